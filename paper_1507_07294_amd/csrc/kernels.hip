// HIP kernels (gfx950) of the time step of the 3D MRT lattice-Boltzmann
// phase-field model of Liang, Shi & Chai (arXiv:1507.07294).
//
// State between steps (pull scheme, two time levels): buffer `cur` holds the
// post-collision populations of the previous step at their source node; a node
// gathers f_i(x) = f*_i(x - c_i), or f*_opp(i)(x) when x - c_i lies beyond a
// wall (half-way bounce-back).  Arrays are structure-of-arrays, one array per
// population, `pitch` elements apart.
//
// The time step itself is one kernel (fused.hip).  This file holds the
// per-node kernels around it:
//   k_phi, k_mu   phi = sum_i f_i (Eq. 13) and mu (Eqs. 2, 36) into arrays,
//                 for read-out, totals and the initial state
//   k_macro       one macroscopic field at the current level
//   k_totals      FP64 sums of phi, momentum and force, non-finite count
//   k_front       lowest and highest zero crossing of phi along z
//   k_init        equilibrium initial state (Eqs. 5, 21)
#include <cmath>

#include "common.h"
#include "device.h"
#include "launch.h"

namespace mplb {
namespace {

using namespace dev;

// ------------------------------------------------------------------ kernels
constexpr int kBlock = 256;

// Q: velocities of the NSE lattice (15 or 19); 16-bit populations of either
// lattice pack f_i with g_i (i = 1..6, the same face velocities).
template <int P, bool COUPLED, int Q>
constexpr bool packed_q() { return packed<P, COUPLED>(); }

template <int P, bool COUPLED, int Q = 15>
__global__ void __launch_bounds__(kBlock) k_phi(Geo G, Bufs B, int cur) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  int x, y, z;
  decode(G, n, x, y, z);
  T f[7];
  pull_f<P, packed_q<P, COUPLED, Q>()>(G, B.f[cur], x, y, z, n, f);
  ((T*)B.phi)[n] = phi_of(f);
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_mu(Geo G, Coef<typename Prec<P>::T> C, Bufs B) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  int x, y, z;
  decode(G, n, x, y, z);
  const T* phi = (const T*)B.phi;
  T c0 = phi[n], gr[3], lap;
  grad_lap(G, phi, x, y, z, c0, gr, lap, false, C.stencil7 != 0);
  ((T*)B.mu)[n] = 4 * C.beta * c0 * (c0 - 1) * (c0 + 1) - C.kappa * lap;
}


// Macroscopic state of node n at the current level (phi and mu arrays must
// hold this level).  Returns false if a pulled population is non-finite.
template <int P, bool COUPLED, int Q = 15>
__device__ inline bool node_macro(const Geo& G, const Coef<typename Prec<P>::T>& C, const Bufs& B, int cur, int n,
                                  Macro<typename Prec<P>::T>& M) {
  using T = typename Prec<P>::T;
  int x, y, z;
  decode(G, n, x, y, z);
  constexpr bool PK = packed_q<P, COUPLED, Q>();
  T f[7];
  pull_f<P, PK>(G, B.f[cur], x, y, z, n, f);
  T phi = phi_of(f);
  bool ok = all_finite(f, 7);
  if (COUPLED) {
    T g[Q];
    pull_g<P, PK, Q>(G, B.f[cur], B.g[cur], x, y, z, n, g);
    ok = ok && all_finite(g, Q);
    const T* mus = (const T*)B.mu;
    T mu = mus[n], gphi[3], lapphi, gd[3], lapmu;
    grad_lap(G, (const T*)B.phi, x, y, z, phi, gphi, lapphi, true, C.stencil7 != 0);
    grad_lap(G, mus, x, y, z, mu, gd, lapmu, false, C.stencil7 != 0);
    if constexpr (Q == 19) flow_macro19(C, g, phi, mu, gphi, lapmu, M);
    else flow_macro(C, g, phi, mu, gphi, lapmu, M);
  } else {
    T gr[3], lap;
    grad_lap(G, (const T*)B.phi, x, y, z, phi, gr, lap, false, C.stencil7 != 0);
    M.phi = phi;
    M.mu = 4 * C.beta * phi * (phi - 1) * (phi + 1) - C.kappa * lap;
    M.rho = (1 + phi) / 2 * C.rho_l + (1 - phi) / 2 * C.rho_g;
    presc_u(G, C, (const T*)B.ufield, x, y, z, n, M.u);
    M.p = 0;
    M.F[0] = M.F[1] = M.F[2] = 0;
    M.gr[0] = M.gr[1] = M.gr[2] = 0;
  }
  return ok;
}

template <int P, bool COUPLED, int Q = 15>
__global__ void __launch_bounds__(kBlock) k_macro(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur, int field) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  Macro<T> M;
  node_macro<P, COUPLED, Q>(G, C, B, cur, n, M);
  T v = 0;
  switch (field) {
    case MPLB_PHI: v = M.phi; break;
    case MPLB_RHO: v = M.rho; break;
    case MPLB_MU: v = M.mu; break;
    case MPLB_UX: v = M.u[0]; break;
    case MPLB_UY: v = M.u[1]; break;
    case MPLB_UZ: v = M.u[2]; break;
    case MPLB_P: v = M.p; break;
  }
  B.out[n] = (double)v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-block FP64 partial sums of phi, j = sum_i c_i g_i, F and the count of
// non-finite nodes; grid-stride over nodes, one slot of 8 doubles per block.
template <int P, bool COUPLED, int Q = 15>
__global__ void __launch_bounds__(kBlock) k_totals(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur) {
  using T = typename Prec<P>::T;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // 64-bit stride: the last node plus one stride can pass INT_MAX
  for (long long nl = (long long)blockIdx.x * kBlock + threadIdx.x; nl < G.N; nl += (long long)gridDim.x * kBlock) {
    const int n = (int)nl;
    Macro<T> M;
    bool ok = node_macro<P, COUPLED, Q>(G, C, B, cur, n, M);
    acc[0] += (double)M.phi;
    if (COUPLED) {
      int x, y, z;
      decode(G, n, x, y, z);
      T g[Q];
      pull_g<P, packed_q<P, COUPLED, Q>(), Q>(G, B.f[cur], B.g[cur], x, y, z, n, g);
      double gd[Q];
      for (int i = 0; i < Q; ++i) gd[i] = (double)g[i];
      for (int i = 0; i < Q; ++i) {
        acc[1] += cq<Q>(i, 0) * gd[i];
        acc[2] += cq<Q>(i, 1) * gd[i];
        acc[3] += cq<Q>(i, 2) * gd[i];
      }
      acc[4] += (double)M.F[0];
      acc[5] += (double)M.F[1];
      acc[6] += (double)M.F[2];
    }
    acc[7] += ok ? 0.0 : 1.0;
  }
  __shared__ double part[kBlock / 64][8];
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    double v = wave_sum(acc[k]);
    if (lane == 0) part[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    double v = 0;
    for (int w = 0; w < kBlock / 64; ++w) v += part[w][threadIdx.x];
    B.red[(size_t)blockIdx.x * 8 + threadIdx.x] = v;
  }
}

// Fixed-order sum of the per-block partials (deterministic).
__global__ void __launch_bounds__(kBlock) k_totals_final(double* red, int nslots) {
  __shared__ double part[kBlock / 64][8];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = threadIdx.x; s < nslots; s += kBlock)
    for (int k = 0; k < 8; ++k) acc[k] += red[(size_t)s * 8 + k];
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < 8; ++k) {
    double v = wave_sum(acc[k]);
    if (lane == 0) part[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    double v = 0;
    for (int w = 0; w < kBlock / 64; ++w) v += part[w][threadIdx.x];
    red[(size_t)kRedSlots * 8 + threadIdx.x] = v;
  }
}

// Interface extremes along z (Rayleigh-Taylor spike tip and bubble front):
// each thread scans columns (x, y) upward through the phi array, locating
// sign changes of phi between layers k and k+1 by linear interpolation at
// z = k + 1/2 + phi_k / (phi_k - phi_{k+1}) (layer k sits at k + 1/2); the
// block keeps the lowest and highest crossing in slots 0 and 1 of its 8.
template <class T>
__global__ void __launch_bounds__(kBlock) k_front(Geo G, Bufs B) {
  const T* phi = (const T*)B.phi;
  const int cols = G.nx * G.ny;
  const size_t plane = (size_t)cols;
  double lo = INFINITY, hi = -INFINITY;
  for (int c = blockIdx.x * kBlock + threadIdx.x; c < cols; c += gridDim.x * kBlock) {
    double a = (double)phi[c];
    for (int k = 0; k + 1 < G.nz; ++k) {
      const double b = (double)phi[(size_t)(k + 1) * plane + c];
      if ((a < 0.0) != (b < 0.0)) {
        const double z = k + 0.5 + a / (a - b);
        lo = fmin(lo, z);
        hi = fmax(hi, z);
      }
      a = b;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  __shared__ double part[kBlock / 64][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    part[wave][0] = lo;
    part[wave][1] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      lo = fmin(lo, part[w][0]);
      hi = fmax(hi, part[w][1]);
    }
    B.red[(size_t)blockIdx.x * 8] = lo;
    B.red[(size_t)blockIdx.x * 8 + 1] = hi;
  }
}

// Extremes over the block slots into the final slot; -1 for both when no
// column crosses.
__global__ void __launch_bounds__(64) k_front_final(double* red, int nslots) {
  double lo = INFINITY, hi = -INFINITY;
  for (int s = threadIdx.x; s < nslots; s += 64) {
    lo = fmin(lo, red[(size_t)s * 8]);
    hi = fmax(hi, red[(size_t)s * 8 + 1]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  if (threadIdx.x == 0) {
    const bool none = !(lo <= hi);
    red[(size_t)kRedSlots * 8] = none ? -1.0 : lo;
    red[(size_t)kRedSlots * 8 + 1] = none ? -1.0 : hi;
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_cvt_in(const double* src, T* dst, int N) {
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n < N) dst[n] = (T)src[n];
}

// Equilibrium populations at every node (Eqs. 5, 21-22 with p = 0), written
// to the storage slot each node will pull them from, so that the first step
// sees f = f^eq and g = g^eq at every node.
template <int P, bool COUPLED, int Q = 15>
__global__ void __launch_bounds__(kBlock) k_init(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  int x, y, z;
  decode(G, n, x, y, z);
  T phi = ((const T*)B.phi)[n], mu = ((const T*)B.mu)[n];
  T* hist = (T*)B.phiu;
  T u[3];
  if (COUPLED) {
    for (int a = 0; a < 3; ++a) u[a] = hist[(size_t)a * G.pitch + n];
  } else {
    presc_u(G, C, (const T*)B.ufield, x, y, z, n, u);
  }
  T w0 = 1 - 3 * C.A, wi = C.A / 2;
  T feq[7];
  feq[0] = phi + (w0 - 1) * C.eta * mu;
#pragma unroll
  for (int i = 1; i < 7; ++i) {
    T cphiu = c7(i, 0) * phi * u[0] + c7(i, 1) * phi * u[1] + c7(i, 2) * phi * u[2];
    feq[i] = wi * C.eta * mu + wi * cphiu / C.A;
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    int s = (i == 0) ? n : pull_src(G, x, y, z, c7(i, 0), c7(i, 1), c7(i, 2));
    if (s >= 0) Lat<P, packed_q<P, COUPLED, Q>()>::stf(B.f[cur], G.pitch, i, s, feq[i]);
    else Lat<P, packed_q<P, COUPLED, Q>()>::stf(B.f[cur], G.pitch, opp(i), n, feq[i]);
  }
  if (COUPLED) {
    T rho = (1 + phi) / 2 * C.rho_l + (1 - phi) / 2 * C.rho_g;
    T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T w = Q == 19 ? ((i == 0) ? (T)(1.0 / 3.0) : (i < 7 ? (T)(1.0 / 18.0) : (T)(1.0 / 36.0)))
                    : ((i == 0) ? (T)(2.0 / 9.0) : (i < 7 ? (T)(1.0 / 9.0) : (T)(1.0 / 72.0)));
      T cu = cq<Q>(i, 0) * u[0] + cq<Q>(i, 1) * u[1] + cq<Q>(i, 2) * u[2];
      T geq = rho * w * (3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);  // Eq. 21 with p = 0
      int s = (i == 0) ? n : pull_src(G, x, y, z, cq<Q>(i, 0), cq<Q>(i, 1), cq<Q>(i, 2));
      if (s >= 0) Lat<P, packed_q<P, COUPLED, Q>()>::stg(B.f[cur], B.g[cur], G.pitch, i, s, geq);
      else Lat<P, packed_q<P, COUPLED, Q>()>::stg(B.f[cur], B.g[cur], G.pitch, opp(i), n, geq);
    }
  }
  if (COUPLED) {
    for (int a = 0; a < 3; ++a) hist[(size_t)a * G.pitch + n] = phi * u[a];
  } else {
    hist[n] = phi;  // CHE-only: the history is phi alone
  }
}

// plain streaming copy with 16-byte accesses (bandwidth reference)
__global__ void __launch_bounds__(kBlock) k_copy16(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) b[i] = a[i];
}

// the same with non-temporal (streaming) stores, the store policy of the
// step kernels on large lattices
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kBlock) k_copy16_nt(const u32x4* __restrict__ a, u32x4* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    __builtin_nontemporal_store(a[i], &b[i]);
}

// four elements per thread and round, non-temporal both ways; the rounds in
// which every thread moves four, then one element per thread up to n
__global__ void __launch_bounds__(kBlock) k_copy16_u4(const u32x4* __restrict__ a, u32x4* __restrict__ b, size_t n) {
  const size_t T = (size_t)gridDim.x * kBlock, tid = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t full = n / (4 * T);
  for (size_t r = 0; r < full; ++r) {
    const size_t base = r * 4 * T + tid;
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(&a[base + u * T]);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], &b[base + u * T]);
  }
  for (size_t i = full * 4 * T + tid; i < n; i += T) __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
}

// each block streams its own contiguous chunk of `chunk` elements, four per
// thread and round, non-temporal both ways (the last chunk may be short)
__global__ void __launch_bounds__(kBlock) k_copy16_chunk(const u32x4* __restrict__ a, u32x4* __restrict__ b, size_t n,
                                                         size_t chunk) {
  const size_t lo = (size_t)blockIdx.x * chunk;
  const size_t hi = lo + chunk < n ? lo + chunk : n;
  for (size_t i = lo + threadIdx.x; i < hi; i += 4 * kBlock) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * kBlock < hi) v[u] = __builtin_nontemporal_load(&a[i + u * kBlock]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * kBlock < hi) __builtin_nontemporal_store(v[u], &b[i + u * kBlock]);
  }
}

__global__ void k_fill_int(int* p, int v, int count) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = v;
}

template <class T>
__global__ void k_fill_zero(T* p, int count) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = (T)0;
}

template <int P, bool COUPLED, int Q = 15>
__global__ void k_poke(Geo G, Bufs B, int cur, int set, int i, int n, double v) {
  using T = typename Prec<P>::T;
  using L = Lat<P, packed_q<P, COUPLED, Q>()>;
  if (set == 0) L::stf(B.f[cur], G.pitch, i, n, (T)v);
  else L::stg(B.f[cur], B.g[cur], G.pitch, i, n, (T)v);
}

template <class T>
Coef<T> cast_coef(const Coef<double>& c) {
  Coef<T> o;
  o.rho_l = (T)c.rho_l; o.rho_g = (T)c.rho_g; o.drho = (T)c.drho;
  o.beta = (T)c.beta; o.kappa = (T)c.kappa; o.eta = (T)c.eta; o.A = (T)c.A; o.mob = (T)c.mob;
  o.rho_ref = (T)c.rho_ref;
  for (int a = 0; a < 3; ++a) o.grav[a] = (T)c.grav[a];
  for (int i = 0; i < 7; ++i) o.sf[i] = (T)c.sf[i];
  for (int i = 0; i < 15; ++i) o.lg[i] = (T)c.lg[i];
  o.vel_kind = c.vel_kind; o.velU = (T)c.velU; o.vel_ct = (T)c.vel_ct; o.vel_ct_prev = (T)c.vel_ct_prev;
  o.stencil7 = c.stencil7; o.forcing28 = c.forcing28;
  o.unit_rates = c.unit_rates;
  o.poison = c.poison;
  return o;
}

inline dim3 grid_for(int N) { return dim3((unsigned)((N + kBlock - 1) / kBlock)); }

template <int P>
hipError_t macro_impl(int mode, const Geo& G, const Coef<double>& Cd, const Bufs& B, int cur, int field, hipStream_t s) {
  using T = typename Prec<P>::T;
  Coef<T> C = cast_coef<T>(Cd);
  if (mode == MPLB_COUPLED) hipLaunchKernelGGL((k_macro<P, true>), grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur, field);
  else if (mode == MPLB_COUPLED_Q19)
    hipLaunchKernelGGL((k_macro<P, true, 19>), grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur, field);
  else hipLaunchKernelGGL((k_macro<P, false>), grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur, field);
  return hipGetLastError();
}

template <int P>
hipError_t totals_impl(int mode, const Geo& G, const Coef<double>& Cd, const Bufs& B, int cur, hipStream_t s) {
  using T = typename Prec<P>::T;
  Coef<T> C = cast_coef<T>(Cd);
  int blocks = (G.N + kBlock - 1) / kBlock;
  if (blocks > kRedSlots) blocks = kRedSlots;
  if (mode == MPLB_COUPLED) hipLaunchKernelGGL((k_totals<P, true>), dim3(blocks), dim3(kBlock), 0, s, G, C, B, cur);
  else if (mode == MPLB_COUPLED_Q19)
    hipLaunchKernelGGL((k_totals<P, true, 19>), dim3(blocks), dim3(kBlock), 0, s, G, C, B, cur);
  else hipLaunchKernelGGL((k_totals<P, false>), dim3(blocks), dim3(kBlock), 0, s, G, C, B, cur);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(kBlock), 0, s, B.red, blocks);
  return hipGetLastError();
}

template <int P>
hipError_t init_impl(int mode, const Geo& G, const Coef<double>& Cd, const Bufs& B, int cur, hipStream_t s) {
  using T = typename Prec<P>::T;
  Coef<T> C = cast_coef<T>(Cd);
  if (mode == MPLB_COUPLED) hipLaunchKernelGGL((k_init<P, true>), grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur);
  else if (mode == MPLB_COUPLED_Q19)
    hipLaunchKernelGGL((k_init<P, true, 19>), grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur);
  else hipLaunchKernelGGL((k_init<P, false>), grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur);
  return hipGetLastError();
}

}  // namespace

#define MPLB_DISPATCH(P, CALL)                      \
  switch (P) {                                      \
    case MPLB_F64: { constexpr int PP = MPLB_F64; CALL; } \
    case MPLB_F32: { constexpr int PP = MPLB_F32; CALL; } \
    case MPLB_F32_F16: { constexpr int PP = MPLB_F32_F16; CALL; } \
    case MPLB_F32_BF16: { constexpr int PP = MPLB_F32_BF16; CALL; } \
    default: return hipErrorInvalidValue;           \
  }

hipError_t launch_phi(int P, int mode, const Geo& G, const Bufs& B, int cur, hipStream_t s) {
  MPLB_DISPATCH(P, {
    if (mode == MPLB_COUPLED) hipLaunchKernelGGL((k_phi<PP, true>), grid_for(G.N), dim3(kBlock), 0, s, G, B, cur);
    else if (mode == MPLB_COUPLED_Q19)
      hipLaunchKernelGGL((k_phi<PP, true, 19>), grid_for(G.N), dim3(kBlock), 0, s, G, B, cur);
    else hipLaunchKernelGGL((k_phi<PP, false>), grid_for(G.N), dim3(kBlock), 0, s, G, B, cur);
    return hipGetLastError();
  })
}

hipError_t launch_mu(int P, const Geo& G, const Coef<double>& Cd, const Bufs& B, hipStream_t s) {
  MPLB_DISPATCH(P, {
    using T = typename Prec<PP>::T;
    hipLaunchKernelGGL(k_mu<PP>, grid_for(G.N), dim3(kBlock), 0, s, G, cast_coef<T>(Cd), B);
    return hipGetLastError();
  })
}

hipError_t launch_macro(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur, int field,
                        hipStream_t s) {
  MPLB_DISPATCH(P, return macro_impl<PP>(mode, G, C, B, cur, field, s))
}

hipError_t launch_totals(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur, hipStream_t s) {
  MPLB_DISPATCH(P, return totals_impl<PP>(mode, G, C, B, cur, s))
}

hipError_t launch_front(int P, const Geo& G, const Bufs& B, hipStream_t s) {
  const int cols = G.nx * G.ny;
  int blocks = (cols + kBlock - 1) / kBlock;
  if (blocks > kRedSlots) blocks = kRedSlots;
  if (P == MPLB_F64) hipLaunchKernelGGL(k_front<double>, dim3(blocks), dim3(kBlock), 0, s, G, B);
  else hipLaunchKernelGGL(k_front<float>, dim3(blocks), dim3(kBlock), 0, s, G, B);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_front_final, dim3(1), dim3(64), 0, s, B.red, blocks);
  return hipGetLastError();
}

// The vertical plane x = y of a field with nx = ny (the diagonal section of a
// Rayleigh-Taylor box): out[z * nx + i] = f(i, i, z).
__global__ void __launch_bounds__(kBlock) k_diag(const double* __restrict__ f, double* __restrict__ out, int nx,
                                                 int nz) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= nx * nz) return;
  const int i = t % nx, z = t / nx;
  out[t] = f[((size_t)z * nx + i) * nx + i];
}

hipError_t launch_diag(const double* f, double* out, int nx, int nz, hipStream_t s) {
  hipLaunchKernelGGL(k_diag, grid_for(nx * nz), dim3(kBlock), 0, s, f, out, nx, nz);
  return hipGetLastError();
}

hipError_t launch_cvt_in(int P, const Geo& G, const Bufs& B, void* dst, hipStream_t s) {
  if (P == MPLB_F64) hipLaunchKernelGGL(k_cvt_in<double>, grid_for(G.N), dim3(kBlock), 0, s, B.out, (double*)dst, G.N);
  else hipLaunchKernelGGL(k_cvt_in<float>, grid_for(G.N), dim3(kBlock), 0, s, B.out, (float*)dst, G.N);
  return hipGetLastError();
}

hipError_t launch_init(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur, hipStream_t s) {
  MPLB_DISPATCH(P, return init_impl<PP>(mode, G, C, B, cur, s))
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int kind, hipStream_t s) {
  if (kind == 3) {
    const size_t n = bytes / 16, chunk = (size_t)16384;  // 256 KB per block
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy16_chunk, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(kBlock), 0, s,
                       (const u32x4*)src, (u32x4*)dst, n, chunk);
  } else if (kind == 2)
    hipLaunchKernelGGL(k_copy16_u4, dim3(16384), dim3(kBlock), 0, s, (const u32x4*)src, (u32x4*)dst, bytes / 16);
  else if (kind == 1)
    hipLaunchKernelGGL(k_copy16_nt, dim3(32768), dim3(kBlock), 0, s, (const u32x4*)src, (u32x4*)dst, bytes / 16);
  else
    hipLaunchKernelGGL(k_copy16, dim3(32768), dim3(kBlock), 0, s, (const float4*)src, (float4*)dst, bytes / 16);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int value, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, grid_for(count), dim3(kBlock), 0, s, p, value, count);
  return hipGetLastError();
}

hipError_t launch_fill_zero(int P, void* p, int count, hipStream_t s) {
  if (P == MPLB_F64) hipLaunchKernelGGL(k_fill_zero<double>, grid_for(count), dim3(kBlock), 0, s, (double*)p, count);
  else hipLaunchKernelGGL(k_fill_zero<float>, grid_for(count), dim3(kBlock), 0, s, (float*)p, count);
  return hipGetLastError();
}

hipError_t launch_poke(int P, int mode, const Geo& G, const Bufs& B, int cur, int set, int i, int n, double v,
                       hipStream_t s) {
  MPLB_DISPATCH(P, {
    if (mode == MPLB_COUPLED) hipLaunchKernelGGL((k_poke<PP, true>), dim3(1), dim3(1), 0, s, G, B, cur, set, i, n, v);
    else if (mode == MPLB_COUPLED_Q19)
      hipLaunchKernelGGL((k_poke<PP, true, 19>), dim3(1), dim3(1), 0, s, G, B, cur, set, i, n, v);
    else hipLaunchKernelGGL((k_poke<PP, false>), dim3(1), dim3(1), 0, s, G, B, cur, set, i, n, v);
    return hipGetLastError();
  })
}

}  // namespace mplb
