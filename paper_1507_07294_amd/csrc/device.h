// Device building blocks of the libmplb kernels: lattice tables, storage
// access, pull streaming with bounce-back, the finite differences of
// Eqs. 35-36, the macroscopic closure (Eqs. 29-30) and the two moment-space
// collisions.  Included by the kernel translation units.
#pragma once

#include <cmath>

#include "common.h"

namespace mplb {
namespace dev {

// ---------------------------------------------------------------- lattices
// D3Q15 velocities in the order of Eq. 23; D3Q7 in the order of Eq. 6.
__host__ __device__ constexpr int c15(int i, int a) {
  constexpr int t[15][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                            {0, 0, 1},   {0, 0, -1},  {1, 1, 1},   {-1, -1, -1}, {1, 1, -1},
                            {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1}, {1, -1, -1}, {-1, 1, 1}};
  return t[i][a];
}
__host__ __device__ constexpr int c7(int i, int a) {
  constexpr int t[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  return t[i][a];
}
// D3Q19 (the other NSE lattice the paper names, after Eq. 22): rest, the
// faces in the order of Eq. 23, then the twelve edges
__host__ __device__ constexpr int c19(int i, int a) {
  constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                            {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                            {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  return t[i][a];
}
// velocity i of the NSE lattice with Q velocities (15 or 19)
template <int Q>
__host__ __device__ constexpr int cq(int i, int a) { return Q == 19 ? c19(i, a) : c15(i, a); }
// all lattices list velocities in antipodal pairs (1,2), (3,4), ...
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// ---------------------------------------------------------------- storage
// Population storage of one time level, in a buffer for f and one for g.
//   f buffer: f_0 (S0, `pitch` elements), then f_1..f_6;
//   g buffer: g_0..g_{Q-1} (S), each array `pitch` elements.
// PACK (16-bit populations of the coupled model): f_i and g_i, i = 1..6,
// share a velocity and therefore a pull source, so they are stored together
// in one 32-bit word (f_i in the low half, g_i in the high half) in six
// arrays after f_0; the g buffer then holds g_0 and g_7..g_{Q-1} (the
// corners of D3Q15, the edges of D3Q19).
template <int P, bool PACK>
struct Lat {
  using T = typename Prec<P>::T;
  using S0 = typename Prec<P>::S0;
  using S = typename Prec<P>::S;
  static_assert(!PACK || sizeof(S) == 2, "packing needs 16-bit populations");
  __device__ static const S0* f0(const void* fb) { return (const S0*)fb; }
  __device__ static S0* f0(void* fb) { return (S0*)fb; }
  // population array i >= 1 of the f buffer (PACK: the 32-bit words as pairs of S)
  __device__ static const S* fi(const void* fb, int pitch) {
    return (const S*)((const char*)fb + (size_t)pitch * sizeof(S0));
  }
  __device__ static S* fi(void* fb, int pitch) { return (S*)((char*)fb + (size_t)pitch * sizeof(S0)); }
  __device__ static const uint32_t* words(const void* fb, int pitch) { return (const uint32_t*)fi(fb, pitch); }
  __device__ static uint32_t* words(void* fb, int pitch) { return (uint32_t*)fi(fb, pitch); }
  // g array holding population i (PACK: 0 -> 0, 7..14 -> 1..8)
  __device__ static size_t gslot(int i) { return PACK ? (i == 0 ? 0 : (size_t)(i - 6)) : (size_t)i; }

  __device__ static T ldf(const void* fb, int pitch, int i, int n) {
    if (i == 0) return (T)f0(fb)[n];
    size_t k = (size_t)(i - 1) * pitch + n;
    return PACK ? (T)fi(fb, pitch)[2 * k] : (T)fi(fb, pitch)[k];
  }
  __device__ static void stf(void* fb, int pitch, int i, int n, T v) {
    if (i == 0) { f0(fb)[n] = (S0)v; return; }
    size_t k = (size_t)(i - 1) * pitch + n;
    if (PACK) fi(fb, pitch)[2 * k] = (S)v;
    else fi(fb, pitch)[k] = (S)v;
  }
  __device__ static T ldg(const void* fb, const void* gb, int pitch, int i, int n) {
    if (PACK && i >= 1 && i <= 6) return (T)fi(fb, pitch)[2 * ((size_t)(i - 1) * pitch + n) + 1];
    return (T)((const S*)gb)[gslot(i) * pitch + n];
  }
  __device__ static void stg(void* fb, void* gb, int pitch, int i, int n, T v) {
    if (PACK && i >= 1 && i <= 6) fi(fb, pitch)[2 * ((size_t)(i - 1) * pitch + n) + 1] = (S)v;
    else ((S*)gb)[gslot(i) * pitch + n] = (S)v;
  }
  // 16-bit halves <-> compute type
  __device__ static T lo(uint32_t w) { return (T)__builtin_bit_cast(S, (uint16_t)(w & 0xffffu)); }
  __device__ static T hi(uint32_t w) { return (T)__builtin_bit_cast(S, (uint16_t)(w >> 16)); }
  // one packed conversion for both halves (round to nearest even)
  __device__ static uint32_t pack(T a, T b) {
    typedef float F2 __attribute__((ext_vector_type(2)));
    typedef S S2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((F2){(float)a, (float)b}, S2));
  }
};

// 16-bit populations of the coupled model are stored packed (see Lat)
template <int P, bool COUPLED>
constexpr bool packed() { return COUPLED && sizeof(typename Prec<P>::S) == 2; }

// ---------------------------------------------------------------- geometry
__device__ inline void decode(const Geo& G, int n, int& x, int& y, int& z) {
  x = n % G.nx;
  int t = n / G.nx;
  y = t % G.ny;
  z = t / G.ny;
}

// Source node of a population with velocity (cx,cy,cz) arriving at (x,y,z),
// or -1 if it left through a wall (then it is the opposite population of
// (x,y,z) reflected back).
__device__ inline int pull_src(const Geo& G, int x, int y, int z, int cx, int cy, int cz) {
  int sx = x - cx, sy = y - cy, sz = z - cz;
  if (sx < 0) { if (G.wall_x) return -1; sx += G.nx; } else if (sx >= G.nx) { if (G.wall_x) return -1; sx -= G.nx; }
  if (sy < 0) { if (G.wall_y) return -1; sy += G.ny; } else if (sy >= G.ny) { if (G.wall_y) return -1; sy -= G.ny; }
  if (sz < 0) { if (G.wall_z) return -1; sz += G.nz; } else if (sz >= G.nz) { if (G.wall_z) return -1; sz -= G.nz; }
  return sx + G.nx * (sy + G.ny * sz);
}

// Neighbour for the finite differences: periodic wrap, or the mirror ghost
// chi(-1) = chi(0), chi(n) = chi(n-1) on wall axes.
__device__ inline int stencil_nb(const Geo& G, int x, int y, int z, int dx, int dy, int dz) {
  int qx = x + dx, qy = y + dy, qz = z + dz;
  if (qx < 0) qx = G.wall_x ? 0 : qx + G.nx; else if (qx >= G.nx) qx = G.wall_x ? G.nx - 1 : qx - G.nx;
  if (qy < 0) qy = G.wall_y ? 0 : qy + G.ny; else if (qy >= G.ny) qy = G.wall_y ? G.ny - 1 : qy - G.ny;
  if (qz < 0) qz = G.wall_z ? 0 : qz + G.nz; else if (qz >= G.nz) qz = G.wall_z ? G.nz - 1 : qz - G.nz;
  return qx + G.nx * (qy + G.ny * qz);
}

template <int P, bool PACK>
__device__ inline void pull_f(const Geo& G, const void* fb, int x, int y, int z, int n, typename Prec<P>::T f[7]) {
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    int s = (i == 0) ? n : pull_src(G, x, y, z, c7(i, 0), c7(i, 1), c7(i, 2));
    f[i] = (s >= 0) ? Lat<P, PACK>::ldf(fb, G.pitch, i, s) : Lat<P, PACK>::ldf(fb, G.pitch, opp(i), n);
  }
}

template <int P, bool PACK, int Q = 15>
__device__ inline void pull_g(const Geo& G, const void* fb, const void* gb, int x, int y, int z, int n,
                              typename Prec<P>::T g[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int s = (i == 0) ? n : pull_src(G, x, y, z, cq<Q>(i, 0), cq<Q>(i, 1), cq<Q>(i, 2));
    g[i] = (s >= 0) ? Lat<P, PACK>::ldg(fb, gb, G.pitch, i, s) : Lat<P, PACK>::ldg(fb, gb, G.pitch, opp(i), n);
  }
}

template <class T>
__device__ inline T phi_of(const T f[7]) {
  return f[0] + (((f[1] + f[2]) + (f[3] + f[4])) + (f[5] + f[6]));
}

// Eq. 35 (gradient) and Eq. 36 (Laplacian) with D3Q15 weights, c_s^2 = 1/3:
// face neighbours weigh 1/3 (gradient) and 2/3 (Laplacian), corners 1/24 and
// 1/12.  s7: the D3Q7 weights instead (w_i / c_s^2 = 1/2: central
// differences and the 7-point Laplacian).
template <class T>
__device__ inline void grad_lap(const Geo& G, const T* chi, int x, int y, int z, T c0, T gr[3], T& lap,
                                bool want_grad, bool s7 = false) {
  if (s7) {
    T v[7];
#pragma unroll
    for (int i = 1; i < 7; ++i) v[i] = chi[stencil_nb(G, x, y, z, c7(i, 0), c7(i, 1), c7(i, 2))];
    lap = (((v[1] - c0) + (v[2] - c0)) + ((v[3] - c0) + (v[4] - c0))) + ((v[5] - c0) + (v[6] - c0));
    gr[0] = (T)0.5 * (v[1] - v[2]);
    gr[1] = (T)0.5 * (v[3] - v[4]);
    gr[2] = (T)0.5 * (v[5] - v[6]);
    return;
  }
  T gx = 0, gy = 0, gz = 0, lf = 0, lc = 0;
#pragma unroll
  for (int i = 1; i < 15; ++i) {
    T v = chi[stencil_nb(G, x, y, z, c15(i, 0), c15(i, 1), c15(i, 2))];
    if (i < 7) {
      lf += v - c0;
      if (want_grad) { gx += c15(i, 0) * v; gy += c15(i, 1) * v; gz += c15(i, 2) * v; }
    } else {
      lc += v - c0;
      if (want_grad) {
        gx += (T)(1.0 / 8.0) * c15(i, 0) * v;
        gy += (T)(1.0 / 8.0) * c15(i, 1) * v;
        gz += (T)(1.0 / 8.0) * c15(i, 2) * v;
      }
    }
  }
  lap = (T)(2.0 / 3.0) * lf + (T)(1.0 / 12.0) * lc;
  gr[0] = gx * (T)(1.0 / 3.0);
  gr[1] = gy * (T)(1.0 / 3.0);
  gr[2] = gz * (T)(1.0 / 3.0);
}

// Prescribed velocity of the interface-tracking runs: a constant field,
// Zalesak's rotation (Eq. 37) or the deformation flow (Eq. 41 times
// cos(pi t / T), the cosine passed in as C.vel_ct).  When up is given it
// receives the velocity of the previous level (the same except for the
// deformation flow, whose cosine there is C.vel_ct_prev).
template <class T>
__device__ inline void presc_u(const Geo& G, const Coef<T>& C, const T* uf, int x, int y, int z, int n, T u[3],
                               T* up = nullptr) {
  u[0] = u[1] = u[2] = 0;
  if (C.vel_kind == MPLB_VEL_FIELD) {
    u[0] = uf[n];
    u[1] = uf[(size_t)G.pitch + n];
    u[2] = uf[2 * (size_t)G.pitch + n];
  } else if (C.vel_kind == MPLB_VEL_ZALESAK) {
    const T pi = (T)3.14159265358979323846;
    T L = (T)G.nx;
    u[1] = (C.velU * pi / L) * (L / 2 - (T)z);
    u[2] = (C.velU * pi / L) * ((T)y - L / 2);
  } else if (C.vel_kind == MPLB_VEL_DEFORM) {
    const T pi = (T)3.14159265358979323846;
    T xh = (T)x / (T)G.nx, yh = (T)y / (T)G.ny, zh = (T)z / (T)G.nz;
    T sx = sin(pi * xh), sy = sin(pi * yh), sz = sin(pi * zh);
    T s2x = sin(2 * pi * xh), s2y = sin(2 * pi * yh), s2z = sin(2 * pi * zh);
    T U = C.velU;
    T b[3] = {2 * U * sx * sx * s2y * s2z, -U * s2x * sy * sy * s2z, -U * s2x * s2y * sz * sz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[a] = b[a] * C.vel_ct;
      if (up) up[a] = b[a] * C.vel_ct_prev;
    }
    return;
  }
  if (up) up[0] = u[0], up[1] = u[1], up[2] = u[2];
}

// presc_u along one lattice column (x, y) of a z march: the deformation
// flow (Eq. 41) is a product of x-y factors, evaluated once per column, and
// z factors, evaluated once per plane; the products keep presc_u's order,
// so the values are the same.
template <class T>
struct PrescColumn {
  T a[3] = {0, 0, 0};  // 2U sx^2 s2y, -U s2x sy^2, -U s2x s2y

  __device__ void init(const Geo& G, const Coef<T>& C, int x, int y) {
    if (C.vel_kind != MPLB_VEL_DEFORM) return;
    const T pi = (T)3.14159265358979323846;
    T xh = (T)x / (T)G.nx, yh = (T)y / (T)G.ny;
    T sx = sin(pi * xh), sy = sin(pi * yh);
    T s2x = sin(2 * pi * xh), s2y = sin(2 * pi * yh);
    T U = C.velU;
    a[0] = 2 * U * sx * sx * s2y;
    a[1] = -U * s2x * sy * sy;
    a[2] = -U * s2x * s2y;
  }

  __device__ void at(const Geo& G, const Coef<T>& C, const T* uf, int x, int y, int z, int n, T u[3],
                     T up[3]) const {
    if (C.vel_kind != MPLB_VEL_DEFORM) {
      presc_u(G, C, uf, x, y, z, n, u, up);
      return;
    }
    const T pi = (T)3.14159265358979323846;
    T zh = (T)z / (T)G.nz;
    T sz = sin(pi * zh), s2z = sin(2 * pi * zh);
    T b[3] = {a[0] * s2z, a[1] * s2z, a[2] * sz * sz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      u[k] = b[k] * C.vel_ct;
      up[k] = b[k] * C.vel_ct_prev;
    }
  }
};

// ------------------------------------------------------------ node physics
// Macroscopic state of a node at level n (coupled model).
template <class T>
struct Macro {
  T phi, rho, mu, u[3], p, F[3], gr[3];
};

// u, p and the forces from pulled g, phi, mu, grad phi and lap mu (Eqs. 29-30;
// F_s = mu grad phi, F_a = (rho_l - rho_g) M lap(mu) u / 2, G = (rho - rho_ref) g).
template <class T>
__device__ inline void flow_macro(const Coef<T>& C, const T g[15], T phi, T mu, const T gphi[3], T lapmu,
                                  Macro<T>& m) {
  m.phi = phi;
  m.mu = mu;
  m.rho = (1 + phi) / 2 * C.rho_l + (1 - phi) / 2 * C.rho_g;
  T half_dr = C.drho / 2;
  T jx = (g[1] - g[2]) + (((g[7] - g[8]) + (g[9] - g[10])) + ((g[11] - g[12]) + (g[13] - g[14])));
  T jy = (g[3] - g[4]) + (((g[7] - g[8]) + (g[9] - g[10])) - ((g[11] - g[12]) + (g[13] - g[14])));
  T jz = (g[5] - g[6]) + (((g[7] - g[8]) - (g[9] - g[10])) + ((g[11] - g[12]) - (g[13] - g[14])));
  T sum_nz = ((g[1] + g[2]) + (g[3] + g[4]) + (g[5] + g[6])) +
             (((g[7] + g[8]) + (g[9] + g[10])) + ((g[11] + g[12]) + (g[13] + g[14])));
  T Fs[3], Gb[3], j[3] = {jx, jy, jz};
  T ml = C.mob * lapmu;
  // one division per node (a correctly rounded reciprocal) instead of three
  const T inv = (T)1 / (m.rho - (T)0.25 * C.drho * ml);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m.gr[a] = half_dr * gphi[a];
    Fs[a] = mu * gphi[a];
    Gb[a] = (m.rho - C.rho_ref) * C.grav[a];
    m.u[a] = (j[a] + (T)0.5 * (Fs[a] + Gb[a])) * inv;
    m.F[a] = Fs[a] + half_dr * ml * m.u[a] + Gb[a];
  }
  T uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
  T ugr = m.u[0] * m.gr[0] + m.u[1] * m.gr[1] + m.u[2] * m.gr[2];
  // c_s^2 / (1 - w_0) = 3/7 and rho s_0(u) = -rho |u|^2 / 3 (Eq. 30)
  m.p = (T)(3.0 / 7.0) * (sum_nz + (T)0.5 * ugr - m.rho * uu * (T)(1.0 / 3.0));
}

// The same on D3Q19 (weights 1/3, 1/18, 1/36): c_s^2 / (1 - w_0) = 1/2 and
// rho s_0(u) = -rho |u|^2 / 2 in Eq. 30.
template <class T>
__device__ inline void flow_macro19(const Coef<T>& C, const T g[19], T phi, T mu, const T gphi[3], T lapmu,
                                    Macro<T>& m) {
  m.phi = phi;
  m.mu = mu;
  m.rho = (1 + phi) / 2 * C.rho_l + (1 - phi) / 2 * C.rho_g;
  T half_dr = C.drho / 2;
  T j[3] = {0, 0, 0}, sum_nz = 0;
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    sum_nz += g[i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (c19(i, a) != 0) j[a] += c19(i, a) > 0 ? g[i] : -g[i];
  }
  T Fs[3], Gb[3];
  T ml = C.mob * lapmu;
  // one division per node (a correctly rounded reciprocal) instead of three
  const T inv = (T)1 / (m.rho - (T)0.25 * C.drho * ml);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m.gr[a] = half_dr * gphi[a];
    Fs[a] = mu * gphi[a];
    Gb[a] = (m.rho - C.rho_ref) * C.grav[a];
    m.u[a] = (j[a] + (T)0.5 * (Fs[a] + Gb[a])) * inv;
    m.F[a] = Fs[a] + half_dr * ml * m.u[a] + Gb[a];
  }
  T uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
  T ugr = m.u[0] * m.gr[0] + m.u[1] * m.gr[1] + m.u[2] * m.gr[2];
  m.p = (T)0.5 * (sum_nz + (T)0.5 * ugr - (T)0.5 * m.rho * uu);
}

// D3Q7 collision in moment space (Eqs. 15, 17, 18, 11): m = M f;
// m* = m - S^f (m - m^eq) + (I - S^f/2) mR; f* = M^-1 m*.
template <class T>
__device__ inline void collide_che(const Coef<T>& C, T f[7], T phi, T mu, const T u[3], const T dphiu[3]) {
  T s12 = f[1] + f[2], s34 = f[3] + f[4], s56 = f[5] + f[6];
  T m1 = f[1] - f[2], m2 = f[3] - f[4], m3 = f[5] - f[6];
  T m4 = 6 * f[0] - ((s12 + s34) + s56);
  T m5 = 2 * s12 - (s34 + s56);
  T m6 = s34 - s56;
  T ms1 = m1 - C.sf[1] * (m1 - phi * u[0]) + (1 - C.sf[1] / 2) * dphiu[0];
  T ms2 = m2 - C.sf[2] * (m2 - phi * u[1]) + (1 - C.sf[2] / 2) * dphiu[1];
  T ms3 = m3 - C.sf[3] * (m3 - phi * u[2]) + (1 - C.sf[3] / 2) * dphiu[2];
  T ms4 = m4 - C.sf[4] * (m4 - (6 * phi - 21 * C.A * C.eta * mu));
  T ms5 = m5 - C.sf[5] * m5;
  T ms6 = m6 - C.sf[6] * m6;
  // M^-1 = M^T diag(1/7, 1/2, 1/2, 1/2, 1/42, 1/12, 1/4)
  T b0 = phi * (T)(1.0 / 7.0), b1 = ms1 / 2, b2 = ms2 / 2, b3 = ms3 / 2;
  T b4 = ms4 * (T)(1.0 / 42.0), b5 = ms5 * (T)(1.0 / 12.0), b6 = ms6 / 4;
  T c = b0 - b4;
  f[0] = b0 + 6 * b4;
  f[1] = c + b1 + 2 * b5;
  f[2] = c - b1 + 2 * b5;
  f[3] = c + b2 - b5 + b6;
  f[4] = c - b2 - b5 + b6;
  f[5] = c + b3 - b5 - b6;
  f[6] = c - b3 - b5 - b6;
}

// m = Gamma v for the D3Q15 basis of d'Humieres on the Eq. 23 order
// (corner pairs (7,8) (9,10) (11,12) (13,14) are antipodal).
template <class T>
__device__ inline void gamma15(const T g[15], T m[15]) {
  T sx = g[1] + g[2], sy = g[3] + g[4], sz = g[5] + g[6];
  T dx = g[1] - g[2], dy = g[3] - g[4], dz = g[5] - g[6];
  T p1 = g[7] + g[8], p2 = g[9] + g[10], p3 = g[11] + g[12], p4 = g[13] + g[14];
  T d1 = g[7] - g[8], d2 = g[9] - g[10], d3 = g[11] - g[12], d4 = g[13] - g[14];
  T Sf = (sx + sy) + sz, Sc = (p1 + p2) + (p3 + p4);
  T Xc = (d1 + d2) + (d3 + d4), Yc = (d1 + d2) - (d3 + d4), Zc = (d1 - d2) + (d3 - d4);
  m[0] = g[0] + Sf + Sc;
  m[1] = -2 * g[0] - Sf + Sc;
  m[2] = 16 * g[0] - 4 * Sf + Sc;
  m[3] = dx + Xc;
  m[4] = -4 * dx + Xc;
  m[5] = dy + Yc;
  m[6] = -4 * dy + Yc;
  m[7] = dz + Zc;
  m[8] = -4 * dz + Zc;
  m[9] = 2 * sx - (sy + sz);
  m[10] = sy - sz;
  m[11] = (p1 + p2) - (p3 + p4);
  m[12] = (p1 - p2) - (p3 - p4);
  m[13] = (p1 - p2) + (p3 - p4);
  m[14] = (d1 - d2) - (d3 - d4);
}

// D3Q15 collision in moment space (Eqs. 20, 27, 31, 32): m = Gamma g;
// m* = m - S^g (m - m^eq) + (I - S^g/2) mT; g* = Gamma^-1 m*.  Gamma's rows are
// d'Humieres' basis on the Eq. 23 velocity order.  F28: mT = Gamma T with T
// of Eq. 28 untruncated, instead of the printed Eq. 32 (a compile-time
// switch: the extra registers would cost the default step occupancy).
// UNIT: S^g = 1 off the stress moments 9..13 (the paper's rates); each such
// row relaxes to m^eq + mT/2 whatever its moment was, so only the five stress
// moments of g are formed (about 50 fewer operations per node; a separate
// instantiation, since a run-time branch between the forms spills registers).
template <bool F28 = false, bool UNIT = false, class T>
__device__ inline void collide_ns(const Coef<T>& C, T g[15], const Macro<T>& M) {
  const T* u = M.u;
  T rho = M.rho, p = M.p;
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  T cs2 = (T)(1.0 / 3.0);
  T eq[15], src[15];
  // Eq. 31
  eq[0] = 0;
  eq[1] = 3 * p + rho * uu;
  eq[2] = -(45 * p + 5 * rho * uu);
  eq[3] = rho * u[0];
  eq[4] = (T)(-7.0 / 3.0) * rho * u[0];
  eq[5] = rho * u[1];
  eq[6] = (T)(-7.0 / 3.0) * rho * u[1];
  eq[7] = rho * u[2];
  eq[8] = (T)(-7.0 / 3.0) * rho * u[2];
  eq[9] = rho * (2 * u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
  eq[10] = rho * (u[1] * u[1] - u[2] * u[2]);
  eq[11] = rho * u[0] * u[1];
  eq[12] = rho * u[1] * u[2];
  eq[13] = rho * u[0] * u[2];
  eq[14] = 0;
  // Eq. 32 with F = F_s + F_a + G and a = c_s^2 grad rho + F
  const T* F = M.F;
  T a[3] = {M.gr[0] * cs2 + F[0], M.gr[1] * cs2 + F[1], M.gr[2] * cs2 + F[2]};
  T ugr = u[0] * M.gr[0] + u[1] * M.gr[1] + u[2] * M.gr[2];
  T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  src[0] = ugr;
  src[1] = -ugr * cs2 + 2 * uF;
  src[2] = -(7 * ugr * cs2 + 10 * uF);
  src[3] = F[0];
  src[4] = (T)(-7.0 / 3.0) * F[0];
  src[5] = F[1];
  src[6] = (T)(-7.0 / 3.0) * F[1];
  src[7] = F[2];
  src[8] = (T)(-7.0 / 3.0) * F[2];
  src[9] = 4 * u[0] * a[0] - 2 * u[1] * a[1] - 2 * u[2] * a[2];
  src[10] = 2 * u[1] * a[1] - 2 * u[2] * a[2];
  src[11] = u[0] * a[1] + u[1] * a[0];
  src[12] = u[1] * a[2] + u[2] * a[1];
  src[13] = u[0] * a[2] + u[2] * a[0];
  src[14] = 0;
  if constexpr (F28) {
    // T_i = 3 [s_i (c_i - u).(a) + w_i (c_i - u).F] with a here the sum
    // c_s^2 grad rho + F of Eq. 28 (s_i + w_i multiplies F)
    T Tv[15];
    T ua = u[0] * a[0] + u[1] * a[1] + u[2] * a[2];
#pragma unroll
    for (int i = 0; i < 15; ++i) {
      const T w = i == 0 ? (T)(2.0 / 9.0) : (i < 7 ? (T)(1.0 / 9.0) : (T)(1.0 / 72.0));
      const T cu = c15(i, 0) * u[0] + c15(i, 1) * u[1] + c15(i, 2) * u[2];
      const T si = w * (3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);
      const T ca = c15(i, 0) * a[0] + c15(i, 1) * a[1] + c15(i, 2) * a[2];
      const T cF = c15(i, 0) * F[0] + c15(i, 1) * F[1] + c15(i, 2) * F[2];
      Tv[i] = 3 * (si * (ca - ua) + w * (cF - uF));
    }
    gamma15(Tv, src);
  }
  T ms[15];
  if constexpr (UNIT) {
    T sx = g[1] + g[2], sy = g[3] + g[4], sz = g[5] + g[6];
    T p1 = g[7] + g[8], p2 = g[9] + g[10], p3 = g[11] + g[12], p4 = g[13] + g[14];
    T m[15];
    m[9] = 2 * sx - (sy + sz);
    m[10] = sy - sz;
    m[11] = (p1 + p2) - (p3 + p4);
    m[12] = (p1 - p2) - (p3 - p4);
    m[13] = (p1 - p2) + (p3 - p4);
#pragma unroll
    for (int r = 0; r < 15; ++r)
      ms[r] = (r >= 9 && r <= 13) ? m[r] - C.lg[r] * (m[r] - eq[r]) + (1 - C.lg[r] / 2) * src[r]
                                  : eq[r] + src[r] / 2;
  } else {
    T m[15];
    gamma15(g, m);
#pragma unroll
    for (int r = 0; r < 15; ++r) ms[r] = m[r] - C.lg[r] * (m[r] - eq[r]) + (1 - C.lg[r] / 2) * src[r];
  }
  // Gamma^-1 = Gamma^T diag(1/15, 1/18, 1/360, 1/10, 1/40, 1/10, 1/40, 1/10, 1/40, 1/12, 1/4, 1/8, 1/8, 1/8, 1/8)
  T a0 = ms[0] * (T)(1.0 / 15.0), a1 = ms[1] * (T)(1.0 / 18.0), a2 = ms[2] * (T)(1.0 / 360.0);
  T a3 = ms[3] * (T)(1.0 / 10.0), a4 = ms[4] * (T)(1.0 / 40.0);
  T a5 = ms[5] * (T)(1.0 / 10.0), a6 = ms[6] * (T)(1.0 / 40.0);
  T a7 = ms[7] * (T)(1.0 / 10.0), a8 = ms[8] * (T)(1.0 / 40.0);
  T a9 = ms[9] * (T)(1.0 / 12.0), a10 = ms[10] / 4;
  T a11 = ms[11] / 8, a12 = ms[12] / 8, a13 = ms[13] / 8, a14 = ms[14] / 8;
  g[0] = a0 - 2 * a1 + 16 * a2;
  T F0 = a0 - a1 - 4 * a2;
  T ex = a3 - 4 * a4, ey = a5 - 4 * a6, ez = a7 - 4 * a8;
  g[1] = F0 + 2 * a9 + ex;
  g[2] = F0 + 2 * a9 - ex;
  g[3] = F0 - a9 + a10 + ey;
  g[4] = F0 - a9 + a10 - ey;
  g[5] = F0 - a9 - a10 + ez;
  g[6] = F0 - a9 - a10 - ez;
  T base = a0 + a1 + a2, X = a3 + a4, Y = a5 + a6, Z = a7 + a8;
  // corner c: base + c.(X,Y,Z) + cx cy a11 + cy cz a12 + cx cz a13 + cx cy cz a14
  T P1 = base + a11 + a12 + a13, Q1 = X + Y + Z + a14;      // (1,1,1)
  T P2 = base + a11 - a12 - a13, Q2 = X + Y - Z - a14;      // (1,1,-1)
  T P3 = base - a11 - a12 + a13, Q3 = X - Y + Z - a14;      // (1,-1,1)
  T P4 = base - a11 + a12 - a13, Q4 = X - Y - Z + a14;      // (1,-1,-1)
  g[7] = P1 + Q1;
  g[8] = P1 - Q1;
  g[9] = P2 + Q2;
  g[10] = P2 - Q2;
  g[11] = P3 + Q3;
  g[12] = P3 - Q3;
  g[13] = P4 + Q4;
  g[14] = P4 - Q4;
}


// D3Q19 collision.  With S^g = 1 except lambda on the five stress moments
// (rows 3pxx, pww, pxy, pyz, pxz of d'Humieres' basis, squared norms 36, 12,
// 4, 4, 4), m* = m - S(m - m^eq) + (I - S/2) m_T with m^eq = Gamma g^eq and
// m_T = Gamma T is, after Gamma^-1,
//   g* = g^eq + T/2 - (lambda - 1) Gamma^-1 P Gamma (g - g^eq + T/2),
// P the projector on the stress moments: only those five moments are formed.
// g^eq from Eqs. 21-22, T from Eq. 28 (F = F_s + F_a + G), both in velocity
// space.  Velocities come in antipodal pairs (i, i+1), c_{i+1} = -c_i, so per
// pair with s_i = E + O (E even, O odd in c):
//   g^eq = G0 +- rho O,  T = Te +- To,
// and the stress-moment weights, quadratic in c, are the same for both: the
// pair enters the moments through (g_i + g_{i+1}) and takes one correction.
// The rest population has no stress weight, so it is g^eq + T/2.
template <class T>
__device__ inline void collide_ns19(const Coef<T>& C, T g[19], const Macro<T>& M) {
  const T* u = M.u;
  const T* F = M.F;
  const T rho = M.rho, p = M.p;
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  // Eq. 28: T_i = 3 [s_i (c_i - u).(a + F) + w_i (c_i - u).F], a = c_s^2 grad rho
  T AF[3], uAF = 0, uF = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    AF[a] = M.gr[a] * (T)(1.0 / 3.0) + F[a];
    uAF += u[a] * AF[a];
    uF += u[a] * F[a];
  }
  {
    const T w = (T)(1.0 / 3.0);
    const T s0 = w * ((T)-1.5 * uu);
    const T T0 = 3 * (s0 * (-uAF) + w * (-uF));
    g[0] = 3 * p * (w - 1) + rho * s0 + T0 / 2;
  }
  T m9 = 0, m11 = 0, m13 = 0, m14 = 0, m15 = 0;
  T be[9], bo[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int i = 2 * k + 1;
    const int cx = c19(i, 0), cy = c19(i, 1), cz = c19(i, 2);
    const T w = i < 7 ? (T)(1.0 / 18.0) : (T)(1.0 / 36.0);
    const T cu = cx * u[0] + cy * u[1] + cz * u[2];
    const T E = w * ((T)4.5 * cu * cu - (T)1.5 * uu);
    const T O = 3 * w * cu;
    const T cAF = cx * AF[0] + cy * AF[1] + cz * AF[2];
    const T cF = cx * F[0] + cy * F[1] + cz * F[2];
    const T G0 = 3 * p * w + rho * E;
    const T Te = 3 * (O * cAF - E * uAF - w * uF);
    const T To = 3 * (E * cAF - O * uAF + w * cF);
    be[k] = G0 + Te / 2;  // g^eq + T/2 of the pair: be +- bo
    bo[k] = rho * O + To / 2;
    // d = g - g^eq + T/2 summed over the pair
    const T dsum = (g[i] + g[i + 1]) - 2 * (G0 - Te / 2);
    const int c2 = cx * cx + cy * cy + cz * cz;
    m9 += (3 * cx * cx - c2) * dsum;
    m11 += (cy * cy - cz * cz) * dsum;
    m13 += (cx * cy) * dsum;
    m14 += (cy * cz) * dsum;
    m15 += (cx * cz) * dsum;
  }
  const T kl = C.lg[9] - 1;
  const T b9 = kl * m9 * (T)(1.0 / 36.0), b11 = kl * m11 * (T)(1.0 / 12.0);
  const T b13 = kl * m13 / 4, b14 = kl * m14 / 4, b15 = kl * m15 / 4;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int i = 2 * k + 1;
    const int cx = c19(i, 0), cy = c19(i, 1), cz = c19(i, 2);
    const int c2 = cx * cx + cy * cy + cz * cz;
    const T corr = (3 * cx * cx - c2) * b9 + (cy * cy - cz * cz) * b11 + (cx * cy) * b13 + (cy * cz) * b14 +
                   (cx * cz) * b15;
    g[i] = (be[k] + bo[k]) - corr;
    g[i + 1] = (be[k] - bo[k]) - corr;
  }
}

template <class T>
__device__ inline bool all_finite(const T* v, int k) {
  T s = 0;
  for (int i = 0; i < k; ++i) s += v[i] * (T)0;
  return s == 0;  // NaN or Inf times 0 is NaN
}

}  // namespace dev
}  // namespace mplb
