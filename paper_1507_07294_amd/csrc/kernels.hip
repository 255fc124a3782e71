// HIP kernels (gfx950) of the time step of the 3D MRT lattice-Boltzmann
// phase-field model of Liang, Shi & Chai (arXiv:1507.07294).
//
// State between steps (pull scheme, two time levels): buffer `cur` holds the
// post-collision populations of the previous step at their source node; a node
// gathers f_i(x) = f*_i(x - c_i), or f*_opp(i)(x) when x - c_i lies beyond a
// wall (half-way bounce-back).  Arrays are structure-of-arrays, one array per
// population, `pitch` elements apart.
//
// One coupled step = three kernels:
//   k_phi   phi = sum_i f_i (Eq. 13)
//   k_mu    mu = 4 beta phi (phi^2 - 1) - k lap phi (Eqs. 2, 36)
//   k_step  grad phi, lap mu (Eqs. 35-36); u, p (Eqs. 29-30); forces (after
//           Eq. 28); d_t(phi u) (Eq. 34); D3Q7 and D3Q15 collisions in moment
//           space (Eqs. 15, 17-18, 20, 31-32) with the sparse structure of M
//           and Gamma written out; stores into buffer 1 - cur.
#include <cmath>

#include "common.h"
#include "launch.h"

namespace mplb {
namespace {

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
// both lattices list velocities in antipodal pairs (1,2), (3,4), ...
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// ---------------------------------------------------------------- storage
template <int P>
struct Lat {
  using T = typename Prec<P>::T;
  using S0 = typename Prec<P>::S0;
  using S = typename Prec<P>::S;
  __device__ static const S0* f0(const void* base) { return (const S0*)base; }
  __device__ static S0* f0(void* base) { return (S0*)base; }
  __device__ static const S* fi(const void* base, int pitch) { return (const S*)((const char*)base + (size_t)pitch * sizeof(S0)); }
  __device__ static S* fi(void* base, int pitch) { return (S*)((char*)base + (size_t)pitch * sizeof(S0)); }
  __device__ static T ldf(const void* base, int pitch, int i, int n) {
    return i == 0 ? (T)f0(base)[n] : (T)fi(base, pitch)[(size_t)(i - 1) * pitch + n];
  }
  __device__ static void stf(void* base, int pitch, int i, int n, T v) {
    if (i == 0) f0(base)[n] = (S0)v;
    else fi(base, pitch)[(size_t)(i - 1) * pitch + n] = (S)v;
  }
  __device__ static T ldg(const void* base, int pitch, int i, int n) { return (T)((const S*)base)[(size_t)i * pitch + n]; }
  __device__ static void stg(void* base, int pitch, int i, int n, T v) { ((S*)base)[(size_t)i * pitch + n] = (S)v; }
};

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

template <int P>
__device__ inline void pull_f(const Geo& G, const void* fb, int x, int y, int z, int n, typename Prec<P>::T f[7]) {
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    int s = (i == 0) ? n : pull_src(G, x, y, z, c7(i, 0), c7(i, 1), c7(i, 2));
    f[i] = (s >= 0) ? Lat<P>::ldf(fb, G.pitch, i, s) : Lat<P>::ldf(fb, G.pitch, opp(i), n);
  }
}

template <int P>
__device__ inline void pull_g(const Geo& G, const void* gb, int x, int y, int z, int n, typename Prec<P>::T g[15]) {
#pragma unroll
  for (int i = 0; i < 15; ++i) {
    int s = (i == 0) ? n : pull_src(G, x, y, z, c15(i, 0), c15(i, 1), c15(i, 2));
    g[i] = (s >= 0) ? Lat<P>::ldg(gb, G.pitch, i, s) : Lat<P>::ldg(gb, G.pitch, opp(i), n);
  }
}

template <class T>
__device__ inline T phi_of(const T f[7]) {
  return f[0] + (((f[1] + f[2]) + (f[3] + f[4])) + (f[5] + f[6]));
}

// Eq. 35 (gradient) and Eq. 36 (Laplacian) with D3Q15 weights, c_s^2 = 1/3:
// face neighbours weigh 1/3 (gradient) and 2/3 (Laplacian), corners 1/24 and 1/12.
template <class T>
__device__ inline void grad_lap(const Geo& G, const T* chi, int x, int y, int z, T c0, T gr[3], T& lap,
                                bool want_grad) {
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
// cos(pi t / T), the cosine passed in as C.vel_ct).
template <class T>
__device__ inline void presc_u(const Geo& G, const Coef<T>& C, const T* uf, int x, int y, int z, int n, T u[3]) {
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
    T U = C.velU, ct = C.vel_ct;
    u[0] = 2 * U * sx * sx * s2y * s2z * ct;
    u[1] = -U * s2x * sy * sy * s2z * ct;
    u[2] = -U * s2x * s2y * sz * sz * ct;
  }
}

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
  T denom = m.rho - (T)0.25 * C.drho * ml;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m.gr[a] = half_dr * gphi[a];
    Fs[a] = mu * gphi[a];
    Gb[a] = (m.rho - C.rho_ref) * C.grav[a];
    m.u[a] = (j[a] + (T)0.5 * (Fs[a] + Gb[a])) / denom;
    m.F[a] = Fs[a] + half_dr * ml * m.u[a] + Gb[a];
  }
  T uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
  T ugr = m.u[0] * m.gr[0] + m.u[1] * m.gr[1] + m.u[2] * m.gr[2];
  // c_s^2 / (1 - w_0) = 3/7 and rho s_0(u) = -rho |u|^2 / 3 (Eq. 30)
  m.p = (T)(3.0 / 7.0) * (sum_nz + (T)0.5 * ugr - m.rho * uu / 3);
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

// D3Q15 collision in moment space (Eqs. 20, 27, 31, 32): m = Gamma g;
// m* = m - S^g (m - m^eq) + (I - S^g/2) mT; g* = Gamma^-1 m*.  Gamma's rows are
// d'Humieres' basis on the Eq. 23 velocity order.
template <class T>
__device__ inline void collide_ns(const Coef<T>& C, T g[15], const Macro<T>& M) {
  // face and corner combinations (corner pairs (7,8) (9,10) (11,12) (13,14) are antipodal)
  T sx = g[1] + g[2], sy = g[3] + g[4], sz = g[5] + g[6];
  T dx = g[1] - g[2], dy = g[3] - g[4], dz = g[5] - g[6];
  T p1 = g[7] + g[8], p2 = g[9] + g[10], p3 = g[11] + g[12], p4 = g[13] + g[14];
  T d1 = g[7] - g[8], d2 = g[9] - g[10], d3 = g[11] - g[12], d4 = g[13] - g[14];
  T Sf = (sx + sy) + sz, Sc = (p1 + p2) + (p3 + p4);
  T Xc = (d1 + d2) + (d3 + d4), Yc = (d1 + d2) - (d3 + d4), Zc = (d1 - d2) + (d3 - d4);
  T m[15];
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
  eq[4] = -7 * rho * u[0] / 3;
  eq[5] = rho * u[1];
  eq[6] = -7 * rho * u[1] / 3;
  eq[7] = rho * u[2];
  eq[8] = -7 * rho * u[2] / 3;
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
  src[4] = -7 * F[0] / 3;
  src[5] = F[1];
  src[6] = -7 * F[1] / 3;
  src[7] = F[2];
  src[8] = -7 * F[2] / 3;
  src[9] = 4 * u[0] * a[0] - 2 * u[1] * a[1] - 2 * u[2] * a[2];
  src[10] = 2 * u[1] * a[1] - 2 * u[2] * a[2];
  src[11] = u[0] * a[1] + u[1] * a[0];
  src[12] = u[1] * a[2] + u[2] * a[1];
  src[13] = u[0] * a[2] + u[2] * a[0];
  src[14] = 0;
  T ms[15];
#pragma unroll
  for (int r = 0; r < 15; ++r) ms[r] = m[r] - C.lg[r] * (m[r] - eq[r]) + (1 - C.lg[r] / 2) * src[r];
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

// ------------------------------------------------------------------ kernels
constexpr int kBlock = 256;

template <int P>
__global__ void __launch_bounds__(kBlock) k_phi(Geo G, Bufs B, int cur) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  int x, y, z;
  decode(G, n, x, y, z);
  T f[7];
  pull_f<P>(G, B.f[cur], x, y, z, n, f);
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
  grad_lap(G, phi, x, y, z, c0, gr, lap, false);
  ((T*)B.mu)[n] = 4 * C.beta * c0 * (c0 - 1) * (c0 + 1) - C.kappa * lap;
}

template <class T>
__device__ inline bool all_finite(const T* v, int k) {
  T s = 0;
  for (int i = 0; i < k; ++i) s += v[i] * (T)0;
  return s == 0;  // NaN or Inf times 0 is NaN
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_step(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  int x, y, z;
  decode(G, n, x, y, z);
  T f[7], g[15];
  pull_f<P>(G, B.f[cur], x, y, z, n, f);
  pull_g<P>(G, B.g[cur], x, y, z, n, g);
  T phi = phi_of(f);
  const T* phis = (const T*)B.phi;
  const T* mus = (const T*)B.mu;
  T mu = mus[n], gphi[3], lapphi, gdummy[3], lapmu;
  grad_lap(G, phis, x, y, z, phi, gphi, lapphi, true);
  grad_lap(G, mus, x, y, z, mu, gdummy, lapmu, false);
  Macro<T> M;
  flow_macro(C, g, phi, mu, gphi, lapmu, M);
  T* hist = (T*)B.phiu;
  T dphiu[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T pu = phi * M.u[a];
    dphiu[a] = pu - hist[(size_t)a * G.pitch + n];
    hist[(size_t)a * G.pitch + n] = pu;
  }
  collide_che(C, f, phi, mu, M.u, dphiu);
  collide_ns(C, g, M);
  void* fo = B.f[1 - cur];
  void* go = B.g[1 - cur];
#pragma unroll
  for (int i = 0; i < 7; ++i) Lat<P>::stf(fo, G.pitch, i, n, f[i]);
#pragma unroll
  for (int i = 0; i < 15; ++i) Lat<P>::stg(go, G.pitch, i, n, g[i]);
  if (!(all_finite(f, 7) && all_finite(g, 15))) *B.flag = 1;
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_step_che(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  int x, y, z;
  decode(G, n, x, y, z);
  T f[7];
  pull_f<P>(G, B.f[cur], x, y, z, n, f);
  T phi = phi_of(f);
  T gr[3], lap;
  grad_lap(G, (const T*)B.phi, x, y, z, phi, gr, lap, false);
  T mu = 4 * C.beta * phi * (phi - 1) * (phi + 1) - C.kappa * lap;
  T u[3];
  presc_u(G, C, (const T*)B.ufield, x, y, z, n, u);
  T* hist = (T*)B.phiu;
  T dphiu[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T pu = phi * u[a];
    dphiu[a] = pu - hist[(size_t)a * G.pitch + n];
    hist[(size_t)a * G.pitch + n] = pu;
  }
  collide_che(C, f, phi, mu, u, dphiu);
  void* fo = B.f[1 - cur];
#pragma unroll
  for (int i = 0; i < 7; ++i) Lat<P>::stf(fo, G.pitch, i, n, f[i]);
  if (!all_finite(f, 7)) *B.flag = 1;
}

// Macroscopic state of node n at the current level (phi and mu arrays must
// hold this level).  Returns false if a pulled population is non-finite.
template <int P, bool COUPLED>
__device__ inline bool node_macro(const Geo& G, const Coef<typename Prec<P>::T>& C, const Bufs& B, int cur, int n,
                                  Macro<typename Prec<P>::T>& M) {
  using T = typename Prec<P>::T;
  int x, y, z;
  decode(G, n, x, y, z);
  T f[7];
  pull_f<P>(G, B.f[cur], x, y, z, n, f);
  T phi = phi_of(f);
  bool ok = all_finite(f, 7);
  if (COUPLED) {
    T g[15];
    pull_g<P>(G, B.g[cur], x, y, z, n, g);
    ok = ok && all_finite(g, 15);
    const T* mus = (const T*)B.mu;
    T mu = mus[n], gphi[3], lapphi, gd[3], lapmu;
    grad_lap(G, (const T*)B.phi, x, y, z, phi, gphi, lapphi, true);
    grad_lap(G, mus, x, y, z, mu, gd, lapmu, false);
    flow_macro(C, g, phi, mu, gphi, lapmu, M);
  } else {
    T gr[3], lap;
    grad_lap(G, (const T*)B.phi, x, y, z, phi, gr, lap, false);
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

template <int P, bool COUPLED>
__global__ void __launch_bounds__(kBlock) k_macro(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur, int field) {
  using T = typename Prec<P>::T;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= G.N) return;
  Macro<T> M;
  node_macro<P, COUPLED>(G, C, B, cur, n, M);
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
template <int P, bool COUPLED>
__global__ void __launch_bounds__(kBlock) k_totals(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur) {
  using T = typename Prec<P>::T;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int n = blockIdx.x * kBlock + threadIdx.x; n < G.N; n += gridDim.x * kBlock) {
    Macro<T> M;
    bool ok = node_macro<P, COUPLED>(G, C, B, cur, n, M);
    acc[0] += (double)M.phi;
    if (COUPLED) {
      int x, y, z;
      decode(G, n, x, y, z);
      T g[15];
      pull_g<P>(G, B.g[cur], x, y, z, n, g);
      double gd[15];
      for (int i = 0; i < 15; ++i) gd[i] = (double)g[i];
      for (int i = 0; i < 15; ++i) {
        acc[1] += c15(i, 0) * gd[i];
        acc[2] += c15(i, 1) * gd[i];
        acc[3] += c15(i, 2) * gd[i];
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

template <class T>
__global__ void __launch_bounds__(kBlock) k_cvt_in(const double* src, T* dst, int N) {
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n < N) dst[n] = (T)src[n];
}

// Equilibrium populations at every node (Eqs. 5, 21-22 with p = 0), written
// to the storage slot each node will pull them from, so that the first step
// sees f = f^eq and g = g^eq at every node.
template <int P, bool COUPLED>
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
    if (s >= 0) Lat<P>::stf(B.f[cur], G.pitch, i, s, feq[i]);
    else Lat<P>::stf(B.f[cur], G.pitch, opp(i), n, feq[i]);
  }
  if (COUPLED) {
    T rho = (1 + phi) / 2 * C.rho_l + (1 - phi) / 2 * C.rho_g;
    T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < 15; ++i) {
      T w = (i == 0) ? (T)(2.0 / 9.0) : (i < 7 ? (T)(1.0 / 9.0) : (T)(1.0 / 72.0));
      T cu = c15(i, 0) * u[0] + c15(i, 1) * u[1] + c15(i, 2) * u[2];
      T geq = rho * w * (3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);  // Eq. 21 with p = 0
      int s = (i == 0) ? n : pull_src(G, x, y, z, c15(i, 0), c15(i, 1), c15(i, 2));
      if (s >= 0) Lat<P>::stg(B.g[cur], G.pitch, i, s, geq);
      else Lat<P>::stg(B.g[cur], G.pitch, opp(i), n, geq);
    }
  }
  for (int a = 0; a < 3; ++a) hist[(size_t)a * G.pitch + n] = phi * u[a];
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

template <int P>
__global__ void k_poke(Geo G, Bufs B, int cur, int set, int i, int n, double v) {
  using T = typename Prec<P>::T;
  if (set == 0) Lat<P>::stf(B.f[cur], G.pitch, i, n, (T)v);
  else Lat<P>::stg(B.g[cur], G.pitch, i, n, (T)v);
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
  o.vel_kind = c.vel_kind; o.velU = (T)c.velU; o.vel_ct = (T)c.vel_ct;
  return o;
}

inline dim3 grid_for(int N) { return dim3((unsigned)((N + kBlock - 1) / kBlock)); }

template <int P>
hipError_t step_impl(int mode, const Geo& G, const Coef<double>& Cd, const Bufs& B, int cur, hipStream_t s) {
  using T = typename Prec<P>::T;
  Coef<T> C = cast_coef<T>(Cd);
  if (mode == MPLB_COUPLED) hipLaunchKernelGGL(k_step<P>, grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur);
  else hipLaunchKernelGGL(k_step_che<P>, grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur);
  return hipGetLastError();
}

template <int P>
hipError_t macro_impl(int mode, const Geo& G, const Coef<double>& Cd, const Bufs& B, int cur, int field, hipStream_t s) {
  using T = typename Prec<P>::T;
  Coef<T> C = cast_coef<T>(Cd);
  if (mode == MPLB_COUPLED) hipLaunchKernelGGL((k_macro<P, true>), grid_for(G.N), dim3(kBlock), 0, s, G, C, B, cur, field);
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

hipError_t launch_phi(int P, const Geo& G, const Bufs& B, int cur, hipStream_t s) {
  MPLB_DISPATCH(P, {
    hipLaunchKernelGGL(k_phi<PP>, grid_for(G.N), dim3(kBlock), 0, s, G, B, cur);
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

hipError_t launch_step(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur, hipStream_t s) {
  MPLB_DISPATCH(P, return step_impl<PP>(mode, G, C, B, cur, s))
}

hipError_t launch_macro(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur, int field,
                        hipStream_t s) {
  MPLB_DISPATCH(P, return macro_impl<PP>(mode, G, C, B, cur, field, s))
}

hipError_t launch_totals(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur, hipStream_t s) {
  MPLB_DISPATCH(P, return totals_impl<PP>(mode, G, C, B, cur, s))
}

hipError_t launch_cvt_in(int P, const Geo& G, const Bufs& B, void* dst, hipStream_t s) {
  if (P == MPLB_F64) hipLaunchKernelGGL(k_cvt_in<double>, grid_for(G.N), dim3(kBlock), 0, s, B.out, (double*)dst, G.N);
  else hipLaunchKernelGGL(k_cvt_in<float>, grid_for(G.N), dim3(kBlock), 0, s, B.out, (float*)dst, G.N);
  return hipGetLastError();
}

hipError_t launch_init(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur, hipStream_t s) {
  MPLB_DISPATCH(P, return init_impl<PP>(mode, G, C, B, cur, s))
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

hipError_t launch_poke(int P, const Geo& G, const Bufs& B, int cur, int set, int i, int n, double v, hipStream_t s) {
  MPLB_DISPATCH(P, {
    hipLaunchKernelGGL(k_poke<PP>, dim3(1), dim3(1), 0, s, G, B, cur, set, i, n, v);
    return hipGetLastError();
  })
}

}  // namespace mplb
