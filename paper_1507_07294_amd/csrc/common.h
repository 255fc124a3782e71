// Internal types shared by the kernels and the host side of libmplb.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mplb.h"

namespace mplb {

// Lattice geometry.  wall[a] != 0: axis a is bounded by no-slip walls.
struct Geo {
  int nx, ny, nz;
  int wall_x, wall_y, wall_z;
  int N;     // nx*ny*nz (< 2^31)
  int pitch; // elements between consecutive population arrays (N rounded up to 256)
};

// Per-lattice coefficients in the compute type (derived on the host).
template <class T>
struct Coef {
  T rho_l, rho_g, drho;   // Eq. 14; drho = rho_l - rho_g (rho_A - rho_B)
  T beta, kappa;          // after Eq. 2
  T eta, A;               // Eqs. 5, 8, 19
  T mob;                  // mobility M
  T rho_ref, grav[3];     // body force
  T sf[7];                // S^f
  T lg[15];               // S^g (lambda_9..13 from nu)
  int vel_kind;           // CHE-only prescribed velocity kind
  T velU;
  T vel_ct;               // cos(pi t / T) of the current step (deformation flow)
  T vel_ct_prev;          // the same at the previous level (step 0: the current one)
  int stencil7;           // Eqs. 35-36 on the D3Q7 weights instead of D3Q15
  int forcing28;          // Gamma T of Eq. 28 instead of the printed Eq. 32 (D3Q15)
  int unit_rates;         // S^g = 1 off the stress moments 9..13 (the paper's choice)
  int poison;             // test hook: the step kernels first fill their LDS with NaN bit patterns
};

// Compute type T, storage of f_0 (S0) and of f_1..f_6 and g (S).
template <int P> struct Prec;
template <> struct Prec<MPLB_F64> { using T = double; using S0 = double; using S = double; };
template <> struct Prec<MPLB_F32> { using T = float; using S0 = float; using S = float; };
template <> struct Prec<MPLB_F32_F16> { using T = float; using S0 = float; using S = _Float16; };
template <> struct Prec<MPLB_F32_BF16> { using T = float; using S0 = float; using S = __bf16; };

// Device pointers of one lattice.  f: f_0 array (S0) followed by f_1..f_6
// arrays (S), each `pitch` elements; g: 15 arrays of S.
struct Bufs {
  void* f[2];
  void* g[2];
  void* phiu;   // T: (phi u) of the previous level, 3 x pitch (coupled);
                //    phi of the previous level, 1 x pitch (CHE-only: u is prescribed)
  void* phi;    // pitch, T
  void* mu;     // pitch, T
  void* ufield; // 3 x pitch, T (CHE-only, prescribed field)
  double* out;  // pitch doubles: read-out / upload staging
  double* red;  // reduction partials (kRedSlots x 8) + final (8)
  int* flag;    // non-finite flag
};

constexpr int kRedSlots = 2048;

// Work split of the z-marching step: tiles of 64 x TY columns, z segments
// of lz planes.
struct Tiling {
  int tiles_x, tiles_y, lz, nseg;
};

// Kernel and work split of one step (launch_shape): the coupled step on
// 64 x 8 or 64 x 16 tiles, the CHE-only step with one node per thread (64 x 8)
// or two (128 x 8).
enum ShapeKind { kShapeCoupled8 = 0, kShapeCoupled16 = 1, kShapeChe1 = 2, kShapeChe2 = 3 };
struct Shape {
  int kind, tile_w, tile_h;
  Tiling tl;
};

// One lattice of a batched step: its geometry, coefficients, buffers, work
// split, buffer parity and first block in the batch grid.
template <class T>
struct BatchItem {
  Geo G;
  Tiling TL;
  Bufs B;
  Coef<T> C;
  int cur0, block0, nblocks, pad;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace mplb
