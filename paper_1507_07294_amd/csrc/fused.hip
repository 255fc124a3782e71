// One-kernel time step of the 3D MRT phase-field lattice-Boltzmann model
// (coupled D3Q7 + D3Q15, and the CHE-only D3Q7 variant), z-marching with
// LDS rings.
//
// A block owns a 64 x TY column of nodes (TY = 16 for the coupled step with
// FP32 populations on a lattice of at least 512 such blocks, else 8) and
// marches along z through a segment [z0, z1).
// At plane z it
//   (a) issues the pulls of the seven f populations of plane z+3 on the tile
//       plus a halo of two nodes,
//   (b) while they are in flight, evaluates mu (Eqs. 2, 36) of plane z+1 on
//       the tile plus a halo of one into an LDS ring of 4 planes, then sums
//       the pulled f into phi (Eq. 13) in an LDS ring of 6 planes,
//   (c) after the one barrier of the plane, finishes the nodes of plane z:
//       grad phi and lap mu (Eqs. 35-36) from LDS, pulls g, forms u, p and
//       the forces (Eqs. 29-30), d_t(phi u) (Eq. 34), collides both lattices
//       in moment space and stores f*, g* and (phi u).
// The rings are deep enough that threads one barrier apart never touch the
// same slot.  (The D3Q19 variant pulls plane z+2 instead and puts a second
// barrier between (a) and (b).)  Each stored population is pulled from HBM once, by the tile
// that owns its destination: the tile's own f, pulled in (a), wait three
// planes in an LDS queue (thread-private slots) for (c).  Only the halo
// pulls of (a) re-read data, which blocks running together on one XCD share
// through its L2 (the block order is remapped so that each XCD gets a
// contiguous run of tiles).
//
// Index arithmetic is hoisted out of the z loop: a thread's x and y source
// offsets (with periodic wrap) are fixed for the whole march, and the plane
// offsets and the bounce-back decisions of a z wall are uniform over the
// block.  Walls on the x or y axis are handled by a separate instantiation.
//
// Finite-difference ghosts: phi beyond a wall is the mirror phi(-1) = phi(0);
// mu at a ghost position is evaluated at its mirror image, so mu(-1) = mu(0).
#include <atomic>
#include <type_traits>

#include "common.h"
#include "device.h"
#include "launch.h"

namespace mplb {
namespace {

using namespace dev;

constexpr int kTX = 64;

// Block -> logical tile with a contiguous run of tiles per XCD (workgroups
// are dispatched round-robin over the 8 XCDs).
__device__ inline int logical_block(int b, int nb) {
  const int X = 8;
  int per = nb / X, rem = nb % X;
  int xcd = b % X, k = b / X;
  return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

// periodic wrap, or clamp onto the wall layer (mirror ghost of phi)
__device__ inline int map_axis(int v, int n, int wall) {
  if (wall) return v < 0 ? 0 : (v >= n ? n - 1 : v);
  v %= n;
  return v < 0 ? v + n : v;
}
__device__ inline int clamp_axis(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }
__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Source offsets of one lattice column (x, y): for a velocity component c in
// {-1, 0, 1}, xs[c+1] is the source x (x - c, wrapped) and xb[c+1] says the
// population comes through an x wall; ys holds y * nx likewise.
struct Column {
  int xs[3], ys[3];
  bool xb[3], yb[3];
};

template <bool XYWALL>
__device__ inline Column make_column(const Geo& G, int x, int y) {
  Column c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int sx = x - (k - 1), sy = y - (k - 1);
    c.xb[k] = XYWALL && G.wall_x && (sx < 0 || sx >= G.nx);
    c.yb[k] = XYWALL && G.wall_y && (sy < 0 || sy >= G.ny);
    c.xs[k] = wrap1(sx, G.nx);
    c.ys[k] = wrap1(sy, G.ny) * G.nx;
  }
  return c;
}

// Plane offsets for the sources of plane z (z - cz) and the z-wall bounce,
// uniform over the block.
struct Plane {
  int zs[3];
  bool zb[3];
  int z;
};

__device__ inline Plane make_plane(const Geo& G, int z) {
  Plane p;
  p.z = z;
  const int nxy = G.nx * G.ny;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int sz = z - (k - 1);
    p.zb[k] = G.wall_z && (sz < 0 || sz >= G.nz);
    p.zs[k] = wrap1(sz, G.nz) * nxy;
  }
  return p;
}

// Pulls into node (column c, plane p).  The bounce-back choice selects an
// array and an index and then issues one load, so that no load sits behind a
// branch and all of them are in flight together; with walls on z only the
// array choice is uniform over the block.
template <bool XYWALL>
__device__ inline bool bounced(const Column& c, const Plane& p, int cx, int cy, int cz) {
  bool b = p.zb[cz + 1];
  if (XYWALL) b = b || c.xb[cx + 1] || c.yb[cy + 1];
  return b;
}
__device__ inline int source(const Column& c, const Plane& p, int cx, int cy, int cz) {
  return p.zs[cz + 1] + c.ys[cy + 1] + c.xs[cx + 1];
}

// Plane-relative addressing.  Every pull of a node reads one z plane per
// velocity, and which plane (and, on a z wall, which array) is uniform over
// the block; so a load is a raw buffer access whose resource holds a scalar
// base (array start plus plane offset, 64-bit scalar arithmetic) and whose
// lane offset is the 32-bit in-plane byte offset: one vector instruction of
// address arithmetic per access.  The in-plane byte offset holds while
// nx*ny*8 < 2^32 (checked when a lattice is created).  The base must be
// uniform over the wave.
template <class S>
__device__ inline const S* plane_base(const void* arr0, size_t arr, int pitch, int zoff) {
  return (const S*)arr0 + (arr * (size_t)pitch + (size_t)zoff);
}
__device__ inline __amdgpu_buffer_rsrc_t rsrc_at(const void* base) {
  // no stride, full 32-bit range, untyped 32-bit data (gfx9 descriptor word 3)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}
// NTL: non-temporal load (cache-policy bit 1), for data that no other block
// reads again.
template <class S, bool NTL = false>
__device__ inline S ld_at(const S* base, int xy) {
  const uint32_t off = (uint32_t)xy * (uint32_t)sizeof(S);
  constexpr int aux = NTL ? 2 : 0;
  if constexpr (sizeof(S) == 2) {
    return __builtin_bit_cast(S, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(rsrc_at(base), off, 0, aux));
  } else if constexpr (sizeof(S) == 4) {
    return __builtin_bit_cast(S, (unsigned int)__builtin_amdgcn_raw_buffer_load_b32(rsrc_at(base), off, 0, aux));
  } else {
    static_assert(sizeof(S) == 8, "2, 4 or 8 bytes");
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(rsrc_at(base), off, 0, aux));
  }
}
// NT: non-temporal (streaming) store, cache-policy bit 1.  It pays when a
// step's traffic is far larger than the last-level cache; for a lattice that
// stays resident there it makes the next step's reads go to HBM.
template <bool NT, class S>
__device__ inline void st_at(S* base, int xy, S v) {
  const uint32_t off = (uint32_t)xy * (uint32_t)sizeof(S);
  constexpr int aux = NT ? 2 : 0;
  if constexpr (sizeof(S) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), rsrc_at(base), off, 0, aux);
  } else if constexpr (sizeof(S) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rsrc_at(base), off, 0, aux);
  } else {
    using U2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), rsrc_at(base), off, 0, aux);
  }
}

// The seven f of the node at in-plane index xy of the plane p (plane offset
// zo), as stored: f_0 in r0, f_1..f_6 in r (PACK: 32-bit words that carry
// g_1..g_6 in their high halves).
template <int P, bool PACK>
struct F7Raw {
  using L = Lat<P, PACK>;
  using QS = typename std::conditional<PACK, uint32_t, typename L::S>::type;
  typename L::S0 r0;
  QS r[6];
};

template <int P, bool PACK, bool XYWALL>
__device__ inline void pull_f7_raw(const Geo& G, const void* fb, const Column& c, const Plane& p, int zo, int xy,
                                   F7Raw<P, PACK>& o) {
  using L = Lat<P, PACK>;
  using QS = typename F7Raw<P, PACK>::QS;
  o.r0 = ld_at(L::f0(fb) + zo, xy);
  const QS* fi = (const QS*)L::fi(fb, G.pitch);
#pragma unroll
  for (int i = 1; i < 7; ++i) {
    const int cx = c7(i, 0), cy = c7(i, 1), cz = c7(i, 2);
    if constexpr (XYWALL) {
      const bool b = bounced<XYWALL>(c, p, cx, cy, cz);
      const int idx = b ? zo + xy : source(c, p, cx, cy, cz);
      o.r[i - 1] = fi[(size_t)((b ? opp(i) : i) - 1) * G.pitch + idx];
    } else {
      // z-wall bounce is uniform: pick array and plane on the scalar side
      const bool b = p.zb[cz + 1];
      const QS* base = plane_base<QS>(fi, (size_t)((b ? opp(i) : i) - 1), G.pitch, b ? zo : p.zs[cz + 1]);
      o.r[i - 1] = ld_at(base, b ? xy : c.ys[cy + 1] + c.xs[cx + 1]);
    }
  }
}

template <int P, bool PACK>
__device__ inline void cvt_f7(const F7Raw<P, PACK>& o, typename Prec<P>::T f[7]) {
  using L = Lat<P, PACK>;
  using T = typename Prec<P>::T;
  f[0] = (T)o.r0;
#pragma unroll
  for (int i = 1; i < 7; ++i) {
    if constexpr (PACK) f[i] = L::lo(o.r[i - 1]);
    else f[i] = (T)o.r[i - 1];
  }
}

// Raw pulls of the g (storage type, no conversion), issued ahead of the
// stage that uses them.
template <int P, bool PACK, bool XYWALL, int Q>
__device__ inline void pull_gq_raw(const Geo& G, const void* gb, const Column& c, const Plane& p, int zo, int xy,
                                   typename Lat<P, PACK>::S raw[Q]) {
  using L = Lat<P, PACK>;
  using S = typename L::S;
  const S* arr = (const S*)gb;
  raw[0] = ld_at(arr + zo, xy);
#pragma unroll
  for (int i = PACK ? 7 : 1; i < Q; ++i) {
    const int cx = cq<Q>(i, 0), cy = cq<Q>(i, 1), cz = cq<Q>(i, 2);
    if constexpr (XYWALL) {
      const bool b = bounced<XYWALL>(c, p, cx, cy, cz);
      const int idx = b ? zo + xy : source(c, p, cx, cy, cz);
      raw[i] = arr[L::gslot(b ? opp(i) : i) * G.pitch + idx];
    } else {
      const bool b = p.zb[cz + 1];
      const S* base = plane_base<S>(arr, L::gslot(b ? opp(i) : i), G.pitch, b ? zo : p.zs[cz + 1]);
      raw[i] = ld_at(base, b ? xy : c.ys[cy + 1] + c.xs[cx + 1]);
    }
  }
}

// The Q g of the NSE lattice (PACK, D3Q15 only: g_0 and the corners g_7..g_14).
template <int P, bool PACK, bool XYWALL, int Q>
__device__ inline void pull_gq(const Geo& G, const void* gb, const Column& c, const Plane& p, int zo, int xy,
                               typename Prec<P>::T g[Q]) {
  using L = Lat<P, PACK>;
  using T = typename Prec<P>::T;
  using S = typename L::S;
  const S* arr = (const S*)gb;
  S raw[Q];
  raw[0] = ld_at(arr + zo, xy);
#pragma unroll
  for (int i = PACK ? 7 : 1; i < Q; ++i) {
    const int cx = cq<Q>(i, 0), cy = cq<Q>(i, 1), cz = cq<Q>(i, 2);
    if constexpr (XYWALL) {
      const bool b = bounced<XYWALL>(c, p, cx, cy, cz);
      const int idx = b ? zo + xy : source(c, p, cx, cy, cz);
      raw[i] = arr[L::gslot(b ? opp(i) : i) * G.pitch + idx];
    } else {
      const bool b = p.zb[cz + 1];
      const S* base = plane_base<S>(arr, L::gslot(b ? opp(i) : i), G.pitch, b ? zo : p.zs[cz + 1]);
      raw[i] = ld_at(base, b ? xy : c.ys[cy + 1] + c.xs[cx + 1]);
    }
  }
  // Issue every load before the first value is used: under register
  // pressure the scheduler otherwise reuses one register per load and waits
  // for each in turn (measured: 16-bit storage 2.8 -> 2.1 ms per step at
  // 256 x 256 x 1024).
  __builtin_amdgcn_sched_barrier(0);
  g[0] = (T)raw[0];
#pragma unroll
  for (int i = PACK ? 7 : 1; i < Q; ++i) g[i] = (T)raw[i];
}

// Eq. 36 at a ring position c of the middle plane pc, with the planes below
// (pm) and above (pp); 2/3 per face and 1/12 per corner (s7: the D3Q7
// weights, 1 per face).
template <class T, int PX>
__device__ inline T lap_lds(const T* pm, const T* pc, const T* pp, int c, bool s7 = false) {
  T c0 = pc[c];
  if (s7)
    return (((pc[c + 1] - c0) + (pc[c - 1] - c0)) + ((pc[c + PX] - c0) + (pc[c - PX] - c0))) +
           ((pp[c] - c0) + (pm[c] - c0));
  T lf = ((pc[c - 1] - c0) + (pc[c + 1] - c0)) + ((pc[c - PX] - c0) + (pc[c + PX] - c0)) + ((pm[c] - c0) + (pp[c] - c0));
  T lc = ((pm[c - PX - 1] - c0) + (pm[c - PX + 1] - c0)) + ((pm[c + PX - 1] - c0) + (pm[c + PX + 1] - c0)) +
         ((pp[c - PX - 1] - c0) + (pp[c - PX + 1] - c0)) + ((pp[c + PX - 1] - c0) + (pp[c + PX + 1] - c0));
  return (T)(2.0 / 3.0) * lf + (T)(1.0 / 12.0) * lc;
}

// Eq. 35: face neighbours weigh 1/3, corners 1/24 (s7: central differences).
template <class T, int PX>
__device__ inline void grad_lds(const T* pm, const T* pc, const T* pp, int c, T gr[3], bool s7 = false) {
  if (s7) {
    gr[0] = (T)0.5 * (pc[c + 1] - pc[c - 1]);
    gr[1] = (T)0.5 * (pc[c + PX] - pc[c - PX]);
    gr[2] = (T)0.5 * (pp[c] - pm[c]);
    return;
  }
  T a = pm[c + PX + 1], b = pm[c + PX - 1], d = pm[c - PX + 1], e = pm[c - PX - 1];
  T A = pp[c + PX + 1], Bv = pp[c + PX - 1], D = pp[c - PX + 1], E = pp[c - PX - 1];
  T cx = ((a - b) + (d - e)) + ((A - Bv) + (D - E));
  T cy = ((a - d) + (b - e)) + ((A - D) + (Bv - E));
  T cz = ((A - a) + (Bv - b)) + ((D - d) + (E - e));
  gr[0] = (T)(1.0 / 3.0) * (pc[c + 1] - pc[c - 1]) + (T)(1.0 / 24.0) * cx;
  gr[1] = (T)(1.0 / 3.0) * (pc[c + PX] - pc[c - PX]) + (T)(1.0 / 24.0) * cy;
  gr[2] = (T)(1.0 / 3.0) * (pp[c] - pm[c]) + (T)(1.0 / 24.0) * cz;
}

// Test hook (Coef::poison): fill shared memory with all-ones words, NaN in
// every storage type, so that a read of a slot no stage has written shows in
// the results.  Callers follow it with a barrier.
__device__ inline void poison_shared(void* p, int bytes) {
  uint32_t* w = (uint32_t*)p;
  for (int i = threadIdx.x; i < bytes / 4; i += blockDim.x) w[i] = 0xffffffffu;
}

template <int P, int TY, int HALO>
struct Ring {
  static constexpr int NT = kTX * TY;
  static constexpr int PX = kTX + 2 * HALO, PY = TY + 2 * HALO;
  static constexpr int NPHI = PX * PY;
  static constexpr int NHALO = NPHI - NT;
  static constexpr int HPT = (NHALO + NT - 1) / NT;  // halo positions per thread
};

// Halo position h of a (PX x PY) padded tile with a halo of H: H rows on each
// side in y, then H columns on each side in x for the interior rows.
template <int PX, int PY, int H>
__device__ inline void halo_pos(int h, int& px, int& py) {
  if (h < H * PX) { py = h / PX; px = h % PX; return; }
  h -= H * PX;
  if (h < H * PX) { py = PY - H + h / PX; px = h % PX; return; }
  h -= H * PX;
  py = H + h / (2 * H);
  int c = h % (2 * H);
  px = c < H ? c : PX - 2 * H + c;
}

// Per-thread phi-load positions: the own tile node plus up to HPT halo nodes,
// each as an LDS slot and the source columns of its seven f pulls.
template <int P, int TY, int HALO, bool XYWALL, bool PACK>
struct PhiLoader {
  using R = Ring<P, TY, HALO>;
  using T = typename Prec<P>::T;
  // queue entry of the own node: the seven f (PACK: f_0's bits and the six raw words)
  using QT = typename std::conditional<PACK, uint32_t, T>::type;
  Column own;
  int own_lds;
  Column halo[R::HPT];
  int halo_lds[R::HPT];
  bool halo_on[R::HPT];
  int own_xy, halo_xy[R::HPT];  // x + nx*y of the (mapped) node

  __device__ void init(const Geo& G, int x0, int y0) {
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    int mx = map_axis(x0 + tx, G.nx, G.wall_x), my = map_axis(y0 + ty, G.ny, G.wall_y);
    own = make_column<XYWALL>(G, mx, my);
    own_xy = mx + G.nx * my;
    own_lds = (ty + HALO) * R::PX + tx + HALO;
#pragma unroll
    for (int k = 0; k < R::HPT; ++k) {
      int h = threadIdx.x + k * R::NT;
      halo_on[k] = h < R::NHALO;
      int px = 0, py = 0;
      if (halo_on[k]) halo_pos<R::PX, R::PY, HALO>(h, px, py);
      int hx = map_axis(x0 - HALO + px, G.nx, G.wall_x), hy = map_axis(y0 - HALO + py, G.ny, G.wall_y);
      halo[k] = make_column<XYWALL>(G, hx, hy);
      halo_xy[k] = hx + G.nx * hy;
      halo_lds[k] = py * R::PX + px;
    }
  }

  // The pulls of logical plane zl (mapped onto the lattice), own node and
  // halo, issued together so that the wave waits for memory once per plane
  // (lanes without a halo position are masked off for the halo pulls).
  struct Pending {
    F7Raw<P, PACK> own, halo[R::HPT];
  };
  __device__ void issue(const Geo& G, const void* fin, int zl, Pending& pd) {
    int mz = map_axis(zl, G.nz, G.wall_z);
    Plane p = make_plane(G, mz);
    int zo = mz * G.nx * G.ny;
    pull_f7_raw<P, PACK, XYWALL>(G, fin, own, p, zo, own_xy, pd.own);
#pragma unroll
    for (int k = 0; k < R::HPT; ++k)
      if (halo_on[k]) pull_f7_raw<P, PACK, XYWALL>(G, fin, halo[k], p, zo, halo_xy[k], pd.halo[k]);
  }
  // phi of the pulled plane into ring slot s; the own node's populations go
  // to q[i * NT + thread] when q is given
  __device__ void finish(const Pending& pd, T* s, QT* q) {
    T f[7];
    cvt_f7<P, PACK>(pd.own, f);
    s[own_lds] = phi_of(f);
    if (q) {
      if constexpr (PACK) {
        q[threadIdx.x] = __builtin_bit_cast(uint32_t, (float)f[0]);
#pragma unroll
        for (int i = 1; i < 7; ++i) q[i * R::NT + threadIdx.x] = (QT)pd.own.r[i - 1];
      } else {
#pragma unroll
        for (int i = 0; i < 7; ++i) q[i * R::NT + threadIdx.x] = (QT)f[i];
      }
    }
#pragma unroll
    for (int k = 0; k < R::HPT; ++k) {
      if (halo_on[k]) {
        T fh[7];
        cvt_f7<P, PACK>(pd.halo[k], fh);
        s[halo_lds[k]] = phi_of(fh);
      }
    }
  }
  __device__ void load(const Geo& G, const void* fin, int zl, T* s, QT* q = nullptr) {
    Pending pd;
    issue(G, fin, zl, pd);
    __builtin_amdgcn_sched_barrier(0);
    finish(pd, s, q);
  }
};

// Per-thread mu positions on the tile + halo 1 (mirror images for walls).
template <int P, int TY>
struct MuMaker {
  using R2 = Ring<P, TY, 2>;
  static constexpr int QX = kTX + 2, QY = TY + 2, NMU = QX * QY;
  static constexpr int MPT = (NMU + R2::NT - 1) / R2::NT;
  int src[MPT];  // phi ring slot index of the position (or its mirror)
  bool on[MPT];

  __device__ void init(const Geo& G, int x0, int y0) {
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      int q = threadIdx.x + k * R2::NT;
      on[k] = q < NMU;
      int qx = q % QX, qy = q / QX;
      int gx = x0 - 1 + qx, gy = y0 - 1 + qy;
      if (G.wall_x) gx = clamp_axis(gx, G.nx);
      if (G.wall_y) gy = clamp_axis(gy, G.ny);
      src[k] = (gy - (y0 - 2)) * R2::PX + (gx - (x0 - 2));
    }
  }

  // mu of logical plane zl >= -1 into smu, from a phi ring of NR slots
  // (plane z in slot (z + 2 NR) % NR)
  template <int NR, bool S7 = false>
  __device__ void run(const Geo& G, const Coef<typename Prec<P>::T>& C, int zl,
                      typename Prec<P>::T (*sphi)[R2::NPHI], typename Prec<P>::T* smu) {
    using T = typename Prec<P>::T;
    int ze = G.wall_z ? clamp_axis(zl, G.nz) : zl;
    const T* pm = sphi[(ze - 1 + 2 * NR) % NR];
    const T* pc = sphi[(ze + 2 * NR) % NR];
    const T* pp = sphi[(ze + 1 + 2 * NR) % NR];
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      if (on[k]) {
        T c0 = pc[src[k]];
        T lap = lap_lds<T, R2::PX>(pm, pc, pp, src[k], S7);
        smu[threadIdx.x + k * R2::NT] = 4 * C.beta * c0 * (c0 - 1) * (c0 + 1) - C.kappa * lap;
      }
    }
  }
};

// at least 4 waves per SIMD for FP32 compute (<= 128 VGPRs), 2 for FP64
template <int P>
constexpr int waves_per_eu() { return P == MPLB_F64 ? 2 : 4; }

// Study variants of a step kernel, compile-time so that the default kernels
// carry no code for them: D3Q7 finite differences (Eqs. 35-36), and Gamma T
// of Eq. 28 in place of the printed Eq. 32.  Built for FP64 and FP32 storage.
constexpr int kVarS7 = 1, kVarF28 = 2;
// S^g = 1 off the stress moments (the host sets it from the rates; any
// precision): the D3Q15 collision forms only the stress moments of g
constexpr int kVarUnit = 4;

// The coupled step of logical block lb of one lattice (NT: streaming stores;
// Q: velocities of the NSE lattice, 15 or 19; V: variant bits, the study
// switches and the collision form).
template <int P, int TY, bool XYWALL, bool NT, int Q = 15, int V = 0>
__device__ inline void fused_body(const Geo& G, const Coef<typename Prec<P>::T>& C, const Bufs& B, int cur,
                                  const Tiling& TL, int lb) {
  using T = typename Prec<P>::T;
  using R = Ring<P, TY, 2>;
  using MU = MuMaker<P, TY>;
  constexpr bool PACK = packed<P, true>();
  using L = Lat<P, PACK>;
  using LD = PhiLoader<P, TY, 2, XYWALL, PACK>;
  using QT = typename LD::QT;
  // rings: phi of planes z-2 .. z+3, mu of planes z-2 .. z+1 (at most one
  // barrier apart, threads read and write disjoint slots), and the own
  // node's pulled populations of planes z .. z+2 (thread-private slots)
  constexpr int NPR = 6, NMR = 4;
  __shared__ T sphi[NPR][R::NPHI];
  __shared__ T smu[NMR][MU::NMU];
  __shared__ QT sfq[3][7 * R::NT];
  if (C.poison) {
    poison_shared(sphi, sizeof sphi);
    poison_shared(smu, sizeof smu);
    poison_shared(sfq, sizeof sfq);
    __syncthreads();
  }
  auto ps = [](int z) { return (z + 2 * NPR) % NPR; };  // z >= -2
  auto ms = [](int z) { return (z + 2 * NMR) % NMR; };  // z >= -2
  auto qs = [](int z) { return (z + 9) % 3; };
  const int tile = lb % (TL.tiles_x * TL.tiles_y), seg = lb / (TL.tiles_x * TL.tiles_y);
  const int x0 = (tile % TL.tiles_x) * kTX, y0 = (tile / TL.tiles_x) * TY;
  const int z0 = seg * TL.lz, z1 = min(G.nz, z0 + TL.lz);
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool own = gx < G.nx && gy < G.ny;
  // selects, not B.f[cur]: a runtime index into a local copy of Bufs (the
  // batched kernel) would put it in scratch memory
  const void* fin = cur ? B.f[1] : B.f[0];
  const void* gin = cur ? B.g[1] : B.g[0];
  void* fo = cur ? B.f[0] : B.f[1];
  void* go = cur ? B.g[0] : B.g[1];
  T* hist = (T*)B.phiu;

  LD ld;
  ld.init(G, x0, y0);
  MU mm;
  mm.init(G, x0, y0);
  // the loader's own column is the node's column for every thread that owns a
  // node (in-plane index gx + nx gy, ring position of the tile node)
  const Column& col = ld.own;
  const int col_xy = ld.own_xy;
  const int lds_c = ld.own_lds;
  const int mu_c = (ty + 1) * MU::QX + tx + 1;

  // The march issues the pulls of plane z+3 before mu of plane z+1 and has
  // one barrier per plane (ONEBAR), or pulls plane z+2 and has a barrier
  // after the pulls and after mu.  Measured at 256 x 256 x 1024: one barrier
  // is 2 % faster for FP64 and 16-bit storage, no different for FP32, and
  // 3 % slower for the D3Q19 lattice.
  constexpr bool ONEBAR = Q == 15;
  // warm-up: phi planes z0-2 .. z0+2 (ONEBAR) or z0+1 with the own
  // populations of z0 on, mu planes z0-1, z0 (read after the first barrier
  // of the march)
  // (three planes' pulls in flight at a time: plane k is issued before
  // plane k-2 is summed)
  {
    constexpr int NW = ONEBAR ? 5 : 4;
    typename LD::Pending pw[3];
#pragma unroll
    for (int k = 0; k < NW + 2; ++k) {
      if (k < NW) ld.issue(G, fin, z0 - 2 + k, pw[k % 3]);
      if (k >= 2) {
        const int zl = z0 - 4 + k;
        ld.finish(pw[(k - 2) % 3], sphi[ps(zl)], zl >= z0 ? sfq[qs(zl)] : nullptr);
      }
    }
  }
  __syncthreads();
  mm.template run<NPR, (V & kVarS7) != 0>(G, C, z0 - 1, sphi, smu[ms(z0 - 1)]);
  mm.template run<NPR, (V & kVarS7) != 0>(G, C, z0, sphi, smu[ms(z0)]);

  // Wave priority of the 16-bit steps, which wait on memory latency rather
  // than bandwidth: high from a plane's stores until the pulls of the next
  // plane are issued, low for the mu stage and the collisions, so that loads
  // and stores go out ahead of other waves' arithmetic.  Measured at
  // 256 x 256 x 1024: FP16 1.76 -> 1.69 ms, BF16 1.76 -> 1.69 ms, D3Q19 FP16
  // 2.11 -> 1.96 ms per step; no change at 32 and 64 bits, where it is off.
  for (int z = z0; z < z1; ++z) {
    const int zo = z * G.nx * G.ny;
    const Plane p = make_plane(G, z);
    T f[7], g[Q];
    if constexpr (PACK) __builtin_amdgcn_s_setprio(1);
    // 16-bit storage: the node's g pulls and (phi u) history loads go out
    // before the phi and mu stages, so that their latency overlaps those of
    // the phi pulls (measured 2.03 -> 1.98 ms per step at 256 x 256 x 1024
    // for the g pulls; at 32 and 64 bits the registers they hold cost more
    // than they save)
    typename L::S graw[Q];
    T hprev[3];
    if constexpr (PACK) {
      if (own) {
        pull_gq_raw<P, PACK, XYWALL, Q>(G, gin, col, p, zo, col_xy, graw);
#pragma unroll
        for (int a = 0; a < 3; ++a) hprev[a] = ld_at<T, true>(hist + ((size_t)a * G.pitch + zo), col_xy);
      }
    }
    QT qv[7];
    if constexpr (ONEBAR) {
      // the own populations of plane z leave their queue slot, which plane
      // z+3 takes over below
#pragma unroll
      for (int i = 0; i < 7; ++i) qv[i] = sfq[qs(z)][i * R::NT + threadIdx.x];
      // the pulls of plane z+3 are in flight while mu of plane z+1 is formed
      // (the last plane of the segment needs none: phi is read up to z1+1)
      const bool more = z + 1 < z1;
      typename LD::Pending pd;
      if (more) ld.issue(G, fin, z + 3, pd);
      if constexpr (PACK) __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_sched_barrier(0);
      mm.template run<NPR, (V & kVarS7) != 0>(G, C, z + 1, sphi, smu[ms(z + 1)]);
      __builtin_amdgcn_sched_barrier(0);
      if (more) ld.finish(pd, sphi[ps(z + 3)], sfq[qs(z + 3)]);
      __syncthreads();
    } else {
      ld.load(G, fin, z + 2, sphi[ps(z + 2)], sfq[qs(z + 2)]);
      if constexpr (PACK) __builtin_amdgcn_s_setprio(0);
      __syncthreads();
      mm.template run<NPR, (V & kVarS7) != 0>(G, C, z + 1, sphi, smu[ms(z + 1)]);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 7; ++i) qv[i] = sfq[qs(z)][i * R::NT + threadIdx.x];
    }
    if (!own) continue;
    if constexpr (PACK) {
      f[0] = (T)__builtin_bit_cast(float, (uint32_t)qv[0]);
#pragma unroll
      for (int i = 1; i < 7; ++i) {
        f[i] = L::lo((uint32_t)qv[i]);
        g[i] = L::hi((uint32_t)qv[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 7; ++i) f[i] = (T)qv[i];
    }
    if constexpr (PACK) {
      g[0] = (T)graw[0];
#pragma unroll
      for (int i = 7; i < Q; ++i) g[i] = (T)graw[i];
    } else {
      pull_gq<P, PACK, XYWALL, Q>(G, gin, col, p, zo, col_xy, g);
    }
    T phi = phi_of(f);
    T gphi[3];
    grad_lds<T, R::PX>(sphi[ps(z - 1)], sphi[ps(z)], sphi[ps(z + 1)], lds_c, gphi, (V & kVarS7) != 0);
    const T* mc = smu[ms(z)];
    T mu = mc[mu_c];
    T lapmu = lap_lds<T, MU::QX>(smu[ms(z - 1)], mc, smu[ms(z + 1)], mu_c, (V & kVarS7) != 0);
    Macro<T> M;
    if constexpr (Q == 19) flow_macro19(C, g, phi, mu, gphi, lapmu, M);
    else flow_macro(C, g, phi, mu, gphi, lapmu, M);
    // The history is read by its own node only: non-temporal loads leave L2
    // to the lines that neighbouring tiles share (256 x 256 x 1024: FP32
    // 2.589 -> 2.580 ms per step, FP16 1.626 -> 1.616, FP64 unchanged; the
    // same hint on the g pulls, whose edge lines two tiles read, costs 3 %).
    T dphiu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T pu = phi * M.u[a];
      T* h = hist + ((size_t)a * G.pitch + zo);
      dphiu[a] = pu - (PACK ? hprev[a] : ld_at<T, true>(h, col_xy));
      st_at<NT>(h, col_xy, pu);
    }
    collide_che(C, f, phi, mu, M.u, dphiu);
    if constexpr (Q == 19) collide_ns19(C, g, M);
    else collide_ns<(V & kVarF28) != 0, (V & kVarUnit) != 0>(C, g, M);
    using S0 = typename L::S0;
    using S = typename L::S;
    if constexpr (PACK) __builtin_amdgcn_s_setprio(1);
    st_at<NT>(L::f0(fo) + zo, col_xy, (S0)f[0]);
    S* ga = (S*)go;
    if constexpr (PACK) {
      uint32_t* wa = L::words(fo, G.pitch);
#pragma unroll
      for (int i = 1; i < 7; ++i) st_at<NT>(wa + ((size_t)(i - 1) * G.pitch + zo), col_xy, L::pack(f[i], g[i]));
      st_at<NT>(ga + zo, col_xy, (S)g[0]);
#pragma unroll
      for (int i = 7; i < Q; ++i) st_at<NT>(ga + (L::gslot(i) * G.pitch + zo), col_xy, (S)g[i]);
    } else {
      S* fa = L::fi(fo, G.pitch);
#pragma unroll
      for (int i = 1; i < 7; ++i) st_at<NT>(fa + ((size_t)(i - 1) * G.pitch + zo), col_xy, (S)f[i]);
#pragma unroll
      for (int i = 0; i < Q; ++i) st_at<NT>(ga + ((size_t)i * G.pitch + zo), col_xy, (S)g[i]);
    }
    if (!(all_finite(f, 7) && all_finite(g, Q))) *B.flag = 1;
  }
}

template <int P, int TY, bool XYWALL, bool NT, int Q, int V = 0>
__global__ void __launch_bounds__(kTX* TY) __attribute__((amdgpu_waves_per_eu(waves_per_eu<P>())))
k_fused(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur, Tiling TL) {
  fused_body<P, TY, XYWALL, NT, Q, V>(G, C, B, cur, TL, logical_block(blockIdx.x, gridDim.x));
}

// Many lattices in one launch (continuous batching): the blocks of all
// lattices form one grid; a block finds its lattice in the device table by
// its (XCD-remapped) index and runs the same body as k_fused, so each
// lattice computes exactly what it computes alone.  Buffer parity of item i
// is cur0 ^ flip.
template <int P, int TY, bool XYWALL, bool NT, int V = 0>
__global__ void __launch_bounds__(kTX* TY) __attribute__((amdgpu_waves_per_eu(waves_per_eu<P>())))
k_fused_many(const BatchItem<typename Prec<P>::T>* __restrict__ tab, int count, int flip) {
  const int b = logical_block(blockIdx.x, gridDim.x);
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (tab[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const BatchItem<typename Prec<P>::T> it = tab[lo];
  fused_body<P, TY, XYWALL, NT, 15, V>(it.G, it.C, it.B, it.cur0 ^ flip, it.TL, b - it.block0);
}

// CHE-only: mu is needed at the node only, so phi needs a halo of one and a
// ring of 4 planes.  At plane z the pulls of plane z+2 are issued, plane z is
// finished while they are in flight, and their phi goes into the ring before
// the one barrier of the plane (threads read planes z-1 .. z+1 and write
// z+2, distinct slots).
template <int P, int TY, bool XYWALL, bool NT, int V = 0>
__global__ void __launch_bounds__(kTX* TY) __attribute__((amdgpu_waves_per_eu(waves_per_eu<P>())))
k_fused_che(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur, Tiling TL) {
  using T = typename Prec<P>::T;
  using R = Ring<P, TY, 1>;
  using L = Lat<P, false>;
  using LD = PhiLoader<P, TY, 1, XYWALL, false>;
  __shared__ T sphi[4][R::NPHI];
  __shared__ T sfq[2][7 * R::NT];  // the own node's pulled f of planes z, z+1
  if (C.poison) {
    poison_shared(sphi, sizeof sphi);
    poison_shared(sfq, sizeof sfq);
    __syncthreads();
  }
  const int lb = logical_block(blockIdx.x, gridDim.x);
  const int tile = lb % (TL.tiles_x * TL.tiles_y), seg = lb / (TL.tiles_x * TL.tiles_y);
  const int x0 = (tile % TL.tiles_x) * kTX, y0 = (tile / TL.tiles_x) * TY;
  const int z0 = seg * TL.lz, z1 = min(G.nz, z0 + TL.lz);
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool own = gx < G.nx && gy < G.ny;
  const void* fin = B.f[cur];
  void* fo = B.f[1 - cur];
  T* hist = (T*)B.phiu;
  LD ld;
  ld.init(G, x0, y0);
  const int col_xy = gx + G.nx * gy;
  const int lds_c = (ty + 1) * R::PX + tx + 1;
  PrescColumn<T> pc;
  pc.init(G, C, gx, gy);
  {
    // the three planes before the march: all pulls in flight together
    typename LD::Pending p0, p1, p2;
    ld.issue(G, fin, z0 - 1, p0);
    ld.issue(G, fin, z0, p1);
    ld.issue(G, fin, z0 + 1, p2);
    __builtin_amdgcn_sched_barrier(0);
    ld.finish(p0, sphi[(z0 - 1 + 8) % 4], nullptr);
    ld.finish(p1, sphi[(z0 + 8) % 4], sfq[z0 % 2]);
    ld.finish(p2, sphi[(z0 + 1 + 8) % 4], sfq[(z0 + 1) % 2]);
  }
  __syncthreads();
  // plane z; PULL: also the pulls of plane z+2, which every plane but the
  // last issues (phi is read up to plane z1, the Laplacian of plane z1-1).
  // The last plane is a separate instantiation, so that no branch around the
  // pulls leaves the compiler unsure how many loads are in flight.
  auto plane = [&](int z, auto pull) {
    constexpr bool PULL = decltype(pull)::value;
    // phi of the previous level first: the memory counter retires in order,
    // so a load issued after the pulls would wait for all of them
    const int zo = z * G.nx * G.ny;
    const T phip = own ? ld_at(hist + zo, col_xy) : (T)0;
    typename LD::Pending pd;
    if constexpr (PULL) ld.issue(G, fin, z + 2, pd);
    __builtin_amdgcn_sched_barrier(0);
    if (own) {
      const int n = zo + col_xy;
      T f[7];
#pragma unroll
      for (int i = 0; i < 7; ++i) f[i] = sfq[z % 2][i * R::NT + threadIdx.x];
      T phi = phi_of(f);
      T lap = lap_lds<T, R::PX>(sphi[(z - 1 + 8) % 4], sphi[(z + 8) % 4], sphi[(z + 1 + 8) % 4], lds_c,
                                (V & kVarS7) != 0);
      T mu = 4 * C.beta * phi * (phi - 1) * (phi + 1) - C.kappa * lap;
      T u[3], up[3];
      pc.at(G, C, (const T*)B.ufield, gx, gy, z, n, u, up);
      // Eq. 34 with u known at both levels: only phi of the previous level is kept
      st_at<NT>(hist + zo, col_xy, phi);
      T dphiu[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) dphiu[a] = phi * u[a] - phip * up[a];
      collide_che(C, f, phi, mu, u, dphiu);
      using S0 = typename L::S0;
      using S = typename L::S;
      st_at<NT>(L::f0(fo) + zo, col_xy, (S0)f[0]);
      S* fa = L::fi(fo, G.pitch);
#pragma unroll
      for (int i = 1; i < 7; ++i) st_at<NT>(fa + ((size_t)(i - 1) * G.pitch + zo), col_xy, (S)f[i]);
      if (!all_finite(f, 7)) *B.flag = 1;
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (PULL) {
      ld.finish(pd, sphi[(z + 2 + 8) % 4], sfq[z % 2]);
      __syncthreads();
    }
  };
  for (int z = z0; z < z1 - 1; ++z) plane(z, std::true_type{});
  plane(z1 - 1, std::false_type{});
}

// CHE-only with two nodes per thread: a block of 64 x 8 threads owns a
// tile of 1024 nodes, TW wide.  TW = 128: a 128 x 8 tile, thread (tx, ty)
// the nodes tx and tx + 64 of row ty; TW = 64: a 64 x 16 tile, thread
// (tx, ty) the nodes of rows ty and ty + 8.  Each wave has twice the loads of
// k_fused_che in flight per plane, and the LDS (a 4-plane phi ring and a
// 2-plane queue for 1024 nodes, 76-78 KB in FP32) still lets two blocks share
// a CU.  The wide tile pulls more halo nodes (27 % of its own against 16 %)
// but its halo columns, each x neighbour in a cache line of its own, cover 20
// rows instead of 36: on 256^3 it takes 236 -> 227 us per step in FP32 and
// 186 -> 176 us with FP16 storage, on 200 x 136 x 300 203 -> 177 us (same
// bits).  Otherwise the march of k_fused_che: at plane z the pulls of plane
// z+2 are issued, plane z is finished while they are in flight, and their phi
// goes into the ring before the one barrier of the plane.
template <int P, bool XYWALL, bool NT, int V = 0, int TW = 128>
__global__ void __launch_bounds__(kTX * 8) __attribute__((amdgpu_waves_per_eu(waves_per_eu<P>())))
k_fused_che2(Geo G, Coef<typename Prec<P>::T> C, Bufs B, int cur, Tiling TL) {
  static_assert(TW == 64 || TW == 128, "64 x 16 or 128 x 8 tiles");
  using T = typename Prec<P>::T;
  using L = Lat<P, false>;
  constexpr int TY = 1024 / TW, NTH = kTX * 8;
  constexpr int PX = TW + 2, PY = TY + 2, NPHI = PX * PY;
  constexpr int NNODE = TW * TY;
  constexpr int NHALO = NPHI - NNODE;
  static_assert(NHALO <= NTH, "one halo position per thread");
  constexpr bool PRIO = sizeof(typename L::S) == 2;
  __shared__ T sphi[4][NPHI];
  __shared__ T sfq[2][7 * NNODE];  // the own nodes' pulled f of planes z, z+1
  if (C.poison) {
    poison_shared(sphi, sizeof sphi);
    poison_shared(sfq, sizeof sfq);
    __syncthreads();
  }
  const int lb = logical_block(blockIdx.x, gridDim.x);
  const int tile = lb % (TL.tiles_x * TL.tiles_y), seg = lb / (TL.tiles_x * TL.tiles_y);
  const int x0 = (tile % TL.tiles_x) * TW, y0 = (tile / TL.tiles_x) * TY;
  const int z0 = seg * TL.lz, z1 = min(G.nz, z0 + TL.lz);
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const void* fin = B.f[cur];
  void* fo = B.f[1 - cur];
  T* hist = (T*)B.phiu;
  // own nodes (a node outside the lattice maps onto its periodic image or
  // its mirror at a wall, whose phi the ring needs there)
  Column oc[2];
  int oxy[2], olds[2], gx[2], gy[2];
  bool own[2];
  PrescColumn<T> pcol[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int lx = TW == 64 ? tx : tx + 64 * r, ly = TW == 64 ? ty + 8 * r : ty;
    gx[r] = x0 + lx;
    gy[r] = y0 + ly;
    own[r] = gx[r] < G.nx && gy[r] < G.ny;
    const int mx = map_axis(gx[r], G.nx, G.wall_x), my = map_axis(gy[r], G.ny, G.wall_y);
    oc[r] = make_column<XYWALL>(G, mx, my);
    oxy[r] = mx + G.nx * my;
    olds[r] = (ly + 1) * PX + lx + 1;
    pcol[r].init(G, C, gx[r], gy[r]);
  }
  // one halo position for each of the first NHALO threads
  const bool hon = threadIdx.x < NHALO;
  int hpx = 0, hpy = 0;
  if (hon) halo_pos<PX, PY, 1>(threadIdx.x, hpx, hpy);
  const int hx = map_axis(x0 - 1 + hpx, G.nx, G.wall_x), hy = map_axis(y0 - 1 + hpy, G.ny, G.wall_y);
  const Column hc = make_column<XYWALL>(G, hx, hy);
  const int hxy = hx + G.nx * hy, hlds = hpy * PX + hpx;

  struct Pending {
    F7Raw<P, false> o[2], h;
  };
  auto issue = [&](int zl, Pending& pd) {
    const int mz = map_axis(zl, G.nz, G.wall_z);
    const Plane p = make_plane(G, mz);
    const int zo = mz * G.nx * G.ny;
    pull_f7_raw<P, false, XYWALL>(G, fin, oc[0], p, zo, oxy[0], pd.o[0]);
    pull_f7_raw<P, false, XYWALL>(G, fin, oc[1], p, zo, oxy[1], pd.o[1]);
    if (hon) pull_f7_raw<P, false, XYWALL>(G, fin, hc, p, zo, hxy, pd.h);
  };
  auto finish = [&](const Pending& pd, T* s, T* q) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      T f[7];
      cvt_f7<P, false>(pd.o[r], f);
      s[olds[r]] = phi_of(f);
      if (q) {
#pragma unroll
        for (int i = 0; i < 7; ++i) q[i * NNODE + threadIdx.x + r * NTH] = f[i];
      }
    }
    if (hon) {
      T fh[7];
      cvt_f7<P, false>(pd.h, fh);
      s[hlds] = phi_of(fh);
    }
  };
  {
    // the three planes before the march: all pulls in flight together
    Pending p0, p1, p2;
    issue(z0 - 1, p0);
    issue(z0, p1);
    issue(z0 + 1, p2);
    __builtin_amdgcn_sched_barrier(0);
    finish(p0, sphi[(z0 - 1 + 8) % 4], nullptr);
    finish(p1, sphi[(z0 + 8) % 4], sfq[z0 % 2]);
    finish(p2, sphi[(z0 + 1 + 8) % 4], sfq[(z0 + 1) % 2]);
  }
  __syncthreads();
  auto plane = [&](int z, auto pull) {
    constexpr bool PULL = decltype(pull)::value;
    const int zo = z * G.nx * G.ny;
    // 16-bit storage: wave priority high from the stores of a plane until the
    // pulls of the next are issued (256^3 with FP16 storage 190 -> 186 us per
    // step; no change in FP32)
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
    // the history loads first: the memory counter retires in order.  No
    // other block reads them, so they are non-temporal and leave L2 to the
    // halo pulls that neighbouring tiles share (256^3: 227 -> 225 us per
    // step in FP32, 176 -> 171 us with FP16 storage).
    T phip[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) phip[r] = own[r] ? ld_at<T, true>(hist + zo, oxy[r]) : (T)0;
    Pending pd;
    if constexpr (PULL) issue(z + 2, pd);
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!own[r]) continue;
      T f[7];
#pragma unroll
      for (int i = 0; i < 7; ++i) f[i] = sfq[z % 2][i * NNODE + threadIdx.x + r * NTH];
      const T phi = phi_of(f);
      const T lap = lap_lds<T, PX>(sphi[(z - 1 + 8) % 4], sphi[(z + 8) % 4], sphi[(z + 1 + 8) % 4], olds[r],
                                   (V & kVarS7) != 0);
      const T mu = 4 * C.beta * phi * (phi - 1) * (phi + 1) - C.kappa * lap;
      T u[3], up[3];
      pcol[r].at(G, C, (const T*)B.ufield, gx[r], gy[r], z, zo + oxy[r], u, up);
      if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
      st_at<NT>(hist + zo, oxy[r], phi);  // Eq. 34: only phi of this level is kept
      T dphiu[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) dphiu[a] = phi * u[a] - phip[r] * up[a];
      collide_che(C, f, phi, mu, u, dphiu);
      st_at<NT>(L::f0(fo) + zo, oxy[r], (typename L::S0)f[0]);
      typename L::S* fa = L::fi(fo, G.pitch);
#pragma unroll
      for (int i = 1; i < 7; ++i)
        st_at<NT>(fa + ((size_t)(i - 1) * G.pitch + zo), oxy[r], (typename L::S)f[i]);
      if (!all_finite(f, 7)) *B.flag = 1;
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (PULL) {
      finish(pd, sphi[(z + 2 + 8) % 4], sfq[z % 2]);
      __syncthreads();
    }
  };
  for (int z = z0; z < z1 - 1; ++z) plane(z, std::true_type{});
  plane(z1 - 1, std::false_type{});
}

template <class T>
Coef<T> cast_coef_f(const Coef<double>& c) {
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

// Rows per tile: 8 (512 threads, two blocks per CU) except for the coupled
// step with FP32 populations on a large lattice, which takes 16 (1024
// threads, one block per CU).
// There the halo of the phi ring falls from 59 % to 33 % of the tile's own
// f pulls, and the step is 3 % faster on D3Q15 and 4 % on D3Q19 (same bits).
// The 16-bit steps wait on memory latency and lose 11 % with one block per
// CU; FP64 does not fit the 160 KB of LDS at 16 rows.
constexpr int kTY = 8;
template <int P>
constexpr int coupled_ty() { return P == MPLB_F32 ? 16 : kTY; }

// Segment length along z: at most the blocks of a few rounds over the 256 CUs
// (four rounds at two 8-row blocks per CU, two at one 16-row block), with
// segments as long as that allows (each segment re-reads a few planes).
// `target` overrides the block count aimed at.
Tiling make_tiling(const Geo& G, int TY, int min_lz, int target = 0, int TW = kTX) {
  Tiling t;
  t.tiles_x = (G.nx + TW - 1) / TW;
  t.tiles_y = (G.ny + TY - 1) / TY;
  int cols = t.tiles_x * t.tiles_y;
  if (target <= 0) target = TY >= 16 ? 512 : 2048;
  // at most `target` blocks: the blocks of a round that the chip cannot
  // start with the others run after them, alone.  Rounding the segment count
  // down instead of up took 160 x 160 x 640 from 0.704 to 0.499 ms per step
  // with FP16 populations, 192 x 192 x 768 from 0.972 to 0.726 ms, and a
  // 224^3 CHE-only step from 210 to 168 us (same bits; the boxes whose
  // planes divide the target evenly, such as 256 x 256 x 1024, unchanged).
  int want = target / cols;
  if (want < 1) want = 1;
  int lz = (G.nz + want - 1) / want;
  if (lz < min_lz) lz = min_lz;
  if (lz > G.nz) lz = G.nz;
  t.lz = lz;
  t.nseg = (G.nz + lz - 1) / lz;
  return t;
}

// Streaming stores pay once a step moves much more than the 256 MB
// last-level cache holds (measured: about 3 % faster at 256 x 256 x 1024,
// 18 % slower for a 128^3 CHE-only box that stays cache-resident).
constexpr size_t kStreamBytes = (size_t)512 << 20;

// One coupled step with TY-row tiles.
template <int P, int TY, bool XYWALL, bool NT, int V>
void launch_coupled(int mode, const Geo& G, const Coef<typename Prec<P>::T>& C, const Bufs& B, int cur,
                    const Tiling& tl, hipStream_t s) {
  dim3 grid((unsigned)(tl.tiles_x * tl.tiles_y * tl.nseg));
  if (mode == MPLB_COUPLED)
    hipLaunchKernelGGL((k_fused<P, TY, XYWALL, NT, 15, V>), grid, dim3(kTX * TY), 0, s, G, C, B, cur, tl);
  else  // D3Q19: its forcing is Gamma T, so only the stencil switch applies
    hipLaunchKernelGGL((k_fused<P, TY, XYWALL, NT, 19, V & kVarS7>), grid, dim3(kTX * TY), 0, s, G, C, B, cur,
                       tl);
}

// The coupled step with 8-row tiles aims at 512 blocks, one round of the chip
// at two blocks per CU, rather than four rounds: the ring's warm-up re-reads
// five planes per segment, and on the 256 x 256 x 1024 box 256-plane
// segments took FP16 1690 -> 1618 us per step, BF16 1665 -> 1624 and FP64
// 5300 -> 5250 (1024 blocks: 1673, 1650, 5285), same bits.  The 16-row FP32
// step keeps two rounds (one round: 2588 -> 2674 us).  FP64 runs one block
// per CU (its registers), so its round is 256 blocks: 256 x 256 x 1024 5180
// -> 5054 us, a W = 64 Rayleigh-Taylor box 100.5 -> 85.4 us; the FP64
// CHE-only step likewise, 96^3 39.7 -> 35.1 us, 128^3 58.6 -> 53.6, 256^3
// 477 -> 428 (64^3 and 192^3 within 1.5 %).
constexpr int kTarget8 = 512;

// A lattice stepped alone whose blocks cannot fill the chip is bound by the
// latency of its march, not by bandwidth: segments of at least 5 planes
// instead of 16 (more, shorter segments, each re-reading its 5 warm-up
// planes) took a 32^3 droplet from 61.1 to 25.8 us per step in FP32 and 81.4
// to 32.9 in FP64, 64^3 from 68.0 to 29.5, 96^3 from 71.8 to 49.1, W = 32 and
// 48 Rayleigh-Taylor boxes from 60.5 and 67.1 to 26.1 and 31.0; boxes whose
// segment count the block target sets (W >= 96) are unchanged (same bits).
// A lattice between 256 and 512 blocks leaves some CUs with one block and
// others with two; where one block per CU marches fewer plane-times (below)
// it is taken: 72^3 droplet 42.7 -> 34.5 us in FP32 and 42.3 -> 31.6 with
// FP16 populations, 80^3 43.8 -> 38.5, W = 56 and 64 Rayleigh-Taylor boxes
// 44.8 -> 40.0 and 49.8 -> 47.4 (FP16 at W = 64: 38.6 -> 39.3), boxes of
// 96^3 and 112^3, which keep two blocks per CU, unchanged.
// The batched step keeps 16: there the lattices fill the chip together, and
// 8 or 5 planes gave 24.5 and 24.0 GLUPS against 24.6 on the serving trace's
// lattices in FP32, 35.0 and 31.7 against 37.5 with FP16 populations.
constexpr int kMinLz8 = 5;

// 16-row tiles only on a lattice that fills two rounds of the chip with them:
// on small lattices (64^3: 16 blocks) they halve the blocks that run at all,
// and 8-row tiles took 26 % less time per step on the serving trace's boxes.
// With the segment count rounded down, that is a lattice whose tile count
// divides the 512 blocks (256 x 256 x 1024: 2.59 ms against 2.87 with 8
// rows); elsewhere 8 rows are as fast or faster (192 x 192 x 768: 1.168 ms
// against 1.171, 160 x 160 x 640: 0.712 against 0.762).
constexpr int kMinBlocksTall = 512;

// CHE-only tiling.  Both kernels size their segments for at most 512
// blocks, one round of the chip at two blocks per CU (FP64, one block per CU:
// 256).  Two nodes per thread
// (k_fused_che2, 128 x 8 tiles, segments of at least 8 planes: 32 at 256^3)
// on lattices of at least 5 M nodes that fill at least 384 such blocks; 8-row
// tiles of 64 (k_fused_che, segments of at least 5 planes) otherwise and for
// FP64, whose two-node LDS would not let two blocks share a CU.  Measured
// (FP32, us per step, one-node against two-node tiles): 96^3 23.9 / 30.2,
// 128^3 32.6 / 35.3, 144^3 51.4 / 61.4, 160^3 61.9 / 71.2, 176^3 106.8 /
// 100.4, 192^3 115.0 / 119.3, 224^3 198 / 161; 256^3 262 / 232 with the
// earlier one-node sizing.  The
// one-node kernel took four rounds with segments of at least 8 planes before
// (96^3 30.5, 100^3 30.6, 144^3 54.9, 160^3 67.9, 192^3 124.4 us; 128^3, one
// round either way, unchanged).  Before the two-node kernel took 128 x 8
// tiles, on 256^3 with 64 x 16 tiles: 254 -> 236 us (8-row tiles with
// 32-plane segments: 248; two rows with 8- or 16-plane segments: 245, 238),
// FP16 storage 219 -> 190 us.  Same bits in every variant.
constexpr int kCheTarget2 = 512, kCheMinLz2 = 8, kCheMinBlocks2 = 384;
constexpr int kCheMinNodes2 = 5000000;
constexpr int kCheTarget1 = 512, kCheMinLz1 = 5;
constexpr int kCheTW = 128;

}  // namespace

// One block per CU instead of two-block tiling t where t would leave some CUs
// with one block and others with two: the CUs that run two take about 1.3
// times as long and set the step time, so the one-block split (longer
// segments) is taken where its march, in planes plus about 8 planes of
// warm-up and start, is shorter than 1.3 times the other's.
static Tiling balance(const Geo& G, int TY, int min_lz, Tiling t, int target) {
  const int nb = t.tiles_x * t.tiles_y * t.nseg;
  if (nb > target / 2 && nb < target) {
    const Tiling t1 = make_tiling(G, TY, min_lz, target / 2);
    if (10 * (t1.lz + 8) <= 13 * (t.lz + 8)) return t1;
  }
  return t;
}

Shape launch_shape(int P, int mode, const Geo& G, int rows) {
  if (mode == MPLB_COUPLED || mode == MPLB_COUPLED_Q19) {
    if (P == MPLB_F32) {
      const Tiling tall = make_tiling(G, 16, 16);
      if (rows == 16 || (rows == 0 && tall.tiles_x * tall.tiles_y * tall.nseg >= kMinBlocksTall))
        return Shape{kShapeCoupled16, kTX, 16, tall};
    }
    // FP64 runs one block per CU (its registers), the other precisions two
    Tiling t8 = make_tiling(G, kTY, kMinLz8, P == MPLB_F64 ? kTarget8 / 2 : kTarget8);
    if (P != MPLB_F64) t8 = balance(G, kTY, kMinLz8, t8, kTarget8);
    return Shape{kShapeCoupled8, kTX, kTY, t8};
  }
  if (P != MPLB_F64) {
    const Tiling t2 = make_tiling(G, 1024 / kCheTW, kCheMinLz2, kCheTarget2, kCheTW);
    if (rows == 16 ||
        (rows == 0 && G.N >= kCheMinNodes2 && t2.tiles_x * t2.tiles_y * t2.nseg >= kCheMinBlocks2))
      return Shape{kShapeChe2, kCheTW, 1024 / kCheTW, t2};
  }
  Tiling tl = make_tiling(G, kTY, kCheMinLz1, P == MPLB_F64 ? kCheTarget1 / 2 : kCheTarget1);
  if (P != MPLB_F64) tl = balance(G, kTY, kCheMinLz1, tl, kCheTarget1);
  return Shape{kShapeChe1, kTX, kTY, tl};
}

namespace {

template <int P, bool XYWALL, bool NT, int V>
hipError_t fused_impl4(int mode, const Geo& G, const Coef<typename Prec<P>::T>& C, const Bufs& B, int cur,
                       hipStream_t s, int rows) {
  const Shape sh = launch_shape(P, mode, G, rows);
  if (mode == MPLB_COUPLED || mode == MPLB_COUPLED_Q19) {
    constexpr int TY = coupled_ty<P>();
    if constexpr (TY != kTY) {
      if (sh.kind == kShapeCoupled16) {
        launch_coupled<P, TY, XYWALL, NT, V>(mode, G, C, B, cur, sh.tl, s);
        return hipGetLastError();
      }
    }
    launch_coupled<P, kTY, XYWALL, NT, V>(mode, G, C, B, cur, sh.tl, s);
  } else {
    if constexpr (sizeof(typename Prec<P>::T) == 4) {
      if (sh.kind == kShapeChe2) {
        hipLaunchKernelGGL((k_fused_che2<P, XYWALL, NT, V & kVarS7, kCheTW>),
                           dim3((unsigned)(sh.tl.tiles_x * sh.tl.tiles_y * sh.tl.nseg)), dim3(kTX * 8), 0, s, G, C, B,
                           cur, sh.tl);
        return hipGetLastError();
      }
    }
    dim3 grid((unsigned)(sh.tl.tiles_x * sh.tl.tiles_y * sh.tl.nseg));
    hipLaunchKernelGGL((k_fused_che<P, kTY, XYWALL, NT, V & kVarS7>), grid, dim3(kTX * kTY), 0, s, G, C, B, cur,
                       sh.tl);
  }
  return hipGetLastError();
}

template <int P, bool XYWALL, bool NT>
hipError_t fused_impl3(int mode, const Geo& G, const Coef<typename Prec<P>::T>& C, const Bufs& B, int cur,
                       hipStream_t s, int rows) {
  const int v = (C.stencil7 ? kVarS7 : 0) | (C.forcing28 ? kVarF28 : 0) | (C.unit_rates ? kVarUnit : 0);
  if (v == 0) return fused_impl4<P, XYWALL, NT, 0>(mode, G, C, B, cur, s, rows);
  if (v == kVarUnit) return fused_impl4<P, XYWALL, NT, kVarUnit>(mode, G, C, B, cur, s, rows);
  if constexpr (P == MPLB_F64 || P == MPLB_F32) {
    switch (v) {
      case kVarS7: return fused_impl4<P, XYWALL, NT, kVarS7>(mode, G, C, B, cur, s, rows);
      case kVarS7 | kVarUnit: return fused_impl4<P, XYWALL, NT, kVarS7 | kVarUnit>(mode, G, C, B, cur, s, rows);
      case kVarF28: return fused_impl4<P, XYWALL, NT, kVarF28>(mode, G, C, B, cur, s, rows);
      case kVarF28 | kVarUnit: return fused_impl4<P, XYWALL, NT, kVarF28 | kVarUnit>(mode, G, C, B, cur, s, rows);
      case kVarS7 | kVarF28: return fused_impl4<P, XYWALL, NT, kVarS7 | kVarF28>(mode, G, C, B, cur, s, rows);
      default: return fused_impl4<P, XYWALL, NT, kVarS7 | kVarF28 | kVarUnit>(mode, G, C, B, cur, s, rows);
    }
  }
  return hipErrorInvalidValue;  // the study switches are built for FP64 and FP32 storage
}

template <int P, bool XYWALL>
hipError_t fused_impl2(int mode, const Geo& G, const Coef<typename Prec<P>::T>& C, const Bufs& B, int cur,
                       hipStream_t s, int rows) {
  if (fused_step_bytes(P, mode, G.N) > kStreamBytes)
    return fused_impl3<P, XYWALL, true>(mode, G, C, B, cur, s, rows);
  return fused_impl3<P, XYWALL, false>(mode, G, C, B, cur, s, rows);
}

template <int P>
hipError_t fused_impl(int mode, const Geo& G, const Coef<double>& Cd, const Bufs& B, int cur, hipStream_t s,
                      int rows) {
  using T = typename Prec<P>::T;
  Coef<T> C = cast_coef_f<T>(Cd);
  if (G.wall_x || G.wall_y) return fused_impl2<P, true>(mode, G, C, B, cur, s, rows);
  return fused_impl2<P, false>(mode, G, C, B, cur, s, rows);
}

template <int P, bool XYWALL, bool NT, int V>
hipError_t many_impl2(const void* dtab, int count, int total_blocks, int flip, hipStream_t s) {
  using T = typename Prec<P>::T;
  hipLaunchKernelGGL((k_fused_many<P, kTY, XYWALL, NT, V>), dim3((unsigned)total_blocks), dim3(kTX * kTY), 0, s,
                     (const BatchItem<T>*)dtab, count, flip);
  return hipGetLastError();
}

// nsteps batched steps as a chain of kernel nodes (flip alternating), built
// directly rather than by stream capture so that it works on any stream.
template <int P, bool XYWALL, bool NT, int V>
hipError_t many_graph2(const void* dtab, int count, int total_blocks, int nsteps, hipGraph_t* out) {
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
    int flip = k & 1;
    const void* tab = dtab;
    void* args[] = {(void*)&tab, (void*)&count, (void*)&flip};
    hipKernelNodeParams kp{};
    kp.func = (void*)k_fused_many<P, kTY, XYWALL, NT, V>;
    kp.gridDim = dim3((unsigned)total_blocks);
    kp.blockDim = dim3(kTX * kTY);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return e;
  }
  *out = g;
  return hipSuccess;
}

template <int P>
int batch_fill_impl(void* table, int i, const Geo& G, const Coef<double>& Cd, const Bufs& B, int cur0, int block0) {
  using T = typename Prec<P>::T;
  BatchItem<T> it{};
  it.G = G;
  it.TL = make_tiling(G, kTY, 16);
  it.B = B;
  it.C = cast_coef_f<T>(Cd);
  it.cur0 = cur0;
  it.block0 = block0;
  it.nblocks = it.TL.tiles_x * it.TL.tiles_y * it.TL.nseg;
  ((BatchItem<T>*)table)[i] = it;
  return it.nblocks;
}

// Batch table of mplb_step_many_noalloc: a file-scope device array, so that
// the call allocates nothing.  Each device holds its own copy until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy (on the host it is only a stand-in for the symbol): its device address
// is looked up once per device and kept.
constexpr size_t kNoAllocTableBytes = (size_t)MPLB_NOALLOC_MAX_LATTICES * sizeof(BatchItem<double>);
static_assert(sizeof(BatchItem<double>) >= sizeof(BatchItem<float>), "the table is sized for FP64 items");
static __device__ __align__(256) unsigned char scratch[kNoAllocTableBytes];
constexpr int kMaxDevices = 64;
// atomic: lattices may be created on several threads at once (each lookup
// of a device stores the same address)
std::atomic<void*> g_scratch_ptr[kMaxDevices];

}  // namespace

hipError_t noalloc_table(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return hipSuccess;
}

size_t noalloc_table_bytes() { return kNoAllocTableBytes; }

hipError_t launch_fused_step(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur,
                             hipStream_t s, int rows) {
  switch (P) {
    case MPLB_F64: return fused_impl<MPLB_F64>(mode, G, C, B, cur, s, rows);
    case MPLB_F32: return fused_impl<MPLB_F32>(mode, G, C, B, cur, s, rows);
    case MPLB_F32_F16: return fused_impl<MPLB_F32_F16>(mode, G, C, B, cur, s, rows);
    case MPLB_F32_BF16: return fused_impl<MPLB_F32_BF16>(mode, G, C, B, cur, s, rows);
    default: return hipErrorInvalidValue;
  }
}

size_t fused_batch_item_bytes(int P) {
  return P == MPLB_F64 ? sizeof(BatchItem<double>) : sizeof(BatchItem<float>);
}

int fused_batch_fill(int P, void* table, int i, const Geo& G, const Coef<double>& C, const Bufs& B, int cur0,
                     int block0) {
  switch (P) {
    case MPLB_F64: return batch_fill_impl<MPLB_F64>(table, i, G, C, B, cur0, block0);
    case MPLB_F32: return batch_fill_impl<MPLB_F32>(table, i, G, C, B, cur0, block0);
    case MPLB_F32_F16: return batch_fill_impl<MPLB_F32_F16>(table, i, G, C, B, cur0, block0);
    case MPLB_F32_BF16: return batch_fill_impl<MPLB_F32_BF16>(table, i, G, C, B, cur0, block0);
    default: return -1;
  }
}

hipError_t launch_fused_many(int P, bool xywall, bool nt, bool unit, const void* dtab, int count, int total_blocks,
                             int flip, hipStream_t s) {
#define MPLB_MANY_V(PP, W, N)                                                                        \
  return unit ? many_impl2<PP, W, N, kVarUnit>(dtab, count, total_blocks, flip, s)                  \
              : many_impl2<PP, W, N, 0>(dtab, count, total_blocks, flip, s);
#define MPLB_MANY(PP)                                                                                \
  if (xywall) {                                                                                      \
    if (nt) MPLB_MANY_V(PP, true, true)                                                              \
    MPLB_MANY_V(PP, true, false)                                                                     \
  }                                                                                                  \
  if (nt) MPLB_MANY_V(PP, false, true)                                                               \
  MPLB_MANY_V(PP, false, false)
  switch (P) {
    case MPLB_F64: MPLB_MANY(MPLB_F64)
    case MPLB_F32: MPLB_MANY(MPLB_F32)
    case MPLB_F32_F16: MPLB_MANY(MPLB_F32_F16)
    case MPLB_F32_BF16: MPLB_MANY(MPLB_F32_BF16)
    default: return hipErrorInvalidValue;
  }
#undef MPLB_MANY
#undef MPLB_MANY_V
}

hipError_t build_fused_many_graph(int P, bool xywall, bool nt, bool unit, const void* dtab, int count,
                                  int total_blocks, int nsteps, hipGraph_t* out) {
#define MPLB_GRAPH_V(PP, W, N)                                                                       \
  return unit ? many_graph2<PP, W, N, kVarUnit>(dtab, count, total_blocks, nsteps, out)             \
              : many_graph2<PP, W, N, 0>(dtab, count, total_blocks, nsteps, out);
#define MPLB_GRAPH(PP)                                                                               \
  if (xywall) {                                                                                      \
    if (nt) MPLB_GRAPH_V(PP, true, true)                                                             \
    MPLB_GRAPH_V(PP, true, false)                                                                    \
  }                                                                                                  \
  if (nt) MPLB_GRAPH_V(PP, false, true)                                                              \
  MPLB_GRAPH_V(PP, false, false)
  switch (P) {
    case MPLB_F64: MPLB_GRAPH(MPLB_F64)
    case MPLB_F32: MPLB_GRAPH(MPLB_F32)
    case MPLB_F32_F16: MPLB_GRAPH(MPLB_F32_F16)
    case MPLB_F32_BF16: MPLB_GRAPH(MPLB_F32_BF16)
    default: return hipErrorInvalidValue;
  }
#undef MPLB_GRAPH
#undef MPLB_GRAPH_V
}

size_t fused_stream_threshold() { return kStreamBytes; }

size_t fused_step_bytes(int P, int mode, long long N) {
  // populations and history read and written once per update
  size_t per = mode == MPLB_COUPLED       ? (P == MPLB_F64 ? 400 : (P == MPLB_F32 ? 200 : 116))
               : mode == MPLB_COUPLED_Q19 ? (P == MPLB_F64 ? 464 : (P == MPLB_F32 ? 232 : 132))
                                          : (P == MPLB_F64 ? 128 : 64);
  return per * (size_t)N;
}

}  // namespace mplb
