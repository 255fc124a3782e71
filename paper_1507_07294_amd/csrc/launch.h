// Host-side launchers of the libmplb kernels (kernels.hip).  Each enqueues on
// `s` and returns the launch status; precision P and mode select the template
// instance at run time.
#pragma once

#include "common.h"

namespace mplb {

// phi = sum_i f_i over the pulled populations of buffer `cur` (Eq. 13)
hipError_t launch_phi(int P, int mode, const Geo& G, const Bufs& B, int cur, hipStream_t s);
// mu from phi (Eqs. 2, 36)
hipError_t launch_mu(int P, const Geo& G, const Coef<double>& C, const Bufs& B, hipStream_t s);
// one step as a single z-marching kernel (fused.hip): reads buffer `cur`,
// writes buffer 1 - cur.  rows: tile height of the coupled step, 0 for the
// automatic choice, 8 or 16 to force one (16: FP32 populations only)
hipError_t launch_fused_step(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur,
                             hipStream_t s, int rows = 0);
// the kernel and work split launch_fused_step uses (host computation only;
// rows as there, assumed valid for P and mode)
Shape launch_shape(int P, int mode, const Geo& G, int rows);
// Batched coupled step over a device table of BatchItem<T> (T of P):
// fused_batch_item_bytes gives the item size, fused_batch_fill writes item i
// of a host table and returns that lattice's block count, launch_fused_many
// runs one step of every item (buffer parity cur0 ^ flip).
size_t fused_batch_item_bytes(int P);
int fused_batch_fill(int P, void* table, int i, const Geo& G, const Coef<double>& C, const Bufs& B, int cur0,
                     int block0);
// (nt: streaming stores, for batches whose step moves more than
// kStreamBytes; see fused_step_bytes; unit: every item has S^g = 1 off the
// stress moments, the form its lattice uses alone)
hipError_t launch_fused_many(int P, bool xywall, bool nt, bool unit, const void* dtab, int count, int total_blocks,
                             int flip, hipStream_t s);
// the same for nsteps steps (flip = k & 1 at step k) as a graph of kernel
// nodes; the caller instantiates, launches and destroys it
hipError_t build_fused_many_graph(int P, bool xywall, bool nt, bool unit, const void* dtab, int count,
                                  int total_blocks, int nsteps, hipGraph_t* out);
// Device address of the static batch table of mplb_step_many_noalloc on
// device `dev` (the current device), looked up on the first call for that
// device and kept; it holds MPLB_NOALLOC_MAX_LATTICES items of any precision
// (noalloc_table_bytes bytes).
hipError_t noalloc_table(int dev, void** out);
size_t noalloc_table_bytes();
// algorithmic bytes one step of an N-node lattice moves (populations and
// history read and written once)
size_t fused_step_bytes(int P, int mode, long long N);
// step traffic above which the step kernels use streaming stores
size_t fused_stream_threshold();
// field (MPLB_PHI..MPLB_P) at the current level into B.out (double)
hipError_t launch_macro(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur,
                        int field, hipStream_t s);
// FP64 totals and non-finite count into B.red[kRedSlots*8 .. +8)
hipError_t launch_totals(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur,
                         hipStream_t s);
// lowest and highest z where phi (the B.phi array) crosses 0 along z, into
// B.red[kRedSlots*8 .. +2) (-1, -1 when there is none)
hipError_t launch_front(int P, const Geo& G, const Bufs& B, hipStream_t s);
// out[z * nx + i] = f[(z * nx + i) * nx + i]: the plane x = y of a field with
// nx = ny (nx * nz elements; out must not overlap f)
hipError_t launch_diag(const double* f, double* out, int nx, int nz, hipStream_t s);
// dst[n] = (T) B.out[n] for n < N (upload of a host field staged in B.out)
hipError_t launch_cvt_in(int P, const Geo& G, const Bufs& B, void* dst, hipStream_t s);
// equilibrium initial state into buffer `cur`, from phi, mu and u (held in phiu)
hipError_t launch_init(int P, int mode, const Geo& G, const Coef<double>& C, const Bufs& B, int cur,
                       hipStream_t s);
hipError_t launch_fill_int(int* p, int value, int count, hipStream_t s);
// dst = src, 16-byte accesses (bandwidth reference); streaming: non-temporal stores
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int kind, hipStream_t s);
hipError_t launch_fill_zero(int P, void* p, int count, hipStream_t s);
// overwrite stored population i (set 0: f, 1: g) at storage index n of buffer cur
hipError_t launch_poke(int P, int mode, const Geo& G, const Bufs& B, int cur, int set, int i, int n, double v,
                       hipStream_t s);

}  // namespace mplb
