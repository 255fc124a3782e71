/*
 * mplb.h -- C-ABI of libmplb, the MI355X (gfx950) implementation of the time
 * step of the three-dimensional MRT lattice-Boltzmann phase-field model of
 * Liang, Shi & Chai, "An efficient three-dimensional multiple-relaxation-time
 * lattice Boltzmann model for multiphase flows" (arXiv:1507.07294).
 *
 * The problem the calls follow (Secs. II-III of the paper): given a lattice,
 * the parameters {sigma, D, rho_l, rho_g, M, A, S^f, nu, S^g, gravity}, an
 * initial order parameter phi (and velocity u) and boundary conditions,
 * advance the D3Q7 MRT scheme for the Cahn-Hilliard equation (Eq. 4) and the
 * D3Q15 MRT scheme for the Navier-Stokes equations (Eq. 20) by N steps and
 * observe phi, rho, mu, u and p.  For the interface-tracking problems
 * (Sec. III A-B) only Eq. 4 is advanced, under a prescribed velocity.
 *
 * Conventions
 *  - Lattice units, dx = dt = c = 1.  Node (x,y,z) has index x + nx*(y + ny*z).
 *  - Host arrays are double, x fastest; a vector field is three consecutive
 *    scalar fields (x component first).  Host arrays are owned by the caller
 *    and only read or written during the call.
 *  - Every call returns MPLB_OK or an error code; nothing throws across the
 *    ABI.  On error, mplb_last_error(h) describes it.  A handle is not
 *    thread-safe; distinct handles may be used from distinct threads.
 *  - Work is enqueued on the handle's HIP stream (default: the null stream).
 *    mplb_step returns once the work is enqueued unless a non-finite check is
 *    due; mplb_read, mplb_totals and mplb_checkpoint synchronise the stream.
 */
#ifndef MPLB_H
#define MPLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MPLB_OK 0
#define MPLB_E_INVAL 1     /* bad argument, size or parameter */
#define MPLB_E_NOMEM 2     /* device allocation failed or arena too small */
#define MPLB_E_DEVICE 3    /* a HIP call failed; text in mplb_last_error */
#define MPLB_E_STATE 4     /* call out of order (e.g. step before init) */
#define MPLB_E_NONFINITE 5 /* a population became NaN or Inf; step index in mplb_last_error */

/* boundary condition per axis */
#define MPLB_PERIODIC 0
#define MPLB_WALL 1 /* no-slip wall, half-way bounce-back, between node 0 / n-1 and the ghost layer */

/* arithmetic and storage precision */
#define MPLB_F64 0       /* FP64 compute and storage */
#define MPLB_F32 1       /* FP32 compute and storage */
#define MPLB_F32_F16 2   /* FP32 compute; f_1..f_6 and g stored in FP16, f_0 and (phi u) in FP32 */
#define MPLB_F32_BF16 3  /* FP32 compute; f_1..f_6 and g stored in BF16, f_0 and (phi u) in FP32 */

/* what a step advances */
#define MPLB_COUPLED 0  /* Eqs. 4 and 20 (Sec. II) */
#define MPLB_CHE_ONLY 1 /* Eq. 4 under a prescribed velocity (Sec. III A-B) */
/* Eqs. 4 and 20 with the NSE populations on D3Q19, the other lattice the
 * paper names (Sec. II B, after Eq. 22): rest, the six faces in the order of
 * Eq. 23, then the twelve edges in antipodal pairs ((1,1,0), (-1,-1,0),
 * (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1),
 * (0,-1,-1), (0,1,-1), (0,-1,1)); weights 1/3, 1/18, 1/36.  The collision
 * relaxes the five stress moments of d'Humieres' D3Q19 basis at 1/tau_g
 * (Eq. 33) and every other moment at 1 (lambda_g is not used); g^eq and the
 * source are Eqs. 21 and 28 taken exactly.  Every storage precision; with
 * 16-bit storage f_i and g_i (i = 1..6) share 32-bit words as on D3Q15.
 * mplb_step_many steps such lattices one after another. */
#define MPLB_COUPLED_Q19 2

/* fields for mplb_read */
#define MPLB_PHI 0 /* order parameter, Eq. 13 */
#define MPLB_RHO 1 /* density, Eq. 14 */
#define MPLB_MU 2  /* chemical potential, Eq. 2 */
#define MPLB_UX 3  /* velocity, Eq. 29 (or the prescribed one) */
#define MPLB_UY 4
#define MPLB_UZ 5
#define MPLB_P 6   /* pressure, Eq. 30 (0 in CHE-only mode) */

/* prescribed velocities for MPLB_CHE_ONLY (mplb_set_velocity) */
#define MPLB_VEL_ZERO 0
#define MPLB_VEL_FIELD 1   /* a constant field given by the caller */
#define MPLB_VEL_ZALESAK 2 /* rigid rotation, Eq. 37, L = nx */
#define MPLB_VEL_DEFORM 3  /* deformation flow, Eq. 41 times cos(pi t/T), t = n U / nx */

typedef struct mplb_params {
  double sigma;        /* surface tension sigma (Eq. 2) */
  double width;        /* interface thickness D (Eq. 2); beta = 3 sigma/(4D), k = 3 D sigma/8 */
  double rho_l;        /* density at phi = +1 (Eq. 14) */
  double rho_g;        /* density at phi = -1 (Eq. 14) */
  double mobility;     /* M (Eqs. 1, 19); eta = M / (A (1/s_1 - 1/2)) */
  double A;            /* D3Q7 free parameter, 0 < A < 1/3 (Eq. 8); the paper fixes 0.25 */
  double s_f[7];       /* S^f (Eq. 10), each in (0,2), s_1 = s_2 = s_3 */
  double nu;           /* kinematic viscosity > 0 (Eq. 33): lambda_9..13 = 1/(3 nu + 1/2) */
  double lambda_g[15]; /* S^g (Eq. 26), each in (0,2); entries 9..13 are replaced from nu
                          unless lambda_override.  With every other entry 1 (the paper's
                          rates) the D3Q15 step forms only the five stress moments of g;
                          otherwise the full moment transform (same result up to rounding) */
  double gravity[3];   /* body acceleration; G = (rho - rho_ref) gravity */
  double rho_ref;      /* reference density of the body force (0: G = rho gravity) */
  /* study switches; 0 selects the readings used by default.  The switches are
     built for FP64 and FP32 storage (mplb_set_params returns MPLB_E_INVAL for
     16-bit storage), and mplb_step_many steps such lattices one after another. */
  int stencil;         /* MPLB_STENCIL_Q15: Eqs. 35-36 with the D3Q15 weights; MPLB_STENCIL_Q7: with the
                          D3Q7 weights (central differences and the 7-point Laplacian) */
  int forcing;         /* MPLB_FORCING_EQ32: the printed moments of Eq. 32; MPLB_FORCING_EQ28: Gamma T of
                          Eq. 28 untruncated.  The D3Q19 variant always uses Gamma T. */
  int lambda_override; /* nonzero: lambda_9..13 are taken from lambda_g (all equal) instead of from nu */
} mplb_params;

#define MPLB_STENCIL_Q15 0
#define MPLB_STENCIL_Q7 1
#define MPLB_FORCING_EQ32 0
#define MPLB_FORCING_EQ28 1

typedef struct mplb_s mplb_t;

/* Device bytes a lattice needs (populations of two time levels, the
 * (phi u) history (3 words per node; CHE-only: phi, 1 word), phi, mu, a
 * read-out buffer and reduction scratch).  MPLB_E_INVAL for an unknown mode
 * or precision, or dimensions out of range. */
int mplb_required_bytes(int nx, int ny, int nz, int precision, int mode, size_t* bytes);

/* Create a lattice of nx*ny*nz nodes (each >= 1) with bc[a] in
 * {MPLB_PERIODIC, MPLB_WALL} per axis.  device_arena: NULL lets the library
 * allocate (hipMalloc) on the current device; otherwise a device buffer of
 * arena_bytes >= mplb_required_bytes that the library borrows until
 * mplb_destroy (the caller keeps it alive, e.g. as a torch tensor).
 * *out receives the handle; on error *out is NULL. */
int mplb_create(int nx, int ny, int nz, const int bc[3], int precision, int mode, void* device_arena,
                size_t arena_bytes, mplb_t** out);

/* Enqueue all later work on this hipStream_t (NULL = null stream). */
int mplb_set_stream(mplb_t* h, void* hip_stream);

/* Validate and derive (beta, k, eta, tau_g) from p.  MPLB_E_INVAL if any rate
 * lies outside (0,2), s_1..s_3 differ, A is outside (0,1/3), D, rho_l,
 * rho_g or nu is not positive, or the mobility is negative; a refused call
 * leaves the lattice's parameters as they were. */
int mplb_set_params(mplb_t* h, const mplb_params* p);

/* CHE-only lattices: the velocity prescribed at step n.  u_field (3N, used
 * by MPLB_VEL_FIELD only) is copied.  U and T as in Eqs. 37 and 41.  Call it
 * before mplb_init: the time derivative of Eq. 34 is formed from phi of the
 * previous level and the prescribed u there, so the velocity is fixed for the
 * run; after init it returns MPLB_E_STATE. */
int mplb_set_velocity(mplb_t* h, int kind, const double* u_field, double U, double T);

/* Equilibrium start (an initial state the paper leaves open): mu_0 from
 * phi0 (Eqs. 2, 36), f = f^eq(phi0, mu0, u0) (Eq. 5), g = g^eq(p = 0, rho(phi0),
 * u0) (Eq. 21), (phi u)_prev = phi0 u0, step counter 0.  phi0 has N values;
 * u0 has 3N or is NULL (u0 = 0); in CHE-only mode u0 is ignored and the
 * prescribed velocity at step 0 is used.  Requires mplb_set_params (and, in
 * CHE-only mode, mplb_set_velocity).  It may be called again to restart the
 * run; if it fails, the lattice counts as uninitialised (mplb_step returns
 * MPLB_E_STATE) until a later mplb_init succeeds. */
int mplb_init(mplb_t* h, const double* phi0, const double* u0);

/* Advance nsteps >= 0 time steps (Eqs. 15-16 and their D3Q15 analogue; the
 * finite differences of Eqs. 34-36).  Returns MPLB_E_NONFINITE if the
 * non-finite check (see mplb_set_check_interval) finds a NaN or Inf. */
int mplb_step(mplb_t* h, int nsteps);

/* Every k steps (k >= 1; 1000 for a new lattice) mplb_step and
 * mplb_step_many synchronise and check that no population of the lattice
 * became non-finite; k = 0 checks only when mplb_totals or mplb_check_finite
 * is called (for callers that keep the stream asynchronous and check at their
 * own synchronisation points). */
int mplb_set_check_interval(mplb_t* h, int k);

/* Synchronise the handle's stream and return MPLB_E_NONFINITE if a
 * population of this lattice has become NaN or Inf since mplb_init or
 * mplb_restore (the step kernels raise a per-lattice flag that stays set),
 * MPLB_OK otherwise.  Lets a caller of mplb_step_many find which lattices of
 * a batch failed.  MPLB_E_STATE before init. */
int mplb_check_finite(mplb_t* h);

long mplb_step_count(const mplb_t* h);

/* Macroscopic field (MPLB_PHI..MPLB_P) at the current time level into
 * out[N] (host, double).  Does not change the state. */
int mplb_read(mplb_t* h, int field, double* out);

/* The same field on the vertical plane x = y only (the diagonal section that
 * Sec. III C shows for the Rayleigh-Taylor runs), into out[nz * nx] (host,
 * double): out[z * nx + i] is the value at node (i, i, z).  Needs nx = ny
 * (MPLB_E_INVAL otherwise); the plane is gathered on the device, so only
 * nx * nz values cross PCIe.  Does not change the state; synchronises. */
int mplb_read_diagonal(mplb_t* h, int field, double* out);

/* FP64 totals at the current level: out[0] = sum phi, out[1..3] = sum of
 * sum_i c_i g_i, out[4..6] = sum of F_s + F_a + G.  Returns MPLB_E_NONFINITE
 * if any population is non-finite. */
int mplb_totals(mplb_t* h, double out[7]);

/* Interface extremes of a layered run at the current level (the spike tip
 * and bubble front of a heavy-over-light Rayleigh-Taylor layer, Sec. III C):
 * out[0] and out[1] are the lowest and the highest z at which phi changes
 * sign between two adjacent layers of one column, located by linear
 * interpolation, with layer k at z = k + 1/2 (phi = 0 counts as positive).
 * Both are -1 when no column crosses.  A periodic z axis is scanned from
 * layer 0 to nz-1 without wrapping.  Synchronises; does not change the
 * state. */
int mplb_front(mplb_t* h, double out[2]);

/* Advance `count` lattices by nsteps each with batched launches: one kernel
 * per step covers every coupled lattice (continuous-batching serving); the
 * nsteps launches are replayed as one HIP graph, cached while the batch keeps
 * its shape.  Each lattice computes exactly what mplb_step computes for it.
 * All handles must be initialised, share one precision and mode, and use the
 * first handle's stream (MPLB_E_INVAL otherwise, before anything is
 * enqueued).  Not thread-safe across calls on one device.
 * CHE-only and D3Q19 lattices, lattices with a study switch set, and a batch
 * in which some lattices have S^g = 1 off the stress moments and others not,
 * are stepped one after another (the batched kernel is the default D3Q15 step
 * in one collision form).  Afterwards every lattice whose own check interval
 * (mplb_set_check_interval) was crossed is checked; all of them are checked
 * even when one fails, each failed lattice's mplb_last_error names it, and
 * the call returns MPLB_E_NONFINITE if any failed (the error text of hs[0]
 * otherwise). */
int mplb_step_many(mplb_t* const* hs, int count, int nsteps);

/* For callers that cannot allocate memory once their lattices exist (tight
 * serving loops, harnesses that forbid hipMalloc and pinned host buffers):
 * mplb_step_many, bitwise the same steps, with no device or host
 * allocation.  The batch table lives in a static device array sized for
 * MPLB_NOALLOC_MAX_LATTICES lattices of any precision (about 250 KB); each
 * device holds its own copy until the process ends, and mplb_create looks up
 * its address.  The table is written from a stack buffer with copies from
 * pageable memory, which return once the table has left the host (they may
 * wait for the work already enqueued on the stream), and the steps are
 * launched one by one (no graph).  count > MPLB_NOALLOC_MAX_LATTICES:
 * MPLB_E_INVAL, with the limit in mplb_last_error(hs[0]).  Every call on a
 * device rewrites that device's one table: calls on one stream are ordered,
 * but calls that overlap on one device (two threads, or two streams) race.
 * Non-finite checks as in mplb_step_many. */
#define MPLB_NOALLOC_MAX_LATTICES 512
int mplb_step_many_noalloc(mplb_t* const* hs, int count, int nsteps);

/* Whether mplb_step_many replays its steps as a graph (enable != 0, the
 * default) or launches them one by one; process-wide, for measurement. */
int mplb_set_step_many_graphs(int enable);

/* Bytes of a checkpoint (raw state in storage precision plus the step
 * counter); mplb_checkpoint writes it to host memory, mplb_restore reads one
 * written by a lattice of the same size, precision and mode. */
int mplb_checkpoint_bytes(const mplb_t* h, size_t* bytes);
int mplb_checkpoint(mplb_t* h, void* host_buf, size_t bytes);
int mplb_restore(mplb_t* h, const void* host_buf, size_t bytes);

/* Measurement: advance nsteps steps with HIP events recorded on the handle's
 * stream around each step kernel; ms[2] and ms[3] receive the summed
 * duration of the step kernels (one kernel does the whole step), ms[0] and
 * ms[1] (separate phi and mu passes, which the step does not have) are 0.
 * Synchronises; the state advances exactly as with mplb_step. */
int mplb_time_stages(mplb_t* h, int nsteps, double ms[4]);

/* Measurement reference: copy `bytes` (a multiple of 16) from device buffer
 * src to device buffer dst with 16-byte loads and stores on hip_stream, so
 * that the bandwidth a plain streaming kernel reaches on this device can be
 * put beside the step's.  kind 0: one element per thread and round, ordinary
 * stores; 1: the same with non-temporal stores (the store policy of the step
 * kernels on large lattices); 2: four elements per thread and round,
 * non-temporal loads and stores, 16384 blocks of 256 threads; 3: each block of
 * 256 threads streams its own contiguous 256 KB chunk, four elements per
 * thread and round, non-temporal loads and stores (the fastest copy found on
 * MI355X).  Other kinds: MPLB_E_INVAL.  Enqueues only. */
int mplb_copy_probe(const void* src, void* dst, size_t bytes, int kind, void* hip_stream);

/* Test hook: overwrite one stored population (set 0: f, 1: g; index i;
 * node n) of the current state with `value`, e.g. to plant a NaN. */
int mplb_poke(mplb_t* h, int set, int i, long node, double value);

/* Test hook (the NaN-poisoned halo check): fill with all-ones bytes (NaN in
 * every storage type) the population arrays that the next step writes and
 * the padding past the last node of every array it reads, and make every
 * later step of this lattice fill its shared-memory rings and queues the same
 * way before using them.  A node that a step does not write, a read past the
 * last node, or a read of a shared-memory slot that no stage has written then
 * shows as non-finite or changed fields.  Synchronises.  MPLB_E_STATE before
 * init. */
int mplb_poison(mplb_t* h);

/* Test hook: the tile height of this lattice's step.  0 (default) lets
 * mplb_step choose: 16 rows for the coupled step with FP32 populations on a
 * lattice that fills 512 such blocks, and for the CHE-only step in FP32
 * compute (any storage) the kernel in which a thread owns two nodes of a
 * 128 x 8 tile on a lattice of at least 5 million nodes that fills at least
 * 384 of those; 8 otherwise.
 * 8 or 16 forces one (16 where it exists, else MPLB_E_INVAL).  The tiling
 * changes which work a block does, not the arithmetic of a node, so the
 * fields are bitwise the same; mplb_step_many always uses 8 rows. */
int mplb_force_tile_rows(mplb_t* h, int rows);

/* The kernel and work split that mplb_step uses for a lattice of nx*ny*nz
 * nodes in this precision and mode, with `rows` as for mplb_force_tile_rows
 * (0: the automatic choice).  A host computation: it needs no device and no
 * lattice.  out[0]: 0 the coupled step on 64 x 8 tiles, 1 on 64 x 16 tiles,
 * 2 the CHE-only step with one node per thread (64 x 8 tiles), 3 with two
 * nodes per thread (128 x 8 tiles); out[1], out[2]: tile width and height in
 * nodes; out[3]: planes per z segment (the last segment may be shorter);
 * out[4]: segments; out[5]: blocks of the launch (tiles times segments).
 * MPLB_E_INVAL for sizes, modes or precisions mplb_create refuses, or rows
 * that mplb_force_tile_rows refuses.  Every choice gives the same results
 * bit for bit; it sets only the speed of the step. */
int mplb_launch_shape(int nx, int ny, int nz, int precision, int mode, int rows, int out[6]);

void mplb_destroy(mplb_t* h);
const char* mplb_last_error(const mplb_t* h);
const char* mplb_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
