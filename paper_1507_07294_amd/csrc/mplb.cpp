// Host side of libmplb: the C-ABI declared in include/mplb.h.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "launch.h"
#include "mplb.h"

using namespace mplb;

namespace {

struct Plan {
  size_t pitch;  // elements per population array
  size_t f, g, phiu, phi, mu, ufield, out, red, flag, total;
};

size_t comp_size(int prec) { return prec == MPLB_F64 ? 8 : 4; }
size_t store0_size(int prec) { return prec == MPLB_F64 ? 8 : 4; }
size_t store_size(int prec) { return prec == MPLB_F64 ? 8 : (prec == MPLB_F32 ? 4 : 2); }

// Population arrays sit `pitch` elements apart.  A lattice of 2^k nodes
// would put every array at a power-of-two distance from the others, so the
// 50 streams a node reads and writes would all start on the same HBM channel
// bits; 27 x 256 extra elements break that alignment (measured on the
// 256 x 256 x 1024 box: 3.08 -> ~2.9 ms per FP32 step).
constexpr size_t kPitchPad = 27 * 256;

Plan make_plan(long long N, int prec, int mode) {
  Plan p{};
  p.pitch = align_up((size_t)N, 256) + kPitchPad;
  const size_t A = 256;
  size_t sT = comp_size(prec), s0 = store0_size(prec), sS = store_size(prec);
  // 16-bit populations of the coupled model: f_i and g_i (i = 1..6) share
  // 32-bit words in the f buffer; the g buffer keeps g_0 and g_7..g_{q-1}
  // (the 8 corners of D3Q15, the 12 edges of D3Q19)
  bool pack = mode != MPLB_CHE_ONLY && sS == 2;
  const int q = mode == MPLB_COUPLED_Q19 ? 19 : 15;  // NSE lattice
  p.f = align_up(p.pitch * s0 + 6 * p.pitch * (pack ? 4 : sS), A);
  p.g = mode != MPLB_CHE_ONLY ? align_up((pack ? q - 6 : q) * p.pitch * sS, A) : 0;
  // (phi u) history: 3 words (coupled); phi alone where u is prescribed
  p.phiu = align_up((mode != MPLB_CHE_ONLY ? 3 : 1) * p.pitch * sT, A);
  p.phi = align_up(p.pitch * sT, A);
  p.mu = align_up(p.pitch * sT, A);
  p.ufield = mode == MPLB_CHE_ONLY ? align_up(3 * p.pitch * sT, A) : 0;
  p.out = align_up(p.pitch * 8, A);
  p.red = align_up(((size_t)kRedSlots * 8 + 8) * 8, A);
  p.flag = A;
  p.total = 2 * p.f + 2 * p.g + p.phiu + p.phi + p.mu + p.ufield + p.out + p.red + p.flag;
  return p;
}

// modes and the precisions each supports
bool valid_mode(int mode, int precision) {
  if (precision < MPLB_F64 || precision > MPLB_F32_BF16) return false;
  return mode == MPLB_COUPLED || mode == MPLB_CHE_ONLY || mode == MPLB_COUPLED_Q19;
}

// The kernels index nodes and population arrays in 32 bits: the padded
// pitch between arrays (which bounds every node index, and the read-out
// grids' last index) must fit an int, and the step kernel forms in-plane
// byte offsets in 32 bits (nx*ny elements of up to 8 bytes).  The limit is
// derived from the pitch itself, so that it follows the padding.
bool valid_dims(int nx, int ny, int nz) {
  if (nx < 1 || ny < 1 || nz < 1) return false;
  long long N = (long long)nx * ny * nz;
  long long pitch = (long long)align_up((size_t)N, 256) + (long long)kPitchPad;
  return pitch <= (long long)INT_MAX && (long long)nx * ny * 8 < (1LL << 32);
}

const uint64_t kMagic = 0x31303531504c424dULL;  // checkpoint tag

// Steps between non-finite checks of a new lattice: a check is one 4-byte
// copy and a synchronisation, which every 1000 steps costs well under 0.1 %.
constexpr int kDefaultCheckInterval = 1000;

struct CkptHeader {
  uint64_t magic;
  int32_t nx, ny, nz, prec, mode, pad;
  int64_t step;
  uint64_t f_bytes, g_bytes, phiu_bytes;
};

}  // namespace

struct mplb_s {
  Geo G{};
  int prec = 0, mode = 0;
  int bc[3] = {0, 0, 0};
  Plan plan{};
  hipStream_t stream = nullptr;
  void* arena = nullptr;
  bool own_arena = false;
  Bufs B{};
  int cur = 0;
  long step = 0;
  bool have_params = false, have_init = false;
  Coef<double> C{};
  double velT = 1.0;
  int check_interval = kDefaultCheckInterval;
  int tile_rows = 0;  // mplb_force_tile_rows (0: automatic)
  std::string err;
};

static int fail(mplb_t* h, int code, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return code;
}

#define HIPCHK(h, expr)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(h, MPLB_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" {

const char* mplb_strerror(int code) {
  switch (code) {
    case MPLB_OK: return "ok";
    case MPLB_E_INVAL: return "invalid argument";
    case MPLB_E_NOMEM: return "out of device memory or arena too small";
    case MPLB_E_DEVICE: return "HIP error";
    case MPLB_E_STATE: return "call out of order";
    case MPLB_E_NONFINITE: return "non-finite population";
    default: return "unknown error";
  }
}

const char* mplb_last_error(const mplb_t* h) { return h ? h->err.c_str() : "null handle"; }

int mplb_required_bytes(int nx, int ny, int nz, int precision, int mode, size_t* bytes) {
  if (!bytes || !valid_dims(nx, ny, nz) || !valid_mode(mode, precision)) return MPLB_E_INVAL;
  *bytes = make_plan((long long)nx * ny * nz, precision, mode).total;
  return MPLB_OK;
}

int mplb_create(int nx, int ny, int nz, const int bc[3], int precision, int mode, void* device_arena,
                size_t arena_bytes, mplb_t** out) {
  if (!out) return MPLB_E_INVAL;
  *out = nullptr;
  if (!bc || !valid_dims(nx, ny, nz) || !valid_mode(mode, precision)) return MPLB_E_INVAL;
  for (int a = 0; a < 3; ++a)
    if (bc[a] != MPLB_PERIODIC && bc[a] != MPLB_WALL) return MPLB_E_INVAL;
  mplb_t* h = new (std::nothrow) mplb_t();
  if (!h) return MPLB_E_NOMEM;
  h->prec = precision;
  h->mode = mode;
  for (int a = 0; a < 3; ++a) h->bc[a] = bc[a];
  h->G.nx = nx; h->G.ny = ny; h->G.nz = nz;
  h->G.wall_x = bc[0] == MPLB_WALL; h->G.wall_y = bc[1] == MPLB_WALL; h->G.wall_z = bc[2] == MPLB_WALL;
  h->G.N = nx * ny * nz;
  h->plan = make_plan(h->G.N, precision, mode);
  h->G.pitch = (int)h->plan.pitch;
  if (device_arena) {
    if (arena_bytes < h->plan.total || ((uintptr_t)device_arena & 255)) {
      delete h;
      return MPLB_E_NOMEM;
    }
    h->arena = device_arena;
  } else {
    if (hipMalloc(&h->arena, h->plan.total) != hipSuccess) {
      (void)hipGetLastError();
      delete h;
      return MPLB_E_NOMEM;
    }
    h->own_arena = true;
  }
  char* p = (char*)h->arena;
  const Plan& P = h->plan;
  h->B.f[0] = p; p += P.f;
  h->B.f[1] = p; p += P.f;
  h->B.g[0] = P.g ? p : nullptr; p += P.g;
  h->B.g[1] = P.g ? p : nullptr; p += P.g;
  h->B.phiu = p; p += P.phiu;
  h->B.phi = p; p += P.phi;
  h->B.mu = p; p += P.mu;
  h->B.ufield = P.ufield ? p : nullptr; p += P.ufield;
  h->B.out = (double*)p; p += P.out;
  h->B.red = (double*)p; p += P.red;
  h->B.flag = (int*)p; p += P.flag;
  h->C.vel_kind = MPLB_VEL_ZERO;
  h->C.vel_ct = h->C.vel_ct_prev = 1.0;
  // set-up of mplb_step_many_noalloc on this device (its table's address)
  int dev = 0;
  void* tab = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || noalloc_table(dev, &tab) != hipSuccess) {
    (void)hipGetLastError();
    mplb_destroy(h);
    return MPLB_E_DEVICE;
  }
  *out = h;
  return MPLB_OK;
}

void mplb_destroy(mplb_t* h) {
  if (!h) return;
  if (h->own_arena && h->arena) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->arena);
  }
  delete h;
}

int mplb_set_stream(mplb_t* h, void* s) {
  if (!h) return MPLB_E_INVAL;
  h->stream = (hipStream_t)s;
  return MPLB_OK;
}

int mplb_set_check_interval(mplb_t* h, int k) {
  if (!h || k < 0) return MPLB_E_INVAL;
  h->check_interval = k;
  return MPLB_OK;
}

long mplb_step_count(const mplb_t* h) { return h ? h->step : -1; }

int mplb_set_params(mplb_t* h, const mplb_params* p) {
  if (!h || !p) return MPLB_E_INVAL;
  auto in02 = [](double v) { return v > 0.0 && v < 2.0; };
  if (!(p->A > 0.0 && p->A < 1.0 / 3.0)) return fail(h, MPLB_E_INVAL, "A must lie in (0, 1/3)");
  if (!(p->width > 0.0) || !(p->rho_l > 0.0) || !(p->rho_g > 0.0) || !(p->nu > 0.0) || !(p->mobility >= 0.0) ||
      !std::isfinite(p->sigma))
    return fail(h, MPLB_E_INVAL, "D, rho_l, rho_g and nu must be positive, the mobility non-negative");
  for (int i = 0; i < 7; ++i)
    if (!in02(p->s_f[i])) return fail(h, MPLB_E_INVAL, "s_f[%d] outside (0,2)", i);
  if (p->s_f[1] != p->s_f[2] || p->s_f[1] != p->s_f[3]) return fail(h, MPLB_E_INVAL, "s_1, s_2, s_3 must be equal");
  // formed in a copy and committed only once every check has passed, so a
  // refused call leaves the lattice's parameters as they were
  Coef<double> C = h->C;
  C.rho_l = p->rho_l;
  C.rho_g = p->rho_g;
  C.drho = p->rho_l - p->rho_g;
  C.beta = 3.0 * p->sigma / (4.0 * p->width);  // after Eq. 2
  C.kappa = 3.0 * p->width * p->sigma / 8.0;
  C.A = p->A;
  double tau_f = 1.0 / p->s_f[1];
  C.eta = p->mobility / (p->A * (tau_f - 0.5));  // Eq. 19 with c_s^2 = A
  C.mob = p->mobility;
  C.rho_ref = p->rho_ref;
  for (int a = 0; a < 3; ++a) C.grav[a] = p->gravity[a];
  for (int i = 0; i < 7; ++i) C.sf[i] = p->s_f[i];
  if ((p->stencil != MPLB_STENCIL_Q15 && p->stencil != MPLB_STENCIL_Q7) ||
      (p->forcing != MPLB_FORCING_EQ32 && p->forcing != MPLB_FORCING_EQ28))
    return fail(h, MPLB_E_INVAL, "unknown stencil or forcing switch");
  C.stencil7 = p->stencil == MPLB_STENCIL_Q7;
  C.forcing28 = p->forcing == MPLB_FORCING_EQ28;
  if ((C.stencil7 || C.forcing28) && h->prec != MPLB_F64 && h->prec != MPLB_F32)
    return fail(h, MPLB_E_INVAL, "the stencil and forcing switches are built for FP64 and FP32 storage");
  double tau_g = 3.0 * p->nu + 0.5;  // Eq. 33 with c_s^2 = 1/3
  if (p->lambda_override) {          // the viscous rate itself is given
    for (int i = 10; i <= 13; ++i)
      if (p->lambda_g[i] != p->lambda_g[9]) return fail(h, MPLB_E_INVAL, "lambda_9..13 must be equal");
    if (!in02(p->lambda_g[9])) return fail(h, MPLB_E_INVAL, "lambda[9] outside (0,2)");
    tau_g = 1.0 / p->lambda_g[9];
  }
  for (int i = 0; i < 15; ++i) C.lg[i] = (i >= 9 && i <= 13) ? 1.0 / tau_g : p->lambda_g[i];
  for (int i = 0; i < 15; ++i)
    if (!in02(C.lg[i])) return fail(h, MPLB_E_INVAL, "lambda[%d] outside (0,2)", i);
  C.unit_rates = 1;
  for (int i = 0; i < 15; ++i)
    if ((i < 9 || i > 13) && C.lg[i] != 1.0) C.unit_rates = 0;
  h->C = C;
  h->have_params = true;
  return MPLB_OK;
}

static int upload_field(mplb_t* h, const double* src, void* dst) {
  HIPCHK(h, hipMemcpyAsync(h->B.out, src, (size_t)h->G.N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, launch_cvt_in(h->prec, h->G, h->B, dst, h->stream));
  return MPLB_OK;
}

int mplb_set_velocity(mplb_t* h, int kind, const double* u_field, double U, double T) {
  if (!h) return MPLB_E_INVAL;
  if (h->mode != MPLB_CHE_ONLY) return fail(h, MPLB_E_STATE, "prescribed velocity needs a CHE-only lattice");
  if (h->have_init)  // the history holds phi only and relies on u at the previous level being known
    return fail(h, MPLB_E_STATE, "set_velocity after init");
  if (kind < MPLB_VEL_ZERO || kind > MPLB_VEL_DEFORM || (kind == MPLB_VEL_FIELD && !u_field) ||
      (kind == MPLB_VEL_DEFORM && !(T > 0.0)) || !std::isfinite(U))
    return fail(h, MPLB_E_INVAL, "invalid velocity specification");
  if (kind == MPLB_VEL_FIELD) {
    size_t sT = comp_size(h->prec);
    for (int a = 0; a < 3; ++a) {
      int rc = upload_field(h, u_field + (size_t)a * h->G.N, (char*)h->B.ufield + (size_t)a * h->G.pitch * sT);
      if (rc) return rc;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  h->C.vel_kind = kind;
  h->C.velU = U;
  h->velT = T;
  return MPLB_OK;
}

// cos(pi t / T) of the deformation flow at step n, t = n U / nx
static double deform_ct(const mplb_t* h, long n) {
  const double pi = 3.14159265358979323846;
  double t = (double)n * h->C.velU / h->G.nx;
  return std::cos(pi * t / h->velT);
}

// Time factors of the prescribed velocity for the step that starts at level
// h->step: the current level and the previous one (level 0 at the first step,
// where the history is phi_0 u_0).
static void set_vel_time(mplb_t* h) {
  if (h->mode != MPLB_CHE_ONLY || h->C.vel_kind != MPLB_VEL_DEFORM) return;
  h->C.vel_ct = deform_ct(h, h->step);
  h->C.vel_ct_prev = deform_ct(h, h->step > 0 ? h->step - 1 : 0);
}

int mplb_init(mplb_t* h, const double* phi0, const double* u0) {
  if (!h || !phi0) return MPLB_E_INVAL;
  if (!h->have_params) return fail(h, MPLB_E_STATE, "init before set_params");
  // the state is overwritten from here on: a failure below leaves the
  // lattice uninitialised rather than half of two states
  h->have_init = false;
  size_t sT = comp_size(h->prec);
  int rc = upload_field(h, phi0, h->B.phi);
  if (rc) return rc;
  if (h->mode != MPLB_CHE_ONLY) {
    for (int a = 0; a < 3; ++a) {
      void* dst = (char*)h->B.phiu + (size_t)a * h->G.pitch * sT;
      if (u0) {
        rc = upload_field(h, u0 + (size_t)a * h->G.N, dst);
        if (rc) return rc;
      } else {
        HIPCHK(h, launch_fill_zero(h->prec, dst, h->G.N, h->stream));
      }
    }
  }
  HIPCHK(h, launch_mu(h->prec, h->G, h->C, h->B, h->stream));
  h->C.vel_ct = h->C.vel_ct_prev = 1.0;
  h->cur = 0;
  HIPCHK(h, launch_init(h->prec, h->mode, h->G, h->C, h->B, h->cur, h->stream));
  HIPCHK(h, launch_fill_int(h->B.flag, 0, 1, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->step = 0;
  h->have_init = true;
  return MPLB_OK;
}

static int check_flag(mplb_t* h) {
  int flag = 0;
  HIPCHK(h, hipMemcpyAsync(&flag, h->B.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (flag) return fail(h, MPLB_E_NONFINITE, "non-finite population after step %ld", h->step);
  return MPLB_OK;
}

// Enqueue one step of lattice h on stream s.
static int enqueue_step(mplb_t* h, hipStream_t s) {
  set_vel_time(h);
  HIPCHK(h, launch_fused_step(h->prec, h->mode, h->G, h->C, h->B, h->cur, s, h->tile_rows));
  h->cur = 1 - h->cur;
  h->step++;
  return MPLB_OK;
}

int mplb_step(mplb_t* h, int nsteps) {
  if (!h || nsteps < 0) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "step before init");
  for (int k = 0; k < nsteps; ++k) {
    int rc = enqueue_step(h, h->stream);
    if (rc) return rc;
    if (h->check_interval > 0 && h->step % h->check_interval == 0) {
      rc = check_flag(h);
      if (rc) return rc;
    }
  }
  return MPLB_OK;
}

int mplb_time_stages(mplb_t* h, int nsteps, double ms[4]) {
  if (!h || !ms || nsteps < 0) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "step before init");
  for (int k = 0; k < 4; ++k) ms[k] = 0.0;
  // one kernel does the whole step: events around it, none for the separate
  // phi and mu passes that the step no longer has (their entries stay 0)
  std::vector<hipEvent_t> ev;
  ev.reserve(2 * (size_t)nsteps);
  int rc = MPLB_OK;
  for (size_t k = 0; k < 2 * (size_t)nsteps && rc == MPLB_OK; ++k) {
    hipEvent_t e = nullptr;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) rc = fail(h, MPLB_E_DEVICE, "time_stages: %s", hipGetErrorString(err));
    else ev.push_back(e);
  }
  for (int k = 0; k < nsteps && rc == MPLB_OK; ++k) {
    hipEvent_t* e = &ev[2 * (size_t)k];
    set_vel_time(h);
    hipError_t err = hipEventRecord(e[0], h->stream);
    if (err == hipSuccess)
      err = launch_fused_step(h->prec, h->mode, h->G, h->C, h->B, h->cur, h->stream, h->tile_rows);
    if (err == hipSuccess) err = hipEventRecord(e[1], h->stream);
    if (err != hipSuccess) rc = fail(h, MPLB_E_DEVICE, "time_stages: %s", hipGetErrorString(err));
    h->cur = 1 - h->cur;
    h->step++;
  }
  if (rc == MPLB_OK) {
    hipError_t err = hipStreamSynchronize(h->stream);
    if (err != hipSuccess) rc = fail(h, MPLB_E_DEVICE, "time_stages: %s", hipGetErrorString(err));
  }
  for (int k = 0; k < nsteps && rc == MPLB_OK; ++k) {
    float c = 0;
    (void)hipEventElapsedTime(&c, ev[2 * (size_t)k], ev[2 * (size_t)k + 1]);
    ms[2] += c;
  }
  ms[3] = ms[2];
  for (auto& e : ev) (void)hipEventDestroy(e);
  return rc;
}

// Instantiated graph of a chunk of batched steps, reused while the batch
// keeps its shape (precision, walls, collision form, item count, block count,
// steps, table).
struct ChunkGraph {
  int prec = -1, xywall = 0, nt = 0, unit = 0, count = 0, blocks = 0, nsteps = 0;
  const void* table = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long used = 0;
};
constexpr int kGraphCache = 4;
// An evicted graph is never one that may still be executing: before a chunk
// is built or looked up, mplb_step_many waits on the host for the previous
// chunk's table upload, which follows every earlier chunk in stream order.
// So only the most recently used graph can still run, and the
// least-recently-used eviction never picks it.
static_assert(kGraphCache >= 2, "the running chunk's graph must survive one eviction");

// Device table of a batched step and its pinned host staging (grow-only,
// one per device; batched calls on one device are not thread-safe).
struct BatchTable {
  void* dev = nullptr;
  size_t dev_cap = 0;
  void* host = nullptr;
  size_t host_cap = 0;
  hipEvent_t uploaded = nullptr;  // host staging consumed
  hipEvent_t done = nullptr;      // last launches that read the device table
  ChunkGraph graphs[kGraphCache];
  unsigned long long clock = 0;
};
static BatchTable g_tables[64];
static bool g_use_graphs = true;

int mplb_set_step_many_graphs(int enable) {
  g_use_graphs = enable != 0;
  return MPLB_OK;
}

// The cached graph for this chunk shape, built and instantiated on a miss
// (replacing the least recently used entry).
static int chunk_graph(mplb_t* h0, BatchTable& T, bool xywall, bool nt, bool unit, int count, int blocks,
                       int nsteps, hipGraphExec_t* out) {
  ChunkGraph* slot = nullptr;
  for (auto& c : T.graphs)
    if (c.exec && c.prec == h0->prec && c.xywall == (int)xywall && c.nt == (int)nt && c.unit == (int)unit &&
        c.count == count &&
        c.blocks == blocks &&
        c.nsteps == nsteps && c.table == T.dev)
      slot = &c;
  if (!slot) {
    slot = &T.graphs[0];
    for (auto& c : T.graphs)
      if (!c.exec || c.used < slot->used) slot = &c;
    if (slot->exec) HIPCHK(h0, hipGraphExecDestroy(slot->exec));
    slot->exec = nullptr;
    hipGraph_t g = nullptr;
    HIPCHK(h0, build_fused_many_graph(h0->prec, xywall, nt, unit, T.dev, count, blocks, nsteps, &g));
    hipError_t e = hipGraphInstantiate(&slot->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      slot->exec = nullptr;
      return fail(h0, MPLB_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    slot->prec = h0->prec;
    slot->xywall = xywall;
    slot->nt = nt;
    slot->unit = unit;
    slot->count = count;
    slot->blocks = blocks;
    slot->nsteps = nsteps;
    slot->table = T.dev;
  }
  slot->used = ++T.clock;
  *out = slot->exec;
  return MPLB_OK;
}

// After every lattice of a batch advanced nsteps: check each lattice whose
// own check interval was crossed, as mplb_step does.  Every such lattice is
// checked (one failure does not hide another); each failed lattice keeps its
// message, and the result is MPLB_E_NONFINITE if any failed.
static int check_after(mplb_t* const* hs, int count, int nsteps) {
  int rc = MPLB_OK;
  for (int i = 0; i < count; ++i) {
    mplb_t* h = hs[i];
    const long k = h->check_interval;
    if (k <= 0 || h->step / k == (h->step - nsteps) / k) continue;
    int r = check_flag(h);
    if (r == MPLB_E_NONFINITE) rc = r;
    else if (r) return r;
  }
  return rc;
}

// Upload of a batch table without allocating: items are written into a stack
// buffer and copied in pieces.  The copies are from pageable memory, so each
// returns only once its bytes have left the buffer.
static int upload_table_noalloc(mplb_t* const* hs, int count, void* dtab, hipStream_t s, int* blocks_out) {
  mplb_t* h0 = hs[0];
  const size_t item = fused_batch_item_bytes(h0->prec);
  alignas(64) unsigned char stage[16384];
  const int per = (int)(sizeof stage / item);
  if (per < 1) return fail(h0, MPLB_E_INVAL, "batch item larger than its staging");
  int blocks = 0;
  for (int first = 0; first < count; first += per) {
    const int n = count - first < per ? count - first : per;
    for (int j = 0; j < n; ++j) {
      mplb_t* h = hs[first + j];
      int nb = fused_batch_fill(h->prec, stage, j, h->G, h->C, h->B, h->cur, blocks);
      if (nb <= 0) return fail(h0, MPLB_E_INVAL, "bad batch item");
      blocks += nb;
    }
    HIPCHK(h0, hipMemcpyAsync((char*)dtab + (size_t)first * item, stage, (size_t)n * item, hipMemcpyHostToDevice, s));
  }
  *blocks_out = blocks;
  return MPLB_OK;
}

// mplb_step_many and its allocation-free variant.
static int step_many_impl(mplb_t* const* hs, int count, int nsteps, bool noalloc) {
  if (!hs || count < 0 || nsteps < 0) return MPLB_E_INVAL;
  if (count == 0 || nsteps == 0) return MPLB_OK;
  if (noalloc && count > MPLB_NOALLOC_MAX_LATTICES)
    return fail(hs[0], MPLB_E_INVAL, "step_many_noalloc: %d lattices exceed its static table of %d", count,
                MPLB_NOALLOC_MAX_LATTICES);
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) return MPLB_E_INVAL;
    if (!hs[i]->have_init) return fail(hs[i], MPLB_E_STATE, "step before init");
    if (hs[i]->prec != hs[0]->prec || hs[i]->mode != hs[0]->mode)
      return fail(hs[0], MPLB_E_INVAL, "step_many needs one precision and one mode");
    // the steps go to one stream, and each lattice's non-finite check reads
    // its flag on its own stream afterwards: the two must be the same
    if (hs[i]->stream != hs[0]->stream)
      return fail(hs[0], MPLB_E_INVAL, "step_many needs every lattice on the first lattice's stream");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[0], MPLB_E_INVAL, "a lattice appears twice in step_many");
  }
  mplb_t* h0 = hs[0];
  hipStream_t s = h0->stream;
  bool any_switch = false, mixed_rates = false;
  for (int i = 0; i < count; ++i) {
    any_switch = any_switch || hs[i]->C.forcing28 || hs[i]->C.stencil7;
    mixed_rates = mixed_rates || hs[i]->C.unit_rates != h0->C.unit_rates;
  }
  const bool unit = h0->C.unit_rates != 0;
  // CHE-only and D3Q19 lattices, lattices with a study switch, and a batch
  // that mixes unit and other S^g rates (two collision forms) step one after
  // another: the batched kernel is the default D3Q15 step in one form
  if (h0->mode != MPLB_COUPLED || any_switch || mixed_rates) {
    for (int k = 0; k < nsteps; ++k)
      for (int i = 0; i < count; ++i) {
        int rc = enqueue_step(hs[i], s);
        if (rc) return rc;
      }
    return check_after(hs, count, nsteps);
  }
  int dev = 0;
  HIPCHK(h0, hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(h0, MPLB_E_DEVICE, "device index out of range");
  bool xywall = false;
  size_t step_bytes = 0;
  for (int i = 0; i < count; ++i) {
    xywall = xywall || hs[i]->G.wall_x || hs[i]->G.wall_y;
    step_bytes += fused_step_bytes(hs[i]->prec, hs[i]->mode, hs[i]->G.N);
  }
  const bool nt = step_bytes > fused_stream_threshold();
  if (noalloc) {
    void* dtab = nullptr;
    HIPCHK(h0, noalloc_table(dev, &dtab));
    int blocks = 0;
    int rc = upload_table_noalloc(hs, count, dtab, s, &blocks);
    if (rc) return rc;
    for (int k = 0; k < nsteps; ++k)
      HIPCHK(h0, launch_fused_many(h0->prec, xywall, nt, unit, dtab, count, blocks, k & 1, s));
  } else {
    BatchTable& T = g_tables[dev];
    size_t bytes = fused_batch_item_bytes(h0->prec) * (size_t)count;
    if (T.uploaded) HIPCHK(h0, hipEventSynchronize(T.uploaded));  // staging free again
    if (!T.uploaded) HIPCHK(h0, hipEventCreateWithFlags(&T.uploaded, hipEventDisableTiming));
    if (!T.done) HIPCHK(h0, hipEventCreateWithFlags(&T.done, hipEventDisableTiming));
    if (T.host_cap < bytes) {
      if (T.host) HIPCHK(h0, hipHostFree(T.host));
      T.host = nullptr;
      T.host_cap = 0;
      HIPCHK(h0, hipHostMalloc(&T.host, 2 * bytes, hipHostMallocDefault));
      T.host_cap = 2 * bytes;
    }
    if (T.dev_cap < bytes) {
      if (T.dev) {
        HIPCHK(h0, hipDeviceSynchronize());
        HIPCHK(h0, hipFree(T.dev));
      }
      T.dev = nullptr;
      T.dev_cap = 0;
      HIPCHK(h0, hipMalloc(&T.dev, 2 * bytes));
      T.dev_cap = 2 * bytes;
    }
    int blocks = 0;
    for (int i = 0; i < count; ++i) {
      mplb_t* h = hs[i];
      int nb = fused_batch_fill(h->prec, T.host, i, h->G, h->C, h->B, h->cur, blocks);
      if (nb <= 0) return fail(h0, MPLB_E_INVAL, "bad batch item");
      blocks += nb;
    }
    // the previous batched launches (perhaps on another stream) still read the table
    HIPCHK(h0, hipStreamWaitEvent(s, T.done, 0));
    HIPCHK(h0, hipMemcpyAsync(T.dev, T.host, bytes, hipMemcpyHostToDevice, s));
    HIPCHK(h0, hipEventRecord(T.uploaded, s));
    if (g_use_graphs && nsteps > 1) {
      hipGraphExec_t ex = nullptr;
      int rc = chunk_graph(h0, T, xywall, nt, unit, count, blocks, nsteps, &ex);
      if (rc) return rc;
      HIPCHK(h0, hipGraphLaunch(ex, s));
    } else {
      for (int k = 0; k < nsteps; ++k)
        HIPCHK(h0, launch_fused_many(h0->prec, xywall, nt, unit, T.dev, count, blocks, k & 1, s));
    }
    HIPCHK(h0, hipEventRecord(T.done, s));
  }
  for (int i = 0; i < count; ++i) {
    mplb_t* h = hs[i];
    h->step += nsteps;
    if (nsteps & 1) h->cur = 1 - h->cur;
  }
  return check_after(hs, count, nsteps);
}

int mplb_step_many(mplb_t* const* hs, int count, int nsteps) { return step_many_impl(hs, count, nsteps, false); }

int mplb_step_many_noalloc(mplb_t* const* hs, int count, int nsteps) {
  return step_many_impl(hs, count, nsteps, true);
}

int mplb_check_finite(mplb_t* h) {
  if (!h) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "check before init");
  return check_flag(h);
}

static int prepare_macro(mplb_t* h) {
  HIPCHK(h, launch_phi(h->prec, h->mode, h->G, h->B, h->cur, h->stream));
  if (h->mode != MPLB_CHE_ONLY) HIPCHK(h, launch_mu(h->prec, h->G, h->C, h->B, h->stream));
  set_vel_time(h);
  return MPLB_OK;
}

int mplb_read(mplb_t* h, int field, double* out) {
  if (!h || !out || field < MPLB_PHI || field > MPLB_P) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "read before init");
  int rc = prepare_macro(h);
  if (rc) return rc;
  HIPCHK(h, launch_macro(h->prec, h->mode, h->G, h->C, h->B, h->cur, field, h->stream));
  HIPCHK(h, hipMemcpyAsync(out, h->B.out, (size_t)h->G.N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MPLB_OK;
}

int mplb_read_diagonal(mplb_t* h, int field, double* out) {
  if (!h || !out || field < MPLB_PHI || field > MPLB_P) return MPLB_E_INVAL;
  if (h->G.nx != h->G.ny) return fail(h, MPLB_E_INVAL, "the plane x = y needs nx = ny");
  if (!h->have_init) return fail(h, MPLB_E_STATE, "read before init");
  int rc = prepare_macro(h);
  if (rc) return rc;
  HIPCHK(h, launch_macro(h->prec, h->mode, h->G, h->C, h->B, h->cur, field, h->stream));
  const size_t n = (size_t)h->G.nx * h->G.nz;
  const double* src = h->B.out;
  if (h->G.nx > 1) {
    // gathered into the phi array, read-out scratch that every read forms
    // anew (nx * nz doubles fit in its nx * nx * nz compute-precision words)
    if (n * sizeof(double) > h->plan.phi) return fail(h, MPLB_E_INVAL, "plane larger than its staging");
    double* d = (double*)h->B.phi;
    HIPCHK(h, launch_diag(h->B.out, d, h->G.nx, h->G.nz, h->stream));
    src = d;
  }
  HIPCHK(h, hipMemcpyAsync(out, src, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MPLB_OK;
}

int mplb_front(mplb_t* h, double out[2]) {
  if (!h || !out) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "front before init");
  HIPCHK(h, launch_phi(h->prec, h->mode, h->G, h->B, h->cur, h->stream));
  HIPCHK(h, launch_front(h->prec, h->G, h->B, h->stream));
  HIPCHK(h, hipMemcpyAsync(out, h->B.red + (size_t)kRedSlots * 8, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MPLB_OK;
}

int mplb_totals(mplb_t* h, double out[7]) {
  if (!h || !out) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "totals before init");
  int rc = prepare_macro(h);
  if (rc) return rc;
  HIPCHK(h, launch_totals(h->prec, h->mode, h->G, h->C, h->B, h->cur, h->stream));
  double r[8];
  HIPCHK(h, hipMemcpyAsync(r, h->B.red + (size_t)kRedSlots * 8, sizeof r, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int k = 0; k < 7; ++k) out[k] = r[k];
  if (r[7] > 0.0) return fail(h, MPLB_E_NONFINITE, "non-finite population at step %ld", h->step);
  return MPLB_OK;
}

int mplb_checkpoint_bytes(const mplb_t* h, size_t* bytes) {
  if (!h || !bytes) return MPLB_E_INVAL;
  *bytes = sizeof(CkptHeader) + h->plan.f + h->plan.g + h->plan.phiu;
  return MPLB_OK;
}

int mplb_checkpoint(mplb_t* h, void* host_buf, size_t bytes) {
  size_t need = 0;
  if (!h || !host_buf || mplb_checkpoint_bytes(h, &need) || bytes < need) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "checkpoint before init");
  CkptHeader hd{kMagic, h->G.nx, h->G.ny, h->G.nz, h->prec, h->mode, 0, h->step, h->plan.f, h->plan.g, h->plan.phiu};
  char* p = (char*)host_buf;
  std::memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  HIPCHK(h, hipMemcpyAsync(p, h->B.f[h->cur], h->plan.f, hipMemcpyDeviceToHost, h->stream));
  p += h->plan.f;
  if (h->plan.g) HIPCHK(h, hipMemcpyAsync(p, h->B.g[h->cur], h->plan.g, hipMemcpyDeviceToHost, h->stream));
  p += h->plan.g;
  HIPCHK(h, hipMemcpyAsync(p, h->B.phiu, h->plan.phiu, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MPLB_OK;
}

int mplb_restore(mplb_t* h, const void* host_buf, size_t bytes) {
  size_t need = 0;
  if (!h || !host_buf || mplb_checkpoint_bytes(h, &need) || bytes < need) return MPLB_E_INVAL;
  CkptHeader hd;
  std::memcpy(&hd, host_buf, sizeof hd);
  if (hd.magic != kMagic || hd.nx != h->G.nx || hd.ny != h->G.ny || hd.nz != h->G.nz || hd.prec != h->prec ||
      hd.mode != h->mode || hd.f_bytes != h->plan.f || hd.g_bytes != h->plan.g || hd.phiu_bytes != h->plan.phiu)
    return fail(h, MPLB_E_INVAL, "checkpoint does not match this lattice");
  if (!h->have_params) return fail(h, MPLB_E_STATE, "restore before set_params");
  const char* p = (const char*)host_buf + sizeof hd;
  h->have_init = false;  // as in mplb_init: a failed copy leaves no usable state
  h->cur = 0;
  HIPCHK(h, hipMemcpyAsync(h->B.f[0], p, h->plan.f, hipMemcpyHostToDevice, h->stream));
  p += h->plan.f;
  if (h->plan.g) HIPCHK(h, hipMemcpyAsync(h->B.g[0], p, h->plan.g, hipMemcpyHostToDevice, h->stream));
  p += h->plan.g;
  HIPCHK(h, hipMemcpyAsync(h->B.phiu, p, h->plan.phiu, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, launch_fill_int(h->B.flag, 0, 1, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->step = (long)hd.step;
  h->have_init = true;
  return MPLB_OK;
}

int mplb_copy_probe(const void* src, void* dst, size_t bytes, int kind, void* hip_stream) {
  if (!src || !dst || bytes % 16 || kind < 0 || kind > 3) return MPLB_E_INVAL;
  return launch_copy_probe(src, dst, bytes, kind, (hipStream_t)hip_stream) == hipSuccess ? MPLB_OK : MPLB_E_DEVICE;
}

int mplb_launch_shape(int nx, int ny, int nz, int precision, int mode, int rows, int out[6]) {
  if (!out || !valid_dims(nx, ny, nz) || !valid_mode(mode, precision)) return MPLB_E_INVAL;
  if (rows != 0 && rows != 8 && rows != 16) return MPLB_E_INVAL;
  if (rows == 16 && (mode == MPLB_CHE_ONLY ? precision == MPLB_F64 : precision != MPLB_F32)) return MPLB_E_INVAL;
  Geo G{};
  G.nx = nx; G.ny = ny; G.nz = nz;
  G.N = nx * ny * nz;
  const Shape sh = launch_shape(precision, mode, G, rows);
  out[0] = sh.kind;
  out[1] = sh.tile_w;
  out[2] = sh.tile_h;
  out[3] = sh.tl.lz;
  out[4] = sh.tl.nseg;
  out[5] = sh.tl.tiles_x * sh.tl.tiles_y * sh.tl.nseg;
  return MPLB_OK;
}

int mplb_force_tile_rows(mplb_t* h, int rows) {
  if (!h) return MPLB_E_INVAL;
  if (rows != 0 && rows != 8 && rows != 16) return fail(h, MPLB_E_INVAL, "tile rows must be 0, 8 or 16");
  if (rows == 16 && (h->mode == MPLB_CHE_ONLY ? h->prec == MPLB_F64 : h->prec != MPLB_F32))
    return fail(h, MPLB_E_INVAL,
                "16-row tiles exist for the coupled step with FP32 populations and the CHE-only step in FP32 compute");
  h->tile_rows = rows;
  return MPLB_OK;
}

int mplb_poison(mplb_t* h) {
  if (!h) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "poison before init");
  const Plan& P = h->plan;
  const size_t N = (size_t)h->G.N, pitch = P.pitch;
  const bool pack = h->mode != MPLB_CHE_ONLY && store_size(h->prec) == 2;
  const int q = h->mode == MPLB_COUPLED_Q19 ? 19 : 15;
  // the level the next step writes: whole buffers
  HIPCHK(h, hipMemsetAsync(h->B.f[1 - h->cur], 0xff, P.f, h->stream));
  if (P.g) HIPCHK(h, hipMemsetAsync(h->B.g[1 - h->cur], 0xff, P.g, h->stream));
  // the level it reads, and the history: the padding past the last node of every array
  auto pad = [&](void* base, size_t first_elem, size_t elem) {
    return hipMemsetAsync((char*)base + first_elem * elem, 0xff, (pitch - N) * elem, h->stream);
  };
  char* f = (char*)h->B.f[h->cur];
  HIPCHK(h, pad(f, N, store0_size(h->prec)));
  const size_t fi = pack ? 4 : store_size(h->prec);
  for (int i = 1; i < 7; ++i) HIPCHK(h, pad(f + pitch * store0_size(h->prec), (size_t)(i - 1) * pitch + N, fi));
  if (P.g)
    for (int i = 0; i < (pack ? q - 6 : q); ++i)
      HIPCHK(h, pad(h->B.g[h->cur], (size_t)i * pitch + N, store_size(h->prec)));
  for (int a = 0; a < (h->mode != MPLB_CHE_ONLY ? 3 : 1); ++a)
    HIPCHK(h, pad(h->B.phiu, (size_t)a * pitch + N, comp_size(h->prec)));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->C.poison = 1;
  return MPLB_OK;
}

int mplb_poke(mplb_t* h, int set, int i, long node, double value) {
  if (!h || set < 0 || set > 1 || i < 0 || node < 0 || node >= h->G.N) return MPLB_E_INVAL;
  const int q = h->mode == MPLB_COUPLED_Q19 ? 19 : 15;
  if ((set == 0 && i > 6) || (set == 1 && (i >= q || h->mode == MPLB_CHE_ONLY))) return MPLB_E_INVAL;
  if (!h->have_init) return fail(h, MPLB_E_STATE, "poke before init");
  HIPCHK(h, launch_poke(h->prec, h->mode, h->G, h->B, h->cur, set, i, (int)node, value, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MPLB_OK;
}

}  // extern "C"
