// Calls every entry point of the libmplb C-ABI, with valid arguments and on
// its error paths, for a sanitizer build of the host code (build.sh here).
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "mplb.h"

static int fails = 0;
#define EXPECT(cond) do { if (!(cond)) { printf("FAIL line %d: %s\n", __LINE__, #cond); fflush(stdout); ++fails; } } while (0)

static mplb_params params(bool che) {
  mplb_params p;
  std::memset(&p, 0, sizeof p);
  p.sigma = 1e-3; p.width = 4.0; p.rho_l = che ? 1.0 : 3.0; p.rho_g = 1.0; p.mobility = 0.05; p.A = 0.25;
  const double sf[7] = {1.0, 1.25, 1.25, 1.25, 1.2, 1.0, 1.0};
  for (int i = 0; i < 7; ++i) p.s_f[i] = sf[i];
  p.nu = 0.1;
  for (int i = 0; i < 15; ++i) p.lambda_g[i] = 1.0;
  p.gravity[2] = che ? 0.0 : -1e-6;
  return p;
}

static std::vector<double> field(int nx, int ny, int nz, unsigned seed) {
  std::vector<double> v((size_t)nx * ny * nz);
  srand(seed);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        v[(size_t)x + nx * ((size_t)y + ny * z)] =
            std::tanh((z - nz / 2.0 + 0.5 * std::sin(0.7 * x) + 0.3 * std::cos(0.5 * y)) / 2.0) +
            1e-3 * ((rand() % 1000) / 1000.0 - 0.5);
  return v;
}

static mplb_t* make(int nx, int ny, int nz, int wz, int prec, int mode, void* arena = nullptr, size_t bytes = 0) {
  int bc[3] = {0, 0, wz};
  mplb_t* h = nullptr;
  EXPECT(mplb_create(nx, ny, nz, bc, prec, mode, arena, bytes, &h) == MPLB_OK && h);
  if (!h) return nullptr;
  mplb_params p = params(mode == MPLB_CHE_ONLY);
  EXPECT(mplb_set_params(h, &p) == MPLB_OK);
  if (mode == MPLB_CHE_ONLY) EXPECT(mplb_set_velocity(h, MPLB_VEL_DEFORM, nullptr, 0.02, 0.05) == MPLB_OK);
  std::vector<double> phi = field(nx, ny, nz, nx * 7 + nz);
  EXPECT(mplb_init(h, phi.data(), nullptr) == MPLB_OK);
  return h;
}

int main() {
  const int nx = 24, ny = 24, nz = 20;
  const size_t N = (size_t)nx * ny * nz;
  // error paths that need no device
  size_t bytes = 0;
  EXPECT(mplb_required_bytes(0, 1, 1, MPLB_F32, MPLB_COUPLED, &bytes) == MPLB_E_INVAL);
  EXPECT(mplb_required_bytes(nx, ny, nz, 9, MPLB_COUPLED, &bytes) == MPLB_E_INVAL);
  EXPECT(mplb_required_bytes(nx, ny, nz, MPLB_F32, MPLB_COUPLED, nullptr) == MPLB_E_INVAL);
  EXPECT(mplb_required_bytes(65536, 65536, 2, MPLB_F32, MPLB_COUPLED, &bytes) == MPLB_E_INVAL);
  EXPECT(std::strlen(mplb_strerror(MPLB_E_NONFINITE)) > 0 && std::strlen(mplb_strerror(99)) > 0);
  EXPECT(std::strcmp(mplb_last_error(nullptr), "null handle") == 0);
  EXPECT(mplb_step(nullptr, 1) == MPLB_E_INVAL && mplb_read(nullptr, 0, nullptr) == MPLB_E_INVAL);
  EXPECT(mplb_step_many(nullptr, 1, 1) == MPLB_E_INVAL);
  mplb_destroy(nullptr);
  int shp[6];
  EXPECT(mplb_launch_shape(256, 256, 1024, MPLB_F32, MPLB_COUPLED, 0, shp) == MPLB_OK && shp[0] == 1 && shp[5] == 512);
  EXPECT(mplb_launch_shape(64, 64, 64, MPLB_F64, MPLB_COUPLED, 16, shp) == MPLB_E_INVAL);
  EXPECT(mplb_launch_shape(64, 64, 64, MPLB_F32, MPLB_CHE_ONLY, 0, nullptr) == MPLB_E_INVAL);

  for (int mode : {MPLB_COUPLED, MPLB_COUPLED_Q19, MPLB_CHE_ONLY})
    for (int prec : {MPLB_F64, MPLB_F32, MPLB_F32_F16, MPLB_F32_BF16}) {
      printf("[case] mode %d precision %d\n", mode, prec);
      fflush(stdout);
      int bc[3] = {0, 0, 1};
      mplb_t* h = nullptr;
      EXPECT(mplb_create(nx, ny, nz, bc, prec, mode, nullptr, 0, &h) == MPLB_OK);
      std::vector<double> out(N), diag((size_t)nx * nz);
      EXPECT(mplb_step(h, 1) == MPLB_E_STATE);                      // before init
      EXPECT(mplb_read(h, MPLB_PHI, out.data()) == MPLB_E_STATE);
      mplb_params p = params(mode == MPLB_CHE_ONLY);
      mplb_params bad = p;
      bad.s_f[2] = 1.1;
      EXPECT(mplb_set_params(h, &bad) == MPLB_E_INVAL && std::strlen(mplb_last_error(h)) > 0);
      bad = p;
      bad.lambda_g[14] = 2.5;
      EXPECT(mplb_set_params(h, &bad) == MPLB_E_INVAL);
      EXPECT(mplb_set_params(h, &p) == MPLB_OK);
      std::vector<double> u(3 * N, 0.01);
      if (mode == MPLB_CHE_ONLY) {
        EXPECT(mplb_set_velocity(h, MPLB_VEL_FIELD, nullptr, 0, 1) == MPLB_E_INVAL);
        EXPECT(mplb_set_velocity(h, MPLB_VEL_FIELD, u.data(), 0, 1) == MPLB_OK);
      } else {
        EXPECT(mplb_set_velocity(h, MPLB_VEL_ZERO, nullptr, 0, 1) == MPLB_E_STATE);
      }
      std::vector<double> phi = field(nx, ny, nz, 3 + prec);
      EXPECT(mplb_init(h, phi.data(), mode == MPLB_CHE_ONLY ? nullptr : u.data()) == MPLB_OK);
      EXPECT(mplb_set_check_interval(h, -1) == MPLB_E_INVAL);
      EXPECT(mplb_set_check_interval(h, 3) == MPLB_OK);
      EXPECT(mplb_step(h, 7) == MPLB_OK && mplb_step_count(h) == 7);
      for (int f = MPLB_PHI; f <= MPLB_P; ++f) EXPECT(mplb_read(h, f, out.data()) == MPLB_OK);
      EXPECT(mplb_read(h, 7, out.data()) == MPLB_E_INVAL);
      EXPECT(mplb_read_diagonal(h, MPLB_UZ, diag.data()) == MPLB_OK);
      double tot[7], fr[2], ms[4];
      EXPECT(mplb_totals(h, tot) == MPLB_OK);
      EXPECT(mplb_front(h, fr) == MPLB_OK);
      EXPECT(mplb_time_stages(h, 3, ms) == MPLB_OK);
      size_t cb = 0;
      EXPECT(mplb_checkpoint_bytes(h, &cb) == MPLB_OK && cb > 0);
      std::vector<unsigned char> ck(cb);
      EXPECT(mplb_checkpoint(h, ck.data(), cb - 1) == MPLB_E_INVAL);
      EXPECT(mplb_checkpoint(h, ck.data(), cb) == MPLB_OK);
      EXPECT(mplb_step(h, 2) == MPLB_OK);
      EXPECT(mplb_restore(h, ck.data(), cb) == MPLB_OK && mplb_step_count(h) == 10);
      std::vector<unsigned char> ck2 = ck;
      ck2[0] ^= 1;
      EXPECT(mplb_restore(h, ck2.data(), cb) == MPLB_E_INVAL);
      int rows = (mode == MPLB_CHE_ONLY ? prec != MPLB_F64 : prec == MPLB_F32) ? 16 : 8;
      EXPECT(mplb_force_tile_rows(h, rows) == MPLB_OK);
      EXPECT(mplb_force_tile_rows(h, 12) == MPLB_E_INVAL);
      EXPECT(mplb_step(h, 2) == MPLB_OK);
      EXPECT(mplb_force_tile_rows(h, 0) == MPLB_OK);
      EXPECT(mplb_poke(h, 0, 7, 0, 0.0) == MPLB_E_INVAL);
      EXPECT(mplb_poke(h, 0, 1, (long)N, 0.0) == MPLB_E_INVAL);
      EXPECT(mplb_poison(h) == MPLB_OK);
      EXPECT(mplb_step(h, 1) == MPLB_OK);
      EXPECT(mplb_poke(h, 0, 1, 5, NAN) == MPLB_OK);
      EXPECT(mplb_step(h, 3) == MPLB_E_NONFINITE && std::strlen(mplb_last_error(h)) > 0);
      EXPECT(mplb_check_finite(h) == MPLB_E_NONFINITE);
      mplb_destroy(h);
    }

  // a borrowed arena, batches (graphs on and off, the allocation-free entry
  // point), a lattice on another stream, a lattice listed twice
  printf("[case] batches\n");
  fflush(stdout);
  size_t need = 0;
  EXPECT(mplb_required_bytes(nx, ny, nz, MPLB_F32, MPLB_COUPLED, &need) == MPLB_OK);
  void* arena = nullptr;
  EXPECT(hipMalloc(&arena, need) == hipSuccess);
  int bc[3] = {0, 0, 1};
  mplb_t* tmp = nullptr;
  EXPECT(mplb_create(nx, ny, nz, bc, MPLB_F32, MPLB_COUPLED, arena, need - 1, &tmp) == MPLB_E_NOMEM && !tmp);
  std::vector<mplb_t*> hs;
  hs.push_back(make(nx, ny, nz, 1, MPLB_F32, MPLB_COUPLED, arena, need));
  hs.push_back(make(17, 9, 33, 0, MPLB_F32, MPLB_COUPLED));
  hs.push_back(make(40, 31, 12, 1, MPLB_F32, MPLB_COUPLED));
  hs.push_back(make(5, 6, 7, 0, MPLB_F32, MPLB_COUPLED));
  EXPECT(mplb_set_step_many_graphs(1) == MPLB_OK);
  EXPECT(mplb_step_many(hs.data(), (int)hs.size(), 5) == MPLB_OK);
  EXPECT(mplb_step_many(hs.data(), (int)hs.size(), 1) == MPLB_OK);
  EXPECT(mplb_set_step_many_graphs(0) == MPLB_OK);
  EXPECT(mplb_step_many(hs.data(), (int)hs.size(), 4) == MPLB_OK);
  EXPECT(mplb_set_step_many_graphs(1) == MPLB_OK);
  EXPECT(mplb_step_many_noalloc(hs.data(), (int)hs.size(), 3) == MPLB_OK);
  std::vector<mplb_t*> twice = {hs[0], hs[1], hs[0]};
  EXPECT(mplb_step_many(twice.data(), 3, 1) == MPLB_E_INVAL);
  hipStream_t s2 = nullptr;
  EXPECT(hipStreamCreate(&s2) == hipSuccess);
  EXPECT(mplb_set_stream(hs[2], s2) == MPLB_OK);
  EXPECT(mplb_step_many(hs.data(), (int)hs.size(), 1) == MPLB_E_INVAL);
  EXPECT(mplb_set_stream(hs[2], nullptr) == MPLB_OK);
  for (auto* h : hs) EXPECT(mplb_step_count(h) == 13);
  std::vector<mplb_t*> many(600, hs[3]);
  EXPECT(mplb_step_many_noalloc(many.data(), 600, 1) == MPLB_E_INVAL);
  // a CHE-only batch (stepped one after another)
  std::vector<mplb_t*> che = {make(30, 20, 16, 0, MPLB_F32_F16, MPLB_CHE_ONLY),
                              make(16, 16, 16, 1, MPLB_F32_F16, MPLB_CHE_ONLY)};
  EXPECT(mplb_step_many(che.data(), 2, 4) == MPLB_OK);
  for (auto* h : che) mplb_destroy(h);
  for (auto* h : hs) mplb_destroy(h);
  EXPECT(hipStreamDestroy(s2) == hipSuccess);
  // copy probe
  void *a = nullptr, *b = nullptr;
  EXPECT(hipMalloc(&a, 1 << 24) == hipSuccess && hipMalloc(&b, 1 << 24) == hipSuccess);
  for (int k = 0; k < 4; ++k) EXPECT(mplb_copy_probe(a, b, 1 << 24, k, nullptr) == MPLB_OK);
  EXPECT(mplb_copy_probe(a, b, 17, 0, nullptr) == MPLB_E_INVAL);
  EXPECT(hipDeviceSynchronize() == hipSuccess);
  EXPECT(hipFree(a) == hipSuccess && hipFree(b) == hipSuccess && hipFree(arena) == hipSuccess);
  printf("%s: %d failed expectations\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
