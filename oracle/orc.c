/*
 * orc.c -- FP64 CPU oracle for one time step of the 3D MRT lattice-Boltzmann
 * phase-field model of Liang, Shi & Chai (arXiv:1507.07294).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow and written to be checked against the
 * paper by eye.  Collisions are done in moment space with the dense matrices
 * M (Eq. 9) and Gamma (Eq. 25) as the paper prescribes (Sec. II A after
 * Eq. 16, Sec. II B after Eq. 30); no blocking or fusion.  The only
 * parallelism is an OpenMP loop over nodes.  Nothing here is shared with the
 * GPU library.
 *
 * One step n -> n+1, all inputs at level n:
 *   S1 phi = sum_i f_i, rho(phi)                              (Eqs. 13, 14)
 *   S2 mu = 4 beta phi (phi - 1)(phi + 1) - k lap phi         (Eqs. 2, 36)
 *   S3 grad phi, grad rho, lap mu                             (Eqs. 35, 36)
 *   S4 F_s, G, u, F_a, p                                      (Eqs. 29, 30; F_a after Eq. 28)
 *   S5 d_t(phi u) = (phi u)(n) - (phi u)(n-1)                 (Eq. 34)
 *   S6 CHE collision in moment space                          (Eqs. 15, 17, 18, 11)
 *   S7 NSE collision in moment space                          (Eqs. 20, 27, 31, 32)
 *      (the D3Q19 variant: Gamma_19 g^eq and Gamma_19 T of Eqs. 21, 28)
 *   S8 streaming, periodic wrap or half-way bounce-back       (Eq. 16)
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - Gamma's columns are labelled by its own rows 3, 5, 7 (the c_x, c_y, c_z
 *     rows) and re-ordered to the velocity order of Eq. 23.
 *   - Eqs. 35-36 use the D3Q15 weights with c_s^2 = 1/3; the c_i inside the
 *     bracket of Eq. 36 is read as absent (the Laplacian is a scalar sum).
 *   - F in Eq. 32 is F_s + F_a + G, as in Eq. 28; rho_A, rho_B = rho_l, rho_g.
 *   - Eq. 32 is used as printed (it is the moment form the paper collides with).
 *   - the sums over g in Eqs. 29-30 use the populations of the current level.
 *   - G = (rho - rho_ref) * gravity.
 *   - no-slip walls: half-way bounce-back for f and g; finite-difference
 *     stencils see a mirror ghost layer (chi(-1) = chi(0)).
 *   - d_t(phi u) at the first step uses (phi u)_prev = phi0 u0.
 */
#include "orc.h"

#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define C_LAT 1.0 /* lattice speed c = dx/dt */

/* ---------------- lattice constants ---------------- */

/* D3Q7 velocities, Eq. 6 */
static const int C7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                             {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* M, Eq. 9, as printed */
static const double M7[7][7] = {
    {1, 1, 1, 1, 1, 1, 1},    {0, 1, -1, 0, 0, 0, 0},    {0, 0, 0, 1, -1, 0, 0},
    {0, 0, 0, 0, 0, 1, -1},   {6, -1, -1, -1, -1, -1, -1}, {0, 2, 2, -1, -1, -1, -1},
    {0, 0, 0, 1, 1, -1, -1}};

/* D3Q15 velocities, Eq. 23 (columns of the printed 3x15 table) */
static const int C15[15][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 1},  {-1, -1, -1}, {1, 1, -1},
    {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1}, {1, -1, -1}, {-1, 1, 1}};

/* D3Q15 weights, Eq. 24 */
static const double W15[15] = {2.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,
                               1.0 / 9,  1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,
                               1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
static const double CS2_G = 1.0 / 3.0; /* c = sqrt(3) c_s (after Eq. 23) */

/* Gamma, Eq. 25, exactly as printed (its own column order) */
static const double G15_PRINTED[15][15] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-2, -1, -1, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1},
    {16, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1},
    {0, 0, 0, 0, 0, -4, 4, 1, 1, 1, 1, -1, -1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1}};

/* D3Q19, the alternative lattice the paper names for the NSE (after Eq. 22):
 * rest, the six faces in the order of Eq. 23, then the twelve edges in
 * antipodal pairs.  Weights 1/3, 1/18, 1/36; c_s^2 = 1/3. */
static const int C19[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                               1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                               1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
/* D3Q19 moments of d'Humieres et al. (2002): density, energy, energy square,
 * momentum and heat flux per axis, the five stress components with their
 * fourth-order partners, and three third-order moments.  Rows 9, 11, 13, 14
 * and 15 are the stress moments that set the viscosity. */
static double g19_row(int r, const int c[3]) {
  const double x = c[0], y = c[1], z = c[2], c2 = x * x + y * y + z * z;
  switch (r) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * c2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * c2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * c2 - 9.0) * z;
    case 9: return 3.0 * x * x - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}
static const int VISC19[5] = {9, 11, 13, 14, 15};

static double G15[15][15];     /* Gamma in the Eq. 23 velocity order */
static double G15_INV[15][15]; /* Gamma^-1 = Gamma^T diag(1/(Gamma Gamma^T)_ii) */
static double M7_INV[7][7];
static double G19[19][19], G19_INV[19][19];
static int OPP7[7], OPP15[15], OPP19[19];
static int tables_ready = 0;

/* Builds Gamma in the Eq. 23 order, the inverses and the opposite-direction
 * maps.  Aborts if a matrix is not orthogonal (the inverses rely on it). */
static void build_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < 15; ++i) {
    int col = -1;
    for (int j = 0; j < 15; ++j)
      if ((int)G15_PRINTED[3][j] == C15[i][0] && (int)G15_PRINTED[5][j] == C15[i][1] &&
          (int)G15_PRINTED[7][j] == C15[i][2])
        col = j;
    if (col < 0) abort();
    for (int r = 0; r < 15; ++r) G15[r][i] = G15_PRINTED[r][col];
  }
  for (int r = 0; r < 7; ++r) {
    double d = 0;
    for (int i = 0; i < 7; ++i) d += M7[r][i] * M7[r][i];
    for (int r2 = 0; r2 < 7; ++r2) {
      double o = 0;
      for (int i = 0; i < 7; ++i) o += M7[r][i] * M7[r2][i];
      if (r2 != r && o != 0.0) abort();
    }
    for (int i = 0; i < 7; ++i) M7_INV[i][r] = M7[r][i] / d;
  }
  for (int r = 0; r < 15; ++r) {
    double d = 0;
    for (int i = 0; i < 15; ++i) d += G15[r][i] * G15[r][i];
    for (int r2 = 0; r2 < 15; ++r2) {
      double o = 0;
      for (int i = 0; i < 15; ++i) o += G15[r][i] * G15[r2][i];
      if (r2 != r && o != 0.0) abort();
    }
    for (int i = 0; i < 15; ++i) G15_INV[i][r] = G15[r][i] / d;
  }
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j)
      if (C7[j][0] == -C7[i][0] && C7[j][1] == -C7[i][1] && C7[j][2] == -C7[i][2]) OPP7[i] = j;
  for (int i = 0; i < 15; ++i)
    for (int j = 0; j < 15; ++j)
      if (C15[j][0] == -C15[i][0] && C15[j][1] == -C15[i][1] && C15[j][2] == -C15[i][2])
        OPP15[i] = j;
  for (int r = 0; r < 19; ++r)
    for (int i = 0; i < 19; ++i) G19[r][i] = g19_row(r, C19[i]);
  for (int r = 0; r < 19; ++r) {
    double d = 0;
    for (int i = 0; i < 19; ++i) d += G19[r][i] * G19[r][i];
    for (int r2 = 0; r2 < 19; ++r2) {
      double o = 0;
      for (int i = 0; i < 19; ++i) o += G19[r][i] * G19[r2][i];
      if (r2 != r && o != 0.0) abort();
    }
    for (int i = 0; i < 19; ++i) G19_INV[i][r] = G19[r][i] / d;
  }
  for (int i = 0; i < 19; ++i)
    for (int j = 0; j < 19; ++j)
      if (C19[j][0] == -C19[i][0] && C19[j][1] == -C19[i][1] && C19[j][2] == -C19[i][2])
        OPP19[i] = j;
  tables_ready = 1;
}

/* D3Q7 weights, Eq. 8 */
static void weights7(double A, double w[7]) {
  w[0] = 1.0 - 3.0 * A;
  for (int i = 1; i < 7; ++i) w[i] = A / 2.0;
}

/* ---------------- state ---------------- */

struct orc_s {
  int n[3], bc[3], mode;
  int q;                  /* NSE lattice: 15 (Eq. 23) or 19 */
  const int (*cg)[3];     /* its velocities, weights and opposite directions */
  const double* wg;
  const int* oppg;
  long N;
  int have_params, have_init;
  orc_params p;
  /* derived parameters */
  double beta, kappa, tau_f, eta, tau_g, drho;
  double sf[7], lg[19];
  /* state at level n */
  double *f, *g, *phiu;
  long step;
  /* per-step work arrays */
  double *fpost, *gpost, *phi, *rho, *mu, *u, *pr, *F, *gradrho;
  /* prescribed velocity */
  int vel_kind;
  double velU, velT;
  double* ufield;
  char err[256];
};

static long idx(const orc_t* s, int x, int y, int z) {
  return (long)x + (long)s->n[0] * ((long)y + (long)s->n[1] * (long)z);
}

/* Node one hop away along (dx,dy,dz) for the finite differences: periodic
 * axes wrap, wall axes repeat the first interior layer (mirror ghost). */
static long stencil_nb(const orc_t* s, int x, int y, int z, int dx, int dy, int dz) {
  int q[3] = {x + dx, y + dy, z + dz};
  for (int a = 0; a < 3; ++a) {
    if (q[a] < 0) q[a] = (s->bc[a] == ORC_WALL) ? 0 : q[a] + s->n[a];
    if (q[a] >= s->n[a]) q[a] = (s->bc[a] == ORC_WALL) ? s->n[a] - 1 : q[a] - s->n[a];
  }
  return idx(s, q[0], q[1], q[2]);
}

orc_t* orc_create(int nx, int ny, int nz, const int bc[3], int mode) {
  build_tables();
  if (nx < 1 || ny < 1 || nz < 1 || !bc) return NULL;
  if (mode != ORC_COUPLED && mode != ORC_CHE_ONLY && mode != ORC_COUPLED_Q19) return NULL;
  for (int a = 0; a < 3; ++a)
    if (bc[a] != ORC_PERIODIC && bc[a] != ORC_WALL) return NULL;
  orc_t* s = (orc_t*)calloc(1, sizeof(orc_t));
  if (!s) return NULL;
  s->n[0] = nx; s->n[1] = ny; s->n[2] = nz;
  for (int a = 0; a < 3; ++a) s->bc[a] = bc[a];
  s->mode = mode;
  s->q = (mode == ORC_COUPLED_Q19) ? 19 : 15;
  s->cg = (s->q == 19) ? C19 : C15;
  s->wg = (s->q == 19) ? W19 : W15;
  s->oppg = (s->q == 19) ? OPP19 : OPP15;
  s->N = (long)nx * ny * nz;
  long N = s->N;
  s->f = calloc(7 * N, sizeof(double));
  s->g = calloc(s->q * N, sizeof(double));
  s->phiu = calloc(3 * N, sizeof(double));
  s->fpost = calloc(7 * N, sizeof(double));
  s->gpost = calloc(s->q * N, sizeof(double));
  s->phi = calloc(N, sizeof(double));
  s->rho = calloc(N, sizeof(double));
  s->mu = calloc(N, sizeof(double));
  s->u = calloc(3 * N, sizeof(double));
  s->pr = calloc(N, sizeof(double));
  s->F = calloc(3 * N, sizeof(double));
  s->gradrho = calloc(3 * N, sizeof(double));
  if (!s->f || !s->g || !s->phiu || !s->fpost || !s->gpost || !s->phi || !s->rho || !s->mu ||
      !s->u || !s->pr || !s->F || !s->gradrho) {
    orc_destroy(s);
    return NULL;
  }
  return s;
}

void orc_destroy(orc_t* s) {
  if (!s) return;
  free(s->f); free(s->g); free(s->phiu); free(s->fpost); free(s->gpost);
  free(s->phi); free(s->rho); free(s->mu); free(s->u); free(s->pr); free(s->F);
  free(s->gradrho); free(s->ufield);
  free(s);
}

const char* orc_last_error(const orc_t* s) { return s ? s->err : "null handle"; }
long orc_step_count(const orc_t* s) { return s ? s->step : -1; }

/* beta, k (after Eq. 2), tau_f and eta (Eq. 19), tau_g and lambda_9..13 (Eq. 33) */
int orc_derived(const orc_params* p, double* d) {
  if (!p || !d) return ORC_E_INVAL;
  double beta = 3.0 * p->sigma / (4.0 * p->width);
  double kappa = 3.0 * p->width * p->sigma / 8.0;
  double tau_f = 1.0 / p->s_f[1];
  double eta = p->mobility / (p->A * C_LAT * C_LAT * (tau_f - 0.5));
  double tau_g = p->nu / CS2_G + 0.5;
  d[0] = beta; d[1] = kappa; d[2] = tau_f; d[3] = eta; d[4] = tau_g; d[5] = 1.0 / tau_g;
  return ORC_OK;
}

int orc_set_params(orc_t* s, const orc_params* p) {
  if (!s || !p) return ORC_E_INVAL;
  if (!(p->A > 0 && p->A < 1.0 / 3.0) || !(p->width > 0) || !(p->rho_l > 0) || !(p->rho_g > 0) ||
      !(p->nu > 0) || p->s_f[1] != p->s_f[2] || p->s_f[1] != p->s_f[3] || !(p->mobility >= 0)) {
    snprintf(s->err, sizeof s->err, "invalid parameters");
    return ORC_E_INVAL;
  }
  for (int i = 0; i < 7; ++i)
    if (!(p->s_f[i] > 0 && p->s_f[i] < 2)) { snprintf(s->err, sizeof s->err, "s_f out of (0,2)"); return ORC_E_INVAL; }
  if ((p->stencil != ORC_STENCIL_Q15 && p->stencil != ORC_STENCIL_Q7) ||
      (p->forcing != ORC_FORCING_EQ32 && p->forcing != ORC_FORCING_EQ28)) {
    snprintf(s->err, sizeof s->err, "unknown stencil or forcing switch");
    return ORC_E_INVAL;
  }
  if (p->lambda_override)
    for (int i = 10; i <= 13; ++i)
      if (p->lambda_g[i] != p->lambda_g[9]) {
        snprintf(s->err, sizeof s->err, "lambda_9..13 must be equal");
        return ORC_E_INVAL;
      }
  double d[6];
  orc_derived(p, d);
  if (p->lambda_override) { /* the viscous rate given, tau_g = 1/lambda_9 (Eq. 33) */
    d[5] = p->lambda_g[9];
    d[4] = 1.0 / d[5];
  }
  s->p = *p;
  s->beta = d[0]; s->kappa = d[1]; s->tau_f = d[2]; s->eta = d[3]; s->tau_g = d[4];
  s->drho = p->rho_l - p->rho_g;
  for (int i = 0; i < 7; ++i) s->sf[i] = p->s_f[i];
  if (s->q == 19) {
    /* D3Q19: the stress moments relax at 1/tau_g (Eq. 33), the others at 1
     * (the paper's choice for S^g, Sec. III C) */
    for (int r = 0; r < 19; ++r) s->lg[r] = 1.0;
    for (int k = 0; k < 5; ++k) s->lg[VISC19[k]] = d[5];
  } else {
    for (int i = 0; i < 15; ++i) s->lg[i] = p->lambda_g[i];
    for (int i = 9; i <= 13; ++i) s->lg[i] = d[5];
  }
  for (int i = 0; i < s->q; ++i)
    if (!(s->lg[i] > 0 && s->lg[i] < 2)) { snprintf(s->err, sizeof s->err, "lambda out of (0,2)"); return ORC_E_INVAL; }
  s->have_params = 1;
  return ORC_OK;
}

/* ---------------- node-level pieces of the paper ---------------- */

void orc_matrices(double* M, double* Gm) {
  build_tables();
  if (M) for (int r = 0; r < 7; ++r) for (int i = 0; i < 7; ++i) M[r * 7 + i] = M7[r][i];
  if (Gm) for (int r = 0; r < 15; ++r) for (int i = 0; i < 15; ++i) Gm[r * 15 + i] = G15[r][i];
}

void orc_lattices(double A, int* c7, double* w7, int* c15, double* w15) {
  double w[7];
  weights7(A, w);
  for (int i = 0; i < 7; ++i) {
    if (c7) for (int a = 0; a < 3; ++a) c7[i * 3 + a] = C7[i][a];
    if (w7) w7[i] = w[i];
  }
  for (int i = 0; i < 15; ++i) {
    if (c15) for (int a = 0; a < 3; ++a) c15[i * 3 + a] = C15[i][a];
    if (w15) w15[i] = W15[i];
  }
}

/* Eq. 5 */
void orc_feq(double A, double eta, double phi, double mu, const double u[3], double feq[7]) {
  double w[7];
  weights7(A, w);
  double cs2 = A * C_LAT * C_LAT; /* Eq. 8 */
  feq[0] = phi + (w[0] - 1.0) * eta * mu;
  for (int i = 1; i < 7; ++i) {
    double cphiu = C_LAT * (C7[i][0] * phi * u[0] + C7[i][1] * phi * u[1] + C7[i][2] * phi * u[2]);
    feq[i] = w[i] * eta * mu + w[i] * cphiu / cs2;
  }
}

/* s_i(u), Eq. 22 */
static double s_of_u(int i, const double u[3]) {
  double cu = C_LAT * (C15[i][0] * u[0] + C15[i][1] * u[1] + C15[i][2] * u[2]);
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return W15[i] * (cu / CS2_G + cu * cu / (2.0 * CS2_G * CS2_G) - uu / (2.0 * CS2_G));
}

/* s_i(u), Eq. 22, for velocity c with weight w */
static double s_of_cw(const int c[3], double w, const double u[3]) {
  double cu = C_LAT * (c[0] * u[0] + c[1] * u[1] + c[2] * u[2]);
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return w * (cu / CS2_G + cu * cu / (2.0 * CS2_G * CS2_G) - uu / (2.0 * CS2_G));
}

/* Eq. 21 on a lattice of q velocities c with weights w */
static void geq_qw(int q, const int (*c)[3], const double* w, double p, double rho, const double u[3],
                   double* geq) {
  for (int i = 0; i < q; ++i) geq[i] = p / CS2_G * (i == 0 ? w[0] - 1.0 : w[i]) + rho * s_of_cw(c[i], w[i], u);
}

/* Eq. 28 on a lattice of q velocities: T_i = (c_i - u)/c_s^2 . [s_i(u)
 * grad(rho c_s^2) + F (s_i(u) + w_i)], with F = F_s + F_a + G */
static void T_qw(int q, const int (*c)[3], const double* w, const double u[3], const double gr[3],
                 const double F[3], double* T) {
  for (int i = 0; i < q; ++i) {
    double si = s_of_cw(c[i], w[i], u), acc = 0.0;
    for (int a = 0; a < 3; ++a) acc += (C_LAT * c[i][a] - u[a]) * (si * gr[a] * CS2_G + F[a] * (si + w[i]));
    T[i] = acc / CS2_G;
  }
}

static void geq_of(const orc_t* s, double p, double rho, const double u[3], double* geq) {
  geq_qw(s->q, s->cg, s->wg, p, rho, u, geq);
}
static void T_of(const orc_t* s, const double u[3], const double gr[3], const double F[3], double* T) {
  T_qw(s->q, s->cg, s->wg, u, gr, F, T);
}

void orc_lattice19(int* c19, double* w19, double* G) {
  build_tables();
  for (int i = 0; i < 19; ++i) {
    if (c19) for (int a = 0; a < 3; ++a) c19[i * 3 + a] = C19[i][a];
    if (w19) w19[i] = W19[i];
  }
  if (G) for (int r = 0; r < 19; ++r) for (int i = 0; i < 19; ++i) G[r * 19 + i] = G19[r][i];
}

void orc_geq19(double p, double rho, const double u[3], double geq[19]) { geq_qw(19, C19, W19, p, rho, u, geq); }

void orc_T(int q, const double u[3], const double gr[3], const double F[3], double* T) {
  if (q == 19) T_qw(19, C19, W19, u, gr, F, T);
  else T_qw(15, C15, W15, u, gr, F, T);
}

/* Eq. 21 */
void orc_geq(double p, double rho, const double u[3], double geq[15]) {
  geq[0] = p / CS2_G * (W15[0] - 1.0) + rho * s_of_u(0, u);
  for (int i = 1; i < 15; ++i) geq[i] = p / CS2_G * W15[i] + rho * s_of_u(i, u);
}

/* Eq. 17 */
void orc_meq_f(double A, double eta, double phi, double mu, const double u[3], double m[7]) {
  m[0] = phi;
  m[1] = phi * u[0] / C_LAT;
  m[2] = phi * u[1] / C_LAT;
  m[3] = phi * u[2] / C_LAT;
  m[4] = 6.0 * phi - 21.0 * A * eta * mu;
  m[5] = 0.0;
  m[6] = 0.0;
}

/* Eq. 18 */
void orc_mR(const double dphiu[3], double m[7]) {
  m[0] = 0.0;
  m[1] = dphiu[0] / C_LAT;
  m[2] = dphiu[1] / C_LAT;
  m[3] = dphiu[2] / C_LAT;
  m[4] = m[5] = m[6] = 0.0;
}

/* Eq. 31 (row 2 divided by c^2; the printed single c is immaterial at c = 1) */
void orc_meq_g(double p, double rho, const double u[3], double m[15]) {
  const double c = C_LAT, c2 = C_LAT * C_LAT;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  m[0] = 0.0;
  m[1] = (3.0 * p + rho * uu) / c2;
  m[2] = -(45.0 * p + 5.0 * rho * uu) / c2;
  m[3] = rho * u[0] / c;
  m[4] = -7.0 * rho * u[0] / (3.0 * c);
  m[5] = rho * u[1] / c;
  m[6] = -7.0 * rho * u[1] / (3.0 * c);
  m[7] = rho * u[2] / c;
  m[8] = -7.0 * rho * u[2] / (3.0 * c);
  m[9] = rho * (2.0 * u[0] * u[0] - u[1] * u[1] - u[2] * u[2]) / c2;
  m[10] = rho * (u[1] * u[1] - u[2] * u[2]) / c2;
  m[11] = rho * u[0] * u[1] / c2;
  m[12] = rho * u[1] * u[2] / c2;
  m[13] = rho * u[0] * u[2] / c2;
  m[14] = 0.0;
}

/* Eq. 32, with F = F_s + F_a + G and a_b = d_b(rho) c_s^2 + F_b */
void orc_mT(const double u[3], const double gr[3], const double F[3], double m[15]) {
  const double c = C_LAT, c2 = C_LAT * C_LAT, cs2 = CS2_G;
  double a[3];
  for (int b = 0; b < 3; ++b) a[b] = gr[b] * cs2 + F[b];
  double ugr = u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2];
  double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  m[0] = ugr;
  m[1] = (-ugr * cs2 + 2.0 * uF) / c2;
  m[2] = -(7.0 * ugr * cs2 + 10.0 * uF) / c2;
  m[3] = F[0] / c;
  m[4] = -7.0 * F[0] / (3.0 * c);
  m[5] = F[1] / c;
  m[6] = -7.0 * F[1] / (3.0 * c);
  m[7] = F[2] / c;
  m[8] = -7.0 * F[2] / (3.0 * c);
  m[9] = (4.0 * u[0] * a[0] - 2.0 * u[1] * a[1] - 2.0 * u[2] * a[2]) / c2;
  m[10] = (2.0 * u[1] * a[1] - 2.0 * u[2] * a[2]) / c2;
  m[11] = (u[0] * a[1] + u[1] * a[0]) / c2;
  m[12] = (u[1] * a[2] + u[2] * a[1]) / c2;
  m[13] = (u[0] * a[2] + u[2] * a[0]) / c2;
  m[14] = 0.0;
}

/* Eq. 35 at one node: D3Q15 weights (default) or, with ORC_STENCIL_Q7, the
 * D3Q7 weights w_i = A/2, c_s^2 = A (Eqs. 7-8), whose ratio is 1/2 */
static void grad_at(const orc_t* s, const double* chi, int x, int y, int z, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  if (s->p.stencil == ORC_STENCIL_Q7) {
    double w[7], cs2 = s->p.A * C_LAT * C_LAT;
    weights7(s->p.A, w);
    for (int i = 1; i < 7; ++i) {
      double v = chi[stencil_nb(s, x, y, z, C7[i][0], C7[i][1], C7[i][2])];
      for (int a = 0; a < 3; ++a) out[a] += w[i] * C_LAT * C7[i][a] * v / cs2;
    }
    return;
  }
  for (int i = 1; i < 15; ++i) {
    double v = chi[stencil_nb(s, x, y, z, C15[i][0], C15[i][1], C15[i][2])];
    for (int a = 0; a < 3; ++a) out[a] += W15[i] * C_LAT * C15[i][a] * v / CS2_G;
  }
}

/* Eq. 36 at one node, on the lattice of grad_at */
static double lap_at(const orc_t* s, const double* chi, int x, int y, int z) {
  double c0 = chi[idx(s, x, y, z)], acc = 0.0;
  if (s->p.stencil == ORC_STENCIL_Q7) {
    double w[7], cs2 = s->p.A * C_LAT * C_LAT;
    weights7(s->p.A, w);
    for (int i = 1; i < 7; ++i) {
      double v = chi[stencil_nb(s, x, y, z, C7[i][0], C7[i][1], C7[i][2])];
      acc += 2.0 * w[i] * (v - c0) / cs2;
    }
    return acc;
  }
  for (int i = 1; i < 15; ++i) {
    double v = chi[stencil_nb(s, x, y, z, C15[i][0], C15[i][1], C15[i][2])];
    acc += 2.0 * W15[i] * (v - c0) / CS2_G;
  }
  return acc;
}

int orc_grad_lap(const orc_t* s, const double* chi, double* grad, double* lap) {
  if (!s || !chi) return ORC_E_INVAL;
  long N = s->N;
#pragma omp parallel for
  for (int z = 0; z < s->n[2]; ++z)
    for (int y = 0; y < s->n[1]; ++y)
      for (int x = 0; x < s->n[0]; ++x) {
        long n = idx(s, x, y, z);
        if (grad) {
          double gv[3];
          grad_at(s, chi, x, y, z, gv);
          for (int a = 0; a < 3; ++a) grad[a * N + n] = gv[a];
        }
        if (lap) lap[n] = lap_at(s, chi, x, y, z);
      }
  return ORC_OK;
}

/* prescribed velocity at step n: Zalesak rotation (Eq. 37) and deformation
 * flow (Eq. 41 times cos(pi t / T), t = n U / L) with L the box edge along x */
static void prescribed_u(const orc_t* s, int x, int y, int z, long n, double u[3]) {
  const double pi = 3.14159265358979323846;
  long id = idx(s, x, y, z);
  u[0] = u[1] = u[2] = 0.0;
  if (s->vel_kind == ORC_VEL_FIELD) {
    for (int a = 0; a < 3; ++a) u[a] = s->ufield[a * s->N + id];
  } else if (s->vel_kind == ORC_VEL_ZALESAK) {
    double L = s->n[0], U = s->velU;
    u[0] = 0.0;
    u[1] = (U * pi / L) * (L / 2.0 - z);
    u[2] = (U * pi / L) * (y - L / 2.0);
  } else if (s->vel_kind == ORC_VEL_DEFORM) {
    double U = s->velU, T = s->velT;
    double xh = (double)x / s->n[0], yh = (double)y / s->n[1], zh = (double)z / s->n[2];
    double t = (double)n * U / s->n[0];
    double ct = cos(pi * t / T);
    double sx = sin(pi * xh), sy = sin(pi * yh), sz = sin(pi * zh);
    u[0] = 2.0 * U * sx * sx * sin(2 * pi * yh) * sin(2 * pi * zh) * ct;
    u[1] = -U * sin(2 * pi * xh) * sy * sy * sin(2 * pi * zh) * ct;
    u[2] = -U * sin(2 * pi * xh) * sin(2 * pi * yh) * sz * sz * ct;
  }
}

int orc_set_velocity(orc_t* s, int kind, const double* u_field, double U, double T) {
  if (!s) return ORC_E_INVAL;
  if (kind < ORC_VEL_ZERO || kind > ORC_VEL_DEFORM || (kind == ORC_VEL_FIELD && !u_field) ||
      (kind == ORC_VEL_DEFORM && !(T > 0))) {
    snprintf(s->err, sizeof s->err, "invalid velocity specification");
    return ORC_E_INVAL;
  }
  s->vel_kind = kind;
  s->velU = U;
  s->velT = T;
  if (kind == ORC_VEL_FIELD) {
    if (!s->ufield) s->ufield = malloc(3 * s->N * sizeof(double));
    if (!s->ufield) return ORC_E_NOMEM;
    memcpy(s->ufield, u_field, 3 * s->N * sizeof(double));
  }
  return ORC_OK;
}

/* ---------------- S1-S4: macroscopic quantities at level n ---------------- */

static void compute_macro(orc_t* s) {
  const long N = s->N;
  const double rl = s->p.rho_l, rg = s->p.rho_g;
  /* S1: Eqs. 13, 14 */
#pragma omp parallel for
  for (long n = 0; n < N; ++n) {
    double phi = 0.0;
    for (int i = 0; i < 7; ++i) phi += s->f[i * N + n];
    s->phi[n] = phi;
    s->rho[n] = (1.0 + phi) / 2.0 * rl + (1.0 - phi) / 2.0 * rg;
  }
  /* S2: Eq. 2 with the Laplacian of Eq. 36 */
#pragma omp parallel for
  for (int z = 0; z < s->n[2]; ++z)
    for (int y = 0; y < s->n[1]; ++y)
      for (int x = 0; x < s->n[0]; ++x) {
        long n = idx(s, x, y, z);
        double phi = s->phi[n];
        s->mu[n] = 4.0 * s->beta * phi * (phi - 1.0) * (phi + 1.0) - s->kappa * lap_at(s, s->phi, x, y, z);
      }
  /* S3, S4 */
#pragma omp parallel for
  for (int z = 0; z < s->n[2]; ++z)
    for (int y = 0; y < s->n[1]; ++y)
      for (int x = 0; x < s->n[0]; ++x) {
        long n = idx(s, x, y, z);
        double u[3], gr[3], F[3];
        if (s->mode == ORC_CHE_ONLY) {
          prescribed_u(s, x, y, z, s->step, u);
          for (int a = 0; a < 3; ++a) {
            s->u[a * N + n] = u[a];
            s->F[a * N + n] = 0.0;
            s->gradrho[a * N + n] = 0.0;
          }
          s->pr[n] = 0.0;
          continue;
        }
        double gphi[3];
        grad_at(s, s->phi, x, y, z, gphi);
        grad_at(s, s->rho, x, y, z, gr);
        double lapmu = lap_at(s, s->mu, x, y, z);
        double mu = s->mu[n], rho = s->rho[n];
        double Fs[3], G[3], j[3] = {0, 0, 0}, sum_nz = 0.0;
        for (int a = 0; a < 3; ++a) {
          Fs[a] = mu * gphi[a];                            /* F_s = mu grad phi (after Eq. 28) */
          G[a] = (rho - s->p.rho_ref) * s->p.gravity[a]; /* external force */
        }
        for (int i = 0; i < s->q; ++i) {
          double gi = s->g[i * N + n];
          for (int a = 0; a < 3; ++a) j[a] += C_LAT * s->cg[i][a] * gi;
          if (i != 0) sum_nz += gi;
        }
        /* Eq. 29 */
        double denom = rho - 0.25 * s->drho * s->p.mobility * lapmu;
        for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * (Fs[a] + G[a])) / denom;
        /* F_a = 0.5 (rho_A - rho_B) M lap(mu) u (after Eq. 28); F = F_s + F_a + G */
        for (int a = 0; a < 3; ++a) F[a] = Fs[a] + 0.5 * s->drho * s->p.mobility * lapmu * u[a] + G[a];
        /* Eq. 30 */
        double ugr = u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2];
        s->pr[n] = CS2_G / (1.0 - s->wg[0]) * (sum_nz + 0.5 * ugr + rho * s_of_cw(s->cg[0], s->wg[0], u));
        for (int a = 0; a < 3; ++a) {
          s->u[a * N + n] = u[a];
          s->F[a * N + n] = F[a];
          s->gradrho[a * N + n] = gr[a];
        }
      }
}

/* ---------------- S5-S8 ---------------- */

static int check_finite(orc_t* s) {
  int bad = 0;
  long N = s->N;
#pragma omp parallel for reduction(| : bad)
  for (long k = 0; k < 7 * N; ++k) bad |= !isfinite(s->f[k]);
#pragma omp parallel for reduction(| : bad)
  for (long k = 0; k < s->q * N; ++k) bad |= !isfinite(s->g[k]);
  return bad;
}

static void step_once(orc_t* s) {
  const long N = s->N;
  compute_macro(s);
#pragma omp parallel for
  for (long n = 0; n < N; ++n) {
    double u[3], phi = s->phi[n], mu = s->mu[n];
    for (int a = 0; a < 3; ++a) u[a] = s->u[a * N + n];
    /* S5: Eq. 34 applied to phi u, then the history moves on */
    double dphiu[3];
    for (int a = 0; a < 3; ++a) {
      dphiu[a] = phi * u[a] - s->phiu[a * N + n];
      s->phiu[a * N + n] = phi * u[a];
    }
    /* S6: m = M f; m* = m - S^f (m - m^eq) + (I - S^f/2) mR; f* = M^-1 m*  (Eqs. 11, 15, 17, 18) */
    double fl[7], m[7], meq[7], mR[7], ms[7];
    for (int i = 0; i < 7; ++i) fl[i] = s->f[i * N + n];
    for (int r = 0; r < 7; ++r) {
      m[r] = 0.0;
      for (int i = 0; i < 7; ++i) m[r] += M7[r][i] * fl[i];
    }
    orc_meq_f(s->p.A, s->eta, phi, mu, u, meq);
    orc_mR(dphiu, mR);
    for (int r = 0; r < 7; ++r) ms[r] = m[r] - s->sf[r] * (m[r] - meq[r]) + (1.0 - s->sf[r] / 2.0) * mR[r];
    for (int i = 0; i < 7; ++i) {
      double v = 0.0;
      for (int r = 0; r < 7; ++r) v += M7_INV[i][r] * ms[r];
      s->fpost[i * N + n] = v;
    }
    if (s->mode == ORC_CHE_ONLY) continue;
    /* S7: m = Gamma g; m* = m - S^g (m - m^eq) + (I - S^g/2) mT; g* = Gamma^-1 m*  (Eqs. 20, 27, 31, 32) */
    double gl[19], mg[19], mgeq[19], mT[19], mgs[19], gr[3], F[3];
    for (int i = 0; i < s->q; ++i) gl[i] = s->g[i * N + n];
    for (int a = 0; a < 3; ++a) {
      gr[a] = s->gradrho[a * N + n];
      F[a] = s->F[a * N + n];
    }
    if (s->q == 19) {
      /* D3Q19: m = Gamma_19 g, m^eq = Gamma_19 g^eq (Eq. 21), m_T = Gamma_19 T
       * (Eq. 28); m* = m - S(m - m^eq) + (I - S/2) m_T; g* = Gamma_19^-1 m* */
      double geq[19], T[19];
      geq_of(s, s->pr[n], s->rho[n], u, geq);
      T_of(s, u, gr, F, T);
      for (int r = 0; r < 19; ++r) {
        mg[r] = mgeq[r] = mT[r] = 0.0;
        for (int i = 0; i < 19; ++i) {
          mg[r] += G19[r][i] * gl[i];
          mgeq[r] += G19[r][i] * geq[i];
          mT[r] += G19[r][i] * T[i];
        }
        mgs[r] = mg[r] - s->lg[r] * (mg[r] - mgeq[r]) + (1.0 - s->lg[r] / 2.0) * mT[r];
      }
      for (int i = 0; i < 19; ++i) {
        double v = 0.0;
        for (int r = 0; r < 19; ++r) v += G19_INV[i][r] * mgs[r];
        s->gpost[i * N + n] = v;
      }
      continue;
    }
    for (int r = 0; r < 15; ++r) {
      mg[r] = 0.0;
      for (int i = 0; i < 15; ++i) mg[r] += G15[r][i] * gl[i];
    }
    orc_meq_g(s->pr[n], s->rho[n], u, mgeq);
    if (s->p.forcing == ORC_FORCING_EQ28) { /* Gamma T of Eq. 28, untruncated */
      double T[15];
      T_of(s, u, gr, F, T);
      for (int r = 0; r < 15; ++r) {
        mT[r] = 0.0;
        for (int i = 0; i < 15; ++i) mT[r] += G15[r][i] * T[i];
      }
    } else {
      orc_mT(u, gr, F, mT);
    }
    for (int r = 0; r < 15; ++r)
      mgs[r] = mg[r] - s->lg[r] * (mg[r] - mgeq[r]) + (1.0 - s->lg[r] / 2.0) * mT[r];
    for (int i = 0; i < 15; ++i) {
      double v = 0.0;
      for (int r = 0; r < 15; ++r) v += G15_INV[i][r] * mgs[r];
      s->gpost[i * N + n] = v;
    }
  }
  /* S8: Eq. 16 (and the left-hand side of Eq. 20): f_i(x + c_i) = f*_i(x);
   * a population leaving through a wall returns to x in the opposite direction */
#pragma omp parallel for
  for (int z = 0; z < s->n[2]; ++z)
    for (int y = 0; y < s->n[1]; ++y)
      for (int x = 0; x < s->n[0]; ++x) {
        long n = idx(s, x, y, z);
        int q[3], p[3] = {x, y, z};
        for (int i = 0; i < 7; ++i) {
          int wall = 0;
          for (int a = 0; a < 3; ++a) {
            q[a] = p[a] + C7[i][a];
            if (q[a] < 0 || q[a] >= s->n[a]) {
              if (s->bc[a] == ORC_WALL) wall = 1;
              else q[a] = (q[a] + s->n[a]) % s->n[a];
            }
          }
          if (wall) s->f[OPP7[i] * N + n] = s->fpost[i * N + n];
          else s->f[i * N + idx(s, q[0], q[1], q[2])] = s->fpost[i * N + n];
        }
        if (s->mode == ORC_CHE_ONLY) continue;
        for (int i = 0; i < s->q; ++i) {
          int wall = 0;
          for (int a = 0; a < 3; ++a) {
            q[a] = p[a] + s->cg[i][a];
            if (q[a] < 0 || q[a] >= s->n[a]) {
              if (s->bc[a] == ORC_WALL) wall = 1;
              else q[a] = (q[a] + s->n[a]) % s->n[a];
            }
          }
          if (wall) s->g[s->oppg[i] * N + n] = s->gpost[i * N + n];
          else s->g[i * N + idx(s, q[0], q[1], q[2])] = s->gpost[i * N + n];
        }
      }
  s->step++;
}

int orc_step(orc_t* s, int nsteps) {
  if (!s || nsteps < 0) return ORC_E_INVAL;
  if (!s->have_params || !s->have_init) {
    snprintf(s->err, sizeof s->err, "step before set_params/init");
    return ORC_E_STATE;
  }
  for (int k = 0; k < nsteps; ++k) {
    step_once(s);
    if (check_finite(s)) {
      snprintf(s->err, sizeof s->err, "non-finite population after step %ld", s->step);
      return ORC_E_NONFINITE;
    }
  }
  return ORC_OK;
}

/* ---------------- initialisation and read-out ---------------- */

int orc_init(orc_t* s, const double* phi0, const double* u0) {
  if (!s || !phi0) return ORC_E_INVAL;
  if (!s->have_params) {
    snprintf(s->err, sizeof s->err, "init before set_params");
    return ORC_E_STATE;
  }
  const long N = s->N;
  /* mu_0 from phi_0 (Eq. 2 with Eq. 36) */
  double* lap = malloc(N * sizeof(double));
  if (!lap) return ORC_E_NOMEM;
  orc_grad_lap(s, phi0, NULL, lap);
  s->step = 0;
#pragma omp parallel for
  for (int z = 0; z < s->n[2]; ++z)
    for (int y = 0; y < s->n[1]; ++y)
      for (int x = 0; x < s->n[0]; ++x) {
        long n = idx(s, x, y, z);
        double phi = phi0[n];
        double mu = 4.0 * s->beta * phi * (phi - 1.0) * (phi + 1.0) - s->kappa * lap[n];
        double u[3] = {0, 0, 0};
        if (s->mode == ORC_CHE_ONLY) prescribed_u(s, x, y, z, 0, u);
        else if (u0) for (int a = 0; a < 3; ++a) u[a] = u0[a * N + n];
        double rho = (1.0 + phi) / 2.0 * s->p.rho_l + (1.0 - phi) / 2.0 * s->p.rho_g;
        double feq[7], geq[19];
        orc_feq(s->p.A, s->eta, phi, mu, u, feq); /* Eq. 5 */
        for (int i = 0; i < 7; ++i) s->f[i * N + n] = feq[i];
        geq_of(s, 0.0, rho, u, geq); /* Eq. 21 with p = 0 */
        for (int i = 0; i < s->q; ++i) s->g[i * N + n] = (s->mode == ORC_CHE_ONLY) ? 0.0 : geq[i];
        for (int a = 0; a < 3; ++a) s->phiu[a * N + n] = phi * u[a];
      }
  free(lap);
  s->have_init = 1;
  return ORC_OK;
}

int orc_read(orc_t* s, int field, double* out) {
  if (!s || !out || field < ORC_PHI || field > ORC_P) return ORC_E_INVAL;
  if (!s->have_init) return ORC_E_STATE;
  compute_macro(s);
  const long N = s->N;
  const double* src = NULL;
  switch (field) {
    case ORC_PHI: src = s->phi; break;
    case ORC_RHO: src = s->rho; break;
    case ORC_MU: src = s->mu; break;
    case ORC_UX: src = s->u; break;
    case ORC_UY: src = s->u + N; break;
    case ORC_UZ: src = s->u + 2 * N; break;
    case ORC_P: src = s->pr; break;
  }
  memcpy(out, src, N * sizeof(double));
  return ORC_OK;
}

int orc_totals(orc_t* s, double out[7]) {
  if (!s || !out) return ORC_E_INVAL;
  if (!s->have_init) return ORC_E_STATE;
  compute_macro(s);
  const long N = s->N;
  for (int k = 0; k < 7; ++k) out[k] = 0.0;
  for (long n = 0; n < N; ++n) out[0] += s->phi[n];
  if (s->mode == ORC_CHE_ONLY) return ORC_OK;
  for (long n = 0; n < N; ++n)
    for (int i = 0; i < s->q; ++i)
      for (int a = 0; a < 3; ++a) out[1 + a] += C_LAT * s->cg[i][a] * s->g[i * N + n];
  for (int a = 0; a < 3; ++a)
    for (long n = 0; n < N; ++n) out[4 + a] += s->F[a * N + n];
  return ORC_OK;
}

int orc_front(orc_t* s, double out[2]) {
  if (!s || !out) return ORC_E_INVAL;
  if (!s->have_init) return ORC_E_STATE;
  compute_macro(s);
  int found = 0;
  double lo = 0.0, hi = 0.0;
  for (int y = 0; y < s->n[1]; ++y)
    for (int x = 0; x < s->n[0]; ++x)
      for (int z = 0; z + 1 < s->n[2]; ++z) {
        double a = s->phi[idx(s, x, y, z)], b = s->phi[idx(s, x, y, z + 1)];
        if ((a < 0.0) == (b < 0.0)) continue;
        /* phi is linear between the layer centres z + 1/2 and z + 3/2 */
        double zc = (z + 0.5) + a / (a - b);
        if (!found || zc < lo) lo = zc;
        if (!found || zc > hi) hi = zc;
        found = 1;
      }
  out[0] = found ? lo : -1.0;
  out[1] = found ? hi : -1.0;
  return ORC_OK;
}

int orc_get_state(const orc_t* s, double* f, double* g, double* phiu) {
  if (!s) return ORC_E_INVAL;
  if (f) memcpy(f, s->f, 7 * s->N * sizeof(double));
  if (g) memcpy(g, s->g, s->q * s->N * sizeof(double));
  if (phiu) memcpy(phiu, s->phiu, 3 * s->N * sizeof(double));
  return ORC_OK;
}

int orc_set_state(orc_t* s, const double* f, const double* g, const double* phiu) {
  if (!s) return ORC_E_INVAL;
  if (f) memcpy(s->f, f, 7 * s->N * sizeof(double));
  if (g) memcpy(s->g, g, s->q * s->N * sizeof(double));
  if (phiu) memcpy(s->phiu, phiu, 3 * s->N * sizeof(double));
  return ORC_OK;
}

int orc_set_threads(int n) {
  if (n < 1) return -1;
  omp_set_num_threads(n);
  return 0;
}

int orc_get_threads(void) { return omp_get_max_threads(); }
