/*
 * orc.h -- FP64 CPU oracle for one time step of the three-dimensional MRT
 * lattice-Boltzmann phase-field model of Liang, Shi & Chai (arXiv:1507.07294):
 * a D3Q7 MRT scheme for the Cahn-Hilliard equation (Sec. II A, Eqs. 4-19) and
 * a D3Q15 MRT scheme for the incompressible Navier-Stokes equations
 * (Sec. II B, Eqs. 20-33), closed by the finite differences of Eqs. 34-36.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference that
 * the GPU library is compared against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * Conventions: lattice units (dx = dt = c = 1).  A node (x,y,z) has index
 * x + nx*(y + ny*z), x fastest.  Every field array is field-major: population
 * i of node n lives at [i*N + n] with N = nx*ny*nz.  All arrays are host
 * memory owned by the caller unless stated otherwise.
 */
#ifndef ORC_H
#define ORC_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_NOMEM = 2, ORC_E_STATE = 4, ORC_E_NONFINITE = 5 };
enum { ORC_PERIODIC = 0, ORC_WALL = 1 };
/* ORC_COUPLED: D3Q7 CHE + D3Q15 NSE (the paper's model); ORC_CHE_ONLY: the
 * interface-tracking runs; ORC_COUPLED_Q19: the NSE on D3Q19, the other
 * lattice the paper names (after Eq. 22): velocities rest, 6 faces (Eq. 23
 * order), 12 edges in antipodal pairs; weights 1/3, 1/18, 1/36; moments of
 * d'Humieres et al. (2002); g^eq (Eq. 21) and T (Eq. 28) transformed exactly
 * (no truncated form of Eq. 32 exists for it); the five stress moments
 * relax at 1/tau_g (Eq. 33), all others at 1, and lambda_g is not used. */
enum { ORC_COUPLED = 0, ORC_CHE_ONLY = 1, ORC_COUPLED_Q19 = 2 };
enum { ORC_PHI = 0, ORC_RHO = 1, ORC_MU = 2, ORC_UX = 3, ORC_UY = 4, ORC_UZ = 5, ORC_P = 6 };
/* prescribed velocity for the interface-tracking runs (Sec. III A-B) */
enum { ORC_VEL_ZERO = 0, ORC_VEL_FIELD = 1, ORC_VEL_ZALESAK = 2, ORC_VEL_DEFORM = 3 };

typedef struct orc_params {
  double sigma;        /* surface tension (Eq. 2) */
  double width;        /* interface thickness D (Eq. 2) */
  double rho_l;        /* density where phi = +1 (Eq. 14) */
  double rho_g;        /* density where phi = -1 (Eq. 14) */
  double mobility;     /* mobility M (Eqs. 1, 19, 28, 29) */
  double A;            /* D3Q7 free parameter, 0 < A < 1/3 (Eq. 8) */
  double s_f[7];       /* S^f diagonal (Eq. 10); s_1 = s_2 = s_3 */
  double nu;           /* kinematic viscosity (Eq. 33): lambda_9..13 = 1/(3 nu + 1/2) */
  double lambda_g[15]; /* S^g diagonal (Eq. 26); entries 9..13 are replaced from nu */
  double gravity[3];   /* body acceleration; G = (rho - rho_ref) * gravity */
  double rho_ref;      /* reference density of the body force (0: G = rho g) */
  /* study switches (0 = the readings of the paper used by default) */
  int stencil;         /* ORC_STENCIL_Q15: Eqs. 35-36 with D3Q15 weights; ORC_STENCIL_Q7: with the
                          D3Q7 weights (central differences, 7-point Laplacian) */
  int forcing;         /* ORC_FORCING_EQ32: the printed moments of Eq. 32; ORC_FORCING_EQ28: Gamma T of
                          Eq. 28 exactly (D3Q15; the D3Q19 variant always uses Gamma T) */
  int lambda_override; /* nonzero: lambda_9..13 come from lambda_g (all equal), not from nu */
} orc_params;

enum { ORC_STENCIL_Q15 = 0, ORC_STENCIL_Q7 = 1 };
enum { ORC_FORCING_EQ32 = 0, ORC_FORCING_EQ28 = 1 };

typedef struct orc_s orc_t;

/* Lattice of nx*ny*nz nodes; bc[a] is ORC_PERIODIC or ORC_WALL (half-way
 * bounce-back) on axis a.  Returns NULL on invalid sizes or no memory. */
orc_t* orc_create(int nx, int ny, int nz, const int bc[3], int mode);
void orc_destroy(orc_t* s);
int orc_set_params(orc_t* s, const orc_params* p);
/* Equilibrium initialisation from phi0[N] and u0[3N] (u0 may be NULL: u = 0),
 * pressure 0, (phi u)_prev = phi0 u0, step counter 0. */
int orc_init(orc_t* s, const double* phi0, const double* u0);
/* CHE-only runs: velocity prescribed at step n.  FIELD copies u_field[3N]. */
int orc_set_velocity(orc_t* s, int kind, const double* u_field, double U, double T);
int orc_step(orc_t* s, int nsteps);
long orc_step_count(const orc_t* s);
/* Macroscopic field at the current time level into out[N]. */
int orc_read(orc_t* s, int field, double* out);
/* out[7] = { sum phi, sum_x sum_i c_i g_i (3), sum F = F_s + F_a + G (3) }. */
int orc_totals(orc_t* s, double out[7]);
/* Spike tip and bubble front of a heavy-over-light layer (Sec. III C):
 * out[0], out[1] = lowest and highest z where phi changes sign between
 * adjacent layers of a column (layer k at z = k + 1/2, linear interpolation,
 * phi = 0 counts as positive); -1, -1 when no column crosses.  Layers are
 * scanned 0..nz-1 without wrapping. */
int orc_front(orc_t* s, double out[2]);
/* D3Q19 tables: velocities c19[19*3], weights w19[19], moment matrix
 * G[19*19] (row-major; any pointer may be NULL). */
void orc_lattice19(int* c19, double* w19, double* G);
/* Eq. 21 on D3Q19 */
void orc_geq19(double p, double rho, const double u[3], double geq[19]);
/* Eq. 28 on D3Q15 (q = 15, the Eq. 23 order) or D3Q19 (q = 19):
 * T[q] for velocity u, grad rho gr and force F = F_s + F_a + G. */
void orc_T(int q, const double u[3], const double gr[3], const double F[3], double* T);
/* Populations at the current level (after streaming): f[7N], g[15N] (g[19N] for ORC_COUPLED_Q19), phiu[3N]
 * holds (phi u) of the previous level.  Any pointer may be NULL. */
int orc_get_state(const orc_t* s, double* f, double* g, double* phiu);
int orc_set_state(orc_t* s, const double* f, const double* g, const double* phiu);
const char* orc_last_error(const orc_t* s);

/* ---- pieces exposed for pinning the oracle against the paper ---- */
/* M (Eq. 9, 7x7 row-major) and Gamma (Eq. 25 re-indexed to the Eq. 23
 * velocity order, 15x15 row-major). */
void orc_matrices(double* M, double* Gamma);
/* c (int triples) and weights of D3Q7 (for parameter A) and D3Q15. */
void orc_lattices(double A, int* c7, double* w7, int* c15, double* w15);
/* derived[6] = { beta, k, tau_f, eta, tau_g, lambda_visc }. */
int orc_derived(const orc_params* p, double* derived);
/* Velocity-space equilibria: f^eq (Eq. 5) and g^eq (Eqs. 21-22). */
void orc_feq(double A, double eta, double phi, double mu, const double u[3], double feq[7]);
void orc_geq(double p, double rho, const double u[3], double geq[15]);
/* Moment-space forms: m^eq_f (Eq. 17), mR (Eq. 18), m^eq_g (Eq. 31), mT (Eq. 32). */
void orc_meq_f(double A, double eta, double phi, double mu, const double u[3], double m[7]);
void orc_mR(const double dphiu[3], double m[7]);
void orc_meq_g(double p, double rho, const double u[3], double m[15]);
void orc_mT(const double u[3], const double grad_rho[3], const double F[3], double m[15]);
/* Isotropic finite differences (Eqs. 35, 36) of chi[N] on the lattice's
 * geometry: grad[3N], lap[N]. */
int orc_grad_lap(const orc_t* s, const double* chi, double* grad, double* lap);
/* Threads of the OpenMP loops (for timing the oracle on a given number of
 * cores): set returns -1 for n < 1; get returns the current maximum. */
int orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
