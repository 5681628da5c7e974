/*
 * FP64 reference ("oracle") of the coupled phase-field lattice Boltzmann step for
 * two-phase electrohydrodynamics of Xiong, Wang, Huang and Luo (arXiv:2407.01654).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or helper with the HIP library; the two meet only through the seeded
 * inputs (parameters and initial fields) that both are given.
 *
 * Layout of every field argument: row-major [ny][nx] doubles, x fastest.
 * Populations: [9][ny][nx], direction-major, directions ordered as Eq. (37).
 */
#ifndef LBM_EHD_ORACLE_H
#define LBM_EHD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_EN_CH = 1, ORA_EN_POT = 2, ORA_EN_NP = 4, ORA_EN_HYDRO = 8 };
/* Sec. 3.3: the paper's potential scheme (Eq. 56-59), or the conventional one
   it improves on, with eps(phi) = chi c_s^2 (tau - 1/2) setting a local
   relaxation time */
enum { ORA_POT_IMPROVED = 0, ORA_POT_CONVENTIONAL = 1 };
/* Charge closure, Eq. (66): q = sum l + R/2.  Algorithm 1 step 4 takes R one
   step behind (lagged); with R = -sigma q / eps + B (Eq. 61) at the same level
   the relation is linear in q and is solved for it (implicit). */
enum { ORA_Q_LAGGED = 0, ORA_Q_IMPLICIT = 1 };

typedef struct {
  int32_t nx, ny;
  int32_t walls_y;                 /* 0: periodic in y; 1: half-way walls at y=-1/2, ny-1/2 */
  double rho_l, rho_v, mu_l, mu_v; /* phase phi=1 is "l", phi=0 is "v" (Eq. 36) */
  double sigma_l, sigma_v, eps_l, eps_v;
  double mobility, width, gamma, alpha_q;   /* M, W, surface tension, charge diffusivity */
  double psi_bottom, psi_top;      /* electrode potentials on the y walls */
  double theta_bottom_deg, theta_top_deg;   /* Young angles of Eq. (72), 90 = neutral */
  double cos_shift_bottom, cos_shift_top;   /* electrowetting shift eta/d of Sec. 4 */
  int32_t enable;                  /* ORA_EN_* bits: which sets advance */
  double pot_tol;                  /* stop test of Algorithm 1 step 3 */
  int32_t pot_max_iter;
  int32_t presolve_iters;          /* 0: stop test; >0: exactly this many at init */
  int32_t pot_scheme;              /* ORA_POT_*: potential scheme of the inner loop */
  double pot_chi;                  /* chi of the conventional scheme (> 0) */
  int32_t charge_closure;          /* ORA_Q_*: how Eq. (66) is closed */
  int32_t pot_stop;                /* ORA_STOP_*: stop test of the inner loop */
} ora_params;

/* Stop test of the inner loop: the successive change of Algorithm 1 step 3,
   or the relative residual of the Poisson equation (ora_residual) below
   pot_tol. */
enum { ORA_STOP_CHANGE = 0, ORA_STOP_RESIDUAL = 1 };

typedef struct ora_state ora_state;

/* Returns NULL and sets *status < 0 on invalid parameters.  ux0/uy0 may be NULL. */
ora_state* ora_create(const ora_params* p, const double* phi0, const double* q0,
                      const double* ux0, const double* uy0, int* status);
void ora_destroy(ora_state* s);
/* Advances n outer steps.  Returns 0, 1 if an inner loop hit pot_max_iter, -4 on NaN. */
int ora_step(ora_state* s, int n);
/* Level-n fields [6][ny][nx]: phi, ux, uy, p, psi, rho_e. */
void ora_fields(const ora_state* s, double* out);
/* Forces the inner-iteration count of the next n steps (n = 0 clears). */
void ora_set_replay(ora_state* s, const int32_t* iters, int n);
/* Inner-iteration counts: entry 0 is the initial potential solve, then one per step. */
int ora_k_history(const ora_state* s, int32_t* out, int max);
/* Final relative change of each inner loop, same indexing as ora_k_history. */
int ora_r_history(const ora_state* s, double* out, int max);
/* Relative change of the second-to-last iteration of each inner loop (how
   close the loop came to stopping one iteration earlier; infinity for a loop
   of one iteration), same indexing as ora_k_history. */
int ora_r_prev_history(const ora_state* s, double* out, int max);
int64_t ora_steps_done(const ora_state* s);
/* Threads of the per-node loops (results do not depend on it). */
void ora_set_threads(int n);
int ora_max_threads(void);
/* Relative residual of the Poisson equation div(eps(phi) grad psi) + q = 0
   (Eq. 52) for the current potential with the order parameter and charge of
   the last main sub-step (phi^0, q^0 before the first step), in the flux form
   of the D2Q9 lattice:
     r(x) = sum_{i=1..8} (2 w_i / c_s^2) eps_i (psi(x + c_i) - psi(x)) + q(x),
   eps_i the harmonic mean of eps(phi) at x and x + c_i (eps(x) where x + c_i
   lies beyond a wall, psi there the electrode ghost 2 psi_w - psi(x + c_i -
   c_iy e_y)); returns sqrt(sum r^2) / sqrt(sum s^2), s(x) the sum of the
   magnitudes of the terms of r(x).  The converged potential of layered
   permittivity is its exact zero. */
double ora_residual(const ora_state* s);
/* Raw state for budget tests: which = 0 g, 1 l, 2 f, 3 h ([9][N] each);
   10 Gamma^{n-1}, 11 R^{n-1}, 12 Fx^{n-1}, 13 Fy^{n-1}, 14 Jx^{n-1}, 15 Jy^{n-1},
   16 psi ([N] each).  Returns the count copied or -1. */
int ora_get(const ora_state* s, int which, double* out);

/* Pointwise building blocks, exported for identity tests (9 outputs each). */
void ora_lattice(int32_t* cx, int32_t* cy, double* w);
void ora_geq(double phi, double mu_c, double* out);
void ora_heq(double psi, double* out);
void ora_leq(double q, double ux, double uy, double* out);
void ora_feq(double p, double rho, double ux, double uy, double* out);
void ora_rbar(double ux, double uy, double grx, double gry, double Fx, double Fy, double* out);
void ora_source_g(double Gamma, double* out);
/* Isotropic gradient and Laplacian of Sec. 3.2 over a whole [ny][nx] field with
   the state's boundaries; kind 0 = order parameter (wetting ghosts), 1 = potential
   (Dirichlet ghosts). */
void ora_stencil(const ora_state* s, const double* field, int kind,
                 double* gx, double* gy, double* lap);

#ifdef __cplusplus
}
#endif
#endif
