/*
 * FP64 reference ("oracle") of the coupled phase-field lattice Boltzmann step for
 * two-phase electrohydrodynamics (Xiong, Wang, Huang, Luo, arXiv:2407.01654).
 *
 * TEST INFRASTRUCTURE ONLY -- see lbm_ehd_oracle.h.  Plain loops over the lattice
 * in natural order; every sub-step is a separate function named after the
 * paper's quantity and cites the equation it follows.  Nothing is fused,
 * blocked or reordered beyond what Algorithm 1 states.
 *
 * Readings taken where the paper is silent, ambiguous or garbled:
 *  - Coupling (Algorithm 1): every sub-step of step n uses level-n quantities;
 *    the only lags are q^{n} = sum l + R^{n-1}/2 and rho u^{n} = sum c f +
 *    F^{n-1}/2 as printed.  The potential sub-step uses eps_hat(phi^n) and q^n.
 *  - Algorithm 1 step 3 writes grad(phi^n) in the h forcing; Eq. (56) and the
 *    local formula Eq. (59) use the potential gradient, which is taken here.
 *  - tau_h = 1/2 + eps_v/c_s^2 and tau_l = 1/2 + alpha/c_s^2 (dt = 1), the
 *    Chapman-Enskog results (A.12) and (B.14).
 *  - E in the chemical potential, the force and the charge source is minus the
 *    isotropic-stencil gradient of the stored potential; grad eps, grad sigma,
 *    grad rho follow from grad phi by the chain rule.
 *  - Walls: half-way bounce-back for f, g, l; anti-bounce-back with the
 *    electrode potential for h; ghost rows for the stencils: order parameter
 *    from the wetting condition Eq. (72) across the half-way wall, potential
 *    by linear extrapolation through the wall value.
 *  - Electrowetting enters as cos(theta_eff) = cos(theta_Y) + cos_shift.
 *  - Stop test: sqrt(sum (psi_new - psi_cur)^2 / sum psi_cur^2) < tol, with the
 *    denominator floored at 1e-300 N, at least one iteration, and a cap.  As
 *    a variant, the relative residual of the Poisson equation in the flux
 *    form of the lattice (ora_residual) below tol instead.
 *  - Initial state: h at equilibrium of a linear potential guess (zero when y
 *    is periodic), potential solved by the inner loop, g = g^eq(phi0, mu0),
 *    l = l^eq(q0, u0), f = f^eq(p = 0, u0); lagged F, R = 0, lagged
 *    Gamma = u0.grad(phi0) and J = q0 u0 so the backward time differences of
 *    the first step vanish.
 *  - Implicit charge closure (a variant beside Algorithm 1's lag): Eq. (66)
 *    with R of Eq. (61) at the same level, R = -(sigma/eps) q + B with
 *    B = (sigma/eps) grad eps . E - grad sigma . E, solved for q:
 *    q = (sum l + B/2) / (1 + sigma / (2 eps)).  Its initial l are
 *    l^eq(q0, u0) - w_i R^0 / 2, so that the closure returns q0 at n = 0.
 */
#include "lbm_ehd_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Loops over nodes or rows run on several threads when the lattice is large
   enough to pay for it.  Every node's update reads only the previous state and
   writes only its own outputs, so the result does not depend on the thread
   count; the sums of the stop test and of the state check stay serial and in
   node order. */
#define PAR_MIN_NODES 4096

/* ---- D2Q9 lattice, Eq. (37) and the weights stated after it ---- */
enum { Q = 9 };
static const int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double w[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int opp[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double cs2 = 1.0 / 3.0;
/* diffusional weights of the potential source, Sec. 3.3 */
static const double varpi[Q] = {0.0, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};

struct ora_state {
  ora_params p;
  int N;
  double beta, kappa;          /* Sec. 2.2: beta = 12 gamma / W, kappa = 3 gamma W / 2 */
  double tau_g, tau_h, tau_l;  /* Eq. (48), (A.12), (B.14) */
  double cos_b, cos_t;         /* effective wall cosines */
  double *g, *l, *f, *h;       /* pre-collision populations, [9][N] */
  double *gs, *ls, *fs, *hs;   /* post-collision populations */
  double *psi;                 /* electric potential at level n */
  double *phi, *qn;            /* phi^n and q^n of the current step */
  double *Gam_prev, *R_prev, *Fx_prev, *Fy_prev, *Jx_prev, *Jy_prev;
  double *Gam_new, *R_new, *Fx_new, *Fy_new, *Jx_new, *Jy_new;
  double *psi_cur;             /* potential before an inner iteration */
  int64_t step;
  int32_t *k_hist;
  double *r_hist, *r_prev_hist;
  int n_hist, cap_hist;
  int32_t *replay;
  int n_replay, replay_pos;
};

#define IDX(s, x, y) ((y) * (s)->p.nx + (x))
#define POP(a, s, i, n) ((a)[(size_t)(i) * (size_t)(s)->N + (size_t)(n)])

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* ---- material laws, Sec. 2 Remark II and Eq. (36) ---- */
static double rho_of(const ora_state* s, double phi) {
  return phi * (s->p.rho_l - s->p.rho_v) + s->p.rho_v;
}
static double mu_of(const ora_state* s, double phi) {
  return phi * (s->p.mu_l - s->p.mu_v) + s->p.mu_v;
}
static double sigma_of(const ora_state* s, double phi) {
  return phi * (s->p.sigma_l - s->p.sigma_v) + s->p.sigma_v;
}
/* Hermite interpolation eps(phi) = eps_v + phi^2 (2 phi - 3)(eps_v - eps_l) */
static double eps_of(const ora_state* s, double phi) {
  return s->p.eps_v + phi * phi * (2.0 * phi - 3.0) * (s->p.eps_v - s->p.eps_l);
}
/* eps_hat of Eq. (55) */
static double eps_hat_of(const ora_state* s, double phi) {
  return phi * phi * (2.0 * phi - 3.0) * (s->p.eps_v - s->p.eps_l);
}
/* d eps / d phi = 6 phi (phi - 1)(eps_v - eps_l) */
static double deps_of(const ora_state* s, double phi) {
  return 6.0 * phi * (phi - 1.0) * (s->p.eps_v - s->p.eps_l);
}

/* ---- ghost values across a half-way wall ---- */
/* Wetting condition Eq. (72), n_w . grad phi = -sqrt(2 beta / kappa) cos(theta)
   (phi - phi^2), n_w the inward normal.  Across the wall n_w . grad phi ~
   phi_adj - phi_ghost; phi at the wall from the second-order extrapolation
   (3 phi_adj - phi_next)/2, clamped to [0, 1]. */
static double phi_ghost(const ora_state* s, double phi_adj, double phi_next, double cos_theta) {
  double phw = 0.5 * (3.0 * phi_adj - phi_next);
  if (phw < 0.0) phw = 0.0;
  if (phw > 1.0) phw = 1.0;
  double slope = -sqrt(2.0 * s->beta / s->kappa) * cos_theta * (phw - phw * phw);
  return phi_adj - slope;
}

/* order parameter at (x, y), y in [-1, ny] */
static double phi_at(const ora_state* s, const double* phi, int x, int y) {
  int nx = s->p.nx, ny = s->p.ny;
  x = wrap(x, nx);
  if (!s->p.walls_y) return phi[IDX(s, x, wrap(y, ny))];
  if (y < 0) return phi_ghost(s, phi[IDX(s, x, 0)], phi[IDX(s, x, 1)], s->cos_b);
  if (y >= ny) return phi_ghost(s, phi[IDX(s, x, ny - 1)], phi[IDX(s, x, ny - 2)], s->cos_t);
  return phi[IDX(s, x, y)];
}

/* potential at (x, y): linear extrapolation through the electrode value */
static double psi_at(const ora_state* s, const double* psi, int x, int y) {
  int nx = s->p.nx, ny = s->p.ny;
  x = wrap(x, nx);
  if (!s->p.walls_y) return psi[IDX(s, x, wrap(y, ny))];
  if (y < 0) return 2.0 * s->p.psi_bottom - psi[IDX(s, x, 0)];
  if (y >= ny) return 2.0 * s->p.psi_top - psi[IDX(s, x, ny - 1)];
  return psi[IDX(s, x, y)];
}

/* Isotropic second-order gradient and Laplacian, Sec. 3.2:
   grad T = sum_{i!=0} w_i c_i T(x + c_i) / c_s^2,
   lap T  = sum_{i!=0} 2 w_i [T(x + c_i) - T(x)] / c_s^2. */
static void grad_lap_at(const ora_state* s, const double* field, int kind, int x, int y,
                        double* gx, double* gy, double* lap) {
  double centre = kind == 0 ? phi_at(s, field, x, y) : psi_at(s, field, x, y);
  double ax = 0.0, ay = 0.0, al = 0.0;
  for (int i = 1; i < Q; ++i) {
    double v = kind == 0 ? phi_at(s, field, x + cx[i], y + cy[i])
                         : psi_at(s, field, x + cx[i], y + cy[i]);
    ax += w[i] * cx[i] * v;
    ay += w[i] * cy[i] * v;
    al += 2.0 * w[i] * (v - centre);
  }
  *gx = ax / cs2;
  *gy = ay / cs2;
  *lap = al / cs2;
}

/* ---- equilibria and forcing terms ---- */
/* Eq. (46): g_0^eq = phi - (1 - w_0) mu_c, g_i^eq = w_i mu_c */
void ora_geq(double phi, double mu_c, double* out) {
  for (int i = 0; i < Q; ++i) out[i] = i == 0 ? phi - (1.0 - w[0]) * mu_c : w[i] * mu_c;
}
/* Eq. (57): h_0^eq = (w_0 - 1) psi, h_i^eq = w_i psi */
void ora_heq(double psi, double* out) {
  for (int i = 0; i < Q; ++i) out[i] = i == 0 ? (w[0] - 1.0) * psi : w[i] * psi;
}
/* Eq. (65): l_i^eq = w_i q (1 + c_i . u / c_s^2) */
void ora_leq(double q, double ux, double uy, double* out) {
  for (int i = 0; i < Q; ++i) out[i] = w[i] * q * (1.0 + (cx[i] * ux + cy[i] * uy) / cs2);
}
/* Eq. (41): s_i(u) = w_i [c.u/c_s^2 + (c.u)^2/(2 c_s^4) - u.u/(2 c_s^2)] */
static double s_i(int i, double ux, double uy) {
  double cu = cx[i] * ux + cy[i] * uy, uu = ux * ux + uy * uy;
  return w[i] * (cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}
/* Eq. (40): f_0^eq = (w_0 - 1) p / c_s^2 + rho s_0, f_i^eq = w_i p / c_s^2 + rho s_i */
void ora_feq(double p, double rho, double ux, double uy, double* out) {
  for (int i = 0; i < Q; ++i)
    out[i] = (i == 0 ? (w[0] - 1.0) : w[i]) * p / cs2 + rho * s_i(i, ux, uy);
}
/* Eq. (39): Rbar_i = w_i [u.grad rho + c_i.F/c_s^2 + (u grad rho):(c_i c_i - c_s^2 I)/c_s^2] */
void ora_rbar(double ux, double uy, double grx, double gry, double Fx, double Fy, double* out) {
  for (int i = 0; i < Q; ++i) {
    double ugr = ux * grx + uy * gry;
    double cF = cx[i] * Fx + cy[i] * Fy;
    /* (u grad rho) : (c c - c_s^2 I) = (c.u)(c.grad rho) - c_s^2 u.grad rho */
    double contr = (cx[i] * ux + cy[i] * uy) * (cx[i] * grx + cy[i] * gry) - cs2 * ugr;
    out[i] = w[i] * (ugr + cF / cs2 + contr / cs2);
  }
}
/* Eq. (47): G_i = w_i (u.grad phi)[-1 + I:(c_i c_i - c_s^2 I)/(2 c_s^2)], D = 2 */
void ora_source_g(double Gamma, double* out) {
  for (int i = 0; i < Q; ++i) {
    double trace = (double)(cx[i] * cx[i] + cy[i] * cy[i]) - 2.0 * cs2;
    out[i] = w[i] * Gamma * (-1.0 + trace / (2.0 * cs2));
  }
}

void ora_lattice(int32_t* ocx, int32_t* ocy, double* ow) {
  for (int i = 0; i < Q; ++i) {
    ocx[i] = cx[i];
    ocy[i] = cy[i];
    ow[i] = w[i];
  }
}

/* ---- streaming ---- */
/* pop_i(x, n+1) = pop*_i(x - c_i, n); half-way bounce-back where x - c_i lies
   beyond a y wall. */
static void stream_bounce_back(const ora_state* s, const double* post, double* pre) {
  int nx = s->p.nx, ny = s->p.ny;
  for (int i = 0; i < Q; ++i)
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int xs = wrap(x - cx[i], nx), ys = y - cy[i];
        int n = IDX(s, x, y);
        if (s->p.walls_y && (ys < 0 || ys >= ny)) {
          POP(pre, s, i, n) = POP(post, s, opp[i], n);
        } else {
          ys = wrap(ys, ny);
          POP(pre, s, i, n) = POP(post, s, i, IDX(s, xs, ys));
        }
      }
}

/* Same, with anti-bounce-back at the electrodes: h_i = -h*_{opp i} + 2 w_i psi_wall. */
static void stream_anti_bounce_back(const ora_state* s, const double* post, double* pre) {
  int nx = s->p.nx, ny = s->p.ny;
  for (int i = 0; i < Q; ++i)
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int xs = wrap(x - cx[i], nx), ys = y - cy[i];
        int n = IDX(s, x, y);
        if (s->p.walls_y && (ys < 0 || ys >= ny)) {
          double psi_w = ys < 0 ? s->p.psi_bottom : s->p.psi_top;
          POP(pre, s, i, n) = -POP(post, s, opp[i], n) + 2.0 * w[i] * psi_w;
        } else {
          ys = wrap(ys, ny);
          POP(pre, s, i, n) = POP(post, s, i, IDX(s, xs, ys));
        }
      }
}

/* ---- Algorithm 1 step 3: potential sub-step ---- */
/* psi = sum_{i != 0} h_i / (1 - w_0), Eq. (58) */
static double psi_from_h(const ora_state* s, const double* h, int n) {
  double a = 0.0;
  for (int i = 1; i < Q; ++i) a += POP(h, s, i, n);
  return a / (1.0 - w[0]);
}

/* One collision of the conventional potential scheme at every node (the model
   Sec. 3.3 starts from): BGK towards the equilibrium of Eq. (57) with the local
   relaxation time given by eps(phi) = chi c_s^2 (tau - 1/2), no forcing term,
   and the source w-bar_i q / chi.  The Chapman-Enskog expansion of Appendix A
   with a node-dependent tau gives div(c_s^2 (tau - 1/2) grad psi) + q / chi = 0,
   i.e. div(eps grad psi) + q = 0. */
static void collide_h_conventional(ora_state* s) {
  const double chi = s->p.pot_chi;
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int n = 0; n < s->N; ++n) {
    double psi = psi_from_h(s, s->h, n);
    s->psi_cur[n] = psi;
    double tau = 0.5 + eps_of(s, s->phi[n]) / (chi * cs2);
    double heq[Q];
    ora_heq(psi, heq);
    for (int i = 0; i < Q; ++i) {
      double hi = POP(s->h, s, i, n);
      POP(s->hs, s, i, n) = hi - (hi - heq[i]) / tau + varpi[i] * s->qn[n] / chi;
    }
  }
}

/* One collision of Eq. (56) at every node, with eps_hat(phi^n) and q^n frozen. */
static void collide_h(ora_state* s) {
  if (s->p.pot_scheme == ORA_POT_CONVENTIONAL) {
    collide_h_conventional(s);
    return;
  }
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int n = 0; n < s->N; ++n) {
    double psi = psi_from_h(s, s->h, n);
    s->psi_cur[n] = psi;
    double eh = eps_hat_of(s, s->phi[n]);
    /* local potential gradient, Eq. (59) / (A.13), from the node's own h */
    double denom = eh + cs2 * s->tau_h;
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < Q; ++i) {
      mx += cx[i] * POP(s->h, s, i, n);
      my += cy[i] * POP(s->h, s, i, n);
    }
    double gpx = -mx / denom, gpy = -my / denom;
    double heq[Q];
    ora_heq(psi, heq);
    for (int i = 0; i < Q; ++i) {
      double hi = POP(s->h, s, i, n);
      double forcing = (eh / cs2) * w[i] * (cx[i] * gpx + cy[i] * gpy) / s->tau_h;
      POP(s->hs, s, i, n) = hi - (hi - heq[i]) / s->tau_h - forcing + varpi[i] * s->qn[n];
    }
  }
}

/* r: relative change of the loop's last iteration; r_prev: of the one before
   it (infinity for a loop of one iteration) */
/* Relative residual of the Poisson equation (see ora_residual in the header)
   for the potential psi, with eps from phi^n and the charge q^n of the
   current step. */
static double residual_of(const ora_state* s, const double* psi) {
  int nx = s->p.nx, ny = s->p.ny;
  double num = 0.0, den = 0.0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = IDX(s, x, y);
      double e0 = eps_of(s, s->phi[n]);
      double r = s->qn[n], a = fabs(s->qn[n]);
      for (int i = 1; i < Q; ++i) {
        int xs = wrap(x + cx[i], nx), ys = y + cy[i];
        double ei, pn;
        if (s->p.walls_y && (ys < 0 || ys >= ny)) {
          double pw = ys < 0 ? s->p.psi_bottom : s->p.psi_top;
          ei = e0;
          pn = 2.0 * pw - psi[IDX(s, xs, y)];
        } else {
          ys = wrap(ys, ny);
          double e1 = eps_of(s, s->phi[IDX(s, xs, ys)]);
          ei = 2.0 * e0 * e1 / (e0 + e1);
          pn = psi[IDX(s, xs, ys)];
        }
        double t = 2.0 * w[i] / cs2 * ei * (pn - psi[n]);
        r += t;
        a += fabs(t);
      }
      num += r * r;
      den += a * a;
    }
  double floor_den = 1e-300 * (double)s->N;
  return sqrt(num / (den > floor_den ? den : floor_den));
}

double ora_residual(const ora_state* s) { return residual_of(s, s->psi); }

static void push_hist(ora_state* s, int k, double r, double r_prev) {
  if (s->n_hist == s->cap_hist) {
    s->cap_hist = s->cap_hist ? 2 * s->cap_hist : 1024;
    s->k_hist = (int32_t*)realloc(s->k_hist, sizeof(int32_t) * s->cap_hist);
    s->r_hist = (double*)realloc(s->r_hist, sizeof(double) * s->cap_hist);
    s->r_prev_hist = (double*)realloc(s->r_prev_hist, sizeof(double) * s->cap_hist);
  }
  s->k_hist[s->n_hist] = k;
  s->r_hist[s->n_hist] = r;
  s->r_prev_hist[s->n_hist] = r_prev;
  s->n_hist++;
}

/* Inner loop of Algorithm 1 step 3: collide-stream h until the relative change
   of the potential falls below pot_tol (or, with the residual stop test, the
   relative residual of the Poisson equation; or exactly `forced`
   iterations).  r records the stop quantity of the loop's last iteration. */
static int potential_substep(ora_state* s, int forced) {
  int k = 0, capped = 0;
  double r = 0.0, r_prev = INFINITY;
  for (;;) {
    ++k;
    if (k > 1) r_prev = r;
    collide_h(s);
    stream_anti_bounce_back(s, s->hs, s->h);
    if (s->p.pot_stop == ORA_STOP_RESIDUAL) {
      /* psi_cur is free again once the collision has used it */
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
      for (int n = 0; n < s->N; ++n) s->psi_cur[n] = psi_from_h(s, s->h, n);
      r = residual_of(s, s->psi_cur);
    } else {
      double num = 0.0, den = 0.0;
      for (int n = 0; n < s->N; ++n) {
        double d = psi_from_h(s, s->h, n) - s->psi_cur[n];
        num += d * d;
        den += s->psi_cur[n] * s->psi_cur[n];
      }
      double floor_den = 1e-300 * (double)s->N;
      r = sqrt(num / (den > floor_den ? den : floor_den));
    }
    if (forced > 0) {
      if (k >= forced) break;
    } else {
      if (r < s->p.pot_tol) break;
      if (k >= s->p.pot_max_iter) {
        capped = 1;
        break;
      }
    }
  }
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int n = 0; n < s->N; ++n) s->psi[n] = psi_from_h(s, s->h, n);
  push_hist(s, k, r, r_prev);
  return capped;
}

/* chemical potential, Eq. (31): 4 beta phi (phi - 1/2)(phi - 1) - kappa lap phi
   - eps'(phi) |E|^2 / 2 */
static double chem_pot(const ora_state* s, double phi, double lap_phi, double Ex, double Ey) {
  return 4.0 * s->beta * phi * (phi - 0.5) * (phi - 1.0) - s->kappa * lap_phi -
         0.5 * deps_of(s, phi) * (Ex * Ex + Ey * Ey);
}

/* B = (sigma/eps) grad eps . E - grad sigma . E, the part of R (Eq. 61) that
   does not depend on q; gE = grad phi . E (grad eps = eps' grad phi) */
static double charge_source_b(const ora_state* s, double phi, double gE) {
  double eps = eps_of(s, phi), sig = sigma_of(s, phi);
  return (sig / eps) * deps_of(s, phi) * gE - (s->p.sigma_l - s->p.sigma_v) * gE;
}

/* q^n at node n from the pre-collision l, Eq. (66): with the lag of Algorithm
   1 step 4, q = sum l + R^{n-1}/2; implicit, q = sum l + R^n/2 with
   R^n = -(sigma/eps) q + B solved for q */
static double charge_of(const ora_state* s, int n, double phi, double gE) {
  double suml = 0.0;
  for (int i = 0; i < Q; ++i) suml += POP(s->l, s, i, n);
  if (s->p.charge_closure == ORA_Q_IMPLICIT) {
    double k = sigma_of(s, phi) / eps_of(s, phi);
    return (suml + 0.5 * charge_source_b(s, phi, gE)) / (1.0 + 0.5 * k);
  }
  return suml + 0.5 * s->R_prev[n];
}

/* ---- Algorithm 1 steps 2, 4, 5: main sub-step at every node ---- */
static void main_substep(ora_state* s) {
  int nx = s->p.nx, ny = s->p.ny;
  int en = s->p.enable;
  /* phi^n = sum_i g_i, Eq. (49) */
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int n = 0; n < s->N; ++n) {
    double a = 0.0;
    for (int i = 0; i < Q; ++i) a += POP(s->g, s, i, n);
    s->phi[n] = a;
  }
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = IDX(s, x, y);
      double phi = s->phi[n];
      double gphx, gphy, lphi, gpsx, gpsy, lpsi;
      grad_lap_at(s, s->phi, 0, x, y, &gphx, &gphy, &lphi);
      grad_lap_at(s, s->psi, 1, x, y, &gpsx, &gpsy, &lpsi);
      double Ex = -gpsx, Ey = -gpsy; /* E = -grad psi, Eq. (32) */
      double rho = rho_of(s, phi);
      double grx = (s->p.rho_l - s->p.rho_v) * gphx, gry = (s->p.rho_l - s->p.rho_v) * gphy;

      /* charge density, Eq. (66) */
      double eps = eps_of(s, phi), sig = sigma_of(s, phi);
      double gE = gphx * Ex + gphy * Ey;
      double q = charge_of(s, n, phi, gE);

      /* rho u^n = sum c f + F^{n-1}/2, Eq. (43) with the lag of step 5 */
      double ux = 0.0, uy = 0.0;
      if (en & ORA_EN_HYDRO) {
        for (int i = 0; i < Q; ++i) {
          ux += cx[i] * POP(s->f, s, i, n);
          uy += cy[i] * POP(s->f, s, i, n);
        }
        ux = (ux + 0.5 * s->Fx_prev[n]) / rho;
        uy = (uy + 0.5 * s->Fy_prev[n]) / rho;
      }
      /* p = c_s^2/(1 - w_0) [sum_{i!=0} f_i + u.grad rho / 2 + rho s_0(u)], Eq. (44) */
      double sumf = 0.0;
      for (int i = 1; i < Q; ++i) sumf += POP(s->f, s, i, n);
      double p = cs2 / (1.0 - w[0]) * (sumf + 0.5 * (ux * grx + uy * gry) + rho * s_i(0, ux, uy));

      double mu_c = chem_pot(s, phi, lphi, Ex, Ey);
      /* F = mu_c grad phi + q E, Eq. (30) */
      double Fx = mu_c * gphx + q * Ex, Fy = mu_c * gphy + q * Ey;
      /* R = -sigma q / eps + (sigma/eps) grad eps . E - grad sigma . E, Eq. (61) */
      double R = -sig * q / eps + charge_source_b(s, phi, gE);
      /* u . grad phi, the argument of G_i in Eq. (47) */
      double Gam = ux * gphx + uy * gphy;
      double Jx = q * ux, Jy = q * uy;

      /* Cahn-Hilliard set, Eq. (45) with the backward difference of d_t G */
      if (en & ORA_EN_CH) {
        double geq[Q], Gn[Q], Gp[Q];
        ora_geq(phi, mu_c, geq);
        ora_source_g(Gam, Gn);
        ora_source_g(s->Gam_prev[n], Gp);
        for (int i = 0; i < Q; ++i) {
          double gi = POP(s->g, s, i, n);
          POP(s->gs, s, i, n) = gi - (gi - geq[i]) / s->tau_g + Gn[i] + 0.5 * (Gn[i] - Gp[i]);
        }
      }
      /* Nernst-Planck set, Eq. (62)-(65) */
      if (en & ORA_EN_NP) {
        double leq[Q];
        ora_leq(q, ux, uy, leq);
        double fac = 1.0 - 1.0 / (2.0 * s->tau_l);
        double dJx = Jx - s->Jx_prev[n], dJy = Jy - s->Jy_prev[n];
        for (int i = 0; i < Q; ++i) {
          double li = POP(s->l, s, i, n);
          double S = fac * w[i] * R;
          double T = fac * w[i] * (cx[i] * dJx + cy[i] * dJy) / cs2;
          POP(s->ls, s, i, n) = li - (li - leq[i]) / s->tau_l + S + T;
        }
      }
      /* hydrodynamic set, Eq. (38)-(42) with the local tau_f */
      if (en & ORA_EN_HYDRO) {
        double tau_f = 0.5 + mu_of(s, phi) / (rho * cs2);
        double feq[Q], rb[Q];
        ora_feq(p, rho, ux, uy, feq);
        ora_rbar(ux, uy, grx, gry, Fx, Fy, rb);
        for (int i = 0; i < Q; ++i) {
          double fi = POP(s->f, s, i, n);
          POP(s->fs, s, i, n) = fi - (fi - feq[i]) / tau_f + (1.0 - 1.0 / (2.0 * tau_f)) * rb[i];
        }
      }
      s->qn[n] = q;
      s->Gam_new[n] = Gam;
      s->R_new[n] = R;
      s->Fx_new[n] = Fx;
      s->Fy_new[n] = Fy;
      s->Jx_new[n] = Jx;
      s->Jy_new[n] = Jy;
    }
  if (en & ORA_EN_CH) stream_bounce_back(s, s->gs, s->g);
  if (en & ORA_EN_NP) stream_bounce_back(s, s->ls, s->l);
  if (en & ORA_EN_HYDRO) stream_bounce_back(s, s->fs, s->f);
  double* t;
#define SWAP(a, b) (t = (a), (a) = (b), (b) = t)
  SWAP(s->Gam_prev, s->Gam_new);
  SWAP(s->R_prev, s->R_new);
  SWAP(s->Fx_prev, s->Fx_new);
  SWAP(s->Fy_prev, s->Fy_new);
  SWAP(s->Jx_prev, s->Jx_new);
  SWAP(s->Jy_prev, s->Jy_new);
#undef SWAP
}

/* ---- life cycle ---- */
static int validate(const ora_params* p) {
  if (p->nx < 1 || p->ny < 1) return -1;
  if (p->walls_y && p->ny < 3) return -1;
  if (p->rho_l <= 0 || p->rho_v <= 0 || p->mu_l <= 0 || p->mu_v <= 0) return -1;
  if (p->eps_l <= 0 || p->eps_v <= 0 || p->mobility <= 0 || p->width <= 0) return -1;
  if (p->gamma < 0 || p->sigma_l < 0 || p->sigma_v < 0) return -1;
  if ((p->enable & ORA_EN_NP) && p->alpha_q <= 0) return -1;
  if (p->pot_max_iter < 1 || p->presolve_iters < 0) return -1;
  if (p->pot_scheme != ORA_POT_IMPROVED && p->pot_scheme != ORA_POT_CONVENTIONAL) return -1;
  if (p->pot_scheme == ORA_POT_CONVENTIONAL && !(p->pot_chi > 0)) return -1;
  if (p->charge_closure != ORA_Q_LAGGED && p->charge_closure != ORA_Q_IMPLICIT) return -1;
  if (p->pot_stop != ORA_STOP_CHANGE && p->pot_stop != ORA_STOP_RESIDUAL) return -1;
  return 0;
}

ora_state* ora_create(const ora_params* p, const double* phi0, const double* q0,
                      const double* ux0, const double* uy0, int* status) {
  if (validate(p) != 0 || !phi0 || !q0) {
    if (status) *status = -1;
    return NULL;
  }
  ora_state* s = (ora_state*)calloc(1, sizeof(ora_state));
  s->p = *p;
  s->N = p->nx * p->ny;
  s->beta = 12.0 * p->gamma / p->width;
  s->kappa = 3.0 * p->gamma * p->width / 2.0;
  s->tau_g = 0.5 + p->mobility / cs2;
  s->tau_h = 0.5 + p->eps_v / cs2;
  s->tau_l = 0.5 + p->alpha_q / cs2;
  s->cos_b = cos(p->theta_bottom_deg * M_PI / 180.0) + p->cos_shift_bottom;
  s->cos_t = cos(p->theta_top_deg * M_PI / 180.0) + p->cos_shift_top;
  size_t N = (size_t)s->N, P = Q * N;
  double** pops[] = {&s->g, &s->l, &s->f, &s->h, &s->gs, &s->ls, &s->fs, &s->hs};
  for (int k = 0; k < 8; ++k) *pops[k] = (double*)calloc(P, sizeof(double));
  double** flds[] = {&s->psi, &s->phi, &s->qn, &s->psi_cur, &s->Gam_prev, &s->R_prev,
                     &s->Fx_prev, &s->Fy_prev, &s->Jx_prev, &s->Jy_prev, &s->Gam_new,
                     &s->R_new, &s->Fx_new, &s->Fy_new, &s->Jx_new, &s->Jy_new};
  for (int k = 0; k < 16; ++k) *flds[k] = (double*)calloc(N, sizeof(double));

  int nx = p->nx, ny = p->ny;
  for (int n = 0; n < s->N; ++n) {
    s->phi[n] = phi0[n];
    s->qn[n] = q0[n];
  }
  /* potential: equilibrium h of a linear guess between the electrodes, then the
     inner loop of Algorithm 1 step 3 with (phi^0, q^0) */
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double guess = 0.0;
      if (p->walls_y) guess = p->psi_bottom + (p->psi_top - p->psi_bottom) * (y + 0.5) / ny;
      double heq[Q];
      ora_heq(guess, heq);
      for (int i = 0; i < Q; ++i) POP(s->h, s, i, IDX(s, x, y)) = heq[i];
      s->psi[IDX(s, x, y)] = guess;
    }
  int st = 0;
  if (p->enable & ORA_EN_POT) st = potential_substep(s, p->presolve_iters);
  else push_hist(s, 0, 0.0, INFINITY);

#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = IDX(s, x, y);
      double phi = s->phi[n];
      double gphx, gphy, lphi, gpsx, gpsy, lpsi;
      grad_lap_at(s, s->phi, 0, x, y, &gphx, &gphy, &lphi);
      grad_lap_at(s, s->psi, 1, x, y, &gpsx, &gpsy, &lpsi);
      double ux = ux0 ? ux0[n] : 0.0, uy = uy0 ? uy0[n] : 0.0;
      if (!(p->enable & ORA_EN_HYDRO)) ux = uy = 0.0;
      double mu_c = chem_pot(s, phi, lphi, -gpsx, -gpsy);
      double geq[Q], leq[Q], feq[Q];
      ora_geq(phi, mu_c, geq);
      ora_leq(q0[n], ux, uy, leq);
      ora_feq(0.0, rho_of(s, phi), ux, uy, feq);
      /* implicit closure: sum l^0 = q0 - R^0 / 2 makes Eq. (66) return q0 */
      double R0 = 0.0;
      if (p->charge_closure == ORA_Q_IMPLICIT)
        R0 = -sigma_of(s, phi) * q0[n] / eps_of(s, phi) +
             charge_source_b(s, phi, -(gphx * gpsx + gphy * gpsy));
      for (int i = 0; i < Q; ++i) {
        POP(s->g, s, i, n) = geq[i];
        POP(s->l, s, i, n) = leq[i] - 0.5 * w[i] * R0;
        POP(s->f, s, i, n) = feq[i];
      }
      s->Gam_prev[n] = ux * gphx + uy * gphy;
      s->Jx_prev[n] = q0[n] * ux;
      s->Jy_prev[n] = q0[n] * uy;
    }
  if (status) *status = st;
  return s;
}

void ora_destroy(ora_state* s) {
  if (!s) return;
  double* all[] = {s->g, s->l, s->f, s->h, s->gs, s->ls, s->fs, s->hs, s->psi, s->phi,
                   s->qn, s->psi_cur, s->Gam_prev, s->R_prev, s->Fx_prev, s->Fy_prev,
                   s->Jx_prev, s->Jy_prev, s->Gam_new, s->R_new, s->Fx_new, s->Fy_new,
                   s->Jx_new, s->Jy_new, s->r_hist, s->r_prev_hist};
  for (size_t k = 0; k < sizeof(all) / sizeof(all[0]); ++k) free(all[k]);
  free(s->k_hist);
  free(s->replay);
  free(s);
}

int ora_step(ora_state* s, int nsteps) {
  int status = 0;
  for (int k = 0; k < nsteps; ++k) {
    main_substep(s);
    if (s->p.enable & ORA_EN_POT) {
      int forced = 0;
      if (s->replay_pos < s->n_replay) forced = s->replay[s->replay_pos++];
      if (potential_substep(s, forced)) status = 1;
    } else {
      push_hist(s, 0, 0.0, INFINITY);
    }
    s->step++;
    double a = 0.0;
    for (int n = 0; n < s->N; ++n) a += s->phi[n] + s->qn[n] + s->psi[n];
    if (!isfinite(a)) return -4;
  }
  return status;
}

void ora_set_replay(ora_state* s, const int32_t* iters, int n) {
  free(s->replay);
  s->replay = NULL;
  s->n_replay = 0;
  s->replay_pos = 0;
  if (n <= 0 || !iters) return;
  s->replay = (int32_t*)malloc(sizeof(int32_t) * n);
  memcpy(s->replay, iters, sizeof(int32_t) * n);
  s->n_replay = n;
}

int ora_k_history(const ora_state* s, int32_t* out, int max) {
  int n = s->n_hist < max ? s->n_hist : max;
  if (out) memcpy(out, s->k_hist, sizeof(int32_t) * n);
  return s->n_hist;
}

int ora_r_history(const ora_state* s, double* out, int max) {
  int n = s->n_hist < max ? s->n_hist : max;
  if (out) memcpy(out, s->r_hist, sizeof(double) * n);
  return s->n_hist;
}

int ora_r_prev_history(const ora_state* s, double* out, int max) {
  int n = s->n_hist < max ? s->n_hist : max;
  if (out) memcpy(out, s->r_prev_hist, sizeof(double) * n);
  return s->n_hist;
}

int64_t ora_steps_done(const ora_state* s) { return s->step; }

void ora_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int ora_max_threads(void) { return omp_get_max_threads(); }

void ora_fields(const ora_state* s, double* out) {
  int nx = s->p.nx, ny = s->p.ny;
  size_t N = (size_t)s->N;
  double* phi = (double*)malloc(sizeof(double) * N);
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int n = 0; n < s->N; ++n) {
    double a = 0.0;
    for (int i = 0; i < Q; ++i) a += POP(s->g, s, i, n);
    phi[n] = a;
  }
#pragma omp parallel for if (s->N >= PAR_MIN_NODES)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = IDX(s, x, y);
      double gphx, gphy, lphi, gpsx, gpsy, lpsi;
      grad_lap_at(s, phi, 0, x, y, &gphx, &gphy, &lphi);
      grad_lap_at(s, s->psi, 1, x, y, &gpsx, &gpsy, &lpsi);
      double rho = rho_of(s, phi[n]);
      double grx = (s->p.rho_l - s->p.rho_v) * gphx, gry = (s->p.rho_l - s->p.rho_v) * gphy;
      double q = charge_of(s, n, phi[n], -(gphx * gpsx + gphy * gpsy));
      double ux = 0.0, uy = 0.0;
      if (s->p.enable & ORA_EN_HYDRO) {
        for (int i = 0; i < Q; ++i) {
          ux += cx[i] * POP(s->f, s, i, n);
          uy += cy[i] * POP(s->f, s, i, n);
        }
        ux = (ux + 0.5 * s->Fx_prev[n]) / rho;
        uy = (uy + 0.5 * s->Fy_prev[n]) / rho;
      }
      double sumf = 0.0;
      for (int i = 1; i < Q; ++i) sumf += POP(s->f, s, i, n);
      double p = cs2 / (1.0 - w[0]) * (sumf + 0.5 * (ux * grx + uy * gry) + rho * s_i(0, ux, uy));
      out[0 * N + n] = phi[n];
      out[1 * N + n] = ux;
      out[2 * N + n] = uy;
      out[3 * N + n] = p;
      out[4 * N + n] = s->psi[n];
      out[5 * N + n] = q;
    }
  free(phi);
}

int ora_get(const ora_state* s, int which, double* out) {
  size_t N = (size_t)s->N;
  const double* src = NULL;
  size_t cnt = N;
  switch (which) {
    case 0: src = s->g; cnt = Q * N; break;
    case 1: src = s->l; cnt = Q * N; break;
    case 2: src = s->f; cnt = Q * N; break;
    case 3: src = s->h; cnt = Q * N; break;
    case 10: src = s->Gam_prev; break;
    case 11: src = s->R_prev; break;
    case 12: src = s->Fx_prev; break;
    case 13: src = s->Fy_prev; break;
    case 14: src = s->Jx_prev; break;
    case 15: src = s->Jy_prev; break;
    case 16: src = s->psi; break;
    default: return -1;
  }
  memcpy(out, src, sizeof(double) * cnt);
  return (int)cnt;
}

void ora_stencil(const ora_state* s, const double* field, int kind, double* gx, double* gy,
                 double* lap) {
  for (int y = 0; y < s->p.ny; ++y)
    for (int x = 0; x < s->p.nx; ++x) {
      int n = IDX(s, x, y);
      grad_lap_at(s, field, kind, x, y, &gx[n], &gy[n], &lap[n]);
    }
}
