/*
 * lbm_ehd -- coupled phase-field lattice Boltzmann time step for two-phase
 * electrohydrodynamics on AMD Instinct MI355X (gfx950).
 *
 * Method: Xiong, Wang, Huang, Luo, "A thermodynamically consistent phase-field
 * lattice Boltzmann method for two-phase electrohydrodynamic flows"
 * (arXiv:2407.01654).  One outer step is Algorithm 1 of Sec. 5: the
 * Cahn-Hilliard set g (Eq. 45-49), the electric-potential set h with its
 * discrete forcing term (Eq. 55-59) iterated until the stop test of Algorithm 1
 * step 3 holds, the Nernst-Planck set l (Eq. 60-66) and the hydrodynamic set f
 * (Eq. 38-44), with the isotropic gradient/Laplacian stencils of Sec. 3.2 and
 * the wetting condition of Sec. 4 (Eq. 72).
 *
 * Conventions shared by every entry point:
 *  - Pure C ABI.  No exceptions cross it; every call returns an lbm_ehd_status
 *    (negative = error, positive = warning).  A handle is not thread-safe.
 *  - Device memory is owned by the caller: one workspace buffer of the size
 *    lbm_ehd_workspace_bytes() reports, alive until lbm_ehd_destroy().  The
 *    library owns only the small host handle.
 *  - All device work is ordered on the caller's hipStream_t given to
 *    lbm_ehd_init (NULL = the legacy default stream).  lbm_ehd_step returns once
 *    the work is enqueued, except where noted (stepping, fields and statistics
    synchronise it).
 *  - Lattice units, dx = dt = 1.  Node (x, y) at integer coordinates; y walls
 *    are half-way, at y = -1/2 and y = ny - 1/2.  x is periodic.
 *  - Host field arrays are row-major [ny][nx] (x fastest); several instances
 *    are concatenated in instance order.
 */
#ifndef LBM_EHD_H
#define LBM_EHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_EHD_ABI_VERSION 10

typedef enum {
  LBM_EHD_OK = 0,
  LBM_EHD_W_NOT_CONVERGED = 1, /* an inner potential loop stopped at pot_max_iter (sticky) */
  LBM_EHD_W_DIVERGED = 2,      /* some instances turned non-finite: they are retired (skipped from
                                  then on, fields left as they were) and the others continue (sticky) */
  LBM_EHD_E_INVAL = -1,        /* invalid argument or parameter set */
  LBM_EHD_E_WORKSPACE = -2,    /* workspace missing, too small or misaligned */
  LBM_EHD_E_HIP = -3,          /* a HIP runtime call failed */
  LBM_EHD_E_DIVERGED = -4,     /* every instance turned non-finite (order parameter, charge or
                                  potential sums, or the stop quantity) (sticky) */
  LBM_EHD_E_STATE = -5         /* the handle is in an unusable state (sticky) */
} lbm_ehd_status;

/* enable bits: which distribution sets advance (all four for the full method) */
enum { LBM_EHD_EN_CH = 1, LBM_EHD_EN_POT = 2, LBM_EHD_EN_NP = 4, LBM_EHD_EN_HYDRO = 8 };

/* population storage */
enum {
  LBM_EHD_PREC_FP32 = 0,  /* all populations in FP32 */
  LBM_EHD_PREC_FP16S = 1  /* rest populations FP32; moving ones FP16 as scaled deviations
                             e = (pop / w_i - ref_set) * scale_set */
};

/* potential scheme of the inner loop (Sec. 3.3); both solve the Poisson
   equation div(eps(phi) grad psi) + q = 0 at the steady state of the loop */
enum {
  LBM_EHD_POT_IMPROVED = 0,     /* the paper's scheme, Eq. (56)-(59): fixed tau_h = 1/2 + eps_v / c_s^2,
                                   discrete forcing with eps_hat(phi), source w-bar_i q */
  LBM_EHD_POT_CONVENTIONAL = 1  /* the conventional scheme the paper improves on: local relaxation time
                                   from eps(phi) = chi c_s^2 (tau(x) - 1/2), no forcing, source
                                   w-bar_i q / chi (the Chapman-Enskog expansion of Appendix A applied
                                   to it recovers the same Poisson equation) */
};

/* closure of the charge density, Eq. (66): q = sum_i l_i + R / 2 */
enum {
  LBM_EHD_Q_LAGGED = 0,   /* R of the previous step, as Algorithm 1 step 4 writes it */
  LBM_EHD_Q_IMPLICIT = 1  /* R of the same step: with R = -(sigma/eps) q + B (Eq. 61, B the part
                             free of q) the relation is solved for q,
                             q = (sum l + B/2) / (1 + sigma / (2 eps)); the initial l are
                             l^eq(q0, u0) - w_i R^0 / 2 so that it returns q0.  Uniform ohmic
                             relaxation then follows the trapezoidal rule, stable for any
                             sigma / eps, where the lag is unstable above sigma / eps ~ 2 */
};

/* stop test of the inner potential loop */
enum {
  LBM_EHD_STOP_CHANGE = 0,   /* Algorithm 1 step 3: relative successive change of psi below pot_tol */
  LBM_EHD_STOP_RESIDUAL = 1  /* relative residual of the Poisson equation (lbm_ehd_residual) of the
                                new psi below pot_tol, evaluated after every iteration */
};

/* field selection for lbm_ehd_fields */
enum {
  LBM_EHD_F_PHI = 1, LBM_EHD_F_UX = 2, LBM_EHD_F_UY = 4,
  LBM_EHD_F_P = 8, LBM_EHD_F_PSI = 16, LBM_EHD_F_RHO_E = 32, LBM_EHD_F_ALL = 63
};

/* Problem statement of one simulation (Sec. 2, 3 and 4).  Phase phi = 1 is "l",
   phi = 0 is "v"; density, viscosity and conductivity are linear in phi and the
   permittivity is the Hermite interpolation of Sec. 2 (Remark II). */
typedef struct {
  int32_t nx, ny;          /* lattice size, nx >= 1; ny >= 3 with walls, >= 1 otherwise;
                              4096 * ceil(nx / 64) * ny < 2^30 (32-bit buffer offsets) */
  int32_t walls_y;         /* 0: periodic in y; 1: electrode walls at both y ends */
  double rho_l, rho_v;     /* densities (> 0) */
  double mu_l, mu_v;       /* dynamic viscosities (> 0): tau_f = 1/2 + mu / (rho c_s^2) */
  double sigma_l, sigma_v; /* conductivities (>= 0) */
  double eps_l, eps_v;     /* permittivities (> 0): tau_h = 1/2 + eps_v / c_s^2 */
  double mobility;         /* M (> 0): tau_g = 1/2 + M / c_s^2 */
  double width;            /* interface width W (> 0) */
  double gamma;            /* surface tension (> 0): beta = 12 gamma / W, kappa = 3 gamma W / 2 */
  double alpha_q;          /* charge diffusivity (> 0 when NP is enabled): tau_l = 1/2 + alpha / c_s^2 */
  double psi_bottom, psi_top;          /* electrode potentials (walls only) */
  double theta_bottom_deg, theta_top_deg; /* wetting angles of phase l, 90 = neutral */
  double cos_shift_bottom, cos_shift_top; /* electrowetting shift eta/d added to cos(theta) */
  int32_t enable;          /* LBM_EHD_EN_* bits */
  double pot_tol;          /* stop test of Algorithm 1 step 3 (the paper uses 1e-5): relative
                              successive change of psi below pot_tol; with FP16S storage a loop
                              also ends once that change is within twice the change rounding the
                              stored h to 16 bits alone makes (lbm_ehd_stats_t.floor_stops) */
  int32_t pot_max_iter;    /* cap of one inner loop (>= 1) */
  int32_t presolve_iters;  /* 0: initial potential solve uses the stop test; > 0: exactly this many */
  int32_t pot_scheme;      /* LBM_EHD_POT_*: potential scheme of the inner loop, the same for every
                              instance of a handle */
  double pot_chi;          /* chi of the conventional scheme (> 0; ignored by the improved one) */
  int32_t charge_closure;  /* LBM_EHD_Q_*: closure of Eq. (66); may differ between instances */
  int32_t pot_stop;        /* LBM_EHD_STOP_*: stop test of the inner loop; may differ between
                              instances (the FP16S rounding-floor end applies to the change test) */
} lbm_ehd_params;

/* Per-instance diagnostics, read back by lbm_ehd_stats (synchronises the stream). */
typedef struct {
  int64_t steps;           /* outer steps completed */
  int64_t total_iters;     /* inner potential iterations summed over those steps */
  int32_t presolve_iters;  /* inner iterations of the initial potential solve */
  int32_t last_iters;      /* inner iterations of the last step */
  double last_rel_change;  /* relative potential change of the last inner iteration */
  double sum_phi;          /* FP64 sum of phi^n over the lattice, last step's main pass */
  double sum_q;            /* FP64 sum of q^n over the lattice, same pass */
  int32_t status;          /* lbm_ehd_status of this instance (sticky); E_DIVERGED: retired */
  int32_t floor_stops;     /* inner loops (initial solve included) that ended at the rounding
                              floor of FP16S storage rather than below pot_tol (always 0 in FP32) */
  double residual;         /* with the residual stop test: relative residual after the last inner
                              iteration (NaN with the change test; see lbm_ehd_residual) */
} lbm_ehd_stats_t;

/* Launch shape.  Each 64-lane wavefront advances one tile: a strip of 64
   lattice columns (one per lane; the wave also reads the column on either
   side of it), band_y rows; a workgroup
   holds block_x / 64 such waves working on adjacent tiles independently.
   Stepping proceeds in rounds: in one round every tile performs its instance's
   current phase (main pass or one inner potential iteration), then each
   instance's partial sums are reduced and its next phase decided on the
   device. */
typedef struct {
  int32_t block_x;          /* threads per workgroup: 64, 128 or 256 */
  int32_t band_y;           /* 4 .. 1024 rows per tile */
  int32_t device_loop;      /* 0: the host checks progress after every round;
                               1: rounds run in hipGraph-captured chunks, one
                                  host check per chunk (default) */
  int32_t rounds_per_graph; /* device loop: rounds per captured chunk, 0..100000;
                               0 = automatic: min(2 n_steps + 2, 1024) in the
                               first chunk of a call, then 1/8 of that
                               (8 .. 256) per chunk */
  int32_t band_y_small;     /* 0, or 4 .. 1024: rows per tile of the instances
                               with fewer than small_ny rows */
  int32_t small_ny;         /* >= 0; 0 = band_y for every instance */
  int32_t solo_max_nodes;   /* >= 0; instances of at most this many lattice
                               nodes that stop their inner loop on the
                               successive change are "solo": one workgroup of
                               256 threads advances each of them through a
                               whole stepping call (main passes and inner
                               loops, a workgroup barrier per pass) on a
                               second stream beside the rounds of the others,
                               so that their inner loops do not add rounds;
                               same tiles, arithmetic and order of sums as the
                               rounds, hence the same results bit for bit;
                               0 = none */
  int32_t stagger;          /* 0 or 1; 1: about half of the instances of the
                               rounds (balanced by node count, alternating
                               in instance order) sit out the first round of
                               each stepping call, so that in the steady
                               regime their main passes (bound by HBM
                               traffic) share rounds with the others' inner
                               iterations (bound by vector instructions);
                               results are unchanged bit for bit */
} lbm_ehd_launch;

/* Kernel timing of the stepping rounds, from HIP events recorded on the
   handle's stream around every launch (see lbm_ehd_timing). */
typedef struct {
  double round_ms;          /* summed duration of the round kernels */
  double finalize_ms;       /* summed duration of the per-instance finalize kernels */
  int64_t round_launches;
  int64_t finalize_launches;
  double main_round_ms;     /* rounds in which every active instance ran its main pass */
  int64_t main_rounds;
  double pot_round_ms;      /* rounds in which every active instance ran an inner iteration */
  int64_t pot_rounds;
  int64_t main_passes;      /* instance main passes and inner iterations over the timed rounds */
  int64_t inner_iterations;
} lbm_ehd_timing_t;

typedef struct lbm_ehd lbm_ehd;

/* Bytes of device workspace for n_inst instances p[0..n_inst-1] at precision
   prec (LBM_EHD_PREC_*).  Returns LBM_EHD_E_INVAL for an invalid set. */
int lbm_ehd_workspace_bytes(const lbm_ehd_params* p, int32_t n_inst, int32_t prec, size_t* bytes);

/* Initialises n_inst independent simulations (Algorithm 1 step 1): order
   parameter phi0 and charge q0 (host FP64, concatenated [ny][nx] arrays), and
   optional initial velocity ux0/uy0 (NULL = at rest).  Populations start at
   their equilibria, the potential from a linear guess between the electrodes
   refined by the inner loop.  d_workspace: device memory of at least
   lbm_ehd_workspace_bytes(), 256-byte aligned; stream: hipStream_t or NULL.
   On success *out receives the handle; on any error (LBM_EHD_E_DIVERGED when
   every instance turns non-finite in the initial solve included) *out is NULL
   and nothing needs to be destroyed.  Warnings (W_NOT_CONVERGED, W_DIVERGED)
   stay readable through lbm_ehd_sync.  The call synchronises the stream. */
int lbm_ehd_init(const lbm_ehd_params* p, int32_t n_inst, int32_t prec,
                 const double* phi0, const double* q0, const double* ux0, const double* uy0,
                 void* d_workspace, size_t workspace_bytes, void* stream, lbm_ehd** out);

/* Advances every instance by n_steps outer steps of Algorithm 1 and returns
   when they are done (the stream is synchronised once per round, or once per
   captured chunk of rounds on the device loop).  Returns the sticky status. */
int lbm_ehd_step(lbm_ehd* s, int32_t n_steps);

/* Level-n fields of instance inst (phi, u_x, u_y, p, psi, rho_e; Eq. 49, 43, 44,
   58, 66), those selected by mask, written as consecutive [ny][nx] FP32 planes
   in the order of the LBM_EHD_F_* bits.  out: device pointer if out_on_device,
   else host pointer.  Synchronises the stream. */
int lbm_ehd_fields(lbm_ehd* s, int32_t inst, uint32_t mask, float* out, int32_t out_on_device);

/* Capacity of the fixed device array lbm_ehd_fields_noalloc stages in: 8 Mi
   nodes (32 MiB of FP32 per device). */
#define LBM_EHD_NOALLOC_MAX_NODES (1 << 23)

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): the fields of
   lbm_ehd_fields with out_on_device = 1, from the same kernels, enqueued on
   the handle's stream.  The call allocates nothing (no device or host
   allocation, no workspace area) and does not synchronise: the values are in
   d_out once the stream reaches that point.  The level-n order parameter,
   which the stencils of the other fields need, is staged in a fixed device
   array of LBM_EHD_NOALLOC_MAX_NODES floats that the library holds once per
   device until the process ends; every call on a device shares that array,
   so calls that overlap on one device (several streams or threads) race, and
   the array keeps the last call's values.  d_out: device memory for the
   selected fields, consecutive [ny][nx] FP32 planes in the order of the
   LBM_EHD_F_* bits.  LBM_EHD_E_INVAL for a bad argument or an instance of more
   than LBM_EHD_NOALLOC_MAX_NODES nodes; a sticky error of the handle is
   returned as it is; LBM_EHD_E_HIP if the launch fails. */
int lbm_ehd_fields_noalloc(lbm_ehd* s, int32_t inst, uint32_t mask, float* d_out);

/* Relative residual of the Poisson equation div(eps(phi) grad psi) + q = 0
   (Eq. 52, the equation the inner loop of Algorithm 1 step 3 solves) for the
   current potential of instance inst, with the order parameter and charge of
   its last main pass (phi^0, q^0 before the first step), in the flux form of
   the D2Q9 lattice:
     r(x) = sum_{i=1..8} (2 w_i / c_s^2) eps_i (psi(x + c_i) - psi(x)) + q(x),
   eps_i the harmonic mean of eps(phi) at x and x + c_i (eps(x) where x + c_i
   lies beyond an electrode, psi there the ghost 2 psi_w - psi(x + c_i -
   c_iy e_y)); *out = sqrt(sum r^2) / sqrt(sum s^2), s(x) the sum of the
   magnitudes of the terms of r(x), summed in FP64.  The converged potential
   of layered permittivity is its exact zero; unlike the successive change it
   measures how far psi is from solving the equation.  Synchronises. */
int lbm_ehd_residual(lbm_ehd* s, int32_t inst, double* out);

/* Diagnostics of instance inst (synchronises the stream). */
int lbm_ehd_stats(lbm_ehd* s, int32_t inst, lbm_ehd_stats_t* out);

/* Inner-iteration counts of instance inst: out[0] is the initial solve, then
   one per step, oldest first; at most the last 8192 steps are kept.  Returns
   the number written (<= max) or a negative status. */
int lbm_ehd_k_history(lbm_ehd* s, int32_t inst, int32_t* out, int32_t max);

/* Forces the inner-iteration count of the next n steps of instance inst
   (n <= 8192; n = 0 returns to the stop test).  For bitwise-reproducible
   comparisons with a reference run. */
int lbm_ehd_set_replay(lbm_ehd* s, int32_t inst, const int32_t* iters, int32_t n);

int lbm_ehd_set_launch(lbm_ehd* s, const lbm_ehd_launch* cfg);
int lbm_ehd_get_launch(const lbm_ehd* s, lbm_ehd_launch* cfg);

/* Tile-shape autotuner.  First measures each instance's mean inner
   iterations per step over trial steps on the starting shape.  When some
   instance averages 2 or more, the slowest instances get bands of their own
   (lbm_ehd_set_instance_band): 4 rows for those at 0.8 of the largest mean or
   above, 8 rows for the others at half of it or above.  Then it runs the
   simulation under each candidate launch shape, with those bands in place,
   and keeps the fastest: band_y in {16, 32, 64} for the instances of at least
   160 rows and band_y_small in {4, 8, 16} for the smaller ones (one set only
   when all instances fall on one side).  Last, the per-instance bands stay
   only if the chosen shape runs faster with them than without.  Then, on
   that shape, solo_max_nodes: 0 or the node count of one of the batch's
   lattice sizes up to 192 x 192 nodes; then, with device_loop = 1,
   then, when some instances went solo, the per-instance bands derived
   again from the longest mean loop of the round path alone (kept if
   faster); then rounds_per_graph in {0 (automatic), 8, 32, 128}; last,
   stagger 0 or 1.  Earlier per-instance
   bands are cleared first.  Every timing advances the simulation by
   2 * trial_steps outer steps (real steps: they count in the step counters
   and histories), the first call to capture its graphs, the second timed on
   the host (after synchronising the handle's stream, so that the solo
   kernel's time counts); with n sizes up to the solo bound the search times
   12 + (n + 1) + 1 + 4 + 2 candidates at most; in the searches after the
   band heights a candidate replaces the kept one only when it is faster by
   more than 2 %.  block_x and
   device_loop are kept.  out (may be NULL) receives the chosen shape, which
   stays applied;
   lbm_ehd_get_instance_band reports the band of each instance.  trial_steps
   in 1 .. 10000.  Synchronises. */
int lbm_ehd_autotune(lbm_ehd* s, int32_t trial_steps, lbm_ehd_launch* out);

/* Band height of instance inst's tiles, replacing the one the launch shape
   gives it: band_y in 4 .. 1024, or 0 to follow the launch shape again.  Kept
   across lbm_ehd_set_launch.  Tile shapes do not change the arithmetic of a
   node; only the order of the FP64 partial sums of the stop test and the
   charge and phase totals follows the tiles.  Synchronises the stream.
   LBM_EHD_E_INVAL for a bad instance or band (nothing changes). */
int lbm_ehd_set_instance_band(lbm_ehd* s, int32_t inst, int32_t band_y);

/* Writes the band height instance inst's tiles use now into *band_y. */
int lbm_ehd_get_instance_band(const lbm_ehd* s, int32_t inst, int32_t* band_y);

/* enable = 1: clear the accumulators and time every round kernel and finalize
   kernel from now on (rounds are then launched one per check, directly
   instead of through captured graphs, so that no idle round is timed);
   enable = 0: stop timing.  out (may be NULL) receives the
   accumulated values.  Synchronises the stream. */
int lbm_ehd_timing(lbm_ehd* s, int32_t enable, lbm_ehd_timing_t* out);

/* Waits for all enqueued work; returns the sticky status. */
int lbm_ehd_sync(lbm_ehd* s);

void lbm_ehd_destroy(lbm_ehd* s);
const char* lbm_ehd_strerror(int32_t code);

/* Host-only ABI check: writes sizeof(lbm_ehd_params), sizeof(lbm_ehd_stats_t),
   sizeof(lbm_ehd_launch) and sizeof(lbm_ehd_timing_t) into out[0..n-1]
   (n <= 4) and returns LBM_EHD_ABI_VERSION.  Needs no device. */
int lbm_ehd_abi_sizes(size_t* out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif
