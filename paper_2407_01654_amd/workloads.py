"""Seeded synthetic workloads for the coupled two-phase EHD lattice Boltzmann step.

This module only builds *inputs*: physical parameters in lattice units and the
initial order-parameter / charge / velocity fields.  It holds none of the
scheme's arithmetic (no equilibria, no collision, no stencils), so both the FP64
oracle and the HIP library can be fed from it without sharing method code.

Lattice units throughout (dx = dt = 1).  Node (x, y) sits at integer
coordinates; walls, when present, are half-way between nodes at y = -1/2 and
y = ny - 1/2.

Parameter choices that the paper leaves open are derived from its dimensionless
groups (Sec. 7.1, the electric capillary number Ca_E = eps_v E0^2 r / gamma and
the Reynolds numbers Re = r^2 rho_v eps_v E0^2 / mu_v^2, Re_E = eps_v^2 E0^2 /
(mu_v sigma_v)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# enable bits: which distribution sets advance
EN_CH, EN_POT, EN_NP, EN_HYDRO = 1, 2, 4, 8
EN_ALL = EN_CH | EN_POT | EN_NP | EN_HYDRO

PARAM_KEYS = (
    "nx", "ny", "walls_y",
    "rho_l", "rho_v", "mu_l", "mu_v", "sigma_l", "sigma_v", "eps_l", "eps_v",
    "mobility", "width", "gamma", "alpha_q",
    "psi_bottom", "psi_top",
    "theta_bottom_deg", "theta_top_deg", "cos_shift_bottom", "cos_shift_top",
    "enable", "pot_tol", "pot_max_iter", "presolve_iters", "pot_scheme", "pot_chi",
    "charge_closure", "pot_stop",
)
POT_IMPROVED, POT_CONVENTIONAL = 0, 1
# closure of q = sum l + R/2 (Eq. 66): R one step behind (Algorithm 1) or at
# the same level, solved for q
Q_LAGGED, Q_IMPLICIT = 0, 1
# stop test of the inner loop: the successive change of Algorithm 1 step 3, or
# the relative residual of the Poisson equation
STOP_CHANGE, STOP_RESIDUAL = 0, 1

EPS_V_DEFAULT = 1.0 / 6.0      # tau_h = 1 with eps_v = c_s^2 (tau_h - 1/2)
ALPHA_Q_FLOOR = 3.3e-3         # keeps tau_l >= 0.51
SIGMA_OVER_EPS_CAP = 0.1       # charge relaxation time >= 10 steps
# Cap of one inner potential loop.  The longest loop of the configs is the
# first outer step of the planar channel (5958 iterations: its initial solve
# stops after one iteration); a loop that stalls ends at the cap with status
# W_NOT_CONVERGED instead of holding the batch up for minutes.
POT_MAX_ITER = 10000
# The batched sweep's loops stay below 220 iterations from the first step on.
SWEEP_POT_MAX_ITER = 2000


def base_params(nx: int, ny: int, **kw) -> dict:
    p = dict(
        nx=int(nx), ny=int(ny), walls_y=1,
        rho_l=1.0, rho_v=1.0, mu_l=1.0 / 6.0, mu_v=1.0 / 6.0,
        sigma_l=0.0, sigma_v=0.0, eps_l=EPS_V_DEFAULT, eps_v=EPS_V_DEFAULT,
        mobility=0.1, width=4.0, gamma=1e-3, alpha_q=0.01,
        psi_bottom=0.0, psi_top=1.0,
        theta_bottom_deg=90.0, theta_top_deg=90.0,
        cos_shift_bottom=0.0, cos_shift_top=0.0,
        enable=EN_ALL, pot_tol=1e-5, pot_max_iter=POT_MAX_ITER, presolve_iters=0,
        pot_scheme=POT_IMPROVED, pot_chi=1.0, charge_closure=Q_LAGGED, pot_stop=STOP_CHANGE,
    )
    p.update(kw)
    unknown = set(p) - set(PARAM_KEYS)
    if unknown:
        raise KeyError(f"unknown parameter(s): {sorted(unknown)}")
    return p


@dataclass
class Workload:
    name: str
    params: dict
    phi0: np.ndarray            # [ny, nx] float64
    q0: np.ndarray              # [ny, nx] float64
    steps: int
    ux0: np.ndarray | None = None
    uy0: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


def _grid(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def tanh_layer(nx, ny, y_if, width, phase_below=1.0):
    """Planar interface at y = y_if; phi = 1 on the side `phase_below` selects."""
    _, y = _grid(nx, ny)
    s = 0.5 - 0.5 * np.tanh(2.0 * (y - y_if) / width)
    return s if phase_below == 1.0 else 1.0 - s


def drop_profile(x, y, nx, cx, cy, r, width, periodic_x=True):
    """phi = 1/2 + 1/2 tanh(2 (r - d) / W) at the points (x, y), the drop
    profile form of Sec. 6.3 (x periodic with period nx)."""
    dx = x - cx
    if periodic_x:
        dx = (dx + nx / 2.0) % nx - nx / 2.0
    d = np.sqrt(dx * dx + (y - cy) ** 2)
    return 0.5 + 0.5 * np.tanh(2.0 * (r - d) / width)


def tanh_drop(nx, ny, cx, cy, r, width, periodic_x=True):
    """drop_profile at the lattice nodes."""
    x, y = _grid(nx, ny)
    return drop_profile(x, y, nx, cx, cy, r, width, periodic_x)


# ---------------------------------------------------------------------------
# Config 1: planar two-layer leaky-dielectric channel
# ---------------------------------------------------------------------------
def planar_layers(nx=8, ny=128, steps=2000, **over) -> Workload:
    """Two superimposed layers (Sec. 6.1): phase 'l' (phi = 1) fills the lower
    half, the walls hold psi = 0 (bottom) and psi = 1 (top).  Ratios
    (l / v): density 1, viscosity 2, permittivity 2, conductivity 5."""
    p = base_params(
        nx, ny, walls_y=1,
        rho_l=1.0, rho_v=1.0, mu_v=1.0 / 6.0, mu_l=2.0 / 6.0,
        eps_v=1.0 / 6.0, eps_l=2.0 / 6.0, sigma_v=0.01, sigma_l=0.05,
        alpha_q=0.01, mobility=0.1, gamma=1e-3, width=4.0,
        psi_bottom=0.0, psi_top=1.0,
    )
    p.update(over)
    phi0 = tanh_layer(nx, ny, ny / 2.0, p["width"], phase_below=1.0)
    q0 = np.zeros((ny, nx))
    return Workload("planar_layers", p, phi0, q0, steps,
                    meta=dict(y_interface=ny / 2.0))


# ---------------------------------------------------------------------------
# Config 2: Gaussian bell charge diffusion (single phase, fully periodic)
# ---------------------------------------------------------------------------
def gaussian_bell(n=64, alpha_q=0.01, steps=None, **over) -> Workload:
    """Charge bell q0 = exp(-|x - c|^2 / (2 s0^2)), s0 = n/16, c = (n/2, n/2),
    periodic both ways, u = 0, no conduction (sigma = 0), potential off.
    Default run length s0^2 / (2 alpha) doubles the bell's variance."""
    s0 = n / 16.0
    if steps is None:
        steps = int(round(s0 * s0 / (2.0 * alpha_q)))
    p = base_params(n, n, walls_y=0, sigma_l=0.0, sigma_v=0.0,
                    alpha_q=alpha_q, enable=EN_NP, psi_bottom=0.0, psi_top=0.0)
    p.update(over)
    x, y = _grid(n, n)
    c = n / 2.0
    q0 = np.exp(-((x - c) ** 2 + (y - c) ** 2) / (2.0 * s0 * s0))
    phi0 = np.zeros((n, n))
    return Workload("gaussian_bell", p, phi0, q0, steps,
                    meta=dict(s0=s0, centre=(c, c)))


# ---------------------------------------------------------------------------
# Drop under a uniform field (configs 3 and 4) and the sessile drop (config 5)
# ---------------------------------------------------------------------------
def drop_params(nx, ny, r, R, S, CaE, rho_ratio=1.0, mu_ratio=1.0,
                dpsi=1.0, eps_v=EPS_V_DEFAULT, Re=1.0, ReE=1e-3,
                alpha_dimless=1e-4, width=4.0, mobility=0.1,
                min_tau_f=0.52, **over) -> dict:
    """Lattice parameters from the dimensionless groups of Sec. 7.1.

    E0 = dpsi / ny; gamma from Ca_E; mu_v from Re; sigma_v from Re_E, capped so
    that sigma / eps <= 0.1 in both phases; charge diffusivity from the
    dimensionless alpha, floored so that tau_l >= 0.51."""
    E0 = abs(dpsi) / ny
    rho_v = 1.0
    gamma = eps_v * E0 * E0 * r / CaE
    mu_v = r * E0 * math.sqrt(rho_v * eps_v / Re)
    rho_l = rho_ratio * rho_v
    mu_l = mu_ratio * mu_v
    cs2 = 1.0 / 3.0
    nu_min = (min_tau_f - 0.5) * cs2
    scale = max(1.0, nu_min / (mu_v / rho_v), nu_min / (mu_l / rho_l))
    mu_v *= scale
    mu_l *= scale
    sigma_v = eps_v * eps_v * E0 * E0 / (mu_v * ReE)
    eps_l = S * eps_v
    sigma_cap = SIGMA_OVER_EPS_CAP * eps_v / max(1.0, R / S)
    sigma_v = min(sigma_v, sigma_cap)
    sigma_l = R * sigma_v
    alpha_q = max(alpha_dimless * eps_v * r * r * E0 * E0 / mu_v, ALPHA_Q_FLOOR)
    p = base_params(nx, ny, walls_y=1, rho_l=rho_l, rho_v=rho_v, mu_l=mu_l,
                    mu_v=mu_v, sigma_l=sigma_l, sigma_v=sigma_v, eps_l=eps_l,
                    eps_v=eps_v, mobility=mobility, width=width, gamma=gamma,
                    alpha_q=alpha_q)
    p.update(over)
    return p


def drop_in_field(n=512, r=None, seed=3, steps=20000, R=None, S=None, CaE=None,
                  rho_ratio=1.0, mu_ratio=1.0, jitter=True, width=4.0, **over) -> Workload:
    """Config 3: centred drop (radius n/8 by default) between electrodes
    psi = 0 (bottom) and psi = 1 (top), periodic sides.

    Draw order from PCG64(seed): log10 R, log10 S in U[-1, 1], Ca_E in
    U[0.05, 0.4], then the centre jitter in U[-1/2, 1/2]^2."""
    rng = np.random.default_rng(seed)
    lr, ls = rng.uniform(-1.0, 1.0, size=2)
    ca = rng.uniform(0.05, 0.4)
    jx, jy = rng.uniform(-0.5, 0.5, size=2)
    R = 10.0 ** lr if R is None else R
    S = 10.0 ** ls if S is None else S
    CaE = ca if CaE is None else CaE
    r = n / 8.0 if r is None else r
    if not jitter:
        jx = jy = 0.0
    cx, cy = n / 2.0 + jx, n / 2.0 + jy
    p = drop_params(n, n, r, R, S, CaE, rho_ratio=rho_ratio, mu_ratio=mu_ratio,
                    width=width, **over)
    phi0 = tanh_drop(n, n, cx, cy, r, width)
    q0 = np.zeros((n, n))
    return Workload("drop_in_field", p, phi0, q0, steps,
                    meta=dict(R=R, S=S, CaE=CaE, r=r, centre=(cx, cy)))



def deformation_drop(R, S, CaE, n=200, r=None, rho_ratio=2.0, mu_ratio=1.0, gamma=1e-3, width=5.0,
                     eps_v=EPS_V_DEFAULT, steps=100000, **over) -> Workload:
    """Drop deformation study of Sec. 7.1 (Table 1, Fig. 8): a drop of radius
    r = n / 8 (the cavity is eight radii wide) centred between electrodes,
    periodic sides, density ratio 2, viscosity ratio 1, surface tension
    gamma = 1e-3, W = 5, M = 0.1, Re = 1, Re_E = 1e-3.  The surface tension is
    held fixed, so the electrode difference follows Ca_E:
    E0^2 = Ca_E gamma / (eps_v r), psi_top - psi_bottom = E0 n."""
    r = n / 8.0 if r is None else r
    E0 = math.sqrt(CaE * gamma / (eps_v * r))
    dpsi = E0 * n
    p = drop_params(n, n, r, R, S, CaE, rho_ratio=rho_ratio, mu_ratio=mu_ratio, dpsi=dpsi,
                    eps_v=eps_v, width=width, psi_bottom=0.0, psi_top=dpsi)
    p.update(over)
    phi0 = tanh_drop(n, n, n / 2.0, n / 2.0, r, width)
    return Workload("deformation_drop", p, phi0, np.zeros((n, n)), steps,
                    meta=dict(R=R, S=S, CaE=CaE, r=r, centre=(n / 2.0, n / 2.0), mu_ratio=mu_ratio))


BATCH_SIDES = (64, 96, 128, 192, 256, 384)


def batch_sweep(n_inst=512, seed=4, steps=5000, sides=BATCH_SIDES, width=4.0):
    """Config 4: independent drops of uneven lattice sizes.

    One PCG64(seed) stream, drawn instance by instance in this order: side
    (uniform over `sides`), log10 R, log10 S in U[-1, 1], Ca_E in U[0.05, 0.4],
    density ratio in U[1, 10], viscosity ratio in U[1, 10].  Drop radius N/4,
    centred, electrodes psi = 0 / 1."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        n = int(sides[rng.integers(0, len(sides))])
        lr, ls = rng.uniform(-1.0, 1.0, size=2)
        ca = rng.uniform(0.05, 0.4)
        rr = rng.uniform(1.0, 10.0)
        mr = rng.uniform(1.0, 10.0)
        R, S = 10.0 ** lr, 10.0 ** ls
        r = n / 4.0
        p = drop_params(n, n, r, R, S, ca, rho_ratio=rr, mu_ratio=mr, width=width,
                        pot_max_iter=SWEEP_POT_MAX_ITER)
        phi0 = tanh_drop(n, n, n / 2.0, n / 2.0, r, width)
        q0 = np.zeros((n, n))
        out.append(Workload(f"batch[{k}]", p, phi0, q0, steps,
                            meta=dict(R=R, S=S, CaE=ca, r=r, rho_ratio=rr,
                                      mu_ratio=mr, index=k)))
    return out


def oracle_subset(batch, n=16):
    """Instances checked against the oracle: the first n, unless a side class
    would be missing, in which case the first instance of each missing class
    replaces the latest-index pick of an over-represented class."""
    pick = list(range(min(n, len(batch))))
    have = {batch[i].params["nx"] for i in pick}
    for side in sorted({w.params["nx"] for w in batch}):
        if side in have:
            continue
        first = next(i for i, w in enumerate(batch) if w.params["nx"] == side)
        counts = {}
        for i in pick:
            counts.setdefault(batch[i].params["nx"], []).append(i)
        big = max(counts.values(), key=len)
        pick.remove(big[-1])
        pick.append(first)
        have.add(side)
    return sorted(pick)


def sessile_drop(nx=2048, ny=4096, r=None, steps=50000, width=5.0, theta_deg=60.0,
                 **over) -> Workload:
    """Config 5: reversed-electrowetting drop on the bottom electrode.

    Semicircular drop (radius nx/8 by default) centred on the wall surface
    (x = nx/2, y = -1/2); bottom wall psi = +1/2 with a 60 degree wetting angle
    for the drop phase, top wall psi = -1/2 and neutral; ratios (drop /
    ambient) density 10, viscosity 10, permittivity 20, conductivity 10;
    W = 5; Ca_E = 0.2."""
    r = nx / 8.0 if r is None else r
    p = drop_params(nx, ny, r, R=10.0, S=20.0, CaE=0.2, rho_ratio=10.0,
                    mu_ratio=10.0, dpsi=1.0, width=width,
                    psi_bottom=0.5, psi_top=-0.5,
                    theta_bottom_deg=theta_deg, theta_top_deg=90.0)
    p.update(over)
    phi0 = tanh_drop(nx, ny, nx / 2.0, -0.5, r, width)
    q0 = np.zeros((ny, nx))
    return Workload("sessile_drop", p, phi0, q0, steps, meta=dict(r=r))


def electrowetting_drop(nx=200, ny=100, r=25.0, theta_deg=120.0, eta_over_d=0.0, field=True,
                        width=4.0, gamma=0.05, nu=0.1, sigma_l=0.5, eps_v=1.0, steps=60000,
                        **over) -> Workload:
    """Equilibrium electrowetting (Sec. 6.3): a conductive drop (phase l) in an
    insulating gas on the bottom electrode, semicircle centred on the wall
    surface.  Ratios (drop / gas): density 100, viscosity 100 (equal kinematic
    viscosity nu), permittivity 81; W = 4; Young angle theta_deg on the bottom
    wall, top wall neutral.  With `field`, the bottom electrode holds psi = 1
    and the top psi = 0, and the bottom wetting condition carries the Lippmann
    shift eta / d (Eq. 69, as an effective liquid-solid tension); without it
    both electrodes hold 0 and the shift is off (the relaxation phase)."""
    p = base_params(nx, ny, walls_y=1, rho_l=100.0, rho_v=1.0, mu_l=100.0 * nu, mu_v=nu,
                    sigma_l=sigma_l, sigma_v=0.0, eps_l=81.0 * eps_v, eps_v=eps_v,
                    mobility=0.1, width=width, gamma=gamma, alpha_q=0.01,
                    psi_bottom=1.0 if field else 0.0, psi_top=0.0,
                    theta_bottom_deg=theta_deg, theta_top_deg=90.0,
                    cos_shift_bottom=eta_over_d if field else 0.0)
    p.update(over)
    phi0 = tanh_drop(nx, ny, nx / 2.0, -0.5, r, width)
    return Workload("electrowetting_drop", p, phi0, np.zeros((ny, nx)), steps,
                    meta=dict(r=r, theta_deg=theta_deg, eta_over_d=eta_over_d, field=field))


def shear_wave(n=64, amp=1e-3, nu=1.0 / 6.0, steps=400) -> Workload:
    """Single-phase shear wave u_x = A sin(2 pi y / n), fully periodic, hydrodynamics only."""
    p = base_params(n, n, walls_y=0, rho_l=1.0, rho_v=1.0, mu_l=nu, mu_v=nu,
                    enable=EN_HYDRO, psi_bottom=0.0, psi_top=0.0)
    _, y = _grid(n, n)
    ux0 = amp * np.sin(2.0 * np.pi * y / n)
    return Workload("shear_wave", p, np.zeros((n, n)), np.zeros((n, n)), steps,
                    ux0=ux0, uy0=np.zeros((n, n)), meta=dict(amp=amp, nu=nu))


def all_configs_small():
    """Reduced sizes of every config, for parity tests the oracle finishes in
    seconds; they keep each config's boundary types and ratios and span several
    GPU tiles plus ragged edges."""
    return {
        "planar": planar_layers(nx=8, ny=128, steps=200),
        "gauss": gaussian_bell(n=32, steps=100),
        "drop": drop_in_field(n=72, r=12.0, seed=3, steps=100),
        "sessile": sessile_drop(nx=136, ny=100, r=24.0, steps=100),
    }
