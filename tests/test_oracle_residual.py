"""The Poisson residual of the oracle (ora_residual), the measure of the
residual stop test that is offered beside the successive change of
Algorithm 1 step 3: r(x) = sum_i (2 w_i / c_s^2) eps_i (psi(x + c_i) - psi(x))
+ q(x) in the flux form of the D2Q9 lattice, eps_i the harmonic mean of
eps(phi) at both ends, relative to the magnitudes of its terms.

Pins: the converged potential of layered permittivity, which is the series-
resistance profile (test_oracle_physics), is the residual's exact zero, for
either potential scheme; an early-stopped potential has a residual many times
the converged one; and a loop with the residual stop test ends at the first
iteration whose residual is below the tolerance."""
import numpy as np
import pytest

from paper_2407_01654_amd import workloads as W

pytestmark = pytest.mark.usefixtures("oracle_lib")

CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
WI = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)


def Oracle(*a, **k):
    import oracle
    oracle.set_threads(4)
    return oracle.Oracle(*a, **k)


def flux_residual(phi, psi, q, p):
    """The flux-form residual written out with numpy shifts (walls in y)."""
    eps = p["eps_v"] + phi ** 2 * (2 * phi - 3) * (p["eps_v"] - p["eps_l"])
    ny, nx = psi.shape
    r = q.copy()
    a = np.abs(q).copy()
    for i in range(1, 9):
        xs = (np.arange(nx) + CX[i]) % nx
        ys = np.arange(ny) + CY[i]
        out = (ys < 0) | (ys >= ny)
        yc = np.clip(ys, 0, ny - 1)
        e1 = eps[yc][:, xs]
        pn = psi[yc][:, xs]
        ei = 2 * eps * e1 / (eps + e1)
        pw = np.where(ys < 0, p["psi_bottom"], p["psi_top"])[:, None]
        ghost = 2 * pw - psi[:, xs]           # mirror of (x + cx, y) through the wall
        ei = np.where(out[:, None], eps, ei)
        pn = np.where(out[:, None], ghost, pn)
        t = 2 * WI[i] * 3.0 * ei * (pn - psi)
        r += t
        a += np.abs(t)
    return np.sqrt((r ** 2).sum() / (a ** 2).sum())


@pytest.mark.parametrize("scheme", [W.POT_IMPROVED, W.POT_CONVENTIONAL])
def test_converged_layered_potential_is_the_residual_zero(scheme):
    wl = W.planar_layers(nx=4, ny=64, width=2.0, eps_l=20.0 / 6.0, sigma_v=0.0, sigma_l=0.0,
                         presolve_iters=40000, enable=W.EN_POT, pot_scheme=scheme)
    o = Oracle(wl.params, wl.phi0, wl.q0)
    assert o.residual() < 1e-12
    early = Oracle(dict(wl.params, presolve_iters=50), wl.phi0, wl.q0)
    assert early.residual() > 1e-3


def test_residual_equals_its_definition_and_separates_early_stops():
    """A drop of permittivity ratio 20 (128 x 128): the residual matches the
    definition evaluated on the oracle's fields, and after the one iteration
    the paper's stop test takes on the linear start it is about 70 times the
    converged value (0.06 against 8.6e-4)."""
    res = {}
    for it in (1, 100, 20000):
        wl = W.drop_in_field(n=128, r=16.0, seed=3, S=20.0, R=1.0, jitter=False, presolve_iters=it,
                             enable=W.EN_POT, sigma_l=0.0, sigma_v=0.0)
        o = Oracle(wl.params, wl.phi0, wl.q0)
        f = o.fields()
        res[it] = o.residual()
        assert abs(res[it] - flux_residual(f["phi"], f["psi"], f["rho_e"], wl.params)) <= 1e-9 * res[it]
    assert res[1] > 30 * res[20000]
    assert res[1] > res[100] > res[20000]
    assert res[20000] < 2e-3


def test_residual_stop_test_ends_at_the_first_iteration_below_tol():
    """pot_stop = residual: each loop's recorded stop quantity is below pot_tol
    and the iteration before it was not, on a coupled drop (all four sets)."""
    wl = W.drop_in_field(n=64, r=12.0, seed=3, pot_stop=W.STOP_RESIDUAL, pot_tol=2e-3)
    o = Oracle(wl.params, wl.phi0, wl.q0)
    o.step(30)
    K, r, rp = o.k_history(), o.r_history(), o.r_prev_history()
    assert (r < 2e-3).all()
    assert (rp[K > 1] >= 2e-3).all()
    assert K.max() > 1
    assert o.residual() == r[-1]
