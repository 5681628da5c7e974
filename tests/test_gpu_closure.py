"""The implicit charge closure on the GPU: Eq. (66) with R of the same step,
R = -(sigma/eps) q + B (Eq. 61) solved for q, beside Algorithm 1's lagged
closure.  Parity with the oracle's implicit closure in the normalisation and
tolerances of test_gpu_parity (FP32 1e-5, FP16S 1e-3, inner counts replayed),
including a conductive drop at sigma / eps = 3 where the lagged closure is
unstable, and uniform ohmic relaxation against the trapezoidal closed form."""
import numpy as np
import pytest

from paper_2407_01654_amd import workloads as W
from test_gpu_parity import assert_parity, run_pair

pytestmark = pytest.mark.gpu


def implicit(wl):
    wl.params.update(charge_closure=W.Q_IMPLICIT)
    return wl


def conductive_drop():
    """Drop 8x more conductive than its surroundings with sigma / eps = 3 in
    the drop (charge relaxes within a step), permittivity ratio 2."""
    wl = W.drop_in_field(n=72, r=12.0, seed=3, R=8.0, S=2.0)
    eps_l = wl.params["eps_l"]
    wl.params.update(sigma_l=3.0 * eps_l, sigma_v=3.0 * eps_l / 8.0)
    return implicit(wl)


CASES = {
    "planar": lambda: (implicit(W.planar_layers(steps=200)), 200),
    "drop": lambda: (implicit(W.drop_in_field(n=72, r=12.0, seed=3)), 60),
    "sessile": lambda: (implicit(W.sessile_drop(nx=136, ny=100, r=24.0)), 60),
    "conductive_drop": lambda: (conductive_drop(), 60),
}


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp16s", 1e-3)])
@pytest.mark.parametrize("case", list(CASES))
def test_implicit_closure_parity_replay(case, prec, tol):
    wl, steps = CASES[case]()
    ora, sim, K = run_pair(wl, steps, prec=prec, launch=dict(block_x=64, band_y=16, device_loop=1))
    assert_parity(ora, sim, wl.params, tol)
    assert np.array_equal(sim.k_history(0), K)


def test_implicit_and_lagged_instances_in_one_batch():
    """The closure is per instance: a batch holding both runs each exactly as
    a handle of its own (bit for bit)."""
    from paper_2407_01654_amd import lbm
    a = W.drop_in_field(n=72, r=12.0, seed=3)
    b = implicit(W.drop_in_field(n=72, r=12.0, seed=3))
    for w in (a, b):
        w.params.update(presolve_iters=50)
    print("\n[case] mixed closures, drop 72x72, 30 steps", flush=True)
    both = lbm.Simulation([a.params, b.params], [a.phi0, b.phi0], [a.q0, b.q0])
    for i in range(2):
        both.set_replay(i, np.full(30, 3, dtype=np.int32))
    both.step(30)
    for i, w in enumerate((a, b)):
        one = lbm.Simulation(w.params, w.phi0, w.q0)
        one.set_replay(0, np.full(30, 3, dtype=np.int32))
        one.step(30)
        fa, fb = both.fields(i), one.fields(0)
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (i, k)
    assert not np.array_equal(both.fields(0)["rho_e"], both.fields(1)["rho_e"])


@pytest.mark.parametrize("k", [0.5, 4.0])
def test_implicit_closure_ohmic_relaxation_closed_form(k):
    """Uniform charge in a uniform medium relaxes as q0 ((1 - k/2)/(1 + k/2))^n,
    k = sigma / eps (FP32: relative 1e-5 of q0 over 12 steps)."""
    from paper_2407_01654_amd import lbm
    n, eps = 64, 0.5
    p = W.base_params(n, n, walls_y=0, enable=W.EN_NP, sigma_v=k * eps, sigma_l=k * eps, eps_v=eps,
                      eps_l=eps, alpha_q=0.01, psi_bottom=0.0, psi_top=0.0, charge_closure=W.Q_IMPLICIT)
    print(f"\n[case] ohmic relaxation k={k}", flush=True)
    sim = lbm.Simulation(p, np.zeros((n, n)), np.ones((n, n)))
    a = (1.0 - 0.5 * k) / (1.0 + 0.5 * k)
    for step in range(1, 13):
        sim.step(1)
        q = sim.fields(0, mask=32)["rho_e"].astype(np.float64)
        assert np.abs(q - a ** step).max() < 1e-5, (step, q.max(), a ** step)
