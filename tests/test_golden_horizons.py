"""The stored free-running oracle runs of tests/golden (configs 3, 4 and 5
over their declared lengths), against the oracle itself: their first
inner-iteration counts are what the oracle takes on the same seeded inputs,
and their samples are consistent with the stored lattice-wide scalars (every
sampled magnitude within the stored maximum; p's stored maximum taken about
its stored mean).  Runs on the CPU in a few seconds per config."""
import os

import numpy as np
import pytest

from paper_2407_01654_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FIELDS = ("phi", "psi", "rho_e", "ux", "uy", "p")


def load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return np.load(path)


def first_counts(wl, steps):
    import oracle
    ora = oracle.Oracle(wl.params, wl.phi0, wl.q0)
    ora.step(steps)
    return ora.k_history()


def check_samples(g, prefix, names):
    for k in FIELDS:
        top = float(g[f"{prefix}/{k}/absmax"])
        shift = float(g[f"{prefix}/{k}/mean"]) if k == "p" else 0.0
        vals = np.concatenate([g[f"{prefix}/{k}/{n}"].astype(np.float64) for n in names])
        assert np.isfinite(vals).all(), (prefix, k)
        # float32 rounding of the samples: 1e-7 relative
        assert np.abs(vals - shift).max() <= top * (1 + 1e-6) + 1e-30, (prefix, k)


def test_config3_store():
    g = load("config3_horizon.npz")
    K = g["k_history"]
    checks = [int(t) for t in g["checkpoints"]]
    assert checks == list(range(5000, 20001, 5000)) and len(K) == checks[-1] + 1
    assert np.array_equal(first_counts(W.drop_in_field(n=512), 3), K[:4])
    for T in checks:
        check_samples(g, str(T), ("column", "row", "random"))


def test_config4_store():
    g = load("config4_horizon.npz")
    wls = W.batch_sweep(n_inst=512, seed=4)
    sub = [int(i) for i in g["subset"]]
    assert sub == W.oracle_subset(wls, 16) and sorted(int(i) for i in g["done"]) == sorted(sub)
    checks = [int(t) for t in g["checkpoints"]]
    assert checks == list(range(1000, 5001, 1000))
    for i in sub[:4]:
        K = g[f"{i}/k_history"]
        assert len(K) == checks[-1] + 1
        assert np.array_equal(first_counts(wls[i], 2), K[:3]), i
    for i in sub:
        for T in checks:
            check_samples(g, f"{i}/{T}", ("column", "row", "random"))


def test_config5_store():
    g = load("config5_horizon.npz")
    K = g["k_history"]
    checks = [int(t) for t in g["checkpoints"]]
    assert checks == list(range(1000, checks[-1] + 1, 1000)) and len(K) == checks[-1] + 1
    assert np.array_equal(first_counts(W.sessile_drop(), 1), K[:2])
    rows = [f"row{int(y)}" for y in g["rows_y"]]
    for T in checks:
        check_samples(g, str(T), ["column", *rows, "random"])
