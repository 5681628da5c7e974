"""Solo instances: lattices of at most solo_max_nodes nodes advanced by a
workgroup of their own through a whole stepping call, beside the rounds of the
other instances.  They run the same tiles, arithmetic and ordered sums as the
round path, so every result is the same bit for bit; the inner loop's stop
test runs inside the kernel, so free-running counts are compared too.  Parity
with the FP64 oracle (replayed counts) in the normalisation of
test_gpu_parity."""
import numpy as np
import pytest

from paper_2407_01654_amd import workloads as W
from test_gpu_parity import CASES, assert_parity, run_pair

pytestmark = pytest.mark.gpu

BASE = dict(block_x=64, band_y=16, device_loop=1)


def snapshot(sim, n):
    out = []
    for i in range(n):
        st = sim.stats(i)
        out.append((sim.fields(i), sim.k_history(i), {k: st[k] for k in
                    ("steps", "total_iters", "floor_stops", "status", "sum_phi", "sum_q")}))
    return out


def assert_same(a, b, tag):
    for i, ((fa, ka, sa), (fb, kb, sb)) in enumerate(zip(a, b)):
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (tag, i, k)
        assert np.array_equal(ka, kb), (tag, i)
        assert sa == sb, (tag, i, sa, sb)


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_solo_matches_round_path_bitwise(prec):
    """Six drops of the sweep (sides 64, 96, 192), free-running from their
    initial state through the start-up transient (inner loops of tens to
    hundreds of iterations) for 60 steps in calls of 7, 13 and 40: the 64 and
    96 sides solo (device loop and host-steered rounds for the others) against
    the round path only, bit for bit in every field, count and sum."""
    from paper_2407_01654_amd import lbm
    batch = W.batch_sweep(n_inst=6, seed=4, steps=60, sides=(64, 96, 192))
    sides = [w.params["nx"] for w in batch]
    print(f"\n[case] solo {prec}, sides {sides}", flush=True)
    assert any(s <= 96 for s in sides) and any(s > 96 for s in sides)
    runs = {}
    for tag, launch in (("rounds", BASE), ("solo", dict(BASE, solo_max_nodes=96 * 96)),
                        ("solo_host", dict(BASE, device_loop=0, solo_max_nodes=96 * 96))):
        sim = lbm.Simulation([w.params for w in batch], [w.phi0 for w in batch], [w.q0 for w in batch],
                             prec=prec, launch=launch)
        for n in (7, 13, 40):
            sim.step(n)
        runs[tag] = snapshot(sim, len(batch))
        print(f"  {tag}: sum K {[int(r[1][1:].sum()) for r in runs[tag]]}", flush=True)
    assert_same(runs["rounds"], runs["solo"], "solo")
    assert_same(runs["rounds"], runs["solo_host"], "solo_host")


@pytest.mark.parametrize("case,prec,tol", [("drop", "fp32", 1e-5), ("planar", "fp32", 1e-5),
                                           ("drop", "fp16s", 1e-3)])
def test_solo_parity_replay(case, prec, tol):
    """A single instance that is solo (the round path then has nothing to do)
    against the FP64 oracle with its counts replayed."""
    wl, steps = CASES[case]()
    ora, sim, K = run_pair(wl, steps, prec=prec, launch=dict(BASE, solo_max_nodes=1 << 20))
    assert_parity(ora, sim, wl.params, tol)
    assert np.array_equal(sim.k_history(0), K)


def test_solo_instance_retired_and_the_others_continue():
    """A conductive drop (sigma / eps = 3, lagged closure) turns non-finite
    within 60 steps: run solo beside a solo drop and a round-path drop, it is
    retired inside the solo kernel (handle W_DIVERGED, instance E_DIVERGED),
    and the two others advance exactly as on their own."""
    from paper_2407_01654_amd import lbm
    good = W.drop_in_field(n=64, r=12.0, seed=3)
    bad = W.drop_in_field(n=64, r=12.0, seed=3, R=8.0, S=2.0)
    eps_l = bad.params["eps_l"]
    bad.params.update(sigma_l=3.0 * eps_l, sigma_v=3.0 * eps_l / 8.0)
    big = W.drop_in_field(n=128, r=24.0, seed=5)
    wls = [good, bad, big]
    print("\n[case] solo retirement: 64^2 good, 64^2 conductive (lagged), 128^2 round path", flush=True)
    sim = lbm.Simulation([w.params for w in wls], [w.phi0 for w in wls], [w.q0 for w in wls],
                         launch=dict(BASE, solo_max_nodes=64 * 64))
    assert sim.step(80) == lbm.W_DIVERGED
    assert sim.stats(1)["status"] == lbm.E_DIVERGED
    for i in (0, 2):
        assert sim.stats(i)["status"] == lbm.OK and sim.stats(i)["steps"] == 80
    assert sim.step(5) == lbm.W_DIVERGED
    for i in (0, 2):
        w = wls[i]
        one = lbm.Simulation(w.params, w.phi0, w.q0, launch=BASE)
        one.step(85)
        a, b = sim.fields(i), one.fields(0)
        for k in a:
            assert np.array_equal(a[k], b[k]), (i, k)
        assert np.array_equal(sim.k_history(i), one.k_history(0)), i


def test_residual_stop_instances_stay_on_the_round_path():
    """Instances that stop on the Poisson residual are never solo (the
    residual pass belongs to the rounds): a batch mixing both stop tests gives
    the same results with and without a solo threshold that covers it."""
    from paper_2407_01654_amd import lbm
    a = W.drop_in_field(n=64, r=12.0, seed=3)
    b = W.drop_in_field(n=64, r=12.0, seed=4, pot_stop=W.STOP_RESIDUAL, pot_tol=2e-3)
    print("\n[case] solo with a residual-stopped instance", flush=True)
    runs = []
    for launch in (BASE, dict(BASE, solo_max_nodes=1 << 20)):
        sim = lbm.Simulation([a.params, b.params], [a.phi0, b.phi0], [a.q0, b.q0], launch=launch)
        sim.step(30)
        runs.append(snapshot(sim, 2))
    assert_same(runs[0], runs[1], "residual")


def test_solo_timing_counts_only_the_rounds():
    """Event timing of the round kernels with solo instances beside them: the
    passes counted are the round path's only (one main pass and the replayed
    inner iterations per step of the one instance there)."""
    from paper_2407_01654_amd import lbm
    small = W.drop_in_field(n=64, r=12.0, seed=3)
    big = W.drop_in_field(n=128, r=24.0, seed=5)
    params = [dict(w.params, presolve_iters=3) for w in (small, big)]
    sim = lbm.Simulation(params, [small.phi0, big.phi0], [small.q0, big.q0],
                         launch=dict(BASE, solo_max_nodes=64 * 64))
    sim.set_replay(0, np.full(20, 4, dtype=np.int32))
    sim.set_replay(1, np.full(20, 2, dtype=np.int32))
    sim.timing(True)
    sim.step(10)
    t = sim.timing(False)
    print("\n[case] solo timing", t, flush=True)
    assert t["main_passes"] == 10 and t["inner_iterations"] == 20
    assert t["round_launches"] == 30
    assert all(sim.stats(i)["steps"] == 10 for i in range(2))
    assert list(sim.k_history(0)[1:11]) == [4] * 10


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_staggered_start_keeps_results_bitwise(prec):
    """A staggered start (half of the round path's instances sit out the
    first round of each call) only moves their passes to other rounds: six
    free-running drops through the start-up transient, in calls of 1, 6 and
    33 steps, alone and together with solo instances, match the plain rounds
    bit for bit."""
    from paper_2407_01654_amd import lbm
    batch = W.batch_sweep(n_inst=6, seed=4, steps=40, sides=(64, 96, 192))
    print(f"\n[case] stagger {prec}, sides {[w.params['nx'] for w in batch]}", flush=True)
    runs = {}
    for tag, launch in (("rounds", BASE), ("stagger", dict(BASE, stagger=1)),
                        ("stagger_solo", dict(BASE, stagger=1, solo_max_nodes=64 * 64)),
                        ("stagger_host", dict(BASE, stagger=1, device_loop=0))):
        sim = lbm.Simulation([w.params for w in batch], [w.phi0 for w in batch], [w.q0 for w in batch],
                             prec=prec, launch=launch)
        for n in (1, 6, 33):
            sim.step(n)
        runs[tag] = snapshot(sim, len(batch))
        assert sim.get_launch()["stagger"] == (0 if tag == "rounds" else 1)
    for tag in ("stagger", "stagger_solo", "stagger_host"):
        assert_same(runs["rounds"], runs[tag], tag)


def test_staggered_start_timing_counts():
    """With a staggered start and every inner loop replayed at one iteration,
    a call of n steps over two instances takes 2 n + 1 rounds: the staggered
    one's idle round counts neither a main pass nor an inner iteration."""
    from paper_2407_01654_amd import lbm
    a = W.drop_in_field(n=64, r=12.0, seed=3)
    b = W.drop_in_field(n=64, r=12.0, seed=4)
    params = [dict(w.params, presolve_iters=3) for w in (a, b)]
    sim = lbm.Simulation(params, [a.phi0, b.phi0], [a.q0, b.q0], launch=dict(BASE, stagger=1))
    for i in range(2):
        sim.set_replay(i, np.full(20, 1, dtype=np.int32))
    sim.timing(True)
    sim.step(8)
    t = sim.timing(False)
    print("\n[case] stagger timing", t, flush=True)
    assert t["main_passes"] == 16 and t["inner_iterations"] == 16
    assert t["round_launches"] == 17
    assert all(sim.stats(i)["steps"] == 8 for i in range(2))


def test_solo_floor_stops_match_the_rounds_bitwise():
    """The FP16S rounding-floor stop inside the solo kernel: drop 502 of the
    sweep (64 x 64, the slowest inner loops, whose FP16S loops end at the
    rounding floor from a few hundred steps on) run solo and on the rounds
    for 600 steps, bit for bit, floor stops included."""
    from paper_2407_01654_amd import lbm
    w = W.batch_sweep(n_inst=512, seed=4)[502]
    print("\n[case] drop 502 fp16s solo vs rounds, 600 steps", flush=True)
    runs = []
    for launch in (BASE, dict(BASE, solo_max_nodes=64 * 64)):
        sim = lbm.Simulation(w.params, w.phi0, w.q0, prec="fp16s", launch=launch)
        for _ in range(3):
            sim.step(200)
        runs.append(snapshot(sim, 1))
        print(f"  floor stops {runs[-1][0][2]['floor_stops']}, sum K {int(runs[-1][0][1][1:].sum())}", flush=True)
    assert runs[0][0][2]["floor_stops"] > 0
    assert_same(runs[0], runs[1], "floor")
