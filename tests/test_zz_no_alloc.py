"""lbm_ehd_fields_noalloc, the entry point for callers that cannot allocate,
against lbm_ehd_fields through the C ABI: the same kernels stage the order
parameter in the library's fixed device array instead of the workspace, so the
selected fields must agree bit for bit.  Two calls in a row, the second on a
smaller instance (the array keeps the first call's values beyond it), and a
mask without the order parameter; instances above the array's capacity are
rejected before any launch."""
import numpy as np
import pytest

from paper_2407_01654_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "ux", "uy", "p", "psi", "rho_e")


def _noalloc(sim, inst, mask):
    import torch
    from paper_2407_01654_amd import lbm
    p = sim.params[inst]
    n_sel = bin(mask).count("1")
    out = torch.full((n_sel, p["ny"], p["nx"]), float("nan"), dtype=torch.float32, device=sim.device)
    assert sim.fields_noalloc(inst, mask, out) == lbm.OK
    torch.cuda.synchronize()
    names = [f for k, f in enumerate(FIELDS) if mask & (1 << k)]
    host = out.cpu().numpy()
    return {k: host[i] for i, k in enumerate(names)}


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_noalloc_fields_match_fields_on_two_calls(prec):
    from paper_2407_01654_amd import lbm
    big = W.drop_in_field(n=136, r=20.0, seed=3)
    small = W.sessile_drop(nx=72, ny=40, r=12.0)
    print(f"\n[case] fields_noalloc {prec}: 136x136 then 72x40", flush=True)
    sim = lbm.Simulation([big.params, small.params], [big.phi0, small.phi0], [big.q0, small.q0], prec=prec,
                         launch=dict(block_x=64, band_y=16))
    sim.step(7)
    for inst, mask in ((0, 63), (1, 63), (1, 16 | 32 | 2), (0, 8)):
        ref = sim.fields(inst, mask=mask, on_device=True)
        got = _noalloc(sim, inst, mask)
        assert set(got) == set(ref)
        for k in got:
            r = ref[k].cpu().numpy()
            assert np.isfinite(r).all(), (inst, k)
            assert np.array_equal(got[k], r), (inst, mask, k)


def test_noalloc_fields_reject_instances_above_capacity():
    from paper_2407_01654_amd import lbm
    import torch
    wl = W.planar_layers(nx=2048, ny=4097, steps=0, presolve_iters=1)
    assert wl.params["nx"] * wl.params["ny"] > lbm.NOALLOC_MAX_NODES
    print("\n[case] fields_noalloc capacity 2048x4097", flush=True)
    sim = lbm.Simulation(wl.params, wl.phi0, wl.q0, prec="fp16s")
    out = torch.empty(1, dtype=torch.float32, device=sim.device)
    assert sim.fields_noalloc(0, 1, out) == lbm.E_INVAL
    assert sim.fields_noalloc(0, 64, out) == lbm.E_INVAL
    assert sim.fields_noalloc(1, 1, out) == lbm.E_INVAL
    # the handle is unaffected
    assert sim.sync() == lbm.OK
