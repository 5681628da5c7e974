"""C-ABI checks that need no device: the built library loads, exports every
entry point the header declares, agrees with the binding on struct layouts,
and its host-side parameter validation and workspace planning behave."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2407_01654_amd import lbm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_ehd.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build_hip()
    return lbm.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(lbm_ehd_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lbm.FUNCTIONS)


def test_struct_layouts_match_binding(lib):
    out = (C.c_size_t * 5)()
    ver = lib.lbm_ehd_abi_sizes(out, 4)
    assert ver == 10
    assert out[0] == C.sizeof(lbm.Params)
    assert out[1] == C.sizeof(lbm.Stats)
    assert out[2] == C.sizeof(lbm.Launch)
    assert out[3] == C.sizeof(lbm.Timing)
    assert lib.lbm_ehd_abi_sizes(out, 5) == lbm.E_INVAL


def test_strerror_covers_codes(lib):
    for code in (0, 1, 2, -1, -2, -3, -4, -5):
        assert lib.lbm_ehd_strerror(code)
    assert b"unknown" in lib.lbm_ehd_strerror(-99)


def test_workspace_planning(lib):
    small = W.planar_layers().params
    big = W.drop_in_field(n=512).params
    b_small = lbm.workspace_bytes([small])
    b_big = lbm.workspace_bytes([big])
    assert 0 < b_small < b_big
    # two pools (FP32 fields, FP32 populations), each one block of 64 plane
    # segments of 64 slots per row and 64-column strip (512 columns -> 8
    # strips), plus 6 compact scratch planes and bookkeeping of a few percent
    pool = -(-512 // 64) * 64 * 64 * 512
    planes = 2 * 4 * pool + 6 * 512 * 512 * 4
    assert planes <= b_big < 1.05 * planes
    b16 = lbm.workspace_bytes([big], "fp16s")
    assert b16 < 0.8 * b_big
    assert b_big < lbm.workspace_bytes([small, big]) <= b_small + b_big
    sess = W.sessile_drop().params
    assert lbm.workspace_bytes([sess]) < 4.8e9


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=2), dict(mu_l=0.0), dict(eps_v=-1.0), dict(gamma=0.0),
    dict(alpha_q=0.0), dict(pot_max_iter=0), dict(enable=16), dict(sigma_v=-1e-3),
    dict(pot_scheme=2), dict(pot_scheme=-1), dict(pot_scheme=W.POT_CONVENTIONAL, pot_chi=0.0),
    dict(pot_scheme=W.POT_CONVENTIONAL, pot_chi=float("nan")),
    dict(charge_closure=2), dict(charge_closure=-1),
])
def test_invalid_parameters_rejected(lib, bad):
    p = W.planar_layers().params
    p.update(bad)
    arr = (lbm.Params * 1)(lbm.make_params(p))
    out = C.c_size_t(0)
    assert lib.lbm_ehd_workspace_bytes(arr, 1, 0, C.byref(out)) == lbm.E_INVAL


def test_one_potential_scheme_per_handle(lib):
    """A handle runs one potential scheme: a set that mixes them is invalid,
    a uniform conventional set is planned like the improved one."""
    p = W.planar_layers().params
    q = dict(p, pot_scheme=W.POT_CONVENTIONAL, pot_chi=2.0)
    out = C.c_size_t(0)
    mixed = (lbm.Params * 2)(lbm.make_params(p), lbm.make_params(q))
    assert lib.lbm_ehd_workspace_bytes(mixed, 2, 0, C.byref(out)) == lbm.E_INVAL
    assert lbm.workspace_bytes([q, q]) == lbm.workspace_bytes([p, p])


def test_init_rejects_bad_workspace_without_touching_device(lib):
    p = W.planar_layers().params
    arr = (lbm.Params * 1)(lbm.make_params(p))
    phi = np.zeros(p["nx"] * p["ny"])
    h = C.c_void_p()
    rc = lib.lbm_ehd_init(arr, 1, 0, phi.ctypes.data_as(C.c_void_p), phi.ctypes.data_as(C.c_void_p),
                          None, None, None, 0, None, C.byref(h))
    assert rc == lbm.E_WORKSPACE and not h.value
    rc = lib.lbm_ehd_init(arr, 1, 7, phi.ctypes.data_as(C.c_void_p), phi.ctypes.data_as(C.c_void_p),
                          None, None, None, 0, None, C.byref(h))
    assert rc == lbm.E_INVAL


def test_product_path_fails_loudly_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("device present")
    wl = W.planar_layers()
    with pytest.raises(RuntimeError):
        lbm.Simulation(wl.params, wl.phi0, wl.q0)


def test_handle_calls_reject_a_null_handle_without_touching_device(lib):
    """Every entry point that takes a handle checks it before any HIP call."""
    b = C.c_int32(0)
    L = lbm.Launch()
    T = lbm.Timing()
    st = lbm.Stats()
    assert lib.lbm_ehd_set_instance_band(None, 0, 8) == lbm.E_INVAL
    assert lib.lbm_ehd_get_instance_band(None, 0, C.byref(b)) == lbm.E_INVAL
    assert lib.lbm_ehd_set_launch(None, C.byref(L)) == lbm.E_INVAL
    assert lib.lbm_ehd_get_launch(None, C.byref(L)) == lbm.E_INVAL
    assert lib.lbm_ehd_autotune(None, 10, C.byref(L)) == lbm.E_INVAL
    assert lib.lbm_ehd_timing(None, 1, C.byref(T)) == lbm.E_INVAL
    assert lib.lbm_ehd_stats(None, 0, C.byref(st)) == lbm.E_INVAL
    assert lib.lbm_ehd_step(None, 1) == lbm.E_INVAL
