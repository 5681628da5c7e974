"""Thin Python binding of the lbm_ehd C ABI (argument marshalling only).

Every step of the method runs in the HIP kernels of liblbm_ehd.so; PyTorch
provides the device workspace and the stream.  If the library is not built or
no HIP device is present, the calls raise: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_ehd.so")

OK, W_NOT_CONVERGED, W_DIVERGED, E_INVAL, E_WORKSPACE, E_HIP, E_DIVERGED, E_STATE = 0, 1, 2, -1, -2, -3, -4, -5
EN_CH, EN_POT, EN_NP, EN_HYDRO = 1, 2, 4, 8
POT_IMPROVED, POT_CONVENTIONAL = 0, 1
STOP_CHANGE, STOP_RESIDUAL = 0, 1
PREC = {"fp32": 0, "fp16s": 1}
FIELDS = ("phi", "ux", "uy", "p", "psi", "rho_e")
F_ALL = 63

FUNCTIONS = (
    "lbm_ehd_workspace_bytes", "lbm_ehd_init", "lbm_ehd_step", "lbm_ehd_fields",
    "lbm_ehd_stats", "lbm_ehd_k_history", "lbm_ehd_set_replay", "lbm_ehd_set_launch",
    "lbm_ehd_get_launch", "lbm_ehd_sync", "lbm_ehd_destroy", "lbm_ehd_strerror",
    "lbm_ehd_abi_sizes", "lbm_ehd_timing", "lbm_ehd_autotune", "lbm_ehd_set_instance_band",
    "lbm_ehd_get_instance_band", "lbm_ehd_fields_noalloc", "lbm_ehd_residual",
)
NOALLOC_MAX_NODES = 1 << 23


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("walls_y", C.c_int32),
        ("rho_l", C.c_double), ("rho_v", C.c_double), ("mu_l", C.c_double), ("mu_v", C.c_double),
        ("sigma_l", C.c_double), ("sigma_v", C.c_double), ("eps_l", C.c_double), ("eps_v", C.c_double),
        ("mobility", C.c_double), ("width", C.c_double), ("gamma", C.c_double), ("alpha_q", C.c_double),
        ("psi_bottom", C.c_double), ("psi_top", C.c_double),
        ("theta_bottom_deg", C.c_double), ("theta_top_deg", C.c_double),
        ("cos_shift_bottom", C.c_double), ("cos_shift_top", C.c_double),
        ("enable", C.c_int32), ("pot_tol", C.c_double), ("pot_max_iter", C.c_int32),
        ("presolve_iters", C.c_int32), ("pot_scheme", C.c_int32), ("pot_chi", C.c_double),
        ("charge_closure", C.c_int32), ("pot_stop", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("total_iters", C.c_int64), ("presolve_iters", C.c_int32),
        ("last_iters", C.c_int32), ("last_rel_change", C.c_double), ("sum_phi", C.c_double),
        ("sum_q", C.c_double), ("status", C.c_int32), ("floor_stops", C.c_int32),
        ("residual", C.c_double),
    ]


class Timing(C.Structure):
    _fields_ = [("round_ms", C.c_double), ("finalize_ms", C.c_double),
                ("round_launches", C.c_int64), ("finalize_launches", C.c_int64),
                ("main_round_ms", C.c_double), ("main_rounds", C.c_int64),
                ("pot_round_ms", C.c_double), ("pot_rounds", C.c_int64),
                ("main_passes", C.c_int64), ("inner_iterations", C.c_int64)]


class Launch(C.Structure):
    _fields_ = [("block_x", C.c_int32), ("band_y", C.c_int32), ("device_loop", C.c_int32),
                ("rounds_per_graph", C.c_int32), ("band_y_small", C.c_int32), ("small_ny", C.c_int32),
                ("solo_max_nodes", C.c_int32), ("stagger", C.c_int32)]


_lib = None


def load():
    """Loads liblbm_ehd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    lib.lbm_ehd_workspace_bytes.argtypes = [C.POINTER(Params), i32, i32, C.POINTER(sz)]
    lib.lbm_ehd_init.argtypes = [C.POINTER(Params), i32, i32, vp, vp, vp, vp, vp, sz, vp, C.POINTER(vp)]
    lib.lbm_ehd_step.argtypes = [vp, i32]
    lib.lbm_ehd_fields.argtypes = [vp, i32, C.c_uint32, vp, i32]
    lib.lbm_ehd_fields_noalloc.argtypes = [vp, i32, C.c_uint32, vp]
    lib.lbm_ehd_stats.argtypes = [vp, i32, C.POINTER(Stats)]
    lib.lbm_ehd_residual.argtypes = [vp, i32, C.POINTER(C.c_double)]
    lib.lbm_ehd_k_history.argtypes = [vp, i32, vp, i32]
    lib.lbm_ehd_set_replay.argtypes = [vp, i32, vp, i32]
    lib.lbm_ehd_set_launch.argtypes = [vp, C.POINTER(Launch)]
    lib.lbm_ehd_get_launch.argtypes = [vp, C.POINTER(Launch)]
    lib.lbm_ehd_sync.argtypes = [vp]
    lib.lbm_ehd_destroy.argtypes = [vp]
    lib.lbm_ehd_destroy.restype = None
    lib.lbm_ehd_strerror.argtypes = [i32]
    lib.lbm_ehd_strerror.restype = C.c_char_p
    lib.lbm_ehd_abi_sizes.argtypes = [C.POINTER(sz), i32]
    lib.lbm_ehd_timing.argtypes = [vp, i32, C.POINTER(Timing)]
    lib.lbm_ehd_autotune.argtypes = [vp, i32, C.POINTER(Launch)]
    lib.lbm_ehd_set_instance_band.argtypes = [vp, i32, i32]
    lib.lbm_ehd_get_instance_band.argtypes = [vp, i32, C.POINTER(i32)]
    _lib = lib
    return lib


class LbmError(RuntimeError):
    def __init__(self, code, what):
        msg = load().lbm_ehd_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


def _check(code, what):
    if code < 0:
        raise LbmError(code, what)
    return code


def make_params(p: dict) -> Params:
    return Params(**{k: p[k] for k, _ in Params._fields_})


def workspace_bytes(params: list, prec: str = "fp32") -> int:
    arr = (Params * len(params))(*[make_params(p) for p in params])
    out = C.c_size_t(0)
    _check(load().lbm_ehd_workspace_bytes(arr, len(params), PREC[prec], C.byref(out)), "workspace_bytes")
    return out.value


def _concat(arrs, params):
    if arrs is None:
        return None
    out = []
    for a, p in zip(arrs, params):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != (p["ny"], p["nx"]):
            raise ValueError(f"field shape {a.shape} != {(p['ny'], p['nx'])}")
        out.append(a.ravel())
    return np.ascontiguousarray(np.concatenate(out))


class Simulation:
    """n independent simulations advanced together on one HIP device."""

    def __init__(self, params, phi0, q0, ux0=None, uy0=None, prec="fp32", device="cuda:0",
                 launch: dict | None = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbm_ehd needs a HIP device")
        single = isinstance(params, dict)
        self.params = [params] if single else list(params)
        if single:
            phi0, q0 = [phi0], [q0]
            ux0 = None if ux0 is None else [ux0]
            uy0 = None if uy0 is None else [uy0]
        lib = load()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.n = len(self.params)
        self.prec = prec
        nbytes = workspace_bytes(self.params, prec)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        arr = (Params * self.n)(*[make_params(p) for p in self.params])
        host = [_concat(a, self.params) for a in (phi0, q0, ux0, uy0)]
        ptr = [None if h is None else h.ctypes.data_as(C.c_void_p) for h in host]
        handle = C.c_void_p()
        _check(lib.lbm_ehd_init(arr, self.n, PREC[prec], ptr[0], ptr[1], ptr[2], ptr[3],
                                C.c_void_p(self.workspace.data_ptr()), nbytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(handle)), "init")
        self._h = handle
        if launch:
            self.set_launch(**launch)

    # -- life cycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lbm_ehd_destroy(self._h)
        self._h = None

    __del__ = close

    # -- stepping ----------------------------------------------------------
    def step(self, n: int) -> int:
        return _check(load().lbm_ehd_step(self._h, int(n)), "step")

    def sync(self) -> int:
        return _check(load().lbm_ehd_sync(self._h), "sync")

    # -- results -----------------------------------------------------------
    def fields(self, inst: int = 0, mask: int = F_ALL, on_device: bool = False):
        p = self.params[inst]
        names = [f for k, f in enumerate(FIELDS) if mask & (1 << k)]
        shape = (len(names), p["ny"], p["nx"])
        if on_device:
            import torch
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
            _check(load().lbm_ehd_fields(self._h, inst, mask, C.c_void_p(out.data_ptr()), 1), "fields")
        else:
            out = np.empty(shape, dtype=np.float32)
            _check(load().lbm_ehd_fields(self._h, inst, mask, out.ctypes.data_as(C.c_void_p), 0), "fields")
        return {k: out[i] for i, k in enumerate(names)}

    def fields_noalloc(self, inst: int, mask: int, out) -> int:
        """lbm_ehd_fields_noalloc into the device tensor `out` (float32,
        contiguous, one [ny][nx] plane per selected field); enqueued on the
        stream, not synchronised.  Returns the status code (no exception), so
        that callers can test the error paths."""
        return load().lbm_ehd_fields_noalloc(self._h, int(inst), int(mask), C.c_void_p(out.data_ptr()))

    def residual(self, inst: int = 0) -> float:
        """Relative residual of the Poisson equation for the current potential."""
        out = C.c_double()
        _check(load().lbm_ehd_residual(self._h, int(inst), C.byref(out)), "residual")
        return out.value

    def stats(self, inst: int = 0) -> dict:
        st = Stats()
        _check(load().lbm_ehd_stats(self._h, inst, C.byref(st)), "stats")
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    def k_history(self, inst: int = 0, max_n: int = 8192) -> np.ndarray:
        out = np.empty(max_n, dtype=np.int32)
        n = _check(load().lbm_ehd_k_history(self._h, inst, out.ctypes.data_as(C.c_void_p), max_n), "k_history")
        return out[:n].copy()

    def set_replay(self, inst: int, iters) -> None:
        arr = np.ascontiguousarray(iters, dtype=np.int32)
        _check(load().lbm_ehd_set_replay(self._h, inst, arr.ctypes.data_as(C.c_void_p), int(arr.size)),
               "set_replay")

    def set_launch(self, block_x=64, band_y=64, device_loop=1, rounds_per_graph=0, band_y_small=0,
                   small_ny=0, solo_max_nodes=0, stagger=0) -> None:
        L = Launch(block_x, band_y, int(device_loop), int(rounds_per_graph), band_y_small, small_ny,
                   int(solo_max_nodes), int(stagger))
        _check(load().lbm_ehd_set_launch(self._h, C.byref(L)), "set_launch")

    def autotune(self, trial_steps: int = 10) -> dict:
        """Chooses band heights, the solo threshold and the rounds per
        captured chunk by timing real steps (2 * trial_steps per candidate);
        returns the launch shape kept."""
        L = Launch()
        _check(load().lbm_ehd_autotune(self._h, int(trial_steps), C.byref(L)), "autotune")
        return {k: getattr(L, k) for k, _ in Launch._fields_}

    def set_instance_band(self, inst: int, band_y: int) -> None:
        """Band height of one instance's tiles (0: the launch shape's)."""
        _check(load().lbm_ehd_set_instance_band(self._h, int(inst), int(band_y)), "set_instance_band")

    def instance_band(self, inst: int) -> int:
        b = C.c_int32()
        _check(load().lbm_ehd_get_instance_band(self._h, int(inst), C.byref(b)), "get_instance_band")
        return b.value

    def timing(self, enable: bool) -> dict:
        """Turns per-launch event timing of the round kernels on/off; returns
        the values accumulated so far."""
        T = Timing()
        _check(load().lbm_ehd_timing(self._h, int(enable), C.byref(T)), "timing")
        return {k: getattr(T, k) for k, _ in Timing._fields_}

    def get_launch(self) -> dict:
        L = Launch()
        _check(load().lbm_ehd_get_launch(self._h, C.byref(L)), "get_launch")
        return {k: getattr(L, k) for k, _ in Launch._fields_}
