"""ctypes binding of the FP64 oracle library (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_ehd_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_ehd_oracle.so")

FIELDS = ("phi", "ux", "uy", "p", "psi", "rho_e")


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, IEEE FP64, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-std=gnu11", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-Wno-unused-parameter",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
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


_lib = None
_variants = {}
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _configure(lib):
    lib.ora_create.restype = C.c_void_p
    lib.ora_create.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.POINTER(C.c_int)]
    lib.ora_destroy.argtypes = [C.c_void_p]
    lib.ora_step.argtypes = [C.c_void_p, C.c_int]
    lib.ora_step.restype = C.c_int
    lib.ora_fields.argtypes = [C.c_void_p, _dp]
    lib.ora_set_replay.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
    lib.ora_k_history.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
    lib.ora_k_history.restype = C.c_int
    lib.ora_r_history.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
    lib.ora_r_history.restype = C.c_int
    lib.ora_r_prev_history.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
    lib.ora_r_prev_history.restype = C.c_int
    lib.ora_set_threads.argtypes = [C.c_int]
    lib.ora_set_threads.restype = None
    lib.ora_max_threads.restype = C.c_int
    lib.ora_steps_done.argtypes = [C.c_void_p]
    lib.ora_steps_done.restype = C.c_int64
    lib.ora_get.argtypes = [C.c_void_p, C.c_int, _dp]
    lib.ora_get.restype = C.c_int
    lib.ora_stencil.argtypes = [C.c_void_p, _dp, C.c_int, _dp, _dp, _dp]
    for name in ("ora_geq",):
        getattr(lib, name).argtypes = [C.c_double, C.c_double, _dp]
    lib.ora_heq.argtypes = [C.c_double, _dp]
    lib.ora_leq.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
    lib.ora_feq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
    lib.ora_rbar.argtypes = [C.c_double] * 6 + [_dp]
    lib.ora_source_g.argtypes = [C.c_double, _dp]
    lib.ora_lattice.argtypes = [C.c_void_p, C.c_void_p, _dp]
    lib.ora_residual.argtypes = [C.c_void_p]
    lib.ora_residual.restype = C.c_double
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _configure(C.CDLL(_LIB))
    return _lib


def build_variant(source: str, out_path: str):
    """Compiles oracle source text (a copy of lbm_ehd_oracle.c with one planted
    change, for the tests that show a pin catches a mistake) into out_path and
    returns it loaded.  The oracle itself is never modified."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(source)
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-std=gnu11", "-fPIC", "-shared", "-w",
                           "-I", _HERE, "-o", out_path, src, "-lm"])
    lib = _configure(C.CDLL(out_path))
    _variants[out_path] = lib
    return lib


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _as_c(a, shape):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if arr.shape != shape:
        raise ValueError(f"expected shape {shape}, got {arr.shape}")
    return arr, arr.ctypes.data_as(C.c_void_p)


class Oracle:
    """One FP64 simulation; `params` uses the keys of workloads.PARAM_KEYS."""

    def __init__(self, params: dict, phi0, q0, ux0=None, uy0=None, lib=None):
        lib = _load() if lib is None else lib
        self._lib = lib
        p = _Params(**{k: params[k] for k, _ in _Params._fields_})
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        shape = (self.ny, self.nx)
        keep = [_as_c(a, shape) for a in (phi0, q0, ux0, uy0)]
        st = C.c_int(0)
        h = lib.ora_create(C.byref(p), *(k[1] for k in keep), C.byref(st))
        if not h:
            raise ValueError(f"oracle rejected parameters (status {st.value})")
        self._h = h
        self.init_status = st.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ora_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, n: int) -> int:
        return self._lib.ora_step(self._h, int(n))

    def fields(self) -> dict:
        out = np.empty((6, self.ny, self.nx), dtype=np.float64)
        self._lib.ora_fields(self._h, out)
        return {k: out[i] for i, k in enumerate(FIELDS)}

    def set_replay(self, iters):
        arr = np.ascontiguousarray(iters, dtype=np.int32)
        self._lib.ora_set_replay(self._h, arr.ctypes.data_as(C.c_void_p), int(arr.size))
        self._replay_keep = arr

    def k_history(self) -> np.ndarray:
        n = self._lib.ora_k_history(self._h, None, 0)
        out = np.empty(n, dtype=np.int32)
        self._lib.ora_k_history(self._h, out.ctypes.data_as(C.c_void_p), n)
        return out

    def r_history(self) -> np.ndarray:
        n = self._lib.ora_r_history(self._h, None, 0)
        out = np.empty(n, dtype=np.float64)
        self._lib.ora_r_history(self._h, out.ctypes.data_as(C.c_void_p), n)
        return out

    def r_prev_history(self) -> np.ndarray:
        n = self._lib.ora_r_prev_history(self._h, None, 0)
        out = np.empty(n, dtype=np.float64)
        self._lib.ora_r_prev_history(self._h, out.ctypes.data_as(C.c_void_p), n)
        return out

    @property
    def steps_done(self) -> int:
        return int(self._lib.ora_steps_done(self._h))

    _GET = {"g": (0, 9), "l": (1, 9), "f": (2, 9), "h": (3, 9), "Gamma_prev": (10, 1),
            "R_prev": (11, 1), "Fx_prev": (12, 1), "Fy_prev": (13, 1), "Jx_prev": (14, 1),
            "Jy_prev": (15, 1), "psi": (16, 1)}

    def get(self, name: str) -> np.ndarray:
        which, k = self._GET[name]
        out = np.empty(k * self.nx * self.ny, dtype=np.float64)
        self._lib.ora_get(self._h, which, out)
        return out.reshape((k, self.ny, self.nx) if k > 1 else (self.ny, self.nx))

    def residual(self) -> float:
        """Relative residual of the Poisson equation for the current potential."""
        return float(self._lib.ora_residual(self._h))

    def stencil(self, field, kind: int):
        f = np.ascontiguousarray(field, dtype=np.float64)
        gx, gy, lap = (np.empty_like(f) for _ in range(3))
        self._lib.ora_stencil(self._h, f, int(kind), gx, gy, lap)
        return gx, gy, lap


def set_threads(n: int) -> None:
    """Threads of the oracle's per-node loops (its results do not depend on it)."""
    _load().ora_set_threads(int(n))


def max_threads() -> int:
    return int(_load().ora_max_threads())


def _nine(fn, *args):
    out = np.empty(9, dtype=np.float64)
    getattr(_load(), fn)(*[float(a) for a in args], out)
    return out


def lattice():
    cx = np.empty(9, dtype=np.int32)
    cy = np.empty(9, dtype=np.int32)
    w = np.empty(9, dtype=np.float64)
    _load().ora_lattice(cx.ctypes.data_as(C.c_void_p), cy.ctypes.data_as(C.c_void_p), w)
    return cx, cy, w


def geq(phi, mu_c):
    return _nine("ora_geq", phi, mu_c)


def heq(psi):
    return _nine("ora_heq", psi)


def leq(q, ux, uy):
    return _nine("ora_leq", q, ux, uy)


def feq(p, rho, ux, uy):
    return _nine("ora_feq", p, rho, ux, uy)


def rbar(ux, uy, grx, gry, Fx, Fy):
    return _nine("ora_rbar", ux, uy, grx, gry, Fx, Fy)


def source_g(Gamma):
    return _nine("ora_source_g", Gamma)
