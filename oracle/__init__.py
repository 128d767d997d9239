"""Plain FP64 CPU oracle of the semi-conservative RSST step (arXiv:1812.04135).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU leg of the
benchmark may use this package; the GPU library never does.  It shares no
code with ``paper_1812_04135_amd``.

The numerics live in ``rsst_oracle.cpp`` (plain loops, explicit ghost
mapping, no fusion); this module only marshals numpy arrays through ctypes.
Which passage of the paper each step follows is stated in that file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsst_oracle.cpp")
_LIB = os.path.join(_HERE, "librsst_oracle.so")

FORMS = {"euler": 0, "pvs": 1, "pms": 2, "dvs": 3, "dms": 4, "pd": 5}
BCS = {"periodic": 0, "reflect": 1, "hydro": 2}
EOS = {"ideal": 0, "vdw": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (strict IEEE: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Config(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("dx", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("dt_rule", ctypes.c_int),
        ("g", ctypes.c_double * 3),
        ("bc_lo", ctypes.c_int * 3),
        ("bc_hi", ctypes.c_int * 3),
        ("form", ctypes.c_int),
        ("cmax", ctypes.c_double),
        ("eos", ctypes.c_int),
        ("eos_a", ctypes.c_double),
        ("eos_b", ctypes.c_double),
        ("p_probe", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(_Config)
        lib.ora_prim.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.ora_flux.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, dp]
        lib.ora_flux_jacobian.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, dp]
        lib.ora_mc.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.ora_mc.restype = ctypes.c_double
        lib.ora_llf.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp,
                                ctypes.c_int, dp]
        lib.ora_llf.restype = ctypes.c_int
        lib.ora_correct.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, dp, dp, dp, dp]
        lib.ora_cfl_dt.argtypes = [cp, dp]
        lib.ora_cfl_dt.restype = ctypes.c_double
        lib.ora_rate.argtypes = [cp, dp, dp]
        lib.ora_rate.restype = ctypes.c_int64
        lib.ora_run.argtypes = [cp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.ora_run.restype = ctypes.c_int64
        lib.ora_run_tangent.argtypes = [cp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double]
        lib.ora_run_tangent.restype = ctypes.c_int64
        lib.ora_diag.argtypes = [cp, dp, dp]
        lib.ora_threads.restype = ctypes.c_int
        lib.ora_set_threads.argtypes = [ctypes.c_int]
        lib.ora_eos.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, dp]
        lib.ora_prim_eos.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, dp, dp]
        lib.ora_correct_eos.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size >= n
    return a


def make_config(cfg: dict) -> _Config:
    """Build the oracle's config from a plain parameter dict.

    Keys: ndim, n (list), dx (list), gamma, xi, cfl, dt_rule, g (list),
    bc_lo/bc_hi (lists of 'periodic'|'reflect' or ints), form (name or int).
    """
    c = _Config()
    c.ndim = int(cfg["ndim"])
    n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
    dx = list(cfg["dx"]) + [1.0] * (3 - len(cfg["dx"]))
    g = list(cfg.get("g", [0.0] * 3)) + [0.0] * 3
    for d in range(3):
        c.n[d] = int(n[d])
        c.dx[d] = float(dx[d])
        c.g[d] = float(g[d])
        lo = cfg.get("bc_lo", ["periodic"] * 3)
        hi = cfg.get("bc_hi", ["periodic"] * 3)
        lo = list(lo) + ["periodic"] * 3
        hi = list(hi) + ["periodic"] * 3
        c.bc_lo[d] = BCS[lo[d]] if isinstance(lo[d], str) else int(lo[d])
        c.bc_hi[d] = BCS[hi[d]] if isinstance(hi[d], str) else int(hi[d])
    c.gamma = float(cfg["gamma"])
    c.xi = float(cfg["xi"])
    c.cfl = float(cfg.get("cfl", 0.4))
    c.dt_rule = int(cfg.get("dt_rule", 0))
    f = cfg.get("form", "pvs")
    c.form = FORMS[f] if isinstance(f, str) else int(f)
    c.cmax = float(cfg.get("cmax", 0.0))
    e = cfg.get("eos", "ideal")
    c.eos = EOS[e] if isinstance(e, str) else int(e)
    c.eos_a = float(cfg.get("eos_a", 0.0))
    c.eos_b = float(cfg.get("eos_b", 0.0))
    c.p_probe = float(cfg.get("p_probe", 0.0))
    return c


def _field(U: np.ndarray, cfg: dict) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    nv = int(cfg["ndim"]) + 2
    ncell = int(np.prod(cfg["n"]))
    assert U.size == nv * ncell, (U.shape, nv, ncell)
    return U


def threads() -> int:
    """OpenMP threads used by the oracle's loops."""
    return int(_load().ora_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's loops for the following calls."""
    _load().ora_set_threads(int(n))


# ----------------------------------------------------------------- per cell

def _gas(gas):
    """(kind, a, b) of an equation-of-state dict {eos, eos_a, eos_b}; None: ideal."""
    if gas is None:
        return 0, 0.0, 0.0
    e = gas.get("eos", "ideal")
    return (EOS[e] if isinstance(e, str) else int(e)), float(gas.get("eos_a", 0.0)), float(gas.get("eos_b", 0.0))


def eos(gamma: float, rho: float, P: float, gas=None) -> dict:
    """The equation of state at (rho, P): e(rho, P), P(rho, e) of that e,
    (de/dP)_rho, (de/drho)_P and a^2."""
    k, a, b = _gas(gas)
    out = np.zeros(5)
    _load().ora_eos(float(gamma), k, a, b, float(rho), float(P), _ptr(out))
    return {"e": out[0], "P_of_e": out[1], "dedP": out[2], "dedrho": out[3], "a2": out[4]}


def prim(u, ndim: int, gamma: float, xi: float = 1.0, cmax: float = 0.0, gas=None) -> dict:
    lib = _load()
    u = _vec(u, ndim + 2)
    out = np.zeros(9)
    if gas is not None:
        assert cmax == 0.0
        lib.ora_prim_eos(ndim, gamma, *_gas(gas), xi, _ptr(u), _ptr(out))
    else:
        lib.ora_prim(ndim, gamma, xi, cmax, _ptr(u), _ptr(out))
    return {"rho": out[0], "v": out[1:1 + ndim].copy(), "P": out[4], "a2": out[5],
            "a": out[6], "vabs": out[7], "ctot": out[8]}


def flux(u, ndim: int, gamma: float, d: int) -> np.ndarray:
    lib = _load()
    u = _vec(u, ndim + 2)
    F = np.zeros(ndim + 2)
    lib.ora_flux(ndim, gamma, _ptr(u), d, _ptr(F))
    return F


def flux_jacobian(u, ndim: int, gamma: float, d: int) -> np.ndarray:
    lib = _load()
    u = _vec(u, ndim + 2)
    nv = ndim + 2
    J = np.zeros(nv * nv)
    lib.ora_flux_jacobian(ndim, gamma, _ptr(u), d, _ptr(J))
    return J.reshape(nv, nv)


def mc(l: float, r: float) -> float:
    return _load().ora_mc(float(l), float(r))


def llf(UL, UR, ndim: int, gamma: float, xi: float, d: int) -> np.ndarray:
    lib = _load()
    UL, UR = _vec(UL, ndim + 2), _vec(UR, ndim + 2)
    F = np.zeros(ndim + 2)
    lib.ora_llf(ndim, gamma, xi, _ptr(UL), _ptr(UR), d, _ptr(F))
    return F


def correct(u, D, ndim: int, gamma: float, xi: float, form, g=(0.0, 0.0, 0.0), cmax: float = 0.0,
            gas=None) -> np.ndarray:
    lib = _load()
    u, D = _vec(u, ndim + 2), _vec(D, ndim + 2)
    gg = _vec(list(g) + [0.0] * 3)
    R = np.zeros(ndim + 2)
    fi = FORMS[form] if isinstance(form, str) else int(form)
    if gas is not None:
        assert cmax == 0.0
        lib.ora_correct_eos(ndim, gamma, *_gas(gas), xi, fi, _ptr(u), _ptr(D), _ptr(gg), _ptr(R))
    else:
        lib.ora_correct(ndim, gamma, xi, cmax, fi, _ptr(u), _ptr(D), _ptr(gg), _ptr(R))
    return R


# ----------------------------------------------------------------- grid

def cfl_dt(cfg: dict, U: np.ndarray) -> float:
    c = make_config(cfg)
    U = _field(U, cfg)
    return _load().ora_cfl_dt(ctypes.byref(c), _ptr(U))


def rate(cfg: dict, U: np.ndarray) -> np.ndarray:
    c = make_config(cfg)
    U = _field(U, cfg)
    R = np.zeros_like(U)
    bad = _load().ora_rate(ctypes.byref(c), _ptr(U), _ptr(R))
    if bad:
        raise FloatingPointError(f"oracle: {bad} non-physical states")
    return R


def run(cfg: dict, U: np.ndarray, nsteps: int, dt_fixed: float = 0.0, t_end: float = 0.0,
        t0: float = 0.0):
    """Advance a copy of U; returns (U_new, t, dt_last)."""
    c = make_config(cfg)
    W = _field(U, cfg).copy()
    t = np.array([t0], dtype=np.float64)
    dtl = np.zeros(1)
    bad = _load().ora_run(ctypes.byref(c), _ptr(W), int(nsteps), float(dt_fixed),
                          float(t_end), _ptr(t), _ptr(dtl))
    if bad:
        raise FloatingPointError(f"oracle: {bad} non-physical states")
    return W, float(t[0]), float(dtl[0])


def run_tangent(cfg: dict, U: np.ndarray, dU: np.ndarray, dxi, nsteps: int, dt: float):
    """Forward-mode tangents of nsteps fixed-dt steps.

    dU has shape [K, nv*ncell] (K <= 8), dxi shape [K].  Returns (U_new, dU_new).
    """
    c = make_config(cfg)
    W = _field(U, cfg).copy()
    T = np.ascontiguousarray(dU, dtype=np.float64).copy()
    K = T.shape[0]
    dx = _vec(dxi)
    assert dx.size == K and T.shape[1] == W.size
    bad = _load().ora_run_tangent(ctypes.byref(c), _ptr(W), _ptr(T), _ptr(dx), K,
                                  int(nsteps), float(dt))
    if bad:
        raise FloatingPointError(f"oracle: {bad} non-physical states")
    return W, T


def diag(cfg: dict, U: np.ndarray) -> np.ndarray:
    c = make_config(cfg)
    U = _field(U, cfg)
    out = np.zeros(8)
    _load().ora_diag(ctypes.byref(c), _ptr(U), _ptr(out))
    return out
