"""MI355X (gfx950) explicit time step of the semi-conservative
reduced-speed-of-sound technique (RSST), arXiv:1812.04135.

Thin ctypes binding of the C ABI in include/rsst.h.  Every step of the path
runs in the HIP kernels of librsst.so; this module only marshals arguments.
PyTorch supplies device memory and the current stream.  If the library is
not built, importing works but every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsst.so")

RSST_OK = 0
RSST_E_DEVICE = -3
RSST_E_NONPHYSICAL = -5
RSST_E_SCRATCH = -6
FORMS = {"euler": 0, "pvs": 1, "pms": 2, "dvs": 3, "dms": 4, "pd": 5}
BCS = {"periodic": 0, "reflect": 1, "hydro": 2}
PRECS = {"fp64": 0, "fp32_pert": 1}
EOS = {"ideal": 0, "vdw": 1}
RSST_WITH_ADJOINT = 1


class rsst_config(ctypes.Structure):
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
        ("prec", ctypes.c_int),
        ("bg", ctypes.c_void_p),
        ("bg_axis", ctypes.c_int),
        ("t_end", ctypes.c_double),
        ("flags", ctypes.c_int),
        ("cmax", ctypes.c_double),
        ("eos", ctypes.c_int),
        ("eos_a", ctypes.c_double),
        ("eos_b", ctypes.c_double),
    ]


_lib = None


def lib():
    """The loaded librsst.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librsst.so not built ({LIB_PATH}); run python -m paper_1812_04135_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.rsst_init.argtypes = [ctypes.POINTER(rsst_config), vp, ctypes.POINTER(vp)]
        L.rsst_prime.argtypes = [vp, vp, ctypes.c_double, vp]
        L.rsst_step.argtypes = [vp, vp, ctypes.c_double, vp]
        L.rsst_step_noalloc.argtypes = [ctypes.POINTER(rsst_config), vp, ctypes.c_double, vp, vp]
        L.rsst_stage.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, vp]
        L.rsst_steps.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, vp]
        L.rsst_get_time.argtypes = [vp, dp, dp, vp]
        L.rsst_diag.argtypes = [vp, vp, dp, vp]
        L.rsst_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
        L.rsst_destroy.argtypes = [vp]
        L.rsst_strerror.argtypes = [ctypes.c_int]
        L.rsst_strerror.restype = ctypes.c_char_p
        L.rsst_version.restype = ctypes.c_char_p
        L.rsst_batch_init.argtypes = [ctypes.POINTER(rsst_config), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_int, vp,
                                      ctypes.POINTER(vp)]
        L.rsst_batch_set_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.rsst_batch_set_times.argtypes = [vp, dp, ctypes.c_uint32, vp]
        L.rsst_batch_set_wait_limit.argtypes = [vp, ctypes.c_double]
        L.rsst_batch_get_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.rsst_batch_run.argtypes = [vp, vp, ctypes.c_int, vp]
        L.rsst_batch_times.argtypes = [vp, dp, vp]
        L.rsst_batch_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
        L.rsst_batch_destroy.argtypes = [vp]
        L.rsst_adjoint_step.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp]
        L.rsst_adjoint_step_u1.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp]
        L.rsst_step_out.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp]
        L.rsst_steps_out.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, ctypes.c_double, vp]
        L.rsst_adjoint_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp,
                                       ctypes.c_double, vp, vp]
        L.rsst_batch_plan.argtypes = [ctypes.POINTER(rsst_config), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        for name in ("rsst_init", "rsst_prime", "rsst_step", "rsst_stage", "rsst_steps", "rsst_get_time",
                     "rsst_diag", "rsst_poll", "rsst_destroy", "rsst_batch_init", "rsst_batch_set_tiles",
                     "rsst_batch_get_tiles", "rsst_batch_run", "rsst_batch_times", "rsst_batch_poll",
                     "rsst_batch_destroy", "rsst_batch_plan", "rsst_adjoint_step", "rsst_adjoint_step_u1",
                     "rsst_step_out", "rsst_adjoint_run", "rsst_steps_out"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class RsstError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib().rsst_strerror(code).decode()} ({code})")


def _check(code: int, where: str):
    if code != RSST_OK:
        raise RsstError(code, where)


def _stream(stream):
    """A raw hipStream_t from None (torch's current stream), a torch stream
    or an integer handle."""
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    if hasattr(t, "data_ptr"):
        assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


def make_config(cfg: dict, prec: str = "fp64", bg=None, bg_axis: int = -1,
                t_end: float = 0.0, adjoint: bool = False) -> rsst_config:
    """rsst_config from a plain parameter dict (the keys of the workloads module)."""
    c = rsst_config()
    c.ndim = int(cfg["ndim"])
    n = list(cfg["n"]) + [1] * 3
    dx = list(cfg["dx"]) + [1.0] * 3
    g = list(cfg.get("g", [])) + [0.0] * 3
    lo = list(cfg.get("bc_lo", [])) + ["periodic"] * 3
    hi = list(cfg.get("bc_hi", [])) + ["periodic"] * 3
    for d in range(3):
        c.n[d] = int(n[d]) if d < c.ndim else 1
        c.dx[d] = float(dx[d])
        c.g[d] = float(g[d]) if d < c.ndim else 0.0
        c.bc_lo[d] = BCS[lo[d]] if isinstance(lo[d], str) else int(lo[d])
        c.bc_hi[d] = BCS[hi[d]] if isinstance(hi[d], str) else int(hi[d])
    c.gamma = float(cfg["gamma"])
    c.xi = float(cfg["xi"])
    c.cfl = float(cfg.get("cfl", 0.4))
    c.dt_rule = int(cfg.get("dt_rule", 0))
    f = cfg.get("form", "pvs")
    c.form = FORMS[f] if isinstance(f, str) else int(f)
    c.prec = PRECS[prec] if isinstance(prec, str) else int(prec)
    c.bg = ctypes.c_void_p(bg.data_ptr()) if bg is not None else None
    c.bg_axis = int(bg_axis)
    c.t_end = float(t_end)
    c.flags = RSST_WITH_ADJOINT if adjoint else 0
    c.cmax = float(cfg.get("cmax", 0.0))
    e = cfg.get("eos", "ideal")
    c.eos = EOS[e] if isinstance(e, str) else int(e)
    c.eos_a = float(cfg.get("eos_a", 0.0))
    c.eos_b = float(cfg.get("eos_b", 0.0))
    return c


# ---- the C ABI, same names -------------------------------------------------

def rsst_init(cfg: rsst_config, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().rsst_init(ctypes.byref(cfg), _stream(stream), ctypes.byref(h)), "rsst_init")
    return h


def rsst_prime(h, U, t0: float = 0.0, stream=None):
    _check(lib().rsst_prime(h, _ptr(U), float(t0), _stream(stream)), "rsst_prime")


def rsst_step(h, U, dt_fixed: float = 0.0, stream=None):
    _check(lib().rsst_step(h, _ptr(U), float(dt_fixed), _stream(stream)), "rsst_step")


def rsst_step_out(h, U, U1, Unext, dt_fixed: float = 0.0, stream=None):
    _check(lib().rsst_step_out(h, _ptr(U), _ptr(U1), _ptr(Unext), float(dt_fixed), _stream(stream)),
           "rsst_step_out")


def rsst_steps_out(h, U_list, U1_list, dt_fixed: float = 0.0, stream=None):
    """len(U1_list) out-of-place steps: U_list[n+1] from U_list[n], keeping
    U1_list[n] (U_list has one entry more)."""
    n = len(U1_list)
    if len(U_list) != n + 1:
        raise ValueError("rsst_steps_out: U_list needs len(U1_list) + 1 entries")
    us = (ctypes.c_void_p * (n + 1))(*[_ptr(u) for u in U_list])
    u1s = (ctypes.c_void_p * max(n, 1))(*[_ptr(u) for u in U1_list])
    _check(lib().rsst_steps_out(h, us, u1s, n, float(dt_fixed), _stream(stream)), "rsst_steps_out")


def rsst_step_noalloc(cfg: rsst_config, U, dt_fixed: float = 0.0, flags=None, stream=None):
    """One step with no allocation (fixed library scratch); flags: None or a
    one-element int32/uint32 device tensor that receives the step's flags."""
    _check(lib().rsst_step_noalloc(ctypes.byref(cfg), _ptr(U), float(dt_fixed),
                                   _ptr(flags) if flags is not None else None, _stream(stream)),
           "rsst_step_noalloc")


def rsst_stage(h, U, stage: int, dt_fixed: float = 0.0, stream=None):
    _check(lib().rsst_stage(h, _ptr(U), int(stage), float(dt_fixed), _stream(stream)), "rsst_stage")


def rsst_steps(h, U, nsteps: int, dt_fixed: float = 0.0, stream=None):
    _check(lib().rsst_steps(h, _ptr(U), int(nsteps), float(dt_fixed), _stream(stream)), "rsst_steps")


def rsst_get_time(h, stream=None):
    t, dt = ctypes.c_double(), ctypes.c_double()
    _check(lib().rsst_get_time(h, ctypes.byref(t), ctypes.byref(dt), _stream(stream)), "rsst_get_time")
    return t.value, dt.value


def rsst_diag(h, U, stream=None) -> np.ndarray:
    out = (ctypes.c_double * 8)()
    _check(lib().rsst_diag(h, _ptr(U), out, _stream(stream)), "rsst_diag")
    return np.array(out[:], dtype=np.float64)


def rsst_poll(h) -> int:
    """Returns the flag word; raises RsstError(RSST_E_NONPHYSICAL) if any flag is set."""
    f = ctypes.c_uint32()
    code = lib().rsst_poll(h, ctypes.byref(f))
    if code not in (RSST_OK, RSST_E_NONPHYSICAL):
        _check(code, "rsst_poll")
    if code == RSST_E_NONPHYSICAL:
        err = RsstError(code, "rsst_poll")
        err.flags = f.value
        raise err
    return f.value


def rsst_destroy(h):
    _check(lib().rsst_destroy(h), "rsst_destroy")


def rsst_adjoint_step(h, U, lam, dt: float, dJdxi, stream=None):
    _check(lib().rsst_adjoint_step(h, _ptr(U), _ptr(lam), float(dt), _ptr(dJdxi), _stream(stream)),
           "rsst_adjoint_step")


def rsst_adjoint_run(h, U_list, U1_list, lam, dt: float, dJdxi, stream=None):
    """Adjoint of len(U_list) steps over a kept trajectory (U1_list: the
    stage values, or None to recompute them)."""
    n = len(U_list)
    us = (ctypes.c_void_p * max(n, 1))(*[_ptr(u) for u in U_list])
    u1s = None
    if U1_list is not None:
        if len(U1_list) != n:
            raise ValueError("rsst_adjoint_run: U1_list and U_list differ in length")
        u1s = (ctypes.c_void_p * max(n, 1))(*[_ptr(u) for u in U1_list])
    _check(lib().rsst_adjoint_run(h, us, u1s, n, _ptr(lam), float(dt), _ptr(dJdxi), _stream(stream)),
           "rsst_adjoint_run")


def rsst_adjoint_step_u1(h, U, U1, lam, dt: float, dJdxi, stream=None):
    _check(lib().rsst_adjoint_step_u1(h, _ptr(U), _ptr(U1), _ptr(lam), float(dt), _ptr(dJdxi), _stream(stream)),
           "rsst_adjoint_step_u1")


def rsst_version() -> str:
    return lib().rsst_version().decode()


# ---- convenience wrapper ----------------------------------------------------

class Solver:
    """Owns one rsst handle.  U is a contiguous CUDA tensor [nvar, ...]
    (float64, or float32 perturbation with prec='fp32_pert' and a float64
    background tensor bg [nvar, nbg])."""

    def __init__(self, cfg: dict, prec: str = "fp64", bg=None, bg_axis: int = -1,
                 t_end: float = 0.0, stream=None, adjoint: bool = False):
        self.cfg = dict(cfg)
        self.prec = prec
        self._bg = bg  # keep the background alive as long as the handle
        self._c = make_config(cfg, prec, bg, bg_axis, t_end, adjoint)
        self.h = rsst_init(self._c, stream)

    def prime(self, U, t0=0.0, stream=None):
        rsst_prime(self.h, U, t0, stream)

    def step(self, U, dt_fixed=0.0, stream=None):
        rsst_step(self.h, U, dt_fixed, stream)

    def stage(self, U, stage, dt_fixed=0.0, stream=None):
        rsst_stage(self.h, U, stage, dt_fixed, stream)

    def steps(self, U, nsteps, dt_fixed=0.0, stream=None):
        rsst_steps(self.h, U, nsteps, dt_fixed, stream)

    def time(self, stream=None):
        return rsst_get_time(self.h, stream)

    def diag(self, U, stream=None):
        return rsst_diag(self.h, U, stream)

    def step_out(self, U, U1, Unext, dt_fixed=0.0, stream=None):
        """One step out of place: U1 = U + dt R(U), Unext = the stepped state
        (U unchanged; same bits as step)."""
        rsst_step_out(self.h, U, U1, Unext, dt_fixed, stream)

    def steps_out(self, U_list, U1_list, dt_fixed=0.0, stream=None):
        """Steps out of place along a kept trajectory (see rsst_steps_out)."""
        rsst_steps_out(self.h, U_list, U1_list, dt_fixed, stream)

    def adjoint_run(self, U_list, U1_list, lam, dt, dJdxi, stream=None):
        """The adjoint of the steps U_list[n] -> U_list[n+1] (stage values
        U1_list[n], or None), last step first, in one library call."""
        rsst_adjoint_run(self.h, U_list, U1_list, lam, dt, dJdxi, stream)

    def adjoint_step(self, U, lam, dt, dJdxi, stream=None, U1=None):
        """lam <- (dU'/dU)^T lam for the fixed-dt step from U; dJdxi (a
        1-element float64 CUDA tensor) += (dU'/dxi)^T lam.  U1: the step's
        stage value as step_out left it (else recomputed)."""
        if U1 is None:
            rsst_adjoint_step(self.h, U, lam, dt, dJdxi, stream)
        else:
            rsst_adjoint_step_u1(self.h, U, U1, lam, dt, dJdxi, stream)

    def poll(self):
        return rsst_poll(self.h)

    def close(self):
        if self.h is not None:
            rsst_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batched boxes ----------------------------------------------------------

def rsst_batch_init(cfgs, offsets, max_steps: int, stream=None) -> ctypes.c_void_p:
    arr = (rsst_config * len(cfgs))(*cfgs)
    off = (ctypes.c_int64 * len(offsets))(*[int(o) for o in offsets])
    h = ctypes.c_void_p()
    _check(lib().rsst_batch_init(arr, len(cfgs), off, int(max_steps), _stream(stream), ctypes.byref(h)),
           "rsst_batch_init")
    return h


BATCH_PLAN_COLS = 13


def rsst_batch_plan(cfgs, strip_rows=(16, 16, 16, 16)) -> np.ndarray:
    """Host-only work-item table of a batch: rows (box, block, first row,
    end row, ndep, dep[8]) -- see rsst.h."""
    cs = [c if isinstance(c, rsst_config) else make_config(c) for c in cfgs]
    arr = (rsst_config * len(cs))(*cs)
    sr = (ctypes.c_int * 4)(*[int(x) for x in strip_rows])
    n = ctypes.c_int()
    _check(lib().rsst_batch_plan(arr, len(cs), sr, None, 0, ctypes.byref(n)), "rsst_batch_plan")
    tab = np.zeros((n.value, BATCH_PLAN_COLS), dtype=np.int32)
    _check(lib().rsst_batch_plan(arr, len(cs), sr, tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 n.value, ctypes.byref(n)), "rsst_batch_plan")
    return tab


def rsst_batch_set_tiles(h, strip_rows):
    a = (ctypes.c_int * 4)(*[int(x) for x in strip_rows])
    _check(lib().rsst_batch_set_tiles(h, a), "rsst_batch_set_tiles")


def rsst_batch_get_tiles(h):
    a = (ctypes.c_int * 4)()
    _check(lib().rsst_batch_get_tiles(h, a), "rsst_batch_get_tiles")
    return list(a)


def rsst_batch_run(h, U_all, nsteps: int, stream=None):
    _check(lib().rsst_batch_run(h, _ptr(U_all), int(nsteps), _stream(stream)), "rsst_batch_run")


def rsst_batch_times(h, nbox: int, stream=None) -> np.ndarray:
    t = np.zeros(nbox)
    _check(lib().rsst_batch_times(h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)),
           "rsst_batch_times")
    return t


def rsst_batch_poll_raw(h) -> int:
    """The batch's flag word (cleared on the device), without raising."""
    f = ctypes.c_uint32()
    code = lib().rsst_batch_poll(h, ctypes.byref(f))
    if code not in (RSST_OK, RSST_E_NONPHYSICAL) and not (code == RSST_E_DEVICE and f.value & 8):
        _check(code, "rsst_batch_poll")
    return f.value


def rsst_batch_poll(h) -> int:
    f = ctypes.c_uint32()
    code = lib().rsst_batch_poll(h, ctypes.byref(f))
    if code == RSST_E_NONPHYSICAL or (code == RSST_E_DEVICE and f.value & 8):
        err = RsstError(code, "rsst_batch_poll")
        err.flags = f.value
        raise err
    _check(code, "rsst_batch_poll")
    return f.value


def rsst_batch_set_wait_limit(h, seconds: float):
    _check(lib().rsst_batch_set_wait_limit(h, float(seconds)), "rsst_batch_set_wait_limit")


def rsst_batch_set_times(h, t, flags: int = 0, stream=None):
    tt = np.ascontiguousarray(t, dtype=np.float64)
    _check(lib().rsst_batch_set_times(h, tt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.c_uint32(int(flags)), _stream(stream)),
           "rsst_batch_set_times")


def rsst_batch_destroy(h):
    _check(lib().rsst_batch_destroy(h), "rsst_batch_destroy")


class Batch:
    """Many 2D boxes in one packed device array.

    cfgs: per-box parameter dicts; for prec='fp32_pert' also a per-box FP64
    background array [nvar, ny] (bg_axis 1) or [nvar, 1] (bg_axis -1).
    Boxes are packed back to back in box order; pack()/unpack() convert
    between per-box numpy arrays and the packed device tensor."""

    def __init__(self, cfgs, prec="fp64", bgs=None, bg_axes=None, max_steps=256, stream=None):
        import torch
        self.cfgs = [dict(c) for c in cfgs]
        self.prec = prec
        self.nv = 4
        self.shapes = [(self.nv, int(c["n"][1]), int(c["n"][0])) for c in cfgs]
        sizes = [int(np.prod(sh)) for sh in self.shapes]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.total = int(sum(sizes))
        self._bgs = None
        cs = []
        if prec == "fp32_pert":
            self._bgs = [torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).cuda() for b in bgs]
            axes = bg_axes if bg_axes is not None else [1] * len(cfgs)
            for c, b, a in zip(cfgs, self._bgs, axes):
                cs.append(make_config(c, prec, b, a))
        else:
            for c in cfgs:
                cs.append(make_config(c, prec))
        self._cs = cs
        self.dtype = torch.float32 if prec == "fp32_pert" else torch.float64
        self.max_steps = int(max_steps)
        self.h = rsst_batch_init(cs, self.offsets, max_steps, stream)

    def pack(self, arrays):
        import torch
        flat = np.concatenate([np.ascontiguousarray(a).ravel() for a in arrays])
        np_dt = np.float32 if self.prec == "fp32_pert" else np.float64
        return torch.from_numpy(flat.astype(np_dt)).cuda()

    def unpack(self, U):
        flat = U.detach().cpu().numpy()
        return [flat[o:o + int(np.prod(sh))].reshape(sh) for o, sh in zip(self.offsets, self.shapes)]

    def set_tiles(self, strip_rows):
        rsst_batch_set_tiles(self.h, strip_rows)

    def tiles(self):
        return rsst_batch_get_tiles(self.h)

    def autotune(self, U, **kw):
        """Measure and set the strip rows (see autotune.tune)."""
        from . import autotune
        return autotune.tune(self, U, **kw)

    def run(self, U, nsteps, stream=None):
        rsst_batch_run(self.h, U, nsteps, stream)

    def times(self, stream=None):
        return rsst_batch_times(self.h, len(self.cfgs), stream)

    def poll(self):
        return rsst_batch_poll(self.h)

    def set_wait_limit(self, seconds):
        rsst_batch_set_wait_limit(self.h, seconds)

    def set_times(self, t, flags=0, stream=None):
        rsst_batch_set_times(self.h, t, flags, stream)

    def close(self):
        if self.h is not None:
            rsst_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
