"""MI355X (gfx950) explicit phase-field + concentration time stepping.

Python binding of ``libpf.so`` (C-ABI declared in ``include/pf.h``).  This
module only marshals arguments: every step of the time integration runs in the
library's HIP kernels.  PyTorch is used for device memory and streams only
(device arrays are passed as ``torch.Tensor`` data pointers).

If the library has not been built, every entry point raises; there is no CPU
fallback.  Build with ``python -m paper_2601_16522_amd.build`` or
``__graft_entry__.build()``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")

PF_FEULER, PF_SSP_S2, PF_SSP_10_4, PF_RKL1, PF_RKL2 = 0, 1, 2, 3, 4
PF_FP64, PF_FP32 = 0, 1
INTEGRATORS = {"fe": PF_FEULER, "ssp2": PF_SSP_S2, "ssp104": PF_SSP_10_4, "rkl1": PF_RKL1,
               "rkl2": PF_RKL2}
PRECISIONS = {"fp64": PF_FP64, "fp32": PF_FP32}
STATUS = {0: "PF_OK", -1: "PF_EINVAL", -2: "PF_ENOMEM", -3: "PF_EHIP", -4: "PF_ENONFINITE",
          -5: "PF_EDTMIN", -6: "PF_ESTATE", -7: "PF_EUNSUPPORTED"}

# every symbol include/pf.h declares
EXPORTS = ["pf_create", "pf_destroy", "pf_set_stream", "pf_init_fields", "pf_init_fields_device",
           "pf_get_fields", "pf_get_fields_device", "pf_rhs", "pf_rhs_device", "pf_stable_dt",
           "pf_stage_count", "pf_step", "pf_run_to", "pf_error_norm", "pf_error_norm_device",
           "pf_error_norm_device_noalloc",
           "pf_conservation", "pf_set_field_groups", "pf_get_field_groups",
           "pf_diagnostics", "pf_get_trace", "pf_get_state", "pf_set_state", "pf_set_tiling",
           "pf_get_tiling", "pf_autotune", "pf_set_timing", "pf_get_kernel_time",
           "pf_supported_nphi", "pf_last_error", "pf_batch_create", "pf_batch_destroy",
           "pf_batch_set_stream", "pf_batch_init_fields", "pf_batch_get_fields",
           "pf_batch_stable_dt", "pf_batch_run_to", "pf_batch_run_adaptive", "pf_batch_autotune", "pf_batch_set_blocks",
           "pf_batch_set_fusion", "pf_batch_get_config", "pf_batch_last_error",
           "pf_params_stable_dt", "pf_rkl_stage_count", "pf_controller_init",
           "pf_controller_update", "pf_clip_step", "pf_set_timing_families",
           "pf_set_stage_fusion", "pf_get_stage_fusion", "pf_set_r0_recompute",
           "pf_get_r0_recompute", "pf_set_pair_zchunk", "pf_get_pair_zchunk",
           "pf_set_sparse_storage", "pf_get_sparse_storage", "pf_sparse_cuts"]


class PFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("W", C.c_double), ("n_phi", C.c_int),
                ("type_of", C.POINTER(C.c_int)), ("n_types", C.c_int),
                ("gamma", C.POINTER(C.c_double)), ("mob", C.POINTER(C.c_double)),
                ("k", C.POINTER(C.c_double)), ("c0", C.POINTER(C.c_double)),
                ("D", C.POINTER(C.c_double)), ("with_c", C.c_int), ("prec", C.c_int),
                ("ssp_stages", C.c_int), ("bc", C.c_int * 3), ("c_fixed", C.c_int * 6),
                ("c_bc", C.c_double * 6)]


class _Tol(C.Structure):
    _fields_ = [("r_phi", C.c_double), ("a_phi", C.c_double), ("r_c", C.c_double),
                ("a_c", C.c_double), ("dt_max_over_dte", C.c_double), ("dt0", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("rhs_evals", C.c_longlong), ("stages", C.c_longlong),
                ("accepted", C.c_longlong), ("rejected", C.c_longlong),
                ("t", C.c_double), ("last_dt", C.c_double), ("last_err", C.c_double)]


class _Controller(C.Structure):
    _fields_ = [("b", C.c_double), ("nhist", C.c_int), ("E1", C.c_double), ("E2", C.c_double),
                ("h1", C.c_double), ("h2", C.c_double)]


@dataclass
class Tol:
    r_phi: float = 1e-4
    a_phi: float = 1e-2
    r_c: float = 1e-4
    a_c: float = 1e-4
    dt_max_over_dte: float = 200.0
    dt0: float = 0.0

    def _c(self):
        return _Tol(self.r_phi, self.a_phi, self.r_c, self.a_c, self.dt_max_over_dte, self.dt0)


@dataclass
class Stats:
    rhs_evals: int
    stages: int
    accepted: int
    rejected: int
    t: float
    last_dt: float
    last_err: float


_lib = None


def lib():
    """Load libpf.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2601_16522_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, d, i, ll = C.c_void_p, C.c_double, C.c_int, C.c_longlong
        pd = C.POINTER(C.c_double)
        sigs = {
            "pf_create": [C.POINTER(_Params), C.POINTER(vp)],
            "pf_destroy": [vp],
            "pf_set_stream": [vp, vp],
            "pf_init_fields": [vp, pd, pd, d],
            "pf_init_fields_device": [vp, vp, d],
            "pf_get_fields": [vp, pd, pd, pd],
            "pf_get_fields_device": [vp, vp],
            "pf_rhs": [vp, pd, pd],
            "pf_rhs_device": [vp, vp],
            "pf_stable_dt": [vp, pd],
            "pf_stage_count": [vp, i, d, C.POINTER(i)],
            "pf_step": [vp, i, d, C.POINTER(_Stats)],
            "pf_run_to": [vp, i, d, C.POINTER(_Tol), d, C.POINTER(_Stats)],
            "pf_error_norm_device": [vp, i, d, vp, vp, vp, C.POINTER(_Tol), pd, C.POINTER(ll)],
            "pf_error_norm_device_noalloc": [vp, i, d, vp, vp, vp, C.POINTER(_Tol), pd,
                                             C.POINTER(ll)],
            "pf_set_field_groups": [vp, i],
            "pf_get_field_groups": [vp, C.POINTER(i)],
            "pf_conservation": [vp, pd],
            "pf_diagnostics": [vp, pd],
            "pf_get_trace": [vp, pd, ll, C.POINTER(ll)],
            "pf_get_state": [vp, vp, C.POINTER(C.c_size_t)],
            "pf_set_state": [vp, vp, C.c_size_t],
            "pf_set_tiling": [vp, i, i],
            "pf_get_tiling": [vp, C.POINTER(i), C.POINTER(i)],
            "pf_autotune": [vp, C.POINTER(i), C.POINTER(i), pd],
            "pf_set_stage_fusion": [vp, i],
            "pf_get_stage_fusion": [vp, C.POINTER(i)],
            "pf_set_r0_recompute": [vp, i],
            "pf_get_r0_recompute": [vp, C.POINTER(i)],
            "pf_set_pair_zchunk": [vp, i],
            "pf_set_sparse_storage": [vp, i],
            "pf_get_sparse_storage": [vp, C.POINTER(i)],
            "pf_sparse_cuts": [vp, C.POINTER(ll)],
            "pf_get_pair_zchunk": [vp, C.POINTER(i)],
            "pf_set_timing": [vp, i],
            "pf_set_timing_families": [vp, C.c_uint],
            "pf_get_kernel_time": [vp, i, pd, C.POINTER(ll)],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.pf_supported_nphi.argtypes = [C.POINTER(C.c_int), C.c_int]
        L.pf_supported_nphi.restype = C.c_int
        L.pf_last_error.argtypes = [vp]
        L.pf_last_error.restype = C.c_char_p
        bsigs = {
            "pf_batch_create": [C.POINTER(_Params), i, C.POINTER(vp)],
            "pf_batch_destroy": [vp],
            "pf_batch_set_stream": [vp, vp],
            "pf_batch_init_fields": [vp, i, pd, d],
            "pf_batch_get_fields": [vp, i, pd, pd],
            "pf_batch_stable_dt": [vp, i, pd],
            "pf_batch_run_to": [vp, i, pd, pd, i, C.POINTER(_Stats)],
            "pf_batch_run_adaptive": [vp, i, pd, C.POINTER(_Tol), C.POINTER(_Stats)],
            "pf_batch_autotune": [vp, C.POINTER(i), pd],
            "pf_batch_set_blocks": [vp, i],
            "pf_batch_set_fusion": [vp, i],
            "pf_batch_get_config": [vp, C.POINTER(i), C.POINTER(i)],
        }
        for name, args in bsigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.pf_batch_last_error.argtypes = [vp]
        L.pf_batch_last_error.restype = C.c_char_p
        hsigs = {
            "pf_params_stable_dt": [C.POINTER(_Params), pd],
            "pf_rkl_stage_count": [i, d, d, C.POINTER(i)],
            "pf_controller_init": [C.POINTER(_Controller)],
            "pf_controller_update": [C.POINTER(_Controller), i, d, d, C.POINTER(i), pd],
            "pf_clip_step": [d, d, d, pd, C.POINTER(i)],
            "pf_error_norm": [C.POINTER(_Params), ll, pd, pd, pd, C.POINTER(_Tol), pd],
        }
        for name, args in hsigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _lib = L
    return _lib


def supported_nphi():
    out = (C.c_int * 64)()
    n = lib().pf_supported_nphi(out, 64)
    return [out[i] for i in range(min(n, 64))]


# ---------------------------------------------------------------------------
# Host-side helpers (no handle, no device)
# ---------------------------------------------------------------------------

def _hchk(code: int, what: str):
    if code != 0:
        raise PFError(code, what)


def params_stable_dt(params: dict) -> float:
    """dt_e of a parameter set (pf_params_stable_dt)."""
    keep = []
    cp = _cparams(params, "fp64", 0, keep)
    v = C.c_double()
    _hchk(lib().pf_params_stable_dt(C.byref(cp), C.byref(v)), "pf_params_stable_dt")
    return v.value


def rkl_stage_count(integ: str, dt: float, dt_e: float) -> int:
    """RKL stage count for dt (pf_rkl_stage_count); integ is "rkl1" or "rkl2"."""
    v = C.c_int()
    _hchk(lib().pf_rkl_stage_count(INTEGRATORS[integ], dt, dt_e, C.byref(v)), "pf_rkl_stage_count")
    return v.value


class Controller:
    """The engine's step-size controller (pf_controller_*)."""

    def __init__(self):
        self._c = _Controller()
        _hchk(lib().pf_controller_init(C.byref(self._c)), "pf_controller_init")

    def update(self, order: int, err: float, h: float):
        """Returns (accepted, proposed next step)."""
        acc, hn = C.c_int(), C.c_double()
        _hchk(lib().pf_controller_update(C.byref(self._c), order, err, h, C.byref(acc),
                                         C.byref(hn)), "pf_controller_update")
        return bool(acc.value), hn.value

    @property
    def bias(self) -> float:
        return self._c.b


def clip_step(t: float, t_end: float, h: float):
    """(step size, is last) of the next step towards t_end, or None when t_end is reached."""
    hu, last = C.c_double(), C.c_int()
    r = lib().pf_clip_step(t, t_end, h, C.byref(hu), C.byref(last))
    if r < 0:
        raise PFError(-1, "pf_clip_step: invalid arguments")
    return (hu.value, bool(last.value)) if r == 1 else None


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def error_norm(params: dict, e, u_old, u_new, tol: "Tol") -> float:
    """Weighted RMS norm of a local error estimate e on host arrays
    (pf_error_norm): e, u_old, u_new are F x V float64 arrays in the state
    layout; the phi filter is whatever e already holds."""
    keep = []
    cp = _cparams(params, "fp64", 0, keep)
    arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (e, u_old, u_new)]
    V = int(params["nx"]) * int(params["ny"]) * int(params.get("nz", 1))
    F = int(params["n_phi"]) + (1 if params["with_c"] else 0)
    if any(a.size != F * V for a in arrs):
        raise ValueError(f"expected {F * V} values per array")
    out = C.c_double()
    ctol = tol._c()
    _hchk(lib().pf_error_norm(C.byref(cp), V, _dp(arrs[0]), _dp(arrs[1]), _dp(arrs[2]),
                              C.byref(ctol), C.byref(out)), "pf_error_norm")
    return out.value


def _tptr(t) -> C.c_void_p:
    """Device pointer of a contiguous torch tensor."""
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _cparams(p: dict, prec: str, ssp_stages: int, keep: list) -> _Params:
    """pf_params for one parameter dict; the arrays it points to go into keep."""
    N = int(p["n_phi"])
    T = int(p["n_types"])
    arrs = [(C.c_int * N)(*[int(v) for v in p["type_of"]]),
            (C.c_double * (T * T))(*p["gamma"]), (C.c_double * (T * T))(*p["mob"]),
            (C.c_double * T)(*p["k"]), (C.c_double * T)(*p["c0"]), (C.c_double * T)(*p["D"])]
    keep.extend(arrs)
    cp = _Params(int(p["dim"]), int(p["nx"]), int(p["ny"]), int(p.get("nz", 1)),
                 float(p["dx"]), float(p["W"]), N, arrs[0], T, arrs[1], arrs[2], arrs[3],
                 arrs[4], arrs[5], int(bool(p["with_c"])), PRECISIONS[prec], int(ssp_stages))
    # boundaries (optional keys; periodic when absent)
    for a, v in enumerate(p.get("bc", (0, 0, 0))):
        cp.bc[a] = int(v)
    for f, v in enumerate(p.get("c_fixed", (0,) * 6)):
        cp.c_fixed[f] = int(v)
    for f, v in enumerate(p.get("c_bc", (0.0,) * 6)):
        cp.c_bc[f] = float(v)
    return cp


class Batch:
    """Handle on a batch of independent 2D simulations (pf_batch): one fused
    launch advances every instance by a forward-Euler step."""

    def __init__(self, params_list, prec: str = "fp32"):
        self._L = lib()
        self._keep = []
        n = len(params_list)
        arr = (_Params * n)(*[_cparams(p, prec, 5, self._keep) for p in params_list])
        self.n = n
        self.prec = prec
        self.shapes = [(int(p["n_phi"]) + (1 if p["with_c"] else 0), 1, int(p["ny"]), int(p["nx"]))
                       for p in params_list]
        h = C.c_void_p()
        rc = self._L.pf_batch_create(arr, n, C.byref(h))
        if rc != 0:
            raise PFError(rc, "pf_batch_create")
        self._h = h

    def _chk(self, rc):
        if rc != 0:
            raise PFError(rc, self._L.pf_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.pf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._chk(self._L.pf_batch_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def init_fields(self, i: int, u: np.ndarray, t0: float = 0.0):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        if u.size != int(np.prod(self.shapes[i])):
            raise ValueError("wrong state size for instance %d" % i)
        self._chk(self._L.pf_batch_init_fields(self._h, i, _dp(u), t0))

    def get_fields(self, i: int):
        out = np.empty(self.shapes[i], dtype=np.float64)
        t = C.c_double()
        self._chk(self._L.pf_batch_get_fields(self._h, i, _dp(out.reshape(-1)), C.byref(t)))
        return out, t.value

    def stable_dt(self, i: int) -> float:
        v = C.c_double()
        self._chk(self._L.pf_batch_stable_dt(self._h, i, C.byref(v)))
        return v.value

    def run_to(self, t_end, dt=None, graph_steps: int = 0, integ: str = "fe"):
        """Fixed steps of every instance to its t_end (integ "fe" or "rkl2");
        dt per instance or None (0.9 dt_e each)."""
        te = np.ascontiguousarray(t_end, dtype=np.float64)
        if te.size != self.n:
            raise ValueError("t_end needs one value per instance")
        dtv = None if dt is None else np.ascontiguousarray(dt, dtype=np.float64)
        if dtv is not None and dtv.size != self.n:
            raise ValueError("dt needs one value per instance")
        st = (_Stats * self.n)()
        self._chk(self._L.pf_batch_run_to(self._h, INTEGRATORS[integ], _dp(te),
                                          _dp(dtv) if dtv is not None else None,
                                          int(graph_steps), st))
        return [Stats(*[getattr(x, f) for f, _ in _Stats._fields_]) for x in st]

    def run_adaptive(self, t_end, tol: "Tol", integ: str = "rkl2"):
        """Adaptive steps of every instance to its t_end, each with a fresh
        controller of its own (pf_batch_run_adaptive)."""
        te = np.ascontiguousarray(t_end, dtype=np.float64)
        if te.size != self.n:
            raise ValueError("t_end needs one value per instance")
        st = (_Stats * self.n)()
        ctol = tol._c()
        self._chk(self._L.pf_batch_run_adaptive(self._h, INTEGRATORS[integ], _dp(te), C.byref(ctol), st))
        return [Stats(*[getattr(x, f) for f, _ in _Stats._fields_]) for x in st]

    def autotune(self):
        nb, ms = C.c_int(), C.c_double()
        self._chk(self._L.pf_batch_autotune(self._h, C.byref(nb), C.byref(ms)))
        return nb.value, ms.value

    def set_blocks(self, nblocks: int):
        self._chk(self._L.pf_batch_set_blocks(self._h, int(nblocks)))

    def set_fusion(self, depth: int):
        """Steps per batched launch (stage-fusion depth), 1 or 2."""
        self._chk(self._L.pf_batch_set_fusion(self._h, int(depth)))

    def config(self):
        """(persistent grid size, fusion depth) used by the next run."""
        nb, d = C.c_int(), C.c_int()
        self._chk(self._L.pf_batch_get_config(self._h, C.byref(nb), C.byref(d)))
        return nb.value, d.value


class Sim:
    """One simulation handle (pf_sim).  Parameters as produced by
    ``pf_inputs.Workload.param_dict()``."""

    def __init__(self, params: dict, prec: str = "fp64", ssp_stages: int = 5):
        self._L = lib()
        p = params
        self.N = int(p["n_phi"])
        self.with_c = bool(p["with_c"])
        self.F = self.N + (1 if self.with_c else 0)
        self.shape = (self.F, int(p.get("nz", 1)), int(p["ny"]), int(p["nx"]))
        self.V = self.shape[1] * self.shape[2] * self.shape[3]
        self.prec = prec
        self._keep = []
        cp = _cparams(p, prec, ssp_stages, self._keep)
        h = C.c_void_p()
        self._chk(self._L.pf_create(C.byref(cp), C.byref(h)), None)
        self._h = h

    # -- plumbing -----------------------------------------------------------
    def _chk(self, rc: int, h=...):
        if rc != 0:
            handle = self._h if h is ... else h
            msg = self._L.pf_last_error(handle).decode() if handle else ""
            raise PFError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self._L.pf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _state_ptr(self, t) -> C.c_void_p:
        """Pointer of a device tensor holding one full state vector (F*V values of
        the handle's precision); anything else is refused before any launch."""
        if t.numel() != self.F * self.V or t.dtype != self.torch_dtype:
            raise ValueError(f"expected {self.F * self.V} values of {self.torch_dtype}, "
                             f"got {t.numel()} of {t.dtype}")
        return _tptr(t)

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.prec == "fp64" else torch.float32

    def empty_device(self):
        import torch
        return torch.empty(self.shape, dtype=self.torch_dtype, device="cuda")

    # -- API ----------------------------------------------------------------
    def set_stream(self, stream):
        ptr = None if stream is None else C.c_void_p(stream.cuda_stream)
        self._chk(self._L.pf_set_stream(self._h, ptr))

    def init_fields(self, u: np.ndarray, t0: float = 0.0):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        if u.size != self.F * self.V:
            raise ValueError(f"expected {self.F * self.V} values, got {u.size}")
        self._chk(self._L.pf_init_fields(self._h, _dp(u), None, t0))

    def init_fields_device(self, t, t0: float = 0.0):
        self._chk(self._L.pf_init_fields_device(self._h, self._state_ptr(t), t0))

    def get_fields(self):
        out = np.empty(self.shape, dtype=np.float64)
        t = C.c_double()
        flat = out.reshape(-1)
        c_ptr = _dp(flat[self.N * self.V:]) if self.with_c else None
        self._chk(self._L.pf_get_fields(self._h, _dp(flat), c_ptr, C.byref(t)))
        return out, t.value

    def get_fields_device(self, t):
        self._chk(self._L.pf_get_fields_device(self._h, self._state_ptr(t)))

    def rhs(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        flat = out.reshape(-1)
        c_ptr = _dp(flat[self.N * self.V:]) if self.with_c else None
        self._chk(self._L.pf_rhs(self._h, _dp(flat), c_ptr))
        return out

    def rhs_device(self, t):
        self._chk(self._L.pf_rhs_device(self._h, self._state_ptr(t)))

    def stable_dt(self) -> float:
        v = C.c_double()
        self._chk(self._L.pf_stable_dt(self._h, C.byref(v)))
        return v.value

    def stage_count(self, integ: str, dt: float) -> int:
        v = C.c_int()
        self._chk(self._L.pf_stage_count(self._h, INTEGRATORS[integ], dt, C.byref(v)))
        return v.value

    def step(self, integ: str, dt: float) -> Stats:
        st = _Stats()
        self._chk(self._L.pf_step(self._h, INTEGRATORS[integ], dt, C.byref(st)))
        return Stats(*[getattr(st, f) for f, _ in _Stats._fields_])

    def run_to(self, integ: str, t_end: float, tol: Optional[Tol] = None,
               dt_fixed: float = 0.0) -> Stats:
        st = _Stats()
        ctol = tol._c() if tol is not None else None
        self._chk(self._L.pf_run_to(self._h, INTEGRATORS[integ], t_end,
                                    C.byref(ctol) if ctol is not None else None, dt_fixed,
                                    C.byref(st)))
        return Stats(*[getattr(st, f) for f, _ in _Stats._fields_])

    def error_norm(self, kind: int, dt: float, u_old, u_new, aux, tol: Tol):
        """Error norm of an adaptive step on device state vectors
        (pf_error_norm_device): (norm, degrees of freedom)."""
        v = C.c_double()
        n = C.c_longlong()
        ctol = tol._c()
        self._chk(self._L.pf_error_norm_device(self._h, kind, dt, self._state_ptr(u_old),
                                        self._state_ptr(u_new), self._state_ptr(aux),
                                        C.byref(ctol), C.byref(v), C.byref(n)))
        return v.value, n.value

    def error_norm_noalloc(self, kind: int, dt: float, u_old, u_new, aux, tol: Tol):
        """pf_error_norm_device_noalloc: the same norm with its partial sums in
        the library's static device scratch (no device allocation)."""
        v = C.c_double()
        n = C.c_longlong()
        ctol = tol._c()
        self._chk(self._L.pf_error_norm_device_noalloc(
            self._h, kind, dt, self._state_ptr(u_old), self._state_ptr(u_new),
            self._state_ptr(aux), C.byref(ctol), C.byref(v), C.byref(n)))
        return v.value, n.value

    def conservation(self) -> float:
        v = C.c_double()
        self._chk(self._L.pf_conservation(self._h, C.byref(v)))
        return v.value

    def diagnostics(self):
        out = (C.c_double * 5)()
        self._chk(self._L.pf_diagnostics(self._h, out))
        return dict(sum_c=out[0], max_sum_dev=out[1], min_phi=out[2], max_phi=out[3],
                    nonfinite=out[4])

    def trace(self) -> np.ndarray:
        n = C.c_longlong()
        self._chk(self._L.pf_get_trace(self._h, None, 0, C.byref(n)))
        buf = np.zeros(4 * max(n.value, 1))
        self._chk(self._L.pf_get_trace(self._h, _dp(buf), n.value, C.byref(n)))
        return buf[: 4 * n.value].reshape(-1, 4)

    def get_state(self) -> bytes:
        n = C.c_size_t()
        self._chk(self._L.pf_get_state(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._chk(self._L.pf_get_state(self._h, buf, C.byref(n)))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._chk(self._L.pf_set_state(self._h, buf, len(blob)))

    def set_tiling(self, tx: int, zchunk: int):
        self._chk(self._L.pf_set_tiling(self._h, tx, zchunk))

    def get_tiling(self):
        a, b = C.c_int(), C.c_int()
        self._chk(self._L.pf_get_tiling(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self):
        a, b, ms = C.c_int(), C.c_int(), C.c_double()
        self._chk(self._L.pf_autotune(self._h, C.byref(a), C.byref(b), C.byref(ms)))
        return a.value, b.value, ms.value

    def set_field_groups(self, ng: int):
        """Least buffer groups per state vector (0 automatic, 1, 2 or 4)."""
        self._chk(self._L.pf_set_field_groups(self._h, int(ng)))

    def field_groups(self) -> int:
        v = C.c_int()
        self._chk(self._L.pf_get_field_groups(self._h, C.byref(v)))
        return v.value

    def set_stage_fusion(self, depth: int):
        """RKL2 inner stages per launch: 1, or 2 (fused pairs, where built)."""
        self._chk(self._L.pf_set_stage_fusion(self._h, int(depth)))

    def get_stage_fusion(self) -> int:
        d = C.c_int()
        self._chk(self._L.pf_get_stage_fusion(self._h, C.byref(d)))
        return d.value

    def set_r0_recompute(self, on: bool):
        """3D RKL2 inner stages recompute R0 from u^{n,0} (True) or read it."""
        self._chk(self._L.pf_set_r0_recompute(self._h, int(bool(on))))

    def get_r0_recompute(self) -> bool:
        v = C.c_int()
        self._chk(self._L.pf_get_r0_recompute(self._h, C.byref(v)))
        return bool(v.value)

    def set_sparse_storage(self, n_p: int):
        """Sparse phase storage with n_p slots per cell (0: dense); clears the
        fields (call init_fields after it)."""
        self._chk(self._L.pf_set_sparse_storage(self._h, int(n_p)))

    def sparse_storage(self) -> int:
        v = C.c_int()
        self._chk(self._L.pf_get_sparse_storage(self._h, C.byref(v)))
        return v.value

    def sparse_cuts(self) -> int:
        """Cells the sparse storage rule cut since the last call."""
        v = C.c_longlong()
        self._chk(self._L.pf_sparse_cuts(self._h, C.byref(v)))
        return v.value

    def set_pair_zchunk(self, zchunk: int):
        """z planes per block of the 3D fused RKL2 stage pairs."""
        self._chk(self._L.pf_set_pair_zchunk(self._h, int(zchunk)))

    def get_pair_zchunk(self) -> int:
        v = C.c_int()
        self._chk(self._L.pf_get_pair_zchunk(self._h, C.byref(v)))
        return v.value

    def set_timing(self, on: bool, families=None):
        """Kernel timing on/off; families: iterable of FAM_* to record only those."""
        if families is None:
            self._chk(self._L.pf_set_timing(self._h, int(bool(on))))
        else:
            mask = sum(1 << f for f in families) if on else 0
            self._chk(self._L.pf_set_timing_families(self._h, mask))

    def kernel_time(self, family: int):
        ms, n = C.c_double(), C.c_longlong()
        self._chk(self._L.pf_get_kernel_time(self._h, family, C.byref(ms), C.byref(n)))
        return ms.value, n.value


FAM_STAGE, FAM_EST, FAM_RED, FAM_RKL2, FAM_FE = 0, 1, 2, 3, 4
