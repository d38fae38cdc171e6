"""FP64 CPU oracle for the explicit phase-field + concentration time step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product (the HIP library and its
binding) never does.  The oracle shares no code with the HIP path.

The arithmetic lives in ``pf_oracle.c`` (plain C, IEEE double, no contraction);
this module only builds it with gcc and marshals numpy arrays through ctypes.
Each C routine cites the passage of Seiz & Takaki (arXiv 2601.16522) it
follows.  State vectors are float64 arrays of shape (F, nz, ny, nx) with
F = n_phi + with_c (phi planes first, then c).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "libpforacle.so")

FE, SSP2, SSP104, RKL1, RKL2 = 0, 1, 2, 3, 4
MAXN, MAXT = 32, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over cells, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("n_phi", C.c_int), ("with_c", C.c_int), ("n_types", C.c_int),
                ("type_of", C.c_int * MAXN),
                ("dx", C.c_double), ("W", C.c_double),
                ("gamma", C.c_double * (MAXT * MAXT)), ("mob", C.c_double * (MAXT * MAXT)),
                ("k", C.c_double * MAXT), ("c0", C.c_double * MAXT), ("D", C.c_double * MAXT),
                ("bc", C.c_int * 3), ("c_fixed", C.c_int * 6), ("c_bc", C.c_double * 6),
                ("n_p", C.c_int)]


class _Tol(C.Structure):
    _fields_ = [("r_phi", C.c_double), ("a_phi", C.c_double), ("r_c", C.c_double),
                ("a_c", C.c_double), ("dt_max_over_dte", C.c_double), ("dt0", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("rhs_evals", C.c_longlong), ("stages", C.c_longlong),
                ("accepted", C.c_longlong), ("rejected", C.c_longlong),
                ("t", C.c_double), ("last_dt", C.c_double), ("last_err", C.c_double)]


class _Ctrl(C.Structure):
    _fields_ = [("b", C.c_double), ("nhist", C.c_int), ("E1", C.c_double), ("E2", C.c_double),
                ("h1", C.c_double), ("h2", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P, D, I, LL = C.POINTER(_Params), C.POINTER(C.c_double), C.c_int, C.c_longlong
        L.pfo_rhs.argtypes = [P, D, D]
        L.pfo_rhs_at.argtypes = [P, D, C.POINTER(C.c_longlong), LL, D]
        L.pfo_delta.argtypes = [P, D, D]
        L.pfo_mu.argtypes = [P, D, D, D]
        L.pfo_simplex.argtypes = [P, D, C.POINTER(C.c_ubyte)]
        L.pfo_simplex.restype = LL
        L.pfo_rkl_coeffs.argtypes = [I, I, I, D, D, D, D]
        L.pfo_step.argtypes = [P, I, I, C.c_double, D, D, C.POINTER(_Stats)]
        L.pfo_step.restype = I
        L.pfo_stable_dt.argtypes = [P]
        L.pfo_stable_dt.restype = C.c_double
        L.pfo_stage_count.argtypes = [I, C.c_double, C.c_double]
        L.pfo_stage_count.restype = I
        L.pfo_error_norm.argtypes = [P, I, C.c_double, D, D, D, C.POINTER(_Tol),
                                     C.POINTER(LL), D, C.POINTER(_Stats)]
        L.pfo_error_norm.restype = C.c_double
        L.pfo_ctrl_init.argtypes = [C.POINTER(_Ctrl)]
        L.pfo_ctrl_update.argtypes = [C.POINTER(_Ctrl), I, C.c_double, C.c_double, C.POINTER(I)]
        L.pfo_ctrl_update.restype = C.c_double
        L.pfo_run_to.argtypes = [P, I, I, C.c_double, C.c_double, C.POINTER(_Tol), C.c_double,
                                 D, C.POINTER(_Stats), D, LL, C.POINTER(LL),
                                 C.POINTER(_Ctrl), C.POINTER(C.c_double)]
        L.pfo_run_to.restype = I
        L.pfo_sum_c.argtypes = [P, D]
        L.pfo_sum_c.restype = C.c_double
        L.pfo_phi_stats.argtypes = [P, D, D, D, D]
        L.pfo_energy.argtypes = [P, D]
        L.pfo_energy.restype = C.c_double
        L.pfo_pair_constants.argtypes = [P, D, D, D]
        L.pfo_num_threads.restype = I
        L.pfo_set_rkl2_r0_correction.argtypes = [I]
        L.pfo_store.argtypes = [P, D]
        L.pfo_store.restype = LL
        L.pfo_store_truncations.restype = LL
        _lib = L
    return _lib


@dataclass
class Params:
    """Model and grid parameters (Table tab:params defaults)."""
    nx: int
    ny: int
    nz: int = 1
    dim: int = 2
    n_phi: int = 2
    type_of: Sequence[int] = ()
    n_types: int = 1
    dx: float = 1.0
    W: float = 2.5
    gamma: Sequence[float] = (1.0,)   # n_types x n_types, row-major
    mob: Sequence[float] = (1.0,)
    k: Sequence[float] = (500.0,)
    c0: Sequence[float] = (0.5,)
    D: Sequence[float] = (1.0,)
    with_c: bool = True
    bc: Sequence[int] = (0, 0, 0)          # per axis: 0 periodic, 1 zero-gradient walls
    c_fixed: Sequence[int] = (0,) * 6      # per face x-, x+, y-, y+, z-, z+ of a walled axis
    c_bc: Sequence[float] = (0.0,) * 6     # the fixed c of those faces
    n_p: int = 0                           # sparse storage: nonzero phi kept per cell (0: all)

    @property
    def F(self) -> int:
        return self.n_phi + (1 if self.with_c else 0)

    @property
    def shape(self):
        return (self.F, self.nz, self.ny, self.nx)

    def _c(self) -> _Params:
        p = _Params()
        p.dim, p.nx, p.ny, p.nz = self.dim, self.nx, self.ny, self.nz
        p.n_phi, p.with_c, p.n_types = self.n_phi, int(bool(self.with_c)), self.n_types
        tof = list(self.type_of) if len(self.type_of) else [0] * self.n_phi
        for i, t in enumerate(tof):
            p.type_of[i] = int(t)
        p.dx, p.W = float(self.dx), float(self.W)
        T = self.n_types
        for i in range(T * T):
            p.gamma[i] = float(self.gamma[i])
            p.mob[i] = float(self.mob[i])
        for i in range(T):
            p.k[i], p.c0[i], p.D[i] = float(self.k[i]), float(self.c0[i]), float(self.D[i])
        p.n_p = int(self.n_p)
        for a in range(3):
            p.bc[a] = int(self.bc[a])
        for f in range(6):
            p.c_fixed[f] = int(self.c_fixed[f])
            p.c_bc[f] = float(self.c_bc[f])
        return p


@dataclass
class Tol:
    r_phi: float = 1e-4
    a_phi: float = 1e-2
    r_c: float = 1e-4
    a_c: float = 1e-4
    dt_max_over_dte: float = 200.0
    dt0: float = 0.0

    def _c(self) -> _Tol:
        return _Tol(self.r_phi, self.a_phi, self.r_c, self.a_c, self.dt_max_over_dte, self.dt0)


@dataclass
class Stats:
    rhs_evals: int = 0
    stages: int = 0
    accepted: int = 0
    rejected: int = 0
    t: float = 0.0
    last_dt: float = 0.0
    last_err: float = 0.0
    trace: Optional[np.ndarray] = field(default=None, repr=False)


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _state(P: Params, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.size == P.F * P.nx * P.ny * P.nz, (u.shape, P.shape)
    return u.reshape(P.shape)


def rhs(P: Params, u) -> np.ndarray:
    u = _state(P, u)
    r = np.zeros_like(u)
    lib().pfo_rhs(C.byref(P._c()), _dp(u), _dp(r))
    return r


def rhs_at(P: Params, u, cells) -> np.ndarray:
    """The right-hand side at the listed cells (flat indices into a plane),
    shape (len(cells), F): the per-cell formula of rhs()."""
    u = _state(P, u)
    idx = np.ascontiguousarray(cells, dtype=np.int64)
    assert idx.ndim == 1 and (idx >= 0).all() and (idx < P.nx * P.ny * P.nz).all()
    out = np.zeros((idx.size, P.F))
    lib().pfo_rhs_at(C.byref(P._c()), _dp(u), idx.ctypes.data_as(C.POINTER(C.c_longlong)),
                     idx.size, _dp(out))
    return out


def delta(P: Params, u) -> np.ndarray:
    """Variational derivative dF/dphi_a at every cell, shape (n_phi, nz, ny, nx)."""
    u = _state(P, u)
    d = np.zeros((P.n_phi,) + u.shape[1:])
    lib().pfo_delta(C.byref(P._c()), _dp(u), _dp(d))
    return d


def mu(P: Params, u):
    u = _state(P, u)
    m = np.zeros(u.shape[1:])
    mc = np.zeros(u.shape[1:])
    lib().pfo_mu(C.byref(P._c()), _dp(u), _dp(m), _dp(mc))
    return m, mc


def simplex(P: Params, u):
    """Project the phi planes of u (a copy) onto the simplex; returns (u, changed mask)."""
    u = _state(P, u).copy()
    ch = np.zeros(u.shape[1:], dtype=np.uint8)
    lib().pfo_simplex(C.byref(P._c()), _dp(u), ch.ctypes.data_as(C.POINTER(C.c_ubyte)))
    return u, ch.astype(bool)


def store(P: Params, u):
    """The sparse storage rule alone applied to every cell of u (a copy);
    returns (u, number of cells it changed)."""
    u = _state(P, u).copy()
    n = lib().pfo_store(C.byref(P._c()), _dp(u))
    return u, int(n)


def store_truncations() -> int:
    """Cells the sparse storage rule changed since the last call (resets)."""
    return int(lib().pfo_store_truncations())


def rkl_coeffs(order: int, s: int, j: int):
    v = [C.c_double() for _ in range(4)]
    lib().pfo_rkl_coeffs(order, s, j, *[C.byref(x) for x in v])
    return tuple(x.value for x in v)


def step(P: Params, integ: int, dt: float, u, s: int = 0, want_aux: bool = False):
    """One fixed step; returns (u_new, aux, stats).  aux = rhs(u^n) (RKL) or the
    embedded solution (SSP(s)2) when want_aux."""
    u = _state(P, u).copy()
    aux = np.zeros_like(u) if want_aux else None
    st = _Stats()
    rc = lib().pfo_step(C.byref(P._c()), integ, s, dt, _dp(u),
                        _dp(aux) if aux is not None else None, C.byref(st))
    if rc:
        raise RuntimeError(f"pfo_step failed: {rc}")
    return u, aux, _stats(st)


def stable_dt(P: Params) -> float:
    return lib().pfo_stable_dt(C.byref(P._c()))


def stage_count(order: int, dt: float, dte: float) -> int:
    return lib().pfo_stage_count(order, dt, dte)


def error_norm(P: Params, kind: int, dt: float, un, unp1, aux, tol: Tol):
    un, unp1, aux = _state(P, un), _state(P, unp1), _state(P, aux)
    nd = C.c_longlong()
    ss = C.c_double()
    e = lib().pfo_error_norm(C.byref(P._c()), kind, dt, _dp(un), _dp(unp1), _dp(aux),
                             C.byref(tol._c()), C.byref(nd), C.byref(ss), None)
    return e, nd.value, ss.value


class Controller:
    """Thin handle on the oracle's PID controller state."""

    def __init__(self):
        self._c = _Ctrl()
        lib().pfo_ctrl_init(C.byref(self._c))

    @property
    def bias(self) -> float:
        return self._c.b

    def update(self, order: int, e: float, h: float):
        acc = C.c_int()
        hn = lib().pfo_ctrl_update(C.byref(self._c), order, e, h, C.byref(acc))
        return hn, bool(acc.value)


class Carry:
    """Controller state and proposed step carried between adaptive run_to calls."""

    def __init__(self):
        self.ctrl = _Ctrl()
        lib().pfo_ctrl_init(C.byref(self.ctrl))
        self.dt = C.c_double(0.0)


def run_to(P: Params, integ: int, u, t_end: float, tol: Optional[Tol] = None,
           dt_fixed: float = 0.0, s: int = 0, t0: float = 0.0, trace_cap: int = 100000,
           carry: Optional[Carry] = None):
    u = _state(P, u).copy()
    st = _Stats()
    tr = np.zeros(4 * trace_cap)
    nt = C.c_longlong()
    rc = lib().pfo_run_to(C.byref(P._c()), integ, s, t0, t_end,
                          C.byref(tol._c()) if tol is not None else None, dt_fixed,
                          _dp(u), C.byref(st), _dp(tr), trace_cap, C.byref(nt),
                          C.byref(carry.ctrl) if carry else None,
                          C.byref(carry.dt) if carry else None)
    out = _stats(st)
    out.trace = tr[: 4 * min(nt.value, trace_cap)].reshape(-1, 4)
    return u, out, rc


def sum_c(P: Params, u) -> float:
    return lib().pfo_sum_c(C.byref(P._c()), _dp(_state(P, u)))


def phi_stats(P: Params, u):
    v = [C.c_double() for _ in range(3)]
    lib().pfo_phi_stats(C.byref(P._c()), _dp(_state(P, u)), *[C.byref(x) for x in v])
    return tuple(x.value for x in v)


def energy(P: Params, u) -> float:
    return lib().pfo_energy(C.byref(P._c()), _dp(_state(P, u)))


def pair_constants(P: Params):
    N = P.n_phi
    A, B, L = np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))
    lib().pfo_pair_constants(C.byref(P._c()), _dp(A), _dp(B), _dp(L))
    return A, B, L


def _stats(st: _Stats) -> Stats:
    return Stats(st.rhs_evals, st.stages, st.accepted, st.rejected, st.t, st.last_dt, st.last_err)


def num_threads() -> int:
    return lib().pfo_num_threads()


class rkl2_r0_correction_off:
    """Context in which the oracle's RKL2 skips the first-stage correction of
    rhs(u^n) (Sec. 3.2, end): only for tests that measure what the correction
    does to the error."""

    def __enter__(self):
        lib().pfo_set_rkl2_r0_correction(0)
        return self

    def __exit__(self, *exc):
        lib().pfo_set_rkl2_r0_correction(1)
        return False
