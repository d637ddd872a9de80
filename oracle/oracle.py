"""ctypes access to the CPU oracle (``liboracle.so``, built from fem_oracle.c).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain FP64 CPU implementation of
the assembly-free theta-scheme heat solver of arXiv:1905.07622 written from the
paper (assembled CSR, Gauss-quadrature element matrices, textbook Jacobi-PCG).
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it; the GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "fem_oracle.c")

OK, EINVAL, ENOMEM, ENOCONV, EBREAKDOWN = 0, -1, -2, -3, -4
GUESS_EXTRAP, GUESS_PREV = 0, 1
STOP_RHS, STOP_INITIAL = 0, 1
PRECOND_JACOBI, PRECOND_CHEBYSHEV = 0, 1
ELEM_HEX8, ELEM_TET6 = 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", LIB_PATH, SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("k_e", _dp), ("rhoc_e", _dp),
                ("dirichlet_mask", ctypes.c_uint32), ("dirichlet_value", ctypes.c_double * 6),
                ("flux_mask", ctypes.c_uint32), ("flux", ctypes.c_double * 6),
                ("flux_schedule", _dp), ("n_schedule", ctypes.c_int32), ("element", ctypes.c_int32)]


class _Controls(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("theta", ctypes.c_double), ("rtol", ctypes.c_double),
                ("nsteps", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("replace_every", ctypes.c_int32), ("guess", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("first_step", ctypes.c_int32),
                ("locked_iters", _ip), ("nthreads", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("cheb_degree", ctypes.c_int32), ("cheb_ratio", ctypes.c_double)]


class _Precond(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("degree", ctypes.c_int32), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double)]


class _Outputs(ctypes.Structure):
    _fields_ = [("T_final", _dp), ("T_saved", _dp), ("save_every", ctypes.c_int32),
                ("sensor_xyz", _dp), ("n_sensors", ctypes.c_int32), ("traces", _dp),
                ("iters", _ip), ("relres", _dp)]


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.POINTER(ctypes.c_int64)), ("col", _ip), ("val", _dp)]


_lib_handle = None


def lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_element_matrices.argtypes = [ctypes.c_double] * 3 + [_dp, _dp]
        L.oracle_tet6_matrices.argtypes = [ctypes.c_double] * 3 + [_dp, _dp]
        L.oracle_assemble.argtypes = [ctypes.POINTER(_Problem), ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(_CSR), ctypes.c_int]
        L.oracle_csr_free.argtypes = [ctypes.POINTER(_CSR)]
        L.oracle_spmv.argtypes = [ctypes.POINTER(_CSR), _dp, _dp, ctypes.c_int]
        L.oracle_element_loop.argtypes = [ctypes.POINTER(_Problem), ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.oracle_load_vector.argtypes = [ctypes.POINTER(_Problem), _dp]
        L.oracle_dirichlet.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_uint8), _dp]
        L.oracle_sensors.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, ctypes.c_int32, _dp]
        L.oracle_run.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, ctypes.POINTER(_Controls),
                                 ctypes.POINTER(_Outputs)]
        L.oracle_pcg.argtypes = [ctypes.POINTER(_CSR), _dp, _dp, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp, _dp, ctypes.c_int]
        L.oracle_pcg_prec.argtypes = [ctypes.POINTER(_CSR), _dp, _dp, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_Precond), _dp,
                                      _dp, _dp, ctypes.c_int]
        L.oracle_cheb_upper.argtypes = [ctypes.c_double] * 3
        L.oracle_cheb_upper.restype = ctypes.c_double
        L.oracle_cheb_apply.argtypes = [ctypes.POINTER(_CSR), _dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        _dp, _dp, ctypes.c_int]
        L.oracle_cheb_apply.restype = None
        for name in ("oracle_assemble", "oracle_run", "oracle_pcg", "oracle_pcg_prec"):
            getattr(L, name).restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp if a.dtype == np.float64 else _ip)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _ProblemRef:
    """A _Problem plus the arrays it points into (kept alive together)."""

    def __init__(self, prob):
        self.k = _f64(prob.k_e)
        self.rhoc = _f64(prob.rhoc_e)
        self.sched = None if prob.flux_schedule is None else _f64(prob.flux_schedule)
        s = _Problem()
        s.nx, s.ny, s.nz = prob.nx, prob.ny, prob.nz
        s.hx, s.hy, s.hz = prob.hx, prob.hy, prob.hz
        s.k_e, s.rhoc_e = _ptr(self.k), _ptr(self.rhoc)
        s.dirichlet_mask = prob.dirichlet_mask
        s.dirichlet_value = (ctypes.c_double * 6)(*[float(v) for v in prob.dirichlet_value])
        s.flux_mask = prob.flux_mask
        s.flux = (ctypes.c_double * 6)(*[float(v) for v in prob.flux])
        s.flux_schedule = _ptr(self.sched)
        s.n_schedule = 0 if self.sched is None else len(self.sched)
        s.element = getattr(prob, "element", ELEM_HEX8)
        self.s = s
        self.N = prob.n_nodes

    @property
    def ref(self):
        return ctypes.byref(self.s)


def element_matrices(hx: float, hy: float, hz: float):
    M = np.zeros(64)
    K = np.zeros(64)
    lib().oracle_element_matrices(hx, hy, hz, _ptr(M), _ptr(K))
    return M.reshape(8, 8), K.reshape(8, 8)


def tet6_matrices(hx: float, hy: float, hz: float):
    M = np.zeros(64)
    K = np.zeros(64)
    lib().oracle_tet6_matrices(hx, hy, hz, _ptr(M), _ptr(K))
    return M.reshape(8, 8), K.reshape(8, 8)


class CSR:
    """An assembled operator held by the oracle library."""

    def __init__(self, prob, cm: float, ck: float, nthreads: int = 1):
        self._p = _ProblemRef(prob)
        self._c = _CSR()
        rc = lib().oracle_assemble(self._p.ref, cm, ck, ctypes.byref(self._c), nthreads)
        if rc != OK:
            raise MemoryError("oracle_assemble failed")
        self.n = self._c.n
        self.nthreads = nthreads

    def matvec(self, x) -> np.ndarray:
        x = _f64(x)
        y = np.zeros(self.n)
        lib().oracle_spmv(ctypes.byref(self._c), _ptr(x), _ptr(y), self.nthreads)
        return y

    def to_arrays(self):
        nnz = self._c.nnz
        rowptr = np.ctypeslib.as_array(self._c.rowptr, shape=(self.n + 1,)).copy()
        col = np.ctypeslib.as_array(self._c.col, shape=(nnz,)).copy()
        val = np.ctypeslib.as_array(self._c.val, shape=(nnz,)).copy()
        return rowptr, col, val

    def to_dense(self) -> np.ndarray:
        rowptr, col, val = self.to_arrays()
        A = np.zeros((self.n, self.n))
        for i in range(self.n):
            A[i, col[rowptr[i]:rowptr[i + 1]]] = val[rowptr[i]:rowptr[i + 1]]
        return A

    def pcg(self, b, x0, *, max_iter=10000, tol=0.0, relative_to_initial=False, replace_every=50,
            locked=-1):
        b = _f64(b)
        x = _f64(x0).copy()
        delta = np.zeros(1)
        tol_used = np.zeros(1)
        it = lib().oracle_pcg(ctypes.byref(self._c), _ptr(b), _ptr(x), max_iter, tol,
                              int(relative_to_initial), replace_every, locked, _ptr(delta),
                              _ptr(tol_used), self.nthreads)
        return x, it, float(delta[0])

    def diagonal(self) -> np.ndarray:
        rowptr, col, val = self.to_arrays()
        P = np.zeros(self.n)
        for i in range(self.n):
            row = slice(rowptr[i], rowptr[i + 1])
            P[i] = val[row][col[row] == i].sum()
        return P

    def cheb_apply(self, r, degree, lo, hi, P=None) -> np.ndarray:
        """s = q(D^-1 A) D^-1 r, the Chebyshev preconditioner (P: the diagonal, 0 on rows left out)."""
        r = _f64(r)
        P = self.diagonal() if P is None else _f64(P)
        s = np.zeros(self.n)
        lib().oracle_cheb_apply(ctypes.byref(self._c), _ptr(P), degree, lo, hi, _ptr(r), _ptr(s), self.nthreads)
        return s

    def pcg_cheb(self, b, x0, *, degree, lo, hi, max_iter=10000, tol=0.0, relative_to_initial=False,
                 replace_every=50, locked=-1):
        b = _f64(b)
        x = _f64(x0).copy()
        delta = np.zeros(1)
        tol_used = np.zeros(1)
        pc = _Precond(PRECOND_CHEBYSHEV, degree, lo, hi)
        it = lib().oracle_pcg_prec(ctypes.byref(self._c), _ptr(b), _ptr(x), max_iter, tol, int(relative_to_initial),
                                   replace_every, locked, ctypes.byref(pc), None, _ptr(delta), _ptr(tol_used),
                                   self.nthreads)
        return x, it, float(delta[0])

    def close(self):
        if self._c.rowptr:
            lib().oracle_csr_free(ctypes.byref(self._c))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def operator_apply(prob, cm: float, ck: float, x, nthreads: int = 1) -> np.ndarray:
    """y = (sum_e cm*rhoc_e*M_e + ck*k_e*K_e) x through the assembled CSR."""
    A = CSR(prob, cm, ck, nthreads)
    try:
        return A.matvec(x)
    finally:
        A.close()


def cheb_upper(hx: float, hy: float, hz: float) -> float:
    """The oracle's bound of the spectrum of D^-1 A on boxes of this shape."""
    return float(lib().oracle_cheb_upper(hx, hy, hz))


def element_loop(prob, cm: float, ck: float, x) -> np.ndarray:
    p = _ProblemRef(prob)
    x = _f64(x)
    y = np.zeros(p.N)
    lib().oracle_element_loop(p.ref, cm, ck, _ptr(x), _ptr(y))
    return y


def load_vector(prob) -> np.ndarray:
    p = _ProblemRef(prob)
    F = np.zeros(p.N)
    lib().oracle_load_vector(p.ref, _ptr(F))
    return F


def dirichlet(prob):
    p = _ProblemRef(prob)
    d = np.zeros(p.N, dtype=np.uint8)
    g = np.zeros(p.N)
    lib().oracle_dirichlet(p.ref, d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _ptr(g))
    return d.astype(bool), g


def sensors(prob, T, xyz) -> np.ndarray:
    p = _ProblemRef(prob)
    T = _f64(T)
    xyz = _f64(xyz).reshape(-1, 3)
    out = np.zeros(len(xyz))
    lib().oracle_sensors(p.ref, _ptr(T), _ptr(xyz), len(xyz), _ptr(out))
    return out


def run(prob, T0=None, T_prev=None, *, nsteps=None, dt=None, theta=None, rtol=None,
        max_iter=10000, replace_every=50, guess=GUESS_EXTRAP, stop_rule=STOP_RHS, first_step=0,
        locked_iters=None, save_every=0, sensor_xyz=None, nthreads=1, precond=PRECOND_JACOBI, cheb_degree=3,
        cheb_ratio=30.0) -> dict:
    """Run the theta-scheme with the problem's controls unless overridden."""
    p = _ProblemRef(prob)
    N = p.N
    nsteps = prob.nsteps if nsteps is None else nsteps
    T0 = _f64(prob.T0 if T0 is None else T0)
    Tp = None if T_prev is None else _f64(T_prev)
    c = _Controls()
    c.dt = prob.dt if dt is None else dt
    c.theta = prob.theta if theta is None else theta
    c.rtol = prob.rtol if rtol is None else rtol
    c.nsteps, c.max_iter, c.replace_every = nsteps, max_iter, replace_every
    c.guess, c.stop_rule, c.first_step = guess, stop_rule, first_step
    locked = None
    if locked_iters is not None:
        locked = np.ascontiguousarray(locked_iters, dtype=np.int32)
        assert len(locked) >= nsteps
        c.locked_iters = locked.ctypes.data_as(_ip)
    c.nthreads = nthreads
    c.precond, c.cheb_degree, c.cheb_ratio = precond, cheb_degree, cheb_ratio
    xyz = prob.sensors if sensor_xyz is None else sensor_xyz
    xyz = None if xyz is None else _f64(xyz).reshape(-1, 3)
    S = 0 if xyz is None else len(xyz)
    T_final = np.zeros(N)
    T_saved = np.zeros(((nsteps // save_every) if save_every else 0, N))
    traces = np.zeros((nsteps, S))
    iters = np.zeros(nsteps, dtype=np.int32)
    relres = np.zeros(nsteps)
    o = _Outputs()
    o.T_final = _ptr(T_final)
    o.T_saved = _ptr(T_saved) if save_every else None
    o.save_every = save_every
    o.sensor_xyz = _ptr(xyz) if S else None
    o.n_sensors = S
    o.traces = _ptr(traces) if S else None
    o.iters = iters.ctypes.data_as(_ip)
    o.relres = _ptr(relres)
    status = lib().oracle_run(p.ref, _ptr(T0), _ptr(Tp), ctypes.byref(c), ctypes.byref(o))
    return dict(status=status, T_final=T_final, T_saved=T_saved, traces=traces, iters=iters,
                relres=relres)
