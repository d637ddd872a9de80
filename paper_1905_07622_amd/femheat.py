"""Python binding of the C ABI in include/fem_heat.h (libfemheat.so).

Argument marshalling only: every step of the solver runs in the HIP library.
The functions keep the C names; ``Heat`` wraps a handle for numpy arrays
(host memory) or torch CUDA tensors (device memory, ``device_ptrs=True``).
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfemheat.so")

FEM_OK, FEM_EINVAL, FEM_ENOMEM, FEM_ENOCONV, FEM_EBREAKDOWN, FEM_EDEVICE, FEM_EBUSY, FEM_ECANCELED = (
    0, -1, -2, -3, -4, -5, -6, -7)
FEM_FP64, FEM_FP32_FP64DOT = 0, 1
FEM_GUESS_EXTRAP, FEM_GUESS_PREV = 0, 1
FEM_STOP_RHS, FEM_STOP_INITIAL = 0, 1
FEM_PRECOND_JACOBI, FEM_PRECOND_CHEBYSHEV = 0, 1
FEM_ELEM_HEX8, FEM_ELEM_TET6 = 0, 1
FEM_DEVICE_PTRS, FEM_TIMING, FEM_ONE_REDUCTION, FEM_ONE_KERNEL = 0x1, 0x2, 0x4, 0x8
FEM_OP_A, FEM_OP_L, FEM_OP_JACOBI, FEM_OP_LOAD, FEM_OP_FP32, FEM_OP_ELEMENTWISE, FEM_OP_ROWWAVE = (
    0, 1, 2, 3, 0x100, 0x200, 0x400)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class fem_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double)]


class fem_bc(ctypes.Structure):
    _fields_ = [("dirichlet_mask", ctypes.c_uint32), ("dirichlet_value", ctypes.c_double * 6),
                ("flux_mask", ctypes.c_uint32), ("flux", ctypes.c_double * 6),
                ("flux_schedule", _dp), ("n_schedule", ctypes.c_int32)]


class fem_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("replace_every", ctypes.c_int32), ("guess", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("hip_stream", ctypes.c_void_p), ("device", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("allocator", ctypes.c_void_p), ("precond", ctypes.c_int32), ("cheb_degree", ctypes.c_int32),
                ("cheb_ratio", ctypes.c_double), ("element", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
                ("batch_groups", ctypes.c_int32)]


class fem_out(ctypes.Structure):
    _fields_ = [("T_final", _dp), ("T_saved", _dp), ("save_every", ctypes.c_int32),
                ("sensor_xyz", _dp), ("n_sensors", ctypes.c_int32), ("traces", _dp),
                ("iters", _ip), ("relres", _dp), ("refine_sweeps", _ip),
                ("first_step", ctypes.c_int32), ("total_iters", ctypes.c_int64),
                ("device_ms", ctypes.c_double)]


class fem_stats(ctypes.Structure):
    _fields_ = [("gather_launches", ctypes.c_int64), ("gather_ms", ctypes.c_double),
                ("update_launches", ctypes.c_int64), ("update_ms", ctypes.c_double),
                ("replace_launches", ctypes.c_int64), ("replace_ms", ctypes.c_double),
                ("grid_blocks", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("apply_calls", ctypes.c_int64), ("apply_ms", ctypes.c_double),
                ("one_kernel_launches", ctypes.c_int64)]


FEM_TUNE_BATCH = 0x1


class fem_tune_result(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("best_us", ctypes.c_double), ("rule_us", ctypes.c_double),
                ("recorded", ctypes.c_int32)]


class fem_request(ctypes.Structure):
    _fields_ = [("grid", fem_grid), ("k_e", _dp), ("rhoc_e", _dp), ("bc", fem_bc),
                ("T0", _dp), ("T_prev", _dp), ("dt", ctypes.c_double), ("theta", ctypes.c_double),
                ("rtol", ctypes.c_double), ("nsteps", ctypes.c_int32), ("out", ctypes.POINTER(fem_out))]


FEM_REQ_QUEUED, FEM_REQ_RUNNING, FEM_REQ_DONE, FEM_REQ_CANCELED = 0, 1, 2, 3


class fem_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32), ("opts", fem_opts)]


class fem_status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("steps_done", ctypes.c_int32),
                ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("bytes", ctypes.c_uint64)]


class fem_server_info(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("canceled", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("epochs", ctypes.c_int64), ("queued", ctypes.c_int32),
                ("running", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("peak_bytes_in_use", ctypes.c_uint64), ("now", ctypes.c_double)]


class FemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{fem_strerror(status)} ({status}): {msg}")
        self.status = status


EXPORTS = ("fem_heat_create", "fem_heat_run", "fem_heat_apply", "fem_heat_apply_noalloc", "fem_heat_stats",
           "fem_heat_tune",
           "fem_heat_destroy",
           "fem_heat_default_opts", "fem_strerror", "fem_last_error", "fem_heat_run_batch",
           "fem_server_create", "fem_server_submit", "fem_server_poll", "fem_server_wait", "fem_server_cancel",
           "fem_server_info_get", "fem_server_destroy")

_lib = None


def lib():
    """Load libfemheat.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.fem_heat_create.argtypes = [ctypes.POINTER(fem_grid), _dp, _dp, ctypes.POINTER(fem_bc),
                                      ctypes.POINTER(fem_opts), ctypes.POINTER(vp)]
        L.fem_heat_run.argtypes = [vp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_double, ctypes.POINTER(fem_out)]
        L.fem_heat_apply.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.fem_heat_apply_noalloc.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, vp, vp]
        L.fem_heat_stats.argtypes = [vp, ctypes.POINTER(fem_stats)]
        L.fem_heat_tune.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                    ctypes.POINTER(fem_tune_result)]
        L.fem_heat_run_batch.argtypes = [ctypes.POINTER(fem_request), ctypes.c_int32, ctypes.POINTER(fem_opts), _ip]
        L.fem_heat_run_batch.restype = ctypes.c_int
        L.fem_server_create.argtypes = [ctypes.POINTER(fem_server_opts), ctypes.POINTER(vp)]
        L.fem_server_submit.argtypes = [vp, ctypes.POINTER(fem_request), ctypes.POINTER(ctypes.c_uint64)]
        L.fem_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(fem_status)]
        L.fem_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(fem_status)]
        L.fem_server_cancel.argtypes = [vp, ctypes.c_uint64]
        L.fem_server_info_get.argtypes = [vp, ctypes.POINTER(fem_server_info)]
        L.fem_server_destroy.argtypes = [vp]
        L.fem_server_destroy.restype = None
        for n in ("fem_server_create", "fem_server_submit", "fem_server_poll", "fem_server_wait",
                  "fem_server_cancel", "fem_server_info_get"):
            getattr(L, n).restype = ctypes.c_int
        L.fem_heat_destroy.argtypes = [vp]
        L.fem_heat_destroy.restype = None
        L.fem_heat_default_opts.argtypes = [ctypes.POINTER(fem_opts)]
        L.fem_heat_default_opts.restype = None
        L.fem_strerror.argtypes = [ctypes.c_int]
        L.fem_strerror.restype = ctypes.c_char_p
        L.fem_last_error.argtypes = [vp]
        L.fem_last_error.restype = ctypes.c_char_p
        for n in ("fem_heat_create", "fem_heat_run", "fem_heat_apply", "fem_heat_apply_noalloc", "fem_heat_stats",
                  "fem_heat_tune"):
            getattr(L, n).restype = ctypes.c_int
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# the C entry points, same names
# ---------------------------------------------------------------------------

def fem_strerror(status: int) -> str:
    return lib().fem_strerror(status).decode()


def fem_last_error(h) -> str:
    return lib().fem_last_error(h).decode()


def fem_heat_default_opts() -> fem_opts:
    o = fem_opts()
    lib().fem_heat_default_opts(ctypes.byref(o))
    return o


def fem_heat_create(grid: fem_grid, k_e_ptr, rhoc_e_ptr, bc: Optional[fem_bc], opts: Optional[fem_opts]):
    h = ctypes.c_void_p()
    st = lib().fem_heat_create(ctypes.byref(grid), k_e_ptr, rhoc_e_ptr,
                               ctypes.byref(bc) if bc is not None else None,
                               ctypes.byref(opts) if opts is not None else None, ctypes.byref(h))
    return st, h


def fem_heat_run(h, T0_ptr, T_prev_ptr, dt, theta, nsteps, rtol, out: Optional[fem_out]) -> int:
    return lib().fem_heat_run(h, T0_ptr, T_prev_ptr, dt, theta, nsteps, rtol,
                              ctypes.byref(out) if out is not None else None)


def fem_heat_apply(h, which, dt, theta, x_ptr, y_ptr) -> int:
    return lib().fem_heat_apply(h, which, dt, theta, x_ptr, y_ptr)


def fem_heat_apply_noalloc(h, which, dt, theta, x_dev_ptr, y_dev_ptr) -> int:
    """Device pointers (ints) in and out; enqueues on the handle's stream and returns."""
    return lib().fem_heat_apply_noalloc(h, which, dt, theta, x_dev_ptr, y_dev_ptr)


def fem_heat_tune(h, dt, theta, flags=0):
    r = fem_tune_result()
    st = lib().fem_heat_tune(h, dt, theta, flags, ctypes.byref(r))
    return st, r


def fem_heat_stats(h) -> fem_stats:
    s = fem_stats()
    st = lib().fem_heat_stats(h, ctypes.byref(s))
    if st != FEM_OK:
        raise FemError(st, "fem_heat_stats")
    return s


def fem_heat_destroy(h) -> None:
    lib().fem_heat_destroy(h)


def fem_heat_run_batch(reqs, n: int, opts: Optional[fem_opts], status_ptr) -> int:
    return lib().fem_heat_run_batch(reqs, n, ctypes.byref(opts) if opts is not None else None, status_ptr)


def fem_server_create(opts: Optional[fem_server_opts]):
    s = ctypes.c_void_p()
    st = lib().fem_server_create(ctypes.byref(opts) if opts is not None else None, ctypes.byref(s))
    return st, s


def fem_server_submit(s, req: fem_request):
    t = ctypes.c_uint64()
    st = lib().fem_server_submit(s, ctypes.byref(req), ctypes.byref(t))
    return st, t.value


def fem_server_poll(s, ticket: int):
    out = fem_status()
    st = lib().fem_server_poll(s, ticket, ctypes.byref(out))
    return st, out


def fem_server_wait(s, ticket: int, timeout_s: float):
    out = fem_status()
    st = lib().fem_server_wait(s, ticket, timeout_s, ctypes.byref(out))
    return st, out


def fem_server_cancel(s, ticket: int) -> int:
    return lib().fem_server_cancel(s, ticket)


def fem_server_info_get(s):
    out = fem_server_info()
    st = lib().fem_server_info_get(s, ctypes.byref(out))
    return st, out


def fem_server_destroy(s) -> None:
    lib().fem_server_destroy(s)


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Arrays:
    """Turns numpy arrays (host) or torch CUDA tensors (device) into pointers,
    keeping the objects alive."""

    def __init__(self, device: bool):
        self.device = device
        self.keep = []

    def inp(self, a, dtype=np.float64):
        if a is None:
            return None
        if self.device:
            import torch
            if not (_is_torch(a) and a.is_cuda):
                raise TypeError("device_ptrs handle: pass torch CUDA tensors")
            t = a.contiguous().to(torch.float64 if dtype == np.float64 else torch.int32)
            self.keep.append(t)
            return ctypes.cast(t.data_ptr(), _dp if dtype == np.float64 else _ip)
        arr = np.ascontiguousarray(a, dtype=dtype)
        self.keep.append(arr)
        return arr.ctypes.data_as(_dp if dtype == np.float64 else _ip)

    def out(self, shape, dtype=np.float64):
        if self.device:
            import torch
            t = torch.empty(shape, dtype=torch.float64 if dtype == np.float64 else torch.int32, device="cuda")
            self.keep.append(t)
            return t, ctypes.cast(t.data_ptr(), _dp if dtype == np.float64 else _ip)
        arr = np.zeros(shape, dtype=dtype)
        self.keep.append(arr)
        return arr, arr.ctypes.data_as(_dp if dtype == np.float64 else _ip)


def make_opts(*, precision=FEM_FP64, max_iter=10000, replace_every=50, guess=FEM_GUESS_EXTRAP,
              stop_rule=FEM_STOP_RHS, max_refine=4, inner_rtol=1e-5, device_ptrs=False, timing=False,
              one_reduction=False, tile=(0, 0, 0), stream=None, device=0, tune_cache=None,
              precond=FEM_PRECOND_JACOBI, cheb_degree=3, cheb_ratio=30.0, element=FEM_ELEM_HEX8,
              batch_groups=0) -> fem_opts:
    o = fem_heat_default_opts()
    o.batch_groups = batch_groups
    o.precond, o.cheb_degree, o.cheb_ratio, o.element = precond, cheb_degree, cheb_ratio, element
    o.precision, o.max_iter, o.replace_every = precision, max_iter, replace_every
    o.guess, o.stop_rule, o.max_refine, o.inner_rtol = guess, stop_rule, max_refine, inner_rtol
    o.flags = ((FEM_DEVICE_PTRS if device_ptrs else 0) | (FEM_TIMING if timing else 0)
               | (FEM_ONE_REDUCTION if one_reduction else 0))
    o.hip_stream = stream
    o.device = device
    o.tile_x, o.tile_y, o.tile_z = tile
    o.tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
    return o


def _bc(p, keep):
    bc = fem_bc()
    bc.dirichlet_mask = p.dirichlet_mask
    bc.dirichlet_value = (ctypes.c_double * 6)(*[float(v) for v in p.dirichlet_value])
    bc.flux_mask = p.flux_mask
    bc.flux = (ctypes.c_double * 6)(*[float(v) for v in p.flux])
    if p.flux_schedule is not None:
        sched = np.ascontiguousarray(p.flux_schedule, dtype=np.float64)
        keep.append(sched)
        bc.flux_schedule = sched.ctypes.data_as(_dp)
        bc.n_schedule = len(sched)
    return bc


def _outputs(a: "_Arrays", N: int, nsteps: int, save_every: int, sensors):
    out = fem_out()
    res = {}
    res["T_final"], out.T_final = a.out((N,))
    n_saved = nsteps // save_every if save_every else 0
    res["T_saved"] = None
    if n_saved:
        res["T_saved"], out.T_saved = a.out((n_saved, N))
    out.save_every = save_every
    res["traces"] = None
    if sensors is not None:
        out.sensor_xyz = a.inp(sensors)
        out.n_sensors = len(sensors)
        res["traces"], out.traces = a.out((nsteps, len(sensors)))
    res["iters"], out.iters = a.out((nsteps,), np.int32)
    res["relres"], out.relres = a.out((nsteps,))
    res["refine_sweeps"], out.refine_sweeps = a.out((nsteps,), np.int32)
    return out, res


def run_batch(problems, *, save_every=0, sensors=False, T_prev=None, check=True, **opt_kw):
    """Runs workloads.Problem instances together through fem_heat_run_batch.

    Each problem brings its grid, coefficients, boundary data, T0, dt, theta,
    nsteps and rtol (and its sensor points when ``sensors`` is true); the
    keyword options (precision, tile, device_ptrs, ...) apply to all.
    Returns (status, list of per-simulation result dicts)."""
    device = bool(opt_kw.get("device_ptrs", False))
    if problems:
        opt_kw.setdefault("element", getattr(problems[0], "element", FEM_ELEM_HEX8))
    a = _Arrays(device)
    n = len(problems)
    reqs = (fem_request * max(n, 1))()
    outs, results = [], []
    for i, p in enumerate(problems):
        r = reqs[i]
        r.grid = fem_grid(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz)
        r.k_e = a.inp(p.k_e)
        r.rhoc_e = a.inp(p.rhoc_e)
        r.bc = _bc(p, a.keep)
        r.T0 = a.inp(p.T0)
        r.T_prev = a.inp(T_prev[i]) if T_prev is not None else None
        r.dt, r.theta, r.rtol, r.nsteps = p.dt, p.theta, p.rtol, p.nsteps
        out, res = _outputs(a, p.n_nodes, p.nsteps, save_every, p.sensors if sensors else None)
        outs.append(out)
        r.out = ctypes.pointer(out)
        results.append(res)
    status = np.zeros(max(n, 1), dtype=np.int32)
    opts = make_opts(**opt_kw)
    st = fem_heat_run_batch(reqs, n, opts, status.ctypes.data_as(_ip))
    if check and st not in (FEM_OK, FEM_ENOCONV):
        raise FemError(st, fem_last_error(None))
    for i, res in enumerate(results):
        res["status"] = int(status[i])
        res["total_iters"] = int(outs[i].total_iters)
        res["device_ms"] = float(outs[i].device_ms)
    return st, results


def _status_dict(st: fem_status) -> dict:
    return {k: getattr(st, k) for k, _ in fem_status._fields_}


class Server:
    """A fem_server: submit workloads.Problem requests, poll or wait for them.

    Output arrays of each request are allocated here and kept alive until the
    request is finished; ``wait`` returns them."""

    def __init__(self, budget_bytes=0, max_slots=0, **opt_kw):
        so = fem_server_opts()
        so.hbm_budget_bytes = int(budget_bytes)
        so.max_slots = int(max_slots)
        so.opts = make_opts(**opt_kw)
        st, self.s = fem_server_create(so)
        if st != FEM_OK:
            raise FemError(st, fem_last_error(None))
        self._pending = {}

    def submit(self, p, *, save_every=0, sensors=False) -> int:
        a = _Arrays(False)
        r = fem_request()
        r.grid = fem_grid(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz)
        r.k_e = a.inp(p.k_e)
        r.rhoc_e = a.inp(p.rhoc_e)
        r.bc = _bc(p, a.keep)
        r.T0 = a.inp(p.T0)
        r.dt, r.theta, r.rtol, r.nsteps = p.dt, p.theta, p.rtol, p.nsteps
        out, res = _outputs(a, p.n_nodes, p.nsteps, save_every, p.sensors if sensors else None)
        r.out = ctypes.pointer(out)
        st, ticket = fem_server_submit(self.s, r)
        if st != FEM_OK:
            raise FemError(st, fem_last_error(None))
        self._pending[ticket] = (a, out, res)
        return ticket

    def poll(self, ticket: int) -> dict:
        st, s = fem_server_poll(self.s, ticket)
        if st != FEM_OK:
            raise FemError(st, "unknown ticket")
        return _status_dict(s)

    def wait(self, ticket: int, timeout: float = -1.0):
        """Returns (status, state dict, result dict or None if not finished)."""
        st, s = fem_server_wait(self.s, ticket, timeout)
        d = _status_dict(s)
        if d["state"] not in (FEM_REQ_DONE, FEM_REQ_CANCELED):
            return st, d, None
        a, out, res = self._pending.pop(ticket)
        res = dict(res)
        res["status"] = d["status"]
        res["total_iters"] = int(out.total_iters)
        res["device_ms"] = float(out.device_ms)
        return st, d, res

    def cancel(self, ticket: int) -> int:
        return fem_server_cancel(self.s, ticket)

    def info(self) -> dict:
        st, i = fem_server_info_get(self.s)
        return {k: getattr(i, k) for k, _ in fem_server_info._fields_}

    def close(self):
        if getattr(self, "s", None):
            fem_server_destroy(self.s)
            self.s = None
            self._pending.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Heat:
    """One solver handle for a grid, coefficient field and boundary conditions."""

    def __init__(self, nx, ny, nz, hx, hy, hz, k_e, rhoc_e, *, dirichlet_mask=0, dirichlet_value=None,
                 flux_mask=0, flux=None, flux_schedule=None, precision=FEM_FP64, max_iter=10000,
                 replace_every=50, guess=FEM_GUESS_EXTRAP, stop_rule=FEM_STOP_RHS, max_refine=4,
                 inner_rtol=1e-5, device_ptrs=False, timing=False, one_reduction=False, tile=(0, 0, 0), stream=None,
                 device=0, tune_cache=None, precond=FEM_PRECOND_JACOBI, cheb_degree=3, cheb_ratio=30.0,
                 element=FEM_ELEM_HEX8, one_kernel=False):
        self.h = None
        self.device_ptrs = device_ptrs
        self.N = (nx + 1) * (ny + 1) * (nz + 1)
        self.E = nx * ny * nz
        self.grid = fem_grid(nx, ny, nz, hx, hy, hz)
        bc = fem_bc()
        bc.dirichlet_mask = dirichlet_mask
        bc.dirichlet_value = (ctypes.c_double * 6)(*([0.0] * 6 if dirichlet_value is None else list(dirichlet_value)))
        bc.flux_mask = flux_mask
        bc.flux = (ctypes.c_double * 6)(*([0.0] * 6 if flux is None else list(flux)))
        self._sched = None if flux_schedule is None else np.ascontiguousarray(flux_schedule, dtype=np.float64)
        bc.flux_schedule = None if self._sched is None else self._sched.ctypes.data_as(_dp)
        bc.n_schedule = 0 if self._sched is None else len(self._sched)
        o = fem_heat_default_opts()
        o.precision, o.max_iter, o.replace_every = precision, max_iter, replace_every
        o.guess, o.stop_rule, o.max_refine, o.inner_rtol = guess, stop_rule, max_refine, inner_rtol
        o.precond, o.cheb_degree, o.cheb_ratio, o.element = precond, cheb_degree, cheb_ratio, element
        o.flags = ((FEM_DEVICE_PTRS if device_ptrs else 0) | (FEM_TIMING if timing else 0)
                   | (FEM_ONE_REDUCTION if one_reduction else 0) | (FEM_ONE_KERNEL if one_kernel else 0))
        o.hip_stream = stream
        o.device = device
        o.tile_x, o.tile_y, o.tile_z = tile
        self._tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
        o.tune_cache = self._tune_cache
        self.opts = o
        arrs = _Arrays(device_ptrs)
        st, h = fem_heat_create(self.grid, arrs.inp(k_e), arrs.inp(rhoc_e), bc, o)
        if st != FEM_OK:
            raise FemError(st, fem_last_error(None))
        self.h = h

    @classmethod
    def from_problem(cls, p, **kw):
        kw.setdefault("element", getattr(p, "element", FEM_ELEM_HEX8))
        return cls(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, p.k_e, p.rhoc_e,
                   dirichlet_mask=p.dirichlet_mask, dirichlet_value=p.dirichlet_value,
                   flux_mask=p.flux_mask, flux=p.flux, flux_schedule=p.flux_schedule, **kw)

    def run(self, T0, T_prev=None, *, dt, theta, nsteps, rtol, save_every=0, sensors=None, first_step=0,
            check=True) -> dict:
        a = _Arrays(self.device_ptrs)
        out = fem_out()
        T_final, out.T_final = a.out((self.N,))
        n_saved = nsteps // save_every if save_every else 0
        T_saved = None
        if n_saved:
            T_saved, out.T_saved = a.out((n_saved, self.N))
        out.save_every = save_every
        S = 0
        traces = None
        if sensors is not None:
            S = len(sensors)
            out.sensor_xyz = a.inp(sensors)
            out.n_sensors = S
            traces, out.traces = a.out((nsteps, S))
        iters, out.iters = a.out((nsteps,), np.int32)
        relres, out.relres = a.out((nsteps,))
        sweeps, out.refine_sweeps = a.out((nsteps,), np.int32)
        out.first_step = first_step
        st = fem_heat_run(self.h, a.inp(T0), a.inp(T_prev), dt, theta, nsteps, rtol, out)
        if check and st not in (FEM_OK, FEM_ENOCONV):
            raise FemError(st, fem_last_error(self.h))
        return dict(status=st, T_final=T_final, T_saved=T_saved, traces=traces, iters=iters, relres=relres,
                    refine_sweeps=sweeps, total_iters=int(out.total_iters), device_ms=float(out.device_ms))

    def apply(self, which, x=None, *, dt, theta, fp32=False, elementwise=False, rowwave=False):
        a = _Arrays(self.device_ptrs)
        y, yp = a.out((self.N,))
        if x is None:
            x = np.zeros(self.N) if not self.device_ptrs else __import__("torch").zeros(self.N, dtype=__import__("torch").float64, device="cuda")
        which = (which | (FEM_OP_FP32 if fp32 else 0) | (FEM_OP_ELEMENTWISE if elementwise else 0)
                 | (FEM_OP_ROWWAVE if rowwave else 0))
        st = fem_heat_apply(self.h, which, dt, theta, a.inp(x), yp)
        if st != FEM_OK:
            raise FemError(st, fem_last_error(self.h))
        return y

    def tune(self, *, dt, theta, batch=False) -> dict:
        """fem_heat_tune: installs (or, with batch=True, records) the fastest gather tile."""
        st, r = fem_heat_tune(self.h, dt, theta, FEM_TUNE_BATCH if batch else 0)
        if st != FEM_OK:
            raise FemError(st, fem_last_error(self.h))
        return {k: getattr(r, k) for k, _ in fem_tune_result._fields_}

    def stats(self) -> dict:
        s = fem_heat_stats(self.h)
        return {k: getattr(s, k) for k, _ in fem_stats._fields_}

    def close(self):
        if self.h:
            fem_heat_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
