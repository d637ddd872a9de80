"""The C-ABI library loads and exports every entry point declared in include/*.h.

CPU-only: no call here touches a GPU (only string/option helpers and argument
validation that fails before any device work).
"""

import glob
import os
import re

import numpy as np
import pytest

from paper_1905_07622_amd import femheat as fh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(fem_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fh.LIB_PATH):
        from paper_1905_07622_amd import build
        build.build()
    return fh.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fem_heat_create", "fem_heat_run", "fem_heat_apply", "fem_heat_destroy", "fem_strerror",
              "fem_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_default_opts(lib):
    for code in range(0, -8, -1):
        assert fh.fem_strerror(code)
    assert "unknown" in fh.fem_strerror(-99)
    o = fh.fem_heat_default_opts()
    assert (o.precision, o.max_iter, o.replace_every, o.guess, o.stop_rule, o.max_refine) == (0, 10000, 50, 0, 0, 4)
    assert abs(o.inner_rtol - 1e-5) < 1e-20


def _create(nx=2, ny=2, nz=2, h=0.5, k=None, rhoc=None, **bc_kw):
    E = nx * ny * nz
    k = np.ones(E) if k is None else k
    rhoc = np.ones(E) if rhoc is None else rhoc
    bc = fh.fem_bc()
    for key, v in bc_kw.items():
        setattr(bc, key, v)
    st, h_ = fh.fem_heat_create(fh.fem_grid(nx, ny, nz, h, h, h), k.ctypes.data_as(fh._dp),
                                rhoc.ctypes.data_as(fh._dp), bc, None)
    return st, h_, fh.fem_last_error(None)


@pytest.mark.parametrize("case", ["grid", "h", "k_neg", "k_nan", "rhoc_zero", "masks", "mask_bits"])
def test_create_rejects_invalid_arguments_before_device_work(lib, case):
    kw = {}
    if case == "grid":
        kw = dict(nx=0)
    elif case == "h":
        kw = dict(h=-1.0)
    elif case == "k_neg":
        kw = dict(k=np.array([1, 1, 1, -1, 1, 1, 1, 1.0]))
    elif case == "k_nan":
        kw = dict(k=np.array([1, 1, 1, np.nan, 1, 1, 1, 1.0]))
    elif case == "rhoc_zero":
        kw = dict(rhoc=np.array([1, 1, 0, 1, 1, 1, 1, 1.0]))
    elif case == "masks":
        kw = dict(dirichlet_mask=1 << 4, flux_mask=1 << 4)
    elif case == "mask_bits":
        kw = dict(flux_mask=1 << 6)
    st, h, msg = _create(**kw)
    assert st == fh.FEM_EINVAL and not h.value and msg


def test_null_handle_calls_are_rejected(lib):
    assert lib.fem_heat_run(None, None, None, 1.0, 1.0, 1, 1.0, None) == fh.FEM_EINVAL
    assert lib.fem_heat_apply(None, 0, 1.0, 1.0, None, None) == fh.FEM_EINVAL
    assert lib.fem_heat_apply_noalloc(None, 0, 1.0, 1.0, None, None) == fh.FEM_EINVAL
    lib.fem_heat_destroy(None)
    assert lib.fem_heat_stats(None, None) == fh.FEM_EINVAL



def _request(nx=2, ny=2, nz=2, dt=1e-3, theta=1.0, rtol=1e-8, nsteps=1, k=None, keep=None):
    from paper_1905_07622_amd import workloads as wl
    p = wl.random_problem(nx, ny, nz, seed=1, nsteps=nsteps, dt=dt, theta=theta, rtol=rtol)
    if k is not None:
        p = p.replace(k_e=k)
    return p


@pytest.mark.parametrize("case", ["dt", "theta", "rtol", "nsteps", "k_neg", "grid"])
def test_run_batch_rejects_invalid_requests_before_device_work(lib, case):
    """One invalid request makes the whole batch fail with FEM_EINVAL before
    anything runs; status[] names the request."""
    good = _request()
    bad = {"dt": dict(dt=0.0), "theta": dict(theta=1.5), "rtol": dict(rtol=-1.0), "nsteps": dict(nsteps=-1),
           "k_neg": dict(k=-np.ones(8)), "grid": {}}[case]
    if case == "grid":
        p = good.replace(nx=0)
    elif case == "nsteps":
        p = good.replace(nsteps=-1)
    else:
        p = _request(**bad)
    a = fh._Arrays(False)
    reqs = (fh.fem_request * 3)()
    for i, q in enumerate([good, p, good]):
        r = reqs[i]
        r.grid = fh.fem_grid(q.nx, q.ny, q.nz, q.hx, q.hy, q.hz)
        r.k_e = a.inp(q.k_e)
        r.rhoc_e = a.inp(q.rhoc_e)
        r.bc = fh._bc(q, a.keep)
        r.T0 = a.inp(q.T0)
        r.dt, r.theta, r.rtol, r.nsteps = q.dt, q.theta, q.rtol, q.nsteps
    status = np.full(3, 99, dtype=np.int32)
    st = fh.fem_heat_run_batch(reqs, 3, fh.make_opts(), status.ctypes.data_as(fh._ip))
    assert st == fh.FEM_EINVAL
    assert list(status) == [fh.FEM_OK, fh.FEM_EINVAL, fh.FEM_OK]
    assert fh.fem_last_error(None).startswith("request 1:")


def test_run_batch_argument_checks(lib):
    assert fh.fem_heat_run_batch(None, 1, None, None) == fh.FEM_EINVAL
    assert fh.fem_heat_run_batch(None, 0, None, None) == fh.FEM_OK
    reqs = (fh.fem_request * 1)()
    bad_opts = fh.make_opts(precision=7)
    assert fh.fem_heat_run_batch(reqs, 1, bad_opts, None) == fh.FEM_EINVAL
    assert fh.fem_heat_run_batch(reqs, 1, fh.make_opts(batch_groups=-1), None) == fh.FEM_EINVAL
    assert "batch_groups" in fh.fem_last_error(None)


STRUCTS = ("fem_grid", "fem_bc", "fem_opts", "fem_out", "fem_stats", "fem_tune_result", "fem_request",
           "fem_server_opts",
           "fem_status", "fem_server_info")


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every ctypes mirror of a header struct has the C compiler's size and
    field offsets (compiled with gcc against include/fem_heat.h)."""
    import ctypes
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fem_heat.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(fh, name)
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n") if l)
    for name in STRUCTS:
        cls = getattr(fh, name)
        assert int(got[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, f"{name}.{field}"


def test_server_rejects_invalid_options_before_device_work(lib):
    so = fh.fem_server_opts()
    so.opts = fh.make_opts(device_ptrs=True)
    st, s = fh.fem_server_create(so)
    assert st == fh.FEM_EINVAL and not s.value
    so.opts = fh.make_opts(precision=5)
    assert fh.fem_server_create(so)[0] == fh.FEM_EINVAL
    so.opts = fh.make_opts()
    so.max_slots = -1
    assert fh.fem_server_create(so)[0] == fh.FEM_EINVAL
    assert fh.fem_server_poll(None, 1)[0] == fh.FEM_EINVAL
    assert fh.fem_server_cancel(None, 1) == fh.FEM_EINVAL
    r = fh.fem_request()
    assert fh.fem_server_submit(None, r)[0] == fh.FEM_EINVAL


@pytest.mark.parametrize("tile", [(128, 2, 4), (1, 64, 4), (200, 0, 0), (0, 4, 0), (257, 1, 1), (64, 9, 1), (513, 1, 1)])
def test_create_rejects_tiles_the_gather_cannot_stage(lib, tile):
    """Tile overrides whose (tx+2)(ty+2) plane tile needs more than two staging
    slots per thread (or out of range) are refused before any device work."""
    k = np.ones(8)
    st, h = fh.fem_heat_create(fh.fem_grid(2, 2, 2, 0.5, 0.5, 0.5), k.ctypes.data_as(fh._dp),
                               k.ctypes.data_as(fh._dp), fh.fem_bc(), fh.make_opts(tile=tile))
    assert st == fh.FEM_EINVAL and not h.value
    assert "tile" in fh.fem_last_error(None)
