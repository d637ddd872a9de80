"""fem_heat_apply_noalloc: the operator apply for callers that cannot
allocate, with the library's static per-GPU scratch.

Checked against fem_heat_apply (the entry point it is a variant of) through
the C-ABI: the same kernels in the same order, so bit-identical results, for
the node-centred gather and the element-by-element form (the one that uses
the 4 N partial sums of the scratch), on two calls in a row whose second has
a smaller grid (the scratch keeps the first call's contents), and again after
a larger grid's call.  Sizes beyond the scratch are rejected before any
device work.
"""
import numpy as np
import pytest
import torch

from _util import say
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _noalloc(h, which, x, dt, theta):
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.full_like(xd, float("nan"))
    torch.cuda.synchronize()
    st = fh.fem_heat_apply_noalloc(h.h, which, dt, theta, xd.data_ptr(), yd.data_ptr())
    assert st == fh.FEM_OK, fh.fem_last_error(h.h)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def _case(p, which, seed, dt=1e-3, theta=0.5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(p.n_nodes)
    with fh.Heat.from_problem(p) as h:
        want = h.apply(which & 0xff, x, dt=dt, theta=theta, elementwise=bool(which & fh.FEM_OP_ELEMENTWISE))
        got = _noalloc(h, which, x, dt, theta)
    return got, want


@pytest.mark.parametrize("form", [0, fh.FEM_OP_ELEMENTWISE])
@pytest.mark.parametrize("op", [fh.FEM_OP_A, fh.FEM_OP_L])
def test_noalloc_equals_apply_two_calls_second_smaller(gpu, op, form):
    big = wl.random_problem(37, 29, 23, seed=3)    # 38 x 30 x 24 nodes, ragged tiles
    small = wl.random_problem(11, 7, 5, seed=4, hx=0.1, hy=0.2, hz=0.15)
    for p, seed in ((big, 1), (small, 2)):
        got, want = _case(p, op | form, seed)
        say(f"noalloc op {op} form {form:#x} grid {p.nx}x{p.ny}x{p.nz}: max |diff| {np.abs(got - want).max():.1e}")
        assert np.array_equal(got, want)


def test_noalloc_headline_grid_and_after_it_a_small_one(gpu):
    p = wl.lognormal_cube()  # 101^3 nodes: within the element-by-element form's 2^20
    for which in (fh.FEM_OP_A | fh.FEM_OP_ELEMENTWISE, fh.FEM_OP_A):
        got, want = _case(p, which, 7, dt=p.dt, theta=p.theta)
        assert np.array_equal(got, want)
    got, want = _case(wl.two_phase_sphere_cube(), fh.FEM_OP_L | fh.FEM_OP_ELEMENTWISE, 8)
    assert np.array_equal(got, want)


def test_noalloc_rejects_beyond_the_scratch_and_other_operators(gpu):
    p = wl.random_problem(103, 101, 100, seed=5)  # 104*102*101 = 1,071,408 nodes > 2^20
    x = torch.zeros(p.n_nodes, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with fh.Heat.from_problem(p) as h:
        st = fh.fem_heat_apply_noalloc(h.h, fh.FEM_OP_A | fh.FEM_OP_ELEMENTWISE, 1e-3, 0.5, x.data_ptr(), y.data_ptr())
        assert st == fh.FEM_EINVAL and "2^20" in fh.fem_last_error(h.h)
        for bad in (fh.FEM_OP_JACOBI, fh.FEM_OP_A | fh.FEM_OP_FP32, fh.FEM_OP_A | fh.FEM_OP_ROWWAVE):
            assert fh.fem_heat_apply_noalloc(h.h, bad, 1e-3, 0.5, x.data_ptr(), y.data_ptr()) == fh.FEM_EINVAL
        assert fh.fem_heat_apply_noalloc(h.h, fh.FEM_OP_A, 1e-3, 0.5, None, y.data_ptr()) == fh.FEM_EINVAL
        # the gather form has no size limit: the same grid applies
        torch.cuda.synchronize()
        assert fh.fem_heat_apply_noalloc(h.h, fh.FEM_OP_A, 1e-3, 0.5, x.data_ptr(), y.data_ptr()) == fh.FEM_OK
        torch.cuda.synchronize()
        assert float(y.abs().max()) == 0.0
