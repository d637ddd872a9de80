"""GPU parity of the gather apply and the setup kernels against the CPU oracle.

Operators: A = M + theta*dt*K and L = M - (1-theta)*dt*K applied by the
node-centred gather (FP64 and FP32), the Jacobi preconditioner and the load
vector.  Bounds: |y - A x| <= rel * (|A||x|) elementwise with rel = 1e-13
in FP64 (27 products per row, each rounded once) and 2e-6 in FP32 (inputs
and coefficients rounded to FP32: ~3 * 2^-24 per term).
"""
import numpy as np
import pytest

from _util import assert_apply_close, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASES = [
    ("1x1x1", (1, 1, 1), {}),
    ("3x5x7", (3, 5, 7), {}),
    ("noncubic_6x5x4", (6, 5, 4), dict(hx=0.11, hy=0.23, hz=0.07)),
    ("cube16", (16, 16, 16), {}),
    ("ragged_70x33x21", (70, 33, 21), dict(zero_k_fraction=0.2)),
    ("noncubic_65x9x30", (65, 9, 30), dict(hx=0.02, hy=0.05, hz=0.03)),
]


@pytest.mark.parametrize("name,dims,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("theta,dt", [(1.0, 1e-3), (0.5, 5e-4), (0.0, 2e-3)])
def test_gather_apply_matches_oracle(gpu, name, dims, kw, theta, dt):
    say(f"apply case {name} theta={theta} dt={dt}")
    prob = wl.random_problem(*dims, seed=sum(dims), **kw)
    x = wl.random_vector(prob.n_nodes, 7)
    with fh.Heat.from_problem(prob) as h:
        yA = h.apply(fh.FEM_OP_A, x, dt=dt, theta=theta)
        yL = h.apply(fh.FEM_OP_L, x, dt=dt, theta=theta)
        yA32 = h.apply(fh.FEM_OP_A, x, dt=dt, theta=theta, fp32=True)
    assert_apply_close(yA, prob, 1.0, theta * dt, x, 1e-13)
    assert_apply_close(yL, prob, 1.0, -(1 - theta) * dt, x, 1e-13)
    assert_apply_close(yA32, prob, 1.0, theta * dt, x, 2e-6)


def test_gather_matches_brute_force_element_loop(gpu):
    prob = wl.random_problem(5, 4, 3, seed=3, hx=0.3, hy=0.2, hz=0.45)
    x = wl.random_vector(prob.n_nodes, 1)
    with fh.Heat.from_problem(prob) as h:
        y = h.apply(fh.FEM_OP_A, x, dt=0.1, theta=0.7)
    ref = oracle.element_loop(prob, 1.0, 0.07, x)
    np.testing.assert_allclose(y, ref, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("tile", [(0, 0, 1), (0, 0, 3), (16, 4, 7), (7, 3, 64), (64, 4, 2)])
def test_tile_shapes_give_identical_bits(gpu, tile):
    say(f"tile {tile}")
    prob = wl.random_problem(40, 23, 17, seed=5)
    x = wl.random_vector(prob.n_nodes, 2)
    with fh.Heat.from_problem(prob) as h0, fh.Heat.from_problem(prob, tile=tile) as h1:
        a = h0.apply(fh.FEM_OP_A, x, dt=1e-3, theta=1.0)
        b = h1.apply(fh.FEM_OP_A, x, dt=1e-3, theta=1.0)
    assert np.array_equal(a, b)


def test_jacobi_and_load_vector(gpu):
    prob = wl.random_problem(9, 7, 5, seed=4, hx=0.1, hy=0.12, hz=0.2,
                             dirichlet_mask=(1 << wl.FACE_ZM) | (1 << wl.FACE_XM),
                             flux_mask=(1 << wl.FACE_ZP) | (1 << wl.FACE_YP),
                             flux=[0, 0, 0, 0.5, 0, 2.0])
    x = wl.random_vector(prob.n_nodes, 3)
    theta, dt = 0.5, 2e-3
    with fh.Heat.from_problem(prob) as h:
        yj = h.apply(fh.FEM_OP_JACOBI, x, dt=dt, theta=theta)
        yj32 = h.apply(fh.FEM_OP_JACOBI, x, dt=dt, theta=theta, fp32=True)
        F = h.apply(fh.FEM_OP_LOAD, dt=dt, theta=theta)
    A = oracle.CSR(prob, 1.0, theta * dt)
    rowptr, col, val = A.to_arrays()
    diag = np.array([val[rowptr[i]:rowptr[i + 1]][col[rowptr[i]:rowptr[i + 1]] == i][0] for i in range(prob.n_nodes)])
    d, _ = oracle.dirichlet(prob)
    ref = np.where(d, 0.0, x / diag)
    np.testing.assert_allclose(yj, ref, rtol=1e-14, atol=0)
    np.testing.assert_allclose(yj32, ref, rtol=2e-7, atol=1e-30)
    np.testing.assert_allclose(F, oracle.load_vector(prob), rtol=1e-14, atol=1e-18)


def test_full_size_apply_100cubed(gpu):
    """The operator at the 1,030,301-node log-normal workload, in the launch
    shape the benchmark uses."""
    say("apply full size lognormal100")
    prob = wl.lognormal_cube()
    x = wl.random_vector(prob.n_nodes, 9)
    with fh.Heat.from_problem(prob) as h:
        y = h.apply(fh.FEM_OP_A, x, dt=prob.dt, theta=prob.theta)
        y32 = h.apply(fh.FEM_OP_A, x, dt=prob.dt, theta=prob.theta, fp32=True)
    assert_apply_close(y, prob, 1.0, prob.theta * prob.dt, x, 1e-13)
    assert_apply_close(y32, prob, 1.0, prob.theta * prob.dt, x, 2e-6)


def test_device_pointer_apply(gpu):
    import torch
    prob = wl.random_problem(12, 11, 10, seed=6)
    x = wl.random_vector(prob.n_nodes, 4)
    with fh.Heat.from_problem(prob) as hh:
        ref = hh.apply(fh.FEM_OP_A, x, dt=1e-3, theta=1.0)
    kd = torch.tensor(prob.k_e, device="cuda")
    rd = torch.tensor(prob.rhoc_e, device="cuda")
    h = fh.Heat(prob.nx, prob.ny, prob.nz, prob.hx, prob.hy, prob.hz, kd, rd,
                dirichlet_mask=prob.dirichlet_mask, device_ptrs=True)
    try:
        y = h.apply(fh.FEM_OP_A, torch.tensor(x, device="cuda"), dt=1e-3, theta=1.0)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), ref)
    finally:
        h.close()


# ---- comparison forms of the apply, kept beside the gather: element by element in two passes
# (FEM_OP_ELEMENTWISE) and node-centred with one wavefront per node row (FEM_OP_ROWWAVE) ----

FORMS = ["elementwise", "rowwave"]

EBE_CASES = CASES + [
    ("seg_61x3x2", (61, 3, 2), {}),
    ("seg_62x2x3", (62, 2, 3), {}),
    ("seg_63x3x2", (63, 3, 2), {}),
    ("seg_124x2x2", (124, 2, 2), {}),
    ("seg_125x4x3", (125, 4, 3), dict(hx=0.01, hy=0.02, hz=0.015)),
]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name,dims,kw", EBE_CASES, ids=[c[0] for c in EBE_CASES])
@pytest.mark.parametrize("theta,dt", [(1.0, 1e-3), (0.5, 5e-4)])
def test_comparison_forms_match_oracle(gpu, form, name, dims, kw, theta, dt):
    """Both operators by each comparison form, against the oracle's assembled
    product to the same FP64 bound as the gather, across x-segment boundaries
    (62 nodes per wavefront) and ragged and non-cubic grids."""
    say(f"{form} apply case {name} theta={theta} dt={dt}")
    prob = wl.random_problem(*dims, seed=sum(dims), **kw)
    x = wl.random_vector(prob.n_nodes, 11)
    f = {form: True}
    with fh.Heat.from_problem(prob) as h:
        yA = h.apply(fh.FEM_OP_A, x, dt=dt, theta=theta, **f)
        yL = h.apply(fh.FEM_OP_L, x, dt=dt, theta=theta, **f)
        gA = h.apply(fh.FEM_OP_A, x, dt=dt, theta=theta)
    assert_apply_close(yA, prob, 1.0, theta * dt, x, 1e-13)
    assert_apply_close(yL, prob, 1.0, -(1 - theta) * dt, x, 1e-13)
    np.testing.assert_allclose(yA, gA, rtol=0, atol=1e-13 * np.abs(gA).max())


@pytest.mark.parametrize("form", FORMS)
def test_comparison_forms_match_brute_force_element_loop(gpu, form):
    prob = wl.random_problem(7, 4, 3, seed=8, hx=0.3, hy=0.2, hz=0.45)
    x = wl.random_vector(prob.n_nodes, 3)
    with fh.Heat.from_problem(prob) as h:
        y = h.apply(fh.FEM_OP_A, x, dt=0.1, theta=0.7, **{form: True})
    ref = oracle.element_loop(prob, 1.0, 0.07, x)
    np.testing.assert_allclose(y, ref, atol=1e-13 * np.abs(ref).max())


def test_comparison_forms_full_size_100cubed_and_timing(gpu):
    """The 1,030,301-node log-normal operator in all three forms, with the
    apply timing of FEM_TIMING handles (one event pair per call)."""
    prob = wl.lognormal_cube()
    x = wl.random_vector(prob.n_nodes, 9)
    with fh.Heat.from_problem(prob, timing=True) as h:
        ys = [h.apply(fh.FEM_OP_A, x, dt=prob.dt, theta=prob.theta, **{f: True}) for f in FORMS]
        g = h.apply(fh.FEM_OP_A, x, dt=prob.dt, theta=prob.theta)
        st = h.stats()
    for y in ys:
        assert_apply_close(y, prob, 1.0, prob.theta * prob.dt, x, 1e-13)
        np.testing.assert_allclose(y, g, rtol=0, atol=1e-13 * np.abs(g).max())
    assert st["apply_calls"] == 3 and st["apply_ms"] > 0


def test_comparison_forms_reject_fp32_other_operators_and_both_flags(gpu):
    prob = wl.random_problem(4, 4, 4, seed=2)
    x = wl.random_vector(prob.n_nodes, 1)
    with fh.Heat.from_problem(prob) as h:
        for form in FORMS:
            for which, fp32 in ((fh.FEM_OP_A, True), (fh.FEM_OP_JACOBI, False), (fh.FEM_OP_LOAD, False)):
                with pytest.raises(fh.FemError):
                    h.apply(which, x, dt=1e-3, theta=1.0, fp32=fp32, **{form: True})
        with pytest.raises(fh.FemError):
            h.apply(fh.FEM_OP_A, x, dt=1e-3, theta=1.0, elementwise=True, rowwave=True)
        st = h.stats()
    assert st["apply_calls"] == 0  # a handle without FEM_TIMING keeps no apply times
