"""GPU parity of the paper's element (six linear tetrahedra per box, Sec. 4.1).

The gather applies the tetrahedra's box matrices from their closed-form
integer tables; the oracle integrates the tetrahedra by quadrature and
assembles a CSR matrix.  Gates as for the hexahedra: operator entries within
1e-13 of |A||x| (FP64), whole runs within 1e-10 of the iteration-locked
oracle, the mixed form within 1e-5, batches bit-identical alone and mixed,
results independent of the tile (both march directions of the z-chunks
meet every node).
"""
import numpy as np
import pytest

from _util import assert_apply_close, rel_l2, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu


def tet(nx, ny, nz, seed, **kw):
    return wl.random_problem(nx, ny, nz, seed, **kw).replace(element=fh.FEM_ELEM_TET6)


@pytest.mark.parametrize("dims", [(1, 1, 1), (13, 9, 11), (70, 5, 33)])
@pytest.mark.parametrize("op", [fh.FEM_OP_A, fh.FEM_OP_L])
def test_tet_operator_against_oracle(gpu, dims, op):
    say(f"tet apply {dims} op {op}")
    p = tet(*dims, seed=11, theta=0.5, dt=3e-3, k_range=(0.01, 100.0))
    x = wl.random_vector(p.n_nodes, 12)
    with fh.Heat.from_problem(p) as h:
        y = h.apply(op, x, dt=p.dt, theta=p.theta)
        y32 = h.apply(op, x, dt=p.dt, theta=p.theta, fp32=True)
    ck = p.theta * p.dt if op == fh.FEM_OP_A else -(1 - p.theta) * p.dt
    assert_apply_close(y, p, 1.0, ck, x, 1e-13)
    assert_apply_close(y32, p, 1.0, ck, x, 2e-6)


@pytest.mark.parametrize("tile", [(0, 0, 1), (0, 0, 3), (16, 4, 7), (7, 3, 64)])
def test_tet_tile_shapes_give_identical_bits(gpu, tile):
    p = tet(40, 23, 37, seed=13, theta=0.5, dt=1e-3)
    x = wl.random_vector(p.n_nodes, 14)
    with fh.Heat.from_problem(p) as h0, fh.Heat.from_problem(p, tile=tile) as h1:
        assert np.array_equal(h0.apply(fh.FEM_OP_A, x, dt=p.dt, theta=p.theta),
                              h1.apply(fh.FEM_OP_A, x, dt=p.dt, theta=p.theta))


def test_tet_jacobi_and_load_vector(gpu):
    p = tet(9, 7, 8, seed=15, theta=1.0, dt=2e-3, dirichlet_mask=1 << wl.FACE_ZM,
            flux_mask=(1 << wl.FACE_ZP) | (1 << wl.FACE_XM), flux=[0.7, 0, 0, 0, 0, 1.3])
    x = wl.random_vector(p.n_nodes, 16)
    with fh.Heat.from_problem(p) as h:
        jx = h.apply(fh.FEM_OP_JACOBI, x, dt=p.dt, theta=p.theta)
        F = h.apply(fh.FEM_OP_LOAD, dt=p.dt, theta=p.theta)
    A = oracle.CSR(p, 1.0, p.theta * p.dt)
    P = A.diagonal()
    d, _ = oracle.dirichlet(p)
    ref = np.where(d, 0.0, x / P)
    np.testing.assert_allclose(jx, ref, rtol=1e-14, atol=0)
    np.testing.assert_allclose(F, oracle.load_vector(p), rtol=1e-14, atol=1e-18)


@pytest.mark.parametrize("name,kw", [
    ("be_dirichlet", dict(theta=1.0)),
    ("cn_flux_neumann", dict(theta=0.5, dirichlet_mask=0, flux_mask=1 << wl.FACE_ZP, flux=[0, 0, 0, 0, 0, 3.0])),
    ("nonzero_dirichlet", dict(dirichlet_mask=(1 << wl.FACE_ZM) | (1 << wl.FACE_XP),
                               dirichlet_value=[0, 1.5, 0, 0, -0.5, 0])),
])
def test_tet_runs_locked_parity(gpu, name, kw):
    say(f"tet run {name}")
    base = dict(seed=17, nsteps=6, rtol=1e-10, dt=5e-3)
    base.update(kw)
    p = tet(13, 9, 11, **base)
    sens = np.array([[0.3, 0.2, 0.4], [0.11, 0.37, 0.05], [0.6, 0.1, 0.52]]) * np.array([1.0, 9 / 13, 11 / 13])
    with fh.Heat.from_problem(p) as h:
        out = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol, save_every=1, sensors=sens)
    ref = oracle.run(p, save_every=1, locked_iters=out["iters"], sensor_xyz=sens)
    assert out["status"] == 0 and ref["status"] == 0
    for n in range(p.nsteps):
        assert rel_l2(out["T_saved"][n], ref["T_saved"][n]) <= 1e-10
    assert rel_l2(out["traces"], ref["traces"]) <= 1e-10
    free = oracle.run(p)
    assert np.abs(out["iters"].astype(int) - free["iters"].astype(int)).max() <= 1


def test_tet_mixed_and_batch(gpu):
    probs = [tet(10 + i, 8, 9, seed=20 + i, nsteps=4, rtol=1e-8, dt=5e-3) for i in range(3)]
    st, mix = fh.run_batch(probs, precision=fh.FEM_FP32_FP64DOT)
    assert st == fh.FEM_OK
    for p, r in zip(probs, mix):
        _, alone = fh.run_batch([p], precision=fh.FEM_FP32_FP64DOT)
        assert np.array_equal(alone[0]["T_final"], r["T_final"])
        ref = oracle.run(p)
        assert rel_l2(r["T_final"], ref["T_final"]) <= 1e-5
    st, fp64 = fh.run_batch(probs)
    for p, r in zip(probs, fp64):
        ref = oracle.run(p, locked_iters=r["iters"])
        assert rel_l2(r["T_final"], ref["T_final"]) <= 1e-10


def test_tet_laminate_paper_workload(gpu):
    """The paper's laminate at its smallest mesh (30 x 30 x 10 cubes, 10,571
    nodes, six tetrahedra per cube), 50 Crank-Nicolson steps: FP64 run
    locked to the oracle, and iteration totals equal to the free oracle's."""
    p = wl.laminate(30)
    with fh.Heat.from_problem(p) as h:
        out = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
    ref = oracle.run(p, locked_iters=out["iters"], nthreads=8)
    free = oracle.run(p, nthreads=8)
    say(f"  laminate30 tet: {int(out['iters'].sum())} iterations over 50 steps (oracle {int(free['iters'].sum())})")
    assert rel_l2(out["T_final"], ref["T_final"]) <= 1e-10
    assert abs(int(out["iters"].sum()) - int(free["iters"].sum())) <= 5


def test_tet_rejections(gpu):
    p = tet(4, 4, 4, seed=3)
    with pytest.raises(fh.FemError):
        fh.Heat.from_problem(p.replace(hz=0.3))
    with pytest.raises(fh.FemError):
        fh.Heat.from_problem(p, precond=fh.FEM_PRECOND_CHEBYSHEV)
    with fh.Heat.from_problem(p) as h:
        with pytest.raises(fh.FemError):
            h.apply(fh.FEM_OP_A, np.zeros(p.n_nodes), dt=1e-3, theta=1.0, elementwise=True)
