"""GPU parity of the mixed-precision form against the FP64 CPU oracle.

The mixed form runs the inner PCG with FP32 operator, vectors and
preconditioner (dot products and alpha/beta/delta in FP64) and corrects the
FP64 field by iterative refinement until the FP64 stop rule holds.  Gate:
relative L2 error <= 1e-5 against the oracle's FP64 field (both stop at the
same relative residual; the error is then ~ condition * rtol, far below the
gate).  The relative residual each step reports is checked against rtol, and
the per-step error is recorded.
"""
import numpy as np
import pytest

from _util import rel_l2, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu

GATE = 1e-5


def run_mixed(p, nsteps=None, save_every=1, sensors=None, **kw):
    nsteps = p.nsteps if nsteps is None else nsteps
    with fh.Heat.from_problem(p, precision=fh.FEM_FP32_FP64DOT, **kw) as h:
        return h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=nsteps, rtol=p.rtol, save_every=save_every,
                     sensors=sensors)


def test_mixed_sphere_cube(gpu):
    say("mixed sphere16")
    p = wl.two_phase_sphere_cube().replace(rtol=1e-8)
    out = run_mixed(p)
    ref = oracle.run(p, save_every=1)
    assert out["status"] == 0
    errs = [rel_l2(out["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)]
    say(f"  per-step rel L2 vs FP64 oracle: max {max(errs):.2e}; sweeps {list(out['refine_sweeps'])}")
    assert max(errs) <= GATE
    assert np.all(out["relres"] <= p.rtol)
    assert np.all(out["refine_sweeps"] >= 1)
    d, g = oracle.dirichlet(p)
    assert np.all(out["T_final"][d] == g[d])


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_mixed_lognormal_and_flux(gpu, theta):
    say(f"mixed lognormal40 theta={theta}")
    p = wl.lognormal_cube(40, seed=7, nsteps=6).replace(theta=theta, dt=1e-3)
    out = run_mixed(p)
    ref = oracle.run(p, save_every=1, nthreads=4)
    errs = [rel_l2(out["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)]
    say(f"  per-step rel L2: {['%.1e' % e for e in errs]}")
    assert out["status"] == 0 and max(errs) <= GATE
    assert np.all(out["relres"] <= p.rtol)


def test_mixed_energy_balance_pure_neumann(gpu):
    q = 1.3
    p = wl.random_problem(12, 10, 8, seed=5, theta=1.0, dt=1e-2, nsteps=5, rtol=1e-12, dirichlet_mask=0,
                          flux_mask=1 << wl.FACE_ZP, flux=[0, 0, 0, 0, 0, q])
    out = run_mixed(p)

    def energy(T):
        T3 = T.reshape(p.nz + 1, p.ny + 1, p.nx + 1)
        c = sum(T3[a:a + p.nz, b:b + p.ny, cc:cc + p.nx] for a in (0, 1) for b in (0, 1) for cc in (0, 1)) / 8
        return float((p.rhoc_e.reshape(p.nz, p.ny, p.nx) * c).sum() * p.hx * p.hy * p.hz)

    area = p.nx * p.hx * p.ny * p.hy
    E0 = energy(p.T0)
    for n in range(p.nsteps):
        assert abs(energy(out["T_saved"][n]) - (E0 + (n + 1) * p.dt * q * area)) < 1e-9


def test_mixed_slab_sensors(gpu):
    say("mixed small defect slab with sensors")
    p = wl.defect_slab(40, 40, 5, seed=3, n_defects=4, nsteps=12, pulse_steps=4, n_sensor=8)
    out = run_mixed(p, sensors=p.sensors)
    ref = oracle.run(p, save_every=1)
    assert rel_l2(out["traces"], ref["traces"]) <= GATE
    errs = [rel_l2(out["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)]
    assert max(errs) <= GATE


def test_mixed_full_size_slab_first_steps(gpu):
    """The 200x200x25 defect slab (1,050,426 nodes, stiff: contrast 500) in
    the mixed form: the first 3 steps against the FP64 oracle, per step."""
    say("mixed full-size slab, 3 steps")
    p = wl.defect_slab()
    out = run_mixed(p, nsteps=3, sensors=p.sensors)
    ref = oracle.run(p, nsteps=3, save_every=1, sensor_xyz=p.sensors, nthreads=8)
    errs = [rel_l2(out["T_saved"][n], ref["T_saved"][n]) for n in range(3)]
    say(f"  iters {list(out['iters'])} sweeps {list(out['refine_sweeps'])} per-step rel L2 {['%.1e' % e for e in errs]}")
    assert max(errs) <= GATE
    assert rel_l2(out["traces"], ref["traces"][:3]) <= GATE
