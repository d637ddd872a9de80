"""GPU parity of whole theta-scheme runs (FP64 path) against the CPU oracle.

Gate: relative L2 error <= 1e-10 with the oracle run iteration-locked to the
GPU's per-step counts (both then perform the same arithmetic up to rounding
order).  Free-running iteration counts are compared too: they may differ by
one near the stopping threshold, since rounding decides that comparison.
"""
import numpy as np
import pytest

from _util import rel_l2, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu


def run_both(prob, *, nsteps=None, save_every=0, sensors=None, heat_kw=None, run_kw=None, oracle_kw=None):
    nsteps = prob.nsteps if nsteps is None else nsteps
    heat_kw = heat_kw or {}
    run_kw = run_kw or {}
    with fh.Heat.from_problem(prob, **heat_kw) as h:
        out = h.run(prob.T0, dt=prob.dt, theta=prob.theta, nsteps=nsteps, rtol=prob.rtol,
                    save_every=save_every, sensors=sensors, **run_kw)
    okw = dict(oracle_kw or {})
    for k in ("max_iter", "replace_every", "guess", "stop_rule"):
        if k in heat_kw:
            okw[k] = heat_kw[k]
    if "T_prev" in run_kw:
        okw["T_prev"] = run_kw["T_prev"]
    if "first_step" in run_kw:
        okw["first_step"] = run_kw["first_step"]
    ref = oracle.run(prob, nsteps=nsteps, save_every=save_every, sensor_xyz=sensors,
                     locked_iters=out["iters"], **okw)
    return out, ref


def test_sphere_cube_full_run(gpu):
    say("run sphere16 20 steps")
    p = wl.two_phase_sphere_cube()
    out, ref = run_both(p, save_every=1)
    assert out["status"] == 0 and ref["status"] == 0
    for n in range(p.nsteps):
        assert rel_l2(out["T_saved"][n], ref["T_saved"][n]) <= 1e-10
    assert rel_l2(out["T_final"], ref["T_final"]) <= 1e-10
    free = oracle.run(p)
    assert np.abs(out["iters"] - free["iters"]).max() <= 1
    assert np.all(out["relres"] <= p.rtol)


@pytest.mark.parametrize("name,kw,heat_kw", [
    ("be_dirichlet", dict(theta=1.0), {}),
    ("cn_flux", dict(theta=0.5, flux_mask=1 << wl.FACE_ZP, flux=[0, 0, 0, 0, 0, 3.0]), {}),
    ("explicit_theta0", dict(theta=0.0, dt=2e-5), {}),
    ("nonzero_dirichlet", dict(dirichlet_mask=(1 << wl.FACE_ZM) | (1 << wl.FACE_XP),
                               dirichlet_value=[0, 1.5, 0, 0, -0.5, 0]), {}),
    ("pure_neumann", dict(dirichlet_mask=0, flux_mask=1 << wl.FACE_YM, flux=[0, 0, 2.0, 0, 0, 0]), {}),
    ("guess_prev", {}, dict(guess=fh.FEM_GUESS_PREV)),
    ("stop_initial", {}, dict(stop_rule=fh.FEM_STOP_INITIAL)),
    ("replace_every_3", dict(rtol=1e-12), dict(replace_every=3)),
    ("no_replacement", {}, dict(replace_every=0)),
    ("zero_k_voids", dict(zero_k_fraction=0.4), {}),
    ("noncubic", dict(hx=0.05, hy=0.08, hz=0.03), {}),
])
def test_small_runs_locked_parity(gpu, name, kw, heat_kw):
    say(f"run case {name}")
    base = dict(seed=31, nsteps=6, rtol=1e-10)
    base.update(kw)
    p = wl.random_problem(13, 9, 11, **base)
    out, ref = run_both(p, save_every=2, heat_kw=heat_kw)
    assert out["status"] == 0 and ref["status"] == 0
    assert rel_l2(out["T_final"], ref["T_final"]) <= 1e-10
    for n in range(len(out["T_saved"])):
        assert rel_l2(out["T_saved"][n], ref["T_saved"][n]) <= 1e-10
    d, g = oracle.dirichlet(p)
    assert np.all(out["T_final"][d] == g[d])


def test_sensor_traces_and_flux_schedule(gpu):
    say("run sensors + schedule")
    p = wl.defect_slab(40, 40, 5, seed=3, n_defects=4, nsteps=12, pulse_steps=4, n_sensor=5)
    out, ref = run_both(p, sensors=p.sensors)
    assert rel_l2(out["traces"], ref["traces"]) <= 1e-10
    # independent: traces equal trilinear interpolation of the GPU's own field
    np.testing.assert_allclose(out["traces"][-1], oracle.sensors(p, out["T_final"], p.sensors), rtol=1e-13, atol=1e-15)


def test_energy_balance_on_gpu(gpu):
    """Pure Neumann: stored energy grows by exactly the injected heat (up to the
    CG residual), computed from the GPU fields alone."""
    q = 1.3
    p = wl.random_problem(12, 10, 8, seed=5, theta=1.0, dt=1e-2, nsteps=5, rtol=1e-12, dirichlet_mask=0,
                          flux_mask=1 << wl.FACE_ZP, flux=[0, 0, 0, 0, 0, q])
    with fh.Heat.from_problem(p) as h:
        out = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol, save_every=1)

    def energy(T):
        T3 = T.reshape(p.nz + 1, p.ny + 1, p.nx + 1)
        c = sum(T3[a:a + p.nz, b:b + p.ny, cc:cc + p.nx] for a in (0, 1) for b in (0, 1) for cc in (0, 1)) / 8
        return float((p.rhoc_e.reshape(p.nz, p.ny, p.nx) * c).sum() * p.hx * p.hy * p.hz)

    area = p.nx * p.hx * p.ny * p.hy
    E0 = energy(p.T0)
    for n in range(p.nsteps):
        assert abs(energy(out["T_saved"][n]) - (E0 + (n + 1) * p.dt * q * area)) < 1e-9


def test_resume_equals_uninterrupted(gpu):
    p = wl.random_problem(10, 8, 9, seed=7, nsteps=10, rtol=1e-9, theta=0.5, flux_mask=1 << wl.FACE_ZP,
                          flux=[0, 0, 0, 0, 0, 1.0]).replace(flux_schedule=np.linspace(1, 0, 10))
    with fh.Heat.from_problem(p) as h:
        full = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=10, rtol=p.rtol, save_every=1)
        a = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=6, rtol=p.rtol, save_every=1)
        b = h.run(a["T_saved"][5], T_prev=a["T_saved"][4], dt=p.dt, theta=p.theta, nsteps=4, rtol=p.rtol,
                  first_step=6)
    assert np.array_equal(full["T_final"], b["T_final"])
    assert list(full["iters"]) == list(a["iters"]) + list(b["iters"])


def test_deterministic_and_edge_cases(gpu):
    p = wl.random_problem(20, 7, 9, seed=8, nsteps=3)
    with fh.Heat.from_problem(p) as h:
        a = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=3, rtol=p.rtol)
        b = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=3, rtol=p.rtol)
        z = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=0, rtol=p.rtol)
        capped = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=2, rtol=p.rtol)
    assert np.array_equal(a["T_final"], b["T_final"]) and np.array_equal(a["iters"], b["iters"])
    d, g = oracle.dirichlet(p)
    assert np.array_equal(z["T_final"], np.where(d, g, p.T0)) and z["status"] == 0
    del capped
    with fh.Heat.from_problem(p, max_iter=1) as h:
        c = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=2, rtol=p.rtol)
    assert c["status"] == fh.FEM_ENOCONV and list(c["iters"]) == [1, 1]
    ref = oracle.run(p, nsteps=2, max_iter=1)
    assert ref["status"] == oracle.ENOCONV and rel_l2(c["T_final"], ref["T_final"]) <= 1e-10
    one = wl.random_problem(1, 1, 1, seed=2, nsteps=3, dirichlet_mask=0)
    out, ref1 = run_both(one)
    assert rel_l2(out["T_final"], ref1["T_final"]) <= 1e-10


def test_zero_rhs_gives_zero_field(gpu):
    p = wl.random_problem(6, 6, 6, seed=9, nsteps=2, random_T0=False).replace(T0=np.zeros(343))
    with fh.Heat.from_problem(p) as h:
        out = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=2, rtol=p.rtol)
    assert np.all(out["T_final"] == 0) and list(out["iters"]) == [0, 0]


def test_run_validation(gpu):
    p = wl.random_problem(3, 3, 3, seed=1)
    with fh.Heat.from_problem(p) as h:
        for kw in (dict(dt=0.0, theta=1.0), dict(dt=1e-3, theta=1.5), dict(dt=1e-3, theta=1.0, rtol=0.0)):
            args = dict(dt=kw["dt"], theta=kw["theta"], nsteps=1, rtol=kw.get("rtol", 1e-8), check=False)
            assert h.run(p.T0, **args)["status"] == fh.FEM_EINVAL
        bad = h.run(p.T0, dt=1e-3, theta=1.0, nsteps=1, rtol=1e-8, sensors=np.array([[2.0, 0, 0]]), check=False)
        assert bad["status"] == fh.FEM_EINVAL


def test_full_size_lognormal_first_steps(gpu):
    """The 1,030,301-node Crank-Nicolson workload in the benchmark's launch
    shape: the first 3 steps against the oracle (iteration-locked)."""
    say("run full size lognormal100, 3 steps")
    p = wl.lognormal_cube()
    out, ref = run_both(p, nsteps=3, oracle_kw=dict(nthreads=8))
    assert out["status"] == 0 and ref["status"] == 0
    err = rel_l2(out["T_final"], ref["T_final"])
    say(f"  iters {list(out['iters'])}, rel L2 {err:.3e}")
    assert err <= 1e-10


def test_above_cache_size_first_steps(gpu):
    """The largest grid the benchmark runs: the log-normal workload at 201^3
    nodes (8,120,601 DOF, beyond the 256 MB Infinity Cache), first 2 steps
    against the iteration-locked oracle, in the benchmark's launch shape."""
    say("run 201^3 lognormal, 2 steps")
    p = wl.lognormal_cube(200, seed=2, nsteps=2)
    out, ref = run_both(p, nsteps=2, oracle_kw=dict(nthreads=16))
    assert out["status"] == 0 and ref["status"] == 0
    err = rel_l2(out["T_final"], ref["T_final"])
    say(f"  iters {list(out['iters'])}, rel L2 {err:.3e}")
    assert err <= 1e-10


def test_timing_changes_nothing_and_samples(gpu):
    """FEM_TIMING records events around a sample of the iterations; the
    results are bit-identical to an untimed run."""
    p = wl.random_problem(14, 12, 10, seed=12, nsteps=4, rtol=1e-11)
    with fh.Heat.from_problem(p) as h:
        a = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
    with fh.Heat.from_problem(p, timing=True) as h:
        b = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
        st = h.stats()
    assert np.array_equal(a["T_final"], b["T_final"]) and np.array_equal(a["iters"], b["iters"])
    total = int(np.sum(b["iters"]))
    assert 0 < st["gather_launches"] < total and st["gather_ms"] > 0
    # iteration 0 of every step is a replacement; one in eight is timed, the first included
    assert 1 <= st["replace_launches"] <= p.nsteps
