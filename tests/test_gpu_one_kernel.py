"""The one-kernel PCG iteration of fem_heat_run (FEM_ONE_KERNEL,
dirupd_kernel): the direction gather, a grid-wide barrier and the x/r update
in one launch, q, r and P^-1 at the own nodes kept in LDS.

Its arithmetic is that of the two kernels except that r^T P^-1 r is summed
per gather block, so it is held to the same gates: the FP64 oracle locked to
its own iteration counts (relative L2 1e-10, every step), counts within one
of the two-kernel form, the stop rule met; the mixed form (its FP32 inner
solves in one kernel) within 1e-5 of the free-running FP64 oracle.  The
statistics show that the one-kernel path ran, and a second run repeats the
first bit for bit.
"""
import numpy as np
import pytest

from _util import rel_l2, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu


def problems():
    return [
        wl.random_problem(13, 9, 11, seed=61, nsteps=5, rtol=1e-10),
        wl.random_problem(20, 7, 5, seed=62, nsteps=4, theta=0.5, rtol=1e-9, flux_mask=1 << wl.FACE_ZP,
                          flux=[0, 0, 0, 0, 0, 2.0]),
        wl.random_problem(9, 12, 8, seed=63, nsteps=5, hx=0.05, hy=0.08, hz=0.03, rtol=1e-10),
        wl.random_problem(17, 15, 16, seed=64, nsteps=4, dt=2e-3, rtol=1e-11,
                          dirichlet_mask=(1 << wl.FACE_ZM) | (1 << wl.FACE_XP),
                          dirichlet_value=[0, 1.5, 0, 0, -0.5, 0]),
        wl.two_phase_sphere_cube().replace(nsteps=6),
        # the paper's element (six tetrahedra per box)
        wl.random_problem(12, 10, 14, seed=65, nsteps=4, rtol=1e-10).replace(element=fh.FEM_ELEM_TET6),
    ]


def _run(p, one_kernel=True, **kw):
    with fh.Heat.from_problem(p, timing=True, one_kernel=one_kernel, **kw) as h:
        out = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol, save_every=1)
        st = h.stats()
    return out, st


@pytest.mark.parametrize("replace_every", [50, 4])
def test_fp64_one_kernel_matches_locked_oracle(gpu, replace_every):
    for p in problems():
        one, st = _run(p, replace_every=replace_every)
        two, st2 = _run(p, replace_every=replace_every, one_kernel=False)
        ref = oracle.run(p, save_every=1, locked_iters=one["iters"], replace_every=replace_every)
        err = max(rel_l2(one["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps))
        say(f"  {p.name} R={replace_every}: iters {list(one['iters'])} (two kernels {list(two['iters'])}), "
            f"one-kernel samples {st['one_kernel_launches']}/{st['gather_launches']}, rel L2 {err:.2e}")
        assert one["status"] == fh.FEM_OK and err <= 1e-10
        assert np.all(one["relres"] <= p.rtol)
        assert np.abs(one["iters"].astype(int) - two["iters"].astype(int)).max() <= 1
        assert st2["one_kernel_launches"] == 0


def test_fp64_one_kernel_repeats_bit_for_bit(gpu):
    p = problems()[3]
    a, _ = _run(p)
    b, _ = _run(p)
    assert np.array_equal(a["T_final"], b["T_final"]) and np.array_equal(a["iters"], b["iters"])


def test_mixed_one_kernel_inner_solves_match_fp64_oracle(gpu):
    for p in problems():
        one, st = _run(p, precision=fh.FEM_FP32_FP64DOT)
        ref = oracle.run(p, save_every=1)
        err = max(rel_l2(one["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps))
        say(f"  {p.name} mixed: inner iters {list(one['iters'])}, rel L2 vs FP64 oracle {err:.2e}")
        assert one["status"] == fh.FEM_OK and err <= 1e-5
        assert np.all(one["relres"] <= p.rtol)


def test_headline_grid_first_steps_locked(gpu):
    p = wl.lognormal_cube(nsteps=3)
    out, st = _run(p)
    ref = oracle.run(p, save_every=1, locked_iters=out["iters"], nthreads=16)
    errs = [rel_l2(out["T_saved"][n], ref["T_saved"][n]) for n in range(3)]
    say(f"  lognormal100: iters {list(out['iters'])}, one-kernel samples {st['one_kernel_launches']}, rel L2 {errs}")
    assert out["status"] == fh.FEM_OK and max(errs) <= 1e-10 and st["one_kernel_launches"] > 0
    mixed, _ = _run(p, precision=fh.FEM_FP32_FP64DOT)
    free = oracle.run(p, save_every=1, nthreads=16)
    assert max(rel_l2(mixed["T_saved"][n], free["T_saved"][n]) for n in range(3)) <= 1e-5


def test_barrier_timeout_fails_the_run_and_the_handle_recovers(gpu, monkeypatch):
    """A grid-barrier wait made to give up at once (a spin limit of 0 set from
    the host): every kernel still exits, the run stops with FEM_EDEVICE at
    the end of its first chunk instead of iterating on void results, and
    the next run on the same handle, with the normal limit, matches the
    two-kernel form."""
    p = problems()[3]
    two, _ = _run(p, one_kernel=False)
    with fh.Heat.from_problem(p, one_kernel=True) as h:
        monkeypatch.setenv("FEMHEAT_BARRIER_SPIN_LIMIT", "0")
        bad = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol, check=False)
        assert bad["status"] == fh.FEM_EDEVICE
        assert "barrier" in fh.fem_last_error(h.h)
        monkeypatch.delenv("FEMHEAT_BARRIER_SPIN_LIMIT")
        good = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
    assert good["status"] == fh.FEM_OK
    assert np.abs(good["iters"].astype(int) - two["iters"].astype(int)).max() <= 1
    assert rel_l2(good["T_final"], two["T_final"]) <= 1e-10
