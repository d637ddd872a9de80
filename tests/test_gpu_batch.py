"""GPU parity of the batched form: many simulations in every kernel launch.

Every simulation of a batch is checked three ways:
  * against the FP64 CPU oracle, iteration-locked to the GPU's per-step
    counts, at the FP64 gate (relative L2 <= 1e-10) or the mixed-form gate
    (1e-5, free-running oracle);
  * against itself run alone (a batch of one): the results must be
    bit-identical, because a simulation's blocks, tiles and reductions do not
    depend on its co-runners;
  * for the FP64 form, against the single-handle path (fem_heat_run), which
    tiles the simulation differently: the same field to the FP64 gate.
The batches mix grid sizes, element shapes (cubic and not), boundary
conditions, dt, theta, tolerances and step counts, including a simulation
with no steps.
"""
import numpy as np
import pytest

from _util import rel_l2, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu

GATE64 = 1e-10
GATE_MIXED = 1e-5


def uneven_batch():
    return [
        wl.random_problem(13, 9, 11, seed=31, nsteps=6, rtol=1e-10),
        wl.random_problem(20, 7, 5, seed=32, nsteps=4, theta=0.5, rtol=1e-9, flux_mask=1 << wl.FACE_ZP,
                          flux=[0, 0, 0, 0, 0, 2.0]).replace(flux_schedule=np.array([1.0, 0.5, 0.0])),
        wl.random_problem(9, 12, 8, seed=33, nsteps=7, hx=0.05, hy=0.08, hz=0.03, rtol=1e-10),
        wl.random_problem(6, 6, 6, seed=34, nsteps=0),
        wl.random_problem(17, 15, 16, seed=35, nsteps=5, dt=2e-3, rtol=1e-11,
                          dirichlet_mask=(1 << wl.FACE_ZM) | (1 << wl.FACE_XP),
                          dirichlet_value=[0, 1.5, 0, 0, -0.5, 0]),
        wl.two_phase_sphere_cube().replace(nsteps=8),
        wl.random_problem(1, 1, 1, seed=36, nsteps=3, dirichlet_mask=0),
    ]


def locked_oracle(p, out, **kw):
    return oracle.run(p, save_every=1, locked_iters=out["iters"], **kw)


def same_bits(a, b):
    for key in ("T_final", "T_saved", "iters", "relres", "refine_sweeps"):
        if a[key] is None:
            assert b[key] is None
            continue
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key


def test_batch_fp64_matches_oracle_and_alone(gpu):
    probs = uneven_batch()
    say(f"batch fp64 of {len(probs)} uneven simulations")
    st, res = fh.run_batch(probs, save_every=1)
    assert st == fh.FEM_OK and all(r["status"] == 0 for r in res)
    for p, r in zip(probs, res):
        if p.nsteps == 0:
            d, g = oracle.dirichlet(p)
            assert np.array_equal(r["T_final"], np.where(d, g, p.T0))
            continue
        ref = locked_oracle(p, r)
        errs = [rel_l2(r["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)]
        say(f"  {p.name}: iters {list(r['iters'])} max rel L2 {max(errs):.2e}")
        assert max(errs) <= GATE64
        assert np.all(r["relres"] <= p.rtol)
        alone_st, alone = fh.run_batch([p], save_every=1)
        assert alone_st == fh.FEM_OK
        same_bits(r, alone[0])


def test_batch_matches_single_handle_path(gpu):
    probs = uneven_batch()[:3]
    st, res = fh.run_batch(probs, save_every=1)
    assert st == fh.FEM_OK
    for p, r in zip(probs, res):
        with fh.Heat.from_problem(p) as h:
            one = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol, save_every=1)
        assert rel_l2(r["T_final"], one["T_final"]) <= GATE64
        assert np.abs(np.asarray(r["iters"]) - np.asarray(one["iters"])).max() <= 1


def test_batch_mixed_matches_oracle_and_alone(gpu):
    probs = [p.replace(rtol=1e-8) for p in uneven_batch() if p.nsteps > 0][:5]
    say(f"batch mixed of {len(probs)}")
    st, res = fh.run_batch(probs, save_every=1, precision=fh.FEM_FP32_FP64DOT)
    assert st == fh.FEM_OK
    for p, r in zip(probs, res):
        ref = oracle.run(p, save_every=1)
        errs = [rel_l2(r["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)]
        say(f"  {p.name}: sweeps {list(r['refine_sweeps'])} max rel L2 vs FP64 oracle {max(errs):.2e}")
        assert max(errs) <= GATE_MIXED
        assert np.all(r["relres"] <= p.rtol)
        _, alone = fh.run_batch([p], save_every=1, precision=fh.FEM_FP32_FP64DOT)
        same_bits(r, alone[0])


@pytest.mark.parametrize("precision", [fh.FEM_FP64, fh.FEM_FP32_FP64DOT])
def test_batch_groups_change_no_bits(gpu, precision):
    """The same batch run as one, two, three or seven concurrent batches
    (fem_opts.batch_groups, each on its own stream and host thread): every
    simulation's outputs bit for bit the same, also with device pointers
    on a caller's stream."""
    import torch
    probs = uneven_batch()
    st, one = fh.run_batch(probs, save_every=1, precision=precision, batch_groups=1)
    assert st == fh.FEM_OK
    for g in (2, 3, 7):
        st, res = fh.run_batch(probs, save_every=1, precision=precision, batch_groups=g)
        assert st == fh.FEM_OK
        for a, b in zip(res, one):
            same_bits(a, b)
    stream = torch.cuda.Stream()
    dev_probs = [p.replace(k_e=torch.tensor(p.k_e, device="cuda"), rhoc_e=torch.tensor(p.rhoc_e, device="cuda"),
                           T0=torch.tensor(p.T0, device="cuda")) for p in probs]
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        st, dev = fh.run_batch(dev_probs, precision=precision, device_ptrs=True, stream=stream.cuda_stream,
                               batch_groups=3)
    stream.synchronize()
    assert st == fh.FEM_OK
    for a, b in zip(dev, one):
        assert np.array_equal(a["T_final"].cpu().numpy(), b["T_final"])
        assert np.array_equal(a["iters"].cpu().numpy() if hasattr(a["iters"], "cpu") else a["iters"], b["iters"])


def test_batch_groups_keep_statuses_per_simulation(gpu):
    easy = wl.random_problem(8, 8, 8, seed=41, nsteps=2, rtol=1e-6)
    hard = wl.random_problem(12, 12, 12, seed=42, nsteps=2, rtol=1e-30)  # below FP64 reach
    st, res = fh.run_batch([easy, hard, easy], max_iter=40, check=False, batch_groups=2)
    assert st == fh.FEM_ENOCONV
    assert [r["status"] for r in res] == [fh.FEM_OK, fh.FEM_ENOCONV, fh.FEM_OK]
    _, alone = fh.run_batch([easy], max_iter=40)
    same_bits(res[0], alone[0])
    same_bits(res[2], alone[0])


def test_batch_sensors_and_device_pointers(gpu):
    import torch
    probs = [wl.defect_slab(30, 24, 5, seed=3, n_defects=3, nsteps=6, pulse_steps=2, n_sensor=4),
             wl.defect_slab(20, 20, 4, seed=4, n_defects=2, nsteps=4, pulse_steps=3, n_sensor=3)]
    st, host = fh.run_batch(probs, sensors=True)
    assert st == fh.FEM_OK
    dev_probs = [p.replace(k_e=torch.tensor(p.k_e, device="cuda"), rhoc_e=torch.tensor(p.rhoc_e, device="cuda"),
                           T0=torch.tensor(p.T0, device="cuda"), sensors=torch.tensor(p.sensors, device="cuda"))
                 for p in probs]
    st2, dev = fh.run_batch(dev_probs, sensors=True, device_ptrs=True)
    assert st2 == fh.FEM_OK
    for p, h_, d_ in zip(probs, host, dev):
        ref = locked_oracle(p, h_, sensor_xyz=p.sensors)
        assert rel_l2(h_["traces"], ref["traces"]) <= GATE64
        assert np.array_equal(h_["traces"], d_["traces"].cpu().numpy())
        assert np.array_equal(h_["T_final"], d_["T_final"].cpu().numpy())


def test_batch_statuses_are_per_simulation(gpu):
    """A simulation that hits max_iter reports FEM_ENOCONV without disturbing
    the others; the call returns the first non-OK status."""
    easy = wl.random_problem(8, 8, 8, seed=41, nsteps=2, rtol=1e-6)
    hard = wl.random_problem(12, 12, 12, seed=42, nsteps=2, rtol=1e-30)  # below FP64 reach
    st, res = fh.run_batch([easy, hard], max_iter=40, check=False)
    say(f"  easy iters {list(res[0]['iters'])}, hard iters {list(res[1]['iters'])}")
    assert st == fh.FEM_ENOCONV
    assert res[0]["status"] == fh.FEM_OK and res[1]["status"] == fh.FEM_ENOCONV
    assert max(res[0]["iters"]) < 40 and list(res[1]["iters"]) == [40, 40]
    _, alone = fh.run_batch([easy], max_iter=40)
    same_bits(res[0], alone[0])
    ref = oracle.run(hard, nsteps=2, max_iter=40)
    assert rel_l2(res[1]["T_final"], ref["T_final"]) <= GATE64


def test_proposal_batch_sampled_parity(gpu):
    """The batched proposal workload shape (48^3 random-sphere fields,
    backward Euler, rtol 1e-8) with 16 simulations for 5 steps in the mixed
    form: three sampled simulations against the FP64 oracle."""
    probs = [wl.sphere_proposal(s, nsteps=5) for s in range(16)]
    say("proposal batch 16 x 48^3, 5 steps, mixed")
    st, res = fh.run_batch(probs, save_every=1, precision=fh.FEM_FP32_FP64DOT)
    assert st == fh.FEM_OK
    for s in (0, 7, 15):
        ref = oracle.run(probs[s], save_every=1, nthreads=4)
        errs = [rel_l2(res[s]["T_saved"][n], ref["T_saved"][n]) for n in range(5)]
        say(f"  sim {s}: iters {list(res[s]['iters'])} max rel L2 {max(errs):.2e}")
        assert max(errs) <= GATE_MIXED


@pytest.mark.parametrize("replace_every,rtol", [(50, 1e-10), (3, 1e-10), (4, 1e-9), (50, 0.5)])
def test_single_simulation_overlap_matches_batch(gpu, replace_every, rtol):
    """A simulation alone starts each step's RHS and initial residual behind
    the previous step's last decide, before the host has read it (and on the
    device only if the solve ended in the iterate buffer assumed); in a batch
    of two it does not.  Both must give the same bits -- also when the
    assumption fails (frequent replacements move the iterate between buffers)
    and when solves take zero or one iteration (loose tolerance)."""
    p = wl.random_problem(13, 9, 11, seed=31, nsteps=6, rtol=rtol)
    partner = wl.random_problem(6, 6, 6, seed=34, nsteps=6)
    _, alone = fh.run_batch([p], save_every=1, replace_every=replace_every)
    _, pair = fh.run_batch([p, partner], save_every=1, replace_every=replace_every)
    say(f"  R={replace_every} rtol={rtol}: iters {list(alone[0]['iters'])}")
    same_bits(alone[0], pair[0])
    with fh.Heat.from_problem(p, replace_every=replace_every) as h:
        one = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol, save_every=1)
    assert np.array_equal(one["iters"], alone[0]["iters"])
    ref = oracle.run(p, save_every=1, locked_iters=one["iters"], replace_every=replace_every)
    assert max(rel_l2(one["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)) <= GATE64


def test_mixed_early_sweep_start_matches_batch(gpu):
    """A simulation alone starts a refinement sweep behind the previous
    sweep's decide, before the host has read it, when its previous step ran
    more sweeps; a step that then needs fewer runs that sweep's inner solve
    idle and ends.  Flux pulses and random initial fields make the sweep
    count per step fall as well as rise.  Alone and in a batch of two (which
    never starts a sweep early) must give the same bits, and the fields must
    match the FP64 oracle."""
    kw = dict(save_every=1, precision=fh.FEM_FP32_FP64DOT, max_refine=6, inner_rtol=1e-3, check=False)
    falls = 0
    for seed, theta, dt, pulse in [(41, 1.0, 1e-3, 3), (42, 0.5, 5e-3, 2), (43, 1.0, 2e-2, 4)]:
        base = wl.random_problem(12, 10, 9, seed=seed, nsteps=9, rtol=1e-11, theta=theta, dt=dt)
        flux = np.zeros(6)
        flux[wl.FACE_ZP] = 50.0
        sched = np.zeros(base.nsteps)
        sched[:pulse] = 1.0
        p = base.replace(flux_mask=wl.face_bit(wl.FACE_ZP), flux=flux, flux_schedule=sched)
        partner = wl.random_problem(6, 6, 6, seed=seed + 100, nsteps=9)
        _, alone = fh.run_batch([p], **kw)
        _, pair = fh.run_batch([p, partner], **kw)
        sw = np.asarray(alone[0]["refine_sweeps"])
        say(f"  seed {seed}: sweeps {list(sw)} iters {list(alone[0]['iters'])} status {alone[0]['status']}")
        assert alone[0]["status"] == fh.FEM_OK == pair[0]["status"]
        same_bits(alone[0], pair[0])
        falls += int(np.sum(np.diff(sw) < 0))
        ref = oracle.run(p, save_every=1)
        assert max(rel_l2(alone[0]["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)) <= GATE_MIXED
    assert falls > 0, "no step ran fewer sweeps than the one before it: the idle early sweep went untested"


@pytest.mark.parametrize("rtol,max_refine,inner_rtol", [(1e-8, 4, 1e-5), (1e-11, 4, 1e-3), (1e-11, 1, 1e-3),
                                                        (0.5, 4, 1e-5)])
def test_mixed_single_simulation_overlap_matches_batch(gpu, rtol, max_refine, inner_rtol):
    """The mixed form alone also starts the next step's RHS and initial
    residual behind the decide of each refinement sweep, before the host
    knows whether that sweep ended the step; on the device they run only if
    it did.  Alone and in a batch of two (no overlap) must give the same bits:
    one sweep per step, several (a loose inner tolerance against a tight
    outer one), steps cut off unconverged by max_refine, and steps that need
    no sweep at all."""
    p = wl.random_problem(13, 9, 11, seed=37, nsteps=6, rtol=rtol)
    partner = wl.random_problem(6, 6, 6, seed=38, nsteps=6)
    kw = dict(save_every=1, precision=fh.FEM_FP32_FP64DOT, max_refine=max_refine, inner_rtol=inner_rtol,
              check=False)
    _, alone = fh.run_batch([p], **kw)
    _, pair = fh.run_batch([p, partner], **kw)
    st = alone[0]["status"]
    say(f"  rtol={rtol} max_refine={max_refine} inner_rtol={inner_rtol}: iters {list(alone[0]['iters'])} "
        f"sweeps {list(alone[0]['refine_sweeps'])} status {st}")
    assert st == pair[0]["status"] and st in (fh.FEM_OK, fh.FEM_ENOCONV)
    same_bits(alone[0], pair[0])
    if st == fh.FEM_OK and rtol <= 1e-8:  # (at rtol 0.5 neither field is near the converged one)
        ref = oracle.run(p, save_every=1)
        assert max(rel_l2(alone[0]["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)) <= GATE_MIXED
