"""GPU tests of the serving loop (fem_server_*): continuous batching,
admission by HBM budget, cancellation, and results that are the same served
in the mix as run alone.

Per request: bit-identical to a batch holding it alone (the server's
simulations join the batched launches at step boundaries and keep their own
tiles and reductions), and within the FP64 gate of the iteration-locked CPU
oracle (or the mixed-form gate of the free-running oracle).
"""
import time

import numpy as np
import pytest

from _util import rel_l2, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu


def same_bits(a, b):
    for key in ("T_final", "T_saved", "iters", "relres", "refine_sweeps"):
        if a[key] is None:
            assert b[key] is None
            continue
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key


def wait_for(srv, ticket, state, timeout=60.0):
    t_end = time.time() + timeout
    while time.time() < t_end:
        if srv.poll(ticket)["state"] >= state:
            return
        time.sleep(0.002)
    raise AssertionError(f"ticket {ticket} did not reach state {state}")


def test_continuous_batching_results_equal_alone_and_oracle(gpu):
    first = [wl.random_problem(20, 18, 16, seed=101, nsteps=150, rtol=1e-9),
             wl.two_phase_sphere_cube().replace(nsteps=120)]
    later = [wl.random_problem(9, 12, 8, seed=102, nsteps=7, hx=0.05, hy=0.08, hz=0.03, rtol=1e-10),
             wl.random_problem(13, 9, 11, seed=103, nsteps=5, theta=0.5, flux_mask=1 << wl.FACE_ZP,
                               flux=[0, 0, 0, 0, 0, 1.0]),
             wl.random_problem(5, 5, 5, seed=104, nsteps=0)]
    say("server: 2 long requests, then 3 more while they run")
    with fh.Server() as srv:
        t_first = [srv.submit(p, save_every=1) for p in first]
        wait_for(srv, t_first[0], fh.FEM_REQ_RUNNING)
        t_later = [srv.submit(p, save_every=1) for p in later]
        got = [srv.wait(t) for t in t_first + t_later]
        info = srv.info()
    say(f"  info {info}")
    assert info["completed"] == 5 and info["failed"] == 0 and info["queued"] == 0 and info["running"] == 0
    assert info["peak_bytes_in_use"] <= info["budget_bytes"] and info["bytes_in_use"] == 0
    states = [d for _, d, _ in got]
    for d in states:
        assert d["state"] == fh.FEM_REQ_DONE and d["status"] == 0
        assert 0.0 <= d["t_arrive"] <= d["t_admit"] <= d["t_done"]
    # continuous batching: the later requests joined while the first ones ran
    assert max(d["t_admit"] for d in states[2:]) < min(d["t_done"] for d in states[:2])
    for p, (st, d, r) in zip(first + later, got):
        assert st == fh.FEM_OK and r["status"] == 0
        _, alone = fh.run_batch([p], save_every=1)
        same_bits(r, alone[0])
        if p.nsteps:
            ref = oracle.run(p, save_every=1, locked_iters=r["iters"], nthreads=4)
            err = max(rel_l2(r["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps))
            say(f"  {p.name}: latency {d['t_done'] - d['t_arrive']:.3f}s max rel L2 {err:.2e}")
            assert err <= 1e-10


def test_admission_respects_a_tiny_budget(gpu):
    probs = [wl.random_problem(16, 16, 16, seed=110 + i, nsteps=4) for i in range(3)]
    with fh.Server() as srv:
        t = srv.submit(probs[0])
        one = srv.poll(t)["bytes"]
        srv.wait(t)
    budget = int(1.5 * one)
    say(f"server with budget {budget} bytes (1.5 requests)")
    with fh.Server(budget_bytes=budget) as srv:
        ts = [srv.submit(p) for p in probs]
        got = [srv.wait(x) for x in ts]
        info = srv.info()
    assert info["peak_bytes_in_use"] <= budget and info["completed"] == 3
    ds = [d for _, d, _ in got]
    for a, b in zip(ds, ds[1:]):  # one at a time, in order
        assert b["t_admit"] >= a["t_done"]
    for p, (_, _, r) in zip(probs, got):
        _, alone = fh.run_batch([p])
        same_bits(r, alone[0])


def test_cancel_queued_and_running(gpu):
    long = wl.random_problem(24, 24, 24, seed=120, nsteps=2000, rtol=1e-10)
    queued = wl.random_problem(8, 8, 8, seed=121, nsteps=3)
    after = wl.random_problem(8, 8, 8, seed=122, nsteps=3)
    with fh.Server(max_slots=1) as srv:
        tl = srv.submit(long)
        tq = srv.submit(queued)
        wait_for(srv, tl, fh.FEM_REQ_RUNNING)
        assert srv.poll(tq)["state"] == fh.FEM_REQ_QUEUED
        assert srv.cancel(tq) == fh.FEM_OK
        st_q, dq, rq = srv.wait(tq)
        assert st_q == fh.FEM_ECANCELED and dq["state"] == fh.FEM_REQ_CANCELED
        assert srv.cancel(tl) == fh.FEM_OK
        st_l, dl, rl = srv.wait(tl, timeout=60.0)
        assert st_l == fh.FEM_ECANCELED and dl["state"] == fh.FEM_REQ_CANCELED
        assert dl["steps_done"] < long.nsteps
        assert np.all(rl["T_final"] == 0)  # outputs of a cancelled request are not written
        ta = srv.submit(after)
        st_a, da, ra = srv.wait(ta)
        info = srv.info()
    assert st_a == fh.FEM_OK and info["canceled"] == 2 and info["completed"] == 1 and info["bytes_in_use"] == 0
    _, alone = fh.run_batch([after])
    same_bits(ra, alone[0])


def test_one_slot_admits_in_arrival_order_across_classes(gpu):
    """With one slot, requests of different size classes (different lanes)
    still run one at a time in arrival order."""
    probs = [wl.random_problem(20, 20, 20, seed=130, nsteps=6), wl.random_problem(5, 5, 5, seed=131, nsteps=2),
             wl.random_problem(12, 12, 12, seed=132, nsteps=3), wl.random_problem(5, 6, 5, seed=133, nsteps=2)]
    with fh.Server(max_slots=1) as srv:
        ts = [srv.submit(p) for p in probs]
        got = [srv.wait(t) for t in ts]
    ds = [d for _, d, _ in got]
    assert all(d["state"] == fh.FEM_REQ_DONE and d["status"] == 0 for d in ds)
    for a, b in zip(ds, ds[1:]):
        assert b["t_admit"] >= a["t_done"]


def test_budget_refusal_and_unknown_ticket(gpu):
    with fh.Server(budget_bytes=1000) as srv:
        with pytest.raises(fh.FemError) as e:
            srv.submit(wl.random_problem(4, 4, 4, seed=1))
        assert e.value.status == fh.FEM_ENOMEM
        with pytest.raises(fh.FemError):
            srv.poll(12345)


def test_mixed_precision_server(gpu):
    probs = [wl.sphere_proposal(s, n=24, nsteps=6) for s in range(4)]
    with fh.Server(precision=fh.FEM_FP32_FP64DOT) as srv:
        ts = [srv.submit(p, save_every=1) for p in probs]
        got = [srv.wait(t) for t in ts]
    for p, (st, d, r) in zip(probs, got):
        assert st == fh.FEM_OK
        _, alone = fh.run_batch([p], save_every=1, precision=fh.FEM_FP32_FP64DOT)
        same_bits(r, alone[0])
        ref = oracle.run(p, save_every=1)
        err = max(rel_l2(r["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps))
        say(f"  {p.name}: sweeps {list(r['refine_sweeps'])} max rel L2 vs FP64 oracle {err:.2e}")
        assert err <= 1e-5
