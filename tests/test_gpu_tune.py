"""The autotuner (fem_heat_tune) and its tile cache.

Tuning changes only the launch shape of the gather.  The operator's value at
every node is formed in a fixed order whatever the tile (the apply is
bit-identical across tiles), but the PCG dot products are summed per block,
so another tile partitions them differently and rounds them differently.
Runs with the tuned tile are therefore checked against the oracle locked to
their own iteration counts (FP64: relative L2 1e-10) or against the FP64
oracle (mixed form: 1e-5), and against the untuned run to rounding; a
handle that takes the tile from the cache repeats the tuned run bit for bit.
The cache makes later handles (single, batch members) take the recorded tile.
"""
import json

import numpy as np
import pytest

from _util import rel_l2, say
from oracle import oracle
from paper_1905_07622_amd import femheat as fh
from paper_1905_07622_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run(h, p, nsteps=4):
    return h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=nsteps, rtol=p.rtol)


@pytest.mark.parametrize("precision", [fh.FEM_FP64, fh.FEM_FP32_FP64DOT])
def test_tuned_single_run_bitwise_equal_and_cached(gpu, tmp_path, precision):
    p = wl.lognormal_cube(36, seed=5, nsteps=4)
    cache = str(tmp_path / "tune.json")
    with fh.Heat.from_problem(p, precision=precision) as h0:
        ref = _run(h0, p)
        rule_tile = [h0.stats()[k] for k in ("tile_x", "tile_y", "tile_z")]
    with fh.Heat.from_problem(p, precision=precision, tune_cache=cache) as h1:
        res = h1.tune(dt=p.dt, theta=p.theta)
        say(f"tuned {res} (rule tile {rule_tile})")
        assert res["candidates"] > 3 and res["recorded"] == 1
        assert res["best_us"] <= res["rule_us"]
        st = h1.stats()
        assert [st["tile_x"], st["tile_y"], st["tile_z"]] == [res["tile_x"], res["tile_y"], res["tile_z"]]
        out = _run(h1, p)
    assert out["status"] == 0
    gate = 1e-10 if precision == fh.FEM_FP64 else 1e-5
    if precision == fh.FEM_FP64:
        want = oracle.run(p, nsteps=4, locked_iters=out["iters"])
    else:
        want = oracle.run(p, nsteps=4)
    err = rel_l2(out["T_final"], want["T_final"])
    say(f"  tuned run vs oracle: rel L2 {err:.2e}; vs untuned run {rel_l2(out['T_final'], ref['T_final']):.2e}")
    assert err <= gate
    assert rel_l2(out["T_final"], ref["T_final"]) <= gate
    assert np.abs(out["iters"].astype(int) - ref["iters"].astype(int)).max() <= 1
    rec = json.load(open(cache))["entries"]
    assert len(rec) == 1 and rec[0]["tile"] == [res["tile_x"], res["tile_y"], res["tile_z"]]
    assert "|single|37x37x37" in rec[0]["key"]
    # a later handle with the same options takes the recorded tile
    with fh.Heat.from_problem(p, precision=precision, tune_cache=cache) as h2:
        st = h2.stats()
        assert [st["tile_x"], st["tile_y"], st["tile_z"]] == rec[0]["tile"]
        again = _run(h2, p)
    assert np.array_equal(again["T_final"], out["T_final"]) and np.array_equal(again["iters"], out["iters"])


def test_tuned_batch_members_match(gpu, tmp_path):
    cache = str(tmp_path / "tune.json")
    probs = [wl.sphere_proposal(s, n=20, nsteps=3) for s in range(5)]
    st0, ref = fh.run_batch(probs, precision=fh.FEM_FP32_FP64DOT)
    p = probs[0]
    with fh.Heat.from_problem(p, precision=fh.FEM_FP32_FP64DOT, tune_cache=cache) as h:
        before = h.stats()
        res = h.tune(dt=p.dt, theta=p.theta, batch=True)
        after = h.stats()
    say(f"batch-member tile {res}")
    assert res["recorded"] == 1
    # with FEM_TUNE_BATCH the handle keeps its own tile; the batch tile is recorded
    assert [before[k] for k in ("tile_x", "tile_y", "tile_z")] == [after[k] for k in ("tile_x", "tile_y", "tile_z")]
    assert "|batch|21x21x21" in json.load(open(cache))["entries"][0]["key"]
    st1, out = fh.run_batch(probs, precision=fh.FEM_FP32_FP64DOT, tune_cache=cache)
    assert st0 == st1 == fh.FEM_OK
    for q, a, b in zip(probs, out, ref):
        want = oracle.run(q, nsteps=3)
        assert rel_l2(a["T_final"], want["T_final"]) <= 1e-5
        assert rel_l2(a["T_final"], b["T_final"]) <= 1e-5
    # the same cache gives the same tiles, so a second batch repeats the first bit for bit
    st2, again = fh.run_batch(probs, precision=fh.FEM_FP32_FP64DOT, tune_cache=cache)
    assert st2 == fh.FEM_OK
    for a, b in zip(again, out):
        assert np.array_equal(a["T_final"], b["T_final"]) and np.array_equal(a["iters"], b["iters"])


def test_tune_rejects_bad_arguments(gpu):
    p = wl.random_problem(5, 4, 3, seed=2)
    with fh.Heat.from_problem(p) as h:
        assert fh.fem_heat_tune(h.h, -1.0, 1.0)[0] == fh.FEM_EINVAL
        assert fh.fem_heat_tune(h.h, 1e-3, 2.0)[0] == fh.FEM_EINVAL
        assert fh.fem_heat_tune(h.h, 1e-3, 1.0, 0x8)[0] == fh.FEM_EINVAL


@pytest.mark.parametrize("precision", [fh.FEM_FP64, fh.FEM_FP32_FP64DOT])
@pytest.mark.parametrize("tile", [(41, 12, 5), (101, 5, 9), (37, 13, 4)])
def test_wide_blocks_of_a_simulation_alone(gpu, precision, tile):
    """Blocks of up to 512 threads (eight waves), which a simulation alone may
    take: the run against the oracle (FP64 locked to its own counts at 1e-10,
    mixed against the FP64 oracle at 1e-5), ragged tiles at every edge and a
    block with idle lanes (41 x 12 = 492 of 512 threads); the operator apply
    with such a tile is bit-identical to the default tile's."""
    p = wl.random_problem(40, 23, 17, seed=71, nsteps=4, rtol=1e-10) if tile[0] != 101 else \
        wl.lognormal_cube(100, seed=2, nsteps=2)
    with fh.Heat.from_problem(p, precision=precision, tile=tile, timing=True) as h:
        out = h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol, save_every=1)
        st = h.stats()
        x = np.random.default_rng(3).standard_normal(p.n_nodes)
        y_wide = h.apply(fh.FEM_OP_A, x, dt=p.dt, theta=p.theta)
    assert [st["tile_x"], st["tile_y"], st["tile_z"]] == list(tile)
    assert out["status"] == fh.FEM_OK
    if precision == fh.FEM_FP64:
        ref = oracle.run(p, save_every=1, locked_iters=out["iters"], nthreads=16)
        gate = 1e-10
    else:
        ref = oracle.run(p, save_every=1, nthreads=16)
        gate = 1e-5
    errs = [rel_l2(out["T_saved"][n], ref["T_saved"][n]) for n in range(p.nsteps)]
    say(f"  tile {tile} ({st['grid_blocks']} blocks): iters {list(out['iters'])}, rel L2 max {max(errs):.2e}")
    assert max(errs) <= gate
    assert np.all(out["relres"] <= p.rtol)
    with fh.Heat.from_problem(p, precision=precision) as h0:
        y_rule = h0.apply(fh.FEM_OP_A, x, dt=p.dt, theta=p.theta)
    assert np.array_equal(y_wide, y_rule)


def test_wide_blocks_refused_for_batch_members(gpu):
    p = wl.random_problem(12, 10, 9, seed=72, nsteps=1)
    st, _ = fh.run_batch([p, p], tile=(41, 12, 5), check=False)
    assert st == fh.FEM_EINVAL
    assert "256" in fh.fem_last_error(None)
