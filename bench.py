"""Benchmark: matrix-free Jacobi-PCG theta-scheme runs at 1M DOF on one MI355X.

One benchmark step is one full run of the log-normal Crank-Nicolson workload
(100^3 hexahedra, 1,030,301 nodes, 200 time steps, rtol 1e-8, q=1 on top,
T=0 at the bottom) with every input already resident in HBM (torch tensors
passed as device pointers).  The headline value is MDOF*iter/s =
N * (PCG iterations) / wall time / 1e6 over the timed steps, FP64.

Printed as one JSON line with a roofline object for the dominant kernel
(algorithmic bytes per launch / average launch time measured with HIP events
over the timed region) and a CPU baseline (the oracle on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(N: int, E: int, w: int) -> dict:
    """Bytes each kernel must move per launch (no re-reads counted).
    gather (direction + apply): read r, P^-1, d_old, rho*c_e, k_e; write d_new, q.
    update: read x, d, r, q, P^-1; write x, r."""
    return {"gather": (5 * N + 2 * E) * w, "update": 7 * N * w}


def committed_traffic(kernel: str, precision: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload, or None when there is none or the
    kernel sources changed since it was taken."""
    from paper_1905_07622_amd.profile_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_lognormal100_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return int(round(rec["traffic_bytes"]))


def cpu_baseline(problem, steps_a=1, steps_b=3):
    """The oracle (serial, 1 thread) on the same workload: the per-iteration
    rate of steps 2..steps_b, taken as the difference of two runs so that the
    one-off CSR assembly is excluded."""
    from oracle import oracle
    t0 = time.perf_counter()
    ra = oracle.run(problem, nsteps=steps_a, nthreads=1)
    t1 = time.perf_counter()
    rb = oracle.run(problem, nsteps=steps_b, nthreads=1)
    t2 = time.perf_counter()
    iters = int(rb["iters"].sum() - ra["iters"].sum())
    secs = (t2 - t1) - (t1 - t0)
    return {"value": problem.n_nodes * iters / secs / 1e6, "unit": "MDOF*iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{problem.name} ({problem.n_nodes} DOF): PCG iterations of steps {steps_a + 1}-{steps_b} "
                      f"({iters} iterations, {secs:.2f} s), serial CSR oracle, assembly excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--nsteps", type=int, default=200, help="time steps per run (the workload has 200)")
    ap.add_argument("--n", type=int, default=100, help="elements per edge (the workload has 100)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="time without per-kernel HIP events")
    ap.add_argument("--tile", type=int, nargs=3, default=(0, 0, 0))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 3 times (scale for rocprof FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the solver has no multi-GPU path; "
              "independent simulations would shard across GPUs with no communication.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 32 * 1024 * 1024  # 32 Mi doubles = 256 MiB per tensor
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "launches": 3}))
        return

    from paper_1905_07622_amd import femheat as fh
    from paper_1905_07622_amd import workloads as wl

    torch.cuda.set_device(0)
    p = wl.lognormal_cube(args.n, seed=2, nsteps=args.nsteps)
    dev = "cuda"
    k = torch.tensor(p.k_e, device=dev)
    rc = torch.tensor(p.rhoc_e, device=dev)
    T0 = torch.tensor(p.T0, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    prec = fh.FEM_FP64 if args.precision == "fp64" else fh.FEM_FP32_FP64DOT
    h = fh.Heat(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, k, rc, dirichlet_mask=p.dirichlet_mask,
                flux_mask=p.flux_mask, flux=p.flux, precision=prec, device_ptrs=True,
                timing=not args.no_timing, tile=tuple(args.tile), stream=stream)
    run_kw = dict(dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
    for w in range(args.warmup):
        h.run(T0, **run_kw)
        print(f"warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    stats = {"gather_launches": 0, "gather_ms": 0.0, "update_launches": 0, "update_ms": 0.0,
             "replace_launches": 0, "replace_ms": 0.0}
    last = None
    for s in range(args.steps):
        last = h.run(T0, **run_kw)
        iters += last["total_iters"]
        st = h.stats()
        for key in stats:
            stats[key] += st[key]
        print(f"step {s + 1}/{args.steps}: {last['total_iters']} iterations, device {last['device_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    value = p.n_nodes * iters / secs / 1e6
    shape = h.stats()
    h.close()

    w = 8 if args.precision == "fp64" else 4
    ab = algorithmic_bytes(p.n_nodes, p.n_elems, w)
    roof = None
    if stats["gather_launches"] and stats["update_launches"]:
        per = {"gather": stats["gather_ms"] / stats["gather_launches"],
               "update": stats["update_ms"] / stats["update_launches"]}
        dom = max(("gather", "update"), key=lambda kname: stats[kname + "_ms"])
        achieved = ab[dom] / (per[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": committed_traffic(dom, args.precision),
                "bytes_per_launch": ab[dom], "avg_launch_us": round(per[dom] * 1e3, 3),
                "other_kernels_us": {kname: round(v * 1e3, 3) for kname, v in per.items() if kname != dom}}

    line = {
        "metric": "PCG MDOF*iter/s at 1M DOF",
        "value": round(value, 1),
        "unit": "MDOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs * 1e3 / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 (f64 dots/scalars/refinement)",
        "data": "synthetic",
        "config": {"workload": f"log-normal k, {p.nx}^3 hex Q1 ({p.n_nodes} DOF), Crank-Nicolson dt=5e-4, "
                               f"{p.nsteps} steps, rtol 1e-8, Jacobi-PCG", "seed": 2,
                   "precision": args.precision, "iterations_per_run": int(last["total_iters"]),
                   "tile": [shape["tile_x"], shape["tile_y"], shape["tile_z"]],
                   "grid_blocks": shape["grid_blocks"]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(line), flush=True)
    del np


if __name__ == "__main__":
    main()
