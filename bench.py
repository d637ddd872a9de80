"""Benchmark: matrix-free Jacobi-PCG theta-scheme runs at 1M DOF on one MI355X.

One benchmark step is one full run of the log-normal Crank-Nicolson workload
(100^3 hexahedra, 1,030,301 nodes, 200 time steps, rtol 1e-8, q=1 on top,
T=0 at the bottom) with every input already resident in HBM (torch tensors
passed as device pointers).  The headline value is MDOF*iter/s =
N * (PCG iterations) / wall time / 1e6 over the timed steps, FP64.

Printed as one JSON line with a roofline object for the dominant kernel
(algorithmic bytes per launch / average launch time measured with HIP events
over the timed region) and a CPU baseline (the oracle on a bounded sample).
The same line carries the batched-proposals result ("batched": 64 x 48^3
simulations in one fem_heat_run_batch call) and the serving result
("served": a Poisson request stream through fem_server), each next to the
plain one-at-a-time FP64 path on the same inputs.
"""
from __future__ import annotations

import argparse
import json
import os
import tempfile
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def deferred_fraction(iters, R: int = 50) -> float:
    """Share of the direction launches that also apply the previous
    iteration's x += alpha d: those of iterations 1..it-1 not preceded by a
    residual replacement (iterations 0, R, 2R, ... of each solve replace)."""
    total = corr = 0
    for it in np.asarray(iters, dtype=np.int64).tolist():
        total += it
        if it >= 1:
            corr += (it - 1) - (0 if it < 2 else (it - 2) // R + 1)
    return corr / total if total else 0.0


def algorithmic_bytes(N: int, E: int, w: int, f_corr: float, form: str = "two-kernel") -> dict:
    """Bytes each kernel must move per launch (no re-reads counted), averaged
    over the launches the timing samples.
    two-kernel: gather (direction + apply) reads r, P^-1, d_old, rho*c_e,
    k_e, writes d_new and q, and in the share f_corr of launches also reads
    and writes x; update reads r, q, P^-1 and writes r.
    one-kernel (both halves in one launch, q, r and P^-1 at the own nodes
    kept on chip): the gather half without q, the update half writing r:
    (5 N + 2 E) w + 2 N w f_corr, no update kernel.
    one-reduction: the gather also reads the previous q and writes the
    advanced r (4 N w f_corr), no update kernel."""
    if form == "one-kernel":
        return {"gather": (5 * N + 2 * E) * w + 2 * N * w * f_corr, "update": 0}
    if form == "one-reduction":
        return {"gather": (5 * N + 2 * E) * w + 4 * N * w * f_corr, "update": 0}
    return {"gather": (5 * N + 2 * E) * w + 2 * N * w * f_corr, "update": 4 * N * w}


def committed_traffic(kernel: str, precision: str, form: str = "two-kernel"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload, or None when there is none or the
    kernel sources changed since it was taken."""
    from paper_1905_07622_amd.profile_summary import kernel_source_hash
    tag = {"two-kernel": "", "one-reduction": "_one_reduction", "one-kernel": "_one_kernel"}[form]
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}{tag}_lognormal100_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return int(round(rec["traffic_bytes"]))


def host_cpu():
    """CPU model and the cores this process may use (the box's share)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def cpu_baseline(problem, gpu_iters, gpu_T_final, steps_a=1, steps_b=3):
    """The oracle on the same workload.  Main figure: the whole 200-step run,
    multi-threaded on the host cores this process may use (at most 16),
    iteration-locked to the GPU's per-step counts (so it also gives the
    headline run's parity), MDOF*iter/s over the PCG part (CSR assembly,
    timed by a 0-step run, excluded).  Beside it: one core on the iterations
    of steps 2-3 (a bounded sample, as a 1-core rate)."""
    from oracle import oracle
    model, cores, ncpu = host_cpu()
    nt = max(1, min(16, cores))
    t0 = time.perf_counter()
    oracle.run(problem, nsteps=0, nthreads=nt)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    full = oracle.run(problem, locked_iters=gpu_iters, nthreads=nt)
    t_full = time.perf_counter() - t0
    iters = int(np.asarray(gpu_iters).sum())
    secs = max(t_full - t_setup, 1e-9)
    ref = full["T_final"]
    parity = float(np.linalg.norm(np.asarray(gpu_T_final) - ref) / np.linalg.norm(ref))
    t0 = time.perf_counter()
    ra = oracle.run(problem, nsteps=steps_a, nthreads=1)
    t1 = time.perf_counter()
    rb = oracle.run(problem, nsteps=steps_b, nthreads=1)
    t2 = time.perf_counter()
    it1 = int(rb["iters"].sum() - ra["iters"].sum())
    s1 = (t2 - t1) - (t1 - t0)
    return {"value": problem.n_nodes * iters / secs / 1e6, "unit": "MDOF*iter/s", "cores": nt, "kind": "oracle",
            "sample": f"{problem.name} ({problem.n_nodes} DOF): the whole {problem.nsteps}-step run, {iters} PCG "
                      f"iterations locked to the GPU's per-step counts, {secs:.1f} s on {nt} threads (CSR assembly, "
                      f"{t_setup:.1f} s, excluded)",
            "cpu_model": model, "nproc": ncpu, "cores_available": cores,
            "headline_rel_l2_vs_oracle": parity,
            "single_core": {"value": problem.n_nodes * it1 / s1 / 1e6, "unit": "MDOF*iter/s", "cores": 1,
                            "sample": f"PCG iterations of steps {steps_a + 1}-{steps_b} ({it1} iterations, "
                                      f"{s1:.2f} s), serial"}}


def _to_device(p, torch):
    dev = "cuda"
    return p.replace(k_e=torch.tensor(p.k_e, device=dev), rhoc_e=torch.tensor(p.rhoc_e, device=dev),
                     T0=torch.tensor(p.T0, device=dev))


def _plain_solve(p, rtol, stream):
    """One forward solve on the plain path: a fresh FP64 handle, fem_heat_run."""
    from paper_1905_07622_amd import femheat as fh
    with fh.Heat(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, p.k_e, p.rhoc_e, dirichlet_mask=p.dirichlet_mask,
                 flux_mask=p.flux_mask, flux=p.flux, device_ptrs=True, stream=stream) as h:
        return h.run(p.T0, dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=rtol)


def _rel(a, b, torch):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def _timed_runs(h, T0, run_kw, nruns):
    """Times nruns full runs after one warm-up; returns (MDOF*iter/s, iterations per run, last result)."""
    h.run(T0, **run_kw)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, last = 0, None
    for _ in range(nruns):
        last = h.run(T0, **run_kw)
        iters += last["total_iters"]
    torch.cuda.synchronize()
    return iters / (time.perf_counter() - t0) / 1e6, last["total_iters"], last


def bench_mixed(args, torch, p, k, rc, T0, T_fp64):
    """The headline workload in the mixed form (FP32 inner PCG with FP64 dot products and scalars inside
    FP64 refinement): MDOF*iter/s counting inner iterations, and the final field against the FP64 run."""
    from paper_1905_07622_amd import femheat as fh
    stream = torch.cuda.current_stream().cuda_stream
    h = fh.Heat(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, k, rc, dirichlet_mask=p.dirichlet_mask,
                flux_mask=p.flux_mask, flux=p.flux, precision=fh.FEM_FP32_FP64DOT, device_ptrs=True,
                stream=stream, one_kernel=args.pcg_form == "one-kernel",
                tune_cache=getattr(args, "tune_cache_path", None))
    run_kw = dict(dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
    tuned = h.tune(dt=p.dt, theta=p.theta) if getattr(args, "tune_cache_path", None) else None
    rate, its, last = _timed_runs(h, T0, run_kw, 2)
    h.close()
    diff = torch.linalg.vector_norm(last["T_final"] - T_fp64) / torch.linalg.vector_norm(T_fp64)
    print(f"mixed: {rate * p.n_nodes:.1f} MDOF*iter/s", file=sys.stderr, flush=True)
    return {"workload": "the headline workload in the mixed form", "value": round(rate * p.n_nodes, 1),
            "unit": "MDOF*iter/s", "iterations_per_run": int(its),
            "sweeps_per_step_max": int(last["refine_sweeps"].max()), "autotuned": tuned,
            "rel_l2_vs_fp64_final_field": float(diff)}


def bench_above_mall(args, torch):
    """The headline field rules at (mall_n+1)^3 nodes, whose FP64 working set (~100 B per node) exceeds
    the 256 MB Infinity Cache: the rate when HBM, not the cache, serves the vectors."""
    from paper_1905_07622_amd import femheat as fh
    from paper_1905_07622_amd import workloads as wl
    p = wl.lognormal_cube(args.mall_n, seed=2, nsteps=args.mall_nsteps)
    dev = "cuda"
    k = torch.tensor(p.k_e, device=dev)
    rc = torch.tensor(p.rhoc_e, device=dev)
    T0 = torch.tensor(p.T0, device=dev)
    h = fh.Heat(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, k, rc, dirichlet_mask=p.dirichlet_mask,
                flux_mask=p.flux_mask, flux=p.flux, device_ptrs=True, timing=True,
                stream=torch.cuda.current_stream().cuda_stream)
    run_kw = dict(dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
    t0 = time.perf_counter()
    rate, its, last = _timed_runs(h, T0, run_kw, 2)
    form = "one-kernel" if h.stats()["one_kernel_launches"] > 0 else "two-kernel"
    h.close()
    f_corr = deferred_fraction(last["iters"].cpu().numpy())
    ab = algorithmic_bytes(p.n_nodes, p.n_elems, 8, f_corr, form)
    mdof = rate * p.n_nodes
    print(f"above MALL: {mdof:.1f} MDOF*iter/s ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    return {"workload": f"log-normal k, {p.nx}^3 hex Q1 ({p.n_nodes} DOF), Crank-Nicolson dt=5e-4, "
                        f"{p.nsteps} steps, rtol 1e-8, FP64", "value": round(mdof, 1), "unit": "MDOF*iter/s",
            "iterations_per_run": int(its), "pcg_form": form,
            "effective_gbs": round((ab["gather"] + ab["update"]) * rate * 1e6 / 1e9, 1)}


def bench_apply_ab(args, torch, p, k, rc, calls=20):
    """The operator apply y = A x of the headline workload three ways: the node-centred gather of the PCG
    path, the two-pass element-by-element form after the paper's coalesced element-by-element method
    (FEM_OP_ELEMENTWISE), and a node-centred form with one wavefront per node row and no block barrier
    (FEM_OP_ROWWAVE).  Device time of the operator kernels per call (HIP events inside the library),
    and the effective rate on the operator's own bytes (read x and the two coefficient arrays, write y)."""
    from paper_1905_07622_amd import femheat as fh
    h = fh.Heat(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, k, rc, dirichlet_mask=p.dirichlet_mask,
                flux_mask=p.flux_mask, flux=p.flux, device_ptrs=True, timing=True,
                stream=torch.cuda.current_stream().cuda_stream)
    x = torch.rand(p.n_nodes, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    own = (2 * p.n_nodes + 2 * p.n_elems) * 8
    res = {}
    ys = {}
    forms = (("gather", {}), ("elementwise_two_pass", {"elementwise": True}), ("row_wavefronts", {"rowwave": True}))
    for name, kw in forms:
        for _ in range(3):
            h.apply(fh.FEM_OP_A, x, dt=p.dt, theta=p.theta, **kw)
        s0 = h.stats()
        for _ in range(calls):
            ys[name] = h.apply(fh.FEM_OP_A, x, dt=p.dt, theta=p.theta, **kw)
        s1 = h.stats()
        us = (s1["apply_ms"] - s0["apply_ms"]) / (s1["apply_calls"] - s0["apply_calls"]) * 1e3
        res[name] = {"us_per_apply": round(us, 2), "operator_gbs": round(own / us / 1e3, 1)}
    h.close()
    res["elementwise_two_pass"]["design_bytes"] = (13 * p.n_nodes + 2 * p.n_elems) * 8
    res["gather"]["design_bytes"] = own
    res["row_wavefronts"]["design_bytes"] = own  # (its nine-row and four-element-row re-reads are L2 traffic)
    nrm = torch.linalg.vector_norm(ys["gather"])
    res["max_rel_l2_between_forms"] = max(float(torch.linalg.vector_norm(ys["gather"] - ys[n]) / nrm)
                                          for n, _ in forms[1:])
    res["calls"] = calls
    res["workload"] = "y = (M + theta dt K) x on the headline grid and coefficients, x ~ U[0,1)"
    print(f"apply A/B: gather {res['gather']['us_per_apply']} us, elementwise "
          f"{res['elementwise_two_pass']['us_per_apply']} us, row wavefronts {res['row_wavefronts']['us_per_apply']} us",
          file=sys.stderr, flush=True)
    return res


def bench_inverse(args, torch, chains=32, iters=48, n=64):
    """The paper's motivating use (Section 5.4) through the batched path: Metropolis-Hastings chains over
    the corrosion depth of the plate stand-in, every proposal a forward solve (mixed form), all chains'
    proposals of an iteration in one fem_heat_run_batch call.  The observed frame is the FP64 GPU solve at
    the true depth through the camera model.  Throughput = forward solves / wall time of the sampling."""
    from paper_1905_07622_amd import femheat as fh
    from paper_1905_07622_amd import inverse as inv
    from paper_1905_07622_amd import workloads as wl

    def make(d):
        return wl.corroded_plate(d, n=n)

    truth = 0.03125
    f_true = inv.batched_frames(make, precision=fh.FEM_FP64)(np.array([truth]))[0]
    obs = inv.camera(f_true, wl.camera_noise(21, f_true.size))
    normals, uniforms = wl.mh_draws(22, iters, chains)
    ll = inv.likelihood_of(inv.batched_frames(make, precision=fh.FEM_FP32_FP64DOT), obs)
    t0 = time.perf_counter()
    out = inv.metropolis(np.linspace(0.01, 0.08, chains), normals, uniforms, 0.004, ll, 0.0, 0.125)
    secs = time.perf_counter() - t0
    late = out["samples"][iters // 2:].ravel()
    p = make(truth)
    print(f"inverse: {out['evaluated'] / secs:.1f} forward solves/s", file=sys.stderr, flush=True)
    return {"workload": f"{chains} Metropolis-Hastings chains x {iters} iterations over the corrosion depth of a "
                        f"{p.nx}x{p.ny}x{p.nz}-element plate ({p.n_nodes} DOF, {p.nsteps} backward-Euler steps, "
                        f"{p.sensors.shape[0]}-pixel camera, noise 0.1 rounded to 0.1), proposals solved in the "
                        "mixed form, one batched call per iteration",
            "forward_solves_per_s": round(out["evaluated"] / secs, 1), "seconds": round(secs, 3),
            "forward_solves": out["evaluated"], "acceptance": round(float(out["accepted"].mean()), 3),
            "true_depth": truth, "second_half_mean": round(float(late.mean()), 5),
            "second_half_std": round(float(late.std()), 5)}


def bench_context(torch, gather_bytes):
    """Reference points for the kernel figures, measured with torch on the same GPU: a device copy moving the
    gather's bytes (half read, half written), and the rate of a 256 MiB copy."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def copy_us(nbytes, reps=20):
        src = torch.empty(nbytes // 16, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    g_us = copy_us(int(gather_bytes))
    big = 2 * 256 * 1024 * 1024
    b_us = copy_us(big, reps=5)
    return {"copy_of_gather_bytes_us": round(g_us, 2),
            "copy_of_gather_bytes_gbs": round(gather_bytes / g_us / 1e3, 1),
            "copy_256MiB_gbs": round(big / b_us / 1e3, 1),
            "note": "torch device copies on the same GPU, (read + write bytes) / time between events"}


def bench_batched(args, torch):
    """Batched proposals: S simulations on 48^3 random-sphere fields, 100
    backward-Euler steps each, in one fem_heat_run_batch call (mixed form),
    against the plain one-at-a-time FP64 path on a sample of the same
    simulations, at the workload's rtol and at a looser rtol that still keeps
    the error within the mixed form's stated accuracy.  Inputs resident in
    HBM; handle set-up inside the timed region on both sides."""
    from paper_1905_07622_amd import femheat as fh
    from paper_1905_07622_amd import workloads as wl
    stream = torch.cuda.current_stream().cuda_stream
    probs = [_to_device(wl.sphere_proposal(s, n=args.batch_n, nsteps=args.batch_nsteps), torch)
             for s in range(args.batch_sims)]
    prec = fh.FEM_FP32_FP64DOT if args.batch_precision == "mixed" else fh.FEM_FP64
    cache = getattr(args, "tune_cache_path", None)
    tuned = None
    if cache:  # batch-member tile for this grid, recorded in the cache the batched call reads
        with fh.Heat.from_problem(probs[0], precision=prec, device_ptrs=True, stream=stream, tune_cache=cache) as th:
            tuned = th.tune(dt=probs[0].dt, theta=probs[0].theta, batch=True)
        print(f"batched: tuned batch-member tile {tuned}", file=sys.stderr, flush=True)
    fh.run_batch(probs[:2], precision=prec, device_ptrs=True, stream=stream, tune_cache=cache)  # warm-up
    times = []
    for _ in range(3):  # the median of three whole batches (each well under a second)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, res = fh.run_batch(probs, precision=prec, device_ptrs=True, stream=stream, tune_cache=cache)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"batched: {len(probs)} simulations in {times[-1]:.2f} s (status {st})", file=sys.stderr, flush=True)
    t_batch = float(np.median(times))
    sample = probs[:args.plain_sample]
    out = {"workload": f"{len(probs)} x {args.batch_n}^3 random-sphere proposals, backward Euler dt=1e-3, "
                       f"{args.batch_nsteps} steps, rtol 1e-8", "precision": args.batch_precision,
           "solves_per_s": round(len(probs) / t_batch, 3), "seconds": round(t_batch, 3),
           "seconds_of_three_runs": [round(t, 3) for t in times],
           "nodes_per_sim": probs[0].n_nodes, "iterations_per_sim_mean": float(np.mean([r["total_iters"] for r in res])),
           "autotuned_member_tile": tuned,
           "concurrent_batches": max(1, min(3, len(probs) // 16, sum(p.n_nodes for p in probs) >> 21))}
    plain = {}
    refs = {}
    for rtol in (1e-8,) + tuple(args.loose_rtols):
        t0 = time.perf_counter()
        outs = [_plain_solve(p, rtol, stream) for p in sample]
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t0
        if rtol == 1e-8:
            refs = outs
        errs = [_rel(o["T_final"], r["T_final"], torch) for o, r in zip(outs, refs)]
        plain[rtol] = {"solves_per_s": round(len(sample) / dt_, 3), "max_rel_err_vs_fp64_rtol_1e-8": max(errs)}
        print(f"plain fp64 rtol {rtol:g}: {len(sample)} solves in {dt_:.2f} s", file=sys.stderr, flush=True)
    errs = [_rel(res[i]["T_final"], refs[i]["T_final"], torch) for i in range(len(sample))]
    out["max_rel_err_vs_plain_fp64"] = max(errs)
    out["plain_fp64"] = {"sample": len(sample), "at_rtol_1e-8": plain[1e-8]}
    ok_loose = [r for r in args.loose_rtols if plain[r]["max_rel_err_vs_fp64_rtol_1e-8"] <= 1e-5]
    if ok_loose:
        loose = max(ok_loose)
        out["plain_fp64"]["loosest_within_1e-5"] = dict(plain[loose], rtol=loose)
        base = plain[loose]["solves_per_s"]
    else:
        base = plain[1e-8]["solves_per_s"]
    out["speedup_vs_plain"] = round(out["solves_per_s"] / base, 3)
    return out


def _fcfs(arrivals, service):
    """Completion times of one-at-a-time FCFS service of the arrival trace."""
    done, out = 0.0, []
    for ta, sv in zip(arrivals, service):
        done = max(ta, done) + sv
        out.append(done)
    return np.array(out)


def _window_stats(arrivals, finish, warm):
    """Solves/s over the measurement window (arrival of the first measured
    request to the last measured completion) and p50/p99 latency, excluding
    the first `warm` requests."""
    a, f = np.asarray(arrivals)[warm:], np.asarray(finish)[warm:]
    lat = f - a
    return {"solves_per_s": round(len(a) / (f.max() - a.min()), 3), "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4)}


def bench_served(args, torch):
    """Serving (the measurement plan for it): a Poisson stream of
    `serve_requests` forward-solve requests (edge from {32,48,64,96,128},
    log-normal or two-phase field, 50-300 steps, theta in {0.5,1}, rtol 1e-8),
    the first `serve_warmup` excluded from the statistics.  The plain path --
    one FP64 handle per request, one request at a time -- is run first over
    the whole mix; its capacity (requests / busy time) sets the arrival rate
    lambda = serve_load x capacity.  The loosest rtol in {1e-6, 1e-7} whose
    plain FP64 result stays within 1e-5 of the rtol-1e-8 result (the mixed
    form's stated accuracy) is probed on the first requests after the
    warm-up.  The stream is then replayed in real time into a server
    (continuous batching, mixed form, HBM budget) at that rtol.  The plain
    path is reported on the same arrival trace (FCFS latencies from its
    measured service times) at rtol 1e-8 and at that rtol (equal stated
    accuracy).  Errors: every served result against the plain FP64 rtol-1e-8
    result; served results of edge <= 64 (a sample) against the CPU oracle
    (FP64, rtol 1e-8); ten sampled requests re-run alone through a fresh
    server, against their served result (bitwise)."""
    from paper_1905_07622_amd import femheat as fh
    from paper_1905_07622_amd import workloads as wl
    stream = torch.cuda.current_stream().cuda_stream
    n, warm = args.serve_requests, args.serve_warmup
    t0 = time.perf_counter()
    reqs = [wl.serve_request(i) for i in range(n)]
    print(f"served: {n} requests generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    prec = fh.FEM_FP32_FP64DOT if args.batch_precision == "mixed" else fh.FEM_FP64

    def plain_pass(rtol, subset=None):
        service, outs = [], []
        for i in (range(n) if subset is None else subset):
            pd = _to_device(reqs[i], torch)
            torch.cuda.synchronize()
            t = time.perf_counter()
            o = _plain_solve(pd, rtol, stream)
            torch.cuda.synchronize()
            service.append(time.perf_counter() - t)
            outs.append(o["T_final"])
        return np.array(service), outs

    cache = getattr(args, "tune_cache_path", None)
    if cache:  # batch-member tiles of every serving grid, recorded in the cache the servers read
        for edge in wl.SERVE_EDGES:
            q = next(r for r in reqs if r.nx == edge)
            with fh.Heat.from_problem(q, precision=prec, tune_cache=cache) as th:
                th.tune(dt=q.dt, theta=q.theta, batch=True)
    _plain_solve(_to_device(reqs[0].replace(nsteps=3), torch), 1e-8, stream)  # warm-up
    service, plain_T = plain_pass(1e-8)
    capacity = n / service.sum()
    rate = args.serve_load * capacity if args.serve_rate <= 0 else args.serve_rate
    print(f"served: plain FP64 busy {service.sum():.1f} s, capacity {capacity:.3f}/s, lambda {rate:.3f}/s",
          file=sys.stderr, flush=True)
    arrivals = wl.poisson_arrivals(n, rate, seed=5)

    # the loosest rtol within the mixed form's stated accuracy (1e-5 against the
    # FP64 rtol-1e-8 result), probed on the plain path; both paths then run at
    # it ("equal stated accuracy"), the served one checked on every request
    probe = list(range(warm, min(n, warm + args.serve_probe)))
    loose = None
    for rtol in sorted(args.loose_rtols, reverse=True):
        _, outs = plain_pass(rtol, probe)
        e = max(_rel(o, plain_T[i], torch) for o, i in zip(outs, probe))
        if e <= 1e-5:
            loose = rtol
            break
    serve_rtol = loose if loose is not None else 1e-8
    reqs_s = [r.replace(rtol=serve_rtol) for r in reqs]

    with fh.Server(precision=prec, tune_cache=cache) as srv:  # warm-up of the server path
        srv.wait(srv.submit(wl.serve_request(10_000).replace(nsteps=3)))
    srv = fh.Server(precision=prec, tune_cache=cache)
    t_start = time.perf_counter()
    tickets = []
    for p, ta in zip(reqs_s, arrivals):
        delay = ta - (time.perf_counter() - t_start)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(p))
    got = [srv.wait(t) for t in tickets]
    t_all = time.perf_counter() - t_start
    info = srv.info()
    srv.close()
    t_arr = np.array([d["t_arrive"] for _, d, _ in got])
    t_done = np.array([d["t_done"] for _, d, _ in got])
    served = _window_stats(t_arr, t_done, warm)
    statuses = sorted({int(d["status"]) for _, d, _ in got})
    served_T = [r["T_final"] for _, _, r in got]
    print(f"served: {n} requests in {t_all:.2f} s, {served}", file=sys.stderr, flush=True)

    errs = np.array([_rel(torch.tensor(T, device="cuda"), P, torch) for T, P in zip(served_T, plain_T)])
    plain_fin = _fcfs(arrivals, service)
    plain = dict(_window_stats(arrivals, plain_fin, warm), rtol=1e-8,
                 busy_solves_per_s=round(n / service.sum(), 3))

    plain_loose = None
    if loose is not None:
        sv_l, outs_l = plain_pass(loose)
        e_l = max(_rel(o, P, torch) for o, P in zip(outs_l[warm:], plain_T[warm:]))
        plain_loose = dict(_window_stats(arrivals, _fcfs(arrivals, sv_l), warm), rtol=loose,
                           busy_solves_per_s=round(n / sv_l.sum(), 3), max_rel_err_vs_rtol_1e_8=e_l)
        print(f"served: plain FP64 at rtol {loose:g}: {plain_loose}", file=sys.stderr, flush=True)

    # ten sampled requests alone, against their result in the mix
    rng = np.random.default_rng(55)
    sample = sorted(rng.choice(np.arange(warm, n), size=min(10, n - warm), replace=False).tolist())
    alone_diff = 0.0
    with fh.Server(precision=prec, tune_cache=cache) as solo:
        for i in sample:
            _, _, r = solo.wait(solo.submit(reqs_s[i]))
            alone_diff = max(alone_diff, float(np.abs(r["T_final"] - served_T[i]).max()))

    # the CPU oracle on served requests of edge <= 64
    from oracle import oracle
    small = [i for i in range(warm, n) if reqs[i].nx <= 64][:args.serve_oracle]
    model, cores, _ = host_cpu()
    oerr = []
    for i in small:
        ref = oracle.run(reqs[i], nthreads=max(1, min(16, cores)))["T_final"]  # FP64 at the config's rtol
        oerr.append(float(np.linalg.norm(served_T[i] - ref) / np.linalg.norm(ref)))
    print(f"served: oracle on {len(small)} requests, max rel L2 {max(oerr) if oerr else float('nan'):.2e}",
          file=sys.stderr, flush=True)
    speed_base = (plain_loose or plain)["solves_per_s"]
    return {"workload": f"{n} Poisson-arrival requests (first {warm} warm-up, excluded), edge in {{32..128}}, "
                        f"50-300 steps, theta in {{0.5,1}}, rtol 1e-8",
            "precision": args.batch_precision, "served_rtol": serve_rtol,
            "served_rtol_rule": "the loosest of the probed rtols whose plain FP64 result stays within 1e-5 of the "
                                "rtol-1e-8 result (the mixed form's stated accuracy); errors below are against "
                                "FP64 at rtol 1e-8", "lambda_per_s": round(rate, 3),
            "lambda_rule": f"{args.serve_load} x plain FP64 capacity ({capacity:.3f}/s on this mix)"
            if args.serve_rate <= 0 else "fixed", **served,
            "statuses": statuses, "peak_hbm_bytes": int(info["peak_bytes_in_use"]), "epochs": int(info["epochs"]),
            "max_rel_err_vs_plain_fp64": float(errs.max()),
            "max_rel_err_vs_oracle": max(oerr) if oerr else None,
            "oracle_checked": len(small),
            "alone_vs_mix_max_abs_diff": alone_diff, "alone_vs_mix_sample": len(sample),
            "plain_fp64": plain, "plain_fp64_loosest_within_1e-5": plain_loose,
            "speedup_vs_plain": round(served["solves_per_s"] / speed_base, 3),
            "p99_ratio_plain_over_served": round((plain_loose or plain)["p99_s"] / served["p99_s"], 3)}


def bench_cheb(args, torch, p, k, rc, T0, jac_ms, jac_iters, T_jac):
    """The headline workload with the Chebyshev-accelerated Jacobi preconditioner (degree m: m - 1 extra
    gathers per PCG iteration) against the Jacobi runs of the headline: iterations, run time and the time-to-
    solution ratio, and the final field against the Jacobi field (both stop at rtol 1e-8 in their own norm)."""
    from paper_1905_07622_amd import femheat as fh
    stream = torch.cuda.current_stream().cuda_stream
    out = {"workload": "the headline workload (FP64) with the Chebyshev preconditioner on [hi/30, hi]",
           "jacobi": {"ms_per_run": round(jac_ms, 2), "iterations_per_run": int(jac_iters)}}
    for m in args.cheb_degrees:
        h = fh.Heat(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, k, rc, dirichlet_mask=p.dirichlet_mask, flux_mask=p.flux_mask,
                    flux=p.flux, device_ptrs=True, stream=stream, precond=fh.FEM_PRECOND_CHEBYSHEV, cheb_degree=m,
                    tune_cache=getattr(args, "tune_cache_path", None))
        kw = dict(dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
        h.run(T0, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = h.run(T0, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        h.close()
        its = int(r["total_iters"])
        out[f"degree_{m}"] = {"ms_per_run": round(ms, 2), "iterations_per_run": its,
                              "gathers_per_run": its * m, "speedup_vs_jacobi": round(jac_ms / ms, 3),
                              "MDOF_iter_per_s": round(p.n_nodes * its / ms / 1e3, 1),
                              "rel_l2_vs_jacobi_field": _rel(r["T_final"], T_jac, torch)}
        print(f"chebyshev m={m}: {its} iterations, {ms:.1f} ms (Jacobi {jac_iters}, {jac_ms:.1f} ms)",
              file=sys.stderr, flush=True)
    return out


def bench_laminate(args, torch):
    """The paper's own performance workload (Sec. 5.1, Table 2): the two-layer laminate, 50 Crank-Nicolson
    steps, rtol 1e-6, with the paper's element (six tetrahedra per cube) at the paper's mesh sizes, FP64:
    PCG iterations over the 50 steps beside the paper's totals (its stop rule and guess may differ from the
    readings here), time per iteration and MDOF*iter/s; the hexahedral element on the same grids for
    comparison."""
    from paper_1905_07622_amd import femheat as fh
    from paper_1905_07622_amd import workloads as wl
    stream = torch.cuda.current_stream().cuda_stream
    paper_iters = {30: 287, 60: 344, 90: 567, 120: 780, 150: 1047, 180: 1278}
    rows = []
    for n in args.laminate_sizes:
        row = {"n": n}
        for name, el in (("tet6", fh.FEM_ELEM_TET6), ("hex8", fh.FEM_ELEM_HEX8)):
            p = _to_device(wl.laminate(n, element=el), torch)
            with fh.Heat.from_problem(p, device_ptrs=True, stream=stream) as h:
                kw = dict(dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
                h.run(p.T0, **dict(kw, nsteps=2))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = h.run(p.T0, **kw)
                torch.cuda.synchronize()
                secs = time.perf_counter() - t0
            its = int(r["total_iters"])
            row["dof"] = p.n_nodes
            row[name] = {"iterations": its, "ms_total": round(secs * 1e3, 2),
                         "us_per_iteration": round(secs * 1e6 / max(its, 1), 2),
                         "MDOF_iter_per_s": round(p.n_nodes * its / secs / 1e6, 1)}
        row["paper_fg_dbd_iterations"] = paper_iters.get(n)
        rows.append(row)
        print(f"laminate n={n}: tet6 {row['tet6']['iterations']} it, hex8 {row['hex8']['iterations']} it "
              f"(paper {row['paper_fg_dbd_iterations']})", file=sys.stderr, flush=True)
    return {"workload": "two-layer laminate [-15,15]^2 x [0,10] mm, steel/oxide at x3 = 5, unit flux on x3 = 0, "
                        "50 CN steps dt 0.01, rtol 1e-6, FP64 Jacobi-PCG", "sizes": rows}


def slab_oracle(nthreads):
    """The FP64 oracle over the whole defect-slab run, every step and the
    surface traces kept (run on the host while the GPU does other work)."""
    from oracle import oracle
    from paper_1905_07622_amd import workloads as wl
    p = wl.defect_slab()
    t0 = time.perf_counter()
    r = oracle.run(p, save_every=1, sensor_xyz=p.sensors, nthreads=nthreads)
    r["seconds"] = time.perf_counter() - t0
    r["nthreads"] = nthreads
    return r


def bench_slab(args, torch, fut):
    """The 200x200x25 defect slab (1,050,426 DOF, two layers, 20 defects of
    k = 0.01, 10-step flux pulse, 300 backward-Euler steps, rtol 1e-8) in the
    mixed form with its 16x16 surface sensors: MDOF*iter/s (inner iterations)
    of a run with inputs resident in HBM, and the error of every step's field
    and traces against the FP64 oracle (which ran on the host meanwhile)."""
    from paper_1905_07622_amd import femheat as fh
    from paper_1905_07622_amd import workloads as wl
    p = wl.defect_slab()
    pd = _to_device(p, torch)
    stream = torch.cuda.current_stream().cuda_stream
    sens = torch.tensor(p.sensors, device="cuda")
    with fh.Heat.from_problem(pd, precision=fh.FEM_FP32_FP64DOT, device_ptrs=True, stream=stream) as h:
        kw = dict(dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
        h.run(pd.T0, **dict(kw, nsteps=3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = h.run(pd.T0, save_every=1, sensors=sens, **kw)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
    rate = p.n_nodes * out["total_iters"] / secs / 1e6
    print(f"slab: {rate:.1f} MDOF*iter/s ({out['total_iters']} inner iterations, {secs:.2f} s); waiting for the oracle",
          file=sys.stderr, flush=True)
    T = out["T_saved"].cpu().numpy()
    tr = out["traces"].cpu().numpy()
    ref = fut.result()
    errs = np.linalg.norm(T - ref["T_saved"], axis=1) / np.linalg.norm(ref["T_saved"], axis=1)
    terr = np.linalg.norm(tr - ref["traces"], axis=1) / np.linalg.norm(ref["traces"], axis=1)
    print(f"slab: per-step rel L2 vs oracle max {errs.max():.2e}; oracle {ref['seconds']:.0f} s", file=sys.stderr,
          flush=True)
    return {"workload": f"defect slab {p.nx}x{p.ny}x{p.nz} ({p.n_nodes} DOF), 2 layers k 1/5, 20 defects k 0.01, "
                        f"flux pulse steps 1-10, backward Euler dt=1e-3, {p.nsteps} steps, rtol 1e-8",
            "precision": "mixed", "value": round(rate, 1), "unit": "MDOF*iter/s", "seconds": round(secs, 3),
            "inner_iterations": int(out["total_iters"]),
            "max_rel_l2_vs_fp64_oracle": float(errs.max()), "worst_step": int(errs.argmax()) + 1,
            "rel_l2_vs_oracle_steps_1_10_11_30_300": [float(errs[:10].max()), float(errs[10:30].max()),
                                                      float(errs[-1])],
            "traces_shape": list(tr.shape), "traces_max_rel_l2_vs_oracle": float(terr.max()),
            "oracle_seconds": round(ref["seconds"], 1), "oracle_threads": ref["nthreads"],
            "oracle_iterations": int(ref["iters"].sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--nsteps", type=int, default=200, help="time steps per run (the workload has 200)")
    ap.add_argument("--n", type=int, default=100, help="elements per edge (the workload has 100)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="time without per-kernel HIP events")
    ap.add_argument("--tile", type=int, nargs=3, default=(0, 0, 0))
    ap.add_argument("--pcg-form", choices=["one-kernel", "two-kernel", "one-reduction"], default="two-kernel",
                    help="Algorithm 1 in one kernel per iteration with a grid-wide barrier (FEM_ONE_KERNEL), "
                         "in two kernels (the library's default), or the one-reduction form")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-proposals measurement")
    ap.add_argument("--no-served", action="store_true", help="skip the serving measurement")
    ap.add_argument("--only-extra", action="store_true", help="skip the 1M-DOF headline run")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-form run of the headline workload")
    ap.add_argument("--no-above-mall", action="store_true", help="skip the 201^3-node (DRAM-bound) run")
    ap.add_argument("--no-apply-ab", action="store_true",
                    help="skip the gather vs element-by-element operator comparison")
    ap.add_argument("--no-inverse", action="store_true", help="skip the coefficient-inverse sampling run")
    ap.add_argument("--mall-n", type=int, default=200)
    ap.add_argument("--mall-nsteps", type=int, default=20)
    ap.add_argument("--batch-sims", type=int, default=64)
    ap.add_argument("--batch-n", type=int, default=48)
    ap.add_argument("--batch-nsteps", type=int, default=100)
    ap.add_argument("--batch-precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--loose-rtols", type=float, nargs="*", default=[1e-6, 1e-7])
    ap.add_argument("--serve-requests", type=int, default=220)
    ap.add_argument("--serve-warmup", type=int, default=20, help="leading requests excluded from the statistics")
    ap.add_argument("--serve-load", type=float, default=1.5, help="arrival rate as a multiple of plain capacity")
    ap.add_argument("--serve-rate", type=float, default=0.0, help="fixed arrival rate (0: serve-load x capacity)")
    ap.add_argument("--serve-probe", type=int, default=20, help="requests that choose the loose plain rtol")
    ap.add_argument("--serve-oracle", type=int, default=6, help="served requests of edge <= 64 checked by the oracle")
    ap.add_argument("--no-slab", action="store_true", help="skip the defect-slab run and its oracle")
    ap.add_argument("--cheb-degrees", type=int, nargs="*", default=[2, 3, 4])
    ap.add_argument("--laminate-sizes", type=int, nargs="*", default=[30, 60, 90, 120, 150])
    ap.add_argument("--no-tune", action="store_true", help="use the library's tile rule (no autotuning)")
    ap.add_argument("--tune-cache", default=os.path.join(tempfile.gettempdir(), "femheat_tune.json"),
                    help="tile cache file of the autotuner (tuned on first use of each shape)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 3 times (scale for rocprof FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the solver has no multi-GPU path; "
              "independent simulations would shard across GPUs with no communication.", file=sys.stderr)
        sys.exit(2)

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
    tune_cache = None if args.no_tune else args.tune_cache
    if tune_cache:
        os.makedirs(os.path.dirname(tune_cache), exist_ok=True)
    args.tune_cache_path = tune_cache
    extra = {}
    if args.only_extra:
        if not args.no_batched:
            extra["batched"] = bench_batched(args, torch)
        if not args.no_served:
            extra["served"] = bench_served(args, torch)
        print(json.dumps(extra), flush=True)
        return
    p = wl.lognormal_cube(args.n, seed=2, nsteps=args.nsteps)
    dev = "cuda"
    k = torch.tensor(p.k_e, device=dev)
    rc = torch.tensor(p.rhoc_e, device=dev)
    T0 = torch.tensor(p.T0, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    prec = fh.FEM_FP64 if args.precision == "fp64" else fh.FEM_FP32_FP64DOT
    h = fh.Heat(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, k, rc, dirichlet_mask=p.dirichlet_mask,
                flux_mask=p.flux_mask, flux=p.flux, precision=prec, device_ptrs=True,
                timing=not args.no_timing, tile=tuple(args.tile), stream=stream,
                one_reduction=args.pcg_form == "one-reduction", one_kernel=args.pcg_form == "one-kernel",
                tune_cache=tune_cache)
    run_kw = dict(dt=p.dt, theta=p.theta, nsteps=p.nsteps, rtol=p.rtol)
    tuned = None
    if tune_cache and args.tile == (0, 0, 0):
        # the autotuner times the hot gather's candidate tiles on this grid and installs the fastest
        tuned = h.tune(dt=p.dt, theta=p.theta)
        print(f"tuned tile {tuned}", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        h.run(T0, **run_kw)
        print(f"warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    stats = {"gather_launches": 0, "gather_ms": 0.0, "update_launches": 0, "update_ms": 0.0,
             "replace_launches": 0, "replace_ms": 0.0, "one_kernel_launches": 0}
    last = None
    run_ms = []
    for s in range(args.steps):
        tr = time.perf_counter()
        last = h.run(T0, **run_kw)
        run_ms.append((time.perf_counter() - tr) * 1e3)  # run() returns once its stream has drained
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
    it_steps = last["iters"]
    f_corr = deferred_fraction(it_steps.cpu().numpy() if hasattr(it_steps, "cpu") else it_steps)
    form = args.pcg_form
    if form == "one-kernel" and stats["one_kernel_launches"] == 0:
        form = "two-kernel"  # the launch could not hold every block at once
    single = form != "two-kernel"
    ab = algorithmic_bytes(p.n_nodes, p.n_elems, w, f_corr, form)
    roof = None
    if stats["gather_launches"] and (stats["update_launches"] or single):
        per = {"gather": stats["gather_ms"] / stats["gather_launches"]}
        if stats["update_launches"]:
            per["update"] = stats["update_ms"] / stats["update_launches"]
        dom = max(per, key=lambda kname: stats[kname + "_ms"])
        achieved = ab[dom] / (per[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": committed_traffic(dom, args.precision, form),
                "bytes_per_launch": int(round(ab[dom])), "avg_launch_us": round(per[dom] * 1e3, 3),
                "deferred_update_share": round(f_corr, 4),
                "other_kernels_us": {kname: round(v * 1e3, 3) for kname, v in per.items() if kname != dom},
                # the other iteration kernels on the same footing (algorithmic bytes / event-timed launch)
                "other_kernels": {kname: {"achieved": round(ab[kname] / (v * 1e-3) / 1e9, 1),
                                          "frac": round(ab[kname] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                          "bytes_per_launch": int(round(ab[kname]))}
                                  for kname, v in per.items() if kname != dom and ab.get(kname)}}

    per_iter = algorithmic_bytes(p.n_nodes, p.n_elems, w, f_corr, form)
    iter_bytes = per_iter["gather"] + per_iter["update"]
    runs = {"n": len(run_ms), "median_ms": round(float(np.median(run_ms)), 2),
            "min_ms": round(min(run_ms), 2), "max_ms": round(max(run_ms), 2),
            "effective_gbs": round(iter_bytes * iters / secs / 1e9, 1),
            "effective_gbs_note": "algorithmic bytes of the iteration kernels (direction gather + update) x "
                                  "iterations / wall time; per-step RHS and initial-residual bytes not counted"}
    # the defect slab's FP64 oracle runs on the host from now on, beside the GPU work
    pool = None
    slab_fut = None
    if not args.no_slab:
        import concurrent.futures
        pool = concurrent.futures.ThreadPoolExecutor(1)
        slab_fut = pool.submit(slab_oracle, max(1, min(8, host_cpu()[1] // 2)))
    if args.precision == "fp64" and not args.no_mixed:
        extra["mixed"] = bench_mixed(args, torch, p, k, rc, T0, last["T_final"])
    if not args.no_above_mall:
        extra["above_mall"] = bench_above_mall(args, torch)
    if args.precision == "fp64" and not args.no_apply_ab:
        extra["apply_ab"] = bench_apply_ab(args, torch, p, k, rc)
    if args.precision == "fp64" and not args.no_inverse:
        extra["inverse"] = bench_inverse(args, torch)
    if args.precision == "fp64" and not args.no_apply_ab:
        extra["context"] = bench_context(torch, per_iter["gather"])
    if args.precision == "fp64" and args.cheb_degrees:
        extra["chebyshev"] = bench_cheb(args, torch, p, k, rc, T0, float(np.median(run_ms)), int(last["total_iters"]),
                                        last["T_final"])
    if args.laminate_sizes:
        extra["laminate_tet6"] = bench_laminate(args, torch)
    if not args.no_batched:
        extra["batched"] = bench_batched(args, torch)
    if not args.no_served:
        extra["served"] = bench_served(args, torch)
    if slab_fut is not None:
        extra["slab"] = bench_slab(args, torch, slab_fut)
        pool.shutdown()

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
                   "precision": args.precision, "pcg_form": form,
                   "iterations_per_run": int(last["total_iters"]),
                   "tile": [shape["tile_x"], shape["tile_y"], shape["tile_z"]],
                   "grid_blocks": shape["grid_blocks"], "autotuned": tuned},
        "roofline": roof,
        "runs": runs,
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        it_np = it_steps.cpu().numpy() if hasattr(it_steps, "cpu") else np.asarray(it_steps)
        Tf = last["T_final"]
        line["cpu_baseline"] = cpu_baseline(p, it_np, Tf.cpu().numpy() if hasattr(Tf, "cpu") else Tf)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
