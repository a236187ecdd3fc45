#!/usr/bin/env python3
"""Throughput of the accurate arrowhead eigensolver on one MI355X.

Default workload (the batched comparison the metric names): 10,000 independent
problems, n = round(exp U(ln 16, ln 1024)), half arrowhead (d ~ U(-1,1) with
minimum gap 1e-6, z ~ U(0.1,1), alpha ~ U(-1,1)), half diagonal-plus-rank-one
(u = g/|g|, rho ~ U(0.1,10)); every eigenvalue and eigenvector of every
problem, inputs resident in HBM.  A step is one run of the hipGraph-captured
batched plan over all of them; the same problems solved with one launch
sequence per problem are timed beside it.  --workload selects a single large
problem instead (the graded n = 4096 arrowhead, uniform n = 16384 or n = 512),
where a step is one full solve.

Prints one JSON line.  Besides the throughput it reports, from HIP events
stamped by the kernels' own dispatches, the duration of each kernel and the
roofline position of the dominant kernel (the root stage, bound by FP64 vector
ALU work) and of the vector kernel (bound by HBM writes), the single graded
n = 4096 solve, the serving loop and the extensions as further legs, and a
bounded sample of the workload solved by the CPU oracle on the host cores,
against which the GPU outputs are checked at the 1e-13 relative bar.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "eigenpairs/s (FP64, rel err≤1e-13) batched vs per-solve launch; p99 latency"

# MI355X published peaks
PEAK_FP64_VECTOR = 78.6e12      # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_HBM = 8.0e12               # bytes/s

# Algorithmic FP64 operations per pole term of each O(n) pass, read off the
# kernel bodies (solver.hpp): +, -, * and a reciprocal count 1, an FMA 2;
# max and abs are not counted.
F_BISECT = 7      # bisection step: e = d_j - d_i (1), fma(-nu, e, 1) (2), e*(.) (1), 1/(.) (1), fma(c_j, ., S) (2)
F_RATIONAL = 14   # rational step: e (1), fma(nu, e, -1) (2), e*(.) (1), 1/(.) (1), v = e q (1), fma(c_j, q, .) (2),
                  # (c_j v) v (2), sum (1), e v (1), fma(d1, e v, .) (2)
F_SELECT = 5      # shift selection: (d_j - d_k) - mid (2), 1/(.) (1), fma(c_j, ., s) (2)
F_DD = 28         # b in double-double: e (1), 1/e (1), the rest of TwoSum(d_j, -d_i) (5), two-digit quotient
                  # (q1 1, TwoProd 3, remainder 5, second digit 1), TwoSum accumulate (8), the upper
                  # bracket end's sum of zeta_j^2 / e_j^2: (1/e)^2 (1), fma (2)
F_NORM = 7        # eigenvector norm: (e_j - s) - mu (3), 1/(.) (1), c_j r (1), fma(., r, acc) (2)

# The roofline's algorithmic work is the hot-path scope's per-unit figure: an eigenpair of an
# order-n problem costs m (48 + 3 I) flops, m = n - 1 pole terms per pass and I its root-finding
# passes (counted by the kernels), a divide counted as one flop -- 4 + 4 for the shift
# selection and the bracket, 40 for b in double-double, 3 per term of each root pass.  The
# per-term recount above (every operation of the passes actually run) is reported beside it.
W_FIXED, W_ITER = 48, 3
ROOF_UNIT = "flops per eigenpair m (48 + 3 I): m = n - 1 pole terms per pass, I = root passes (kernel counters)"

BATCH_DESC = ("10,000 problems in one plan: n = round(exp U(ln16, ln1024)); even: arrowhead (d~U(-1,1) min gap "
              "1e-6, z~U(0.1,1), alpha~U(-1,1)), odd: DPR1 (d as above, u = g/|g|, rho~U(0.1,10)); all eigenvalues "
              "+ vectors (9.6 GB)")

WORKLOADS = {
    "batch_mixed": (BATCH_DESC, "batch_mixed"),
    "graded_4096": ("single graded arrowhead n=4096: |d| log-uniform [1e-10,1e10] with random signs "
                    "+ 64 clusters of 8 poles (relative gaps ~1e-12), z log-uniform [1e-8,1], alpha=1e-3; "
                    "all eigenvalues + full V (128 MiB)", "single_graded_4096"),
    "uniform_512": ("single arrowhead n=512: d~U(-1,1) min gap 1e-6, z~U(0.1,1), alpha~U(-1,1); "
                    "all eigenvalues + full V", "single_uniform_512"),
    "uniform_16384": ("single arrowhead n=16384: d~U(-1e4,1e4) min gap 1e-6, z~U(0.1,1), alpha~U(-1,1); "
                      "all eigenvalues + full V (2 GiB)", "single_uniform_16384"),
}


def profiled_traffic(workload, prefix):
    """HBM bytes per launch of the kernel whose name starts with `prefix`, from the committed
    rocprofv3 counter summary of this workload (FETCH_SIZE + WRITE_SIZE, scaled by the copy
    probe); None when there is none or the kernel sources changed since it was taken."""
    from paper_1302_7203_amd import profiling

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    if doc.get("source_sha256") != profiling.source_hash():
        return None
    for name, k in doc["kernels"].items():
        if name.startswith(prefix) and "hbm_bytes" in k:
            return k["hbm_bytes"]
    return None


def measured_peaks(binding, dev):
    """What the device sustains: FP64 FMA issue (arrow_probe_fma), 16-byte streaming stores
    (arrow_probe_fill, 2 GiB) and a plain copy (arrow_probe_copy, 1 GiB each way), each the best
    of 5 launches timed with HIP events on torch's current stream."""
    import ctypes

    import torch

    L = binding.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count

    def best(fn, reps=5):
        fn()
        t = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            t.append(a.elapsed_time(b) * 1e-3)
        return min(t)

    blocks, iters = cus * 32, 4096
    out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    t_fma = best(lambda: binding._check(L.arrow_probe_fma(ctypes.c_void_p(out.data_ptr()), blocks, iters, st),
                                        "arrow_probe_fma"))
    fill_bytes = 2 << 30
    buf = torch.empty(fill_bytes // 8, dtype=torch.float64, device=dev)
    t_fill = best(lambda: binding._check(L.arrow_probe_fill(ctypes.c_void_p(buf.data_ptr()), fill_bytes, 1.0, st),
                                         "arrow_probe_fill"))
    half = fill_bytes // 2
    src, dst = buf[: half // 8], buf[half // 8:]
    t_copy = best(lambda: binding._check(L.arrow_probe_copy(ctypes.c_void_p(dst.data_ptr()),
                                                            ctypes.c_void_p(src.data_ptr()), half, st),
                                         "arrow_probe_copy"))
    del out, buf, src, dst
    torch.cuda.empty_cache()
    return {"fp64_fma_tflops": blocks * 256 * iters * 16 / t_fma / 1e12,
            "store_gbs": fill_bytes / t_fill / 1e9,
            "copy_gbs": 2 * half / t_copy / 1e9,
            "how": "arrow_probe_fma (8 FMA chains/lane), arrow_probe_fill (2 GiB, 16-B non-temporal stores), "
                   "arrow_probe_copy (1 GiB read + 1 GiB write); best of 5, HIP events"}


def batched_headline(args, workloads, dev, steps, cpu=True):
    """The metric's workload: 10,000 problems of uneven order in one hipGraph-captured plan (the
    timed steps), the same plan's kernels timed by their own dispatch events over further eager
    runs, the algorithmic work from the plan's pass counters, and the same problems solved with
    one launch sequence per problem."""
    import numpy as np
    import torch

    from paper_1302_7203_amd import batch

    probs = workloads.batch_mixed()
    pairs = sum(p.n for p in probs)
    g = batch.Batch(probs, device=dev, graph=not args.no_graph)
    for _ in range(max(1, args.warmup)):
        g.run()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        g.run()
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t0
    # the plan's five kernels, each timed by the events its dispatch stamps
    tp = batch.Batch(probs, device=dev, timing=True)
    tp.run()
    stages = np.zeros(5)
    for _ in range(args.timing_runs):
        tp.run()
        stages += np.array(tp.timing())
    stages /= max(1, args.timing_runs)
    cnt = tp.counters()
    same_eager = bool(torch.equal(tp.out_pool, g.out_pool))
    info = tp.info_pool.cpu().numpy().astype(np.uint32)
    info_counts = {name: int(np.sum((info & bit) != 0)) for name, bit in
                   (("dd_b", 1), ("remedy_a", 2), ("remedy_b", 4), ("near_zero", 8), ("pole_shift", 512),
                    ("not_solved", 304))}
    tp.close()
    del tp
    torch.cuda.empty_cache()
    # one launch sequence per problem, on the same stream
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    g.run_sequential()
    torch.cuda.synchronize(dev)
    t_seq = time.perf_counter() - t0
    out = g.out_pool.clone()          # the sequential results, for the comparison below
    g.run()
    torch.cuda.synchronize(dev)
    f_iter = F_RATIONAL if args.root == "rational" else F_BISECT
    recount = f_iter * cnt["root_iter_terms"] + F_DD * cnt["root_dd_terms"] + F_SELECT * cnt["root_plain_terms"]
    root_flops = W_FIXED * float(sum(p.n * (p.n - 1) for p in probs)) + W_ITER * cnt["root_iter_terms"]
    t_root = stages[1] * 1e-3
    roof = {"kernel": "k_b_root (root stage)", "bound": "alu", "achieved": root_flops / t_root / 1e12,
            "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s", "traffic": profiled_traffic("batch_mixed", "k_b_root"),
            "flops_per_launch": root_flops, "per_unit": ROOF_UNIT,
            "recount": {"flops_per_launch": recount, "achieved": recount / t_root / 1e12,
                        "frac": recount / t_root / PEAK_FP64_VECTOR}}
    roof["frac"] = roof["achieved"] / roof["peak"]
    vec_bytes = float(sum(8.0 * p.n * p.n + 16.0 * p.n for p in probs))
    roof_v = {"kernel": "k_b_vec", "bound": "hbm", "achieved": vec_bytes / (stages[4] * 1e-3) / 1e9,
              "peak": PEAK_HBM / 1e9, "unit": "GB/s", "traffic": profiled_traffic("batch_mixed", "k_b_vec"),
              "bytes_per_launch": vec_bytes}
    roof_v["frac"] = roof_v["achieved"] / roof_v["peak"]
    res = {"value": pairs * steps / elapsed, "ms_per_step": elapsed / steps * 1e3, "steps": steps,
           "config": {"workload": BATCH_DESC, "problems": len(probs), "eigenpairs_per_step": pairs,
                      "parallelism": "single GPU", "schedule": "persistent work queues" +
                      (", hipGraph-captured plan" if not args.no_graph else ", eager launches"),
                      "root_finder": args.root},
           "stages_ms": {k: float(v) for k, v in zip(("prologue", "root", "check", "repair", "vectors"), stages)},
           "stage_timing": {"runs": args.timing_runs,
                            "how": "an eager plan of the same problems whose five kernels stamp HIP events by their "
                                   "own dispatches (hipExtLaunchKernel) on the plan's stream; its outputs are "
                                   "bitwise those of the timed graph plan: " + str(same_eager)},
           "counters": cnt, "info_counts": info_counts, "roofline": roof, "roofline_vector": roof_v,
           "per_solve_launch": {"ms": t_seq * 1e3, "eigenpairs_per_s": pairs / t_seq,
                                "how": "arrow_solve_sequential: the single-problem launch sequence per problem, "
                                       "back to back on the same stream"}}
    res["vs_per_solve_launch"] = res["value"] / res["per_solve_launch"]["eigenpairs_per_s"]
    if cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
        oracle.build(force=False)
        sample = list(range(0, len(probs), args.cpu_every))
        worst_l = worst_v = 0.0
        spairs = 0
        t_cpu = 0.0
        for p in sample:
            pr = probs[p]
            t1 = time.perf_counter()
            ref = (oracle.arrow_eig if pr.kind == 0 else oracle.dpr1_eig)(pr.d, pr.z, pr.scalar, threads=threads)
            t_cpu += time.perf_counter() - t1
            spairs += pr.n
            lam, V, _, _ = g.result(p)
            worst_l = max(worst_l, float(np.max(np.abs(lam.cpu().numpy() - ref.lam) / np.abs(ref.lam))))
            worst_v = max(worst_v, float(np.max(np.abs(V.cpu().numpy() - ref.vec) / np.abs(ref.vec))))
        res["cpu_baseline"] = {"value": spairs / t_cpu, "unit": "eigenpairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"every {args.cpu_every}th problem of the same 10,000 ({len(sample)} problems, "
                                         f"{spairs} eigenpairs, every eigenvalue and eigenvector), binary128 oracle, "
                                         f"{t_cpu:.1f} s wall"}
        res["parity"] = {"sample_problems": len(sample), "sample_eigenpairs": spairs, "max_rel_err_lambda": worst_l,
                         "max_rel_err_V": worst_v, "tolerance": 1e-13,
                         "pass": bool(worst_l <= 1e-13 and worst_v <= 1e-13)}
        # the one-launch-per-problem results agree to rounding (other sums' order), checked on the same sample
        wl = 0.0
        for p in sample:
            D = g.packed.descs[p]
            a = out[D.lam_off:D.lam_off + D.n]
            b = g.out_pool[D.lam_off:D.lam_off + D.n]
            wl = max(wl, float(torch.max(torch.abs(a - b) / torch.abs(b)).item()))
        res["per_solve_launch"]["max_rel_diff_lambda_vs_batched"] = wl
    g.close()
    del g, out
    torch.cuda.empty_cache()
    return res


SERVE_DESC = ("Poisson stream, n = round(exp U(ln32, ln8192)); 60% arrowhead eigen (d~U(-1,1) min gap 1e-6, "
              "z~U(0.1,1)), 25% DPR1 eigen (rho~U(0.1,10), u = g/|g|), 15% SVD of an upper-triangular arrowhead "
              "(d~U(0,1), z~U(0.1,1)); all values + vectors; admission by an HBM budget")


def serving_leg(args, dev):
    """The serving loop: saturated capacity (batched, and one launch per request), then a
    Poisson stream offered at a fixed fraction of that capacity, with p50/p99 latency.
    Sampled requests of the offered-load run are checked against the oracle."""
    import numpy as np
    import torch

    from paper_1302_7203_amd import serve, workloads

    arr = workloads.serving_requests(count=args.serve_requests, nmin=32, nmax=8192, rate=1.0)
    probs = [p for _, p in arr]
    budget = int(args.serve_budget_gib * (1 << 30))
    pairs = sum(p.n for p in probs)

    rng = np.random.default_rng(5)
    check_rids = sorted(int(i) for i in rng.choice(len(probs), 8, replace=False)) if not args.no_cpu_baseline else []
    got = {}

    def grab(srv, r):
        # the sampled requests are served again after the timed runs (each request's results
        # are the same in any batch): reading results back inside the loop would stall it
        rid = check_rids[r.rid]
        lam, V, U, info = srv.result(r)
        n = r.problem.n
        ks = np.unique(np.linspace(0, n - 1, min(n, 16)).astype(np.int64))
        kt = torch.from_numpy(ks).to(dev)
        got[rid] = (ks, lam[kt].cpu().numpy(), V[:, kt].cpu().numpy(),
                    None if U is None else U[:, kt].cpu().numpy())

    # the process holds the other legs' data (10,000 problems and their results): a full
    # collection of that heap during the 0.1-s stream stalls the loop for tens of ms, so the
    # heap is collected once and frozen out of the collector for the serving runs
    import gc
    gc.collect()
    gc.freeze()
    srv = serve.Server(hbm_budget=budget, device=dev, streams=4, max_batch=args.serve_max_batch, split_n=2048)
    srv.run([(0.0, p) for p in probs[:200]])                     # warm-up
    torch.cuda.synchronize(dev)
    sat = serve.latency_stats(srv.run([(0.0, p) for p in probs]))
    l0 = srv.launches
    rate = args.serve_load * sat["solves_per_s"]
    # the stream lasts about 0.1 s, so its p99 (its 20 slowest requests) turns on a burst or
    # two: it is offered several times and the run with the median p99 is reported, every
    # run's p50 and p99 beside it
    runs = [serve.latency_stats(srv.run([(t / rate, p) for t, p in arr])) for _ in range(max(1, args.serve_repeats))]
    st = sorted(runs, key=lambda r: r["p99_ms"])[len(runs) // 2]
    launches = (srv.launches - l0) / len(runs)
    peak = srv.peak_used
    if check_rids:
        srv.on_done = grab
        srv.run([(0.0, probs[i]) for i in check_rids])
    srv.close()
    del srv
    torch.cuda.empty_cache()

    one = serve.Server(hbm_budget=budget, device=dev, streams=1, max_batch=1)
    one.run([(0.0, p) for p in probs[:16]])
    per_solve = serve.latency_stats(one.run([(0.0, p) for p in probs]))
    one.close()
    del one
    torch.cuda.empty_cache()
    gc.unfreeze()

    res = {"workload": SERVE_DESC, "requests": len(probs), "eigenpairs": pairs, "hbm_budget_gib": args.serve_budget_gib,
           "max_batch": args.serve_max_batch,
           "saturated_batched": {k: sat[k] for k in ("solves_per_s", "eigenpairs_per_s", "wall_s")},
           "saturated_per_solve_launch": {k: per_solve[k] for k in ("solves_per_s", "eigenpairs_per_s", "wall_s")},
           "speedup_vs_per_solve": sat["eigenpairs_per_s"] / per_solve["eigenpairs_per_s"],
           "offered_load": args.serve_load, "offered_solves_per_s": rate,
           "achieved_solves_per_s": st["solves_per_s"], "achieved_eigenpairs_per_s": st["eigenpairs_per_s"],
           "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
           "repeats": len(runs), "p50_ms_runs": [round(r["p50_ms"], 3) for r in runs],
           "p99_ms_runs": [round(r["p99_ms"], 3) for r in runs],
           "latency_parts_ms": {k: round(v, 4) for k, v in st.items()
                                if k.startswith(("admit_wait", "launch_wait", "device"))},
           "slowest_1pct_mean_n": st["n_mean_slowest_1pct"], "streams": 4, "aging_ms": 20.0, "split_n": 2048,
           "launches": launches, "mean_batch": len(probs) / max(1, launches), "peak_arena_gib": peak / (1 << 30)}
    if got:
        import oracle
        worst_l = worst_v = 0.0
        for rid, (ks, lam, V, U) in got.items():
            pr = probs[rid]
            if pr.kind == 2:
                ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar, ks=ks)
                rl, rV = ref.sigma, ref.V
                worst_v = max(worst_v, float(np.max(np.abs(U - ref.U) / np.abs(ref.U))))
            else:
                ref = (oracle.arrow_eig if pr.kind == 0 else oracle.dpr1_eig)(pr.d, pr.z, pr.scalar, ks=ks)
                rl, rV = ref.lam, ref.vec
            worst_l = max(worst_l, float(np.max(np.abs(lam - rl) / np.abs(rl))))
            worst_v = max(worst_v, float(np.max(np.abs(V - rV) / np.abs(rV))))
        res["parity"] = {"sample_requests": len(got), "eigenpairs_each": "16 evenly spaced (all if n<16)",
                         "max_rel_err_values": worst_l, "max_rel_err_vectors": worst_v,
                         "pass": bool(worst_l <= 1e-13 and worst_v <= 1e-13)}
    return res


def sampled_steps(step, steps, every, dev):
    """Run `steps` calls of `step` back to back between two synchronisations and
    return (mean stage times in ms, info).  Every `every`-th call records the
    stage events (stamped by the kernels' own dispatches); its stages are read
    once the following call is queued, so the stream never drains and the
    untimed calls run without the events' dispatch gaps."""
    import numpy as np
    import torch

    from paper_1302_7203_amd import binding

    stages = np.zeros(5)
    nsamp = 0
    pending = False
    last = None
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for s in range(steps):
        timed = s % every == 0
        if timed:
            binding.set_option(binding.OPT_TIMING, 1)
        last = step()
        if timed:
            binding.set_option(binding.OPT_TIMING, 0)
        if pending:
            stages += np.array(binding.timing_of(1 if timed else 0))
            nsamp += 1
        pending = timed
    if pending:
        stages += np.array(binding.timing_of(0))
        nsamp += 1
    torch.cuda.synchronize(dev)
    el = time.perf_counter() - t0
    return stages / max(nsamp, 1), {"elapsed_s": el, "sampled_steps": nsamp, "last": last}


def extensions_leg(args, binding, workloads, dev):
    """The solver's extensions at n = 4096, each timed like the main workload (inputs resident,
    HIP-event stage times): a Hermitian arrowhead (Sec. 6.1; complex vectors, 16 bytes per entry),
    a reducible arrowhead deflated on the device (Sec. 1), a DPR1 matrix with rho < 0, and the
    divide-and-conquer tridiagonal solver built on the DPR1 merge.  Throughput (and the vector
    phase's HBM rate) only; their parity is checked by the GPU tests on the same generators."""
    import numpy as np
    import torch
    rng = np.random.default_rng(workloads.SEED_BASE + 7)
    n = 4096
    herm = workloads.herm_arrow(n, rng)
    red = workloads.reducible_arrow(n, rng, zero_frac=0.1, repeat_every=13)
    neg = workloads.dpr1(n, rng)
    cases = {
        "hermitian_4096": (lambda d, z: binding.arrow_eig_herm(d, z, herm.scalar), herm, 16.0,
                           "Hermitian arrowhead, uniform poles shuffled, z = r e^{i theta}, r~U(0.1,1); complex U"),
        "reducible_4096": (lambda d, z: binding.arrow_eig(d, z, red.scalar), red, 8.0,
                           "uniform arrowhead shuffled with 10% z_j = 0 and every 13th pole repeated, deflated"),
        "dpr1_negative_4096": (lambda d, z: binding.dpr1_eig(d, z, -neg.scalar), neg, 8.0,
                               "D + rho u u^T with rho = -U(0.1,10), u = g/||g||"),
    }
    out = {}
    steps = max(5, args.steps // 2)
    for name, (solve, pr, entry_bytes, desc) in cases.items():
        d = torch.from_numpy(pr.d).to(dev)
        z = torch.from_numpy(np.ascontiguousarray(pr.z)).to(dev)
        for _ in range(2):
            res = solve(d, z)
        st, sampled = sampled_steps(lambda: solve(d, z), steps, max(1, args.timing_every), dev)
        el = sampled["elapsed_s"]
        res = sampled["last"]
        info = res.info.cpu().numpy().astype(np.uint32)
        out[name] = {"workload": desc, "n": n, "steps": steps, "value": n * steps / el, "unit": "eigenpairs/s",
                     "ms_per_step": el / steps * 1e3,
                     "stages_ms": {k: float(v) for k, v in zip(("front", "sort", "root", "check", "vectors"), st)},
                     "vector_hbm_gbs": entry_bytes * n * n / (st[4] * 1e-3) / 1e9,
                     "vector_hbm_frac": entry_bytes * n * n / (st[4] * 1e-3) / PEAK_HBM,
                     "deflated": int(np.sum((info & 1024) != 0)),
                     "not_solved": int(np.sum((info & 304) != 0))}
    # divide-and-conquer tridiagonal solve (synchronous: its allocations, the host
    # planning of every tree level and the rocBLAS GEMMs are inside the time)
    a = torch.from_numpy(rng.uniform(-1.0, 1.0, n)).to(dev)
    b = torch.from_numpy(rng.uniform(-1.0, 1.0, n - 1)).to(dev)
    res = binding.tridiag_eig(a, b)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(3):
        res = binding.tridiag_eig(a, b)
    torch.cuda.synchronize(dev)
    el = (time.perf_counter() - t0) / 3

    def gemm_flops(lo, hi):   # Q = diag(Q1, Q2) Qh at every merge, 2 m n k each
        if hi - lo < 2:
            return 0.0
        mid = lo + (hi - lo) // 2
        s, sl, sr = hi - lo, mid - lo, hi - mid
        return 2.0 * s * (sl * sl + sr * sr) + gemm_flops(lo, mid) + gemm_flops(mid, hi)
    gf = gemm_flops(0, n)
    info = res.info.cpu().numpy().astype(np.uint32)
    out["tridiag_4096"] = {"workload": "symmetric tridiagonal, a, b ~ U(-1,1), divide and conquer with batched DPR1 "
                                       "merges and FP64 GEMM updates", "n": n, "steps": 3,
                           "value": n / el, "unit": "eigenpairs/s", "ms_per_step": el * 1e3,
                           "gemm_flops": gf, "gemm_tflops_over_whole_solve": gf / el / 1e12,
                           "deflated_at_top": int(np.sum((info & 1024) != 0))}
    return out


def single_run(args, workload, binding, workloads, dev, steps, cpu=True):
    """One large problem (graded n = 4096, uniform n = 16384 or n = 512): `steps` full solves back
    to back, the stage events stamped on every k-th one, the root and vector kernels' rooflines,
    and (cpu) a bounded oracle sample that also checks the outputs."""
    import numpy as np
    import torch

    desc, gen = WORKLOADS[workload]
    pr = getattr(workloads, gen)()
    n = pr.n
    d = torch.from_numpy(pr.d).to(dev)
    z = torch.from_numpy(pr.z).to(dev)
    torch.cuda.synchronize(dev)
    for _ in range(max(1, args.warmup)):
        out = binding.arrow_eig(d, z, pr.scalar)
    torch.cuda.synchronize(dev)
    stages, sampled = sampled_steps(lambda: binding.arrow_eig(d, z, pr.scalar), steps,
                                    max(1, args.timing_every), dev)
    elapsed = sampled["elapsed_s"]
    out = sampled["last"]
    cnt = binding.last_counters()
    m = n - 1
    f_iter = F_RATIONAL if args.root == "rational" else F_BISECT
    recount = m * (f_iter * cnt["root_bisect"] + F_DD * cnt["root_dd"] + F_SELECT * cnt["root_plain"])
    root_flops = m * (W_FIXED * float(n) + W_ITER * cnt["root_bisect"])
    t_root = stages[2] * 1e-3
    roof = {"kernel": "k_root", "bound": "alu", "achieved": root_flops / t_root / 1e12,
            "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s", "traffic": profiled_traffic(workload, "k_root<"),
            "flops_per_launch": root_flops, "per_unit": ROOF_UNIT,
            "recount": {"flops_per_launch": recount, "achieved": recount / t_root / 1e12,
                        "frac": recount / t_root / PEAK_FP64_VECTOR}}
    roof["frac"] = roof["achieved"] / roof["peak"]
    vec_bytes = 8.0 * n * n + 16.0 * n
    roof_v = {"kernel": "k_vec", "bound": "hbm", "achieved": vec_bytes / (stages[4] * 1e-3) / 1e9,
              "peak": PEAK_HBM / 1e9, "unit": "GB/s", "traffic": profiled_traffic(workload, "k_vec<"),
              "bytes_per_launch": vec_bytes}
    roof_v["frac"] = roof_v["achieved"] / roof_v["peak"]
    res = {"value": n * steps / elapsed, "unit": "eigenpairs/s", "steps": steps,
           "ms_per_step": elapsed / steps * 1e3,
           "config": {"workload": desc, "n": n, "problems_per_step": 1, "parallelism": "single GPU",
                      "root_finder": args.root},
           "stages_ms": {k: float(v) for k, v in zip(("front", "sort", "root", "check", "vectors"), stages)},
           "stage_timing": {"sampled_steps": sampled["sampled_steps"], "every": max(1, args.timing_every),
                            "how": "HIP events stamped by the kernels' own dispatches (hipExtLaunchKernel) on the "
                                   "solve's stream, on every k-th timed step; root and vectors are the kernels' "
                                   "durations"},
           "counters": cnt, "roofline": roof, "roofline_vector": roof_v}
    info = out.info.cpu().numpy().astype(np.uint32)
    res["info_counts"] = {name: int(np.sum((info & bit) != 0)) for name, bit in
                          (("dd_b", 1), ("remedy_a", 2), ("remedy_b", 4), ("near_zero", 8), ("not_solved", 304))}
    if cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
        step = max(1, n // args.cpu_sample)
        ks = np.arange(0, n, step, dtype=np.int64)[: args.cpu_sample]
        oracle.build(force=False)
        t0 = time.perf_counter()
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks, threads=threads)
        t_cpu = time.perf_counter() - t0
        res["cpu_baseline"] = {
            "value": ks.size / t_cpu, "unit": "eigenpairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{ks.size} of {n} eigenpairs (every {step}th, eigenvalue + full eigenvector) of the "
                      f"same workload, binary128 oracle, {t_cpu:.1f} s wall"}
        Vs = out.V[:, torch.from_numpy(ks).to(dev)].cpu().numpy()
        el = np.abs(out.lam.cpu().numpy()[ks] - ref.lam) / np.abs(ref.lam)
        ev = np.abs(Vs - ref.vec) / np.abs(ref.vec)
        res["parity"] = {"sample_eigenpairs": int(ks.size), "max_rel_err_lambda": float(el.max()),
                         "max_rel_err_V": float(ev.max()), "tolerance": 1e-13,
                         "pass": bool(el.max() <= 1e-13 and ev.max() <= 1e-13)}
    del out, d, z
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 batched runs, or 40 single solves)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--timing-every", type=int, default=10,
                    help="single solves: record the stage events on every k-th timed step (each event adds a "
                         "dispatch gap)")
    ap.add_argument("--timing-runs", type=int, default=3, help="batched: eager runs whose kernels are timed")
    ap.add_argument("--workload", default="batch_mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--no-graph", action="store_true", help="batched: time eager launches instead of the graph")
    ap.add_argument("--cpu-sample", type=int, default=512,
                    help="single solves: eigenpairs the oracle solves for the CPU baseline")
    ap.add_argument("--cpu-every", type=int, default=50, help="batched: the oracle solves every k-th problem")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--root", default="rational", choices=["rational", "bisect"],
                    help="root finder for the extreme eigenvalue of the shifted inverse")
    ap.add_argument("--no-single", action="store_true", help="batched headline: skip the single n=4096 solve leg")
    ap.add_argument("--single-steps", type=int, default=40)
    ap.add_argument("--no-batch", action="store_true", help="single headline: skip the batched leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop leg")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.7, help="offered load as a fraction of saturated capacity")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-max-batch", type=int, default=4096, help="most requests one launch may take")
    ap.add_argument("--serve-repeats", type=int, default=3,
                    help="offered-load runs of the same stream; the one with the median p99 is reported")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the Hermitian / reducible / rho < 0 legs")
    ap.add_argument("--no-peaks", action="store_true", help="skip the calibration kernels")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (every eigenpair and every "
              f"problem is independent: the work would shard by whole problems, or by eigenvalue ranges of one "
              f"problem, with no collective on the solve path)", file=sys.stderr)
        sys.exit(2)
    batched = args.workload == "batch_mixed"
    if args.steps is None:
        args.steps = 20 if batched else 40

    import torch

    from paper_1302_7203_amd import binding, workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    binding.set_option(binding.OPT_ROOT, binding.ROOT_RATIONAL if args.root == "rational" else binding.ROOT_BISECT)
    binding.set_option(binding.OPT_TIMING, 0)

    head = batched_headline(args, workloads, dev, args.steps, cpu=not args.no_cpu_baseline) if batched else \
        single_run(args, args.workload, binding, workloads, dev, args.steps, cpu=not args.no_cpu_baseline)
    result = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head.pop("config"),
    }
    head.pop("unit", None)
    head.pop("steps", None)
    result.update(head)
    if not args.no_peaks:
        peaks = measured_peaks(binding, dev)
        result["measured_peaks"] = peaks
        result["roofline"]["frac_of_measured"] = result["roofline"]["achieved"] / peaks["fp64_fma_tflops"]
        result["roofline_vector"]["frac_of_measured"] = result["roofline_vector"]["achieved"] / peaks["store_gbs"]
    if batched and not args.no_single:
        result["single_graded_4096"] = single_run(args, "graded_4096", binding, workloads, dev, args.single_steps,
                                                  cpu=not args.no_cpu_baseline)
    if not batched and not args.no_batch:
        result["batched"] = batched_headline(args, workloads, dev, 5, cpu=False)
    if not args.no_serve:
        result["serving"] = serving_leg(args, dev)
    if not args.no_extensions:
        result["extensions"] = extensions_leg(args, binding, workloads, dev)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
