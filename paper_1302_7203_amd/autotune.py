"""Autotuner for the solver's schedule: lanes of a wavefront per eigenvalue.

The kernels let G = 1, 2, 4, ..., 64 lanes cooperate on one eigenvalue (G = 64:
a wavefront per eigenvalue; smaller G: 64/G eigenvalues share a wavefront and
its loads of the pole data, with shorter reductions but longer per-lane
loops).  The best G depends on the order n, on how many eigenvalues are in
flight (one problem, or a whole batch) and on the device, so it is measured:

* single problems: one arrowhead solve (all eigenvalues and vectors) of each
  order in SINGLE_NS, timed for every G;
* batches: a mixed batch (60% arrowhead, 25% DPR1, 15% SVD) of orders drawn
  log-uniformly in each bucket of BATCH_BUCKETS, about BATCH_PAIRS
  eigenpairs in all, one hipGraph-captured plan per G.

The fastest G per size becomes a table entry (n_max, lanes); the tables are
written as JSON (binding.TUNED_PATH by default), and the binding installs them
into every handle it creates through arrow_set_lanes_table.  Results do not
depend on the table beyond rounding: every G meets the same accuracy bar.

    python -m paper_1302_7203_amd.autotune [--out PATH] [--reps 5] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import batch, binding, workloads

SINGLE_NS = [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
LANES_SINGLE = [1, 2, 4, 8, 16, 32, 64]
BATCH_BUCKETS = [(8, 24), (24, 48), (48, 96), (96, 192), (192, 384), (384, 768), (768, 1536), (1536, 3072),
                 (3072, 8192)]
LANES_BATCH = [4, 8, 16, 32, 64]
BATCH_PAIRS = 400_000


def _time(fn, reps, dev):
    fn()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize(dev)
    return (time.perf_counter() - t0) / reps


def tune_single(dev, reps=5, ns=SINGLE_NS, log=print):
    rng = np.random.default_rng(workloads.SEED_BASE + 90)
    meas = {}
    best = []
    for n in ns:
        pr = workloads.uniform_arrow(n, rng)
        d = torch.from_numpy(pr.d).to(dev)
        z = torch.from_numpy(pr.z).to(dev)
        row = {}
        for g in LANES_SINGLE:
            if g > max(1, n):
                continue
            binding.set_option(binding.OPT_LANES, g, device=dev)
            row[g] = _time(lambda: binding.arrow_eig(d, z, pr.scalar), reps, dev) * 1e3
        binding.set_option(binding.OPT_LANES, 0, device=dev)
        g_best = min(row, key=row.get)
        meas[n] = row
        best.append(g_best)
        log(f"single n={n}: " + " ".join(f"G{g}={t:.3f}ms" for g, t in row.items()) + f" -> {g_best}")
    # entry k covers n up to the geometric midpoint between the tuned orders k and k+1
    n_max = [int(math.sqrt(a * b)) for a, b in zip(ns, ns[1:])] + [binding.INT32_MAX]
    return _merge(n_max, best), meas


def _mixed_bucket(lo, hi, pairs, rng):
    out, total = [], 0
    while total < pairs:
        n = int(round(math.exp(rng.uniform(math.log(lo + 1), math.log(hi)))))
        u = rng.uniform()
        pr = (workloads.uniform_arrow(n, rng) if u < 0.60 else workloads.dpr1(n, rng) if u < 0.85
              else workloads.svd_arrow(n, rng))
        out.append(pr)
        total += n
    return out


def tune_batch(dev, reps=3, buckets=BATCH_BUCKETS, pairs=BATCH_PAIRS, log=print):
    rng = np.random.default_rng(workloads.SEED_BASE + 91)
    meas = {}
    best = []
    h = binding.handle(dev)
    for lo, hi in buckets:
        probs = _mixed_bucket(lo, hi, pairs, rng)
        packed = batch.pack(probs)
        row = {}
        for g in LANES_BATCH:
            binding.set_lanes_table(binding.SCHEDULE_BATCH, [binding.INT32_MAX], [g], h=h)
            b = batch.Batch(probs, device=dev, graph=True, packed=packed)
            row[g] = _time(b.run, reps, dev) * 1e3
            b.close()
            del b
        g_best = min(row, key=row.get)
        meas[f"{lo}-{hi}"] = {"problems": len(probs), "eigenpairs": sum(p.n for p in probs), "ms": row}
        best.append(g_best)
        log(f"batch n in ({lo},{hi}] x{len(probs)}: " + " ".join(f"G{g}={t:.2f}ms" for g, t in row.items())
            + f" -> {g_best}")
        torch.cuda.empty_cache()
    binding.set_lanes_table(binding.SCHEDULE_BATCH, [], [], h=h)
    n_max = [hi for _, hi in buckets[:-1]] + [binding.INT32_MAX]
    return _merge(n_max, best), meas


def _merge(n_max, lanes):
    """Drop entries whose successor has the same lanes (the successor's n_max covers them)."""
    out_n, out_g = [], []
    for k, (n, g) in enumerate(zip(n_max, lanes)):
        if k + 1 < len(lanes) and lanes[k + 1] == g:
            continue
        out_n.append(int(n))
        out_g.append(int(g))
    return out_n, out_g


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=binding.TUNED_PATH)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="few sizes and a small batch (a smoke run)")
    args = ap.parse_args(argv)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # measure from the built-in schedule, whatever table is installed
    h = binding.handle(dev)
    binding.set_lanes_table(binding.SCHEDULE_SINGLE, [], [], h=h)
    binding.set_lanes_table(binding.SCHEDULE_BATCH, [], [], h=h)
    log = lambda s: print(s, flush=True)   # noqa: E731
    if args.quick:
        single, ms = tune_single(dev, reps=2, ns=[16, 256], log=log)
        btab, mb = tune_batch(dev, reps=1, buckets=[(24, 48), (192, 384)], pairs=20_000, log=log)
    else:
        single, ms = tune_single(dev, reps=args.reps, log=log)
        btab, mb = tune_batch(dev, reps=max(2, args.reps // 2), log=log)
    props = torch.cuda.get_device_properties(dev)
    doc = {
        "device": getattr(props, "gcnArchName", props.name),
        "device_name": props.name,
        "compute_units": props.multi_processor_count,
        "command": "python -m paper_1302_7203_amd.autotune" + (" --quick" if args.quick else ""),
        "single": {"n_max": single[0], "lanes": single[1]},
        "batch": {"n_max": btab[0], "lanes": btab[1]},
        "measurements_ms": {"single": {str(k): v for k, v in ms.items()}, "batch": mb},
    }
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    binding.read_tuned(args.out)   # validates what was written
    print(json.dumps({"single": doc["single"], "batch": doc["batch"]}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
