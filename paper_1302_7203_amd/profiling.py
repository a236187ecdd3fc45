"""Summaries of rocprofv3 output for the committed profiles.

Reads the CSV output of three rocprofv3 runs of the same command -- a kernel
trace with statistics, a ``--pmc FETCH_SIZE`` pass and a ``--pmc WRITE_SIZE``
pass -- and produces, per kernel, the average dispatch duration and the HBM
bytes fetched and written per dispatch.  The counters are scaled by what they
read for ``arrow_probe_copy`` (a plain copy of known size that bench.py runs
while measuring the device's peaks): a factor of known bytes / counted bytes
for each direction.  The result also records a hash of the kernel sources;
bench.py reports the traffic only while the sources still hash the same, since
counters taken on other kernels say nothing about these.

    python -m paper_1302_7203_amd.profiling --trace DIR --fetch DIR --write DIR \\
        --copy-bytes N --out profiles/NAME.json --command "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNEL = "k_probe_copy"


def source_hash() -> str:
    """sha256 over the kernel sources (csrc/*.hip, *.hpp, include/arrow.h), in name order."""
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp")))
    files.append(os.path.join(os.path.dirname(HERE), "include", "arrow.h"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(kernel: str) -> str:
    """'void k_root<0, 64, true>(ahd::ProbDesc, ...)' -> 'k_root<0, 64, true>'."""
    s = kernel.replace("void ", "").replace("(anonymous namespace)::", "")
    return s.split("(")[0].strip()


def _one_csv(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return sorted(hits)[0]


def kernel_stats(trace_dir: str) -> dict:
    """name -> {calls, avg_us, total_us} from the kernel-trace statistics."""
    out = {}
    with open(_one_csv(trace_dir, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            out[short_name(r["Name"])] = {"calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                                          "total_us": float(r["TotalDurationNs"]) / 1e3}
    return out


def counter_means(pmc_dir: str, counter: str) -> dict:
    """name -> mean over dispatches of one counter (rocprofv3 sums each dispatch over its dimensions)."""
    acc = defaultdict(list)
    with open(_one_csv(pmc_dir, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize(trace_dir, fetch_dir, write_dir, copy_bytes, command=""):
    stats = kernel_stats(trace_dir)
    fetch = counter_means(fetch_dir, "FETCH_SIZE")
    write = counter_means(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if COPY_KERNEL in k]
    if not copy:
        raise ValueError(f"{COPY_KERNEL} is not in the counter runs: nothing to scale by")
    ck = copy[0]
    f_fetch = copy_bytes / (fetch[ck] * 1024.0)
    f_write = copy_bytes / (write[ck] * 1024.0)
    kernels = {}
    for k, st in stats.items():
        entry = dict(st)
        if k in fetch and k in write:
            entry["fetch_kib"] = fetch[k]
            entry["write_kib"] = write[k]
            entry["hbm_bytes"] = fetch[k] * 1024.0 * f_fetch + write[k] * 1024.0 * f_write
        kernels[k] = entry
    return {"command": command, "source_sha256": source_hash(),
            "copy_probe": {"kernel": ck, "bytes_each_way": copy_bytes, "fetch_kib": fetch[ck],
                           "write_kib": write[ck], "fetch_scale": f_fetch, "write_scale": f_write},
            "kernels": kernels}


def markdown(doc, title, extra=None):
    """A short text summary of `doc` (and of optional extra per-kernel counter columns)."""
    extra = extra or {}
    lines = [f"# {title}", "", "Commands (repository root, one MI355X, `cd /tmp && export TMPDIR=/tmp` first):", ""]
    for c in doc["command"].split(" ;; "):
        lines.append(f"    {c}")
    cp = doc["copy_probe"]
    lines += ["", f"Kernel sources sha256 `{doc['source_sha256'][:16]}…` (bench.py reports traffic only while "
              "the sources match).", "",
              f"Calibration: `{cp['kernel']}` copies {cp['bytes_each_way']} bytes; FETCH_SIZE reads "
              f"{cp['fetch_kib']:.0f} KiB (scale {cp['fetch_scale']:.4f}), WRITE_SIZE {cp['write_kib']:.0f} KiB "
              f"(scale {cp['write_scale']:.4f}).", ""]
    cols = list(extra)
    lines.append("| kernel | calls | avg µs | fetch KiB | write KiB | HBM bytes/launch (scaled) |"
                 + "".join(f" {c} |" for c in cols))
    lines.append("|---|---|---|---|---|---|" + "---|" * len(cols))
    rows = sorted(doc["kernels"].items(), key=lambda kv: -kv[1]["total_us"])
    for name, k in rows:
        f = f"{k['fetch_kib']:.1f}" if "fetch_kib" in k else ""
        w = f"{k['write_kib']:.1f}" if "write_kib" in k else ""
        b = f"{k['hbm_bytes']:.4g}" if "hbm_bytes" in k else ""
        ex = "".join(f" {extra[c].get(name, float('nan')):.4g} |" for c in cols)
        lines.append(f"| {name} | {k['calls']} | {k['avg_us']:.2f} | {f} | {w} | {b} |{ex}")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True, help="bytes arrow_probe_copy read (= wrote)")
    ap.add_argument("--out", required=True, help="JSON summary (read by bench.py)")
    ap.add_argument("--md", help="text summary")
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--extra", action="append", default=[],
                    help="DIR:COUNTER -- add the per-dispatch mean of COUNTER from the pmc run in DIR")
    ap.add_argument("--command", default="", help="the commands that made the runs, joined by ' ;; '")
    a = ap.parse_args(argv)
    doc = summarize(a.trace, a.fetch, a.write, a.copy_bytes, a.command)
    with open(a.out, "w") as f:
        json.dump(doc, f, indent=1)
    if a.md:
        extra = {}
        for spec in a.extra:
            d, c = spec.rsplit(":", 1)
            extra[c] = counter_means(d, c)
        with open(a.md, "w") as f:
            f.write(markdown(doc, a.title, extra))
    print(json.dumps({k: v for k, v in doc["kernels"].items() if "hbm_bytes" in v}, indent=1))


if __name__ == "__main__":
    main()
