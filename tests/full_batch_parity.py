"""Every eigenvalue and every eigenvector entry of the 10,000-problem mixed batch (the plan the
benchmark times) against the oracle, at the 1e-13 relative bar.

Not collected by pytest (about ten minutes of oracle time on 16 host threads); run it on a GPU
machine from the repository root:

    python tests/full_batch_parity.py

It prints its progress every 500 problems and, at the end, the worst relative errors and the
number of entries compared; it exits 1 if any entry misses the bar or any reference is not
trusted (oracle relerr above REF_RELERR).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from parity import REF_RELERR, TOL, relerr  # noqa: E402


def main():
    import torch

    from paper_1302_7203_amd import batch, workloads as W

    dev = torch.device("cuda", 0)
    probs = W.batch_mixed()
    b = batch.Batch(probs, device=dev, graph=True)
    b.run()
    torch.cuda.synchronize()
    worst_l = worst_v = 0.0
    entries = 0
    bad = []
    t0 = time.time()
    for p, pr in enumerate(probs):
        lam, V, _, _ = b.result(p)
        ref = (oracle.arrow_eig if pr.kind == W.KIND_ARROW else oracle.dpr1_eig)(pr.d, pr.z, pr.scalar)
        if ref.relerr.size and float(np.max(ref.relerr)) > REF_RELERR:
            bad.append((p, "untrusted reference", float(np.max(ref.relerr))))
        el = relerr(lam.cpu().numpy(), ref.lam)
        ev = relerr(V.cpu().numpy(), ref.vec)
        entries += el.size + ev.size
        wl, wv = float(el.max()), float(ev.max())
        worst_l, worst_v = max(worst_l, wl), max(worst_v, wv)
        if not (wl <= TOL and wv <= TOL):
            bad.append((p, pr.n, wl, wv))
        if (p + 1) % 500 == 0:
            print(f"{p + 1} problems, worst lambda {worst_l:.2e}, V {worst_v:.2e}, {time.time() - t0:.0f} s",
                  flush=True)
    b.close()
    print(f"all {len(probs)} problems ({sum(pr.n for pr in probs)} eigenpairs, {entries} entries): "
          f"worst lambda {worst_l:.3e}, worst V {worst_v:.3e}, bar {TOL:.0e}; misses {len(bad)}", flush=True)
    for x in bad[:20]:
        print("  ", x, flush=True)
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())
