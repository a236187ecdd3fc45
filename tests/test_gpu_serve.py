"""The serving loop on the GPU: continuous batching under an HBM budget, results
identical to solving each request alone, and parity with the oracle."""
import numpy as np
import pytest

import oracle
from paper_1302_7203_amd import workloads as W
from parity import assert_close

pytestmark = pytest.mark.gpu


def _stream(count, seed, nmax=400, rate=2000.0):
    reqs = W.serving_requests(count=count, nmin=32, nmax=nmax, rate=rate, seed=seed)
    out = [(t, p) for t, p in reqs]
    # every 6th request becomes a Hermitian arrowhead of the same order (odd and even n)
    rng = np.random.default_rng(seed + 100)
    return [(t, W.herm_arrow(p.n, rng) if i % 6 == 5 else p) for i, (t, p) in enumerate(out)]


def test_served_results_equal_alone_and_oracle(oracle_lib):
    import torch
    from paper_1302_7203_amd import batch, serve
    dev = torch.device("cuda", 0)
    arr = _stream(80, 11)
    biggest = max(serve.request_bytes(p) for _, p in arr)
    srv = serve.Server(hbm_budget=max(6 * biggest, 64 << 20), device=dev, streams=3)
    reqs = srv.run(arr, keep_results=True)
    torch.cuda.synchronize()
    assert all(r.done >= r.arrival for r in reqs)
    assert srv.peak_used <= srv.arena.capacity
    for r in reqs[:: 7] + [r for r in reqs if r.problem.kind == W.KIND_HERM][:3]:
        lam, V, U, info = srv.result(r)
        one = batch.Batch([r.problem], device=dev)
        one.run()
        torch.cuda.synchronize()
        l1, V1, U1, _ = one.result(0)
        assert torch.equal(lam, l1) and torch.equal(V, V1)
        if U is not None:
            assert torch.equal(U, U1)
        one.close()
        pr = r.problem
        if pr.kind == W.KIND_ARROW:
            ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
            rl, rV = ref.lam, ref.vec
        elif pr.kind == W.KIND_DPR1:
            ref = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
            rl, rV = ref.lam, ref.vec
        elif pr.kind == W.KIND_HERM:
            ref = oracle.herm_eig(pr.d, pr.z, pr.scalar)
            rl, rV = ref.lam, ref.vec
        else:
            ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
            rl, rV = ref.sigma, ref.V
            assert_close(U.cpu().numpy(), ref.U, f"request {r.rid} U")
        assert_close(lam.cpu().numpy(), rl, f"request {r.rid} values")
        assert_close(V.cpu().numpy(), rV, f"request {r.rid} vectors")
    srv.close()


def test_tight_budget_forces_waiting_but_finishes():
    import torch
    from paper_1302_7203_amd import serve
    dev = torch.device("cuda", 0)
    arr = [(0.0, p) for _, p in _stream(40, 12, nmax=300)]
    biggest = max(serve.request_bytes(p) for _, p in arr)
    srv = serve.Server(hbm_budget=2 * biggest + (4 << 20), device=dev, streams=2)
    reqs = srv.run(arr)
    assert all(r.done > 0 for r in reqs)
    waited = sum(1 for r in reqs if r.admitted > r.arrival)
    assert waited > 0
    assert srv.arena.used == 0
    srv.close()


def test_batches_overlap_on_the_device():
    """With several streams, batches run at the same time: the batches' device intervals
    (timing events around each batch's kernels) add up to more than the span they cover,
    which a one-at-a-time execution could not do."""
    import torch
    from paper_1302_7203_amd import serve
    dev = torch.device("cuda", 0)
    arr = [(0.0, p) for _, p in _stream(200, 14, nmax=2000)]
    srv = serve.Server(hbm_budget=8 << 30, device=dev, streams=3, max_batch=16, trace=True)
    reqs = srv.run(arr)
    torch.cuda.synchronize(dev)
    assert all(r.done > 0 for r in reqs)
    iv = srv.device_intervals()
    assert len(iv) >= 10 and len({s for _, _, s in iv}) == 3
    busy = sum(b - a for a, b, _ in iv)
    span = max(b for _, b, _ in iv) - min(a for a, _, _ in iv)
    assert busy > 1.2 * span, (busy, span)
    srv.close()
