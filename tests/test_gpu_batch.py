"""Batched plans (arrow_batch_*) and the sequential reference path against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1302_7203_amd import workloads as W
from parity import assert_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1302_7203_amd import batch, binding
    assert torch.cuda.is_available()
    binding.lib()
    return torch, batch, torch.device("cuda", 0)


def _mixed(count, seed, nmin=16, nmax=300):
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        k = p % 3
        out.append(W.uniform_arrow(n, rng) if k == 0 else W.dpr1(n, rng) if k == 1 else W.svd_arrow(n, rng))
    # a graded problem, two reducible ones (deflated, Sec. 1) and the edge orders
    out.append(W.graded_arrow(200, rng, clusters=4, cluster_size=8))
    out.append(W.reducible_arrow(40, rng))
    out.append(W.reducible_arrow(150, rng, zero_frac=0.3, repeat_every=4))
    neg = W.dpr1(120, rng)          # rho < 0
    neg.scalar = -neg.scalar
    out.append(neg)
    out += [W.herm_arrow(33, rng), W.herm_arrow(90, rng)]   # Hermitian (Sec. 6.1)
    inc = W.uniform_arrow(77, rng)                          # poles in increasing order
    inc.d, inc.z = inc.d[::-1].copy(), inc.z[::-1].copy()
    out.append(inc)
    # spectra spread over 250 decades: eigenvalues within 1e-240 of their poles
    out += [W.wide_arrow(W.KIND_ARROW, 180, rng, 250), W.wide_arrow(W.KIND_DPR1, 120, rng, 250),
            W.wide_arrow(W.KIND_SVD, 90, rng, 250)]
    out += [W.uniform_arrow(1, rng), W.uniform_arrow(2, rng), W.dpr1(1, rng), W.svd_arrow(2, rng)]
    return out


def _oracle(pr):
    if pr.kind == W.KIND_ARROW:
        r = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
        return r.lam, r.vec, None
    if pr.kind == W.KIND_DPR1:
        r = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
        return r.lam, r.vec, None
    if pr.kind == W.KIND_HERM:
        r = oracle.herm_eig(pr.d, pr.z, pr.scalar)
        return r.lam, r.vec, None
    r = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
    return r.sigma, r.V, r.U


def _check(b, problems, torch, idx=None):
    torch.cuda.synchronize()
    for p in (range(len(problems)) if idx is None else idx):
        lam, V, U, info = b.result(p)
        rl, rV, rU = _oracle(problems[p])
        assert_close(lam.cpu().numpy(), rl, f"problem {p} values")
        assert_close(V.cpu().numpy(), rV, f"problem {p} vectors")
        if rU is not None:
            assert_close(U.cpu().numpy(), rU, f"problem {p} left vectors")


def test_batched_plan_matches_oracle(env, oracle_lib):
    torch, batch, dev = env
    probs = _mixed(45, 1)
    b = batch.Batch(probs, device=dev)
    b.run()
    _check(b, probs, torch)
    b.close()


def test_sequential_path_matches_oracle(env, oracle_lib):
    torch, batch, dev = env
    probs = _mixed(20, 2)
    b = batch.Batch(probs, device=dev)
    b.run_sequential()
    _check(b, probs, torch)
    b.close()


def test_alone_equals_in_the_mix_bitwise(env):
    torch, batch, dev = env
    probs = _mixed(30, 3)
    mix = batch.Batch(probs, device=dev)
    mix.run()
    for p in (0, 7, 13, len(probs) - 5):
        one = batch.Batch([probs[p]], device=dev)
        one.run()
        torch.cuda.synchronize()
        a, b_ = mix.result(p), one.result(0)
        assert torch.equal(a[0], b_[0]) and torch.equal(a[1], b_[1])
        if a[2] is not None:
            assert torch.equal(a[2], b_[2])
        one.close()
    mix.close()


def test_graph_replays_equal_eager(env):
    torch, batch, dev = env
    probs = _mixed(25, 4)
    eager = batch.Batch(probs, device=dev)
    eager.run()
    torch.cuda.synchronize()
    ref = [[None if t is None else t.clone() for t in eager.result(p)] for p in range(len(probs))]
    g = batch.Batch(probs, device=dev, graph=True)
    for rep in range(3):
        g.out_pool.fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        g.run()
        torch.cuda.synchronize()
        for p in range(len(probs)):             # every output of every problem (the pools' padding aside)
            for a, b in zip(g.result(p), ref[p]):
                assert (a is None) == (b is None) and (a is None or torch.equal(a, b)), f"replay {rep} problem {p}"
    g.close()
    eager.close()


def test_bad_problem_is_isolated(env, oracle_lib):
    torch, batch, dev = env
    probs = _mixed(6, 5)
    bad = W.Problem(W.KIND_ARROW, 4, np.array([1.0, np.inf, 0.5]), np.array([1.0, 2.0, 3.0]), 0.0)
    probs.insert(3, bad)
    b = batch.Batch(probs, device=dev)
    b.run()
    torch.cuda.synchronize()
    lam, V, U, info = b.result(3)
    assert bool((info.cpu() & 32).all()) and bool(torch.isnan(lam).all())
    _check(b, probs, torch, idx=[p for p in range(len(probs)) if p != 3])
    b.close()


def test_reducible_row_tiles(env, oracle_lib):
    """Deflated problems large enough for the row-tiled vector kernel, odd (one row per
    store) and even (16-byte stores), beside ordinary problems."""
    torch, batch, dev = env
    rng = np.random.default_rng(61)
    probs = [W.reducible_arrow(701, rng), W.uniform_arrow(600, rng), W.reducible_arrow(1024, rng, zero_frac=0.2),
             W.dpr1(520, rng), W.dpr1(777, rng), W.herm_arrow(701, rng)]
    probs[-2].scalar = -probs[-2].scalar     # rho < 0, odd n
    b = batch.Batch(probs, device=dev)
    b.run()
    _check(b, probs, torch)
    b.close()


def test_invalid_descriptor_rejected(env):
    torch, batch, dev = env
    pr = W.uniform_arrow(5, np.random.default_rng(1))
    pk = batch.pack([pr])
    pk.descs[0].n = 0
    with pytest.raises(Exception):
        batch.Batch([pr], device=dev, packed=pk)


def test_full_size_batch_sampled(env, oracle_lib):
    """The 10,000-problem mixed batch (n log-uniform in [16, 1024]) in the plan the benchmark times."""
    torch, batch, dev = env
    probs = W.batch_mixed()
    b = batch.Batch(probs, device=dev, graph=True)
    b.run()
    torch.cuda.synchronize()
    # 320 problems stratified by kind and by order: 24 from each (kind, octave of n) class up
    # to n = 512 and 8 from each of (512, 768] and (768, 1024] (the oracle's cost grows as n^2)
    rng = np.random.default_rng(7)
    idx = set()
    for kind in (W.KIND_ARROW, W.KIND_DPR1):
        for lo, hi, take in ((8, 16, 24), (16, 32, 24), (32, 64, 24), (64, 128, 24), (128, 256, 24),
                             (256, 512, 24), (512, 768, 8), (768, 1024, 8)):
            pool = [p for p, pr in enumerate(probs) if pr.kind == kind and lo < pr.n <= hi]
            idx |= set(int(i) for i in rng.choice(pool, min(take, len(pool)), replace=False))
    idx = sorted(idx | {0, 1, len(probs) - 1})
    print(f"10,000-problem plan: oracle for {len(idx)} problems", flush=True)
    _check(b, probs, torch, idx=idx)
    info = b.info_pool.cpu().numpy().astype(np.uint32)
    assert not np.any(info & (16 | 32 | 256))
    b.close()
    del b
    torch.cuda.empty_cache()


def test_root_staging_boundaries_sampled(env, oracle_lib):
    """Orders at the edges of the root stage's LDS staging (poles and weights while 2 ns <= 1280,
    the poles alone while ns <= 1280, nothing above; ns = n - 1, DPR1 n) and the regrouped
    root stage at 8 and 16 lanes per eigenvalue, against the oracle on 24 eigenpairs each."""
    torch, batch, dev = env
    rng = np.random.default_rng(63)
    probs = ([W.uniform_arrow(n, rng) for n in (641, 642, 1281, 1282, 3100)]
             + [W.dpr1(n, rng) for n in (640, 641, 1280, 1281)] + [W.svd_arrow(1281, rng)])
    b = batch.Batch(probs, device=dev)
    b.run()
    torch.cuda.synchronize()
    for p, pr in enumerate(probs):
        lam, V, U, info = b.result(p)
        ks = np.unique(np.linspace(0, pr.n - 1, 24).astype(np.int64))
        kt = torch.from_numpy(ks).to(dev)
        if pr.kind == W.KIND_SVD:
            r = oracle.arrow_svd(pr.d, pr.z, pr.scalar, ks=ks)
            rl, rV = r.sigma, r.V
            assert_close(U[:, kt].cpu().numpy(), r.U, f"n={pr.n} kind {pr.kind} left vectors")
        else:
            r = (oracle.arrow_eig if pr.kind == W.KIND_ARROW else oracle.dpr1_eig)(pr.d, pr.z, pr.scalar, ks=ks)
            rl, rV = r.lam, r.vec
        assert_close(lam[kt].cpu().numpy(), rl, f"n={pr.n} kind {pr.kind} values")
        assert_close(V[:, kt].cpu().numpy(), rV, f"n={pr.n} kind {pr.kind} vectors")
    b.close()


def test_options_fixed_at_creation(env):
    """A plan keeps the handle's options from its creation: changing the root
    finder (ARROW_OPT_ROOT) or the FP64-b bound (ARROW_OPT_TAU_B) afterwards
    changes neither its eager nor its graph runs (bitwise)."""
    torch, batch, dev = env
    from paper_1302_7203_amd import binding
    probs = _mixed(12, 21, nmax=200)
    eager = batch.Batch(probs, device=dev)
    graph = batch.Batch(probs, device=dev, graph=True)
    eager.run()
    torch.cuda.synchronize()
    ref = [tuple(t.clone() if t is not None else None for t in eager.result(p)) for p in range(len(probs))]
    try:
        binding.set_option(binding.OPT_ROOT, binding.ROOT_BISECT)
        binding.set_option(binding.OPT_TAU_B, 4.0)
        for b in (eager, graph):
            b.run()
            torch.cuda.synchronize()
            for p in range(len(probs)):
                got = b.result(p)
                for a, r in zip(got, ref[p]):
                    assert (a is None and r is None) or torch.equal(a, r), p
    finally:
        binding.set_option(binding.OPT_ROOT, binding.ROOT_RATIONAL)
        binding.set_option(binding.OPT_TAU_B, 0.0)
