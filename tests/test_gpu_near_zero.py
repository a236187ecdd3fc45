"""Eigenvalues near the origin on the GPU (Sec. 3, Remark 1; the exceptions
(a)-(c) of condition (C1) in Theorem 2), through the C ABI, against the oracle:
every eigenvalue and vector entry within 1e-13, and the eigenvalue nearest 0
flagged ARROW_INFO_NEAR_ZERO (taken from A^{-1}), never F0_UNRESOLVED."""
import numpy as np
import pytest

import near_zero_cases as NZ
import oracle
from paper_1302_7203_amd import workloads as W
from parity import assert_close

pytestmark = pytest.mark.gpu

NEAR_ZERO, F0_UNRESOLVED = 8, 2048


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1302_7203_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return torch, binding, torch.device("cuda", 0)


def _t(gpu, x):
    torch, _, dev = gpu
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _flag(info, k):
    f = int(info[k])
    assert f & NEAR_ZERO, f"eigenvalue {k}: info {f} lacks NEAR_ZERO"
    assert not f & F0_UNRESOLVED


@pytest.mark.parametrize("case", NZ.arrow_cases(), ids=lambda c: c[0])
def test_arrow(gpu, case, oracle_lib):
    torch, binding, dev = gpu
    name, d, z, a = case
    print(f"arrow_eig near zero: {name} n={d.size + 1}", flush=True)
    out = binding.arrow_eig(_t(gpu, d), _t(gpu, z), a, pairs=True)
    torch.cuda.synchronize(dev)
    ref = oracle.arrow_eig(d, z, a)
    assert_close(out.lam.cpu().numpy(), ref.lam, "lambda")
    assert_close(out.V.cpu().numpy(), ref.vec, "V")
    k = int(np.argmin(np.abs(ref.lam)))
    _flag(out.info.cpu().numpy(), k)
    # Remark 1 measures lambda from the origin: shift 0, mu = lambda
    assert out.shift.cpu().numpy()[k] == 0.0


@pytest.mark.parametrize("case", NZ.dpr1_cases(), ids=lambda c: c[0])
def test_dpr1(gpu, case, oracle_lib):
    torch, binding, dev = gpu
    name, d, u, rho = case
    print(f"dpr1_eig near zero: {name} n={d.size}", flush=True)
    out = binding.dpr1_eig(_t(gpu, d), _t(gpu, u), rho)
    torch.cuda.synchronize(dev)
    ref = oracle.dpr1_eig(d, u, rho)
    assert_close(out.lam.cpu().numpy(), ref.lam, "lambda")
    assert_close(out.V.cpu().numpy(), ref.vec, "Q")
    _flag(out.info.cpu().numpy(), int(np.argmin(np.abs(ref.lam))))


@pytest.mark.parametrize("case", NZ.svd_cases(), ids=lambda c: c[0])
def test_svd(gpu, case, oracle_lib):
    torch, binding, dev = gpu
    name, d, z, a = case
    print(f"arrow_svd near zero: {name} n={d.size + 1}", flush=True)
    out = binding.arrow_svd(_t(gpu, d), _t(gpu, z), a)
    torch.cuda.synchronize(dev)
    ref = oracle.arrow_svd(d, z, a)
    assert_close(out.lam.cpu().numpy(), ref.sigma, "sigma")
    assert_close(out.V.cpu().numpy(), ref.V, "V")
    assert_close(out.U.cpu().numpy(), ref.U, "U")
    _flag(out.info.cpu().numpy(), d.size)


@pytest.mark.parametrize("case", NZ.herm_cases(), ids=lambda c: c[0])
def test_hermitian(gpu, case, oracle_lib):
    torch, binding, dev = gpu
    name, d, z, a = case
    print(f"arrow_eig_herm near zero: {name}", flush=True)
    out = binding.arrow_eig_herm(_t(gpu, d), _t(gpu, z), a)
    torch.cuda.synchronize(dev)
    ref = oracle.herm_eig(d, z, a)
    assert_close(out.lam.cpu().numpy(), ref.lam, "lambda")
    got, want = out.V.cpu().numpy(), ref.vec
    e = np.abs(got - want) / np.abs(want)
    assert float(e.max()) <= 1e-13
    _flag(out.info.cpu().numpy(), int(np.argmin(np.abs(ref.lam))))


def test_batched_alone_and_in_the_mix(gpu, oracle_lib):
    """The same problems in one batched plan (repairs in k_b_repair) against the
    oracle, and each alone in a plan of its own, bitwise."""
    torch, _, dev = gpu
    from paper_1302_7203_amd import batch
    probs = [W.Problem(W.KIND_ARROW, d.size + 1, d, z, a) for _, d, z, a in NZ.arrow_cases()]
    probs += [W.Problem(W.KIND_DPR1, d.size, d, u, r) for _, d, u, r in NZ.dpr1_cases()]
    probs += [W.Problem(W.KIND_SVD, d.size + 1, d, z, a) for _, d, z, a in NZ.svd_cases()]
    probs += [W.Problem(W.KIND_HERM, d.size + 1, d, z, a) for _, d, z, a in NZ.herm_cases()]
    rng = np.random.default_rng(3)
    probs += [W.uniform_arrow(100, rng), W.dpr1(80, rng)]   # ordinary neighbours in the queue
    print(f"batched near-zero plan: {len(probs)} problems", flush=True)
    mix = batch.Batch(probs, device=dev)
    mix.run()
    torch.cuda.synchronize(dev)
    for p, pr in enumerate(probs):
        lam, V, U, info = mix.result(p)
        if pr.kind == W.KIND_ARROW:
            r = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
            rl, rV, rU = r.lam, r.vec, None
        elif pr.kind == W.KIND_DPR1:
            r = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
            rl, rV, rU = r.lam, r.vec, None
        elif pr.kind == W.KIND_HERM:
            r = oracle.herm_eig(pr.d, pr.z, pr.scalar)
            rl, rV, rU = r.lam, r.vec, None
        else:
            r = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
            rl, rV, rU = r.sigma, r.V, r.U
        assert_close(lam.cpu().numpy(), rl, f"problem {p} values")
        if pr.kind == W.KIND_HERM:
            assert float((np.abs(V.cpu().numpy() - rV) / np.abs(rV)).max()) <= 1e-13
        else:
            assert_close(V.cpu().numpy(), rV, f"problem {p} vectors")
        if rU is not None:
            assert_close(U.cpu().numpy(), rU, f"problem {p} left vectors")
        one = batch.Batch([pr], device=dev)
        one.run()
        torch.cuda.synchronize(dev)
        l1, V1, _, i1 = one.result(0)
        assert torch.equal(l1, lam) and torch.equal(V1, V) and torch.equal(i1, info), p
