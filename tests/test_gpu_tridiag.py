"""Divide-and-conquer tridiagonal eigensolver with DPR1 merges (tridiag_eig) against
the binary128 oracle.

Divide and conquer is normwise accurate, so the bars are derived from that
arithmetic rather than the componentwise 1e-13 of the arrowhead path:
eigenvalues within C n eps ||T||, residual ||T q - lambda q|| and
orthogonality within C n eps (||T||), and each eigenvector, compared up to
sign, within C n eps ||T|| / gap_k (the perturbation bound), gap_k its
distance to the other eigenvalues.  C = 4."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53
C = 4.0


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1302_7203_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return torch, binding, torch.device("cuda", 0)


def _solve(gpu, a, b):
    torch, binding, dev = gpu
    out = binding.tridiag_eig(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
    torch.cuda.synchronize(dev)
    return out.lam.cpu().numpy(), out.V.cpu().numpy(), out.info.cpu().numpy()


def _check(a, b, lam, Q, ks=None):
    """The bars above on the columns ks (all by default)."""
    n = a.size
    tn = float(np.max(np.abs(a) + np.concatenate([[0.0], np.abs(b)]) + np.concatenate([np.abs(b), [0.0]])))
    ks = np.arange(n) if ks is None else np.asarray(ks)
    near = np.unique(np.clip(np.concatenate([ks - 1, ks, ks + 1]), 0, n - 1))
    ev = dict(zip(near, oracle.tridiag_eig(a, b, ks=near, vectors=False)[0]))
    rl, rQ = oracle.tridiag_eig(a, b, ks=ks)
    assert np.all(np.diff(lam) <= 0)
    assert np.max(np.abs(lam[ks] - rl)) <= C * n * EPS * tn
    Qk = Q[:, ks].astype(np.longdouble)
    TQ = a[:, None] * Qk                      # T Q[:, ks] without forming T
    TQ[:-1] += b[:, None] * Qk[1:]
    TQ[1:] += b[:, None] * Qk[:-1]
    assert np.max(np.abs(TQ - Qk * lam[ks].astype(np.longdouble))) <= C * n * EPS * tn
    G = Q.astype(np.longdouble).T @ Qk        # columns ks against every column
    G[ks, np.arange(ks.size)] -= 1
    assert np.max(np.abs(G)) <= C * n * EPS
    for i, k in enumerate(ks):
        gap = min([abs(ev[j] - ev[k]) for j in (k - 1, k + 1) if 0 <= j < n] or [np.inf])
        q = Q[:, k] * np.sign(Q[np.argmax(np.abs(Q[:, k])), k])
        err = np.max(np.abs(q - rQ[:, i]))
        assert err <= min(2.0, C * n * EPS * tn / gap), (k, err, gap)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 255, 700])
def test_random_tridiagonal(gpu, n, oracle_lib):
    rng = np.random.default_rng(500 + n)
    a, b = rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))
    lam, Q, info = _solve(gpu, a, b)
    assert not np.any(info & (16 | 32))
    _check(a, b, lam, Q)


def test_graded_and_signed(gpu, oracle_lib):
    """Entries over ten decades with both signs of the off-diagonal (rho < 0 merges)."""
    rng = np.random.default_rng(7)
    n = 300
    a = rng.standard_normal(n) * 10.0 ** rng.uniform(-5, 5, n)
    b = rng.standard_normal(n - 1) * 10.0 ** rng.uniform(-5, 5, n - 1)
    lam, Q, _ = _solve(gpu, a, b)
    _check(a, b, lam, Q)


def test_zero_off_diagonals_split(gpu, oracle_lib):
    """b_k = 0 splits T: those merges are list merges with a permutation."""
    rng = np.random.default_rng(8)
    n = 200
    a, b = rng.standard_normal(n), rng.standard_normal(n - 1)
    b[[0, 49, 99, 100, 150, 198]] = 0.0
    lam, Q, info = _solve(gpu, a, b)
    assert not np.any(info & (16 | 32))
    _check(a, b, lam, Q)


def test_large_sampled(gpu, oracle_lib):
    n = 4096
    rng = np.random.default_rng(9)
    a, b = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n - 1)
    lam, Q, _ = _solve(gpu, a, b)
    _check(a, b, lam, Q, ks=np.arange(0, n, 97))
