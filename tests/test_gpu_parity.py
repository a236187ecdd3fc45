"""GPU path (through the C ABI) against the oracle, element by element, at the
1e-13 relative bar for every eigenvalue and every vector entry."""
import numpy as np
import pytest

import oracle
from paper_1302_7203_amd import workloads as W
from parity import assert_close, relerr

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1302_7203_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return torch, binding, torch.device("cuda", 0)


def _arrow(gpu, d, z, a, vectors=True, pairs=False):
    torch, binding, dev = gpu
    out = binding.arrow_eig(torch.from_numpy(np.ascontiguousarray(d)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(z)).to(dev), a, vectors=vectors, pairs=pairs)
    torch.cuda.synchronize(dev)
    return out


def _np(t):
    return None if t is None else t.cpu().numpy()


EXAMPLES = {
    "ex1": (np.array([2e-3, 1e-7, 0.0, -1e-7, -2e-3]), np.array([1e7, 1e7, 1.0, 1e7, 1e7]), 1e20),
    "ex2": (np.array([1 + 4 * EPS, 1 + 3 * EPS, 1 + 2 * EPS, 1 + EPS]), np.array([1.0, 2, 3, 4]), 0.0),
    "ex3": (np.array([1e10, 4, 3, 2, 1.0]), np.array([1e10, 1, 1, 1, 1.0]), 1e10),
}


@pytest.mark.parametrize("name", sorted(EXAMPLES))
def test_examples(gpu, name, oracle_lib):
    d, z, a = EXAMPLES[name]
    out = _arrow(gpu, d, z, a, pairs=True)
    ref = oracle.arrow_eig(d, z, a)
    assert_close(_np(out.lam), ref.lam, "lambda")
    assert_close(_np(out.V), ref.vec, "V")
    # Remark 3 pairs: shift + mu represents lambda
    lam2 = _np(out.shift) + _np(out.mu)
    assert_close(lam2, ref.lam, "shift+mu")


def test_example2_pairs_carry_32_digits(gpu, oracle_lib):
    d, z, a = EXAMPLES["ex2"]
    out = _arrow(gpu, d, z, a, pairs=True)
    ref = oracle.arrow_eig(d, z, a)
    sh, mu = _np(out.shift), _np(out.mu)
    # lambda_2..lambda_4: the pair (d_i, mu) equals the oracle's (pole, tau) to ~1e-13 in mu
    for k in (1, 2, 3):
        assert sh[k] == d[ref.pole[k]]
        assert abs(mu[k] - ref.tau[k]) <= 1e-13 * abs(ref.tau[k])


def test_uniform_512_full(gpu, oracle_lib):
    pr = W.single_uniform_512()
    out = _arrow(gpu, pr.d, pr.z, pr.scalar)
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    assert_close(_np(out.lam), ref.lam, "lambda")
    assert_close(_np(out.V), ref.vec, "V")


def _sample_ks(n, info, step, extra=16):
    ks = set(range(0, n, step)) | {0, 1, n - 2, n - 1}
    flagged = np.flatnonzero(info & (2 | 4 | 8))
    ks |= set(int(k) for k in flagged[:: max(1, flagged.size // 64)]) if flagged.size else set()
    rng = np.random.default_rng(n)
    ks |= set(int(k) for k in rng.integers(0, n, extra))
    return np.array(sorted(ks), dtype=np.int64)


def test_graded_4096_full(gpu, oracle_lib):
    """The graded n = 4096 workload in full: every eigenvalue and every entry of V (16.8M)
    against the oracle."""
    torch, _, _ = gpu
    pr = W.single_graded_4096()
    out = _arrow(gpu, pr.d, pr.z, pr.scalar)
    lam, info = _np(out.lam), _np(out.info).astype(np.uint32)
    assert np.all(info & 1)                       # b in double-double everywhere
    assert np.all(np.diff(lam) < 0)
    print("graded n=4096: oracle for all 4096 eigenpairs", flush=True)
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    assert_close(lam, ref.lam, "lambda")
    assert_close(_np(out.V), ref.vec, "V")


def test_uniform_16384_sampled(gpu, oracle_lib):
    torch, _, _ = gpu
    pr = W.single_uniform_16384()
    out = _arrow(gpu, pr.d, pr.z, pr.scalar)
    lam, info = _np(out.lam), _np(out.info).astype(np.uint32)
    # interlacing with the (sorted) poles for every eigenvalue
    assert np.all(lam[:-1] > pr.d) and np.all(pr.d > lam[1:])
    # every 16th eigenpair (1024 eigenvalues and columns, 16.8M entries), every one that
    # took a remedy, and the ends
    ks = _sample_ks(pr.n, info, 16)
    flagged = np.flatnonzero(info & (2 | 4 | 8))
    ks = np.union1d(ks, flagged).astype(np.int64)
    print(f"uniform n=16384: oracle for {ks.size} eigenpairs", flush=True)
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks)
    assert_close(lam[ks], ref.lam, "lambda")
    V = out.V[:, torch.from_numpy(ks).to(out.V.device)].cpu().numpy()
    assert_close(V, ref.vec, "V columns")
    del out
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_uniform_16384_every_eigenvalue(gpu, oracle_lib, capsys):
    """Every one of the 16384 eigenvalues of the uniform n = 16384 workload against the
    oracle (about four minutes of the oracle on 16 host threads; progress is printed per
    chunk of 2048)."""
    torch, _, _ = gpu
    pr = W.single_uniform_16384()
    out = _arrow(gpu, pr.d, pr.z, pr.scalar, vectors=False)
    lam = _np(out.lam)
    for c0 in range(0, pr.n, 2048):
        ks = np.arange(c0, min(pr.n, c0 + 2048), dtype=np.int64)
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks, vectors=False)
        assert_close(lam[ks], ref.lam, f"lambda {c0}..{ks[-1]}")
        with capsys.disabled():
            print(f"uniform n=16384: eigenvalues {c0}..{ks[-1]} match the oracle", flush=True)


@pytest.mark.parametrize("kind", [W.KIND_ARROW, W.KIND_DPR1, W.KIND_SVD])
def test_odd_order_above_4096_sampled(gpu, kind, oracle_lib):
    """n = 5001: the tall vector tiles with one row per store (odd n), for every kind."""
    torch, binding, _ = gpu
    rng = np.random.default_rng(5001 + kind)
    n = 5001
    if kind == W.KIND_ARROW:
        pr = W.uniform_arrow(n, rng)
        out = _arrow(gpu, pr.d, pr.z, pr.scalar)
        ks = np.unique(np.r_[0, 1, 2500, n - 2, n - 1, rng.integers(0, n, 12)])
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks)
        rl, rV, V = ref.lam, ref.vec, out.V
    elif kind == W.KIND_DPR1:
        pr = W.dpr1(n, rng)
        out = binding.dpr1_eig(torch.from_numpy(pr.d).cuda(), torch.from_numpy(pr.z).cuda(), pr.scalar)
        ks = np.unique(np.r_[0, 1, 2500, n - 2, n - 1, rng.integers(0, n, 12)])
        ref = oracle.dpr1_eig(pr.d, pr.z, pr.scalar, ks=ks)
        rl, rV, V = ref.lam, ref.vec, out.V
    else:
        pr = W.svd_arrow(n, rng)
        out = binding.arrow_svd(torch.from_numpy(pr.d).cuda(), torch.from_numpy(pr.z).cuda(), pr.scalar)
        ks = np.unique(np.r_[0, 1, 2500, n - 2, n - 1, rng.integers(0, n, 12)])
        ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar, ks=ks)
        rl, rV, V = ref.sigma, ref.V, out.V
        assert_close(out.U[:, torch.from_numpy(ks).cuda()].cpu().numpy(), ref.U, "U columns")
    torch.cuda.synchronize()
    kt = torch.from_numpy(ks).to(out.lam.device)
    assert_close(out.lam[kt].cpu().numpy(), rl, "values")
    assert_close(V[:, kt].cpu().numpy(), rV, "vector columns")
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_every_lane_count(gpu, lanes, oracle_lib):
    _, binding, _ = gpu
    pr = W.uniform_arrow(301, np.random.default_rng(3))
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    binding.set_option(binding.OPT_LANES, lanes)
    try:
        out = _arrow(gpu, pr.d, pr.z, pr.scalar)
    finally:
        binding.set_option(binding.OPT_LANES, 0)
    assert_close(_np(out.lam), ref.lam, "lambda")
    assert_close(_np(out.V), ref.vec, "V")


@pytest.mark.parametrize("n", [1, 2, 3, 255, 1025])
def test_small_ragged_shuffled(gpu, n, oracle_lib):
    pr = W.shuffled(W.uniform_arrow(n, np.random.default_rng(n)), 9)
    out = _arrow(gpu, pr.d, pr.z, pr.scalar)
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    assert_close(_np(out.lam), ref.lam, "lambda")
    assert_close(_np(out.V), ref.vec, "V")


def test_order_and_sign_invariance_bitwise(gpu):
    pr = W.uniform_arrow(200, np.random.default_rng(8))
    base = _arrow(gpu, pr.d, pr.z, pr.scalar)
    sh = W.shuffled(pr, 2)
    perm = sh.meta["perm"]
    out = _arrow(gpu, sh.d, sh.z, sh.scalar)
    assert np.array_equal(_np(out.lam), _np(base.lam))
    assert np.array_equal(_np(out.V)[:-1], _np(base.V)[perm])
    z2 = pr.z.copy()
    z2[7] = -z2[7]
    fl = _arrow(gpu, pr.d, z2, pr.scalar)
    assert np.array_equal(_np(fl.V)[7], -_np(base.V)[7])


@pytest.mark.parametrize("n", [3, 700, 5000])
def test_increasing_input_equals_decreasing_bitwise(gpu, n):
    """Poles given in increasing order take the front end's reversed copy: the same
    eigenvalues bit for bit, and the vectors with their rows reversed."""
    pr = W.uniform_arrow(n, np.random.default_rng(300 + n))
    a = _arrow(gpu, pr.d, pr.z, pr.scalar)
    b = _arrow(gpu, pr.d[::-1].copy(), pr.z[::-1].copy(), pr.scalar)
    assert np.array_equal(_np(a.lam), _np(b.lam))
    Va, Vb = _np(a.V), _np(b.V)
    assert np.array_equal(Va[:-1][::-1], Vb[:-1]) and np.array_equal(Va[-1], Vb[-1])


def test_repeat_is_bitwise_deterministic(gpu):
    pr = W.single_graded_4096()
    a = _arrow(gpu, pr.d, pr.z, pr.scalar)
    b = _arrow(gpu, pr.d, pr.z, pr.scalar)
    assert np.array_equal(_np(a.lam), _np(b.lam))
    assert bool((a.V == b.V).all())


REDUCIBLE = [
    (np.array([1.0, 3.0, 1.0, 0.5, 1.0, -2.0]), np.array([2.0, 1.0, -1.5, 3.0, 0.25, 0.0]), 0.3),
    (np.array([0.5, -1.0, 2.0]), np.array([0.0, 0.0, 0.0]), 0.7),
    (np.array([2.0, 2.0, 2.0, 2.0]), np.array([1.0, -2.0, 0.5, 3.0]), -1.0),
    (np.array([0.0, 1.0, 0.0, 1.0]), np.array([0.0, 1.0, 1.0, 2.0]), 0.0),
]


@pytest.mark.parametrize("i", range(len(REDUCIBLE)))
def test_reducible_deflated(gpu, i, oracle_lib):
    """Zero shaft entries and repeated poles are deflated (Sec. 1), as in the oracle."""
    d, z, a = REDUCIBLE[i]
    out = _arrow(gpu, d, z, a, pairs=True)
    ref = oracle.arrow_eig(d, z, a)
    assert_close(_np(out.lam), ref.lam, "lambda")
    assert_close(_np(out.V), ref.vec, "V")
    assert_close(_np(out.shift) + _np(out.mu), ref.lam, "shift+mu")
    assert np.array_equal((_np(out.info) & 1024) != 0, ref.tau == 0)


@pytest.mark.parametrize("n", [2, 9, 300, 513, 1000, 4096, 5001])
def test_reducible_sizes_sampled(gpu, n, oracle_lib):
    """Every vector-tile shape, odd and even n, with ~10% zero shaft entries and
    repeated poles, unsorted; ~60 sampled columns plus every deflated one."""
    pr = W.reducible_arrow(n, np.random.default_rng(n), zero_frac=0.1, repeat_every=13)
    out = _arrow(gpu, pr.d, pr.z, pr.scalar, pairs=True)
    info = _np(out.info)
    defl = np.flatnonzero(info & 1024)
    assert defl.size >= int(0.1 * (n - 1))
    ks = np.union1d(np.arange(0, n, max(1, n // 60)), defl)
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks)
    assert_close(_np(out.lam)[ks], ref.lam, "lambda")
    assert_close(_np(out.V)[:, ks], ref.vec, "V")
    assert np.array_equal(info[ks] & 1024 != 0, ref.tau == 0)
    assert np.all(np.diff(_np(out.lam)) <= 0)


def test_reducible_sorted_input(gpu, oracle_lib):
    """Strictly decreasing poles with zero shaft entries: the one-kernel front end deflates."""
    rng = np.random.default_rng(77)
    pr = W.reducible_arrow(700, rng, zero_frac=0.3, repeat_every=0, triple=False)
    o = np.argsort(-pr.d, kind="stable")
    d, z = pr.d[o].copy(), pr.z[o].copy()
    assert np.all(np.diff(d) < 0)
    out = _arrow(gpu, d, z, pr.scalar)
    ks = np.arange(0, 700, 7)
    ref = oracle.arrow_eig(d, z, pr.scalar, ks=ks)
    assert_close(_np(out.lam)[ks], ref.lam, "lambda")
    assert_close(_np(out.V)[:, ks], ref.vec, "V")


def test_reducible_other_kinds_and_nonfinite_reported(gpu):
    _, binding, dev = gpu
    import torch
    t = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64)).to(dev)   # noqa: E731
    out = binding.dpr1_eig(t([1.0, 1.0, 0.5]), t([1.0, 2.0, 3.0]), 1.0)
    torch.cuda.synchronize(dev)
    assert np.all(_np(out.info) & 16) and np.all(np.isnan(_np(out.lam)))
    out = binding.arrow_svd(t([1.0, 0.7, 0.5]), t([1.0, 0.0, 3.0]), 0.5)
    torch.cuda.synchronize(dev)
    assert np.all(_np(out.info) & 16) and np.all(np.isnan(_np(out.lam)))
    out = _arrow(gpu, np.array([1.0, np.inf, 0.5]), np.array([1.0, 2.0, 3.0]), 0.0)
    assert np.all(_np(out.info) & 32)
    out = _arrow(gpu, np.array([1.0, 1.0, np.nan]), np.array([0.0, 2.0, 3.0]), 0.0)
    assert np.all(_np(out.info) & 32) and np.all(np.isnan(_np(out.lam)))
    # a good call after a bad one is unaffected
    pr = W.uniform_arrow(50, np.random.default_rng(1))
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    out = _arrow(gpu, pr.d, pr.z, pr.scalar)
    assert_close(_np(out.lam), ref.lam, "lambda")


def test_fp64_b_negative_control(gpu, oracle_lib):
    _, binding, _ = gpu
    d, z, a = EXAMPLES["ex3"]
    ref = oracle.arrow_eig(d, z, a)
    binding.set_option(binding.OPT_FP64_B, 1)
    binding.set_option(binding.OPT_REMEDIES, 0)
    try:
        out = _arrow(gpu, d, z, a)
    finally:
        binding.set_option(binding.OPT_FP64_B, 0)
        binding.set_option(binding.OPT_REMEDIES, 1)
    e = relerr(_np(out.lam), ref.lam)
    assert e[4] > 1e-9 and e[5] > 1e-8      # the digits Algorithm 1 loses (Sec. 5, Ex. 3)
    good = _arrow(gpu, d, z, a)
    assert relerr(_np(good.lam), ref.lam).max() < 1e-15


@pytest.mark.parametrize("n", [1, 2, 97, 1000])
def test_dpr1(gpu, n, oracle_lib):
    torch, binding, dev = gpu
    pr = W.dpr1(n, np.random.default_rng(60 + n))
    out = binding.dpr1_eig(torch.from_numpy(pr.d).to(dev), torch.from_numpy(pr.z).to(dev), pr.scalar)
    torch.cuda.synchronize(dev)
    ref = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
    assert_close(_np(out.lam), ref.lam, "lambda")
    assert_close(_np(out.V), ref.vec, "Q")


@pytest.mark.parametrize("n", [1, 2, 97, 1000, 4097])
def test_dpr1_negative_rho(gpu, n, oracle_lib):
    """rho < 0 (solved as the negation of (-D) + |rho| u u^T), every tile shape up to n = 4097."""
    torch, binding, dev = gpu
    pr = W.dpr1(n, np.random.default_rng(65 + n))
    out = binding.dpr1_eig(torch.from_numpy(pr.d).to(dev), torch.from_numpy(pr.z).to(dev), -pr.scalar)
    torch.cuda.synchronize(dev)
    ks = np.arange(n) if n <= 1000 else np.arange(0, n, 41)
    ref = oracle.dpr1_eig(pr.d, pr.z, -pr.scalar, ks=ks)
    assert_close(_np(out.lam)[ks], ref.lam, "lambda")
    assert_close(_np(out.V)[:, ks], ref.vec, "Q")


def _herm_case(n, seed):
    rng = np.random.default_rng(seed)
    m = n - 1
    d = W._sorted_with_gap(rng, m, -1.0, 1.0)[rng.permutation(m)]
    z = rng.uniform(0.1, 1.0, m) * np.exp(2j * np.pi * rng.uniform(0.0, 1.0, m))
    return d, z, float(rng.uniform(-1.0, 1.0))


def _herm(gpu, d, z, a, pairs=False):
    torch, binding, dev = gpu
    out = binding.arrow_eig_herm(torch.from_numpy(np.ascontiguousarray(d)).to(dev),
                                 torch.from_numpy(np.ascontiguousarray(z, dtype=np.complex128)).to(dev), a,
                                 pairs=pairs)
    torch.cuda.synchronize(dev)
    return out


def _assert_close_c(got, ref, what, tol=1e-13):
    den = np.abs(ref)
    e = np.abs(got - ref) / np.where(den == 0, 1.0, den)
    worst = float(e.max()) if e.size else 0.0
    assert np.all(np.isfinite(e)) and worst <= tol, f"{what}: max relative error {worst:.3e}"


@pytest.mark.parametrize("n", [1, 2, 97, 1000, 4097])
def test_hermitian(gpu, n, oracle_lib):
    """Hermitian arrowhead (Sec. 6.1), every complex vector tile shape; sampled above n = 1000."""
    d, z, a = _herm_case(n, 95 + n)
    out = _herm(gpu, d, z, a, pairs=True)
    ks = np.arange(n) if n <= 1000 else np.arange(0, n, 41)
    ref = oracle.herm_eig(d, z, a, ks=ks)
    assert_close(_np(out.lam)[ks], ref.lam, "lambda")
    assert_close(_np(out.shift)[ks] + _np(out.mu)[ks], ref.lam, "shift+mu")
    _assert_close_c(_np(out.V)[:, ks], ref.vec, "U")


def test_hermitian_real_case_bitwise(gpu):
    """Real z: the Hermitian path gives the symmetric path's results bit for bit."""
    pr = W.uniform_arrow(600, np.random.default_rng(96))
    pr.z[::3] *= -1
    h = _herm(gpu, pr.d, pr.z.astype(np.complex128), pr.scalar)
    r = _arrow(gpu, pr.d, pr.z, pr.scalar)
    assert np.array_equal(_np(h.lam), _np(r.lam))
    U = _np(h.V)
    assert np.array_equal(U.real, _np(r.V)) and np.all(U.imag == 0)


def test_hermitian_reducible_reported(gpu):
    out = _herm(gpu, np.array([1.0, 0.5, 0.2]), np.array([1.0 + 1j, 0.0, 2.0]), 0.0)
    assert np.all(_np(out.info) & 16) and np.all(np.isnan(_np(out.lam)))


@pytest.mark.parametrize("n", [1, 2, 97, 1000])
def test_svd(gpu, n, oracle_lib):
    torch, binding, dev = gpu
    pr = W.svd_arrow(n, np.random.default_rng(70 + n))
    out = binding.arrow_svd(torch.from_numpy(pr.d).to(dev), torch.from_numpy(pr.z).to(dev), pr.scalar)
    torch.cuda.synchronize(dev)
    ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
    assert_close(_np(out.lam), ref.sigma, "sigma")
    assert_close(_np(out.V), ref.V, "V")
    assert_close(_np(out.U), ref.U, "U")


def test_bisection_method_matches_oracle(gpu, oracle_lib):
    """Algorithm 3 (bisection) instead of the default rational iteration."""
    torch, binding, _ = gpu
    binding.set_option(binding.OPT_ROOT, binding.ROOT_BISECT)
    try:
        pr = W.single_uniform_512()
        out = _arrow(gpu, pr.d, pr.z, pr.scalar)
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
        assert_close(_np(out.lam), ref.lam, "lambda (bisection)")
        assert_close(_np(out.V), ref.vec, "V (bisection)")
        pr = W.single_graded_4096()
        out = _arrow(gpu, pr.d, pr.z, pr.scalar)
        ks = _sample_ks(pr.n, _np(out.info).astype(np.uint32), 32)
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks)
        assert_close(_np(out.lam)[ks], ref.lam, "lambda (bisection, graded)")
        V = out.V[:, torch.from_numpy(ks).to(out.V.device)].cpu().numpy()
        assert_close(V, ref.vec, "V (bisection, graded)")
    finally:
        binding.set_option(binding.OPT_ROOT, binding.ROOT_RATIONAL)


def test_unsorted_large_input_matches_sorted(gpu):
    """The rank sort over several comparison chunks gives the same bits as sorted input."""
    pr = W.single_graded_4096()
    base = _arrow(gpu, pr.d, pr.z, pr.scalar)
    sh = W.shuffled(pr, 11)
    out = _arrow(gpu, sh.d, sh.z, sh.scalar)
    assert np.array_equal(_np(out.lam), _np(base.lam))
    perm = sh.meta["perm"]
    Vb, Vo = _np(base.V), _np(out.V)
    assert np.array_equal(Vo[:-1], Vb[perm]) and np.array_equal(Vo[-1], Vb[-1])


@pytest.mark.parametrize("k", [-100, 20, 100])
def test_power_of_two_scaling_is_exact(gpu, k):
    """2^k times every input: eigenvalues (singular values) times 2^k and the same vectors,
    bit for bit, for every kind (no absolute threshold anywhere)."""
    torch, binding, dev = gpu
    s = 2.0 ** k
    rng = np.random.default_rng(61)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)   # noqa: E731
    pr = W.graded_arrow(1000, rng, clusters=8, cluster_size=8)
    a, b = _arrow(gpu, pr.d, pr.z, pr.scalar), _arrow(gpu, pr.d * s, pr.z * s, pr.scalar * s)
    assert np.array_equal(_np(b.lam), _np(a.lam) * s) and np.array_equal(_np(b.V), _np(a.V))
    pr = W.dpr1(700, rng)
    a, b = binding.dpr1_eig(t(pr.d), t(pr.z), pr.scalar), binding.dpr1_eig(t(pr.d * s), t(pr.z), pr.scalar * s)
    torch.cuda.synchronize(dev)
    assert np.array_equal(_np(b.lam), _np(a.lam) * s) and np.array_equal(_np(b.V), _np(a.V))
    pr = W.svd_arrow(500, rng)
    a = binding.arrow_svd(t(pr.d), t(pr.z), pr.scalar)
    b = binding.arrow_svd(t(pr.d * s), t(pr.z * s), pr.scalar * s)
    torch.cuda.synchronize(dev)
    assert np.array_equal(_np(b.lam), _np(a.lam) * s)
    assert np.array_equal(_np(b.V), _np(a.V)) and np.array_equal(_np(b.U), _np(a.U))
    d, z, al = _herm_case(600, 62)
    a, b = _herm(gpu, d, z, al), _herm(gpu, d * s, z * s, al * s)
    assert np.array_equal(_np(b.lam), _np(a.lam) * s) and np.array_equal(_np(b.V), _np(a.V))


@pytest.mark.parametrize("kind", [W.KIND_ARROW, W.KIND_DPR1, W.KIND_SVD])
def test_spectrum_spread_over_250_decades(gpu, kind, oracle_lib):
    """Eigenvalues within 1e-240 of their poles, where a square of an x-space
    quantity would overflow."""
    torch, binding, dev = gpu
    pr = W.wide_arrow(kind, 700, np.random.default_rng(80 + kind), 250)
    d = torch.from_numpy(pr.d).to(dev)
    z = torch.from_numpy(pr.z).to(dev)
    if kind == W.KIND_DPR1:
        out = binding.dpr1_eig(d, z, pr.scalar)
        ref = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
        lam, vec = ref.lam, ref.vec
    elif kind == W.KIND_SVD:
        out = binding.arrow_svd(d, z, pr.scalar)
        ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
        lam, vec = ref.sigma, ref.V
    else:
        out = binding.arrow_eig(d, z, pr.scalar)
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
        lam, vec = ref.lam, ref.vec
    torch.cuda.synchronize(dev)
    assert_close(_np(out.lam), lam, "lambda")
    assert_close(_np(out.V), vec, "V")
    if kind == W.KIND_SVD:
        assert_close(_np(out.U), ref.U, "U")


def test_fp64_b_where_kb_is_small(gpu, oracle_lib):
    """ARROW_OPT_TAU_B = 4: b from the FP64 pass where K_b <= 4 (Algorithm 5), the
    double-double pass elsewhere; same bar against the oracle.  Bad values are refused."""
    torch, binding, dev = gpu
    cases = [(W.single_graded_4096(), np.arange(0, 4096, 16)), (W.single_uniform_512(), None)]
    binding.set_option(binding.OPT_TAU_B, 4.0)
    try:
        for pr, ks in cases:
            out = _arrow(gpu, pr.d, pr.z, pr.scalar)
            ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks)
            kk = np.arange(pr.n) if ks is None else ks
            assert_close(_np(out.lam)[kk], ref.lam, "lambda")
            assert_close(_np(out.V)[:, kk], ref.vec, "V")
        for bad in (-1.0, float("inf"), float("nan")):
            with pytest.raises(binding.ArrowError):
                binding.set_option(binding.OPT_TAU_B, bad)
    finally:
        binding.set_option(binding.OPT_TAU_B, 0.0)


def test_example3_conditions_kb_knu(gpu):
    """arrow_conditions after Example 3 (Sec. 5): the printed K_b (eq. K2) of
    lambda_2..lambda_6 to 1e-6, and K_nu (eq. K0), printed 7.941165469988994 for
    lambda_6 and about 1 for the others (their printed digits carry ~1e-7 of the
    first pass's noise, so 1e-6)."""
    torch, binding, dev = gpu
    d, z, a = EXAMPLES["ex3"]
    _arrow(gpu, d, z, a)
    kb, knu = binding.conditions(6, dev)
    torch.cuda.synchronize(dev)
    kb, knu = kb.cpu().numpy(), knu.cpu().numpy()
    kb_printed = [3.243243243540540e9, 3.636363636818182e9, 4.444444445000000e9, 5.217390439488477e9,
                  5.217390439488477e9]
    knu_printed = [9.999999090793056e-1, 9.999996083428923e-1, 1.000000117045544, 9.999998561319470e-1,
                   7.941165469988994]
    for k in range(1, 6):
        assert abs(kb[k] - kb_printed[k - 1]) <= 1e-6 * kb_printed[k - 1], (k, kb[k])
        assert abs(knu[k] - knu_printed[k - 1]) <= 1e-6 * knu_printed[k - 1], (k, knu[k])
