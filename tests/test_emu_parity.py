"""The library's kernel bodies, driven on the host with one lane per eigenvalue,
against the oracle (no GPU).  This checks the method as implemented; the GPU
tests check the same bodies under the real grid."""
import numpy as np
import pytest

import oracle
from emu import emu
from paper_1302_7203_amd import workloads as W
from parity import TOL, assert_close, relerr

EPS = 2.0 ** -52


def _examples():
    return {
        "ex1": (np.array([2e-3, 1e-7, 0.0, -1e-7, -2e-3]), np.array([1e7, 1e7, 1.0, 1e7, 1e7]), 1e20),
        "ex2": (np.array([1 + 4 * EPS, 1 + 3 * EPS, 1 + 2 * EPS, 1 + EPS]), np.array([1.0, 2, 3, 4]), 0.0),
        "ex3": (np.array([1e10, 4, 3, 2, 1.0]), np.array([1e10, 1, 1, 1, 1.0]), 1e10),
    }


@pytest.mark.parametrize("name", ["ex1", "ex2", "ex3"])
def test_examples(name, oracle_lib):
    d, z, a = _examples()[name]
    r = emu.solve(0, d, z, a)
    ref = oracle.arrow_eig(d, z, a)
    assert_close(r["lam"], ref.lam, f"{name} lambda")
    assert_close(r["V"], ref.vec, f"{name} V")


def test_example3_negative_control_and_kb(oracle_lib):
    """With b in FP64 only (Algorithm 2) the example's eigenvalues lose the digits the
    paper's Algorithm 1 column loses; with double-double b they are exact (Sec. 5, Ex. 3)."""
    d, z, a = _examples()["ex3"]
    ref = oracle.arrow_eig(d, z, a)
    good = emu.solve(0, d, z, a)
    bad = emu.solve(0, d, z, a, fp64_b=1, remedies=0)
    e_good = relerr(good["lam"], ref.lam)
    e_bad = relerr(bad["lam"], ref.lam)
    assert e_good.max() < 1e-15
    # printed Algorithm 1 errors: ~8e-12 (lambda_2) ... 2e-8 (lambda_5), 3.4e-7 (lambda_6)
    assert e_bad[1] > 1e-12 and e_bad[4] > 1e-9 and e_bad[5] > 1e-8
    printed_basic = [4.150396802313551, 3.161498641452035, 2.188045596352105, 1.216093560005649,
                     -7.160348702977373e-1]
    for k in range(1, 6):
        e_printed = abs(printed_basic[k - 1] - ref.lam[k]) / abs(ref.lam[k])
        assert 0.01 * e_printed < e_bad[k] < 100 * e_printed, (k, e_bad[k], e_printed)
    # K_b table of the example (lambda_2..lambda_6); the printed K_nu ~ 1 values carry noise
    kb_printed = [3.243243243540540e9, 3.636363636818182e9, 4.444444445000000e9, 5.217390439488477e9,
                  5.217390439488477e9]
    for k in range(1, 6):
        assert abs(good["kb"][k] - kb_printed[k - 1]) <= 1e-6 * kb_printed[k - 1], (k, good["kb"][k])
    # K_nu (eq. K0) of lambda_6, printed 7.941165469988994; the K_nu ~ 1 values to 1e-6
    knu_printed = [9.999999090793056e-1, 9.999996083428923e-1, 1.000000117045544, 9.999998561319470e-1,
                   7.941165469988994]
    for k in range(1, 6):
        assert abs(good["knu"][k] - knu_printed[k - 1]) <= 1e-6 * knu_printed[k - 1], (k, good["knu"][k])


def test_uniform_512(oracle_lib):
    pr = W.single_uniform_512()
    r = emu.solve(0, pr.d, pr.z, pr.scalar)
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "V")
    assert np.all(np.diff(r["lam"]) < 0)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 130])
def test_small_and_ragged(n, oracle_lib):
    pr = W.uniform_arrow(n, np.random.default_rng(n))
    sh = W.shuffled(pr, 5)
    r = emu.solve(0, sh.d, sh.z, sh.scalar)
    ref = oracle.arrow_eig(sh.d, sh.z, sh.scalar)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "V")


def test_graded_with_clusters(oracle_lib):
    pr = W.graded_arrow(400, np.random.default_rng(17), clusters=10, cluster_size=8)
    r = emu.solve(0, pr.d, pr.z, pr.scalar)
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "V")


@pytest.mark.parametrize("n", [1, 2, 60, 300])
def test_dpr1(n, oracle_lib):
    pr = W.dpr1(n, np.random.default_rng(40 + n))
    r = emu.solve(1, pr.d, pr.z, pr.scalar)
    ref = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "Q")


@pytest.mark.parametrize("n", [1, 2, 97, 600])
def test_dpr1_negative_rho(n, oracle_lib):
    """rho < 0: solved as the negation of (-D) + |rho| u u^T."""
    pr = W.dpr1(n, np.random.default_rng(45 + n))
    r = emu.solve(1, pr.d, pr.z, -pr.scalar)
    ref = oracle.dpr1_eig(pr.d, pr.z, -pr.scalar)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "Q")


def _herm_case(n, seed):
    rng = np.random.default_rng(seed)
    m = n - 1
    d = W._sorted_with_gap(rng, m, -1.0, 1.0)[rng.permutation(m)]
    z = rng.uniform(0.1, 1.0, m) * np.exp(2j * np.pi * rng.uniform(0.0, 1.0, m))
    return d, z, float(rng.uniform(-1.0, 1.0))


def assert_close_c(got, ref, what, tol=TOL):
    """Complex entries: |got - ref| / |ref| componentwise."""
    den = np.abs(ref)
    e = np.where(den == 0, np.abs(got - ref), np.abs(got - ref) / np.where(den == 0, 1, den))
    worst = float(e.max()) if e.size else 0.0
    assert worst <= tol, f"{what}: max relative error {worst:.3e}"


@pytest.mark.parametrize("n", [1, 2, 97, 400])
def test_hermitian(n, oracle_lib):
    """Hermitian arrowhead (Sec. 6.1): the real solver on |z|, vectors with the complex z."""
    d, z, a = _herm_case(n, 90 + n)
    r = emu.solve(3, d, z, a)
    ref = oracle.herm_eig(d, z, a)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close_c(r["V"], ref.vec, "U")


def test_hermitian_reducible_reported(oracle_lib):
    r = emu.solve(3, np.array([1.0, 0.5]), np.array([0.0, 1.0 + 1.0j]), 0.0)
    assert np.all(r["info"] & 16) and np.all(np.isnan(r["lam"]))


@pytest.mark.parametrize("n", [2, 60, 300])
def test_svd(n, oracle_lib):
    pr = W.svd_arrow(n, np.random.default_rng(50 + n))
    r = emu.solve(2, pr.d, pr.z, pr.scalar)
    ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
    assert_close(r["lam"], ref.sigma, "sigma")
    assert_close(r["V"], ref.V, "V")
    assert_close(r["U"], ref.U, "U")


REDUCIBLE = [
    (np.array([1.0, 3.0, 1.0, 0.5, 1.0, -2.0]), np.array([2.0, 1.0, -1.5, 3.0, 0.25, 0.0]), 0.3),
    (np.array([0.5, -1.0, 2.0]), np.array([0.0, 0.0, 0.0]), 0.7),
    (np.array([2.0, 2.0, 2.0, 2.0]), np.array([1.0, -2.0, 0.5, 3.0]), -1.0),
    (np.array([0.0, 1.0, 0.0, 1.0]), np.array([0.0, 1.0, 1.0, 2.0]), 0.0),
]


@pytest.mark.parametrize("i", range(len(REDUCIBLE)))
def test_reducible_deflated(i, oracle_lib):
    """Deflation of zero shaft entries and repeated poles (Sec. 1) against the oracle's."""
    d, z, a = REDUCIBLE[i]
    r = emu.solve(0, d, z, a)
    ref = oracle.arrow_eig(d, z, a)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "V")
    assert np.array_equal((r["info"] & 1024) != 0, ref.tau == 0)
    assert_close(r["shift"] + r["mu"], ref.lam, "shift+mu")


@pytest.mark.parametrize("n,seed", [(2, 1), (9, 2), (300, 3), (1001, 4)])
def test_reducible_random(n, seed, oracle_lib):
    pr = W.reducible_arrow(n, np.random.default_rng(seed), zero_frac=0.2, repeat_every=5)
    r = emu.solve(0, pr.d, pr.z, pr.scalar)
    ks = np.arange(0, n, max(1, n // 60))
    ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar, ks=ks)
    assert_close(r["lam"][ks], ref.lam, "lambda")
    assert_close(r["V"][:, ks], ref.vec, "V")


def test_other_kinds_reducible_reported(oracle_lib):
    """DPR1 and SVD inputs that are reducible are reported, not solved."""
    r = emu.solve(1, np.array([1.0, 1.0, 0.5]), np.array([1.0, 2.0, 3.0]), 1.0)
    assert np.all(r["info"] & 16) and np.all(np.isnan(r["lam"]))
    r = emu.solve(2, np.array([1.0, 0.7, 0.5]), np.array([1.0, 0.0, 3.0]), 0.5)
    assert np.all(r["info"] & 16) and np.all(np.isnan(r["lam"]))


@pytest.mark.parametrize("k", [-100, 20, 100])
def test_power_of_two_scaling_is_exact(k, oracle_lib):
    """Scaling every input by 2^k scales every eigenvalue (singular value) by 2^k and leaves
    the vectors unchanged, bit for bit: no step of the method uses an absolute threshold.
    (k stays where no intermediate square or product leaves the normal range; at 2^-300 the
    graded and SVD cases reach subnormals.)"""
    s = 2.0 ** k
    rng = np.random.default_rng(60)
    cases = [(0, W.graded_arrow(300, rng, clusters=4, cluster_size=8)), (1, W.dpr1(200, rng)),
             (2, W.svd_arrow(150, rng))]
    for kind, pr in cases:
        a = emu.solve(kind, pr.d, pr.z, pr.scalar)
        zs = pr.z if kind == 1 else pr.z * s          # DPR1: D and rho scale, u does not
        b = emu.solve(kind, pr.d * s, zs, pr.scalar * s)
        assert np.array_equal(b["lam"], a["lam"] * s), kind
        assert np.array_equal(b["V"], a["V"]), kind


@pytest.mark.parametrize("case,mean_max,worst_max", [
    ("graded_1024", 2.5, 7), ("graded_2048_c16", 2.4, 6), ("uniform_512", 4.0, 7), ("graded_4096", 2.3, 8)])
def test_rational_passes_stay_few(case, mean_max, worst_max):
    """The secular iteration for the extreme eigenvalue of A_i^{-1}, with each step confined by
    the lower (tangent of the far poles) and upper (nearest-pole fit) model bounds on the zero:
    spectra spread over 20 decades with tight clusters converge in a few O(n) passes, the worst
    eigenvalue included (it took 8-10 before the bounds were kept)."""
    pr = {"graded_1024": lambda: W.graded_arrow(1024, np.random.default_rng(201)),
          "graded_2048_c16": lambda: W.graded_arrow(2048, np.random.default_rng(202), clusters=16),
          "uniform_512": W.single_uniform_512, "graded_4096": W.single_graded_4096}[case]()
    r = emu.solve(0, pr.d, pr.z, pr.scalar, vectors=False)
    it = r["cnt"][:, 0]
    assert it.mean() <= mean_max and it.max() <= worst_max, (it.mean(), it.max())


@pytest.mark.parametrize("kind,decades,n,seed", [(0, 250, 160, 320), (0, 300, 160, 370), (1, 250, 160, 321),
                                                 (2, 250, 160, 322), (0, 250, 700, 80), (1, 250, 700, 81),
                                                 (2, 250, 700, 82)])
def test_spectrum_spread_over_hundreds_of_decades(kind, decades, n, seed, oracle_lib):
    """Eigenvalues within 1e-240 of their poles: the x-space quantities are then near
    1e240, so no square of one may be formed (bracket end, residue, norms).  The
    n = 700 cases are the GPU test's; their eigenvalue nearest 0 takes Remark 1
    with poles near 1e-250 on both sides of it."""
    pr = W.wide_arrow(kind, n, np.random.default_rng(seed), decades)
    r = emu.solve(kind, pr.d, pr.z, pr.scalar)
    if kind == 1:
        ref = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
        lam, vec = ref.lam, ref.vec
    elif kind == 2:
        ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
        lam, vec = ref.sigma, ref.V
        assert_close(r["U"], ref.U, "U")
    else:
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
        lam, vec = ref.lam, ref.vec
    assert np.abs(lam ** 2 if kind == 2 else lam).min() < 1e-200   # SVD: the poles are d_j^2
    assert_close(r["lam"], lam, "lambda")
    assert_close(r["V"], vec, "V")


@pytest.mark.parametrize("kind,name", [(0, "graded_1024"), (0, "uniform_512"), (1, "dpr1_600"), (2, "svd_500")])
def test_fp64_b_where_kb_is_small(kind, name, oracle_lib):
    """Algorithm 5's choice: b from the FP64 pass where its K_b is at most tau_b, the
    double-double pass elsewhere.  Still within the bar, and on graded poles most
    eigenvalues skip the double-double pass."""
    rng = np.random.default_rng(90 + kind)
    pr = {"graded_1024": lambda: W.graded_arrow(1024, rng), "uniform_512": W.single_uniform_512,
          "dpr1_600": lambda: W.dpr1(600, rng), "svd_500": lambda: W.svd_arrow(500, rng)}[name]()
    r = emu.solve(kind, pr.d, pr.z, pr.scalar, tau_b=4.0)
    if kind == 1:
        ref = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
        lam, vec = ref.lam, ref.vec
    elif kind == 2:
        ref = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
        lam, vec = ref.sigma, ref.V
    else:
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
        lam, vec = ref.lam, ref.vec
    assert_close(r["lam"], lam, "lambda")
    assert_close(r["V"], vec, "V")
    dd = r["cnt"][:, 1]                    # double-double b passes per eigenvalue
    assert np.all(dd[r["kb"] > 4.0] >= 1)   # large K_b: double-double
    if name == "graded_1024":
        assert dd.mean() < 0.2


# ---------------------------------------------------------------------------
# eigenvalues near the origin (Sec. 3, Remark 1): f(0) summed exactly where its
# terms cancel beyond double-double, the root in lambda, the norm at the scale of
# the nearest pole

import near_zero_cases as NZ  # noqa: E402


@pytest.mark.parametrize("case", NZ.arrow_cases(), ids=lambda c: c[0])
def test_near_zero_arrow(case, oracle_lib):
    _, d, z, a = case
    r = emu.solve(0, d, z, a)
    ref = oracle.arrow_eig(d, z, a)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "V")
    k = int(np.argmin(np.abs(ref.lam)))
    assert r["info"][k] & 8 and not r["info"][k] & 2048


@pytest.mark.parametrize("case", NZ.dpr1_cases(), ids=lambda c: c[0])
def test_near_zero_dpr1(case, oracle_lib):
    _, d, u, rho = case
    r = emu.solve(1, d, u, rho)
    ref = oracle.dpr1_eig(d, u, rho)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close(r["V"], ref.vec, "Q")
    k = int(np.argmin(np.abs(ref.lam)))
    assert r["info"][k] & 8 and not r["info"][k] & 2048


@pytest.mark.parametrize("case", NZ.svd_cases(), ids=lambda c: c[0])
def test_near_zero_svd(case, oracle_lib):
    _, d, z, a = case
    r = emu.solve(2, d, z, a)
    ref = oracle.arrow_svd(d, z, a)
    assert_close(r["lam"], ref.sigma, "sigma")
    assert_close(r["V"], ref.V, "V")
    assert_close(r["U"], ref.U, "U")
    assert r["info"][-1] & 8


@pytest.mark.parametrize("case", NZ.herm_cases(), ids=lambda c: c[0])
def test_near_zero_hermitian(case, oracle_lib):
    _, d, z, a = case
    r = emu.solve(3, d, z, a)
    ref = oracle.herm_eig(d, z, a)
    assert_close(r["lam"], ref.lam, "lambda")
    assert_close_c(r["V"], ref.vec, "U")
    assert r["info"][int(np.argmin(np.abs(ref.lam)))] & 8


def test_batched_check_stage_order(oracle_lib):
    """The batched plan's check stage (Remark 2 and the DPR1 re-measure in the check itself,
    eigenvalues near the origin listed and repaired afterwards) against the oracle, over the
    mixed problems of the GPU batch tests and the near-zero cases."""
    import test_gpu_batch as TB
    probs = TB._mixed(45, 1)
    probs += [W.Problem(W.KIND_ARROW, d.size + 1, d, z, a) for _, d, z, a in NZ.arrow_cases()]
    probs += [W.Problem(W.KIND_DPR1, d.size, d, u, r) for _, d, u, r in NZ.dpr1_cases()]
    emu.set_batch_check(True)
    try:
        for p, pr in enumerate(probs):
            r = emu.solve(pr.kind, pr.d, pr.z, pr.scalar)
            rl, rV, rU = TB._oracle(pr)
            assert_close(r["lam"], rl, f"problem {p} values")
            if pr.kind == W.KIND_HERM:
                assert_close_c(r["V"], rV, f"problem {p} vectors")
            else:
                assert_close(r["V"], rV, f"problem {p} vectors")
            if rU is not None:
                assert_close(r["U"], rU, f"problem {p} left vectors")
    finally:
        emu.set_batch_check(False)
