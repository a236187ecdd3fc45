"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's formulas: eigenvalues are checked against
exact-rational inertia bisection and mpmath's dense Jacobi solver, against the
paper's worked examples (tests/golden/), and against identities the oracle
never evaluates (trace, determinant, the Loewner reconstruction of z from the
spectrum in Sec. 1, the eigenvector-eigenvalue identity, orthogonality, exact
invariances).  The last test plants mistakes in copies of the oracle and
checks that these pins catch every one.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import brute
import oracle
from paper_1302_7203_amd import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def F(x):
    return Fraction(float(x))


def hilo(hi, lo):
    return F(hi) + F(lo)


def mpf2(hi, lo):
    return mp.mpf(float(hi)) + mp.mpf(float(lo))


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = rest
    return vals


def within_printed(value, printed: str, units=1.5):
    """|value - printed| <= units * (one unit of the last printed digit)."""
    s = printed.lower()
    mant, _, exp = s.partition("e")
    exp = int(exp) if exp else 0
    mant = mant.lstrip("+-")
    if "." in mant:
        ndec = len(mant.split(".")[1])
    else:
        ndec = 0
    unit = mp.mpf(10) ** (exp - ndec)
    return abs(mp.mpf(value) - mp.mpf(printed)) <= units * unit


# ---------------------------------------------------------------------------
# small cases with exact answers

def _tiny_cases():
    eps = 2.0 ** -52
    rng = np.random.default_rng(11)
    cases = []
    for n in (2, 3, 4, 5, 6):
        d = np.sort(rng.uniform(-1, 1, n - 1))[::-1]
        z = rng.uniform(0.1, 1, n - 1) * np.where(rng.uniform(size=n - 1) < 0.5, -1, 1)
        cases.append((d, z, float(rng.uniform(-1, 1))))
    # graded magnitudes, tiny shaft entries
    cases.append((np.array([3e8, 2.5, -1e-6, -7e3]), np.array([1e-7, 2.0, 3e-5, 1e2]), 1e-3))
    # poles 1 + k*eps (Example 2 style)
    cases.append((np.array([1 + 3 * eps, 1 + 2 * eps, 1 + eps]), np.array([1.0, 2.0, 3.0]), 0.0))
    # a zero pole and an eigenvalue near zero
    cases.append((np.array([2e-3, 0.0, -2e-3]), np.array([1e3, 1.0, 1e3]), 1e9))
    return cases


@pytest.mark.parametrize("case", range(8))
def test_arrow_exact_inertia(case, oracle_lib):
    d, z, alpha = _tiny_cases()[case]
    n = d.size + 1
    A = brute.dense_arrow(d, z, alpha)
    lam_exact = brute.exact_eigvals(A, rel_bits=170)
    r = oracle.arrow_eig(d, z, alpha)
    for k in range(n):
        got = hilo(r.lam[k], r.lam_lo[k])
        assert abs(got - lam_exact[k]) <= abs(lam_exact[k]) * Fraction(1, 10 ** 25), (k, float(got), float(lam_exact[k]))
        assert r.lam[k] == float(lam_exact[k])  # the double itself is the rounding of the exact value
        x = brute.exact_null_vector(A, lam_exact[k])
        col = r.vec[:, k]
        assert col[-1] < 0                      # sign convention x_n = -1 (eq. Aeigenvec)
        scale = -F(col[-1])
        for j in range(n - 1):
            ratio = F(col[j]) / scale
            assert abs(ratio - x[j]) <= abs(x[j]) * Fraction(4, 10 ** 16), (k, j)
        nrm = sum(F(c) ** 2 for c in col)
        assert abs(nrm - 1) < Fraction(1, 10 ** 15)


@pytest.mark.parametrize("n,seed,graded", [(9, 1, False), (16, 2, False), (14, 3, True), (24, 4, True)])
def test_arrow_mpmath_dense(n, seed, graded, oracle_lib):
    rng = np.random.default_rng(seed)
    pr = W.graded_arrow(n, rng, clusters=1, cluster_size=3) if graded else W.uniform_arrow(n, rng)
    r = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    lam, vec = brute.mp_eigsy(brute.arrow_np(pr.d, pr.z, pr.scalar), dps=70)
    with mp.workdps(70):
        for k in range(n):
            got = mpf2(r.lam[k], r.lam_lo[k])
            assert abs(got - lam[k]) <= abs(lam[k]) * mp.mpf("1e-25"), k
            v = [mp.mpf(float(x)) for x in r.vec[:, k]]
            s = 1 if sum(a * b for a, b in zip(v, vec[k])) > 0 else -1
            for j in range(n):
                ref = s * vec[k][j]
                assert abs(v[j] - ref) <= abs(ref) * mp.mpf("2.3e-16") + mp.mpf("1e-55"), (k, j)


# ---------------------------------------------------------------------------
# worked examples of Sec. 5

def test_example1_printed_values(oracle_lib):
    g = read_golden("ex1.txt")
    d = np.array([float(x) for x in g["d"]])
    z = np.array([float(x) for x in g["z"]])
    alpha = float(g["alpha"][0])
    r = oracle.arrow_eig(d, z, alpha)
    with mp.workdps(40):
        for k, p in enumerate(g["lambda"]):
            assert within_printed(mpf2(r.lam[k], r.lam_lo[k]), p), (k, p)
        v4 = r.vec[:, 3]
        printed = g["v4"]
        sgn = -1.0   # reading 2: the printed vector is -x/||x||
        for j, p in enumerate(printed):
            assert within_printed(sgn * v4[j], p, units=float(g["v4_units"][0])), (j, p, v4[j])


def test_example2_32_digits_and_pairs(oracle_lib):
    g = read_golden("ex2.txt")
    eps = 2.0 ** int(g["eps_pow2"][0])
    d = np.array([1 + int(k) * eps for k in g["dk"]])
    z = np.array([float(x) for x in g["z"]])
    r = oracle.arrow_eig(d, z, float(g["alpha"][0]))
    with mp.workdps(50):
        for k, p in enumerate(g["lambda32"]):
            # 32 printed digits; the oracle itself is good to relerr (~1e-28 relative)
            got = mpf2(r.lam[k], r.lam_lo[k])
            slack = 2 * mp.mpf(float(r.relerr[k])) * abs(got)
            assert abs(got - mp.mpf(p)) <= slack + mp.mpf(10) ** -31 * 0.51 * abs(mp.mpf(p)) * 10, (k, p)
    # lambda_2..lambda_4 round to 1 + 4e, 1 + 3e, 1 + 2e
    for k, mult in zip(g["lambda_fp64_k"], g["lambda_fp64_epsmult"]):
        assert r.lam[int(k)] == 1 + int(mult) * eps
    # the (pole, mu) pairs of Remark 3: reference pole and mu / eps to 10 digits
    for i, k in enumerate((1, 2, 3)):
        assert r.pole[k] == k - 1
        assert within_printed(r.tau[k] / eps, g["mu_over_eps"][i], units=0.51)


def test_example3_printed_values(oracle_lib):
    g = read_golden("ex3.txt")
    d = np.array([float(x) for x in g["d"]])
    z = np.array([float(x) for x in g["z"]])
    r = oracle.arrow_eig(d, z, float(g["alpha"][0]))
    with mp.workdps(40):
        for k, p in enumerate(g["lambda"]):
            assert within_printed(mpf2(r.lam[k], r.lam_lo[k]), p), (k, p)
        # the FP64-only column is really wrong: it misses the exact values by >1e-12 for k=1..5
        for k in range(1, 6):
            ex = mpf2(r.lam[k], r.lam_lo[k])
            assert abs(mp.mpf(g["lambda_basic"][k]) - ex) > abs(ex) * mp.mpf("1e-12")


# ---------------------------------------------------------------------------
# identities the oracle never evaluates

def _mp_pole_diff(r, d, k, i):
    """lam_k - d_i from the oracle's (pole, tau) pair, exactly in mp."""
    return (mp.mpf(float(d[r.pole[k]])) - mp.mpf(float(d[i]))) + mpf2(r.tau[k], r.tau_lo[k])


@pytest.mark.parametrize("which", ["uniform", "graded"])
def test_arrow_identities(which, oracle_lib):
    rng = np.random.default_rng(5)
    pr = W.uniform_arrow(160, rng) if which == "uniform" else W.graded_arrow(160, rng, clusters=4, cluster_size=8)
    d, z, alpha = pr.d, pr.z, pr.scalar
    n = d.size + 1
    r = oracle.arrow_eig(d, z, alpha)
    assert np.all(r.relerr < 1e-26)
    with mp.workdps(60):
        lam = [mpf2(a, b) for a, b in zip(r.lam, r.lam_lo)]
        # strict interlacing (eq. interlace)
        for k in range(n - 1):
            assert lam[k] > mp.mpf(float(d[k])) > lam[k + 1]
        # trace
        tr = sum(mp.mpf(float(x)) for x in d) + mp.mpf(alpha)
        assert abs(sum(lam) - tr) <= mp.mpf("1e-26") * max(abs(x) for x in lam) * n
        # determinant via the Schur complement of D
        det = mp.fprod(mp.mpf(float(x)) for x in d) * (
            mp.mpf(alpha) - mp.fsum(mp.mpf(float(zz)) ** 2 / mp.mpf(float(dd)) for dd, zz in zip(d, z)))
        assert abs(mp.fprod(lam) - det) <= abs(det) * mp.mpf("1e-22")
        # Loewner reconstruction of zeta_i^2 from the spectrum (Sec. 1): pins every tau
        for i in range(0, n - 1, 7):
            num = mp.fprod(-_mp_pole_diff(r, d, k, i) for k in range(n))
            den = mp.fprod(mp.mpf(float(d[i])) - mp.mpf(float(d[l])) for l in range(n - 1) if l != i)
            z2 = -num / den
            assert abs(z2 - mp.mpf(float(z[i])) ** 2) <= mp.mpf(float(z[i])) ** 2 * mp.mpf("1e-22"), i
        # eigenvector-eigenvalue identity for the last row
        for k in range(0, n, 9):
            num = mp.fprod(_mp_pole_diff(r, d, k, j) for j in range(n - 1))
            den = mp.fprod(_mp_pole_diff(r, d, k, r.pole[l]) - mpf2(r.tau[l], r.tau_lo[l]) for l in range(n) if l != k)
            assert abs(mp.mpf(float(r.vec[-1, k])) ** 2 - num / den) <= abs(num / den) * mp.mpf("1e-14"), k
    V = r.vec.astype(np.longdouble)
    assert np.max(np.abs(V.T @ V - np.eye(n))) < 1e-14
    A = brute.arrow_np(d, z, alpha).astype(np.longdouble)
    res = A @ V - V * r.lam.astype(np.longdouble)
    assert np.max(np.abs(res)) <= 1e-14 * np.max(np.abs(r.lam))


def test_special_and_invariances(oracle_lib):
    r = oracle.arrow_eig(np.zeros(0), np.zeros(0), 0.75)
    assert r.lam[0] == 0.75 and r.vec.shape == (1, 1) and r.vec[0, 0] == -1.0
    # n = 2 closed form
    d, z, a = np.array([0.3]), np.array([0.7]), -0.2
    r = oracle.arrow_eig(d, z, a)
    with mp.workdps(50):
        c, h = (mp.mpf(0.3) + mp.mpf(-0.2)) / 2, (mp.mpf(0.3) - mp.mpf(-0.2)) / 2
        rt = mp.sqrt(h * h + mp.mpf(0.7) ** 2)
        for k, ex in enumerate((c + rt, c - rt)):
            assert abs(mpf2(r.lam[k], r.lam_lo[k]) - ex) <= abs(ex) * mp.mpf("1e-27")
    pr = W.uniform_arrow(40, np.random.default_rng(9))
    base = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    # exact scaling by a power of two
    sc = oracle.arrow_eig(pr.d * 2.0 ** 37, pr.z * 2.0 ** 37, pr.scalar * 2.0 ** 37)
    assert np.array_equal(sc.lam, base.lam * 2.0 ** 37) and np.array_equal(sc.vec, base.vec)
    # permutation of the input order permutes rows only
    sh = W.shuffled(pr, 3)
    ps = oracle.arrow_eig(sh.d, sh.z, sh.scalar)
    perm = sh.meta["perm"]
    assert np.array_equal(ps.lam, base.lam)
    assert np.array_equal(ps.vec[:-1], base.vec[perm]) and np.array_equal(ps.vec[-1], base.vec[-1])
    # sign flip of one shaft entry flips one row
    z2 = pr.z.copy()
    z2[5] = -z2[5]
    fl = oracle.arrow_eig(pr.d, z2, pr.scalar)
    assert np.array_equal(fl.lam, base.lam)
    assert np.array_equal(fl.vec[5], -base.vec[5])
    other = np.arange(pr.n) != 5
    assert np.array_equal(fl.vec[other], base.vec[other])


# ---------------------------------------------------------------------------
# reducible input (Sec. 1): deflation

# (d, z, alpha): unsorted, with a zero shaft entry and a pole taken three
# times; a diagonal matrix; all poles equal; a zero pole with a zero shaft
# entry beside an equal pair
REDUCIBLE = [
    (np.array([1.0, 3.0, 1.0, 0.5, 1.0, -2.0]), np.array([2.0, 1.0, -1.5, 3.0, 0.25, 0.0]), 0.3),
    (np.array([0.5, -1.0, 2.0]), np.array([0.0, 0.0, 0.0]), 0.7),
    (np.array([2.0, 2.0, 2.0, 2.0]), np.array([1.0, -2.0, 0.5, 3.0]), -1.0),
    (np.array([0.0, 1.0, 0.0, 1.0]), np.array([0.0, 1.0, 1.0, 2.0]), 0.0),
]
_EXACT = {}


def _exact_reducible(i):
    if i not in _EXACT:
        d, z, a = REDUCIBLE[i]
        _EXACT[i] = brute.exact_eigvals(brute.dense_arrow(d, z, a))
    return _EXACT[i]


def _deflation_failures(i, r):
    """What the mathematics fixes for REDUCIBLE[i] and the oracle's result r."""
    d, z, a = REDUCIBLE[i]
    n = d.size + 1
    bad = []
    for k, e in enumerate(_exact_reducible(i)):       # rounded once: within half an ulp
        if abs(F(r.lam[k]) - e) > abs(e) * Fraction(1, 2 ** 53) + Fraction(1, 2 ** 399):   # the bisection floor
            bad.append(f"lambda_{k}")
    A = brute.arrow_np(d, z, a).astype(np.longdouble)
    V = r.vec.astype(np.longdouble)
    tol = 4 * n * 2.0 ** -53
    if np.max(np.abs(V.T @ V - np.eye(n))) > tol:
        bad.append("orthonormal")
    if np.max(np.abs(A @ V - V * r.lam.astype(np.longdouble))) > tol * float(np.max(np.abs(A))):
        bad.append("residual")
    # z_j = 0: the eigenpair (d_j, e_j)
    for j in np.flatnonzero(z == 0):
        e = np.zeros(n)
        e[j] = 1.0
        if not any(r.lam[k] == d[j] and np.array_equal(r.vec[:, k], e) for k in range(n)):
            bad.append(f"unit vector e_{j}")
    for k in range(n):
        p = int(r.pole[k])
        if r.tau[k] == 0 and p >= 0 and z[p] != 0:
            # a direction removed from a run of equal poles: supported on the
            # run, negative on its own row
            off = (d != d[p]) & (r.vec[:-1, k] != 0)
            if off.any() or r.vec[-1, k] != 0 or not r.vec[p, k] < 0:
                bad.append(f"rotation vector {k}")
        elif r.tau[k] != 0 and not r.vec[-1, k] < 0:
            bad.append(f"corner sign {k}")
    return bad


@pytest.mark.parametrize("i", range(len(REDUCIBLE)))
def test_deflation_pins(i, oracle_lib):
    d, z, a = REDUCIBLE[i]
    r = oracle.arrow_eig(d, z, a)
    assert _deflation_failures(i, r) == []


def test_deflation_larger_random(oracle_lib):
    """n = 60 with zero shaft entries and repeated poles: against mpmath's dense solver at 40 digits."""
    pr = W.reducible_arrow(60, np.random.default_rng(31), zero_frac=0.15, repeat_every=7)
    r = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    lam, _ = brute.mp_eigsy(brute.arrow_np(pr.d, pr.z, pr.scalar), dps=40)
    for k in range(pr.n):
        assert abs(mp.mpf(float(r.lam[k])) - lam[k]) <= abs(lam[k]) * mp.mpf(2.0 ** -53) + mp.mpf("1e-30")
    A = brute.arrow_np(pr.d, pr.z, pr.scalar).astype(np.longdouble)
    V = r.vec.astype(np.longdouble)
    assert np.max(np.abs(V.T @ V - np.eye(pr.n))) < 1e-14
    assert np.max(np.abs(A @ V - V * r.lam.astype(np.longdouble))) < 1e-14
    assert np.all(np.diff(r.lam) <= 0)


# ---------------------------------------------------------------------------
# DPR1 (Sec. 6.3) and SVD (Sec. 6.2)

@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (6, 3)])
def test_dpr1_exact_inertia(n, seed, oracle_lib):
    pr = W.dpr1(n, np.random.default_rng(seed))
    M = brute.dense_dpr1(pr.d, pr.z, pr.scalar)
    lam_exact = brute.exact_eigvals(M, rel_bits=170)
    r = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
    for k in range(n):
        got = hilo(r.lam[k], r.lam_lo[k])
        assert abs(got - lam_exact[k]) <= abs(lam_exact[k]) * Fraction(1, 10 ** 25)
        x = brute.exact_null_vector(M, lam_exact[k])
        col = r.vec[:, k]
        for j in range(n - 1):
            ratio = F(col[j]) / F(col[-1])
            assert abs(ratio - x[j] / x[-1]) <= abs(x[j] / x[-1]) * Fraction(4, 10 ** 16)
        # convention q ~ +(D - lam I)^{-1} u: the row of the smallest pole (lam > d_min)
        jmin = int(np.argmin(pr.d))
        assert np.sign(col[jmin]) == -np.sign(pr.z[jmin])
    # interlacing (eq. lld) and trace
    ds = np.sort(pr.d)[::-1]
    for k in range(n):
        assert r.lam[k] > ds[k] if r.lam_lo[k] >= 0 or r.lam[k] != ds[k] else False


def _dpr1_negative_failures(pr, r):
    """D + rho u u^T with rho < 0: exact eigenvalues, interlacing from below
    (d_{k+1} < lambda_k < d_k), exact null vectors and q ~ +(D - lambda I)^{-1} u."""
    bad = []
    n = pr.n
    M = brute.dense_dpr1(pr.d, pr.z, pr.scalar)
    lam_exact = brute.exact_eigvals(M, rel_bits=170)
    ds = np.sort(pr.d)[::-1]
    for k in range(n):
        if abs(hilo(r.lam[k], r.lam_lo[k]) - lam_exact[k]) > abs(lam_exact[k]) * Fraction(1, 10 ** 25):
            bad.append(f"lambda_{k}")
        if not (lam_exact[k] < F(ds[k]) and (k == n - 1 or lam_exact[k] > F(ds[k + 1]))):
            bad.append(f"interlacing {k}")
        x = brute.exact_null_vector(M, lam_exact[k]) if n > 1 else [Fraction(-1)]
        col = r.vec[:, k]
        for j in range(n - 1):
            if abs(F(col[j]) / F(col[-1]) - x[j] / x[-1]) > abs(x[j] / x[-1]) * Fraction(4, 10 ** 16):
                bad.append(f"vector {k}")
                break
        # the row of the largest pole: lambda_k < d_max, so (d_max - lambda) u > 0 in sign
        jmax = int(np.argmax(pr.d))
        if np.sign(col[jmax]) != np.sign(pr.z[jmax]):
            bad.append(f"sign {k}")
    return bad


@pytest.mark.parametrize("n,seed", [(1, 6), (3, 7), (6, 8)])
def test_dpr1_negative_rho(n, seed, oracle_lib):
    pr = W.dpr1(n, np.random.default_rng(seed))
    pr.scalar = -pr.scalar
    assert _dpr1_negative_failures(pr, oracle.dpr1_eig(pr.d, pr.z, pr.scalar)) == []


@pytest.mark.parametrize("n,seed", [(12, 4), (20, 5)])
def test_dpr1_mpmath_dense(n, seed, oracle_lib):
    pr = W.dpr1(n, np.random.default_rng(seed))
    r = oracle.dpr1_eig(pr.d, pr.z, pr.scalar)
    Mnp = np.diag(pr.d) + pr.scalar * np.outer(pr.z, pr.z)
    with mp.workdps(70):
        Mmp = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                Mmp[i, j] = (mp.mpf(float(pr.d[i])) if i == j else 0) + mp.mpf(pr.scalar) * mp.mpf(float(pr.z[i])) * mp.mpf(float(pr.z[j]))
        E, Q = mp.eigsy(Mmp)
        order = sorted(range(n), key=lambda i: -E[i])
        for k, i in enumerate(order):
            got = mpf2(r.lam[k], r.lam_lo[k])
            assert abs(got - E[i]) <= abs(E[i]) * mp.mpf("1e-25")
            v = [mp.mpf(float(x)) for x in r.vec[:, k]]
            s = 1 if sum(v[j] * Q[j, i] for j in range(n)) > 0 else -1
            for j in range(n):
                assert abs(v[j] - s * Q[j, i]) <= abs(Q[j, i]) * mp.mpf("2.3e-16") + mp.mpf("1e-55")
        tr = mp.fsum(mp.mpf(float(x)) for x in pr.d) + mp.mpf(pr.scalar) * mp.fsum(mp.mpf(float(x)) ** 2 for x in pr.z)
        assert abs(mp.fsum(mpf2(a, b) for a, b in zip(r.lam, r.lam_lo)) - tr) < mp.mpf("1e-26") * n
    assert Mnp.shape == (n, n)


@pytest.mark.parametrize("n,seed", [(6, 1), (14, 2)])
def test_svd_mpmath_dense(n, seed, oracle_lib):
    pr = W.svd_arrow(n, np.random.default_rng(seed))
    r = oracle.arrow_svd(pr.d, pr.z, pr.scalar)
    m = n - 1
    B = np.zeros((n, n))
    B[np.arange(m), np.arange(m)] = pr.d
    B[:m, m] = pr.z
    B[m, m] = pr.scalar
    s, u, v = brute.mp_svd(B, dps=70)
    with mp.workdps(70):
        for k in range(n):
            got = mpf2(r.sigma[k], r.sigma_lo[k])
            assert abs(got - s[k]) <= s[k] * mp.mpf("1e-25")
            vv = [mp.mpf(float(x)) for x in r.V[:, k]]
            uu = [mp.mpf(float(x)) for x in r.U[:, k]]
            sg = 1 if sum(a * b for a, b in zip(vv, v[k])) > 0 else -1
            for j in range(n):
                assert abs(vv[j] - sg * v[k][j]) <= abs(v[k][j]) * mp.mpf("2.3e-16") + mp.mpf("1e-50")
                assert abs(uu[j] - sg * u[k][j]) <= abs(u[k][j]) * mp.mpf("4.5e-16") + mp.mpf("1e-50")
        fro = mp.fsum(mp.mpf(float(x)) ** 2 for x in B.ravel())
        assert abs(mp.fsum(mpf2(a, b) ** 2 for a, b in zip(r.sigma, r.sigma_lo)) - fro) < fro * mp.mpf("1e-26")
        det = abs(mp.mpf(pr.scalar) * mp.fprod(mp.mpf(float(x)) for x in pr.d))
        assert abs(mp.fprod(mpf2(a, b) for a, b in zip(r.sigma, r.sigma_lo)) - det) < det * mp.mpf("1e-24")
    Bl = B.astype(np.longdouble)
    U, V = r.U.astype(np.longdouble), r.V.astype(np.longdouble)
    assert np.max(np.abs(Bl @ V - U * r.sigma.astype(np.longdouble))) < 1e-15 * r.sigma[0]
    assert np.max(np.abs(U.T @ U - np.eye(n))) < 1e-14


# ---------------------------------------------------------------------------
# Hermitian arrowhead (Sec. 6.1)

def _herm_case(n, seed):
    rng = np.random.default_rng(seed)
    m = n - 1
    d = W._sorted_with_gap(rng, m, -1.0, 1.0)[rng.permutation(m)]
    z = rng.uniform(0.1, 1.0, m) * np.exp(2j * np.pi * rng.uniform(0.0, 1.0, m))
    return d, z, float(rng.uniform(-1.0, 1.0))


def _herm_failures(d, z, a, r, dps=40):
    """Against mpmath's dense Hermitian solver: eigenvalues to 1e-25 relative,
    eigenvectors (phase fixed by the real negative corner entry) to 2.3e-16."""
    bad = []
    n = d.size + 1
    with mp.workdps(dps):
        C = mp.matrix(n, n)
        for j in range(n - 1):
            C[j, j] = mp.mpf(float(d[j]))
            C[j, n - 1] = mp.mpc(float(z[j].real), float(z[j].imag))
            C[n - 1, j] = mp.mpc(float(z[j].real), -float(z[j].imag))
        C[n - 1, n - 1] = mp.mpf(a)
        E, Q = mp.eighe(C)
        order = sorted(range(n), key=lambda i: -E[i])
        for k, i in enumerate(order):
            if abs(mpf2(r.lam[k], r.lam_lo[k]) - E[i]) > abs(E[i]) * mp.mpf("1e-25"):
                bad.append(f"lambda_{k}")
            c = Q[n - 1, i]
            ph = -mp.conj(c) / abs(c)          # makes the corner entry real and negative
            for j in range(n):
                want = Q[j, i] * ph
                got = mp.mpc(float(r.vec[j, k].real), float(r.vec[j, k].imag))
                if abs(got - want) > abs(want) * mp.mpf("2.3e-16") + mp.mpf("1e-50"):
                    bad.append(f"vector {k}")
                    break
    return bad


@pytest.mark.parametrize("n,seed", [(1, 81), (2, 82), (7, 83), (16, 84)])
def test_herm_mpmath_dense(n, seed, oracle_lib):
    d, z, a = _herm_case(n, seed)
    assert _herm_failures(d, z, a, oracle.herm_eig(d, z, a)) == []


def test_herm_phase_invariance(oracle_lib):
    """Phi^* C Phi only sees |z_j| (Sec. 6.1): z_j -> i z_j leaves every eigenvalue and
    multiplies row j of U by i, exactly."""
    d, z, a = _herm_case(30, 85)
    base = oracle.herm_eig(d, z, a)
    z2 = z.copy()
    z2[[3, 11]] *= 1j
    r = oracle.herm_eig(d, z2, a)
    assert np.array_equal(r.lam, base.lam) and np.array_equal(r.lam_lo, base.lam_lo)
    assert np.array_equal(r.vec[[3, 11]], 1j * base.vec[[3, 11]])
    keep = np.setdiff1d(np.arange(30), [3, 11])
    assert np.array_equal(r.vec[keep], base.vec[keep])


def test_herm_real_case(oracle_lib):
    """Real z: the symmetric arrowhead's decomposition (values to the last bit, vectors to an ulp)."""
    pr = W.uniform_arrow(200, np.random.default_rng(86))
    pr.z[::3] *= -1
    h = oracle.herm_eig(pr.d, pr.z.astype(np.complex128), pr.scalar)
    r = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
    assert np.array_equal(h.lam, r.lam)
    assert np.all(h.vec.imag == 0)
    assert np.max(np.abs(h.vec.real - r.vec) / np.abs(r.vec)) <= 2.3e-16


# ---------------------------------------------------------------------------
# symmetric tridiagonal (the divide-and-conquer application of Sec. 1)

def _dense_tridiag(a, b):
    n = len(a)
    T = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        T[i][i] = F(a[i])
        if i + 1 < n:
            T[i][i + 1] = T[i + 1][i] = F(b[i])
    return T


def _tridiag_failures(a, b, lam, Q):
    """Exact eigenvalues (rounded once: half an ulp, or the bisection floor), the null
    vector of T - lambda I, and the sign rule (largest entry positive)."""
    bad = []
    n = len(a)
    T = _dense_tridiag(a, b)
    ex = brute.exact_eigvals(T)
    for k in range(n):
        if abs(F(lam[k]) - ex[k]) > abs(ex[k]) * Fraction(1, 2 ** 53) + Fraction(1, 2 ** 399):
            bad.append(f"lambda_{k}")
        q = Q[:, k]
        j = int(np.argmax(np.abs(q)))
        if not q[j] > 0:
            bad.append(f"sign {k}")
        # T q = lambda q to the rounding of q: the exact residual of the rounded vector
        res = max(abs(sum(T[i][l] * F(q[l]) for l in range(n)) - ex[k] * F(q[i])) for i in range(n))
        if res > Fraction(8 * n, 2 ** 53) * (1 + max(abs(x) for x in ex)):
            bad.append(f"vector {k}")
    return bad


@pytest.mark.parametrize("n,seed", [(1, 41), (2, 42), (5, 43), (6, 44)])
def test_tridiag_exact(n, seed, oracle_lib):
    rng = np.random.default_rng(seed)
    a, b = rng.standard_normal(n), rng.standard_normal(n - 1)
    lam, Q = oracle.tridiag_eig(a, b)
    assert _tridiag_failures(a, b, lam, Q) == []


@pytest.mark.parametrize("n,seed", [(40, 45), (200, 46)])
def test_tridiag_against_lapack(n, seed, oracle_lib):
    """LAPACK's dsyevd (numpy) is normwise accurate: eigenvalues agree to a few n eps ||T||;
    the oracle's vectors are orthonormal with residual at its own rounding."""
    rng = np.random.default_rng(seed)
    a, b = rng.standard_normal(n), rng.standard_normal(n - 1)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    lam, Q = oracle.tridiag_eig(a, b)
    ev = np.linalg.eigvalsh(T)[::-1]
    tn = np.abs(T).sum(axis=1).max()
    assert np.max(np.abs(lam - ev)) <= 4 * n * 2.0 ** -53 * tn
    Tl, Ql = T.astype(np.longdouble), Q.astype(np.longdouble)
    assert np.max(np.abs(Tl @ Ql - Ql * lam.astype(np.longdouble))) <= 4 * 2.0 ** -53 * tn
    assert np.max(np.abs(Ql.T @ Ql - np.eye(n))) <= 4 * n * 2.0 ** -53


# ---------------------------------------------------------------------------
# eigenvalues near the origin: Sec. 3, Remark 1 and the exceptions (a)-(c) of
# condition (C1) in Theorem 2 (an eigenvalue far closer to 0 than to any pole)

FINE = Fraction(1, 2 ** 1400)     # bisection floor well below the smallest double


def _bracket_count(A, lam, k, rel=Fraction(1, 10 ** 25)):
    """Exact inertia on both sides of lam: True when exactly the eigenvalue of
    rank k (0 = largest) lies within lam (1 +- rel)."""
    n = len(A)
    w = abs(lam) * rel + Fraction(1, 2 ** 1072)    # hi + lo with a subnormal lo word
    lo, hi = brute._count_below(A, lam - w), brute._count_below(A, lam + w)
    return lo == n - 1 - k and hi == n - k


# (d, z, alpha): 3x3 cases have closed forms near alpha/(1 + sum z^2/d^2); the
# quotients z^2/d of (3, -3) and (6, 3, -2) are not dyadic, so their exact
# cancellation needs more than one binary128 digit
NEAR_ZERO = [
    ([1.0, -1.0], [1.0, 1.0], 1e-12),
    ([1.0, -1.0], [1.0, 1.0], 1e-20),
    ([1.0, -1.0], [1.0, 1.0], 1e-30),
    ([1.0, -1.0], [1.0, 1.0], -3e-200),
    ([3.0, -3.0], [1.0, 1.0], 1e-30),
    ([3.0, -3.0], [1.0, 1.0], -3e-200),
    ([6.0, 3.0, -2.0], [1.0, 1.0, 1.0], 1e-30),
    ([6.0, 3.0, -2.0], [1.0, 1.0, 1.0], -2.5e-300),
    ([6.0, 3.0, -2.0], [1.0, 1.0, 1.0], 3e-3),       # inside the window, |l/d| ~ 1e-3
    ([-0.5, -4.0], [1.0, 2.0], -3.0 + 2.0 ** -40),    # exterior: poles < 0, f(0) = 2^-40, l_1 ~ 2e-13
    ([2.0, 2.0, -1.0], [1.0, 1.0, 1.0], 1e-30),       # reducible: a repeated pole merged first
]


@pytest.mark.parametrize("case", range(len(NEAR_ZERO)))
def test_near_zero_exact(case, oracle_lib):
    d, z, alpha = (np.array(NEAR_ZERO[case][0]), np.array(NEAR_ZERO[case][1]), NEAR_ZERO[case][2])
    n = d.size + 1
    A = brute.dense_arrow(d, z, alpha)
    lam_exact = brute.exact_eigvals(A, rel_bits=170, abs_floor=FINE)
    r = oracle.arrow_eig(d, z, alpha)
    assert np.all(r.relerr <= 1e-25), r.relerr
    k0 = int(np.argmin(np.abs(r.lam)))
    for k in range(n):
        got = hilo(r.lam[k], r.lam_lo[k])
        # the lo word of a value near 1e-300 is subnormal: its last bit is 2^-1074
        tol = abs(lam_exact[k]) * Fraction(1, 10 ** 25) + Fraction(1, 2 ** 1074)
        assert abs(got - lam_exact[k]) <= tol, (k, float(got), float(lam_exact[k]))
        assert r.lam[k] == float(lam_exact[k])
        if k == k0 and d.size == len(set(d.tolist())):
            x = brute.exact_null_vector(A, lam_exact[k])
            scale = -F(r.vec[-1, k])
            for j in range(n - 1):
                assert abs(F(r.vec[j, k]) / scale - x[j]) <= abs(x[j]) * Fraction(4, 10 ** 16), (k, j)


def test_near_zero_random_200(oracle_lib):
    """n = 201, poles of both signs, alpha the double nearest to sum z_j^2/d_j, so
    that f(0) is a rounding error: the eigenvalue near 0 is ~1e-20, pinned by
    exact inertia on both sides of it."""
    rng = np.random.default_rng(5)
    d = np.sort(rng.uniform(-1, 1, 200))[::-1]
    z = rng.uniform(0.1, 1, 200)
    alpha = float(sum(F(b) ** 2 / F(a) for a, b in zip(d, z)))
    r = oracle.arrow_eig(d, z, alpha)
    assert np.all(r.relerr <= 1e-25)
    k = int(np.argmin(np.abs(r.lam)))
    assert abs(r.lam[k]) < 1e-15 * np.min(np.abs(d))
    assert _bracket_count(brute.dense_arrow(d, z, alpha), hilo(r.lam[k], r.lam_lo[k]), k)


@pytest.mark.parametrize("rho", [4.0, 4.0 + 2.0 ** -50, 4.0 - 2.0 ** -48])
def test_near_zero_dpr1(rho, oracle_lib):
    """D + rho uu^T with d = (2, -1, 4), u = 1: singular at rho = 4 exactly (an
    eigenvalue 0), and an eigenvalue of size ~1e-15 next to it."""
    d, u = np.array([2.0, -1.0, 4.0]), np.ones(3)
    M = brute.dense_dpr1(d, u, rho)
    lam_exact = brute.exact_eigvals(M, rel_bits=170, abs_floor=FINE)
    r = oracle.dpr1_eig(d, u, rho)
    assert np.all(r.relerr <= 1e-25)
    for k in range(3):
        got = hilo(r.lam[k], r.lam_lo[k])
        if lam_exact[k] == 0 or abs(lam_exact[k]) < FINE:
            assert got == 0 and rho == 4.0
        else:
            assert abs(got - lam_exact[k]) <= abs(lam_exact[k]) * Fraction(1, 10 ** 25), (k, float(got))


def test_near_zero_dpr1_random(oracle_lib):
    """Random d of both signs and u, rho the double nearest to -1/sum(u_j^2/d_j)."""
    rng = np.random.default_rng(8)
    d = W._sorted_with_gap(rng, 8, -1.0, 1.0)
    u = rng.uniform(0.2, 1.0, 8)
    s = sum(F(b) ** 2 / F(a) for a, b in zip(d, u))
    if s > 0:
        d = -d
        s = -s
    rho = float(-1 / s)
    M = brute.dense_dpr1(d, u, rho)
    r = oracle.dpr1_eig(d, u, rho)
    assert np.all(r.relerr <= 1e-25)
    k = int(np.argmin(np.abs(r.lam)))
    assert abs(r.lam[k]) < 1e-12
    assert _bracket_count(M, hilo(r.lam[k], r.lam_lo[k]), k)


@pytest.mark.parametrize("alpha", [1e-30, -1e-100, 3e-150])
def test_near_zero_svd(alpha, oracle_lib):
    """B = [D z; 0 alpha] with tiny alpha: the smallest singular value is ~|alpha|,
    so B^T B has an eigenvalue ~alpha^2 next to its corner alpha^2 + z^T z.
    Pinned by exact inertia of B^T B and by prod(sigma) = |alpha prod d|."""
    d, z = np.array([0.5, 0.75, 0.3]), np.array([0.9, 0.4, 0.7])
    n = 4
    B = [[Fraction(0)] * n for _ in range(n)]
    for j in range(3):
        B[j][j] = F(d[j])
        B[j][3] = F(z[j])
    B[3][3] = F(alpha)
    BtB = [[sum(B[r][i] * B[r][j] for r in range(n)) for j in range(n)] for i in range(n)]
    lam_exact = brute.exact_eigvals(BtB, rel_bits=170, abs_floor=FINE)
    r = oracle.arrow_svd(d, z, alpha)
    assert np.all(r.relerr <= 1e-25)
    with mp.workdps(80):
        for k in range(n):
            s2 = mpf2(r.sigma[k], r.sigma_lo[k]) ** 2
            ex = mp.mpf(lam_exact[k].numerator) / lam_exact[k].denominator
            assert abs(s2 - ex) <= ex * mp.mpf("1e-25"), k
        prod = mp.fprod([mpf2(a, b) for a, b in zip(r.sigma, r.sigma_lo)])
        ref = abs(mp.mpf(alpha) * mp.fprod([mp.mpf(float(x)) for x in d]))
        assert abs(prod - ref) <= ref * mp.mpf("1e-25")


def test_near_zero_hermitian(oracle_lib):
    """[diag(6, 3, -2) z; z^* alpha] with |z_j| = 1 and alpha = 1e-30, against
    mpmath's dense Hermitian solver."""
    d = np.array([6.0, 3.0, -2.0])
    z = np.array([1j, -1.0, 1j * -1.0])
    assert _herm_failures(d, z, 1e-30, oracle.herm_eig(d, z, 1e-30), dps=90) == []
    assert np.all(oracle.herm_eig(d, z, 1e-30).relerr <= 1e-25)


def test_origin_unresolved_is_reported(oracle_lib):
    """f(0) = 0 exactly with non-dyadic quotients (1/3 - 1/3): no finite number of
    binary128 digits settles it, and the oracle says so instead of guessing."""
    r = oracle.arrow_eig(np.array([3.0, -3.0]), np.array([1.0, 1.0]), 0.0)
    assert r.relerr[1] >= 1 and abs(r.lam[1]) < 1e-300
    assert np.all(r.relerr[[0, 2]] <= 1e-25)


# ---------------------------------------------------------------------------
# planted mistakes: every one must be caught by the pins above

_MUTANTS = {
    "tau_sign_in_secular": ("R t = s->c[j] / ((s->d[j] - dp) - tau);", "R t = s->c[j] / ((s->d[j] - dp) + tau);"),
    "zeta_not_squared": ("cq[j] = zz * zz;", "cq[j] = fabsq(zz);"),
    "dropped_last_term": ("  for (int64_t j = 0; j < s->m; ++j) {\n    R t = s->c[j] / ((s->d[j] - dp) - tau);",
                          "  for (int64_t j = 0; j < s->m - 1; ++j) {\n    R t = s->c[j] / ((s->d[j] - dp) - tau);"),
    "corner_sign": ("col[m] = (double)(-1 / nrm);", "col[m] = (double)(1 / nrm);"),
    "norm_without_corner": ("      R nrm2 = 1;\n      R dp = dq[r.p];", "      R nrm2 = 0;\n      R dp = dq[r.p];"),
    "dpr1_dropped_rho": ("cq[j] = (R)rho * (uu * uu);", "cq[j] = (uu * uu);"),
    "svd_corner_alpha_not_squared": ("R corner = (R)alpha * (R)alpha,", "R corner = (R)alpha,"),
    "svd_u_times_d": ("uc[j] = (double)(sg * v / dj);", "uc[j] = (double)(sg * v * dj);"),
    "ascending_order": ("return (x > y) ? -1 : (x < y) ? 1 :", "return (x < y) ? -1 : (x > y) ? 1 :"),
    "deflation_rotation_sign": ("out[row] = (double)(-cs);", "out[row] = (double)(cs);"),
    "deflation_weight_dropped": ("c += (R)zq * (R)zq;", "c += 0;"),
    "deflation_unit_row_sorted": ("out[t->row] = 1.0;", "out[t->pos] = 1.0;"),
    "deflation_merge_count": ("if (g > err) c = P + 1;", "if (g < -err) c = P + 1;"),
    "dpr1_negative_order": ("kr[i] = n - 1 - k;", "kr[i] = k;"),
    "dpr1_negative_tau_sign": ("t = -((R)th[i] + (R)tl[i])", "t = ((R)th[i] + (R)tl[i])"),
    "herm_conjugated_vector": ("col[2 * j + 1] = (double)((R)zi[j] / den);", "col[2 * j + 1] = (double)(-(R)zi[j] / den);"),
    "herm_modulus_real_part_only": ("cq[j] = (R)zr[o] * (R)zr[o] + (R)zi[o] * (R)zi[o];", "cq[j] = (R)zr[o] * (R)zr[o];"),
    "tridiag_sturm_b_not_squared": ("b2[i] = bq[i] * bq[i];", "b2[i] = fabsq(bq[i]);"),
    "tridiag_back_substitution_sign": ("s -= u1[i] * x[i + 1];", "s += u1[i] * x[i + 1];"),
    "origin_one_digit": ("for (int level = 0; level < 24; ++level)", "for (int level = 0; level < 1; ++level)"),
    "origin_digit_sign": ("ex_add(&x, -q);", "ex_add(&x, q);"),
    "origin_inexact_remainder": ("r[t] = (r[t] - p) - pe;", "r[t] = (r[t] - p);"),
    "origin_slope_sign": ("S += s->c[j] / (s->d[j] * (s->d[j] - l));", "S += s->c[j] / (s->d[j] * (s->d[j] + l));"),
    "origin_window_skipped": ("if (lo_end < 0 && hi_end > 0) {", "if (0) {"),
    "origin_dpr1_low_part_dropped": ("q_two_prod((R)rho, uu * uu, &tn[2 * j], &tn[2 * j + 1]);",
                                     "tn[2 * j] = cq[j]; tn[2 * j + 1] = 0;"),
    "origin_svd_corner_dropped": ("k0[0] = (R)alpha * (R)alpha;", "k0[0] = 0;"),
    "vector_tau_sign": ("R x = (R)z[j] / (((R)d[j] - dp) - r.tau);\n        col[j]",
                        "R x = (R)z[j] / (((R)d[j] - dp) + r.tau);\n        col[j]"),
}


def _quick_pins(lib):
    """Cheap versions of the pins above; returns the list of those that fail."""
    failed = []
    pr = W.uniform_arrow(10, np.random.default_rng(21))
    try:
        r = oracle.arrow_eig(pr.d, pr.z, pr.scalar, lib=lib)
        lam, vec = brute.mp_eigsy(brute.arrow_np(pr.d, pr.z, pr.scalar), dps=40)
        for k in range(pr.n):
            with mp.workdps(40):
                bad = abs(mpf2(r.lam[k], r.lam_lo[k]) - lam[k]) > abs(lam[k]) * mp.mpf("1e-25")
            if bad:
                failed.append("arrow eigenvalue")
                break
            v = r.vec[:, k]
            if v[-1] >= 0 or max(abs(float(a) - float(b)) for a, b in zip(v, vec[k] if vec[k][-1] < 0 else [-x for x in vec[k]])) > 1e-15:
                failed.append("arrow vector")
                break
    except oracle.oracle.OracleError:
        failed.append("arrow error")
    pr = W.dpr1(8, np.random.default_rng(22))
    try:
        r = oracle.dpr1_eig(pr.d, pr.z, pr.scalar, lib=lib)
        tr = float(np.sum(pr.d) + pr.scalar * np.sum(pr.z ** 2))
        if abs(np.sum(r.lam) - tr) > 1e-13:
            failed.append("dpr1 trace")
    except oracle.oracle.OracleError:
        failed.append("dpr1 error")
    pr = W.svd_arrow(6, np.random.default_rng(23))
    try:
        r = oracle.arrow_svd(pr.d, pr.z, pr.scalar, lib=lib)
        m = pr.n - 1
        B = np.zeros((pr.n, pr.n))
        B[np.arange(m), np.arange(m)] = pr.d
        B[:m, m] = pr.z
        B[m, m] = pr.scalar
        if np.max(np.abs(np.linalg.svd(B, compute_uv=False) - r.sigma)) > 1e-13:
            failed.append("svd values")
        if np.max(np.abs(B @ r.V - r.U * r.sigma)) > 1e-13:
            failed.append("svd BV=US")
    except oracle.oracle.OracleError:
        failed.append("svd error")
    return failed


def _quick_extension_pins(lib):
    failed = []
    rng = np.random.default_rng(47)
    a, b = rng.standard_normal(5), rng.standard_normal(4)
    try:
        lam, Q = oracle.tridiag_eig(a, b, lib=lib)
        if _tridiag_failures(a, b, lam, Q):
            failed.append("tridiagonal")
    except (oracle.oracle.OracleError, ValueError, ZeroDivisionError):
        failed.append("tridiagonal error")
    d, z, a = _herm_case(5, 87)
    try:
        if _herm_failures(d, z, a, oracle.herm_eig(d, z, a, lib=lib), dps=30):
            failed.append("hermitian")
    except (oracle.oracle.OracleError, ValueError, ZeroDivisionError):
        failed.append("hermitian error")
    pr = W.dpr1(5, np.random.default_rng(9))
    pr.scalar = -pr.scalar
    try:
        if _dpr1_negative_failures(pr, oracle.dpr1_eig(pr.d, pr.z, pr.scalar, lib=lib)):
            failed.append("dpr1 rho < 0")
    except (oracle.oracle.OracleError, ValueError, ZeroDivisionError):   # NaN or zero where a value belongs
        failed.append("dpr1 rho < 0 error")
    for i in range(len(REDUCIBLE)):
        d, z, a = REDUCIBLE[i]
        try:
            if _deflation_failures(i, oracle.arrow_eig(d, z, a, lib=lib)):
                failed.append(f"deflation {i}")
        except (oracle.oracle.OracleError, ValueError, ZeroDivisionError):
            failed.append(f"deflation {i} error")
    return failed


def _quick_origin_pins(lib):
    """Eigenvalues near the origin, each bracketed by exact inertia."""
    failed = []
    try:
        d, z = np.array([6.0, 3.0, -2.0]), np.ones(3)
        for alpha in (1e-30, -2.5e-300, 3e-3):
            r = oracle.arrow_eig(d, z, alpha, lib=lib)
            k = int(np.argmin(np.abs(r.lam)))
            if not _bracket_count(brute.dense_arrow(d, z, alpha), hilo(r.lam[k], r.lam_lo[k]), k):
                failed.append(f"arrow near zero {alpha}")
        rng = np.random.default_rng(8)
        d = W._sorted_with_gap(rng, 8, -1.0, 1.0)
        u = rng.uniform(0.2, 1.0, 8)
        sm = sum(F(b) ** 2 / F(a) for a, b in zip(d, u))
        if sm > 0:
            d, sm = -d, -sm
        rho = float(-1 / sm)
        r = oracle.dpr1_eig(d, u, rho, lib=lib)
        k = int(np.argmin(np.abs(r.lam)))
        if not _bracket_count(brute.dense_dpr1(d, u, rho), hilo(r.lam[k], r.lam_lo[k]), k):
            failed.append("dpr1 near zero")
        d, z, alpha = np.array([0.5, 0.75, 0.3]), np.array([0.9, 0.4, 0.7]), 1e-30
        r = oracle.arrow_svd(d, z, alpha, lib=lib)
        with mp.workdps(60):
            prod = mp.fprod([mpf2(a, b) for a, b in zip(r.sigma, r.sigma_lo)])
            ref = abs(mp.mpf(alpha) * mp.fprod([mp.mpf(float(x)) for x in d]))
            if not abs(prod - ref) <= ref * mp.mpf("1e-25"):
                failed.append("svd near zero")
    except (oracle.oracle.OracleError, ValueError, ZeroDivisionError):
        failed.append("near zero error")
    return failed


def test_pins_catch_planted_mistakes(oracle_lib):
    assert _quick_pins(None) == [] and _quick_extension_pins(None) == [] and _quick_origin_pins(None) == []
    src = open(os.path.join(os.path.dirname(oracle.oracle.__file__), "oracle.c")).read()
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        for name, (old, new) in _MUTANTS.items():
            assert src.count(old) == 1, name
            path = os.path.join(tmp, f"{name}.c")
            with open(path, "w") as f:
                f.write(src.replace(old, new))
            so = os.path.join(tmp, f"lib_{name}.so")
            subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", so, path, "-lquadmath"], check=True)
            assert _quick_pins(so) + _quick_extension_pins(so) + _quick_origin_pins(so) != [], \
                f"planted mistake '{name}' not caught"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def test_parity_helper_refuses_unresolved_reference(oracle_lib, monkeypatch):
    """tests/parity.py refuses a reference whose zero the oracle could not resolve."""
    import parity
    parity.guard_oracle(monkeypatch)
    with pytest.raises(parity.UntrustedReference):
        oracle.arrow_eig(np.array([3.0, -3.0]), np.array([1.0, 1.0]), 0.0)
    assert oracle.arrow_eig(np.array([3.0, -3.0]), np.array([1.0, 1.0]), 1e-30).lam[1] > 0
