"""Brute-force references that know nothing about arrowhead structure.

* ``exact_eigvals``: eigenvalues of a dense symmetric matrix of exact rationals,
  located by bisection on Sylvester's law of inertia (the number of negative
  pivots of an exact LDL^T of A - xI is the number of eigenvalues below x).
* ``exact_null_vector``: a null vector of A - lam*I by exact Gaussian
  elimination of its first n-1 rows, with the last coordinate fixed to -1.
* ``mp_eigsy`` / ``mp_svd``: mpmath's dense Jacobi eigensolver / SVD at a
  chosen number of digits (the paper's own check used 100-digit Mathematica).

Binary FP64 inputs are exact dyadic rationals (Sec. 4.1, binary convention),
so ``Fraction(x)`` is the exact input.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath as mp
import numpy as np


def dense_arrow(d, z, alpha):
    m = len(d)
    n = m + 1
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(m):
        A[i][i] = Fraction(float(d[i]))
        A[i][m] = A[m][i] = Fraction(float(z[i]))
    A[m][m] = Fraction(float(alpha))
    return A


def dense_dpr1(d, u, rho):
    n = len(d)
    r = Fraction(float(rho))
    uu = [Fraction(float(x)) for x in u]
    return [[(Fraction(float(d[i])) if i == j else Fraction(0)) + r * uu[i] * uu[j]
             for j in range(n)] for i in range(n)]


def _count_below(A, x):
    n = len(A)
    M = [[A[i][j] - (x if i == j else 0) for j in range(n)] for i in range(n)]
    neg = 0
    for k in range(n):
        piv = M[k][k]
        if piv == 0:
            return None
        if piv < 0:
            neg += 1
        rowk = M[k]
        for i in range(k + 1, n):
            f = M[i][k] / piv
            if f:
                Mi = M[i]
                for j in range(k + 1, n):
                    Mi[j] -= f * rowk[j]
    return neg


def exact_eigvals(A, rel_bits=110, abs_floor=Fraction(1, 2 ** 400)):
    """All eigenvalues (descending) as Fractions, each within 2^-rel_bits relative."""
    n = len(A)
    radius = [sum(abs(A[i][j]) for j in range(n) if j != i) for i in range(n)]
    lo0 = min(A[i][i] - radius[i] for i in range(n)) - 1
    hi0 = max(A[i][i] + radius[i] for i in range(n)) + 1
    out = []
    for k in range(n):
        target = n - 1 - k           # eigenvalues strictly below lambda_k
        lo, hi = lo0, hi0
        while True:
            w = hi - lo
            scale = max(abs(lo), abs(hi))
            if w <= scale / 2 ** rel_bits or w <= abs_floor:
                break
            mid = (lo + hi) / 2
            c = _count_below(A, mid)
            bump = Fraction(1, 2 ** 600)
            while c is None:
                mid += bump
                bump *= 2
                c = _count_below(A, mid)
            if c <= target:
                lo = mid
            else:
                hi = mid
        out.append((lo + hi) / 2)
    return out


def exact_null_vector(A, lam):
    """x with x[-1] = -1 solving the first n-1 rows of (A - lam I) x = 0 exactly."""
    n = len(A)
    m = n - 1
    M = [[A[i][j] - (lam if i == j else 0) for j in range(m)] for i in range(m)]
    rhs = [A[i][m] for i in range(m)]          # (A - lam I)[i, m] * (-1) moved over: +A[i][m]
    for k in range(m):
        p = max(range(k, m), key=lambda r: abs(M[r][k]))
        M[k], M[p] = M[p], M[k]
        rhs[k], rhs[p] = rhs[p], rhs[k]
        piv = M[k][k]
        for i in range(k + 1, m):
            f = M[i][k] / piv
            if f:
                for j in range(k, m):
                    M[i][j] -= f * M[k][j]
                rhs[i] -= f * rhs[k]
    x = [Fraction(0)] * m
    for i in reversed(range(m)):
        s = rhs[i] - sum(M[i][j] * x[j] for j in range(i + 1, m))
        x[i] = s / M[i][i]
    return x + [Fraction(-1)]


def mp_eigsy(A_np, dps=50):
    """Dense symmetric eigen-decomposition in mpmath; eigenvalues descending."""
    with mp.workdps(dps):
        n = A_np.shape[0]
        A = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                A[i, j] = mp.mpf(float(A_np[i, j]))
        E, Q = mp.eigsy(A)
        order = sorted(range(n), key=lambda i: -E[i])
        lam = [E[i] for i in order]
        vec = [[Q[r, i] for r in range(n)] for i in order]
    return lam, vec


def mp_svd(B_np, dps=50):
    with mp.workdps(dps):
        n = B_np.shape[0]
        B = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                B[i, j] = mp.mpf(float(B_np[i, j]))
        U, S, V = mp.svd_r(B)
        order = sorted(range(n), key=lambda i: -S[i])
        s = [S[i] for i in order]
        u = [[U[r, i] for r in range(n)] for i in order]
        v = [[V[i, r] for r in range(n)] for i in order]   # V is returned transposed
    return s, u, v


def arrow_np(d, z, alpha):
    m = len(d)
    A = np.zeros((m + 1, m + 1))
    A[np.arange(m), np.arange(m)] = d
    A[:m, m] = z
    A[m, :m] = z
    A[m, m] = alpha
    return A
