"""Inputs whose eigenvalue nearest 0 lies far closer to 0 than to any pole: the
regime of Sec. 3, Remark 1 and the exceptions (a)-(c) of condition (C1) in
Theorem 2.  Inputs only (exact rationals fix alpha or rho where the cancellation
is planted); no solver arithmetic."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from paper_1302_7203_amd import workloads as W


def _F(x):
    return Fraction(float(x))


def arrow_cases():
    """(name, d, z, alpha).  The 3x3 cases have l ~ alpha / (1 + sum z^2/d^2); the
    quotients z^2/d of (3, -3) and (6, 3, -2) are not dyadic, so f(0) cancels
    beyond any fixed precision of their roundings."""
    out = []
    for a in (1e-12, 1e-20, 1e-30, -3e-200):
        out.append((f"pm1_{a:g}", np.array([1.0, -1.0]), np.array([1.0, 1.0]), a))
    for a in (1e-30, -3e-200):
        out.append((f"pm3_{a:g}", np.array([3.0, -3.0]), np.array([1.0, 1.0]), a))
    for a in (1e-30, -2.5e-300, 3e-3):
        out.append((f"six_{a:g}", np.array([6.0, 3.0, -2.0]), np.ones(3), a))
    out.append(("exterior", np.array([-0.5, -4.0]), np.array([1.0, 2.0]), -3.0 + 2.0 ** -40))
    out.append(("reducible", np.array([2.0, 2.0, -1.0]), np.ones(3), 1e-30))
    # n = 301, poles of both signs, alpha the double nearest to sum z_j^2 / d_j
    rng = np.random.default_rng(5)
    d = W._sorted_with_gap(rng, 300, -1.0, 1.0)[rng.permutation(300)]
    z = rng.uniform(0.1, 1.0, 300)
    out.append(("random_301", d, z, float(sum(_F(b) ** 2 / _F(a) for a, b in zip(d, z)))))
    return out


def dpr1_cases():
    """(name, d, u, rho): D + rho u u^T singular at rho = 4 (an eigenvalue 0), one
    eigenvalue ~1e-16 next to it, their negations, and a random n = 64 case with
    rho the double nearest to -1 / sum u_j^2 / d_j."""
    d, u = np.array([2.0, -1.0, 4.0]), np.ones(3)
    out = []
    for rho in (4.0, 4.0 + 2.0 ** -50, 4.0 - 2.0 ** -48):
        out.append((f"three_{rho!r}", d, u, rho))
        out.append((f"three_neg_{rho!r}", -d, u, -rho))
    rng = np.random.default_rng(8)
    d = W._sorted_with_gap(rng, 64, -1.0, 1.0)
    u = rng.uniform(0.2, 1.0, 64)
    s = sum(_F(b) ** 2 / _F(a) for a, b in zip(d, u))
    if s > 0:
        d, s = -d, -s
    out.append(("random_64", d, u, float(-1 / s)))
    return out


def svd_cases():
    """(name, d, z, alpha): B = [D z; 0 alpha] with tiny alpha, so sigma_n ~ |alpha|."""
    d, z = np.array([0.5, 0.75, 0.3]), np.array([0.9, 0.4, 0.7])
    out = [(f"three_{a:g}", d, z, a) for a in (1e-30, -1e-100, 3e-150)]
    rng = np.random.default_rng(9)
    dd_ = W._sorted_with_gap(rng, 150, 0.0, 1.0)
    out.append(("random_151", dd_, rng.uniform(0.1, 1.0, 150), 1e-40))
    return out


def herm_cases():
    return [("six", np.array([6.0, 3.0, -2.0]), np.array([1j, -1.0, -1j]), 1e-30)]
