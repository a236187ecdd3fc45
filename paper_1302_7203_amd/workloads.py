"""Seeded synthetic inputs for the arrowhead, DPR1 and triangular-arrowhead SVD problems.

This module only draws random numbers and arranges them; it contains none of
the solver's arithmetic, so both the GPU path and the CPU oracle may use it.
Every generator uses numpy's PCG64 ``default_rng`` with a fixed seed.  A "min
gap" condition is met by sampling the conditional law directly (see
``_sorted_with_gap``); the graded poles are redrawn until they are distinct.

The paper publishes no dataset (its quantum-dot matrix of Example 4 is given
only by ranges), so these laws stand in for its workloads:

  uniform   d ~ U(lo, hi) sorted descending with min gap >= 1e-6,
            z ~ U(0.1, 1), alpha ~ U(-1, 1)
  graded    |d| log-uniform in [1e-10, 1e10] with random signs, plus tight
            clusters of 8 poles with relative gaps ~1e-12; z log-uniform in
            [1e-8, 1]; alpha = 1e-3  (forces the double-double element b)
  dpr1      d as ``uniform``, u = g/||g|| with g ~ N(0, I), rho ~ U(0.1, 10)
  svd       d ~ U(0, 1) sorted with min gap >= 1e-6, z ~ U(0.1, 1), alpha ~ U(0, 1)
  reducible ``uniform`` with some z_j = 0, repeated poles and signed z, shuffled
  herm      ``uniform`` poles shuffled, z = r e^{i theta}, r ~ U(0.1, 1), theta ~ U(0, 2 pi)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KIND_ARROW = 0
KIND_DPR1 = 1
KIND_SVD = 2
KIND_HERM = 3

SEED_BASE = 72030


@dataclass
class Problem:
    kind: int                 # KIND_ARROW / KIND_DPR1 / KIND_SVD
    n: int                    # matrix order
    d: np.ndarray             # arrow/svd: n-1 poles; dpr1: n diagonal entries
    z: np.ndarray             # arrow/svd: n-1 shaft entries; dpr1: u (n entries); herm: complex
    scalar: float             # arrow/svd: alpha; dpr1: rho
    meta: dict = field(default_factory=dict)


def _sorted_with_gap(rng, m, lo, hi, min_gap=1e-6):
    """m points uniform on (lo, hi) conditioned on every gap between neighbours being
    >= min_gap, in descending order.  Drawn exactly rather than by redrawing (which
    never ends for thousands of points): sort m uniforms on (lo, hi - (m-1)*min_gap)
    and move the k-th smallest up by k*min_gap.  That map is a bijection with unit
    Jacobian onto the constrained set, so the law equals the rejection sampler's."""
    if m < 1:
        return np.zeros(0)
    span = (hi - lo) - (m - 1) * min_gap
    if span <= 0:
        raise ValueError(f"{m} points with gaps >= {min_gap} do not fit in ({lo}, {hi})")
    u = np.sort(rng.uniform(lo, lo + span, m))
    return (u + min_gap * np.arange(m))[::-1].copy()


def uniform_arrow(n, rng, lo=-1.0, hi=1.0):
    m = n - 1
    d = _sorted_with_gap(rng, m, lo, hi)
    z = rng.uniform(0.1, 1.0, m)
    alpha = float(rng.uniform(-1.0, 1.0))
    return Problem(KIND_ARROW, n, d, z, alpha)


def graded_arrow(n, rng, clusters=64, cluster_size=8, alpha=1e-3):
    m = n - 1
    singles = m - clusters * cluster_size
    if singles < 0:
        clusters, singles = m // cluster_size, m % cluster_size
    while True:
        mags = 10.0 ** rng.uniform(-10.0, 10.0, singles)
        signs = np.where(rng.uniform(size=singles) < 0.5, -1.0, 1.0)
        vals = [signs * mags]
        for _ in range(clusters):
            c = (1.0 if rng.uniform() < 0.5 else -1.0) * 10.0 ** rng.uniform(-10.0, 10.0)
            gaps = 10.0 ** rng.uniform(-12.3, -11.7, cluster_size - 1)
            mem = c * np.concatenate([[1.0], np.cumprod(1.0 + gaps)])
            vals.append(mem)
        d = np.sort(np.concatenate(vals))[::-1].copy()
        if np.all(d[:-1] > d[1:]) and np.all(d != 0):
            break
    z = 10.0 ** rng.uniform(-8.0, 0.0, m)
    return Problem(KIND_ARROW, n, d, z, float(alpha))


def dpr1(n, rng):
    d = _sorted_with_gap(rng, n, -1.0, 1.0)
    g = rng.standard_normal(n)
    u = g / np.linalg.norm(g)
    rho = float(rng.uniform(0.1, 10.0))
    return Problem(KIND_DPR1, n, d, u, rho)


def svd_arrow(n, rng):
    m = n - 1
    d = _sorted_with_gap(rng, m, 0.0, 1.0)
    d = np.where(d == 0.0, np.nextafter(0.0, 1.0), d)
    z = rng.uniform(0.1, 1.0, m)
    alpha = float(rng.uniform(0.0, 1.0))
    return Problem(KIND_SVD, n, d, z, alpha)


# ---------------------------------------------------------------------------
# The five workloads (sizes as named in the benchmark configurations).

def single_uniform_512():
    """One arrowhead, n=512, poles U(-1,1)."""
    return uniform_arrow(512, np.random.default_rng(SEED_BASE + 0))


def single_graded_4096():
    """One graded arrowhead, n=4096, with 64 clusters of 8 poles."""
    return graded_arrow(4096, np.random.default_rng(SEED_BASE + 1))


def single_uniform_16384():
    """One arrowhead, n=16384, poles U(-1e4, 1e4)."""
    return uniform_arrow(16384, np.random.default_rng(SEED_BASE + 2), -1e4, 1e4)


def batch_mixed(count=10000, nmin=16, nmax=1024):
    """Independent problems, n log-uniform in [nmin, nmax]; even: arrowhead, odd: DPR1."""
    ss = np.random.SeedSequence(SEED_BASE + 3).spawn(count)
    out = []
    for p, s in enumerate(ss):
        rng = np.random.default_rng(s)
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        out.append(uniform_arrow(n, rng) if p % 2 == 0 else dpr1(n, rng))
    return out


def serving_requests(count=2200, nmin=32, nmax=8192, rate=1.0, seed=SEED_BASE + 4):
    """Poisson request stream: (arrival time in units of 1/rate, Problem).

    Type by U: < 0.60 arrowhead eigen, < 0.85 DPR1 eigen, else triangular
    arrowhead SVD; n log-uniform in [nmin, nmax]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        u = rng.uniform()
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        if u < 0.60:
            pr = uniform_arrow(n, rng)
        elif u < 0.85:
            pr = dpr1(n, rng)
        else:
            pr = svd_arrow(n, rng)
        out.append((t, pr))
    return out


def wide_arrow(kind, n, rng, decades=300):
    """Poles whose magnitudes spread log-uniformly over `decades` decades below 1
    (signed for ARROW and DPR1, non-negative for SVD, whose poles are the squares
    of d), shaft entries of order 1: eigenvalues lie far closer to their poles
    than the square root of the smallest normal number."""
    m = n if kind == KIND_DPR1 else n - 1
    span = decades if kind != KIND_SVD else decades / 2
    mag = 10.0 ** rng.uniform(-span, 0.0, m)
    d = mag if kind == KIND_SVD else mag * np.where(rng.random(m) < 0.5, 1.0, -1.0)
    d = np.sort(d)[::-1].copy()
    z = rng.uniform(0.5, 1.5, m)
    scalar = 0.7 if kind == KIND_DPR1 else 0.3
    return Problem(kind, n, d, z, scalar)


def herm_arrow(n, rng):
    """Hermitian arrowhead (Sec. 6.1): ``uniform`` poles in random order, z = r e^{i theta}
    with r ~ U(0.1, 1), theta ~ U(0, 2 pi)."""
    m = n - 1
    d = _sorted_with_gap(rng, m, -1.0, 1.0)[rng.permutation(m)]
    z = rng.uniform(0.1, 1.0, m) * np.exp(2j * np.pi * rng.uniform(0.0, 1.0, m))
    return Problem(KIND_HERM, n, d.copy(), z, float(rng.uniform(-1.0, 1.0)))


def reducible_arrow(n, rng, zero_frac=0.1, repeat_every=97, triple=True):
    """A reducible arrowhead (Sec. 1) in random order: ``uniform`` poles and
    shaft, then a fraction ``zero_frac`` of the shaft entries set to 0 (random
    signs on the rest), every ``repeat_every``-th pole repeated in the next
    slot (0: none), and, if ``triple``, one pole taken three times."""
    m = n - 1
    d = _sorted_with_gap(rng, m, -1.0, 1.0)
    z = rng.uniform(0.1, 1.0, m) * rng.choice([-1.0, 1.0], m)
    if m > 0:
        z[rng.choice(m, int(zero_frac * m), replace=False)] = 0.0
    if repeat_every > 0:
        for i in range(0, m - 1, repeat_every):
            d[i + 1] = d[i]
    if triple and m >= 8:
        c = m // 2
        d[c + 1] = d[c + 2] = d[c]
    perm = rng.permutation(m)
    alpha = float(rng.uniform(-1.0, 1.0))
    return Problem(KIND_ARROW, n, d[perm].copy(), z[perm].copy(), alpha)


def shuffled(pr: Problem, seed: int) -> Problem:
    """Same problem with its poles presented in a random order."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(pr.d.size)
    return Problem(pr.kind, pr.n, pr.d[perm].copy(), pr.z[perm].copy(), pr.scalar, {"perm": perm})
