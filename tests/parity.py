"""Element-by-element comparison against the oracle at the 1e-13 relative bar."""
from __future__ import annotations

import numpy as np

TOL = 1e-13   # relative, componentwise, for every eigenvalue and every vector entry


def relerr(got, ref):
    """|got - ref| / |ref| entrywise (complex entries by modulus)."""
    dt = np.complex128 if (np.iscomplexobj(got) or np.iscomplexobj(ref)) else np.float64
    got = np.asarray(got, dtype=dt)
    ref = np.asarray(ref, dtype=dt)
    den = np.abs(ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.abs(got - ref) / den
    e = np.where((den == 0) & (got == ref), 0.0, e)
    return e


def assert_close(got, ref, what, tol=TOL):
    e = relerr(got, ref)
    assert np.all(np.isfinite(e)), f"{what}: non-finite entries"
    worst = float(e.max()) if e.size else 0.0
    if worst > tol:
        idx = np.unravel_index(int(np.argmax(e)), e.shape)
        raise AssertionError(f"{what}: max relative error {worst:.3e} > {tol:.0e} at {idx}: "
                             f"got {np.asarray(got)[idx]!r} ref {np.asarray(ref)[idx]!r}")
    return worst
