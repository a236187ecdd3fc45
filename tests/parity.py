"""Element-by-element comparison against the oracle at the 1e-13 relative bar."""
from __future__ import annotations

import numpy as np

TOL = 1e-13   # relative, componentwise, for every eigenvalue and every vector entry
REF_RELERR = 1e-20   # the oracle's own uncertainty must sit far below TOL to be a reference


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


class UntrustedReference(AssertionError):
    pass


def trusted(res):
    """The oracle's result, refused when any of its located zeros carries a
    reported relative uncertainty above REF_RELERR."""
    rel = np.asarray(getattr(res, "relerr", []), dtype=np.float64)
    if rel.size and not np.all(rel <= REF_RELERR):
        i = int(np.argmax(np.where(np.isfinite(rel), rel, np.inf)))
        raise UntrustedReference(f"oracle reference not resolved: relerr {rel[i]:.3e} > {REF_RELERR:.0e} "
                                 f"at output {i}")
    return res


GUARDED = ("arrow_eig", "dpr1_eig", "arrow_svd", "herm_eig")


def guard_oracle(monkeypatch):
    """Route every oracle reference used by a comparison test through trusted()."""
    import oracle

    for name in GUARDED:
        f = getattr(oracle, name)

        def wrapped(*a, _f=f, **k):
            return trusted(_f(*a, **k))

        monkeypatch.setattr(oracle, name, wrapped)
