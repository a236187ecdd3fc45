"""ctypes front end of the binary128 oracle in ``oracle.c`` (test infrastructure only).

Each function returns numpy arrays of the exact eigen/singular decomposition
rounded once to FP64 (see the header of ``oracle.c`` for the definitions it
follows: Sec. 1 eqs. (Pick), (Aeigenvec), (interlace); Sec. 6.2; Sec. 6.3 and
Remark 1 for the DPR1 secular equation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_libs = {}


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lquadmath"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load(path=None):
    """Load the built oracle (or, for the planted-mistake tests, another build of it)."""
    key = path or _LIB
    if key not in _libs:
        if path is None and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(key)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_arrow_eig.argtypes = [I64, P, P, D, I64, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_dpr1_eig.argtypes = [I64, P, P, D, I64, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_arrow_svd.argtypes = [I64, P, P, D, I64, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_herm_eig.argtypes = [I64, P, P, P, D, I64, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_tridiag_eig.argtypes = [I64, P, P, I64, P, P, P, ctypes.c_int]
        for f in (lib.oracle_arrow_eig, lib.oracle_dpr1_eig, lib.oracle_arrow_svd, lib.oracle_herm_eig,
                  lib.oracle_tridiag_eig):
            f.restype = ctypes.c_int
        _libs[key] = lib
    return _libs[key]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


@dataclass
class EigResult:
    lam: np.ndarray        # eigenvalues (nearest double), descending order of ks
    lam_lo: np.ndarray     # binary128 remainder: lam + lam_lo ~ exact to ~2^-100
    tau: np.ndarray        # eigenvalue minus reference pole
    tau_lo: np.ndarray
    pole: np.ndarray       # caller index of the reference pole
    vec: np.ndarray | None  # n x nk eigenvectors (caller row order)
    relerr: np.ndarray     # relative uncertainty of the located zero
    ks: np.ndarray


def _ks(n, ks):
    if ks is None:
        return np.arange(n, dtype=np.int64)
    return np.ascontiguousarray(np.asarray(ks, dtype=np.int64))


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what}: oracle returned {rc}")


def arrow_eig(d, z, alpha, ks=None, vectors=True, threads=0, lib=None) -> EigResult:
    """Eigenpairs of A = [diag(d) z; z^T alpha] (d, z of length n-1, any order)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = d.size + 1
    k = _ks(n, ks)
    nk = k.size
    out = [np.empty(nk) for _ in range(4)]
    pole = np.empty(nk, dtype=np.int64)
    rel = np.empty(nk)
    V = np.empty((nk, n)) if vectors else None  # row i = column i of the n x nk result
    rc = _load(lib).oracle_arrow_eig(n, _ptr(d), _ptr(z), float(alpha), nk, _ptr(k),
                                  _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(out[3]),
                                  _ptr(pole), _ptr(V), _ptr(rel), int(threads))
    _check(rc, "oracle_arrow_eig")
    return EigResult(out[0], out[1], out[2], out[3], pole, None if V is None else V.T, rel, k)


def herm_eig(d, z, alpha, ks=None, vectors=True, threads=0, lib=None) -> EigResult:
    """Eigenpairs of the Hermitian arrowhead [diag(d) z; z^* alpha] (d real, z complex, n-1 each);
    ``vec`` is complex."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.complex128)
    zr = np.ascontiguousarray(z.real)
    zi = np.ascontiguousarray(z.imag)
    n = d.size + 1
    k = _ks(n, ks)
    nk = k.size
    out = [np.empty(nk) for _ in range(4)]
    pole = np.empty(nk, dtype=np.int64)
    rel = np.empty(nk)
    U = np.empty((nk, n), dtype=np.complex128) if vectors else None
    rc = _load(lib).oracle_herm_eig(n, _ptr(d), _ptr(zr), _ptr(zi), float(alpha), nk, _ptr(k),
                                 _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(out[3]),
                                 _ptr(pole), _ptr(U), _ptr(rel), int(threads))
    _check(rc, "oracle_herm_eig")
    return EigResult(out[0], out[1], out[2], out[3], pole, None if U is None else U.T, rel, k)


def dpr1_eig(d, u, rho, ks=None, vectors=True, threads=0, lib=None) -> EigResult:
    """Eigenpairs of M = diag(d) + rho u u^T, rho > 0 (d, u of length n, any order)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = d.size
    k = _ks(n, ks)
    nk = k.size
    out = [np.empty(nk) for _ in range(4)]
    pole = np.empty(nk, dtype=np.int64)
    rel = np.empty(nk)
    Q = np.empty((nk, n)) if vectors else None
    rc = _load(lib).oracle_dpr1_eig(n, _ptr(d), _ptr(u), float(rho), nk, _ptr(k),
                                 _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(out[3]),
                                 _ptr(pole), _ptr(Q), _ptr(rel), int(threads))
    _check(rc, "oracle_dpr1_eig")
    return EigResult(out[0], out[1], out[2], out[3], pole, None if Q is None else Q.T, rel, k)


@dataclass
class SvdResult:
    sigma: np.ndarray
    sigma_lo: np.ndarray
    U: np.ndarray | None
    V: np.ndarray | None
    relerr: np.ndarray
    ks: np.ndarray


def arrow_svd(d, z, alpha, ks=None, vectors=True, threads=0, lib=None) -> SvdResult:
    """SVD of B = [diag(d) z; 0 alpha] (d, z of length n-1, any order)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = d.size + 1
    k = _ks(n, ks)
    nk = k.size
    s = np.empty(nk)
    slo = np.empty(nk)
    rel = np.empty(nk)
    U = np.empty((nk, n)) if vectors else None
    V = np.empty((nk, n)) if vectors else None
    rc = _load(lib).oracle_arrow_svd(n, _ptr(d), _ptr(z), float(alpha), nk, _ptr(k),
                                  _ptr(s), _ptr(slo), _ptr(U), _ptr(V), _ptr(rel), int(threads))
    _check(rc, "oracle_arrow_svd")
    return SvdResult(s, slo, None if U is None else U.T, None if V is None else V.T, rel, k)


def tridiag_eig(a, b, ks=None, vectors=True, threads=0, lib=None):
    """Eigenpairs of the symmetric tridiagonal matrix with diagonal a (n) and off-diagonal b (n-1):
    (lam, Q) with lam descending over ks and Q[:, i] the i-th vector, largest-magnitude entry > 0."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = a.size
    k = _ks(n, ks)
    lam = np.empty(k.size)
    Q = np.empty((k.size, n)) if vectors else None
    rc = _load(lib).oracle_tridiag_eig(n, _ptr(a), _ptr(b), k.size, _ptr(k), _ptr(lam), _ptr(Q), int(threads))
    _check(rc, "oracle_tridiag_eig")
    return lam, (None if Q is None else Q.T)
