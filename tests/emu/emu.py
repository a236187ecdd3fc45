"""Build and call the host-only driver of the library's kernel bodies (tests only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host_emu.hip")
LIB = os.path.join(HERE, "libarrow_emu.so")
CSRC = os.path.join(os.path.dirname(os.path.dirname(HERE)), "paper_1302_7203_amd", "csrc")
_lib = None


def build():
    deps = [SRC] + [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    if os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(p) for p in deps):
        return LIB
    tmp = f"{LIB}.{os.getpid()}.tmp"   # concurrent test workers may build at once
    subprocess.run(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-fPIC",
                    "-shared", "-ffp-contract=off", "-fopenmp", "-o", tmp, SRC], check=True,
                   capture_output=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        L.emu_solve.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, ctypes.c_double, P, P, P, P, P, P,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P,
                                ctypes.c_double, P]
        L.emu_solve.restype = ctypes.c_int
        L.emu_set_batch_check.argtypes = [ctypes.c_int]
        L.emu_set_batch_check.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def set_batch_check(on: bool):
    """Run the check stage as the batched plan does: Remark 2 and the DPR1 re-measure inline,
    eigenvalues near the origin listed and repaired afterwards."""
    _load().emu_set_batch_check(1 if on else 0)


def solve(kind, d, z, scalar, vectors=True, tau_nu=100.0, tau_zero=10.0, fp64_b=0, remedies=1, root=1, tau_b=0.0):
    """kind 0 arrowhead, 1 DPR1, 2 SVD, 3 Hermitian arrowhead (complex z; complex V).
    Returns dict of numpy arrays (V[:, k] = k-th vector)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.complex128 if kind == 3 else np.float64)
    n = d.size + (0 if kind == 1 else 1)
    lam = np.empty(n)
    Vb = np.empty((n, n), dtype=np.complex128 if kind == 3 else np.float64) if vectors else None
    Ub = np.empty((n, n)) if (vectors and kind == 2) else None
    sh, mu, kb, knu = np.empty(n), np.empty(n), np.empty(n), np.empty(n)
    info = np.empty(n, dtype=np.uint32)
    cnt = np.empty((n, 6), dtype=np.int32)
    _load().emu_solve(kind, n, _p(d), _p(z), float(scalar), _p(lam), _p(Vb), _p(Ub), _p(sh), _p(mu), _p(info),
                      tau_nu, tau_zero, fp64_b, remedies, _p(kb), root, _p(cnt), tau_b, _p(knu))
    return {"lam": lam, "V": None if Vb is None else Vb.T, "U": None if Ub is None else Ub.T,
            "shift": sh, "mu": mu, "info": info, "kb": kb, "knu": knu, "cnt": cnt}
