"""Thin ctypes binding of ``libarrow.so`` (C ABI in include/arrow.h).

Only argument marshalling happens here: torch supplies device memory and the
current HIP stream; every step of the solve runs in the library's kernels.
There is no fallback: if the library is missing the calls raise.
"""
from __future__ import annotations

import ctypes
import json
import os
import threading
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; ARROW_LIBRARY may name another build of the same sources
LIB_PATH = os.environ.get("ARROW_LIBRARY") or os.path.join(_HERE, "libarrow.so")
# lanes-per-eigenvalue tables measured by the autotuner (paper_1302_7203_amd.autotune)
TUNED_PATH = os.path.join(_HERE, "tuned", "schedule_gfx950.json")

INFO_DD_B = 1
INFO_REMEDY_A = 2
INFO_REMEDY_B = 4
INFO_NEAR_ZERO = 8
INFO_REDUCIBLE = 16
INFO_NONFINITE = 32
INFO_KB_LARGE = 64
INFO_BAD_INPUT = 256
INFO_POLE_SHIFT = 512
INFO_NOT_SOLVED = INFO_REDUCIBLE | INFO_NONFINITE | INFO_BAD_INPUT

OPT_TAU_NU = 1
OPT_TAU_ZERO = 2
OPT_FP64_B = 3
OPT_REMEDIES = 4
OPT_LANES = 5
OPT_TIMING = 6
OPT_ROOT = 7
OPT_TAU_B = 8
OPT_CHECK_LANES = 9
ROOT_BISECT = 0
ROOT_RATIONAL = 1
NOALLOC_N_MAX = 32768   # ARROW_NOALLOC_N_MAX: largest order arrow_eig_noalloc takes
SCHEDULE_SINGLE = 0
SCHEDULE_BATCH = 1
INT32_MAX = 2147483647


class ArrowError(RuntimeError):
    pass


_lib = None
_lock = threading.Lock()
_handles: dict[int, ctypes.c_void_p] = {}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise ArrowError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
                L = ctypes.CDLL(LIB_PATH)
                P, I64, D, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
                L.arrow_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), I]
                L.arrow_destroy.argtypes = [P]
                L.arrow_set_stream.argtypes = [P, P]
                L.arrow_set_option.argtypes = [P, I, D]
                L.arrow_workspace_size.argtypes = [I64]
                L.arrow_workspace_size.restype = ctypes.c_size_t
                L.arrow_eig.argtypes = [P, I64, P, P, D, P, P, I64, P, P, P]
                L.arrow_eig_noalloc.argtypes = [P, I64, P, P, D, P, P, I64, P, P, P]
                L.arrow_eig_herm.argtypes = [P, I64, P, P, D, P, P, I64, P, P, P]
                L.tridiag_eig.argtypes = [P, I64, P, P, P, P, I64, P]
                L.dpr1_eig.argtypes = [P, I64, P, P, D, P, P, I64, P]
                L.arrow_svd.argtypes = [P, I64, P, P, D, P, P, I64, P, I64, P]
                L.arrow_last_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
                L.arrow_timing_of.argtypes = [P, I, ctypes.POINTER(ctypes.c_double)]
                L.arrow_last_counters.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
                L.arrow_conditions.argtypes = [P, P, P]
                L.arrow_set_lanes_table.argtypes = [P, I, ctypes.c_int32, P, P]
                L.arrow_probe_fma.argtypes = [P, I64, I, P]
                L.arrow_probe_fill.argtypes = [P, I64, D, P]
                L.arrow_probe_copy.argtypes = [P, P, I64, P]
                L.arrow_probe_rcp.argtypes = [P, P, I64, P]
                for f in ("arrow_probe_fma", "arrow_probe_fill", "arrow_probe_copy", "arrow_probe_rcp",
                          "arrow_create", "arrow_destroy", "arrow_set_stream", "arrow_set_option",
                          "arrow_eig", "arrow_eig_noalloc", "arrow_eig_herm", "tridiag_eig", "dpr1_eig", "arrow_svd",
                          "arrow_last_timing", "arrow_timing_of", "arrow_last_counters", "arrow_conditions",
                          "arrow_set_lanes_table"):
                    getattr(L, f).restype = ctypes.c_int
                _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise ArrowError(f"{what} returned {rc}")


def read_tuned(path: str = TUNED_PATH) -> dict | None:
    """The autotuner's tables {"single": (n_max, lanes), "batch": (n_max, lanes)}, validated;
    None when the file does not exist."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    out = {}
    for scope, gmin in (("single", 1), ("batch", 4)):
        t = doc[scope]
        n_max, lanes = [int(x) for x in t["n_max"]], [int(x) for x in t["lanes"]]
        if not (1 <= len(n_max) == len(lanes) <= 16):
            raise ArrowError(f"{path}: {scope} table has a bad length")
        if any(b <= a for a, b in zip(n_max, n_max[1:])) or n_max[0] < 1 or n_max[-1] > INT32_MAX:
            raise ArrowError(f"{path}: {scope} n_max must increase strictly within [1, 2^31-1]")
        if any(g < gmin or g > 64 or g & (g - 1) for g in lanes):
            raise ArrowError(f"{path}: {scope} lanes must be powers of two in [{gmin}, 64]")
        out[scope] = (n_max, lanes)
    return out


def set_lanes_table(scope: int, n_max, lanes, h: ctypes.c_void_p | None = None, device=None):
    """Install a lanes-per-eigenvalue table (arrow_set_lanes_table); empty lists restore the default."""
    h = handle(device) if h is None else h
    a = (ctypes.c_int32 * max(1, len(n_max)))(*[int(x) for x in n_max])
    b = (ctypes.c_int32 * max(1, len(lanes)))(*[int(x) for x in lanes])
    _check(lib().arrow_set_lanes_table(h, scope, len(n_max), a, b), "arrow_set_lanes_table")


def apply_tuned(h: ctypes.c_void_p, path: str = TUNED_PATH):
    """Load the autotuned tables, if any, into handle h."""
    t = read_tuned(path)
    if t is not None:
        set_lanes_table(SCHEDULE_SINGLE, *t["single"], h=h)
        set_lanes_table(SCHEDULE_BATCH, *t["batch"], h=h)


def handle(device: int | torch.device | None = None) -> ctypes.c_void_p:
    """The per-device default handle (created on first use, with the autotuned schedule)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx not in _handles:
        h = ctypes.c_void_p()
        _check(lib().arrow_create(ctypes.byref(h), idx), "arrow_create")
        _handles[idx] = h
        apply_tuned(h)
    return _handles[idx]


def set_option(option: int, value: float, device=None):
    _check(lib().arrow_set_option(handle(device), option, float(value)), "arrow_set_option")


def last_timing(device=None) -> list[float]:
    """Stage times (ms) of the last timed call: front, sort, root, check, vectors."""
    ms = (ctypes.c_double * 5)()
    _check(lib().arrow_last_timing(handle(device), ms), "arrow_last_timing")
    return list(ms)


def timing_of(age: int, device=None) -> list[float]:
    """Stage times (ms) of the most recent timed call (age 0) or the one before it (age 1)."""
    ms = (ctypes.c_double * 5)()
    _check(lib().arrow_timing_of(handle(device), int(age), ms), "arrow_timing_of")
    return list(ms)


def last_counters(device=None) -> dict:
    """Pass counters of the last call (see arrow_last_counters)."""
    out = (ctypes.c_int64 * 7)()
    _check(lib().arrow_last_counters(handle(device), out), "arrow_last_counters")
    keys = ("root_bisect", "root_dd", "root_plain", "check_bisect", "check_dd", "check_plain", "n")
    return dict(zip(keys, list(out)))


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def conditions(n: int, device=None):
    """(K_b, K_nu) per output column of the last single-problem call on the default handle
    of `device` (see arrow_conditions), as float64 tensors of length n on that device."""
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = handle(device)
    with torch.cuda.device(device):
        _bind_stream(h, device)
        kb = torch.empty(n, dtype=torch.float64, device=device)
        knu = torch.empty(n, dtype=torch.float64, device=device)
        _check(lib().arrow_conditions(h, _ptr(kb), _ptr(knu)), "arrow_conditions")
    return kb, knu


def _dev_vec(x, n, device, name):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.device.type != "cuda" or x.dtype != torch.float64 or x.dim() != 1 or x.numel() != n:
        raise ValueError(f"{name} must be a 1-D float64 CUDA tensor of length {n}")
    return x.contiguous()


def _bind_stream(h, device):
    s = torch.cuda.current_stream(device)
    _check(lib().arrow_set_stream(h, ctypes.c_void_p(s.cuda_stream)), "arrow_set_stream")


@dataclass
class EigOut:
    lam: torch.Tensor             # eigenvalues (singular values), descending
    V: torch.Tensor | None        # n x n, column k = k-th vector (a transposed view of col-major storage)
    U: torch.Tensor | None = None
    shift: torch.Tensor | None = None
    mu: torch.Tensor | None = None
    info: torch.Tensor | None = None


def _colmajor(n, device):
    buf = torch.empty((n, n), dtype=torch.float64, device=device)   # buf[k, r] = V[r, k]
    return buf


def arrow_eig(d: torch.Tensor, z: torch.Tensor, alpha: float, *, vectors: bool = True,
              pairs: bool = False, noalloc: bool = False) -> EigOut:
    """Eigenpairs of A = [diag(d) z; z^T alpha]; d, z float64 CUDA tensors of length n-1.
    noalloc: call arrow_eig_noalloc (the library allocates nothing; n <= NOALLOC_N_MAX)."""
    device = d.device
    n = d.numel() + 1
    d = _dev_vec(d, n - 1, device, "d")
    z = _dev_vec(z, n - 1, device, "z")
    h = handle(device)
    with torch.cuda.device(device):
        _bind_stream(h, device)
        lam = torch.empty(n, dtype=torch.float64, device=device)
        buf = _colmajor(n, device) if vectors else None
        shift = torch.empty(n, dtype=torch.float64, device=device) if pairs else None
        mu = torch.empty(n, dtype=torch.float64, device=device) if pairs else None
        info = torch.empty(n, dtype=torch.int32, device=device)
        f = lib().arrow_eig_noalloc if noalloc else lib().arrow_eig
        rc = f(h, n, _ptr(d), _ptr(z), float(alpha), _ptr(lam), _ptr(buf), n, _ptr(shift), _ptr(mu), _ptr(info))
    _check(rc, "arrow_eig_noalloc" if noalloc else "arrow_eig")
    return EigOut(lam, None if buf is None else buf.t(), None, shift, mu, info)


def arrow_eig_herm(d: torch.Tensor, z: torch.Tensor, alpha: float, *, vectors: bool = True,
                   pairs: bool = False) -> EigOut:
    """Eigenpairs of the Hermitian arrowhead [diag(d) z; z^* alpha]; d float64 and z complex128
    CUDA tensors of length n-1.  V is complex128."""
    device = d.device
    n = d.numel() + 1
    d = _dev_vec(d, n - 1, device, "d")
    if not isinstance(z, torch.Tensor) or z.device.type != "cuda" or z.dtype != torch.complex128 \
            or z.dim() != 1 or z.numel() != n - 1:
        raise ValueError(f"z must be a 1-D complex128 CUDA tensor of length {n - 1}")
    z = z.contiguous()
    h = handle(device)
    with torch.cuda.device(device):
        _bind_stream(h, device)
        lam = torch.empty(n, dtype=torch.float64, device=device)
        buf = torch.empty((n, n), dtype=torch.complex128, device=device) if vectors else None
        shift = torch.empty(n, dtype=torch.float64, device=device) if pairs else None
        mu = torch.empty(n, dtype=torch.float64, device=device) if pairs else None
        info = torch.empty(n, dtype=torch.int32, device=device)
        rc = lib().arrow_eig_herm(h, n, _ptr(d), _ptr(z), float(alpha), _ptr(lam), _ptr(buf), n,
                                  _ptr(shift), _ptr(mu), _ptr(info))
    _check(rc, "arrow_eig_herm")
    return EigOut(lam, None if buf is None else buf.t(), None, shift, mu, info)


def tridiag_eig(a: torch.Tensor, b: torch.Tensor) -> EigOut:
    """Eigenpairs of the symmetric tridiagonal matrix with diagonal a (n) and off-diagonal b (n-1),
    float64 CUDA tensors, by divide and conquer with DPR1 merges.  Synchronous."""
    device = a.device
    n = a.numel()
    a = _dev_vec(a, n, device, "a")
    b = _dev_vec(b, n - 1, device, "b") if n > 1 else torch.zeros(1, dtype=torch.float64, device=device)
    h = handle(device)
    with torch.cuda.device(device):
        _bind_stream(h, device)
        lam = torch.empty(n, dtype=torch.float64, device=device)
        buf = _colmajor(n, device)
        info = torch.empty(n, dtype=torch.int32, device=device)
        rc = lib().tridiag_eig(h, n, _ptr(a), _ptr(b), _ptr(lam), _ptr(buf), n, _ptr(info))
    _check(rc, "tridiag_eig")
    return EigOut(lam, buf.t(), None, None, None, info)


def dpr1_eig(d: torch.Tensor, u: torch.Tensor, rho: float, *, vectors: bool = True) -> EigOut:
    """Eigenpairs of diag(d) + rho u u^T (rho != 0); d, u float64 CUDA tensors of length n."""
    device = d.device
    n = d.numel()
    d = _dev_vec(d, n, device, "d")
    u = _dev_vec(u, n, device, "u")
    h = handle(device)
    with torch.cuda.device(device):
        _bind_stream(h, device)
        lam = torch.empty(n, dtype=torch.float64, device=device)
        buf = _colmajor(n, device) if vectors else None
        info = torch.empty(n, dtype=torch.int32, device=device)
        rc = lib().dpr1_eig(h, n, _ptr(d), _ptr(u), float(rho), _ptr(lam), _ptr(buf), n, _ptr(info))
    _check(rc, "dpr1_eig")
    return EigOut(lam, None if buf is None else buf.t(), None, None, None, info)


def arrow_svd(d: torch.Tensor, z: torch.Tensor, alpha: float, *, vectors: bool = True) -> EigOut:
    """SVD of B = [diag(d) z; 0 alpha]; returns sigma in ``lam``, U and V."""
    device = d.device
    n = d.numel() + 1
    d = _dev_vec(d, n - 1, device, "d")
    z = _dev_vec(z, n - 1, device, "z")
    h = handle(device)
    with torch.cuda.device(device):
        _bind_stream(h, device)
        sig = torch.empty(n, dtype=torch.float64, device=device)
        vb = _colmajor(n, device) if vectors else None
        ub = _colmajor(n, device) if vectors else None
        info = torch.empty(n, dtype=torch.int32, device=device)
        rc = lib().arrow_svd(h, n, _ptr(d), _ptr(z), float(alpha), _ptr(sig), _ptr(ub), n, _ptr(vb), n,
                             _ptr(info))
    _check(rc, "arrow_svd")
    return EigOut(sig, None if vb is None else vb.t(), None if ub is None else ub.t(), None, None, info)
