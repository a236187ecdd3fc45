"""Batched solves through the C ABI (arrow_batch_* in include/arrow.h).

The problems of a batch are packed into three device pools (inputs, float
outputs, info words) described by ``arrow_desc_t`` records; torch provides the
memory and the stream, the library does all the work.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import binding
from .workloads import KIND_ARROW, KIND_DPR1, KIND_HERM, KIND_SVD, Problem

BATCH_GRAPH = 1
BATCH_TIMING = 2


class ArrowDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("d_off", ctypes.c_int64),
                ("z_off", ctypes.c_int64), ("scalar", ctypes.c_double), ("lam_off", ctypes.c_int64),
                ("vec_off", ctypes.c_int64), ("left_off", ctypes.c_int64), ("info_off", ctypes.c_int64)]


assert ctypes.sizeof(ArrowDesc) == 64


def _setup(L):
    if getattr(L, "_batch_ready", False):
        return L
    P, I64, I, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    L.arrow_batch_workspace_size.argtypes = [I64, P]
    L.arrow_batch_workspace_size.restype = SZ
    L.arrow_batch_create.argtypes = [P, I64, P, P, P, P, P, SZ, I, ctypes.POINTER(ctypes.c_void_p)]
    L.arrow_batch_run.argtypes = [P]
    L.arrow_batch_destroy.argtypes = [P]
    L.arrow_solve_batched.argtypes = [P, I64, P, P, P, P]
    L.arrow_solve_sequential.argtypes = [P, I64, P, P, P, P]
    L.arrow_batch_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    L.arrow_batch_counters.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    for f in ("arrow_batch_create", "arrow_batch_run", "arrow_batch_destroy", "arrow_solve_batched",
              "arrow_solve_sequential", "arrow_batch_timing", "arrow_batch_counters"):
        getattr(L, f).restype = I
    L._batch_ready = True
    return L


def lib():
    return _setup(binding.lib())


def set_lanes_table(n_max, lanes, device=None):
    """Batched schedule of the default handle: lanes per eigenvalue for n <= n_max[e]."""
    binding.set_lanes_table(binding.SCHEDULE_BATCH, n_max, lanes, device=device)


def sorted_len(kind, n):
    return n if kind == KIND_DPR1 else n - 1


@dataclass
class Packed:
    """Problems packed into pools: descriptors plus the host-side input pool."""
    descs: ctypes.Array
    in_host: np.ndarray
    out_size: int
    info_size: int
    kinds: list
    ns: list


def pack(problems: list[Problem], vectors: bool = True, left: bool = True, info: bool = True) -> Packed:
    count = len(problems)
    descs = (ArrowDesc * count)()
    ins, ioff, ooff, foff = [], 0, 0, 0
    for p, pr in enumerate(problems):
        ms = sorted_len(pr.kind, pr.n)
        D = descs[p]
        D.kind, D.n, D.scalar = pr.kind, pr.n, float(pr.scalar)
        D.d_off, D.z_off = ioff, ioff + ms
        if pr.kind == KIND_HERM:   # z as (re, im) pairs
            ins += [np.asarray(pr.d, dtype=np.float64), np.asarray(pr.z, dtype=np.complex128).view(np.float64)]
            ioff += 3 * ms
        else:
            ins += [np.asarray(pr.d, dtype=np.float64), np.asarray(pr.z, dtype=np.float64)]
            ioff += 2 * ms
        D.lam_off = ooff
        ooff += pr.n
        D.vec_off, D.left_off = -1, -1
        if vectors and pr.kind == KIND_HERM:
            ooff += ooff & 1               # complex entries start on 16 bytes
            D.vec_off = ooff
            ooff += 2 * pr.n * pr.n
        elif vectors:
            D.vec_off = ooff
            ooff += pr.n * pr.n
            if pr.kind == KIND_SVD and left:
                D.left_off = ooff
                ooff += pr.n * pr.n
        D.info_off = foff if info else -1
        foff += pr.n if info else 0
    in_host = np.concatenate(ins) if ins else np.zeros(0)
    if in_host.size == 0:
        in_host = np.zeros(1)
    return Packed(descs, in_host, max(ooff, 1), max(foff, 1), [p.kind for p in problems], [p.n for p in problems])


class Batch:
    """Device pools and a plan for a list of problems."""

    def __init__(self, problems: list[Problem], device=None, vectors=True, graph=False, packed: Packed | None = None,
                 in_pool: torch.Tensor | None = None, out_pool: torch.Tensor | None = None,
                 info_pool: torch.Tensor | None = None, workspace: torch.Tensor | None = None, timing=False):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.packed = packed or pack(problems, vectors=vectors)
        pk = self.packed
        self.in_pool = in_pool if in_pool is not None else torch.from_numpy(pk.in_host).to(self.device)
        self.out_pool = out_pool if out_pool is not None else torch.empty(pk.out_size, dtype=torch.float64,
                                                                            device=self.device)
        self.info_pool = info_pool if info_pool is not None else torch.empty(pk.info_size, dtype=torch.int32,
                                                                             device=self.device)
        L = lib()
        self.h = binding.handle(self.device)
        self.count = len(pk.kinds)
        self.plan = ctypes.c_void_p()
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
        with torch.cuda.device(self.device):
            binding._bind_stream(self.h, self.device)
            rc = L.arrow_batch_create(self.h, self.count, ctypes.cast(pk.descs, ctypes.c_void_p),
                                      ctypes.c_void_p(self.in_pool.data_ptr()),
                                      ctypes.c_void_p(self.out_pool.data_ptr()),
                                      ctypes.c_void_p(self.info_pool.data_ptr()), ws_ptr, ws_bytes,
                                      (BATCH_GRAPH if graph else 0) | (BATCH_TIMING if timing else 0),
                                      ctypes.byref(self.plan))
        binding._check(rc, "arrow_batch_create")

    def run(self):
        with torch.cuda.device(self.device):
            binding._bind_stream(self.h, self.device)
            binding._check(lib().arrow_batch_run(self.plan), "arrow_batch_run")

    def run_sequential(self):
        """The same problems, one single-problem launch sequence each (reference path)."""
        with torch.cuda.device(self.device):
            binding._bind_stream(self.h, self.device)
            rc = lib().arrow_solve_sequential(self.h, self.count, ctypes.cast(self.packed.descs, ctypes.c_void_p),
                                              ctypes.c_void_p(self.in_pool.data_ptr()),
                                              ctypes.c_void_p(self.out_pool.data_ptr()),
                                              ctypes.c_void_p(self.info_pool.data_ptr()))
        binding._check(rc, "arrow_solve_sequential")

    def timing(self) -> list[float]:
        """Durations (ms) of the latest timed run's kernels: prologue, root, check, repairs, vectors."""
        ms = (ctypes.c_double * 5)()
        binding._check(lib().arrow_batch_timing(self.plan, ms), "arrow_batch_timing")
        return list(ms)

    def counters(self) -> dict:
        """Pole terms visited by the latest run's passes, summed over problems (m_p x steps)."""
        out = (ctypes.c_double * 7)()
        with torch.cuda.device(self.device):
            binding._bind_stream(self.h, self.device)
            binding._check(lib().arrow_batch_counters(self.plan, out), "arrow_batch_counters")
        keys = ("root_iter_terms", "root_dd_terms", "root_plain_terms", "check_iter_terms", "check_dd_terms",
                "check_plain_terms", "eigenpairs")
        return {k: float(v) for k, v in zip(keys, out)}

    def result(self, p: int):
        """(values, vectors or None, left vectors or None, info or None) views of problem p."""
        D = self.packed.descs[p]
        n = D.n
        lam = self.out_pool[D.lam_off:D.lam_off + n]
        if D.vec_off >= 0 and D.kind == KIND_HERM:
            V = torch.view_as_complex(self.out_pool[D.vec_off:D.vec_off + 2 * n * n].view(n * n, 2)).view(n, n).t()
        else:
            V = self.out_pool[D.vec_off:D.vec_off + n * n].view(n, n).t() if D.vec_off >= 0 else None
        U = self.out_pool[D.left_off:D.left_off + n * n].view(n, n).t() if D.left_off >= 0 else None
        info = self.info_pool[D.info_off:D.info_off + n] if D.info_off >= 0 else None
        return lam, V, U, info

    def close(self):
        if self.plan:
            binding._check(lib().arrow_batch_destroy(self.plan), "arrow_batch_destroy")
            self.plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size(packed: Packed) -> int:
    return int(lib().arrow_batch_workspace_size(len(packed.kinds), ctypes.cast(packed.descs, ctypes.c_void_p)))


def arrow_solve_batched(problems: list[Problem], device=None, vectors=True):
    """Solve every problem in one plan; returns the Batch (results via .result(p))."""
    b = Batch(problems, device=device, vectors=vectors)
    b.run()
    return b
