"""Serving loop: continuous batching of eigen/SVD solve requests on one GPU.

Requests (arrowhead eigen, DPR1 eigen, triangular-arrowhead SVD) arrive over
time.  The loop

* admits them in arrival order whenever their device bytes (inputs, outputs,
  info words and solver workspace) fit in a fixed HBM budget -- one arena
  allocated once, so the loop itself never allocates device memory.  A request
  that does not fit is passed over by later, smaller ones until it has waited
  `aging_s`; from then on nothing is admitted past it, so the space it needs
  frees up as batches finish and it cannot starve.  Requests of order below
  `split_n` and the larger ones go to separate batches, so that a small
  request is not held until a large one in its batch is done;
* packs everything admitted since the last launch into one batch plan
  (arrow_batch_create with workspace carved from the arena) and launches it
  on one of a few streams, so batches that arrive while others run overlap
  with them on the device;
* polls completion events, records each request's arrival, admission, launch
  and completion times (latency: arrival to results resident on the device)
  and returns the arena space of finished requests.

Each request's results are the same as if it were solved alone: a problem's
kernels depend only on its own data and its order n (which fixes its lanes).
"""
from __future__ import annotations

import bisect
import ctypes
import functools
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import batch, binding
from .workloads import KIND_DPR1, KIND_HERM, KIND_SVD, Problem

ALIGN = 256


class Arena:
    """First-fit allocator over [0, capacity) with coalescing free list (byte offsets)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free_list = [(0, self.capacity)]     # sorted (offset, size)
        self.used = 0

    def alloc(self, nbytes: int):
        size = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for idx, (off, sz) in enumerate(self.free_list):
            if sz >= size:
                if sz == size:
                    del self.free_list[idx]
                else:
                    self.free_list[idx] = (off + size, sz - size)
                self.used += size
                return off, size
        return None

    def free(self, off: int, size: int):
        self.used -= size
        i = bisect.bisect_left(self.free_list, (off, 0))
        self.free_list.insert(i, (off, size))
        # coalesce with neighbours
        if i + 1 < len(self.free_list) and self.free_list[i][0] + self.free_list[i][1] == self.free_list[i + 1][0]:
            self.free_list[i] = (off, size + self.free_list[i + 1][1])
            del self.free_list[i + 1]
        if i > 0 and self.free_list[i - 1][0] + self.free_list[i - 1][1] == self.free_list[i][0]:
            self.free_list[i - 1] = (self.free_list[i - 1][0], self.free_list[i - 1][1] + self.free_list[i][1])
            del self.free_list[i]

    def largest_free(self):
        return max((sz for _, sz in self.free_list), default=0)


def _ms(pr: Problem):
    return pr.n if pr.kind == KIND_DPR1 else pr.n - 1


def _vec_at(pr: Problem):
    """Offset (doubles) of a request's vectors after its n values: Hermitian vectors are
    complex and start on 16 bytes."""
    return pr.n + (pr.n & 1 if pr.kind == KIND_HERM else 0)


def _in_doubles(pr: Problem):
    return _ms(pr) * (3 if pr.kind == KIND_HERM else 2)   # Hermitian z: (re, im) pairs


def out_doubles(pr: Problem, vectors=True):
    k = (2 if pr.kind in (KIND_SVD, KIND_HERM) else 1) if vectors else 0
    return _vec_at(pr) + k * pr.n * pr.n


def _up(nbytes: int) -> int:
    return (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN


# Arena bytes a batch needs once, whatever its size: the plan's counter block and the
# rounding of its descriptor, table, input and workspace chunks to ALIGN.
BATCH_OVERHEAD = 8 * ALIGN


@functools.lru_cache(maxsize=None)
def _plan_bytes(kind: int, n: int, vectors: bool) -> int:
    """Device bytes of a batch plan holding this one problem (the library's own layout:
    counters, descriptor, tables -- one word per vector tile among them -- and solver
    workspace); a plan of many problems needs at most the sum of these."""
    d = (batch.ArrowDesc * 1)()
    d[0].kind, d[0].n, d[0].scalar = kind, n, 1.0
    d[0].d_off, d[0].z_off, d[0].lam_off = 0, 0, 0
    d[0].vec_off = 0 if vectors else -1
    d[0].left_off = -1
    d[0].info_off = 0
    got = int(batch.lib().arrow_batch_workspace_size(1, ctypes.cast(d, ctypes.c_void_p)))
    if got <= 0:
        raise ValueError(f"no batch plan for kind {kind}, n = {n}")
    return got


def request_parts(pr: Problem, vectors=True):
    """(outputs, info, rest): arena bytes of a request's results, of its info words, and of
    its share of the batch's input chunk and plan workspace."""
    out = _up(8 * out_doubles(pr, vectors))
    info = _up(4 * pr.n)
    rest = _up(8 * _in_doubles(pr)) + _plan_bytes(pr.kind, pr.n, vectors)
    return out, info, rest


def request_bytes(pr: Problem, vectors=True):
    """Device bytes one request holds while in flight."""
    return sum(request_parts(pr, vectors))


@dataclass
class Request:
    rid: int
    problem: Problem
    arrival: float                 # seconds on the loop's clock
    admitted: float = -1.0         # its results' arena space granted
    launched: float = -1.0         # its batch's kernels queued on a stream
    done: float = -1.0             # results complete on the device (seen by the poll)
    out: tuple | None = None       # (offset, size) in the arena: values, vectors, left vectors
    info: tuple | None = None
    desc_fields: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.done - self.arrival


class Scheduler:
    """Admission policy (no device work): requests in arrival order by byte budget, batches
    capped in size; later requests may pass one that does not fit, until it has waited
    aging_s (at most `lookahead` pending requests are looked at per admission)."""

    def __init__(self, arena: Arena, max_batch=4096, vectors=True, aging_s=0.02, lookahead=256, max_work=None,
                 split_n=None):
        self.arena = arena
        self.max_batch = max_batch
        self.max_work = max_work      # cap on the sum of n^2 over a batch (None: none)
        # requests of order below split_n and the others go to separate batches (None: mixed):
        # a small request is complete only when its whole batch is
        self.split_n = split_n
        self.vectors = vectors
        self.aging_s = aging_s
        self.lookahead = lookahead
        self.pending: deque[Request] = deque()

    def submit(self, req: Request):
        if request_bytes(req.problem, self.vectors) + BATCH_OVERHEAD > self.arena.capacity:
            raise ValueError(f"request {req.rid} needs more than the whole HBM budget")
        self.pending.append(req)

    def _take(self, req: Request, reserve: int, now: float) -> int:
        """Grant req its results' and info words' space if it fits next to `reserve` bytes
        kept for the batch; returns its share of the batch's input chunk and workspace,
        or -1 when it does not fit."""
        out_b, info_b, rest = request_parts(req.problem, self.vectors)
        if self.arena.capacity - self.arena.used - reserve < out_b + info_b + rest:
            return -1
        got = self.arena.alloc(out_b)
        if got is None:
            return -1
        inf = self.arena.alloc(info_b)
        if inf is None:
            self.arena.free(*got)
            return -1
        req.out, req.info, req.admitted = got, inf, now
        return rest

    def admit(self, now: float, allow_big: bool = True) -> list[Request]:
        """Requests admitted now, in arrival order, as one batch.  Their results and info
        words are allocated here; room for the batch's inputs and plan workspace is kept
        free for the launch that follows at once.  A request that does not fit is passed
        over while it is younger than aging_s; an older one stops the scan, so that no
        later request takes the space it waits for.  With split_n, the batch takes the size
        class of the oldest pending request, or only small ones when allow_big is false."""
        out = []
        reserve = BATCH_OVERHEAD
        skipped = []
        looked = 0
        work = 0
        big = None
        if self.split_n is not None and self.pending:
            big = allow_big and self.pending[0].problem.n >= self.split_n
        while self.pending and len(out) < self.max_batch and looked < self.lookahead:
            req = self.pending.popleft()
            looked += 1
            if big is not None and (req.problem.n >= self.split_n) != big:
                skipped.append(req)            # the other size class: a batch of its own
                continue
            if out and self.max_work is not None and work + req.problem.n ** 2 > self.max_work:
                self.pending.appendleft(req)   # the batch is full; the next one starts here
                break
            rest = self._take(req, reserve, now)
            work += req.problem.n ** 2 if rest >= 0 else 0
            if rest >= 0:
                reserve += rest
                out.append(req)
                continue
            skipped.append(req)
            if now - req.arrival >= self.aging_s:
                break
        for req in reversed(skipped):   # passed-over requests keep their place in line
            self.pending.appendleft(req)
        return out

    def release(self, req: Request):
        self.arena.free(*req.out)
        self.arena.free(*req.info)


@dataclass
class InFlight:
    reqs: list
    plan: "batch.Batch | None"
    ws: tuple
    event: object
    stream: object
    staging_slot: int
    big: bool = False


class Server:
    """Continuous batching of requests on one device within an HBM budget."""

    def __init__(self, hbm_budget: int, device=None, streams=4, max_batch=4096, vectors=True,
                 staging_bytes=64 << 20, on_done=None, aging_s=0.02, max_work=None, trace=False, split_n=2048):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.arena = Arena(hbm_budget)
        self.sched = Scheduler(self.arena, max_batch=max_batch, vectors=vectors, aging_s=aging_s, max_work=max_work,
                               split_n=split_n)
        self.vectors = vectors
        self.buf = torch.empty(hbm_budget // 8, dtype=torch.float64, device=self.device)   # the arena
        self.base = self.buf.data_ptr()
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.handles = []
        L = batch.lib()
        for s in self.streams:
            h = ctypes.c_void_p()
            binding._check(L.arrow_create(ctypes.byref(h), self.device.index or 0), "arrow_create")
            binding._check(L.arrow_set_stream(h, ctypes.c_void_p(s.cuda_stream)), "arrow_set_stream")
            binding.apply_tuned(h)
            self.handles.append(h)
        self.staging = torch.empty(staging_bytes // 8 * streams, dtype=torch.float64).pin_memory()
        self.slot_doubles = staging_bytes // 8
        self.slot_busy = [None] * streams          # event of the last copy out of each staging slot
        self.inflight: list[InFlight] = []
        self.finished: list[Request] = []
        self.next_stream = 0
        self.peak_used = 0
        self.launches = 0
        # on_done(server, req) runs when req's results are complete on the device and
        # before its arena space is returned; it may read server.result(req) synchronously.
        self.on_done = on_done
        # trace: timing events around every batch's kernels, for device_intervals()
        self.trace = trace
        self.traced: list[tuple] = []

    # -- device bookkeeping -------------------------------------------------
    def _free_stream(self):
        busy = {f.staging_slot for f in self.inflight}
        for k in range(len(self.streams)):
            s = (self.next_stream + k) % len(self.streams)
            if s not in busy:
                self.next_stream = (s + 1) % len(self.streams)
                return s
        return None

    def _launch(self, reqs: list[Request], now: float) -> bool:
        s = self._free_stream()
        if s is None:
            return False
        # inputs of the batch: one contiguous arena chunk, one H2D copy
        ins = []
        for r in reqs:
            z = r.problem.z
            z = np.asarray(z, dtype=np.complex128).view(np.float64) if r.problem.kind == KIND_HERM \
                else np.asarray(z, dtype=np.float64)
            ins += [np.asarray(r.problem.d, dtype=np.float64), z]
        in_host = np.concatenate(ins) if ins else np.zeros(1)
        if in_host.size > self.slot_doubles:
            raise ValueError("batch inputs exceed the staging slot")
        descs = (batch.ArrowDesc * len(reqs))()
        ioff = 0
        for q, r in enumerate(reqs):
            pr, D = r.problem, descs[q]
            ms = _ms(pr)
            D.kind, D.n, D.scalar = pr.kind, pr.n, float(pr.scalar)
            D.d_off, D.z_off = ioff, ioff + ms     # relative; shifted below
            ioff += _in_doubles(pr)
            o = r.out[0] // 8
            D.lam_off = o
            D.vec_off = o + _vec_at(pr) if self.vectors else -1
            D.left_off = o + pr.n + pr.n * pr.n if (self.vectors and pr.kind == KIND_SVD) else -1
            D.info_off = r.info[0] // 4
        in_chunk = self.arena.alloc(8 * max(1, in_host.size))
        if in_chunk is None:
            return False
        for q in range(len(reqs)):
            descs[q].d_off += in_chunk[0] // 8
            descs[q].z_off += in_chunk[0] // 8
        L = batch.lib()
        ws_bytes = int(L.arrow_batch_workspace_size(len(reqs), ctypes.cast(descs, ctypes.c_void_p)))
        ws = self.arena.alloc(ws_bytes)
        if ws is None:
            self.arena.free(*in_chunk)
            return False
        self.peak_used = max(self.peak_used, self.arena.used)
        stream = self.streams[s]
        if self.slot_busy[s] is not None:
            self.slot_busy[s].synchronize()
        slot = self.staging[s * self.slot_doubles: s * self.slot_doubles + in_host.size]
        slot.numpy()[:] = in_host
        with torch.cuda.stream(stream):
            self.buf[in_chunk[0] // 8: in_chunk[0] // 8 + in_host.size].copy_(slot, non_blocking=True)
            copied = torch.cuda.Event()
            copied.record(stream)
            self.slot_busy[s] = copied
            if self.trace:
                t_start = torch.cuda.Event(enable_timing=True)
                t_start.record(stream)
            plan = ctypes.c_void_p()
            rc = L.arrow_batch_create(self.handles[s], len(reqs), ctypes.cast(descs, ctypes.c_void_p),
                                      ctypes.c_void_p(self.base), ctypes.c_void_p(self.base),
                                      ctypes.c_void_p(self.base), ctypes.c_void_p(self.base + ws[0]), ws[1], 0,
                                      ctypes.byref(plan))
            binding._check(rc, "arrow_batch_create")
            binding._check(L.arrow_batch_run(plan), "arrow_batch_run")
            if self.trace:
                t_end = torch.cuda.Event(enable_timing=True)
                t_end.record(stream)
                self.traced.append((t_start, t_end, s))
            ev = torch.cuda.Event()
            ev.record(stream)
        for r in reqs:
            r.launched = now
        split = self.sched.split_n
        big = split is not None and any(r.problem.n >= split for r in reqs)
        self.inflight.append(InFlight(reqs, plan, (in_chunk, ws), ev, stream, s, big))
        self.launches += 1
        return True

    def _poll(self, now_fn, keep_results):
        still = []
        for f in self.inflight:
            if f.event.query():
                t = now_fn()
                binding._check(batch.lib().arrow_batch_destroy(f.plan), "arrow_batch_destroy")
                self.arena.free(*f.ws[0])
                self.arena.free(*f.ws[1])
                for r in f.reqs:
                    r.done = t
                    self.finished.append(r)
                    if self.on_done is not None:
                        self.on_done(self, r)
                    if not keep_results:
                        self.sched.release(r)
            else:
                still.append(f)
        self.inflight = still

    def device_intervals(self):
        """(start ms, end ms, stream) of every traced batch on the device, relative to the
        first batch's start (call once they are complete)."""
        if not self.traced:
            return []
        t0 = self.traced[0][0]
        return [(t0.elapsed_time(a), t0.elapsed_time(b), s) for a, b, s in self.traced]

    def release(self, req: Request):
        """The client is done with req's results: return its arena space."""
        self.sched.release(req)

    def result(self, req: Request):
        pr, n = req.problem, req.problem.n
        o = req.out[0] // 8
        lam = self.buf[o:o + n]
        v = o + _vec_at(pr)
        if self.vectors and pr.kind == KIND_HERM:
            V = torch.view_as_complex(self.buf[v:v + 2 * n * n].view(n * n, 2)).view(n, n).t()
        else:
            V = self.buf[v:v + n * n].view(n, n).t() if self.vectors else None
        U = (self.buf[o + n + n * n:o + n + 2 * n * n].view(n, n).t()
             if (self.vectors and pr.kind == KIND_SVD) else None)
        info = self.buf.view(torch.int32)[req.info[0] // 4: req.info[0] // 4 + n]
        return lam, V, U, info

    # -- the loop -------------------------------------------------------------
    def _try_launch(self, adm: list[Request], now: float) -> list[Request]:
        """Launch adm (splitting it when the arena is too fragmented); returns what could not go."""
        if self._launch(adm, now):
            return []
        if len(adm) > 1 and not self.inflight:
            half = len(adm) // 2
            rest = self._try_launch(adm[:half], now)
            return rest + adm[half:]
        if not self.inflight:
            raise RuntimeError("a single request does not fit the HBM budget next to its workspace")
        return adm

    def run(self, arrivals: list[tuple[float, Problem]], keep_results=False, progress=None):
        """Serve requests arriving at the given times (seconds from start); returns them, finished."""
        reqs = [Request(i, pr, t) for i, (t, pr) in enumerate(arrivals)]
        for r in reqs:
            if request_bytes(r.problem, self.vectors) + BATCH_OVERHEAD > self.arena.capacity:
                raise ValueError(f"request {r.rid} exceeds the HBM budget")
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0   # noqa: E731
        nxt = 0
        reported = 0
        while nxt < len(reqs) or self.sched.pending or self.inflight:
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                self.sched.submit(reqs[nxt])
                nxt += 1
            if self.sched.pending and self._free_stream() is not None:
                # batches of large requests never take the last stream: small ones always have one
                busy_big = sum(1 for f in self.inflight if f.big)
                adm = self.sched.admit(t, allow_big=len(self.streams) < 2 or busy_big < len(self.streams) - 1)
                if adm:
                    back = self._try_launch(adm, t)
                    for r in sorted(back, key=lambda q: q.rid, reverse=True):
                        self.sched.release(r)
                        r.admitted = -1.0
                        self.sched.pending.appendleft(r)
                elif not self.inflight:
                    # nothing runs that could free space: only kept results hold the arena
                    raise RuntimeError(f"request {self.sched.pending[0].rid} cannot be admitted: the HBM budget "
                                       f"is held by results that were kept and not released")
            self._poll(now, keep_results)
            if progress and len(self.finished) - reported >= 500:
                reported = len(self.finished)
                progress(reported)
            if not self.inflight and not self.sched.pending and nxt < len(reqs):
                wait = reqs[nxt].arrival - now()
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        return reqs

    def close(self):
        for f in self.inflight:
            f.event.synchronize()
        self._poll(lambda: 0.0, True)
        L = batch.lib()
        for h in self.handles:
            L.arrow_destroy(h)
        self.handles = []
        self.buf = None          # the arena goes back to torch's caching allocator


def latency_stats(reqs: list[Request]):
    """Throughput and latency percentiles, with the latency split into its parts: waiting
    for admission (arrival to admitted), admitted but not launched (a free stream, the
    batch's inputs and plan), and on the device (launch to completion seen)."""
    lat = np.array([r.latency for r in reqs])
    t_end = max(r.done for r in reqs)
    t_start = min(r.arrival for r in reqs)
    pairs = sum(r.problem.n for r in reqs)
    parts = {"admit_wait": np.array([r.admitted - r.arrival for r in reqs]),
             "launch_wait": np.array([r.launched - r.admitted for r in reqs]),
             "device": np.array([r.done - r.launched for r in reqs])}
    slow = lat >= np.percentile(lat, 99)
    out = {"requests": len(reqs), "wall_s": t_end - t_start, "solves_per_s": len(reqs) / (t_end - t_start),
           "eigenpairs_per_s": pairs / (t_end - t_start), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}
    for k, v in parts.items():
        out[f"{k}_p50_ms"] = float(np.percentile(v, 50) * 1e3)
        out[f"{k}_p99_ms"] = float(np.percentile(v, 99) * 1e3)
        out[f"{k}_mean_ms_slowest_1pct"] = float(v[slow].mean() * 1e3)
    out["n_mean_slowest_1pct"] = float(np.mean([r.problem.n for r, s_ in zip(reqs, slow) if s_]))
    return out
