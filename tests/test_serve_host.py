"""Host-side logic of the serving loop: arena allocator and admission policy (no GPU)."""
import ctypes

import numpy as np

from paper_1302_7203_amd import workloads as W
from paper_1302_7203_amd.serve import (ALIGN, BATCH_OVERHEAD, Arena, Request, Scheduler, request_bytes,
                                      request_parts)


def test_arena_first_fit_and_coalescing():
    a = Arena(10 * ALIGN)
    x = a.alloc(3 * ALIGN)
    y = a.alloc(1)
    z = a.alloc(2 * ALIGN)
    assert x == (0, 3 * ALIGN) and y == (3 * ALIGN, ALIGN) and z == (4 * ALIGN, 2 * ALIGN)
    assert a.used == 6 * ALIGN
    assert a.alloc(5 * ALIGN) is None            # only 4 left
    a.free(*y)
    assert a.alloc(2 * ALIGN)[0] == 6 * ALIGN    # hole of 1 too small: first fit goes past it
    a.free(*x)
    a.free(*z)
    # x, y's hole and z coalesce into [0, 6*ALIGN)
    assert a.free_list[0] == (0, 6 * ALIGN)
    assert a.alloc(6 * ALIGN) == (0, 6 * ALIGN)


def test_arena_random_alloc_free_keeps_invariants():
    rng = np.random.default_rng(0)
    a = Arena(1 << 20)
    live = []
    for _ in range(2000):
        if live and rng.uniform() < 0.45:
            a.free(*live.pop(int(rng.integers(len(live)))))
        else:
            got = a.alloc(int(rng.integers(1, 40000)))
            if got:
                live.append(got)
        fl = a.free_list
        assert all(fl[i][0] + fl[i][1] < fl[i + 1][0] for i in range(len(fl) - 1))   # sorted, coalesced
        assert a.used == sum(s for _, s in live)
        spans = sorted(live + fl)
        assert all(spans[i][0] + spans[i][1] == spans[i + 1][0] for i in range(len(spans) - 1))
    for x in live:
        a.free(*x)
    assert a.free_list == [(0, 1 << 20)] and a.used == 0


def _side(r):
    return request_parts(r.problem)[2]


def test_fifo_admission_by_budget():
    """Each admit() forms one batch that the server launches at once (allocating its
    inputs and workspace, here simulated) before the next admit()."""
    rng = np.random.default_rng(1)
    probs = [W.uniform_arrow(n, rng) for n in (100, 400, 50, 50, 60)]
    cap = request_bytes(probs[0]) + request_bytes(probs[1]) + BATCH_OVERHEAD
    s = Scheduler(Arena(cap))
    for i, p in enumerate(probs):
        s.submit(Request(i, p, 0.0))
    first = s.admit(0.0)
    assert [r.rid for r in first] == [0, 1]           # request 2 would fit alone but waits its turn
    launch1 = s.arena.alloc(sum(_side(r) for r in first))
    assert launch1 is not None                        # the reserve kept room for the launch
    assert [r.rid for r in s.admit(0.0)] == []
    s.arena.free(*launch1)                            # batch 1 finished ...
    s.release(first[1])                               # ... and request 1's results were taken
    nxt = s.admit(1.0)
    assert [r.rid for r in nxt] == [2, 3, 4][: len(nxt)] and len(nxt) >= 1   # FIFO prefix
    launch2 = s.arena.alloc(sum(_side(r) for r in nxt))
    assert launch2 is not None
    assert s.arena.used <= cap
    s.arena.free(*launch2)
    for r in [first[0]] + nxt:
        s.release(r)
    assert s.arena.used == 0


def test_admission_passes_a_blocked_request_until_it_ages():
    """A request that does not fit is passed over by later ones that do, while it is
    younger than aging_s; once older, nothing is admitted past it, and it goes first
    when the space frees up."""
    rng = np.random.default_rng(4)
    big = [W.uniform_arrow(300, rng) for _ in range(2)]
    small = [W.uniform_arrow(40, rng) for _ in range(4)]
    cap = request_bytes(big[0]) + 2 * request_bytes(small[0]) + BATCH_OVERHEAD
    assert cap < 2 * request_bytes(big[0])
    s = Scheduler(Arena(cap), aging_s=0.05)
    for i, p in enumerate([big[0], big[1], small[0], small[1]]):
        s.submit(Request(i, p, 0.0))
    first = s.admit(0.01)                       # request 1 (young, no room) is passed over
    assert [r.rid for r in first] == [0, 2, 3]
    assert [r.rid for r in s.pending] == [1]
    launch1 = s.arena.alloc(sum(_side(r) for r in first))
    assert launch1 is not None
    s.arena.free(*launch1)                      # the batch finished ...
    s.release(first[1])                         # ... and two small results were taken
    s.release(first[2])
    s.submit(Request(4, small[2], 0.06))
    # request 1 is now older than aging_s and still does not fit: request 4 would, but may
    # not pass it
    assert s.admit(0.07) == [] and [r.rid for r in s.pending] == [1, 4]
    s.release(first[0])
    second = s.admit(0.08)
    assert [r.rid for r in second][0] == 1
    for r in second:
        s.release(r)
    assert s.arena.used == 0


def test_size_classes_form_separate_batches():
    """With split_n, a batch holds only requests below it or only the others: the class of
    the oldest pending request; the rest wait for the next admission, in order."""
    rng = np.random.default_rng(6)
    ns = (50, 900, 60, 1200, 70)
    probs = [W.uniform_arrow(n, rng) for n in ns]
    s = Scheduler(Arena(1 << 30), split_n=512)
    for i, p in enumerate(probs):
        s.submit(Request(i, p, 0.0))
    first = s.admit(0.0)
    assert [r.rid for r in first] == [0, 2, 4]
    assert [r.rid for r in s.pending] == [1, 3]
    second = s.admit(0.0)
    assert [r.rid for r in second] == [1, 3] and not s.pending
    for r in first + second:
        s.release(r)
    assert s.arena.used == 0


def test_request_bytes_cover_the_plan_workspace():
    """A batch's input chunk and plan workspace fit in its requests' reserved share plus
    the per-batch overhead, for batches of one and of many."""
    from paper_1302_7203_amd import batch, build
    if build.stale():
        build.build()
    L = batch.lib()
    rng = np.random.default_rng(2)
    for trial in range(6):
        k = 1 if trial < 2 else 20
        gen = (W.uniform_arrow, W.dpr1, W.svd_arrow, W.herm_arrow)
        hi = 300 if trial % 2 == 0 else 3000     # small problems, and row-tiled ones with long tile tables
        probs = [gen[c](int(n), rng) for n, c in zip(rng.integers(1, hi, k), rng.integers(0, 4, k))]
        pk = batch.pack(probs)
        ws = int(L.arrow_batch_workspace_size(len(probs), ctypes.cast(pk.descs, ctypes.c_void_p)))
        up = lambda x: (x + ALIGN - 1) // ALIGN * ALIGN   # noqa: E731
        reserved = sum(request_parts(p)[2] for p in probs) + BATCH_OVERHEAD
        assert up(ws) + up(8 * pk.in_host.size) <= reserved


def test_hermitian_packing_aligns_complex_vectors():
    """Hermitian z goes in as (re, im) pairs and its complex vectors start on 16 bytes."""
    from paper_1302_7203_amd import batch
    rng = np.random.default_rng(3)
    probs = [W.uniform_arrow(4, rng), W.herm_arrow(5, rng), W.dpr1(3, rng), W.herm_arrow(4, rng)]
    pk = batch.pack(probs)
    for p, pr in enumerate(probs):
        D = pk.descs[p]
        if pr.kind == W.KIND_HERM:
            assert D.vec_off % 2 == 0
            z = pk.in_host[D.z_off:D.z_off + 2 * (pr.n - 1)].view(np.complex128)
            assert np.array_equal(z, pr.z)
    assert pk.descs[2].d_off == pk.descs[1].z_off + 2 * (probs[1].n - 1)
