"""The continuous-batching scheduler on the CPU: a simulated executor with a
virtual clock checks admission by memory and slots, FIFO order, overlap of
batches, and that every query gets its own result.  No GPU."""
from __future__ import annotations

import pytest

from paper_2603_25206_amd.serve import Executor, Query, Server, make_queries, summary


class Clock:
    """Virtual time: every reading advances it by a fixed tick."""

    def __init__(self, tick=2e-6):
        self.t = 0.0
        self.tick = tick

    def __call__(self):
        self.t += self.tick
        return self.t


class FakeExecutor(Executor):
    def __init__(self, clock, n_slots=2, per_batch=2e-4, per_elem=2e-11):
        self.clock, self.n_slots = clock, n_slots
        self.per_batch, self.per_elem = per_batch, per_elem
        self.busy = set()
        self.launch_log = []

    def result_bytes(self, q):
        return 48 if q.op != "gradmag" else 4 * q.volume()

    def launch(self, slot, queries):
        assert slot not in self.busy, "a slot ran two batches at once"
        self.busy.add(slot)
        self.launch_log.append([q.qid for q in queries])
        work = sum(q.volume() for q in queries)
        return {"slot": slot, "end": self.clock.t + self.per_batch + work * self.per_elem, "qs": queries}

    def done(self, h):
        return self.clock.t >= h["end"]

    def collect(self, h):
        self.busy.discard(h["slot"])
        return [("result-of", q.qid, q.op, q.box) for q in h["qs"]]


SHAPES = [(512, 512, 512), (100, 500, 500)]


def test_all_queries_served_in_fifo_order_with_own_results():
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, mem_budget=256 << 20, max_batch=16, clock=clock)
    qs = make_queries(SHAPES, 400, rate_hz=4000, seed=7)
    done = srv.run(qs)
    assert len(done) == 400
    for q in done:
        assert q.result == ("result-of", q.qid, q.op, q.box)
        assert q.t_arrival <= q.t_launch <= q.t_done
    # launches follow arrival order
    order = [qid for batch in ex.launch_log for qid in batch]
    assert order == sorted(order)
    assert srv.stats.max_mem <= 256 << 20
    assert srv.stats.max_in_flight <= ex.n_slots


def test_batches_overlap_and_grow_under_load():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=3, per_batch=1e-3)
    srv = Server(ex, mem_budget=1 << 34, max_batch=64, clock=clock)
    qs = make_queries(SHAPES, 600, rate_hz=20000, seed=3)
    srv.run(qs)
    assert srv.stats.max_in_flight == 3  # batches ran concurrently
    assert max(srv.stats.batch_sizes) > 1  # arrivals during execution were batched together
    s = summary(srv.done, wall_s=clock.t, bytes_per_elem=4)
    assert s["queries"] == 600 and s["p99_ms"] >= s["p50_ms"] > 0


def test_memory_budget_limits_admission():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=4)
    budget = 80 << 20  # room for one 256^3 gradient result (64 MiB) at a time
    srv = Server(ex, mem_budget=budget, max_batch=64, clock=clock)
    qs = [Query(i, 0, "gradmag", ((0, 0, 0), (256, 256, 256)), t_arrival=0.0) for i in range(6)]
    srv.run(qs)
    assert len(srv.done) == 6
    assert srv.stats.max_mem <= budget
    assert all(len(b) == 1 for b in ex.launch_log)  # never two of them in flight together
    assert srv.stats.max_in_flight == 1


def test_oversized_query_is_refused():
    clock = Clock()
    srv = Server(FakeExecutor(clock), mem_budget=1 << 20, clock=clock)
    with pytest.raises(ValueError):
        srv.submit(Query(0, 0, "gradmag", ((0, 0, 0), (256, 256, 256))))


def test_query_generator_is_seeded_and_bounded():
    a = make_queries(SHAPES, 50, rate_hz=2000, seed=11)
    b = make_queries(SHAPES, 50, rate_hz=2000, seed=11)
    assert [(q.snap, q.op, q.box, q.t_arrival) for q in a] == [(q.snap, q.op, q.box, q.t_arrival) for q in b]
    for q in a:
        shape = SHAPES[q.snap]
        for lo, hi, dim in zip(q.box[0], q.box[1], shape):
            assert 0 <= lo < hi <= dim and 32 <= hi - lo <= 256


def test_held_results_stay_charged_until_released():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=4)
    budget = 80 << 20  # one 256^3 gradient result at a time
    srv = Server(ex, mem_budget=budget, max_batch=64, clock=clock, hold_results=True)
    released = []

    def consume(q):
        assert srv.mem_used <= budget
        released.append(q.qid)
        srv.release(q)
    srv.on_done = consume
    qs = [Query(i, 0, "gradmag", ((0, 0, 0), (256, 256, 256)), t_arrival=0.0) for i in range(5)]
    srv.run(qs)
    assert released == [0, 1, 2, 3, 4] and srv.mem_used == 0
    assert all(len(b) == 1 for b in ex.launch_log)


def test_held_results_block_admission_without_release():
    clock = Clock()
    ex = FakeExecutor(clock, n_slots=4)
    srv = Server(ex, mem_budget=80 << 20, max_batch=64, clock=clock, hold_results=True)
    qs = [Query(i, 0, "gradmag", ((0, 0, 0), (256, 256, 256)), t_arrival=0.0) for i in range(2)]
    for q in qs:
        srv.submit(q)
    for _ in range(200):  # 2 ms of virtual time: the first finishes, the second waits for memory
        srv.poll()
        clock.t += 1e-5
    assert len(srv.done) == 1 and len(srv.pending) == 1
    srv.release(srv.done[0])
    while not srv.idle():
        srv.poll()
        clock.t += 1e-5
    assert len(srv.done) == 2


def test_arena_first_fit_and_coalescing():
    from paper_2603_25206_amd.serve import _Arena
    a = _Arena(4096)
    x = a.alloc(1000)  # rounded to 1024
    y = a.alloc(1024)
    z = a.alloc(2048)
    assert (x, y, z) == ((0, 1024), (1024, 1024), (2048, 2048))
    assert a.alloc(1) is None
    a.free(*y)
    assert a.alloc(2048) is None  # 1024 free in the middle only
    a.free(*x)
    assert a.free_list == [(0, 2048)]
    a.free(*z)
    assert a.free_list == [(0, 4096)] and a.free_bytes() == 4096
