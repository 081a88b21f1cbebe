"""Serving: analytical queries against compressed snapshots resident in HBM,
with memory-admitted continuous batching.

A query is (snapshot, operation, box); operations are mean, variance and
gradient magnitude over a sub-box.  The scheduler keeps a FIFO of arrived
queries and a fixed number of execution slots (one HIP stream and one
workspace each).  Whenever a slot is free it admits, in arrival order, the
queries whose result memory fits the budget still free (up to a batch-size
cap), and launches them as ONE batched pass on that slot's stream.  Batches
on different slots run concurrently on the device; a query that arrives
while others are executing joins the next batch as soon as a slot and
memory free up.  Completion is observed through stream events; latency is
completion minus arrival.  With hold_results, a query's result memory stays
charged after completion until the consumer releases it (Server.release,
typically from the on_done callback), so the budget bounds what results
occupy, not only what is in flight.

The executor is injectable: GpuExecutor runs batches through the C ABI with
everything it needs on the device allocated when it is built; tests drive
the same scheduler with a simulated executor and a virtual clock.
"""
from __future__ import annotations

import collections
import gc
import threading
import time
from dataclasses import dataclass, field

import numpy as np

OPS = ("mean", "var", "gradmag")


@dataclass
class Query:
    qid: int
    snap: int
    op: str
    box: tuple  # ((lo...), (hi...)) in the snapshot's own axes
    t_arrival: float = 0.0
    t_launch: float | None = None
    t_done: float | None = None
    result: object = None
    mem: int = 0          # result memory charged to the budget
    held: bool = False    # charged until released
    slot_mem: object = None  # the executor's record of the memory it gave this query

    def volume(self) -> int:
        v = 1
        for lo, hi in zip(*self.box):
            v *= int(hi) - int(lo)
        return v

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def make_queries(shapes, count: int, rate_hz: float, seed: int = 7, side_lo: int = 32, side_hi: int = 256):
    """Poisson arrivals (exponential gaps, mean 1/rate), snapshot and operation
    uniform, box sides uniform in [side_lo, side_hi] clipped to the snapshot,
    origin uniform.  Returns queries with t_arrival relative to 0."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        s = int(rng.integers(0, len(shapes)))
        op = OPS[int(rng.integers(0, len(OPS)))]
        shape = shapes[s]
        lo, hi = [], []
        for dim in shape:
            side = min(int(rng.integers(side_lo, side_hi + 1)), dim)
            a = int(rng.integers(0, dim - side + 1))
            lo.append(a)
            hi.append(a + side)
        out.append(Query(i, s, op, (tuple(lo), tuple(hi)), t_arrival=float(t[i])))
    return out


class Executor:
    """What the scheduler needs from a backend."""

    n_slots: int = 1

    def result_bytes(self, q: Query) -> int:
        raise NotImplementedError

    def alloc(self, q: Query) -> bool:
        """Place q's result (called at admission); False if it does not fit now."""
        return True

    def free(self, q: Query):
        """Give back what alloc gave q."""

    def launch(self, slot: int, queries: list) -> object:
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def collect(self, handle) -> list:
        raise NotImplementedError


@dataclass
class _InFlight:
    slot: int
    queries: list
    handle: object
    mem: int


@dataclass
class ServerStats:
    launched_batches: int = 0
    max_in_flight: int = 0
    max_mem: int = 0
    batch_sizes: list = field(default_factory=list)
    # where the scheduler's own time goes (seconds): the longest gap between
    # two scheduling rounds, the longest launch and collect calls, and the
    # interpreter's garbage-collection pauses during run()
    max_round_gap: float = 0.0
    max_launch: float = 0.0
    max_collect: float = 0.0
    gc_pauses: int = 0
    gc_max_pause: float = 0.0


class Server:
    """Continuous-batching scheduler (FIFO, memory- and slot-admitted)."""

    def __init__(self, executor: Executor, mem_budget: int, max_batch: int = 64, clock=time.perf_counter,
                 hold_results: bool = False, on_done=None):
        self.ex = executor
        if getattr(executor, "max_batch", None) is not None and max_batch > executor.max_batch:
            raise ValueError("the executor was sized for smaller batches")
        self.hold_results = bool(hold_results)
        self.on_done = on_done
        self.mem_budget = int(mem_budget)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.pending = collections.deque()
        self.free_slots = list(range(executor.n_slots))
        self.in_flight: list[_InFlight] = []
        self.mem_used = 0
        self.done: list[Query] = []
        self.stats = ServerStats()
        self._lock = threading.Lock()

    def submit(self, q: Query):
        if self.ex.result_bytes(q) > self.mem_budget:
            raise ValueError(f"query {q.qid} needs more memory than the whole budget")
        with self._lock:
            self.pending.append(q)

    def poll(self) -> int:
        """One scheduling round: retire finished batches, then admit and launch
        into every free slot.  Returns the number of queries completed."""
        finished = 0
        still = []
        for f in self.in_flight:
            if self.ex.done(f.handle):
                t_c = self.clock()
                results = self.ex.collect(f.handle)
                now = self.clock()
                self.stats.max_collect = max(self.stats.max_collect, now - t_c)
                for q, r in zip(f.queries, results):
                    q.result = r
                    q.t_done = now
                    self.done.append(q)
                self.free_slots.append(f.slot)
                finished += len(f.queries)
                for q in f.queries:
                    if not self.hold_results:
                        self.release(q)
                    if self.on_done is not None:
                        self.on_done(q)
            else:
                still.append(f)
        self.in_flight = still
        while self.free_slots:
            batch, mem = [], 0
            with self._lock:
                while self.pending and len(batch) < self.max_batch:
                    q = self.pending[0]
                    need = self.ex.result_bytes(q)
                    if self.mem_used + mem + need > self.mem_budget or not self.ex.alloc(q):
                        break  # FIFO: wait for memory rather than overtake
                    q.mem, q.held = need, True
                    batch.append(self.pending.popleft())
                    mem += need
            if not batch:
                break
            slot = self.free_slots.pop(0)
            now = self.clock()
            for q in batch:
                q.t_launch = now
            handle = self.ex.launch(slot, batch)
            self.stats.max_launch = max(self.stats.max_launch, self.clock() - now)
            self.in_flight.append(_InFlight(slot, batch, handle, mem))
            self.mem_used += mem
            self.stats.launched_batches += 1
            self.stats.batch_sizes.append(len(batch))
            self.stats.max_in_flight = max(self.stats.max_in_flight, len(self.in_flight))
            self.stats.max_mem = max(self.stats.max_mem, self.mem_used)
        return finished

    def release(self, q: Query):
        """Return a completed query's result memory to the budget.  The
        consumer may have work reading the result still queued on its current
        stream (a copy, say): the executor reuses the memory only after that
        stream's work up to this call has run."""
        if q.held:
            self.ex.free(q)
            self.mem_used -= q.mem
            q.held = False

    def idle(self) -> bool:
        return not self.pending and not self.in_flight

    def run(self, queries, time_scale: float = 1.0, timeout_s: float = 600.0, freeze_gc: bool = True):
        """Replay an arrival trace open-loop: each query is submitted when the
        clock passes its arrival time; returns the completed queries.

        freeze_gc: objects that exist before the replay (snapshots, the
        executor, the trace) move to the interpreter's permanent generation,
        so a full garbage collection during the replay scans only what the
        replay itself creates."""
        order = sorted(queries, key=lambda q: q.t_arrival)
        gc_t = [0.0]

        def on_gc(phase, info):
            if phase == "start":
                gc_t[0] = time.perf_counter()
            else:
                d = time.perf_counter() - gc_t[0]
                self.stats.gc_pauses += 1
                self.stats.gc_max_pause = max(self.stats.gc_max_pause, d)
        if freeze_gc:
            gc.collect()
            gc.freeze()
        gc.callbacks.append(on_gc)
        try:
            t0 = self.clock()
            last = t0
            i = 0
            while i < len(order) or not self.idle():
                now = self.clock()
                self.stats.max_round_gap = max(self.stats.max_round_gap, now - last)
                last = now
                if now - t0 > timeout_s:
                    raise TimeoutError("serving trace did not finish")
                while i < len(order) and order[i].t_arrival * time_scale <= now - t0:
                    q = order[i]
                    q.t_arrival = t0 + q.t_arrival * time_scale
                    self.submit(q)
                    i += 1
                self.poll()
        finally:
            gc.callbacks.remove(on_gc)
            if freeze_gc:
                gc.unfreeze()
        return self.done


def summary(done, wall_s: float, bytes_per_elem: int) -> dict:
    """Latency percentiles, throughput, and for the slowest query the split of
    its latency into waiting for admission and being served."""
    lat = np.array([q.latency for q in done]) * 1e3
    vol = sum(q.volume() for q in done)
    worst = max(done, key=lambda q: q.latency)
    return {
        "queries": len(done),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "p999_ms": float(np.percentile(lat, 99.9)),
        "mean_ms": float(lat.mean()),
        "max_ms": float(lat.max()),
        "max_wait_ms": float((worst.t_launch - worst.t_arrival) * 1e3),
        "max_service_ms": float((worst.t_done - worst.t_launch) * 1e3),
        "qps": len(done) / wall_s,
        "gbs_orig": vol * bytes_per_elem / wall_s / 1e9,
    }


class _Arena:
    """First-fit placement of result byte ranges in one device buffer
    (offsets 256-byte aligned, neighbours coalesced on free)."""

    def __init__(self, nbytes: int):
        self.size = int(nbytes)
        self.free_list = [(0, self.size)] if self.size > 0 else []  # sorted (offset, length)

    def alloc(self, n: int):
        n = (int(n) + 255) // 256 * 256
        for i, (off, ln) in enumerate(self.free_list):
            if ln >= n:
                if ln == n:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + n, ln - n)
                return off, n
        return None

    def free(self, off: int, n: int):
        import bisect
        i = bisect.bisect_left(self.free_list, (off, 0))
        self.free_list.insert(i, (off, n))
        # coalesce with the next, then with the previous range
        if i + 1 < len(self.free_list) and off + n == self.free_list[i + 1][0]:
            self.free_list[i] = (off, n + self.free_list[i + 1][1])
            self.free_list.pop(i + 1)
        if i > 0 and self.free_list[i - 1][0] + self.free_list[i - 1][1] == off:
            po, pn = self.free_list[i - 1]
            self.free_list[i - 1] = (po, pn + self.free_list[i][1])
            self.free_list.pop(i)

    def free_bytes(self) -> int:
        return sum(ln for _, ln in self.free_list)


class GpuExecutor(Executor):
    """Runs each admitted batch as one pass on a slot's stream, with nothing
    allocated on the request path: everything is carved out of mem_budget
    when the executor is built.

    Per slot: a context (hsz_ctx) whose scratch is the batch workspace, sized
    for the largest batch the scheduler admits (max_batch jobs of any mix);
    its pinned ring carries the work tables to the device.  A device region
    takes the batch's statistics and status word and a pinned host mirror
    receives them by an asynchronous copy at the end of the pass, so
    completion is read from host memory.  Gradient results are placed in one
    device arena (the rest of the budget) at admission and stay there until
    the consumer releases the query (Server(hold_results=True)); a query's
    result is a view of the arena.

    Statistics go through the exact integer route of 'stats_via' (mean via the
    decorrelated stage, variance via the quantized stage by default), the
    gradient magnitude through 'grad_via'.  Snapshot block indexes are built
    once at construction."""

    def __init__(self, snapshots, n_slots: int = 4, tune=None, mean_via=None, var_via=None, grad_via=None,
                 mem_budget: int = 1 << 30, max_batch: int = 64):
        import torch

        from . import hsz
        self.torch, self.hsz = torch, hsz
        self.snaps = snapshots
        self.n_slots = n_slots
        self.max_batch = int(max_batch)
        self.tune = tune
        self.via = {"mean": mean_via or hsz.DELTA, "var": var_via or hsz.QUANT, "gradmag": grad_via or hsz.QUANT}
        dev = snapshots[0].data.device
        for c in snapshots:
            c.build_index()
        # the workspace of the largest admissible batch: max_batch statistics
        # jobs plus max_batch gradient jobs bound any mix of max_batch jobs
        # (the table's size does not depend on the boxes: one-element boxes and
        # a shared dummy result keep this sizing from allocating results)
        c0 = snapshots[0]
        nd = int(c0.header.ndim)
        one = ((0,) * nd, (1,) * nd)
        dummy = torch.empty(256, dtype=torch.uint8, device=dev)
        ws = 0
        for op in ("var", "gradmag"):
            b = hsz._Batch([hsz.Job(c0, op, self.via[op], box=one)] * self.max_batch,
                           outs=[(dummy, None if op == "var" else (1,) * nd)] * self.max_batch)
            ws += b.workspace_bytes()
        del dummy
        self.ws_bytes = ws + (64 << 10)
        self.stat_bytes = 48 * self.max_batch + 256  # statistics, then the status word
        fixed = n_slots * ((self.ws_bytes + (1 << 20) - 1) // (1 << 20) * (1 << 20) + self.stat_bytes)
        arena_bytes = int(mem_budget) - fixed
        if arena_bytes <= 0:
            raise ValueError(f"mem_budget {mem_budget} does not cover the slots' workspaces ({fixed} bytes)")
        self.arena = torch.empty(arena_bytes // 256 * 256, dtype=torch.uint8, device=dev)
        self.placer = _Arena(self.arena.numel())
        self.result_budget = self.arena.numel()  # what results may occupy: the scheduler's budget
        self.budget_fixed = fixed
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_slots)]
        self.ctx = [hsz.Context(scratch_bytes=self.ws_bytes, host_bytes=1 << 20, device=dev) for _ in range(n_slots)]
        self.dstat = [torch.zeros(self.stat_bytes, dtype=torch.uint8, device=dev) for _ in range(n_slots)]
        self.hstat = [torch.zeros(self.stat_bytes, dtype=torch.uint8, pin_memory=True) for _ in range(n_slots)]
        self.events = [torch.cuda.Event() for _ in range(n_slots)]
        # released result ranges wait for the consumer's stream: an event
        # recorded at release (from a pool made here), the range placed again
        # once it has passed
        self.release_pool = [torch.cuda.Event() for _ in range(2 * self.max_batch * n_slots)]
        self.deferred = []  # (event, offset, length)
        torch.cuda.synchronize()

    def result_bytes(self, q: Query) -> int:
        if q.op in ("mean", "var"):
            return 0  # in the slot's statistics region, charged at construction
        esz = 4 if self.snaps[q.snap].header.dtype == 1 else 8
        return (esz * q.volume() + 255) // 256 * 256

    def _settle(self, wait: bool = False):
        """Place again the released ranges whose consumer work has run (all of
        them, waiting, with wait)."""
        keep = []
        for ev, off, n in self.deferred:
            if wait:
                ev.synchronize()
            if wait or ev.query():
                self.placer.free(off, n)
                self.release_pool.append(ev)
            else:
                keep.append((ev, off, n))
        self.deferred = keep

    def alloc(self, q: Query) -> bool:
        n = self.result_bytes(q)
        if n == 0:
            return True
        if self.deferred:
            self._settle()
        got = self.placer.alloc(n)
        if got is None:
            return False
        q.slot_mem = got
        return True

    def free(self, q: Query):
        if q.slot_mem is not None:
            cur = self.torch.cuda.current_stream()
            if self.release_pool:
                ev = self.release_pool.pop()
                ev.record(cur)
                self.deferred.append((ev, *q.slot_mem))
            else:  # every pooled event in use: wait for the consumer instead
                cur.synchronize()
                self.placer.free(*q.slot_mem)
            q.slot_mem = None

    def launch(self, slot: int, queries: list):
        hsz = self.hsz
        s = self.streams[slot]
        jobs = [hsz.Job(self.snaps[q.snap], q.op, self.via[q.op], box=q.box) for q in queries]
        dstat = self.dstat[slot]
        outs, k = [], 0
        for q in queries:
            if q.op == "gradmag":
                off, n = q.slot_mem
                shape = tuple(int(hi) - int(lo) for lo, hi in zip(*q.box))
                outs.append((self.arena[off:off + n], shape))
            else:
                outs.append((dstat[48 * k: 48 * k + 48], None))
                k += 1
        status = dstat[48 * self.max_batch: 48 * self.max_batch + 4].view(self.torch.int32)
        b = self.ctx[slot].batch_run(jobs, tune=self.tune, stream=s, outs=outs, status=status)
        with self.torch.cuda.stream(s):
            self.hstat[slot].copy_(dstat, non_blocking=True)
        ev = self.events[slot]
        ev.record(s)
        return (ev, b, queries, slot)

    def done(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle) -> list:
        ev, b, queries, slot = handle
        hsz = self.hsz
        host = self.hstat[slot].numpy()
        st = int(host[48 * self.max_batch: 48 * self.max_batch + 4].view(np.int32)[0])
        if st != hsz.OK:
            raise hsz.HszError(st, "serving batch")
        raw = host[: 48 * self.max_batch].tobytes()
        out, k = [], 0
        for q, buf, shape in zip(queries, b.results, b.shapes):
            if q.op == "gradmag":
                h = self.snaps[q.snap].header
                esz = 4 if h.dtype == 1 else 8
                out.append(buf[: esz * q.volume()].view(h.torch_dtype).view(shape))
            else:
                out.append(hsz._stats_from_raw(raw[48 * k: 48 * k + 48]))
                k += 1
        return out

    def close(self):
        self._settle(wait=True)
        for c in self.ctx:
            c.close()
