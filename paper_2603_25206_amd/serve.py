"""Serving: analytical queries against compressed snapshots resident in HBM,
with memory-admitted continuous batching.

A query is (snapshot, operation, box); operations are mean, variance and
gradient magnitude over a sub-box.  The scheduler keeps a FIFO of arrived
queries and a fixed number of execution slots (one HIP stream and one
workspace each).  Whenever a slot is free it admits, in arrival order, the
queries whose result memory fits the budget still free (up to a batch-size
cap), and launches them as ONE batched pass (hsz_batch_run) on that slot's
stream.  Batches on different slots run concurrently on the device; a query
that arrives while others are executing joins the next batch as soon as a
slot and memory free up.  Completion is observed through stream events;
latency is completion minus arrival.

The executor is injectable: GpuExecutor runs batches through the C ABI;
tests drive the same scheduler with a simulated executor and a virtual
clock.
"""
from __future__ import annotations

import collections
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


class Server:
    """Continuous-batching scheduler (FIFO, memory- and slot-admitted)."""

    def __init__(self, executor: Executor, mem_budget: int, max_batch: int = 64, clock=time.perf_counter):
        self.ex = executor
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
                results = self.ex.collect(f.handle)
                now = self.clock()
                for q, r in zip(f.queries, results):
                    q.result = r
                    q.t_done = now
                    self.done.append(q)
                self.mem_used -= f.mem
                self.free_slots.append(f.slot)
                finished += len(f.queries)
            else:
                still.append(f)
        self.in_flight = still
        while self.free_slots:
            batch, mem = [], 0
            with self._lock:
                while self.pending and len(batch) < self.max_batch:
                    need = self.ex.result_bytes(self.pending[0])
                    if self.mem_used + mem + need > self.mem_budget:
                        break  # FIFO: wait for memory rather than overtake
                    batch.append(self.pending.popleft())
                    mem += need
            if not batch:
                break
            slot = self.free_slots.pop(0)
            now = self.clock()
            for q in batch:
                q.t_launch = now
            handle = self.ex.launch(slot, batch)
            self.in_flight.append(_InFlight(slot, batch, handle, mem))
            self.mem_used += mem
            self.stats.launched_batches += 1
            self.stats.batch_sizes.append(len(batch))
            self.stats.max_in_flight = max(self.stats.max_in_flight, len(self.in_flight))
            self.stats.max_mem = max(self.stats.max_mem, self.mem_used)
        return finished

    def idle(self) -> bool:
        return not self.pending and not self.in_flight

    def run(self, queries, time_scale: float = 1.0, timeout_s: float = 600.0):
        """Replay an arrival trace open-loop: each query is submitted when the
        clock passes its arrival time; returns the completed queries."""
        order = sorted(queries, key=lambda q: q.t_arrival)
        t0 = self.clock()
        i = 0
        while i < len(order) or not self.idle():
            now = self.clock()
            if now - t0 > timeout_s:
                raise TimeoutError("serving trace did not finish")
            while i < len(order) and order[i].t_arrival * time_scale <= now - t0:
                q = order[i]
                q.t_arrival = t0 + q.t_arrival * time_scale
                self.submit(q)
                i += 1
            self.poll()
        return self.done


def summary(done, wall_s: float, bytes_per_elem: int) -> dict:
    lat = np.array([q.latency for q in done]) * 1e3
    vol = sum(q.volume() for q in done)
    return {
        "queries": len(done),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "max_ms": float(lat.max()),
        "qps": len(done) / wall_s,
        "gbs_orig": vol * bytes_per_elem / wall_s / 1e9,
    }


class GpuExecutor(Executor):
    """Runs each admitted batch as one hsz_batch_run pass on a slot's stream.

    Statistics go through the exact integer route of 'stats_via' (mean via the
    decorrelated stage, variance via the quantized stage by default), the
    gradient magnitude through 'grad_via'.  Snapshot block indexes are built
    once at construction."""

    def __init__(self, snapshots, n_slots: int = 4, tune=None, mean_via=None, var_via=None, grad_via=None):
        import torch

        from . import hsz
        self.torch, self.hsz = torch, hsz
        self.snaps = snapshots
        self.n_slots = n_slots
        self.tune = tune
        self.via = {"mean": mean_via or hsz.DELTA, "var": var_via or hsz.QUANT, "gradmag": grad_via or hsz.QUANT}
        dev = snapshots[0].data.device
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_slots)]
        self.ws = [None] * n_slots
        for c in snapshots:
            c.build_index()
        torch.cuda.synchronize()

    def result_bytes(self, q: Query) -> int:
        if q.op in ("mean", "var"):
            return 48
        esz = 4 if self.snaps[q.snap].header.dtype == 1 else 8
        return esz * q.volume()

    def launch(self, slot: int, queries: list):
        torch, hsz = self.torch, self.hsz
        s = self.streams[slot]
        with torch.cuda.stream(s):
            jobs = [hsz.Job(self.snaps[q.snap], q.op, self.via[q.op], box=q.box) for q in queries]
            nstats = sum(1 for q in queries if q.op != "gradmag")
            sbuf = torch.empty(max(1, nstats) * 48, dtype=torch.uint8, device=self.snaps[0].data.device)
            outs, k = [], 0
            for q, j in zip(queries, jobs):
                if q.op == "gradmag":
                    buf, shape = hsz._result_for(j, sbuf.device)
                    outs.append((buf, shape))
                else:
                    outs.append((sbuf[48 * k: 48 * k + 48], None))
                    k += 1
            b = hsz._Batch(jobs, outs=outs)
            need = b.workspace_bytes()
            if self.ws[slot] is None or self.ws[slot].numel() < need:
                self.ws[slot] = hsz._empty_bytes(max(need, 1 << 20), sbuf.device)
            ws = self.ws[slot]
            hsz._check(hsz.load().hsz_batch_run(b.items, len(jobs), hsz._tuning(self.tune),
                                                hsz.ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                                hsz.ctypes.c_void_p(s.cuda_stream)), "batch_run")
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, b, sbuf, queries, slot)

    def done(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle) -> list:
        ev, b, sbuf, queries, slot = handle
        hsz = self.hsz
        st = hsz.read_status(self.ws[slot], self.streams[slot])
        if st != hsz.OK:
            raise hsz.HszError(st, "serving batch")
        host = sbuf.cpu().numpy().tobytes()
        out, k = [], 0
        for q, buf, shape in zip(queries, b.results, b.shapes):
            if q.op == "gradmag":
                h = self.snaps[q.snap].header
                esz = 4 if h.dtype == 1 else 8
                out.append(buf[: esz * q.volume()].view(h.torch_dtype).view(shape))
            else:
                out.append(hsz._stats_from_raw(host[48 * k: 48 * k + 48]))
                k += 1
        return out
