"""Serving on the GPU: compressed snapshots resident in HBM, a Poisson query
stream, continuous batching over several streams with every device buffer
allocated when the executor is built -- every query's result in the mix
equals the same query run alone, bit for bit, batches overlap on the
device, and result memory stays within the budget until it is released."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU visible", allow_module_level=True)

from paper_2603_25206_amd import hsz, synth  # noqa: E402
from paper_2603_25206_amd.serve import GpuExecutor, Server, make_queries, summary  # noqa: E402


def test_results_same_alone_and_in_the_mix():
    print("[case] serving mix", flush=True)
    sys.stdout.flush()
    shapes = [(48, 64, 80), (30, 50, 60)] * 3
    snaps = []
    for k, shape in enumerate(shapes):
        x = synth.gaussian_mixture(shape, 6, (3.0, 12.0), seed=300 + k).astype(np.float32)
        snaps.append(hsz.compress(torch.from_numpy(x).cuda(), 1e-3, rel=True, block=32))
    ex = GpuExecutor(snaps, n_slots=3, mem_budget=8 << 20, max_batch=32)
    arena_before = ex.arena.data_ptr()
    srv = Server(ex, mem_budget=ex.result_budget, max_batch=32, hold_results=True)
    peak = [0]

    def consume(q):  # a client that reads its result, then gives the memory back
        peak[0] = max(peak[0], srv.mem_used)
        if q.op == "gradmag":
            q.result = q.result.clone()
        srv.release(q)
    srv.on_done = consume
    qs = make_queries(shapes, 240, rate_hz=30000, seed=7, side_lo=4, side_hi=40)
    done = srv.run(qs)
    ex.close()
    assert len(done) == 240
    assert max(srv.stats.batch_sizes) > 1
    assert srv.stats.max_in_flight > 1  # batches overlapped on the device
    assert srv.stats.max_mem <= ex.result_budget and peak[0] <= ex.result_budget
    assert srv.mem_used == 0 and ex.placer.free_bytes() == ex.arena.numel()
    assert ex.arena.data_ptr() == arena_before
    for q in done:
        via = ex.via[q.op]
        alone = hsz.op_fused(snaps[q.snap], via, q.op, box=q.box)
        if q.op == "gradmag":
            assert torch.equal(q.result, alone), q.qid
        else:
            r = q.result
            assert (r["n"], r["s1"], r["mean"]) == (alone["n"], alone["s1"], alone["mean"]), q.qid
            if q.op == "var":
                assert (r["s2"], r["var"]) == (alone["s2"], alone["var"]), q.qid
    s = summary(done, wall_s=max(q.t_done for q in done) - min(q.t_arrival for q in done), bytes_per_elem=4)
    assert s["p99_ms"] >= s["p50_ms"] > 0
