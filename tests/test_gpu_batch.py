"""Batches and graph plans: every job of a batch -- many fields of uneven
shapes, dtypes, block sizes, stages and boxes in one pass of persistent
kernels -- equals the same operation run alone (hsz_op_fused) bit for bit,
for every launch shape the autotuner may pick, and on every replay of a
captured graph, including after the plan's table is rewritten."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU visible", allow_module_level=True)

from paper_2603_25206_amd import hsz, synth  # noqa: E402

DEV = "cuda:0"

FIELDS = [
    ((40, 48, 70), np.float32, 1e-3, 32),
    ((33, 61), np.float64, 1e-6, 64),
    ((20, 30, 100), np.float32, 1e-4, 64),
    ((5000,), np.float32, 1e-2, 32),
    ((9, 300, 270), np.float32, 1e-4, 32),  # wider than one gradient tile
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def streams():
    out = []
    for i, (shape, dt, rel, S) in enumerate(FIELDS):
        x = synth.gaussian_mixture(shape, 5, (2.0, max(3.0, min(shape) / 2.0)), seed=50 + i).astype(dt)
        c = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S)
        out.append((x, c))
    torch.cuda.synchronize()
    return out


def rand_box(shape, rng):
    lo, hi = [], []
    for s in shape:
        a = int(rng.integers(0, s))
        lo.append(a)
        hi.append(int(rng.integers(a + 1, s + 1)))
    return tuple(lo), tuple(hi)


def make_jobs(streams, seed):
    rng = np.random.default_rng(seed)
    jobs = []
    for x, c in streams:
        nd = x.ndim
        jobs += [
            hsz.Job(c, "mean", hsz.DELTA),
            hsz.Job(c, "var", hsz.QUANT),
            hsz.Job(c, "var", hsz.DELTA, box=rand_box(x.shape, rng)),
            hsz.Job(c, "mean", hsz.QUANT, box=rand_box(x.shape, rng)),
            hsz.Job(c, "gradmag", hsz.QUANT),
            hsz.Job(c, "gradmag", hsz.QUANT, box=rand_box(x.shape, rng)),
            hsz.Job(c, "deriv", hsz.FLOAT, axis=int(rng.integers(0, nd)), box=rand_box(x.shape, rng)),
            hsz.Job(c, "deriv", hsz.QUANT, axis=nd - 1, box=rand_box(x.shape, rng)),
        ]
    return jobs


def alone(job):
    return hsz.op_fused(job.c, job.via, job.op, axis=job.axis, box=job.box)


def same(a, b):
    if isinstance(a, dict):
        return a == b or (a["n"], a["s1"], a["s2"], a["mean"]) == (b["n"], b["s1"], b["s2"], b["mean"]) and \
            (np.isnan(a["var"]) and np.isnan(b["var"]))
    return torch.equal(a, b)


def test_batch_equals_single_ops(streams):
    say("[case] batch vs single ops")
    jobs = make_jobs(streams, seed=1)
    got = hsz.batch_run(jobs)
    for k, (j, g) in enumerate(zip(jobs, got)):
        assert same(g, alone(j)), (k, j.op, j.via, j.box)


def test_batch_against_oracle(streams):
    say("[case] batch vs oracle")
    x, c = streams[0]
    buf = oracle.compress(x, 1e-3, rel=True, block=32)
    q = oracle.decompress(buf, oracle.QUANT)
    h = oracle.read_header(buf)
    xh = oracle.dequantize64(q, h.quantum)
    box = ((3, 5, 7), (30, 40, 66))
    got = hsz.batch_run([hsz.Job(c, "var", hsz.QUANT, box=box), hsz.Job(c, "gradmag", hsz.QUANT, box=box)])
    n, s1, s2 = oracle.int_sums(q, box)
    assert (got[0]["n"], got[0]["s1"], got[0]["s2"]) == (n, s1, s2)
    assert got[0]["var"] == pytest.approx(oracle.var(xh, box), rel=1e-12)
    want = oracle.gradmag(xh, box)
    g = got[1].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g - want) <= 1e-6 * np.abs(want))


@pytest.mark.parametrize("tune", [
    {"stats_waves_per_cu": 4, "grad_groups_per_cu": 2, "grad_tz": 8},
    {"stats_waves_per_cu": 16, "grad_groups_per_cu": 6, "grad_tz": 64},
    {"stats_waves_per_cu": 1, "grad_groups_per_cu": 1, "grad_tz": 3},
    {"stats_waves_per_cu": 8, "grad_groups_per_cu": 4, "grad_tz": 32, "separate_stats": 1},
])
def test_results_independent_of_launch_shape(streams, tune):
    say(f"[case] tuning {tune}")
    jobs = make_jobs(streams, seed=2)
    ref = hsz.batch_run(jobs)
    got = hsz.batch_run(jobs, tune=tune)
    for k, (a, b) in enumerate(zip(ref, got)):
        assert same(a, b), k


@pytest.mark.parametrize("graph_replay", [0, 1])
def test_plan_replays_and_updates(streams, graph_replay):
    say(f"[case] plan, graph replay {graph_replay}")
    jobs1 = make_jobs(streams, seed=3)
    plan = hsz.Plan(jobs1, tune={"grad_tz": 16, "graph_replay": graph_replay})
    want1 = [alone(j) for j in jobs1]
    for rep in range(3):
        plan.launch()
        got = plan.results()
        for k, (a, b) in enumerate(zip(got, want1)):
            assert same(a, b), (rep, k)
        # eager work and synchronisation between replays
        hsz.decompress_to_stage(streams[0][1], hsz.QUANT)
        torch.cuda.synchronize()
    jobs2 = make_jobs(streams, seed=4)  # same structure, new boxes and axes
    plan.update(jobs2)
    want2 = [alone(j) for j in jobs2]
    for rep in range(3):
        plan.launch()
        got = plan.results()
        for k, (a, b) in enumerate(zip(got, want2)):
            assert same(a, b), (rep, k)
        torch.cuda.synchronize()
    plan.close()


def test_shared_decode_statistics(streams):
    """Mean and variance over the same stream and box as a gradient job
    through D_q are summed inside the gradient tiles; the results equal the
    separate statistics pass and the single operations bit for bit (small
    and large max|q|, whole fields and boxes)."""
    say("[case] shared decode")
    rng = np.random.default_rng(11)
    jobs = []
    for x, c in streams:
        box = rand_box(x.shape, rng)
        for b in (None, box):
            jobs += [
                hsz.Job(c, "gradmag", hsz.QUANT, box=b),
                hsz.Job(c, "mean", hsz.DELTA, box=b),
                hsz.Job(c, "var", hsz.QUANT, box=b),
                hsz.Job(c, "mean", hsz.QUANT, box=b),
                hsz.Job(c, "deriv", hsz.QUANT, axis=x.ndim - 1, box=b),
            ]
    assert any(c.header.max_abs_q >= 65536 for _, c in streams)
    assert any(c.header.max_abs_q < 65536 for _, c in streams)
    shared = hsz.batch_run(jobs)
    separate = hsz.batch_run(jobs, tune={"separate_stats": 1})
    for k, (j, a, b) in enumerate(zip(jobs, shared, separate)):
        assert same(a, b), (k, j.op, j.via, j.box)
        assert same(a, alone(j)), (k, j.op, j.via, j.box)
    plan = hsz.Plan(jobs, tune={"grad_tz": 8})
    for rep in range(3):
        plan.launch()
        for k, (a, b) in enumerate(zip(plan.results(), separate)):
            assert same(a, b), (rep, k)
        torch.cuda.synchronize()
    plan.close()


def test_batch_of_every_stream_mode_and_operation(streams):
    """Items the batch kernels do not take (HSZp-nd, HSZp and block-mean
    streams, the Laplacian, the spread about the metadata mean, statistics
    through D_f) run inside the batch as operations of their own, mixed with
    kernel jobs: every result equals the operation run alone, bit for bit,
    in one-shot batches, plans launched directly and replayed as graphs, and
    after a plan update to other streams (the graph captured again)."""
    say("[case] batch of every mode")
    x0, c0 = streams[0]
    shape = (24, 20, 40)
    xs = [np.ascontiguousarray(synth.gaussian_mixture(shape, 4, (2.0, 6.0), seed=90 + k).astype(np.float32))
          for k in range(2)]

    def modes(x):
        xt = torch.from_numpy(x).to(DEV)
        return (hsz.compress(xt, 1e-3, rel=True, block=32, lorenzo=True),
                hsz.compress(xt, 1e-3, rel=True, block=32, inter_block=True),
                hsz.compress(xt, 1e-3, rel=True, block=32, mean_dec=True))

    def jobs_of(nd, flat, bm):
        box = ((2, 3, 5), (20, 17, 33))
        return [hsz.Job(c0, "gradmag", hsz.QUANT), hsz.Job(c0, "var", hsz.QUANT),
                hsz.Job(c0, "mean", hsz.FLOAT), hsz.Job(c0, "laplacian", hsz.QUANT),
                hsz.Job(nd, "mean", hsz.DELTA), hsz.Job(nd, "var", hsz.DELTA), hsz.Job(nd, "var", hsz.QUANT, box=box),
                hsz.Job(nd, "deriv", hsz.DELTA, axis=1), hsz.Job(nd, "laplacian", hsz.DELTA),
                hsz.Job(nd, "gradmag", hsz.QUANT, box=box),
                hsz.Job(flat, "var", hsz.DELTA), hsz.Job(flat, "gradmag", hsz.QUANT),
                hsz.Job(bm, "var_mt", hsz.DELTA), hsz.Job(bm, "mean", hsz.META), hsz.Job(bm, "var", hsz.QUANT)]

    jobs = jobs_of(*modes(xs[0]))
    want = [alone(j) for j in jobs]
    for k, (j, g) in enumerate(zip(jobs, hsz.batch_run(jobs))):
        assert same(g, want[k]), (k, j.op, j.via)
    jobs2 = jobs_of(*modes(xs[1]))
    want2 = [alone(j) for j in jobs2]
    for graph in (False, True):
        plan = hsz.Plan(jobs, tune={"graph_replay": graph})
        for rep in range(2):
            plan.launch()
            for k, g in enumerate(plan.results()):
                assert same(g, want[k]), (graph, rep, k)
            torch.cuda.synchronize()
        plan.update(jobs2)
        plan.launch()
        for k, g in enumerate(plan.results()):
            assert same(g, want2[k]), (graph, "updated", k)
        plan.close()


def test_batch_with_prebuilt_block_indexes(streams):
    """Jobs that carry the stream's prebuilt block index (the serving path)
    give the same results as jobs that let the batch build it."""
    say("[case] prebuilt indexes")
    jobs = make_jobs(streams, seed=5)
    ref = hsz.batch_run(jobs)
    idx_streams = [(x, hsz.Compressed(c.data, c.header)) for x, c in streams]
    for _, c in idx_streams:
        c.build_index()
    jobs_i = [hsz.Job(idx_streams[[id(c) for _, c in streams].index(id(j.c))][1], j.op, j.via, j.axis, j.box)
              for j in jobs]
    got = hsz.batch_run(jobs_i)
    for k, (a, b) in enumerate(zip(ref, got)):
        assert same(a, b), k
