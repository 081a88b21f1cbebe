"""GPU tests of contexts (hsz_ctx): the pipeline of Sec. III-A -- compress,
decode to a stage, operate there, batch -- issued through one context on
one stream, and the out-of-core operation of Alg. 3 enqueued on the
caller's stream.

Bars: the calls return while a spin kernel enqueued before them still runs
(none waits on the host); after the stream completes, q equals the oracle's
bit for bit, integer sums equal the oracle's exactly, the gradient
magnitude is within 1e-6 relative of the oracle's (zeros exact), batch
results equal the single operations bit for bit, and the asynchronous
out-of-core results equal the synchronous entry point's bit for bit.
"""
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


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def spin_cycles(ms: float) -> int:
    """Cycles of torch.cuda._sleep that take about 'ms' on this device."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(1000)
    e0.record(s)
    torch.cuda._sleep(1_000_000)
    e1.record(s)
    e1.synchronize()
    per_ms = 1_000_000 / max(e0.elapsed_time(e1), 1e-3)
    return int(per_ms * ms)


def _check_mag(got, want, what):
    got = got.cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    assert not (err > 1e-6 * np.abs(want)).any(), what
    assert np.all(got[want == 0] == 0), what


def test_pipeline_through_context_does_not_wait():
    shape = (24, 40, 96)
    say(f"[case] ctx pipeline {shape}")
    x = synth.make_field(synth.FieldSpec(shape, "f32", k=5, sigma=(2.0, 9.0), noise=1e-3, seed=7))
    ref = oracle.compress(x, 1e-3, rel=True, block=32)
    q_ref = oracle.decompress(ref, oracle.QUANT)
    h_ref = oracle.read_header(ref)
    xh = oracle.dequantize64(q_ref, h_ref.quantum)
    c = hsz.compress(torch.from_numpy(x).to(DEV), 1e-3, rel=True, block=32)  # reads its header back (explicit)
    c.build_index()
    h = c.header
    ctx = hsz.Context(scratch_bytes=64 << 20, host_bytes=1 << 20)
    try:
        s = torch.cuda.Stream()
        n = int(h.n)
        qbuf = torch.empty(4 * n, dtype=torch.uint8, device=DEV)
        s_var = torch.empty(64, dtype=torch.uint8, device=DEV)
        gbuf = torch.empty(4 * n, dtype=torch.uint8, device=DEV)
        jobs = [hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
        cycles = spin_cycles(300.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            torch.cuda._sleep(cycles)
        qv = ctx.decompress_to_stage(c, hsz.QUANT, out=qbuf, stream=s)
        ctx.op_on_stage(qv, h, hsz.QUANT, hsz.VAR, out=s_var, stream=s)
        ctx.op_fused(c, hsz.QUANT, hsz.GRADMAG, out=gbuf, stream=s)
        b = ctx.batch_run(jobs, stream=s)
        busy = not s.query()
        s.synchronize()
        assert busy, "a context call waited for the stream"
        assert ctx.status(s) == hsz.OK
        assert np.array_equal(qv.cpu().numpy(), q_ref)
        st = hsz.stats_of(s_var)
        assert (st["n"], st["s1"], st["s2"]) == oracle.int_sums(q_ref)
        mag = gbuf.view(torch.float32)[:n].view(shape)
        _check_mag(mag, oracle.gradmag(xh), "op_fused")
        bvar, bmag = b.outputs()
        assert (bvar["n"], bvar["s1"], bvar["s2"]) == (st["n"], st["s1"], st["s2"])
        assert torch.equal(bmag, mag)
    finally:
        ctx.close()


def test_context_capacity_and_tuning():
    shape = (8, 16, 64)
    x = synth.make_field(synth.FieldSpec(shape, "f32", k=3, sigma=(2.0, 5.0), noise=1e-3, seed=3))
    c = hsz.compress(torch.from_numpy(x).to(DEV), 1e-3, rel=True, block=32)
    ctx = hsz.Context(scratch_bytes=0, host_bytes=1 << 16)
    try:
        with pytest.raises(hsz.HszError) as e:
            ctx.batch_run([hsz.Job(c, "var", hsz.QUANT)])
        assert e.value.code == hsz.ERR_CAPACITY
        ctx.reserve(16 << 20)
        assert ctx.scratch.numel() >= 16 << 20
        assert ctx.get_tuning("none") is None
        ctx.set_tuning("k", {"grad_tz": 16, "grad_tile_x": 256})
        t = ctx.get_tuning("k")
        assert t["grad_tz"] == 16 and t["grad_tile_x"] == 256
        b = ctx.batch_run([hsz.Job(c, "var", hsz.QUANT)], tune=t)
        torch.cuda.synchronize()
        (v,) = b.outputs()
        q = oracle.decompress(oracle.compress(x, 1e-3, rel=True, block=32), oracle.QUANT)
        assert (v["n"], v["s1"], v["s2"]) == oracle.int_sums(q)
    finally:
        ctx.close()


@pytest.mark.parametrize("mode", ["delta", "nd"])
@pytest.mark.parametrize("op", ["mean", "var", "gradmag"])
def test_out_of_core_async_equals_sync(op, mode):
    shape = (37, 41, 32)
    say(f"[case] ctx ooc {op} {mode}")
    f = synth.gaussian_mixture(shape, 5, (2.0, 12.0), seed=11)
    x = np.ascontiguousarray(f.astype(np.float32))
    slabs = hsz.compress_slabs(torch.from_numpy(x), 1e-3, 8, rel=True, block=32, device=DEV,
                               lorenzo=mode == "nd")
    want = hsz.ooc_op(slabs, op)
    ctx = hsz.Context(scratch_bytes=0, host_bytes=1 << 16)
    try:
        ctx.reserve(hsz.ooc_workspace_bytes(slabs, op))
        s = torch.cuda.Stream()
        status = torch.full((1,), -99, dtype=torch.int32, device=DEV)
        cycles = spin_cycles(200.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            torch.cuda._sleep(cycles)
        out1 = ctx.ooc_op(slabs, op, stream=s)
        out2 = ctx.ooc_op(slabs, op, stream=s, status=status)  # ordered after the first on the device
        busy = not s.query()
        s.synchronize()
        assert busy, "the out-of-core call waited for the stream"
        assert int(status.item()) == hsz.OK
        for out in (out1, out2):
            if op == "gradmag":
                got = out.view(torch.float32).view(want.shape)
                assert torch.equal(got, want)
            else:
                got = hsz.stats_of_host(out)
                for k in ("n", "s1", "mean"):
                    assert got[k] == want[k], (k, got[k], want[k])
                if op == "var":
                    assert got["s2"] == want["s2"] and got["var"] == want["var"]
    finally:
        ctx.close()
