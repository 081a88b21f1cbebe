"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (a plan of mean via D_p, variance via D_q and gradient magnitude via
D_q per field, statistics summed inside the gradient tiles):

  * 512^3 binary32 field, rel eb 1e-4, S = 32: compressed bytes identical to
    the oracle's; sum q and sum q^2 exact; mean and variance within 1e-12;
    the magnitude on EVERY element within 1e-6; the full-decompress
    baseline's stage-4 mean and variance against the oracle's on the stored
    binary32 values within 1e-12;
  * the other large-field variants (rel eb 1e-2 with S = 32, rel eb 1e-4 and
    1e-2 with S = 64): bytes, exact sums and every element of the magnitude;
  * 8 binary64 256^3 fields with tanh fronts, rel eb 1e-6 (large max|q|: the
    general accumulator and binary64 squared sums): the same bars on every
    field, binary64 tolerance for the magnitude;
  * 12 uneven binary32 fields (100x500x500, 256x384x384, 1800x3600): bytes,
    sums and every element of each magnitude.
The oracle runs its plain C loops over whole fields; worker threads overlap
the fields of a batch (the C calls release the interpreter lock).
"""
from __future__ import annotations

import sys
from concurrent.futures import ThreadPoolExecutor

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


def check_stats(got, q, xh, op, exact_var=True):
    n, s1, s2 = oracle.int_sums(q)
    assert (got["n"], got["s1"]) == (n, s1)
    scale = max(abs(oracle.mean(xh)), float(np.mean(np.abs(xh))))
    assert abs(got["mean"] - oracle.mean(xh)) <= 1e-12 * scale
    if op == "var":
        assert got["s2"] == s2
        want = oracle.var(xh)
        assert got["var"] == pytest.approx(want, rel=1e-12)


def check_gradmag_whole(out, xh, f64, what=""):
    """Every element of a whole-field magnitude against the oracle's."""
    want = oracle.gradmag(xh)
    got = out.reshape(want.shape).cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    if f64:
        tol = 1e-12 * np.abs(want) + 4 * 2.0 ** -53 * float(np.max(np.abs(xh)))
    else:
        tol = 1e-6 * np.abs(want)
    bad = err > tol
    assert not bad.any(), (what, int(bad.sum()), float(err.max()))
    assert np.all(got[want == 0] == 0), what


def oracle_side(x, rel):
    """The oracle's stream, q and d' = q Delta of one field (runs in a worker
    thread: the C calls release the interpreter lock)."""
    ref = oracle.compress(x, rel, rel=True, block=32)
    q = oracle.decompress(ref, oracle.QUANT)
    return ref, q, oracle.dequantize64(q, oracle.read_header(ref).quantum)


def step_plan(c):
    c.build_index()
    jobs = [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
    plan = hsz.Plan(jobs)
    plan.launch()
    res = plan.results()
    plan.close()
    return res


def test_large_field_512cube():
    say("[case] 512^3 f32 rel 1e-4 S=32: bytes, step plan vs oracle, every element")
    x = synth.make_field(synth.large_field_spec(seed=0))
    ref = oracle.compress(x, 1e-4, rel=True, block=32)
    c = hsz.compress(torch.from_numpy(x).to(DEV), 1e-4, rel=True, block=32)
    got_bytes = c.data[: c.nbytes].cpu().numpy()
    assert got_bytes.size == ref.size and np.array_equal(got_bytes, ref)
    h = oracle.read_header(ref)
    q = oracle.decompress(ref, oracle.QUANT)
    xh = oracle.dequantize64(q, h.quantum)
    mean, var, mag = step_plan(c)
    check_stats(mean, q, xh, "mean")
    check_stats(var, q, xh, "var")
    check_gradmag_whole(mag, xh, f64=False, what="512^3 step")
    # the single-operation kernel gives the same magnitudes bit for bit
    assert torch.equal(hsz.op_fused(c, hsz.QUANT, "gradmag"), mag)
    del mag, xh, q
    # the full-decompress baseline: decode to binary32, then mean and variance
    # of the stored values in binary64 (stage 4), against the oracle's own
    # stage-4 values
    say("[case] 512^3 f32 stage-4 statistics vs oracle")
    xs = oracle.decompress(ref, oracle.FLOAT).astype(np.float64)
    fbuf = hsz.decompress_to_stage(c, hsz.FLOAT)
    want_m, want_v = oracle.mean(xs), oracle.var(xs)
    scale = max(abs(want_m), float(np.mean(np.abs(xs))))
    for got in (hsz.op_on_stage(fbuf, c.header, hsz.FLOAT, "var"), hsz.op_fused(c, hsz.FLOAT, "var")):
        assert abs(got["mean"] - want_m) <= 1e-12 * scale
        assert got["var"] == pytest.approx(want_v, rel=1e-12)
    got = hsz.op_on_stage(fbuf, c.header, hsz.FLOAT, "mean")
    assert abs(got["mean"] - want_m) <= 1e-12 * scale


@pytest.mark.parametrize("rel,S", [(1e-2, 32), (1e-4, 64), (1e-2, 64)])
def test_large_field_variants(rel, S):
    """The large field's other bound and block variants: bytes, exact sums
    and every element of the magnitude, through the step's plan."""
    say(f"[case] 512^3 f32 rel {rel:g} S={S}: bytes, step plan vs oracle, every element")
    x = synth.make_field(synth.large_field_spec(seed=0))
    ref = oracle.compress(x, rel, rel=True, block=S)
    c = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S)
    got_bytes = c.data[: c.nbytes].cpu().numpy()
    assert got_bytes.size == ref.size and np.array_equal(got_bytes, ref)
    h = oracle.read_header(ref)
    # q from the oracle's quantizer (its decoder's output for this stream:
    # the bytes are identical and decode(encode(q)) = q is pinned)
    q = oracle.quantize(x, h.quantum).reshape(x.shape)
    xh = oracle.dequantize64(q, h.quantum)
    mean, var, mag = step_plan(c)
    check_stats(mean, q, xh, "mean")
    check_stats(var, q, xh, "var")
    check_gradmag_whole(mag, xh, f64=False, what=f"rel {rel:g} S={S}")


def test_front_fields_f64():
    say("[case] 8 x 256^3 f64 fronts rel 1e-6: batch plan vs oracle")
    fields = [synth.make_field(synth.front_field_spec(i)) for i in range(8)]
    comps, jobs = [], []
    for x in fields:
        c = hsz.compress(torch.from_numpy(x).to(DEV), 1e-6, rel=True, block=32)
        c.build_index()
        comps.append(c)
        jobs += [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
    assert max(c.header.max_abs_q for c in comps) >= 65536  # the general accumulator
    plan = hsz.Plan(jobs)
    plan.launch()
    res = plan.results()
    plan.close()
    with ThreadPoolExecutor(8) as pool:
        sides = list(pool.map(lambda x: oracle_side(x, 1e-6), fields))
    for k, x in enumerate(fields):
        ref, q, xh = sides[k]
        assert np.array_equal(comps[k].data[: comps[k].nbytes].cpu().numpy(), ref), k
        check_stats(res[3 * k], q, xh, "mean")
        check_stats(res[3 * k + 1], q, xh, "var")
        check_gradmag_whole(res[3 * k + 2], xh, f64=True, what=f"front field {k}")


def test_uneven_f32_batch():
    say("[case] 12 uneven f32 fields: batch plan vs oracle")
    specs = synth.batch_specs()
    fields, comps, jobs = [], [], []
    for sp, rel in specs:
        x = synth.make_field(sp)
        c = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=32)
        fields.append((x, rel))
        comps.append(c)
        jobs += [hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)]
    plan = hsz.Plan(jobs, tune={"stats_waves_per_cu": 8, "grad_groups_per_cu": 4, "grad_tz": 32})
    plan.launch()
    res = plan.results()
    plan.close()
    with ThreadPoolExecutor(8) as pool:
        sides = list(pool.map(lambda f: oracle_side(*f), fields))
    for k, (x, rel) in enumerate(fields):
        ref, q, xh = sides[k]
        assert np.array_equal(comps[k].data[: comps[k].nbytes].cpu().numpy(), ref), k
        check_stats(res[3 * k], q, xh, "mean")
        check_stats(res[3 * k + 1], q, xh, "var")
        check_gradmag_whole(res[3 * k + 2], xh, f64=False, what=f"uneven field {k}")
