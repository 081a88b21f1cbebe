"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, on the
same seeded inputs.

Bars:
  * integer and byte work bit-exact: compressed bytes, q0, widths, p, q,
    the stored binary32/binary64 decompressed values, sum q and sum q^2;
  * mean / variance: 1e-12 relative (the mean against the scale
    max(|mean|, mean |d'|) so a near-zero mean is not a false failure);
  * derivatives and gradient magnitude of binary32 fields: 1e-6 relative
    per element, exact zeros stay zero; binary64 fields: 1e-12 relative plus
    the oracle's own rounding of d' = q*Delta (4 * 2^-53 * max |d'|).
The integer routes (stages 2, 3) are compared with the oracle's operations
on the decompressed values in binary64 (q*Delta); the float route (stage 4)
with the oracle's operations on the stored decompressed field.
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


def field(shape, dtype, seed):
    k = 6
    f = synth.gaussian_mixture(shape, k, (2.0, max(3.0, min(shape) / 3.0)), seed=seed)
    rng = np.random.default_rng(seed + 1000)
    f = f * np.exp(rng.normal(0.0, 0.05, size=shape))
    return np.ascontiguousarray(f.astype(dtype))


CASES = [
    # (shape, dtype, rel eb, block)
    ((64, 64, 64), np.float32, 1e-3, 32),
    ((37, 41, 29), np.float32, 1e-4, 32),  # ragged: n % 32 != 0, nb % 64 != 0
    ((37, 41, 29), np.float32, 1e-2, 64),
    ((5, 300, 211), np.float32, 1e-4, 64),
    ((6, 37, 264), np.float32, 1e-3, 32),  # whole 256 x 16 gradient tiles beside partial ones in x and y
    ((181, 367), np.float64, 1e-6, 32),
    ((20, 33, 70), np.float64, 1e-6, 64),
    ((100003,), np.float32, 1e-3, 32),
    ((3, 5, 7), np.float32, 1e-3, 32),  # a single partial block
]


def case_id(c):
    shape, dt, rel, S = c
    return f"{'x'.join(map(str, shape))}-{np.dtype(dt).name}-{rel:g}-S{S}"


@pytest.fixture(scope="module", params=CASES, ids=[case_id(c) for c in CASES])
def case(request):
    shape, dt, rel, S = request.param
    say(f"[case] {case_id(request.param)}")
    x = field(shape, dt, seed=sum(shape) + S)
    ref = oracle.compress(x, rel, rel=True, block=S)
    xg = torch.from_numpy(x).to(DEV)
    c = hsz.compress(xg, rel, rel=True, block=S)
    torch.cuda.synchronize()
    h = oracle.read_header(ref)
    q = oracle.decompress(ref, oracle.QUANT)
    xh64 = oracle.dequantize64(q, h.quantum)
    x_stored = oracle.decompress(ref, oracle.FLOAT).astype(np.float64)
    return dict(x=x, ref=ref, c=c, h=h, q=q, xh64=xh64, x_stored=x_stored, S=S, shape=shape)


def boxes_for(shape, seed, count=3):
    rng = np.random.default_rng(seed)
    out = [None]
    for _ in range(count):
        lo, hi = [], []
        for s in shape:
            a = int(rng.integers(0, s))
            b = int(rng.integers(a + 1, s + 1))
            lo.append(a)
            hi.append(b)
        out.append((tuple(lo), tuple(hi)))
    return out


def test_compressed_bytes_identical(case):
    got = case["c"].to_bytes()
    ref = case["ref"]
    assert got.size == ref.size
    assert np.array_equal(got, ref)


def test_decode_stages_bit_exact(case):
    c, ref, h = case["c"], case["ref"], case["h"]
    # decode the oracle's own stream on the GPU (cross-decode)
    c_ref = hsz.from_bytes(ref, DEV)
    for cc in (c, c_ref):
        q0 = hsz.decompress_to_stage(cc, hsz.META, check=True)
        assert np.array_equal(q0.cpu().numpy(), oracle.decompress(ref, oracle.META))
        p, q0b = hsz.decompress_to_stage(cc, hsz.DELTA, check=True)
        op, oq0 = oracle.decompress(ref, oracle.DELTA)
        assert np.array_equal(p.cpu().numpy(), op)
        assert np.array_equal(q0b.cpu().numpy(), oq0)
        q = hsz.decompress_to_stage(cc, hsz.QUANT, check=True)
        assert np.array_equal(q.cpu().numpy(), case["q"])
        f = hsz.decompress_to_stage(cc, hsz.FLOAT, check=True)
        of = oracle.decompress(ref, oracle.FLOAT)
        assert f.dtype == (torch.float32 if h.dtype == 1 else torch.float64)
        assert np.array_equal(f.cpu().numpy().view(np.uint8), of.view(np.uint8))
    # the error bound of Sec. III-A on every element
    x = case["x"].astype(np.float64)
    if case["x"].dtype == np.float32:
        assert np.all(np.abs(x - case["x_stored"]) <= h.eb_abs)


def _check_stats(got, want_mean, want_var, scale, op, exact=None):
    assert got["mean"] == pytest.approx(want_mean, rel=0, abs=1e-12 * scale)
    if op == "var":
        assert got["var"] == pytest.approx(want_var, rel=1e-12, abs=0)
    if exact is not None:
        n, s1, s2 = exact
        assert got["n"] == n
        assert got["s1"] == s1
        if op == "var":
            assert got["s2"] == s2


@pytest.mark.parametrize("op", ["mean", "var"])
def test_stats_all_routes(case, op):
    c, h = case["c"], case["h"]
    stage_bufs = {st: hsz.decompress_to_stage(c, st) for st in (hsz.DELTA, hsz.QUANT, hsz.FLOAT)}
    for box in boxes_for(case["shape"], seed=len(case["shape"]) * 7 + case["S"]):
        exact = oracle.int_sums(case["q"], box)
        m64, v64 = oracle.mean(case["xh64"], box), oracle.var(case["xh64"], box)
        ms, vs = oracle.mean(case["x_stored"], box), oracle.var(case["x_stored"], box)
        sl = tuple(slice(l, hh) for l, hh in zip(*box)) if box else tuple(slice(None) for _ in case["shape"])
        scale64 = max(abs(m64), float(np.mean(np.abs(case["xh64"][sl]))))
        if exact[0] < 2 and op == "var":
            continue
        for st in (hsz.DELTA, hsz.QUANT):
            got = hsz.op_on_stage(stage_bufs[st], h_of(c), st, op, box=box)
            _check_stats(got, m64, v64, scale64, op, exact)
            got = hsz.op_fused(c, st, op, box=box)
            _check_stats(got, m64, v64, scale64, op, exact)
        got = hsz.op_on_stage(stage_bufs[hsz.FLOAT], h_of(c), hsz.FLOAT, op, box=box)
        _check_stats(got, ms, vs, scale64, op)
        got = hsz.op_fused(c, hsz.FLOAT, op, box=box)
        _check_stats(got, ms, vs, scale64, op)


def h_of(c):
    return c.header


def _grad_tol(case, want, route):
    if case["x"].dtype == np.float32:
        return 1e-6 * np.abs(want)
    base = case["xh64"] if route == "int" else case["x_stored"]
    return 1e-12 * np.abs(want) + 4 * 2.0 ** -53 * float(np.max(np.abs(base)))


@pytest.mark.parametrize("op", ["deriv", "gradmag"])
def test_gradient_stage_routes(case, op):
    c, h = case["c"], case["h"]
    nd = len(case["shape"])
    qbuf = hsz.decompress_to_stage(c, hsz.QUANT)
    fbuf = hsz.decompress_to_stage(c, hsz.FLOAT)
    axes = range(nd) if op == "deriv" else [0]
    for box in boxes_for(case["shape"], seed=nd * 13 + case["S"], count=2):
        for ax in axes:
            for route, st, buf, base in (("int", hsz.QUANT, qbuf, case["xh64"]),
                                         ("float", hsz.FLOAT, fbuf, case["x_stored"])):
                if op == "deriv":
                    want = oracle.derivative(base, ax, box)
                else:
                    want = oracle.gradmag(base, box)
                got = hsz.op_on_stage(buf, c.header, st, op, axis=ax, box=box).cpu().numpy().astype(np.float64)
                assert got.shape == want.shape
                err = np.abs(got - want)
                tol = _grad_tol(case, want, route)
                bad = err > tol
                assert not bad.any(), (route, ax, box, int(bad.sum()), float(err.max()))
                assert np.all(got[want == 0] == 0)


@pytest.mark.parametrize("op", ["deriv", "gradmag"])
def test_gradient_fused_routes(case, op):
    """Gradient straight from the compressed stream: via D_q (integers) and via
    D_f (floats) against the oracle, as for the stage buffers."""
    c = case["c"]
    nd = len(case["shape"])
    axes = range(nd) if op == "deriv" else [0]
    for box in boxes_for(case["shape"], seed=nd * 17 + case["S"], count=3):
        for ax in axes:
            for route, via, base in (("int", hsz.QUANT, case["xh64"]), ("float", hsz.FLOAT, case["x_stored"])):
                want = oracle.derivative(base, ax, box) if op == "deriv" else oracle.gradmag(base, box)
                got = hsz.op_fused(c, via, op, axis=ax, box=box).cpu().numpy().astype(np.float64)
                assert got.shape == want.shape
                err = np.abs(got - want)
                bad = err > _grad_tol(case, want, route)
                assert not bad.any(), (route, ax, box, int(bad.sum()), float(err.max()))
                assert np.all(got[want == 0] == 0)


def test_fast_axis_derivative_on_deltas(case):
    """Stage 2 (D_p): the derivative along the fast axis from p_j + p_{j+1}
    and the block metadata, as a stage buffer and straight from the stream;
    the other axes and the magnitude are not defined there."""
    c = case["c"]
    nd = len(case["shape"])
    fast = nd - 1
    dbuf = hsz.decompress_to_stage(c, hsz.DELTA)
    for box in boxes_for(case["shape"], seed=nd * 19 + case["S"], count=4):
        want = oracle.derivative(case["xh64"], fast, box)
        for got in (hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "deriv", axis=fast, box=box),
                    hsz.op_fused(c, hsz.DELTA, "deriv", axis=fast, box=box)):
            got = got.cpu().numpy().astype(np.float64)
            err = np.abs(got - want)
            bad = err > _grad_tol(case, want, "int")
            assert not bad.any(), (box, int(bad.sum()), float(err.max()))
            assert np.all(got[want == 0] == 0)
        # identical to the integer route on D_q, bit for bit
        qroute = hsz.op_fused(c, hsz.QUANT, "deriv", axis=fast, box=box).cpu().numpy()
        assert np.array_equal(hsz.op_fused(c, hsz.DELTA, "deriv", axis=fast, box=box).cpu().numpy(), qroute)
    for op, ax in (("gradmag", 0), ("deriv", 0)):
        if op == "deriv" and nd == 1:
            continue
        with pytest.raises(hsz.HszError) as e:
            hsz.op_fused(c, hsz.DELTA, op, axis=ax)
        assert e.value.code == hsz.ERR_UNSUPPORTED


def _lap_tol(case, want, route):
    """Integer route: the exact numerator rounded once to the field dtype,
    against the oracle's binary64 sums of d' = q*Delta (their own rounding:
    16 * 2^-53 * max|d'|).  Float route: the stencil in the field's own
    precision (a few roundings of values up to max|d'|)."""
    base = case["xh64"] if route == "int" else case["x_stored"]
    m = float(np.max(np.abs(base)))
    f32 = case["x"].dtype == np.float32
    rel = 1e-6 if f32 else 1e-12
    if route == "int":
        return rel * np.abs(want) + 16 * 2.0 ** -53 * m
    eps = 2.0 ** -24 if f32 else 2.0 ** -53
    return rel * np.abs(want) + 16 * eps * m


def test_laplacian_all_routes(case):
    """Laplacian on the materialised stages 3 and 4 and straight from the
    stream via D_q and D_f, whole field and boxes, against the oracle."""
    c = case["c"]
    qbuf = hsz.decompress_to_stage(c, hsz.QUANT)
    fbuf = hsz.decompress_to_stage(c, hsz.FLOAT)
    nd = len(case["shape"])
    for box in boxes_for(case["shape"], seed=nd * 17 + case["S"], count=2):
        for route, st, buf, base in (("int", hsz.QUANT, qbuf, case["xh64"]),
                                     ("float", hsz.FLOAT, fbuf, case["x_stored"])):
            want = oracle.laplacian(base, box)
            tol = _lap_tol(case, want, route)
            for got in (hsz.op_on_stage(buf, c.header, st, "laplacian", box=box),
                        hsz.op_fused(c, st, "laplacian", box=box)):
                got = got.cpu().numpy().astype(np.float64)
                assert got.shape == want.shape
                err = np.abs(got - want)
                bad = err > tol
                assert not bad.any(), (route, box, int(bad.sum()), float(err.max()))
            if route == "int":
                # the integer route is exact before its one rounding: stage and fused agree bit for bit
                a = hsz.op_on_stage(buf, c.header, st, "laplacian", box=box)
                b = hsz.op_fused(c, st, "laplacian", box=box)
                assert torch.equal(a, b)
    with pytest.raises(hsz.HszError) as e:
        hsz.op_fused(c, hsz.DELTA, "laplacian")
    assert e.value.code == hsz.ERR_UNSUPPORTED


def test_laplacian_large_integers_and_batches():
    """max|q| >= 2^27: the integer Laplacian is refused (its 32-bit numerator
    could overflow) while the float route still matches the oracle; in a
    batch the Laplacian runs as an operation of its own, with the same
    result and the same refusal."""
    say("[case] laplacian: max|q| >= 2^27, in a batch")
    x = field((6, 9, 40), np.float64, seed=77)
    c = hsz.compress(torch.from_numpy(x).to(DEV), 1e-9, rel=True, block=32)
    assert c.header.max_abs_q >= 2 ** 27
    with pytest.raises(hsz.HszError) as e:
        hsz.op_fused(c, hsz.QUANT, "laplacian")
    assert e.value.code == hsz.ERR_UNSUPPORTED
    ref = oracle.compress(x, 1e-9, rel=True, block=32)
    xs = oracle.decompress(ref, oracle.FLOAT).astype(np.float64)
    want = oracle.laplacian(xs)
    got = hsz.op_fused(c, hsz.FLOAT, "laplacian").cpu().numpy()
    assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want) + 16 * 2.0 ** -53 * float(np.max(np.abs(xs))))
    plan = hsz.Plan([hsz.Job(c, "laplacian", hsz.FLOAT), hsz.Job(c, "var", hsz.QUANT)])
    plan.launch()
    lap, var = plan.results()
    plan.close()
    assert torch.equal(lap.cpu(), torch.from_numpy(got))
    v1 = hsz.op_fused(c, hsz.QUANT, "var")
    assert (var["n"], var["s1"], var["s2"], var["var"]) == (v1["n"], v1["s1"], v1["s2"], v1["var"])
    with pytest.raises(hsz.HszError) as e:
        hsz.Plan([hsz.Job(c, "laplacian", hsz.QUANT)])
    assert e.value.code == hsz.ERR_UNSUPPORTED


def test_repeat_runs_identical(case):
    c = case["c"]
    a = hsz.op_fused(c, hsz.QUANT, "var")
    b = hsz.op_fused(c, hsz.QUANT, "var")
    assert a == b
    q1 = hsz.decompress_to_stage(c, hsz.QUANT).clone()
    q2 = hsz.decompress_to_stage(c, hsz.QUANT)
    assert torch.equal(q1, q2)


# ---- data-dependent errors are reported through the status word --------------

def test_nonfinite_range_and_eb_errors():
    say("[case] error statuses")
    x = torch.linspace(0, 1, 4096, device=DEV, dtype=torch.float32)
    bad = x.clone()
    bad[100] = float("nan")
    with pytest.raises(hsz.HszError) as e:
        hsz.compress(bad, 1e-3)
    assert e.value.code == hsz.ERR_NONFINITE
    with pytest.raises(hsz.HszError) as e:
        hsz.compress(x, 1e-12)
    assert e.value.code == hsz.ERR_EB
    with pytest.raises(hsz.HszError) as e:
        hsz.compress(x.double(), 1e-12)
    assert e.value.code == hsz.ERR_RANGE


def test_corrupt_width_reported_not_faulting():
    say("[case] corrupt stream")
    x = field((16, 16, 64), np.float32, 3)
    ref = oracle.compress(x, 1e-4, block=32)
    h = oracle.read_header(ref)
    bad = ref.copy()
    bad[h.off_width + 5] = 29  # widths no longer match the chunk table
    c = hsz.from_bytes(bad, DEV)
    with pytest.raises(hsz.HszError) as e:
        hsz.decompress_to_stage(c, hsz.QUANT, check=True)
    assert e.value.code == hsz.ERR_BAD_STREAM
    with pytest.raises(hsz.HszError) as e:
        hsz.op_fused(c, hsz.QUANT, "var")
    assert e.value.code == hsz.ERR_BAD_STREAM


def test_small_field_step_against_the_oracle():
    """The 64^3 field of the latency row (synth.small_field_spec, seed 0; rel
    eb 1e-3, S = 32): bytes identical to the oracle's, and the step's plan
    (mean via D_p, variance via D_q, gradient magnitude via D_q) gives the
    exact integer sums and the magnitude within 1e-6 on every element."""
    say("[case] 64^3 small field step")
    x = synth.make_field(synth.small_field_spec(seed=0))
    ref = oracle.compress(x, 1e-3, rel=True, block=32)
    c = hsz.compress(torch.from_numpy(x).to(DEV), 1e-3, rel=True, block=32)
    c.build_index()
    assert np.array_equal(c.to_bytes(), ref)
    q = oracle.decompress(ref, oracle.QUANT)
    n, s1, s2 = oracle.int_sums(q)
    want = oracle.gradmag(oracle.dequantize64(q, oracle.read_header(ref).quantum))
    plan = hsz.Plan([hsz.Job(c, "mean", hsz.DELTA), hsz.Job(c, "var", hsz.QUANT), hsz.Job(c, "gradmag", hsz.QUANT)])
    plan.launch()
    mean, var, mag = plan.results()
    plan.close()
    assert (mean["n"], mean["s1"]) == (n, s1)
    assert (var["n"], var["s1"], var["s2"]) == (n, s1, s2)
    got = mag.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-6 * np.abs(want))
    assert np.all(got[want == 0] == 0)
