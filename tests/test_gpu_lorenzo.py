"""GPU parity for HSZp-nd streams (Sec. IV, multidimensional Lorenzo
decorrelation) and HSZp streams (deltas across the blocks of the flat
field) against the oracle: compressed bytes, stages 2-4, the mean with its
weights and Alg. 4 (the running sum for HSZp) on D_p, the derivative of
Eq. (derivative_Dp) on D_p of HSZp-nd, the Laplacian of Eq. (laplacian_Dp)
and the divergence and curl of HSZp-nd vector fields on D_p, every
operation through D_q and D_f, and the routes these modes refuse.

Bars: bytes, stages and integer sums bit-exact; means and variances 1e-12
relative (the mean against max(|mean|, mean |d'|)); the D_p derivative,
Laplacian, divergence and curl equal the D_q route's bit for bit (same
integer numerators, same scaling) and the oracle's within 1e-6 (binary32)
or 1e-12 (binary64) relative plus a few 2^-53 * max|d'|.
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


CASES = [
    ((64, 64, 64), np.float32, 1e-3, 32),
    ((37, 41, 29), np.float32, 1e-4, 64),  # ragged blocks on every axis
    ((20, 37, 264), np.float32, 1e-3, 32),
    ((181, 367), np.float64, 1e-6, 32),
    ((90, 300), np.float32, 1e-3, 64),
    ((1, 17, 40), np.float32, 1e-3, 32),  # a 3D field of one plane
    ((3, 5), np.float32, 1e-3, 32),  # one partial block
    ((19, 23, 70), np.float64, 1e-6, 32),  # binary64 3D
    ((6, 9, 1100), np.float32, 1e-3, 32),  # rows of several residual tiles, the last partial
    ((30, 1300), np.float32, 1e-3, 64),
    ((13, 21, 45), np.float64, 1e-5, 64),
    ((35, 8, 128), np.float32, 1e-3, 32),  # z segments of two layers, the last one partial
    ((24, 30, 96), np.float64, 1e-6, 64),  # binary64 D_q in two passes
    ((6, 10, 512), np.float32, 1e-3, 64),  # the widest rows the two-pass D_q takes
]


def case_id(c):
    shape, dt, rel, S = c
    return f"{'x'.join(map(str, shape))}-{np.dtype(dt).name}-{rel:g}-S{S}"


@pytest.fixture(scope="module", params=CASES, ids=[case_id(c) for c in CASES])
def lcase(request):
    shape, dt, rel, S = request.param
    say(f"[case] lorenzo {case_id(request.param)}")
    f = synth.gaussian_mixture(shape, 6, (2.0, max(3.0, min(shape) / 3.0)), seed=sum(shape) + S)
    rng = np.random.default_rng(sum(shape) + 5)
    x = np.ascontiguousarray((f * np.exp(rng.normal(0.0, 0.05, size=shape))).astype(dt))
    ref = oracle.compress(x, rel, rel=True, block=S, lorenzo=True)
    c = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S, lorenzo=True)
    torch.cuda.synchronize()
    h = oracle.read_header(ref)
    q = oracle.decompress(ref, oracle.QUANT)
    p, _ = oracle.decompress(ref, oracle.DELTA)
    return dict(x=x, ref=ref, c=c, h=h, q=q, p=p, xh64=oracle.dequantize64(q, h.quantum),
                x_stored=oracle.decompress(ref, oracle.FLOAT).astype(np.float64), shape=shape, S=S,
                f32=dt == np.float32)


def test_bytes_and_stages_bit_exact(lcase):
    c, ref = lcase["c"], lcase["ref"]
    assert c.header.flags == hsz.FLAG_LORENZO
    assert np.array_equal(c.to_bytes(), ref)
    for cc in (c, hsz.from_bytes(ref, DEV)):
        p, q0 = hsz.decompress_to_stage(cc, hsz.DELTA, check=True)
        assert q0.numel() == 0
        assert np.array_equal(p.cpu().numpy(), lcase["p"])
        assert np.array_equal(hsz.decompress_to_stage(cc, hsz.QUANT, check=True).cpu().numpy(), lcase["q"])
        f = hsz.decompress_to_stage(cc, hsz.FLOAT, check=True).cpu().numpy()
        assert np.array_equal(f.view(np.uint8), oracle.decompress(ref, oracle.FLOAT).view(np.uint8))
    with pytest.raises(hsz.HszError) as e:
        hsz.decompress_to_stage(c, hsz.META)
    assert e.value.code == hsz.ERR_UNSUPPORTED


def test_statistics_on_dp(lcase):
    """Mean with the nd weights and Alg. 4, fused and on the stage-2 buffer."""
    c, h = lcase["c"], lcase["h"]
    n, s1, s2 = oracle.int_sums(lcase["q"], None)
    ms1, mmean = oracle.lz_mean_p(lcase["p"], h.quantum)
    vr = oracle.lz_var_p(lcase["p"], h.quantum)
    assert (ms1, vr["s1"], vr["s2"]) == (s1, s1, s2)  # the oracle's D_p routes against its sums of q
    dbuf = hsz.decompress_to_stage(c, hsz.DELTA)
    scale = max(abs(mmean), float(np.mean(np.abs(lcase["xh64"]))))
    for got in (hsz.op_fused(c, hsz.DELTA, "mean"), hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "mean")):
        assert (got["n"], got["s1"]) == (n, s1)
        assert got["mean"] == pytest.approx(mmean, rel=0, abs=1e-12 * scale)
    for got in (hsz.op_fused(c, hsz.DELTA, "var"), hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "var")):
        assert (got["n"], got["s1"], got["s2"]) == (n, s1, s2)
        if n > 1:
            assert got["var"] == pytest.approx(vr["var"], rel=1e-12, abs=0)
    # the caller's stage-2 buffer is left as it was
    assert np.array_equal(dbuf[0].cpu().numpy(), lcase["p"])


def _boxes(shape, seed):
    rng = np.random.default_rng(seed)
    out = [None]
    for _ in range(2):
        lo, hi = [], []
        for s in shape:
            a = int(rng.integers(0, s))
            lo.append(a)
            hi.append(int(rng.integers(a + 1, s + 1)))
        out.append((tuple(lo), tuple(hi)))
    return out


@pytest.mark.parametrize("op", ["mean", "var"])
def test_statistics_on_dq_and_df(lcase, op):
    c = lcase["c"]
    bufs = {st: hsz.decompress_to_stage(c, st) for st in (hsz.QUANT, hsz.FLOAT)}
    for box in _boxes(lcase["shape"], seed=len(lcase["shape"]) + lcase["S"]):
        n, s1, s2 = oracle.int_sums(lcase["q"], box)
        if n < 2 and op == "var":
            continue
        m64, v64 = oracle.mean(lcase["xh64"], box), oracle.var(lcase["xh64"], box)
        ms, vs = oracle.mean(lcase["x_stored"], box), oracle.var(lcase["x_stored"], box)
        sl = tuple(slice(l, hh) for l, hh in zip(*box)) if box else tuple(slice(None) for _ in lcase["shape"])
        scale = max(abs(m64), float(np.mean(np.abs(lcase["xh64"][sl]))))
        for st in (hsz.QUANT, hsz.FLOAT):
            for got in (hsz.op_fused(c, st, op, box=box), hsz.op_on_stage(bufs[st], c.header, st, op, box=box)):
                wm, wv = (m64, v64) if st == hsz.QUANT else (ms, vs)
                assert got["mean"] == pytest.approx(wm, rel=0, abs=1e-12 * scale)
                if op == "var":
                    assert got["var"] == pytest.approx(wv, rel=1e-12, abs=0)
                if st == hsz.QUANT:
                    assert (got["n"], got["s1"]) == (n, s1)
                    if op == "var":
                        assert got["s2"] == s2


def test_derivative_on_dp(lcase):
    """Eq. (derivative_Dp) along every axis, fused and on the stage-2 buffer:
    bit for bit the D_q route's result, and the oracle's recursion."""
    c, h = lcase["c"], lcase["h"]
    dbuf = hsz.decompress_to_stage(c, hsz.DELTA)
    qbuf = hsz.decompress_to_stage(c, hsz.QUANT)
    m = float(np.max(np.abs(lcase["xh64"])))
    for ax in range(len(lcase["shape"])):
        via_q = hsz.op_on_stage(qbuf, c.header, hsz.QUANT, "deriv", axis=ax).cpu().numpy()
        _, want = oracle.lz_deriv_p(lcase["p"], ax, h.quantum)
        tol = (1e-6 if lcase["f32"] else 1e-12) * np.abs(want) + 4 * 2.0 ** -53 * m
        for got in (hsz.op_fused(c, hsz.DELTA, "deriv", axis=ax),
                    hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "deriv", axis=ax)):
            g = got.cpu().numpy()
            assert g.shape == tuple(lcase["shape"])
            assert np.array_equal(g.view(np.uint8), via_q.view(np.uint8)), ax
            err = np.abs(g.astype(np.float64) - want)
            assert not (err > tol).any(), (ax, float(err.max()))


def test_laplacian_on_dp(lcase):
    """Eq. (laplacian_Dp) in the field's rank, fused and on the stage-2
    buffer: bit for bit the D_q route's result, and the oracle's Laplacian
    of d' = q Delta."""
    c = lcase["c"]
    dbuf = hsz.decompress_to_stage(c, hsz.DELTA)
    qbuf = hsz.decompress_to_stage(c, hsz.QUANT)
    via_q = hsz.op_on_stage(qbuf, c.header, hsz.QUANT, "laplacian").cpu().numpy()
    want = oracle.laplacian(lcase["xh64"])
    m = float(np.max(np.abs(lcase["xh64"])))
    tol = (1e-6 if lcase["f32"] else 1e-12) * np.abs(want) + 16 * 2.0 ** -53 * m
    for got in (hsz.op_fused(c, hsz.DELTA, "laplacian"), hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "laplacian")):
        g = got.cpu().numpy()
        assert g.shape == tuple(lcase["shape"])
        assert np.array_equal(g.view(np.uint8), via_q.view(np.uint8))
        assert not (np.abs(g.astype(np.float64) - want) > tol).any()


@pytest.mark.parametrize("op", ["gradmag", "laplacian"])
def test_stencils_through_dq_and_df(lcase, op):
    """Fused via D_q / D_f (the stage rebuilt in the workspace) equals the
    operation on the materialised stage, bit for bit, and the oracle."""
    c = lcase["c"]
    box = _boxes(lcase["shape"], seed=3)[1]
    for st in (hsz.QUANT, hsz.FLOAT):
        buf = hsz.decompress_to_stage(c, st)
        for b in (None, box):
            a = hsz.op_on_stage(buf, c.header, st, op, box=b).cpu().numpy()
            f = hsz.op_fused(c, st, op, box=b).cpu().numpy()
            assert np.array_equal(a.view(np.uint8), f.view(np.uint8)), (st, b)
    ofn = oracle.gradmag if op == "gradmag" else oracle.laplacian
    want = ofn(lcase["xh64"])
    got = hsz.op_fused(c, hsz.QUANT, op).cpu().numpy().astype(np.float64)
    m = float(np.max(np.abs(lcase["xh64"])))
    tol = (1e-6 if lcase["f32"] else 1e-12) * np.abs(want) + 16 * 2.0 ** -53 * m
    assert not (np.abs(got - want) > tol).any()


def test_refused_routes(lcase):
    c = lcase["c"]
    shape = lcase["shape"]
    box = (tuple(0 for _ in shape), tuple(shape[:-1]) + (shape[-1] - 1,)) if shape[-1] > 1 else None
    dbuf = hsz.decompress_to_stage(c, hsz.DELTA)
    bad = [lambda: hsz.op_fused(c, hsz.DELTA, "gradmag"),
           lambda: hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "gradmag"),
           lambda: hsz.op_fused(c, hsz.META, "mean"),
           lambda: hsz.op_fused(c, hsz.QUANT, "var_mt"),
           lambda: hsz.Plan([hsz.Job(c, "gradmag", hsz.DELTA)]),  # in a batch: the operation's own refusal
           lambda: c.build_index()]
    if box is not None:
        bad += [lambda: hsz.op_fused(c, hsz.DELTA, "mean", box=box),
                lambda: hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "deriv", axis=0, box=box),
                lambda: hsz.op_fused(c, hsz.DELTA, "laplacian", box=box)]
    for fn in bad:
        with pytest.raises(hsz.HszError) as e:
            fn()
        assert e.value.code == hsz.ERR_UNSUPPORTED
    # in a batch HSZp-nd streams run as operations of their own
    plan = hsz.Plan([hsz.Job(c, "mean", hsz.QUANT), hsz.Job(c, "var", hsz.DELTA)])
    plan.launch()
    mean, var = plan.results()
    plan.close()
    m1, v1 = hsz.op_fused(c, hsz.QUANT, "mean"), hsz.op_fused(c, hsz.DELTA, "var")
    assert (mean["n"], mean["s1"], mean["mean"]) == (m1["n"], m1["s1"], m1["mean"])
    assert (var["n"], var["s1"], var["s2"], var["mean"], var["var"]) == \
        (v1["n"], v1["s1"], v1["s2"], v1["mean"], v1["var"])


VCASES = [
    ((24, 30, 40), np.float32, 1e-3, 32),
    ((37, 41, 29), np.float32, 1e-4, 64),  # ragged blocks on every axis
    ((60, 90), np.float64, 1e-6, 32),
    ((1, 20, 36), np.float32, 1e-3, 32),  # one plane: the z terms are 0
    ((45, 70), np.float32, 1e-3, 64),
]


@pytest.mark.parametrize("case", VCASES, ids=[case_id(c) for c in VCASES])
@pytest.mark.parametrize("op", ["divergence", "curl"])
def test_vector_ops_on_dp(case, op):
    """Divergence and curl of HSZp-nd vector fields on D_p (each term from
    its component's p by Eq. (derivative_Dp)), on stage-2 buffers and fused
    via D_p: bit for bit the D_q route's result, and the oracle's operation
    on the components' d' = q Delta."""
    shape, dt, rel, S = case
    say(f"[case] lorenzo vector {op} {case_id(case)}")
    nd = len(shape)
    xs = [np.ascontiguousarray(synth.gaussian_mixture(shape, 5, (2.0, max(3.0, min(shape) / 3.0)),
                                                      seed=40 + 7 * k + S).astype(dt)) for k in range(nd)]
    comps = [hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S, lorenzo=True) for x in xs]
    hs = [c.header for c in comps]
    pbufs = [hsz.decompress_to_stage(c, hsz.DELTA)[0] for c in comps]
    qbufs = [hsz.decompress_to_stage(c, hsz.QUANT) for c in comps]
    ref = [g.cpu().numpy() for g in _as_list(hsz.vector_op_on_stage(qbufs, hs, hsz.QUANT, op))]
    ints = [oracle.dequantize64(oracle.decompress(c.to_bytes(), oracle.QUANT), c.header.quantum) for c in comps]
    want = (oracle.divergence if op == "divergence" else oracle.curl)(ints)
    wants = list(want) if (op == "curl" and nd == 3) else [want]
    m = max(float(np.abs(i).max()) for i in ints)
    for run in (lambda: hsz.vector_op_on_stage(pbufs, hs, hsz.DELTA, op),
                lambda: hsz.vector_op_fused(comps, op, via=hsz.DELTA)):
        got = [g.cpu().numpy() for g in _as_list(run())]
        assert len(got) == len(ref) == len(wants)
        for g, r, w in zip(got, ref, wants):
            assert np.array_equal(g.view(np.uint8), r.view(np.uint8))
            tol = (1e-6 if dt == np.float32 else 1e-12) * np.abs(w) + 16 * 2.0 ** -53 * m
            assert not (np.abs(g.astype(np.float64) - w) > tol).any()
    box = (tuple(0 for _ in shape), tuple(shape[:-1]) + (shape[-1] - 1,))
    for fn in (lambda: hsz.vector_op_on_stage(pbufs, hs, hsz.DELTA, op, box=box),
               lambda: hsz.vector_op_fused(comps, op, via=hsz.DELTA, box=box)):
        with pytest.raises(hsz.HszError) as e:
            fn()
        assert e.value.code == hsz.ERR_UNSUPPORTED


def _as_list(r):
    return list(r) if isinstance(r, tuple) else [r]


def test_vector_fields_and_one_dimensional_fields_refused():
    x = np.ascontiguousarray(synth.gaussian_mixture((12, 40), 3, (2.0, 6.0), seed=1).astype(np.float32))
    comps = [hsz.compress(torch.from_numpy(x * (k + 1)).to(DEV), 1e-3, lorenzo=True) for k in range(2)]
    with pytest.raises(hsz.HszError) as e:
        hsz.vector_op_fused(comps, "divergence")  # fused windows through D_q decode delta streams
    assert e.value.code == hsz.ERR_UNSUPPORTED
    plain = [hsz.compress(torch.from_numpy(x * (k + 1)).to(DEV), 1e-3) for k in range(2)]
    pb = [hsz.decompress_to_stage(cc, hsz.DELTA)[0] for cc in plain]
    for fn in (lambda: hsz.vector_op_on_stage(pb, [cc.header for cc in plain], hsz.DELTA, "divergence"),
               lambda: hsz.vector_op_fused(plain, "divergence", via=hsz.DELTA)):
        with pytest.raises(hsz.HszError) as e:
            fn()  # stage 2 of delta streams keeps no multidimensional neighbours
        assert e.value.code == hsz.ERR_UNSUPPORTED
    qb = [hsz.decompress_to_stage(cc, hsz.QUANT) for cc in comps]  # materialised stage 3 works
    got = hsz.vector_op_on_stage(qb, [cc.header for cc in comps], hsz.QUANT, "divergence").cpu().numpy()
    ints = [oracle.dequantize64(oracle.decompress(cc.to_bytes(), oracle.QUANT), cc.header.quantum) for cc in comps]
    want = oracle.divergence(ints)
    assert np.allclose(got, want, rtol=1e-6, atol=16 * 2.0 ** -53 * max(float(np.abs(i).max()) for i in ints))
    with pytest.raises(hsz.HszError) as e:
        hsz.compress(torch.from_numpy(x.ravel().copy()).to(DEV), 1e-3, lorenzo=True)
    assert e.value.code == hsz.ERR_UNSUPPORTED


@pytest.mark.parametrize("shape,dt,S", [((201, 400, 40), np.float32, 32), ((201, 400, 40), np.float64, 32),
                                        ((180, 400, 300), np.float32, 64)],
                         ids=["201x400x40-f32-S32", "201x400x40-f64-S32", "180x400x300-f32-S64"])
def test_compress_runs_of_block_planes(shape, dt, S):
    """Fields with enough rows of blocks that one residual work item walks
    several block planes (the halo plane carried between them), the last run
    shorter: the stream equals the oracle's byte for byte."""
    say(f"[case] lorenzo long runs {shape} {np.dtype(dt).name} S{S}")
    x = np.ascontiguousarray(synth.gaussian_mixture(shape, 4, (3.0, 30.0), seed=7).astype(dt))
    ref = oracle.compress(x, 1e-4, rel=True, block=S, lorenzo=True)
    c = hsz.compress(torch.from_numpy(x).to(DEV), 1e-4, rel=True, block=S, lorenzo=True)
    assert np.array_equal(c.to_bytes(), ref)


def test_residual_range_error():
    """A binary64 checkerboard with |q| near 2.5e8 has 3D residuals near 2e9,
    beyond 2^30 - 1: the compressor reports a range error, as the oracle."""
    idx = np.indices((4, 4, 4)).sum(axis=0)
    x = np.where(idx % 2 == 0, 1.0, -1.0).astype(np.float64)
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(x, 1e-9, rel=True, block=64, lorenzo=True)
    assert e.value.code == oracle.ERR_RANGE
    with pytest.raises(hsz.HszError) as e:
        hsz.compress(torch.from_numpy(x).to(DEV), 1e-9, rel=True, block=64, lorenzo=True)
    assert e.value.code == hsz.ERR_RANGE


# ---- HSZp: deltas across the blocks of the flat field ---------------------------------

FLAT_CASES = [
    ((1000003,), np.float32, 1e-3, 32),  # 245 scan tiles, ragged last tile and block
    ((64, 64, 64), np.float32, 1e-4, 64),
    ((181, 367), np.float64, 1e-6, 32),
    ((3000,), np.float32, 1e-3, 32),  # below one scan tile
    ((5,), np.float32, 1e-3, 32),
]


@pytest.fixture(scope="module", params=FLAT_CASES, ids=[case_id(c) for c in FLAT_CASES])
def fcase(request):
    shape, dt, rel, S = request.param
    say(f"[case] inter-block {case_id(request.param)}")
    f = synth.gaussian_mixture(shape, 5, (2.0, max(3.0, min(shape) / 3.0)), seed=sum(shape) + 2 * S)
    x = np.ascontiguousarray(f.astype(dt))
    ref = oracle.compress(x, rel, rel=True, block=S, inter_block=True)
    c = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S, inter_block=True)
    torch.cuda.synchronize()
    h = oracle.read_header(ref)
    q = oracle.decompress(ref, oracle.QUANT)
    p, _ = oracle.decompress(ref, oracle.DELTA)
    return dict(x=x, ref=ref, c=c, h=h, q=q, p=p, xh64=oracle.dequantize64(q, h.quantum), shape=shape)


def test_inter_block_bytes_stages_and_dp_statistics(fcase):
    c, ref, h = fcase["c"], fcase["ref"], fcase["h"]
    assert c.header.flags == hsz.FLAG_INTER_BLOCK
    assert np.array_equal(c.to_bytes(), ref)
    p, q0 = hsz.decompress_to_stage(c, hsz.DELTA, check=True)
    assert q0.numel() == 0 and np.array_equal(p.cpu().numpy(), fcase["p"])
    assert np.array_equal(hsz.decompress_to_stage(c, hsz.QUANT, check=True).cpu().numpy(), fcase["q"])
    f = hsz.decompress_to_stage(c, hsz.FLOAT, check=True).cpu().numpy()
    assert np.array_equal(f.view(np.uint8), oracle.decompress(ref, oracle.FLOAT).view(np.uint8))
    n, s1, s2 = oracle.int_sums(fcase["q"], None)
    ms1, mmean = oracle.lz_mean_p(fcase["p"].ravel(), h.quantum)
    vr = oracle.lz_var_p(fcase["p"].ravel(), h.quantum)
    assert (ms1, vr["s2"]) == (s1, s2)
    scale = max(abs(mmean), float(np.mean(np.abs(fcase["xh64"]))))
    dbuf = (p, q0)
    for got in (hsz.op_fused(c, hsz.DELTA, "mean"), hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "mean")):
        assert (got["n"], got["s1"]) == (n, s1)
        assert got["mean"] == pytest.approx(mmean, rel=0, abs=1e-12 * scale)
    for got in (hsz.op_fused(c, hsz.DELTA, "var"), hsz.op_on_stage(dbuf, c.header, hsz.DELTA, "var"),
                hsz.op_fused(c, hsz.QUANT, "var")):
        assert (got["n"], got["s1"], got["s2"]) == (n, s1, s2)
        if n > 1:
            assert got["var"] == pytest.approx(vr["var"], rel=1e-12, abs=0)


def test_inter_block_stencils_and_refusals(fcase):
    c = fcase["c"]
    nd = len(fcase["shape"])
    qbuf = hsz.decompress_to_stage(c, hsz.QUANT)
    a = hsz.op_on_stage(qbuf, c.header, hsz.QUANT, "gradmag").cpu().numpy()
    f = hsz.op_fused(c, hsz.QUANT, "gradmag").cpu().numpy()
    assert np.array_equal(a.view(np.uint8), f.view(np.uint8))
    want = oracle.gradmag(fcase["xh64"])
    m = float(np.max(np.abs(fcase["xh64"])))
    tol = (1e-6 if fcase["x"].dtype == np.float32 else 1e-12) * np.abs(want) + 4 * 2.0 ** -53 * m
    assert not (np.abs(a.astype(np.float64) - want) > tol).any()
    for fn in (lambda: hsz.op_fused(c, hsz.DELTA, "deriv", axis=nd - 1),
               lambda: hsz.op_fused(c, hsz.DELTA, "laplacian"),
               lambda: hsz.decompress_to_stage(c, hsz.META),
               lambda: hsz.Plan([hsz.Job(c, "deriv", hsz.DELTA, axis=nd - 1)])):
        with pytest.raises(hsz.HszError) as e:
            fn()
        assert e.value.code == hsz.ERR_UNSUPPORTED
