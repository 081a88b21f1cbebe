"""GPU parity for fields held as compressed slabs in host memory and the
out-of-core operations over them (the sliding window of Alg. 3), for
delta, block-mean, HSZp-nd and HSZp slabs.

Bars: each slab's stream equals the oracle's encoding of that slab with
the whole field's quantizer, byte for byte apart from the recorded
extremes; statistics over the slabs give the whole field's exact integer
sums; stencils over the slabs (each slab decoded between one-plane halos
from its neighbours) agree with the oracle's operation on the whole
decompressed field (1e-6 relative for binary32, 1e-12 plus the oracle's own
rounding for binary64) and equal the same operation on the whole field's
materialised D_q bit for bit.
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
    ((37, 41, 29), np.float32, 1e-3, 32, 8, False),   # 5 slabs, the last shorter
    ((9, 17, 40), np.float32, 1e-4, 64, 1, False),    # one-plane slabs: halos on both sides
    ((181, 367), np.float64, 1e-6, 32, 50, False),
    ((100003,), np.float32, 1e-3, 32, 30000, False),  # 1D: slabs of the only axis
    ((20, 33, 30), np.float32, 1e-3, 32, 6, True),    # block-mean streams
    ((12, 10, 8), np.float32, 1e-3, 32, 64, False),   # a single slab
    ((23, 30, 64), np.float32, 1e-3, 32, 6, "lorenzo"),  # HSZp-nd slabs (two-pass D_q), the last shorter
    ((19, 21, 45), np.float64, 1e-5, 64, 5, "lorenzo"),  # HSZp-nd binary64, ragged blocks
    ((90, 300), np.float32, 1e-3, 32, 25, "lorenzo"),    # HSZp-nd 2D
    ((16, 20, 70), np.float32, 1e-3, 32, 5, "inter"),    # HSZp slabs (deltas across blocks)
]


def case_id(c):
    shape, dt, rel, S, planes, mode = c
    tag = {True: "-mean", "lorenzo": "-nd", "inter": "-flat"}.get(mode, "")
    return f"{'x'.join(map(str, shape))}-{np.dtype(dt).name}-S{S}-p{planes}" + tag


def mode_kw(mode):
    """compress() keywords of a case's decorrelation (mode True: block mean)."""
    return {"mean_dec": mode is True, "lorenzo": mode == "lorenzo", "inter_block": mode == "inter"}


@pytest.fixture(scope="module", params=CASES, ids=[case_id(c) for c in CASES])
def ocase(request):
    shape, dt, rel, S, planes, mode = request.param
    say(f"[case] ooc {case_id(request.param)}")
    f = synth.gaussian_mixture(shape, 5, (2.0, max(3.0, min(shape) / 3.0)), seed=sum(shape) + planes)
    x = np.ascontiguousarray(f.astype(dt))
    kw = mode_kw(mode)
    slabs = hsz.compress_slabs(torch.from_numpy(x), rel, planes, rel=True, block=S, device=DEV, **kw)
    whole = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S, **kw)
    torch.cuda.synchronize()
    return dict(x=x, rel=rel, S=S, planes=planes, mean=mode is True, mode=mode, slabs=slabs, whole=whole,
                shape=shape)


def test_slab_streams_match_the_oracle(ocase):
    x, S = ocase["x"], ocase["S"]
    dt = oracle.F32 if x.dtype == np.float32 else oracle.F64
    eps, quantum = oracle.quant_params(float(x.min()), float(x.max()), ocase["rel"], True, dt)
    assert ocase["whole"].header.quantum == quantum
    qs = []
    for k, (host, h) in enumerate(ocase["slabs"]):
        a = k * ocase["planes"]
        xs = x[a:a + ocase["planes"]]
        assert h.quantum == quantum and h.eb_abs == eps
        q = oracle.quantize(xs, quantum).reshape(xs.shape)
        ref = oracle.encode_q(q, xs.shape, quantum, S, dtype=dt, eb_abs=eps, **mode_kw(ocase["mode"]))
        got = host.numpy()
        assert got.size == ref.size
        keep = np.ones(ref.size, dtype=bool)
        keep[72:88] = False  # the header's extremes: the whole field's here, zero in the oracle's encoding
        assert np.array_equal(got[keep], ref[keep]), k
        qs.append(q)
    whole_q = oracle.decompress(ocase["whole"].to_bytes(), oracle.QUANT)
    assert np.array_equal(np.concatenate(qs, axis=0), whole_q)


@pytest.mark.parametrize("op", ["mean", "var"])
def test_statistics_over_slabs(ocase, op):
    c = ocase["whole"]
    q = oracle.decompress(c.to_bytes(), oracle.QUANT)
    n, s1, s2 = oracle.int_sums(q, None)
    for via in (hsz.DELTA, hsz.QUANT):
        got = hsz.ooc_op(ocase["slabs"], op, via=via, device=DEV)
        want = hsz.op_fused(c, via, op)
        assert (got["n"], got["s1"]) == (n, s1)
        assert got["mean"] == want["mean"]
        if op == "var":
            assert got["s2"] == s2
            if n > 1:
                assert got["var"] == want["var"]


def _oracle_stencil(xh, op, ax):
    if op == "deriv":
        return oracle.derivative(xh, ax)
    return oracle.gradmag(xh) if op == "gradmag" else oracle.laplacian(xh)


def _stencil_tol(x, xh, want, op):
    """1e-6 (binary32) or 1e-12 (binary64) relative per element, plus the
    oracle's own binary64 rounding of d' = q Delta where it can show: 4 units
    of 2^-53 max|d'| for a binary64 difference, 16 for the Laplacian's sums."""
    m = float(np.max(np.abs(xh)))
    if op == "laplacian":
        return (1e-6 if x.dtype == np.float32 else 1e-12) * np.abs(want) + 16 * 2.0 ** -53 * m
    if x.dtype == np.float32:
        return 1e-6 * np.abs(want)
    return 1e-12 * np.abs(want) + 4 * 2.0 ** -53 * m


@pytest.mark.parametrize("op", ["deriv", "gradmag", "laplacian"])
def test_stencils_over_slabs(ocase, op):
    """Each stencil over the host slabs against the oracle's operation on
    the whole decompressed field (d' = q Delta in binary64), and bit for bit
    against the same operation on the whole field's materialised D_q."""
    c = ocase["whole"]
    q = oracle.decompress(c.to_bytes(), oracle.QUANT)
    xh = oracle.dequantize64(q, c.header.quantum)
    qbuf = hsz.decompress_to_stage(c, hsz.QUANT)
    axes = range(len(ocase["shape"])) if op == "deriv" else [0]
    for ax in axes:
        got = hsz.ooc_op(ocase["slabs"], op, axis=ax, device=DEV).numpy()
        want = _oracle_stencil(xh, op, ax)
        assert got.shape == want.shape
        g64 = got.astype(np.float64)
        err = np.abs(g64 - want)
        bad = err > _stencil_tol(ocase["x"], xh, want, op)
        assert not bad.any(), (op, ax, int(bad.sum()), float(err.max()))
        assert np.all(g64[want == 0] == 0), (op, ax)
        same = hsz.op_on_stage(qbuf, c.header, hsz.QUANT, op, axis=ax).cpu().numpy()
        assert np.array_equal(got.view(np.uint8), same.view(np.uint8)), (op, ax)


def test_refusals():
    x = np.ascontiguousarray(synth.gaussian_mixture((16, 12, 10), 3, (2.0, 4.0), seed=5).astype(np.float32))
    slabs = hsz.compress_slabs(torch.from_numpy(x), 1e-3, 8, device=DEV)
    other = hsz.compress_slabs(torch.from_numpy(x * 3), 1e-3, 8, device=DEV)  # another quantum
    with pytest.raises(hsz.HszError) as e:
        hsz.ooc_op([slabs[0], other[1]], "mean", device=DEV)
    assert e.value.code == hsz.ERR_INVALID_ARG
    with pytest.raises(hsz.HszError) as e:
        hsz.ooc_op(slabs, "gradmag", via=hsz.DELTA, device=DEV)
    assert e.value.code == hsz.ERR_UNSUPPORTED
    with pytest.raises(hsz.HszError) as e:
        hsz.ooc_op(slabs, "deriv", axis=3, device=DEV)
    assert e.value.code == hsz.ERR_INVALID_ARG
    # a slab outside the given extremes cannot keep the bound with their quantizer
    with pytest.raises(hsz.HszError) as e:
        hsz.compress_range(torch.from_numpy(x).to(DEV), 1e-3, float(x.min()) / 2, float(x.max()) / 2)
    assert e.value.code == hsz.ERR_EB
