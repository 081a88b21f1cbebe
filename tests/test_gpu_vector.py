"""GPU parity for divergence and curl of vector fields (one compressed stream
per component) against the oracle.

Bars: the integer route (fused from the streams through D_q, and on stage-3
buffers) sums exact integer numerators scaled by each component's quantum
and rounds once, so it must agree with the oracle's binary64 operators on
d' = q*Delta within 1e-6 relative for binary32 (1e-12 for binary64) plus the
oracle's own rounding (16 * 2^-53 * max|d'|); the two integer paths agree
bit for bit.  The float route (stage-4 buffers) differences the stored
values in the field's precision: 1e-6 (1e-12) relative plus 16 units of
that precision times max|d'|.  The binary32 cases (blocks at most 16 bits
wide) take the fused kernel's pair decode, blocks of 32 and of 64; the
binary64 ones (wider blocks) its slot-by-slot decode.
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
    # (shape, dtype, rel eb per component, block)
    ((1000,), np.float32, (1e-3,), 32),
    ((90, 300), np.float32, (1e-3, 1e-4), 32),
    ((37, 150), np.float64, (1e-6, 1e-5), 64),
    ((20, 37, 264), np.float32, (1e-3, 1e-4, 1e-2), 32),  # whole and partial tiles, ragged blocks
    ((9, 33, 70), np.float64, (1e-6, 1e-6, 1e-7), 32),
    ((1, 17, 40), np.float32, (1e-3, 1e-3, 1e-3), 32),   # length-1 axis 0
    ((30, 200), np.float32, (1e-3, 1e-2), 64),            # blocks of 64 decoded in pairs
    ((11, 20, 130), np.float32, (1e-3, 1e-2, 1e-3), 64),
]


def case_id(c):
    shape, dt, rels, S = c
    return f"{'x'.join(map(str, shape))}-{np.dtype(dt).name}-S{S}"


@pytest.fixture(scope="module", params=CASES, ids=[case_id(c) for c in CASES])
def vcase(request):
    shape, dt, rels, S = request.param
    say(f"[case] vector {case_id(request.param)}")
    comps, ints, stored = [], [], []
    for k, rel in enumerate(rels):
        f = synth.gaussian_mixture(shape, 5, (2.0, max(3.0, min(shape) / 3.0)), seed=31 * k + sum(shape))
        x = np.ascontiguousarray(f.astype(dt))
        ref = oracle.compress(x, rel, rel=True, block=S)
        c = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S)
        assert np.array_equal(c.to_bytes(), ref)
        h = oracle.read_header(ref)
        q = oracle.decompress(ref, oracle.QUANT)
        comps.append(c)
        ints.append(oracle.dequantize64(q, h.quantum))
        stored.append(oracle.decompress(ref, oracle.FLOAT).astype(np.float64))
    return dict(shape=shape, f32=dt == np.float32, comps=comps, ints=ints, stored=stored)


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


def _tol(want, base, f32, route):
    m = max(float(np.max(np.abs(b))) for b in base)
    rel = 1e-6 if f32 else 1e-12
    unit = 2.0 ** -53 if (route == "int" or not f32) else 2.0 ** -24
    return rel * np.abs(want) + 16 * unit * m


def _as_list(r):
    return list(r) if isinstance(r, tuple) else [r]


@pytest.mark.parametrize("op", ["divergence", "curl"])
def test_vector_ops_all_routes(vcase, op):
    shape, comps = vcase["shape"], vcase["comps"]
    nd = len(shape)
    if op == "curl" and nd < 2:
        with pytest.raises(hsz.HszError) as e:
            hsz.vector_op_fused(comps, op)
        assert e.value.code == hsz.ERR_INVALID_ARG
        return
    headers = [c.header for c in comps]
    qbufs = [hsz.decompress_to_stage(c, hsz.QUANT) for c in comps]
    fbufs = [hsz.decompress_to_stage(c, hsz.FLOAT) for c in comps]
    ofn = oracle.divergence if op == "divergence" else oracle.curl
    for box in _boxes(shape, seed=nd * 5 + len(comps)):
        for route, base, runs in (
                ("int", vcase["ints"], (lambda: hsz.vector_op_fused(comps, op, box=box),
                                        lambda: hsz.vector_op_on_stage(qbufs, headers, hsz.QUANT, op, box=box))),
                ("float", vcase["stored"], (lambda: hsz.vector_op_on_stage(fbufs, headers, hsz.FLOAT, op,
                                                                          box=box),))):
            want = ofn(base, box)
            wants = list(want) if (op == "curl" and nd == 3) else [want]
            results = []
            for run in runs:
                got = [g.cpu().numpy().astype(np.float64) for g in _as_list(run())]
                assert len(got) == len(wants)
                for g, w in zip(got, wants):
                    assert g.shape == w.shape
                    err = np.abs(g - w)
                    bad = err > _tol(w, base, vcase["f32"], route)
                    assert not bad.any(), (op, route, box, int(bad.sum()), float(err.max()))
                results.append(got)
            if route == "int":
                for a, b in zip(results[0], results[1]):
                    assert np.array_equal(a, b)  # fused and stage route: same terms, same order


def test_vector_ops_refuse_bad_requests(vcase):
    comps = vcase["comps"]
    headers = [c.header for c in comps]
    with pytest.raises(hsz.HszError) as e:
        hsz.vector_op_fused(comps, "divergence", via=hsz.FLOAT)
    assert e.value.code == hsz.ERR_UNSUPPORTED
    pbufs = [hsz.decompress_to_stage(c, hsz.DELTA)[0] for c in comps]
    with pytest.raises(hsz.HszError) as e:
        hsz.vector_op_on_stage(pbufs, headers, hsz.DELTA, "divergence")
    assert e.value.code == hsz.ERR_UNSUPPORTED
    if len(comps) > 1:
        with pytest.raises(hsz.HszError) as e:  # one component short of the field's dims
            hsz.vector_op_fused(comps[:-1], "divergence")
        assert e.value.code == hsz.ERR_INVALID_ARG
