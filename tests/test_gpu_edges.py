"""Degenerate inputs on the GPU against the oracle: constant and all-zero
fields, a single element, length-1 axes (including a length-1 fast axis,
where every block spans many rows), and a field whose max|q| comes close to
the 2^29 - 1 limit (widths near 30 bits, the general accumulators and the
binary64 squared sums).  Empty input is rejected before any launch."""
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


def run_all(x, rel, S):
    """Bytes, every stage, the integer-route statistics and gradients (fused,
    and in a batch with shared statistics) against the oracle."""
    ref = oracle.compress(x, rel, rel=True, block=S)
    c = hsz.compress(torch.from_numpy(x).to(DEV), rel, rel=True, block=S)
    assert np.array_equal(c.data[: c.nbytes].cpu().numpy(), ref)
    h = oracle.read_header(ref)
    q = oracle.decompress(ref, oracle.QUANT)
    assert np.array_equal(hsz.decompress_to_stage(c, hsz.QUANT).cpu().numpy().reshape(x.shape), q)
    xh = oracle.dequantize64(q, h.quantum)
    n, s1, s2 = oracle.int_sums(q)
    f64 = x.dtype == np.float64
    for via in (hsz.DELTA, hsz.QUANT):
        st = hsz.op_fused(c, via, "var")
        assert (st["n"], st["s1"], st["s2"]) == (n, s1, s2)
    want = oracle.gradmag(xh)
    for got in (hsz.op_fused(c, hsz.QUANT, "gradmag"),
                hsz.batch_run([hsz.Job(c, "gradmag", hsz.QUANT), hsz.Job(c, "var", hsz.QUANT)])[0]):
        g = got.cpu().numpy().astype(np.float64).reshape(want.shape)
        tol = (1e-12 * np.abs(want) + 4 * 2.0 ** -53 * float(np.max(np.abs(xh)))) if f64 else 1e-6 * np.abs(want)
        assert np.all(np.abs(g - want) <= tol)
        assert np.all(g[want == 0] == 0)
    st = hsz.batch_run([hsz.Job(c, "gradmag", hsz.QUANT), hsz.Job(c, "var", hsz.QUANT)])[1]
    assert (st["n"], st["s1"], st["s2"]) == (n, s1, s2)
    for ax in range(x.ndim):
        got = hsz.op_fused(c, hsz.QUANT, "deriv", axis=ax).cpu().numpy().astype(np.float64)
        want = oracle.derivative(xh, ax)
        tol = (1e-12 * np.abs(want) + 4 * 2.0 ** -53 * float(np.max(np.abs(xh)))) if f64 else 1e-6 * np.abs(want)
        assert np.all(np.abs(got.reshape(want.shape) - want) <= tol), ax
    return c, st


@pytest.mark.parametrize("value", [0.0, 3.25, -7.5])
def test_constant_fields(value):
    say(f"[case] constant field {value}")
    x = np.full((20, 30, 70), value, dtype=np.float32)
    c, st = run_all(x, 1e-3, 32)
    assert st["var"] == 0.0
    assert torch.count_nonzero(hsz.op_fused(c, hsz.QUANT, "gradmag")) == 0


@pytest.mark.parametrize("shape", [(1,), (1, 1, 1), (2,), (1, 64, 64), (40, 1, 70), (33, 45, 1), (7, 1, 1),
                                   (300, 1), (1, 1000)])
def test_length_one_axes(shape):
    say(f"[case] shape {shape}")
    x = (synth.gaussian_mixture(shape, 4, (1.0, 8.0), seed=sum(shape)) + 0.1).astype(np.float32)
    run_all(x, 1e-3, 32)


def test_near_range_limit_f64():
    say("[case] max|q| near 2^29")
    x = synth.gaussian_mixture((24, 40, 96), 5, (2.0, 10.0), seed=5)
    x = np.ascontiguousarray(x)
    rel = 1.0e-9  # range / (2 eps) ~ 5e8 < 2^29 - 1
    ref = oracle.compress(x, rel, rel=True, block=64)
    h = oracle.read_header(ref)
    assert h.max_abs_q > 2 ** 27
    run_all(x, rel, 64)


def test_empty_input_rejected():
    with pytest.raises(hsz.HszError) as e:
        hsz.compress(torch.empty(0, dtype=torch.float32, device=DEV), 1e-3)
    assert e.value.code == hsz.ERR_INVALID_ARG
