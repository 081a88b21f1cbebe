"""Pins for the CPU oracle: checks against what the paper and mathematics fix,
never against the oracle itself.  No GPU needed.

Pins used:
  * the paper's worked example (Sec. IV, HSZx-nd paragraph): Y, eps = 0.1
    and the printed Y_q (tests/golden/worked_example.txt);
  * quantities derived by hand from that example with the SZp rules
    (metadata = first q of a block, p_i = q_i - q_{i-1}), and the bytes
    they encode to, derived by hand from the format rules;
  * a second reading of the byte format (tests/format_ref.py);
  * brute force over every small integer vector;
  * library routines the operations reduce to (math.fsum, numpy.var with
    ddof=1, numpy.gradient) and exact Python integers;
  * the error bound |d - d'| <= eps of Sec. III-A on adversarial inputs.
"""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import format_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = [float(v) for v in rest]
    return vals


# ---------------------------------------------------------------- quantizer

def test_quantizer_reproduces_paper_worked_example():
    g = _golden()
    y = np.array(g["Y"])
    yq = np.array(g["Yq"], dtype=np.int32)
    quantum = 2 * g["eb"][0]
    assert list(oracle.quantize(y, quantum)) == list(yq)
    # the same from binary32 inputs
    assert list(oracle.quantize(y.astype(np.float32).astype(np.float64), quantum)) == list(yq)


def test_other_tie_rules_do_not_reproduce_the_example():
    """The example discriminates the rounding rule: half-to-even (numpy.rint)
    and half-away-from-zero both miss at least one printed integer, so a
    quantizer with either rule fails the test above."""
    g = _golden()
    y = np.array(g["Y"])
    yq = np.array(g["Yq"])
    t = y / (2 * g["eb"][0])
    assert not np.array_equal(np.rint(t), yq)
    assert not np.array_equal(np.sign(t) * np.floor(np.abs(t) + 0.5), yq)


def test_quantizer_large_values_and_ties():
    quantum = 0.25
    x = np.array([0.125, -0.125, 0.375, -0.375, 1e3, -1e3, 0.0, -0.0])
    # ties go up: 0.5 -> 1, -0.5 -> 0, 1.5 -> 2, -1.5 -> -1
    assert list(oracle.quantize(x, quantum)) == [1, 0, 2, -1, 4000, -4000, 0, 0]


# ---------------------------------------------------- decorrelate + encode

# Hand derivation from the worked example with blocks of S = 4 over the
# row-major flat array:
#   block 0: q = 6 8 -11 -12 -> q0 = 6,  p = 0 2 -19 -1,  max|p| = 19 -> w = 5
#   block 1: q = 13 -5 10 9  -> q0 = 13, p = 0 -18 15 -1, max|p| = 18 -> w = 5
#   sign words: block 0 slots 2,3 negative -> 0b1100 = 12;
#               block 1 slots 1,3 negative -> 0b1010 = 10
#   magnitude words (5 bits each, least significant first):
#     block 0: 0 | 2<<5 | 19<<10 | 1<<15 = 52288
#     block 1: 0 | 18<<5 | 15<<10 | 1<<15 = 48704
WORKED_P = [0, 2, -19, -1, 0, -18, 15, -1]
WORKED_Q0 = [6, 13]
WORKED_WIDTH = [5, 5]
WORKED_PAYLOAD = [12, 52288, 10, 48704]


def test_encode_worked_example():
    g = _golden()
    yq = np.array(g["Yq"], dtype=np.int32)
    buf = oracle.encode_q(yq, (2, 4), quantum=0.2, block=4, eb_abs=0.1)
    h = oracle.read_header(buf)
    assert (h.n, h.block, h.nb, h.nchunks, h.dims) == (8, 4, 2, 1, (2, 4))
    assert h.max_abs_q == 13
    p, q0 = oracle.decompress(buf, oracle.DELTA)
    assert list(p.ravel()) == WORKED_P
    assert list(q0) == WORKED_Q0
    assert list(oracle.decompress(buf, oracle.META)) == WORKED_Q0
    assert list(oracle.decompress(buf, oracle.QUANT).ravel()) == list(yq)
    x32 = oracle.decompress(buf, oracle.FLOAT)
    assert x32.dtype == np.float32
    assert list(x32.ravel()) == [np.float32(v * 0.2) for v in yq]
    ref = format_ref.parse(buf.tobytes())
    assert ref["width"] == WORKED_WIDTH
    assert ref["payload"] == WORKED_PAYLOAD
    assert ref["q0"] == WORKED_Q0


# ------------------------------------------------------------- operations

def test_stats_on_worked_example():
    """Hand-derived from Y_q: sum q = 18, sum q^2 = 740, so with the quantum
    0.2 the mean is 18*0.2/8 = 0.45 and the sample variance is
    (8*740 - 18^2)/(8*7) * 0.04 = 3.99714285714...  The paper's HSZx route
    prints sigma = 2.000 for the same field (Sec. V-A); the SZp route is
    exact on D_q, so it may differ from that by at most eps = 0.1 (the bias
    bound of Sec. V-D for the block-mean route)."""
    g = _golden()
    yq = np.array(g["Yq"], dtype=np.int32).reshape(2, 4)
    assert oracle.int_sums(yq) == (8, 18, 740)
    xh = oracle.dequantize64(yq, 0.2)
    assert oracle.mean(xh) == pytest.approx(0.45, rel=1e-15)
    v = oracle.var(xh)
    assert v == pytest.approx((8 * 740 - 18 ** 2) / (8 * 7) * 0.04, rel=1e-14)
    assert v == pytest.approx(np.var(xh, ddof=1), rel=1e-14)
    assert abs(math.sqrt(v) - g["sigma_hszx_p"][0]) <= g["eb"][0]


def test_gradient_on_worked_example():
    """Row 0 of d' = 0.2*Y_q is 1.2 1.6 -2.2 -2.4; along the fast axis the
    derivative is 0.4, -1.7, -2.0, -0.2 (one-sided at the ends)."""
    g = _golden()
    yq = np.array(g["Yq"], dtype=np.int32).reshape(2, 4)
    xh = oracle.dequantize64(yq, 0.2)
    d1 = oracle.derivative(xh, axis=1)
    np.testing.assert_allclose(d1[0], [0.4, -1.7, -2.0, -0.2], rtol=0, atol=1e-14)
    d0 = oracle.derivative(xh, axis=0)  # length-2 axis: one-sided everywhere
    np.testing.assert_allclose(d0[0], xh[1] - xh[0], rtol=0, atol=0)


# ----------------------------------------------------- brute force: codec

@pytest.mark.parametrize("S", [1, 2, 3, 4, 5])
def test_brute_force_all_small_vectors(S):
    """Every q vector in [-3, 3]^S, one vector per block, plus a ragged tail."""
    vecs = np.array(list(itertools.product(range(-3, 4), repeat=S)), dtype=np.int32)
    tail = np.array([2, -3, 1][: max(1, S - 1)], dtype=np.int32) if S > 1 else np.zeros(0, np.int32)
    q = np.concatenate([vecs.ravel(), tail])
    buf = oracle.encode_q(q, (q.size,), quantum=1.0, block=S)
    got_q = oracle.decompress(buf, oracle.QUANT)
    assert np.array_equal(got_q, q)
    p, q0 = oracle.decompress(buf, oracle.DELTA)
    nb = -(-q.size // S)
    assert np.array_equal(q0, q[::S])
    exp_p = np.zeros(q.size, dtype=np.int64)
    for b in range(nb):
        blk = q[b * S:(b + 1) * S].astype(np.int64)
        exp_p[b * S + 1:b * S + blk.size] = np.diff(blk)
    assert np.array_equal(p, exp_p)
    ref = format_ref.parse(buf.tobytes())
    assert np.array_equal(ref["q"], q)
    for b in range(nb):
        mx = int(np.abs(exp_p[b * S:(b + 1) * S]).max())
        assert ref["width"][b] == mx.bit_length()


@pytest.mark.parametrize("S", [32, 64, 7])
def test_codec_random_wide_values(S):
    rng = np.random.default_rng(11)
    q = np.cumsum(rng.integers(-2 ** 20, 2 ** 20, size=5 * 64 * S + 13)).astype(np.int64)
    q = np.clip(q, -(2 ** 29 - 1), 2 ** 29 - 1).astype(np.int32)
    q[: 64 * S] = 5  # a run of constant blocks (w = 0)
    buf = oracle.encode_q(q, (q.size,), quantum=1.0, block=S)
    ref = format_ref.parse(buf.tobytes())
    assert np.array_equal(ref["q"], q)
    assert np.array_equal(oracle.decompress(buf, oracle.QUANT), q)
    assert all(w == 0 for w in ref["width"][:64])
    h = oracle.read_header(buf)
    assert h.max_abs_q == int(np.abs(q.astype(np.int64)).max())


# --------------------------------------- closed forms of the stage data

def test_block_sum_and_delta_derivative_closed_forms():
    """Sec. V-A (mean on D_p): inside a block q_i is q0 plus the prefix sum of
    p, so sum_{i<S_b} q_i = S_b*q0 + sum_{i>=1} (S_b - i) p_i; and the
    central difference inside a block is q_{i+1} - q_{i-1} = p_i + p_{i+1}."""
    rng = np.random.default_rng(3)
    x = np.cumsum(rng.normal(size=10 * 32 + 9)).astype(np.float32)
    buf = oracle.compress(x, 1e-3, rel=True, block=32)
    p, q0 = oracle.decompress(buf, oracle.DELTA)
    q = oracle.decompress(buf, oracle.QUANT).astype(np.int64)
    S = 32
    for b in range(q0.size):
        blk = q[b * S:(b + 1) * S]
        pb = p[b * S:(b + 1) * S].astype(np.int64)
        sb = blk.size
        assert blk.sum() == sb * int(q0[b]) + sum((sb - i) * int(pb[i]) for i in range(1, sb))
        for i in range(1, sb - 1):
            assert blk[i + 1] - blk[i - 1] == pb[i] + pb[i + 1]


# ------------------------------------------------ operations vs libraries

@pytest.mark.parametrize("shape", [(9,), (6, 7), (5, 6, 7), (1, 4, 5), (3, 1, 6)])
def test_ops_match_numpy(shape):
    rng = np.random.default_rng(5)
    x = rng.normal(size=shape) * 3 + 1
    assert oracle.mean(x) == pytest.approx(math.fsum(x.ravel()) / x.size, rel=1e-15)
    assert oracle.var(x) == pytest.approx(np.var(x, ddof=1), rel=1e-13)
    gs = []
    for a in range(x.ndim):
        g = np.gradient(x, axis=a) if shape[a] > 1 else np.zeros(shape)
        gs.append(g)
        np.testing.assert_array_equal(oracle.derivative(x, a), g)
    np.testing.assert_allclose(oracle.gradmag(x), np.sqrt(sum(g * g for g in gs)), rtol=1e-15, atol=0)
    # sub-box: statistics of the box, gradient = restriction of the full gradient
    lo = tuple(s // 3 for s in shape)
    hi = tuple(max(l + 1, s - s // 4) for l, s in zip(lo, shape))
    sl = tuple(slice(l, h) for l, h in zip(lo, hi))
    sub = x[sl]
    assert oracle.mean(x, (lo, hi)) == pytest.approx(math.fsum(sub.ravel()) / sub.size, rel=1e-15)
    if sub.size > 1:
        assert oracle.var(x, (lo, hi)) == pytest.approx(np.var(sub, ddof=1), rel=1e-13)
    for a in range(x.ndim):
        np.testing.assert_array_equal(oracle.derivative(x, a, (lo, hi)), gs[a][sl])
    np.testing.assert_allclose(oracle.gradmag(x, (lo, hi)), np.sqrt(sum(g * g for g in gs))[sl],
                               rtol=1e-15, atol=0)


def test_int_sums_exact():
    rng = np.random.default_rng(8)
    q = rng.integers(-(2 ** 29 - 1), 2 ** 29, size=(4, 5, 33)).astype(np.int32)
    n, s1, s2 = oracle.int_sums(q)
    vals = [int(v) for v in q.ravel()]
    assert (n, s1, s2) == (len(vals), sum(vals), sum(v * v for v in vals))
    box = ((1, 2, 3), (3, 5, 30))
    sub = [int(v) for v in q[1:3, 2:5, 3:30].ravel()]
    assert oracle.int_sums(q, box) == (len(sub), sum(sub), sum(v * v for v in sub))


# ----------------------------------------------------------- error bound

def _exact_abs_err_ok(x, xh, eps):
    """|x - x'| <= eps decided exactly (binary64 inputs via Fractions)."""
    if x.dtype == np.float32:
        return np.all(np.abs(x.astype(np.float64) - xh.astype(np.float64)) <= eps)
    fe = Fraction(eps)
    return all(abs(Fraction(float(a)) - Fraction(float(b))) <= fe for a, b in zip(x, xh))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("rel", [1e-2, 1e-4, 1e-6])
def test_error_bound_adversarial(dtype, rel):
    """Values placed exactly on, and one ulp either side of, the quantizer's
    rounding ties, plus zeros, subnormals and the extremes.  Every
    decompressed value must lie within eps of its input (Sec. III-A)."""
    anchors = np.array([-3.0, 5.0])
    eps, quantum = oracle.quant_params(-3.0, 5.0, rel, True, 1 if dtype == np.float32 else 2)
    assert eps == rel * 8.0 and quantum < 2 * eps
    ks = np.concatenate([np.arange(-40, 40), np.arange(-40, 40) + int(2.9 / quantum) - 40])
    ties = ((ks + 0.5) * quantum).astype(dtype)
    ties = ties[(ties > -3) & (ties < 5)]
    up = np.nextafter(ties, dtype(np.inf))
    dn = np.nextafter(ties, dtype(-np.inf))
    special = np.array([0.0, -0.0, np.finfo(dtype).tiny, -np.finfo(dtype).tiny, 4.999999, -2.999999],
                       dtype=dtype)
    x = np.concatenate([anchors.astype(dtype), ties, up, dn, special]).astype(dtype)
    buf = oracle.compress(x, rel, rel=True, block=32)
    h = oracle.read_header(buf)
    assert h.eb_abs == eps and h.quantum == quantum
    xh = oracle.decompress(buf, oracle.FLOAT)
    assert xh.dtype == dtype
    assert _exact_abs_err_ok(x, xh, eps)


# Hand-derived quanta (Sec. III-A bound, reading R3: Delta = 2 (eps - m ulp(max|x| + eps)),
# m = 1 for binary32, 8 for binary64).  Each ulp is fixed by the binade of
# max|x| + eps, worked out by hand: [4, 8) has binary32 spacing 2^-21 and
# binary64 spacing 2^-50; [2, 4) has 2^-22 and 2^-51.  A margin off by a
# binade, a wrong multiplier m, or max|x| taken from the wrong end of the
# range changes Delta and fails one of these.
QUANTUM_PINS = [
    # (vmin, vmax, rel, dtype, eps, ulp multiple subtracted from eps)
    (-3.0, 5.0, 1e-4, 1, 8.0 * 1e-4, 2.0 ** -21),            # 5.0008 in [4, 8)
    (-3.0, 5.0, 1e-4, 2, 8.0 * 1e-4, 8 * 2.0 ** -50),        # binary64: m = 8
    (-3.0, 3.99, 1e-4, 1, 6.99 * 1e-4, 2.0 ** -22),          # 3.990699 in [2, 4)
    (-3.0, 3.9999, 1e-4, 1, 6.9999 * 1e-4, 2.0 ** -21),      # 4.00059999 crosses into [4, 8)
    (-6.0, 1.0, 1e-3, 1, 7.0 * 1e-3, 2.0 ** -21),            # max|x| is |vmin| = 6: 6.007 in [4, 8)
    (-6.0, 1.0, 1e-3, 2, 7.0 * 1e-3, 8 * 2.0 ** -50),
]


@pytest.mark.parametrize("vmin,vmax,rel,dtype,eps_want,margin", QUANTUM_PINS)
def test_quantum_exact_hand_derived(vmin, vmax, rel, dtype, eps_want, margin):
    eps, quantum = oracle.quant_params(vmin, vmax, rel, True, dtype)
    # eps = rel (max - min) in binary64: the range is an exact small number,
    # so only the product with rel rounds
    assert eps == rel * (vmax - vmin)
    assert eps == pytest.approx(eps_want, rel=1e-15)
    assert quantum == 2.0 * (eps - margin)


def test_signed_zero_extremes_are_canonical():
    """A field whose extreme is zero stores +0.0 whichever zero the scan met
    first, so the header bytes do not depend on the order of -0.0 / +0.0."""
    a = np.array([-0.0, 0.0, 1.0, 2.0] * 8, dtype=np.float32)
    b = np.array([0.0, -0.0, 1.0, 2.0] * 8, dtype=np.float32)
    ba, bb = oracle.compress(a, 1e-3), oracle.compress(b, 1e-3)
    ha = oracle.read_header(ba)
    assert ha.vmin == 0.0 and np.signbit(ha.vmin) == False  # noqa: E712
    assert np.array_equal(ba, bb)


def test_margin_is_needed_for_binary32_ties():
    """Without the margin (quantum exactly 2*eps) rounding the decompressed
    value to binary32 breaks the bound on tie inputs: the reading that
    shrinks the quantum is load-bearing, not decoration."""
    eps = 1e-4 * 8.0
    quantum = 2 * eps
    ks = np.arange(1000, 3000)
    x = ((ks + 0.5) * quantum).astype(np.float32).astype(np.float64)
    q = oracle.quantize(x, quantum)
    xh = (q.astype(np.float64) * quantum).astype(np.float32).astype(np.float64)
    assert np.any(np.abs(x - xh) > eps)


@pytest.mark.parametrize("dtype,rel", [(np.float32, 1e-3), (np.float32, 1e-4), (np.float64, 1e-6)])
def test_round_trip_smooth_field(dtype, rel):
    from paper_2603_25206_amd import synth
    x = synth.gaussian_mixture((20, 24, 40), 6, (3.0, 9.0), seed=1).astype(dtype)
    for S in (32, 64):
        buf = oracle.compress(x, rel, rel=True, block=S)
        h = oracle.read_header(buf)
        xh = oracle.decompress(buf, oracle.FLOAT)
        assert _exact_abs_err_ok(x.ravel(), xh.ravel(), h.eb_abs)
        q = oracle.decompress(buf, oracle.QUANT)
        assert np.array_equal(q.ravel(), oracle.quantize(x.ravel().astype(np.float64), h.quantum))
        ref = format_ref.parse(buf.tobytes())
        assert np.array_equal(ref["q"], q.ravel())
        assert h.total_bytes == buf.size < x.nbytes


def test_constant_and_zero_fields():
    x = np.full((3, 40), 2.5, dtype=np.float32)
    buf = oracle.compress(x, 1e-3, rel=True, block=32)
    h = oracle.read_header(buf)
    assert h.eb_abs == 1e-3 * 2.5
    assert _exact_abs_err_ok(x.ravel(), oracle.decompress(buf, oracle.FLOAT).ravel(), h.eb_abs)
    assert h.payload_words == 0  # every block has p = 0
    z = np.zeros(100, dtype=np.float64)
    buf = oracle.compress(z, 1e-3, rel=True, block=32)
    h = oracle.read_header(buf)
    assert h.eb_abs == 1e-3
    assert np.all(oracle.decompress(buf, oracle.FLOAT) == 0)


# ----------------------------------------------------------------- errors

def test_rejects_bad_inputs():
    x = np.linspace(0, 1, 100).astype(np.float32)
    bad = x.copy()
    bad[7] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(bad, 1e-3)
    assert e.value.code == oracle.ERR_NONFINITE
    bad[7] = np.inf
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(bad, 1e-3)
    assert e.value.code == oracle.ERR_NONFINITE
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(x, 0.0)
    assert e.value.code == oracle.ERR_EB
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(x, 1e-12)  # eps is below binary32 spacing: no quantum left
    assert e.value.code == oracle.ERR_EB
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(x.astype(np.float64), 1e-12)  # |q| would reach 5e11 > 2^29 - 1
    assert e.value.code == oracle.ERR_RANGE


def test_rejects_corrupt_streams():
    x = np.sin(np.linspace(0, 20, 5000)).astype(np.float32)
    buf = oracle.compress(x, 1e-3)
    h = oracle.read_header(buf)
    bad = buf.copy()
    bad[0] = ord("X")
    with pytest.raises(oracle.OracleError):
        oracle.read_header(bad)
    with pytest.raises(oracle.OracleError):
        oracle.decompress(buf[:-4], oracle.QUANT)
    bad = buf.copy()
    bad[h.off_width + 3] = 31
    with pytest.raises(oracle.OracleError) as e:
        oracle.decompress(bad, oracle.QUANT)
    assert e.value.code == oracle.ERR_STREAM
    bad = buf.copy()
    bad[h.off_chunk + 8] ^= 1  # second chunk's offset
    with pytest.raises(oracle.OracleError) as e:
        oracle.decompress(bad, oracle.QUANT)
    assert e.value.code == oracle.ERR_STREAM
