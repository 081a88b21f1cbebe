"""Pins for the oracle's block-mean decorrelation (HSZx, Sec. IV) and the mean
from its metadata (Sec. V-A, Eq. (mean_m)).

The worked example of Sec. IV prints, for the 2x2 blocks of Y_q, the integer
block means M = (5, -1) and the decorrelated data Y_p; the 1D encoder applied
to each printed block's four values (gathered in block order) must reproduce
both.  The rounding rule of the block mean is pinned against exact rational
arithmetic (fractions.Fraction) by brute force, the metadata mean against the
paper's mu~ = 2 and the bias bound of the error analysis (|mu_M - mu_f| <=
eps), and the decoder by round trips.
"""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def _golden():
    g = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        g[k] = [float(t) for t in v]
    return g


def _round_half_down(fr: Fraction) -> int:
    """Nearest integer, halves going down: the largest m with m - 1/2 < fr <= m + 1/2."""
    m = math.floor(fr)
    return m + 1 if fr - m > Fraction(1, 2) else m


def test_block_mean_worked_example():
    g = _golden()
    yq = np.array(g["Yq"], dtype=np.int32).reshape(2, 4)
    # the two 2x2 blocks of Y_q, each read row by row, one after the other
    blocks = np.concatenate([yq[:, 0:2].ravel(), yq[:, 2:4].ravel()])
    buf = oracle.encode_q(blocks, (8,), quantum=0.2, block=4, eb_abs=0.1, mean_dec=True)
    assert oracle.read_header(buf).flags == 1
    meta = oracle.decompress(buf, oracle.META)
    assert list(meta) == [int(v) for v in g["M"]]  # printed M_1 = 5, M_2 = -1
    p, _ = oracle.decompress(buf, oracle.DELTA)
    yp = np.array(g["Yp"], dtype=np.int32).reshape(2, 4)
    want_p = np.concatenate([yp[:, 0:2].ravel(), yp[:, 2:4].ravel()])
    assert np.array_equal(p, want_p)  # printed Y_p
    assert np.array_equal(oracle.decompress(buf, oracle.QUANT), blocks)
    # Eq. (mean_m): (5*4 + (-1)*4) / 8 * 0.2 = 0.4; the paper's mu~ = round(16 / 8) = 2
    msum, mean = oracle.meta_mean(buf)
    assert msum == 16 and mean == pytest.approx(0.4, abs=1e-15)
    assert msum // 8 == 2
    exact = float(blocks.sum()) / 8 * 0.2  # 18 / 8 * 0.2 = 0.45
    assert abs(mean - exact) <= 0.1  # the bias bound of the metadata mean: eps


@pytest.mark.parametrize("S", [1, 2, 3, 4])
def test_block_mean_brute_force(S):
    """Every integer vector in [-3, 3]^S: the metadata is the block mean
    rounded half down (exact rationals), |mean - M| <= 1/2, p = q - M, and
    the decoder returns q."""
    for vals in itertools.product(range(-3, 4), repeat=S):
        q = np.array(vals, dtype=np.int32)
        buf = oracle.encode_q(q, (S,), quantum=1.0, block=S, mean_dec=True)
        m = int(oracle.decompress(buf, oracle.META)[0])
        fr = Fraction(int(q.sum()), S)
        assert m == _round_half_down(fr), (vals, m)
        assert abs(fr - m) <= Fraction(1, 2)
        p, _ = oracle.decompress(buf, oracle.DELTA)
        assert np.array_equal(p, q - m)
        assert np.array_equal(oracle.decompress(buf, oracle.QUANT), q)


def test_halves_round_down():
    for q, m in (([1, 2], 1), ([-1, -2], -2), ([5, 6], 5), ([-5, -6], -6), ([0, 0, 1], 0), ([1, 1, 0], 1)):
        buf = oracle.encode_q(np.array(q, dtype=np.int32), (len(q),), 1.0, block=len(q), mean_dec=True)
        assert int(oracle.decompress(buf, oracle.META)[0]) == m


@pytest.mark.parametrize("shape,S,rel", [((5, 7, 33), 32, 1e-3), ((1000,), 64, 1e-4), ((3, 5, 7), 32, 1e-2)])
def test_metadata_mean_bias_and_round_trip(shape, S, rel):
    """Random fields (ragged last block included): decode in the block-mean
    mode returns the same quantization integers as the delta mode, and the
    metadata mean is within eps of the mean of the decompressed field."""
    rng = np.random.default_rng(sum(shape) + S)
    x = (rng.normal(size=shape) * 3 + 1).astype(np.float32)
    a = oracle.compress(x, rel, rel=True, block=S)
    b = oracle.compress(x, rel, rel=True, block=S, mean_dec=True)
    ha, hb = oracle.read_header(a), oracle.read_header(b)
    assert hb.flags == 1 and hb.quantum == ha.quantum and hb.max_abs_q == ha.max_abs_q
    q = oracle.decompress(b, oracle.QUANT)
    assert np.array_equal(q, oracle.decompress(a, oracle.QUANT))
    xh = oracle.decompress(b, oracle.FLOAT).astype(np.float64)
    assert np.all(np.abs(xh - x.astype(np.float64)) <= hb.eb_abs)
    msum, mean = oracle.meta_mean(b)
    qq = q.ravel().astype(np.int64)
    want = 0
    for k in range(hb.nb):
        blk = qq[k * S:(k + 1) * S]
        want += _round_half_down(Fraction(int(blk.sum()), len(blk))) * len(blk)
    assert msum == want
    exact = oracle.mean(oracle.dequantize64(q, hb.quantum))
    assert abs(mean - exact) <= hb.eb_abs


def test_rejects_unknown_flags_and_meta_mean_of_delta_streams():
    x = np.linspace(0, 1, 100).astype(np.float32)
    buf = oracle.compress(x, 1e-3)
    with pytest.raises(oracle.OracleError) as e:
        oracle.meta_mean(buf)
    assert e.value.code == oracle.ERR_UNSUPPORTED
    bad = buf.copy()
    bad[92] = 2  # flags: only bit 0 is defined
    with pytest.raises(oracle.OracleError) as e:
        oracle.read_header(bad)
    assert e.value.code == oracle.ERR_STREAM


# ---- standard deviation on D_p about the integer metadata mean (Sec. V-A) ----------------

def test_std_about_metadata_mean_worked_example():
    """Sec. V-A continues the example of Sec. IV: mu~ = round((5*4 + (-1)*4) / 8)
    = 2 and sigma = 2.000 on Y_p (the exact sample deviation would be 1.9993)."""
    g = _golden()
    yq = np.array(g["Yq"], dtype=np.int32).reshape(2, 4)
    blocks = np.concatenate([yq[:, 0:2].ravel(), yq[:, 2:4].ravel()])
    buf = oracle.encode_q(blocks, (8,), quantum=0.2, block=4, eb_abs=0.1, mean_dec=True)
    r = oracle.var_mt(buf)
    assert (r["n"], r["msum"], r["mu_t"]) == (8, 16, 2)
    assert r["s2"] == sum((int(v) - 2) ** 2 for v in blocks) == 700
    assert round(math.sqrt(r["var"]), 3) == g["sigma_hszx_p"][0]
    assert math.sqrt(r["var"]) == pytest.approx(2.0, rel=1e-15)
    exact = float(np.std(blocks.astype(np.float64), ddof=1)) * 0.2
    assert round(exact, 3) != g["sigma_hszx_p"][0]  # the printed value is the mu~ form


@pytest.mark.parametrize("S,N", [(1, 4), (2, 5), (3, 4), (4, 6)])
def test_std_about_metadata_mean_brute_force(S, N):
    """Every integer vector in [-2, 2]^N (ragged last block when S does not
    divide N): mu~ is the rounded (halves down) mean of the block means
    weighted by their sizes, and the sum is of (q - mu~)^2 taken straight
    from q, with exact rationals."""
    for vals in itertools.product(range(-2, 3), repeat=N):
        q = np.array(vals, dtype=np.int32)
        buf = oracle.encode_q(q, (N,), quantum=1.0, block=S, mean_dec=True)
        r = oracle.var_mt(buf)
        ms = 0
        for b in range(0, N, S):
            blk = vals[b:b + S]
            ms += _round_half_down(Fraction(sum(blk), len(blk))) * len(blk)
        mt = _round_half_down(Fraction(ms, N))
        want = sum((v - mt) ** 2 for v in vals)
        assert (r["msum"], r["mu_t"], r["s2"]) == (ms, mt, want), vals
        assert r["var"] == pytest.approx(want / (N - 1), rel=1e-15, abs=0)


@pytest.mark.parametrize("shape,S,rel", [((7, 9, 35), 32, 1e-3), ((3001,), 64, 1e-5), ((1,), 32, 1e-3)])
def test_std_about_metadata_mean_shift_identity(shape, S, rel):
    """Sum (q - mu~)^2 = sum (q - mu)^2 + N (mu - mu~)^2 exactly (mu = the exact
    mean of q): the spread about mu~ exceeds the sample variance by the
    squared shift only, and |mu - mu~| <= 1 (each rounding moves by at most
    one half)."""
    rng = np.random.default_rng(sum(shape) * S)
    x = (rng.normal(size=shape) * 2 - 5).astype(np.float32)
    buf = oracle.compress(x, rel, rel=True, block=S, mean_dec=True)
    h = oracle.read_header(buf)
    q = [int(v) for v in oracle.decompress(buf, oracle.QUANT).ravel()]
    r = oracle.var_mt(buf)
    n = len(q)
    mu = Fraction(sum(q), n)
    assert abs(mu - r["mu_t"]) <= 1
    assert r["msum"] == oracle.meta_mean(buf)[0]
    assert Fraction(r["s2"]) == sum((Fraction(v) - mu) ** 2 for v in q) + n * (mu - r["mu_t"]) ** 2
    if n > 1:
        assert r["var"] == pytest.approx(r["s2"] / (n - 1) * h.quantum ** 2, rel=1e-15)
    else:
        assert math.isnan(r["var"])


def test_std_about_metadata_mean_constant_field_and_delta_streams():
    x = np.full((5, 70), 3.25, dtype=np.float32)
    r = oracle.var_mt(oracle.compress(x, 1e-3, block=32, mean_dec=True))
    assert r["s2"] == 0 and r["var"] == 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.var_mt(oracle.compress(x, 1e-3, block=32))
    assert e.value.code == oracle.ERR_UNSUPPORTED
