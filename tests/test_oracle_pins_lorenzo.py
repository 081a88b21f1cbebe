"""Pins for the oracle's HSZp-nd mode (Sec. IV, multidimensional Lorenzo
decorrelation) and its operations on D_p (Sec. V-A mean with nd weights,
Alg. 4 standard deviation, Eq. (derivative_Dp)).

The paper prints no HSZp-nd example, so each function is pinned against
what the mathematics fixes: the Lorenzo residual is the mixed backward
difference of the zero-padded field (numpy.diff), its inverse the nd
cumulative sum (numpy.cumsum); the nd partition is re-derived with numpy
reshapes and read back with the independent format reader; the D_p mean,
Alg. 4 and the derivative recursion equal sum q, sum q^2 and
numpy.gradient of the decoded q, exactly in integers.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.format_ref import parse

SHAPES = [((5, 9, 13), 32), ((7, 4, 10), 64), ((33, 41), 32), ((9, 70), 64), ((1, 1, 5), 32), ((2, 3), 32),
          ((16, 8, 8), 64), ((3, 3, 3), 8), ((5, 6), 4)]


def _field(shape, seed):
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.linspace(0, 3, s) for s in shape], indexing="ij")
    f = sum(np.sin((k + 1) * g) for k, g in enumerate(grids)) + 0.05 * rng.normal(size=shape)
    return f.astype(np.float32)


def _residual(q):
    """Mixed backward difference with q = 0 before index 0 on every axis."""
    r = np.asarray(q, dtype=np.int64)
    for ax in range(r.ndim):
        r = np.diff(r, axis=ax, prepend=0)
    return r


def _block_shape(ndim, S):
    return {(2, 4): (2, 2), (2, 32): (4, 8), (2, 64): (8, 8), (3, 8): (2, 2, 2), (3, 32): (2, 4, 4),
            (3, 64): (4, 4, 4)}[(ndim, S)]


def _blocks_of(p, bs):
    """p in the nd partition: blocks in raster order, slots in raster order,
    zero outside the field (numpy reshapes, no loops)."""
    pad = [(0, (-s) % b) for s, b in zip(p.shape, bs)]
    pp = np.pad(p, pad)
    nbs = [s // b for s, b in zip(pp.shape, bs)]
    inter = []
    for nb_, b in zip(nbs, bs):
        inter += [nb_, b]
    v = pp.reshape(inter)
    nd = p.ndim
    v = v.transpose(list(range(0, 2 * nd, 2)) + list(range(1, 2 * nd, 2)))
    return v.reshape(int(np.prod(nbs)), int(np.prod(bs)))


@pytest.mark.parametrize("shape,S", SHAPES)
def test_residual_partition_and_inverse(shape, S):
    x = _field(shape, sum(shape))
    buf = oracle.compress(x, 1e-3, rel=True, block=S, lorenzo=True)
    h = oracle.read_header(buf)
    assert h.flags == 2 and h.off_width == h.off_q0  # no metadata section
    q_ref = oracle.decompress(oracle.compress(x, 1e-3, rel=True, block=32), oracle.QUANT)  # same quantizer
    p, q0 = oracle.decompress(buf, oracle.DELTA)
    assert q0.size == 0
    assert np.array_equal(p, _residual(q_ref))
    q = oracle.decompress(buf, oracle.QUANT)
    assert np.array_equal(q, q_ref)
    c = p.astype(np.int64)
    for ax in range(p.ndim):
        c = np.cumsum(c, axis=ax)
    assert np.array_equal(c, q_ref)
    bs = _block_shape(len(shape), S)
    want_blocks = _blocks_of(p.astype(np.int64), bs)
    fr = parse(buf.tobytes())
    assert fr["nb"] == want_blocks.shape[0] == h.nb
    assert np.array_equal(fr["pblocks"], want_blocks)
    widths = [int(np.max(np.abs(b))).bit_length() for b in want_blocks]
    assert fr["width"] == widths


def test_block_shapes_of_the_device_sizes():
    """S = 32 / 64: 4x8 and 8x8 in 2D, 2x4x4 and 4x4x4 in 3D (read back from
    where a single nonzero residual lands)."""
    for shape, S, bs in (((8, 16), 32, (4, 8)), ((16, 16), 64, (8, 8)), ((4, 8, 8), 32, (2, 4, 4)),
                         ((8, 8, 8), 64, (4, 4, 4))):
        q = np.zeros(shape, dtype=np.int64)
        last = tuple(b - 1 for b in bs)  # the last slot of block 0
        q[last] = 1
        buf = oracle.encode_q(q.cumsum(0).cumsum(1) if len(shape) == 2 else q.cumsum(0).cumsum(1).cumsum(2),
                              shape, 1.0, S, lorenzo=True)
        fr = parse(buf.tobytes())
        nz = np.argwhere(fr["pblocks"] != 0)
        assert nz.tolist() == [[0, S - 1]], (shape, S)


def test_range_limit_on_the_residual():
    """|q| <= 2^29 - 1 but a 3D checkerboard makes |p| = 8 (2^29 - 1) > 2^30 - 1."""
    m = (1 << 29) - 1
    idx = np.indices((2, 2, 2)).sum(axis=0)
    q = np.where(idx % 2 == 0, m, -m).astype(np.int32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.encode_q(q, q.shape, 1.0, 8, lorenzo=True)
    assert e.value.code == oracle.ERR_RANGE
    small = np.where(idx % 2 == 0, 1 << 26, -(1 << 26)).astype(np.int32)
    oracle.encode_q(small, small.shape, 1.0, 8, lorenzo=True)  # 8 * 2^26 = 2^29 fits


def test_invalid_requests():
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress(np.ones(100, dtype=np.float32), 1e-3, lorenzo=True)  # 1D: no nd partition
    assert e.value.code == oracle.ERR_ARG
    with pytest.raises(oracle.OracleError) as e:
        oracle.encode_q(np.zeros((6, 8), np.int32), (6, 8), 1.0, 48, lorenzo=True)  # S not a power of two
    assert e.value.code == oracle.ERR_ARG
    with pytest.raises(ValueError):
        oracle.compress(np.ones((4, 4), dtype=np.float32), 1e-3, mean_dec=True, lorenzo=True)
    buf = oracle.compress(_field((6, 7), 1), 1e-3, lorenzo=True)
    with pytest.raises(oracle.OracleError) as e:
        oracle.decompress(buf, oracle.META)
    assert e.value.code == oracle.ERR_UNSUPPORTED
    bad = buf.copy()
    bad[92] = 3  # both decorrelation bits
    with pytest.raises(oracle.OracleError) as e:
        oracle.read_header(bad)
    assert e.value.code == oracle.ERR_STREAM


@pytest.mark.parametrize("shape,S", SHAPES)
def test_mean_and_std_on_dp(shape, S):
    """The nd weights give sum q exactly; Alg. 4 (3D form) gives sum q and
    sum q^2 exactly; both means and the variance match binary64 numpy."""
    x = _field(shape, 7 + sum(shape))
    buf = oracle.compress(x, 1e-3, rel=True, block=S, lorenzo=True)
    h = oracle.read_header(buf)
    p, _ = oracle.decompress(buf, oracle.DELTA)
    q = oracle.decompress(buf, oracle.QUANT).astype(np.int64)
    qi = [int(v) for v in q.ravel()]
    s1, mean = oracle.lz_mean_p(p, h.quantum)
    assert s1 == sum(qi)
    assert mean == pytest.approx(float(np.mean(q * h.quantum)), rel=1e-12, abs=1e-300)
    r = oracle.lz_var_p(p, h.quantum)
    assert (r["n"], r["s1"], r["s2"]) == (q.size, sum(qi), sum(v * v for v in qi))
    if q.size > 1:
        assert r["var"] == pytest.approx(float(np.var(q * h.quantum, ddof=1)), rel=1e-12)


def test_weights_of_the_mean_catch_an_index_shift():
    """A single residual at (s, t) contributes (n1 - s)(n2 - t) copies of
    itself to sum q (0-based s, t): every point of the quadrant after it."""
    for s, t in ((0, 0), (2, 3), (4, 6)):
        p = np.zeros((5, 7), dtype=np.int32)
        p[s, t] = 3
        s1, _ = oracle.lz_mean_p(p, 1.0)
        assert s1 == 3 * (5 - s) * (7 - t)


@pytest.mark.parametrize("shape,S", SHAPES)
def test_derivative_recursion_on_dp(shape, S):
    """Eq. (derivative_Dp): the numerators are 2x numpy.gradient of q
    (central inside, one-sided at the ends) along every axis, exactly."""
    x = _field(shape, 11 + sum(shape))
    buf = oracle.compress(x, 1e-3, rel=True, block=S, lorenzo=True)
    h = oracle.read_header(buf)
    p, _ = oracle.decompress(buf, oracle.DELTA)
    q = oracle.decompress(buf, oracle.QUANT).astype(np.float64)
    for ax in range(len(shape)):
        num, out = oracle.lz_deriv_p(p, ax, h.quantum)
        if shape[ax] == 1:
            want = np.zeros(shape)
        else:
            want = 2 * np.gradient(q, axis=ax, edge_order=1)
        assert np.array_equal(num.astype(np.float64), want), ax
        assert np.array_equal(out, num * (h.quantum * 0.5))
        deriv_ref = oracle.derivative(oracle.dequantize64(q.astype(np.int32), h.quantum), ax)
        assert np.allclose(out, deriv_ref, rtol=1e-12, atol=8 * 2.0 ** -53 * float(np.max(np.abs(q))) * h.quantum)


# ---- HSZp: deltas across block borders over the flat field (Sec. IV) -------------------

@pytest.mark.parametrize("shape,S", [((5, 9, 13), 32), ((1000,), 64), ((33, 41), 32), ((3,), 32), ((7, 70), 64)])
def test_inter_block_deltas(shape, S):
    """p = numpy.diff of the flat q with a leading 0 (crossing block borders),
    q = numpy.cumsum of p; blocks of S in flat order (read back by the
    independent format reader); the paper's HSZp mean and running-sum
    standard deviation on D_p give sum q and sum q^2 exactly."""
    x = _field(shape, 3 + sum(shape))
    buf = oracle.compress(x, 1e-3, rel=True, block=S, inter_block=True)
    h = oracle.read_header(buf)
    assert h.flags == 4 and h.off_width == h.off_q0 and h.nb == -(-h.n // S)
    q_ref = oracle.decompress(oracle.compress(x, 1e-3, rel=True, block=S), oracle.QUANT).ravel().astype(np.int64)
    p, q0 = oracle.decompress(buf, oracle.DELTA)
    assert q0.size == 0
    assert np.array_equal(p.ravel(), np.diff(q_ref, prepend=0))
    assert np.array_equal(oracle.decompress(buf, oracle.QUANT).ravel(), q_ref)
    assert np.array_equal(np.cumsum(p.ravel().astype(np.int64)), q_ref)
    fr = parse(buf.tobytes())
    padded = np.zeros(h.nb * S, dtype=np.int64)
    padded[: h.n] = p.ravel()
    assert np.array_equal(fr["pblocks"], padded.reshape(h.nb, S))
    qi = [int(v) for v in q_ref]
    s1, _ = oracle.lz_mean_p(p.ravel(), h.quantum)  # weights N - i + 1 (1-based)
    assert s1 == sum(qi)
    r = oracle.lz_var_p(p.ravel(), h.quantum)  # the running sum eta of Sec. V-A
    assert (r["s1"], r["s2"]) == (sum(qi), sum(v * v for v in qi))


@pytest.mark.parametrize("S,N", [(2, 5), (3, 5), (4, 4)])
def test_inter_block_brute_force(S, N):
    """Every integer vector in [-2, 2]^N, ragged last block included."""
    import itertools
    for vals in itertools.product(range(-2, 3), repeat=N):
        q = np.array(vals, dtype=np.int32)
        buf = oracle.encode_q(q, (N,), 1.0, S, inter_block=True)
        p, _ = oracle.decompress(buf, oracle.DELTA)
        assert np.array_equal(p, np.diff(q.astype(np.int64), prepend=0)), vals
        assert np.array_equal(oracle.decompress(buf, oracle.QUANT), q), vals


def test_flag_values():
    buf = oracle.compress(_field((6, 7), 2), 1e-3, inter_block=True)
    for fl in (3, 5, 6, 8):
        bad = buf.copy()
        bad[92] = fl
        with pytest.raises(oracle.OracleError) as e:
            oracle.read_header(bad)
        assert e.value.code == oracle.ERR_STREAM
    with pytest.raises(oracle.OracleError) as e:
        oracle.decompress(buf, oracle.META)
    assert e.value.code == oracle.ERR_UNSUPPORTED
