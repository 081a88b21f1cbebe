"""Pins for the oracle's Laplacian, divergence and curl (Sec. III-B,
Eq. (laplacian), Eq. (divergence), Eq. (curl)).

Each function is pinned by values derived by hand from the paper's worked
example (Sec. IV, the 2x4 field Y and its printed Y_q), by library routines
that implement the same operators independently (scipy.ndimage.laplace with
mode='reflect', numpy.gradient), by closed forms on polynomial fields, and
by identities of the discrete operators (the mirrored Laplacian sums to
zero; curl of a gradient and divergence of a curl vanish because the
difference operators along different axes commute).
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def _yq():
    for line in open(GOLDEN):
        if line.startswith("Yq "):
            return np.array([int(t) for t in line.split()[1:]], dtype=np.int32).reshape(2, 4)
    raise AssertionError("Yq missing from the golden file")


# ------------------------------------------------------------------ Laplacian

def test_laplacian_worked_example():
    """Integer numerators of the Laplacian of Y_q (rows 6 8 -11 -12 and
    13 -5 10 9), derived by hand with the end value standing in for the
    missing neighbour, e.g. at (0,0): (6 + 13 - 12) + (6 + 8 - 12) = 9.
    d' = 0.2 * Y_q, so the Laplacian of d' is 0.2 times them."""
    num = [9, -34, 39, 22, -25, 46, -37, -20]
    xh = oracle.dequantize64(_yq(), 0.2)
    got = oracle.laplacian(xh).ravel()
    np.testing.assert_allclose(got, 0.2 * np.array(num, dtype=np.float64), rtol=0, atol=1e-14)
    assert sum(num) == 0  # mirrored ends: the discrete Laplacian sums to zero


@pytest.mark.parametrize("shape", [(9,), (6, 7), (5, 6, 7), (1, 4, 5), (3, 1, 6), (1, 1, 1), (2, 3, 1)])
def test_laplacian_matches_scipy(shape):
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(11)
    x = rng.normal(size=shape) * 3 + 1
    want = ndimage.laplace(x, mode="reflect")
    np.testing.assert_allclose(oracle.laplacian(x), want, rtol=0, atol=1e-13)
    lo = tuple(s // 3 for s in shape)
    hi = tuple(max(l + 1, s - s // 4) for l, s in zip(lo, shape))
    sl = tuple(slice(l, h) for l, h in zip(lo, hi))
    np.testing.assert_allclose(oracle.laplacian(x, (lo, hi)), want[sl], rtol=0, atol=1e-13)


def test_laplacian_closed_form_and_zero_sum():
    """f = a z^2 + b y^2 + c x^2 + linear terms: 2(a + b + c) at every
    interior point; any field's mirrored Laplacian sums to zero."""
    z, y, x = np.meshgrid(np.arange(7.0), np.arange(8.0), np.arange(9.0), indexing="ij")
    a, b, c = 3.0, -2.0, 5.0
    f = a * z * z + b * y * y + c * x * x + 4 * z - 7 * y + x + 11
    lap = oracle.laplacian(f)
    assert np.all(lap[1:-1, 1:-1, 1:-1] == 2 * (a + b + c))
    q = np.random.default_rng(3).integers(-1000, 1000, size=(5, 6, 7)).astype(np.float64)
    assert oracle.laplacian(q).sum() == 0.0  # integer-valued: every sum is exact


# --------------------------------------------------------- divergence, curl

def _grad(f, axis):
    return np.gradient(f, axis=axis) if f.shape[axis] > 1 else np.zeros(f.shape)


@pytest.mark.parametrize("shape", [(7, 9), (5, 6, 7), (1, 4, 5), (4, 1, 6)])
def test_divergence_and_curl_match_numpy(shape):
    rng = np.random.default_rng(21)
    F = [rng.normal(size=shape) for _ in shape]
    div = sum(_grad(F[k], k) for k in range(len(shape)))
    np.testing.assert_allclose(oracle.divergence(F), div, rtol=0, atol=1e-13)
    if len(shape) == 2:
        want = _grad(F[0], 1) - _grad(F[1], 0)
    else:
        want = np.stack([_grad(F[1], 2) - _grad(F[2], 1),
                         _grad(F[2], 0) - _grad(F[0], 2),
                         _grad(F[0], 1) - _grad(F[1], 0)])
    np.testing.assert_allclose(oracle.curl(F), want, rtol=0, atol=1e-13)
    lo = tuple(s // 3 for s in shape)
    hi = tuple(max(l + 1, s - s // 4) for l, s in zip(lo, shape))
    sl = tuple(slice(l, h) for l, h in zip(lo, hi))
    np.testing.assert_allclose(oracle.divergence(F, (lo, hi)), div[sl], rtol=0, atol=1e-13)
    wsl = sl if len(shape) == 2 else (slice(None),) + sl
    np.testing.assert_allclose(oracle.curl(F, (lo, hi)), want[wsl], rtol=0, atol=1e-13)


def test_divergence_curl_closed_forms():
    z, y, x = np.meshgrid(np.arange(6.0), np.arange(7.0), np.arange(8.0), indexing="ij")
    # F = (2z, -3y, 5x): divergence 2 - 3 + 5 = 4 everywhere (one-sided ends are exact on linear fields)
    assert np.all(oracle.divergence([2 * z, -3 * y, 5 * x]) == 4.0)
    # 2D, Eq. (curl) as printed: delta_y u - delta_x v with u = c*j, v = e*i gives c - e
    i, j = np.meshgrid(np.arange(5.0), np.arange(6.0), indexing="ij")
    assert np.all(oracle.curl([3.0 * j, 7.0 * i]) == 3.0 - 7.0)
    # 3D, axes (z, y, x) = (0, 1, 2): F = (5x + y, 2x + 7z, 3z + 4y) gives
    # (d2 F1 - d1 F2, d0 F2 - d2 F0, d1 F0 - d0 F1) = (2 - 4, 3 - 5, 1 - 7)
    c = oracle.curl([5 * x + y, 2 * x + 7 * z, 3 * z + 4 * y])
    assert np.all(c[0] == -2.0) and np.all(c[1] == -2.0) and np.all(c[2] == -6.0)


def test_curl_of_gradient_and_divergence_of_curl_vanish():
    rng = np.random.default_rng(8)
    phi = rng.integers(-50, 50, size=(6, 7, 8)).astype(np.float64)
    g = [oracle.derivative(phi, k) for k in range(3)]
    np.testing.assert_allclose(oracle.curl(g), 0.0, rtol=0, atol=1e-12)
    phi2 = phi[0]
    g2 = [oracle.derivative(phi2, k) for k in range(2)]
    np.testing.assert_allclose(oracle.curl(g2), 0.0, rtol=0, atol=1e-12)
    F = [rng.integers(-50, 50, size=(6, 7, 8)).astype(np.float64) for _ in range(3)]
    np.testing.assert_allclose(oracle.divergence(list(oracle.curl(F))), 0.0, rtol=0, atol=1e-12)


def test_vector_ops_reject_bad_shapes():
    with pytest.raises(ValueError):
        oracle.divergence([np.zeros((3, 4))])  # one component for a 2D field
    with pytest.raises(ValueError):
        oracle.curl([np.zeros(5)])
