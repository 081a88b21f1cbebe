"""Seeded synthetic scientific fields.

This module only draws inputs: it holds none of the compressor's or the
operations' arithmetic, and it is shared by the tests (which feed the same
arrays to the GPU library and to the CPU checker) and by the benchmark.

The paper evaluates on Ocean (2400x3600), Miranda (256x384x384), Hurricane
(100x500x500), NYX (512^3) and JHTDB fields, all binary32 (Sec. VI-A,
Table III).  None of those datasets is available here, so the workloads use
smooth synthetic stand-ins with the same shapes: sums of isotropic Gaussian
bumps, with optional i.i.d. noise, multiplicative log-normal texture (which
makes neighbouring values less predictable and lowers the compression
ratio), and sharp tanh fronts for the binary64 workload.

Draw order for a Gaussian mixture (fixed, so a seed names one field):
centres ~ U[0, dim) per axis (K x ndim), sigma ~ U[sig_lo, sig_hi] (K),
amplitude ~ U[0.5, 2] (K); then per-element noise in C order.  All
arithmetic is binary64, cast to the field dtype at the end.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _pad3(shape):
    shape = tuple(int(s) for s in shape)
    return (1,) * (3 - len(shape)) + shape


def gaussian_mixture(shape, k: int, sigma, seed: int | None = None, rng=None) -> np.ndarray:
    """Sum of k separable isotropic Gaussians in binary64, shaped `shape`."""
    if rng is None:
        rng = np.random.default_rng(seed)
    nd = len(shape)
    dims = np.array(shape, dtype=np.float64)
    centres = rng.uniform(0.0, 1.0, size=(k, nd)) * dims
    sig = rng.uniform(sigma[0], sigma[1], size=k)
    amp = rng.uniform(0.5, 2.0, size=k)
    z3, y3, x3 = _pad3(shape)
    c3 = np.zeros((k, 3))
    c3[:, 3 - nd:] = centres

    def axis_profile(n, c):
        i = np.arange(n, dtype=np.float64)
        return np.exp(-((i[None, :] - c[:, None]) ** 2) / (2.0 * sig[:, None] ** 2))

    gz = axis_profile(z3, c3[:, 0]) if z3 > 1 else np.ones((k, 1))
    gy = axis_profile(y3, c3[:, 1]) if y3 > 1 else np.ones((k, 1))
    gx = axis_profile(x3, c3[:, 2])
    gzy = (amp[:, None, None] * gz[:, :, None] * gy[:, None, :]).reshape(k, z3 * y3)
    f = gzy.T @ gx  # (z*y, x): sum over the k bumps
    return f.reshape(shape)


def _tanh_fronts(shape, nfronts: int, rng) -> np.ndarray:
    """nfronts planes through uniform points with N(0, I)-drawn normals;
    each adds B * tanh(s / 2), s = signed distance in cells."""
    z3, y3, x3 = _pad3(shape)
    out = np.zeros((z3, y3, x3))
    zz = np.arange(z3, dtype=np.float64)[:, None, None]
    yy = np.arange(y3, dtype=np.float64)[None, :, None]
    xx = np.arange(x3, dtype=np.float64)[None, None, :]
    for _ in range(nfronts):
        point = rng.uniform(0.0, 1.0, size=3) * np.array([z3, y3, x3], dtype=np.float64)
        nrm = rng.standard_normal(3)
        nrm /= np.linalg.norm(nrm)
        b = rng.uniform(0.5, 2.0)
        s = (zz - point[0]) * nrm[0] + (yy - point[1]) * nrm[1] + (xx - point[2]) * nrm[2]
        out += b * np.tanh(s / 2.0)
    return out.reshape(shape)


@dataclass(frozen=True)
class FieldSpec:
    shape: tuple
    dtype: str  # "f32" | "f64"
    k: int
    sigma: tuple
    noise: float = 0.0  # std of additive N(0, noise)
    texture: float = 0.0  # std of the log of the multiplicative log-normal texture
    fronts: int = 0
    seed: int = 0


def make_field(spec: FieldSpec) -> np.ndarray:
    rng = np.random.default_rng(spec.seed)
    f = gaussian_mixture(spec.shape, spec.k, spec.sigma, rng=rng)
    if spec.fronts:
        f = f + _tanh_fronts(spec.shape, spec.fronts, rng)
    if spec.noise:
        f = f + rng.normal(0.0, spec.noise, size=spec.shape)
    if spec.texture:
        f = f * np.exp(rng.normal(0.0, spec.texture, size=spec.shape))
    return np.ascontiguousarray(f.astype(np.float32 if spec.dtype == "f32" else np.float64))


# ---- the workloads ----------------------------------------------------------

def small_field_spec(seed: int = 0) -> FieldSpec:
    """64^3 binary32: 8 bumps (sigma 4..16 cells) plus N(0, 1e-3) noise."""
    return FieldSpec((64, 64, 64), "f32", k=8, sigma=(4.0, 16.0), noise=1e-3, seed=seed)


def large_field_spec(seed: int = 0, shape=(512, 512, 512)) -> FieldSpec:
    """512^3 binary32 (NYX-sized): 64 bumps (sigma 8..64) times a log-normal(0, 0.1) texture."""
    return FieldSpec(tuple(shape), "f32", k=64, sigma=(8.0, 64.0), texture=0.1, seed=seed)


BATCH_SHAPES = [(100, 500, 500)] * 4 + [(256, 384, 384)] * 4 + [(1800, 3600)] * 4
BATCH_REL_EB = (1e-2, 1e-3, 1e-4)


def batch_specs():
    """12 uneven binary32 fields (Hurricane-, Miranda-, Ocean-like shapes),
    the large-field recipe, seeds 100+i, relative bounds cycling 1e-2/1e-3/1e-4."""
    return [(large_field_spec(seed=100 + i, shape=s), BATCH_REL_EB[i % 3]) for i, s in enumerate(BATCH_SHAPES)]


def front_field_spec(i: int, shape=(256, 256, 256)) -> FieldSpec:
    """binary64 field: 16 bumps (sigma 8..32) plus 4 tanh fronts of width 2 cells."""
    return FieldSpec(tuple(shape), "f64", k=16, sigma=(8.0, 32.0), fronts=4, seed=200 + i)


def snapshot_spec(k: int) -> FieldSpec:
    """Serving snapshot k: even k -> 512^3, odd k -> 100x500x500; large-field recipe."""
    shape = (512, 512, 512) if k % 2 == 0 else (100, 500, 500)
    return large_field_spec(seed=300 + k, shape=shape)


def make_field_torch(spec: FieldSpec, device="cuda"):
    """The same recipe generated on the GPU with torch's seeded generator (a
    different random stream from make_field, so different values): used where
    many large fields are needed quickly and no CPU reference consumes them
    (the serving snapshots).  binary64 arithmetic, cast at the end."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(spec.seed))
    f64 = torch.float64
    shape = tuple(int(s) for s in spec.shape)
    nd = len(shape)
    k = spec.k
    dims = torch.tensor(shape, dtype=f64, device=device)
    centres = torch.rand(k, nd, generator=g, dtype=f64, device=device) * dims
    sig = spec.sigma[0] + (spec.sigma[1] - spec.sigma[0]) * torch.rand(k, generator=g, dtype=f64, device=device)
    amp = 0.5 + 1.5 * torch.rand(k, generator=g, dtype=f64, device=device)
    z3, y3, x3 = _pad3(shape)
    c3 = torch.zeros(k, 3, dtype=f64, device=device)
    c3[:, 3 - nd:] = centres

    def prof(n, c):
        i = torch.arange(n, dtype=f64, device=device)
        return torch.exp(-((i[None, :] - c[:, None]) ** 2) / (2.0 * sig[:, None] ** 2))

    gz = prof(z3, c3[:, 0]) if z3 > 1 else torch.ones(k, 1, dtype=f64, device=device)
    gy = prof(y3, c3[:, 1]) if y3 > 1 else torch.ones(k, 1, dtype=f64, device=device)
    gx = prof(x3, c3[:, 2])
    gzy = (amp[:, None, None] * gz[:, :, None] * gy[:, None, :]).reshape(k, z3 * y3)
    f = (gzy.T @ gx).reshape(shape)
    if spec.fronts:
        zz = torch.arange(z3, dtype=f64, device=device)[:, None, None]
        yy = torch.arange(y3, dtype=f64, device=device)[None, :, None]
        xx = torch.arange(x3, dtype=f64, device=device)[None, None, :]
        dims3 = torch.tensor([z3, y3, x3], dtype=f64, device=device)
        acc = torch.zeros((z3, y3, x3), dtype=f64, device=device)
        for _ in range(spec.fronts):
            point = torch.rand(3, generator=g, dtype=f64, device=device) * dims3
            nrm = torch.randn(3, generator=g, dtype=f64, device=device)
            nrm = nrm / torch.linalg.norm(nrm)
            b = 0.5 + 1.5 * torch.rand((), generator=g, dtype=f64, device=device)
            s = (zz - point[0]) * nrm[0] + (yy - point[1]) * nrm[1] + (xx - point[2]) * nrm[2]
            acc += b * torch.tanh(s / 2.0)
        f = f + acc.reshape(shape)
    if spec.noise:
        f = f + spec.noise * torch.randn(shape, generator=g, dtype=f64, device=device)
    if spec.texture:
        f = f * torch.exp(spec.texture * torch.randn(shape, generator=g, dtype=f64, device=device))
    return f.to(torch.float32 if spec.dtype == "f32" else torch.float64).contiguous()
