"""CPU oracle for the homomorphic SZp path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product (the HIP library and its
binding) never imports it, and it never imports the product: the two share
no code.  Everything computed here is done by ``hsz_oracle.c`` (plain C,
binary64, no fused multiply-add); this module only marshals numpy arrays
through ctypes.

Functions and the passages of the paper they follow:
  quantize           Sec. IV quantization paragraph, Alg. 1 quantize loop
  quant_params       error bound -> quantum (value-range relative bound,
                     Sec. VI-B; safety margin: a reading, see the C file)
  encode_q           Alg. 1 partition/metadata/decorrelate/encode (SZp)
  compress           Alg. 1 end to end
  decompress         Alg. 2 (stages: 1 metadata, 2 decorrelated,
                     3 quantized, 4 floats)
  compress(mean_dec) Sec. IV HSZx paragraph: block-mean decorrelation
  meta_mean          Sec. V-A Eq. (mean_m), the mean from the metadata
  mean, var          Sec. III-B Eq. (var) on the decompressed field
  derivative,        Sec. III-B Eq. (derivatives), unit spacing, one-sided
  gradmag            at the ends of an axis
  laplacian          Sec. III-B Eq. (laplacian) over every axis, the end
                     value standing in for the missing neighbour
  divergence, curl   Sec. III-B Eq. (divergence) and Eq. (curl), component
                     k paired with axis k; 3D curl is the vector whose last
                     component is the printed 2D formula
  int_sums           sum q and sum q^2 of the quantized field (exact)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsz_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_STREAM, ERR_UNSUPPORTED, ERR_RANGE, ERR_EB, ERR_NONFINITE, ERR_CAPACITY = (
    0, -1, -2, -3, -4, -5, -6, -7)
F32, F64 = 1, 2
META, DELTA, QUANT, FLOAT = 1, 2, 3, 4


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile hsz_oracle.c into liboracle.so with gcc (no FMA contraction)."""
    import subprocess
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
            "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    u64, u32, i32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
    lib.or_compress_bound.restype = u64
    lib.or_compress_bound.argtypes = [u64, u32]
    lib.or_compress_bound_dims.restype = u64
    lib.or_compress_bound_dims.argtypes = [u32, P, u32, u32]
    lib.or_lz_mean_p.restype = i32
    lib.or_lz_mean_p.argtypes = [P, u32, P, dbl, P, P]
    lib.or_lz_var_p.restype = i32
    lib.or_lz_var_p.argtypes = [P, u32, P, dbl, P, P, P, P, P]
    lib.or_lz_deriv_p.restype = i32
    lib.or_lz_deriv_p.argtypes = [P, u32, P, i32, dbl, P, P]
    lib.or_ulp.restype = dbl
    lib.or_ulp.argtypes = [dbl, i32]
    lib.or_quant_params.restype = i32
    lib.or_quant_params.argtypes = [dbl, dbl, dbl, i32, i32, P, P]
    lib.or_quantize.restype = u64
    lib.or_quantize.argtypes = [P, u64, dbl, P]
    lib.or_encode_q.restype = i32
    lib.or_encode_q.argtypes = [P, u32, P, u32, dbl, dbl, u32, u32, P, u64, P]
    lib.or_compress.restype = i32
    lib.or_compress.argtypes = [P, u32, u32, P, dbl, i32, u32, u32, P, u64, P]
    lib.or_meta_mean.restype = i32
    lib.or_meta_mean.argtypes = [P, u64, P, P]
    lib.or_var_mt.restype = i32
    lib.or_var_mt.argtypes = [P, u64, P, P, P, P, P, P]
    lib.or_read_header.restype = i32
    lib.or_read_header.argtypes = [P, u64, P]
    lib.or_stage_bytes.restype = u64
    lib.or_stage_bytes.argtypes = [P, u64, i32]
    lib.or_decompress.restype = i32
    lib.or_decompress.argtypes = [P, u64, i32, P]
    lib.or_dequantize64.restype = None
    lib.or_dequantize64.argtypes = [P, u64, dbl, P]
    for name in ("or_mean", "or_var"):
        getattr(lib, name).restype = i32
        getattr(lib, name).argtypes = [P, P, P, P, P]
    lib.or_derivative.restype = i32
    lib.or_derivative.argtypes = [P, P, i32, P, P, P]
    lib.or_gradmag.restype = i32
    lib.or_gradmag.argtypes = [P, P, P, P, P]
    lib.or_laplacian.restype = i32
    lib.or_laplacian.argtypes = [P, P, P, P, P]
    for name in ("or_divergence", "or_curl"):
        getattr(lib, name).restype = i32
        getattr(lib, name).argtypes = [P, i32, P, P, P, P]
    lib.or_int_sums.restype = i32
    lib.or_int_sums.argtypes = [P, P, P, P, P, P, P, P]
    _lib = lib
    return lib


class _Hdr(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_uint32), ("ndim", ctypes.c_uint32),
        ("dims", ctypes.c_uint64 * 3), ("n", ctypes.c_uint64),
        ("block", ctypes.c_uint32), ("chunk_blocks", ctypes.c_uint32),
        ("eb_abs", ctypes.c_double), ("quantum", ctypes.c_double),
        ("inv_quantum", ctypes.c_double), ("vmin", ctypes.c_double),
        ("vmax", ctypes.c_double), ("max_abs_q", ctypes.c_uint32),
        ("flags", ctypes.c_uint32), ("nb", ctypes.c_uint64),
        ("nchunks", ctypes.c_uint64), ("off_chunk", ctypes.c_uint64),
        ("off_q0", ctypes.c_uint64), ("off_width", ctypes.c_uint64),
        ("off_payload", ctypes.c_uint64), ("payload_words", ctypes.c_uint64),
        ("total_bytes", ctypes.c_uint64),
    ]


@dataclass
class Header:
    dtype: int
    ndim: int
    dims: tuple  # the field's own shape (ndim entries), slow -> fast
    dims3: tuple  # 3D view with leading ones
    n: int
    block: int
    eb_abs: float
    quantum: float
    inv_quantum: float
    vmin: float
    vmax: float
    max_abs_q: int
    nb: int
    nchunks: int
    off_chunk: int
    off_q0: int
    off_width: int
    off_payload: int
    payload_words: int
    total_bytes: int
    flags: int = 0  # bit 0: block-mean decorrelation


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


def _dims3(shape) -> np.ndarray:
    shape = tuple(int(s) for s in shape)
    if not 1 <= len(shape) <= 3:
        raise ValueError("fields are 1D, 2D or 3D")
    return np.array((1,) * (3 - len(shape)) + shape, dtype=np.uint64)


def _box3(shape, box):
    """box = None or (lo, hi) sequences in the field's own axes -> 3D arrays."""
    nd = len(shape)
    if box is None:
        return None, None
    lo, hi = box
    lo3 = np.array((0,) * (3 - nd) + tuple(int(v) for v in lo), dtype=np.int64)
    hi3 = np.array((1,) * (3 - nd) + tuple(int(v) for v in hi), dtype=np.int64)
    return lo3, hi3


def compress_bound(n: int, block: int) -> int:
    return int(_load().or_compress_bound(n, block))


def _flags(mean_dec: bool, lorenzo: bool, inter_block: bool = False) -> int:
    if int(bool(mean_dec)) + int(bool(lorenzo)) + int(bool(inter_block)) > 1:
        raise ValueError("block-mean, Lorenzo and inter-block decorrelation are exclusive")
    return 1 if mean_dec else (2 if lorenzo else (4 if inter_block else 0))


def compress_bound_dims(shape, block: int, flags: int = 0) -> int:
    dims = np.array([int(v) for v in shape], dtype=np.uint64)
    return int(_load().or_compress_bound_dims(len(shape), _ptr(dims), block, flags))


def ulp(v: float, dtype: int) -> float:
    return float(_load().or_ulp(v, dtype))


def quant_params(vmin: float, vmax: float, eb: float, rel: bool, dtype: int):
    """-> (eps_abs, quantum)."""
    lib = _load()
    e = ctypes.c_double()
    d = ctypes.c_double()
    _check(lib.or_quant_params(vmin, vmax, eb, int(rel), dtype, ctypes.byref(e), ctypes.byref(d)),
           "quant_params")
    return e.value, d.value


def quantize(x, quantum: float) -> np.ndarray:
    """q = floor(x * (1/quantum) + 0.5) in binary64; out-of-range values clamp."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    q = np.empty(x.size, dtype=np.int32)
    _load().or_quantize(_ptr(x), x.size, quantum, _ptr(q))
    return q


def encode_q(q, shape, quantum: float, block: int, dtype: int = F32, eb_abs: float = 0.0,
             mean_dec: bool = False, lorenzo: bool = False, inter_block: bool = False) -> np.ndarray:
    """Encode given quantization integers; mean_dec selects block-mean
    decorrelation (HSZx), lorenzo the nd Lorenzo decorrelation of HSZp-nd,
    inter_block HSZp's deltas across block borders, instead of in-block
    deltas."""
    q = np.ascontiguousarray(np.asarray(q, dtype=np.int32).ravel())
    dims = np.array([int(s) for s in shape], dtype=np.uint64)
    fl = _flags(mean_dec, lorenzo, inter_block)
    cap = max(compress_bound_dims(shape, block, fl), 1)
    out = np.zeros(cap, dtype=np.uint8)
    size = ctypes.c_uint64()
    _check(_load().or_encode_q(_ptr(q), len(shape), _ptr(dims), dtype, eb_abs, quantum, block,
                               fl, _ptr(out), cap, ctypes.byref(size)), "encode_q")
    return out[: size.value].copy()


def meta_mean(buf: np.ndarray):
    """Eq. (mean_m) on a block-mean stream: -> (sum_b M_b S_b as int, mean)."""
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    ms, mean = ctypes.c_int64(), ctypes.c_double()
    _check(_load().or_meta_mean(_ptr(buf), buf.size, ctypes.byref(ms), ctypes.byref(mean)), "meta_mean")
    return ms.value, mean.value


def var_mt(buf: np.ndarray) -> dict:
    """Standard deviation on D_p of a block-mean stream (Sec. V-A, about
    the integer metadata mean mu~): -> {n, msum, mu_t, s2 (exact
    sum (p + M_b - mu~)^2 as int), var}."""
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    n, ms, mt, hi = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lo, var = ctypes.c_uint64(), ctypes.c_double()
    _check(_load().or_var_mt(_ptr(buf), buf.size, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(mt),
                             ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(var)), "var_mt")
    return {"n": n.value, "msum": ms.value, "mu_t": mt.value, "s2": (hi.value << 64) + lo.value, "var": var.value}


def lz_mean_p(p: np.ndarray, quantum: float):
    """Mean on D_p of HSZp-nd (Sec. V-A, nd weights): -> (sum q as int, mean)."""
    pp = np.ascontiguousarray(p, dtype=np.int32)
    dims = np.array(pp.shape, dtype=np.uint64)
    s1, mean = ctypes.c_int64(), ctypes.c_double()
    _check(_load().or_lz_mean_p(_ptr(pp), pp.ndim, _ptr(dims), quantum, ctypes.byref(s1), ctypes.byref(mean)),
           "lz_mean_p")
    return s1.value, mean.value


def lz_var_p(p: np.ndarray, quantum: float) -> dict:
    """Alg. 4 (and its 3D form) on D_p of HSZp-nd: -> {n, s1, s2, var}."""
    pp = np.ascontiguousarray(p, dtype=np.int32)
    dims = np.array(pp.shape, dtype=np.uint64)
    n, s1, hi, lo, var = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_double()
    _check(_load().or_lz_var_p(_ptr(pp), pp.ndim, _ptr(dims), quantum, ctypes.byref(n), ctypes.byref(s1),
                               ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(var)), "lz_var_p")
    return {"n": n.value, "s1": s1.value, "s2": (hi.value << 64) + lo.value, "var": var.value}


def lz_deriv_p(p: np.ndarray, axis: int, quantum: float):
    """Eq. (derivative_Dp) on D_p of HSZp-nd along 'axis': -> (integer
    numerators int64, derivative = num * quantum / 2 in binary64)."""
    pp = np.ascontiguousarray(p, dtype=np.int32)
    dims = np.array(pp.shape, dtype=np.uint64)
    num = np.empty(pp.shape, dtype=np.int64)
    out = np.empty(pp.shape, dtype=np.float64)
    _check(_load().or_lz_deriv_p(_ptr(pp), pp.ndim, _ptr(dims), axis, quantum, _ptr(num), _ptr(out)), "lz_deriv_p")
    return num, out


def compress(x: np.ndarray, eb: float, rel: bool = True, block: int = 32, mean_dec: bool = False,
             lorenzo: bool = False, inter_block: bool = False) -> np.ndarray:
    x = np.ascontiguousarray(x)
    if x.dtype == np.float32:
        dt = F32
    elif x.dtype == np.float64:
        dt = F64
    else:
        raise TypeError("field must be float32 or float64")
    dims = np.array(x.shape, dtype=np.uint64)
    fl = _flags(mean_dec, lorenzo, inter_block)
    cap = max(compress_bound_dims(x.shape, block, fl), 1)
    out = np.empty(cap, dtype=np.uint8)
    size = ctypes.c_uint64()
    _check(_load().or_compress(_ptr(x), dt, x.ndim, _ptr(dims), eb, int(rel), block, fl,
                               _ptr(out), cap, ctypes.byref(size)), "compress")
    return out[: size.value].copy()


def read_header(buf: np.ndarray) -> Header:
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    h = _Hdr()
    _check(_load().or_read_header(_ptr(buf), buf.size, ctypes.byref(h)), "read_header")
    dims3 = tuple(int(v) for v in h.dims)
    return Header(
        dtype=h.dtype, ndim=h.ndim, dims=dims3[3 - h.ndim:], dims3=dims3, n=h.n, block=h.block,
        eb_abs=h.eb_abs, quantum=h.quantum, inv_quantum=h.inv_quantum, vmin=h.vmin, vmax=h.vmax,
        max_abs_q=h.max_abs_q, nb=h.nb, nchunks=h.nchunks, off_chunk=h.off_chunk,
        off_q0=h.off_q0, off_width=h.off_width, off_payload=h.off_payload,
        payload_words=h.payload_words, total_bytes=h.total_bytes, flags=h.flags)


def decompress(buf: np.ndarray, stage: int):
    """Alg. 2 to the given stage.

    stage 1 -> q0 (int32[nb]); stage 2 -> (p int32[n] shaped like the field,
    q0 int32[nb], empty for HSZp-nd streams); stage 3 -> q int32 shaped like
    the field; stage 4 -> the decompressed field in its own dtype.
    """
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    h = read_header(buf)
    lib = _load()
    if stage == META and h.flags & 6:
        raise OracleError(ERR_UNSUPPORTED, "decompress: an HSZp-nd or HSZp stream has no metadata stage")
    nbytes = int(lib.or_stage_bytes(_ptr(buf), buf.size, stage))
    if nbytes == 0:
        raise OracleError(ERR_ARG, "decompress: bad stage")
    raw = np.empty(nbytes, dtype=np.uint8)
    _check(lib.or_decompress(_ptr(buf), buf.size, stage, _ptr(raw)), "decompress")
    if stage == META:
        return raw.view(np.int32).copy()
    if stage == DELTA:
        v = raw.view(np.int32)
        return v[: h.n].reshape(h.dims).copy(), v[h.n:].copy()
    if stage == QUANT:
        return raw.view(np.int32).reshape(h.dims).copy()
    return raw.view(np.float32 if h.dtype == F32 else np.float64).reshape(h.dims).copy()


def dequantize64(q: np.ndarray, quantum: float) -> np.ndarray:
    """d' = q * quantum in binary64, shaped like q."""
    qq = np.ascontiguousarray(q, dtype=np.int32)
    out = np.empty(qq.shape, dtype=np.float64)
    _load().or_dequantize64(_ptr(qq), qq.size, quantum, _ptr(out))
    return out


def _field(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return x, _dims3(x.shape)


def mean(x, box=None) -> float:
    x, d = _field(x)
    lo, hi = _box3(x.shape, box)
    r = ctypes.c_double()
    _check(_load().or_mean(_ptr(x), _ptr(d), None if lo is None else _ptr(lo),
                           None if hi is None else _ptr(hi), ctypes.byref(r)), "mean")
    return r.value


def var(x, box=None) -> float:
    x, d = _field(x)
    lo, hi = _box3(x.shape, box)
    r = ctypes.c_double()
    _check(_load().or_var(_ptr(x), _ptr(d), None if lo is None else _ptr(lo),
                          None if hi is None else _ptr(hi), ctypes.byref(r)), "var")
    return r.value


def _box_shape(shape, box):
    if box is None:
        return tuple(shape)
    lo, hi = box
    return tuple(int(h) - int(l) for l, h in zip(lo, hi))


def derivative(x, axis: int, box=None) -> np.ndarray:
    """Derivative along the field's own axis (0 = slowest), restricted to box."""
    x, d = _field(x)
    nd = x.ndim
    if not 0 <= axis < nd:
        raise ValueError("axis out of range")
    lo, hi = _box3(x.shape, box)
    out = np.empty(_box_shape(x.shape, box), dtype=np.float64)
    _check(_load().or_derivative(_ptr(x), _ptr(d), axis + 3 - nd, None if lo is None else _ptr(lo),
                                 None if hi is None else _ptr(hi), _ptr(out)), "derivative")
    return out


def gradmag(x, box=None) -> np.ndarray:
    x, d = _field(x)
    lo, hi = _box3(x.shape, box)
    out = np.empty(_box_shape(x.shape, box), dtype=np.float64)
    _check(_load().or_gradmag(_ptr(x), _ptr(d), None if lo is None else _ptr(lo),
                              None if hi is None else _ptr(hi), _ptr(out)), "gradmag")
    return out


def laplacian(x, box=None) -> np.ndarray:
    """Laplacian (Eq. (laplacian) summed over the field's axes, mirrored ends),
    restricted to box."""
    x, d = _field(x)
    lo, hi = _box3(x.shape, box)
    out = np.empty(_box_shape(x.shape, box), dtype=np.float64)
    _check(_load().or_laplacian(_ptr(x), _ptr(d), None if lo is None else _ptr(lo),
                                None if hi is None else _ptr(hi), _ptr(out)), "laplacian")
    return out


def _components(comps):
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in comps]
    shape = cs[0].shape
    if len(cs) != len(shape) or any(c.shape != shape for c in cs):
        raise ValueError("one component per axis, all of the field's shape")
    arr = (ctypes.c_void_p * len(cs))(*[c.ctypes.data for c in cs])
    return cs, shape, arr


def divergence(comps, box=None) -> np.ndarray:
    """sum_k d F_k / d x_k (Eq. (divergence)); comps[k] pairs with axis k."""
    cs, shape, arr = _components(comps)
    d = _dims3(shape)
    lo, hi = _box3(shape, box)
    out = np.empty(_box_shape(shape, box), dtype=np.float64)
    _check(_load().or_divergence(ctypes.cast(arr, ctypes.c_void_p), len(cs), _ptr(d),
                                 None if lo is None else _ptr(lo), None if hi is None else _ptr(hi),
                                 _ptr(out)), "divergence")
    return out


def curl(comps, box=None) -> np.ndarray:
    """Eq. (curl): 2D fields -> delta_1 F_0 - delta_0 F_1 (box-shaped);
    3D fields -> array (3, *box) of the components
    (delta_2 F_1 - delta_1 F_2, delta_0 F_2 - delta_2 F_0, delta_1 F_0 - delta_0 F_1)."""
    cs, shape, arr = _components(comps)
    if len(shape) not in (2, 3):
        raise ValueError("curl needs a 2D or 3D field")
    d = _dims3(shape)
    lo, hi = _box3(shape, box)
    bs = _box_shape(shape, box)
    out = np.empty(bs if len(shape) == 2 else (3,) + bs, dtype=np.float64)
    _check(_load().or_curl(ctypes.cast(arr, ctypes.c_void_p), len(cs), _ptr(d),
                           None if lo is None else _ptr(lo), None if hi is None else _ptr(hi),
                           _ptr(out)), "curl")
    return out


def int_sums(q, box=None):
    """-> (N, sum q, sum q^2) as Python ints, over the box."""
    q = np.ascontiguousarray(q, dtype=np.int32)
    d = _dims3(q.shape)
    lo, hi = _box3(q.shape, box)
    n, s1, s2lo, s2hi = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64()
    _check(_load().or_int_sums(_ptr(q), _ptr(d), None if lo is None else _ptr(lo),
                               None if hi is None else _ptr(hi), ctypes.byref(n), ctypes.byref(s1),
                               ctypes.byref(s2lo), ctypes.byref(s2hi)), "int_sums")
    return n.value, s1.value, (s2hi.value << 64) + s2lo.value
