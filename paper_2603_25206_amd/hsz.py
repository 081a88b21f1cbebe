"""Python binding of libhsz (include/hsz.h) -- argument marshalling only.

Every step of compression, decompression and the operations runs in the HIP
kernels of libhsz.so; this module allocates device buffers with torch,
passes raw pointers and the current torch stream through ctypes, and turns
results back into tensors.  There is no fallback: if the library is not
built, or no GPU is visible, the calls raise.

Names follow the C ABI: compress, read_header, decompress_to_stage,
op_on_stage, op_fused (plus helpers).
"""
from __future__ import annotations

import ctypes
import os
import struct
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsz.so")

OK = 0
ERR_INVALID_ARG, ERR_BAD_STREAM, ERR_UNSUPPORTED, ERR_RANGE, ERR_EB, ERR_NONFINITE, ERR_CAPACITY, ERR_HIP = (
    -1, -2, -3, -4, -5, -6, -7, -8)
F32, F64 = 1, 2
META, DELTA, QUANT, FLOAT = 1, 2, 3, 4
MEAN, VAR, DERIV, GRADMAG, LAPLACIAN, DIVERGENCE, CURL, VAR_MT = 1, 2, 3, 4, 5, 6, 7, 8
FLAG_BLOCK_MEAN = 1  # header flag: block-mean decorrelation (HSZx)
FLAG_LORENZO = 2  # header flag: Lorenzo decorrelation over the whole field, nd blocks (HSZp-nd)
FLAG_INTER_BLOCK = 4  # header flag: deltas across the blocks of the flat field (HSZp)
HEADER_BYTES = 256

_OPS = {"mean": MEAN, "var": VAR, "var_mt": VAR_MT, "deriv": DERIV, "gradmag": GRADMAG, "laplacian": LAPLACIAN,
        "divergence": DIVERGENCE, "curl": CURL}
_STAGES = {"meta": META, "delta": DELTA, "quant": QUANT, "float": FLOAT}
_STATS = (MEAN, VAR, VAR_MT)
NOALLOC_SCRATCH_BYTES = 16 << 20  # HSZ_NOALLOC_SCRATCH_BYTES: the fixed workspace of op_fused_noalloc


class HszError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        msg = f"{what}: {code}"
        if _lib is not None:
            msg += f" ({_lib.hsz_strerror(code).decode()})"
        if detail:
            msg += f" {detail}"
        super().__init__(msg)
        self.code = code


class Header(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * 3),
        ("n", ctypes.c_int64), ("block", ctypes.c_int32), ("chunk_blocks", ctypes.c_int32),
        ("eb_abs", ctypes.c_double), ("quantum", ctypes.c_double), ("inv_quantum", ctypes.c_double),
        ("vmin", ctypes.c_double), ("vmax", ctypes.c_double), ("max_abs_q", ctypes.c_uint32),
        ("flags", ctypes.c_uint32), ("nb", ctypes.c_int64), ("nchunks", ctypes.c_int64),
        ("off_chunk", ctypes.c_uint64), ("off_q0", ctypes.c_uint64), ("off_width", ctypes.c_uint64),
        ("off_payload", ctypes.c_uint64), ("payload_words", ctypes.c_uint64),
        ("total_bytes", ctypes.c_uint64),
    ]

    @property
    def shape(self):
        return tuple(int(self.dims[k]) for k in range(self.ndim))

    @property
    def torch_dtype(self):
        return torch.float32 if self.dtype == F32 else torch.float64


class Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int64 * 3), ("hi", ctypes.c_int64 * 3)]


class Work(ctypes.Structure):
    _fields_ = [("d_c", ctypes.c_void_p), ("h", ctypes.POINTER(Header)), ("op", ctypes.c_int32),
                ("via", ctypes.c_int32), ("axis", ctypes.c_int32), ("use_box", ctypes.c_int32), ("box", Box),
                ("d_result", ctypes.c_void_p), ("result_bytes", ctypes.c_uint64), ("d_index", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("stats_waves_per_cu", ctypes.c_int32), ("grad_groups_per_cu", ctypes.c_int32),
                ("grad_tz", ctypes.c_int32), ("separate_stats", ctypes.c_int32), ("graph_replay", ctypes.c_int32),
                ("grad_tile_x", ctypes.c_int32)]


EXPORTS = (
    "hsz_strerror", "hsz_version", "hsz_last_hip_error", "hsz_read_status", "hsz_compress_bound",
    "hsz_compress_workspace", "hsz_compress", "hsz_compress_flags", "hsz_read_header", "hsz_stage_bytes",
    "hsz_decompress_to_stage", "hsz_decompress_workspace", "hsz_op_workspace", "hsz_op_on_stage", "hsz_op_fused",
    "hsz_batch_workspace", "hsz_batch_run", "hsz_plan_create", "hsz_plan_update", "hsz_plan_launch",
    "hsz_plan_destroy", "hsz_block_index_bytes", "hsz_block_index", "hsz_vector_workspace",
    "hsz_vector_op_on_stage", "hsz_vector_op_fused", "hsz_compress_range", "hsz_extremes_workspace",
    "hsz_extremes", "hsz_ooc_workspace", "hsz_ooc_op", "hsz_compress_workspace_mode", "hsz_op_fused_noalloc",
    "hsz_ctx_create", "hsz_ctx_destroy", "hsz_ctx_reserve", "hsz_ctx_scratch", "hsz_ctx_set_tuning",
    "hsz_ctx_get_tuning", "hsz_ctx_batch_run", "hsz_ooc_op_async",
)

_lib = None


def load(path: str = LIB_PATH):
    """Load libhsz.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhsz.so is not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
    pi64, pu64 = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)
    sig = {
        "hsz_strerror": (ctypes.c_char_p, [i32]),
        "hsz_version": (i32, []),
        "hsz_last_hip_error": (i32, []),
        "hsz_read_status": (i32, [P, P, ctypes.POINTER(ctypes.c_int)]),
        "hsz_compress_bound": (i32, [i32, i32, pi64, i32, pu64]),
        "hsz_compress_workspace": (i32, [i32, pi64, i32, pu64]),
        "hsz_compress_workspace_mode": (i32, [i32, pi64, i32, ctypes.c_uint32, pu64]),
        "hsz_compress": (i32, [P, i32, i32, pi64, dbl, i32, i32, P, u64, P, u64, P]),
        "hsz_compress_flags": (i32, [P, i32, i32, pi64, dbl, i32, i32, ctypes.c_uint32, P, u64, P, u64, P]),
        "hsz_read_header": (i32, [P, u64, u64, ctypes.POINTER(Header)]),
        "hsz_stage_bytes": (i32, [ctypes.POINTER(Header), i32, pu64]),
        "hsz_decompress_to_stage": (i32, [P, ctypes.POINTER(Header), i32, P, u64, P, u64, P]),
        "hsz_decompress_workspace": (i32, [ctypes.POINTER(Header), i32, ctypes.POINTER(ctypes.c_uint64)]),
        "hsz_op_workspace": (i32, [ctypes.POINTER(Header), i32, pu64]),
        "hsz_op_on_stage": (i32, [P, ctypes.POINTER(Header), i32, i32, i32, ctypes.POINTER(Box), P, u64, P,
                                  u64, P]),
        "hsz_op_fused": (i32, [P, ctypes.POINTER(Header), i32, i32, i32, ctypes.POINTER(Box), P, u64, P, u64,
                               P]),
        "hsz_op_fused_noalloc": (i32, [P, ctypes.POINTER(Header), i32, i32, i32, ctypes.POINTER(Box), P, u64,
                                       P, P]),
        "hsz_batch_workspace": (i32, [ctypes.POINTER(Work), i32, pu64]),
        "hsz_batch_run": (i32, [ctypes.POINTER(Work), i32, ctypes.POINTER(Tuning), P, u64, P]),
        "hsz_plan_create": (i32, [ctypes.POINTER(Work), i32, ctypes.POINTER(Tuning), P, u64, P,
                                  ctypes.POINTER(ctypes.c_void_p)]),
        "hsz_plan_update": (i32, [P, ctypes.POINTER(Work), i32]),
        "hsz_plan_launch": (i32, [P, P]),
        "hsz_plan_destroy": (None, [P]),
        "hsz_block_index_bytes": (i32, [ctypes.POINTER(Header), pu64]),
        "hsz_block_index": (i32, [P, ctypes.POINTER(Header), P, u64, P]),
        "hsz_vector_workspace": (i32, [P, i32, pu64]),
        "hsz_vector_op_on_stage": (i32, [P, P, i32, i32, i32, ctypes.POINTER(Box), P, u64, P, u64, P]),
        "hsz_vector_op_fused": (i32, [P, P, i32, i32, i32, ctypes.POINTER(Box), P, u64, P, u64, P]),
        "hsz_compress_range": (i32, [P, i32, i32, pi64, dbl, i32, dbl, dbl, i32, ctypes.c_uint32, P, u64, P, u64,
                                     P]),
        "hsz_extremes_workspace": (i32, [pu64]),
        "hsz_extremes": (i32, [P, i32, u64, P, P, u64, P]),
        "hsz_ooc_workspace": (i32, [P, i32, i32, pu64]),
        "hsz_ooc_op": (i32, [P, P, i32, i32, i32, i32, P, u64, P, u64, P]),
        "hsz_ctx_create": (i32, [u64, u64, ctypes.POINTER(ctypes.c_void_p)]),
        "hsz_ctx_destroy": (None, [P]),
        "hsz_ctx_reserve": (i32, [P, u64]),
        "hsz_ctx_scratch": (i32, [P, ctypes.POINTER(ctypes.c_void_p), pu64]),
        "hsz_ctx_set_tuning": (i32, [P, ctypes.c_char_p, ctypes.POINTER(Tuning)]),
        "hsz_ctx_get_tuning": (i32, [P, ctypes.c_char_p, ctypes.POINTER(Tuning)]),
        "hsz_ctx_batch_run": (i32, [P, ctypes.POINTER(Work), i32, ctypes.POINTER(Tuning), P, P]),
        "hsz_ooc_op_async": (i32, [P, P, P, i32, i32, i32, i32, P, u64, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != OK:
        detail = ""
        if rc == ERR_HIP:
            detail = f"hipError {_lib.hsz_last_hip_error()}"
        raise HszError(rc, what, detail)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dims(shape):
    arr = (ctypes.c_int64 * 3)(*([int(v) for v in shape] + [1] * (3 - len(shape))))
    return arr


def _box(box, ndim):
    if box is None:
        return None
    lo, hi = box
    b = Box()
    for k in range(ndim):
        b.lo[k] = int(lo[k])
        b.hi[k] = int(hi[k])
    return ctypes.byref(b)


def _empty_bytes(nbytes: int, device) -> torch.Tensor:
    # rounded up to 16 bytes so every buffer is 16-byte aligned and whole
    return torch.empty(((int(nbytes) + 15) // 16) * 16, dtype=torch.uint8, device=device)


_ws_cache: dict = {}


def workspace(nbytes: int, device=None, key: str = "op") -> torch.Tensor:
    """A cached device workspace of at least nbytes (per device and key)."""
    dev = torch.device(device if device is not None else "cuda")
    k = (str(dev), key)
    t = _ws_cache.get(k)
    if t is None or t.numel() < nbytes:
        t = _empty_bytes(max(int(nbytes), 256), dev)
        _ws_cache[k] = t
    return t


def read_status(ws: torch.Tensor, stream=None) -> int:
    lib = load()
    st = ctypes.c_int(0)
    _check(lib.hsz_read_status(ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(_stream(stream)),
                               ctypes.byref(st)), "read_status")
    return st.value


@dataclass
class Compressed:
    """A compressed stream resident in device memory, with its parsed header
    (and, once built with build_index(), its block index)."""
    data: torch.Tensor  # uint8, at least header.total_bytes long
    header: Header
    index: torch.Tensor | None = None

    def build_index(self, stream=None) -> torch.Tensor:
        """Build (once) the per-block payload offsets used by batches."""
        if self.index is None:
            lib = load()
            nbytes = ctypes.c_uint64()
            _check(lib.hsz_block_index_bytes(ctypes.byref(self.header), ctypes.byref(nbytes)), "block_index_bytes")
            idx = _empty_bytes(nbytes.value, self.data.device)
            _check(lib.hsz_block_index(ctypes.c_void_p(self.data.data_ptr()), ctypes.byref(self.header),
                                       ctypes.c_void_p(idx.data_ptr()), idx.numel(),
                                       ctypes.c_void_p(_stream(stream))), "block_index")
            self.index = idx
        return self.index

    @property
    def nbytes(self) -> int:
        return int(self.header.total_bytes)

    @property
    def ratio(self) -> float:
        esz = 4 if self.header.dtype == F32 else 8
        return self.header.n * esz / self.nbytes

    def to_bytes(self):
        return self.data[: self.nbytes].cpu().numpy()


def read_header(buf, len_stream: int | None = None) -> Header:
    """Parse a header from host bytes (numpy/bytes) or a device uint8 tensor."""
    lib = load()
    if isinstance(buf, torch.Tensor):
        if len_stream is None:
            len_stream = buf.numel()
        host = buf[:HEADER_BYTES].cpu().numpy().tobytes()
    else:
        host = bytes(memoryview(buf)[:HEADER_BYTES])
        if len_stream is None:
            len_stream = len(memoryview(buf))
    h = Header()
    cbuf = ctypes.create_string_buffer(host, len(host))
    _check(lib.hsz_read_header(cbuf, len(host), int(len_stream), ctypes.byref(h)), "read_header")
    return h


def compress_bound(shape, dtype: int, block: int) -> int:
    lib = load()
    out = ctypes.c_uint64()
    _check(lib.hsz_compress_bound(dtype, len(shape), _dims(shape), block, ctypes.byref(out)), "compress_bound")
    return out.value


def compress(x: torch.Tensor, eb: float, rel: bool = True, block: int = 32, stream=None,
             out: torch.Tensor | None = None, check: bool = True, mean_dec: bool = False,
             lorenzo: bool = False, inter_block: bool = False) -> Compressed:
    """c = C(x, eb) on the GPU.  x: contiguous float32/float64 CUDA tensor.
    mean_dec selects the block-mean decorrelation (HSZx), lorenzo the nd
    Lorenzo decorrelation of HSZp-nd (2D / 3D fields), inter_block HSZp's
    deltas across block borders, instead of in-block deltas."""
    if int(bool(mean_dec)) + int(bool(lorenzo)) + int(bool(inter_block)) > 1:
        raise ValueError("block-mean, Lorenzo and inter-block decorrelation are exclusive")
    flags = FLAG_BLOCK_MEAN if mean_dec else (FLAG_LORENZO if lorenzo else (FLAG_INTER_BLOCK if inter_block else 0))
    lib = load()
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous GPU tensor")
    dt = F32 if x.dtype == torch.float32 else F64 if x.dtype == torch.float64 else None
    if dt is None:
        raise TypeError("x must be float32 or float64")
    shape = tuple(x.shape)
    dims = _dims(shape)
    cap = compress_bound(shape, dt, block)
    if out is None:
        out = _empty_bytes(cap, x.device)
    wsb = ctypes.c_uint64()
    _check(lib.hsz_compress_workspace_mode(len(shape), dims, block, flags, ctypes.byref(wsb)), "compress_workspace")
    ws = workspace(wsb.value, x.device, key="compress")
    s = _stream(stream)
    _check(lib.hsz_compress_flags(ctypes.c_void_p(x.data_ptr()), dt, len(shape), dims, float(eb), int(rel),
                                  block, flags, ctypes.c_void_p(out.data_ptr()),
                                  out.numel(), ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(s)),
           "compress")
    if not check:
        return Compressed(out, Header())
    st = read_status(ws, stream)
    if st != OK:
        raise HszError(st, "compress")
    return Compressed(out, read_header(out))


def op_workspace_bytes(h: Header, op) -> int:
    lib = load()
    op = _OPS.get(op, op)
    wsb = ctypes.c_uint64()
    _check(lib.hsz_op_workspace(ctypes.byref(h), op, ctypes.byref(wsb)), "op_workspace")
    return wsb.value


def stage_bytes(h: Header, stage: int) -> int:
    lib = load()
    out = ctypes.c_uint64()
    _check(lib.hsz_stage_bytes(ctypes.byref(h), stage, ctypes.byref(out)), "stage_bytes")
    return out.value


def decompress_to_stage(c: Compressed, stage, stream=None, out: torch.Tensor | None = None, ws=None,
                        check: bool = False):
    """Alg. 2 to stage 1..4.  Returns (for stage 2) (p, q0), else one tensor
    shaped like the field (stage 1: q0 of shape [nb])."""
    lib = load()
    stage = _STAGES.get(stage, stage)
    h = c.header
    nbytes = stage_bytes(h, stage)
    if out is None:
        out = _empty_bytes(nbytes, c.data.device)
    wsb = ctypes.c_uint64()
    _check(lib.hsz_decompress_workspace(ctypes.byref(h), stage, ctypes.byref(wsb)), "decompress_workspace")
    if ws is None or ws.numel() < wsb.value:
        ws = workspace(wsb.value, c.data.device, key="decode")
    _check(lib.hsz_decompress_to_stage(ctypes.c_void_p(c.data.data_ptr()), ctypes.byref(h), stage,
                                       ctypes.c_void_p(out.data_ptr()), out.numel(),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       ctypes.c_void_p(_stream(stream))), "decompress_to_stage")
    if check:
        st = read_status(ws, stream)
        if st != OK:
            raise HszError(st, "decompress_to_stage")
    return stage_view(out, h, stage)


def stage_view(buf: torch.Tensor, h: Header, stage: int):
    n, nb = int(h.n), int(h.nb)
    if stage == META:
        return buf[: 4 * nb].view(torch.int32)
    if stage == DELTA:
        nq = 0 if h.flags & (FLAG_LORENZO | FLAG_INTER_BLOCK) else nb  # no metadata in these modes
        v = buf[: 4 * (n + nq)].view(torch.int32)
        return v[:n].view(h.shape), v[n:]
    if stage == QUANT:
        return buf[: 4 * n].view(torch.int32).view(h.shape)
    esz = 4 if h.dtype == F32 else 8
    return buf[: esz * n].view(h.torch_dtype).view(h.shape)


def _stats_from_raw(raw: bytes) -> dict:
    n, s1, s2lo, s2hi, mean, var = struct.unpack("<qqQqdd", raw)
    return {"n": n, "s1": s1, "s2": (s2hi << 64) + s2lo, "mean": mean, "var": var}


def _result_buffer(h: Header, op: int, box, device):
    if op in _STATS:
        return _empty_bytes(48, device), None
    if box is None:
        shape = h.shape
    else:
        shape = tuple(int(hi) - int(lo) for lo, hi in zip(*box))
    esz = 4 if h.dtype == F32 else 8
    vol = 1
    for s in shape:
        vol *= s
    return _empty_bytes(esz * vol, device), shape


def stats_of(buf: torch.Tensor) -> dict:
    """Decode a 48-byte hsz_stats result buffer (synchronises)."""
    return _stats_from_raw(buf[:48].cpu().numpy().tobytes())


def _finish(buf, shape, h, op, ws, stream, check, raw=False):
    if raw:
        return buf
    if check:
        st = read_status(ws, stream)
        if st != OK:
            raise HszError(st, "operation")
    if op in _STATS:
        return _stats_from_raw(buf[:48].cpu().numpy().tobytes())
    vol = 1
    for s in shape:
        vol *= s
    esz = 4 if h.dtype == F32 else 8
    return buf[: esz * vol].view(h.torch_dtype).view(shape)


def op_on_stage(stage_buf, h: Header, stage, op, axis: int = 0, box=None, stream=None, check: bool = True,
                out: torch.Tensor | None = None, ws: torch.Tensor | None = None, raw: bool = False):
    """Operation on a materialised stage buffer (the tensor(s) returned by
    decompress_to_stage).  Stats return a dict; derivatives a tensor."""
    lib = load()
    stage = _STAGES.get(stage, stage)
    op = _OPS.get(op, op)
    base = stage_buf[0] if isinstance(stage_buf, tuple) else stage_buf
    dev = base.device
    buf, shape = _result_buffer(h, op, box, dev) if out is None else (out, None)
    if shape is None and op not in _STATS:
        shape = h.shape if box is None else tuple(int(hi) - int(lo) for lo, hi in zip(*box))
    if ws is None:
        ws = workspace(op_workspace_bytes(h, op), dev)
    _check(lib.hsz_op_on_stage(ctypes.c_void_p(base.data_ptr()), ctypes.byref(h), stage, op, axis,
                               _box(box, h.ndim), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(_stream(stream))),
           "op_on_stage")
    return _finish(buf, shape, h, op, ws, stream, check, raw)


def op_fused(c: Compressed, via, op, axis: int = 0, box=None, stream=None, check: bool = True,
             out: torch.Tensor | None = None, ws: torch.Tensor | None = None, raw: bool = False):
    """Operation computed straight from the compressed stream through stage via."""
    lib = load()
    via = _STAGES.get(via, via)
    op = _OPS.get(op, op)
    h = c.header
    dev = c.data.device
    buf, shape = _result_buffer(h, op, box, dev) if out is None else (out, None)
    if shape is None and op not in _STATS:
        shape = h.shape if box is None else tuple(int(hi) - int(lo) for lo, hi in zip(*box))
    if ws is None:
        ws = workspace(op_workspace_bytes(h, op), dev)
    _check(lib.hsz_op_fused(ctypes.c_void_p(c.data.data_ptr()), ctypes.byref(h), via, op, axis,
                            _box(box, h.ndim), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(_stream(stream))),
           "op_fused")
    return _finish(buf, shape, h, op, ws, stream, check, raw)


def op_fused_noalloc(c: Compressed, via, op, axis: int = 0, box=None, stream=None, out: torch.Tensor | None = None,
                     status: torch.Tensor | None = None):
    """op_fused without a caller workspace: the library's fixed per-device
    scratch array serves as the workspace, so the call allocates nothing
    (pass 'out' and 'status' to keep this wrapper allocation-free too).
    Returns the raw result buffer; 'status' (int32 on the device) receives
    the call's status word.  Calls on one device must not overlap."""
    lib = load()
    via = _STAGES.get(via, via)
    op = _OPS.get(op, op)
    h = c.header
    dev = c.data.device
    buf = _result_buffer(h, op, box, dev)[0] if out is None else out
    st_ptr = ctypes.c_void_p(status.data_ptr()) if status is not None else None
    _check(lib.hsz_op_fused_noalloc(ctypes.c_void_p(c.data.data_ptr()), ctypes.byref(h), via, op, axis,
                                    _box(box, h.ndim), ctypes.c_void_p(buf.data_ptr()), buf.numel(), st_ptr,
                                    ctypes.c_void_p(_stream(stream))), "op_fused_noalloc")
    return buf


# ---- vector fields -------------------------------------------------------------------

def _headers_array(headers):
    arr = (ctypes.POINTER(Header) * len(headers))(*[ctypes.pointer(h) for h in headers])
    return arr


def vector_workspace_bytes(headers) -> int:
    out = ctypes.c_uint64()
    arr = _headers_array(headers)
    _check(load().hsz_vector_workspace(ctypes.cast(arr, ctypes.c_void_p), len(headers), ctypes.byref(out)),
           "vector_workspace")
    return out.value


def _vector_results(h: Header, op: int, box, device, outs):
    nout = 3 if (op == CURL and h.ndim == 3) else 1
    if outs is None:
        outs = [_result_buffer(h, DERIV, box, device)[0] for _ in range(nout)]
    shape = h.shape if box is None else tuple(int(hi) - int(lo) for lo, hi in zip(*box))
    return outs, shape


def _vector_call(fn_name, ptrs, headers, dev, mode, op, box, stream, check, outs, ws, what):
    lib = load()
    op = _OPS.get(op, op)
    h = headers[0]
    outs, shape = _vector_results(h, op, box, dev, outs)
    if ws is None:
        ws = workspace(vector_workspace_bytes(headers), dev)
    harr = _headers_array(headers)
    parr = (ctypes.c_void_p * len(ptrs))(*ptrs)
    oarr = (ctypes.c_void_p * 3)(*([o.data_ptr() for o in outs] + [None] * (3 - len(outs))))
    cap = min(o.numel() for o in outs)
    _check(getattr(lib, fn_name)(ctypes.cast(parr, ctypes.c_void_p), ctypes.cast(harr, ctypes.c_void_p),
                                 len(headers), mode, op, _box(box, h.ndim), ctypes.cast(oarr, ctypes.c_void_p),
                                 cap, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 ctypes.c_void_p(_stream(stream))), what)
    if check:
        st = read_status(ws, stream)
        if st != OK:
            raise HszError(st, what)
    vol = 1
    for n in shape:
        vol *= n
    esz = 4 if h.dtype == F32 else 8
    res = [o[: esz * vol].view(h.torch_dtype).view(shape) for o in outs]
    return res[0] if len(res) == 1 else tuple(res)


def vector_op_fused(comps, op, via=QUANT, box=None, stream=None, check: bool = True, outs=None, ws=None):
    """Divergence or curl of the vector field whose component k is the
    compressed stream comps[k], computed from the streams through D_q.
    Returns one tensor, or three for the curl of a 3D field."""
    via = _STAGES.get(via, via)
    return _vector_call("hsz_vector_op_fused", [c.data.data_ptr() for c in comps], [c.header for c in comps],
                        comps[0].data.device, via, op, box, stream, check, outs, ws, "vector_op_fused")


def vector_op_on_stage(bufs, headers, stage, op, box=None, stream=None, check: bool = True, outs=None, ws=None):
    """Divergence or curl on materialised stage-3 or stage-4 buffers (one per
    component, from decompress_to_stage)."""
    stage = _STAGES.get(stage, stage)
    return _vector_call("hsz_vector_op_on_stage", [b.data_ptr() for b in bufs], list(headers), bufs[0].device,
                        stage, op, box, stream, check, outs, ws, "vector_op_on_stage")


def from_bytes(data, device="cuda") -> Compressed:
    """Upload a compressed stream held in host memory."""
    import numpy as np
    arr = np.frombuffer(bytes(memoryview(data)), dtype=np.uint8)
    h = read_header(arr)
    t = _empty_bytes(arr.size, device)
    t[: arr.size].copy_(torch.from_numpy(arr.copy()))
    return Compressed(t, h)


# ---- batches --------------------------------------------------------------------------

@dataclass
class Job:
    """One operation of a batch: op on stream c through stage via (box optional)."""
    c: Compressed
    op: int
    via: int
    axis: int = 0
    box: tuple | None = None


def _result_for(job: Job, device):
    h = job.c.header
    op = _OPS.get(job.op, job.op)
    buf, shape = _result_buffer(h, op, job.box, device)
    return buf, shape


class _Batch:
    """Marshalled work items of a batch (keeps the ctypes objects alive)."""

    def __init__(self, jobs, outs=None, device=None):
        self.jobs = list(jobs)
        dev = device if device is not None else self.jobs[0].c.data.device
        self.results, self.shapes = [], []
        for k, j in enumerate(self.jobs):
            if outs is not None:
                buf, shape = outs[k]
            else:
                buf, shape = _result_for(j, dev)
            self.results.append(buf)
            self.shapes.append(shape)
        self.items = (Work * len(self.jobs))()
        self._headers = []
        for k, j in enumerate(self.jobs):
            w = self.items[k]
            hh = j.c.header
            self._headers.append(hh)
            w.d_c = j.c.data.data_ptr()
            w.h = ctypes.pointer(hh)
            w.op = _OPS.get(j.op, j.op)
            w.via = _STAGES.get(j.via, j.via)
            w.axis = j.axis
            w.use_box = 0 if j.box is None else 1
            if j.box is not None:
                lo, hi = j.box
                for a in range(hh.ndim):
                    w.box.lo[a] = int(lo[a])
                    w.box.hi[a] = int(hi[a])
            w.d_result = self.results[k].data_ptr()
            w.result_bytes = self.results[k].numel()
            w.d_index = j.c.index.data_ptr() if j.c.index is not None else None

    def workspace_bytes(self) -> int:
        out = ctypes.c_uint64()
        _check(load().hsz_batch_workspace(self.items, len(self.jobs), ctypes.byref(out)), "batch_workspace")
        return out.value

    def outputs(self):
        """Results as dicts (statistics) or tensors (derivatives); synchronises."""
        res = []
        for j, buf, shape in zip(self.jobs, self.results, self.shapes):
            op = _OPS.get(j.op, j.op)
            res.append(_finish(buf, shape, j.c.header, op, None, None, False))
        return res


def _tuning(tune):
    if tune is None:
        return None
    t = Tuning()
    t.stats_waves_per_cu = int(tune.get("stats_waves_per_cu", 0))
    t.grad_groups_per_cu = int(tune.get("grad_groups_per_cu", 0))
    t.grad_tz = int(tune.get("grad_tz", 0))
    t.separate_stats = int(bool(tune.get("separate_stats", False)))
    t.graph_replay = int(bool(tune.get("graph_replay", False)))
    t.grad_tile_x = int(tune.get("grad_tile_x", 0))
    if t.grad_tile_x not in (0, 256, 512, -1):
        raise ValueError("grad_tile_x must be 0, 256, 512 or -1")
    return ctypes.byref(t)


def batch_run(jobs, tune: dict | None = None, stream=None, ws: torch.Tensor | None = None, sync: bool = True):
    """Run a batch of jobs in one pass; returns the results (or the _Batch when
    sync is False: call .outputs() after the stream completes)."""
    lib = load()
    b = _Batch(jobs)
    need = b.workspace_bytes()
    if ws is None or ws.numel() < need:
        ws = workspace(need, b.results[0].device, key="batch")
    _check(lib.hsz_batch_run(b.items, len(b.jobs), _tuning(tune), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                             ctypes.c_void_p(_stream(stream))), "batch_run")
    if not sync:
        b.ws = ws
        return b
    st = read_status(ws, stream)
    if st != OK:
        raise HszError(st, "batch_run")
    return b.outputs()


class Plan:
    """A batch captured as a HIP graph; replay with launch(), retarget with update()."""

    def __init__(self, jobs, tune: dict | None = None, stream=None):
        lib = load()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.batch = _Batch(jobs)
        need = self.batch.workspace_bytes()
        self.ws = _empty_bytes(need, self.batch.results[0].device)
        handle = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(lib.hsz_plan_create(self.batch.items, len(self.batch.jobs), _tuning(tune),
                                   ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)), "plan_create")
        self.handle = handle

    def update(self, jobs, outs=None):
        """New jobs of the same structure (new streams, boxes, axes); results go
        to 'outs' ((buffer, shape) per job) or to freshly allocated buffers."""
        nb = _Batch(jobs, outs=outs)
        _check(load().hsz_plan_update(self.handle, nb.items, len(nb.jobs)), "plan_update")
        self.batch = nb

    def launch(self):
        _check(load().hsz_plan_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)), "plan_launch")

    def results(self):
        self.stream.synchronize()
        st = read_status(self.ws, self.stream)
        if st != OK:
            raise HszError(st, "plan")
        return self.batch.outputs()

    def close(self):
        if getattr(self, "handle", None):
            load().hsz_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- slabs and out-of-core operations (Alg. 3's window over host-resident slabs) ------

def extremes(x: torch.Tensor, stream=None):
    """(vmin, vmax, has_nonfinite) of a contiguous float32/float64 GPU tensor."""
    lib = load()
    dt = F32 if x.dtype == torch.float32 else F64
    wsb = ctypes.c_uint64()
    _check(lib.hsz_extremes_workspace(ctypes.byref(wsb)), "extremes_workspace")
    ws = workspace(wsb.value, x.device, key="extremes")
    out = torch.empty(4, dtype=torch.float64, device=x.device)
    _check(lib.hsz_extremes(ctypes.c_void_p(x.data_ptr()), dt, x.numel(), ctypes.c_void_p(out.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(_stream(stream))),
           "extremes")
    v = out.cpu().tolist()
    return v[0], v[1], bool(v[2])


def compress_range(x: torch.Tensor, eb: float, vmin: float, vmax: float, rel: bool = True, block: int = 32,
                   stream=None, mean_dec: bool = False, lorenzo: bool = False,
                   inter_block: bool = False) -> Compressed:
    """Compress one slab of a larger field with the whole field's quantizer:
    eps and the quantum come from the field's extremes [vmin, vmax]; the
    decorrelation as in compress()."""
    lib = load()
    if int(bool(mean_dec)) + int(bool(lorenzo)) + int(bool(inter_block)) > 1:
        raise ValueError("at most one of mean_dec, lorenzo, inter_block")
    flags = FLAG_BLOCK_MEAN if mean_dec else (FLAG_LORENZO if lorenzo else (FLAG_INTER_BLOCK if inter_block else 0))
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous GPU tensor")
    dt = F32 if x.dtype == torch.float32 else F64
    shape = tuple(x.shape)
    dims = _dims(shape)
    out = _empty_bytes(compress_bound(shape, dt, block), x.device)
    wsb = ctypes.c_uint64()
    _check(lib.hsz_compress_workspace_mode(len(shape), dims, block, flags, ctypes.byref(wsb)), "compress_workspace")
    ws = workspace(wsb.value, x.device, key="compress")
    _check(lib.hsz_compress_range(ctypes.c_void_p(x.data_ptr()), dt, len(shape), dims, float(eb), int(rel),
                                  float(vmin), float(vmax), block, flags,
                                  ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel(), ctypes.c_void_p(_stream(stream))), "compress_range")
    st = read_status(ws, stream)
    if st != OK:
        raise HszError(st, "compress_range")
    return Compressed(out, read_header(out))


def compress_slabs(x: torch.Tensor, eb: float, planes: int, rel: bool = True, block: int = 32,
                   mean_dec: bool = False, device="cuda", lorenzo: bool = False, inter_block: bool = False):
    """Compress a host-resident field slab by slab (ranges of 'planes' indices
    of its slowest axis) with the whole field's quantizer, keeping only one
    slab on the device at a time: a first pass reduces the extremes, a
    second compresses.  Returns [(pinned host uint8 tensor, Header)]."""
    if x.is_cuda:
        raise ValueError("x must be a host tensor")
    n0 = x.shape[0]
    lo, hi = float("inf"), float("-inf")
    for a in range(0, n0, planes):
        vmin, vmax, bad = extremes(x[a:a + planes].contiguous().to(device))
        if bad:
            raise HszError(ERR_NONFINITE, "compress_slabs")
        lo, hi = min(lo, vmin), max(hi, vmax)
    out = []
    for a in range(0, n0, planes):
        c = compress_range(x[a:a + planes].contiguous().to(device), eb, lo, hi, rel=rel, block=block,
                           mean_dec=mean_dec, lorenzo=lorenzo, inter_block=inter_block)
        nbytes = int(c.header.total_bytes)
        host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        host.copy_(c.data[:nbytes])
        out.append((host, c.header))
    return out


def ooc_workspace_bytes(slabs, op) -> int:
    """Workspace (bytes) an out-of-core operation over these slabs needs."""
    hdrs = [h for _, h in slabs]
    harr = _headers_array(hdrs)
    wsb = ctypes.c_uint64()
    _check(load().hsz_ooc_workspace(ctypes.cast(harr, ctypes.c_void_p), len(slabs), _OPS.get(op, op),
                                    ctypes.byref(wsb)), "ooc_workspace")
    return wsb.value


def ooc_op(slabs, op, via=QUANT, axis: int = 0, stream=None, device="cuda"):
    """An operation on the field held as host-resident compressed slabs
    (compress_slabs), streamed through the device: a stats dict for mean /
    var, else a pinned host tensor shaped like the whole field."""
    lib = load()
    op = _OPS.get(op, op)
    via = _STAGES.get(via, via)
    hdrs = [h for _, h in slabs]
    harr = _headers_array(hdrs)
    ptrs = (ctypes.c_void_p * len(slabs))(*[t.data_ptr() for t, _ in slabs])
    wsb = ctypes.c_uint64()
    _check(lib.hsz_ooc_workspace(ctypes.cast(harr, ctypes.c_void_p), len(slabs), op, ctypes.byref(wsb)),
           "ooc_workspace")
    ws = workspace(wsb.value, torch.device(device), key="ooc")
    h0 = hdrs[0]
    if op in _STATS:
        res = torch.empty(48, dtype=torch.uint8, pin_memory=True)
    else:
        shape = (sum(int(h.dims[0]) for h in hdrs),) + tuple(h0.shape[1:])
        n = 1
        for v in shape:
            n *= v
        res = torch.empty(n * (4 if h0.dtype == F32 else 8), dtype=torch.uint8, pin_memory=True)
    _check(lib.hsz_ooc_op(ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(harr, ctypes.c_void_p), len(slabs), via,
                          op, axis, ctypes.c_void_p(res.data_ptr()), res.numel(), ctypes.c_void_p(ws.data_ptr()),
                          ws.numel(), ctypes.c_void_p(_stream(stream))), "ooc_op")
    if op in _STATS:
        return _stats_from_raw(res.numpy().tobytes())
    return res.view(h0.torch_dtype).view(shape)


# ---- contexts: persistent scratch, pinned staging and streams (hsz_ctx) ---------------

class _DevBuf:
    """A device buffer the library owns, in the form the wrappers above take
    for a workspace (data_ptr, numel in bytes)."""

    def __init__(self, ptr: int, nbytes: int):
        self._ptr, self._n = int(ptr or 0), int(nbytes)

    def data_ptr(self) -> int:
        return self._ptr

    def numel(self) -> int:
        return self._n


class Context:
    """One device's hsz_ctx: a device scratch buffer that is the workspace of
    every call made through this object, a ring of pinned host memory through
    which batch tables reach the device, the out-of-core copy stream, and
    stored launch shapes.  The calls return once their work is enqueued:
    none waits on the host unless the scratch must grow (reserve() it up
    front) or the staging ring is exhausted.  Results of statistics are read
    after the stream has completed (status(), or outputs() of a batch)."""

    def __init__(self, scratch_bytes: int = 256 << 20, host_bytes: int = 4 << 20, device=None):
        lib = load()
        self.device = torch.device(device if device is not None else "cuda")
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.hsz_ctx_create(int(scratch_bytes), int(host_bytes), ctypes.byref(h)), "ctx_create")
        self.handle = h

    @property
    def scratch(self) -> _DevBuf:
        p, n = ctypes.c_void_p(), ctypes.c_uint64()
        _check(load().hsz_ctx_scratch(self.handle, ctypes.byref(p), ctypes.byref(n)), "ctx_scratch")
        return _DevBuf(p.value, n.value)

    def reserve(self, nbytes: int):
        """Grow the scratch to nbytes (waits for the context's work if it grows)."""
        _check(load().hsz_ctx_reserve(self.handle, int(nbytes)), "ctx_reserve")

    def decompress_to_stage(self, c: Compressed, stage, out: torch.Tensor, stream=None):
        return decompress_to_stage(c, stage, stream=stream, out=out, ws=self.scratch)

    def op_fused(self, c: Compressed, via, op, out: torch.Tensor, axis: int = 0, box=None, stream=None):
        return op_fused(c, via, op, axis=axis, box=box, stream=stream, check=False, out=out, ws=self.scratch,
                        raw=True)

    def op_on_stage(self, stage_buf, h: Header, stage, op, out: torch.Tensor, axis: int = 0, box=None, stream=None):
        return op_on_stage(stage_buf, h, stage, op, axis=axis, box=box, stream=stream, check=False, out=out,
                           ws=self.scratch, raw=True)

    def batch_run(self, jobs, tune: dict | None = None, stream=None, outs=None,
                  status: torch.Tensor | None = None) -> "_Batch":
        """Enqueue one pass over the jobs (results into 'outs', (buffer, shape)
        per job, or fresh buffers); call .outputs() of the returned batch after
        the stream has completed.  status: a device int32 that receives the
        pass's status word."""
        b = _Batch(jobs, outs=outs)
        _check(load().hsz_ctx_batch_run(self.handle, b.items, len(b.jobs), _tuning(tune),
                                        None if status is None else ctypes.c_void_p(status.data_ptr()),
                                        ctypes.c_void_p(_stream(stream))), "ctx_batch_run")
        return b

    def ooc_op(self, slabs, op, via=QUANT, axis: int = 0, stream=None, out: torch.Tensor | None = None,
               status: torch.Tensor | None = None) -> torch.Tensor:
        """Enqueue an out-of-core operation (see ooc_op); returns the pinned
        host tensor the result lands in once the stream reaches this point:
        48 raw bytes of statistics (stats_of_host) or the field's result."""
        lib = load()
        op = _OPS.get(op, op)
        via = _STAGES.get(via, via)
        hdrs = [h for _, h in slabs]
        harr = _headers_array(hdrs)
        ptrs = (ctypes.c_void_p * len(slabs))(*[t.data_ptr() for t, _ in slabs])
        h0 = hdrs[0]
        if out is None:
            if op in _STATS:
                out = torch.empty(48, dtype=torch.uint8, pin_memory=True)
            else:
                n = sum(int(h.dims[0]) for h in hdrs)
                for v in h0.shape[1:]:
                    n *= int(v)
                out = torch.empty(n * (4 if h0.dtype == F32 else 8), dtype=torch.uint8, pin_memory=True)
        self._keep = (ptrs, harr, hdrs, slabs)  # alive until the next call
        _check(lib.hsz_ooc_op_async(self.handle, ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(harr, ctypes.c_void_p),
                                    len(slabs), via, op, axis, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                    None if status is None else ctypes.c_void_p(status.data_ptr()),
                                    ctypes.c_void_p(_stream(stream))), "ooc_op_async")
        return out

    def status(self, stream=None) -> int:
        """The status word of the last call made through the context
        (synchronises the stream)."""
        return read_status(self.scratch, stream)

    def set_tuning(self, key: str, tune: dict):
        _check(load().hsz_ctx_set_tuning(self.handle, key.encode(), _tuning(tune)), "ctx_set_tuning")

    def get_tuning(self, key: str):
        t = Tuning()
        rc = load().hsz_ctx_get_tuning(self.handle, key.encode(), ctypes.byref(t))
        if rc != OK:
            return None
        return {f: int(getattr(t, f)) for f, _ in Tuning._fields_}

    def close(self):
        if getattr(self, "handle", None):
            load().hsz_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stats_of_host(raw: torch.Tensor) -> dict:
    """Statistics from the 48 raw bytes an out-of-core call left in host memory."""
    return _stats_from_raw(raw[:48].numpy().tobytes())
