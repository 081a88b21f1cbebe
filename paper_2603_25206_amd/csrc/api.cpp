// api.cpp -- the C ABI of libhsz (declared in include/hsz.h): argument and
// stream validation on the host, then stream-ordered kernel launches.
#include "abi_util.hpp"
#include "hsz_nd.hpp"

namespace hsz_abi {
int& last_hip() {
  thread_local int v = 0;
  return v;
}
}  // namespace hsz_abi

namespace {

using namespace hsz_abi;

__global__ void k_reset_status(int* status) {
  if (threadIdx.x == 0) *status = 0;
}

// Stage 1 supports one operation: the mean of a block-mean stream over the
// whole field (Eq. (mean_m)).
bool meta_mean_ok(const hsz_header* h, int op, const hsz::OpTarget& t) {
  const hsz::Box3& b = t.box;
  const bool whole = b.z0 == 0 && b.y0 == 0 && b.x0 == 0 && b.z1 == t.d.z && b.y1 == t.d.y && b.x1 == t.d.x;
  return (h->flags & HSZ_FLAG_BLOCK_MEAN) && op == HSZ_MEAN && whole;
}

bool is_stats(int op) { return op == HSZ_MEAN || op == HSZ_VAR || op == HSZ_VAR_MT; }

bool whole_box(const hsz::Box3& b, const hsz::Dims3& d) {
  return b.z0 == 0 && b.y0 == 0 && b.x0 == 0 && b.z1 == d.z && b.y1 == d.y && b.x1 == d.x;
}
bool whole_box(const hsz::OpTarget& t) { return whole_box(t.box, t.d); }

// the Lorenzo family: HSZp-nd (nd blocks) and HSZp (deltas across the blocks
// of the flat field); neither stores metadata
bool is_nd(const hsz_header* h) { return (h->flags & (HSZ_FLAG_LORENZO | HSZ_FLAG_INTER_BLOCK)) != 0; }
bool is_flat(const hsz_header* h) { return (h->flags & HSZ_FLAG_INTER_BLOCK) != 0; }

hsz::NdGrid grid_of(const hsz_header* h) {
  if (is_flat(h)) return hsz::flat_grid(h->n, h->block);
  int64_t d3[3], n;
  dims3_of(h->ndim, h->dims, d3, &n);
  return hsz::nd_grid(d3, h->ndim, h->block);
}

// tile sums of the device-wide scan of HSZp's single row (stages 3 and 4)
// HSZp: tile sums of the flat row's scan; HSZp-nd: the z segments' totals of
// the two-pass D_q (rows of at most 512 columns)
uint64_t lz_tmp_bytes(const hsz_header* h) {
  if (is_flat(h)) return hsz::lz_scan_tmp_bytes(h->n);
  return is_nd(h) ? hsz::lz_dq_tmp_bytes(grid_of(h)) : 0;
}

// HSZp-nd streams: the fused routes and the D_p operations rebuild a stage
// in scratch memory after the operation's own workspace (4 bytes per point,
// 8 for the binary64 floats of stage 4).
uint64_t nd_scratch_off(const hsz_header* h) {
  const uint64_t a = hsz::op_workspace_bytes(), b = hsz::grad_workspace_bytes(h->nb);
  return ((a > b ? a : b) + 255) / 256 * 256;
}
uint64_t nd_scratch_bytes(const hsz_header* h) {
  return ((h->dtype == HSZ_F64 ? 8 : 4) * (uint64_t)h->n + 255) / 256 * 256;
}
uint64_t nd_workspace(const hsz_header* h) { return nd_scratch_off(h) + nd_scratch_bytes(h) + lz_tmp_bytes(h); }
// the Laplacian on D_p of an HSZp-nd stream also keeps one int32 field per
// axis (the prefix sums of p over the other axes)
uint64_t nd_lap_bytes(const hsz_header* h) { return ((4 * (uint64_t)h->n + 255) / 256 * 256) * (uint64_t)h->ndim; }
uint64_t nd_workspace_op(const hsz_header* h, int op) {
  return nd_workspace(h) + (op == HSZ_LAPLACIAN && !is_flat(h) ? nd_lap_bytes(h) : 0);
}
bool is_stencil(int op) { return op >= HSZ_DERIV && op <= HSZ_LAPLACIAN; }

// The spread about the integer metadata mean (Sec. V-A, standard deviation
// on D_p of HSZx) needs the block means of every block: block-mean streams,
// whole field, through stage 2 (or 3 in the fused path, whose stream still
// holds the metadata).
bool var_mt_ok(const hsz_header* h, const hsz::OpTarget& t, int stage, bool fused) {
  const hsz::Box3& b = t.box;
  const bool whole = b.z0 == 0 && b.y0 == 0 && b.x0 == 0 && b.z1 == t.d.z && b.y1 == t.d.y && b.x1 == t.d.x;
  return (h->flags & HSZ_FLAG_BLOCK_MEAN) && whole && (stage == HSZ_DELTA || (fused && stage == HSZ_QUANT));
}

// The integer Laplacian numerator is a sum of 12 terms of |q| in 32 bits.
constexpr uint32_t kLapMaxQ = 1u << 27;

int reset_status(void* ws, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, (int*)ws);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int op_common(const hsz_header* h, int op, int axis, const hsz_box* box, uint64_t cap, void* d_result,
              void* d_ws, uint64_t ws_bytes, hsz::OpTarget* t, int* axis3) {
  int rc = check_header(h);
  if (rc) return rc;
  if (!is_stats(op) && !is_stencil(op)) return HSZ_ERR_INVALID_ARG;
  if (!d_result || !d_ws || !aligned16(d_ws)) return HSZ_ERR_INVALID_ARG;
  if (ws_bytes < hsz::op_workspace_bytes()) return HSZ_ERR_CAPACITY;
  int64_t d3[3], n;
  dims3_of(h->ndim, h->dims, d3, &n);
  t->d = hsz::Dims3{d3[0], d3[1], d3[2]};
  if (!box3_of(h, box, &t->box)) return HSZ_ERR_INVALID_ARG;
  if (op == HSZ_DERIV) {
    if (axis < 0 || axis >= h->ndim) return HSZ_ERR_INVALID_ARG;
    *axis3 = axis + 3 - h->ndim;
  } else {
    *axis3 = 0;
  }
  if (is_stencil(op) && ws_bytes < hsz::grad_workspace_bytes(h->nb)) return HSZ_ERR_CAPACITY;
  const uint64_t esz = h->dtype == HSZ_F32 ? 4 : 8;
  const uint64_t need = is_stats(op) ? sizeof(hsz_stats) : esz * (uint64_t)t->box.volume();
  if (cap < need) return HSZ_ERR_CAPACITY;
  if (is_stencil(op) && !aligned16(d_result)) return HSZ_ERR_INVALID_ARG;
  return HSZ_OK;
}

// Operations on HSZp-nd streams.  d_c != nullptr: fused from the stream
// through 'stage' (decoded into the scratch area as far as needed); else on
// the caller's stage buffer d_stage.  Stage 2 (D_p, whole field): the mean
// with nd weights, Alg. 4 and Eq. (derivative_Dp) along any axis; stages 3
// and 4 hold the field's layout, so the kernels of delta streams apply.
int nd_op(const void* d_c, const void* d_stage, const hsz_header* h, int stage, int op, int axis3,
          const hsz::OpTarget& t, void* d_result, void* d_ws, uint64_t ws_bytes, hipStream_t s) {
  if (stage == HSZ_META) return HSZ_ERR_UNSUPPORTED;  // no metadata
  if (stage < HSZ_DELTA || stage > HSZ_FLOAT) return HSZ_ERR_INVALID_ARG;
  if (op == HSZ_VAR_MT) return HSZ_ERR_UNSUPPORTED;  // block-mean streams only
  // on D_p: the whole field; the derivative for HSZp-nd only (a 1D partition
  // keeps no multidimensional layout)
  const bool dp_stencil = (op == HSZ_DERIV || op == HSZ_LAPLACIAN) && !is_flat(h);
  if (stage == HSZ_DELTA && (!whole_box(t) || !(op == HSZ_MEAN || op == HSZ_VAR || dp_stencil)))
    return HSZ_ERR_UNSUPPORTED;
  if (op == HSZ_LAPLACIAN && stage <= HSZ_QUANT && h->max_abs_q >= kLapMaxQ) return HSZ_ERR_UNSUPPORTED;
  if (ws_bytes < (stage == HSZ_DELTA ? nd_workspace_op(h, op) : nd_workspace(h))) return HSZ_ERR_CAPACITY;
  uint8_t* ws = (uint8_t*)d_ws;
  int32_t* scratch = (int32_t*)(ws + nd_scratch_off(h));
  int32_t* tmp = lz_tmp_bytes(h) ? (int32_t*)(ws + nd_scratch_off(h) + nd_scratch_bytes(h)) : nullptr;
  const hsz::StreamView v = view_of(d_c, h);
  const hsz::NdGrid g = grid_of(h);
  int rc = reset_status(d_ws, s);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  if (stage == HSZ_DELTA && !is_stencil(op)) {
    e = hsz::launch_lz_stats(d_c ? nullptr : (const int32_t*)d_stage, v, g, op, d_result, ws, scratch, tmp, s);
  } else if (stage == HSZ_DELTA) {
    const int32_t* p = (const int32_t*)d_stage;
    if (d_c) {
      e = hsz::lz_decode(v, g, HSZ_DELTA, scratch, (int*)d_ws, tmp, s);
      p = scratch;
    }
    if (e == hipSuccess && op == HSZ_DERIV) e = hsz::lz_deriv_p(p, v, g, axis3, d_result, s);
    if (e == hipSuccess && op == HSZ_LAPLACIAN)
      e = hsz::lz_laplacian_p(p, g, h->quantum, h->dtype, (int32_t*)(ws + nd_workspace(h)), d_result, s);
  } else {
    const void* buf = d_stage;
    if (d_c) {
      e = hsz::lz_decode(v, g, stage, scratch, (int*)d_ws, tmp, s);
      buf = scratch;
    }
    if (e == hipSuccess)
      e = is_stats(op) ? hsz::launch_stats_stage(buf, stage, v, op, t, d_result, ws, s)
                       : hsz::launch_grad_stage(buf, stage, v, op, axis3, t, d_result, ws, s);
  }
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

}  // namespace

extern "C" {

const char* hsz_strerror(int code) {
  switch (code) {
    case HSZ_OK: return "ok";
    case HSZ_ERR_INVALID_ARG: return "invalid argument";
    case HSZ_ERR_BAD_STREAM: return "corrupt or truncated compressed stream";
    case HSZ_ERR_UNSUPPORTED: return "operation or block size not supported at this stage";
    case HSZ_ERR_RANGE: return "quantization integer out of range (|q| > 2^29 - 1)";
    case HSZ_ERR_EB: return "error bound not positive or below the field's floating-point spacing";
    case HSZ_ERR_NONFINITE: return "non-finite value in the input field";
    case HSZ_ERR_CAPACITY: return "buffer too small";
    case HSZ_ERR_HIP: return "HIP runtime error";
  }
  return "unknown error";
}

int hsz_version(void) { return 100; }

int hsz_last_hip_error(void) { return hsz_abi::last_hip(); }

int hsz_read_status(const void* d_workspace, void* stream, int* h_status) {
  if (!d_workspace || !h_status) return HSZ_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  int st = 0;
  e = hipMemcpy(&st, d_workspace, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  *h_status = st;
  return HSZ_OK;
}

int hsz_compress_bound(int dtype, int ndim, const int64_t* h_dims, int block, uint64_t* h_bytes) {
  int64_t d3[3], n;
  if (!h_bytes || (dtype != HSZ_F32 && dtype != HSZ_F64) || !dims3_of(ndim, h_dims, d3, &n))
    return HSZ_ERR_INVALID_ARG;
  if (!valid_block(block)) return HSZ_ERR_UNSUPPORTED;
  // the larger of the 1D partition and (2D / 3D fields) the nd partition
  const uint64_t per_block = 4 * (uint64_t)((block / 32) * (1 + hsz::kMaxWidth));
  const hsz::Layout L = hsz::make_layout(n, block);
  uint64_t bound = L.off_payload + per_block * (uint64_t)L.nb;
  if (ndim >= 2) {
    const hsz::Layout Ln = hsz::make_layout_nd(d3, ndim, block);
    const uint64_t bn = Ln.off_payload + per_block * (uint64_t)Ln.nb;
    bound = bn > bound ? bn : bound;
  }
  *h_bytes = bound;
  return HSZ_OK;
}

int hsz_compress_workspace(int ndim, const int64_t* h_dims, int block, uint64_t* h_bytes) {
  int64_t d3[3], n;
  if (!h_bytes || !dims3_of(ndim, h_dims, d3, &n)) return HSZ_ERR_INVALID_ARG;
  if (!valid_block(block)) return HSZ_ERR_UNSUPPORTED;
  uint64_t w = hsz::compress_workspace_bytes(hsz::make_layout(n, block));
  const uint64_t wf = hsz::compress_workspace_bytes_nd(hsz::make_layout_flat(n, block));
  w = wf > w ? wf : w;
  if (ndim >= 2) {
    const uint64_t wn = hsz::compress_workspace_bytes_nd(hsz::make_layout_nd(d3, ndim, block));
    w = wn > w ? wn : w;
  }
  *h_bytes = w;
  return HSZ_OK;
}

int hsz_compress_workspace_mode(int ndim, const int64_t* h_dims, int block, uint32_t flags, uint64_t* h_bytes) {
  int64_t d3[3], n;
  if (!h_bytes || !dims3_of(ndim, h_dims, d3, &n)) return HSZ_ERR_INVALID_ARG;
  if (flags != 0 && flags != HSZ_FLAG_BLOCK_MEAN && flags != HSZ_FLAG_LORENZO && flags != HSZ_FLAG_INTER_BLOCK)
    return HSZ_ERR_INVALID_ARG;
  if (!valid_block(block)) return HSZ_ERR_UNSUPPORTED;
  if (flags == HSZ_FLAG_LORENZO && ndim < 2) return HSZ_ERR_UNSUPPORTED;
  *h_bytes = flags == HSZ_FLAG_LORENZO       ? hsz::compress_workspace_bytes_nd(hsz::make_layout_nd(d3, ndim, block))
             : flags == HSZ_FLAG_INTER_BLOCK ? hsz::compress_workspace_bytes_nd(hsz::make_layout_flat(n, block))
                                             : hsz::compress_workspace_bytes(hsz::make_layout(n, block));
  return HSZ_OK;
}

int hsz_compress(const void* d_x, int dtype, int ndim, const int64_t* h_dims, double eb, int eb_is_rel, int block,
                 void* d_out, uint64_t cap, void* d_workspace, uint64_t workspace_bytes, void* stream) {
  return hsz_compress_flags(d_x, dtype, ndim, h_dims, eb, eb_is_rel, block, 0u, d_out, cap, d_workspace,
                            workspace_bytes, stream);
}

static int compress_impl(const void* d_x, int dtype, int ndim, const int64_t* h_dims, double eb, int eb_is_rel,
                         int block, uint32_t flags, int fixed, double vmin, double vmax, void* d_out, uint64_t cap,
                         void* d_workspace, uint64_t workspace_bytes, void* stream) {
  int64_t d3[3], n;
  if (flags != 0 && flags != HSZ_FLAG_BLOCK_MEAN && flags != HSZ_FLAG_LORENZO && flags != HSZ_FLAG_INTER_BLOCK)
    return HSZ_ERR_INVALID_ARG;
  if (!d_x || !d_out || !d_workspace || (dtype != HSZ_F32 && dtype != HSZ_F64) || !dims3_of(ndim, h_dims, d3, &n))
    return HSZ_ERR_INVALID_ARG;
  if (!aligned16(d_x) || !aligned16(d_out) || !aligned16(d_workspace)) return HSZ_ERR_INVALID_ARG;
  if (!valid_block(block)) return HSZ_ERR_UNSUPPORTED;
  if (flags == HSZ_FLAG_LORENZO && ndim < 2) return HSZ_ERR_UNSUPPORTED;  // the nd partition needs 2D / 3D
  if (!(eb > 0.0) || eb != eb || eb > 1e300) return HSZ_ERR_EB;
  hsz::Layout L = flags == HSZ_FLAG_LORENZO       ? hsz::make_layout_nd(d3, ndim, block)
                  : flags == HSZ_FLAG_INTER_BLOCK ? hsz::make_layout_flat(n, block)
                                                  : hsz::make_layout(n, block);
  const bool lorenzo = flags == HSZ_FLAG_LORENZO || flags == HSZ_FLAG_INTER_BLOCK;
  if (workspace_bytes < (lorenzo ? hsz::compress_workspace_bytes_nd(L) : hsz::compress_workspace_bytes(L)))
    return HSZ_ERR_CAPACITY;
  if (cap < L.off_payload) return HSZ_ERR_CAPACITY;
  hsz::CompressArgs a;
  a.x = d_x;
  a.dtype = dtype;
  a.ndim = ndim;
  a.dims[0] = d3[0];
  a.dims[1] = d3[1];
  a.dims[2] = d3[2];
  a.eb = eb;
  a.eb_is_rel = eb_is_rel ? 1 : 0;
  a.flags = flags;
  a.fixed_range = fixed;
  a.vmin = vmin;
  a.vmax = vmax;
  a.lay = L;
  a.out = (uint8_t*)d_out;
  a.cap = cap;
  a.ws = (uint8_t*)d_workspace;
  a.ws_bytes = workspace_bytes;
  hipError_t e = lorenzo ? hsz::launch_compress_nd(a, (hipStream_t)stream)
                     : hsz::launch_compress(a, (hipStream_t)stream);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int hsz_compress_flags(const void* d_x, int dtype, int ndim, const int64_t* h_dims, double eb, int eb_is_rel,
                       int block, uint32_t flags, void* d_out, uint64_t cap, void* d_workspace,
                       uint64_t workspace_bytes, void* stream) {
  return compress_impl(d_x, dtype, ndim, h_dims, eb, eb_is_rel, block, flags, 0, 0.0, 0.0, d_out, cap, d_workspace,
                       workspace_bytes, stream);
}

int hsz_compress_range(const void* d_x, int dtype, int ndim, const int64_t* h_dims, double eb, int eb_is_rel,
                       double vmin, double vmax, int block, uint32_t flags, void* d_out, uint64_t cap,
                       void* d_workspace, uint64_t workspace_bytes, void* stream) {
  if (!(vmin <= vmax) || vmin != vmin || vmax != vmax || vmin - vmin != 0.0 || vmax - vmax != 0.0)
    return HSZ_ERR_INVALID_ARG;
  return compress_impl(d_x, dtype, ndim, h_dims, eb, eb_is_rel, block, flags, 1, vmin, vmax, d_out, cap,
                       d_workspace, workspace_bytes, stream);
}

int hsz_read_header(const void* h_bytes, uint64_t len, uint64_t len_stream, hsz_header* o) {
  if (!h_bytes || !o) return HSZ_ERR_INVALID_ARG;
  if (len < HSZ_HEADER_BYTES) return HSZ_ERR_BAD_STREAM;
  const uint8_t* p = (const uint8_t*)h_bytes;
  if (memcmp(p, "HSZ1", 4) != 0 || rd16(p + 4) != 1) return HSZ_ERR_BAD_STREAM;
  hsz_header h;
  memset(&h, 0, sizeof h);
  h.dtype = p[6];
  h.ndim = p[7];
  if (h.dtype != HSZ_F32 && h.dtype != HSZ_F64) return HSZ_ERR_BAD_STREAM;
  if (h.ndim < 1 || h.ndim > 3) return HSZ_ERR_BAD_STREAM;
  uint64_t d3[3] = {rd64(p + 8), rd64(p + 16), rd64(p + 24)};
  for (int k = 0; k < 3 - h.ndim; ++k)
    if (d3[k] != 1) return HSZ_ERR_BAD_STREAM;
  for (int k = 0; k < h.ndim; ++k) {
    if (d3[3 - h.ndim + k] > (uint64_t(1) << 40)) return HSZ_ERR_BAD_STREAM;
    h.dims[k] = (int64_t)d3[3 - h.ndim + k];
  }
  h.n = (int64_t)rd64(p + 32);
  h.block = (int32_t)rd32(p + 40);
  h.chunk_blocks = (int32_t)rd32(p + 44);
  h.eb_abs = rdf64(p + 48);
  h.quantum = rdf64(p + 56);
  h.inv_quantum = rdf64(p + 64);
  h.vmin = rdf64(p + 72);
  h.vmax = rdf64(p + 80);
  h.max_abs_q = rd32(p + 88);
  h.flags = rd32(p + 92);
  if (h.flags != 0 && h.flags != HSZ_FLAG_BLOCK_MEAN && h.flags != HSZ_FLAG_LORENZO &&
      h.flags != HSZ_FLAG_INTER_BLOCK)
    return HSZ_ERR_BAD_STREAM;
  h.nb = (int64_t)rd64(p + 96);
  h.nchunks = (int64_t)rd64(p + 104);
  h.off_chunk = rd64(p + 112);
  h.off_q0 = rd64(p + 120);
  h.off_width = rd64(p + 128);
  h.off_payload = rd64(p + 136);
  h.payload_words = rd64(p + 144);
  h.total_bytes = rd64(p + 152);
  if (h.chunk_blocks != hsz::kChunkBlocks || h.block < 1 || h.block > 64) return HSZ_ERR_BAD_STREAM;
  if (h.inv_quantum != 1.0 / h.quantum) return HSZ_ERR_BAD_STREAM;
  int64_t dd[3], n;
  if (!dims3_of(h.ndim, h.dims, dd, &n) || n != h.n) return HSZ_ERR_BAD_STREAM;
  if (!(h.quantum > 0.0) || h.max_abs_q > (uint32_t)hsz::kQMax) return HSZ_ERR_BAD_STREAM;
  // the layout follows from n and S (the 1D partition) or from the dims and S
  // (the nd partition of HSZp-nd, which has no q0 section)
  if (h.flags == HSZ_FLAG_LORENZO && (h.ndim < 2 || (h.block != 32 && h.block != 64))) return HSZ_ERR_BAD_STREAM;
  const hsz::Layout L = h.flags == HSZ_FLAG_LORENZO       ? hsz::make_layout_nd(dd, h.ndim, h.block)
                        : h.flags == HSZ_FLAG_INTER_BLOCK ? hsz::make_layout_flat(h.n, h.block)
                                                          : hsz::make_layout(h.n, h.block);
  const int64_t nb = L.nb;
  const uint64_t op = L.off_payload;
  if (h.nb != L.nb || h.nchunks != L.nchunks || h.off_chunk != L.off_chunk || h.off_q0 != L.off_q0 ||
      h.off_width != L.off_width || h.off_payload != L.off_payload)
    return HSZ_ERR_BAD_STREAM;
  if (h.payload_words > (uint64_t)nb * 64 || h.total_bytes != op + 4 * h.payload_words) return HSZ_ERR_BAD_STREAM;
  if (h.total_bytes > len_stream) return HSZ_ERR_BAD_STREAM;
  *o = h;
  return HSZ_OK;
}

int hsz_stage_bytes(const hsz_header* h, int stage, uint64_t* h_bytes) {
  if (!h || !h_bytes) return HSZ_ERR_INVALID_ARG;
  const uint64_t n = (uint64_t)h->n, nb = (uint64_t)h->nb;
  const bool nd = is_nd(h);  // HSZp-nd and HSZp: no metadata
  switch (stage) {
    case HSZ_META:
      if (nd) return HSZ_ERR_UNSUPPORTED;
      *h_bytes = 4 * nb;
      return HSZ_OK;
    case HSZ_DELTA: *h_bytes = 4 * n + (nd ? 0 : 4 * nb); return HSZ_OK;
    case HSZ_QUANT: *h_bytes = 4 * n; return HSZ_OK;
    case HSZ_FLOAT: *h_bytes = (h->dtype == HSZ_F32 ? 4 : 8) * n; return HSZ_OK;
  }
  return HSZ_ERR_INVALID_ARG;
}

int hsz_decompress_workspace(const hsz_header* h, int stage, uint64_t* h_bytes) {
  int rc = check_header(h);
  if (rc) return rc;
  if (!h_bytes || stage < HSZ_META || stage > HSZ_FLOAT) return HSZ_ERR_INVALID_ARG;
  *h_bytes = 256 + (stage >= HSZ_QUANT ? lz_tmp_bytes(h) : 0);
  return HSZ_OK;
}

int hsz_decompress_to_stage(const void* d_c, const hsz_header* h, int stage, void* d_out, uint64_t cap,
                            void* d_workspace, uint64_t workspace_bytes, void* stream) {
  int rc = check_header(h);
  if (rc) return rc;
  if (!d_c || !d_out || !d_workspace || !aligned16(d_c) || !aligned16(d_out) || !aligned16(d_workspace))
    return HSZ_ERR_INVALID_ARG;
  uint64_t wneed = 0;
  if ((rc = hsz_decompress_workspace(h, stage, &wneed))) return rc;
  if (workspace_bytes < wneed) return HSZ_ERR_CAPACITY;
  uint64_t need = 0;
  if ((rc = hsz_stage_bytes(h, stage, &need))) return rc == HSZ_ERR_UNSUPPORTED ? rc : HSZ_ERR_INVALID_ARG;
  if (cap < need) return HSZ_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = reset_status(d_workspace, s))) return rc;
  hipError_t e = is_nd(h) ? hsz::lz_decode(view_of(d_c, h), grid_of(h), stage, d_out, (int*)d_workspace,
                                           (int32_t*)((uint8_t*)d_workspace + 256), s)
                          : hsz::launch_decode(view_of(d_c, h), stage, d_out, (int*)d_workspace, s);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int hsz_block_index_bytes(const hsz_header* h, uint64_t* h_bytes) {
  if (!h || !h_bytes) return HSZ_ERR_INVALID_ARG;
  int rc = check_header(h);
  if (rc) return rc;
  *h_bytes = 2 * (uint64_t)h->nb;
  return HSZ_OK;
}

int hsz_block_index(const void* d_c, const hsz_header* h, void* d_index, uint64_t cap, void* stream) {
  int rc = check_header(h);
  if (rc) return rc;
  if (!d_c || !d_index || !aligned16(d_c) || !aligned16(d_index)) return HSZ_ERR_INVALID_ARG;
  if (cap < 2 * (uint64_t)h->nb) return HSZ_ERR_CAPACITY;
  if (is_nd(h)) return HSZ_ERR_UNSUPPORTED;  // the index serves the fused tiles of 1D partitions
  hipError_t e = hsz::launch_block_index(view_of(d_c, h), (uint16_t*)d_index, (hipStream_t)stream);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int hsz_op_workspace(const hsz_header* h, int op, uint64_t* h_bytes) {
  if (!h || !h_bytes || (!is_stats(op) && !is_stencil(op))) return HSZ_ERR_INVALID_ARG;
  uint64_t a = hsz::op_workspace_bytes(), b = hsz::grad_workspace_bytes(h->nb);
  *h_bytes = (is_stencil(op) && b > a) ? b : a;
  if (is_nd(h)) *h_bytes = nd_workspace_op(h, op);
  return HSZ_OK;
}

int hsz_op_on_stage(const void* d_stage, const hsz_header* h, int stage, int op, int axis, const hsz_box* h_box,
                    void* d_result, uint64_t cap, void* d_workspace, uint64_t workspace_bytes, void* stream) {
  hsz::OpTarget t;
  int axis3 = 0;
  int rc = op_common(h, op, axis, h_box, cap, d_result, d_workspace, workspace_bytes, &t, &axis3);
  if (rc) return rc;
  if (!d_stage || !aligned16(d_stage)) return HSZ_ERR_INVALID_ARG;
  if (is_nd(h))
    return nd_op(nullptr, d_stage, h, stage, op, axis3, t, d_result, d_workspace, workspace_bytes, (hipStream_t)stream);
  if (stage == HSZ_META && !meta_mean_ok(h, op, t)) return HSZ_ERR_UNSUPPORTED;
  if (stage < HSZ_META || stage > HSZ_FLOAT) return HSZ_ERR_INVALID_ARG;
  if (op == HSZ_VAR_MT && !var_mt_ok(h, t, stage, false)) return HSZ_ERR_UNSUPPORTED;
  // a block-mean stream keeps no deltas between neighbours: no stencil on its stage 2
  if ((h->flags & HSZ_FLAG_BLOCK_MEAN) && is_stencil(op) && stage == HSZ_DELTA) return HSZ_ERR_UNSUPPORTED;
  // on the decorrelated stage only the derivative along the fast axis is
  // defined (the 1D partition keeps no other neighbour relation)
  if (is_stencil(op) && stage == HSZ_DELTA && !(op == HSZ_DERIV && axis3 == 2)) return HSZ_ERR_UNSUPPORTED;
  if (op == HSZ_LAPLACIAN && stage == HSZ_QUANT && h->max_abs_q >= kLapMaxQ) return HSZ_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = reset_status(d_workspace, s))) return rc;
  const hsz::StreamView v = view_of(nullptr, h);
  hipError_t e = is_stats(op)
                     ? hsz::launch_stats_stage(d_stage, stage, v, op, t, d_result, (uint8_t*)d_workspace, s)
                     : hsz::launch_grad_stage(d_stage, stage, v, op, axis3, t, d_result, (uint8_t*)d_workspace, s);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int hsz_op_fused(const void* d_c, const hsz_header* h, int via, int op, int axis, const hsz_box* h_box,
                 void* d_result, uint64_t cap, void* d_workspace, uint64_t workspace_bytes, void* stream) {
  hsz::OpTarget t;
  int axis3 = 0;
  int rc = op_common(h, op, axis, h_box, cap, d_result, d_workspace, workspace_bytes, &t, &axis3);
  if (rc) return rc;
  if (!d_c || !aligned16(d_c)) return HSZ_ERR_INVALID_ARG;
  if (is_nd(h))
    return nd_op(d_c, nullptr, h, via, op, axis3, t, d_result, d_workspace, workspace_bytes, (hipStream_t)stream);
  if (via == HSZ_META && !meta_mean_ok(h, op, t)) return HSZ_ERR_UNSUPPORTED;
  if (via < HSZ_META || via > HSZ_FLOAT) return HSZ_ERR_INVALID_ARG;
  if (op == HSZ_VAR_MT && !var_mt_ok(h, t, via, true)) return HSZ_ERR_UNSUPPORTED;
  // fused stencils decode delta streams only
  if ((h->flags & HSZ_FLAG_BLOCK_MEAN) && is_stencil(op)) return HSZ_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const hsz::StreamView v = view_of(d_c, h);
  if (is_stencil(op)) {
    if (via == HSZ_DELTA && !(op == HSZ_DERIV && axis3 == 2)) return HSZ_ERR_UNSUPPORTED;
    if (op == HSZ_LAPLACIAN && via == HSZ_QUANT && h->max_abs_q >= kLapMaxQ) return HSZ_ERR_UNSUPPORTED;
    if ((rc = reset_status(d_workspace, s))) return rc;
    hipError_t e = hsz::launch_grad_fused(v, via, op, axis3, t, d_result, (uint8_t*)d_workspace, s);
    if (e == hipErrorNotSupported) return HSZ_ERR_UNSUPPORTED;
    return e == hipSuccess ? HSZ_OK : hip_fail(e);
  }
  if ((rc = reset_status(d_workspace, s))) return rc;
  hipError_t e = hsz::launch_stats_fused(v, via, op, t, d_result, (uint8_t*)d_workspace, s);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

// ---- vector fields ------------------------------------------------------------
namespace {
// HSZp-nd components (the D_p route): the components' p and one numerator
// field per term of the largest operation on top of the common workspace
bool vec_nd(const hsz_header* const* h, int nc) {
  for (int c = 0; c < nc; ++c)
    if (h[c]->flags != HSZ_FLAG_LORENZO) return false;
  return true;
}
uint64_t field4(const hsz_header* h) { return (4 * (uint64_t)h->n + 255) / 256 * 256; }
int vec_max_terms(int nc) { return nc == 3 ? 6 : nc; }
uint64_t vec_ws(const hsz_header* const* h, int nc) {
  int64_t nb[3] = {0, 0, 0};
  for (int c = 0; c < nc; ++c) nb[c] = h[c]->nb;
  uint64_t b = hsz::vector_workspace_bytes(nb, nc);
  if (vec_nd(h, nc)) b += (uint64_t)(nc + vec_max_terms(nc)) * field4(h[0]);
  return b;
}

// Divergence / curl of an HSZp-nd vector field on D_p (whole field): the
// terms' numerators from each component's p, combined like the D_q route.
int vec_dp(const hsz::VecJob& j, const hsz_header* const* h, int nc, const int32_t* const* p, uint8_t* ws,
           hipStream_t s) {
  int tc[6], ta[6], ts[6], to[6], nout = 0;
  const int nt = hsz::vector_terms(j.op, nc, tc, ta, ts, to, &nout);
  if (nt == 0) return HSZ_ERR_INVALID_ARG;
  int64_t nb[3] = {0, 0, 0};
  for (int c = 0; c < nc; ++c) nb[c] = h[c]->nb;
  int32_t* nbuf = (int32_t*)(ws + hsz::vector_workspace_bytes(nb, nc) + (uint64_t)nc * field4(h[0]));
  void* out[3] = {j.out[0], j.out[1], j.out[2]};
  hipError_t e = hsz::lz_vector_p(p, grid_of(h[0]), nt, tc, ta, ts, to, nout, j.halfq, h[0]->dtype, nbuf, out, s);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

// Validate the component headers of a vector field and fill the job.
int vec_common(const hsz_header* const* h, int nc, int op, const hsz_box* box, void* const* d_result,
               uint64_t cap, void* d_ws, uint64_t ws_bytes, hsz::VecJob* j) {
  if (!h || nc < 1 || nc > 3 || !d_result) return HSZ_ERR_INVALID_ARG;
  if (op != HSZ_DIVERGENCE && op != HSZ_CURL) return HSZ_ERR_INVALID_ARG;
  for (int c = 0; c < nc; ++c) {
    if (!h[c]) return HSZ_ERR_INVALID_ARG;
    int rc = check_header(h[c]);
    if (rc) return rc;
  }
  const hsz_header* h0 = h[0];
  if (h0->ndim != nc) return HSZ_ERR_INVALID_ARG;  // one component per axis of the field
  if (op == HSZ_CURL && nc < 2) return HSZ_ERR_INVALID_ARG;
  for (int c = 1; c < nc; ++c) {
    if (h[c]->ndim != nc || h[c]->dtype != h0->dtype || h[c]->block != h0->block) return HSZ_ERR_INVALID_ARG;
    for (int k = 0; k < nc; ++k)
      if (h[c]->dims[k] != h0->dims[k]) return HSZ_ERR_INVALID_ARG;
  }
  if (!d_ws || !aligned16(d_ws)) return HSZ_ERR_INVALID_ARG;
  if (ws_bytes < vec_ws(h, nc)) return HSZ_ERR_CAPACITY;
  int64_t d3[3], n;
  dims3_of(h0->ndim, h0->dims, d3, &n);
  *j = hsz::VecJob{};
  j->d = hsz::Dims3{d3[0], d3[1], d3[2]};
  if (!box3_of(h0, box, &j->b)) return HSZ_ERR_INVALID_ARG;
  j->nc = nc;
  j->op = op == HSZ_DIVERGENCE ? hsz::kOpDivergence : hsz::kOpCurl;
  const int nout = (op == HSZ_CURL && nc == 3) ? 3 : 1;
  const uint64_t esz = h0->dtype == HSZ_F32 ? 4 : 8;
  if (cap < esz * (uint64_t)j->b.volume()) return HSZ_ERR_CAPACITY;
  for (int o = 0; o < nout; ++o) {
    if (!d_result[o] || !aligned16(d_result[o])) return HSZ_ERR_INVALID_ARG;
    j->out[o] = d_result[o];
  }
  for (int c = 0; c < nc; ++c) j->halfq[c] = 0.5 * h[c]->quantum;
  return HSZ_OK;
}
}  // namespace

int hsz_vector_workspace(const hsz_header* const* h, int ncomp, uint64_t* h_bytes) {
  if (!h || !h_bytes || ncomp < 1 || ncomp > 3) return HSZ_ERR_INVALID_ARG;
  for (int c = 0; c < ncomp; ++c)
    if (!h[c]) return HSZ_ERR_INVALID_ARG;
  *h_bytes = vec_ws(h, ncomp);
  return HSZ_OK;
}

int hsz_vector_op_on_stage(const void* const* d_stage, const hsz_header* const* h, int ncomp, int stage, int op,
                           const hsz_box* h_box, void* const* d_result, uint64_t cap, void* d_workspace,
                           uint64_t workspace_bytes, void* stream) {
  hsz::VecJob j;
  int rc = vec_common(h, ncomp, op, h_box, d_result, cap, d_workspace, workspace_bytes, &j);
  if (rc) return rc;
  if (!d_stage) return HSZ_ERR_INVALID_ARG;
  if (stage == HSZ_META) return HSZ_ERR_UNSUPPORTED;
  // on D_p: HSZp-nd components, whole field (Eq. (derivative_Dp) per term)
  if (stage == HSZ_DELTA && (!vec_nd(h, ncomp) || !whole_box(j.b, j.d))) return HSZ_ERR_UNSUPPORTED;
  if (stage < HSZ_DELTA || stage > HSZ_FLOAT) return HSZ_ERR_INVALID_ARG;
  for (int c = 0; c < ncomp; ++c) {
    if (!d_stage[c] || !aligned16(d_stage[c])) return HSZ_ERR_INVALID_ARG;
    j.buf[c] = d_stage[c];
  }
  hipStream_t s = (hipStream_t)stream;
  if ((rc = reset_status(d_workspace, s))) return rc;
  if (stage == HSZ_DELTA) {
    const int32_t* p[3] = {(const int32_t*)d_stage[0], ncomp > 1 ? (const int32_t*)d_stage[1] : nullptr,
                           ncomp > 2 ? (const int32_t*)d_stage[2] : nullptr};
    return vec_dp(j, h, ncomp, p, (uint8_t*)d_workspace, s);
  }
  hipError_t e = hsz::launch_vector_stage(j, stage, h[0]->dtype, s);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int hsz_vector_op_fused(const void* const* d_c, const hsz_header* const* h, int ncomp, int via, int op,
                        const hsz_box* h_box, void* const* d_result, uint64_t cap, void* d_workspace,
                        uint64_t workspace_bytes, void* stream) {
  hsz::VecJob j;
  int rc = vec_common(h, ncomp, op, h_box, d_result, cap, d_workspace, workspace_bytes, &j);
  if (rc) return rc;
  if (!d_c) return HSZ_ERR_INVALID_ARG;
  if (via == HSZ_DELTA && vec_nd(h, ncomp)) {
    // HSZp-nd: each component decoded to D_p in the workspace, then the
    // terms on D_p (whole field)
    if (!whole_box(j.b, j.d)) return HSZ_ERR_UNSUPPORTED;
    for (int c = 0; c < ncomp; ++c)
      if (!d_c[c] || !aligned16(d_c[c])) return HSZ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = reset_status(d_workspace, s))) return rc;
    int64_t nb[3] = {0, 0, 0};
    for (int c = 0; c < ncomp; ++c) nb[c] = h[c]->nb;
    uint8_t* ws = (uint8_t*)d_workspace;
    const int32_t* p[3] = {nullptr, nullptr, nullptr};
    for (int c = 0; c < ncomp; ++c) {
      int32_t* pc = (int32_t*)(ws + hsz::vector_workspace_bytes(nb, ncomp) + (uint64_t)c * field4(h[0]));
      hipError_t e = hsz::lz_decode(view_of(d_c[c], h[c]), grid_of(h[c]), HSZ_DELTA, pc, (int*)d_workspace, nullptr, s);
      if (e != hipSuccess) return hip_fail(e);
      p[c] = pc;
    }
    return vec_dp(j, h, ncomp, p, ws, s);
  }
  if (via == HSZ_META || via == HSZ_DELTA || via == HSZ_FLOAT) return HSZ_ERR_UNSUPPORTED;
  if (via != HSZ_QUANT) return HSZ_ERR_INVALID_ARG;
  for (int c = 0; c < ncomp; ++c) {
    if (!d_c[c] || !aligned16(d_c[c])) return HSZ_ERR_INVALID_ARG;
    if (h[c]->flags) return HSZ_ERR_UNSUPPORTED;  // fused windows decode delta streams
    j.v[c] = view_of(d_c[c], h[c]);
  }
  hipStream_t s = (hipStream_t)stream;
  if ((rc = reset_status(d_workspace, s))) return rc;
  hipError_t e = hsz::launch_vector_fused(j, (uint8_t*)d_workspace, s);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

}  // extern "C"
