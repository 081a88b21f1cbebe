// ooc.cpp -- operations on a field held as compressed slabs (consecutive
// ranges of its slowest axis, each an independent stream with the whole
// field's quantizer) that live in host memory and pass through the device a
// few at a time: the GPU form of the sliding window of Alg. 3, for fields
// whose compressed or decompressed form does not fit in device memory.
//
// Pipeline (one copy stream beside the caller's compute stream, events
// between them):
//   - the compressed slabs go host -> device into a ring of three buffers,
//     up to two slabs ahead of the one being decoded;
//   - statistics: the fused integer route of each slab adds (n, sum q,
//     sum q^2) into its own record; the records are combined exactly at
//     the end, so the result equals the whole field's;
//   - stencils: slab k is decoded to D_q into one of two window buffers
//     between a one-plane halo on each side (the last plane of slab k-1,
//     kept from the previous window, and the first plane of slab k+1,
//     decoded into the other window next), the stage-3 kernel runs on the
//     window with the slab as its box, and the slab of results goes device
//     -> host from one of two output buffers while the next slab computes.
// At most three compressed slabs, two windows and two output slabs are in
// device memory at any time.
#include <algorithm>
#include <vector>

#include "abi_util.hpp"
#include "ctx.hpp"
#include "hsz_nd.hpp"

using namespace hsz_abi;

namespace {

__global__ void k_ooc_reset(int* status) {
  if (threadIdx.x == 0) *status = 0;
}

uint64_t a256(uint64_t v) { return (v + 255) / 256 * 256; }

struct SlabSet {
  int K = 0, ndim = 0, dtype = 0;
  int64_t plane = 1;                   // elements per index of the slowest axis
  int64_t dims[3] = {0, 0, 0};          // the whole field's dims (its own axes)
  std::vector<int64_t> planes, first;   // per slab: its planes, its first plane
  int64_t max_planes = 0;
  uint64_t max_bytes = 0;
  uint32_t max_abs_q = 0;
  bool lz = false;         // HSZp-nd or HSZp slabs: decoded and reduced by the single-stream calls
  uint64_t lz_ws = 0;      // the workspace those calls need for the largest slab
};

bool is_stencil_op(int op) { return op == HSZ_DERIV || op == HSZ_GRADMAG || op == HSZ_LAPLACIAN; }

// The slabs must be one field cut along its slowest axis: same dtype, rank,
// block, decorrelation (delta or block-mean), quantum and other dims.
int describe(const hsz_header* const* h, int K, SlabSet* S) {
  if (!h || K < 1) return HSZ_ERR_INVALID_ARG;
  for (int k = 0; k < K; ++k) {
    if (!h[k]) return HSZ_ERR_INVALID_ARG;
    int rc = check_header(h[k]);
    if (rc) return rc;
  }
  const hsz_header* h0 = h[0];
  S->K = K;
  S->lz = (h0->flags & (HSZ_FLAG_LORENZO | HSZ_FLAG_INTER_BLOCK)) != 0;
  S->ndim = h0->ndim;
  S->dtype = h0->dtype;
  S->plane = 1;
  for (int a = 1; a < h0->ndim; ++a) S->plane *= h0->dims[a];
  int64_t total = 0;
  for (int k = 0; k < K; ++k) {
    const hsz_header* hk = h[k];
    if (hk->dtype != h0->dtype || hk->ndim != h0->ndim || hk->block != h0->block || hk->flags != h0->flags ||
        hk->quantum != h0->quantum || hk->eb_abs != h0->eb_abs)
      return HSZ_ERR_INVALID_ARG;
    for (int a = 1; a < h0->ndim; ++a)
      if (hk->dims[a] != h0->dims[a]) return HSZ_ERR_INVALID_ARG;
    S->planes.push_back(hk->dims[0]);
    S->first.push_back(total);
    total += hk->dims[0];
    if (hk->dims[0] > S->max_planes) S->max_planes = hk->dims[0];
    if (hk->total_bytes > S->max_bytes) S->max_bytes = hk->total_bytes;
    if (hk->max_abs_q > S->max_abs_q) S->max_abs_q = hk->max_abs_q;
  }
  S->dims[0] = total;
  for (int a = 1; a < h0->ndim; ++a) S->dims[a] = h0->dims[a];
  return HSZ_OK;
}

// HSZp-nd / HSZp slabs: workspace of the single-stream calls per slab (the
// statistics operation, or decoding to D_q for stencils), the largest
uint64_t lz_workspace(const hsz_header* const* h, int K, int op) {
  uint64_t need = 0;
  for (int k = 0; k < K; ++k) {
    uint64_t b = 0;
    const int rc = (op == HSZ_MEAN || op == HSZ_VAR) ? hsz_op_workspace(h[k], op, &b)
                                                     : hsz_decompress_workspace(h[k], HSZ_QUANT, &b);
    if (rc) return 0;
    need = std::max(need, b);
  }
  return need;
}

// Workspace: op workspace (status word first) | 3 compressed slabs | 2
// windows + 2 output slabs (stencils) or K statistics records | for
// HSZp-nd / HSZp slabs, the single-stream calls' workspace (its own status
// word, merged into the first after each call).
struct WsLayout {
  uint64_t cbuf[3], win[2], out[2], stats, final, lzws, total;
};

WsLayout ws_layout(const SlabSet& S, int op) {
  WsLayout L{};
  uint64_t off = a256(hsz::op_workspace_bytes());
  for (int i = 0; i < 3; ++i) {
    L.cbuf[i] = off;
    off += a256(S.max_bytes);
  }
  if (is_stencil_op(op)) {
    const uint64_t esz = S.dtype == HSZ_F32 ? 4 : 8;
    // a window: [pad | halo plane | slab planes | halo plane], the pad
    // placing the slab's first plane on a 256-byte boundary
    for (int i = 0; i < 2; ++i) {
      L.win[i] = off;
      off += a256(a256(4 * (uint64_t)S.plane) + 4 * (uint64_t)(S.max_planes + 1) * (uint64_t)S.plane);
    }
    for (int i = 0; i < 2; ++i) {
      L.out[i] = off;
      off += a256(esz * (uint64_t)S.max_planes * (uint64_t)S.plane);
    }
  } else {
    L.stats = off;
    off += a256(48 * (uint64_t)S.K);
    L.final = off;  // the combined record (asynchronous calls)
    off += 256;
  }
  L.lzws = off;
  off += a256(S.lz_ws);
  L.total = off;
  return L;
}

// the 3D view of a field of this rank with 'p' indices on its slowest axis
hsz::Dims3 view_dims(const SlabSet& S, int64_t p) {
  int64_t d[3] = {p, S.dims[1], S.dims[2]};
  int64_t d3[3], n;
  dims3_of(S.ndim, d, d3, &n);
  return hsz::Dims3{d3[0], d3[1], d3[2]};
}

// The pipeline's events: created per call (hsz_ooc_op) or borrowed from a
// context (hsz_ooc_op_async), indexed as in ctx.hpp.
struct Events {
  hipEvent_t e[kOocEvents] = {};
  bool used_set[3] = {false, false, false}, done_set[2] = {false, false};
  bool owned = false;
  hipEvent_t& h2d(int i) { return e[kOocH2d + i]; }
  hipEvent_t& used(int i) { return e[kOocUsed + i]; }
  hipEvent_t& out_ready(int i) { return e[kOocOutReady + i]; }
  hipEvent_t& out_done(int i) { return e[kOocOutDone + i]; }
  hipError_t create() {
    owned = true;
    for (int i = 0; i < kOocEvents; ++i) {
      hipError_t r = hipEventCreateWithFlags(&e[i], hipEventDisableTiming);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
  void borrow(const hipEvent_t* src) {
    for (int i = 0; i < kOocEvents; ++i) e[i] = src[i];
  }
  ~Events() {
    if (owned)
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
  }
};

// combine per-slab statistics records exactly and finish them as one
// (the device finalize's formulas, in the same order)
void combine(const std::vector<uint8_t>& rec, int K, int op, double quantum, hsz_stats* out) {
  int64_t n = 0, s1 = 0;
  unsigned __int128 s2 = 0;
  for (int k = 0; k < K; ++k) {
    hsz_stats r;
    memcpy(&r, rec.data() + 48 * (size_t)k, sizeof r);
    n += r.n;
    s1 += r.s1;
    s2 += ((unsigned __int128)(uint64_t)r.s2_hi << 64) | r.s2_lo;
  }
  hsz_stats o;
  memset(&o, 0, sizeof o);
  o.n = n;
  o.s1 = s1;
  o.mean = (double)s1 * quantum / (double)n;
  o.var = __builtin_nan("");
  if (op == HSZ_VAR) {
    o.s2_lo = (uint64_t)s2;
    o.s2_hi = (int64_t)(uint64_t)(s2 >> 64);
    const unsigned __int128 a = (unsigned __int128)(uint64_t)n * s2;
    const uint64_t m = (uint64_t)(s1 < 0 ? -s1 : s1);
    const unsigned __int128 b = (unsigned __int128)m * m;
    const unsigned __int128 d = a - b;
    const double num = (double)(uint64_t)(d >> 64) * 18446744073709551616.0 + (double)(uint64_t)d;
    if (n > 1) o.var = num / ((double)n * (double)(n - 1)) * (quantum * quantum);
  }
  *out = o;
}

// Arguments both entry points check before anything is enqueued.
int ooc_check(const void* const* h_slabs, const hsz_header* const* hdrs, int nslabs, int via, int op, int axis,
              const void* h_result, uint64_t result_bytes, SlabSet* S) {
  int rc = describe(hdrs, nslabs, S);
  if (rc) return rc;
  if (S->lz && !(S->lz_ws = lz_workspace(hdrs, nslabs, op))) return HSZ_ERR_UNSUPPORTED;
  if (!h_slabs || !h_result) return HSZ_ERR_INVALID_ARG;
  for (int k = 0; k < nslabs; ++k)
    if (!h_slabs[k]) return HSZ_ERR_INVALID_ARG;
  const bool stencil = is_stencil_op(op);
  if (!stencil && op != HSZ_MEAN && op != HSZ_VAR) return HSZ_ERR_INVALID_ARG;
  if (stencil && via != HSZ_QUANT) return HSZ_ERR_UNSUPPORTED;
  if (!stencil && via != HSZ_DELTA && via != HSZ_QUANT) return HSZ_ERR_UNSUPPORTED;
  if (op == HSZ_DERIV && (axis < 0 || axis >= S->ndim)) return HSZ_ERR_INVALID_ARG;
  if (op == HSZ_LAPLACIAN && S->max_abs_q >= (1u << 27)) return HSZ_ERR_UNSUPPORTED;
  const uint64_t esz = S->dtype == HSZ_F32 ? 4 : 8;
  const int64_t n_total = S->dims[0] * S->plane;
  if (result_bytes < (stencil ? esz * (uint64_t)n_total : sizeof(hsz_stats))) return HSZ_ERR_CAPACITY;
  return HSZ_OK;
}

// Enqueue the pass: kernels on 's', host <-> device copies on 'cs', events
// between them.  The status word is at the start of ws.  async: statistics
// are combined on the device (ws + L.final) and copied into h_result on 's',
// and the stencil results' last copies on 'cs' are joined into 's'; else the
// caller drains both streams and combines the records on the host.
// A single-stream call that refuses (HSZp-nd / HSZp slabs) leaves its code
// in *call_rc and stops the pass.
hipError_t ooc_enqueue(const void* const* h_slabs, const hsz_header* const* hdrs, const SlabSet& S, int via, int op,
                       int axis, void* h_result, uint8_t* ws, const WsLayout& L, hipStream_t s, hipStream_t cs,
                       Events& ev, bool async, int* call_rc) {
  int* status = (int*)ws;
  const int K = S.K;
  const int64_t P = S.plane;
  const bool stencil = is_stencil_op(op);
  const uint64_t esz = S.dtype == HSZ_F32 ? 4 : 8;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
    return e == hipSuccess;
  };
  auto issue = [&](int k) -> hipError_t {  // compressed slab k -> ring slot k % 3
    const int slot = k % 3;
    if (ev.used_set[slot]) {
      hipError_t r = hipStreamWaitEvent(cs, ev.used(slot), 0);
      if (r != hipSuccess) return r;
    }
    hipError_t r = hipMemcpyAsync(ws + L.cbuf[slot], h_slabs[k], hdrs[k]->total_bytes, hipMemcpyHostToDevice, cs);
    if (r != hipSuccess) return r;
    return hipEventRecord(ev.h2d(slot), cs);
  };
  auto mark_used = [&](int k) -> hipError_t {
    ev.used_set[k % 3] = true;
    return hipEventRecord(ev.used(k % 3), s);
  };
  hipLaunchKernelGGL(k_ooc_reset, dim3(1), dim3(64), 0, s, status);
  if (!chk(hipGetLastError())) return e;
  // the first copies read the ring after the reset's predecessors on 's'
  if (!chk(hipEventRecord(ev.e[kOocFinal], s)) || !chk(hipStreamWaitEvent(cs, ev.e[kOocFinal], 0))) return e;
  if (!stencil) {
    // statistics: every slab through the fused integer route, one record each
    chk(issue(0));
    if (K > 1) chk(issue(1));
    for (int k = 0; k < K && e == hipSuccess; ++k) {
      if (!chk(hipStreamWaitEvent(s, ev.h2d(k % 3), 0))) break;
      if (S.lz) {
        // the slab's own statistics through the single-stream call, then its
        // status word merged into the pass's
        const int rc = hsz_op_fused(ws + L.cbuf[k % 3], hdrs[k], via, op, 0, nullptr, ws + L.stats + 48 * (uint64_t)k,
                                    48, ws + L.lzws, S.lz_ws, s);
        if (rc) {
          *call_rc = rc;
          if (e == hipSuccess) e = hipErrorInvalidValue;
        }
        chk(hsz::launch_merge_status((const int*)(ws + L.lzws), status, s));
      } else {
        hsz::OpTarget t;
        t.d = view_dims(S, S.planes[k]);
        t.box = hsz::Box3{0, t.d.z, 0, t.d.y, 0, t.d.x};
        chk(hsz::launch_stats_fused(view_of(ws + L.cbuf[k % 3], hdrs[k]), via, op, t,
                                    ws + L.stats + 48 * (uint64_t)k, ws, s));
      }
      chk(mark_used(k));
      if (k + 2 < K) chk(issue(k + 2));
    }
    if (async && e == hipSuccess) {
      chk(hsz::launch_stats_combine(ws + L.stats, K, op, hdrs[0]->quantum, ws + L.final, s));
      chk(hipMemcpyAsync(h_result, ws + L.final, sizeof(hsz_stats), hipMemcpyDeviceToHost, s));
    }
    // the copy stream's last work (slab uploads) is joined into 's'
    if (chk(hipEventRecord(ev.e[kOocFinal], cs))) chk(hipStreamWaitEvent(s, ev.e[kOocFinal], 0));
    return e;
  }
  // stencils: windows of D_q with one-plane halos, results streamed out
  const int axis3 = op == HSZ_DERIV ? axis + 3 - S.ndim : 0;
  const int a_s = 3 - S.ndim;  // the slowest axis in the 3D view
  const uint64_t pb = 4 * (uint64_t)P;  // bytes of one plane of q
  // each window starts at its halo plane, so its slab planes (win + pb)
  // start on a 256-byte boundary
  uint8_t* win[2] = {ws + L.win[0] + (a256(pb) - pb), ws + L.win[1] + (a256(pb) - pb)};
  uint8_t* out[2] = {ws + L.out[0], ws + L.out[1]};
  hsz::StreamView vq = view_of(nullptr, hdrs[0]);
  auto decode = [&](int k, uint8_t* dst) -> bool {
    if (!chk(hipStreamWaitEvent(s, ev.h2d(k % 3), 0))) return false;
    if (S.lz) {
      // HSZp-nd / HSZp: the single-stream decode to D_q, its status merged
      const int rc = hsz_decompress_to_stage(ws + L.cbuf[k % 3], hdrs[k], HSZ_QUANT, dst,
                                             4 * (uint64_t)S.planes[k] * (uint64_t)P, ws + L.lzws, S.lz_ws, s);
      if (rc) {
        *call_rc = rc;
        if (e == hipSuccess) e = hipErrorInvalidValue;
        return false;
      }
      if (!chk(hsz::launch_merge_status((const int*)(ws + L.lzws), status, s))) return false;
    } else if (!chk(hsz::launch_decode(view_of(ws + L.cbuf[k % 3], hdrs[k]), HSZ_QUANT, dst, status, s))) {
      return false;
    }
    return chk(mark_used(k));
  };
  chk(issue(0));
  if (K > 1) chk(issue(1));
  if (e == hipSuccess) decode(0, win[0] + pb);
  if (K > 2) chk(issue(2));
  for (int k = 0; k < K && e == hipSuccess; ++k) {
    uint8_t* cur = win[k % 2];
    uint8_t* nxt = win[(k + 1) % 2];
    if (k >= 1)  // the halo before: the last plane of slab k-1, still in the other window
      chk(hipMemcpyAsync(cur, nxt + pb * (uint64_t)S.planes[k - 1], pb, hipMemcpyDeviceToDevice, s));
    if (k + 1 < K && e == hipSuccess) {
      if (!decode(k + 1, nxt + pb)) break;
      if (k + 3 < K) chk(issue(k + 3));
      // the halo after: the first plane of slab k+1
      chk(hipMemcpyAsync(cur + pb * (uint64_t)(1 + S.planes[k]), nxt + pb, pb, hipMemcpyDeviceToDevice, s));
    }
    if (e != hipSuccess) break;
    const int before = k > 0 ? 1 : 0, after = k + 1 < K ? 1 : 0;
    const int64_t wplanes = S.planes[k] + before + after;
    hsz::OpTarget t;
    t.d = view_dims(S, wplanes);
    t.box = hsz::Box3{0, t.d.z, 0, t.d.y, 0, t.d.x};
    if (a_s == 0) { t.box.z0 = before; t.box.z1 = before + S.planes[k]; }
    else if (a_s == 1) { t.box.y0 = before; t.box.y1 = before + S.planes[k]; }
    else { t.box.x0 = before; t.box.x1 = before + S.planes[k]; }
    const int o = k % 2;
    if (ev.done_set[o] && !chk(hipStreamWaitEvent(s, ev.out_done(o), 0))) break;
    const uint8_t* wbuf = cur + (before ? 0 : pb);
    if (!chk(hsz::launch_grad_stage(wbuf, HSZ_QUANT, vq, op, axis3, t, out[o], ws, s))) break;
    if (!chk(hipEventRecord(ev.out_ready(o), s))) break;
    if (!chk(hipStreamWaitEvent(cs, ev.out_ready(o), 0))) break;
    const uint64_t ob = esz * (uint64_t)S.planes[k] * (uint64_t)P;
    if (!chk(hipMemcpyAsync((uint8_t*)h_result + esz * (uint64_t)S.first[k] * (uint64_t)P, out[o], ob,
                            hipMemcpyDeviceToHost, cs)))
      break;
    ev.done_set[o] = true;
    chk(hipEventRecord(ev.out_done(o), cs));
  }
  // the result copies on the copy stream are joined into 's'
  if (chk(hipEventRecord(ev.e[kOocFinal], cs))) chk(hipStreamWaitEvent(s, ev.e[kOocFinal], 0));
  return e;
}

}  // namespace

extern "C" {

int hsz_extremes(const void* d_x, int dtype, uint64_t n, double* d_out, void* d_workspace, uint64_t workspace_bytes,
                 void* stream) {
  if (!d_x || !d_out || !d_workspace || n == 0 || (dtype != HSZ_F32 && dtype != HSZ_F64)) return HSZ_ERR_INVALID_ARG;
  if (!aligned16(d_x) || !aligned16(d_workspace) || ((uintptr_t)d_out & 7u)) return HSZ_ERR_INVALID_ARG;
  if (workspace_bytes < hsz::extremes_workspace_bytes()) return HSZ_ERR_CAPACITY;
  hipError_t e = hsz::launch_extremes(d_x, dtype, (int64_t)n, d_out, (uint8_t*)d_workspace, (hipStream_t)stream);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int hsz_extremes_workspace(uint64_t* h_bytes) {
  if (!h_bytes) return HSZ_ERR_INVALID_ARG;
  *h_bytes = hsz::extremes_workspace_bytes();
  return HSZ_OK;
}

int hsz_ooc_workspace(const hsz_header* const* h_slabs, int nslabs, int op, uint64_t* h_bytes) {
  if (!h_bytes) return HSZ_ERR_INVALID_ARG;
  SlabSet S;
  int rc = describe(h_slabs, nslabs, &S);
  if (rc) return rc;
  if (S.lz && !(S.lz_ws = lz_workspace(h_slabs, nslabs, op))) return HSZ_ERR_UNSUPPORTED;
  *h_bytes = ws_layout(S, op).total;
  return HSZ_OK;
}

int hsz_ooc_op(const void* const* h_slabs, const hsz_header* const* hdrs, int nslabs, int via, int op, int axis,
               void* h_result, uint64_t result_bytes, void* d_workspace, uint64_t workspace_bytes, void* stream) {
  SlabSet S;
  int rc = ooc_check(h_slabs, hdrs, nslabs, via, op, axis, h_result, result_bytes, &S);
  if (rc) return rc;
  if (!d_workspace || !aligned16(d_workspace)) return HSZ_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(S, op);
  if (workspace_bytes < L.total) return HSZ_ERR_CAPACITY;
  uint8_t* ws = (uint8_t*)d_workspace;
  hipStream_t s = (hipStream_t)stream;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e);
  Events ev;
  e = ev.create();
  std::vector<uint8_t> records;
  int call_rc = HSZ_OK;
  if (e == hipSuccess) e = ooc_enqueue(h_slabs, hdrs, S, via, op, axis, h_result, ws, L, s, cs, ev, false, &call_rc);
  // drain both streams whatever happened, so no copy is in flight on return
  hipError_t e1 = hipStreamSynchronize(cs);
  hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e1 != hipSuccess ? e1 : e2;
  int st = 0;
  if (e == hipSuccess) e = hipMemcpy(&st, ws, sizeof st, hipMemcpyDeviceToHost);
  if (e == hipSuccess && !is_stencil_op(op)) {
    records.resize(48 * (size_t)nslabs);
    e = hipMemcpy(records.data(), ws + L.stats, records.size(), hipMemcpyDeviceToHost);
  }
  (void)hipStreamDestroy(cs);
  if (call_rc != HSZ_OK) return call_rc;
  if (e != hipSuccess) return hip_fail(e);
  if (st != 0) return st;
  if (!is_stencil_op(op)) combine(records, nslabs, op, hdrs[0]->quantum, (hsz_stats*)h_result);
  return HSZ_OK;
}

int hsz_ooc_op_async(hsz_ctx* ctx, const void* const* h_slabs, const hsz_header* const* hdrs, int nslabs, int via,
                     int op, int axis, void* h_result, uint64_t result_bytes, int* d_status, void* stream) {
  if (!ctx || ((uintptr_t)d_status & 3u)) return HSZ_ERR_INVALID_ARG;
  int rc = hsz_ctx_util::check_device(ctx);
  if (rc) return rc;
  SlabSet S;
  if ((rc = ooc_check(h_slabs, hdrs, nslabs, via, op, axis, h_result, result_bytes, &S))) return rc;
  std::lock_guard<std::mutex> g(ctx->mu);
  const WsLayout L = ws_layout(S, op);
  if (!ctx->d_scratch || ctx->scratch_bytes < L.total) return HSZ_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  hipStream_t cs = ctx->copy;
  Events ev;
  ev.borrow(ctx->ooc);
  // after the context's previous call on both streams (the ring slots, the
  // windows and the status word are reused)
  hipError_t e = hsz_ctx_util::order_after_last(ctx, s);
  if (e == hipSuccess) e = hsz_ctx_util::order_after_last(ctx, cs);
  int call_rc = HSZ_OK;
  if (e == hipSuccess)
    e = ooc_enqueue(h_slabs, hdrs, S, via, op, axis, h_result, ctx->d_scratch, L, s, cs, ev, true, &call_rc);
  if (e == hipSuccess && d_status) {
    e = hsz::launch_copy_status((const int*)ctx->d_scratch, d_status, s);
  }
  // the context's last call ends here whatever happened: everything enqueued
  // on either stream is joined into 's'
  hipError_t e2 = hsz_ctx_util::mark_last(ctx, s);
  if (e == hipSuccess) e = e2;
  if (call_rc != HSZ_OK) return call_rc;
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

}  // extern "C"
