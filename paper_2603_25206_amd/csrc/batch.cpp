// batch.cpp -- many jobs (fields, boxes, operations) in one pass of
// persistent kernels, and replayable HIP-graph plans of such a pass.
//
// The host lays out a device work table in the caller's workspace:
//   counts      int64 pairs (jobs, units) per kernel, read by the kernels
//   stats jobs  per block size (32, 64): StatsJob[] + first unit of each job
//   grad jobs   per kernel variant (S, via, op, dtype): GradJob[] + first tile
//   index jobs  every gradient job again + its first chunk (offset index)
//   acc         kAccStripes BatchAcc per statistics job (exact sums)
//   rel         one 16-bit offset index per gradient job
// then enqueues: reset -> offset index -> statistics -> gradients -> finalize.
// A statistics job over the same stream and box as a gradient job through
// the quantized stage is computed inside that job's tiles (one decode for
// both); hsz_tuning.separate_stats turns this off.
// Because job and unit counts are read from device memory, a captured graph
// can be replayed after the table is rewritten for a batch of the same
// structure (hsz_plan_update).
#include <algorithm>
#include <vector>

#include "abi_util.hpp"
#include "ctx.hpp"
#include "hsz_stats.hpp"

namespace {

using namespace hsz_abi;

// S(2) x via(2) x op(2) x dtype(2) x shared-statistics mode(3) for the general
// tile, then S(2) x column tile(2) x shared-statistics mode(2) for the
// four-column binary32 magnitude tile (grad4.hip)
constexpr int kVariantsGeneral = 48;
constexpr int kVariants = kVariantsGeneral + 8;
constexpr uint64_t kAlign = 256;

uint64_t up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int variant_of(int S, int via, int op, int dtype, int acc) {
  return 16 * acc + (((S == 64) << 3) | ((via == HSZ_FLOAT) << 2) | ((op == HSZ_GRADMAG) << 1) | (dtype == HSZ_F64));
}
int variant_q4(int S, int txl, int acc) { return kVariantsGeneral + 4 * (S == 64) + 2 * (txl == 512) + acc; }
bool is_q4(int g) { return g >= kVariantsGeneral; }

struct Layout {
  uint64_t counts = 0;                   // int64[2 * (2 + kVariants + 1)]
  uint64_t stats_jobs[2] = {0, 0}, stats_start[2] = {0, 0};
  uint64_t grad_jobs[kVariants] = {}, grad_start[kVariants] = {};
  uint64_t index_jobs = 0, index_start = 0;
  uint64_t acc[2] = {0, 0};
  uint64_t table_end = 0;                // [counts, table_end) is copied from the host
  std::vector<uint64_t> rel;             // per gradient job (in input order)
  uint64_t total = 0;
};

struct Item {
  int kind;  // 0 stats, 1 gradient, 2 an operation of its own (hsz_op_fused)
  int S, via, op, dtype, axis3;
  hsz::StreamView v;
  hsz::OpTarget t;
  void* out;
  const uint16_t* index;  // caller's block index, or null
  hsz_work w;             // kind 2: the work item (w.h unused) and its header
  hsz_header hdr;
  uint64_t ws_bytes;      // kind 2: hsz_op_workspace
};

// A kind-2 job of a built batch: enqueued as its own fused operation on the
// pass's stream, with its workspace in the batch's (its status word merged
// into the pass's afterwards).
struct Single {
  hsz_work w;
  hsz_header hdr;
  uint64_t ws_off, ws_bytes;
};

// counts slots
int cslot_stats(int si) { return si; }             // si: 0 (S=32), 1 (S=64)
int cslot_grad(int var) { return 2 + var; }
int cslot_index() { return 2 + kVariants; }
constexpr int kCountSlots = 2 + kVariants + 1;

// Validate one work item and classify it.
int classify(const hsz_work& w, Item* it) {
  const hsz_header* h = w.h;
  int rc = check_header(h);
  if (rc) return rc;
  if (!w.d_c || ((uintptr_t)w.d_c & 15u) || !w.d_result) return HSZ_ERR_INVALID_ARG;
  int64_t d3[3], n;
  dims3_of(h->ndim, h->dims, d3, &n);
  it->t.d = hsz::Dims3{d3[0], d3[1], d3[2]};
  if (!box3_of(h, w.use_box ? &w.box : nullptr, &it->t.box)) return HSZ_ERR_INVALID_ARG;
  it->S = h->block;
  it->via = w.via;
  it->op = w.op;
  it->dtype = h->dtype;
  it->v = view_of(w.d_c, h);
  it->out = w.d_result;
  it->index = (const uint16_t*)w.d_index;
  if (w.d_index && ((uintptr_t)w.d_index & 1u)) return HSZ_ERR_INVALID_ARG;
  // The batch kernels decode delta streams through the exact integer
  // statistics and the derivative / magnitude stencils; every other item
  // (HSZp-nd, HSZp and block-mean streams, the Laplacian, the spread about
  // the metadata mean, statistics through D_f) runs as an operation of its
  // own inside the pass.
  const bool stats = w.op == HSZ_MEAN || w.op == HSZ_VAR;
  const bool grad = w.op == HSZ_DERIV || w.op == HSZ_GRADMAG;
  if (h->flags || (!stats && !grad) || (stats && w.via != HSZ_DELTA && w.via != HSZ_QUANT)) {
    if ((w.op < HSZ_MEAN || w.op > HSZ_LAPLACIAN) && w.op != HSZ_VAR_MT) return HSZ_ERR_INVALID_ARG;
    uint64_t b = 0;
    if ((rc = hsz_op_workspace(h, w.op, &b))) return rc;
    it->kind = 2;
    it->w = w;
    it->w.h = nullptr;
    it->hdr = *h;
    it->ws_bytes = b;
    it->axis3 = 0;
    return HSZ_OK;
  }
  if (stats) {
    if (w.result_bytes < sizeof(hsz_stats)) return HSZ_ERR_CAPACITY;
    it->kind = 0;
    it->axis3 = 0;
    return HSZ_OK;
  }
  if (grad) {
    if (w.via != HSZ_QUANT && w.via != HSZ_FLOAT) return HSZ_ERR_UNSUPPORTED;
    if (w.op == HSZ_DERIV && (w.axis < 0 || w.axis >= h->ndim)) return HSZ_ERR_INVALID_ARG;
    if ((uintptr_t)w.d_result & 15u) return HSZ_ERR_INVALID_ARG;
    const uint64_t esz = h->dtype == HSZ_F32 ? 4 : 8;
    if (w.result_bytes < esz * (uint64_t)it->t.box.volume()) return HSZ_ERR_CAPACITY;
    it->kind = 1;
    it->axis3 = w.op == HSZ_DERIV ? w.axis + 3 - h->ndim : 0;
    return HSZ_OK;
  }
  return HSZ_ERR_INVALID_ARG;
}

struct Built {
  Layout L;
  std::vector<Single> singles;
  std::vector<uint8_t> table;  // bytes [L.counts, L.table_end)
  int stats_kmax[2] = {0, 0};
  int grad_kmax[kVariants] = {};
  int n_stats[2] = {0, 0};
  int n_grad[kVariants] = {};
  int n_index = 0;
  int64_t stats_units[2] = {0, 0};
  int64_t grad_tile_total[kVariants] = {};
  int64_t index_chunks = 0;
};

bool same_box(const hsz::Box3& a, const hsz::Box3& b) {
  return a.z0 == b.z0 && a.z1 == b.z1 && a.y0 == b.y0 && a.y1 == b.y1 && a.x0 == b.x0 && a.x1 == b.x1;
}

int tz_for(const hsz::Box3& b, int want) {
  const int64_t bz = b.z1 - b.z0;
  int64_t tz = want > 0 ? want : 32;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tz, bz));
}

// Planes per tile of a gradient job in variant g: the tuning's value, else
// 32, halved (down to 4) while the job has fewer than 256 tiles, so a
// small field's planes are not marched by a few workgroups one after
// another (each tile walks its planes in order).
int tz_pick(const hsz::Box3& b, int want, int g) {
  if (want > 0) return tz_for(b, want);
  auto tiles = [&](int tz) -> int64_t {
    if (!is_q4(g)) return hsz::grad_tiles(b, tz);
    return hsz::q4_tiles(b, tz, ((g - kVariantsGeneral) & 2) ? 512 : 256);
  };
  int tz = tz_for(b, 32);
  while (tz > 4 && tiles(tz) < 256) tz = (tz + 1) / 2;
  return tz;
}

// Lay out and fill the table for 'items' in the workspace at d_ws.
int build(const std::vector<Item>& items, const hsz_tuning& tune, uint8_t* d_ws, Built* B) {
  Layout& L = B->L;
  // Statistics that share a gradient job's decode: same stream and box, the
  // gradient through the quantized stage.  Such a job gets no units of its
  // own; the gradient tiles add its sums (exact, so the result is the same).
  std::vector<int> host(items.size(), -1), slot(items.size(), -1), acc_mode(items.size(), 0);
  if (!tune.separate_stats) {
    for (int i = 0; i < (int)items.size(); ++i) {
      if (items[i].kind != 0) continue;
      for (int g = 0; g < (int)items.size(); ++g) {
        const Item& G = items[g];
        if (G.kind == 1 && G.via == HSZ_QUANT && G.v.base == items[i].v.base && same_box(G.t.box, items[i].t.box)) {
          host[i] = g;
          acc_mode[g] = (G.v.max_abs_q < 65536u && tz_for(G.t.box, tune.grad_tz) <= 2048) ? 1 : 2;
          break;
        }
      }
    }
  }
  std::vector<int> order_stats[2], order_grad[kVariants];
  std::vector<int> grads, var_of(items.size(), -1);
  for (int i = 0; i < (int)items.size(); ++i) {
    const Item& it = items[i];
    if (it.kind == 2) continue;  // an operation of its own (below)
    if (it.kind == 0) order_stats[it.S == 64].push_back(i);
    else {
      const bool q4 =
          tune.grad_tile_x >= 0 && acc_mode[i] != 2 && hsz::q4_eligible(it.v, it.via, it.op, it.t.d, it.t.box);
      const int txl = tune.grad_tile_x == 256 ? 256 : hsz::q4_txl(it.t.box);
      var_of[i] = q4 ? variant_q4(it.S, txl, acc_mode[i]) : variant_of(it.S, it.via, it.op, it.dtype, acc_mode[i]);
      order_grad[var_of[i]].push_back(i);
      if (!it.index) grads.push_back(i);  // jobs that need an index built here
    }
  }
  uint64_t off = kAlign;  // [0, 256): status
  L.counts = off;
  off = up(off + sizeof(int64_t) * 2 * kCountSlots);
  for (int si = 0; si < 2; ++si) {
    L.stats_jobs[si] = off;
    off = up(off + sizeof(hsz::StatsJob) * order_stats[si].size());
    L.stats_start[si] = off;
    off = up(off + sizeof(int64_t) * order_stats[si].size());
  }
  for (int g = 0; g < kVariants; ++g) {
    L.grad_jobs[g] = off;
    off = up(off + sizeof(hsz::GradJob) * order_grad[g].size());
    L.grad_start[g] = off;
    off = up(off + sizeof(int64_t) * order_grad[g].size());
  }
  L.index_jobs = off;
  off = up(off + sizeof(hsz::GradJob) * grads.size());
  L.index_start = off;
  off = up(off + sizeof(int64_t) * grads.size());
  L.table_end = off;
  for (int si = 0; si < 2; ++si) {
    L.acc[si] = off;
    off = up(off + sizeof(hsz::BatchAcc) * hsz::kAccStripes * order_stats[si].size());
  }
  L.rel.assign(items.size(), 0);
  for (int i : grads) {
    L.rel[i] = off;
    off = up(off + 2 * (uint64_t)items[i].v.nb);
  }
  B->singles.clear();
  for (const Item& it : items) {
    if (it.kind != 2) continue;
    B->singles.push_back(Single{it.w, it.hdr, off, it.ws_bytes});
    off = up(off + it.ws_bytes);
  }
  L.total = off;

  B->table.assign(L.table_end - L.counts, 0);
  auto at = [&](uint64_t o) { return B->table.data() + (o - L.counts); };
  int64_t* counts = (int64_t*)at(L.counts);
  for (int si = 0; si < 2; ++si) {
    int64_t u = 0;
    int km = 0;
    for (size_t k = 0; k < order_stats[si].size(); ++k) {
      const int i = order_stats[si][k];
      const Item& it = items[i];
      hsz::StatsJob J{};
      J.v = it.v;
      J.rows = hsz::make_rows(it.t.d, it.t.box);
      J.whole = J.rows.count() == 1 && J.rows.base == 0 && J.rows.len == it.v.n;
      J.per_row = (J.rows.len + it.S - 2) / it.S + 1;
      J.op = it.op;
      J.via = it.via;
      J.acc = (int32_t)k;
      J.out = it.out;
      J.rel = it.index;
      ((int64_t*)at(L.stats_start[si]))[k] = u;
      if (host[i] >= 0) {
        if (slot[host[i]] < 0) slot[host[i]] = (int)k;
        J.acc = slot[host[i]];
      } else {
        u += J.whole ? it.v.nchunks : (J.rows.count() * J.per_row + hsz::kWave - 1) / hsz::kWave;
      }
      ((hsz::StatsJob*)at(L.stats_jobs[si]))[k] = J;
      km = std::max(km, hsz::stats_kmax(it.v));
    }
    counts[2 * cslot_stats(si)] = (int64_t)order_stats[si].size();
    counts[2 * cslot_stats(si) + 1] = u;
    B->n_stats[si] = (int)order_stats[si].size();
    B->stats_units[si] = u;
    B->stats_kmax[si] = km;
  }
  std::vector<hsz::GradJob> gj(items.size());
  for (int i = 0; i < (int)items.size(); ++i) {
    const Item& it = items[i];
    if (it.kind != 1) continue;
    hsz::GradJob J{};
    J.v = it.v;
    J.rel = it.index ? it.index : (const uint16_t*)(d_ws + L.rel[i]);
    J.d = it.t.d;
    J.b = it.t.box;
    J.axis = it.axis3;
    J.tz = tz_pick(it.t.box, tune.grad_tz, var_of[i]);
    J.kmax = hsz::grad_kmax(it.v);
    J.halfq = 0.5 * it.v.quantum;
    J.out = it.out;
    if (slot[i] >= 0) {
      J.acc = d_ws + L.acc[it.S == 64] + sizeof(hsz::BatchAcc) * hsz::kAccStripes * (uint64_t)slot[i];
      J.acc_mode = acc_mode[i];
    }
    gj[i] = J;
  }
  for (int g = 0; g < kVariants; ++g) {
    int64_t tiles = 0;
    int km = 0;
    for (size_t k = 0; k < order_grad[g].size(); ++k) {
      const hsz::GradJob& J = gj[order_grad[g][k]];
      ((hsz::GradJob*)at(L.grad_jobs[g]))[k] = J;
      ((int64_t*)at(L.grad_start[g]))[k] = tiles;
      tiles += is_q4(g) ? hsz::q4_tiles(J.b, J.tz, ((g - kVariantsGeneral) & 2) ? 512 : 256)
                        : hsz::grad_tiles(J.b, J.tz);
      km = std::max(km, J.kmax);
    }
    counts[2 * cslot_grad(g)] = (int64_t)order_grad[g].size();
    counts[2 * cslot_grad(g) + 1] = tiles;
    B->n_grad[g] = (int)order_grad[g].size();
    B->grad_tile_total[g] = tiles;
    B->grad_kmax[g] = km;
  }
  int64_t chunks = 0;
  for (size_t k = 0; k < grads.size(); ++k) {
    ((hsz::GradJob*)at(L.index_jobs))[k] = gj[grads[k]];
    ((int64_t*)at(L.index_start))[k] = chunks;
    chunks += items[grads[k]].v.nchunks;
  }
  counts[2 * cslot_index()] = (int64_t)grads.size();
  counts[2 * cslot_index() + 1] = chunks;
  B->n_index = (int)grads.size();
  B->index_chunks = chunks;
  return HSZ_OK;
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

// The one gradient variant of a batch that can finish itself: every job is
// a 512-column sixteen-bit tile with statistics summed inside (and every
// statistic is), no block index is built per pass.  -1 if none.
int self_finishing(const Built& B) {
  if (B.n_index > 0 || B.stats_units[0] > 0 || B.stats_units[1] > 0 || B.n_stats[0] + B.n_stats[1] == 0 ||
      !B.singles.empty())
    return -1;
  int only = -1;
  for (int g = 0; g < kVariants; ++g) {
    if (B.n_grad[g] == 0) continue;
    if (only >= 0) return -1;
    only = g;
  }
  return only == variant_q4(32, 512, 1) ? only : -1;
}

// Enqueue the kernels of a built batch ('kmax' values fix the LDS sizes).
// 'primed': the workspace's accumulators, live word and done count are zero
// (a plan, after its first reset): a batch that can finish itself is then
// one kernel.
int enqueue(const Built& B, uint8_t* d_ws, const hsz_tuning& tune, hipStream_t s, bool primed = false) {
  const Layout& L = B.L;
  const int64_t* counts = (const int64_t*)(d_ws + L.counts);
  int* status = (int*)d_ws;
  const int cus = device_cus();
  const int self = primed ? self_finishing(B) : -1;
  if (self >= 0) {
    hsz::BatchTail T;
    for (int c = 0; c < 2; ++c) {
      T.jobs[c] = (const hsz::StatsJob*)(d_ws + L.stats_jobs[c]);
      T.counts[c] = counts + 2 * cslot_stats(c);
      T.acc[c] = (hsz::BatchAcc*)(d_ws + L.acc[c]);
      T.n[c] = B.n_stats[c];
    }
    T.status_out = status;
    T.live = status + 1;
    T.done = (unsigned*)(status + 2);
    const int per_cu = std::min(2, tune.grad_groups_per_cu > 0 ? tune.grad_groups_per_cu : 2);
    hipError_t e = hsz::launch_batch_gradmag_q8_tail((const hsz::GradJob*)(d_ws + L.grad_jobs[self]),
                                                     (const int64_t*)(d_ws + L.grad_start[self]),
                                                     counts + 2 * cslot_grad(self), std::max(1, cus * per_cu), T, s);
    return e == hipSuccess ? HSZ_OK : hip_fail(e);
  }
  const int stats_grid = std::max(1, cus * (tune.stats_waves_per_cu > 0 ? tune.stats_waves_per_cu : 8) / 4);
  const int grad_grid = std::max(1, cus * (tune.grad_groups_per_cu > 0 ? tune.grad_groups_per_cu : 4));
  hipError_t e;
  // every pass first zeroes the status word and the accumulators of both
  // classes (adjacent in the workspace), in one small kernel: no memset nodes
  if ((e = hsz::launch_batch_reset((hsz::BatchAcc*)(d_ws + L.acc[0]), B.n_stats[0] + B.n_stats[1], status, s)) !=
      hipSuccess)
    return hip_fail(e);
  if (B.n_index > 0) {
    if ((e = hsz::launch_batch_block_index((const hsz::GradJob*)(d_ws + L.index_jobs),
                                           (const int64_t*)(d_ws + L.index_start), counts + 2 * cslot_index(),
                                           std::max(1, cus * 8), s)) != hipSuccess)
      return hip_fail(e);
  }
  for (int si = 0; si < 2; ++si) {
    if (B.stats_units[si] == 0) continue;  // none, or all summed inside gradient tiles
    if ((e = hsz::launch_batch_stats(si ? 64 : 32, (const hsz::StatsJob*)(d_ws + L.stats_jobs[si]),
                                     (const int64_t*)(d_ws + L.stats_start[si]), counts + 2 * cslot_stats(si),
                                     B.stats_kmax[si], (hsz::BatchAcc*)(d_ws + L.acc[si]), status, stats_grid, s)) !=
        hipSuccess)
      return hip_fail(e);
  }
  for (int g = 0; g < kVariants; ++g) {
    if (B.n_grad[g] == 0) continue;
    if (is_q4(g)) {
      // persistent: as many workgroups as fit at once (two per compute unit by
      // their LDS), at most the tuning's count
      const int q = g - kVariantsGeneral, per_cu = std::min(2, tune.grad_groups_per_cu > 0 ? tune.grad_groups_per_cu : 2);
      if ((e = hsz::launch_batch_gradmag_q4(32, (q & 2) ? 512 : 256, q & 1,
                                            (const hsz::GradJob*)(d_ws + L.grad_jobs[g]),
                                            (const int64_t*)(d_ws + L.grad_start[g]), counts + 2 * cslot_grad(g),
                                            std::max(1, cus * per_cu), status, s)) != hipSuccess)
        return hip_fail(e);
      continue;
    }
    const int S = ((g >> 3) & 1) ? 64 : 32, via = ((g >> 2) & 1) ? HSZ_FLOAT : HSZ_QUANT;
    const int op = ((g >> 1) & 1) ? HSZ_GRADMAG : HSZ_DERIV, dtype = (g & 1) ? HSZ_F64 : HSZ_F32, acc = g >> 4;
    if ((e = hsz::launch_batch_grad(S, via, op, dtype, acc, (const hsz::GradJob*)(d_ws + L.grad_jobs[g]),
                                    (const int64_t*)(d_ws + L.grad_start[g]), counts + 2 * cslot_grad(g),
                                    B.grad_kmax[g], grad_grid, status, s)) != hipSuccess)
      return hip_fail(e);
  }
  // the operations of their own, each followed by its status word's merge
  for (const Single& one : B.singles) {
    hsz_header hdr = one.hdr;
    const hsz_work& w = one.w;
    const int rc = hsz_op_fused(w.d_c, &hdr, w.via, w.op, w.axis, w.use_box ? &w.box : nullptr, w.d_result,
                                w.result_bytes, d_ws + one.ws_off, one.ws_bytes, s);
    if (rc) return rc;
    if ((e = hsz::launch_merge_status((const int*)(d_ws + one.ws_off), status, s)) != hipSuccess) return hip_fail(e);
  }
  const hsz::StatsJob* fj[2] = {(const hsz::StatsJob*)(d_ws + L.stats_jobs[0]),
                                (const hsz::StatsJob*)(d_ws + L.stats_jobs[1])};
  const int64_t* fc[2] = {counts + 2 * cslot_stats(0), counts + 2 * cslot_stats(1)};
  const hsz::BatchAcc* fa[2] = {(const hsz::BatchAcc*)(d_ws + L.acc[0]), (const hsz::BatchAcc*)(d_ws + L.acc[1])};
  if ((e = hsz::launch_batch_finalize(fj, fc, fa, B.n_stats, s)) != hipSuccess) return hip_fail(e);
  return HSZ_OK;
}

int collect(const hsz_work* items, int n, std::vector<Item>* out) {
  if (!items || n <= 0) return HSZ_ERR_INVALID_ARG;
  out->resize(n);
  for (int i = 0; i < n; ++i) {
    int rc = classify(items[i], &(*out)[i]);
    if (rc) return rc;
  }
  return HSZ_OK;
}

}  // namespace

struct hsz_plan {
  Built built;
  hsz_tuning tune;
  uint8_t* d_ws = nullptr;
  uint64_t ws_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool launched = false;
};

extern "C" {

int hsz_batch_workspace(const hsz_work* items, int n, uint64_t* h_bytes) {
  if (!h_bytes) return HSZ_ERR_INVALID_ARG;
  std::vector<Item> its;
  int rc = collect(items, n, &its);
  if (rc) return rc;
  Built B;
  hsz_tuning t{};
  build(its, t, nullptr, &B);
  *h_bytes = B.L.total;
  return HSZ_OK;
}

int hsz_batch_run(const hsz_work* items, int n, const hsz_tuning* tune, void* d_workspace, uint64_t workspace_bytes,
                  void* stream) {
  std::vector<Item> its;
  int rc = collect(items, n, &its);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 15u)) return HSZ_ERR_INVALID_ARG;
  hsz_tuning t = tune ? *tune : hsz_tuning{};
  Built B;
  build(its, t, (uint8_t*)d_workspace, &B);
  if (workspace_bytes < B.L.total) return HSZ_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync((uint8_t*)d_workspace + B.L.counts, B.table.data(), B.table.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e);
  return enqueue(B, (uint8_t*)d_workspace, t, s);
}

int hsz_ctx_batch_run(hsz_ctx* ctx, const hsz_work* items, int n, const hsz_tuning* tune, int* d_status,
                      void* stream) {
  if (!ctx || ((uintptr_t)d_status & 3u)) return HSZ_ERR_INVALID_ARG;
  int rc = hsz_ctx_util::check_device(ctx);
  if (rc) return rc;
  std::vector<Item> its;
  if ((rc = collect(items, n, &its))) return rc;
  std::lock_guard<std::mutex> g(ctx->mu);
  hsz_tuning t = tune ? *tune : hsz_tuning{};
  Built B;
  build(its, t, ctx->d_scratch, &B);
  if (!ctx->d_scratch || ctx->scratch_bytes < B.L.total) return HSZ_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hsz_ctx_util::order_after_last(ctx, s);
  if (e != hipSuccess) return hip_fail(e);
  if ((rc = hsz_ctx_util::stage_copy(ctx, B.table.data(), B.table.size(), ctx->d_scratch + B.L.counts, s))) return rc;
  if ((rc = enqueue(B, ctx->d_scratch, t, s))) return rc;
  if (d_status && (e = hsz::launch_copy_status((const int*)ctx->d_scratch, d_status, s)) != hipSuccess)
    return hip_fail(e);
  e = hsz_ctx_util::mark_last(ctx, s);
  return e == hipSuccess ? HSZ_OK : hip_fail(e);
}

int hsz_plan_create(const hsz_work* items, int n, const hsz_tuning* tune, void* d_workspace, uint64_t workspace_bytes,
                    void* stream, hsz_plan** out) {
  if (!out || !stream) return HSZ_ERR_INVALID_ARG;  // capture needs a created stream
  *out = nullptr;
  std::vector<Item> its;
  int rc = collect(items, n, &its);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 15u)) return HSZ_ERR_INVALID_ARG;
  hsz_plan* p = new hsz_plan();
  p->tune = tune ? *tune : hsz_tuning{};
  p->d_ws = (uint8_t*)d_workspace;
  p->ws_bytes = workspace_bytes;
  build(its, p->tune, p->d_ws, &p->built);
  if (workspace_bytes < p->built.L.total) {
    delete p;
    return HSZ_ERR_CAPACITY;
  }
  // the table is uploaded here and by hsz_plan_update, not by the graph: a
  // replay runs kernels only
  hipError_t e = hipMemcpy(p->d_ws + p->built.L.counts, p->built.table.data(), p->built.table.size(),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e);
  }
  hipStream_t s = (hipStream_t)stream;
  if ((e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming)) != hipSuccess) {
    hsz_plan_destroy(p);
    return hip_fail(e);
  }
  // a batch that finishes itself leaves its accumulators, live word and
  // done count zero after every pass: zero them once here, before any pass
  // (and wait, so a pass on another stream finds them zero)
  if (self_finishing(p->built) >= 0 &&
      ((e = hsz::launch_batch_reset((hsz::BatchAcc*)(p->d_ws + p->built.L.acc[0]),
                                    p->built.n_stats[0] + p->built.n_stats[1], (int*)p->d_ws, s)) != hipSuccess ||
       (e = hipStreamSynchronize(s)) != hipSuccess)) {
    hsz_plan_destroy(p);
    return hip_fail(e);
  }
  if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    hsz_plan_destroy(p);
    return hip_fail(e);
  }
  int erc = enqueue(p->built, p->d_ws, p->tune, s, true);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (erc != HSZ_OK || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    hsz_plan_destroy(p);
    return erc != HSZ_OK ? erc : hip_fail(e2);
  }
  p->graph = g;
  if ((e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
    hsz_plan_destroy(p);
    return hip_fail(e);
  }
  *out = p;
  return HSZ_OK;
}

int hsz_plan_update(hsz_plan* p, const hsz_work* items, int n) {
  if (!p) return HSZ_ERR_INVALID_ARG;
  std::vector<Item> its;
  int rc = collect(items, n, &its);
  if (rc) return rc;
  Built B;
  build(its, p->tune, p->d_ws, &B);
  // the captured launches fix the table layout, the kernel variants and the
  // LDS sizes: a new batch must have the same structure and fit them
  const Built& A = p->built;
  bool same = B.L.total <= p->ws_bytes && B.table.size() == A.table.size() && B.n_index == A.n_index;
  for (int si = 0; si < 2 && same; ++si)
    same = B.n_stats[si] == A.n_stats[si] && B.stats_kmax[si] <= A.stats_kmax[si] && B.L.acc[si] == A.L.acc[si] &&
           (B.stats_units[si] > 0) == (A.stats_units[si] > 0);
  for (int g = 0; g < kVariants && same; ++g) same = B.n_grad[g] == A.n_grad[g] && B.grad_kmax[g] <= A.grad_kmax[g];
  for (size_t i = 0; i < B.L.rel.size() && same; ++i) same = B.L.rel[i] == A.L.rel[i];
  same = same && B.singles.size() == A.singles.size();
  for (size_t k = 0; k < B.singles.size() && same; ++k)
    same = B.singles[k].ws_off == A.singles[k].ws_off && B.singles[k].ws_bytes <= A.singles[k].ws_bytes;
  if (!same) return HSZ_ERR_UNSUPPORTED;
  if (p->launched) {
    hipError_t e = hipEventSynchronize(p->done);  // the last replay has read the table
    if (e != hipSuccess) return hip_fail(e);
  }
  hipError_t e = hipMemcpy(p->d_ws + B.L.counts, B.table.data(), B.table.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e);
  if (!B.singles.empty()) {
    // the operations of their own take their streams and results as launch
    // arguments: direct launches read the new ones from here, and the graph
    // is captured again with them
    for (size_t k = 0; k < B.singles.size(); ++k) {
      p->built.singles[k].w = B.singles[k].w;
      p->built.singles[k].hdr = B.singles[k].hdr;
    }
    hipStream_t cs = nullptr;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e);
    hipGraph_t g = nullptr;
    int erc = HSZ_OK;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) == hipSuccess) {
      erc = enqueue(p->built, p->d_ws, p->tune, cs, true);
      e = hipStreamEndCapture(cs, &g);
    }
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess && erc == HSZ_OK) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || erc != HSZ_OK) {
      if (g) (void)hipGraphDestroy(g);
      return erc != HSZ_OK ? erc : hip_fail(e);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph = g;
    p->exec = x;
  }
  return HSZ_OK;
}

int hsz_plan_launch(hsz_plan* p, void* stream) {
  if (!p || !p->exec) return HSZ_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (p->tune.graph_replay) {
    if ((e = hipGraphLaunch(p->exec, s)) != hipSuccess) return hip_fail(e);
  } else {
    // the table is on the device since create/update: the pass is a handful
    // of kernel launches, which reach the GPU sooner than a graph launch
    const int erc = enqueue(p->built, p->d_ws, p->tune, s, true);
    if (erc != HSZ_OK) return erc;
  }
  if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e);
  p->launched = true;
  return HSZ_OK;
}

void hsz_plan_destroy(hsz_plan* p) {
  if (!p) return;
  if (p->launched && p->done) (void)hipEventSynchronize(p->done);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->done) (void)hipEventDestroy(p->done);
  delete p;
}

}  // extern "C"
