// vector.hip -- divergence and curl of vector fields (Eq. (divergence),
// Eq. (curl), Sec. V-C "multivariate derivation"), one compressed stream per
// component.
//
// Both reduce to derivatives of single components (Eq. (derivatives)):
// component k of the field pairs with the field's own axis k, interior
// points take central differences and the two ends of an axis one-sided
// ones.  Divergence = sum_k delta_k F_k.  Curl of a 2D field = delta_1 F_0 -
// delta_0 F_1 (Eq. (curl) as printed); of a 3D field the vector
// (delta_2 F_1 - delta_1 F_2, delta_0 F_2 - delta_2 F_0, delta_1 F_0 -
// delta_0 F_1), whose last component is the 2D formula.
//
// Integer route (D_q): every term is an exact integer numerator n of one
// component (q_{+1} - q_{-1}, or 2 (q_1 - q_0) at an end), scaled by that
// component's Delta/2; the terms of an output are summed in binary64 in a
// fixed order and rounded once to the field dtype.  The fused kernel decodes
// a plane of every component from its stream in one pass, each into its own
// LDS window (the blockwise window of Alg. 3, one per component, with only
// the halo that component's terms need); the stage kernel reads
// materialised q buffers and sums the same terms in the same order, so the
// two agree bit for bit.  Float route (D_f, stage buffers):
// the same differences on the decompressed values in the field's precision.
#include <algorithm>

#include "hsz_device.hpp"
#include "hsz_launch.hpp"

namespace hsz {

namespace {

// One derivative term: component c, axis a of the 3D view (0 z, 1 y, 2 x),
// sign s, output o.
struct VTerm {
  int c, a, s, o;
};

template <int OP, int NC>
struct VTerms;
// divergence of 1D, 2D, 3D fields (field axis k = view axis k + 3 - NC)
template <>
struct VTerms<kOpDivergence, 1> {
  static constexpr int n = 1, nout = 1;
  static constexpr VTerm t[1] = {{0, 2, 1, 0}};
};
template <>
struct VTerms<kOpDivergence, 2> {
  static constexpr int n = 2, nout = 1;
  static constexpr VTerm t[2] = {{0, 1, 1, 0}, {1, 2, 1, 0}};
};
template <>
struct VTerms<kOpDivergence, 3> {
  static constexpr int n = 3, nout = 1;
  static constexpr VTerm t[3] = {{0, 0, 1, 0}, {1, 1, 1, 0}, {2, 2, 1, 0}};
};
// curl of a 2D field: delta_1 F_0 - delta_0 F_1 (field axes 0, 1 = view y, x)
template <>
struct VTerms<kOpCurl, 2> {
  static constexpr int n = 2, nout = 1;
  static constexpr VTerm t[2] = {{0, 2, 1, 0}, {1, 1, -1, 0}};
};
// curl of a 3D field, output by output
template <>
struct VTerms<kOpCurl, 3> {
  static constexpr int n = 6, nout = 3;
  static constexpr VTerm t[6] = {{1, 2, 1, 0}, {2, 1, -1, 0}, {2, 0, 1, 1},
                                 {0, 2, -1, 1}, {0, 1, 1, 2}, {1, 0, -1, 2}};
};

// whether some term differentiates component c along view axis a
template <class Tm>
__host__ __device__ constexpr bool needs_axis(int c, int a) {
  for (int k = 0; k < Tm::n; ++k)
    if (Tm::t[k].c == c && Tm::t[k].a == a) return true;
  return false;
}

// integer numerator along one axis at coordinate i of length L
__device__ __forceinline__ int vnum(int vm, int v0, int vp, int64_t i, int64_t L) {
  if (L < 2) return 0;
  if (i == 0) return 2 * (vp - v0);
  if (i == L - 1) return 2 * (v0 - vm);
  return vp - vm;
}
// float derivative along one axis in the field's precision
template <typename T>
__device__ __forceinline__ T vder(T vm, T v0, T vp, int64_t i, int64_t L) {
  if (L < 2) return T(0);
  if (i == 0) return vp - v0;
  if (i == L - 1) return v0 - vm;
  return (vp - vm) * T(0.5);
}

// ---- stage buffers: one thread per output point --------------------------------
template <int SRC, int OP, int NC, typename T>
__global__ void __launch_bounds__(256) k_vector_buf(VecJob j) {
  using Tm = VTerms<OP, NC>;
  const Box3 b = j.b;
  const Dims3 d = j.d;
  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int64_t vol = bx * by * (b.z1 - b.z0);
  const int64_t sy = d.x, sz = d.x * d.y;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < vol; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = b.x0 + e % bx, y = b.y0 + (e / bx) % by, z = b.z0 + e / (bx * by);
    const int64_t pos[3] = {z, y, x}, len[3] = {d.z, d.y, d.x}, str[3] = {sz, sy, 1};
    const int64_t f = z * sz + y * sy + x;
    double acc[Tm::nout];
    T facc[Tm::nout];
#pragma unroll
    for (int o = 0; o < Tm::nout; ++o) { acc[o] = 0.0; facc[o] = T(0); }
#pragma unroll
    for (int k = 0; k < Tm::n; ++k) {
      const VTerm tm = Tm::t[k];
      const int64_t i = pos[tm.a], L = len[tm.a], st = str[tm.a];
      if constexpr (SRC == 3) {
        const int32_t* q = (const int32_t*)j.buf[tm.c];
        const int v0 = q[f], vm = i > 0 ? q[f - st] : v0, vp = i + 1 < L ? q[f + st] : v0;
        acc[tm.o] += (double)(tm.s * vnum(vm, v0, vp, i, L)) * j.halfq[tm.c];
      } else {
        const T* v = (const T*)j.buf[tm.c];
        const T v0 = v[f], vm = i > 0 ? v[f - st] : v0, vp = i + 1 < L ? v[f + st] : v0;
        const T g = vder<T>(vm, v0, vp, i, L);
        facc[tm.o] = tm.s > 0 ? facc[tm.o] + g : facc[tm.o] - g;
      }
    }
#pragma unroll
    for (int o = 0; o < Tm::nout; ++o) ((T*)j.out[o])[e] = SRC == 3 ? (T)acc[o] : facc[o];
  }
}

// ---- fused from the compressed streams (D_q) ------------------------------------
constexpr int kVTx = 256, kVThreads = 256;
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

template <int S, int TY>
struct VRow {
  static constexpr int kRows = TY + 2, kCols = kVTx + 2;
  static constexpr int kNbr = (kCols + S - 2) / S + 1;  // blocks covering one decoded row
  static constexpr int kOff = S - 1;                    // extended column of tile column 0
  static constexpr int kExt = kCols + 2 * (S - 1);
  // a pitch congruent to kNbr (S + S/32) mod 64: decode lane i writes slot j
  // of its block to bank i (S + S/32) + const, distinct over a wave for S = 32
  static constexpr int pitch() {
    int p = kExt + (kExt >> 5);
    while (p % 64 != (kNbr * (S + S / 32)) % 64) ++p;
    return p;
  }
  static constexpr int kPitch = pitch();
  static __host__ __device__ constexpr int at(int e) { return e + (e >> 5); }
};

template <int OP, int NC>
constexpr int vty() { return (OP == kOpCurl && NC == 3) ? 4 : 8; }

// The windows of one plane, one per component, all decoded in one pass (one
// decode item per thread).  Component c's window holds TY rows, plus the
// rows above and below when one of c's terms is a y difference (hy), and
// the tile's columns, plus one either side when one of c's terms is an x
// difference (hx): a divergence decodes each component with the one halo
// its own axis needs.  The windows sit one after another in LDS, row by row
// (row r of the window is tile row r - 1; windows without hy hold rows 1..TY).
template <int S, int OP, int NC>
struct VWin {
  using Tm = VTerms<OP, NC>;
  static constexpr int TY = vty<OP, NC>();
  using R = VRow<S, TY>;
  static constexpr int kNb0 = (kVTx + S - 2) / S + 1;  // blocks covering the tile's columns
  static constexpr bool hy(int c) { return needs_axis<Tm>(c, 1); }
  static constexpr bool hx(int c) { return needs_axis<Tm>(c, 2); }
  static constexpr int rows(int c) { return TY + (hy(c) ? 2 : 0); }
  static constexpr int nb(int c) { return hx(c) ? R::kNbr : kNb0; }
  static constexpr int items(int c) { return rows(c) * nb(c); }
  static constexpr int item_off(int c) {
    int o = 0;
    for (int k = 0; k < c; ++k) o += items(k);
    return o;
  }
  static constexpr int row_off(int c) {
    int o = 0;
    for (int k = 0; k < c; ++k) o += rows(k);
    return o;
  }
  // LDS word of window c's row r (r = 0 .. TY + 1 for hy, else 1 .. TY)
  static constexpr int base(int c) { return (row_off(c) - (hy(c) ? 0 : 1)) * R::kPitch; }
  static constexpr int kItems = item_off(NC);
  static constexpr int kStageOff = (row_off(NC) * R::kPitch + 63) / 64 * 64;
};

// A staged block decoded two slots per funnel shift: with every width at most
// 16 bits (the stream's max|q| below 2^15, which bounds every delta's width),
// slots j and j + 1 lie in one 32-bit window of the magnitude words, so a
// pair costs one pair of LDS reads and one shift where the slot-by-slot
// decode of the general case costs two each.  Same slots, same values.
constexpr int kVPairW = 16;
template <int S, bool ALIGNED>
__device__ __forceinline__ void decode_block_pairs(const uint32_t* col, int w, int q0, int* dst, int jx) {
  const uint32_t sg0 = col[0];
  const uint32_t sg1 = S == 64 ? col[kVThreads] : 0u;
  const uint32_t* mag = col + (S / 32) * kVThreads;
  int* dst1 = dst + 1;
  int q = q0;
  const uint32_t uw = (uint32_t)w, w2 = 2u * uw;
  uint32_t pos = 0;
#pragma unroll
  for (int g = 0; g < S; g += 8) {
    // bit positions of the four pairs by additions (the empty asm keeps the
    // compiler from computing all of them up front)
    asm volatile("" : "+v"(pos));
    uint32_t lo[4], hi[4], pp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      pp[u] = pos;
      pos += w2;
      uint32_t k = pp[u] >> 5;
      asm("" : "+v"(k));  // one shift-add per address
      const uint32_t* a = mag + k * kVThreads;
      lo[u] = a[0];
      hi[u] = a[kVThreads];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = g + 2 * u;
      const uint32_t win = __builtin_amdgcn_alignbit(hi[u], lo[u], pp[u]);
      const uint32_t sgw = j < 32 ? sg0 : sg1;
      const int s0 = __builtin_amdgcn_sbfe((int)sgw, (uint32_t)(j & 31), 1u);
      const int s1 = __builtin_amdgcn_sbfe((int)sgw, (uint32_t)((j + 1) & 31), 1u);
      const uint32_t m0 = __builtin_amdgcn_ubfe(win, 0u, uw), m1 = __builtin_amdgcn_ubfe(win, uw, uw);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jj = j + h, sg = h ? s1 : s0;
        q = (int)(((h ? m1 : m0) ^ (uint32_t)sg) + (uint32_t)q) - sg;  // q += (m ^ s) - s
        if constexpr (ALIGNED) {
          dst[jj + (jj >> 5)] = q;
        } else {
          int* d = ((jj & 31) >= jx) ? dst1 : dst;
          d[jj + (jj >> 5)] = q;
        }
      }
    }
  }
}

// One workgroup: a tile of kVTx columns x TY rows over tz planes.  Per plane
// p, every thread with a decode item stages and decodes its block of plane
// p into its component's window; after a barrier every column thread writes
// the one-sided ghosts of its column and takes the in-plane numerators of
// every term (plane p) and the z numerators (plane p - 1, from q of planes
// p and p - 2 kept in registers); a barrier frees the windows for the next
// plane, whose payload words were loaded during the stencil.  Then plane
// p - 1 is emitted.
template <int S, int OP, int NC, typename T, bool PAIRS>
__global__ void __launch_bounds__(kVThreads) k_vector_fused(VecJob j, int* status) {
  using Tm = VTerms<OP, NC>;
  using W = VWin<S, OP, NC>;
  constexpr int TY = W::TY;
  using R = typename W::R;
  constexpr int P = R::kPitch, NT = Tm::n;
  static_assert(W::kItems <= kVThreads, "one decode item per thread");
  extern __shared__ uint32_t smem[];
  int* const pl = (int*)smem;
  uint32_t* const stage = smem + W::kStageOff;
  const int t = threadIdx.x;
  const Dims3 d = j.d;
  const Box3 b = j.b;
  const int tz = j.tz, kmax = j.kmax;

  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int64_t ntx = (bx + kVTx - 1) / kVTx, nty = (by + TY - 1) / TY;
  int64_t blk = blockIdx.x;
  const int64_t tx = blk % ntx;
  blk /= ntx;
  const int64_t ty = blk % nty;
  const int64_t tzi = blk / nty;
  const int64_t x0 = b.x0 + tx * kVTx, y0 = b.y0 + ty * TY, z0 = b.z0 + tzi * tz;
  if (z0 >= b.z1) return;
  const int xs = (int)min((int64_t)kVTx, b.x1 - x0), ys = (int)min((int64_t)TY, b.y1 - y0);
  const int64_t zs = min((int64_t)tz, b.z1 - z0);
  const int64_t cA = max((int64_t)0, x0 - 1), cB = min(d.x, x0 + xs + 1);
  const int64_t rA = max((int64_t)0, y0 - 1), rB = min(d.y, y0 + ys + 1);
  const int64_t za = max((int64_t)0, z0 - 1), zb = min(d.z, z0 + zs + 1);
  const bool aligned = (d.x & 31) == 0 && (x0 & 31) == 0;

  // this thread's decode item: component dc, window row dr, block dk (the
  // same for every plane); none past the last item
  int dc = -1, dr = 0, dk = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (t >= W::item_off(c) && t < W::item_off(c) + W::items(c)) {
      dc = c;
      dr = (t - W::item_off(c)) / W::nb(c);
      dk = (t - W::item_off(c)) % W::nb(c);
    }
  bool dhy = false, dhx = false;
  int dbase = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c == dc) {
      dhy = W::hy(c);
      dhx = W::hx(c);
      dbase = W::base(c);
    }
  const int64_t dy = (dhy ? rA : y0) + dr;
  const bool decoder = dc >= 0 && dy < (dhy ? rB : y0 + ys);
  const int64_t dxa = dhx ? cA : x0, dxb = dhx ? cB : x0 + xs;  // the window's columns
  // the item's stream, picked from the kernel arguments once (selects of
  // uniform values, not loads: the planes' metadata loads then depend on
  // nothing but the plane)
  const uint8_t* s_width = j.v[0].width;
  const int32_t* s_q0 = j.v[0].q0;
  const uint64_t* s_chunk = j.v[0].chunk_off;
  const uint32_t* s_pay = j.v[0].payload;
  uint64_t s_words = j.v[0].payload_words;
  const uint16_t* s_rel = j.rel[0];
#pragma unroll
  for (int c = 1; c < NC; ++c)
    if (c == dc) {
      s_width = j.v[c].width;
      s_q0 = j.v[c].q0;
      s_chunk = j.v[c].chunk_off;
      s_pay = j.v[c].payload;
      s_words = j.v[c].payload_words;
      s_rel = j.rel[c];
    }
  int* const drow = pl + dbase + (int)(dy - (y0 - 1)) * P;
  uint32_t* const col = stage + t;

  // stencil column of this thread
  const int ec = R::at(t + 1 + R::kOff), em = R::at(t + R::kOff), ep = R::at(t + 2 + R::kOff);
  const int64_t x = x0 + t;
  const bool active = t < xs;
  const bool ylo = y0 == 0, yhi = y0 + ys == d.y, xlo = x == 0, xhi = x == d.x - 1;
  const bool y2 = d.y >= 2, x2 = d.x >= 2;

  int ipc[NT][TY], ipp[NT][TY], zn[NT][TY], h1[NT][TY], h2[NT][TY];
#pragma unroll
  for (int k = 0; k < NT; ++k)
#pragma unroll
    for (int i = 0; i < TY; ++i) { ipc[k][i] = 0; ipp[k][i] = 0; zn[k][i] = 0; h1[k][i] = 0; h2[k][i] = 0; }

  // Staging of one plane's block: the item's metadata and the first PF
  // payload words of its block, loaded into registers ahead of use.
  constexpr int PF = 16 * (S / 32);
  struct Pending {
    int w, q0, words, e0;
    uint64_t off;
    bool valid;
    uint32_t pw[PF];
  };
  auto issue = [&](int64_t p, Pending& m) {
    m.valid = false;
    m.w = 0;
    m.words = 0;
    if (!decoder || p >= zb) return;
    const int64_t f = (p * d.y + dy) * d.x;
    const int64_t bA = (f + dxa) / S, bB = (f + dxb - 1) / S, bk = bA + dk;
    if (bk > bB) return;
    m.valid = true;
    m.w = (int)s_width[bk];
    m.q0 = s_q0[bk];
    m.off = s_chunk[bk / kChunkBlocks] + s_rel[bk];
    m.e0 = (int)(bk * S - f);
    m.words = block_words<S>(m.w);
    if (m.w > kMaxWidth || m.words > kmax || m.off + (uint64_t)m.words > s_words) {
      record_status(status, kErrBadStream);
      m.w = 0;
      m.words = 0;
    }
    prefetch_words<PF>(s_pay, s_words, m.off, m.words, m.pw);
  };
  // staged words to this thread's column, then the block into its window
  auto commit = [&](const Pending& m) {
    if (!m.valid) return;
#pragma unroll
    for (int k = 0; k < PF; ++k)
      if (k < m.words) col[k * kVThreads] = m.pw[k];
    const uint32_t* src = s_pay + m.off;
    for (int k = PF; k < m.words; ++k) col[k * kVThreads] = src[k];
    const int cb = m.e0 - (int)(x0 - 1) + R::kOff;  // extended column of slot 0 (>= 0)
    int* dst = drow + R::at(cb);
    // (a block of width 0 decodes as q0 everywhere: zero magnitudes)
    if constexpr (PAIRS) {
      if (aligned) decode_block_pairs<S, true>(col, m.w, m.q0, dst, 32);
      else decode_block_pairs<S, false>(col, m.w, m.q0, dst, 32 - (cb & 31));
    } else {
      if (aligned) decode_block_q<S, true, kVThreads>(col, m.w, m.q0, dst, 32);
      else decode_block_q<S, false, kVThreads>(col, m.w, m.q0, dst, 32 - (cb & 31));
    }
  };
  // the one-sided ghosts of this thread's column in window c (after the
  // decode barrier): rows for a window with y terms, columns for x terms
  auto ghosts = [&](int c) {
    if (!active) return;
    int* const w0 = pl + W::base(c);
    if (W::hy(c)) {
      if (ylo) w0[ec] = y2 ? 2 * w0[P + ec] - w0[2 * P + ec] : w0[P + ec];
      if (yhi) {
        int* r = w0 + ys * P + ec;
        r[P] = y2 ? 2 * r[0] - r[-P] : r[0];
      }
    }
    if (W::hx(c) && (xlo || xhi)) {
#pragma unroll
      for (int i = 0; i < TY; ++i) {
        int* r = w0 + (i + 1) * P;
        if (xlo) r[em] = x2 ? 2 * r[ec] - r[ep] : r[ec];
        if (xhi) r[ep] = x2 ? 2 * r[ec] - r[em] : r[ec];
      }
    }
  };

  // One output value of plane o per row from the numerators of its terms.
  // Every wave issues the same TY x nout buffer stores whatever the plane,
  // row or lane (a row outside the box gets a descriptor of 0 bytes, a lane
  // past the tile's columns an offset past its xs values: the hardware
  // discards both), so the wait for the next plane's payload loads, issued
  // before these stores, need not drain them.
  auto emit = [&](int64_t o, bool last) {
    const bool plane_ok = o >= z0 && o < z0 + zs;
#pragma unroll
    for (int i = 0; i < TY; ++i) {
      const bool row_ok = plane_ok && i < ys;
      const int64_t r0 = ((o - b.z0) * by + (y0 + i - b.y0)) * bx + (x0 - b.x0);
#pragma unroll
      for (int oo = 0; oo < Tm::nout; ++oo) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          const VTerm tm = Tm::t[k];
          if (tm.o != oo) continue;
          int n;
          if (tm.a == 0) n = last ? ((d.z >= 2) ? 2 * (h1[k][i] - h2[k][i]) : 0) : zn[k][i];
          else n = ipp[k][i];
          acc += (double)(tm.s * n) * j.halfq[tm.c];
        }
        T* const row = (T*)j.out[oo] + (row_ok ? r0 : 0);
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void*)row, (short)0, row_ok ? xs * (int)sizeof(T) : 0, 0x00020000);
        const int off = t * (int)sizeof(T);
        if constexpr (sizeof(T) == 4)
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, (float)acc), r, off, 0, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, acc), r, off, 0, 0);
      }
    }
  };

  // planes in order; the next plane's metadata and words load while this
  // plane's stencil runs.  Each plane's payload loads are followed by
  // exactly kStores stores (the emit of the plane before; ahead of the
  // first plane, an emit whose stores are all discarded), so one wait for
  // all but the kStores newest memory operations, at the top of every
  // iteration whatever the thread's item, retires them without draining
  // the stores.
  constexpr int kStores = TY * Tm::nout;
  static_assert(kStores < 64, "vmcnt holds 6 bits");
  // s_waitcnt immediate: vmcnt = kStores (bits 3:0 and 15:14), expcnt and
  // lgkmcnt at their maxima (no wait)
  constexpr int kWaitImm = (kStores & 15) | (7 << 4) | (15 << 8) | ((kStores >> 4) << 14);
  Pending cur, nxt;
  issue(za, cur);
  emit(za - 1, false);
  for (int64_t p = za; p < zb; ++p) {
    const int64_t o = p - 1;
    __builtin_amdgcn_s_waitcnt(kWaitImm);
    commit(cur);
    lds_barrier();
    issue(p + 1, nxt);
#pragma unroll
    for (int c = 0; c < NC; ++c) ghosts(c);
    if (active) {
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const VTerm tm = Tm::t[k];
        const int* const w0 = pl + W::base(tm.c);
#pragma unroll
        for (int i = 0; i < TY; ++i) {
          const int r = i + 1;
          const int qc = w0[r * P + ec];
          if (tm.a == 0) {
            // z numerator of plane o = p - 1; the field's first plane uses
            // the ghost 2 q_0 - q_1 below it
            if (o == 0) h2[k][i] = d.z >= 2 ? 2 * h1[k][i] - qc : h1[k][i];
            zn[k][i] = qc - h2[k][i];
            h2[k][i] = h1[k][i];
            h1[k][i] = qc;
          } else if (tm.a == 1) {
            ipc[k][i] = w0[(r + 1) * P + ec] - w0[(r - 1) * P + ec];
          } else {
            ipc[k][i] = w0[r * P + ep] - w0[r * P + em];
          }
        }
      }
    }
    lds_barrier();
    cur = nxt;
    emit(o, false);
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
      for (int i = 0; i < TY; ++i) ipp[k][i] = ipc[k][i];
  }
  // the field's last plane: one-sided in z (or 0 on a single plane)
  if (z0 + zs == zb && zb == d.z) emit(zb - 1, true);
}

template <int OP, int NC, typename T>
hipError_t vec_buf(const VecJob& j, int stage, hipStream_t s) {
  const int64_t vol = j.b.volume();
  const int64_t g = (vol + 255) / 256;
  const unsigned grid = (unsigned)(g < 65536 ? g : 65536);
  if (stage == 3) hipLaunchKernelGGL((k_vector_buf<3, OP, NC, T>), dim3(grid), dim3(256), 0, s, j);
  else hipLaunchKernelGGL((k_vector_buf<4, OP, NC, T>), dim3(grid), dim3(256), 0, s, j);
  return hipGetLastError();
}

// compute units of the current device (cached per device)
int vec_device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

template <int S, int OP, int NC, typename T>
hipError_t vec_fused(const VecJob& j0, uint8_t* ws, hipStream_t s) {
  VecJob j = j0;
  using W = VWin<S, OP, NC>;
  constexpr int TY = W::TY;
  const Box3& b = j.b;
  const int64_t ntx = (b.x1 - b.x0 + kVTx - 1) / kVTx, nty = (b.y1 - b.y0 + TY - 1) / TY;
  const int64_t bz = b.z1 - b.z0;
  const size_t lds = (size_t)W::kStageOff * 4 + (size_t)(j.kmax + 1) * kVThreads * 4;
  // z chunks: about as many workgroups as the chip holds at once (by LDS,
  // at most four of these register-heavy workgroups per compute unit), each
  // marching one chunk; chunks of at least 8 planes (two halo planes each)
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(4, (int64_t)(160 * 1024) / (int64_t)lds));
  const int64_t resident = per_cu * vec_device_cus();
  const int64_t nzc = std::max<int64_t>(1, std::min<int64_t>((resident + ntx * nty - 1) / (ntx * nty), (bz + 7) / 8));
  const int64_t tz = (bz + nzc - 1) / nzc;
  j.tz = (int)tz;
  const int64_t grid = ntx * nty * ((bz + tz - 1) / tz);
  // every block at most kVPairW bits wide (wider ones are refused as corrupt)
  if (j.kmax <= (S / 32) * (1 + kVPairW))
    hipLaunchKernelGGL((k_vector_fused<S, OP, NC, T, true>), dim3((unsigned)grid), dim3(kVThreads), lds, s, j, (int*)ws);
  else
    hipLaunchKernelGGL((k_vector_fused<S, OP, NC, T, false>), dim3((unsigned)grid), dim3(kVThreads), lds, s, j, (int*)ws);
  return hipGetLastError();
}

template <int OP, typename T>
hipError_t by_nc_buf(const VecJob& j, int stage, hipStream_t s) {
  if constexpr (OP == kOpDivergence) {
    if (j.nc == 1) return vec_buf<OP, 1, T>(j, stage, s);
    if (j.nc == 2) return vec_buf<OP, 2, T>(j, stage, s);
    return vec_buf<OP, 3, T>(j, stage, s);
  } else {
    if (j.nc == 2) return vec_buf<OP, 2, T>(j, stage, s);
    return vec_buf<OP, 3, T>(j, stage, s);
  }
}

template <int S, int OP, typename T>
hipError_t by_nc_fused(const VecJob& j, uint8_t* ws, hipStream_t s) {
  if constexpr (OP == kOpDivergence) {
    if (j.nc == 1) return vec_fused<S, OP, 1, T>(j, ws, s);
    if (j.nc == 2) return vec_fused<S, OP, 2, T>(j, ws, s);
    return vec_fused<S, OP, 3, T>(j, ws, s);
  } else {
    if (j.nc == 2) return vec_fused<S, OP, 2, T>(j, ws, s);
    return vec_fused<S, OP, 3, T>(j, ws, s);
  }
}

template <int S, typename T>
hipError_t fused_s(const VecJob& j, uint8_t* ws, hipStream_t s) {
  return j.op == kOpDivergence ? by_nc_fused<S, kOpDivergence, T>(j, ws, s) : by_nc_fused<S, kOpCurl, T>(j, ws, s);
}

}  // namespace

template <int OP, int NC>
int terms_of(int* c, int* a, int* s, int* o, int* nout) {
  using Tm = VTerms<OP, NC>;
  for (int k = 0; k < Tm::n; ++k) {
    c[k] = Tm::t[k].c;
    a[k] = Tm::t[k].a;
    s[k] = Tm::t[k].s;
    o[k] = Tm::t[k].o;
  }
  *nout = Tm::nout;
  return Tm::n;
}

int vector_terms(int op, int nc, int* c, int* a, int* s, int* o, int* nout) {
  if (op == kOpDivergence) {
    if (nc == 1) return terms_of<kOpDivergence, 1>(c, a, s, o, nout);
    if (nc == 2) return terms_of<kOpDivergence, 2>(c, a, s, o, nout);
    if (nc == 3) return terms_of<kOpDivergence, 3>(c, a, s, o, nout);
  } else if (op == kOpCurl) {
    if (nc == 2) return terms_of<kOpCurl, 2>(c, a, s, o, nout);
    if (nc == 3) return terms_of<kOpCurl, 3>(c, a, s, o, nout);
  }
  return 0;
}

uint64_t vector_workspace_bytes(const int64_t* nb, int nc) {
  uint64_t off = kGradIndexOff;
  for (int c = 0; c < nc; ++c) off += ((2 * (uint64_t)nb[c] + 255) / 256) * 256;
  return off;
}

hipError_t launch_vector_stage(const VecJob& j, int stage, int dtype, hipStream_t s) {
  if (j.op == kOpDivergence)
    return dtype == 1 ? by_nc_buf<kOpDivergence, float>(j, stage, s) : by_nc_buf<kOpDivergence, double>(j, stage, s);
  return dtype == 1 ? by_nc_buf<kOpCurl, float>(j, stage, s) : by_nc_buf<kOpCurl, double>(j, stage, s);
}

hipError_t launch_vector_fused(const VecJob& j0, uint8_t* ws, hipStream_t s) {
  VecJob j = j0;
  // per-component block indexes in the workspace after the status words
  uint64_t off = kGradIndexOff;
  int kmax = 1;
  for (int c = 0; c < j.nc; ++c) {
    uint16_t* rel = (uint16_t*)(ws + off);
    hipError_t e = launch_block_index(j.v[c], rel, s);
    if (e != hipSuccess) return e;
    j.rel[c] = rel;
    off += ((2 * (uint64_t)j.v[c].nb + 255) / 256) * 256;
    kmax = std::max(kmax, grad_kmax(j.v[c]));
  }
  j.kmax = kmax;
  const int dtype = j.v[0].dtype, S = j.v[0].block;
  if (S == 32) return dtype == 1 ? fused_s<32, float>(j, ws, s) : fused_s<32, double>(j, ws, s);
  return dtype == 1 ? fused_s<64, float>(j, ws, s) : fused_s<64, double>(j, ws, s);
}

}  // namespace hsz
