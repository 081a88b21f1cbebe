// ops.hip -- analytical operations Q_i on the stages (Sec. V): mean and
// sample variance (Eq. (var), Sec. V-A), derivatives and gradient magnitude
// (Eq. (derivatives), Sec. V-B), on materialised stage buffers and fused
// with decoding straight from the compressed stream.
//
// Integer routes (stages 2 and 3) accumulate exact sums of q and q^2
// (int64 and 128-bit) and scale by the quantum once, in the finalize kernel.
// The stage-2 mean uses the block-sum identity of Sec. V-A for SZp
// (sum_i q_i = S_b*q0 + sum_{i>=1} (S_b - i) p_i, generalised to a slot
// range [a, z] of the block) and never forms q.  The stage-4 routes work on
// floats in binary64, shifted by the box's first value.
#include <algorithm>

#include "hsz_device.hpp"
#include "hsz_launch.hpp"
#include "hsz_nd.hpp"
#include "hsz_stats.hpp"

namespace hsz {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerGroup = kThreads / kWave;
constexpr uint64_t kPartialOff = 256;
constexpr uint64_t kMetaOff = 64;  // finalized metadata sum (op 8), 48 bytes

// Per-workgroup partial: integer sums or binary64 sums.
struct Partial {
  int64_t s1;
  uint64_t s2lo, s2hi;
  int64_t cnt;
  double f1, f2;
  double pad0, pad1;
};

// ---- accumulation helpers ------------------------------------------------------
struct IntAcc {
  int64_t s1 = 0;
  U128 s2 = {0, 0};
  int64_t cnt = 0;
  __device__ void add(int q, bool want_sq) {
    s1 += q;
    if (want_sq) add_u64(s2, (uint64_t)((int64_t)q * (int64_t)q));
    cnt += 1;
  }
};

// Reduce a lane's integer accumulators over the workgroup and store one
// partial per workgroup.
__device__ void store_int_partial(IntAcc a, Partial* parts) {
  __shared__ int64_t ss1[kWavesPerGroup], scnt[kWavesPerGroup];
  __shared__ uint64_t slo[kWavesPerGroup], shi[kWavesPerGroup];
  // 128-bit sum across lanes: add the low words as 64-bit with carries
  // counted through the high words (lane values of s2.lo are < 2^64).
  int64_t s1 = wave_sum64(a.s1);
  int64_t cnt = wave_sum64(a.cnt);
  U128 s2 = a.s2;
  for (int m = 32; m >= 1; m >>= 1) {
    U128 o;
    o.lo = __shfl_xor(s2.lo, m);
    o.hi = __shfl_xor(s2.hi, m);
    add_u128(s2, o);
  }
  const int wv = wave_in_group();
  if (lane_id() == 0) { ss1[wv] = s1; scnt[wv] = cnt; slo[wv] = s2.lo; shi[wv] = s2.hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kWavesPerGroup; ++k) {
      s1 += ss1[k];
      cnt += scnt[k];
      add_u128(s2, U128{slo[k], shi[k]});
    }
    Partial p{};
    p.s1 = s1; p.s2lo = s2.lo; p.s2hi = s2.hi; p.cnt = cnt;
    parts[blockIdx.x] = p;
  }
}

__device__ void store_f64_partial(double f1, double f2, int64_t cnt, double K, Partial* parts) {
  __shared__ double sf1[kWavesPerGroup], sf2[kWavesPerGroup];
  __shared__ int64_t scnt[kWavesPerGroup];
  f1 = wave_sum_f64(f1);
  f2 = wave_sum_f64(f2);
  cnt = wave_sum64(cnt);
  const int wv = wave_in_group();
  if (lane_id() == 0) { sf1[wv] = f1; sf2[wv] = f2; scnt[wv] = cnt; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kWavesPerGroup; ++k) { f1 += sf1[k]; f2 += sf2[k]; cnt += scnt[k]; }
    Partial p{};
    p.f1 = f1; p.f2 = f2; p.cnt = cnt; p.pad0 = K;
    parts[blockIdx.x] = p;
  }
}

// ---- stats on a stage-3 buffer (q) or stage-4 buffer (floats) -------------------
constexpr int64_t kSeg = 4096;

template <int OP>
__global__ void __launch_bounds__(kThreads) k_stats_q(const int32_t* __restrict__ q, Rows rows, Partial* parts) {
  IntAcc acc;
  const int64_t segs = (rows.len + kSeg - 1) / kSeg;
  const int64_t items = rows.count() * segs;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t r = it / segs, sg = it % segs;
    const int64_t lo = sg * kSeg, hi = min(rows.len, lo + kSeg);
    const int32_t* src = q + rows.start(r);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) acc.add(src[i], OP == 2);
  }
  store_int_partial(acc, parts);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_stats_f(const T* __restrict__ x, Rows rows, Partial* parts) {
  const double K = (double)x[rows.base];
  double f1 = 0.0, f2 = 0.0;
  int64_t cnt = 0;
  const int64_t segs = (rows.len + kSeg - 1) / kSeg;
  const int64_t items = rows.count() * segs;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t r = it / segs, sg = it % segs;
    const int64_t lo = sg * kSeg, hi = min(rows.len, lo + kSeg);
    const T* src = x + rows.start(r);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
      const double e = (double)src[i] - K;
      f1 += e;
      f2 += e * e;
      cnt += 1;
    }
  }
  store_f64_partial(f1, f2, cnt, K, parts);
}

// ---- whole contiguous ranges: 16-byte loads, four in flight per thread ----------
// Used when the box is one contiguous, 4-element-aligned flat range (the whole
// field, or whole planes).  Elements [0, len) of 'src'.
constexpr int kUnroll = 4;

template <int OP>
__global__ void __launch_bounds__(kThreads) k_stats_q_flat(const int32_t* __restrict__ q, int64_t len,
                                                          Partial* parts) {
  IntAcc acc;
  typedef int32_t i4 __attribute__((ext_vector_type(4)));
  const i4* v4 = (const i4*)q;
  const int64_t nv = len / 4;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
    i4 t[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) t[u] = v4[i + u * stride];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      acc.add(t[u].x, OP == 2); acc.add(t[u].y, OP == 2); acc.add(t[u].z, OP == 2); acc.add(t[u].w, OP == 2);
    }
  }
  for (; i < nv; i += stride) {
    const i4 t = v4[i];
    acc.add(t.x, OP == 2); acc.add(t.y, OP == 2); acc.add(t.z, OP == 2); acc.add(t.w, OP == 2);
  }
  if (blockIdx.x == 0 && threadIdx.x < (len & 3)) acc.add(q[nv * 4 + threadIdx.x], OP == 2);
  store_int_partial(acc, parts);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_stats_f_flat(const T* __restrict__ x, int64_t len, Partial* parts) {
  constexpr int kPer = 16 / sizeof(T);
  typedef T vt __attribute__((ext_vector_type(kPer)));
  const double K = (double)x[0];
  double f1 = 0.0, f2 = 0.0;
  int64_t cnt = 0;
  const vt* v = (const vt*)x;
  const int64_t nv = len / kPer;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  auto add = [&](T val) {
    const double e = (double)val - K;
    f1 += e;
    f2 += e * e;
  };
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * stride < nv; i += kUnroll * stride) {
    vt t[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) t[u] = v[i + u * stride];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int k = 0; k < kPer; ++k) add(t[u][k]);
    cnt += kUnroll * kPer;
  }
  for (; i < nv; i += stride) {
    const vt t = v[i];
#pragma unroll
    for (int k = 0; k < kPer; ++k) add(t[k]);
    cnt += kPer;
  }
  if (blockIdx.x == 0 && threadIdx.x < (len % kPer)) {
    add(x[nv * kPer + threadIdx.x]);
    cnt += 1;
  }
  store_f64_partial(f1, f2, cnt, K, parts);
}

// Stage 2 over the whole field: thread i holds p[4i .. 4i+3] (one block is
// S/4 consecutive threads).  Mean: sum_j (S_b - j) p_j per block plus
// S_b q0_b (the q0 term is added by the thread holding slot 0).  Variance:
// in-thread prefix, then an exclusive scan over the block's S/4 threads.
template <int S, int OP>
__global__ void __launch_bounds__(kThreads) k_stats_delta_flat(const int32_t* __restrict__ p,
                                                              const int32_t* __restrict__ q0s, int64_t n,
                                                              int64_t nb, Partial* parts) {
  constexpr int G = S / 4;  // threads per block
  IntAcc acc;
  typedef int32_t i4 __attribute__((ext_vector_type(4)));
  const i4* v4 = (const i4*)p;
  const int64_t nvec = nb * G;  // vectors covering whole blocks (the tail is read element-wise)
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t base = blockIdx.x * (int64_t)kThreads; base < nvec; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool ok = i < nvec;
    const int64_t b = i / G;
    const int j0 = (int)(i % G) * 4;
    const int64_t e0 = i * 4;
    int t4[4] = {0, 0, 0, 0};
    if (ok) {
      if (e0 + 4 <= n) {
        const i4 t = v4[i];
        t4[0] = t.x; t4[1] = t.y; t4[2] = t.z; t4[3] = t.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) t4[u] = (e0 + u < n) ? p[e0 + u] : 0;
      }
    }
    const int sb = ok ? (int)min((int64_t)S, n - b * S) : 0;  // the block's valid length
    const int q0 = (ok && j0 == 0) || OP == 2 ? (ok ? q0s[b] : 0) : 0;
    if constexpr (OP == 1) {
      int64_t s = (j0 == 0) ? (int64_t)sb * q0 : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u < sb) s += (int64_t)(sb - (j0 + u)) * t4[u];
      acc.s1 += s;
      acc.cnt += max(0, min(4, sb - j0));
    } else {
      int run = t4[0] + t4[1] + t4[2] + t4[3];
      int incl = run;
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        const int o = __shfl_up(incl, d, G);
        if ((int)(i % G) >= d) incl += o;
      }
      int q = q0 + incl - run;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        q += t4[u];
        if (ok && j0 + u < sb) acc.add(q, true);
      }
    }
  }
  store_int_partial(acc, parts);
}

// Stage-2 statistics from a p buffer (p[n], q0[nb]).
template <int S, int OP>
__global__ void __launch_bounds__(kThreads) k_stats_delta(const int32_t* __restrict__ p,
                                                         const int32_t* __restrict__ q0s, Segs<S> segs,
                                                         Partial* parts) {
  IntAcc acc;
  const int64_t items = segs.count();
  for (int64_t it = blockIdx.x * (int64_t)kThreads + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * kThreads) {
    int64_t b;
    int a, z;
    if (!segs.get(it, b, a, z)) continue;
    const int32_t* pb = p + b * S;
    const int q0 = q0s[b];
    if constexpr (OP == 1) {
      // sum_{i=a}^{z} q_i = (z-a+1) q0 + sum_{t=1}^{z} (z - max(a,t) + 1) p_t
      int64_t s = (int64_t)(z - a + 1) * q0;
      for (int t = 1; t <= z; ++t) s += (int64_t)(z - (a > t ? a : t) + 1) * pb[t];
      acc.s1 += s;
      acc.cnt += z - a + 1;
    } else {
      int q = q0;
      for (int t = 0; t <= z; ++t) {
        if (t > 0) q += pb[t];
        if (t >= a) acc.add(q, true);
      }
    }
  }
  store_int_partial(acc, parts);
}

// ---- block-mean streams (HSZx) ---------------------------------------------------------
// Stage-2 buffer (p[n], M[nb]) of a block-mean stream: q = M_b + p over the
// box rows (the D_p mean of Sec. V-A: sum_b (sum p + M_b S_b)).
template <int S, int OP>
__global__ void __launch_bounds__(kThreads) k_stats_delta_mean(const int32_t* __restrict__ p,
                                                              const int32_t* __restrict__ ms, Rows rows,
                                                              Partial* parts) {
  IntAcc acc;
  const int64_t segs = (rows.len + kSeg - 1) / kSeg;
  const int64_t items = rows.count() * segs;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t r = it / segs, sg = it % segs;
    const int64_t lo = sg * kSeg, hi = min(rows.len, lo + kSeg);
    const int64_t f0 = rows.start(r);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) acc.add(ms[(f0 + i) / S] + p[f0 + i], OP == 2);
  }
  store_int_partial(acc, parts);
}

// Eq. (mean_m): the mean from the metadata alone, sum_b M_b S_b (S_b = S but
// for a shorter last block), as an exact integer partial per workgroup.
__global__ void __launch_bounds__(kThreads) k_meta_mean(const int32_t* __restrict__ ms, int64_t n, int64_t nb,
                                                       int S, Partial* parts) {
  IntAcc acc;
  for (int64_t b = blockIdx.x * (int64_t)kThreads + threadIdx.x; b < nb; b += (int64_t)gridDim.x * kThreads) {
    const int64_t sb = min((int64_t)S, n - b * S);
    acc.s1 += (int64_t)ms[b] * sb;
    acc.cnt += sb;
  }
  store_int_partial(acc, parts);
}

// ---- whole blocks of streams with small integers -----------------------------------
// Exact sums over one whole block (slots 0 .. S-1 all counted) when the
// stream's max|q| is below small_q_limit<MODE>(): the block's terms are
// summed in 32 bits with 24-bit multiply-adds and widened once per block.
//   MODE 0, the stage-2 block sum S q0 + sum_{j>=1} (S - j) p_j: |p| < 2^23
//     fits the 24-bit operands, terms are below 2^29 and every partial sum
//     is bounded by 2 S max|q| < 2^29 (summation by parts);
//   MODE 1, sum q: below S 2^22;
//   MODE 2, sum q and sum q^2: q^2 < 2^26 and S q^2 < 2^32 (unsigned).
template <int MODE>
__host__ __device__ constexpr uint32_t small_q_limit() { return MODE == 2 ? 8192u : (1u << 22); }

// MEAN: a block-mean stream (q0 = M): the stage-2 block sum is S M + sum p.
template <int S, int MODE, bool MEAN = false>
__device__ __forceinline__ void whole_block_sums(const uint32_t* col, int w, int q0, IntAcc& a) {
  int s1 = 0;
  uint32_t s2 = 0;
  if constexpr (MODE == 0 && MEAN) {
    decode_lane_block<S, kWave, true>(col, w, q0, [&](int, int p, int) { s1 += p; });
    a.s1 += (int64_t)S * q0 + s1;
  } else if constexpr (MODE == 0) {
    decode_lane_block<S>(col, w, q0, [&](int j, int p, int) {
      if (j >= 1) s1 = __mul24(S - j, p) + s1;
    });
    a.s1 += (int64_t)S * q0 + s1;
  } else {
    decode_lane_block<S, kWave, MEAN>(col, w, q0, [&](int, int, int q) {
      s1 += q;
      if constexpr (MODE == 2) s2 = (uint32_t)__mul24(q, q) + s2;
    });
    a.s1 += s1;
    if constexpr (MODE == 2) add_u64(a.s2, (uint64_t)s2);
  }
  a.cnt += S;
}

// ---- fused statistics straight from the compressed stream ------------------------
// VIA: 2 (decorrelated), 3 (quantized), 4 (floats).  WHOLE: the items are
// every block in order (chunk-aligned waves use the chunk scan).
template <int S, int VIA, int OP, typename T, bool WHOLE, bool MEAN>
__global__ void __launch_bounds__(kThreads) k_stats_fused(StreamView v, Segs<S> segs, int kmax, const double* Kp,
                                                         Partial* parts, int* status) {
  extern __shared__ uint32_t smem[];
  const int wv = wave_in_group();
  uint32_t* tile = smem + wv * (kmax + 1) * kWave;
  const int l = lane_id();
  IntAcc acc;
  double f1 = 0.0, f2 = 0.0;
  int64_t fcnt = 0;
  const double quantum = v.quantum;
  const double K = (VIA == 4) ? *Kp : 0.0;
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  const int64_t items = WHOLE ? v.nchunks * kChunkBlocks : segs.count();
  constexpr int kMode = (VIA == 2 && OP == 1) ? 0 : OP;
  const bool small = v.max_abs_q < small_q_limit<kMode>();
  // one block of the lane: slots a..z counted
  auto process = [&](int w, int q0, int a, int z) {
    if constexpr (VIA != 4) {
      if (small && a == 0 && z == S - 1) {
        whole_block_sums<S, kMode, MEAN>(tile + l, w, q0, acc);
        return;
      }
    }
    if constexpr (VIA == 2 && OP == 1 && MEAN) {
      // block-mean stream: (z - a + 1) M + the sum of its deltas
      int64_t s = (int64_t)(z - a + 1) * q0;
      decode_lane_block<S, kWave, true>(tile + l, w, q0, [&](int j, int p, int) {
        if (j >= a && j <= z) s += p;
      });
      acc.s1 += s;
      acc.cnt += z - a + 1;
    } else if constexpr (VIA == 2 && OP == 1) {
      // weighted block sum, no recorrelation
      int64_t s = (int64_t)(z - a + 1) * q0;
      decode_lane_block<S>(tile + l, w, q0, [&](int j, int p, int) {
        if (j >= 1 && j <= z) s += (int64_t)(z - (a > j ? a : j) + 1) * p;
      });
      acc.s1 += s;
      acc.cnt += z - a + 1;
    } else if constexpr (VIA == 4) {
      decode_lane_block<S, kWave, MEAN>(tile + l, w, q0, [&](int j, int, int q) {
        if (j >= a && j <= z) {
          const double e = (double)(T)dequant64(q, quantum) - K;
          f1 += e;
          f2 += e * e;
          fcnt += 1;
        }
      });
    } else {
      decode_lane_block<S, kWave, MEAN>(tile + l, w, q0, [&](int j, int, int q) {
        if (j >= a && j <= z) acc.add(q, OP == 2);
      });
    }
  };
  if constexpr (WHOLE) {
    // chunks c, c + W, ... (W = waves of the grid); the next chunk's
    // metadata and first words load while this one decodes
    constexpr int PF = 16;
    int64_t c = blockIdx.x * (int64_t)kWavesPerGroup + wv;
    ChunkStage<PF> cs;
    if (c < v.nchunks)
      chunk_begin<S, PF>(v.width, v.q0, v.chunk_off, v.payload, v.payload_words, v.n, v.nb, c, kmax, cs, status);
    for (; c < v.nchunks; c += waves) {
      chunk_end<PF>(cs, tile);
      const LaneBlock lb = cs.lb;
      if (c + waves < v.nchunks)
        chunk_begin<S, PF>(v.width, v.q0, v.chunk_off, v.payload, v.payload_words, v.n, v.nb, c + waves, kmax, cs,
                           status);
      if (lb.len > 0) process(lb.w, lb.q0, 0, lb.len - 1);
    }
  } else {
    for (int64_t base = (blockIdx.x * (int64_t)kWavesPerGroup + wv) * kWave; base < items; base += waves * kWave) {
      const int64_t it = base + l;
      int64_t b;
      int a = 0, z = -1, q0 = 0, w = 0;
      if (it < items && segs.get(it, b, a, z))
        w = stage_block<S, kWave>(v.width, v.q0, v.chunk_off, v.payload, v.payload_words, v.nb, b, tile + l, kmax,
                                  q0, status);
      else
        z = -1;
      if (z >= 0) process(w, q0, a, z);
    }
  }
  if constexpr (VIA == 4) store_f64_partial(f1, f2, fcnt, K, parts);
  else store_int_partial(acc, parts);
}

// ---- finalize: partials -> hsz_stats (StatsOut, stats_from_sums) ---------------------
__global__ void k_copy_status_word(const int* status, int* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = *status;
}

// an error in *src becomes *dst's unless *dst holds one already
__global__ void k_merge_status_word(const int* src, int* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *src != 0) atomicCAS(dst, 0, *src);
}

// Records of the same field's slabs (each its own exact sums) combined into
// one: the sums add exactly (int64, 128 bits) and are finished once.
__global__ void k_stats_combine(const StatsOut* rec, int K, int op, double quantum, StatsOut* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t n = 0, s1 = 0;
  unsigned __int128 s2 = 0;
  for (int k = 0; k < K; ++k) {
    n += rec[k].n;
    s1 += rec[k].s1;
    s2 += ((unsigned __int128)(uint64_t)rec[k].s2hi << 64) | rec[k].s2lo;
  }
  *out = stats_from_sums(n, s1, (uint64_t)s2, (uint64_t)(s2 >> 64), op, quantum);
}

// The standard deviation on D_p of a block-mean stream (Sec. V-A) is taken
// about the integer mean mu~ = round(sum_b M_b S_b / n), halves down like the
// block means.  With the exact sums s1 = sum q and s2 = sum q^2 the spread is
// sum (q - mu~)^2 = s2 - 2 mu~ s1 + n mu~^2, an exact 128-bit integer equal
// to the paper's sum over blocks of (p + M_b - mu~)^2.  The result holds n,
// s1 = sum_b M_b S_b, s2 = that spread, mean = mu~ Delta and var = spread /
// (n - 1) Delta^2.
__device__ int64_t round_half_down_div(int64_t a, int64_t b) {
  const int64_t num = 2 * a - b, den = 2 * b;
  return num >= 0 ? (num + den - 1) / den : -((-num) / den);
}

__device__ StatsOut stats_about_meta_mean(int64_t n, int64_t s1, uint64_t s2lo, uint64_t s2hi, int64_t msum,
                                          double quantum) {
  StatsOut r{};
  const int64_t mt = round_half_down_div(msum, n);
  const __int128 S2 = (__int128)(((unsigned __int128)s2hi << 64) | s2lo);
  const __int128 spread = S2 - (__int128)2 * mt * s1 + (__int128)n * ((__int128)mt * mt);
  r.n = n;
  r.s1 = msum;
  r.s2lo = (uint64_t)spread;
  r.s2hi = (int64_t)(spread >> 64);
  r.mean = (double)mt * quantum;
  r.var = n > 1 ? u128_to_f64((unsigned __int128)spread) / (double)(n - 1) * (quantum * quantum)
                : __builtin_nan("");
  return r;
}

// One workgroup of 256 threads: thread t sums partials t, t+256, ... in
// order, then a fixed-shape tree combines the 256 sums, so the result does
// not depend on timing.  op 8 takes the metadata sum from 'meta' (the
// finalized k_meta_mean of the same stream).
constexpr int kFinThreads = 256;

__global__ void __launch_bounds__(kFinThreads) k_finalize(const Partial* parts, int groups, int op, int fl,
                                                          double quantum, const StatsOut* meta, StatsOut* out) {
  __shared__ int64_t s1s[kFinThreads], cnts[kFinThreads];
  __shared__ uint64_t los[kFinThreads], his[kFinThreads];
  __shared__ double f1s[kFinThreads], f2s[kFinThreads];
  const int t = threadIdx.x;
  int64_t s1 = 0, cnt = 0;
  U128 s2 = {0, 0};
  double f1 = 0.0, f2 = 0.0;
  for (int g = t; g < groups; g += kFinThreads) {
    const Partial p = parts[g];
    s1 += p.s1;
    cnt += p.cnt;
    add_u128(s2, U128{p.s2lo, p.s2hi});
    f1 += p.f1;
    f2 += p.f2;
  }
  s1s[t] = s1; cnts[t] = cnt; los[t] = s2.lo; his[t] = s2.hi; f1s[t] = f1; f2s[t] = f2;
  __syncthreads();
  for (int half = kFinThreads / 2; half >= 1; half >>= 1) {
    if (t < half) {
      s1s[t] += s1s[t + half];
      cnts[t] += cnts[t + half];
      U128 a{los[t], his[t]};
      add_u128(a, U128{los[t + half], his[t + half]});
      los[t] = a.lo;
      his[t] = a.hi;
      f1s[t] += f1s[t + half];
      f2s[t] += f2s[t + half];
    }
    __syncthreads();
  }
  if (t != 0) return;
  StatsOut r{};
  r.n = cnts[0];
  const int64_t n = cnts[0];
  if (op == kOpVarMetaMean) {
    r = stats_about_meta_mean(n, s1s[0], los[0], his[0], meta->s1, quantum);
  } else if (!fl) {
    r = stats_from_sums(n, s1s[0], los[0], his[0], op, quantum);
  } else {
    const double K = parts[0].pad0;
    r.mean = K + f1s[0] / (double)n;
    r.var = (op == 2 && n > 1) ? (f2s[0] - f1s[0] * f1s[0] / (double)n) / (double)(n - 1) : __builtin_nan("");
  }
  *out = r;
}

// ---- batches: many jobs, one persistent launch --------------------------------------
// Integer-route statistics of every job of one block size.  Units: a chunk
// of a whole field, or 64 block segments of a box.  A wave walks the units
// u = wave, wave + W, ...; it accumulates per job and adds its sums to the
// job's accumulator with 64-bit atomics when the job changes (the 128-bit
// sum of q^2 carries by hand).  Integer atomics make the totals exact and
// independent of the schedule, so a job's result equals the one-op result.
// One unit of a statistics job: MODE 0 = weighted delta sum (mean through
// D_p), 1 = sum of q, 2 = sums of q and q^2.
template <int S, int MODE, bool WHOLE>
__device__ __forceinline__ void stats_unit(const StatsJob& J, int64_t lu, uint32_t* tile, int kmax, IntAcc& a,
                                           int* status) {
  const int l = lane_id();
  int w = 0, q0 = 0, sa = 0, sz = -1;
  if constexpr (WHOLE) {
    LaneBlock lb;
    stage_chunk<S>(J.v.width, J.v.q0, J.v.chunk_off, J.v.payload, J.v.payload_words, J.v.n, J.v.nb, lu, tile, kmax,
                   lb, status);
    w = lb.w; q0 = lb.q0; sz = lb.len - 1;
  } else {
    Segs<S> segs;
    segs.rows = J.rows;
    segs.per_row = J.per_row;
    int64_t b;
    if (lu * kWave + l < segs.count() && segs.get(lu * kWave + l, b, sa, sz))
      w = stage_block<S, kWave>(J.v.width, J.v.q0, J.v.chunk_off, J.v.payload, J.v.payload_words, J.v.nb, b,
                                tile + l, kmax, q0, status, J.rel);
    else
      sz = -1;
  }
  if (sz < 0) return;
  if (J.v.max_abs_q < small_q_limit<MODE>() && sa == 0 && sz == S - 1) {
    whole_block_sums<S, MODE>(tile + l, w, q0, a);
    return;
  }
  if constexpr (MODE == 0) {
    int64_t s = (int64_t)(sz - sa + 1) * q0;
    decode_lane_block<S>(tile + l, w, q0, [&](int j, int p, int) {
      if (j >= 1 && j <= sz) s += (int64_t)(sz - (sa > j ? sa : j) + 1) * p;
    });
    a.s1 += s;
    a.cnt += sz - sa + 1;
  } else {
    decode_lane_block<S>(tile + l, w, q0, [&](int j, int, int q) {
      if (j >= sa && j <= sz) a.add(q, MODE == 2);
    });
  }
}

// ---- batches: many jobs, one persistent launch --------------------------------------
// Integer-route statistics of every job of one block size.  Units: a chunk
// of a whole field, or 64 block segments of a box.  A wave walks the units
// u = wave, wave + W, ... (increasing, so the job index only moves forward);
// it accumulates per job and adds its sums to the job's accumulator with
// 64-bit atomics when the job changes (the 128-bit sum of q^2 carries by
// hand).  Integer atomics make the totals exact and independent of the
// schedule, so a job's result equals the one-op result.  The job entry and
// the unit index are wave-uniform, so the table is read with scalar loads.
template <int S>
__global__ void __launch_bounds__(kThreads) k_batch_stats(const StatsJob* __restrict__ jobs,
                                                         const int64_t* __restrict__ unit_start,
                                                         const int64_t* __restrict__ counts, int kmax,
                                                         BatchAcc* __restrict__ acc, int* status) {
  extern __shared__ uint32_t smem[];
  const int wv = wave_in_group();
  uint32_t* tile = smem + wv * (kmax + 1) * kWave;
  const int n = (int)counts[0];
  const int64_t total = counts[1];
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  IntAcc a;
  auto flush = [&](int slot) {
    acc_add_wave(acc + (int64_t)slot * kAccStripes, a.s1, a.cnt, a.s2);
    a = IntAcc{};
  };
  int64_t u = blockIdx.x * (int64_t)kWavesPerGroup + wv;
  if (u >= total) return;
  int cur = 0;  // last job whose first unit is <= u
  while (cur + 1 < n && unit_start[cur + 1] <= u) ++cur;
  StatsJob J = load_job(jobs, cur);
  int64_t first = unit_start[cur], next = cur + 1 < n ? unit_start[cur + 1] : total;
  int mode = J.via == 2 && J.op == 1 ? 0 : J.op == 2 ? 2 : 1;
  for (; u < total; u += waves) {
    if (u >= next) {
      flush(J.acc);
      while (cur + 1 < n && unit_start[cur + 1] <= u) ++cur;
      J = load_job(jobs, cur);
      first = unit_start[cur];
      next = cur + 1 < n ? unit_start[cur + 1] : total;
      mode = J.via == 2 && J.op == 1 ? 0 : J.op == 2 ? 2 : 1;
    }
    const int64_t lu = u - first;
    if (J.whole) {
      if (mode == 0) stats_unit<S, 0, true>(J, lu, tile, kmax, a, status);
      else if (mode == 1) stats_unit<S, 1, true>(J, lu, tile, kmax, a, status);
      else stats_unit<S, 2, true>(J, lu, tile, kmax, a, status);
    } else {
      if (mode == 0) stats_unit<S, 0, false>(J, lu, tile, kmax, a, status);
      else if (mode == 1) stats_unit<S, 1, false>(J, lu, tile, kmax, a, status);
      else stats_unit<S, 2, false>(J, lu, tile, kmax, a, status);
    }
  }
  flush(J.acc);
}

// status[0] is the status word; status[1] and status[2] are the live word
// and the done count of a batch that finishes itself (BatchTail)
__global__ void k_batch_reset(BatchAcc* acc, int slots, int* status) {
  const int n = slots * kAccStripes;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc[i] = BatchAcc{0, 0, 0, 0};
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    status[0] = 0;
    status[1] = 0;
    status[2] = 0;
  }
}

struct FinalizeArgs {
  const StatsJob* jobs[2];
  const int64_t* counts[2];
  const BatchAcc* acc[2];
  int n0;
};

// One wave per job of either class (finish_stats_job).
__global__ void __launch_bounds__(256) k_batch_finalize(FinalizeArgs fa) {
  const int w = blockIdx.x * (blockDim.x / kWave) + wave_in_group();
  const int c = w < fa.n0 ? 0 : 1;
  const int i = c ? w - fa.n0 : w;
  if (i >= (int)fa.counts[c][0]) return;
  const StatsJob J = load_job(fa.jobs[c], i);
  finish_stats_job<false>(J, fa.acc[c] + (int64_t)J.acc * kAccStripes);
}

int grid_for(int64_t work_items, int per_group) {
  int64_t g = (work_items + per_group - 1) / per_group;
  if (g < 1) g = 1;
  return (int)(g < kOpWorkgroups ? g : kOpWorkgroups);
}

int kmax_for(const StreamView& v) {
  int wmax = 32 - __builtin_clz(2u * v.max_abs_q | 1u);
  wmax = wmax < 1 ? 1 : (wmax > kMaxWidth ? kMaxWidth : wmax);
  return (v.block / 32) * (1 + wmax);
}

// One wave: decode the value at flat index f (the shift of the binary64
// float-route sums) into *K.
template <int S, typename T, bool MEAN>
__global__ void k_first_value(StreamView v, int64_t f, int kmax, double* K, int* status) {
  extern __shared__ uint32_t smem[];
  const int64_t b = f / S;
  const int slot = (int)(f - b * S);
  int q0 = 0;
  const int w = lane_id() == 0 ? stage_block<S, kWave>(v.width, v.q0, v.chunk_off, v.payload, v.payload_words, v.nb, b, smem, kmax, q0, status) : 0;
  if (lane_id() != 0) return;
  int qv = 0;
  decode_lane_block<S, kWave, MEAN>(smem, w, q0, [&](int j, int, int q) {
    if (j == slot) qv = q;
  });
  *K = (double)(T)dequant64(qv, v.quantum);
}

template <int S, int VIA, int OP, typename T, bool MEAN>
hipError_t run_fused_stats_m(const StreamView& v, const Rows& rows, bool whole, double* K, Partial* parts, int& grid,
                             int* status, hipStream_t s) {
  const int kmax = kmax_for(v);
  const size_t lds = (size_t)kWavesPerGroup * (kmax + 1) * kWave * sizeof(uint32_t);
  Segs<S> segs = make_segs<S>(rows);
  if (VIA == 4)
    hipLaunchKernelGGL((k_first_value<S, T, MEAN>), dim3(1), dim3(kWave), (kmax + 1) * kWave * sizeof(uint32_t), s, v,
                       rows.base, kmax, K, status);
  const int64_t items = whole ? v.nchunks * kChunkBlocks : segs.count();
  grid = grid_for(items, kThreads);
  if (whole)
    hipLaunchKernelGGL((k_stats_fused<S, VIA, OP, T, true, MEAN>), dim3(grid), dim3(kThreads), lds, s, v, segs,
                       kmax, K, parts, status);
  else
    hipLaunchKernelGGL((k_stats_fused<S, VIA, OP, T, false, MEAN>), dim3(grid), dim3(kThreads), lds, s, v, segs,
                       kmax, K, parts, status);
  return hipGetLastError();
}

template <int S, int VIA, int OP, typename T>
hipError_t run_fused_stats(const StreamView& v, const Rows& rows, bool whole, double* K, Partial* parts, int& grid,
                           int* status, hipStream_t s) {
  return (v.flags & 1u) ? run_fused_stats_m<S, VIA, OP, T, true>(v, rows, whole, K, parts, grid, status, s)
                        : run_fused_stats_m<S, VIA, OP, T, false>(v, rows, whole, K, parts, grid, status, s);
}

template <int S, int OP>
hipError_t fused_by_via(const StreamView& v, int via, const Rows& rows, bool whole, double* K, Partial* parts,
                        int& grid, int* status, hipStream_t s) {
  switch (via) {
    case 2: return run_fused_stats<S, 2, OP, float>(v, rows, whole, K, parts, grid, status, s);
    case 3: return run_fused_stats<S, 3, OP, float>(v, rows, whole, K, parts, grid, status, s);
    case 4:
      return v.dtype == 1 ? run_fused_stats<S, 4, OP, float>(v, rows, whole, K, parts, grid, status, s)
                          : run_fused_stats<S, 4, OP, double>(v, rows, whole, K, parts, grid, status, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_copy_status(const int* status, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_status_word, dim3(1), dim3(64), 0, s, status, out);
  return hipGetLastError();
}

hipError_t launch_merge_status(const int* src, int* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_status_word, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_stats_combine(const void* records, int K, int op, double quantum, void* out, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_combine, dim3(1), dim3(64), 0, s, (const StatsOut*)records, K, op, quantum,
                     (StatsOut*)out);
  return hipGetLastError();
}

hipError_t launch_batch_reset(BatchAcc* acc, int slots, int* status, hipStream_t s) {
  const int n = slots * kAccStripes;
  const unsigned grid = (unsigned)std::min(64, std::max(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_batch_reset, dim3(grid), dim3(256), 0, s, acc, slots, status);
  return hipGetLastError();
}

hipError_t launch_batch_stats(int S, const StatsJob* jobs, const int64_t* unit_start, const int64_t* counts, int kmax,
                              BatchAcc* acc, int* status, int grid, hipStream_t s) {
  const size_t lds = (size_t)kWavesPerGroup * (kmax + 1) * kWave * sizeof(uint32_t);
  if (S == 32)
    hipLaunchKernelGGL(k_batch_stats<32>, dim3(grid), dim3(kThreads), lds, s, jobs, unit_start, counts, kmax, acc,
                       status);
  else
    hipLaunchKernelGGL(k_batch_stats<64>, dim3(grid), dim3(kThreads), lds, s, jobs, unit_start, counts, kmax, acc,
                       status);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const StatsJob* const jobs[2], const int64_t* const counts[2],
                                 const BatchAcc* const acc[2], const int n[2], hipStream_t s) {
  FinalizeArgs fa;
  for (int c = 0; c < 2; ++c) {
    fa.jobs[c] = jobs[c];
    fa.counts[c] = counts[c];
    fa.acc[c] = acc[c];
  }
  fa.n0 = n[0];
  const int waves = n[0] + n[1];
  if (waves == 0) return hipSuccess;
  const int per = 256 / kWave;
  hipLaunchKernelGGL(k_batch_finalize, dim3((waves + per - 1) / per), dim3(256), 0, s, fa);
  return hipGetLastError();
}

int stats_kmax(const StreamView& v) { return kmax_for(v); }

uint64_t op_workspace_bytes() { return kPartialOff + sizeof(Partial) * (uint64_t)kOpWorkgroups; }

// Sum of the block means (k_meta_mean, finalized into the workspace at
// kMetaOff) that the spread about the metadata mean needs first.
hipError_t launch_meta_sum(const int32_t* ms, const StreamView& v, Partial* parts, uint8_t* ws, hipStream_t s) {
  const int grid = grid_for(v.nb, kThreads);
  hipLaunchKernelGGL(k_meta_mean, dim3(grid), dim3(kThreads), 0, s, ms, v.n, v.nb, v.block, parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, parts, grid, 1, 0, v.quantum,
                     (const StatsOut*)nullptr, (StatsOut*)(ws + kMetaOff));
  return hipGetLastError();
}

hipError_t launch_stats_stage(const void* buf, int stage, const StreamView& v, int op_in, const OpTarget& t,
                              void* result, uint8_t* ws, hipStream_t s) {
  Partial* parts = (Partial*)(ws + kPartialOff);
  if (op_in == kOpVarMetaMean) {  // stage 2 of a block-mean stream, whole field (checked by the caller)
    hipError_t e = launch_meta_sum((const int32_t*)buf + v.n, v, parts, ws, s);
    if (e != hipSuccess) return e;
  }
  const int op = op_in == kOpVarMetaMean ? 2 : op_in;
  const Rows rows = make_rows(t.d, t.box);
  const bool contiguous = rows.count() == 1 && rows.base % 4 == 0;
  const bool whole = contiguous && rows.base == 0 && rows.len == v.n;
  int grid = 1;
  if (stage == 3 && contiguous) {
    const int32_t* q = (const int32_t*)buf + rows.base;
    grid = grid_for(rows.len / 4, kThreads * kUnroll);
    if (op == 1) hipLaunchKernelGGL(k_stats_q_flat<1>, dim3(grid), dim3(kThreads), 0, s, q, rows.len, parts);
    else hipLaunchKernelGGL(k_stats_q_flat<2>, dim3(grid), dim3(kThreads), 0, s, q, rows.len, parts);
  } else if (stage == 3) {
    grid = grid_for(rows.count() * ((rows.len + kSeg - 1) / kSeg), 1);
    if (op == 1) hipLaunchKernelGGL(k_stats_q<1>, dim3(grid), dim3(kThreads), 0, s, (const int32_t*)buf, rows, parts);
    else hipLaunchKernelGGL(k_stats_q<2>, dim3(grid), dim3(kThreads), 0, s, (const int32_t*)buf, rows, parts);
  } else if (stage == 4 && contiguous) {
    const int per = v.dtype == 1 ? 4 : 2;
    grid = grid_for(rows.len / per, kThreads * kUnroll);
    if (v.dtype == 1)
      hipLaunchKernelGGL(k_stats_f_flat<float>, dim3(grid), dim3(kThreads), 0, s, (const float*)buf + rows.base,
                         rows.len, parts);
    else
      hipLaunchKernelGGL(k_stats_f_flat<double>, dim3(grid), dim3(kThreads), 0, s,
                         (const double*)buf + rows.base, rows.len, parts);
  } else if (stage == 4) {
    grid = grid_for(rows.count() * ((rows.len + kSeg - 1) / kSeg), 1);
    if (v.dtype == 1)
      hipLaunchKernelGGL(k_stats_f<float>, dim3(grid), dim3(kThreads), 0, s, (const float*)buf, rows, parts);
    else
      hipLaunchKernelGGL(k_stats_f<double>, dim3(grid), dim3(kThreads), 0, s, (const double*)buf, rows, parts);
  } else if (stage == 1) {
    // metadata (block means) of a block-mean stream, whole field (checked by the caller)
    grid = grid_for(v.nb, kThreads);
    hipLaunchKernelGGL(k_meta_mean, dim3(grid), dim3(kThreads), 0, s, (const int32_t*)buf, v.n, v.nb, v.block, parts);
  } else if (stage == 2 && (v.flags & 1u)) {
    const int32_t* p = (const int32_t*)buf;
    const int32_t* ms = p + v.n;
    grid = grid_for(rows.count() * ((rows.len + kSeg - 1) / kSeg), 1);
    if (v.block == 32 && op == 1)
      hipLaunchKernelGGL((k_stats_delta_mean<32, 1>), dim3(grid), dim3(kThreads), 0, s, p, ms, rows, parts);
    else if (v.block == 32)
      hipLaunchKernelGGL((k_stats_delta_mean<32, 2>), dim3(grid), dim3(kThreads), 0, s, p, ms, rows, parts);
    else if (op == 1)
      hipLaunchKernelGGL((k_stats_delta_mean<64, 1>), dim3(grid), dim3(kThreads), 0, s, p, ms, rows, parts);
    else
      hipLaunchKernelGGL((k_stats_delta_mean<64, 2>), dim3(grid), dim3(kThreads), 0, s, p, ms, rows, parts);
  } else if (stage == 2) {
    const int32_t* p = (const int32_t*)buf;
    const int32_t* q0 = p + v.n;
    if (whole) {
      const int G = v.block / 4;
      grid = grid_for(v.nb * G, kThreads * 2);
      if (v.block == 32) {
        if (op == 1) hipLaunchKernelGGL((k_stats_delta_flat<32, 1>), dim3(grid), dim3(kThreads), 0, s, p, q0, v.n, v.nb, parts);
        else hipLaunchKernelGGL((k_stats_delta_flat<32, 2>), dim3(grid), dim3(kThreads), 0, s, p, q0, v.n, v.nb, parts);
      } else {
        if (op == 1) hipLaunchKernelGGL((k_stats_delta_flat<64, 1>), dim3(grid), dim3(kThreads), 0, s, p, q0, v.n, v.nb, parts);
        else hipLaunchKernelGGL((k_stats_delta_flat<64, 2>), dim3(grid), dim3(kThreads), 0, s, p, q0, v.n, v.nb, parts);
      }
    } else if (v.block == 32) {
      Segs<32> sg = make_segs<32>(rows);
      grid = grid_for(sg.count(), kThreads);
      if (op == 1) hipLaunchKernelGGL((k_stats_delta<32, 1>), dim3(grid), dim3(kThreads), 0, s, p, q0, sg, parts);
      else hipLaunchKernelGGL((k_stats_delta<32, 2>), dim3(grid), dim3(kThreads), 0, s, p, q0, sg, parts);
    } else {
      Segs<64> sg = make_segs<64>(rows);
      grid = grid_for(sg.count(), kThreads);
      if (op == 1) hipLaunchKernelGGL((k_stats_delta<64, 1>), dim3(grid), dim3(kThreads), 0, s, p, q0, sg, parts);
      else hipLaunchKernelGGL((k_stats_delta<64, 2>), dim3(grid), dim3(kThreads), 0, s, p, q0, sg, parts);
    }
  } else {
    return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // stage 4 sums are shifted by the box's first value; every partial carries it
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, parts, grid, op_in, stage == 4 ? 1 : 0,
                     v.quantum, (const StatsOut*)(ws + kMetaOff), (StatsOut*)result);
  return hipGetLastError();
}

hipError_t launch_stats_fused(const StreamView& v, int via, int op_in, const OpTarget& t, void* result, uint8_t* ws,
                              hipStream_t s) {
  Partial* parts = (Partial*)(ws + kPartialOff);
  if (op_in == kOpVarMetaMean) {  // via 2 or 3 of a block-mean stream, whole field (checked by the caller)
    hipError_t e = launch_meta_sum(v.q0, v, parts, ws, s);
    if (e != hipSuccess) return e;
  }
  const int op = op_in == kOpVarMetaMean ? 2 : op_in;
  int* status = (int*)ws;
  const Rows rows = make_rows(t.d, t.box);
  const bool whole = rows.count() == 1 && rows.base == 0 && rows.len == v.n;
  double* K = (double*)(ws + 8);
  int grid = 1;
  hipError_t e;
  if (via == 1) {  // the stream's own metadata section (block means)
    grid = grid_for(v.nb, kThreads);
    hipLaunchKernelGGL(k_meta_mean, dim3(grid), dim3(kThreads), 0, s, v.q0, v.n, v.nb, v.block, parts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, parts, grid, op, 0, v.quantum,
                       (const StatsOut*)nullptr, (StatsOut*)result);
    return hipGetLastError();
  }
  if (v.block == 32)
    e = op == 1 ? fused_by_via<32, 1>(v, via, rows, whole, K, parts, grid, status, s)
                : fused_by_via<32, 2>(v, via, rows, whole, K, parts, grid, status, s);
  else
    e = op == 1 ? fused_by_via<64, 1>(v, via, rows, whole, K, parts, grid, status, s)
                : fused_by_via<64, 2>(v, via, rows, whole, K, parts, grid, status, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, parts, grid, op_in, via == 4 ? 1 : 0, v.quantum,
                     (const StatsOut*)(ws + kMetaOff), (StatsOut*)result);
  return hipGetLastError();
}

// ---- HSZp-nd on D_p (Sec. V-A) ------------------------------------------------------
namespace {

// Mean: sum q = sum over points of (Z - z)(Y - y)(X - x) p (0-based), the nd
// weights of Sec. V-A (HSZp's flat field: N - i).  Products and running sums
// wrap modulo 2^64, which is exact because the total, sum q, fits in 64
// bits.  One segment of kSeg points of a row (z, y) per workgroup step.
__global__ void __launch_bounds__(kThreads) k_lz_mean_buf(const int32_t* __restrict__ p, NdGrid g, Partial* parts) {
  IntAcc acc;
  uint64_t s = 0;
  const int64_t segs = (g.X + kSeg - 1) / kSeg;
  const int64_t items = g.Z * g.Y * segs;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t r = it / segs, x0 = (it % segs) * kSeg;
    const int64_t z = r / g.Y, y = r % g.Y;
    const uint64_t wzy = (uint64_t)(g.Z - z) * (uint64_t)(g.Y - y);
    const int32_t* row = p + r * g.X;
    const int64_t x1 = min(g.X, x0 + (int64_t)kSeg);
    for (int64_t x = x0 + threadIdx.x; x < x1; x += kThreads) {
      s += wzy * (uint64_t)(g.X - x) * (uint64_t)(int64_t)row[x];
      acc.cnt += 1;
    }
  }
  acc.s1 = (int64_t)s;
  store_int_partial(acc, parts);
}

// The same sum straight from the stream: a wave per 64-block chunk, a lane
// per nd block, each decoded slot weighted by its coordinates.
template <int S, int ND>
__global__ void __launch_bounds__(kThreads) k_lz_mean_fused(StreamView v, NdGrid g, int kmax, Partial* parts,
                                                           int* status) {
  using Sh = NdShape<ND, S>;
  extern __shared__ uint32_t smem[];
  uint32_t* tile = smem + wave_in_group() * (kmax + 1) * kWave;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  IntAcc acc;
  uint64_t s = 0;
  for (int64_t c = blockIdx.x * (int64_t)kWavesPerGroup + wave_in_group(); c < v.nchunks; c += waves) {
    const int w = lz_stage<S>(v, c, tile, kmax, status);
    const int64_t b = c * kChunkBlocks + l;
    if (b < v.nb) {
      const int64_t oz = (b / (g.nby * g.nbx)) * Sh::BZ, oy = ((b / g.nbx) % g.nby) * Sh::BY,
                    ox = (b % g.nbx) * Sh::BX;
      int vals[S];
      decode_lane_block<S, kWave, true>(tile + l, w, 0, [&](int j, int p, int) { vals[j] = p; });
      // weights factor as (Z - z)(Y - y)(X - x): each row of the block sums
      // (X - x) p, then is scaled once by (Z - z)(Y - y); slots outside the
      // field carry a weight factor <= 0 and are skipped
      const int64_t A = g.Z - oz, B = g.Y - oy, C = g.X - ox;
#pragma unroll
      for (int r = 0; r < Sh::BZ * Sh::BY; ++r) {
        const int64_t wz = A - r / Sh::BY, wy = B - r % Sh::BY;
        uint64_t row = 0;
#pragma unroll
        for (int sx = 0; sx < Sh::BX; ++sx) {
          const int64_t wx = C - sx;
          row += wx > 0 ? (uint64_t)wx * (uint64_t)(int64_t)vals[r * Sh::BX + sx] : 0;
        }
        if (wz > 0 && wy > 0) s += (uint64_t)(wz * wy) * row;
      }
      acc.cnt += min(A, (int64_t)Sh::BZ) * min(B, (int64_t)Sh::BY) * min(C, (int64_t)Sh::BX);
    }
    __builtin_amdgcn_wave_barrier();
  }
  acc.s1 = (int64_t)s;
  store_int_partial(acc, parts);
}

__global__ void __launch_bounds__(kThreads) k_copy_i32(const int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ b) {
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) b[i] = a[i];
}

// Alg. 4 on the GPU: with the prefix sums over every axis but the field's
// slowest already taken, one thread per column walks that axis with a
// running sum, which is q, and sums q and q^2 (nothing is written back).
__global__ void __launch_bounds__(kThreads) k_lz_scan_stats(const int32_t* __restrict__ buf, int64_t len,
                                                           int64_t inner, Partial* parts) {
  IntAcc acc;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < inner; t += (int64_t)gridDim.x * kThreads) {
    int run = 0;
#pragma unroll 8
    for (int64_t i = 0; i < len; ++i) {
      run += buf[i * inner + t];
      acc.add(run, true);
    }
  }
  store_int_partial(acc, parts);
}

// Alg. 4 on the two-pass D_q: the second pass's running sum along y (t plus
// the earlier z segments' totals) is q; its sums of q and q^2 are taken and
// nothing is written.
__global__ void __launch_bounds__(kThreads) k_lz_dq2_stats(const int32_t* __restrict__ buf, int64_t Z, int64_t Y,
                                                          int64_t X, const int32_t* __restrict__ carry,
                                                          int64_t seg_planes, Partial* parts) {
  typedef int i2 __attribute__((ext_vector_type(2)));
  constexpr int kRows = 8;  // rows of t and of the carries in flight per thread
  IntAcc acc;
  const int64_t h2 = X / 2, cols = Z * h2;
  for (int64_t c = blockIdx.x * (int64_t)kThreads + threadIdx.x; c < cols; c += (int64_t)gridDim.x * kThreads) {
    const int64_t z = c / h2, k = c % h2;
    const i2* p = (const i2*)(buf + z * Y * X) + k;
    const i2* cr = (const i2*)(carry + (z / seg_planes) * Y * X) + k;
    i2 run = {0, 0};
    int64_t y = 0;
    for (; y + kRows <= Y; y += kRows) {
      i2 a[kRows], b[kRows];
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        a[u] = p[(y + u) * h2];
        b[u] = cr[(y + u) * h2];
      }
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        run += a[u] + b[u];
        acc.add(run.x, true);
        acc.add(run.y, true);
      }
    }
    for (; y < Y; ++y) {
      run += p[y * h2] + cr[y * h2];
      acc.add(run.x, true);
      acc.add(run.y, true);
    }
  }
  store_int_partial(acc, parts);
}

// Alg. 4 on HSZp's flat row from lz_flat_front's p and tile carries: each
// tile's q (the in-tile prefix sum of p plus the carry, as the device-wide
// scan's last pass forms it) is summed, q and q^2, and not written.  Thread
// t of a tile owns its kFlatStatsPer consecutive words (16-byte loads),
// scans them in registers, and one workgroup scan of the thread totals
// places them: q = the tile's carry + the threads before + the thread's own
// prefix.  The prefix sums are taken modulo 2^32: every q fits 32 bits, so
// the wrapped sums are exact.
constexpr int kFlatStatsPer = (int)(kFlatTile / kThreads);
static_assert(kFlatStatsPer % 4 == 0, "16-byte loads");
__global__ void __launch_bounds__(kThreads) k_flat_stats(const int32_t* __restrict__ p, int64_t n,
                                                        const int32_t* __restrict__ carry, Partial* parts) {
  typedef int i4 __attribute__((ext_vector_type(4)));
  __shared__ uint32_t wt[kWavesPerGroup];
  IntAcc acc;
  const int64_t ntiles = (n + kFlatTile - 1) / kFlatTile;
  const int wv = wave_in_group();
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t i0 = t * kFlatTile + (int64_t)threadIdx.x * kFlatStatsPer;
    uint32_t v[kFlatStatsPer];
    if (i0 + kFlatStatsPer <= n) {
#pragma unroll
      for (int k = 0; k < kFlatStatsPer; k += 4) {
        const i4 w = *(const i4*)(p + i0 + k);
        v[k] = (uint32_t)w.x;
        v[k + 1] = (uint32_t)w.y;
        v[k + 2] = (uint32_t)w.z;
        v[k + 3] = (uint32_t)w.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kFlatStatsPer; ++k) v[k] = i0 + k < n ? (uint32_t)p[i0 + k] : 0u;
    }
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kFlatStatsPer; ++k) {
      tot += v[k];
      v[k] = tot;
    }
    // the threads before this one: a wave scan, then the waves before
    const uint32_t incl = (uint32_t)wave_incl_scan((int)tot);
    if (lane_id() == kWave - 1) wt[wv] = incl;
    lds_barrier();
    uint32_t before = incl - tot;
#pragma unroll
    for (int w = 0; w < kWavesPerGroup; ++w) before += w < wv ? wt[w] : 0u;
    lds_barrier();  // wt is rewritten by the next tile
    const uint32_t base = (uint32_t)carry[t] + before;
    const int valid = (int)min((int64_t)kFlatStatsPer, max((int64_t)0, n - i0));
    int64_t s1 = 0;
#pragma unroll
    for (int k = 0; k < kFlatStatsPer; ++k) {
      const int q = k < valid ? (int)(base + v[k]) : 0;
      s1 += q;
      add_u64(acc.s2, (uint64_t)((int64_t)q * (int64_t)q));
    }
    acc.s1 += s1;
    acc.cnt += valid;
  }
  store_int_partial(acc, parts);
}

template <int S, int ND>
int launch_lz_mean_fused(const StreamView& v, const NdGrid& g, Partial* parts, int* status, hipStream_t s) {
  const int kmax = lz_kmax<S, ND>(v.max_abs_q);
  const size_t lds = (size_t)kWavesPerGroup * (kmax + 1) * kWave * sizeof(uint32_t);
  const int grid = grid_for(v.nchunks, kWavesPerGroup);
  hipLaunchKernelGGL((k_lz_mean_fused<S, ND>), dim3(grid), dim3(kThreads), lds, s, v, g, kmax, parts, status);
  return grid;
}

}  // namespace

hipError_t launch_lz_stats(const int32_t* p, const StreamView& v, const NdGrid& g, int op, void* result,
                           uint8_t* ws, int32_t* scratch, int32_t* tmp, hipStream_t s) {
  Partial* parts = (Partial*)(ws + kPartialOff);
  int* status = (int*)ws;
  int grid = 1;
  if (op == 1 && p) {
    grid = grid_for(g.Z * g.Y * ((g.X + kSeg - 1) / kSeg), 1);
    hipLaunchKernelGGL(k_lz_mean_buf, dim3(grid), dim3(kThreads), 0, s, p, g, parts);
  } else if (op == 1) {
    if (g.ndim == 3)
      grid = v.block == 32 ? launch_lz_mean_fused<32, 3>(v, g, parts, status, s)
                           : launch_lz_mean_fused<64, 3>(v, g, parts, status, s);
    else if (g.ndim == 2)
      grid = v.block == 32 ? launch_lz_mean_fused<32, 2>(v, g, parts, status, s)
                           : launch_lz_mean_fused<64, 2>(v, g, parts, status, s);
    else
      grid = v.block == 32 ? launch_lz_mean_fused<32, 1>(v, g, parts, status, s)
                           : launch_lz_mean_fused<64, 1>(v, g, parts, status, s);
  } else if (op == 2) {
    const int64_t n = g.Z * g.Y * g.X;
    // the prefix sums over every axis but the field's slowest (3D view: z for
    // 3D, y for 2D); HSZp's single row is scanned whole and then only read,
    // so from compressed bytes it is decoded straight to D_q (the decoder
    // then also provides the scan's tile sums)
    const int last = g.ndim == 3 ? 0 : (g.ndim == 2 ? 1 : -1);
    const bool to_q = !p && g.ndim == 1;
    if (!p && tmp && g.ndim == 1 && g.Z * g.Y == 1 && g.X > kFlatTile) {
      // HSZp from the stream: decode to p with the tile sums, their prefix,
      // then one pass summing q as the scan's last pass would form it
      hipError_t e = lz_flat_front(v, g, scratch, tmp, status, s);
      if (e != hipSuccess) return e;
      const int64_t ntiles = (g.X + kFlatTile - 1) / kFlatTile;
      grid = (int)(ntiles < kOpWorkgroups ? ntiles : kOpWorkgroups);
      hipLaunchKernelGGL(k_flat_stats, dim3(grid), dim3(kThreads), 0, s, scratch, g.X, tmp, parts);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, parts, grid, op, 0, v.quantum,
                         (const StatsOut*)nullptr, (StatsOut*)result);
      return hipGetLastError();
    }
    if (!p && tmp && lz_dq_ok(g)) {
      // from the stream: the two-pass D_q's first pass, then its second
      // pass summing instead of writing
      int64_t seg_planes = 1;
      hipError_t e = lz_dq_front(v, g, scratch, tmp, status, s, &seg_planes);
      if (e != hipSuccess) return e;
      grid = grid_for(g.Z * g.X / 2, kThreads);
      hipLaunchKernelGGL(k_lz_dq2_stats, dim3(grid), dim3(kThreads), 0, s, scratch, g.Z, g.Y, g.X, tmp, seg_planes,
                         parts);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, parts, grid, op, 0, v.quantum,
                         (const StatsOut*)nullptr, (StatsOut*)result);
      return hipGetLastError();
    }
    if (p) hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(n, kThreads * 4)), dim3(kThreads), 0, s, p, n, scratch);
    else {
      hipError_t e = lz_decode(v, g, to_q ? 3 : 2, scratch, status, tmp, s);
      if (e != hipSuccess) return e;
    }
    if (!to_q) {
      hipError_t e = lz_scan_axes(scratch, g.Z, g.Y, g.X, 1, last, tmp, s);
      if (e != hipSuccess) return e;
    }
    const int64_t len = last == 0 ? g.Z : (last == 1 ? g.Y : 1);
    const int64_t inner = last == 0 ? g.Y * g.X : g.X;
    grid = grid_for(inner, kThreads);
    hipLaunchKernelGGL(k_lz_scan_stats, dim3(grid), dim3(kThreads), 0, s, scratch, len, inner, parts);
  } else {
    return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, parts, grid, op, 0, v.quantum,
                     (const StatsOut*)nullptr, (StatsOut*)result);
  return hipGetLastError();
}

}  // namespace hsz
