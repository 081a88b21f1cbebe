// compress.hip -- c = C(d, eps) on the GPU (Sec. IV, Alg. 1).
//
//   k_minmax      one read of the field (16-byte loads): extremes and a
//                 non-finite flag
//   k_params      eps -> eps_q -> Delta, 1/Delta (binary64)
//   k_quant_meta  quantize and decorrelate; block widths, q0, payload words
//                 per 64-block chunk, max |q|
//   k_scan_sums,  exclusive scan of the chunk word counts -> chunk table
//   k_scan_write
//   k_pack        quantize again and bit-pack each chunk in LDS, then copy it
//                 out with coalesced stores
//   k_header      the 256-byte header and the zero padding between sections
//
// Work layout of k_quant_meta and k_pack: a wavefront owns a 64-block chunk
// and walks it 64 consecutive elements at a time, lane l <-> element l of
// the step, so every load is coalesced.  With S = 32 a step holds two blocks
// (lanes 0-31 and 32-63), with S = 64 one.  q_{i-1} comes from the lane
// below (a shuffle); slot 0 of a block has p = 0; a block's width is the bit
// length of the OR of |p| over its lanes; its sign word is a ballot; each
// magnitude is OR-ed into its (at most two) words of the LDS chunk image.
//
// Block-mean mode (MEAN; the HSZx decorrelation of Sec. IV): the metadata of
// a block is its integer mean M = round-half-down(sum q / S_b), p = q - M on
// every slot.  The block sum comes from a segmented DPP scan of the low and
// high 16-bit halves of q (neither sum can overflow 32 bits); M is
// ceil((2 sum - S_b) / (2 S_b)) through one binary64 division, which is exact
// here: a quotient that is not an integer lies at least 1/128 from one,
// far beyond the division's rounding.  k_pack reads M back from the
// metadata section.
//
// Quantization is q = floor(x * (1/Delta) + 0.5) in binary64 with no fused
// multiply-add (compiled with contraction off); the same expression and
// parameter arithmetic as the CPU reference, so streams are byte-identical.
#include "hsz_device.hpp"
#include "hsz_launch.hpp"
#include "hsz_nd.hpp"

#include <math.h>

namespace hsz {

namespace {

constexpr int kThreads = 256;
constexpr int kMinmaxGroups = 1024;

struct CompressWs {
  int status;
  uint32_t max_abs_q;
  double eps, quantum, inv_quantum, vmin, vmax;
  uint64_t total_words;
};
constexpr uint64_t kWsPartials = 256;  // byte offset of the min/max partials

__host__ __device__ inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// 16-byte vector of the field type
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int k = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int k = 2;
};

template <typename T>
__device__ __forceinline__ void mm_add(T v, T& lo, T& hi, int& bad) {
  bad |= !(v - v == T(0));  // NaN or infinity
  lo = v < lo ? v : lo;
  hi = v > hi ? v : hi;
}

// Extremes in the field's own type (exact), four 16-byte loads in flight
// per thread; the scalar tail (n not a multiple of the vector) by one group.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_minmax(const T* __restrict__ x, int64_t n, double* partial) {
  using V = typename Vec16<T>::type;
  constexpr int K = Vec16<T>::k;
  constexpr int U = 4;
  T lo = (T)INFINITY, hi = (T)-INFINITY;
  int bad = 0;
  const V* xv = (const V*)x;
  const int64_t nv = n / K;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i0 = blockIdx.x * (int64_t)kThreads + threadIdx.x; i0 < nv; i0 += stride * U) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < nv) v[u] = xv[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * stride < nv) {
        const T* e = (const T*)&v[u];
#pragma unroll
        for (int k = 0; k < K; ++k) mm_add(e[k], lo, hi, bad);
      }
    }
  }
  if (blockIdx.x == 0)
    for (int64_t i = nv * K + threadIdx.x; i < n; i += kThreads) mm_add(x[i], lo, hi, bad);
  double dlo = (double)lo, dhi = (double)hi;
  for (int m = 32; m >= 1; m >>= 1) {
    dlo = fmin(dlo, __shfl_xor(dlo, m));
    dhi = fmax(dhi, __shfl_xor(dhi, m));
    bad |= __shfl_xor(bad, m);
  }
  __shared__ double slo[kThreads / kWave], shi[kThreads / kWave];
  __shared__ int sbad[kThreads / kWave];
  const int wv = wave_in_group();
  if (lane_id() == 0) { slo[wv] = dlo; shi[wv] = dhi; sbad[wv] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kThreads / kWave; ++k) {
      dlo = fmin(dlo, slo[k]);
      dhi = fmax(dhi, shi[k]);
      bad |= sbad[k];
    }
    partial[3 * blockIdx.x + 0] = dlo;
    partial[3 * blockIdx.x + 1] = dhi;
    partial[3 * blockIdx.x + 2] = bad ? 1.0 : 0.0;
  }
}

// spacing of the field's numbers in the binade holding v > 0
__device__ double ulp_of(double v, int dtype) {
  int e;
  frexp(v, &e);
  return ldexp(1.0, e - 1 - (dtype == 1 ? 23 : 52));
}

// One workgroup: reduce the min/max partials (256 threads, then a tree),
// then thread 0 derives eps, eps_q, Delta and 1/Delta.
// fixed: derive eps and the quantum from the given extremes (those of the
// whole field a slab belongs to) instead of the reduced ones; a reduced
// extreme outside them is an error-bound failure (the margin would not hold).
__global__ void __launch_bounds__(kThreads) k_params(const double* partial, int groups, double eb, int eb_is_rel,
                                                     int dtype, int fixed, double gmin, double gmax, CompressWs* ws) {
  __shared__ double slo[kThreads], shi[kThreads];
  __shared__ int sbad[kThreads];
  const int t = threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int g = t; g < groups; g += kThreads) {
    lo = fmin(lo, partial[3 * g + 0]);
    hi = fmax(hi, partial[3 * g + 1]);
    bad |= partial[3 * g + 2] != 0.0;
  }
  slo[t] = lo; shi[t] = hi; sbad[t] = bad;
  __syncthreads();
  for (int half = kThreads / 2; half >= 1; half >>= 1) {
    if (t < half) {
      slo[t] = fmin(slo[t], slo[t + half]);
      shi[t] = fmax(shi[t], shi[t + half]);
      sbad[t] |= sbad[t + half];
    }
    __syncthreads();
  }
  if (t != 0) return;
  ws->status = 0;
  lo = slo[0];
  hi = shi[0];
  bad = sbad[0];
  // + 0.0 turns a -0.0 extreme into +0.0 so the stored bytes are canonical
  lo = lo + 0.0;
  hi = hi + 0.0;
  const bool outside = fixed && !bad && (lo < gmin || hi > gmax);
  if (fixed) {
    lo = gmin + 0.0;
    hi = gmax + 0.0;
  }
  ws->vmin = lo;
  ws->vmax = hi;
  ws->max_abs_q = 0;
  ws->total_words = 0;
  if (bad) {
    record_status(&ws->status, kErrNonFinite);
    ws->quantum = 1.0;
    ws->inv_quantum = 1.0;
    ws->eps = 0.0;
    return;
  }
  double eps;
  if (eb_is_rel) {
    double range = hi - lo;
    if (range > 0.0) eps = eb * range;
    else if (fabs(hi) > 0.0) eps = eb * fabs(hi);
    else eps = eb;
  } else {
    eps = eb;
  }
  double maxabs = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
  double margin = (dtype == 1 ? 1.0 : 8.0) * ulp_of(maxabs + eps, dtype);
  double eps_q = eps - margin;
  if (!(eps_q > 0.0) || outside) {
    record_status(&ws->status, kErrEb);
    ws->quantum = 1.0;
    ws->inv_quantum = 1.0;
    ws->eps = eps;
    return;
  }
  ws->eps = eps;
  ws->quantum = 2.0 * eps_q;
  ws->inv_quantum = 1.0 / ws->quantum;
}

// quantize one value; returns q clamped to +-kQMax and flags overflow
__device__ __forceinline__ int quantize(double x, double inv, bool& over) {
  double r = floor(x * inv + 0.5);
  over |= !(fabs(r) <= (double)kQMax);
  r = fmin(fmax(r, -(double)kQMax), (double)kQMax);
  return (int)r;
}

__device__ __forceinline__ int bitlen(uint32_t v) { return 32 - __clz((int)v); }

// Inclusive prefix-OR within each block's lanes by DPP: rows of 16 first,
// then row 0 -> 1 and 2 -> 3; with S = 64 also the first half into the
// second.  The block's OR ends up in its last lane (31, 63).
template <int S>
__device__ __forceinline__ int block_or_scan(int v) {
  v |= dpp<0x111>(v);
  v |= dpp<0x112>(v);
  v |= dpp<0x114>(v);
  v |= dpp<0x118>(v);
  v |= dpp<0x142, 0xa>(v);
  if (S == 64) v |= dpp<0x143, 0xc>(v);
  return v;
}

// Sum over each block's lanes by DPP (rows of 16, then row 0 -> 1 and
// 2 -> 3; with S = 64 the first half into the second): the block's sum ends
// up in its last lane.  Exact for |v| sums below 2^31.
template <int S>
__device__ __forceinline__ int block_add_scan(int v) {
  v += dpp<0x111>(v);
  v += dpp<0x112>(v);
  v += dpp<0x114>(v);
  v += dpp<0x118>(v);
  v += dpp<0x142, 0xa>(v);
  if (S == 64) v += dpp<0x143, 0xc>(v);
  return v;
}

// Integer mean of each block, rounded half down, for the lanes of one step
// (q of invalid lanes is 0; 'len' is the lane's block length, >= 1): the
// ceiling of (2 sum - len) / (2 len).  A whole block (FULL, len = S) divides
// by the power of two 2S, so the ceiling is exact in integers:
// floor((2 sum + S - 1) / 2S), an arithmetic shift; a partial block takes
// the binary64 quotient (exact: both operands are integers below 2^36).
// SMALL: every |q| of the step is below 2^30 / S, so the block sum fits one
// 32-bit scan; otherwise the low and high 16 bits are summed apart.
template <int S, bool FULL, bool SMALL>
__device__ __forceinline__ int block_mean(int q, int len) {
  auto block_total = [](int t) {  // the scan's value in the block's last lane
    if (S == 32) {
      const bool up = lane_id() >= 32;
      return up ? __builtin_amdgcn_readlane(t, 63) : __builtin_amdgcn_readlane(t, 31);
    }
    return __builtin_amdgcn_readlane(t, 63);
  };
  int64_t sum;
  if constexpr (SMALL) {
    sum = block_total(block_add_scan<S>(q));
  } else {
    const int lo = block_add_scan<S>(q & 0xffff), hi = block_add_scan<S>(q >> 16);
    sum = (int64_t)block_total(hi) * 65536 + (int64_t)block_total(lo);
  }
  if constexpr (FULL) {
    constexpr int kShift = S == 32 ? 6 : 7;  // log2(2S)
    return (int)((2 * sum + (S - 1)) >> kShift);
  } else {
    const double num = 2.0 * (double)sum - (double)len, den = 2.0 * (double)len;
    return (int)ceil(num / den);
  }
}

// the value of the lane below (wave shift right by one; lane 0 gets 0).  The
// empty asm keeps the shifted value in a register of its own: folded into
// the subtraction that follows (as a v_subrev with a DPP operand) it gave
// q_{i-1} - q_i instead of q_i - q_{i-1} for S = 64.
__device__ __forceinline__ int from_lane_below(int v) {
  int r = dpp<0x138>(v);
  asm volatile("" : "+v"(r));
  return r;
}

// Steps of 64 elements per chunk, and how many are loaded ahead.
template <int S>
constexpr int kSteps = kChunkBlocks * S / kWave;
constexpr int kAhead = 16;

// max|q| is reduced per workgroup into group_max[] (k_header takes the max
// of those): one atomic per wave on a single word serialized the end of the
// kernel.
constexpr int kMetaGroups = 4096;

template <typename T, int S, bool MEAN>
__global__ void __launch_bounds__(kThreads) k_quant_meta(const T* __restrict__ x, int64_t n, int64_t nb,
                                                        int64_t nchunks, CompressWs* ws, int32_t* q0s,
                                                        uint8_t* widths, uint32_t* chunk_words,
                                                        uint32_t* group_max) {
  if (ws->status != 0) {
    if (threadIdx.x == 0) group_max[blockIdx.x] = 0;
    return;
  }
  // per wave: the q0 and width of each block of its current chunk, written
  // by the block's first / last lane as the steps go, read back by lane l
  // (block 64c + l) for coalesced stores
  __shared__ int meta_all[(kThreads / kWave) * 2 * kChunkBlocks];
  int* mq0 = meta_all + wave_in_group() * 2 * kChunkBlocks;
  int* mw = mq0 + kChunkBlocks;
  const double inv = ws->inv_quantum;
  const int l = lane_id();
  const int slot = l % S;
  const int64_t waves = (int64_t)gridDim.x * (kThreads / kWave);
  uint32_t maxq = 0;
  bool over = false;
  // a chunk: FULL when all its elements exist (no bounds tests, so the
  // kAhead loads are issued back to back)
  auto chunk = [&](int64_t c, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    const int64_t e0 = c * (int64_t)(kChunkBlocks * S);
    for (int st = 0; st < kSteps<S>; st += kAhead) {
      T v[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int64_t e = e0 + (int64_t)(st + u) * kWave + l;
        v[u] = (FULL || e < n) ? x[e] : T(0);
      }
      // quantize and decorrelate the kAhead steps, then run their block
      // prefix-OR scans stage by stage: the independent DPP chains interleave
      // instead of stalling on each other's results
      int qv[kAhead];
      uint32_t step_max = 0;
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const bool valid = FULL || e0 + (int64_t)(st + u) * kWave + l < n;
        qv[u] = valid ? quantize((double)v[u], inv, over) : 0;
        const uint32_t aq = (uint32_t)(qv[u] < 0 ? -qv[u] : qv[u]);
        step_max = aq > step_max ? aq : step_max;
      }
      maxq = step_max > maxq ? step_max : maxq;
      int ab[kAhead];
      auto decorrelate = [&](auto small_tag) {
        constexpr bool SMALL = decltype(small_tag)::value;
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
          const bool valid = FULL || e0 + (int64_t)(st + u) * kWave + l < n;
          const int q = qv[u];
          int p, meta;
          if constexpr (MEAN) {
            const int64_t bstart = e0 + (int64_t)(st + u) * kWave + (l / S) * S;
            const int64_t rem = n - bstart;
            const int len = FULL ? S : (int)(rem < S ? (rem > 0 ? rem : 1) : S);
            meta = block_mean<S, FULL, SMALL>(q, len);
            p = valid ? q - meta : 0;
          } else {
            const int qp = from_lane_below(q);
            p = (slot == 0 || !valid) ? 0 : q - qp;
            meta = q;
          }
          ab[u] = p < 0 ? -p : p;
          if (slot == 0) mq0[(st + u) * (kWave / S) + l / S] = meta;
        }
      };
      if constexpr (MEAN) {
        // one vote per kAhead steps, so the branch is the whole wave's
        if (__all(step_max < (uint32_t)((1 << 30) / S))) decorrelate(std::true_type{});
        else decorrelate(std::false_type{});
      } else {
        decorrelate(std::false_type{});
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) ab[u] |= dpp<0x111>(ab[u]);
#pragma unroll
      for (int u = 0; u < kAhead; ++u) ab[u] |= dpp<0x112>(ab[u]);
#pragma unroll
      for (int u = 0; u < kAhead; ++u) ab[u] |= dpp<0x114>(ab[u]);
#pragma unroll
      for (int u = 0; u < kAhead; ++u) ab[u] |= dpp<0x118>(ab[u]);
#pragma unroll
      for (int u = 0; u < kAhead; ++u) ab[u] |= dpp<0x142, 0xa>(ab[u]);
      if (S == 64) {
#pragma unroll
        for (int u = 0; u < kAhead; ++u) ab[u] |= dpp<0x143, 0xc>(ab[u]);
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u)  // the block's OR is in its last lane
        if (slot == S - 1) mw[(st + u) * (kWave / S) + l / S] = bitlen((uint32_t)ab[u]);
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t b = c * kChunkBlocks + l;
    const bool exists = FULL || b < nb;
    const int my_w = mw[l], my_q0 = mq0[l];
    if (exists) {
      q0s[b] = my_q0;
      widths[b] = (uint8_t)my_w;
    }
    const int words = wave_incl_scan(exists ? block_words<S>(my_w) : 0);
    if (l == kWave - 1) chunk_words[c] = (uint32_t)words;
    __builtin_amdgcn_wave_barrier();
  };
  for (int64_t c = blockIdx.x * (int64_t)(kThreads / kWave) + wave_in_group(); c < nchunks; c += waves) {
    if ((c + 1) * (int64_t)(kChunkBlocks * S) <= n) chunk(c, std::true_type{});
    else chunk(c, std::false_type{});
  }
  maxq = (uint32_t)wave_max((int)maxq);
  __shared__ uint32_t wmax[kThreads / kWave];
  if (l == 0) wmax[wave_in_group()] = maxq;
  if (__any(over) && l == 0) record_status(&ws->status, kErrRange);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int k = 0; k < kThreads / kWave; ++k) m = wmax[k] > m ? wmax[k] : m;
    group_max[blockIdx.x] = m;
  }
}

// Exclusive scan of the chunk word counts into the chunk table, in ranges of
// kScanRange chunks (one workgroup each, 4 per thread): k_scan_sums adds each
// range, k_scan_write starts every range at the sum of the ranges before it
// and scans inside it.  A range's total is below 2^31 (a chunk holds at most
// 64 * 62 words).
constexpr int kScanThreads = 1024, kScanPer = 4, kScanRange = kScanThreads * kScanPer;

// sum of 'v' over the workgroup (every thread gets it)
__device__ __forceinline__ uint64_t group_sum(uint64_t v, uint64_t* red) {
  v = wave_sum_u64(v);
  const int wv = wave_in_group();
  if (lane_id() == 0) red[wv] = v;
  __syncthreads();
  uint64_t t = 0;
  for (int k = 0; k < kScanThreads / kWave; ++k) t += red[k];
  __syncthreads();
  return t;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(const uint32_t* __restrict__ chunk_words,
                                                            int64_t nchunks, uint64_t* range_sums) {
  __shared__ uint64_t red[kScanThreads / kWave];
  const int64_t i0 = blockIdx.x * (int64_t)kScanRange + threadIdx.x * (int64_t)kScanPer;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) s += i0 + k < nchunks ? chunk_words[i0 + k] : 0u;
  s = group_sum(s, red);
  if (threadIdx.x == 0) range_sums[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_write(const uint32_t* __restrict__ chunk_words,
                                                             int64_t nchunks, const uint64_t* __restrict__ range_sums,
                                                             uint64_t* chunk_off, CompressWs* ws,
                                                             uint64_t off_payload, uint64_t cap) {
  __shared__ uint64_t red[kScanThreads / kWave];
  __shared__ int wtot[kScanThreads / kWave];
  const int t = threadIdx.x, l = lane_id(), wv = wave_in_group();
  uint64_t before = 0;
  for (int64_t g = t; g < blockIdx.x; g += kScanThreads) before += range_sums[g];
  before = group_sum(before, red);
  const int64_t i0 = blockIdx.x * (int64_t)kScanRange + t * (int64_t)kScanPer;
  uint32_t v[kScanPer];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = i0 + k < nchunks ? chunk_words[i0 + k] : 0u;
    sum += (int)v[k];
  }
  const int incl = wave_incl_scan(sum);
  if (l == kWave - 1) wtot[wv] = incl;
  __syncthreads();
  int prior = 0, range = 0;
  for (int k = 0; k < kScanThreads / kWave; ++k) {
    const int wt = wtot[k];
    prior += k < wv ? wt : 0;
    range += wt;
  }
  uint64_t run = before + (uint64_t)(prior + incl - sum);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (i0 + k < nchunks) chunk_off[i0 + k] = run;
    run += v[k];
  }
  if (t == 0 && (int64_t)(blockIdx.x + 1) * kScanRange >= nchunks) {  // the last range
    const uint64_t total = before + (uint64_t)range;
    chunk_off[nchunks] = total;
    ws->total_words = total;
    if (off_payload + 4 * total > cap) record_status(&ws->status, kErrCapacity);
  }
}

template <typename T, int S, bool MEAN>
__global__ void __launch_bounds__(kThreads) k_pack(const T* __restrict__ x, int64_t n, int64_t nb,
                                                  int64_t nchunks, const CompressWs* ws,
                                                  const int32_t* __restrict__ metas,
                                                  const uint8_t* __restrict__ widths,
                                                  const uint64_t* __restrict__ chunk_off,
                                                  uint32_t* payload) {
  if (ws->status != 0) return;
  constexpr int kRows = (S / 32) * (1 + kMaxWidth);  // words of the widest block
  __shared__ uint32_t lin_all[(kThreads / kWave) * kRows * kWave];
  uint32_t* lin = lin_all + wave_in_group() * kRows * kWave;
  const double inv = ws->inv_quantum;
  const int l = lane_id();
  const int slot = l % S;
  const int64_t waves = (int64_t)gridDim.x * (kThreads / kWave);
  for (int64_t c = blockIdx.x * (int64_t)(kThreads / kWave) + wave_in_group(); c < nchunks; c += waves) {
    // word offsets of the chunk's blocks (lane l <-> block 64c + l)
    const int64_t bl = c * kChunkBlocks + l;
    const int wl = bl < nb ? (int)widths[bl] : 0;
    const int ml = (MEAN && bl < nb) ? metas[bl] : 0;  // block means (block-mean mode)
    const int nwl = block_words<S>(wl);
    const int incl = wave_incl_scan(nwl);
    const int offl = incl - nwl;
    const int total = __shfl(incl, kWave - 1);
    if (total < 0 || total > kRows * kWave) continue;  // widths are <= 30, so never taken
    for (int k = l; k < total; k += kWave) lin[k] = 0u;
    __builtin_amdgcn_wave_barrier();
    const int64_t e0 = c * (int64_t)(kChunkBlocks * S);
    auto steps = [&](auto full_tag) {  // FULL: every element of the chunk exists
      constexpr bool FULL = decltype(full_tag)::value;
    for (int st = 0; st < kSteps<S>; st += kAhead) {
      T v[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int64_t e = e0 + (int64_t)(st + u) * kWave + l;
        v[u] = (FULL || e < n) ? x[e] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int64_t base = e0 + (int64_t)(st + u) * kWave;
        const bool valid = FULL || base + l < n;
        bool ov = false;
        const int q = valid ? quantize((double)v[u], inv, ov) : 0;
        const int blk = (st + u) * (kWave / S);  // first block of the step within the chunk
        int p;
        if constexpr (MEAN) {
          int mb = __builtin_amdgcn_readlane(ml, blk);
          if (S == 32 && l >= 32) mb = __builtin_amdgcn_readlane(ml, blk + 1);
          p = valid ? q - mb : 0;
        } else {
          const int qp = from_lane_below(q);
          p = (slot == 0 || !valid) ? 0 : q - qp;
        }
        int w = __builtin_amdgcn_readlane(wl, blk), off = __builtin_amdgcn_readlane(offl, blk);
        if (S == 32 && l >= 32) {
          w = __builtin_amdgcn_readlane(wl, blk + 1);
          off = __builtin_amdgcn_readlane(offl, blk + 1);
        }
        const uint64_t neg = __ballot(p < 0);
        if (w > 0) {
          if (S == 32) {
            if (slot == 0) lin[off] = (uint32_t)(l < 32 ? neg : neg >> 32);
          } else {
            if (l == 0) lin[off] = (uint32_t)neg;
            if (l == 32) lin[off + 1] = (uint32_t)(neg >> 32);
          }
          const uint32_t m = (uint32_t)(p < 0 ? -p : p);
          if (m) {
            const uint32_t pos = (uint32_t)slot * (uint32_t)w;
            const uint32_t k = pos >> 5, sh = pos & 31u;
            uint32_t* mag = lin + off + S / 32;
            atomicOr(&mag[k], m << sh);
            if (sh + (uint32_t)w > 32u) atomicOr(&mag[k + 1], m >> (32u - sh));
          }
        }
      }
    }
    };
    if (e0 + (int64_t)(kChunkBlocks * S) <= n) steps(std::true_type{});
    else steps(std::false_type{});
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t* dst = payload + chunk_off[c];
    for (int k = l; k < total; k += kWave) dst[k] = lin[k];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

__device__ void put_bytes(uint8_t* h, int off, const void* v, int nbytes) {
  const uint8_t* s = (const uint8_t*)v;
  for (int k = 0; k < nbytes; ++k) h[off + k] = s[k];
}

// Header and zero padding.  One workgroup.
__global__ void k_header(uint8_t* out, CompressWs* ws, const uint32_t* __restrict__ group_max, int groups,
                         uint32_t flags, int dtype, int ndim, int64_t d0, int64_t d1, int64_t d2, int64_t n,
                         int block, int64_t nb,
                         int64_t nchunks, uint64_t off_chunk, uint64_t off_q0, uint64_t off_width,
                         uint64_t off_payload) {
  __shared__ uint8_t h[kHeaderBytes];
  __shared__ uint32_t smax[kHeaderBytes];
  const int t = threadIdx.x;
  if (t < kHeaderBytes) h[t] = 0;
  uint32_t m = 0;
  for (int g = t; g < groups; g += blockDim.x) m = group_max[g] > m ? group_max[g] : m;
  smax[t] = m;
  __syncthreads();
  for (int half = kHeaderBytes / 2; half >= 1; half >>= 1) {
    if (t < half && smax[t + half] > smax[t]) smax[t] = smax[t + half];
    __syncthreads();
  }
  if (t == 0) ws->max_abs_q = smax[0];
  __syncthreads();
  if (t == 0) {
    h[0] = 'H'; h[1] = 'S'; h[2] = 'Z'; h[3] = '1';
    uint16_t ver = 1;
    put_bytes(h, 4, &ver, 2);
    h[6] = (uint8_t)dtype;
    h[7] = (uint8_t)ndim;
    uint64_t dd[3] = {(uint64_t)d0, (uint64_t)d1, (uint64_t)d2};
    put_bytes(h, 8, dd, 24);
    uint64_t nn = (uint64_t)n;
    put_bytes(h, 32, &nn, 8);
    uint32_t bs = (uint32_t)block, cb = (uint32_t)kChunkBlocks;
    put_bytes(h, 40, &bs, 4);
    put_bytes(h, 44, &cb, 4);
    put_bytes(h, 48, &ws->eps, 8);
    put_bytes(h, 56, &ws->quantum, 8);
    put_bytes(h, 64, &ws->inv_quantum, 8);
    put_bytes(h, 72, &ws->vmin, 8);
    put_bytes(h, 80, &ws->vmax, 8);
    put_bytes(h, 88, &ws->max_abs_q, 4);
    put_bytes(h, 92, &flags, 4);
    uint64_t v[8] = {(uint64_t)nb, (uint64_t)nchunks, off_chunk, off_q0, off_width, off_payload,
                     ws->total_words, off_payload + 4 * ws->total_words};
    put_bytes(h, 96, v, 64);
  }
  __syncthreads();
  if (t < kHeaderBytes) out[t] = h[t];
  // padding after each metadata section (each gap is shorter than 256 bytes)
  const uint64_t ends[3] = {off_chunk + 8 * (uint64_t)(nchunks + 1), off_q0 + 4 * (uint64_t)nb,
                            off_width + (uint64_t)nb};
  const uint64_t next[3] = {off_q0, off_width, off_payload};
  for (int s = 0; s < 3; ++s)
    if (ends[s] + t < next[s]) out[ends[s] + t] = 0;
}

// workspace: CompressWs | min/max partials | chunk word counts | range sums | group max|q|
uint64_t ws_range_sums_off(const Layout& L) {
  return kWsPartials + 24 * (uint64_t)kMinmaxGroups + align_up(4 * (uint64_t)L.nchunks, 256);
}
uint64_t ws_group_max_off(const Layout& L) {
  const uint64_t ranges = (L.nchunks + kScanRange - 1) / kScanRange;
  return align_up(ws_range_sums_off(L) + 8 * ranges, 256);
}
// residuals of the Lorenzo modes, one int32 per slot of the partition
uint64_t ws_resid_off(const Layout& L) { return align_up(ws_group_max_off(L) + 4 * (uint64_t)kMetaGroups, 256); }

template <typename T, int S, bool MEAN>
hipError_t run(const CompressArgs& a, hipStream_t s) {
  const Layout& L = a.lay;
  CompressWs* ws = (CompressWs*)a.ws;
  double* partial = (double*)(a.ws + kWsPartials);
  uint32_t* chunk_words = (uint32_t*)(a.ws + kWsPartials + 24 * kMinmaxGroups);
  uint8_t* out = a.out;
  const T* x = (const T*)a.x;
  int g = (int)((L.n + kThreads * 16 - 1) / (kThreads * 16));
  g = g < 1 ? 1 : (g > kMinmaxGroups ? kMinmaxGroups : g);
  hipLaunchKernelGGL(k_minmax<T>, dim3(g), dim3(kThreads), 0, s, x, L.n, partial);
  hipLaunchKernelGGL(k_params, dim3(1), dim3(kThreads), 0, s, partial, g, a.eb, a.eb_is_rel, a.dtype,
                     a.fixed_range, a.vmin, a.vmax, ws);
  const int64_t cg = (L.nchunks + 3) / 4;
  const int grid = (int)(cg < kMetaGroups ? cg : kMetaGroups);
  uint32_t* group_max = (uint32_t*)(a.ws + ws_group_max_off(L));
  hipLaunchKernelGGL((k_quant_meta<T, S, MEAN>), dim3(grid), dim3(kThreads), 0, s, x, L.n, L.nb, L.nchunks, ws,
                     (int32_t*)(out + L.off_q0), out + L.off_width, chunk_words, group_max);
  const unsigned ranges = (unsigned)((L.nchunks + kScanRange - 1) / kScanRange);
  uint64_t* range_sums = (uint64_t*)(a.ws + ws_range_sums_off(L));
  hipLaunchKernelGGL(k_scan_sums, dim3(ranges), dim3(kScanThreads), 0, s, chunk_words, L.nchunks, range_sums);
  hipLaunchKernelGGL(k_scan_write, dim3(ranges), dim3(kScanThreads), 0, s, chunk_words, L.nchunks, range_sums,
                     (uint64_t*)(out + L.off_chunk), ws, L.off_payload, a.cap);
  hipLaunchKernelGGL((k_pack<T, S, MEAN>), dim3(grid), dim3(kThreads), 0, s, x, L.n, L.nb, L.nchunks, ws,
                     (const int32_t*)(out + L.off_q0), (const uint8_t*)(out + L.off_width),
                     (const uint64_t*)(out + L.off_chunk),
                     (uint32_t*)(out + L.off_payload));
  hipLaunchKernelGGL(k_header, dim3(1), dim3(kHeaderBytes), 0, s, out, ws, (const uint32_t*)group_max, grid,
                     MEAN ? 1u : 0u, a.dtype, a.ndim, a.dims[0], a.dims[1], a.dims[2], L.n, L.block, L.nb, L.nchunks, L.off_chunk,
                     L.off_q0, L.off_width, L.off_payload);
  return hipGetLastError();
}

// ---- HSZp-nd and HSZp: Lorenzo residual over the whole field -------------------
// (HSZp-nd: the field's own axes, nd blocks; HSZp: the field as one row of n,
// ND = 1, blocks of S consecutive elements)
// The residual of a point is the sum over the corners c of {0,1}^ND of
// (-1)^|c| q(point - c), with q = 0 before index 0 on any axis.  Three
// passes: k_resid_nd quantizes the field row by row and writes every slot's
// residual in block order into the workspace (4 bytes per slot of the
// partition, 0 on the slots past the field's end) and each block's width;
// k_chunk_words_nd sums the payload words per chunk and k_pack_nd takes the
// same wave-per-chunk walk as k_pack over the residuals.  |p| beyond
// 2^30 - 1 is a range error.

// One tile: U x 256 consecutive x positions of one row of blocks (BZ planes
// by BY rows).  A thread loads its columns (and the columns before them) on
// those rows and on the row before them (the corners' halo), every load
// issued before any is used, then forms the BZ x BY residuals of each
// column.  In 3D a work item walks a run of zper block planes of the same
// row of blocks: the halo plane is loaded once per run, and each block
// plane's last plane is carried, quantized, as the next one's halo.  The nd
// modes gather the tile's blocks in LDS (BX pad words after each block keep
// the column writes on distinct banks) and store them as one contiguous run;
// the flat mode's blocks are already in field order.  Either way the lanes
// then hold whole blocks (slot l % S), and the last lane of each writes the
// block's width.
template <typename T, int S, int ND>
struct ResidTile {
  using Sh = NdShape<ND, S>;
  static constexpr int HZ = ND == 3 ? 1 : 0, HY = ND >= 2 ? 1 : 0;  // halo plane / row
  static constexpr int NZ = Sh::BZ + HZ, NY = Sh::BY + HY;
  static constexpr int U = ND == 1 ? 8 : (NZ * NY * (int)sizeof(T) <= 64 ? 2 : 1);
  static constexpr int kSpan = U * kThreads;
  static constexpr int kPad = Sh::BX;
  static constexpr int kLds = ND == 1 ? 1 : kSpan / Sh::BX * (S + kPad);
};

template <typename T, int S, int ND>
__global__ void __launch_bounds__(kThreads) k_resid_nd(const T* __restrict__ x, NdGrid g, int64_t nxt, int64_t zper,
                                                      int64_t count, CompressWs* ws, int32_t* __restrict__ resid,
                                                      uint8_t* __restrict__ widths, uint32_t* group_max, int groups) {
  using Sh = NdShape<ND, S>;
  using R = ResidTile<T, S, ND>;
  constexpr int HZ = R::HZ, HY = R::HY, NY = R::NY, U = R::U;
  __shared__ int32_t tile[R::kLds];
  if (ws->status != 0) return;
  const double inv = ws->inv_quantum;
  const int t = threadIdx.x, l = lane_id();
  const int64_t xp = g.nbx * Sh::BX;  // padded row length
  uint32_t maxq = 0;
  bool over = false, wide = false;
  // q on (x, x - 1) of one row of the field, 0 outside it
  auto load_row = [&](int64_t z, int64_t y, int64_t xx, T& va, T& vb) {
    const bool row = z >= 0 && z < g.Z && y >= 0 && y < g.Y;
    const int64_t base = row ? (z * g.Y + y) * g.X : 0;
    const bool ia = row && xx < g.X, ib = row && xx >= 1 && xx - 1 < g.X;
    va = x[ia ? base + xx : 0];
    vb = x[ib ? base + xx - 1 : 0];
  };
  auto quant_row = [&](int64_t z, int64_t y, int64_t xx, T va, T vb, int& qa, int& qb) {
    const bool row = z >= 0 && z < g.Z && y >= 0 && y < g.Y;
    const bool ia = row && xx < g.X, ib = row && xx >= 1 && xx - 1 < g.X;
    qa = ia ? quantize((double)va, inv, over) : 0;
    qb = ib ? quantize((double)vb, inv, over) : 0;
  };
  for (int64_t w = blockIdx.x; w < count; w += gridDim.x) {
    // work item: x tile, row of blocks, run of zper block planes
    const int64_t xt = w % nxt, rest = w / nxt;
    const int64_t by = rest % g.nby, zc = rest / g.nby;
    const int64_t xbase = xt * R::kSpan;
    const int64_t bz0 = zc * zper, bz1 = ND < 3 ? bz0 + 1 : (bz0 + zper < g.nbz ? bz0 + zper : g.nbz);
    // the plane before the run (the corners' halo plane), carried from one
    // block plane to the next
    int ha[U][NY], hb[U][NY];
    if constexpr (HZ) {
      T pa[U][NY], pb[U][NY];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int iy = 0; iy < NY; ++iy)
          load_row(bz0 * Sh::BZ - 1, by * Sh::BY + iy - HY, xbase + u * kThreads + t, pa[u][iy], pb[u][iy]);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int iy = 0; iy < NY; ++iy)
          quant_row(bz0 * Sh::BZ - 1, by * Sh::BY + iy - HY, xbase + u * kThreads + t, pa[u][iy], pb[u][iy],
                    ha[u][iy], hb[u][iy]);
    }
    for (int64_t bz = bz0; bz < bz1; ++bz) {
      T va[U][Sh::BZ][NY], vb[U][Sh::BZ][NY];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int dz = 0; dz < Sh::BZ; ++dz)
#pragma unroll
          for (int iy = 0; iy < NY; ++iy)
            load_row(bz * Sh::BZ + dz, by * Sh::BY + iy - HY, xbase + u * kThreads + t, va[u][dz][iy], vb[u][dz][iy]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t xx = xbase + u * kThreads + t;
        const bool inx = xx < g.X;
        int qa[Sh::BZ + HZ][NY], qb[Sh::BZ + HZ][NY];
#pragma unroll
        for (int iy = 0; iy < NY; ++iy) {
          if constexpr (HZ) {
            qa[0][iy] = ha[u][iy];
            qb[0][iy] = hb[u][iy];
          }
#pragma unroll
          for (int dz = 0; dz < Sh::BZ; ++dz) {
            quant_row(bz * Sh::BZ + dz, by * Sh::BY + iy - HY, xx, va[u][dz][iy], vb[u][dz][iy], qa[dz + HZ][iy],
                      qb[dz + HZ][iy]);
            if (iy >= HY) {
              const int q = qa[dz + HZ][iy];
              const uint32_t aq = (uint32_t)(q < 0 ? -q : q);
              maxq = aq > maxq ? aq : maxq;
            }
          }
        }
        const int loc = u * kThreads + t;  // column within the tile
#pragma unroll
        for (int dz = 0; dz < Sh::BZ; ++dz) {
#pragma unroll
          for (int dy = 0; dy < Sh::BY; ++dy) {
            const int iz = dz + HZ, iy = dy + HY;
            const bool inside = inx && bz * Sh::BZ + dz < g.Z && by * Sh::BY + dy < g.Y;
            int64_t r = (int64_t)qa[iz][iy] - qb[iz][iy];
            if constexpr (ND >= 2) r += (int64_t)qb[iz][iy - 1] - qa[iz][iy - 1];
            if constexpr (ND == 3) {
              r += (int64_t)qb[iz - 1][iy] - qa[iz - 1][iy];
              r += (int64_t)qa[iz - 1][iy - 1] - qb[iz - 1][iy - 1];
            }
            if (!inside) r = 0;  // a slot past the field's end
            const int64_t ar = r < 0 ? -r : r;
            wide |= ar > kPMax;
            if constexpr (ND == 1) {
              // one row of blocks: slot order is field order, block xx / S in lanes of l / S
              const int ab = block_or_scan<S>((int)(ar > kPMax ? kPMax : ar));
              if (xx < xp) {
                resid[xx] = (int32_t)r;
                if (l % S == S - 1) widths[xx / S] = (uint8_t)bitlen((uint32_t)ab);
              }
            } else {
              tile[(loc / Sh::BX) * (S + R::kPad) + (dz * Sh::BY + dy) * Sh::BX + loc % Sh::BX] = (int32_t)r;
            }
          }
        }
        if constexpr (HZ) {
#pragma unroll
          for (int iy = 0; iy < NY; ++iy) {
            ha[u][iy] = qa[Sh::BZ][iy];
            hb[u][iy] = qb[Sh::BZ][iy];
          }
        }
      }
      if constexpr (ND >= 2) {
        __syncthreads();
        const int64_t xe = xp < xbase + R::kSpan ? xp : xbase + R::kSpan;
        const int total = (int)((xe - xbase) / Sh::BX) * S;  // words of the tile's blocks inside the partition
        const int64_t b0 = (bz * g.nby + by) * g.nbx + xbase / Sh::BX;
        int32_t* dst = resid + b0 * S;
        for (int k0 = 0; k0 < total; k0 += kThreads) {  // every lane takes part in the block OR
          const int k = k0 + t;
          const int v = k < total ? tile[(k / S) * (S + R::kPad) + k % S] : 0;
          const int ab = block_or_scan<S>(v < 0 ? -v : v);  // |v| <= kPMax unless a range error stops the stream
          if (k < total) {
            dst[k] = v;
            if (l % S == S - 1) widths[b0 + k / S] = (uint8_t)bitlen((uint32_t)ab);
          }
        }
        __syncthreads();
      }
    }
  }
  maxq = (uint32_t)wave_max((int)maxq);
  __shared__ uint32_t wmax[kThreads / kWave];
  if (l == 0) wmax[wave_in_group()] = maxq;
  if (__any(over || wide) && l == 0) record_status(&ws->status, kErrRange);
  __syncthreads();
  if (t == 0) {
    uint32_t m = 0;
    for (int k = 0; k < kThreads / kWave; ++k) m = wmax[k] > m ? wmax[k] : m;
    if (m) atomicMax(&group_max[blockIdx.x % groups], m);
  }
}

__global__ void __launch_bounds__(kThreads) k_zero_u32(uint32_t* p, int n) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) p[i] = 0u;
}

// payload words of each chunk of 64 blocks from the widths k_resid_nd wrote
template <int S>
__global__ void __launch_bounds__(kThreads) k_chunk_words_nd(const uint8_t* __restrict__ widths, int64_t nb,
                                                            int64_t nchunks, const CompressWs* ws,
                                                            uint32_t* chunk_words) {
  if (ws->status != 0) return;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (kThreads / kWave);
  for (int64_t c = blockIdx.x * (int64_t)(kThreads / kWave) + wave_in_group(); c < nchunks; c += waves) {
    const int64_t b = c * kChunkBlocks + l;
    const int words = wave_incl_scan(b < nb ? block_words<S>((int)widths[b]) : 0);
    if (l == kWave - 1) chunk_words[c] = (uint32_t)words;
  }
}

template <int S>
__global__ void __launch_bounds__(kThreads) k_pack_nd(const int32_t* __restrict__ resid, int64_t nb, int64_t nchunks,
                                                     const CompressWs* ws, const uint8_t* __restrict__ widths,
                                                     const uint64_t* __restrict__ chunk_off, uint32_t* payload) {
  if (ws->status != 0) return;
  constexpr int kRows = (S / 32) * (1 + kMaxWidth);  // words of the widest block
  __shared__ uint32_t lin_all[(kThreads / kWave) * kRows * kWave];
  uint32_t* lin = lin_all + wave_in_group() * kRows * kWave;
  const int l = lane_id();
  const int slot = l % S;
  const int64_t waves = (int64_t)gridDim.x * (kThreads / kWave);
  for (int64_t c = blockIdx.x * (int64_t)(kThreads / kWave) + wave_in_group(); c < nchunks; c += waves) {
    const int64_t bl = c * kChunkBlocks + l;
    const int wl = bl < nb ? (int)widths[bl] : 0;
    const int nwl = block_words<S>(wl);
    const int incl = wave_incl_scan(nwl);
    const int offl = incl - nwl;
    const int total = __shfl(incl, kWave - 1);
    if (total < 0 || total > kRows * kWave) continue;  // widths are <= 30, so never taken
    for (int k = l; k < total; k += kWave) lin[k] = 0u;
    __builtin_amdgcn_wave_barrier();
    // slot l % S of block 64c + st (64/S) + l/S is residual word 64 S c + 64 st + l
    const int64_t e0 = c * (int64_t)(kChunkBlocks * S), words = nb * (int64_t)S;
#pragma unroll
    for (int st0 = 0; st0 < kSteps<S>; st0 += kAhead) {
      int pv[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int64_t e = e0 + (int64_t)(st0 + u) * kWave + l;
        pv[u] = e < words ? resid[e] : 0;
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int st = st0 + u;
        const int blk = st * (kWave / S);  // first block of the step within the chunk
        const int p = pv[u];
        int w = __builtin_amdgcn_readlane(wl, blk), off = __builtin_amdgcn_readlane(offl, blk);
        if (S == 32 && l >= 32) {
          w = __builtin_amdgcn_readlane(wl, blk + 1);
          off = __builtin_amdgcn_readlane(offl, blk + 1);
        }
        const uint64_t neg = __ballot(p < 0);
        if (w > 0) {
          if (S == 32) {
            if (slot == 0) lin[off] = (uint32_t)(l < 32 ? neg : neg >> 32);
          } else {
            if (l == 0) lin[off] = (uint32_t)neg;
            if (l == 32) lin[off + 1] = (uint32_t)(neg >> 32);
          }
          const uint32_t m = (uint32_t)(p < 0 ? -p : p);
          if (m) {
            const uint32_t pos = (uint32_t)slot * (uint32_t)w;
            const uint32_t k = pos >> 5, sh = pos & 31u;
            uint32_t* mag = lin + off + S / 32;
            atomicOr(&mag[k], m << sh);
            if (sh + (uint32_t)w > 32u) atomicOr(&mag[k + 1], m >> (32u - sh));
          }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t* dst = payload + chunk_off[c];
    for (int k = l; k < total; k += kWave) dst[k] = lin[k];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

template <typename T, int S, int ND>
hipError_t run_nd(const CompressArgs& a, const NdGrid& g, hipStream_t s) {
  const Layout& L = a.lay;
  CompressWs* ws = (CompressWs*)a.ws;
  double* partial = (double*)(a.ws + kWsPartials);
  uint32_t* chunk_words = (uint32_t*)(a.ws + kWsPartials + 24 * kMinmaxGroups);
  uint8_t* out = a.out;
  const T* x = (const T*)a.x;
  int gm = (int)((L.n + kThreads * 16 - 1) / (kThreads * 16));
  gm = gm < 1 ? 1 : (gm > kMinmaxGroups ? kMinmaxGroups : gm);
  hipLaunchKernelGGL(k_minmax<T>, dim3(gm), dim3(kThreads), 0, s, x, L.n, partial);
  hipLaunchKernelGGL(k_params, dim3(1), dim3(kThreads), 0, s, partial, gm, a.eb, a.eb_is_rel, a.dtype,
                     a.fixed_range, a.vmin, a.vmax, ws);
  const int64_t cg = (L.nchunks + 3) / 4;
  const int grid = (int)(cg < kMetaGroups ? cg : kMetaGroups);
  uint32_t* group_max = (uint32_t*)(a.ws + ws_group_max_off(L));
  int32_t* resid = (int32_t*)(a.ws + ws_resid_off(L));
  using Sh = NdShape<ND, S>;
  const int64_t nxt = (g.nbx * Sh::BX + ResidTile<T, S, ND>::kSpan - 1) / ResidTile<T, S, ND>::kSpan;
  // runs of block planes per work item (3D): long enough to amortise the
  // halo plane, short enough to leave about 4096 work items
  const int64_t tiles2 = nxt * g.nby;
  int64_t zper = ND == 3 ? (tiles2 * g.nbz) / 4096 : 1;
  zper = zper < 1 ? 1 : (zper > 16 ? 16 : zper);
  const int64_t rcount = tiles2 * ((g.nbz + zper - 1) / zper);
  const int rgrid = (int)(rcount < (int64_t)(1 << 20) ? rcount : (int64_t)(1 << 20));
  hipLaunchKernelGGL(k_zero_u32, dim3((grid + kThreads - 1) / kThreads), dim3(kThreads), 0, s, group_max, grid);
  if (rgrid > 0)
    hipLaunchKernelGGL((k_resid_nd<T, S, ND>), dim3(rgrid), dim3(kThreads), 0, s, x, g, nxt, zper, rcount, ws, resid,
                       out + L.off_width, group_max, grid);
  hipLaunchKernelGGL((k_chunk_words_nd<S>), dim3(grid), dim3(kThreads), 0, s, (const uint8_t*)(out + L.off_width),
                     L.nb, L.nchunks, ws, chunk_words);
  const unsigned ranges = (unsigned)((L.nchunks + kScanRange - 1) / kScanRange);
  uint64_t* range_sums = (uint64_t*)(a.ws + ws_range_sums_off(L));
  hipLaunchKernelGGL(k_scan_sums, dim3(ranges), dim3(kScanThreads), 0, s, chunk_words, L.nchunks, range_sums);
  hipLaunchKernelGGL(k_scan_write, dim3(ranges), dim3(kScanThreads), 0, s, chunk_words, L.nchunks, range_sums,
                     (uint64_t*)(out + L.off_chunk), ws, L.off_payload, a.cap);
  hipLaunchKernelGGL((k_pack_nd<S>), dim3(grid), dim3(kThreads), 0, s, resid, L.nb, L.nchunks, ws,
                     (const uint8_t*)(out + L.off_width), (const uint64_t*)(out + L.off_chunk),
                     (uint32_t*)(out + L.off_payload));
  hipLaunchKernelGGL(k_header, dim3(1), dim3(kHeaderBytes), 0, s, out, ws, (const uint32_t*)group_max, grid,
                     a.flags, a.dtype, a.ndim, a.dims[0], a.dims[1], a.dims[2], L.n, L.block, L.nb, L.nchunks,
                     L.off_chunk, L.off_q0, L.off_width, L.off_payload);
  return hipGetLastError();
}

// extremes and the non-finite flag of a field from the k_minmax partials:
// out = {vmin, vmax, 1.0 if a value is NaN or infinite else 0.0}
__global__ void __launch_bounds__(kThreads) k_extremes(const double* partial, int groups, double* out) {
  __shared__ double slo[kThreads], shi[kThreads], sbad[kThreads];
  const int t = threadIdx.x;
  double lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (int g = t; g < groups; g += kThreads) {
    lo = fmin(lo, partial[3 * g + 0]);
    hi = fmax(hi, partial[3 * g + 1]);
    bad = partial[3 * g + 2] != 0.0 ? 1.0 : bad;
  }
  slo[t] = lo; shi[t] = hi; sbad[t] = bad;
  __syncthreads();
  for (int half = kThreads / 2; half >= 1; half >>= 1) {
    if (t < half) {
      slo[t] = fmin(slo[t], slo[t + half]);
      shi[t] = fmax(shi[t], shi[t + half]);
      sbad[t] = fmax(sbad[t], sbad[t + half]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = slo[0] + 0.0;
    out[1] = shi[0] + 0.0;
    out[2] = sbad[0];
  }
}

template <typename T, int ND>
hipError_t compress_nd_block(const CompressArgs& a, hipStream_t s) {
  const NdGrid g = ND == 1 ? flat_grid(a.lay.n, a.lay.block) : nd_grid(a.dims, a.ndim, a.lay.block);
  return a.lay.block == 32 ? run_nd<T, 32, ND>(a, g, s) : run_nd<T, 64, ND>(a, g, s);
}

}  // namespace

Layout make_layout_nd(const int64_t d3[3], int ndim, int block) {
  const NdGrid g = nd_grid(d3, ndim, block);
  Layout L;
  L.n = d3[0] * d3[1] * d3[2];
  L.block = block;
  L.nb = g.nbz * g.nby * g.nbx;
  L.nchunks = (L.nb + kChunkBlocks - 1) / kChunkBlocks;
  L.off_chunk = kHeaderBytes;
  L.off_q0 = align_up(L.off_chunk + 8 * (uint64_t)(L.nchunks + 1), kSectionAlign);
  L.off_width = L.off_q0;  // no metadata
  L.off_payload = align_up(L.off_width + (uint64_t)L.nb, kSectionAlign);
  return L;
}

uint64_t extremes_workspace_bytes() { return 24 * (uint64_t)kMinmaxGroups; }

hipError_t launch_extremes(const void* x, int dtype, int64_t n, double* out, uint8_t* ws, hipStream_t s) {
  double* partial = (double*)ws;
  int g = (int)((n + kThreads * 16 - 1) / (kThreads * 16));
  g = g < 1 ? 1 : (g > kMinmaxGroups ? kMinmaxGroups : g);
  if (dtype == 1) hipLaunchKernelGGL(k_minmax<float>, dim3(g), dim3(kThreads), 0, s, (const float*)x, n, partial);
  else hipLaunchKernelGGL(k_minmax<double>, dim3(g), dim3(kThreads), 0, s, (const double*)x, n, partial);
  hipLaunchKernelGGL(k_extremes, dim3(1), dim3(kThreads), 0, s, partial, g, out);
  return hipGetLastError();
}

Layout make_layout_flat(int64_t n, int block) {
  Layout L = make_layout(n, block);
  L.off_width = L.off_q0;  // no metadata
  L.off_payload = align_up(L.off_width + (uint64_t)L.nb, kSectionAlign);
  return L;
}

hipError_t launch_compress_nd(const CompressArgs& a, hipStream_t s) {
  if (a.flags == kFlagInterBlock)
    return a.dtype == 1 ? compress_nd_block<float, 1>(a, s) : compress_nd_block<double, 1>(a, s);
  if (a.ndim == 3)
    return a.dtype == 1 ? compress_nd_block<float, 3>(a, s) : compress_nd_block<double, 3>(a, s);
  return a.dtype == 1 ? compress_nd_block<float, 2>(a, s) : compress_nd_block<double, 2>(a, s);
}

Layout make_layout(int64_t n, int block) {
  Layout L;
  L.n = n;
  L.block = block;
  L.nb = (n + block - 1) / block;
  L.nchunks = (L.nb + kChunkBlocks - 1) / kChunkBlocks;
  L.off_chunk = kHeaderBytes;
  L.off_q0 = align_up(L.off_chunk + 8 * (uint64_t)(L.nchunks + 1), kSectionAlign);
  L.off_width = align_up(L.off_q0 + 4 * (uint64_t)L.nb, kSectionAlign);
  L.off_payload = align_up(L.off_width + (uint64_t)L.nb, kSectionAlign);
  return L;
}

uint64_t compress_workspace_bytes(const Layout& lay) { return ws_group_max_off(lay) + 4 * (uint64_t)kMetaGroups; }
uint64_t compress_workspace_bytes_nd(const Layout& lay) {
  return ws_resid_off(lay) + 4 * (uint64_t)lay.nb * (uint64_t)lay.block;
}

template <bool MEAN>
hipError_t compress_mode(const CompressArgs& a, hipStream_t s) {
  if (a.dtype == 1)
    return a.lay.block == 32 ? run<float, 32, MEAN>(a, s) : run<float, 64, MEAN>(a, s);
  return a.lay.block == 32 ? run<double, 32, MEAN>(a, s) : run<double, 64, MEAN>(a, s);
}

hipError_t launch_compress(const CompressArgs& a, hipStream_t s) {
  return (a.flags & 1u) ? compress_mode<true>(a, s) : compress_mode<false>(a, s);
}

}  // namespace hsz
