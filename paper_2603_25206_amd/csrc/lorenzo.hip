// lorenzo.hip -- decoding of HSZp-nd streams (Sec. IV, multidimensional
// Lorenzo decorrelation) and HSZp streams (deltas across block borders, the
// one-dimensional case over the flat field), and the derivative on the
// decorrelated data of HSZp-nd (Eq. (derivative_Dp)).
//
// D_p: one wavefront per 64-block chunk, one lane per nd block; the lane
// decodes its block slot by slot from its LDS column and writes each slot to
// its coordinates in the field (rows of BX consecutive words).
// D_q: q is the nd prefix sum of p (the inverse of the residual), built in
// place with one pass per axis: along x a wave per row (four words per lane,
// a wave scan, a carry across 256-word segments), along y and z a thread per
// column walking the axis with a running sum (consecutive threads own
// consecutive x, so every step is a coalesced row).  HSZp's single row of n
// is scanned device-wide instead: tile sums, a scan of those, and each tile
// scanned again with its offset.  Partial sums never
// overflow 32 bits: after the x pass a value is a mixed difference of at most
// four q (|q| < 2^29), after the y pass of two.
// D_f: D_q, then each word is converted in place.  A binary64 output keeps q
// in the low word of each 8-byte element (element stride 2), so the
// conversion of element i reads and writes only element i's own bytes.
//
// Derivative on D_p along axis a: with r the prefix sum of p over the other
// axes, q_{i+1} - q_{i-1} = r_i + r_{i+1}; so t_i = p_i + p_{i+1} (2 p_1 and
// 2 p_{n-1} at the one-sided ends, 0 on an axis of length 1) is formed, the
// prefix sums run over the other axes only, and the numerator is scaled by
// Delta/2 as on D_q: one axis fewer to scan than rebuilding q.
#include "hsz_device.hpp"
#include "hsz_nd.hpp"

namespace hsz {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerGroup = kThreads / kWave;

// D_p -> out (int32 words at element stride es), the field's layout.  The
// flat field (ND = 1) covers 64 S consecutive words per chunk: each lane
// puts its block's S values in row l of a (64 x (S+1))-word LDS tile (the +1
// keeps the writes conflict-free) and the wave stores the chunk 64 words at
// a time; nd blocks are written row by row (BX consecutive words).  With
// tsums the flat decoder also adds each chunk's residuals (the words inside
// the field) to the sum of its kFlatTile-word scan tile, which the device-wide
// scan then takes instead of reading the field again.
template <int S, int ND>
__global__ void __launch_bounds__(kThreads) k_lz_decode_p(StreamView v, NdGrid g, int kmax, int wave_words,
                                                         int32_t* __restrict__ out, int es, int* status,
                                                         int32_t* __restrict__ tsums) {
  using Sh = NdShape<ND, S>;
  extern __shared__ uint32_t smem[];
  const int wv = wave_in_group();
  uint32_t* tile = smem + wv * wave_words;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  for (int64_t c = blockIdx.x * (int64_t)kWavesPerGroup + wv; c < v.nchunks; c += waves) {
    const int w = lz_stage<S>(v, c, tile, kmax, status);
    const int64_t b = c * kChunkBlocks + l;
    if constexpr (ND == 1) {
      int vals[S];
      decode_lane_block<S, kWave, true>(tile + l, w, 0, [&](int j, int p, int) { vals[j] = p; });
      if (tsums) {
        // a chunk's words are one tile (S = 64) or half of one (S = 32); the
        // sum of any run of p is a difference of two q, so it fits 32 bits
        // (partial sums may wrap, hence unsigned)
        uint32_t bs = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) bs += (b * S + j < g.X) ? (uint32_t)vals[j] : 0u;
        for (int m = kWave / 2; m >= 1; m >>= 1) bs += (uint32_t)__shfl_xor((int)bs, m);
        constexpr int kPerTile = (int)(kFlatTile / (S * kChunkBlocks));
        if (l == 0) {
          if (kPerTile == 1) tsums[c] = (int32_t)bs;
          else atomicAdd(&tsums[c / kPerTile], (int)bs);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < S; ++j) tile[l * (S + 1) + j] = (uint32_t)vals[j];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int64_t base = c * kChunkBlocks * S;
#pragma unroll
      for (int m = 0; m < S; ++m) {
        const int e = m * kWave + l;
        const int64_t i = base + e;
        if (i < g.X) out[i * es] = (int32_t)tile[(e / S) * (S + 1) + (e % S)];
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      continue;
    }
    if (b < v.nb) {
      const int64_t oz = (b / (g.nby * g.nbx)) * Sh::BZ, oy = ((b / g.nbx) % g.nby) * Sh::BY,
                    ox = (b % g.nbx) * Sh::BX;
      const bool whole = oz + Sh::BZ <= g.Z && oy + Sh::BY <= g.Y && ox + Sh::BX <= g.X;
      int32_t* base = out + ((oz * g.Y + oy) * g.X + ox) * es;
      int vals[S];
      decode_lane_block<S, kWave, true>(tile + l, w, 0, [&](int j, int p, int) { vals[j] = p; });
      if (whole && es == 1 && (g.X & 3) == 0) {
        // rows of BX (4 or 8) words start 16-byte aligned: vector stores
        typedef int i4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int r = 0; r < Sh::BZ * Sh::BY; ++r) {
          int32_t* row = base + ((r / Sh::BY) * g.Y + (r % Sh::BY)) * g.X;
#pragma unroll
          for (int x4 = 0; x4 < Sh::BX; x4 += 4)
            *(i4*)(row + x4) = i4{vals[r * Sh::BX + x4], vals[r * Sh::BX + x4 + 1], vals[r * Sh::BX + x4 + 2],
                                  vals[r * Sh::BX + x4 + 3]};
        }
      } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const int sz = j / (Sh::BY * Sh::BX), sy = (j / Sh::BX) % Sh::BY, sx = j % Sh::BX;
          if (whole || (oz + sz < g.Z && oy + sy < g.Y && ox + sx < g.X))
            base[((sz * g.Y + sy) * g.X + sx) * es] = vals[j];
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// prefix sum along x of every row (rows = Z*Y), one wave per row
__global__ void __launch_bounds__(kThreads) k_scan_x(int32_t* __restrict__ buf, int64_t rows, int64_t X, int es) {
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  for (int64_t r = blockIdx.x * (int64_t)kWavesPerGroup + wave_in_group(); r < rows; r += waves) {
    int32_t* row = buf + r * X * es;
    int carry = 0;
    if (es == 1 && (X & 3) == 0) {  // 16-byte loads and stores, lane l <-> words 4l .. 4l+3
      typedef int i4 __attribute__((ext_vector_type(4)));
      for (int64_t x0 = 0; x0 < X; x0 += 4 * kWave) {
        const int64_t x = x0 + 4 * l;
        i4 v = x < X ? *(const i4*)(row + x) : i4{0, 0, 0, 0};
        v.y += v.x;
        v.z += v.y;
        v.w += v.z;
        const int incl = wave_incl_scan(v.w);
        const int before = carry + incl - v.w;
        if (x < X) *(i4*)(row + x) = i4{v.x + before, v.y + before, v.z + before, v.w + before};
        carry += __shfl(incl, kWave - 1);
      }
      continue;
    }
    for (int64_t x0 = 0; x0 < X; x0 += 4 * kWave) {
      int v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t x = x0 + 4 * l + k;
        v[k] = x < X ? row[x * es] : 0;
      }
      v[1] += v[0];
      v[2] += v[1];
      v[3] += v[2];
      const int incl = wave_incl_scan(v[3]);
      const int before = carry + incl - v[3];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t x = x0 + 4 * l + k;
        if (x < X) row[x * es] = v[k] + before;
      }
      carry += __shfl(incl, kWave - 1);
    }
  }
}

constexpr int kBatch = 16;  // rows in flight per thread in the column scans

// prefix sum along a strided axis: element (o, i, k) at ((o len + i) inner + k) es,
// one thread per (o, k) walking i
__global__ void __launch_bounds__(kThreads) k_scan_strided(int32_t* __restrict__ buf, int64_t outer, int64_t len,
                                                          int64_t inner, int es) {
  const int64_t cols = outer * inner;
  const int64_t step = inner * es;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < cols; t += (int64_t)gridDim.x * kThreads) {
    const int64_t o = t / inner, k = t % inner;
    int32_t* p = buf + (o * len * inner + k) * es;
    int run = 0;
    // a batch of kBatch rows is loaded before any is stored (a store could
    // alias the next load, so the compiler would not move loads ahead)
    int64_t i = 0;
    for (; i + kBatch <= len; i += kBatch) {
      int v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = p[(i + u) * step];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        run += v[u];
        p[(i + u) * step] = run;
      }
    }
    for (; i < len; ++i) {
      run += p[i * step];
      p[i * step] = run;
    }
  }
}

// ---- one long row (HSZp's flat field): reduce, scan the tile sums, apply ----------
// Tiles of kFlatTile words; a workgroup of 256 threads, 16 words per thread.
constexpr int kFlatPer = (int)(kFlatTile / kThreads);

// workgroup inclusive scan of one int per thread; 'total' gets the sum
__device__ __forceinline__ int group_incl_scan(int v, int* wsum, int& total) {
  const int incl = wave_incl_scan(v);
  const int wv = wave_in_group();
  if (lane_id() == kWave - 1) wsum[wv] = incl;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int k = 0; k < kWavesPerGroup; ++k) {
    const int t = wsum[k];
    before += k < wv ? t : 0;
    total += t;
  }
  __syncthreads();
  return before + incl;
}

__global__ void __launch_bounds__(kThreads) k_flat_tile_sums(const int32_t* __restrict__ buf, int64_t n, int es,
                                                            int32_t* __restrict__ sums) {
  __shared__ int wsum[kWavesPerGroup];
  const int64_t ntiles = (n + kFlatTile - 1) / kFlatTile;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int v = 0;
#pragma unroll
    for (int k = 0; k < kFlatPer; ++k) {
      const int64_t i = t * kFlatTile + (int64_t)k * kThreads + threadIdx.x;
      v += i < n ? buf[i * es] : 0;
    }
    int total;
    group_incl_scan(v, wsum, total);
    if (threadIdx.x == 0) sums[t] = total;
  }
}

// exclusive scan of the tile sums in place (one workgroup; each thread owns
// kSumsPer consecutive sums per step)
constexpr int kSumsPer = 32;
__global__ void __launch_bounds__(kThreads) k_flat_scan_sums(int32_t* __restrict__ sums, int64_t ntiles) {
  __shared__ int wsum[kWavesPerGroup];
  int carry = 0;
  for (int64_t b = 0; b < ntiles; b += (int64_t)kThreads * kSumsPer) {
    const int64_t i0 = b + (int64_t)threadIdx.x * kSumsPer;
    int v[kSumsPer];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < kSumsPer; ++k) {
      v[k] = i0 + k < ntiles ? sums[i0 + k] : 0;
      tot += v[k];
    }
    int total;
    const int incl = group_incl_scan(tot, wsum, total);
    int run = carry + incl - tot;
#pragma unroll
    for (int k = 0; k < kSumsPer; ++k) {
      if (i0 + k < ntiles) sums[i0 + k] = run;
      run += v[k];
    }
    carry += total;
  }
}

// each tile: word k*256 + t of the tile is thread t's k-th (coalesced loads
// and stores); each wave scans its 64 words of every row of 256, the wave
// totals of all 16 rows meet in LDS once, and every word gets the tile's
// offset plus the rows before it plus the waves before it in its row
__global__ void __launch_bounds__(kThreads) k_flat_apply(int32_t* __restrict__ buf, int64_t n, int es,
                                                        const int32_t* __restrict__ sums) {
  __shared__ int wt[kFlatPer * kWavesPerGroup];
  const int64_t ntiles = (n + kFlatTile - 1) / kFlatTile;
  const int wv = wave_in_group();
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t i0 = t * kFlatTile + threadIdx.x;
    int v[kFlatPer];
#pragma unroll
    for (int k = 0; k < kFlatPer; ++k) {
      const int64_t i = i0 + (int64_t)k * kThreads;
      v[k] = i < n ? buf[i * es] : 0;
    }
#pragma unroll
    for (int k = 0; k < kFlatPer; ++k) {
      v[k] = wave_incl_scan(v[k]);
      if (lane_id() == kWave - 1) wt[k * kWavesPerGroup + wv] = v[k];
    }
    lds_barrier();
    int run = sums[t];
#pragma unroll
    for (int k = 0; k < kFlatPer; ++k) {
      int before = 0, row = 0;
#pragma unroll
      for (int w = 0; w < kWavesPerGroup; ++w) {
        const int x = wt[k * kWavesPerGroup + w];
        before += w < wv ? x : 0;
        row += x;
      }
      const int64_t i = i0 + (int64_t)k * kThreads;
      if (i < n) buf[i * es] = run + before + v[k];
      run += row;
    }
    lds_barrier();  // each thread reads and writes only its own words of buf
  }
}

// the same over four neighbouring columns per thread with 16-byte loads
// (es = 1, inner a multiple of 4)
__global__ void __launch_bounds__(kThreads) k_scan_strided4(int32_t* __restrict__ buf, int64_t outer, int64_t len,
                                                           int64_t inner) {
  typedef int i4 __attribute__((ext_vector_type(4)));
  const int64_t q4 = inner / 4;
  const int64_t cols = outer * q4;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < cols; t += (int64_t)gridDim.x * kThreads) {
    const int64_t o = t / q4, k = t % q4;
    i4* p = (i4*)(buf + o * len * inner) + k;
    i4 run = {0, 0, 0, 0};
    int64_t i = 0;
    for (; i + kBatch <= len; i += kBatch) {
      i4 v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = p[(i + u) * q4];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        run += v[u];
        p[(i + u) * q4] = run;
      }
    }
    for (; i < len; ++i) {
      run += p[i * q4];
      p[i * q4] = run;
    }
  }
}

// ---- D_q in two passes (HSZp-nd, rows of at most kDqMaxX columns) -------------
// q = prefix sums of p along x, y and z.  First pass: a workgroup owns one
// block row (BY rows, all columns) and a segment of block layers along z.
// Per layer its blocks are decoded into an LDS copy of the layer's BZ x BY
// rows; wave w then prefix-sums rows w, w + 4, .. of each plane along x
// (eight consecutive columns per lane, a wave scan of the lane totals) and
// adds the running sum along z of each position, kept in registers from
// plane to plane within the segment, writing t (prefix over x and over the
// segment's planes up to z); at the segment's end the running sums, the
// segment's totals, go to tot[segment][y][x].  Second pass: a thread per
// (z, two columns) walks y with a running sum of t plus the totals of the
// earlier segments (the exclusive prefix of tot over segments), which is q.
// Two passes over the field instead of decoding and three prefix passes.
// The lane that scans eight columns also owns their running sums along z
// and stores them (two 16-byte words), so the scanned row never returns to
// LDS; a layer's chunk metadata is loaded two layers ahead and its first
// payload words one layer ahead (the pipeline at the end of k_lz_dq1).
typedef int i4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr uint32_t kDqNoStore = 0x80000000u;  // a buffer offset past every row: the store is discarded
constexpr int kDqPrefetch = 16;  // payload words per lane kept in flight a layer ahead
constexpr int kDqMaxX = 512;   // eight columns per lane
constexpr int kDqMaxSeg = 16;  // z segments, at most

template <int S, int ND>
__global__ void __launch_bounds__(kThreads) k_lz_dq1(StreamView v, NdGrid g, int kmax, int wave_words, int ndec,
                                                    int pitch, int64_t seg_layers, int32_t* __restrict__ t,
                                                    int32_t* __restrict__ tot, int* status) {
  using Sh = NdShape<ND, S>;
  constexpr int BZ = Sh::BZ, BY = Sh::BY, BX = Sh::BX;
  constexpr int RPW = (BY + kWavesPerGroup - 1) / kWavesPerGroup;  // rows per wave
  constexpr int V = kDqMaxX / kWave;
  static_assert(BX == 4, "three-dimensional blocks: rows of four words");
  extern __shared__ uint32_t smem[];
  const int wv = wave_in_group(), l = lane_id();
  // a layer's blocks span at most ndec chunks (the host's count); chunk k
  // of layer bz is decoded by wave (k - bz) mod 4 in staging tile k, so the
  // decoding turns over all four waves (and their SIMDs) layer by layer
  int32_t* lay = (int32_t*)(smem + ndec * wave_words);
  auto slot_of = [&](int bz) { return (wv + bz) & (kWavesPerGroup - 1); };
  const int64_t by = blockIdx.x % g.nby, seg = blockIdx.x / g.nby;
  const int L0 = (int)(seg * seg_layers), L1 = (int)min(L0 + seg_layers, g.nbz);
  const int nbx = (int)g.nbx;
  const int64_t X = g.X, YX = g.Y * g.X;
  int carry[RPW][V];
#pragma unroll
  for (int k = 0; k < RPW; ++k)
#pragma unroll
    for (int m = 0; m < V; ++m) carry[k][m] = 0;
  // the wave's chunk of layer bz (blocks b0..b1 of the layer are consecutive
  // in the stream, one lane each), or -1
  // (32-bit tests: the layer's first block sits b0 % 64 into its chunk)
  auto chunk_of = [&](int bz, int64_t& b0) {
    b0 = ((int64_t)bz * g.nby + by) * g.nbx;
    const int in_chunk = (int)(b0 % kChunkBlocks), k = slot_of(bz);
    return (bz < L1 && k < ndec && k * kChunkBlocks - in_chunk < nbx) ? b0 / kChunkBlocks + k : (int64_t)-1;
  };
  // metadata of chunk c, loaded unconditionally (chunk 0 stands in for none)
  // so the waits count the loads exactly
  auto meta_of = [&](int64_t c) { return lz_meta(v, c >= 0 ? c : 0); };
  using Pend = LzPending<kDqPrefetch>;
  auto decode = [&](int bz, int64_t c, int64_t b0, const Pend& P) {
    if (c < 0) return;
    uint32_t* stage = smem + slot_of(bz) * wave_words;
    const int w = lz_commit<kDqPrefetch>(v, P, stage, kmax);
    const int64_t b = c * kChunkBlocks + l;
    if (b >= b0 && b < b0 + nbx) {
      // a block row is BX = 4 consecutive words of the layer: written as one
      // 16-byte word (lanes 16 bytes apart, no bank conflicts)
      int32_t* dst = lay + (b - b0) * BX;
      i4v row4 = {0, 0, 0, 0};
      decode_lane_block<S, kWave, true>(stage + l, w, 0, [&](int j, int p, int) {
        row4[j % BX] = p;
        if (j % BX == BX - 1) *(i4v*)&dst[((j / BX) / BY % BZ * BY + (j / BX) % BY) * pitch] = row4;
      });
    }
  };
  auto rows = [&](int bz) {
#pragma unroll
    for (int sz = 0; sz < BZ; ++sz) {
      const int64_t z = (int64_t)bz * BZ + sz;
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int sy = wv + kWavesPerGroup * k;
        if (BY % kWavesPerGroup != 0 && sy >= BY) continue;
        const int64_t y = by * BY + sy;
        const bool ok = z < g.Z && y < g.Y;
        const int32_t* row = lay + (sz * BY + sy) * pitch;
        // x prefix: the lane's eight consecutive columns, then the lane totals
        const i4v lo = *(const i4v*)(row + V * l), hi = *(const i4v*)(row + V * l + 4);
        const int in[V] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        int vals[V], run = 0;
#pragma unroll
        for (int m = 0; m < V; ++m) {
          run += V * l + m < X ? in[m] : 0;
          vals[m] = run;
        }
        const int off = wave_incl_scan(run) - run;
        // then the running sum along z (rows past the field add nothing), and
        // the row stored as two 16-byte words per lane; every lane stores,
        // offsets past the row (or a row past the field) are discarded, so
        // the stores are the same on every path
#pragma unroll
        for (int m = 0; m < V; ++m) carry[k][m] += ok ? vals[m] + off : 0;
        const __amdgpu_buffer_rsrc_t r_row = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(ok ? t + z * YX + y * X : t), (short)0, ok ? (int)(4 * X) : 0, 0x00020000);
        const uint32_t o = 4u * (uint32_t)(V * l);
        __builtin_amdgcn_raw_buffer_store_b128(i4v{carry[k][0], carry[k][1], carry[k][2], carry[k][3]}, r_row,
                                               V * l < X ? o : kDqNoStore, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(i4v{carry[k][4], carry[k][5], carry[k][6], carry[k][7]}, r_row,
                                               V * l + 4 < X ? o + 16u : kDqNoStore, 0, 0);
      }
    }
  };
  // Software pipeline over the segment's layers, in pairs with two register
  // sets in turn: while layer L is decoded and its rows scanned and stored,
  // the payload of layer L + 1 is in flight (issued before layer L's
  // stores, so its wait includes none of them) and the metadata of layer
  // L + 2 too.
  // The first layer is peeled off so that the loop is entered, as it is
  // repeated, just after a layer's stores: the wait for a payload then
  // counts the same operations on both ways in.
  int64_t bA = 0, bB = 0;
  int64_t cA = chunk_of(L0, bA), cB = chunk_of(L0 + 1, bB);
  LzMeta mA = meta_of(cA), mB = meta_of(cB);
  Pend PA = lz_issue<S, kDqPrefetch>(v, mA, cA >= 0, kmax, status), PB;
  decode(L0, cA, bA, PA);
  cA = chunk_of(L0 + 2, bA);
  mA = meta_of(cA);
  PB = lz_issue<S, kDqPrefetch>(v, mB, cB >= 0, kmax, status);
  lds_barrier();
  rows(L0);
  lds_barrier();
  for (int bz = L0 + 1; bz < L1; bz += 2) {
    decode(bz, cB, bB, PB);
    const int64_t cB2 = chunk_of(bz + 2, bB);
    mB = meta_of(cB2);
    PA = lz_issue<S, kDqPrefetch>(v, mA, cA >= 0, kmax, status);
    lds_barrier();
    rows(bz);
    lds_barrier();
    cB = cB2;
    if (bz + 1 >= L1) break;
    decode(bz + 1, cA, bA, PA);
    const int64_t cA2 = chunk_of(bz + 3, bA);
    mA = meta_of(cA2);
    PB = lz_issue<S, kDqPrefetch>(v, mB, cB >= 0, kmax, status);
    lds_barrier();
    rows(bz + 1);
    lds_barrier();
    cA = cA2;
  }
  // the segment's totals
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int sy = wv + kWavesPerGroup * k;
    const int64_t y = by * BY + sy;
    if (sy >= BY || y >= g.Y) continue;
#pragma unroll
    for (int m = 0; m < V; ++m) {
      const int x = V * l + m;
      if (x < X) tot[seg * YX + y * X + x] = carry[k][m];
    }
  }
}

// tot[s] <- sum of tot[s'] for s' < s, per position (in place)
__global__ void __launch_bounds__(kThreads) k_lz_seg_carry(int32_t* __restrict__ tot, int nseg, int64_t YX) {
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < YX; i += (int64_t)gridDim.x * kThreads) {
    int run = 0;
    for (int s = 0; s < nseg; ++s) {
      const int v = tot[s * YX + i];
      tot[s * YX + i] = run;
      run += v;
    }
  }
}

// Second pass (X even): MODE 0 writes q, MODE 1 (float)(q Delta).  Two
// columns per thread (twice the waves of four, for latency), kDqBatch rows
// of t and of the carries per load batch, the next batch's loads issued
// before this batch's stores.
constexpr int kDqBatch = 8;

template <int MODE>
__device__ __forceinline__ void dq2_put(int32_t* p, int a, int b, double quantum) {
  typedef int i2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  if constexpr (MODE == 0) *(i2*)p = i2{a, b};
  else *(f2*)p = f2{(float)dequant64(a, quantum), (float)dequant64(b, quantum)};
}

template <int MODE>
__device__ __forceinline__ void dq2_load(const int32_t* p, const int32_t* cr, int64_t y, int64_t h2, int2* a) {
  typedef int i2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int u = 0; u < kDqBatch; ++u) {
    const i2 t = ((const i2*)p)[(y + u) * h2];
    const i2 c = ((const i2*)cr)[(y + u) * h2];
    a[2 * u] = make_int2(t.x, t.y);
    a[2 * u + 1] = make_int2(c.x, c.y);
  }
}

template <int MODE>
__device__ __forceinline__ void dq2_emit(int32_t* p, int64_t y, int64_t h2, const int2* a, int& rx, int& ry,
                                         double quantum) {
#pragma unroll
  for (int u = 0; u < kDqBatch; ++u) {
    rx += a[2 * u].x + a[2 * u + 1].x;
    ry += a[2 * u].y + a[2 * u + 1].y;
    dq2_put<MODE>(p + 2 * (y + u) * h2, rx, ry, quantum);
  }
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_lz_dq2(int32_t* __restrict__ buf, int64_t Z, int64_t Y, int64_t X,
                                                    const int32_t* __restrict__ carry, int64_t seg_planes,
                                                    double quantum) {
  const int64_t h2 = X / 2, cols = Z * h2;
  const int64_t nfull = Y / kDqBatch;
  for (int64_t c = blockIdx.x * (int64_t)kThreads + threadIdx.x; c < cols; c += (int64_t)gridDim.x * kThreads) {
    const int64_t z = c / h2, k = c % h2;
    int32_t* p = buf + z * Y * X + 2 * k;
    const int32_t* cr = carry + (z / seg_planes) * Y * X + 2 * k;
    int rx = 0, ry = 0;
    // two register sets in turn: a batch's loads are issued one batch of
    // stores ahead of their use.  The loads are unconditional (past the last
    // batch they read it again) so the waits count them exactly.
    int2 A[2 * kDqBatch], B[2 * kDqBatch];
    const int64_t last = nfull > 0 ? nfull - 1 : 0;
    if (nfull > 0) dq2_load<MODE>(p, cr, 0, h2, A);
    for (int64_t i = 0; i < nfull; i += 2) {
      dq2_load<MODE>(p, cr, min(i + 1, last) * kDqBatch, h2, B);
      dq2_emit<MODE>(p, i * kDqBatch, h2, A, rx, ry, quantum);
      if (i + 1 >= nfull) break;
      dq2_load<MODE>(p, cr, min(i + 2, last) * kDqBatch, h2, A);
      dq2_emit<MODE>(p, (i + 1) * kDqBatch, h2, B, rx, ry, quantum);
    }
    for (int64_t y = nfull * kDqBatch; y < Y; ++y) {
      rx += p[2 * y * h2] + cr[2 * y * h2];
      ry += p[2 * y * h2 + 1] + cr[2 * y * h2 + 1];
      dq2_put<MODE>(p + 2 * y * h2, rx, ry, quantum);
    }
  }
}

// ---- the derivative on D_p with its first and last passes fused ---------------
// For binary32 outputs (element stride 1, X a multiple of 4) and a derivative
// along z or y (so four x neighbours share their index along the axis): the
// first pass forms t along the axis from p on the fly and scans it along x;
// the last pass of the prefix sums writes (float)num * (float)(Delta/2)
// instead of the integer.  Two passes over the field fewer than pair, scans
// and scale one after another.
__device__ __forceinline__ i4v pair4(const i4v* __restrict__ p4, int64_t e4, int64_t i, int64_t L, int64_t s4) {
  if (L < 2) return i4v{0, 0, 0, 0};
  if (i == 0) return 2 * p4[e4 + s4];
  if (i == L - 1) return 2 * p4[e4];
  return p4[e4] + p4[e4 + s4];
}

// first pass (t along axis a in {0, 1}) scanned along x, one wave per row; with
// SCALE it is also the last pass (a 2D field's derivative along its rows' axis)
template <bool SCALE>
__global__ void __launch_bounds__(kThreads) k_scan_x_pair(const int32_t* __restrict__ p, NdGrid g, int a,
                                                         int32_t* __restrict__ out, float h) {
  const int l = lane_id();
  const int64_t rows = g.Z * g.Y, X = g.X;
  const int64_t L = a == 0 ? g.Z : g.Y;
  const int64_t s4 = (a == 0 ? g.Y * g.X : g.X) / 4;
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  const i4v* p4 = (const i4v*)p;
  for (int64_t r = blockIdx.x * (int64_t)kWavesPerGroup + wave_in_group(); r < rows; r += waves) {
    const int64_t i = a == 0 ? r / g.Y : r % g.Y;  // the row's index along the axis
    int carry = 0;
    for (int64_t x0 = 0; x0 < X; x0 += 4 * kWave) {
      const int64_t x = x0 + 4 * l;
      i4v v = x < X ? pair4(p4, (r * X + x) / 4, i, L, s4) : i4v{0, 0, 0, 0};
      v.y += v.x;
      v.z += v.y;
      v.w += v.z;
      const int incl = wave_incl_scan(v.w);
      const int before = carry + incl - v.w;
      if (x < X) {
        const i4v o = i4v{v.x + before, v.y + before, v.z + before, v.w + before};
        if constexpr (SCALE) *(f4v*)(out + r * X + x) = f4v{(float)o.x * h, (float)o.y * h, (float)o.z * h, (float)o.w * h};
        else *(i4v*)(out + r * X + x) = o;
      }
      carry += __shfl(incl, kWave - 1);
    }
  }
}

// first pass for a derivative along x: t along x (p_x + p_{x+1}; 2 p_1 and
// 2 p_{X-1} at the ends) formed from four words and the next one, scanned
// along the strided axis (y); with SCALE also the last pass (a 2D field)
template <bool SCALE>
__global__ void __launch_bounds__(kThreads) k_scan_strided4_pairx(const int32_t* __restrict__ p,
                                                                 int32_t* __restrict__ out, int64_t outer,
                                                                 int64_t len, int64_t X, float h) {
  const int64_t q4 = X / 4;
  const int64_t cols = outer * q4;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < cols; t += (int64_t)gridDim.x * kThreads) {
    const int64_t o = t / q4, k = t % q4;
    const int64_t x = 4 * k;
    const int64_t base = o * len * X + x;
    i4v run = {0, 0, 0, 0};
    for (int64_t i = 0; i < len; ++i) {
      const int64_t e = base + i * X;
      const i4v v = *(const i4v*)(p + e);
      const int nx = x + 4 < X ? p[e + 4] : 0;
      i4v tv;
      if (X < 2) {
        tv = i4v{0, 0, 0, 0};
      } else {
        tv = i4v{v.x + v.y, v.y + v.z, v.z + v.w, v.w + nx};
        if (x == 0) tv.x = 2 * v.y;
        if (x + 3 == X - 1) tv.w = 2 * v.w;
      }
      run += tv;
      if constexpr (SCALE)
        *(f4v*)(out + e) = f4v{(float)run.x * h, (float)run.y * h, (float)run.z * h, (float)run.w * h};
      else
        *(i4v*)(out + e) = run;
    }
  }
}

// last pass: the prefix sum along a strided axis, written as the scaled float
__global__ void __launch_bounds__(kThreads) k_scan_strided4_scale(int32_t* __restrict__ buf, int64_t outer,
                                                                 int64_t len, int64_t inner, float h) {
  const int64_t q4 = inner / 4;
  const int64_t cols = outer * q4;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < cols; t += (int64_t)gridDim.x * kThreads) {
    const int64_t o = t / q4, k = t % q4;
    i4v* p = (i4v*)(buf + o * len * inner) + k;
    i4v run = {0, 0, 0, 0};
    int64_t i = 0;
    for (; i + kBatch <= len; i += kBatch) {
      i4v v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = p[(i + u) * q4];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        run += v[u];
        *(f4v*)&p[(i + u) * q4] = f4v{(float)run.x * h, (float)run.y * h, (float)run.z * h, (float)run.w * h};
      }
    }
    for (; i < len; ++i) {
      run += p[i * q4];
      *(f4v*)&p[i * q4] = f4v{(float)run.x * h, (float)run.y * h, (float)run.z * h, (float)run.w * h};
    }
  }
}

// last pass of D_f (binary32): the prefix sum along a strided axis written as
// (float)(q * Delta), the dequantization of Alg. 2, in place
__global__ void __launch_bounds__(kThreads) k_scan_strided4_deq(int32_t* __restrict__ buf, int64_t outer,
                                                               int64_t len, int64_t inner, double quantum) {
  const int64_t q4 = inner / 4;
  const int64_t cols = outer * q4;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < cols; t += (int64_t)gridDim.x * kThreads) {
    const int64_t o = t / q4, k = t % q4;
    i4v* p = (i4v*)(buf + o * len * inner) + k;
    i4v run = {0, 0, 0, 0};
    int64_t i = 0;
    for (; i + kBatch <= len; i += kBatch) {
      i4v v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = p[(i + u) * q4];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        run += v[u];
        *(f4v*)&p[(i + u) * q4] = f4v{(float)dequant64(run.x, quantum), (float)dequant64(run.y, quantum),
                                      (float)dequant64(run.z, quantum), (float)dequant64(run.w, quantum)};
      }
    }
    for (; i < len; ++i) {
      run += p[i * q4];
      *(f4v*)&p[i * q4] = f4v{(float)dequant64(run.x, quantum), (float)dequant64(run.y, quantum),
                              (float)dequant64(run.z, quantum), (float)dequant64(run.w, quantum)};
    }
  }
}

// q (int32 at element stride es) -> T in place
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_dequant(void* buf, int64_t n, int es, double quantum) {
  if (sizeof(T) == 4 && es == 1) {  // four words per thread, 16-byte accesses, then the tail
    typedef int i4 __attribute__((ext_vector_type(4)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int64_t n4 = n / 4;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kThreads) {
      const i4 q = ((const i4*)buf)[i];
      ((f4*)buf)[i] = f4{(float)dequant64(q.x, quantum), (float)dequant64(q.y, quantum),
                         (float)dequant64(q.z, quantum), (float)dequant64(q.w, quantum)};
    }
    for (int64_t i = 4 * n4 + blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
      ((T*)buf)[i] = (T)dequant64(((const int32_t*)buf)[i], quantum);
    return;
  }
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const int q = ((const int32_t*)buf)[i * es];
    ((T*)buf)[i] = (T)dequant64(q, quantum);
  }
}

// t along axis a (see the file comment) -> out words at element stride es
__global__ void __launch_bounds__(kThreads) k_lz_pair(const int32_t* __restrict__ p, NdGrid g, int a,
                                                     int32_t* __restrict__ out, int es) {
  const int64_t n = g.Z * g.Y * g.X;
  const int64_t L = a == 0 ? g.Z : a == 1 ? g.Y : g.X;
  const int64_t stride = a == 0 ? g.Y * g.X : a == 1 ? g.X : 1;
  if (a != 2 && es == 1 && (g.X & 3) == 0) {
    // four neighbours along x share their index along the axis: 16-byte accesses
    typedef int i4 __attribute__((ext_vector_type(4)));
    const int64_t n4 = n / 4, s4 = stride / 4;
    const i4* p4 = (const i4*)p;
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < n4; e += (int64_t)gridDim.x * kThreads) {
      const int64_t i = (e / s4) % L;
      i4 t;
      if (L < 2) t = i4{0, 0, 0, 0};
      else if (i == 0) t = 2 * p4[e + s4];
      else if (i == L - 1) t = 2 * p4[e];
      else t = p4[e] + p4[e + s4];
      ((i4*)out)[e] = t;
    }
    return;
  }
  for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = (e / stride) % L;
    int t;
    if (L < 2) t = 0;
    else if (i == 0) t = 2 * p[e + stride];
    else if (i == L - 1) t = 2 * p[e];
    else t = p[e] + p[e + stride];
    out[e * es] = t;
  }
}

// numerator (int32 at element stride es) -> (T)num * (T)(Delta/2) in place
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_scale(void* buf, int64_t n, int es, double halfq) {
  const T h = (T)halfq;
  if (sizeof(T) == 4 && es == 1) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int64_t n4 = n / 4;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kThreads) {
      const i4 q = ((const i4*)buf)[i];
      ((f4*)buf)[i] = f4{(float)q.x * (float)h, (float)q.y * (float)h, (float)q.z * (float)h, (float)q.w * (float)h};
    }
    for (int64_t i = 4 * n4 + blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
      ((T*)buf)[i] = (T)((const int32_t*)buf)[i] * h;
    return;
  }
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const int num = ((const int32_t*)buf)[i * es];
    ((T*)buf)[i] = (T)num * h;
  }
}

unsigned grid_of(int64_t items, int per) {
  const int64_t g = (items + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

// The Laplacian on D_p (Eq. (laplacian_Dp), in any rank): c_a holds the
// prefix sums of p over every axis but a, which is q's backward difference
// along a (c_a at index 0 is q there).  The second difference along a is
// c_a one step further minus c_a here; the end value standing in for the
// missing neighbour drops the first term at the far end and the second at
// index 0 (an axis of length 1 adds 0).  The integer numerator is the D_q
// route's exactly, scaled by Delta once.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_lap(const int32_t* __restrict__ cz, const int32_t* __restrict__ cy,
                                                    const int32_t* __restrict__ cx, NdGrid g, double quantum,
                                                    T* __restrict__ out) {
  const int64_t n = g.Z * g.Y * g.X, sz = g.Y * g.X;
  for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
    const int64_t z = e / sz, y = (e / g.X) % g.Y, x = e % g.X;
    int num = 0;
    if (cz) num += (z + 1 < g.Z ? cz[e + sz] : 0) - (z > 0 ? cz[e] : 0);
    if (cy) num += (y + 1 < g.Y ? cy[e + g.X] : 0) - (y > 0 ? cy[e] : 0);
    num += (x + 1 < g.X ? cx[e + 1] : 0) - (x > 0 ? cx[e] : 0);
    out[e] = (T)((double)num * quantum);
  }
}

// Divergence / curl terms on D_p: term k is component c_k's central-
// difference numerator along its axis (an int32 field), signed s_k, scaled
// by that component's Delta/2 and added in binary64 to output o_k, in the
// order of the D_q route's terms (so the results equal it bit for bit).
struct LzVecTerms {
  const int32_t* num[6];
  double halfq[6];
  int s[6], o[6];
  int n, nout;
  void* out[3];
};

template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_vec(LzVecTerms t, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < t.n; ++k) acc[t.o[k]] += (double)(t.s[k] * t.num[k][e]) * t.halfq[k];
    for (int o = 0; o < t.nout; ++o) ((T*)t.out[o])[e] = (T)acc[o];
  }
}

__global__ void __launch_bounds__(kThreads) k_clear_i32(int32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) p[i] = 0;
}

template <int S, int ND>
hipError_t decode_p(const StreamView& v, const NdGrid& g, int32_t* out, int es, int* status, hipStream_t s,
                    int32_t* tsums) {
  const int kmax = lz_kmax<S, ND>(v.max_abs_q);
  int wave_words = (kmax + 1) * kWave;
  if (ND == 1 && wave_words < kWave * (S + 1)) wave_words = kWave * (S + 1);
  const size_t lds = (size_t)kWavesPerGroup * wave_words * sizeof(uint32_t);
  const int64_t groups = (v.nchunks + kWavesPerGroup - 1) / kWavesPerGroup;
  const unsigned grid = (unsigned)(groups < 8192 ? (groups < 1 ? 1 : groups) : 8192);
  hipLaunchKernelGGL((k_lz_decode_p<S, ND>), dim3(grid), dim3(kThreads), lds, s, v, g, kmax, wave_words, out, es,
                     status, ND == 1 ? tsums : nullptr);
  return hipGetLastError();
}

// tsums: tile sums of the flat field's scan (ND = 1 only; cleared here), or null
hipError_t decode_p_any(const StreamView& v, const NdGrid& g, int32_t* out, int es, int* status, hipStream_t s,
                        int32_t* tsums = nullptr) {
  if (g.ndim == 3)
    return v.block == 32 ? decode_p<32, 3>(v, g, out, es, status, s, nullptr)
                         : decode_p<64, 3>(v, g, out, es, status, s, nullptr);
  if (g.ndim == 2)
    return v.block == 32 ? decode_p<32, 2>(v, g, out, es, status, s, nullptr)
                         : decode_p<64, 2>(v, g, out, es, status, s, nullptr);
  if (tsums) {
    const int64_t ntiles = (g.X + kFlatTile - 1) / kFlatTile;
    hipLaunchKernelGGL(k_clear_i32, dim3(grid_of(ntiles, kThreads)), dim3(kThreads), 0, s, tsums, ntiles);
  }
  return v.block == 32 ? decode_p<32, 1>(v, g, out, es, status, s, tsums)
                       : decode_p<64, 1>(v, g, out, es, status, s, tsums);
}

// compute units of the current device (cached per device)
int device_cu_count() {
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

template <int S, int ND>
hipError_t dq_front(const StreamView& v, const NdGrid& g, int32_t* t, int32_t* tot, int* status, hipStream_t s,
                    int64_t* seg_planes) {
  using Sh = NdShape<ND, S>;
  const int kmax = lz_kmax<S, ND>(v.max_abs_q);
  const int wave_words = std::max(kmax + 1, kDqPrefetch) * kWave;  // the prefetched rows are all written
  const int pitch = kDqMaxX + 4;
  // chunks a layer's blocks can touch: nbx / 64 when layers start on chunk
  // borders, else one more (nbx <= 128 here, so at most 3)
  const int ndec = (int)(g.nbx % kChunkBlocks == 0 ? g.nbx / kChunkBlocks : g.nbx / kChunkBlocks + 2);
  if (ndec > kWavesPerGroup) return hipErrorInvalidValue;
  const size_t lds = ((size_t)ndec * wave_words + (size_t)Sh::BZ * Sh::BY * pitch) * sizeof(uint32_t);
  // z segments: as many workgroups as fit on the chip at once (by LDS, at
  // most eight per compute unit)
  const int64_t per_cu = std::min<int64_t>(8, (int64_t)(160 * 1024) / (int64_t)lds);
  const int64_t resident = std::max<int64_t>(1, per_cu) * device_cu_count();
  int64_t nseg = resident / g.nby;
  nseg = nseg < 1 ? 1 : (nseg > kDqMaxSeg ? kDqMaxSeg : nseg);
  nseg = nseg > g.nbz ? g.nbz : nseg;
  const int64_t seg_layers = (g.nbz + nseg - 1) / nseg;
  nseg = (g.nbz + seg_layers - 1) / seg_layers;
  hipLaunchKernelGGL((k_lz_dq1<S, ND>), dim3((unsigned)(g.nby * nseg)), dim3(kThreads), lds, s, v, g, kmax, wave_words,
                     ndec, pitch, seg_layers, t, tot, status);
  hipLaunchKernelGGL(k_lz_seg_carry, dim3(grid_of(g.Y * g.X, kThreads)), dim3(kThreads), 0, s, tot, (int)nseg,
                     g.Y * g.X);
  *seg_planes = seg_layers * Sh::BZ;
  return hipGetLastError();
}

}  // namespace

bool lz_dq_ok(const NdGrid& g) { return g.ndim == 3 && g.X <= kDqMaxX && (g.X & 3) == 0; }

uint64_t lz_dq_tmp_bytes(const NdGrid& g) {
  return lz_dq_ok(g) ? (uint64_t)kDqMaxSeg * (uint64_t)(g.Y * g.X) * sizeof(int32_t) : 0;
}

hipError_t lz_flat_front(const StreamView& v, const NdGrid& g, int32_t* p, int32_t* tsums, int* status,
                         hipStream_t s) {
  if (g.ndim != 1 || g.Z * g.Y != 1 || g.X <= kFlatTile || !tsums) return hipErrorNotSupported;
  hipError_t e = decode_p_any(v, g, p, 1, status, s, tsums);
  if (e != hipSuccess) return e;
  const int64_t ntiles = (g.X + kFlatTile - 1) / kFlatTile;
  hipLaunchKernelGGL(k_flat_scan_sums, dim3(1), dim3(kThreads), 0, s, tsums, ntiles);
  return hipGetLastError();
}

hipError_t lz_dq_front(const StreamView& v, const NdGrid& g, int32_t* t, int32_t* tot, int* status, hipStream_t s,
                       int64_t* seg_planes) {
  if (!lz_dq_ok(g) || !tot) return hipErrorNotSupported;  // three dimensions only
  return v.block == 32 ? dq_front<32, 3>(v, g, t, tot, status, s, seg_planes)
                       : dq_front<64, 3>(v, g, t, tot, status, s, seg_planes);
}

namespace {
// D_q (mode 0) or binary32 D_f (mode 1) of an HSZp-nd stream in two passes
hipError_t lz_dq(const StreamView& v, const NdGrid& g, int mode, int32_t* out, int32_t* tot, int* status,
                 hipStream_t s) {
  int64_t seg_planes = 1;
  hipError_t e = lz_dq_front(v, g, out, tot, status, s, &seg_planes);
  if (e != hipSuccess) return e;
  const unsigned grid = grid_of(g.Z * g.X / 2, kThreads);
  if (mode == 0)
    hipLaunchKernelGGL(k_lz_dq2<0>, dim3(grid), dim3(kThreads), 0, s, out, g.Z, g.Y, g.X, tot, seg_planes, 0.0);
  else
    hipLaunchKernelGGL(k_lz_dq2<1>, dim3(grid), dim3(kThreads), 0, s, out, g.Z, g.Y, g.X, tot, seg_planes,
                       v.quantum);
  return hipGetLastError();
}
}  // namespace

hipError_t lz_scan_axes(int32_t* buf, int64_t Z, int64_t Y, int64_t X, int es, int skip, int32_t* tmp,
                        hipStream_t s, bool sums_ready) {
  if (skip != 2 && Z * Y == 1 && X > kFlatTile) {
    if (!tmp) return hipErrorInvalidValue;
    const int64_t ntiles = (X + kFlatTile - 1) / kFlatTile;
    if (!sums_ready)
      hipLaunchKernelGGL(k_flat_tile_sums, dim3(grid_of(ntiles, 1)), dim3(kThreads), 0, s, buf, X, es, tmp);
    hipLaunchKernelGGL(k_flat_scan_sums, dim3(1), dim3(kThreads), 0, s, tmp, ntiles);
    hipLaunchKernelGGL(k_flat_apply, dim3(grid_of(ntiles, 1)), dim3(kThreads), 0, s, buf, X, es, tmp);
  } else if (skip != 2) {
    const int64_t rows = Z * Y;
    hipLaunchKernelGGL(k_scan_x, dim3(grid_of(rows, kWavesPerGroup)), dim3(kThreads), 0, s, buf, rows, X, es);
  }
  const bool v4 = es == 1 && (X & 3) == 0;
  if (skip != 1 && Y > 1) {
    if (v4)
      hipLaunchKernelGGL(k_scan_strided4, dim3(grid_of(Z * X / 4, kThreads)), dim3(kThreads), 0, s, buf, Z, Y, X);
    else
      hipLaunchKernelGGL(k_scan_strided, dim3(grid_of(Z * X, kThreads)), dim3(kThreads), 0, s, buf, Z, Y, X, es);
  }
  if (skip != 0 && Z > 1) {
    if (v4)
      hipLaunchKernelGGL(k_scan_strided4, dim3(grid_of(Y * X / 4, kThreads)), dim3(kThreads), 0, s, buf, (int64_t)1,
                         Z, Y * X);
    else
      hipLaunchKernelGGL(k_scan_strided, dim3(grid_of(Y * X, kThreads)), dim3(kThreads), 0, s, buf, (int64_t)1, Z,
                         Y * X, es);
  }
  return hipGetLastError();
}

hipError_t lz_decode(const StreamView& v, const NdGrid& g, int stage, void* out, int* status, int32_t* tmp,
                     hipStream_t s) {
  if (stage < 2 || stage > 4) return hipErrorInvalidValue;
  const int es = (stage == 4 && v.dtype == 2) ? 2 : 1;
  // rows of at most kDqMaxX columns: two passes (tmp holds the z segments' totals)
  if (es == 1 && stage >= 3 && tmp && lz_dq_ok(g)) return lz_dq(v, g, stage == 3 ? 0 : 1, (int32_t*)out, tmp, status, s);
  // the flat field's device-wide scan takes its tile sums from the decoder
  const bool fused_sums = stage >= 3 && g.ndim == 1 && g.Z * g.Y == 1 && g.X > kFlatTile && tmp;
  hipError_t e = decode_p_any(v, g, (int32_t*)out, es, status, s, fused_sums ? tmp : nullptr);
  if (e != hipSuccess || stage == 2) return e;
  if (stage == 4 && v.dtype == 1 && g.ndim >= 2 && (g.X & 3) == 0) {
    // all axes but the field's slowest, then the slowest writing the floats
    const int last = g.ndim == 3 ? 0 : 1;
    e = lz_scan_axes((int32_t*)out, g.Z, g.Y, g.X, 1, last, tmp, s);
    if (e != hipSuccess) return e;
    if (last == 0)
      hipLaunchKernelGGL(k_scan_strided4_deq, dim3(grid_of(g.Y * g.X / 4, kThreads)), dim3(kThreads), 0, s,
                         (int32_t*)out, (int64_t)1, g.Z, g.Y * g.X, v.quantum);
    else
      hipLaunchKernelGGL(k_scan_strided4_deq, dim3(grid_of(g.X / 4, kThreads)), dim3(kThreads), 0, s, (int32_t*)out,
                         (int64_t)1, g.Y, g.X, v.quantum);
    return hipGetLastError();
  }
  e = lz_scan_axes((int32_t*)out, g.Z, g.Y, g.X, es, -1, tmp, s, fused_sums);
  if (e != hipSuccess || stage == 3) return e;
  const int64_t n = g.Z * g.Y * g.X;
  if (v.dtype == 1)
    hipLaunchKernelGGL(k_lz_dequant<float>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es, v.quantum);
  else
    hipLaunchKernelGGL(k_lz_dequant<double>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es,
                       v.quantum);
  return hipGetLastError();
}

hipError_t lz_numerator_p(const int32_t* p, const NdGrid& g, int axis3, int32_t* out, hipStream_t s) {
  const int64_t n = g.Z * g.Y * g.X;
  hipLaunchKernelGGL(k_lz_pair, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, p, g, axis3, out, 1);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? lz_scan_axes(out, g.Z, g.Y, g.X, 1, axis3, nullptr, s) : e;
}

hipError_t lz_laplacian_p(const int32_t* p, const NdGrid& g, double quantum, int dtype, int32_t* cbuf, void* out,
                          hipStream_t s) {
  const int64_t n = g.Z * g.Y * g.X;
  const int first = 3 - g.ndim;  // the field's slowest axis in the 3D view
  const int32_t* c[3] = {nullptr, nullptr, nullptr};
  for (int a = first; a < 3; ++a) {
    int32_t* ca = cbuf + (uint64_t)(a - first) * (uint64_t)n;
    hipError_t e = hipMemcpyAsync(ca, p, 4 * (uint64_t)n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = lz_scan_axes(ca, g.Z, g.Y, g.X, 1, a, nullptr, s);
    if (e != hipSuccess) return e;
    c[a] = ca;
  }
  if (dtype == 1)
    hipLaunchKernelGGL(k_lz_lap<float>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, c[0], c[1], c[2], g, quantum,
                       (float*)out);
  else
    hipLaunchKernelGGL(k_lz_lap<double>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, c[0], c[1], c[2], g,
                       quantum, (double*)out);
  return hipGetLastError();
}

hipError_t lz_vector_p(const int32_t* const* p, const NdGrid& g, int nterms, const int* tc, const int* ta,
                       const int* ts, const int* to, int nout, const double* halfq, int dtype, int32_t* nbuf,
                       void* const* out, hipStream_t s) {
  if (nterms < 1 || nterms > 6 || nout < 1 || nout > 3) return hipErrorInvalidValue;
  const int64_t n = g.Z * g.Y * g.X;
  LzVecTerms t{};
  t.n = nterms;
  t.nout = nout;
  for (int k = 0; k < nterms; ++k) {
    int32_t* num = nbuf + (uint64_t)k * (uint64_t)n;
    hipError_t e = lz_numerator_p(p[tc[k]], g, ta[k], num, s);
    if (e != hipSuccess) return e;
    t.num[k] = num;
    t.halfq[k] = halfq[tc[k]];
    t.s[k] = ts[k];
    t.o[k] = to[k];
  }
  for (int o = 0; o < nout; ++o) t.out[o] = out[o];
  if (dtype == 1)
    hipLaunchKernelGGL(k_lz_vec<float>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, t, n);
  else
    hipLaunchKernelGGL(k_lz_vec<double>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, t, n);
  return hipGetLastError();
}

hipError_t lz_deriv_p(const int32_t* p, const StreamView& v, const NdGrid& g, int axis3, void* out, hipStream_t s) {
  const int es = v.dtype == 2 ? 2 : 1;
  const int64_t n = g.Z * g.Y * g.X;
  if (v.dtype == 1 && (g.X & 3) == 0 && axis3 == 2) {
    const float h = (float)(0.5 * v.quantum);
    if (g.ndim == 2) {  // y is the only other axis: one pass
      hipLaunchKernelGGL(k_scan_strided4_pairx<true>, dim3(grid_of(g.X / 4, kThreads)), dim3(kThreads), 0, s, p,
                         (int32_t*)out, (int64_t)1, g.Y, g.X, h);
      return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_strided4_pairx<false>, dim3(grid_of(g.Z * g.X / 4, kThreads)), dim3(kThreads), 0, s,
                       p, (int32_t*)out, g.Z, g.Y, g.X, h);
    hipLaunchKernelGGL(k_scan_strided4_scale, dim3(grid_of(g.Y * g.X / 4, kThreads)), dim3(kThreads), 0, s,
                       (int32_t*)out, (int64_t)1, g.Z, g.Y * g.X, h);
    return hipGetLastError();
  }
  if (v.dtype == 1 && (g.X & 3) == 0 && axis3 != 2) {
    const float h = (float)(0.5 * v.quantum);
    const unsigned gx = grid_of(g.Z * g.Y, kWavesPerGroup);
    if (g.ndim == 2) {  // the rows' axis is the only other one: one pass
      hipLaunchKernelGGL(k_scan_x_pair<true>, dim3(gx), dim3(kThreads), 0, s, p, g, axis3, (int32_t*)out, h);
      return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_x_pair<false>, dim3(gx), dim3(kThreads), 0, s, p, g, axis3, (int32_t*)out, h);
    if (axis3 == 0)  // then along y, scaled
      hipLaunchKernelGGL(k_scan_strided4_scale, dim3(grid_of(g.Z * g.X / 4, kThreads)), dim3(kThreads), 0, s,
                         (int32_t*)out, g.Z, g.Y, g.X, h);
    else  // then along z, scaled
      hipLaunchKernelGGL(k_scan_strided4_scale, dim3(grid_of(g.Y * g.X / 4, kThreads)), dim3(kThreads), 0, s,
                         (int32_t*)out, (int64_t)1, g.Z, g.Y * g.X, h);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_lz_pair, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, p, g, axis3, (int32_t*)out, es);
  hipError_t e = lz_scan_axes((int32_t*)out, g.Z, g.Y, g.X, es, axis3, nullptr, s);
  if (e != hipSuccess) return e;
  const double halfq = 0.5 * v.quantum;
  if (v.dtype == 1)
    hipLaunchKernelGGL(k_lz_scale<float>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es, halfq);
  else
    hipLaunchKernelGGL(k_lz_scale<double>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es, halfq);
  return hipGetLastError();
}

}  // namespace hsz
