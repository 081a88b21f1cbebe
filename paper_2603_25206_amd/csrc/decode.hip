// decode.hip -- partial decompression d^(i) = D_i(...D_1(c)) (Alg. 2).
//
// One wavefront per 64-block chunk, one lane per block.  The lane decodes
// its block slot by slot from its LDS column (stage_chunk /
// decode_lane_block), keeps the S outputs in registers and writes them as
// whole 16-byte vectors, so every lane stores one full 128- or 256-byte
// segment of the output.
//   stage 2 (D_p): p[n] then q0[nb]      stage 3 (D_q): q[n]
//   (block-mean streams: q0 holds the block means and q = M + p)
//   stage 4 (D_f): (dtype)(q * Delta)    stage 1 (D_m): q0[nb] (a copy)
#include "hsz_device.hpp"
#include "hsz_launch.hpp"

namespace hsz {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerGroup = kThreads / kWave;

template <typename T, int S>
__device__ __forceinline__ void store_block(T* dst, const T (&v)[S], int len) {
  if (len == S) {
    constexpr int kPerVec = 16 / sizeof(T);
    typedef T vec_t __attribute__((ext_vector_type(kPerVec)));
#pragma unroll
    for (int j = 0; j < S; j += kPerVec) {
      vec_t t;
#pragma unroll
      for (int u = 0; u < kPerVec; ++u) t[u] = v[j + u];
      *(vec_t*)(dst + j) = t;
    }
  } else {
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (j < len) dst[j] = v[j];
  }
}

// STAGE: 2, 3 or 4.  T: output element type (int32 for 2/3, float/double for 4).
// 4-byte outputs leave through an LDS transpose: lane l writes its block's S
// values to row l of a (64 x (S+1))-word tile (the +1 keeps the writes
// conflict-free), then every lane reads four consecutive outputs of the
// chunk and the wave stores 1 KB of contiguous memory per instruction.
template <int S, int STAGE, typename T, bool MEAN>
__global__ void __launch_bounds__(kThreads) k_decode(StreamView v, int kmax, int wave_words, T* __restrict__ out,
                                                    int32_t* __restrict__ out_q0, int* status) {
  extern __shared__ uint32_t smem[];
  const int wv = wave_in_group();
  uint32_t* tile = smem + wv * wave_words;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  const double quantum = v.quantum;
  constexpr bool kTranspose = sizeof(T) == 4;
  for (int64_t c = blockIdx.x * (int64_t)kWavesPerGroup + wv; c < v.nchunks; c += waves) {
    LaneBlock lb;
    stage_chunk<S>(v.width, v.q0, v.chunk_off, v.payload, v.payload_words, v.n, v.nb, c, tile, kmax, lb,
                   status);
    T vals[S];
    decode_lane_block<S, kWave, MEAN>(tile + l, lb.w, lb.q0, [&](int j, int p, int q) {
      if constexpr (STAGE == 2) vals[j] = p;
      else if constexpr (STAGE == 3) vals[j] = q;
      else vals[j] = (T)dequant64(q, quantum);
    });
    if constexpr (STAGE == 2) {
      if (lb.len > 0) out_q0[lb.b] = lb.q0;
    }
    if constexpr (kTranspose) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < S; ++j) tile[l * (S + 1) + j] = __builtin_bit_cast(uint32_t, vals[j]);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int64_t base = c * kChunkBlocks * S;
      const bool full = base + (int64_t)kChunkBlocks * S <= v.n;
#pragma unroll
      for (int m = 0; m < S / 4; ++m) {
        const int e = m * 4 * kWave + 4 * l;
        const int a = (e / S) * (S + 1) + (e % S);
        uint32_t w4[4] = {tile[a], tile[a + 1], tile[a + 2], tile[a + 3]};
        if (full) {
          typedef uint32_t u4 __attribute__((ext_vector_type(4)));
          *(u4*)((uint32_t*)out + base + e) = u4{w4[0], w4[1], w4[2], w4[3]};
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (base + e + u < v.n) ((uint32_t*)out)[base + e + u] = w4[u];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    } else {
      if (lb.len > 0) store_block<T, S>(out + lb.b * S, vals, lb.len);
    }
  }
}

// Per-block payload offsets relative to the block's chunk (16 bits: a chunk
// holds at most 64 * 62 words), so that any block's words can be located
// with two independent loads: chunk_off[b / 64] + rel[b].  A wave takes four
// chunks at a time: lane l the blocks 4l .. 4l + 3 of them (one 16-lane row
// per chunk), their word counts summed in the lane and scanned over the row;
// one 8-byte store writes the lane's four offsets.
constexpr int kIndexChunks = kWave * 4 / kChunkBlocks;  // chunks per wave and step
static_assert(kChunkBlocks % 4 == 0 && kChunkBlocks / 4 == 16, "one 16-lane row per chunk");
template <int S>
__global__ void __launch_bounds__(kThreads) k_block_index(StreamView v, uint16_t* __restrict__ rel) {
  const int wv = wave_in_group();
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  const int64_t steps = (v.nchunks + kIndexChunks - 1) / kIndexChunks;
  for (int64_t c = blockIdx.x * (int64_t)kWavesPerGroup + wv; c < steps; c += waves) {
    const int64_t b0 = c * (kIndexChunks * kChunkBlocks) + 4 * l;
    int nw[4], pre[4], tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int w = b0 + k < v.nb ? (int)v.width[b0 + k] : 0;
      nw[k] = block_words<S>(w < kMaxWidth ? w : kMaxWidth);
      pre[k] = tot;
      tot += nw[k];
    }
    // exclusive scan of the lane totals within the lane's 16-lane row
    int incl = tot;
    incl += dpp<0x111>(incl);
    incl += dpp<0x112>(incl);
    incl += dpp<0x114>(incl);
    incl += dpp<0x118>(incl);
    const int ex = incl - tot;
    if (b0 + 3 < v.nb) {
      typedef uint32_t u2v __attribute__((ext_vector_type(2)));
      const u2v pk = {(uint32_t)(ex + pre[0]) | ((uint32_t)(ex + pre[1]) << 16),
                      (uint32_t)(ex + pre[2]) | ((uint32_t)(ex + pre[3]) << 16)};
      *(u2v*)(rel + b0) = pk;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (b0 + k < v.nb) rel[b0 + k] = (uint16_t)(ex + pre[k]);
    }
  }
}

// The same index for every gradient job of a batch: units are the chunks of
// all jobs (counts[0] jobs, counts[1] chunks in total).
__global__ void __launch_bounds__(kThreads) k_batch_block_index(const GradJob* __restrict__ jobs,
                                                               const int64_t* __restrict__ chunk_start,
                                                               const int64_t* __restrict__ counts) {
  const int wv = wave_in_group();
  const int l = lane_id();
  const int n = (int)counts[0];
  const int64_t total = counts[1];
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  for (int64_t u = blockIdx.x * (int64_t)kWavesPerGroup + wv; u < total; u += waves) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (chunk_start[mid] <= u) lo = mid;
      else hi = mid - 1;
    }
    const GradJob J = load_job(jobs, lo);
    const int64_t b = (u - chunk_start[lo]) * kChunkBlocks + l;
    const int w = b < J.v.nb ? (int)J.v.width[b] : 0;
    const int wc = w < kMaxWidth ? w : kMaxWidth;
    const int nw = wc ? (J.v.block / 32) * (1 + wc) : 0;
    const int incl = wave_incl_scan(nw);
    if (b < J.v.nb) ((uint16_t*)J.rel)[b] = (uint16_t)(incl - nw);
  }
}

__global__ void k_copy_q0(const int32_t* __restrict__ q0, int64_t nb, int32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = q0[i];
}

template <int S, int STAGE, typename T>
hipError_t run(const StreamView& v, void* out, int* status, hipStream_t s) {
  const int wmax = max(1, 32 - __builtin_clz(2u * v.max_abs_q | 1u));
  const int kmax = tile_rows<S>(wmax > kMaxWidth ? kMaxWidth : wmax) - 1;
  int wave_words = (kmax + 1) * kWave;
  if (sizeof(T) == 4 && wave_words < kWave * (S + 1)) wave_words = kWave * (S + 1);
  const size_t lds = (size_t)kWavesPerGroup * wave_words * sizeof(uint32_t);
  const int64_t groups = (v.nchunks + kWavesPerGroup - 1) / kWavesPerGroup;
  const int grid = (int)(groups < 8192 ? groups : 8192);
  int32_t* q0out = (STAGE == 2) ? (int32_t*)out + v.n : nullptr;
  if (v.flags & 1u)
    hipLaunchKernelGGL((k_decode<S, STAGE, T, true>), dim3(grid), dim3(kThreads), lds, s, v, kmax, wave_words,
                       (T*)out, q0out, status);
  else
    hipLaunchKernelGGL((k_decode<S, STAGE, T, false>), dim3(grid), dim3(kThreads), lds, s, v, kmax, wave_words,
                       (T*)out, q0out, status);
  return hipGetLastError();
}

template <int S>
hipError_t dispatch(const StreamView& v, int stage, void* out, int* status, hipStream_t s) {
  switch (stage) {
    case 2: return run<S, 2, int32_t>(v, out, status, s);
    case 3: return run<S, 3, int32_t>(v, out, status, s);
    case 4:
      return v.dtype == 1 ? run<S, 4, float>(v, out, status, s) : run<S, 4, double>(v, out, status, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_block_index(const StreamView& v, uint16_t* rel, hipStream_t s) {
  const int64_t steps = (v.nchunks + kIndexChunks - 1) / kIndexChunks;
  const int64_t groups = (steps + kWavesPerGroup - 1) / kWavesPerGroup;
  const unsigned grid = (unsigned)(groups < 8192 ? groups : 8192);
  if (v.block == 32) hipLaunchKernelGGL(k_block_index<32>, dim3(grid), dim3(kThreads), 0, s, v, rel);
  else hipLaunchKernelGGL(k_block_index<64>, dim3(grid), dim3(kThreads), 0, s, v, rel);
  return hipGetLastError();
}

hipError_t launch_batch_block_index(const GradJob* jobs, const int64_t* chunk_start, const int64_t* counts, int grid,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_batch_block_index, dim3(grid), dim3(kThreads), 0, s, jobs, chunk_start, counts);
  return hipGetLastError();
}

hipError_t launch_decode(const StreamView& v, int stage, void* out, int* status, hipStream_t s) {
  if (stage == 1) {
    const int64_t g = (v.nb + 255) / 256;
    hipLaunchKernelGGL(k_copy_q0, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, v.q0, v.nb,
                       (int32_t*)out);
    return hipGetLastError();
  }
  return v.block == 32 ? dispatch<32>(v, stage, out, status, s) : dispatch<64>(v, stage, out, status, s);
}

}  // namespace hsz
