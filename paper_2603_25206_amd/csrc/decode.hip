// decode.hip -- partial decompression d^(i) = D_i(...D_1(c)) (Alg. 2).
//
// One wavefront per 64-block chunk, one lane per block.  The lane decodes
// its block slot by slot from its LDS column (stage_chunk /
// decode_lane_block), keeps the S outputs in registers and writes them as
// whole 16-byte vectors, so every lane stores one full 128- or 256-byte
// segment of the output.
//   stage 2 (D_p): p[n] then q0[nb]      stage 3 (D_q): q[n]
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
template <int S, int STAGE, typename T>
__global__ void __launch_bounds__(kThreads) k_decode(StreamView v, int kmax, T* __restrict__ out,
                                                    int32_t* __restrict__ out_q0, int* status) {
  extern __shared__ uint32_t smem[];
  const int wv = threadIdx.x / kWave;
  uint32_t* tile = smem + wv * (kmax + 1) * kWave;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  const double quantum = v.quantum;
  for (int64_t c = blockIdx.x * (int64_t)kWavesPerGroup + wv; c < v.nchunks; c += waves) {
    LaneBlock lb;
    stage_chunk<S>(v.width, v.q0, v.chunk_off, v.payload, v.payload_words, v.n, v.nb, c, tile, kmax, lb,
                   status);
    if (lb.len == 0) continue;
    T vals[S];
    decode_lane_block<S>(tile + l, lb.w, lb.q0, [&](int j, int p, int q) {
      if constexpr (STAGE == 2) vals[j] = p;
      else if constexpr (STAGE == 3) vals[j] = q;
      else vals[j] = (T)dequant64(q, quantum);
    });
    store_block<T, S>(out + lb.b * S, vals, lb.len);
    if constexpr (STAGE == 2) out_q0[lb.b] = lb.q0;
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
  const size_t lds = (size_t)kWavesPerGroup * (kmax + 1) * kWave * sizeof(uint32_t);
  const int64_t groups = (v.nchunks + kWavesPerGroup - 1) / kWavesPerGroup;
  const int grid = (int)(groups < 8192 ? groups : 8192);
  int32_t* q0out = (STAGE == 2) ? (int32_t*)out + v.n : nullptr;
  hipLaunchKernelGGL((k_decode<S, STAGE, T>), dim3(grid), dim3(kThreads), lds, s, v, kmax, (T*)out, q0out,
                     status);
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
