// lorenzo.hip -- decoding of HSZp-nd streams (Sec. IV, multidimensional
// Lorenzo decorrelation) and the derivative on their decorrelated data
// (Eq. (derivative_Dp)).
//
// D_p: one wavefront per 64-block chunk, one lane per nd block; the lane
// decodes its block slot by slot from its LDS column and writes each slot to
// its coordinates in the field (rows of BX consecutive words).
// D_q: q is the nd prefix sum of p (the inverse of the residual), built in
// place with one pass per axis: along x a wave per row (four words per lane,
// a wave scan, a carry across 256-word segments), along y and z a thread per
// column walking the axis with a running sum (consecutive threads own
// consecutive x, so every step is a coalesced row).  Partial sums never
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

// D_p -> out (int32 words at element stride es), the field's layout.
template <int S, int ND>
__global__ void __launch_bounds__(kThreads) k_lz_decode_p(StreamView v, NdGrid g, int kmax, int32_t* __restrict__ out,
                                                         int es, int* status) {
  using Sh = NdShape<ND, S>;
  extern __shared__ uint32_t smem[];
  const int wv = wave_in_group();
  uint32_t* tile = smem + wv * (kmax + 1) * kWave;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kWavesPerGroup;
  for (int64_t c = blockIdx.x * (int64_t)kWavesPerGroup + wv; c < v.nchunks; c += waves) {
    const int w = lz_stage<S>(v, c, tile, kmax, status);
    const int64_t b = c * kChunkBlocks + l;
    if (b < v.nb) {
      const int64_t oz = (b / (g.nby * g.nbx)) * Sh::BZ, oy = ((b / g.nbx) % g.nby) * Sh::BY,
                    ox = (b % g.nbx) * Sh::BX;
      const bool whole = oz + Sh::BZ <= g.Z && oy + Sh::BY <= g.Y && ox + Sh::BX <= g.X;
      int32_t* base = out + ((oz * g.Y + oy) * g.X + ox) * es;
      decode_lane_block<S, kWave, true>(tile + l, w, 0, [&](int j, int p, int) {
        const int sz = j / (Sh::BY * Sh::BX), sy = (j / Sh::BX) % Sh::BY, sx = j % Sh::BX;
        if (whole || (oz + sz < g.Z && oy + sy < g.Y && ox + sx < g.X))
          base[((sz * g.Y + sy) * g.X + sx) * es] = p;
      });
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
#pragma unroll 8
    for (int64_t i = 0; i < len; ++i) {
      run += p[i * step];
      p[i * step] = run;
    }
  }
}

// q (int32 at element stride es) -> T in place
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_dequant(void* buf, int64_t n, int es, double quantum) {
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
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const int num = ((const int32_t*)buf)[i * es];
    ((T*)buf)[i] = (T)num * h;
  }
}

unsigned grid_of(int64_t items, int per) {
  const int64_t g = (items + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

template <int S, int ND>
hipError_t decode_p(const StreamView& v, const NdGrid& g, int32_t* out, int es, int* status, hipStream_t s) {
  const int kmax = lz_kmax<S, ND>(v.max_abs_q);
  const size_t lds = (size_t)kWavesPerGroup * (kmax + 1) * kWave * sizeof(uint32_t);
  const int64_t groups = (v.nchunks + kWavesPerGroup - 1) / kWavesPerGroup;
  const unsigned grid = (unsigned)(groups < 8192 ? (groups < 1 ? 1 : groups) : 8192);
  hipLaunchKernelGGL((k_lz_decode_p<S, ND>), dim3(grid), dim3(kThreads), lds, s, v, g, kmax, out, es, status);
  return hipGetLastError();
}

hipError_t decode_p_any(const StreamView& v, const NdGrid& g, int32_t* out, int es, int* status, hipStream_t s) {
  if (g.ndim == 3) return v.block == 32 ? decode_p<32, 3>(v, g, out, es, status, s) : decode_p<64, 3>(v, g, out, es, status, s);
  return v.block == 32 ? decode_p<32, 2>(v, g, out, es, status, s) : decode_p<64, 2>(v, g, out, es, status, s);
}

}  // namespace

hipError_t lz_scan_axes(int32_t* buf, int64_t Z, int64_t Y, int64_t X, int es, int skip, hipStream_t s) {
  if (skip != 2) {
    const int64_t rows = Z * Y;
    hipLaunchKernelGGL(k_scan_x, dim3(grid_of(rows, kWavesPerGroup)), dim3(kThreads), 0, s, buf, rows, X, es);
  }
  if (skip != 1 && Y > 1)
    hipLaunchKernelGGL(k_scan_strided, dim3(grid_of(Z * X, kThreads)), dim3(kThreads), 0, s, buf, Z, Y, X, es);
  if (skip != 0 && Z > 1)
    hipLaunchKernelGGL(k_scan_strided, dim3(grid_of(Y * X, kThreads)), dim3(kThreads), 0, s, buf, (int64_t)1, Z,
                       Y * X, es);
  return hipGetLastError();
}

hipError_t lz_decode(const StreamView& v, const NdGrid& g, int stage, void* out, int* status, hipStream_t s) {
  if (stage < 2 || stage > 4) return hipErrorInvalidValue;
  const int es = (stage == 4 && v.dtype == 2) ? 2 : 1;
  hipError_t e = decode_p_any(v, g, (int32_t*)out, es, status, s);
  if (e != hipSuccess || stage == 2) return e;
  e = lz_scan_axes((int32_t*)out, g.Z, g.Y, g.X, es, -1, s);
  if (e != hipSuccess || stage == 3) return e;
  const int64_t n = g.Z * g.Y * g.X;
  if (v.dtype == 1)
    hipLaunchKernelGGL(k_lz_dequant<float>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es, v.quantum);
  else
    hipLaunchKernelGGL(k_lz_dequant<double>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es,
                       v.quantum);
  return hipGetLastError();
}

hipError_t lz_deriv_p(const int32_t* p, const StreamView& v, const NdGrid& g, int axis3, void* out, hipStream_t s) {
  const int es = v.dtype == 2 ? 2 : 1;
  const int64_t n = g.Z * g.Y * g.X;
  hipLaunchKernelGGL(k_lz_pair, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, p, g, axis3, (int32_t*)out, es);
  hipError_t e = lz_scan_axes((int32_t*)out, g.Z, g.Y, g.X, es, axis3, s);
  if (e != hipSuccess) return e;
  const double halfq = 0.5 * v.quantum;
  if (v.dtype == 1)
    hipLaunchKernelGGL(k_lz_scale<float>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es, halfq);
  else
    hipLaunchKernelGGL(k_lz_scale<double>, dim3(grid_of(n, kThreads)), dim3(kThreads), 0, s, out, n, es, halfq);
  return hipGetLastError();
}

}  // namespace hsz
