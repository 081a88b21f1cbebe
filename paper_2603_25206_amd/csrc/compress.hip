// compress.hip -- c = C(d, eps) on the GPU (Sec. IV, Alg. 1).
//
//   k_minmax      one read of the field: extremes and a non-finite flag
//   k_params      eps -> eps_q -> Delta, 1/Delta (one thread, binary64)
//   k_quant_meta  one lane per block: quantize, decorrelate, block width,
//                 q0, payload words per 64-block chunk, max |q|
//   k_scan_chunks exclusive scan of the chunk word counts -> chunk table
//   k_pack        one lane per block: re-quantize and bit-pack the block
//                 into an LDS copy of the chunk's payload, then copy it out
//                 with coalesced stores
//   k_header      the 256-byte header and the zero padding between sections
//
// Quantization is q = floor(x * (1/Delta) + 0.5) in binary64 with no fused
// multiply-add (compiled with contraction off); the same expression and
// parameter arithmetic as the CPU reference, so streams are byte-identical.
#include "hsz_device.hpp"
#include "hsz_launch.hpp"

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

template <typename T>
__global__ void __launch_bounds__(kThreads) k_minmax(const T* __restrict__ x, int64_t n, double* partial) {
  double lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double v = (double)x[i];
    bad |= !isfinite(v);
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  for (int m = 32; m >= 1; m >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, m));
    hi = fmax(hi, __shfl_xor(hi, m));
    bad |= __shfl_xor(bad, m);
  }
  __shared__ double slo[kThreads / kWave], shi[kThreads / kWave];
  __shared__ int sbad[kThreads / kWave];
  const int wv = wave_in_group();
  if (lane_id() == 0) { slo[wv] = lo; shi[wv] = hi; sbad[wv] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kThreads / kWave; ++k) {
      lo = fmin(lo, slo[k]);
      hi = fmax(hi, shi[k]);
      bad |= sbad[k];
    }
    partial[3 * blockIdx.x + 0] = lo;
    partial[3 * blockIdx.x + 1] = hi;
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
__global__ void __launch_bounds__(kThreads) k_params(const double* partial, int groups, double eb, int eb_is_rel,
                                                     int dtype, CompressWs* ws) {
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
  if (!(eps_q > 0.0)) {
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

template <typename T, int S>
__global__ void __launch_bounds__(kThreads) k_quant_meta(const T* __restrict__ x, int64_t n, int64_t nb,
                                                        int64_t nchunks, CompressWs* ws, int32_t* q0s,
                                                        uint8_t* widths, uint32_t* chunk_words) {
  if (ws->status != 0) return;
  const double inv = ws->inv_quantum;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (kThreads / kWave);
  uint32_t maxq = 0;
  bool over = false;
  for (int64_t c = blockIdx.x * (int64_t)(kThreads / kWave) + wave_in_group(); c < nchunks; c += waves) {
    const int64_t b = c * kChunkBlocks + l;
    int w = 0;
    if (b < nb) {
      const T* xb = x + b * S;
      const int len = (int)((n - b * S) < S ? (n - b * S) : S);
      int qprev = 0;
      uint32_t orp = 0;
      int q0 = 0;
#pragma unroll 8
      for (int j = 0; j < S; ++j) {
        if (j < len) {
          int q = quantize((double)xb[j], inv, over);
          uint32_t aq = (uint32_t)(q < 0 ? -q : q);
          maxq = aq > maxq ? aq : maxq;
          if (j == 0) q0 = q;
          int p = (j == 0) ? 0 : q - qprev;
          orp |= (uint32_t)(p < 0 ? -p : p);
          qprev = q;
        }
      }
      w = bitlen(orp);
      q0s[b] = q0;
      widths[b] = (uint8_t)w;
    }
    int words = block_words<S>(w);
    int tot = wave_incl_scan(words);
    if (l == kWave - 1) chunk_words[c] = (uint32_t)tot;
  }
  maxq = (uint32_t)wave_max((int)maxq);
  if (l == 0) atomicMax(&ws->max_abs_q, maxq);
  if (__any(over) && l == 0) record_status(&ws->status, kErrRange);
}

// One workgroup: exclusive scan of chunk_words into the stream's chunk table.
__global__ void __launch_bounds__(1024) k_scan_chunks(const uint32_t* chunk_words, int64_t nchunks,
                                                      uint64_t* chunk_off, CompressWs* ws,
                                                      uint64_t off_payload, uint64_t cap) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (nchunks + 1023) / 1024;
  const int64_t lo = t * per, hi = (lo + per < nchunks) ? lo + per : nchunks;
  uint64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += chunk_words[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint64_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint64_t run = part[t] - s;  // exclusive prefix of this thread's segment
  for (int64_t i = lo; i < hi; ++i) {
    chunk_off[i] = run;
    run += chunk_words[i];
  }
  if (t == 1023) {
    const uint64_t total = part[1023];
    chunk_off[nchunks] = total;
    ws->total_words = total;
    if (off_payload + 4 * total > cap) record_status(&ws->status, kErrCapacity);
  }
}

template <typename T, int S>
__global__ void __launch_bounds__(kThreads) k_pack(const T* __restrict__ x, int64_t n, int64_t nb,
                                                  int64_t nchunks, const CompressWs* ws,
                                                  const uint8_t* __restrict__ widths,
                                                  const uint64_t* __restrict__ chunk_off,
                                                  uint32_t* payload) {
  if (ws->status != 0) return;
  constexpr int kRows = (S / 32) * (1 + kMaxWidth);
  __shared__ uint32_t lin_all[(kThreads / kWave) * kRows * kWave];
  uint32_t* lin = lin_all + (wave_in_group()) * kRows * kWave;
  const double inv = ws->inv_quantum;
  const int l = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (kThreads / kWave);
  for (int64_t c = blockIdx.x * (int64_t)(kThreads / kWave) + wave_in_group(); c < nchunks; c += waves) {
    const int64_t b = c * kChunkBlocks + l;
    const int w = (b < nb) ? (int)widths[b] : 0;
    const int nw = block_words<S>(w);
    const int incl = wave_incl_scan(nw);
    const int woff = incl - nw;
    const int total = __shfl(incl, kWave - 1);
    if (total < 0 || total > kRows * kWave) continue;  // widths are <= 30, so never taken
    for (int k = 0; k < nw; ++k) lin[woff + k] = 0u;
    if (w > 0) {
      const T* xb = x + b * S;
      const int len = (int)((n - b * S) < S ? (n - b * S) : S);
      uint32_t sg0 = 0, sg1 = 0;
      uint32_t* mag = lin + woff + S / 32;
      int qprev = 0;
      bool over = false;
      for (int j = 0; j < len; ++j) {
        int q = quantize((double)xb[j], inv, over);
        int p = (j == 0) ? 0 : q - qprev;
        qprev = q;
        if (p < 0) {
          if (j < 32) sg0 |= 1u << j;
          else sg1 |= 1u << (j - 32);
        }
        uint32_t m = (uint32_t)(p < 0 ? -p : p);
        uint32_t pos = (uint32_t)j * (uint32_t)w;
        uint32_t k = pos >> 5, sh = pos & 31u;
        mag[k] |= m << sh;
        if (sh + (uint32_t)w > 32u) mag[k + 1] |= m >> (32u - sh);
      }
      lin[woff] = sg0;
      if (S == 64) lin[woff + 1] = sg1;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t* dst = payload + chunk_off[c];
    for (int t = l; t < total; t += kWave) dst[t] = lin[t];
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
__global__ void k_header(uint8_t* out, const CompressWs* ws, int dtype, int ndim, int64_t d0, int64_t d1,
                         int64_t d2, int64_t n, int block, int64_t nb, int64_t nchunks, uint64_t off_chunk,
                         uint64_t off_q0, uint64_t off_width, uint64_t off_payload) {
  __shared__ uint8_t h[kHeaderBytes];
  const int t = threadIdx.x;
  if (t < kHeaderBytes) h[t] = 0;
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
    uint32_t flags = 0;
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

template <typename T, int S>
hipError_t run(const CompressArgs& a, hipStream_t s) {
  const Layout& L = a.lay;
  CompressWs* ws = (CompressWs*)a.ws;
  double* partial = (double*)(a.ws + kWsPartials);
  uint32_t* chunk_words = (uint32_t*)(a.ws + kWsPartials + 24 * kMinmaxGroups);
  uint8_t* out = a.out;
  const T* x = (const T*)a.x;
  int g = (int)((L.n + kThreads * 8 - 1) / (kThreads * 8));
  g = g < 1 ? 1 : (g > kMinmaxGroups ? kMinmaxGroups : g);
  hipLaunchKernelGGL(k_minmax<T>, dim3(g), dim3(kThreads), 0, s, x, L.n, partial);
  hipLaunchKernelGGL(k_params, dim3(1), dim3(kThreads), 0, s, partial, g, a.eb, a.eb_is_rel, a.dtype, ws);
  const int64_t cg = (L.nchunks + 3) / 4;
  const int grid = (int)(cg < 4096 ? cg : 4096);
  hipLaunchKernelGGL((k_quant_meta<T, S>), dim3(grid), dim3(kThreads), 0, s, x, L.n, L.nb, L.nchunks, ws,
                     (int32_t*)(out + L.off_q0), out + L.off_width, chunk_words);
  hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, s, chunk_words, L.nchunks,
                     (uint64_t*)(out + L.off_chunk), ws, L.off_payload, a.cap);
  hipLaunchKernelGGL((k_pack<T, S>), dim3(grid), dim3(kThreads), 0, s, x, L.n, L.nb, L.nchunks, ws,
                     (const uint8_t*)(out + L.off_width), (const uint64_t*)(out + L.off_chunk),
                     (uint32_t*)(out + L.off_payload));
  hipLaunchKernelGGL(k_header, dim3(1), dim3(kHeaderBytes), 0, s, out, ws, a.dtype, a.ndim, a.dims[0],
                     a.dims[1], a.dims[2], L.n, L.block, L.nb, L.nchunks, L.off_chunk, L.off_q0,
                     L.off_width, L.off_payload);
  return hipGetLastError();
}

}  // namespace

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

uint64_t compress_workspace_bytes(const Layout& lay) {
  return kWsPartials + 24 * (uint64_t)kMinmaxGroups + 4 * (uint64_t)lay.nchunks + 256;
}

hipError_t launch_compress(const CompressArgs& a, hipStream_t s) {
  if (a.dtype == 1)
    return a.lay.block == 32 ? run<float, 32>(a, s) : run<float, 64>(a, s);
  return a.lay.block == 32 ? run<double, 32>(a, s) : run<double, 64>(a, s);
}

}  // namespace hsz
