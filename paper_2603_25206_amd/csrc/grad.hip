// grad.hip -- derivatives and gradient magnitude (Eq. (derivatives),
// Sec. V-B) on materialised stage buffers.
//
// Stage 3 (D_q): integer numerators n = q_{+1} - q_{-1} inside the field and
// n = 2 (q_1 - q_0) at its ends (the one-sided difference, expressed over the
// same denominator), scaled once by Delta/2:  g = n * Delta/2.
// Stage 4 (D_f): the same stencil on the decompressed floats in the field's
// own precision: (x_{+1} - x_{-1}) / 2 inside, x_1 - x_0 at the ends.
// Gradient magnitude = sqrt(sum_k g_k^2); an axis of length 1 adds 0.
#include "hsz_device.hpp"
#include "hsz_launch.hpp"

namespace hsz {

namespace {

constexpr int kThreads = 256;

// integer numerator along one axis at coordinate i of length L, stride st
__device__ __forceinline__ int qnum(const int32_t* __restrict__ q, int64_t e, int64_t i, int64_t L, int64_t st) {
  if (L < 2) return 0;
  if (i == 0) return 2 * (q[e + st] - q[e]);
  if (i == L - 1) return 2 * (q[e] - q[e - st]);
  return q[e + st] - q[e - st];
}

template <typename T>
__device__ __forceinline__ T fdiff(const T* __restrict__ x, int64_t e, int64_t i, int64_t L, int64_t st) {
  if (L < 2) return T(0);
  if (i == 0) return x[e + st] - x[e];
  if (i == L - 1) return x[e] - x[e - st];
  return (x[e + st] - x[e - st]) * T(0.5);
}

// SRC 3: int32 q in; SRC 4: T floats in.  OP 3: derivative along axis, 4: magnitude.
template <int SRC, int OP, typename T>
__global__ void __launch_bounds__(kThreads) k_grad_buf(const void* __restrict__ in, Dims3 d, Box3 b, int axis,
                                                      double halfq, T* __restrict__ out) {
  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0, bz = b.z1 - b.z0;
  const int64_t tiles = (bx + kThreads - 1) / kThreads;
  const int64_t items = bz * by * tiles;
  const T h = (T)halfq;
  const int64_t sy = d.x, sz = d.x * d.y;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t tile = it % tiles, row = it / tiles;
    const int64_t ox = tile * kThreads + threadIdx.x;
    if (ox >= bx) continue;
    const int64_t iy = row % by, iz = row / by;
    const int64_t x = b.x0 + ox, y = b.y0 + iy, z = b.z0 + iz;
    const int64_t e = (z * d.y + y) * d.x + x;
    T r;
    if constexpr (SRC == 3) {
      const int32_t* q = (const int32_t*)in;
      if constexpr (OP == 3) {
        int n = axis == 0 ? qnum(q, e, z, d.z, sz) : axis == 1 ? qnum(q, e, y, d.y, sy) : qnum(q, e, x, d.x, 1);
        r = (T)n * h;
      } else {
        const T gz = (T)qnum(q, e, z, d.z, sz), gy = (T)qnum(q, e, y, d.y, sy), gx = (T)qnum(q, e, x, d.x, 1);
        r = sqrt(gz * gz + gy * gy + gx * gx) * h;
      }
    } else {
      const T* f = (const T*)in;
      if constexpr (OP == 3) {
        r = axis == 0 ? fdiff(f, e, z, d.z, sz) : axis == 1 ? fdiff(f, e, y, d.y, sy) : fdiff(f, e, x, d.x, (int64_t)1);
      } else {
        const T gz = fdiff(f, e, z, d.z, sz), gy = fdiff(f, e, y, d.y, sy), gx = fdiff(f, e, x, d.x, (int64_t)1);
        r = sqrt(gz * gz + gy * gy + gx * gx);
      }
    }
    out[(iz * by + iy) * bx + ox] = r;
  }
}

template <int SRC, typename T>
hipError_t run(const void* buf, int op, int axis, const OpTarget& t, double halfq, void* out, hipStream_t s) {
  const Box3& b = t.box;
  const int64_t tiles = (b.x1 - b.x0 + kThreads - 1) / kThreads;
  const int64_t items = (b.z1 - b.z0) * (b.y1 - b.y0) * tiles;
  const int grid = (int)(items < 65536 ? items : 65536);
  if (op == 3)
    hipLaunchKernelGGL((k_grad_buf<SRC, 3, T>), dim3(grid), dim3(kThreads), 0, s, buf, t.d, b, axis, halfq, (T*)out);
  else
    hipLaunchKernelGGL((k_grad_buf<SRC, 4, T>), dim3(grid), dim3(kThreads), 0, s, buf, t.d, b, axis, halfq, (T*)out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grad_stage(const void* buf, int stage, const StreamView& v, int op, int axis3, const OpTarget& t,
                             void* result, uint8_t*, hipStream_t s) {
  const double halfq = 0.5 * v.quantum;
  if (stage == 3)
    return v.dtype == 1 ? run<3, float>(buf, op, axis3, t, halfq, result, s)
                        : run<3, double>(buf, op, axis3, t, halfq, result, s);
  if (stage == 4)
    return v.dtype == 1 ? run<4, float>(buf, op, axis3, t, halfq, result, s)
                        : run<4, double>(buf, op, axis3, t, halfq, result, s);
  return hipErrorInvalidValue;
}

hipError_t launch_grad_fused(const StreamView&, int, int, int, const OpTarget&, void*, uint8_t*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace hsz
