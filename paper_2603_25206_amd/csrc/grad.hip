// grad.hip -- derivatives and gradient magnitude (Eq. (derivatives),
// Sec. V-B) on materialised stage buffers and fused with decoding.
//
// Integer route (D_q): numerators n = q_{+1} - q_{-1} inside the field and
// n = 2 (q_1 - q_0) at its ends (the one-sided difference over the same
// denominator), scaled once by Delta/2: g = n * Delta/2.
// Float route (D_f): the same stencil on the decompressed values in the
// field's own precision: (x_{+1} - x_{-1}) * 0.5 inside, x_1 - x_0 at the ends.
// Gradient magnitude = sqrt(g_z^2 + g_y^2 + g_x^2); an axis of length 1 adds 0.
// Laplacian (Eq. (laplacian), op 5): the sum over the axes of the second
// difference v_{-1} + v_{+1} - 2 v, the end value standing in for a missing
// neighbour; the integer route scales the exact numerator once by Delta.
//
// Both kernels march along z (the slowest axis) and keep the z-neighbours of
// every (x, y) column in registers, so each value is read from memory once
// per pass; in-plane neighbours come from the cache (buffer kernel) or from
// one LDS plane (fused kernel).  The fused kernel is the blockwise sliding
// window of Alg. 3 mapped to the GPU: it decodes each plane of its tile
// (plus a one-cell halo) from the compressed bytes into LDS, one lane per
// block, and never writes the stage to memory.
#include "hsz_device.hpp"
#include "hsz_launch.hpp"

namespace hsz {

namespace {

// ---- numerators -------------------------------------------------------------------
// v(-1), v(0), v(+1) along one axis at coordinate i of length L.
__device__ __forceinline__ int inum(int vm, int v0, int vp, int64_t i, int64_t L) {
  if (L < 2) return 0;
  if (i == 0) return 2 * (vp - v0);
  if (i == L - 1) return 2 * (v0 - vm);
  return vp - vm;
}

template <typename T>
__device__ __forceinline__ T fnum(T vm, T v0, T vp, int64_t i, int64_t L) {
  if (L < 2) return T(0);
  if (i == 0) return vp - v0;
  if (i == L - 1) return v0 - vm;
  return (vp - vm) * T(0.5);
}

// second difference along one axis at coordinate i of length L, the end
// value standing in for a missing neighbour (0 on an axis of length 1)
template <typename N>
__device__ __forceinline__ N lap1(N vm, N v0, N vp, int64_t i, int64_t L) {
  const N a = i > 0 ? vm : v0, b = i + 1 < L ? vp : v0;
  return (a + b) - (v0 + v0);
}

// an exact integer Laplacian numerator n -> n * Delta, rounded once
template <typename T>
__device__ __forceinline__ T lap_value(int n, double quantum) {
  return (T)((double)n * quantum);
}

// square root: v_sqrt_f32 (within 1 ulp) for binary32, the IEEE one for binary64
__device__ __forceinline__ float vsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double vsqrt(double a) { return sqrt(a); }

// in-plane part of the squared magnitude, gy^2 + gx^2
template <bool INT, typename T, typename N>
__device__ __forceinline__ T sq_xy(N ny, N nx) {
  const T gy = (T)ny, gx = (T)nx;
  return gy * gy + gx * gx;
}

// a z/y/x-numerator triple -> output; the magnitude is sqrt(gz^2 + (gy^2 + gx^2))
template <int OP, bool INT, typename T, typename N>
__device__ __forceinline__ T finish(N nz, N ny, N nx, int axis, T h) {
  if constexpr (OP == 3) {
    const N n = axis == 0 ? nz : axis == 1 ? ny : nx;
    if constexpr (INT) return (T)n * h;
    else return n;
  } else {
    const T gz = (T)nz;
    const T m = vsqrt(gz * gz + sq_xy<INT, T, N>(ny, nx));
    if constexpr (INT) return m * h;
    else return m;
  }
}

// ---- stage buffers: 2.5D z-march, one thread per (x, y) column -------------------
constexpr int kBx = 64, kBy = 4, kBufThreads = kBx * kBy;

// SRC 3: int32 q; SRC 4: T floats.  OP 3: derivative along axis, 4: magnitude.
template <int SRC, int OP, typename T>
__global__ void __launch_bounds__(kBufThreads) k_grad_buf(const void* __restrict__ in, Dims3 d, Box3 b, int axis,
                                                          int tz, double halfq, T* __restrict__ out) {
  using V = typename std::conditional<SRC == 3, int, T>::type;
  constexpr bool INT = SRC == 3;
  const V* src = (const V*)in;
  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int64_t ntx = (bx + kBx - 1) / kBx, nty = (by + kBy - 1) / kBy;
  int64_t blk = blockIdx.x;
  const int64_t tx = blk % ntx;
  blk /= ntx;
  const int64_t ty = blk % nty;
  const int64_t tzi = blk / nty;
  const int64_t x = b.x0 + tx * kBx + (threadIdx.x % kBx);
  const int64_t y = b.y0 + ty * kBy + (threadIdx.x / kBx);
  if (x >= b.x1 || y >= b.y1) return;
  const int64_t z0 = b.z0 + tzi * tz;
  const int64_t z1 = min(b.z1, z0 + tz);
  const int64_t sy = d.x, sz = d.x * d.y;
  const T h = (T)halfq;
  const bool need_z = OP >= 4 || axis == 0, need_y = OP >= 4 || axis == 1, need_x = OP >= 4 || axis == 2;
  const V* col = src + y * sy + x;
  using N = typename std::conditional<INT, int, T>::type;
  constexpr int U = 4;  // planes per iteration: their loads are issued together
  V qm = z0 > 0 ? col[(z0 - 1) * sz] : V(0);
  V qc = col[z0 * sz];
  for (int64_t zb = z0; zb < z1; zb += U) {
    V qn[U], ym[U], yp[U], xm[U], xp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t z = zb + u;
      const bool in = z < z1;
      qn[u] = (in && z + 1 < d.z) ? col[(z + 1) * sz] : V(0);
      const V* e = col + z * sz;
      ym[u] = (in && need_y && y > 0) ? e[-sy] : V(0);
      yp[u] = (in && need_y && y + 1 < d.y) ? e[sy] : V(0);
      xm[u] = (in && need_x && x > 0) ? e[-1] : V(0);
      xp[u] = (in && need_x && x + 1 < d.x) ? e[1] : V(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t z = zb + u;
      if (z < z1 && OP == 5) {
        const N lz = lap1<N>(qm, qc, qn[u], z, d.z), ly = lap1<N>(ym[u], qc, yp[u], y, d.y);
        const N l = lz + ly + lap1<N>(xm[u], qc, xp[u], x, d.x);
        T r;
        if constexpr (INT) r = lap_value<T>(l, 2.0 * halfq);
        else r = l;
        out[((z - b.z0) * by + (y - b.y0)) * bx + (x - b.x0)] = r;
        qm = qc;
        qc = qn[u];
      } else if (z < z1) {
        N nz = 0, ny = 0, nx = 0;
        if constexpr (INT) {
          if (need_z) nz = inum(qm, qc, qn[u], z, d.z);
          if (need_y) ny = inum(ym[u], qc, yp[u], y, d.y);
          if (need_x) nx = inum(xm[u], qc, xp[u], x, d.x);
        } else {
          if (need_z) nz = fnum<T>(qm, qc, qn[u], z, d.z);
          if (need_y) ny = fnum<T>(ym[u], qc, yp[u], y, d.y);
          if (need_x) nx = fnum<T>(xm[u], qc, xp[u], x, d.x);
        }
        out[((z - b.z0) * by + (y - b.y0)) * bx + (x - b.x0)] = finish<OP, INT, T>(nz, ny, nx, axis, h);
        qm = qc;
        qc = qn[u];
      }
    }
  }
}

// ---- fused: decode tiles from the compressed stream --------------------------------
constexpr int kTx = 256, kTy = 16, kRows = kTy + 2, kCols = kTx + 2;
constexpr int kFusedThreads = kTx;

// LDS row pitch of a decoded plane.  Rows hold one pad word per 32 columns,
// so consecutive blocks of a row start (S + S/32) words apart; decode lane i
// owns block i % NBR of row i / NBR.  A pitch congruent to NBR (S + S/32)
// modulo 64 places lane i's slot j at i (S + S/32) + const (mod 64): for
// S = 32 (an odd block span) the 64 lanes of a wave write 64 distinct banks.
constexpr int conflict_free_pitch(int min_pitch, int nbr, int span) {
  int p = min_pitch;
  while (p % 64 != (nbr * span) % 64) ++p;
  return p;
}
template <int S>
constexpr int kNbr = (kCols + S - 2) / S + 1;  // max blocks covering one decoded row
template <int S>
constexpr int kPitch = conflict_free_pitch(kCols + (kCols >> 5), kNbr<S>, S + S / 32);

// One workgroup: a tile of kTx columns x kTy rows, marching over tz planes.
// Every decoded row's covering blocks get one thread each (decode items);
// every tile column gets one thread (stencil).  Per plane p:
//   A  each decode thread decodes its staged block of plane p into the LDS
//      plane tile (its staging column is private, so no barrier is needed)
//   -- barrier --
//   B  it issues the payload loads of its block of plane p+1 into registers
//      and the metadata loads (width, q0, offset) of plane p+2
//   C  every stencil thread processes its column for all rows of plane p
//      while those loads are in flight
//   D  the prefetched words go to the staging column
//   -- barrier --
// so the global-memory latency of the next planes overlaps the stencil.
// Block offsets come from the chunk table plus the per-block index 'rel'.
// z-neighbours and the in-plane part of the previous plane stay in registers.
// ACC (quantized route only): also sum q and q^2 over the tile's own
// elements (each element of the box is emitted by exactly one tile) and add
// the sums to job.acc -- statistics that share this decode.  ACC 1 needs
// max|q| < 2^16 (squares fit 32 bits), ACC 2 takes any q.
template <int S, int VIA, int OP, typename T>
__device__ __forceinline__ void grad_tile(const GradJob& job, int64_t tile, uint32_t* smem, int* status) {
  const StreamView& v = job.v;
  const uint16_t* __restrict__ rel = job.rel;
  const Dims3 d = job.d;
  const Box3 b = job.b;
  const int axis = job.axis, tz = job.tz, kmax = job.kmax;
  const double halfq = job.halfq;
  T* __restrict__ out = (T*)job.out;
  using V = typename std::conditional<VIA == 3, int, T>::type;
  constexpr bool INT = VIA == 3;
  using N = typename std::conditional<INT, int, T>::type;
  // per-row state from the previous plane: one in-plane numerator (a single
  // derivative) or gy^2 + gx^2 (the magnitude)
  using G = typename std::conditional<OP == 3, N, T>::type;
  constexpr int NBR = kNbr<S>;
  constexpr int PF = 16 * (S / 32);  // payload words prefetched per thread
  constexpr int kP = kPitch<S>;
  static_assert(kRows * NBR <= kFusedThreads, "one decode item per thread");
  V* plane = (V*)smem;
  uint32_t* stage = smem + (kRows * kP * sizeof(V) + 3) / 4;
  const int t = threadIdx.x;

  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int64_t ntx = (bx + kTx - 1) / kTx, nty = (by + kTy - 1) / kTy;
  int64_t blk = tile;
  const int64_t tx = blk % ntx;
  blk /= ntx;
  const int64_t ty = blk % nty;
  const int64_t tzi = blk / nty;
  const int64_t x0 = b.x0 + tx * kTx, y0 = b.y0 + ty * kTy, z0 = b.z0 + tzi * tz;
  const int xs = (int)min((int64_t)kTx, b.x1 - x0), ys = (int)min((int64_t)kTy, b.y1 - y0);
  const int64_t zs = min((int64_t)tz, b.z1 - z0);
  const int64_t cA = max((int64_t)0, x0 - 1), cB = min(d.x, x0 + xs + 1);
  const int64_t rA = max((int64_t)0, y0 - 1), rB = min(d.y, y0 + ys + 1);
  const int64_t za = max((int64_t)0, z0 - 1), zb = min(d.z, z0 + zs + 1);
  const int nrows = (int)(rB - rA);
  const double quantum = v.quantum;
  const T h = (T)halfq;
  const bool need_z = OP >= 4 || axis == 0, need_y = OP >= 4 || axis == 1, need_x = OP >= 4 || axis == 2;

  // decode item of this thread: decoded row dr, dk-th block of the row
  const int dr = t / NBR, dk = t % NBR;
  const int64_t dy = rA + dr;
  const bool decoder = dr < nrows;
  V* prow = plane + (int)(dy - (y0 - 1)) * kP;
  uint32_t* col = stage + t;

  struct Meta {
    int w, q0, words, e0;
    uint64_t off;
    bool valid;
  };
  // metadata of this thread's block in plane p (loads only; checked in use)
  auto meta_of = [&](int64_t p) {
    Meta m{0, 0, 0, 0, 0, false};
    if (decoder && p < zb) {
      const int64_t f = (p * d.y + dy) * d.x;
      const int64_t bA = (f + cA) / S, bB = (f + cB - 1) / S, bk = bA + dk;
      if (bk <= bB) {
        m.valid = true;
        m.w = (int)v.width[bk];
        m.q0 = v.q0[bk];
        m.off = v.chunk_off[bk / kChunkBlocks] + rel[bk];
        m.e0 = (int)(bk * S - f);
      }
    }
    return m;
  };
  auto check = [&](Meta& m) {
    if (!m.valid) return;
    m.words = block_words<S>(m.w);
    if (m.w > kMaxWidth || m.words > kmax || m.off + (uint64_t)m.words > v.payload_words) {
      record_status(status, kErrBadStream);
      m.w = 0;
      m.words = 0;
    }
  };
  auto stage_rest = [&](const Meta& m, int from) {  // words [from, m.words) straight to LDS
    const uint32_t* src = v.payload + m.off;
    for (int k = from; k < m.words; ++k) col[k * kFusedThreads] = src[k];
  };
  auto decode = [&](const Meta& m) {
    if (!m.valid) return;
    const int cb = m.e0 - (int)(x0 - 1);  // LDS column of slot 0
    const int ja = max(0, (int)(cA - m.e0)), jb = min(S, (int)(cB - m.e0));
    decode_lane_block<S, kFusedThreads>(col, m.w, m.q0, [&](int j, int, int q) {
      if (j >= ja && j < jb) {
        const int cc = cb + j;
        if constexpr (INT) prow[cc + (cc >> 5)] = q;
        else prow[cc + (cc >> 5)] = (T)dequant64(q, quantum);
      }
    });
  };

  // stencil column of this thread
  const int c = t + 1;
  const int64_t x = x0 + t;
  const bool active = t < xs;
  const int ac = c + (c >> 5);              // LDS address of column c in row 0
  const int am = (c - 1) + ((c - 1) >> 5);  // column c-1
  const int ap = (c + 1) + ((c + 1) >> 5);  // column c+1
  const bool xlo = x == 0, xhi = x == d.x - 1, xone = d.x < 2;
  const int64_t obase = x - b.x0;

  V qm2[kTy], qm1[kTy];
  G g1[kTy];
#pragma unroll
  for (int i = 0; i < kTy; ++i) { qm2[i] = V(0); qm1[i] = V(0); g1[i] = G(0); }
  auto emit = [&](int64_t o, int i, N nz) {
    const int64_t row = ((o - b.z0) * by + (y0 + i - b.y0)) * bx;
    T r;
    if constexpr (OP == 5) {
      r = (T)g1[i] + (T)nz;  // the float route only (INT is false here)
    } else if constexpr (OP == 3) {
      if (axis == 0) r = INT ? (T)nz * h : (T)nz;
      else r = INT ? (T)g1[i] * h : (T)g1[i];
    } else {
      const T gz = (T)nz;
      const T m = vsqrt(gz * gz + g1[i]);
      r = INT ? m * h : m;
    }
    out[row + obase] = r;
  };

  // prologue: plane za staged, metadata of za+1 in flight
  Meta cur = meta_of(za);
  check(cur);
  stage_rest(cur, 0);
  Meta nxt = meta_of(za + 1);

  for (int64_t p = za; p < zb; ++p) {
    decode(cur);  // A
    lds_barrier();
    // B: prefetch plane p+1's payload, request plane p+2's metadata
    check(nxt);
    uint32_t pw[PF];
    {
      const uint32_t* src = v.payload + nxt.off;
#pragma unroll
      for (int k = 0; k < PF; ++k) pw[k] = (k < nxt.words) ? src[k] : 0u;
    }
    const Meta nn = meta_of(p + 2);
    // C: stencil on this thread's column
    if (active) {
      const int64_t o = p - 1;
      const bool out_prev = o >= z0 && o < z0 + zs;
#pragma unroll
      for (int i = 0; i < kTy; ++i) {
        if (i < ys) {
          const int r = i + 1;
          const int64_t y = y0 + i;
          const V qc = plane[r * kP + ac];
          N nx = 0, ny = 0;
          if (OP == 5) {
            nx = lap1<N>(plane[r * kP + am], qc, plane[r * kP + ap], x, d.x);
            ny = lap1<N>(plane[(r - 1) * kP + ac], qc, plane[(r + 1) * kP + ac], y, d.y);
          } else if (need_x) {
            const V vm = plane[r * kP + am], vp = plane[r * kP + ap];
            const V lo = xlo ? qc : vm, hi = xhi ? qc : vp;
            if constexpr (INT) nx = xone ? 0 : (hi - lo) * ((xlo || xhi) ? 2 : 1);
            else nx = xone ? T(0) : (xlo || xhi) ? hi - lo : (hi - lo) * T(0.5);
          }
          if (need_y && OP != 5) {
            const bool ylo = y == 0, yhi = y == d.y - 1;
            const V lo = ylo ? qc : plane[(r - 1) * kP + ac];
            const V hi = yhi ? qc : plane[(r + 1) * kP + ac];
            if constexpr (INT) ny = d.y < 2 ? 0 : (hi - lo) * ((ylo || yhi) ? 2 : 1);
            else ny = d.y < 2 ? T(0) : (ylo || yhi) ? hi - lo : (hi - lo) * T(0.5);
          }
          if (out_prev) {
            N nz = 0;
            if constexpr (OP == 5) {
              nz = lap1<N>(qm2[i], qm1[i], qc, o, d.z);
            } else if (need_z) {
              if constexpr (INT) nz = inum(qm2[i], qm1[i], qc, o, d.z);
              else nz = fnum<T>(qm2[i], qm1[i], qc, o, d.z);
            }
            emit(o, i, nz);
          }
          qm2[i] = qm1[i];
          qm1[i] = qc;
          if constexpr (OP == 3) g1[i] = axis == 1 ? ny : nx;
          else if constexpr (OP == 5) g1[i] = nx + ny;
          else g1[i] = sq_xy<INT, T, N>(ny, nx);
        }
      }
    }
    // D: plane p+1's words into this thread's staging column
#pragma unroll
    for (int k = 0; k < PF; ++k)
      if (k < nxt.words) col[k * kFusedThreads] = pw[k];
    stage_rest(nxt, PF);
    cur = nxt;
    nxt = nn;
    lds_barrier();
  }
  // the field's last plane has no plane after it: one-sided (or 0 if nz = 1)
  if (active && z0 + zs == zb) {
    const int64_t o = zb - 1;
#pragma unroll
    for (int i = 0; i < kTy; ++i) {
      if (i < ys) {
        N nz = 0;
        if constexpr (OP == 5) {
          nz = d.z >= 2 ? qm2[i] - qm1[i] : N(0);  // the missing z+1 neighbour is the end value
        } else if (need_z && d.z >= 2) {
          if constexpr (INT) nz = 2 * (qm1[i] - qm2[i]);
          else nz = qm1[i] - qm2[i];
        }
        emit(o, i, nz);
      }
    }
  }
}

// ---- fused, quantized route (D_q) --------------------------------------------------
// The same z-march and pipeline as above, laid out for the integer route:
//  * A row of the LDS plane holds the tile's columns x0-1 .. x0+kTx plus S-1
//    spare columns on each side, so every slot of every block covering the
//    row has a place: the decoder writes whole blocks, with no range tests.
//    Column e of a row sits at e + e/32 (one pad word per 32 columns, so the
//    64 lanes of a wave, each writing slot j of its own block, hit distinct
//    banks).  When rows start on a 32-column boundary (d.x and the box's x0
//    multiples of 32) the pad positions are compile-time offsets.
//  * Domain edges use ghost cells: q_{-1} = 2 q_0 - q_1 (and the mirror at
//    the far end) makes the central numerator q_{+1} - q_{-1} equal the
//    one-sided 2 (q_1 - q_0) exactly in integers, and a length-1 axis gets
//    q itself (numerator 0).  Each thread writes the ghosts of its own
//    column (y, and x at the two edge columns) after the decode barrier, so
//    the stencil has no per-row edge tests; z edges are patched once per
//    tile in registers.
//  * The squared magnitude is summed exactly in integers when max|q| < 8192
//    (|numerator| < 2^15, three squares < 2^32) for binary32 output, and in
//    binary64 for binary64 output (exact while the sum is below 2^53, that is
//    max|q| < 2^23); binary32 output with larger q sums in binary32.
//  * ACC: exact sums of q and q^2 over the tile's own elements for
//    statistics sharing this decode (ACC 1: max|q| < 2^16 and tz <= 2048, so
//    a thread's sum of q fits 32 bits; ACC 2: any q).
template <int S>
struct QRow {
  static constexpr int kOff = S - 1;  // extended column of tile column 0 (x = x0 - 1)
  static constexpr int kExt = kCols + 2 * (S - 1);
  static constexpr int kPitch = conflict_free_pitch(kExt + (kExt >> 5), kNbr<S>, S + S / 32);
  static __host__ __device__ constexpr int at(int e) { return e + (e >> 5); }
  // staging columns start on a 256-byte boundary, so the constant part of
  // every staging address fits the offset field of a strided LDS read
  static constexpr int kStageOff = (kRows * kPitch + 63) / 64 * 64;
};

template <int S, int OP, typename T, int ACC, bool SMALL>
__device__ __forceinline__ void grad_tile_q(const GradJob& job, int64_t tile, uint32_t* smem, int* status) {
  static_assert(!SMALL || (OP == 4 && sizeof(T) == 4), "32-bit squared sums: binary32 magnitude only");
  using R = QRow<S>;
  constexpr int P = R::kPitch;
  const StreamView& v = job.v;
  const uint16_t* __restrict__ rel = job.rel;
  const Dims3 d = job.d;
  const Box3 b = job.b;
  const int axis = job.axis, tz = job.tz, kmax = job.kmax;
  const double halfq = job.halfq;
  T* __restrict__ out = (T*)job.out;
  constexpr int NBR = kNbr<S>;
  constexpr int PF = 16 * (S / 32);  // payload words prefetched per thread
  static_assert(kRows * NBR <= kFusedThreads, "one decode item per thread");
  int* const pl = (int*)smem;
  uint32_t* stage = smem + R::kStageOff;
  const int t = threadIdx.x;

  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int64_t ntx = (bx + kTx - 1) / kTx, nty = (by + kTy - 1) / kTy;
  int64_t blk = tile;
  const int64_t tx = blk % ntx;
  blk /= ntx;
  const int64_t ty = blk % nty;
  const int64_t tzi = blk / nty;
  const int64_t x0 = b.x0 + tx * kTx, y0 = b.y0 + ty * kTy, z0 = b.z0 + tzi * tz;
  const int xs = (int)min((int64_t)kTx, b.x1 - x0), ys = (int)min((int64_t)kTy, b.y1 - y0);
  const int64_t zs = min((int64_t)tz, b.z1 - z0);
  const int64_t cA = max((int64_t)0, x0 - 1), cB = min(d.x, x0 + xs + 1);
  const int64_t rA = max((int64_t)0, y0 - 1), rB = min(d.y, y0 + ys + 1);
  const int64_t za = max((int64_t)0, z0 - 1), zb = min(d.z, z0 + zs + 1);
  const int nrows = (int)(rB - rA);
  const T h = (T)halfq;
  const double quantum = v.quantum;
  const bool need_z = OP >= 4 || axis == 0, need_y = OP >= 4 || axis == 1, need_x = OP >= 4 || axis == 2;
  const bool aligned = (d.x & 31) == 0 && (x0 & 31) == 0;

  // decode item of this thread: decoded row dr, dk-th block of the row
  const int dr = t / NBR, dk = t % NBR;
  const int64_t dy = rA + dr;
  const bool decoder = dr < nrows;
  int* const prow = pl + (int)(dy - (y0 - 1)) * P;
  uint32_t* col = stage + t;

  struct Meta {
    int w, q0, words, e0;
    uint64_t off;
    bool valid;
  };
  auto meta_of = [&](int64_t p) {
    Meta m{0, 0, 0, 0, 0, false};
    if (decoder && p < zb) {
      const int64_t f = (p * d.y + dy) * d.x;
      const int64_t bA = (f + cA) / S, bB = (f + cB - 1) / S, bk = bA + dk;
      if (bk <= bB) {
        m.valid = true;
        m.w = (int)v.width[bk];
        m.q0 = v.q0[bk];
        m.off = v.chunk_off[bk / kChunkBlocks] + rel[bk];
        m.e0 = (int)(bk * S - f);
      }
    }
    return m;
  };
  auto check = [&](Meta& m) {
    if (!m.valid) return;
    m.words = block_words<S>(m.w);
    if (m.w > kMaxWidth || m.words > kmax || m.off + (uint64_t)m.words > v.payload_words) {
      record_status(status, kErrBadStream);
      m.w = 0;
      m.words = 0;
    }
  };
  auto stage_rest = [&](const Meta& m, int from) {
    const uint32_t* src = v.payload + m.off;
    for (int k = from; k < m.words; ++k) col[k * kFusedThreads] = src[k];
  };
  auto decode = [&](const Meta& m) {
    if (!m.valid) return;
    const int cb = m.e0 - (int)(x0 - 1) + R::kOff;  // extended column of slot 0 (>= 0)
    int* dst = prow + R::at(cb);
    if (aligned) decode_block_q<S, true, kFusedThreads>(col, m.w, m.q0, dst, 32);
    else decode_block_q<S, false, kFusedThreads>(col, m.w, m.q0, dst, 32 - (cb & 31));
  };

  // stencil column of this thread and its neighbours (row-relative offsets)
  const int ec = R::at(t + 1 + R::kOff), em = R::at(t + R::kOff), ep = R::at(t + 2 + R::kOff);
  const int64_t x = x0 + t;
  const bool active = t < xs;
  const bool ylo = y0 == 0, yhi = y0 + ys == d.y, xlo = x == 0, xhi = x == d.x - 1;
  const bool y2 = d.y >= 2, x2 = d.x >= 2;

  // per row: q of the two previous planes; in-plane part of the previous
  // plane (squared sum, the one numerator of a single derivative, or the
  // in-plane second differences of the Laplacian)
  using G = typename std::conditional<OP == 3 || OP == 5, int,
                                      typename std::conditional<SMALL, uint32_t, T>::type>::type;
  int qm2[kTy], qm1[kTy];
  G g1[kTy];
#pragma unroll
  for (int i = 0; i < kTy; ++i) { qm2[i] = 0; qm1[i] = 0; g1[i] = G(0); }
  using S1 = typename std::conditional<ACC == 1, int, int64_t>::type;
  S1 as1 = 0;
  uint64_t as2s = 0;
  U128 as2 = {0, 0};

  // one output value from the numerators (in-plane part already squared)
  auto value = [&](int i, int nz) -> T {
    if constexpr (OP == 3) {
      const int n = axis == 0 ? nz : (int)g1[i];
      return (T)n * h;
    } else if constexpr (SMALL) {
      const uint32_t s2 = g1[i] + (uint32_t)__mul24(nz, nz);
      return vsqrt((float)s2) * h;
    } else {
      const T dz = (T)nz;
      return vsqrt(g1[i] + dz * dz) * h;
    }
  };
  auto accumulate = [&](int q) {
    if constexpr (ACC == 1) {
      as1 += q;
      as2s += (uint32_t)__mul24(q, q);
    } else if constexpr (ACC == 2) {
      as1 += q;
      add_u64(as2, (uint64_t)((int64_t)q * (int64_t)q));
    }
  };

  // stencil over the rows of plane p (in LDS); emits plane o = p - 1
  auto rows = [&](int64_t p) {
    const int64_t o = p - 1;
    const bool emit = o >= z0 && o < z0 + zs;
    // ghosts of this thread's column: 2 q_0 - q_1 for differences (the
    // one-sided numerator), q_0 itself for the Laplacian (mirrored end)
    constexpr bool kMirror = OP == 5;
    if (ylo) pl[ec] = (y2 && !kMirror) ? 2 * pl[P + ec] - pl[2 * P + ec] : pl[P + ec];
    if (yhi) {
      int* r = pl + ys * P + ec;
      r[P] = (y2 && !kMirror) ? 2 * r[0] - r[-P] : r[0];
    }
    if (need_x && (xlo || xhi)) {
#pragma unroll
      for (int i = 0; i < kTy; ++i) {
        int* r = pl + (i + 1) * P;
        if (xlo) r[em] = (x2 && !kMirror) ? 2 * r[ec] - r[ep] : r[ec];
        if (xhi) r[ep] = (x2 && !kMirror) ? 2 * r[ec] - r[em] : r[ec];
      }
    }
    // the field's first plane: ghost plane q_{-1} = 2 q_0 - q_1 (or q_0)
    if (o == 0 && need_z) {
#pragma unroll
      for (int i = 0; i < kTy; ++i) {
        const int c1 = pl[(i + 1) * P + ec];
        qm2[i] = (d.z >= 2 && !kMirror) ? 2 * qm1[i] - c1 : qm1[i];
      }
    }
    // rows to store this plane (kTy, ys, or none): it depends on the plane,
    // so the compiler keeps no per-row masks across the march
    const int nr = emit ? ys : 0;
    T* orow = out + ((o - b.z0) * by + (y0 - b.y0)) * bx + (x0 - b.x0);
#pragma unroll
    for (int hh = 0; hh < kTy; hh += kTy / 4) {
      constexpr int H = kTy / 4;
      int cv[H + 2], xm[H], xp[H];
#pragma unroll
      for (int k = 0; k < H + 2; ++k) cv[k] = pl[(hh + k) * P + ec];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        xm[k] = need_x ? pl[(hh + k + 1) * P + em] : 0;
        xp[k] = need_x ? pl[(hh + k + 1) * P + ep] : 0;
      }
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int i = hh + k;
        const int qc = cv[k + 1];
        if (i < nr) {
          T* rowp = orow + (int64_t)i * bx;
          if constexpr (OP == 5) {
            rowp[(uint32_t)t] = lap_value<T>(g1[i] + (qc + qm2[i]) - (qm1[i] + qm1[i]), quantum);
          } else {
            const int nz = need_z ? qc - qm2[i] : 0;
            rowp[(uint32_t)t] = value(i, nz);
          }
          accumulate(qm1[i]);
        }
        const int nx = xp[k] - xm[k], ny = need_y ? cv[k + 2] - cv[k] : 0;
        qm2[i] = qm1[i];
        qm1[i] = qc;
        if constexpr (OP == 3) g1[i] = axis == 1 ? ny : nx;
        else if constexpr (OP == 5) g1[i] = ((xp[k] + xm[k]) - (qc + qc)) + ((cv[k + 2] + cv[k]) - (qc + qc));
        else if constexpr (SMALL) g1[i] = (uint32_t)__mul24(nx, nx) + (uint32_t)__mul24(ny, ny);
        else g1[i] = (T)nx * (T)nx + (T)ny * (T)ny;
      }
    }
  };

  // prologue: plane za staged, metadata of za+1 in flight
  Meta cur = meta_of(za);
  check(cur);
  stage_rest(cur, 0);
  Meta nxt = meta_of(za + 1);

  for (int64_t p = za; p < zb; ++p) {
    decode(cur);  // A
    lds_barrier();
    // B: prefetch plane p+1's payload, request plane p+2's metadata
    check(nxt);
    uint32_t pw[PF];
    prefetch_words<PF>(v.payload, v.payload_words, nxt.off, nxt.words, pw);
    const Meta nn = meta_of(p + 2);
    if (active) rows(p);  // C
    // D: plane p+1's words into this thread's staging column
#pragma unroll
    for (int k = 0; k < PF; ++k)
      if (k < nxt.words) col[k * kFusedThreads] = pw[k];
    stage_rest(nxt, PF);
    cur = nxt;
    nxt = nn;
    lds_barrier();
  }
  // the field's last plane has no plane after it: one-sided (or 0 if nz = 1)
  if (active && z0 + zs == zb) {
    const int64_t o = zb - 1;
    T* orow = out + ((o - b.z0) * by + (y0 - b.y0)) * bx + (x0 - b.x0);
#pragma unroll
    for (int i = 0; i < kTy; ++i) {
      if (i < ys) {
        T* rowp = orow + (int64_t)i * bx;
        if constexpr (OP == 5) {
          // the missing z+1 neighbour is the end value qm1 itself; a field of
          // one plane has no z term (qm2 never held a plane there)
          rowp[(uint32_t)t] = lap_value<T>(g1[i] + (d.z >= 2 ? qm2[i] - qm1[i] : 0), quantum);
        } else {
          const int nz = (need_z && d.z >= 2) ? 2 * (qm1[i] - qm2[i]) : 0;
          rowp[(uint32_t)t] = value(i, nz);
        }
        accumulate(qm1[i]);
      }
    }
  }
  if constexpr (ACC != 0) {
    const int64_t cnt = active ? (int64_t)ys * zs : 0;
    if constexpr (ACC == 1) as2.lo = as2s;
    acc_add_wave((BatchAcc*)job.acc, (int64_t)as1, cnt, as2);
  }
}

// One tile of a job: the quantized route by the integer tile (32-bit squared
// sums when the stream's max|q| allows), the float route by the float tile.
template <int S, int VIA, int OP, typename T, int ACC>
__device__ __forceinline__ void any_tile(const GradJob& job, int64_t tile, uint32_t* smem, int* status) {
  if constexpr (VIA == 3) {
    if constexpr (OP == 4 && sizeof(T) == 4) {
      if (job.v.max_abs_q < 8192u) {
        grad_tile_q<S, OP, T, ACC, true>(job, tile, smem, status);
        return;
      }
    }
    grad_tile_q<S, OP, T, ACC, false>(job, tile, smem, status);
  } else {
    static_assert(ACC == 0, "shared statistics need the quantized route");
    grad_tile<S, VIA, OP, T>(job, tile, smem, status);
  }
}

// Four waves per SIMD (128 registers) for the binary32 quantized route with
// S = 32; the others (binary64 squared sums, twice the prefetch for S = 64)
// take the registers they need.
template <int S, int VIA, typename T>
constexpr int kGradWaves = (S == 32 && VIA == 3 && sizeof(T) == 4) ? 4 : 1;

template <int S, int VIA, int OP, typename T>
__global__ void __launch_bounds__(kFusedThreads, (kGradWaves<S, VIA, T>)) k_grad_fused(GradJob job, int* status) {
  extern __shared__ uint32_t smem[];
  any_tile<S, VIA, OP, T, 0>(job, blockIdx.x, smem, status);
}

// Persistent batch: the tiles of every job of one kernel variant, listed in
// a device table (count and tile offsets read from device memory, so a
// captured graph can be replayed with a new table).  ACC is the variant's
// shared-statistics mode (one instantiation each, so a variant without
// statistics keeps the plain kernel's registers and code size).
template <int S, int VIA, int OP, typename T, int ACC>
__global__ void __launch_bounds__(kFusedThreads, (kGradWaves<S, VIA, T>)) k_batch_grad(const GradJob* __restrict__ jobs,
                                                              const int64_t* __restrict__ tile_start,
                                                              const int64_t* __restrict__ counts, int* status) {
  extern __shared__ uint32_t smem[];
  const int n = (int)counts[0];
  const int64_t total = counts[1];
  for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
    int lo = 0, hi = n - 1;  // last job whose first tile is <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (tile_start[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    const GradJob job = load_job(jobs, lo);
    any_tile<S, VIA, OP, T, ACC>(job, tile - tile_start[lo], smem, status);
  }
}

// ---- stage 2 (D_p): derivative along the fast axis, no recorrelation -----------
// Inside a block the central difference is q_{j+1} - q_{j-1} = p_j + p_{j+1}
// (p_j = q_j - q_{j-1}).  At a block edge the missing neighbour comes from
// the metadata: the next block's q0, or the previous block's last value
// q0 + (sum of its deltas).  One lane per (box row, block) segment; the
// previous block's last value is taken from the neighbouring lane when that
// lane holds it, else summed from its deltas.
template <int S, bool FROM_STREAM, typename T>
__global__ void __launch_bounds__(256) k_deriv_fast_delta(const int32_t* __restrict__ pbuf,
                                                          const int32_t* __restrict__ q0buf, StreamView v,
                                                          Segs<S> segs, Dims3 d, Box3 b, int kmax, double halfq,
                                                          T* __restrict__ out, int* status) {
  extern __shared__ uint32_t smem[];
  const int t = threadIdx.x;
  const int64_t items = segs.count();
  const T h = (T)halfq;
  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int32_t* q0s = FROM_STREAM ? v.q0 : q0buf;
  uint32_t* col = smem + t;
  // p of block k, the block's first q, and its last q = q0 + sum of deltas
  auto load_block = [&](int64_t k, int (&pv)[S], int& q0) {
    if constexpr (FROM_STREAM) {
      const int w = stage_block<S, 256>(v.width, v.q0, v.chunk_off, v.payload, v.payload_words, v.nb, k, col,
                                        kmax, q0, status);
      decode_lane_block<S, 256>(col, w, q0, [&](int j, int p, int) { pv[j] = p; });
    } else {
      q0 = q0buf[k];
#pragma unroll
      for (int j = 0; j < S; ++j) pv[j] = (k * S + j < v.n) ? pbuf[k * S + j] : 0;
    }
    int sum = 0;
#pragma unroll
    for (int j = 1; j < S; ++j) sum += pv[j];
    return q0 + sum;
  };
  for (int64_t base = (int64_t)blockIdx.x * 256; base < items; base += (int64_t)gridDim.x * 256) {
    const int64_t it = base + t;
    int64_t blk = -1;
    int a = 0, z = -1;
    const bool ok = it < items && segs.get(it, blk, a, z);
    int pv[S];
    int q0 = 0, qlast = 0;
    if (ok) qlast = load_block(blk, pv, q0);
    const int64_t prev_blk = __shfl_up(blk, 1);
    const int prev_last = __shfl_up(qlast, 1);
    const int prev_ok = __shfl_up((int)ok, 1);
    if (!ok) continue;
    const int64_t r = it / segs.per_row;
    const int64_t f = segs.rows.start(r);  // flat index of the box row's first element
    const int64_t e0 = blk * S;
    const int64_t x_of0 = b.x0 + (e0 - f);  // x of slot 0 (may lie left of the box)
    int qprev = 0;
    if (a == 0 && x_of0 > 0) {
      if (lane_id() > 0 && prev_ok && prev_blk == blk - 1) {
        qprev = prev_last;
      } else {
        int pp[S];
        int q0p;
        qprev = load_block(blk - 1, pp, q0p);  // pv stays in registers
      }
    }
    const int q0next = (z == S - 1 && x_of0 + S - 1 < d.x - 1) ? q0s[blk + 1] : 0;
    const int64_t iz = r / segs.rows.nry, iy = r % segs.rows.nry;
    const int64_t orow = (iz * by + iy) * bx - b.x0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      if (j >= a && j <= z) {
        const int64_t x = x_of0 + j;
        int nn;
        if (d.x < 2) nn = 0;
        else if (x == 0) nn = 2 * (j + 1 <= S - 1 ? pv[j + 1 < S ? j + 1 : S - 1] : q0next - qlast);
        else if (x == d.x - 1) nn = 2 * (j >= 1 ? pv[j] : q0 - qprev);
        else if (j == 0) nn = q0 + pv[1] - qprev;
        else if (j == S - 1) nn = q0next - (qlast - pv[S - 1]);
        else nn = pv[j] + pv[j + 1 < S ? j + 1 : S - 1];
        out[orow + x] = (T)nn * h;
      }
    }
  }
}

int kmax_for(const StreamView& v) {
  int wmax = 32 - __builtin_clz(2u * v.max_abs_q | 1u);
  wmax = wmax < 1 ? 1 : (wmax > kMaxWidth ? kMaxWidth : wmax);
  return (v.block / 32) * (1 + wmax);
}

template <int SRC, typename T>
hipError_t run_buf(const void* buf, int op, int axis, const OpTarget& t, double halfq, void* out, hipStream_t s) {
  const Box3& b = t.box;
  const int64_t ntx = (b.x1 - b.x0 + kBx - 1) / kBx, nty = (b.y1 - b.y0 + kBy - 1) / kBy;
  const int64_t bz = b.z1 - b.z0;
  // enough workgroups to fill the chip, long enough z runs to reuse the column registers
  int64_t tz = bz;
  while (tz > 16 && ntx * nty * ((bz + tz - 1) / tz) < 16384) tz = (tz + 1) / 2;
  const int64_t grid = ntx * nty * ((bz + tz - 1) / tz);
  if (op == 3)
    hipLaunchKernelGGL((k_grad_buf<SRC, 3, T>), dim3((unsigned)grid), dim3(kBufThreads), 0, s, buf, t.d, b, axis,
                       (int)tz, halfq, (T*)out);
  else if (op == 5)
    hipLaunchKernelGGL((k_grad_buf<SRC, 5, T>), dim3((unsigned)grid), dim3(kBufThreads), 0, s, buf, t.d, b, axis,
                       (int)tz, halfq, (T*)out);
  else
    hipLaunchKernelGGL((k_grad_buf<SRC, 4, T>), dim3((unsigned)grid), dim3(kBufThreads), 0, s, buf, t.d, b, axis,
                       (int)tz, halfq, (T*)out);
  return hipGetLastError();
}

size_t grad_lds_bytes(int S, int dtype, int via, int kmax);

template <int S, int VIA, typename T>
hipError_t run_fused(const StreamView& v, int op, int axis, const OpTarget& t, void* out, uint8_t* ws,
                     hipStream_t s) {
  int* status = (int*)ws;
  uint16_t* rel = (uint16_t*)(ws + kGradIndexOff);
  hipError_t e = launch_block_index(v, rel, s);
  if (e != hipSuccess) return e;
  const Box3& b = t.box;
  const int kmax = kmax_for(v);
  const size_t lds = grad_lds_bytes(S, v.dtype, VIA, kmax);
  const int64_t ntx = (b.x1 - b.x0 + kTx - 1) / kTx, nty = (b.y1 - b.y0 + kTy - 1) / kTy;
  const int64_t bz = b.z1 - b.z0;
  int64_t tz = bz;
  while (tz > 8 && ntx * nty * ((bz + tz - 1) / tz) < 1024) tz = (tz + 1) / 2;
  const int64_t grid = ntx * nty * ((bz + tz - 1) / tz);
  GradJob job{v, rel, t.d, b, axis, (int)tz, kmax, 0.5 * v.quantum, out};
  if (op == 3)
    hipLaunchKernelGGL((k_grad_fused<S, VIA, 3, T>), dim3((unsigned)grid), dim3(kFusedThreads), lds, s, job, status);
  else if (op == 5)
    hipLaunchKernelGGL((k_grad_fused<S, VIA, 5, T>), dim3((unsigned)grid), dim3(kFusedThreads), lds, s, job, status);
  else
    hipLaunchKernelGGL((k_grad_fused<S, VIA, 4, T>), dim3((unsigned)grid), dim3(kFusedThreads), lds, s, job, status);
  return hipGetLastError();
}

template <int S>
hipError_t fused_by_via(const StreamView& v, int via, int op, int axis, const OpTarget& t, void* out, uint8_t* ws,
                        hipStream_t s) {
  if (via == 3)
    return v.dtype == 1 ? run_fused<S, 3, float>(v, op, axis, t, out, ws, s)
                        : run_fused<S, 3, double>(v, op, axis, t, out, ws, s);
  if (via == 4)
    return v.dtype == 1 ? run_fused<S, 4, float>(v, op, axis, t, out, ws, s)
                        : run_fused<S, 4, double>(v, op, axis, t, out, ws, s);
  return hipErrorNotSupported;
}

template <int S, bool FROM_STREAM, typename T>
hipError_t run_fast_delta(const int32_t* p, const StreamView& v, const OpTarget& t, void* out, int* status,
                          hipStream_t s) {
  const Box3& b = t.box;
  Rows rows;
  rows.nrz = b.z1 - b.z0;
  rows.nry = b.y1 - b.y0;
  rows.len = b.x1 - b.x0;
  rows.base = (b.z0 * t.d.y + b.y0) * t.d.x + b.x0;
  rows.sz = t.d.x * t.d.y;
  rows.sy = t.d.x;
  const Segs<S> segs = make_segs<S>(rows);
  const int kmax = kmax_for(v);
  const size_t lds = FROM_STREAM ? (size_t)(kmax + 1) * 256 * sizeof(uint32_t) : 0;
  const int64_t g = (segs.count() + 255) / 256;
  const unsigned grid = (unsigned)(g < 8192 ? g : 8192);
  hipLaunchKernelGGL((k_deriv_fast_delta<S, FROM_STREAM, T>), dim3(grid), dim3(256), lds, s, p,
                     p ? p + v.n : nullptr, v, segs, t.d, b, kmax, 0.5 * v.quantum, (T*)out, status);
  return hipGetLastError();
}

template <bool FROM_STREAM>
hipError_t fast_delta(const int32_t* p, const StreamView& v, const OpTarget& t, void* out, int* status,
                      hipStream_t s) {
  if (v.block == 32)
    return v.dtype == 1 ? run_fast_delta<32, FROM_STREAM, float>(p, v, t, out, status, s)
                        : run_fast_delta<32, FROM_STREAM, double>(p, v, t, out, status, s);
  return v.dtype == 1 ? run_fast_delta<64, FROM_STREAM, float>(p, v, t, out, status, s)
                      : run_fast_delta<64, FROM_STREAM, double>(p, v, t, out, status, s);
}

// LDS of one gradient tile: the plane (integer rows of QRow for the quantized
// route, padded rows of T for the float route) and the staging columns.
size_t grad_lds_bytes(int S, int dtype, int via, int kmax) {
  const size_t stage = (size_t)(kmax + 1) * kFusedThreads * sizeof(uint32_t);
  if (via == 3) return (size_t)(S == 32 ? QRow<32>::kStageOff : QRow<64>::kStageOff) * sizeof(int) + stage;
  const size_t vsz = dtype == 2 ? 8 : 4;
  return ((kRows * (S == 32 ? kPitch<32> : kPitch<64>) * vsz + 3) / 4) * 4 + stage;
}

template <int S, int VIA, int OP, typename T, int ACC>
hipError_t batch_grad_v(const GradJob* jobs, const int64_t* tile_start, const int64_t* counts, int kmax, int grid,
                        int* status, hipStream_t s) {
  const size_t lds = grad_lds_bytes(S, sizeof(T) == 4 ? 1 : 2, VIA, kmax);
  hipLaunchKernelGGL((k_batch_grad<S, VIA, OP, T, ACC>), dim3(grid), dim3(kFusedThreads), lds, s, jobs, tile_start,
                     counts, status);
  return hipGetLastError();
}

template <int S, int VIA, int OP, int ACC>
hipError_t batch_grad_t(int dtype, const GradJob* jobs, const int64_t* tile_start, const int64_t* counts, int kmax,
                        int grid, int* status, hipStream_t s) {
  return dtype == 1 ? batch_grad_v<S, VIA, OP, float, ACC>(jobs, tile_start, counts, kmax, grid, status, s)
                    : batch_grad_v<S, VIA, OP, double, ACC>(jobs, tile_start, counts, kmax, grid, status, s);
}

template <int S, int OP>
hipError_t batch_grad_acc(int acc, int dtype, const GradJob* jobs, const int64_t* tile_start, const int64_t* counts,
                          int kmax, int grid, int* status, hipStream_t s) {
  return acc == 1   ? batch_grad_t<S, 3, OP, 1>(dtype, jobs, tile_start, counts, kmax, grid, status, s)
         : acc == 2 ? batch_grad_t<S, 3, OP, 2>(dtype, jobs, tile_start, counts, kmax, grid, status, s)
                    : batch_grad_t<S, 3, OP, 0>(dtype, jobs, tile_start, counts, kmax, grid, status, s);
}

template <int S>
hipError_t batch_grad_s(int via, int op, int dtype, int acc, const GradJob* jobs, const int64_t* tile_start,
                        const int64_t* counts, int kmax, int grid, int* status, hipStream_t s) {
  if (via == 3)
    return op == 3 ? batch_grad_acc<S, 3>(acc, dtype, jobs, tile_start, counts, kmax, grid, status, s)
                   : batch_grad_acc<S, 4>(acc, dtype, jobs, tile_start, counts, kmax, grid, status, s);
  if (acc) return hipErrorInvalidValue;
  return op == 3 ? batch_grad_t<S, 4, 3, 0>(dtype, jobs, tile_start, counts, kmax, grid, status, s)
                 : batch_grad_t<S, 4, 4, 0>(dtype, jobs, tile_start, counts, kmax, grid, status, s);
}

}  // namespace

uint64_t grad_workspace_bytes(int64_t nb) { return kGradIndexOff + ((2 * (uint64_t)nb + 255) / 256) * 256; }

size_t batch_grad_lds(int S, int dtype, int via, int kmax) { return grad_lds_bytes(S, dtype, via, kmax); }

hipError_t launch_batch_grad(int S, int via, int op, int dtype, int acc, const GradJob* jobs,
                             const int64_t* tile_start, const int64_t* counts, int kmax, int grid, int* status,
                             hipStream_t s) {
  return S == 32 ? batch_grad_s<32>(via, op, dtype, acc, jobs, tile_start, counts, kmax, grid, status, s)
                 : batch_grad_s<64>(via, op, dtype, acc, jobs, tile_start, counts, kmax, grid, status, s);
}

int grad_tiles(const Box3& b, int tz) {
  const int64_t ntx = (b.x1 - b.x0 + kTx - 1) / kTx, nty = (b.y1 - b.y0 + kTy - 1) / kTy;
  return (int)(ntx * nty * ((b.z1 - b.z0 + tz - 1) / tz));
}

int grad_kmax(const StreamView& v) { return kmax_for(v); }

hipError_t launch_grad_stage(const void* buf, int stage, const StreamView& v, int op, int axis3, const OpTarget& t,
                             void* result, uint8_t* ws, hipStream_t s) {
  const double halfq = 0.5 * v.quantum;
  if (stage == 2) {
    if (op != 3 || axis3 != 2) return hipErrorNotSupported;
    return fast_delta<false>((const int32_t*)buf, v, t, result, (int*)ws, s);
  }
  if (stage == 3)
    return v.dtype == 1 ? run_buf<3, float>(buf, op, axis3, t, halfq, result, s)
                        : run_buf<3, double>(buf, op, axis3, t, halfq, result, s);
  if (stage == 4)
    return v.dtype == 1 ? run_buf<4, float>(buf, op, axis3, t, halfq, result, s)
                        : run_buf<4, double>(buf, op, axis3, t, halfq, result, s);
  return hipErrorInvalidValue;
}

hipError_t launch_grad_fused(const StreamView& v, int via, int op, int axis3, const OpTarget& t, void* result,
                             uint8_t* ws, hipStream_t s) {
  int* status = (int*)ws;
  if (via == 2) {
    if (op != 3 || axis3 != 2) return hipErrorNotSupported;
    return fast_delta<true>(nullptr, v, t, result, status, s);
  }
  if (q4_eligible(v, via, op, t.d, t.box)) {
    uint16_t* rel = (uint16_t*)(ws + kGradIndexOff);
    hipError_t e = launch_block_index(v, rel, s);
    if (e != hipSuccess) return e;
    const int tz = q4_tz(t.box);
    GradJob job{v, rel, t.d, t.box, 0, tz, kmax_for(v), 0.5 * v.quantum, result};
    return launch_gradmag_q4(job, status, s);
  }
  return v.block == 32 ? fused_by_via<32>(v, via, op, axis3, t, result, ws, s)
                       : fused_by_via<64>(v, via, op, axis3, t, result, ws, s);
}

}  // namespace hsz
