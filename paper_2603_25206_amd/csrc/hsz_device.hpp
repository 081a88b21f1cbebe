// hsz_device.hpp -- device-side building blocks shared by the HIP kernels:
// the byte-format constants, wave64 primitives (DPP scans, reductions), the
// status word, and the block decoder used by every stage and operation.
//
// Work layout used throughout: one wavefront owns a chunk of 64 consecutive
// blocks and each lane owns ONE block (lane l <-> block 64*c + l).  A lane
// walks the S slots of its block serially, so recorrelation (the prefix sum
// q_i = q_{i-1} + p_i of Alg. 2) is a single add per element, and all
// per-block metadata (width, q0, payload offset) lives in the lane's own
// registers.  The chunk's payload words are staged in LDS transposed,
// word k of lane l at tile[k*64 + l], so that when every lane reads "its"
// word k (k differs per lane) the 64 addresses fall in 64 distinct banks.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#include "hsz_launch.hpp"

namespace hsz {

constexpr int kHeaderBytes = 256;
constexpr int kSectionAlign = 256;
constexpr int kChunkBlocks = 64;
constexpr int kMaxWidth = 30;  // |p| < 2^30 because |q| <= 2^29 - 1
constexpr int32_t kQMax = 536870911;
constexpr int kWave = 64;

// Status codes recorded by kernels (same values as the C ABI).
constexpr int kErrBadStream = -2;
constexpr int kErrRange = -4;
constexpr int kErrEb = -5;
constexpr int kErrNonFinite = -6;
constexpr int kErrCapacity = -7;

// First error wins; later ones are dropped.  A vector atomic on global
// memory (never a scalar-cache store).
__device__ __forceinline__ void record_status(int* status, int code) {
  if (status) atomicCAS(status, 0, code);
}

// Payload words of a block of S slots with bit width w: S/32 sign words and
// S*w/32 magnitude words, nothing when w = 0.
template <int S>
__device__ __forceinline__ int block_words(int w) {
  return w ? (S / 32) * (1 + w) : 0;
}

// ---- wave64 primitives -------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// DPP controls (GFX9 encoding): row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.  Lanes whose source is outside the row read 'old' = 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes of the wave.
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += dpp<0x111>(x);
  x += dpp<0x112>(x);
  x += dpp<0x114>(x);
  x += dpp<0x118>(x);
  x += dpp<0x142, 0xa>(x);  // lane 15 -> row 1, lane 47 -> row 3
  x += dpp<0x143, 0xc>(x);  // lane 31 -> rows 2 and 3
  return x;
}

__device__ __forceinline__ int wave_max(int x) {
  for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m));
  return x;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

__device__ __forceinline__ double wave_sum_f64(double x) {
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

// ---- row sets and block segments (boxes) -------------------------------------
inline Rows make_rows(const Dims3& d, const Box3& b) {
  Rows r;
  const int64_t plane = d.y * d.x;
  if (b.x0 == 0 && b.x1 == d.x && b.y0 == 0 && b.y1 == d.y) {
    r.nrz = 1; r.nry = 1; r.len = (b.z1 - b.z0) * plane; r.base = b.z0 * plane; r.sz = 0; r.sy = 0;
  } else if (b.x0 == 0 && b.x1 == d.x) {
    r.nrz = b.z1 - b.z0; r.nry = 1; r.len = (b.y1 - b.y0) * d.x; r.base = b.z0 * plane + b.y0 * d.x;
    r.sz = plane; r.sy = 0;
  } else {
    r.nrz = b.z1 - b.z0; r.nry = b.y1 - b.y0; r.len = b.x1 - b.x0;
    r.base = b.z0 * plane + b.y0 * d.x + b.x0; r.sz = plane; r.sy = d.x;
  }
  return r;
}

// ---- block segments: the part of one block that lies inside one row -------------
// Items are (row, k-th block touched by the row).  For a row [f, f+len) the
// blocks are f/S .. (f+len-1)/S; inside block b the row covers slots a..z.
template <int S>
struct Segs {
  Rows rows;
  int64_t per_row;  // upper bound of blocks touched by one row
  __host__ __device__ int64_t count() const { return rows.count() * per_row; }
  // returns false if item k lies past the row's last block
  __device__ bool get(int64_t item, int64_t& b, int& a, int& z) const {
    const int64_t r = item / per_row, k = item % per_row;
    const int64_t f = rows.start(r), e = f + rows.len;  // [f, e)
    b = f / S + k;
    if (b > (e - 1) / S) return false;
    const int64_t bs = b * S;
    a = (int)(f > bs ? f - bs : 0);
    z = (int)((e < bs + S ? e : bs + S) - 1 - bs);
    return true;
  }
};
template <int S>
inline Segs<S> make_segs(const Rows& r) {
  Segs<S> s;
  s.rows = r;
  s.per_row = (r.len + S - 2) / S + 1;
  return s;
}

// ---- 128-bit unsigned accumulator (sum of q^2 can pass 2^64) ----------------
struct U128 {
  uint64_t lo, hi;
};
__device__ __forceinline__ void add_u64(U128& a, uint64_t v) {
  uint64_t t = a.lo + v;
  a.hi += (t < v);
  a.lo = t;
}
__device__ __forceinline__ void add_u128(U128& a, U128 b) {
  uint64_t t = a.lo + b.lo;
  a.hi += b.hi + (t < b.lo);
  a.lo = t;
}

// ---- job tables in device memory ------------------------------------------------
// A pointer loaded from a device-side job table has an unknown address space
// to the compiler, which then emits flat loads and stores.  Flat accesses
// count against the LDS wait counter too, so every LDS wait also waits for
// outstanding memory traffic and prefetching stops overlapping.  The mirror
// structs below have the same layout as the host-built ones with the
// pointers typed as global; a kernel reads its table entry through them and
// converts, and every access derived from that entry is emitted as global.
#define HSZ_GLOBAL __attribute__((address_space(1)))

struct StreamViewG {
  const HSZ_GLOBAL uint8_t* base;
  const HSZ_GLOBAL uint64_t* chunk_off;
  const HSZ_GLOBAL int32_t* q0;
  const HSZ_GLOBAL uint8_t* width;
  const HSZ_GLOBAL uint32_t* payload;
  uint64_t payload_words;
  int64_t n, nb, nchunks;
  int block;
  int dtype;
  double quantum;
  uint32_t max_abs_q;
  uint32_t flags;
};
static_assert(sizeof(StreamViewG) == sizeof(StreamView), "mirror layout");
static_assert(offsetof(StreamViewG, flags) == offsetof(StreamView, flags), "mirror layout");
static_assert(offsetof(StreamViewG, payload_words) == offsetof(StreamView, payload_words), "mirror layout");
static_assert(offsetof(StreamViewG, max_abs_q) == offsetof(StreamView, max_abs_q), "mirror layout");

struct GradJobG {
  StreamViewG v;
  const HSZ_GLOBAL uint16_t* rel;
  Dims3 d;
  Box3 b;
  int axis, tz, kmax;
  double halfq;
  HSZ_GLOBAL void* out;
  HSZ_GLOBAL void* acc;
  int acc_mode;
};
static_assert(sizeof(GradJobG) == sizeof(GradJob), "mirror layout");
static_assert(offsetof(GradJobG, acc_mode) == offsetof(GradJob, acc_mode), "mirror layout");
static_assert(offsetof(GradJobG, rel) == offsetof(GradJob, rel), "mirror layout");
static_assert(offsetof(GradJobG, halfq) == offsetof(GradJob, halfq), "mirror layout");
static_assert(offsetof(GradJobG, out) == offsetof(GradJob, out), "mirror layout");

struct StatsJobG {
  StreamViewG v;
  Rows rows;
  int64_t per_row;
  int32_t op, via, whole, acc;
  HSZ_GLOBAL void* out;
  const HSZ_GLOBAL uint16_t* rel;
};
static_assert(sizeof(StatsJobG) == sizeof(StatsJob), "mirror layout");
static_assert(offsetof(StatsJobG, per_row) == offsetof(StatsJob, per_row), "mirror layout");
static_assert(offsetof(StatsJobG, out) == offsetof(StatsJob, out), "mirror layout");
static_assert(offsetof(StatsJobG, rel) == offsetof(StatsJob, rel), "mirror layout");

__device__ __forceinline__ StreamView view_of(const StreamViewG& g) {
  StreamView v;
  v.base = (const uint8_t*)g.base;
  v.chunk_off = (const uint64_t*)g.chunk_off;
  v.q0 = (const int32_t*)g.q0;
  v.width = (const uint8_t*)g.width;
  v.payload = (const uint32_t*)g.payload;
  v.payload_words = g.payload_words;
  v.n = g.n;
  v.nb = g.nb;
  v.nchunks = g.nchunks;
  v.block = g.block;
  v.dtype = g.dtype;
  v.quantum = g.quantum;
  v.max_abs_q = g.max_abs_q;
  v.flags = g.flags;
  return v;
}

// Table entry k, read as uniform (scalar) loads with global pointers.
__device__ __forceinline__ GradJob load_job(const GradJob* jobs, int k) {
  const GradJobG g = ((const GradJobG*)jobs)[k];
  GradJob j;
  j.v = view_of(g.v);
  j.rel = (const uint16_t*)g.rel;
  j.d = g.d;
  j.b = g.b;
  j.axis = g.axis;
  j.tz = g.tz;
  j.kmax = g.kmax;
  j.halfq = g.halfq;
  j.out = (void*)g.out;
  j.acc = (void*)g.acc;
  j.acc_mode = g.acc_mode;
  return j;
}

__device__ __forceinline__ StatsJob load_job(const StatsJob* jobs, int k) {
  const StatsJobG g = ((const StatsJobG*)jobs)[k];
  StatsJob j;
  j.v = view_of(g.v);
  j.rows = g.rows;
  j.per_row = g.per_row;
  j.op = g.op;
  j.via = g.via;
  j.whole = g.whole;
  j.acc = g.acc;
  j.out = (void*)g.out;
  j.rel = (const uint16_t*)g.rel;
  return j;
}

// Add a wave's exact sums (s1, count, s2 < 2^96) to a batch accumulator
// slot: reduce over the wave, then lane 0 adds to the slot's stripe for this
// wave with no-return 64-bit atomics (s2 split as hi * 2^32 + lo).
__device__ __forceinline__ void acc_add_wave(BatchAcc* slot, int64_t s1, int64_t cnt, U128 s2) {
  s1 = wave_sum64(s1);
  cnt = wave_sum64(cnt);
  for (int m = 32; m >= 1; m >>= 1) {
    U128 o;
    o.lo = __shfl_xor(s2.lo, m);
    o.hi = __shfl_xor(s2.hi, m);
    add_u128(s2, o);
  }
  if (lane_id() == 0) {
    const unsigned stripe = (blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) % kAccStripes;
    BatchAcc* a = slot + stripe;
    atomicAdd((unsigned long long*)&a->s1, (unsigned long long)s1);
    atomicAdd((unsigned long long*)&a->cnt, (unsigned long long)cnt);
    atomicAdd((unsigned long long*)&a->s2lo, (unsigned long long)(s2.lo & 0xffffffffull));
    atomicAdd((unsigned long long*)&a->s2hi, (unsigned long long)((s2.lo >> 32) | (s2.hi << 32)));
  }
}

// Workgroup barrier that orders LDS only.  __syncthreads() also fences
// global memory, which makes every wave wait at each barrier until all its
// global stores are acknowledged; the tiles below never read back what they
// store (outputs) and only read global data nobody writes during the kernel,
// so their barriers need the LDS ordering alone, and the stores of one
// step then drain while the next step computes.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum (s1, cnt, s2) over the calling workgroup and add it to one stripe of
// 'slot' with one set of atomics per workgroup rather than per wave (device-
// scope atomics on a few addresses serialise): each wave reduces its lanes,
// lane 0 leaves the wave's sums in red[wave] (LDS, one BatchAcc per wave),
// and after a barrier wave 0 adds them up.  Every thread of the workgroup
// calls it; 'red' is not touched again before the caller's next barrier.
__device__ __forceinline__ void acc_add_group(BatchAcc* slot, int64_t s1, int64_t cnt, U128 s2, BatchAcc* red,
                                              int nwaves) {
  s1 = wave_sum64(s1);
  cnt = wave_sum64(cnt);
  for (int m = 32; m >= 1; m >>= 1) {
    U128 o;
    o.lo = __shfl_xor(s2.lo, m);
    o.hi = __shfl_xor(s2.hi, m);
    add_u128(s2, o);
  }
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (lane_id() == 0) red[w] = BatchAcc{s1, cnt, s2.lo, s2.hi};
  lds_barrier();
  if (w != 0) return;
  const bool mine = lane_id() < nwaves;
  const BatchAcc v = mine ? red[lane_id()] : BatchAcc{0, 0, 0, 0};
  int64_t t1 = wave_sum64(v.s1), tc = wave_sum64(v.cnt);
  U128 t2 = {v.s2lo, v.s2hi};
  for (int m = 32; m >= 1; m >>= 1) {
    U128 o;
    o.lo = __shfl_xor(t2.lo, m);
    o.hi = __shfl_xor(t2.hi, m);
    add_u128(t2, o);
  }
  if (lane_id() == 0) {
    BatchAcc* a = slot + blockIdx.x % kAccStripes;
    atomicAdd((unsigned long long*)&a->s1, (unsigned long long)t1);
    atomicAdd((unsigned long long*)&a->cnt, (unsigned long long)tc);
    atomicAdd((unsigned long long*)&a->s2lo, (unsigned long long)(t2.lo & 0xffffffffull));
    atomicAdd((unsigned long long*)&a->s2hi, (unsigned long long)((t2.lo >> 32) | (t2.hi << 32)));
  }
}

// Index of the calling wave within its workgroup, as a wave-uniform value.
__device__ __forceinline__ int wave_in_group() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

// ---- chunk staging -----------------------------------------------------------
// Per-lane metadata of one block of a chunk.
struct LaneBlock {
  int w;        // bit width (0..30), 0 for lanes past the last block
  int q0;       // first quantization integer of the block
  int len;      // valid slots (S for all but the field's last block, 0 if none)
  int64_t b;    // block index
};

// Staging of chunk c in two halves, so that a wave can load chunk c+1 while
// it decodes chunk c.  chunk_begin: lane l loads the width and q0 of block
// 64c+l, the wave scans the payload word counts and checks them against the
// chunk table, and the lane loads the first PF words of its block into
// registers (16-byte loads, dword aligned, where the four-word group stays
// inside the payload; a group may run into the next block's words, which
// are ignored).  chunk_end: the words go to the lane's column of the LDS
// tile (tile rows = kmax+1, row k at tile + k*64); words past PF are copied
// there directly.  An inconsistent chunk records a status and its lanes
// decode as all-zero blocks.
template <int PF>
struct ChunkStage {
  LaneBlock lb;
  int nw;                  // payload words of the lane's block
  const uint32_t* src;     // the block's first payload word
  uint32_t pw[PF];         // words [0, PF) of the block
};

template <int S, int PF>
__device__ __forceinline__ void chunk_begin(const uint8_t* __restrict__ width, const int32_t* __restrict__ q0s,
                                            const uint64_t* __restrict__ chunk_off,
                                            const uint32_t* __restrict__ payload, uint64_t payload_words, int64_t n,
                                            int64_t nb, int64_t c, int kmax, ChunkStage<PF>& cs, int* status) {
  static_assert(PF % 4 == 0, "four-word groups");
  const int l = lane_id();
  LaneBlock& lb = cs.lb;
  lb.b = c * kChunkBlocks + l;
  const bool valid = lb.b < nb;
  int w = valid ? (int)width[lb.b] : 0;
  lb.q0 = valid ? q0s[lb.b] : 0;
  int64_t first = lb.b * S;
  lb.len = valid ? (int)((n - first) < S ? (n - first) : S) : 0;
  int nw = block_words<S>(w);
  bool bad = (w > kMaxWidth) || (nw > kmax);
  int incl = wave_incl_scan(bad ? 0 : nw);
  int woff = incl - (bad ? 0 : nw);
  int total = __shfl(incl, kWave - 1);
  uint64_t base = chunk_off[c];
  uint64_t next = chunk_off[c + 1];
  int any_bad = __any(bad);
  if (any_bad || next - base != (uint64_t)total || next > payload_words) {
    if (l == 0) record_status(status, kErrBadStream);
    w = 0;
    nw = 0;
  }
  lb.w = w;
  cs.nw = nw;
  cs.src = payload + base + woff;
  const uint64_t avail = payload_words - (base + woff);
  typedef uint32_t u4 __attribute__((ext_vector_type(4), aligned(4)));
#pragma unroll
  for (int k = 0; k < PF; k += 4) {
    if ((uint64_t)(k + 4) <= avail) {
      u4 t = {0u, 0u, 0u, 0u};
      if (k < nw) t = *(const u4*)(cs.src + k);
      cs.pw[k] = t.x; cs.pw[k + 1] = t.y; cs.pw[k + 2] = t.z; cs.pw[k + 3] = t.w;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) cs.pw[k + u] = (k + u < nw) ? cs.src[k + u] : 0u;
    }
  }
}

template <int PF>
__device__ __forceinline__ void chunk_end(const ChunkStage<PF>& cs, uint32_t* tile) {
  const int l = lane_id();
#pragma unroll
  for (int k = 0; k < PF; ++k)
    if (k < cs.nw) tile[k * kWave + l] = cs.pw[k];
  for (int k = PF; k < cs.nw; ++k) tile[k * kWave + l] = cs.src[k];
}

// Both halves at once.
template <int S>
__device__ __forceinline__ void stage_chunk(const uint8_t* __restrict__ width,
                                           const int32_t* __restrict__ q0s,
                                           const uint64_t* __restrict__ chunk_off,
                                           const uint32_t* __restrict__ payload,
                                           uint64_t payload_words, int64_t n, int64_t nb,
                                           int64_t c, uint32_t* tile, int kmax, LaneBlock& lb,
                                           int* status) {
  ChunkStage<8> cs;
  chunk_begin<S, 8>(width, q0s, chunk_off, payload, payload_words, n, nb, c, kmax, cs, status);
  chunk_end<8>(cs, tile);
  lb = cs.lb;
}

// ---- random access to one block ----------------------------------------------
// Word offset (within the payload) of block b: the chunk table entry plus the
// words of the blocks before b in its 64-block chunk, read as up to 16 words
// of packed widths (byte sums with v_sad_u8, non-zero bytes by bit tricks).
template <int S>
__device__ __forceinline__ uint64_t block_offset(const uint8_t* __restrict__ width,
                                                 const uint64_t* __restrict__ chunk_off, int64_t nb,
                                                 int64_t b) {
  const int64_t c = b / kChunkBlocks;
  const int cnt = (int)(b - c * kChunkBlocks);
  const uint32_t* wq = (const uint32_t*)(width + c * kChunkBlocks);
  const int64_t avail = nb - c * kChunkBlocks;  // bytes of this chunk inside the section
  uint32_t sumw = 0, nz = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (4 * k < cnt) {
      // the width section is padded to 256 bytes, so whole words are readable
      uint32_t dw = (4 * k < avail) ? wq[k] : 0u;
      const int keep = cnt - 4 * k;
      if (keep < 4) dw &= (1u << (8 * keep)) - 1u;
      sumw += __builtin_amdgcn_sad_u8(dw, 0u, 0u);
      const uint32_t t = ((dw & 0x7f7f7f7fu) + 0x7f7f7f7fu) | dw;
      nz += __builtin_popcount(t & 0x80808080u);
    }
  }
  return chunk_off[c] + (uint64_t)(S / 32) * (sumw + nz);
}

// Stage block b into one LDS column (rows STRIDE words apart).  Returns the
// width, 0 when the block is corrupt (status recorded) -- it then decodes as
// the constant q0.
template <int S, int STRIDE>
__device__ __forceinline__ int stage_block(const uint8_t* __restrict__ width, const int32_t* __restrict__ q0s,
                                           const uint64_t* __restrict__ chunk_off,
                                           const uint32_t* __restrict__ payload, uint64_t payload_words,
                                           int64_t nb, int64_t b, uint32_t* col, int kmax, int& q0,
                                           int* status, const uint16_t* __restrict__ rel = nullptr) {
  const int w = (int)width[b];
  q0 = q0s[b];
  const int nw = block_words<S>(w);
  const uint64_t off = rel ? chunk_off[b / kChunkBlocks] + rel[b] : block_offset<S>(width, chunk_off, nb, b);
  if (w > kMaxWidth || nw > kmax || off + (uint64_t)nw > payload_words) {
    record_status(status, kErrBadStream);
    return 0;
  }
  const uint32_t* src = payload + off;
  for (int k0 = 0; k0 < nw; k0 += 8) {
    uint32_t t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = (k0 + u < nw) ? src[k0 + u] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < nw) col[(k0 + u) * STRIDE] = t[u];
  }
  return w;
}

// Decode the lane's block from its LDS column.  For every slot j in order
// it calls sink(j, p_j, q_j) with p the decorrelated integer (stage 2) and
// q the recorrelated quantization integer (stage 3).  Slot 0 has p = 0 and
// q = q0.  col = tile + lane (column base); rows hold sign word(s) first,
// then magnitude words.
// MEAN: a block-mean stream (q0 holds the block mean M): q_j = M + p_j.
template <int S, int STRIDE = kWave, bool MEAN = false, class Sink>
__device__ __forceinline__ void decode_lane_block(const uint32_t* col, int w, int q0, Sink&& sink) {
  const uint32_t sg0 = w ? col[0] : 0u;
  const uint32_t sg1 = (S == 64 && w) ? col[STRIDE] : 0u;
  const uint32_t* mag = col + (S / 32) * STRIDE;
  int q = q0;
  uint32_t uw = (uint32_t)w;
#pragma unroll
  for (int g = 0; g < S; g += 8) {
    // an empty asm that "changes" uw keeps the compiler from computing the
    // bit positions of all S slots up front (S live registers)
    asm volatile("" : "+v"(uw));
    uint32_t lo[8], hi[8], pos[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      // bit position j*w (24-bit multiply, full rate); word pos/32 and the next
      pos[u] = __umul24((uint32_t)(g + u), uw);
      // the word index, opaque to the optimiser: otherwise it folds j*w into
      // each address (multiply, mask, add) and recomputes j*w for the bit
      // offset, sometimes with the quarter-rate 32-bit multiply
      uint32_t k = pos[u] >> 5;
      asm("" : "+v"(k));
      const uint32_t* a = mag + k * STRIDE;
      lo[u] = a[0];
      hi[u] = a[STRIDE];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = g + u;
      const uint32_t m = __builtin_amdgcn_ubfe(__builtin_amdgcn_alignbit(hi[u], lo[u], pos[u]), 0u, uw);
      const int sg = __builtin_amdgcn_sbfe((int)(j < 32 ? sg0 : sg1), (uint32_t)(j & 31), 1u);
      // p = (m ^ sg) - sg applies the sign (sg = 0 or -1); q is formed as
      // ((m ^ sg) + q) - sg so that a sink using only q costs one xor-add
      const uint32_t x = m ^ (uint32_t)sg;
      const int p = (int)x - sg;
      if constexpr (MEAN) q = (int)(x + (uint32_t)q0) - sg;
      else q = (int)(x + (uint32_t)q) - sg;
      sink(j, p, q);
    }
  }
}

// Decode one staged block (column 'col', rows STRIDE words apart) and write its
// S values of q to dst[j + j/32 + pad_j], pad_j = ((j & 31) >= jx) (jx = 32:
// none).  Reads are issued eight slots at a time, ahead of the writes.
template <int S, bool ALIGNED, int STRIDE>
__device__ __forceinline__ void decode_block_q(const uint32_t* col, int w, int q0, int* dst, int jx) {
  const uint32_t sg0 = col[0];
  const uint32_t sg1 = S == 64 ? col[STRIDE] : 0u;
  const uint32_t* mag = col + (S / 32) * STRIDE;
  int* dst1 = dst + 1;
  int q = q0;
  uint32_t uw = (uint32_t)w;
#pragma unroll
  for (int g = 0; g < S; g += 8) {
    // an empty asm that "changes" uw keeps the compiler from computing the
    // bit positions of all S slots up front (S live registers)
    asm volatile("" : "+v"(uw));
    uint32_t lo[8], hi[8], pos[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      pos[u] = __umul24((uint32_t)(g + u), uw);  // full-rate 24-bit multiply
      uint32_t k = pos[u] >> 5;
      asm("" : "+v"(k));  // one shift-add per address (see decode_lane_block)
      const uint32_t* a = mag + k * STRIDE;
      lo[u] = a[0];
      hi[u] = a[STRIDE];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = g + u;
      const uint32_t m = __builtin_amdgcn_ubfe(__builtin_amdgcn_alignbit(hi[u], lo[u], pos[u]), 0u, uw);
      const int sg = __builtin_amdgcn_sbfe((int)(j < 32 ? sg0 : sg1), (uint32_t)(j & 31), 1u);
      q = (int)((m ^ (uint32_t)sg) + (uint32_t)q) - sg;  // q += (m ^ sg) - sg
      if constexpr (ALIGNED) {
        dst[j + (j >> 5)] = q;
      } else {
        int* d = ((j & 31) >= jx) ? dst1 : dst;
        d[j + (j >> 5)] = q;
      }
    }
  }
}

// Words [0, min(words, N)) of a block at payload word 'off' into w[] (the
// rest 0).  A block's words are contiguous and the blocks of a decoded row
// follow each other in the payload, so each lane reads its words four at a
// time: one 16-byte load per four words (dword aligned) instead of four
// scattered dword loads.  Four-word groups may run into the next block's
// words (ignored); near the end of the payload the lane reads word by word.
template <int N>
__device__ __forceinline__ void prefetch_words(const uint32_t* __restrict__ payload, uint64_t payload_words,
                                               uint64_t off, int words, uint32_t (&w)[N]) {
  static_assert(N % 4 == 0, "four-word groups");
  typedef uint32_t u4 __attribute__((ext_vector_type(4), aligned(4)));
  const uint32_t* src = payload + off;
  if (off + N <= payload_words) {
#pragma unroll
    for (int k = 0; k < N; k += 4) {
      u4 t = {0u, 0u, 0u, 0u};
      if (k < words) t = *(const u4*)(src + k);
      w[k] = t.x; w[k + 1] = t.y; w[k + 2] = t.z; w[k + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) w[k] = (k < words) ? src[k] : 0u;
  }
}

// Rows of the staging tile needed for blocks of width <= wmax: sign words,
// magnitude words, and one spare row read (never used) past the last word.
template <int S>
__host__ __device__ constexpr int tile_rows(int wmax) {
  return (S / 32) * (1 + wmax) + 1;
}

// Exact (float)(q * quantum) and q * quantum: the dequantization of Alg. 2,
// always through binary64 so every platform rounds the same way.
__device__ __forceinline__ double dequant64(int q, double quantum) { return (double)q * quantum; }

}  // namespace hsz
