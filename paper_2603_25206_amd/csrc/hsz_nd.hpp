// hsz_nd.hpp -- HSZp-nd streams (Sec. IV): the multidimensional Lorenzo
// decorrelation over the whole field, encoded in nd blocks.  Host and device
// helpers shared by the compressor, the decoder, the operations and the ABI.
#pragma once

#include "hsz_device.hpp"
#include "hsz_launch.hpp"

namespace hsz {

constexpr uint32_t kFlagLorenzo = 2u;  // header flags bit 1: HSZp-nd
constexpr uint32_t kFlagInterBlock = 4u;  // header flags bit 2: HSZp, deltas across blocks of the flat field
constexpr int32_t kPMax = (1 << 30) - 1;  // largest |p| of a Lorenzo residual

// Block shape (slow -> fast, in the 3D view) of the nd partition: S = 2^k
// elements with k split over the field's axes as evenly as possible, the
// faster axes taking the remainder (2D: 4x8 for S = 32, 8x8 for 64; 3D:
// 2x4x4 and 4x4x4).  false for a 1D field or another S.
__host__ __device__ constexpr bool nd_block_shape(int ndim, int S, int b[3]) {
  if (ndim < 2 || ndim > 3 || (S != 32 && S != 64)) return false;
  const int k = S == 32 ? 5 : 6;
  const int ez = ndim == 3 ? k / 3 : 0;
  const int ey = (k - ez) / 2;
  const int ex = k - ez - ey;
  b[0] = 1 << ez;
  b[1] = 1 << ey;
  b[2] = 1 << ex;
  return true;
}

// ND = 1: the flat field of HSZp, blocks of S consecutive elements.
template <int ND, int S>
struct NdShape {
  static constexpr int k = S == 32 ? 5 : 6;
  static constexpr int ez = ND == 3 ? k / 3 : 0;
  static constexpr int ey = ND >= 2 ? (k - ez) / 2 : 0;
  static constexpr int ex = k - ez - ey;
  static constexpr int BZ = 1 << ez, BY = 1 << ey, BX = 1 << ex;
};

// Block grid of a field in the 3D view.
struct NdGrid {
  int64_t Z, Y, X;  // field dims (leading ones)
  int64_t nbz, nby, nbx;
  int ndim;         // the field's own rank (2 or 3): it fixes the block shape
};

// HSZp: the field as one row of n (ndim 1 selects blocks of S in a row)
inline NdGrid flat_grid(int64_t n, int S) { return NdGrid{1, 1, n, 1, 1, (n + S - 1) / S, 1}; }

inline NdGrid nd_grid(const int64_t d3[3], int ndim, int S) {
  int b[3] = {1, 1, 1};
  nd_block_shape(ndim, S, b);
  return NdGrid{d3[0], d3[1], d3[2], (d3[0] + b[0] - 1) / b[0], (d3[1] + b[1] - 1) / b[1],
                (d3[2] + b[2] - 1) / b[2], ndim};
}

// Sections of an HSZp-nd stream: blocks counted over the nd partition, an
// empty q0 section.
Layout make_layout_nd(const int64_t d3[3], int ndim, int block);
// Sections of an HSZp stream (inter-block deltas): the 1D partition, no q0.
Layout make_layout_flat(int64_t n, int block);
// Compression workspace of the Lorenzo modes (nd or flat layout): the delta
// mode's plus one int32 residual per slot of the partition.
uint64_t compress_workspace_bytes_nd(const Layout& lay);

// Extremes of a field ({vmin, vmax, non-finite flag} as three doubles at
// 'out'), with extremes_workspace_bytes() of scratch: the first pass of a
// field compressed slab by slab with the whole field's quantizer.
uint64_t extremes_workspace_bytes();
hipError_t launch_extremes(const void* x, int dtype, int64_t n, double* out, uint8_t* ws, hipStream_t s);

// Compression of an HSZp-nd (a.flags = kFlagLorenzo, a.lay from
// make_layout_nd) or HSZp stream (kFlagInterBlock, make_layout_flat).
hipError_t launch_compress_nd(const CompressArgs& a, hipStream_t s);

// Rows of a chunk's LDS staging tile: |p| of a residual is at most 2^ND max|q|
// (and at most 2^30 - 1).
template <int S, int ND>
inline int lz_kmax(uint32_t max_abs_q) {
  uint64_t pm = (uint64_t)max_abs_q << ND;
  if (pm > (uint64_t)kPMax) pm = kPMax;
  const int wmax = pm ? 64 - __builtin_clzll(pm) : 1;
  return tile_rows<S>(wmax > kMaxWidth ? kMaxWidth : wmax) - 1;
}

// payload words per lane in flight per round trip of the chunk staging below
constexpr int kStageBatch = 8;

// a value every lane of the wave holds, moved to scalar registers
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
}

// A chunk's metadata as loaded: the lane's block width (through a
// descriptor of the chunk's blocks: a lane past the last block reads 0) and
// the chunk's word offsets, all in one round trip.  Nothing here waits for
// the loads, so a caller may issue them a step ahead of their use.
struct LzMeta {
  int w;
  uint64_t base, next;
};

__device__ __forceinline__ LzMeta lz_meta(const StreamView& v, int64_t c) {
  const int64_t b0 = c * kChunkBlocks;
  const int64_t nbc = v.nb - b0 < kChunkBlocks ? v.nb - b0 : kChunkBlocks;
  const __amdgpu_buffer_rsrc_t r_w =
      __builtin_amdgcn_make_buffer_rsrc((void*)(v.width + b0), (short)0, (int)(nbc > 0 ? nbc : 0), 0x00020000);
  LzMeta m;
  m.w = (int)__builtin_amdgcn_raw_buffer_load_b8(r_w, (uint32_t)lane_id(), 0, 0);
  m.base = v.chunk_off[c];
  m.next = v.chunk_off[c + 1];
  return m;
}

// Stage the payload of chunk c (metadata m) into the lane columns of 'tile'
// (row k at tile + k*64, lane l <-> block 64c + l) and return the lane's
// block width; an inconsistent chunk records a status and its blocks decode
// as zeros.
template <int S>
__device__ __forceinline__ int lz_stage_meta(const StreamView& v, const LzMeta& m, uint32_t* tile, int kmax,
                                             int* status) {
  const int l = lane_id();
  // the offsets are the wave's (c is): moved to scalar registers, so the
  // payload descriptor below is one
  const uint64_t base = uniform_u64(m.base), next = uniform_u64(m.next);
  int w = m.w;
  int nw = block_words<S>(w);
  const bool bad = (w > kMaxWidth) || (nw > kmax);
  const int incl = wave_incl_scan(bad ? 0 : nw);
  const int woff = incl - (bad ? 0 : nw);
  const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
  if (__any(bad) || next - base != (uint64_t)total || next > v.payload_words) {
    if (l == 0) record_status(status, kErrBadStream);
    w = 0;
    nw = 0;
  }
  // kStageBatch words per lane in flight per round trip (a load, its wait
  // and the LDS write per word would make the chunk's latency its width in
  // trips).  Loads through a descriptor of the chunk's words: past a lane's
  // own words the offset leaves the descriptor and the load returns 0, so no
  // lane branches; rows past the lane's width are written with those zeros,
  // up to the tile's last row.
  const uint32_t chunk_bytes = (uint32_t)total * 4u;
  const __amdgpu_buffer_rsrc_t r_pay =
      __builtin_amdgcn_make_buffer_rsrc((void*)(v.payload + base), (short)0, (int)chunk_bytes, 0x00020000);
  for (int k0 = 0; __any(k0 < nw); k0 += kStageBatch) {
    uint32_t r[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      r[u] = __builtin_amdgcn_raw_buffer_load_b32(r_pay, k0 + u < nw ? 4u * (uint32_t)(woff + k0 + u) : 0x80000000u,
                                                  0, 0);
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (k0 + u <= kmax) tile[(k0 + u) * kWave + l] = r[u];
  }
  return w;
}

// The staging split in two for callers that keep a chunk's payload in
// flight while they do other work: lz_issue takes the metadata (whose loads
// must have landed) and issues the loads of the lane's first PF payload
// words into registers; lz_commit writes them to the tile (which holds at
// least PF rows: all PF are written, without branches, so the wait for them
// counts exactly the memory operations issued since) and stages the rest
// (widths past PF words), which then waits.  A chunk of none (ok false)
// issues loads that all fall past their descriptor.
template <int PF>
struct LzPending {
  uint32_t r[PF];
  int w, nw, woff;
  uint64_t base;
  int total;
};

template <int S, int PF>
__device__ __forceinline__ LzPending<PF> lz_issue(const StreamView& v, const LzMeta& m, bool ok, int kmax,
                                                  int* status) {
  LzPending<PF> P;
  const uint64_t base = uniform_u64(m.base), next = uniform_u64(m.next);
  int w = ok ? m.w : 0;
  int nw = block_words<S>(w);
  const bool bad = (w > kMaxWidth) || (nw > kmax);
  const int incl = wave_incl_scan(bad ? 0 : nw);
  const int woff = incl - (bad ? 0 : nw);
  const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
  if (ok && (__any(bad) || next - base != (uint64_t)total || next > v.payload_words)) {
    if (lane_id() == 0) record_status(status, kErrBadStream);
    w = 0;
    nw = 0;
  }
  if (!ok) nw = 0;
  const __amdgpu_buffer_rsrc_t r_pay =
      __builtin_amdgcn_make_buffer_rsrc((void*)(v.payload + base), (short)0, (int)((uint32_t)total * 4u), 0x00020000);
#pragma unroll
  for (int u = 0; u < PF; ++u)
    P.r[u] = __builtin_amdgcn_raw_buffer_load_b32(r_pay, u < nw ? 4u * (uint32_t)(woff + u) : 0x80000000u, 0, 0);
  P.w = w;
  P.nw = nw;
  P.woff = woff;
  P.base = base;
  P.total = total;
  return P;
}

template <int PF>
__device__ __forceinline__ int lz_commit(const StreamView& v, const LzPending<PF>& P, uint32_t* tile, int kmax) {
  const int l = lane_id();
#pragma unroll
  for (int u = 0; u < PF; ++u) tile[u * kWave + l] = P.r[u];
  if (kmax >= PF) {
    const __amdgpu_buffer_rsrc_t r_pay = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(v.payload + P.base), (short)0, (int)((uint32_t)P.total * 4u), 0x00020000);
    for (int k0 = PF; __any(k0 < P.nw); k0 += kStageBatch) {
      uint32_t r[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u)
        r[u] = __builtin_amdgcn_raw_buffer_load_b32(
            r_pay, k0 + u < P.nw ? 4u * (uint32_t)(P.woff + k0 + u) : 0x80000000u, 0, 0);
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u)
        if (k0 + u <= kmax) tile[(k0 + u) * kWave + l] = r[u];
    }
  }
  return P.w;
}

// The two steps above at once.
template <int S>
__device__ __forceinline__ int lz_stage(const StreamView& v, int64_t c, uint32_t* tile, int kmax, int* status) {
  return lz_stage_meta<S>(v, lz_meta(v, c), tile, kmax, status);
}

// Decoding of an HSZp-nd stream to stage 2 (p, int32, the field's layout),
// 3 (q, int32) or 4 (the field's dtype).  Stage 3 and 4 rebuild q with
// prefix sums along every axis (the inverse of the Lorenzo residual) in the
// output itself; the binary64 stage 4 keeps q in the low word of each
// element until its conversion, so no scratch memory is needed.
// 'tmp' holds lz_scan_tmp_bytes(n) bytes for a single long row (HSZp).
hipError_t lz_decode(const StreamView& v, const NdGrid& g, int stage, void* out, int* status, int32_t* tmp,
                     hipStream_t s);

// Derivative along axis3 (of the 3D view) on D_p (Eq. (derivative_Dp)):
// p (int32, the field's layout) -> out (field dtype, whole field).
hipError_t lz_deriv_p(const int32_t* p, const StreamView& v, const NdGrid& g, int axis3, void* out, hipStream_t s);

// D_q of an HSZp-nd stream in two passes for fields of three dimensions
// whose rows hold at most 512 columns, a multiple of 4 (lz_dq_ok): lz_dq_front decodes and takes the prefix sums along x and,
// within z segments, along z into t (the field's layout) and the segments'
// totals into tot (lz_dq_tmp_bytes), then the exclusive prefix of those over
// segments; q is then the prefix sum along y of t plus tot of the element's
// segment (seg_planes planes each).  lz_decode takes this route for stages
// 3 and 4 (binary32) when given tmp of lz_dq_tmp_bytes.
bool lz_dq_ok(const NdGrid& g);
// HSZp (one row of more than kFlatTile words) from the stream: p into 'p'
// with the sum of each kFlatTile tile in 'tsums', then the exclusive prefix
// of the sums (tile t's carry); q is p prefix-summed within its tile plus
// the carry.
hipError_t lz_flat_front(const StreamView& v, const NdGrid& g, int32_t* p, int32_t* tsums, int* status,
                         hipStream_t s);
uint64_t lz_dq_tmp_bytes(const NdGrid& g);
hipError_t lz_dq_front(const StreamView& v, const NdGrid& g, int32_t* t, int32_t* tot, int* status, hipStream_t s,
                       int64_t* seg_planes);

// The central-difference numerator along axis3 on D_p (Eq. (derivative_Dp)
// before its scaling): int32 over the whole field, the D_q route's exactly.
hipError_t lz_numerator_p(const int32_t* p, const NdGrid& g, int axis3, int32_t* out, hipStream_t s);

// The Laplacian on D_p (Eq. (laplacian_Dp)) of the whole field into out
// (field dtype); cbuf holds g.ndim int32 fields of scratch.
hipError_t lz_laplacian_p(const int32_t* p, const NdGrid& g, double quantum, int dtype, int32_t* cbuf, void* out,
                          hipStream_t s);

// Divergence / curl on D_p of an HSZp-nd vector field (whole field): term k
// is component tc[k] differentiated along view axis ta[k], signed ts[k],
// added to output to[k]; p[c] the components' D_p buffers, halfq[c] their
// Delta/2; nbuf holds nterms int32 fields of scratch.
hipError_t lz_vector_p(const int32_t* const* p, const NdGrid& g, int nterms, const int* tc, const int* ta,
                       const int* ts, const int* to, int nout, const double* halfq, int dtype, int32_t* nbuf,
                       void* const* out, hipStream_t s);

// Prefix sums along the 3D view's axes z..x except 'skip' (-1: none) of an
// int32 field stored at element stride es (1 or 2 words), in place.  A
// single row (Z = Y = 1) is scanned device-wide in tiles of 4096 words whose
// sums go to 'tmp' (lz_scan_tmp_bytes(X) bytes); sums_ready: the decoder
// already wrote them there.
hipError_t lz_scan_axes(int32_t* buf, int64_t Z, int64_t Y, int64_t X, int es, int skip, int32_t* tmp,
                        hipStream_t s, bool sums_ready = false);
constexpr int64_t kFlatTile = 4096;
inline uint64_t lz_scan_tmp_bytes(int64_t n) { return ((uint64_t)(4 * ((n + kFlatTile - 1) / kFlatTile)) + 255) / 256 * 256; }

// Statistics of an HSZp-nd stream on D_p (whole field): MEAN through the
// nd weights of Sec. V-A (from a stage-2 buffer, or fused from the stream
// when p == nullptr), VAR through the prefix sums of Alg. 4 (p copied to
// 'scratch', 4n bytes, and rebuilt there; fused: decoded there).
hipError_t launch_lz_stats(const int32_t* p, const StreamView& v, const NdGrid& g, int op, void* result,
                           uint8_t* ws, int32_t* scratch, int32_t* tmp, hipStream_t s);

}  // namespace hsz
