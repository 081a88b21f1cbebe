// abi_util.hpp -- host-side helpers shared by the C-ABI translation units:
// header checks, dims/box conversion, stream views, HIP error capture.
#pragma once

#include <hip/hip_runtime.h>
#include <string.h>

#include "../../include/hsz.h"
#include "hsz_device.hpp"
#include "hsz_launch.hpp"
#include "hsz_nd.hpp"

namespace hsz_abi {

// the last HIP error seen by the library on this thread
int& last_hip();

inline int hip_fail(hipError_t e) {
  last_hip() = (int)e;
  return HSZ_ERR_HIP;
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

inline uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
inline uint32_t rd32(const uint8_t* p) {
  uint32_t v = 0;
  for (int k = 3; k >= 0; --k) v = (v << 8) | p[k];
  return v;
}
inline uint64_t rd64(const uint8_t* p) {
  uint64_t v = 0;
  for (int k = 7; k >= 0; --k) v = (v << 8) | p[k];
  return v;
}
inline double rdf64(const uint8_t* p) {
  uint64_t v = rd64(p);
  double d;
  memcpy(&d, &v, 8);
  return d;
}

// dims of the field's own axes -> 3D view with leading ones
inline bool dims3_of(int ndim, const int64_t* dims, int64_t out[3], int64_t* n) {
  if (ndim < 1 || ndim > 3 || !dims) return false;
  out[0] = out[1] = out[2] = 1;
  int64_t prod = 1;
  for (int k = 0; k < ndim; ++k) {
    if (dims[k] < 1) return false;
    out[3 - ndim + k] = dims[k];
    if (prod > (int64_t(1) << 40) / dims[k]) return false;
    prod *= dims[k];
  }
  *n = prod;
  return true;
}

inline bool valid_block(int block) { return block == 32 || block == 64; }

inline hsz::StreamView view_of(const void* d_c, const hsz_header* h) {
  hsz::StreamView v;
  const uint8_t* base = (const uint8_t*)d_c;
  v.base = base;
  v.chunk_off = (const uint64_t*)(base + h->off_chunk);
  v.q0 = (const int32_t*)(base + h->off_q0);
  v.width = base + h->off_width;
  v.payload = (const uint32_t*)(base + h->off_payload);
  v.payload_words = h->payload_words;
  v.n = h->n;
  v.nb = h->nb;
  v.nchunks = h->nchunks;
  v.block = h->block;
  v.dtype = h->dtype;
  v.quantum = h->quantum;
  v.max_abs_q = h->max_abs_q;
  v.flags = h->flags;
  return v;
}

// Re-check a header the caller hands back (it may have been edited).
inline int check_header(const hsz_header* h) {
  if (!h) return HSZ_ERR_INVALID_ARG;
  if (h->dtype != HSZ_F32 && h->dtype != HSZ_F64) return HSZ_ERR_BAD_STREAM;
  int64_t d3[3], n;
  if (!dims3_of(h->ndim, h->dims, d3, &n) || n != h->n) return HSZ_ERR_BAD_STREAM;
  if (!valid_block(h->block)) return HSZ_ERR_UNSUPPORTED;
  if (h->flags != 0 && h->flags != HSZ_FLAG_BLOCK_MEAN && h->flags != HSZ_FLAG_LORENZO &&
      h->flags != HSZ_FLAG_INTER_BLOCK)
    return HSZ_ERR_BAD_STREAM;
  if (h->flags == HSZ_FLAG_LORENZO && h->ndim < 2) return HSZ_ERR_BAD_STREAM;
  hsz::Layout L = h->flags == HSZ_FLAG_LORENZO       ? hsz::make_layout_nd(d3, h->ndim, h->block)
                  : h->flags == HSZ_FLAG_INTER_BLOCK ? hsz::make_layout_flat(h->n, h->block)
                                                     : hsz::make_layout(h->n, h->block);
  if (L.nb != h->nb || L.nchunks != h->nchunks || L.off_chunk != h->off_chunk || L.off_q0 != h->off_q0 ||
      L.off_width != h->off_width || L.off_payload != h->off_payload)
    return HSZ_ERR_BAD_STREAM;
  if (h->total_bytes != h->off_payload + 4 * h->payload_words) return HSZ_ERR_BAD_STREAM;
  if (!(h->quantum > 0.0) || h->max_abs_q > (uint32_t)hsz::kQMax) return HSZ_ERR_BAD_STREAM;
  return HSZ_OK;
}

// box in the field's axes -> 3D box; NULL = whole field
inline bool box3_of(const hsz_header* h, const hsz_box* b, hsz::Box3* o) {
  int64_t d3[3], n;
  dims3_of(h->ndim, h->dims, d3, &n);
  int64_t lo[3] = {0, 0, 0}, hi[3] = {d3[0], d3[1], d3[2]};
  if (b) {
    for (int k = 0; k < h->ndim; ++k) {
      const int a = 3 - h->ndim + k;
      lo[a] = b->lo[k];
      hi[a] = b->hi[k];
      if (lo[a] < 0 || hi[a] > d3[a] || lo[a] >= hi[a]) return false;
    }
  }
  *o = hsz::Box3{lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]};
  return true;
}

}  // namespace hsz_abi
