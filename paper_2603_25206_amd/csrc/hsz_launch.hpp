// hsz_launch.hpp -- host-side interface between the C-ABI layer (api.cpp)
// and the kernel launchers in the .hip files.  Plain structs of sizes and
// device pointers; no torch or Python types.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsz {

// Section placement of a stream (depends only on n and S).
struct Layout {
  int64_t n, nb, nchunks;
  int block;
  uint64_t off_chunk, off_q0, off_width, off_payload;
};
Layout make_layout(int64_t n, int block);

// 3D view of a field: dims slow -> fast with leading ones.
struct Dims3 {
  int64_t z, y, x;
};
// Box in the 3D view, half-open.
struct Box3 {
  int64_t z0, z1, y0, y1, x0, x1;
  int64_t volume() const { return (z1 - z0) * (y1 - y0) * (x1 - x0); }
};

// Device view of a compressed stream.
struct StreamView {
  const uint8_t* base;
  const uint64_t* chunk_off;
  const int32_t* q0;
  const uint8_t* width;
  const uint32_t* payload;
  uint64_t payload_words;
  int64_t n, nb, nchunks;
  int block;
  int dtype;
  double quantum;
  uint32_t max_abs_q;
};

// ---- compression -------------------------------------------------------------
struct CompressArgs {
  const void* x;
  int dtype;
  int ndim;
  int64_t dims[3];  // 3D view
  double eb;
  int eb_is_rel;
  Layout lay;
  uint8_t* out;
  uint64_t cap;
  uint8_t* ws;
  uint64_t ws_bytes;
};
uint64_t compress_workspace_bytes(const Layout& lay);
hipError_t launch_compress(const CompressArgs& a, hipStream_t s);

// ---- decompression -----------------------------------------------------------
hipError_t launch_decode(const StreamView& v, int stage, void* out, int* status, hipStream_t s);
// per-block payload offsets within their chunk (uint16[nb])
hipError_t launch_block_index(const StreamView& v, uint16_t* rel, hipStream_t s);

// ---- operations ----------------------------------------------------------------
// Workspace: [0,256) status + scratch words, then per-workgroup partials.
constexpr int kOpWorkgroups = 2048;  // max workgroups of a reduction launch
uint64_t op_workspace_bytes();
// gradient operations also keep a per-block offset index in the workspace
uint64_t grad_workspace_bytes(int64_t nb);
constexpr uint64_t kGradIndexOff = 256;

struct OpTarget {
  Dims3 d;
  Box3 box;
};

// Statistics (op = 1 mean, 2 var) on a stage buffer or fused from a stream.
hipError_t launch_stats_stage(const void* stage_buf, int stage, const StreamView& v, int op,
                              const OpTarget& t, void* result, uint8_t* ws, hipStream_t s);
hipError_t launch_stats_fused(const StreamView& v, int via, int op, const OpTarget& t, void* result,
                              uint8_t* ws, hipStream_t s);

// Derivative (op = 3, axis in the 3D view) or gradient magnitude (op = 4).
hipError_t launch_grad_stage(const void* stage_buf, int stage, const StreamView& v, int op, int axis3,
                             const OpTarget& t, void* result, uint8_t* ws, hipStream_t s);
hipError_t launch_grad_fused(const StreamView& v, int via, int op, int axis3, const OpTarget& t,
                             void* result, uint8_t* ws, hipStream_t s);

}  // namespace hsz
