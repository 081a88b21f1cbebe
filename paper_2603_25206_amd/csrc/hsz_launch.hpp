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
  uint32_t flags;  // bit 0: block-mean decorrelation (metadata = block means)
};

// ---- compression -------------------------------------------------------------
struct CompressArgs {
  const void* x;
  int dtype;
  int ndim;
  int64_t dims[3];  // 3D view
  double eb;
  int eb_is_rel;
  uint32_t flags;  // bit 0: block-mean decorrelation
  int fixed_range = 0;  // quantizer parameters from [vmin, vmax] (a slab of a larger field)
  double vmin = 0.0, vmax = 0.0;
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

// ---- batches -----------------------------------------------------------------------
// A set of contiguous flat ranges ("rows"): row r = iz*nry + iy starts at
// base + iz*sz + iy*sy and has len elements.
struct Rows {
  int64_t nrz, nry, len, base, sz, sy;
  __host__ __device__ int64_t count() const { return nrz * nry; }
  __device__ int64_t start(int64_t r) const { return base + (r / nry) * sz + (r % nry) * sy; }
};

// One statistics job of a batch (integer routes only).
struct StatsJob {
  StreamView v;
  Rows rows;        // the box as contiguous rows
  int64_t per_row;  // blocks a row can touch
  int32_t op, via, whole;
  int32_t acc;          // accumulator slot (its own index, or the slot it shares)
  void* out;            // hsz_stats (device)
  const uint16_t* rel;  // block index, or null (offsets from the widths)
};
// Exact accumulator of one statistics slot: sum q, count, and sum q^2 as
// s2hi * 2^32 + s2lo, so that every wave adds with plain (no-return) 64-bit
// atomics: its low 32 bits to s2lo, the rest to s2hi.  A slot is
// kAccStripes consecutive accumulators; a wave adds to one chosen by its
// index, which keeps simultaneous atomics on one address few.
struct BatchAcc {
  int64_t s1, cnt;
  uint64_t s2lo, s2hi;
};
constexpr int kAccStripes = 64;
// Zero 'slots' accumulator slots at acc, the status word and the two words
// after it (the live status and the done count of a batch that finishes
// itself).
hipError_t launch_batch_reset(BatchAcc* acc, int slots, int* status, hipStream_t s);
hipError_t launch_batch_stats(int S, const StatsJob* jobs, const int64_t* unit_start, const int64_t* counts,
                              int kmax, BatchAcc* acc, int* status, int grid, hipStream_t s);
// Finish the statistics jobs of both block-size classes (n[c] jobs each, one
// wave per job summing its slot's stripes).
// *out = *status (device ints), ordered on 's'
hipError_t launch_copy_status(const int* status, int* out, hipStream_t s);
// *dst takes *src's error code if *dst has none
hipError_t launch_merge_status(const int* src, int* dst, hipStream_t s);
// K per-slab statistics records (48 bytes each, the hsz_stats layout) of one
// field combined exactly into one record at 'out' (device)
hipError_t launch_stats_combine(const void* records, int K, int op, double quantum, void* out, hipStream_t s);
hipError_t launch_batch_finalize(const StatsJob* const jobs[2], const int64_t* const counts[2],
                                 const BatchAcc* const acc[2], const int n[2], hipStream_t s);

// Statistics (op = 1 mean, 2 var, 8 var about the integer metadata mean of a
// block-mean stream) on a stage buffer or fused from a stream.
constexpr int kOpVarMetaMean = 8;
hipError_t launch_stats_stage(const void* stage_buf, int stage, const StreamView& v, int op,
                              const OpTarget& t, void* result, uint8_t* ws, hipStream_t s);
hipError_t launch_stats_fused(const StreamView& v, int via, int op, const OpTarget& t, void* result,
                              uint8_t* ws, hipStream_t s);

// One fused-gradient job: a box of one stream, its block-offset index, the
// z-extent of a tile (tz) and the staging rows needed (kmax).
struct GradJob {
  StreamView v;
  const uint16_t* rel;
  Dims3 d;
  Box3 b;
  int axis, tz, kmax;
  double halfq;
  void* out;
  // Statistics sharing this job's decode (batches only): the exact sums of
  // q over the box go to *acc.  acc_mode 0: none; 1: max|q| < 2^16 (32-bit
  // squares); 2: any q.
  void* acc;
  int acc_mode;
};

hipError_t launch_batch_block_index(const GradJob* jobs, const int64_t* chunk_start, const int64_t* counts, int grid,
                                    hipStream_t s);
// acc: the variant's shared-statistics mode (GradJob::acc_mode of all its jobs)
hipError_t launch_batch_grad(int S, int via, int op, int dtype, int acc, const GradJob* jobs,
                             const int64_t* tile_start, const int64_t* counts, int kmax, int grid, int* status,
                             hipStream_t s);
size_t batch_grad_lds(int S, int dtype, int via, int kmax);
int grad_tiles(const Box3& b, int tz);  // tiles of one fused-gradient job
int grad_kmax(const StreamView& v);     // staging rows a stream needs
int stats_kmax(const StreamView& v);

// Binary32 gradient magnitude through D_q with four columns per lane
// (grad4.hip): streams with max|q| < 8192 and boxes whose rows start on block
// boundaries (q4_eligible); the same values as the general tile, bit for bit.
bool q4_eligible(const StreamView& v, int via, int op, const Dims3& d, const Box3& b);
int q4_txl(const Box3& b);                            // column tile: 256 or 512 (widest admitted)
int64_t q4_tiles(const Box3& b, int tz, int txl);     // tiles of a box with txl-column tiles
int q4_tz(const Box3& b);                             // planes per tile of a single launch
int q4_kmax(int S);
hipError_t launch_gradmag_q4(const GradJob& job, int* status, hipStream_t s);
hipError_t launch_batch_gradmag_q4(int S, int txl, int acc, const GradJob* jobs, const int64_t* tile_start,
                                   const int64_t* counts, int grid, int* status, hipStream_t s);
// The 512-column tile with every statistic of the batch summed in its tiles,
// finishing the batch itself (BatchTail, hsz_stats.hpp): its last workgroup
// writes the statistics records, zeroes the accumulators and publishes the
// status word, so no reset or finalize kernel runs around it once the
// accumulators, the live word and the count are zero.
struct BatchTail;
hipError_t launch_batch_gradmag_q8_tail(const GradJob* jobs, const int64_t* tile_start, const int64_t* counts,
                                        int grid, const BatchTail& tail, hipStream_t s);
size_t batch_gradmag_q4_lds(int S, int txl);

// Derivative (op = 3, axis in the 3D view) or gradient magnitude (op = 4).
hipError_t launch_grad_stage(const void* stage_buf, int stage, const StreamView& v, int op, int axis3,
                             const OpTarget& t, void* result, uint8_t* ws, hipStream_t s);
hipError_t launch_grad_fused(const StreamView& v, int via, int op, int axis3, const OpTarget& t,
                             void* result, uint8_t* ws, hipStream_t s);

// ---- vector fields: divergence and curl, one stream (or buffer) per component ----
constexpr int kOpDivergence = 6, kOpCurl = 7;
struct VecJob {
  StreamView v[3];         // component streams (fused route)
  const uint16_t* rel[3];  // their block indexes (filled by launch_vector_fused)
  const void* buf[3];      // component stage buffers (stage route)
  double halfq[3];         // Delta/2 of each component
  Dims3 d;
  Box3 b;
  int nc, op, tz, kmax;    // components (= field dims), kOpDivergence / kOpCurl
  void* out[3];            // result buffers (1, or 3 for the curl of a 3D field)
};
// status words, then one block index per component
uint64_t vector_workspace_bytes(const int64_t* nb, int nc);
// the terms of an operation (component c, view axis a, sign s, output o) in
// the order the kernels add them; returns their count (0: none)
int vector_terms(int op, int nc, int* c, int* a, int* s, int* o, int* nout);
hipError_t launch_vector_stage(const VecJob& j, int stage, int dtype, hipStream_t s);
hipError_t launch_vector_fused(const VecJob& j, uint8_t* ws, hipStream_t s);

}  // namespace hsz
