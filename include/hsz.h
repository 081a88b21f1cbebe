/*
 * hsz.h -- C ABI of libhsz: error-bounded SZp-style compression, multi-stage
 * decompression and homomorphic analytical operations on MI355X (gfx950).
 *
 * The operations follow the problem statement of Sec. III-A of "Enabling
 * Homomorphic Analytical Operations on Compressed Scientific Data with
 * Multi-stage Decompression": a compressor c = C(d, eps), a decompressor
 * split into stages D = D_m o ... o D_1 with intermediate representations
 * d^(i), and operations Q_i evaluated directly on d^(i).  Stage numbers are
 * those of Table I: 1 metadata (D_m), 2 decorrelated data (D_p),
 * 3 quantized data (D_q), 4 fully decompressed floats (D_f).
 *
 * Conventions shared by every entry point
 *   - Pointers named d_* are DEVICE pointers (HIP global memory of the
 *     current device); pointers named h_* are HOST pointers.  The caller owns
 *     every buffer; the library never allocates, frees or retains caller
 *     memory.  Device buffers must be 16-byte aligned.
 *   - 'stream' is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call that takes a stream only enqueues work on it and returns;
 *     results are valid after the stream is synchronised.
 *   - Every entry point returns HSZ_OK (0) or a negative HSZ_ERR_* code and
 *     never throws.  Argument errors are detected on the host before any
 *     work is enqueued.  Errors that depend on data (non-finite input, an
 *     out-of-range quantization integer, a corrupt block width) are
 *     detected by the kernels and recorded in a status word at the start of
 *     the call's workspace; read it with hsz_read_status().
 *   - Fields are C-order (row-major) arrays of 1, 2 or 3 dimensions, dims
 *     listed slow -> fast.  Boxes are half-open [lo, hi) per axis in the
 *     field's own axes; a NULL box means the whole field.
 *   - The library is reentrant: calls that use distinct workspaces may run
 *     concurrently on different streams.
 */
#ifndef HSZ_H
#define HSZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- codes ---------------------------------------------------------------- */
enum {
  HSZ_OK = 0,
  HSZ_ERR_INVALID_ARG = -1, /* bad pointer, size, shape, alignment, enum    */
  HSZ_ERR_BAD_STREAM = -2,  /* corrupt or truncated compressed stream       */
  HSZ_ERR_UNSUPPORTED = -3, /* op not defined at that stage, or block size  */
  HSZ_ERR_RANGE = -4,       /* |q| would exceed 2^29 - 1                    */
  HSZ_ERR_EB = -5,          /* error bound <= 0 or below the dtype spacing   */
  HSZ_ERR_NONFINITE = -6,   /* NaN or Inf in the input field                */
  HSZ_ERR_CAPACITY = -7,    /* output or workspace buffer too small         */
  HSZ_ERR_HIP = -8          /* a HIP runtime call failed (hsz_last_hip_error) */
};

enum { HSZ_F32 = 1, HSZ_F64 = 2 };                                  /* field dtype */
enum { HSZ_META = 1, HSZ_DELTA = 2, HSZ_QUANT = 3, HSZ_FLOAT = 4 }; /* Table I     */
enum { HSZ_MEAN = 1, HSZ_VAR = 2, HSZ_DERIV = 3, HSZ_GRADMAG = 4, HSZ_LAPLACIAN = 5, /* operations */
       HSZ_DIVERGENCE = 6, HSZ_CURL = 7,                    /* vector fields (below) */
       HSZ_VAR_MT = 8 };            /* spread about the metadata mean (block-mean streams) */

/* Size of the fixed header at the start of every compressed stream. */
#define HSZ_HEADER_BYTES 256

/* Parsed header of a compressed stream (host-side copy). */
typedef struct hsz_header {
  int32_t dtype;          /* HSZ_F32 / HSZ_F64                               */
  int32_t ndim;           /* 1..3                                            */
  int64_t dims[3];        /* the field's own dims, slow -> fast (ndim used)  */
  int64_t n;              /* element count                                   */
  int32_t block;          /* S: elements per block (32 or 64 on the GPU)     */
  int32_t chunk_blocks;   /* blocks per chunk-offset entry (64)              */
  double eb_abs;          /* eps: absolute error bound the stream honours    */
  double quantum;         /* Delta = 2*eps_q, d' = q * Delta                 */
  double inv_quantum;     /* 1 / Delta, the quantizer's multiplier           */
  double vmin, vmax;      /* extremes of the input field                     */
  uint32_t max_abs_q;     /* max |q| over the field                          */
  uint32_t flags;         /* 0 or one HSZ_FLAG_* decorrelation mode          */
  int64_t nb;             /* number of blocks = ceil(n / S)                  */
  int64_t nchunks;        /* ceil(nb / 64)                                   */
  uint64_t off_chunk;     /* byte offsets of the sections in the stream      */
  uint64_t off_q0;
  uint64_t off_width;
  uint64_t off_payload;
  uint64_t payload_words; /* 32-bit words in the payload section             */
  uint64_t total_bytes;   /* stream length                                   */
} hsz_header;

/* Half-open box [lo, hi) in the field's own axes (first ndim entries used). */
typedef struct hsz_box {
  int64_t lo[3];
  int64_t hi[3];
} hsz_box;

/* Result of HSZ_MEAN / HSZ_VAR (48 bytes, written to device memory).
 * On stages 2 and 3 (and the fused path via 2 or 3), s1 = sum q and
 * s2 = sum q^2 over the box are exact (s2 is a two's-complement 128-bit
 * integer s2_hi:s2_lo); mean = s1*Delta/n and var = (n*s2 - s1^2) /
 * (n*(n-1)) * Delta^2 are rounded once from the exact integers.  HSZ_MEAN
 * leaves s2 = 0 and var = NaN.  On stage 4 the sums are 0 and mean/var are
 * computed from the floats in binary64.  HSZ_VAR_MT: n; s1 = sum_b M_b S_b
 * (the block means times their sizes); s2 = sum (q - mu~)^2, exact, with
 * mu~ = round(s1 / n) (halves down); mean = mu~ * Delta; var = s2 / (n - 1)
 * * Delta^2 (NaN for n = 1). */
typedef struct hsz_stats {
  int64_t n;
  int64_t s1;
  uint64_t s2_lo;
  int64_t s2_hi;
  double mean;
  double var;
} hsz_stats;

/* ---- housekeeping ----------------------------------------------------------- */

/* Static string for a code; never NULL. */
const char *hsz_strerror(int code);

/* Library version: major*10000 + minor*100 + patch. */
int hsz_version(void);

/* Last HIP error code seen by the library on this thread (hipError_t). */
int hsz_last_hip_error(void);

/* Read the status word at the start of a workspace after the stream that
 * used it has completed: synchronises 'stream', then stores HSZ_OK or the
 * first data-dependent error any kernel of the call recorded. */
int hsz_read_status(const void *d_workspace, void *stream, int *h_status);

/* ---- compression: c = C(d, eps), Sec. IV, Alg. 1 -------------------------------
 * Quantize q = floor(x/Delta + 0.5) (binary64, the division done as a
 * multiply by 1/Delta), partition the flat array into blocks of S, keep the
 * first q of each block (q0), decorrelate p_i = q_i - q_{i-1} inside the
 * block, and encode each block as its sign bits followed by |p| at the
 * block's bit width.  eps is absolute (eb_is_rel = 0) or relative to the
 * value range max - min (eb_is_rel = 1).  The quantum is
 * Delta = 2*(eps - m*ulp(max|x| + eps)) with m = 1 (binary32) or 8
 * (binary64), so |x - x'| <= eps holds for every element after rounding. */

/* Worst-case stream size for a field (bytes), in any decorrelation mode
 * (for 2D and 3D fields the larger of the 1D and the nd partition). */
int hsz_compress_bound(int dtype, int ndim, const int64_t *h_dims, int block, uint64_t *h_bytes);

/* Workspace hsz_compress / hsz_compress_flags need (bytes), any mode.  The
 * Lorenzo modes (HSZ_FLAG_LORENZO, HSZ_FLAG_INTER_BLOCK) keep one int32
 * residual per slot of their partition there, about 4 bytes per element;
 * the other modes need a few kilobytes plus 4 bytes per 64 blocks. */
int hsz_compress_workspace(int ndim, const int64_t *h_dims, int block, uint64_t *h_bytes);

/* Workspace of one mode (flags as for hsz_compress_flags): what that mode
 * needs, at most hsz_compress_workspace().  INVALID_ARG for other flags,
 * UNSUPPORTED for HSZ_FLAG_LORENZO on a 1D field or a block other than 32 / 64. */
int hsz_compress_workspace_mode(int ndim, const int64_t *h_dims, int block, uint32_t flags, uint64_t *h_bytes);

/* Compress d_x (dtype, dims) into d_out (capacity 'cap' bytes, at least
 * hsz_compress_bound()).  The stream's length is header.total_bytes; after
 * the stream completes, read the header back (HSZ_HEADER_BYTES from d_out)
 * and check hsz_read_status(d_workspace).  block must be 32 or 64. */
int hsz_compress(const void *d_x, int dtype, int ndim, const int64_t *h_dims, double eb,
                 int eb_is_rel, int block, void *d_out, uint64_t cap, void *d_workspace,
                 uint64_t workspace_bytes, void *stream);

/* The same with header flags: HSZ_FLAG_BLOCK_MEAN selects the block-mean
 * decorrelation of HSZx (Sec. IV): the metadata of each block is its
 * integer mean M_b = sum q / S_b rounded to the nearest integer, halves
 * down, and p_i = q_i - M_b on every slot (none is forced to 0); decoding is
 * q_i = M_b + p_i.  The stage-1 buffer (and the q0 section) then holds the
 * block means, and HSZ_MEAN is defined on stage 1 (Eq. (mean_m), the whole
 * field only): mean = (sum_b M_b S_b / n) * Delta, exact integer sum in s1,
 * within eps of the mean of the decompressed field.  Streams of this mode
 * support every statistic and the materialised stages 3 and 4 of the
 * stencil and vector-field operations; fused stencils and fused vector
 * fields return HSZ_ERR_UNSUPPORTED for them (in a batch they run as
 * operations of their own). */
#define HSZ_FLAG_BLOCK_MEAN 1u
/* HSZ_FLAG_LORENZO selects HSZp-nd (Sec. IV) for 2D and 3D fields: the
 * Lorenzo residual over the whole field, p = sum over the corners c of
 * {0,1}^d of (-1)^|c| q(i - c) with q = 0 before index 0 on every axis (the
 * paper's 2D and 3D formulas), encoded in nd blocks of S elements (2D: 4x8
 * for S = 32, 8x8 for 64; 3D: 2x4x4, 4x4x4; blocks and their slots in
 * raster order, slots outside the field 0).  There is no metadata: stage 1
 * is HSZ_ERR_UNSUPPORTED and the stage-2 buffer is p int32[n] in the field's
 * layout.  A residual beyond 2^30 - 1 is HSZ_ERR_RANGE (status word).  On
 * stage 2 (materialised or fused, whole field only): HSZ_MEAN through the
 * nd weights of Sec. V-A, HSZ_VAR through the prefix sums of Alg. 4,
 * HSZ_DERIV along any axis through Eq. (derivative_Dp), HSZ_LAPLACIAN
 * through Eq. (laplacian_Dp) in any rank (the prefix sums of p over every
 * axis but one are q's backward differences along that one; the integer
 * numerator, and so the result, equals the stage-3 route's; max|q| < 2^27),
 * and divergence and curl of HSZp-nd vector fields (below); stages 3 and 4
 * take every operation of a delta stream.  The fused routes rebuild what
 * they need in the workspace (hsz_op_workspace: 4 bytes per point, 8 for
 * binary64 fields, beyond the operation's own, plus 16 planes of int32 for
 * the two-pass D_q of 3D fields with rows of at most 512 columns; the
 * Laplacian on stage 2 keeps one more int32 field per axis).  Block
 * indexes return HSZ_ERR_UNSUPPORTED for these streams; in a batch they run
 * as operations of their own. */
#define HSZ_FLAG_LORENZO 2u
/* HSZ_FLAG_INTER_BLOCK selects HSZp's decorrelation (Sec. IV, prediction
 * across block borders) for fields of any rank: p_i = q_i - q_{i-1} over the
 * field read as one flat array, q_{-1} = 0, in the 1D partition of S; no
 * metadata (stage 1 is HSZ_ERR_UNSUPPORTED, stage 2 is p int32[n]).  q is
 * the prefix sum of p over the whole field, computed device-wide in tiles
 * (stages 3 and 4 need hsz_decompress_workspace bytes).  On stage 2 (whole
 * field): HSZ_MEAN through the weights N - i of Sec. V-A and HSZ_VAR through
 * the running sum of q; derivatives need stage 3 (a 1D partition keeps no
 * multidimensional layout); stages 3 and 4 take every operation.  Batches,
 * block indexes and fused vector fields return HSZ_ERR_UNSUPPORTED. */
#define HSZ_FLAG_INTER_BLOCK 4u
int hsz_compress_flags(const void *d_x, int dtype, int ndim, const int64_t *h_dims, double eb,
                       int eb_is_rel, int block, uint32_t flags, void *d_out, uint64_t cap,
                       void *d_workspace, uint64_t workspace_bytes, void *stream);

/* The same for one slab of a larger field (a range of its slowest axis):
 * eps and the quantum are derived from the given extremes [vmin, vmax] of
 * the whole field (as hsz_compress_flags derives them from a field's own),
 * so every slab shares the whole field's quantizer and q.  The header
 * records vmin and vmax as given; a slab value outside them is
 * HSZ_ERR_EB (status word). */
int hsz_compress_range(const void *d_x, int dtype, int ndim, const int64_t *h_dims, double eb,
                       int eb_is_rel, double vmin, double vmax, int block, uint32_t flags, void *d_out,
                       uint64_t cap, void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Extremes of a field: d_out (device, 3 doubles) = {vmin, vmax, 1.0 if a
 * value is NaN or infinite else 0.0}; d_workspace of
 * hsz_extremes_workspace bytes.  Reduce the slabs' extremes to the field's
 * before hsz_compress_range. */
int hsz_extremes_workspace(uint64_t *h_bytes);
int hsz_extremes(const void *d_x, int dtype, uint64_t n, double *d_out, void *d_workspace,
                 uint64_t workspace_bytes, void *stream);

/* Parse and validate a header held in HOST memory.  'len' is the number of
 * stream bytes the caller holds (at least HSZ_HEADER_BYTES); the stream's
 * own length must not exceed 'len_stream' (pass the device buffer size). */
int hsz_read_header(const void *h_bytes, uint64_t len, uint64_t len_stream, hsz_header *h_out);

/* ---- multi-stage decompression: d^(i) = D_i(...D_1(c)), Alg. 2 ---------------
 * Stage buffer layouts (bytes from hsz_stage_bytes):
 *   HSZ_META  : q0 int32[nb]                   (first q of each block)
 *   HSZ_DELTA : p int32[n], then q0 int32[nb]  (p = 0 at each block's slot 0)
 *   HSZ_QUANT : q int32[n]
 *   HSZ_FLOAT : d' = (dtype)(q * Delta), dtype[n] */
int hsz_stage_bytes(const hsz_header *h, int stage, uint64_t *h_bytes);

/* Workspace hsz_decompress_to_stage needs for this stream and stage: 256
 * bytes (the status word), plus for stages 3 and 4 the tile sums of
 * HSZ_FLAG_INTER_BLOCK streams, or for HSZ_FLAG_LORENZO streams of 3D
 * fields whose rows hold at most 512 columns (a multiple of 4) the totals
 * of the z segments of the two-pass decode (16 planes of int32). */
int hsz_decompress_workspace(const hsz_header *h, int stage, uint64_t *h_bytes);

/* Decode the stream d_c (device) to 'stage' into d_out (capacity 'cap').
 * d_workspace (hsz_decompress_workspace bytes) receives the status word: a block whose
 * width or payload disagrees with the chunk table is reported as
 * HSZ_ERR_BAD_STREAM and decoded as constant q0 (never read out of bounds). */
int hsz_decompress_to_stage(const void *d_c, const hsz_header *h, int stage, void *d_out,
                            uint64_t cap, void *d_workspace, uint64_t workspace_bytes,
                            void *stream);

/* ---- operations Q_i(d^(i)), Sec. V ------------------------------------------
 * op = HSZ_MEAN, HSZ_VAR : result = one hsz_stats (Eq. (var), sample
 *      variance with N - 1; the standard deviation is sqrt(var)).
 * op = HSZ_VAR_MT        : result = one hsz_stats; the standard deviation
 *      on D_p of HSZx (Sec. V-A): each term of Eq. (var) is taken about the
 *      integer mean mu~ of the block means instead of the exact mean, so
 *      var = sum_b sum_{p in D_p[B_b]} (p + M_b - mu~)^2 / (N - 1) * Delta^2
 *      (the sample variance plus N (mu - mu~)^2 / (N - 1) Delta^2).  Block-
 *      mean streams only, the whole field only, via stage 2 (on_stage and
 *      fused) or stage 3 (fused); anything else HSZ_ERR_UNSUPPORTED.
 * op = HSZ_DERIV (axis)  : result = derivative along 'axis' (0 = slowest)
 *      at every point of the box, field dtype, box-shaped C order.
 * op = HSZ_GRADMAG       : result = sqrt(sum over axes of derivative^2).
 * op = HSZ_LAPLACIAN     : result = Laplacian, Eq. (laplacian) summed over
 *      the field's axes: sum_k (d_{-1} + d_{+1} - 2 d) along axis k, unit
 *      spacing, the end value standing in for the missing neighbour at the
 *      two ends of an axis (an axis of length 1 adds 0).  On stage 3 (and
 *      the fused path via 3) the integer numerator sum_k (q_{-1} + q_{+1} -
 *      2 q) is exact and scaled once by Delta (Eq. (laplacian_Dq)); this
 *      needs max|q| < 2^27 (else HSZ_ERR_UNSUPPORTED; stage 4 has no limit).
 *      Stage 2: HSZp-nd streams only (whole field, see HSZ_FLAG_LORENZO);
 *      delta and block-mean streams: HSZ_ERR_UNSUPPORTED (a 1D partition
 *      keeps no multidimensional neighbours, Sec. V-B).
 * Derivatives follow Eq. (derivatives): central differences (q_{+1} -
 * q_{-1}) * Delta/2 inside the field and one-sided (q_1 - q_0) * Delta at
 * its ends, unit spacing, neighbours taken from the whole field even when
 * they lie outside the box; an axis of length 1 contributes 0.
 * Stage support: MEAN/VAR on stages 2, 3, 4; DERIV/GRADMAG on 2, 3, 4;
 * LAPLACIAN on 3, 4 (and 2 for HSZp-nd); stage 1 supports none
 * (HSZ_ERR_UNSUPPORTED), as Table II lists for SZp. */

/* Workspace an operation needs (bytes; at least 256). */
int hsz_op_workspace(const hsz_header *h, int op, uint64_t *h_bytes);

/* Operation on a materialised stage buffer produced by
 * hsz_decompress_to_stage (d_stage, 'stage'). */
int hsz_op_on_stage(const void *d_stage, const hsz_header *h, int stage, int op, int axis,
                    const hsz_box *h_box, void *d_result, uint64_t cap, void *d_workspace,
                    uint64_t workspace_bytes, void *stream);

/* The same operation computed directly from the compressed stream d_c in one
 * pass, the intermediate stage 'via' (2, 3 or 4) existing only in registers
 * and on-chip memory (the blockwise pipeline of Alg. 3).  Results equal
 * hsz_op_on_stage on the same stage bit for bit for integer sums, within
 * rounding for floating-point results. */
int hsz_op_fused(const void *d_c, const hsz_header *h, int via, int op, int axis,
                 const hsz_box *h_box, void *d_result, uint64_t cap, void *d_workspace,
                 uint64_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops that must not call the allocator): hsz_op_fused
 * with its workspace taken from a fixed device array the library owns, of
 * HSZ_NOALLOC_SCRATCH_BYTES per device, held until the process ends.  The
 * caller passes the stream, the result buffer and, optionally, d_status
 * (device, 4-byte aligned, or NULL): after the operation the call's status
 * word (HSZ_OK or the first data-dependent error) is copied there.  The
 * call itself never allocates or frees memory; its first call on a device
 * resolves the array's device address (with that device current).
 * HSZ_ERR_CAPACITY when hsz_op_workspace(h, op) exceeds the array (e.g. a
 * gradient of more than about 8.4 million blocks, or fused HSZp-nd routes
 * beyond about 4 million points).  Every call on a device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (different streams, or host threads) race and must be serialised
 * by the caller. */
#define HSZ_NOALLOC_SCRATCH_BYTES (16u << 20)
int hsz_op_fused_noalloc(const void *d_c, const hsz_header *h, int via, int op, int axis,
                         const hsz_box *h_box, void *d_result, uint64_t cap, int *d_status,
                         void *stream);

/* ---- out of core: a field as compressed slabs in host memory (Alg. 3) -----
 * h_slabs[k] (HOST memory; pinned memory lets the copies overlap) holds the
 * stream of slab k, hdrs[k] its header: consecutive ranges of the field's
 * slowest axis in order, compressed by hsz_compress_range with the whole
 * field's extremes (same dtype, rank, block, decorrelation, quantum and
 * other dims; delta, block-mean, HSZp-nd or HSZp streams: the last two are
 * reduced or decoded slab by slab through hsz_op_fused /
 * hsz_decompress_to_stage, whose workspace hsz_ooc_workspace includes).
 * The slabs pass through the device a few at a time: at most three
 * compressed slabs, and for stencils two windows of D_q and two result
 * slabs.
 *   op = HSZ_MEAN / HSZ_VAR, via HSZ_DELTA or HSZ_QUANT: h_result = one
 *        hsz_stats of the whole field, from exact per-slab integer sums.
 *   op = HSZ_DERIV (axis) / HSZ_GRADMAG / HSZ_LAPLACIAN, via HSZ_QUANT:
 *        h_result (HOST, n * dtype bytes) = the whole field's result; each
 *        slab is decoded between one-plane halos from its neighbours (the
 *        window of Alg. 3), so it equals the operation on the whole field.
 * d_workspace: hsz_ooc_workspace bytes.  Synchronous: returns when the
 * result is in h_result (or a status code of the stream decoding). */
int hsz_ooc_workspace(const hsz_header *const *hdrs, int nslabs, int op, uint64_t *h_bytes);
int hsz_ooc_op(const void *const *h_slabs, const hsz_header *const *hdrs, int nslabs, int via, int op,
               int axis, void *h_result, uint64_t result_bytes, void *d_workspace,
               uint64_t workspace_bytes, void *stream);

/* ---- vector fields: divergence and curl, Sec. III-B and Sec. V-C -----------------
 * A vector field of an n-dimensional grid (n = 1..3) is held as n streams of
 * the same dims, dtype and block size, component k paired with the field's
 * own axis k (delta_x = axis 0, the slowest).  Each component keeps its own
 * error bound and quantum.  The derivative is the one of HSZ_DERIV (central
 * differences inside, one-sided at the ends of an axis, 0 on an axis of
 * length 1), taken over the whole field even where it lies outside the box.
 *   HSZ_DIVERGENCE (Eq. (divergence)): sum_k delta_k F_k; one result.
 *   HSZ_CURL (Eq. (curl)), n = 2: delta_1 F_0 - delta_0 F_1 (as printed);
 *     one result.  n = 3: three results, (delta_2 F_1 - delta_1 F_2,
 *     delta_0 F_2 - delta_2 F_0, delta_1 F_0 - delta_0 F_1), the last being
 *     the 2D formula.
 * Results are box-shaped C-order arrays of the field dtype, each at
 * d_result[o] (16-byte aligned, 'cap' bytes each).  On the quantized
 * stage every term is an exact integer numerator of one component times
 * that component's Delta/2, the terms of a result summed in binary64 in a
 * fixed order and rounded once; on the float stage the same differences are
 * taken on the decompressed values in the field's precision.  On stage 2
 * (HSZp-nd components, whole field; on stage buffers, or fused via 2 from
 * the streams, each decoded to D_p in the workspace): every term's integer
 * numerator comes from the component's p through Eq. (derivative_Dp) (the
 * pair p_i + p_{i+1} along the term's axis, prefix-summed over the other
 * axes, one-sided at the ends), and the terms are combined exactly as on
 * stage 3, so the results equal the stage-3 route's bit for bit.  Stage 1,
 * and stage 2 of delta and block-mean streams: HSZ_ERR_UNSUPPORTED (the 1D
 * partition keeps no multidimensional neighbours, Sec. V-B).  Arrays
 * d_stage / d_c / h hold ncomp entries. */

/* Workspace of a vector-field operation (status words and one block index
 * per component; for HSZp-nd components also ncomp + 6 (3D) or ncomp (1D,
 * 2D) int32 fields for the stage-2 route). */
int hsz_vector_workspace(const hsz_header *const *h, int ncomp, uint64_t *h_bytes);

/* On materialised stage buffers (stage = HSZ_QUANT or HSZ_FLOAT, or
 * HSZ_DELTA for HSZp-nd components; one buffer per component from
 * hsz_decompress_to_stage). */
int hsz_vector_op_on_stage(const void *const *d_stage, const hsz_header *const *h, int ncomp, int stage,
                           int op, const hsz_box *h_box, void *const *d_result, uint64_t cap,
                           void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Straight from the component streams through D_q (via = HSZ_QUANT, delta
 * streams): each component's planes are decoded on chip in turn; the result
 * equals hsz_vector_op_on_stage on the quantized stage bit for bit.  HSZp-nd
 * components through D_p (via = HSZ_DELTA): each decoded to p in the
 * workspace, then the stage-2 route. */
int hsz_vector_op_fused(const void *const *d_c, const hsz_header *const *h, int ncomp, int via, int op,
                        const hsz_box *h_box, void *const *d_result, uint64_t cap, void *d_workspace,
                        uint64_t workspace_bytes, void *stream);

/* ---- batches: many fields, boxes and operations in one pass ------------------
 * One persistent launch per kernel family works through a device table of
 * (job, unit) pairs: statistics units are 64-block chunks (whole fields) or
 * groups of 64 block segments (boxes); gradient units are tiles.  Statistics
 * are accumulated as exact integers with 64-bit atomics, so every job's
 * result is bit-identical to hsz_op_fused on the same stream, box and stage,
 * whatever else is in the batch.  The kernels take delta streams with
 * HSZ_MEAN / HSZ_VAR via HSZ_DELTA or HSZ_QUANT and HSZ_DERIV / HSZ_GRADMAG
 * via HSZ_QUANT or HSZ_FLOAT.  Every other item hsz_op_fused accepts
 * (HSZp-nd, HSZp and block-mean streams, HSZ_LAPLACIAN, HSZ_VAR_MT,
 * statistics via HSZ_FLOAT) runs in the pass as an operation of its own,
 * with its workspace inside the batch's and its status word merged into the
 * batch's; its refusals (hsz_op_fused's codes) are the batch's.  Vector
 * operations are HSZ_ERR_INVALID_ARG. */
typedef struct hsz_work {
  const void *d_c;      /* compressed stream (device, 16-byte aligned)          */
  const hsz_header *h;  /* its parsed header (host)                             */
  int32_t op;           /* an operation of one stream (HSZ_MEAN .. HSZ_VAR_MT)   */
  int32_t via;          /* the stage held on chip (see above)                   */
  int32_t axis;         /* HSZ_DERIV: axis in the field's own order             */
  int32_t use_box;      /* 0: the whole field; 1: 'box'                         */
  hsz_box box;
  void *d_result;       /* hsz_stats, or the box-shaped result (16-byte aligned) */
  uint64_t result_bytes;
  const void *d_index;  /* optional: the stream's block index (hsz_block_index);
                           NULL builds one in the workspace for gradient jobs  */
} hsz_work;

/* Block index of a stream: for every block, the offset of its payload
 * within its 64-block chunk (uint16[nb]).  With it any block is located by
 * two independent loads (chunk table + index) instead of a prefix over the
 * chunk's widths; streams that stay resident (serving) build it once. */
int hsz_block_index_bytes(const hsz_header *h, uint64_t *h_bytes);
int hsz_block_index(const void *d_c, const hsz_header *h, void *d_index, uint64_t cap, void *stream);

/* Launch shape of a batch; zeros select the defaults. */
typedef struct hsz_tuning {
  int32_t stats_waves_per_cu;  /* statistics launch: waves per compute unit (8)   */
  int32_t grad_groups_per_cu;  /* gradient launch: workgroups per compute unit (4) */
  int32_t grad_tz;             /* planes per gradient tile; 0: 32, halved (to 4 at
                                  least) while a job has fewer than 256 tiles        */
  int32_t separate_stats;      /* 1: statistics never share a gradient job's decode
                                  (by default a mean/variance job over the same stream
                                  and box as a gradient job through D_q is summed
                                  inside that job's tiles; results are identical)  */
  int32_t graph_replay;        /* plans: 1 replays the HIP graph captured at create;
                                  0 (default) enqueues the pass's kernels directly,
                                  which reaches the GPU sooner for these few-kernel
                                  passes (the work table is on the device either way) */
  int32_t grad_tile_x;         /* workgroup shape of binary32 gradient-magnitude jobs
                                  through D_q that admit the narrow tiles (max|q| < 8192,
                                  blocks of 32, rows on block boundaries): 0 (default) the
                                  widest admitted -- 512 columns x 16 rows by 512 threads
                                  for boxes wider than 256 columns with a width divisible
                                  by 8, else 256 x 16 by 256 threads; 256 always the
                                  latter; -1 the general tile (any stream).  The values
                                  are bit-identical whichever tile runs */
} hsz_tuning;

/* Workspace a batch needs (bytes). */
int hsz_batch_workspace(const hsz_work *h_items, int n, uint64_t *h_bytes);

/* Validate, copy the work table into d_workspace and enqueue the pass. */
int hsz_batch_run(const hsz_work *h_items, int n, const hsz_tuning *h_tune, void *d_workspace,
                  uint64_t workspace_bytes, void *stream);

/* A batch prepared once and launched many times: its work table is
 * uploaded (synchronously) by hsz_plan_create and by hsz_plan_update, never
 * by a launch, and its kernels are captured as a HIP graph.  A launch
 * enqueues the kernels, or replays the graph when the tuning's
 * graph_replay is set.  'stream' must be a created
 * (non-null) stream.  hsz_plan_update rewrites the table for a batch of the
 * same structure (same jobs per kernel variant, the same classes with
 * separately summed statistics, no larger index or staging needs) -- new
 * streams, boxes, axes and result buffers; it first waits for the previous
 * replay to finish (a plan holding operations of their own captures its
 * graph again with the new items).  The workspace belongs to the plan
 * until hsz_plan_destroy. */
typedef struct hsz_plan hsz_plan;
int hsz_plan_create(const hsz_work *h_items, int n, const hsz_tuning *h_tune, void *d_workspace,
                    uint64_t workspace_bytes, void *stream, hsz_plan **out);
int hsz_plan_update(hsz_plan *plan, const hsz_work *h_items, int n);
int hsz_plan_launch(hsz_plan *plan, void *stream);
void hsz_plan_destroy(hsz_plan *plan);

/* ---- contexts: persistent scratch, staging and streams for one device ------------
 * The decompression pipeline of Sec. III-A (compress once, then decode to a
 * stage and operate there, many times) issued without allocation or hidden
 * synchronisation.  A context belongs to the device current at
 * hsz_ctx_create and owns:
 *   - a device scratch buffer (scratch_bytes; hsz_ctx_reserve grows it) that
 *     serves as the workspace of the calls made through the context;
 *   - a ring of pinned host memory (host_bytes) through which batch work
 *     tables reach the device with asynchronous copies (a region is reused
 *     once the copy that read it has completed; a table larger than the
 *     ring is HSZ_ERR_CAPACITY);
 *   - the copy stream and events of the out-of-core pipeline;
 *   - launch shapes chosen by an autotuner, per batch shape class (a string
 *     key the caller forms; hsz_ctx_set_tuning / hsz_ctx_get_tuning).
 * Work issued through a context runs in the order it is issued: each call
 * orders itself after the context's previous call (device-side waits, never
 * a host wait), so calls on different streams do not race on the scratch.
 * hsz_ctx_scratch hands the scratch to the plain entry points (as their
 * d_workspace) for callers that order those calls themselves.
 * hsz_ctx_destroy waits for the context's outstanding work, then frees it. */
typedef struct hsz_ctx hsz_ctx;
int hsz_ctx_create(uint64_t scratch_bytes, uint64_t host_bytes, hsz_ctx **out);
void hsz_ctx_destroy(hsz_ctx *ctx);
/* Grow the scratch to at least 'bytes' (waits for the context's work first;
 * a no-op when it is already that large). */
int hsz_ctx_reserve(hsz_ctx *ctx, uint64_t bytes);
int hsz_ctx_scratch(hsz_ctx *ctx, void **d_scratch, uint64_t *bytes);
/* Launch shape stored under 'key' (NUL-terminated, < 1024 bytes);
 * hsz_ctx_get_tuning returns HSZ_ERR_INVALID_ARG for an unknown key. */
int hsz_ctx_set_tuning(hsz_ctx *ctx, const char *key, const hsz_tuning *h_tune);
int hsz_ctx_get_tuning(hsz_ctx *ctx, const char *key, hsz_tuning *h_tune);
/* hsz_batch_run with the context's scratch as workspace (HSZ_ERR_CAPACITY
 * when it holds less than hsz_batch_workspace) and its table copied from
 * the pinned ring: returns once the pass is enqueued on 'stream'.  The
 * status word is at the start of the scratch (hsz_read_status); d_status
 * (device int, 4-byte aligned, or NULL) also receives it when the pass
 * completes. */
int hsz_ctx_batch_run(hsz_ctx *ctx, const hsz_work *h_items, int n, const hsz_tuning *h_tune,
                      int *d_status, void *stream);
/* hsz_ooc_op enqueued on 'stream' and the context's copy stream, with the
 * context's scratch as workspace (HSZ_ERR_CAPACITY below hsz_ooc_workspace):
 * returns once the pass is enqueued.  Every part of it, the device-to-host
 * copies of the result included, completes before any work the caller
 * enqueues on 'stream' afterwards (record an event there to wait for it).
 * Statistics are combined on the device, exactly as hsz_ooc_op combines
 * them, and copied into h_result.  h_slabs and h_result should be pinned
 * host memory: a copy from or to pageable memory can make the call wait.
 * d_status (device int, or NULL): after completion HSZ_OK or the first
 * data-dependent error of the pass. */
int hsz_ooc_op_async(hsz_ctx *ctx, const void *const *h_slabs, const hsz_header *const *hdrs,
                     int nslabs, int via, int op, int axis, void *h_result, uint64_t result_bytes,
                     int *d_status, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HSZ_H */
