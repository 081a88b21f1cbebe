/*
 * hsz_oracle.c -- plain, slow, obviously correct CPU reference for the
 * homomorphic SZp path (error-bounded compression, multi-stage
 * decompression, and analytical operations on the decompressed field).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT THE PRODUCT.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library: it is a
 * second, independent implementation of the same arithmetic and the same
 * byte format, written for a reader who checks it against the paper by eye.
 *
 * What it follows (paper: "Enabling Homomorphic Analytical Operations on
 * Compressed Scientific Data with Multi-stage Decompression"):
 *   - Sec. IV, quantization paragraph and Alg. 1 (quantize loop):
 *       q_i = round(d_i / (2 eps)),  d'_i = 2 q_i eps,  |d_i - d'_i| <= eps.
 *   - Sec. IV, data partition / metadata / decorrelation paragraphs and
 *     Alg. 1 (block loop), SZp flavour: blocks of S consecutive elements of
 *     the field read as a flat array, metadata = first q of the block,
 *     p_i = q_i - q_{i-1} inside the block.
 *   - Sec. IV, encoding paragraph and Alg. 1 (encode): per block the sign
 *     bits are stored together, then each |p| with the block's bit width
 *     (enough bits for the largest |p|).
 *   - Alg. 2: partial decompression to decorrelated data, quantized data, or
 *     floats (decode, recorrelate, dequantize).
 *   - Sec. III-B, Eq. (var), Eq. (derivatives), Eq. (laplacian),
 *     Eq. (divergence) and Eq. (curl): mean, standard deviation (N-1),
 *     central differences, the five-point (2D) / seven-point (3D) Laplacian,
 *     divergence and curl of vector fields.  The operations here are
 *     computed plainly on the fully decompressed field, never with
 *     homomorphic shortcuts.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   R1 round() is round-half-up: q = floor(t + 0.5).  The worked example of
 *      Sec. IV (HSZx-nd paragraph) reproduces only under this rule.
 *   R2 t = x * (1/Delta) in IEEE binary64 with no fused multiply-add.
 *   R3 the quantum is Delta = 2*eps_q with eps_q = eps - m*ulp(max|x| + eps),
 *      m = 1 for binary32 fields and m = 8 for binary64 fields, so that the
 *      bound |x - x'| <= eps of Sec. III-A holds after floating-point
 *      rounding.  A relative bound is eps = rel * (max - min) (value-range
 *      relative, Sec. VI-B); a constant field uses rel * |max|, and an
 *      all-zero field uses rel.
 *   R4 slot 0 of every block holds p = 0 (its q is the metadata q0).
 *   R5 width w = bit length of max |p| over the block (0 if all zero); a
 *      block with w = 0 stores nothing.  A block with w > 0 stores
 *      ceil(S/32) sign words then ceil(S*w/32) magnitude words; element i
 *      owns stream bits [i*w, i*w + w), bit k of the stream is bit k%32 of
 *      word k/32 (little-endian, least significant bit first).
 *   R6 |q| <= 2^29 - 1, else the compressor reports a range error.
 *   R7 derivatives use unit spacing; interior points use central
 *      differences, the two ends of an axis use one-sided differences
 *      (the rule of numpy.gradient with edge_order=1); an axis of length 1
 *      has derivative 0.  Gradient magnitude = sqrt(sum_k g_k^2).
 *   R10 block-mean decorrelation (HSZx, Sec. IV: p_i = q_i - mean(B_i0)),
 *      selected by bit 0 of the header flags: the metadata of block b is the
 *      integer mean M_b = round_half_down(sum of its q / S_b), i.e.
 *      ceil((2 sum - S_b) / (2 S_b)) -- the printed M_1 = 5 for a block
 *      mean of 5.5 and the bound |sum/S_b - M_b| <= 1/2 used by the bias
 *      analysis of the metadata mean both hold; p_i = q_i - M_b on every
 *      slot (none is forced to 0); q_i = M_b + p_i.  Padding slots of the
 *      last block (past n) hold p = 0 as in the delta mode.
 *   R11 the integer mean of the standard deviation on D_p for HSZx
 *      (Sec. V-A), mu~ = round(sum_b M_b S_b / N), rounds halves down like
 *      the block means of R10 (the paper's example, 16 / 8 = 2, has no
 *      tie); the spread is taken over the whole field only, since mu~ comes
 *      from the metadata of every block.
 *   R12 HSZp-nd (Sec. IV): bit 1 of the header flags.  Decorrelation is
 *      the Lorenzo residual over the whole field (prediction crosses block
 *      boundaries, as HSZp's does), with q = 0 outside the field:
 *      p = sum over the corners c of {0,1}^3 of (-1)^|c| q(i - c) in the
 *      3D view (a 2D field is one plane, so this is the printed 2D form).
 *      The partition for encoding is into blocks of S = 2^k elements shaped
 *      by splitting k over the axes as evenly as possible, the faster axes
 *      taking the remainder (2D: 4x8 for S = 32, 8x8 for 64; 3D: 2x4x4
 *      and 4x4x4), blocks and their slots in raster order, slots outside
 *      the field p = 0.  No metadata is stored (the q0 section is empty);
 *      stage 2 is p in the field's own layout.  For 2D and 3D fields only.
 *   R14 HSZp (Sec. IV, inter-block prediction): bit 2 of the header flags.
 *      p_i = q_i - q_{i-1} over the field read as one flat array, across
 *      block borders, with q_{-1} = 0 (so p_0 = q_0); the 1D partition of S
 *      elements; no metadata.  This is R12's residual in one dimension, and
 *      it applies to fields of any rank.
 *   R13 the residual of HSZp-nd sums up to eight quantization integers, so
 *      besides R6 it must satisfy |p| <= 2^30 - 1 (the delta mode's width
 *      limit), else the compressor reports a range error.
 *   R8 the Laplacian of Eq. (laplacian) on n axes is the sum over the axes
 *      of d_{-1} + d_{+1} - 2 d (unit spacing); at the two ends of an axis
 *      the missing neighbour is the end value itself (the field mirrored
 *      about its last sample), so an axis of length 1 adds 0.
 *   R9 divergence and curl, Eq. (divergence) and Eq. (curl), use the
 *      derivative of R7 with component k of the vector field paired with
 *      the field's own axis k (delta_x = axis 0).  Divergence =
 *      sum_k delta_k F_k.  Curl of a 2D field = delta_1 F_0 - delta_0 F_1
 *      (Eq. (curl) as printed); of a 3D field, the vector
 *      (delta_2 F_1 - delta_1 F_2, delta_0 F_2 - delta_2 F_0,
 *       delta_1 F_0 - delta_0 F_1), whose last component is the 2D
 *      formula.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- error codes (the same numbers the library reports) ---------------- */
#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_STREAM (-2)
#define OR_ERR_UNSUPPORTED (-3)
#define OR_ERR_RANGE (-4)
#define OR_ERR_EB (-5)
#define OR_ERR_NONFINITE (-6)
#define OR_ERR_CAPACITY (-7)

/* ---- byte format constants --------------------------------------------- */
#define OR_HEADER_BYTES 256u
#define OR_SECTION_ALIGN 256u
#define OR_CHUNK_BLOCKS 64u
#define OR_QMAX 536870911 /* 2^29 - 1 */
#define OR_PMAX 1073741823 /* 2^30 - 1 (R13) */
#define OR_FLAG_MEAN 1u
#define OR_FLAG_LORENZO 2u
#define OR_FLAG_INTER 4u

typedef struct {
  uint32_t dtype;   /* 1 = binary32, 2 = binary64 */
  uint32_t ndim;    /* 1..3 */
  uint64_t dims[3]; /* slow -> fast, unused = 1 (leading) */
  uint64_t n;
  uint32_t block;   /* S */
  uint32_t chunk_blocks;
  double eb_abs;    /* user bound eps (absolute) */
  double quantum;   /* Delta = 2 eps_q */
  double inv_quantum;
  double vmin, vmax;
  uint32_t max_abs_q;
  uint32_t flags;
  uint64_t nb, nchunks;
  uint64_t off_chunk, off_q0, off_width, off_payload;
  uint64_t payload_words;
  uint64_t total_bytes;
} or_header;

/* little-endian field writers/readers, byte by byte */
static void put_u16(uint8_t *p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put_u32(uint8_t *p, uint32_t v) { for (int k = 0; k < 4; k++) p[k] = (uint8_t)(v >> (8 * k)); }
static void put_u64(uint8_t *p, uint64_t v) { for (int k = 0; k < 8; k++) p[k] = (uint8_t)(v >> (8 * k)); }
static void put_f64(uint8_t *p, double d) { uint64_t v; memcpy(&v, &d, 8); put_u64(p, v); }
static uint16_t get_u16(const uint8_t *p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t get_u32(const uint8_t *p) { uint32_t v = 0; for (int k = 3; k >= 0; k--) v = (v << 8) | p[k]; return v; }
static uint64_t get_u64(const uint8_t *p) { uint64_t v = 0; for (int k = 7; k >= 0; k--) v = (v << 8) | p[k]; return v; }
static double get_f64(const uint8_t *p) { uint64_t v = get_u64(p); double d; memcpy(&d, &v, 8); return d; }

static uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }
static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

/* Block shape of the HSZp-nd partition (R12) in the 3D view (slow -> fast);
 * 0 if ndim or S does not allow one. */
static int nd_block_shape(uint32_t ndim, uint32_t S, uint64_t b[3]) {
  if (ndim < 2 || ndim > 3 || S < 4 || S > 64 || (S & (S - 1))) return 0;
  int k = 0;
  while ((1u << k) < S) k++;
  const int ez = ndim == 3 ? k / 3 : 0;
  const int ey = (k - ez) / 2;
  const int ex = k - ez - ey;
  b[0] = 1ull << ez;
  b[1] = 1ull << ey;
  b[2] = 1ull << ex;
  return 1;
}

/* The residual's view of the field for the Lorenzo family: HSZp-nd (R12)
 * uses the field's own dims and the nd block shape; HSZp (R14) the field as
 * one row of n with blocks of S.  0 for the other modes. */
static int lz_view(const or_header *h, uint64_t d[3], uint64_t bs[3]) {
  if (h->flags & OR_FLAG_INTER) {
    d[0] = d[1] = 1;
    d[2] = h->n;
    bs[0] = bs[1] = 1;
    bs[2] = h->block;
    return 1;
  }
  if (h->flags & OR_FLAG_LORENZO) {
    if (!nd_block_shape(h->ndim, h->block, bs)) return 0;
    for (int k = 0; k < 3; k++) d[k] = h->dims[k];
    return 1;
  }
  return 0;
}

/* Section placement: header, chunk offsets, q0, widths, payload.  Streams of
 * the Lorenzo family count blocks over their partition and store no q0. */
static void layout(or_header *h) {
  uint64_t d[3], bs[3];
  const int lz = lz_view(h, d, bs);
  if (lz) {
    h->nb = 1;
    for (int k = 0; k < 3; k++) h->nb *= ceil_div(d[k], bs[k]);
  } else {
    h->nb = ceil_div(h->n, h->block);
  }
  h->nchunks = ceil_div(h->nb, h->chunk_blocks);
  h->off_chunk = OR_HEADER_BYTES;
  h->off_q0 = round_up(h->off_chunk + 8 * (h->nchunks + 1), OR_SECTION_ALIGN);
  h->off_width = round_up(h->off_q0 + (lz ? 0 : 4 * h->nb), OR_SECTION_ALIGN);
  h->off_payload = round_up(h->off_width + h->nb, OR_SECTION_ALIGN);
}

/* words one block occupies in the payload (rule R5) */
static uint64_t block_words(uint32_t S, uint32_t w) {
  if (w == 0) return 0;
  return ceil_div(S, 32) + ceil_div((uint64_t)S * w, 32);
}

static void write_header(uint8_t *out, const or_header *h) {
  memset(out, 0, OR_HEADER_BYTES);
  memcpy(out + 0, "HSZ1", 4);
  put_u16(out + 4, 1);
  out[6] = (uint8_t)h->dtype;
  out[7] = (uint8_t)h->ndim;
  put_u64(out + 8, h->dims[0]);
  put_u64(out + 16, h->dims[1]);
  put_u64(out + 24, h->dims[2]);
  put_u64(out + 32, h->n);
  put_u32(out + 40, h->block);
  put_u32(out + 44, h->chunk_blocks);
  put_f64(out + 48, h->eb_abs);
  put_f64(out + 56, h->quantum);
  put_f64(out + 64, h->inv_quantum);
  put_f64(out + 72, h->vmin);
  put_f64(out + 80, h->vmax);
  put_u32(out + 88, h->max_abs_q);
  put_u32(out + 92, h->flags);
  put_u64(out + 96, h->nb);
  put_u64(out + 104, h->nchunks);
  put_u64(out + 112, h->off_chunk);
  put_u64(out + 120, h->off_q0);
  put_u64(out + 128, h->off_width);
  put_u64(out + 136, h->off_payload);
  put_u64(out + 144, h->payload_words);
  put_u64(out + 152, h->total_bytes);
}

/* Parse and validate a header.  Returns OR_OK or OR_ERR_STREAM. */
int or_read_header(const uint8_t *buf, uint64_t len, or_header *h) {
  if (!buf || !h) return OR_ERR_ARG;
  if (len < OR_HEADER_BYTES) return OR_ERR_STREAM;
  if (memcmp(buf, "HSZ1", 4) != 0 || get_u16(buf + 4) != 1) return OR_ERR_STREAM;
  memset(h, 0, sizeof *h);
  h->dtype = buf[6];
  h->ndim = buf[7];
  h->dims[0] = get_u64(buf + 8);
  h->dims[1] = get_u64(buf + 16);
  h->dims[2] = get_u64(buf + 24);
  h->n = get_u64(buf + 32);
  h->block = get_u32(buf + 40);
  h->chunk_blocks = get_u32(buf + 44);
  h->eb_abs = get_f64(buf + 48);
  h->quantum = get_f64(buf + 56);
  h->inv_quantum = get_f64(buf + 64);
  h->vmin = get_f64(buf + 72);
  h->vmax = get_f64(buf + 80);
  h->max_abs_q = get_u32(buf + 88);
  h->flags = get_u32(buf + 92);
  h->nb = get_u64(buf + 96);
  h->nchunks = get_u64(buf + 104);
  h->off_chunk = get_u64(buf + 112);
  h->off_q0 = get_u64(buf + 120);
  h->off_width = get_u64(buf + 128);
  h->off_payload = get_u64(buf + 136);
  h->payload_words = get_u64(buf + 144);
  h->total_bytes = get_u64(buf + 152);
  if (h->dtype != 1 && h->dtype != 2) return OR_ERR_STREAM;
  /* bit 0: block-mean decorrelation (R10); bit 1: HSZp-nd (R12); bit 2:
     HSZp's inter-block prediction (R14); at most one */
  if (h->flags != 0 && h->flags != 1u && h->flags != 2u && h->flags != 4u) return OR_ERR_STREAM;
  if (h->ndim < 1 || h->ndim > 3) return OR_ERR_STREAM;
  uint64_t bs[3];
  if ((h->flags & OR_FLAG_LORENZO) && !nd_block_shape(h->ndim, h->block, bs)) return OR_ERR_STREAM;
  if (h->block < 1 || h->block > 64 || h->chunk_blocks != OR_CHUNK_BLOCKS) return OR_ERR_STREAM;
  uint64_t prod = 1;
  for (int k = 0; k < 3; k++) {
    if (h->dims[k] == 0) return OR_ERR_STREAM;
    if (k < 3 - (int)h->ndim && h->dims[k] != 1) return OR_ERR_STREAM;
    prod *= h->dims[k];
  }
  if (prod != h->n || h->n == 0) return OR_ERR_STREAM;
  if (!(h->quantum > 0.0) || h->inv_quantum != 1.0 / h->quantum) return OR_ERR_STREAM;
  or_header ref = *h;
  layout(&ref);
  if (ref.nb != h->nb || ref.nchunks != h->nchunks || ref.off_chunk != h->off_chunk ||
      ref.off_q0 != h->off_q0 || ref.off_width != h->off_width || ref.off_payload != h->off_payload)
    return OR_ERR_STREAM;
  if (h->total_bytes != h->off_payload + 4 * h->payload_words) return OR_ERR_STREAM;
  if (h->total_bytes > len) return OR_ERR_STREAM;
  return OR_OK;
}

uint64_t or_compress_bound(uint64_t n, uint32_t S) {
  if (n == 0 || S < 1 || S > 64) return 0;
  or_header h;
  memset(&h, 0, sizeof h);
  h.n = n;
  h.block = S;
  h.chunk_blocks = OR_CHUNK_BLOCKS;
  layout(&h);
  /* |q| <= 2^29 - 1 (R6) bounds |p| below 2^30, so no block is wider than 30 bits */
  return h.off_payload + 4 * h.nb * block_words(S, 30);
}

/* The same bound for a stream of the given flags over a field of the given
 * dims (HSZp-nd streams count blocks over the nd partition). */
uint64_t or_compress_bound_dims(uint32_t ndim, const uint64_t *dims, uint32_t S, uint32_t flags) {
  if (!dims || ndim < 1 || ndim > 3 || S < 1 || S > 64 || (flags != 0 && flags != 1u && flags != 2u && flags != 4u))
    return 0;
  or_header h;
  memset(&h, 0, sizeof h);
  h.ndim = ndim;
  for (int k = 0; k < 3; k++) h.dims[k] = 1;
  h.n = 1;
  for (uint32_t k = 0; k < ndim; k++) { h.dims[3 - ndim + k] = dims[k]; h.n *= dims[k]; }
  uint64_t bs[3];
  if (h.n == 0 || ((flags & OR_FLAG_LORENZO) && !nd_block_shape(ndim, S, bs))) return 0;
  h.block = S;
  h.flags = flags;
  h.chunk_blocks = OR_CHUNK_BLOCKS;
  layout(&h);
  return h.off_payload + 4 * h.nb * block_words(S, 30);
}

/* ---- quantizer parameters (rule R3) ------------------------------------ */

/* spacing of the field's floating-point numbers in the binade holding v>0 */
double or_ulp(double v, int dtype) {
  int e;
  frexp(v, &e); /* v = m * 2^e, 0.5 <= m < 1, so v lies in [2^(e-1), 2^e) */
  return ldexp(1.0, e - 1 - (dtype == 1 ? 23 : 52));
}

/* From the field's extremes and the user's bound, compute eps (absolute)
 * and the quantum Delta.  Returns OR_ERR_EB when no positive quantum is
 * left after the safety margin. */
int or_quant_params(double vmin, double vmax, double eb, int eb_is_rel, int dtype,
                    double *eb_abs, double *quantum) {
  if (!(eb > 0.0) || !isfinite(eb)) return OR_ERR_EB;
  double eps;
  if (eb_is_rel) {
    double range = vmax - vmin;
    if (range > 0.0) eps = eb * range;
    else if (fabs(vmax) > 0.0) eps = eb * fabs(vmax);
    else eps = eb;
  } else {
    eps = eb;
  }
  double maxabs = fabs(vmin) > fabs(vmax) ? fabs(vmin) : fabs(vmax);
  double margin = (dtype == 1 ? 1.0 : 8.0) * or_ulp(maxabs + eps, dtype);
  double eps_q = eps - margin;
  if (!(eps_q > 0.0)) return OR_ERR_EB;
  *eb_abs = eps;
  *quantum = 2.0 * eps_q;
  return OR_OK;
}

/* ---- Alg. 1, quantize loop --------------------------------------------- */

/* q_i = round(x_i / Delta), round-half-up, the division done as a multiply
 * by the stored reciprocal (rules R1, R2).  Returns the number of elements
 * whose |q| exceeds 2^29 - 1 (their q is clamped). */
uint64_t or_quantize(const double *x, uint64_t n, double quantum, int32_t *q) {
  double inv = 1.0 / quantum;
  uint64_t bad = 0;
  for (uint64_t i = 0; i < n; i++) {
    double t = x[i] * inv;
    double r = floor(t + 0.5);
    if (r > OR_QMAX) { r = OR_QMAX; bad++; }
    if (r < -OR_QMAX) { r = -OR_QMAX; bad++; }
    q[i] = (int32_t)r;
  }
  return bad;
}

/* ---- Alg. 1, partition + metadata + decorrelate + encode --------------- */

static uint32_t bit_length(uint32_t v) {
  uint32_t w = 0;
  while (v) { w++; v >>= 1; }
  return w;
}

static void stream_set_bits(uint32_t *words, uint64_t bitpos, uint32_t value, uint32_t nbits) {
  for (uint32_t k = 0; k < nbits; k++)
    if ((value >> k) & 1u) words[(bitpos + k) / 32] |= 1u << ((bitpos + k) % 32);
}

static uint32_t stream_get_bits(const uint32_t *words, uint64_t bitpos, uint32_t nbits) {
  uint32_t v = 0;
  for (uint32_t k = 0; k < nbits; k++)
    if ((words[(bitpos + k) / 32] >> ((bitpos + k) % 32)) & 1u) v |= 1u << k;
  return v;
}

/* round(a / b) with halves rounded down, b > 0: ceil((2a - b) / (2b)) in
 * exact integer arithmetic (C division truncates toward zero) */
static int64_t round_half_down_div(int64_t a, int64_t b) {
  const int64_t num = 2 * a - b, den = 2 * b;
  return num >= 0 ? (num + den - 1) / den : -((-num) / den);
}

/* Encode already-quantized integers q[n] (the field read as a flat array)
 * into the byte format.  'h' carries dtype, dims, eps, Delta, extremes; the
 * layout fields are filled here.  The output must be zero-filled by this
 * function's caller or it is cleared here up to the bound. */
static int encode_q(const int32_t *q, or_header *h, uint8_t *out, uint64_t cap, uint64_t *out_size) {
  const uint32_t S = h->block;
  const int mean_mode = (h->flags & OR_FLAG_MEAN) != 0;
  const int lorenzo = (h->flags & (OR_FLAG_LORENZO | OR_FLAG_INTER)) != 0;
  uint64_t vd[3] = {1, 1, 1}, bs[3] = {1, 1, 1};
  if (lorenzo && !lz_view(h, vd, bs)) return OR_ERR_ARG;
  h->chunk_blocks = OR_CHUNK_BLOCKS;
  layout(h);
  uint64_t bound = h->off_payload + 4 * h->nb * block_words(S, 30);
  if (cap < h->off_payload) { if (out_size) *out_size = bound; return OR_ERR_CAPACITY; }

  uint32_t max_abs_q = 0;
  for (uint64_t e = 0; e < h->n; e++) {
    uint32_t aq = (uint32_t)(q[e] < 0 ? -(int64_t)q[e] : q[e]);
    if (aq > max_abs_q) max_abs_q = aq;
  }

  /* decorrelated data p, block by block (slot i of block b at b*S + i; slots
     outside the field stay 0), and the metadata of the 1D modes */
  int32_t *p = (int32_t *)calloc(h->nb * S, sizeof(int32_t));
  uint32_t *width = (uint32_t *)calloc(h->nb, sizeof(uint32_t));
  int32_t *q0 = (int32_t *)calloc(h->nb, sizeof(int32_t));
  if (!p || !width || !q0) { free(p); free(width); free(q0); return OR_ERR_ARG; }
  if (lorenzo) {
    /* Lorenzo residual of every point (R12, R14), q = 0 outside the field */
    const uint64_t Z = vd[0], Y = vd[1], X = vd[2];
    const uint64_t nbz = ceil_div(Z, bs[0]), nby = ceil_div(Y, bs[1]), nbx = ceil_div(X, bs[2]);
    for (uint64_t bz = 0; bz < nbz; bz++)
      for (uint64_t by = 0; by < nby; by++)
        for (uint64_t bx = 0; bx < nbx; bx++) {
          const uint64_t b = (bz * nby + by) * nbx + bx;
          uint32_t i = 0;
          for (uint64_t sz = 0; sz < bs[0]; sz++)
            for (uint64_t sy = 0; sy < bs[1]; sy++)
              for (uint64_t sx = 0; sx < bs[2]; sx++, i++) {
                const uint64_t z = bz * bs[0] + sz, y = by * bs[1] + sy, x = bx * bs[2] + sx;
                if (z >= Z || y >= Y || x >= X) continue;
                int64_t r = 0;
                for (int c = 0; c < 8; c++) {
                  const int dz = (c >> 2) & 1, dy = (c >> 1) & 1, dx = c & 1;
                  if ((dz && z == 0) || (dy && y == 0) || (dx && x == 0)) continue;
                  const int64_t v = q[((z - dz) * Y + (y - dy)) * X + (x - dx)];
                  r += ((dz + dy + dx) & 1) ? -v : v;
                }
                if (r > OR_PMAX || r < -OR_PMAX) { free(p); free(width); free(q0); return OR_ERR_RANGE; }
                p[b * S + i] = (int32_t)r;
              }
        }
  } else {
    for (uint64_t b = 0; b < h->nb; b++) {
      uint64_t first = b * S;
      uint64_t len = (h->n - first < S) ? h->n - first : S;
      if (mean_mode) {
        int64_t sum = 0;
        for (uint64_t i = 0; i < len; i++) sum += q[first + i];
        q0[b] = (int32_t)round_half_down_div(sum, (int64_t)len);
      } else {
        q0[b] = q[first];
      }
      for (uint64_t i = 0; i < len; i++)
        p[first + i] = mean_mode ? q[first + i] - q0[b] : (i == 0) ? 0 : q[first + i] - q[first + i - 1];
    }
  }
  uint64_t words = 0;
  for (uint64_t b = 0; b < h->nb; b++) {
    uint32_t maxp = 0;
    for (uint32_t i = 0; i < S; i++) {
      int32_t pi = p[b * S + i];
      uint32_t ap = (uint32_t)(pi < 0 ? -(int64_t)pi : pi);
      if (ap > maxp) maxp = ap;
    }
    width[b] = bit_length(maxp);
    words += block_words(S, width[b]);
  }
  h->max_abs_q = max_abs_q;
  h->payload_words = words;
  h->total_bytes = h->off_payload + 4 * words;
  if (out_size) *out_size = h->total_bytes;
  if (cap < h->total_bytes) { free(p); free(width); free(q0); return OR_ERR_CAPACITY; }

  memset(out, 0, h->total_bytes);
  write_header(out, h);
  uint32_t *payload = (uint32_t *)calloc(words ? words : 1, sizeof(uint32_t));
  if (!payload) { free(p); free(width); free(q0); return OR_ERR_ARG; }
  uint64_t pos = 0;
  for (uint64_t b = 0; b < h->nb; b++) {
    if (b % OR_CHUNK_BLOCKS == 0) put_u64(out + h->off_chunk + 8 * (b / OR_CHUNK_BLOCKS), pos);
    if (!lorenzo) put_u32(out + h->off_q0 + 4 * b, (uint32_t)q0[b]);
    out[h->off_width + b] = (uint8_t)width[b];
    uint32_t w = width[b];
    if (w == 0) continue;
    uint32_t *sign = payload + pos;
    uint32_t *mag = sign + ceil_div(S, 32);
    for (uint32_t i = 0; i < S; i++) {
      int32_t pi = p[b * S + i];
      if (pi < 0) sign[i / 32] |= 1u << (i % 32);
      uint32_t ap = (uint32_t)(pi < 0 ? -(int64_t)pi : pi);
      stream_set_bits(mag, (uint64_t)i * w, ap, w);
    }
    pos += block_words(S, w);
  }
  put_u64(out + h->off_chunk + 8 * h->nchunks, pos);
  for (uint64_t k = 0; k < words; k++) put_u32(out + h->off_payload + 4 * k, payload[k]);
  free(payload); free(p); free(width); free(q0);
  return OR_OK;
}

/* Encode given quantization integers (used to pin the decorrelation and the
 * encoding on the paper's worked example, where the quantum is fixed). */
int or_encode_q(const int32_t *q, uint32_t ndim, const uint64_t *dims, uint32_t dtype,
                double eb_abs, double quantum, uint32_t S, uint32_t flags, uint8_t *out, uint64_t cap,
                uint64_t *out_size) {
  if (!q || !dims || ndim < 1 || ndim > 3 || S < 1 || S > 64 || (dtype != 1 && dtype != 2))
    return OR_ERR_ARG;
  or_header h;
  memset(&h, 0, sizeof h);
  h.dtype = dtype;
  h.ndim = ndim;
  for (int k = 0; k < 3; k++) h.dims[k] = 1;
  h.n = 1;
  for (uint32_t k = 0; k < ndim; k++) { h.dims[3 - ndim + k] = dims[k]; h.n *= dims[k]; }
  if (h.n == 0) return OR_ERR_ARG;
  h.block = S;
  h.eb_abs = eb_abs;
  h.quantum = quantum;
  h.inv_quantum = 1.0 / quantum;
  h.vmin = 0.0;
  h.vmax = 0.0;
  if (flags != 0 && flags != 1u && flags != 2u && flags != 4u) return OR_ERR_ARG;
  h.flags = flags;
  return encode_q(q, &h, out, cap, out_size);
}

/* Full compressor C(d, eps): extremes -> parameters -> quantize -> encode. */
int or_compress(const void *x, uint32_t dtype, uint32_t ndim, const uint64_t *dims, double eb,
                int eb_is_rel, uint32_t S, uint32_t flags, uint8_t *out, uint64_t cap, uint64_t *out_size) {
  if (!x || !dims || ndim < 1 || ndim > 3 || S < 1 || S > 64 || (dtype != 1 && dtype != 2) ||
      (flags != 0 && flags != 1u && flags != 2u && flags != 4u))
    return OR_ERR_ARG;
  or_header h;
  memset(&h, 0, sizeof h);
  h.dtype = dtype;
  h.ndim = ndim;
  for (int k = 0; k < 3; k++) h.dims[k] = 1;
  h.n = 1;
  for (uint32_t k = 0; k < ndim; k++) { h.dims[3 - ndim + k] = dims[k]; h.n *= dims[k]; }
  if (h.n == 0) return OR_ERR_ARG;
  h.block = S;
  h.flags = flags;

  double *xd = (double *)malloc(h.n * sizeof(double));
  if (!xd) return OR_ERR_ARG;
  for (uint64_t i = 0; i < h.n; i++)
    xd[i] = (dtype == 1) ? (double)((const float *)x)[i] : ((const double *)x)[i];
  double vmin = xd[0], vmax = xd[0];
  for (uint64_t i = 0; i < h.n; i++) {
    if (!isfinite(xd[i])) { free(xd); return OR_ERR_NONFINITE; }
    if (xd[i] < vmin) vmin = xd[i];
    if (xd[i] > vmax) vmax = xd[i];
  }
  /* + 0.0 turns a -0.0 extreme into +0.0, so the stored extremes have one
     byte pattern whichever of two equal zeros came first */
  vmin = vmin + 0.0;
  vmax = vmax + 0.0;
  h.vmin = vmin;
  h.vmax = vmax;
  int rc = or_quant_params(vmin, vmax, eb, eb_is_rel, (int)dtype, &h.eb_abs, &h.quantum);
  if (rc != OR_OK) { free(xd); return rc; }
  h.inv_quantum = 1.0 / h.quantum;

  int32_t *q = (int32_t *)malloc(h.n * sizeof(int32_t));
  if (!q) { free(xd); return OR_ERR_ARG; }
  uint64_t bad = or_quantize(xd, h.n, h.quantum, q);
  free(xd);
  if (bad) { free(q); return OR_ERR_RANGE; }
  rc = encode_q(q, &h, out, cap, out_size);
  free(q);
  return rc;
}

/* ---- Alg. 2: partial decompression ------------------------------------- */

/* stage: 1 = metadata (q0[nb]); 2 = decorrelated data (p[n] then q0[nb]);
 * 3 = quantized data (q[n]); 4 = decompressed floats (field dtype, n).
 * 'out' must hold or_stage_bytes(...) bytes. */
uint64_t or_stage_bytes(const uint8_t *buf, uint64_t len, int stage) {
  or_header h;
  if (or_read_header(buf, len, &h) != OR_OK) return 0;
  const int lorenzo = (h.flags & (OR_FLAG_LORENZO | OR_FLAG_INTER)) != 0;
  switch (stage) {
    case 1: return lorenzo ? 0 : 4 * h.nb;
    case 2: return 4 * h.n + (lorenzo ? 0 : 4 * h.nb);
    case 3: return 4 * h.n;
    case 4: return (h.dtype == 1 ? 4 : 8) * h.n;
    default: return 0;
  }
}

/* stage 1 of an HSZp-nd or HSZp stream does not exist (no metadata):
 * OR_ERR_UNSUPPORTED */
int or_decompress(const uint8_t *buf, uint64_t len, int stage, void *out) {
  or_header h;
  int rc = or_read_header(buf, len, &h);
  if (rc != OR_OK) return rc;
  if (!out || stage < 1 || stage > 4) return OR_ERR_ARG;
  const uint32_t S = h.block;
  const int lorenzo = (h.flags & (OR_FLAG_LORENZO | OR_FLAG_INTER)) != 0;
  if (lorenzo && stage == 1) return OR_ERR_UNSUPPORTED;
  int32_t *q0 = (int32_t *)calloc(h.nb, sizeof(int32_t));
  if (!q0) return OR_ERR_ARG;
  if (!lorenzo)
    for (uint64_t b = 0; b < h.nb; b++) q0[b] = (int32_t)get_u32(buf + h.off_q0 + 4 * b);
  if (stage == 1) { memcpy(out, q0, h.nb * sizeof(int32_t)); free(q0); return OR_OK; }

  /* decode: signs and magnitudes -> pb (slot i of block b at b*S + i) */
  int32_t *pb = (int32_t *)calloc(h.nb * S, sizeof(int32_t));
  if (!pb) { free(q0); return OR_ERR_ARG; }
  uint64_t pos = 0;
  for (uint64_t b = 0; b < h.nb; b++) {
    if (b % OR_CHUNK_BLOCKS == 0 && get_u64(buf + h.off_chunk + 8 * (b / OR_CHUNK_BLOCKS)) != pos) {
      free(pb); free(q0); return OR_ERR_STREAM;
    }
    uint32_t w = buf[h.off_width + b];
    if (w > 30) { free(pb); free(q0); return OR_ERR_STREAM; }
    if (w == 0) continue;
    uint64_t nw = block_words(S, w);
    if (pos + nw > h.payload_words) { free(pb); free(q0); return OR_ERR_STREAM; }
    uint32_t *blk = (uint32_t *)malloc(nw * sizeof(uint32_t));
    if (!blk) { free(pb); free(q0); return OR_ERR_ARG; }
    for (uint64_t k = 0; k < nw; k++) blk[k] = get_u32(buf + h.off_payload + 4 * (pos + k));
    const uint32_t *mag = blk + ceil_div(S, 32);
    for (uint32_t i = 0; i < S; i++) {
      uint32_t a = stream_get_bits(mag, (uint64_t)i * w, w);
      int neg = (blk[i / 32] >> (i % 32)) & 1u;
      pb[b * S + i] = neg ? -(int32_t)a : (int32_t)a;
    }
    free(blk);
    pos += nw;
  }
  if (pos != h.payload_words) { free(pb); free(q0); return OR_ERR_STREAM; }

  /* p in the field's own layout: the 1D modes read blocks in order; HSZp-nd
     places each slot of each nd block at its coordinates (R12) */
  int32_t *p = (int32_t *)calloc(h.n, sizeof(int32_t));
  if (!p) { free(pb); free(q0); return OR_ERR_ARG; }
  uint64_t vd[3] = {h.dims[0], h.dims[1], h.dims[2]}, bs[3] = {1, 1, 1};
  if (lorenzo) lz_view(&h, vd, bs);
  const uint64_t Z = vd[0], Y = vd[1], X = vd[2];
  if (lorenzo) {
    const uint64_t nby = ceil_div(Y, bs[1]), nbx = ceil_div(X, bs[2]);
    for (uint64_t b = 0; b < h.nb; b++) {
      const uint64_t bz = b / (nby * nbx), by = (b / nbx) % nby, bx = b % nbx;
      for (uint32_t i = 0; i < S; i++) {
        const uint64_t sz = i / (bs[1] * bs[2]), sy = (i / bs[2]) % bs[1], sx = i % bs[2];
        const uint64_t z = bz * bs[0] + sz, y = by * bs[1] + sy, x = bx * bs[2] + sx;
        if (z < Z && y < Y && x < X) p[(z * Y + y) * X + x] = pb[b * S + i];
      }
    }
  } else {
    memcpy(p, pb, h.n * sizeof(int32_t));
  }
  free(pb);
  if (stage == 2) {
    memcpy(out, p, h.n * sizeof(int32_t));
    if (!lorenzo) memcpy((int32_t *)out + h.n, q0, h.nb * sizeof(int32_t));
    free(p); free(q0);
    return OR_OK;
  }

  /* recorrelate: q_i = q_{i-1} + p_i inside a block, starting from q0 (delta
     mode); q_i = M_b + p_i (block-mean mode, R10); HSZp-nd: q = p plus the
     Lorenzo prediction from the points before it in raster order (R12) */
  int32_t *q = (int32_t *)malloc(h.n * sizeof(int32_t));
  if (!q) { free(p); free(q0); return OR_ERR_ARG; }
  for (uint64_t e = 0; e < h.n; e++) {
    uint64_t b = e / S;
    if (lorenzo) {
      const uint64_t z = e / (Y * X), y = (e / X) % Y, x = e % X;
      int64_t v = p[e];
      for (int c = 1; c < 8; c++) {
        const int dz = (c >> 2) & 1, dy = (c >> 1) & 1, dx = c & 1;
        if ((dz && z == 0) || (dy && y == 0) || (dx && x == 0)) continue;
        const int64_t u = q[((z - dz) * Y + (y - dy)) * X + (x - dx)];
        v += ((dz + dy + dx) & 1) ? u : -u;
      }
      if (v > OR_QMAX || v < -OR_QMAX) { free(q); free(p); free(q0); return OR_ERR_STREAM; }
      q[e] = (int32_t)v;
    } else if (h.flags & OR_FLAG_MEAN) {
      q[e] = q0[b] + p[e];
    } else {
      q[e] = (e % S == 0) ? q0[b] : q[e - 1] + p[e];
    }
  }
  free(p); free(q0);
  if (stage == 3) { memcpy(out, q, h.n * sizeof(int32_t)); free(q); return OR_OK; }

  /* dequantize: d' = q * Delta (Delta = 2 eps_q) */
  for (uint64_t e = 0; e < h.n; e++) {
    double v = (double)q[e] * h.quantum;
    if (h.dtype == 1) ((float *)out)[e] = (float)v;
    else ((double *)out)[e] = v;
  }
  free(q);
  return OR_OK;
}

/* d' = q * Delta in binary64 (the decompressed value before it is stored in
 * the field's own type). */
void or_dequantize64(const int32_t *q, uint64_t n, double quantum, double *out) {
  for (uint64_t i = 0; i < n; i++) out[i] = (double)q[i] * quantum;
}

/* ---- operations on the decompressed field (Sec. III-B) ----------------- */

/* dims3: slow -> fast, box lo/hi half-open, all 3D (leading axes of length
 * 1 for 1D and 2D fields).  NULL box = whole field. */
typedef struct { int64_t lo[3], hi[3]; } or_box;

static int box_ok(const uint64_t *d, const int64_t *lo, const int64_t *hi, or_box *b) {
  for (int k = 0; k < 3; k++) {
    b->lo[k] = lo ? lo[k] : 0;
    b->hi[k] = hi ? hi[k] : (int64_t)d[k];
    if (b->lo[k] < 0 || b->hi[k] > (int64_t)d[k] || b->lo[k] >= b->hi[k]) return 0;
  }
  return 1;
}

/* Neumaier-compensated running sum */
typedef struct { double s, c; } ksum;
static void ksum_add(ksum *k, double v) {
  double t = k->s + v;
  if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
  else k->c += (v - t) + k->s;
  k->s = t;
}
static double ksum_get(const ksum *k) { return k->s + k->c; }

/* mean = (sum of d_i) / N over the box */
int or_mean(const double *x, const uint64_t *d, const int64_t *lo, const int64_t *hi, double *mean) {
  or_box b;
  if (!box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  ksum k = {0, 0};
  int64_t cnt = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) {
        ksum_add(&k, x[((uint64_t)z * d[1] + (uint64_t)y) * d[2] + (uint64_t)xx]);
        cnt++;
      }
  *mean = ksum_get(&k) / (double)cnt;
  return OR_OK;
}

/* sample variance sum (d_i - mu)^2 / (N - 1), two passes */
int or_var(const double *x, const uint64_t *d, const int64_t *lo, const int64_t *hi, double *var) {
  or_box b;
  if (!box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  double mu;
  or_mean(x, d, lo, hi, &mu);
  ksum k = {0, 0};
  int64_t cnt = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) {
        double e = x[((uint64_t)z * d[1] + (uint64_t)y) * d[2] + (uint64_t)xx] - mu;
        ksum_add(&k, e * e);
        cnt++;
      }
  *var = (cnt > 1) ? ksum_get(&k) / (double)(cnt - 1) : NAN;
  return OR_OK;
}

/* derivative of the field along axis a (0 = slowest of the 3D view) at one
 * point, unit spacing, rule R7 */
static double deriv_at(const double *x, const uint64_t *d, int a, int64_t z, int64_t y, int64_t xx) {
  int64_t idx[3] = {z, y, xx};
  int64_t len = (int64_t)d[a];
  if (len < 2) return 0.0;
  int64_t im = idx[a] - 1, ip = idx[a] + 1;
  double denom = 2.0;
  if (idx[a] == 0) { im = 0; denom = 1.0; }
  if (idx[a] == len - 1) { ip = len - 1; denom = 1.0; }
  int64_t jm[3] = {z, y, xx}, jp[3] = {z, y, xx};
  jm[a] = im;
  jp[a] = ip;
  double vm = x[((uint64_t)jm[0] * d[1] + (uint64_t)jm[1]) * d[2] + (uint64_t)jm[2]];
  double vp = x[((uint64_t)jp[0] * d[1] + (uint64_t)jp[1]) * d[2] + (uint64_t)jp[2]];
  return (vp - vm) / denom;
}

/* out[box volume] = derivative along axis a (3D view axis) */
int or_derivative(const double *x, const uint64_t *d, int a, const int64_t *lo, const int64_t *hi, double *out) {
  or_box b;
  if (a < 0 || a > 2 || !box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  uint64_t o = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) out[o++] = deriv_at(x, d, a, z, y, xx);
  return OR_OK;
}

/* out[box volume] = sqrt(sum over axes of derivative^2) */
int or_gradmag(const double *x, const uint64_t *d, const int64_t *lo, const int64_t *hi, double *out) {
  or_box b;
  if (!box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  uint64_t o = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) {
        double s = 0.0;
        for (int a = 0; a < 3; a++) {
          double g = deriv_at(x, d, a, z, y, xx);
          s += g * g;
        }
        out[o++] = sqrt(s);
      }
  return OR_OK;
}

/* second difference of the field along axis a at one point, rule R8 */
static double second_diff_at(const double *x, const uint64_t *d, int a, int64_t z, int64_t y, int64_t xx) {
  int64_t idx[3] = {z, y, xx};
  int64_t len = (int64_t)d[a];
  int64_t im = idx[a] > 0 ? idx[a] - 1 : idx[a];
  int64_t ip = idx[a] < len - 1 ? idx[a] + 1 : idx[a];
  int64_t jm[3] = {z, y, xx}, jp[3] = {z, y, xx};
  jm[a] = im;
  jp[a] = ip;
  double v0 = x[((uint64_t)z * d[1] + (uint64_t)y) * d[2] + (uint64_t)xx];
  double vm = x[((uint64_t)jm[0] * d[1] + (uint64_t)jm[1]) * d[2] + (uint64_t)jm[2]];
  double vp = x[((uint64_t)jp[0] * d[1] + (uint64_t)jp[1]) * d[2] + (uint64_t)jp[2]];
  return vm + vp - 2.0 * v0;
}

/* out[box volume] = Laplacian (Eq. (laplacian), rule R8) */
int or_laplacian(const double *x, const uint64_t *d, const int64_t *lo, const int64_t *hi, double *out) {
  or_box b;
  if (!box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  uint64_t o = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) {
        double s = 0.0;
        for (int a = 0; a < 3; a++) s += second_diff_at(x, d, a, z, y, xx);
        out[o++] = s;
      }
  return OR_OK;
}

/* Divergence (Eq. (divergence), rule R9) of a vector field with one
 * component per axis of the field: comp[k] is component k (field axis k =
 * 3D-view axis k + 3 - ndim).  out[box volume]. */
int or_divergence(const double *const *comp, int ndim, const uint64_t *d, const int64_t *lo, const int64_t *hi,
                  double *out) {
  or_box b;
  if (ndim < 1 || ndim > 3 || !box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  uint64_t o = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) {
        double s = 0.0;
        for (int k = 0; k < ndim; k++) s += deriv_at(comp[k], d, k + 3 - ndim, z, y, xx);
        out[o++] = s;
      }
  return OR_OK;
}

/* Curl (Eq. (curl), rule R9).  ndim 2: out[box volume] = delta_1 F_0 -
 * delta_0 F_1.  ndim 3: out holds the three components one after the
 * other, each of box volume. */
int or_curl(const double *const *comp, int ndim, const uint64_t *d, const int64_t *lo, const int64_t *hi,
            double *out) {
  or_box b;
  if ((ndim != 2 && ndim != 3) || !box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  const uint64_t vol = (uint64_t)(b.hi[0] - b.lo[0]) * (uint64_t)(b.hi[1] - b.lo[1]) * (uint64_t)(b.hi[2] - b.lo[2]);
  const int base = 3 - ndim; /* 3D-view axis of field axis 0 */
  uint64_t o = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) {
        if (ndim == 2) {
          out[o] = deriv_at(comp[0], d, base + 1, z, y, xx) - deriv_at(comp[1], d, base + 0, z, y, xx);
        } else {
          out[o] = deriv_at(comp[1], d, 2, z, y, xx) - deriv_at(comp[2], d, 1, z, y, xx);
          out[vol + o] = deriv_at(comp[2], d, 0, z, y, xx) - deriv_at(comp[0], d, 2, z, y, xx);
          out[2 * vol + o] = deriv_at(comp[0], d, 1, z, y, xx) - deriv_at(comp[1], d, 0, z, y, xx);
        }
        o++;
      }
  return OR_OK;
}

/* Eq. (mean_m): mean from the metadata alone, (1/N sum_b M_b S_b) * Delta,
 * for a block-mean stream (R10); the exact integer sum_b M_b S_b is returned
 * too.  The stream is read from its bytes. */
int or_meta_mean(const uint8_t *buf, uint64_t len, int64_t *msum, double *mean) {
  or_header h;
  int rc = or_read_header(buf, len, &h);
  if (rc != OR_OK) return rc;
  if (!(h.flags & 1u)) return OR_ERR_UNSUPPORTED;
  int64_t s = 0;
  for (uint64_t b = 0; b < h.nb; b++) {
    const uint64_t first = b * h.block;
    const int64_t sb = (int64_t)((h.n - first < h.block) ? h.n - first : h.block);
    s += (int64_t)(int32_t)get_u32(buf + h.off_q0 + 4 * b) * sb;
  }
  *msum = s;
  *mean = (double)s / (double)h.n * h.quantum;
  return OR_OK;
}

/* Standard deviation on D_p for a block-mean stream (Sec. V-A): with the
 * integer mean mu~ = round(sum_b M_b S_b / N) (R11), every term of Eq. (var)
 * is split as (q_i - M_b) + (M_b - mu~) = p_i + M_b - mu~, and
 * sigma^2 = sum_b sum_{p in D_p[B_b]} (p + M_b - mu~)^2 / (N - 1) * Delta^2.
 * The sum of squares is exact (128-bit, split into lo/hi words); msum is
 * sum_b M_b S_b and mu~ the integer mean.  var is NaN when N = 1.  The
 * stream is decoded to stage 2 from its bytes. */
int or_var_mt(const uint8_t *buf, uint64_t len, int64_t *n, int64_t *msum, int64_t *mu_t, uint64_t *s2_lo,
              int64_t *s2_hi, double *var) {
  or_header h;
  int rc = or_read_header(buf, len, &h);
  if (rc != OR_OK) return rc;
  if (!(h.flags & 1u)) return OR_ERR_UNSUPPORTED;
  int32_t *st = (int32_t *)malloc((h.n + h.nb) * sizeof(int32_t));
  if (!st) return OR_ERR_ARG;
  rc = or_decompress(buf, len, 2, st);
  if (rc != OR_OK) { free(st); return rc; }
  const int32_t *p = st, *M = st + h.n;
  int64_t ms = 0;
  for (uint64_t b = 0; b < h.nb; b++) {
    const uint64_t first = b * h.block;
    ms += (int64_t)M[b] * (int64_t)((h.n - first < h.block) ? h.n - first : h.block);
  }
  const int64_t mt = round_half_down_div(ms, (int64_t)h.n);
  __int128 acc = 0;
  for (uint64_t b = 0; b < h.nb; b++) {
    const uint64_t first = b * h.block;
    const uint64_t last = (h.n - first < h.block) ? h.n : first + h.block;
    for (uint64_t e = first; e < last; e++) {
      const int64_t t = (int64_t)p[e] + (int64_t)M[b] - mt;
      acc += (__int128)t * t;
    }
  }
  free(st);
  *n = (int64_t)h.n;
  *msum = ms;
  *mu_t = mt;
  *s2_lo = (uint64_t)acc;
  *s2_hi = (int64_t)(acc >> 64);
  *var = h.n > 1 ? (double)acc / (double)(h.n - 1) * (h.quantum * h.quantum) : NAN;
  return OR_OK;
}

/* ---- HSZp-nd on its decorrelated data D_p (Sec. V) ------------------------
 * p is stage 2 of an HSZp-nd stream (the field's layout); dims are the
 * field's own (ndim of them, slow -> fast).  q at index -1 of any axis is 0. */

static void dims3_from(uint32_t ndim, const uint64_t *dims, uint64_t d[3]) {
  for (int k = 0; k < 3; k++) d[k] = 1;
  for (uint32_t k = 0; k < ndim; k++) d[3 - ndim + k] = dims[k];
}

/* Sec. V-A, mean on D_p of HSZp-nd: q is the nd prefix sum of p, so
 * sum q = sum over points of prod_k (n_k - i_k) p_i (0-based i_k; the
 * paper's 2D weights (n_1 - s + 1)(n_2 - t + 1) with 1-based s, t). */
int or_lz_mean_p(const int32_t *p, uint32_t ndim, const uint64_t *dims, double quantum, int64_t *s1,
                 double *mean) {
  if (!p || !dims || ndim < 1 || ndim > 3) return OR_ERR_ARG;
  uint64_t d[3];
  dims3_from(ndim, dims, d);
  __int128 acc = 0;
  for (uint64_t z = 0; z < d[0]; z++)
    for (uint64_t y = 0; y < d[1]; y++)
      for (uint64_t x = 0; x < d[2]; x++) {
        const __int128 w = (__int128)(d[0] - z) * (__int128)(d[1] - y) * (__int128)(d[2] - x);
        acc += w * p[(z * d[1] + y) * d[2] + x];
      }
  const uint64_t n = d[0] * d[1] * d[2];
  *s1 = (int64_t)acc;
  *mean = (double)acc / (double)n * quantum;
  return OR_OK;
}

/* Standard deviation on D_p of HSZp-nd (Alg. 4, Sec. V-A).  Alg. 4 rebuilds
 * q from p by running sums and accumulates sum q and sum q^2 on the way;
 * the oracle takes the same mathematical steps in their plainest form: q is
 * the nd prefix sum of p (the inverse of the Lorenzo residual), formed here
 * as one cumulative sum along each axis in turn (x, then y, then z; the
 * order does not matter for a separable sum), in 64-bit integers; then
 * s1 = sum q and s2 = sum q^2 exactly (128 bits) and var as Eq. (var) with
 * N - 1, rounded once from (n s2 - s1^2) / (n (n - 1)) Delta^2. */
int or_lz_var_p(const int32_t *p, uint32_t ndim, const uint64_t *dims, double quantum, int64_t *n_out,
                int64_t *s1, uint64_t *s2_lo, int64_t *s2_hi, double *var) {
  if (!p || !dims || ndim < 1 || ndim > 3) return OR_ERR_ARG;
  uint64_t d[3];
  dims3_from(ndim, dims, d);
  const uint64_t Z = d[0], Y = d[1], X = d[2], n = Z * Y * X;
  int64_t *q = (int64_t *)malloc(n * sizeof(int64_t));
  if (!q) return OR_ERR_ARG;
  for (uint64_t i = 0; i < n; i++) q[i] = p[i];
  for (uint64_t z = 0; z < Z; z++) /* along x */
    for (uint64_t y = 0; y < Y; y++)
      for (uint64_t x = 1; x < X; x++) q[(z * Y + y) * X + x] += q[(z * Y + y) * X + x - 1];
  for (uint64_t z = 0; z < Z; z++) /* along y */
    for (uint64_t y = 1; y < Y; y++)
      for (uint64_t x = 0; x < X; x++) q[(z * Y + y) * X + x] += q[(z * Y + y - 1) * X + x];
  for (uint64_t z = 1; z < Z; z++) /* along z */
    for (uint64_t y = 0; y < Y; y++)
      for (uint64_t x = 0; x < X; x++) q[(z * Y + y) * X + x] += q[((z - 1) * Y + y) * X + x];
  int64_t a1 = 0;
  __int128 a2 = 0;
  for (uint64_t i = 0; i < n; i++) {
    a1 += q[i];
    a2 += (__int128)q[i] * q[i];
  }
  free(q);
  *n_out = (int64_t)n;
  *s1 = a1;
  *s2_lo = (uint64_t)a2;
  *s2_hi = (int64_t)(a2 >> 64);
  const __int128 num = (__int128)n * a2 - (__int128)a1 * a1;
  *var = n > 1 ? (double)num / ((double)n * (double)(n - 1)) * (quantum * quantum) : NAN;
  return OR_OK;
}

/* Eq. (derivative_Dp) in the 3D view: along axis a (of the field's axes),
 * q_{i+1} - q_{i-1} is the prefix sum over the other axes of
 * t_i = p_i + p_{i+1}; the one-sided ends (R7) use 2 (q_1 - q_0) with
 * t_0 = 2 p_1 and 2 (q_{n-1} - q_{n-2}) with t = 2 p_{n-1}; an axis of
 * length 1 has t = 0.  The prefix sums follow the paper's recursion: along
 * the fastest other axis a running sum per point (the scalar eta), then a
 * running sum per column over the slower other axis.  num holds the exact
 * integers; out = num * Delta / 2 (the paper's factor eps_q). */
int or_lz_deriv_p(const int32_t *p, uint32_t ndim, const uint64_t *dims, int axis, double quantum, int64_t *num,
                  double *out) {
  if (!p || !dims || !num || !out || ndim < 1 || ndim > 3 || axis < 0 || axis >= (int)ndim) return OR_ERR_ARG;
  uint64_t d[3];
  dims3_from(ndim, dims, d);
  const int a = axis + 3 - (int)ndim;
  const uint64_t na = d[a];
  /* t along axis a */
  for (uint64_t z = 0; z < d[0]; z++)
    for (uint64_t y = 0; y < d[1]; y++)
      for (uint64_t x = 0; x < d[2]; x++) {
        const uint64_t c[3] = {z, y, x};
        const uint64_t i = c[a];
        uint64_t cn[3] = {z, y, x};
        int64_t t;
        if (na == 1) {
          t = 0;
        } else if (i == 0) {
          cn[a] = 1;
          t = 2 * (int64_t)p[(cn[0] * d[1] + cn[1]) * d[2] + cn[2]];
        } else if (i == na - 1) {
          t = 2 * (int64_t)p[(z * d[1] + y) * d[2] + x];
        } else {
          cn[a] = i + 1;
          t = (int64_t)p[(z * d[1] + y) * d[2] + x] + p[(cn[0] * d[1] + cn[1]) * d[2] + cn[2]];
        }
        num[(z * d[1] + y) * d[2] + x] = t;
      }
  /* prefix sums over each of the other axes, fastest first */
  for (int o = 2; o >= 0; o--) {
    if (o == a) continue;
    const uint64_t stride = o == 2 ? 1 : (o == 1 ? d[2] : d[1] * d[2]);
    for (uint64_t e = 0; e < d[0] * d[1] * d[2]; e++) {
      const uint64_t c[3] = {e / (d[1] * d[2]), (e / d[2]) % d[1], e % d[2]};
      if (c[o] > 0) num[e] += num[e - stride];
    }
  }
  const double half = quantum * 0.5;
  for (uint64_t e = 0; e < d[0] * d[1] * d[2]; e++) out[e] = (double)num[e] * half;
  return OR_OK;
}

/* Exact integer sums over the box of the quantized field: N, sum q, sum q^2
 * (the last as a 128-bit two's-complement value split into lo/hi words). */
int or_int_sums(const int32_t *q, const uint64_t *d, const int64_t *lo, const int64_t *hi,
                int64_t *n, int64_t *s1, uint64_t *s2_lo, int64_t *s2_hi) {
  or_box b;
  if (!box_ok(d, lo, hi, &b)) return OR_ERR_ARG;
  int64_t cnt = 0, a1 = 0;
  __int128 a2 = 0;
  for (int64_t z = b.lo[0]; z < b.hi[0]; z++)
    for (int64_t y = b.lo[1]; y < b.hi[1]; y++)
      for (int64_t xx = b.lo[2]; xx < b.hi[2]; xx++) {
        int64_t v = q[((uint64_t)z * d[1] + (uint64_t)y) * d[2] + (uint64_t)xx];
        cnt++;
        a1 += v;
        a2 += (__int128)(v * v);
      }
  *n = cnt;
  *s1 = a1;
  *s2_lo = (uint64_t)a2;
  *s2_hi = (int64_t)(a2 >> 64);
  return OR_OK;
}
