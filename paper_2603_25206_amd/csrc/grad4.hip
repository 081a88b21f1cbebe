// grad4.hip -- the binary32 gradient magnitude (Eq. (derivatives), Sec. V-B)
// straight from the compressed stream through D_q, laid out for the common
// case of the quantized route: blocks of 32, max|q| < 8192 (every numerator
// below 2^15, the squared sum exact in 32 bits) and rows whose blocks start
// on 32-column boundaries (the field's width and the box's first column
// multiples of 32, the box width a multiple of 4).  Other streams and boxes take
// the general tile of grad.hip; both give the same values bit for bit.
//
// A workgroup of 256 threads owns a tile of TXL columns x kTY rows and marches
// along z (the blockwise window of Alg. 3 with the planes as its blocks).
//  * Every stencil lane owns 4 consecutive columns x 4 rows: one 16-byte LDS
//    read per row gives a row's four values (x-neighbours inside the lane in
//    registers), one 16-byte store writes four results.
//  * The decoded planes are double-buffered in LDS, so one barrier per plane
//    separates "plane p+1 decoded" from "plane p read".  A decode thread owns
//    one block of one decoded row (rows y0-1 .. y0+kTY, the blocks covering
//    columns x0-1 .. x0+TXL); its payload words are staged in a private LDS
//    column, so staging needs no barrier.  The two plane buffers and the
//    staging columns take under 64 KiB, two workgroups per compute unit.  While the stencil of plane p runs,
//    the payload of plane p+2 and the metadata of plane p+3 are in flight.
//  * A block is decoded two slots per 32-bit window (2 w <= 28 bits), and four
//    decoded slots go to LDS in one 16-byte write.  A row of the plane buffer
//    holds one 4-word pad per 32 columns, which keeps both the decode writes
//    and the stencil reads free of bank conflicts.
//  * z-neighbours live in registers: the loop is unrolled by three so the
//    planes p-2, p-1, p rotate through three register sets without copies.
//  * Domain edges use ghost values q_{-1} = 2 q_0 - q_1 (and the mirror at the
//    far end), formed in registers: the central numerator then equals the
//    one-sided 2 (q_1 - q_0) exactly in integers (a length-1 axis adds 0).
//  * ACC (batches): the exact sums of q and q^2 over the tile's own elements,
//    for statistics sharing this decode; per plane in 32 bits (16 values of
//    |q| < 8192), then widened.
#include "hsz_device.hpp"
#include "hsz_launch.hpp"
#include "hsz_stats.hpp"

namespace hsz {

namespace {

constexpr int kQ4Threads = 256;
constexpr int kQ4MaxW = 14;  // |p| < 2^14 when max|q| < 8192
constexpr int kQ4NS = 256;   // staging columns (words between two rows of a column)

typedef __attribute__((address_space(3))) int lds_i32;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef int i4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <int S, int TXL>
struct Q4 {
  static constexpr int kG = TXL / 4;            // stencil lanes per row group
  static constexpr int kRG = kQ4Threads / kG;   // row groups (one or more whole waves each)
  static constexpr int kRY = 4;                 // rows per stencil lane
  static constexpr int kTY = kRG * kRY;         // output rows per tile
  static constexpr int kRows = kTY + 2;         // decoded rows (one halo row each side)
  static constexpr int kNBR = TXL / S + 2;      // blocks per decoded row, at most
  static constexpr int kItems = kRows * kNBR;   // decode items
  static constexpr int kIPW = (kItems + 3) / 4; // decode items per wave
  static constexpr int kPitch = 36 * ((TXL + 2 * S) / 32);  // words per LDS row
  static constexpr int kPlane = kRows * kPitch;             // words per plane buffer
  static constexpr int kPF = (S / 32) * (1 + kQ4MaxW) + 1;  // words staged per block (+ the spare a window reads)
  static constexpr int kStageOff = (2 * kPlane + 63) / 64 * 64;  // 256-byte aligned: row offsets fold into ds_read2st64
  static constexpr int kLdsWords = kStageOff + kPF * kQ4NS;
  static_assert(S == 32 && kPF == 16, "blocks of 32: at most 15 payload words");
  static_assert(kIPW <= kWave && 3 * kIPW + kWave <= kQ4NS, "one staging column per item, spares for idle lanes");
  static_assert(kG % kWave == 0 && kRG * kG == kQ4Threads, "whole waves per row group");
  static_assert(kStageOff * 4 < 65536, "staging rows addressed with instruction offsets");
};

// LDS word of extended column e of a row (e = x - x0 + S, so the block that
// holds column x0 - 1 starts at e = 0): one 4-word pad per 32 columns
__device__ __forceinline__ int q4w(int e) { return 36 * (e >> 5) + (e & 31); }

// buffer descriptor of 'bytes' bytes at 'base': loads past the end return 0
__device__ __forceinline__ __amdgpu_buffer_rsrc_t q4_rsrc(const void* base, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(uint32_t)bytes, 0x00020000);
}

// An offset past the end of every output (outputs stay below 2 GiB): a
// buffer store there is discarded by the hardware.
constexpr uint32_t kNoStore = 0x80000000u;

// 16-byte store at byte offset 'off' of r, the whole offset in the vector
// operand and soffset zero.  The store reads its data registers after issue,
// and a VALU write to them in the very next instruction corrupts the last
// lanes read; the backend pads that case with a wait state only for stores
// whose soffset is not a register, so an offset split into an SGPR soffset
// would leave it unguarded.  The results are written once and not read by
// the kernel: non-temporal (cache policy nt), which measured a few percent
// faster for the magnitude than the default policy.
constexpr int kStoreNT = 2;
__device__ __forceinline__ void store_b128(const f4& v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i4, v), r, off, 0, kStoreNT);
}

// Decode one staged block (payload words in LDS column 'col', rows kQ4NS
// words apart) into row[q4w(e0 + j)], e0 a multiple of 32: two slots per
// 32-bit window, four slots per 16-byte LDS write.  gl / gr: also write the
// ghost column before the row (2 q_0 - q_1) / after it (2 q_31 - q_30).
template <int S>
__device__ __forceinline__ void decode_q4(const lds_u32* col, int w, int q0, lds_i32* row, int e0, bool gl,
                                          bool gr) {
  const uint32_t sg0 = col[0];
  const lds_u32* mag = col + kQ4NS;
  int q = q0;
  uint32_t uw = (uint32_t)w, pos = 0;
  const uint32_t w2 = 2u * uw;
  int first[2] = {0, 0}, last[2] = {0, 0};
#pragma unroll
  for (int g = 0; g < S; g += 8) {
    // bit positions j w of the four pairs, by additions (the empty asm keeps
    // the compiler from folding them into multiplies or hoisting later groups)
    asm volatile("" : "+v"(pos));
    uint32_t lo[4], hi[4], pp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      pp[u] = pos;
      pos += w2;
      uint32_t k = pp[u] >> 5;
      asm("" : "+v"(k));  // one shift-add per address
      const lds_u32* a = mag + k * kQ4NS;
      lo[u] = a[0];
      hi[u] = a[kQ4NS];
    }
    int vals[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = g + 2 * u;
      const uint32_t win = __builtin_amdgcn_alignbit(hi[u], lo[u], pp[u]);
      const uint32_t m0 = __builtin_amdgcn_ubfe(win, 0u, uw);
      const uint32_t m1 = __builtin_amdgcn_ubfe(win, uw, uw);
      const int s0 = __builtin_amdgcn_sbfe((int)sg0, (uint32_t)j, 1u);
      const int s1 = __builtin_amdgcn_sbfe((int)sg0, (uint32_t)(j + 1), 1u);
      q = (int)((m0 ^ (uint32_t)s0) + (uint32_t)q) - s0;  // q += (m ^ s) - s
      vals[2 * u] = q;
      q = (int)((m1 ^ (uint32_t)s1) + (uint32_t)q) - s1;
      vals[2 * u + 1] = q;
    }
    *(__attribute__((address_space(3))) i4*)(row + q4w(e0 + g)) = i4{vals[0], vals[1], vals[2], vals[3]};
    *(__attribute__((address_space(3))) i4*)(row + q4w(e0 + g + 4)) = i4{vals[4], vals[5], vals[6], vals[7]};
    if (g == 0) { first[0] = vals[0]; first[1] = vals[1]; }
    if (g == S - 8) { last[0] = vals[7]; last[1] = vals[6]; }
  }
  if (gl) row[q4w(e0 - 1)] = 2 * first[0] - first[1];
  if (gr) row[q4w(e0 + S)] = 2 * last[0] - last[1];
}

template <int S, int TXL, int ACC>
__device__ __forceinline__ void gradmag_tile_q4(const GradJob& job, int64_t tile, uint32_t* smem_g, int* status) {
  using L = Q4<S, TXL>;
  constexpr int P = L::kPitch;
  const StreamView& v = job.v;
  const Dims3 d = job.d;
  const Box3 b = job.b;
  const int tz = job.tz, kmax = job.kmax;
  const float h = (float)job.halfq;
  lds_u32* const smem = (lds_u32*)smem_g;
  lds_i32* const planes = (lds_i32*)smem;
  lds_u32* const stage = smem + L::kStageOff;
  const int t = threadIdx.x;

  // bounds-checked views of the stream's sections and of the result
  // metadata sections through one view of the stream (section offsets as the
  // scalar offset; every metadata index is in range), the payload through its
  // own (words past its end read 0)
  const __amdgpu_buffer_rsrc_t r_meta = q4_rsrc(v.base, (const uint8_t*)v.payload - v.base);
  const int so_w = (int)(v.width - v.base), so_q0 = (int)((const uint8_t*)v.q0 - v.base);
  const int so_co = (int)((const uint8_t*)v.chunk_off - v.base);
  const __amdgpu_buffer_rsrc_t r_pay = q4_rsrc(v.payload, v.payload_words * 4);
  const __amdgpu_buffer_rsrc_t r_rel = q4_rsrc(job.rel, 2 * (uint64_t)v.nb);
  const __amdgpu_buffer_rsrc_t r_out = q4_rsrc(job.out, 4 * (uint64_t)((b.z1 - b.z0) * (b.y1 - b.y0) * (b.x1 - b.x0)));

  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int64_t ntx = (bx + TXL - 1) / TXL, nty = (by + L::kTY - 1) / L::kTY;
  int64_t blk = tile;
  const int64_t tx = blk % ntx;
  blk /= ntx;
  const int64_t ty = blk % nty;
  const int64_t tzi = blk / nty;
  const int64_t x0 = b.x0 + tx * TXL, y0 = b.y0 + ty * L::kTY, z0 = b.z0 + tzi * tz;
  const int xs = (int)min((int64_t)TXL, b.x1 - x0), ys = (int)min((int64_t)L::kTY, b.y1 - y0);
  const int64_t zs = min((int64_t)tz, b.z1 - z0);
  const int64_t za = max((int64_t)0, z0 - 1), zb = min(d.z, z0 + zs + 1);
  const uint32_t bpr = (uint32_t)(d.x / S);  // blocks per field row (d.x is a multiple of S)

  // ---- decode item of this thread: the items are spread evenly over the four
  // waves, and consecutive lanes own consecutive staging columns
  const int lane = t % kWave;
  const int item = (t / kWave) * L::kIPW + lane;
  const int dr = item / L::kNBR, dk = item % L::kNBR;
  const int64_t dy = y0 - 1 + dr;
  const int64_t fb = x0 > 0 ? x0 / S - 1 : 0;      // first block of the row range
  const int64_t lb = min((int64_t)bpr - 1, (x0 + xs) / S);  // last block
  const bool decoder = lane < L::kIPW && item < L::kItems && dr <= ys + 1 && dy >= 0 && dy < d.y && fb + dk <= lb;
  const int e0 = (int)((fb + dk) * S - x0 + S);     // extended column of slot 0
  const bool gl = decoder && x0 == 0 && dk == 0;    // ghost column before the field's first column
  const bool gr = decoder && x0 + xs == d.x && fb + dk == (int64_t)bpr - 1;  // after its last
  const int drow = dr * P;
  // staging column: the item's own; idle lanes write their (unused) words to
  // columns no decode item owns
  lds_u32* const col = stage + (lane < L::kIPW ? item : 4 * L::kIPW + (lane - L::kIPW));
  // block of this item in plane za, and the step from one plane to the next
  const uint32_t bk0 = decoder ? (uint32_t)((za * d.y + dy) * (int64_t)bpr + fb + dk) : 0u;
  const uint32_t pstride = (uint32_t)(d.y * (int64_t)bpr);

  struct Meta {
    int w, q0, words;
    uint32_t off;
    bool valid;
  };
  auto meta_of = [&](int64_t p) {
    Meta m;
    m.valid = decoder && p < zb;
    const uint32_t bk = m.valid ? bk0 + (uint32_t)(p - za) * pstride : 0u;
    m.w = (int)__builtin_amdgcn_raw_buffer_load_b8(r_meta, bk, so_w, 0);
    m.q0 = (int)__builtin_amdgcn_raw_buffer_load_b32(r_meta, 4 * bk, so_q0, 0);
    const uint32_t rel = __builtin_amdgcn_raw_buffer_load_b16(r_rel, 2 * bk, 0, 0);
    const uint32_t cl = __builtin_amdgcn_raw_buffer_load_b32(r_meta, 8 * (bk / kChunkBlocks), so_co, 0);
    m.off = cl + rel;  // payload words stay below 2^29 (the eligibility test)
    m.words = 0;
    return m;
  };
  auto check = [&](Meta& m) {
    m.words = m.valid ? block_words<S>(m.w) : 0;
    if (m.valid && (m.w > kQ4MaxW || m.words > kmax || (uint64_t)m.off + (uint64_t)m.words > v.payload_words)) {
      record_status(status, kErrBadStream);
      m.w = 0;
      m.words = 0;
    }
  };
  // the block's first kPF payload words (loads past the payload return 0;
  // an invalid block reads nothing) into registers, then to the staging column
  auto fetch = [&](const Meta& m, uint32_t (&pw)[L::kPF]) {
    const uint32_t base = m.words ? 4 * m.off : 0x80000000u;
#pragma unroll
    for (int k = 0; k < L::kPF; ++k) pw[k] = __builtin_amdgcn_raw_buffer_load_b32(r_pay, base + 4 * k, 0, 0);
  };
  auto stage_words = [&](const uint32_t (&pw)[L::kPF]) {
#pragma unroll
    for (int k = 0; k < L::kPF; ++k) col[k * kQ4NS] = pw[k];
  };

  // ---- stencil lanes: 4 columns x 4 rows; the row group is wave-uniform
  const int rg = __builtin_amdgcn_readfirstlane(t / L::kG);
  const int c4 = 4 * (t % L::kG);
  const bool active = c4 < xs;
  const int cw = q4w(S + c4), cwm = q4w(S + c4 - 1), cwp = q4w(S + c4 + 4);
  const bool top = y0 == 0 && rg == 0;                          // row 0 of the tile: ghost above the field
  const int kb = (y0 + ys == d.y) ? ys + 1 - L::kRY * rg : -1;  // lane-row of the ghost below, if any
  const bool y2 = d.y >= 2, z2 = d.z >= 2;
  int nrows = ys - L::kRY * rg;                                 // output rows of the row group
  nrows = nrows < 0 ? 0 : (nrows > L::kRY ? L::kRY : nrows);
  // byte offsets in the result: this lane's columns, and the row group's first row
  const uint32_t ocol = 4u * (uint32_t)((x0 - b.x0) + c4);
  const int64_t orow0 = (y0 + L::kRY * rg - b.y0) * bx;

  int Q[3][4][4];    // q of three consecutive planes (rotating roles)
  uint32_t G[4][4];  // nx^2 + ny^2 of the previous plane
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) Q[r][i][j] = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) G[i][j] = 0u;
  int as1 = 0;
  uint64_t as2 = 0;

  // one output plane o from the numerators of plane o (G, nz); sums of its q
  auto emit = [&](int64_t o, const int (&qo)[4][4], const int (&nz)[4][4]) {
    const int64_t orow = ((o - b.z0) * by) * bx + orow0;
    uint32_t s2p = 0;
    int s1p = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i < nrows) {
        f4 r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t s = G[i][j] + (uint32_t)__mul24(nz[i][j], nz[i][j]);
          r[j] = __builtin_amdgcn_sqrtf((float)s) * h;
        }
        if (active) store_b128(r, r_out, ocol + (uint32_t)(4 * (orow + i * bx)));
        if constexpr (ACC == 1) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            s1p += qo[i][j];
            s2p += (uint32_t)__mul24(qo[i][j], qo[i][j]);
          }
        }
      }
    }
    if constexpr (ACC == 1) {
      if (active) {
        as1 += s1p;
        as2 += s2p;
      }
    }
  };

  // plane p is in buffer 'buf'; emits plane p - 1.  C: register set of plane p.
  auto stencil = [&](auto RC, int64_t p, const lds_i32* buf) {
    constexpr int C = decltype(RC)::value, M1 = (C + 2) % 3, M2 = (C + 1) % 3;
    const lds_i32* rb = buf + L::kRY * rg * P;
    int vv[6][4];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const i4 a = *(const __attribute__((address_space(3))) i4*)(rb + k * P + cw);
      vv[k][0] = a.x; vv[k][1] = a.y; vv[k][2] = a.z; vv[k][3] = a.w;
    }
    int xm[4], xp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xm[i] = rb[(i + 1) * P + cwm];
      xp[i] = rb[(i + 1) * P + cwp];
    }
    if (top) {
#pragma unroll
      for (int j = 0; j < 4; ++j) vv[0][j] = y2 ? 2 * vv[1][j] - vv[2][j] : vv[1][j];
    }
    if (kb >= 2 && kb <= 5) {
#pragma unroll
      for (int k = 2; k < 6; ++k)
        if (k == kb) {
#pragma unroll
          for (int j = 0; j < 4; ++j) vv[k][j] = y2 ? 2 * vv[k - 1][j] - vv[k - 2][j] : vv[k - 1][j];
        }
    }
    const int64_t o = p - 1;
    if (o == 0) {  // the field's first plane: ghost plane q_{-1} = 2 q_0 - q_1 (q_0 on a length-1 axis)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) Q[M2][i][j] = z2 ? 2 * Q[M1][i][j] - vv[i + 1][j] : Q[M1][i][j];
    }
    if (o >= z0 && o < z0 + zs) {
      int nz[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) nz[i][j] = vv[i + 1][j] - Q[M2][i][j];
      emit(o, Q[M1], nz);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int qc = vv[i + 1][j];
        const int nx = (j < 3 ? vv[i + 1][j + 1] : xp[i]) - (j > 0 ? vv[i + 1][j - 1] : xm[i]);
        const int ny = vv[i + 2][j] - vv[i][j];
        G[i][j] = (uint32_t)__mul24(nx, nx) + (uint32_t)__mul24(ny, ny);
        Q[C][i][j] = qc;
      }
    }
  };

  // one plane of the march: decode plane p+1 into the other buffer, fetch
  // plane p+2's payload and plane p+3's metadata, stencil on plane p
  Meta cur, nn;
  auto step = [&](auto RC, int64_t p) {
    const bool odd = ((p - za) & 1) != 0;
    const lds_i32* buf = planes + (odd ? L::kPlane : 0);
    lds_i32* nbuf = planes + (odd ? 0 : L::kPlane);
    if (cur.valid) decode_q4<S>(col, cur.w, cur.q0, nbuf + drow, e0, gl, gr);
    check(nn);
    uint32_t pw[L::kPF];
    fetch(nn, pw);
    const Meta n3 = meta_of(p + 3);
    stencil(RC, p, buf);
    stage_words(pw);
    cur = nn;
    nn = n3;
    lds_barrier();
  };

  // prologue: plane za decoded into buffer 0, plane za+1 staged, metadata of za+2 in flight
  {
    uint32_t pw[L::kPF];
    cur = meta_of(za);
    Meta nx = meta_of(za + 1);
    check(cur);
    fetch(cur, pw);
    stage_words(pw);
    if (cur.valid) decode_q4<S>(col, cur.w, cur.q0, planes + drow, e0, gl, gr);
    check(nx);
    fetch(nx, pw);
    stage_words(pw);
    cur = nx;
    nn = meta_of(za + 2);
    lds_barrier();
  }

  // the march, unrolled by three (plane p's values go to register set (p - za) % 3)
  int64_t p = za;
  for (; p + 3 <= zb; p += 3) {
    step(std::integral_constant<int, 0>{}, p);
    step(std::integral_constant<int, 1>{}, p + 1);
    step(std::integral_constant<int, 2>{}, p + 2);
  }
  const int rem = (int)(zb - p);
  if (rem >= 1) step(std::integral_constant<int, 0>{}, p);
  if (rem >= 2) step(std::integral_constant<int, 1>{}, p + 1);

  // the field's last plane has no plane after it: one-sided (0 if d.z = 1)
  if (z0 + zs == zb) {
    const int64_t o = zb - 1;
    const int last = rem == 0 ? 2 : rem - 1;  // register set of plane zb - 1
    auto tail = [&](auto RC) {
      constexpr int C = decltype(RC)::value, M1 = (C + 2) % 3;
      int nz[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) nz[i][j] = z2 ? 2 * (Q[C][i][j] - Q[M1][i][j]) : 0;
      emit(o, Q[C], nz);
    };
    if (last == 0) tail(std::integral_constant<int, 0>{});
    else if (last == 1) tail(std::integral_constant<int, 1>{});
    else tail(std::integral_constant<int, 2>{});
  }
  if constexpr (ACC == 1) {
    const int64_t cnt = active ? (int64_t)nrows * 4 * zs : 0;
    U128 s2 = {as2, 0};
    acc_add_group((BatchAcc*)job.acc, (int64_t)as1, cnt, s2, (BatchAcc*)(smem_g + L::kLdsWords), kQ4Threads / kWave);
  }
}

// ---- wide rows: q as 16-bit pairs -------------------------------------------------
// Boxes wider than 256 columns take a 512 x 16 tile of 512 threads (eight
// waves).  With max|q| < 8192 every q, every ghost value (2 q_0 - q_1) and
// every numerator fits 16 bits, so the decoded planes hold q as 16-bit pairs
// (half the LDS of the tile above: two workgroups of eight waves per compute
// unit) and the stencil works on pairs: numerators by packed subtractions,
// squares summed by 16-bit dot products into 32 bits (exact: three squares
// of |n| < 2^15 stay below 2^32).  Wave w
// owns rows 2w, 2w+1 of the tile and lane l the columns 4l .. 4l+3 and
// 256+4l .. 256+4l+3, so each 16-byte store of a wave writes 1 KiB of one
// row contiguously; a lane's x-neighbours come from the lanes beside it
// (wave shifts), the wave's outer ones from LDS.
constexpr int kQ8Threads = 512;
constexpr int kQ8TXL = 512;
constexpr int kQ8RY = 2;                             // rows per lane
constexpr int kQ8TY = kQ8RY * (kQ8Threads / kWave);  // 16
constexpr int kQ8Rows = kQ8TY + 2;
constexpr int kQ8NBR = kQ8TXL / 32 + 2;              // blocks per decoded row, at most
constexpr int kQ8Items = kQ8Rows * kQ8NBR;           // 324
constexpr int kQ8NS = 512;                           // staging columns
// words per LDS row: 576 16-bit columns (288 words), padded to 4 (mod 64) so
// the 16-byte decode writes of consecutive rows fall in distinct banks
constexpr int kQ8Pitch = 324;
constexpr int kQ8Plane = kQ8Rows * kQ8Pitch;
constexpr int kQ8StageOff = (2 * kQ8Plane + 63) / 64 * 64;
constexpr int kQ8PF = 16;
constexpr int kQ8LdsWords = kQ8StageOff + kQ8PF * kQ8NS;
static_assert(kQ8Items + kWave <= kQ8NS, "a staging column per item, spares for the idle lanes of a wave");
static_assert(kQ8Pitch * 2 >= (kQ8TXL + 64) && kQ8Pitch % 64 == 4, "row pitch");
static_assert((kQ8LdsWords * 4 + (kQ8Threads / kWave) * 32) * 2 <= 163840, "two workgroups per compute unit");

typedef short s2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) short lds_i16;

__device__ __forceinline__ int pk_sub(int a, int b) {
  return __builtin_bit_cast(int, __builtin_bit_cast(s2, a) - __builtin_bit_cast(s2, b));
}
__device__ __forceinline__ int pk_add(int a, int b) {
  return __builtin_bit_cast(int, __builtin_bit_cast(s2, a) + __builtin_bit_cast(s2, b));
}
// squares of 16-bit halves through 16-bit dot products (all 32-bit sums are
// taken modulo 2^32 and read as unsigned: a sum of three squares of |n| < 2^15
// stays below 2^32): sq2lo(x, y, c) = c + x.lo^2 + y.lo^2, sq2hi the high
// halves; sq1lo(z, c) = c + z.lo^2, sq1hi(z, c) = c + z.hi^2
__device__ __forceinline__ int dot2(int a, int b, int c);
__device__ __forceinline__ uint32_t sq2lo(int x, int y, uint32_t c) {
  const int p = (int)__builtin_amdgcn_perm((uint32_t)y, (uint32_t)x, 0x05040100u);  // (x.lo, y.lo)
  return (uint32_t)dot2(p, p, (int)c);
}
__device__ __forceinline__ uint32_t sq2hi(int x, int y, uint32_t c) {
  const int p = (int)__builtin_amdgcn_perm((uint32_t)y, (uint32_t)x, 0x07060302u);  // (x.hi, y.hi)
  return (uint32_t)dot2(p, p, (int)c);
}
__device__ __forceinline__ uint32_t sq1lo(int z, uint32_t c) { return (uint32_t)dot2(z, z & 0xffff, (int)c); }
__device__ __forceinline__ uint32_t sq1hi(int z, uint32_t c) { return (uint32_t)dot2(z, z & (int)0xffff0000u, (int)c); }
__device__ __forceinline__ int dot2(int a, int b, int c) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(s2, a), __builtin_bit_cast(s2, b), c, false);
}
// the 16-bit pair (lo, hi)
__device__ __forceinline__ int pk(int lo, int hi) { return (int)__builtin_amdgcn_perm((uint32_t)hi, (uint32_t)lo, 0x05040100u); }

// Decode one staged block into 16-bit q at halfwords e0 .. e0+31 of 'row'
// (e0 a multiple of 32), with the optional ghost columns before and after.
__device__ __forceinline__ void decode_q8(const lds_u32* col, int w, int q0, lds_i16* row, int e0, bool gl, bool gr) {
  const uint32_t sg0 = col[0];
  const lds_u32* mag = col + kQ8NS;
  int q = q0;
  uint32_t uw = (uint32_t)w, pos = 0;
  const uint32_t w2 = 2u * uw;
  int first[2] = {0, 0}, last[2] = {0, 0};
#pragma unroll
  for (int g = 0; g < 32; g += 8) {
    asm volatile("" : "+v"(pos));
    uint32_t lo[4], hi[4], pp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      pp[u] = pos;
      pos += w2;
      uint32_t k = pp[u] >> 5;
      asm("" : "+v"(k));
      const lds_u32* a = mag + k * kQ8NS;
      lo[u] = a[0];
      hi[u] = a[kQ8NS];
    }
    int packed[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = g + 2 * u;
      const uint32_t win = __builtin_amdgcn_alignbit(hi[u], lo[u], pp[u]);
      const uint32_t m0 = __builtin_amdgcn_ubfe(win, 0u, uw);
      const uint32_t m1 = __builtin_amdgcn_ubfe(win, uw, uw);
      const int s0 = __builtin_amdgcn_sbfe((int)sg0, (uint32_t)j, 1u);
      const int s1 = __builtin_amdgcn_sbfe((int)sg0, (uint32_t)(j + 1), 1u);
      const int qa = (int)((m0 ^ (uint32_t)s0) + (uint32_t)q) - s0;
      q = (int)((m1 ^ (uint32_t)s1) + (uint32_t)qa) - s1;
      packed[u] = pk(qa, q);
      if (g == 0 && u == 0) { first[0] = qa; first[1] = q; }
      if (g == 24 && u == 3) { last[0] = q; last[1] = qa; }
    }
    *(__attribute__((address_space(3))) i4*)(row + e0 + g) = i4{packed[0], packed[1], packed[2], packed[3]};
  }
  if (gl) row[e0 - 1] = (short)(2 * first[0] - first[1]);
  if (gr) row[e0 + 32] = (short)(2 * last[0] - last[1]);
}

template <int ACC>
__device__ __forceinline__ void gradmag_tile_q8(const GradJob& job, int64_t tile, uint32_t* smem_g, int* status) {
  constexpr int S = 32, P = kQ8Pitch;
  const StreamView& v = job.v;
  const Dims3 d = job.d;
  const Box3 b = job.b;
  const int tz = job.tz, kmax = job.kmax;
  const float h = (float)job.halfq;
  lds_u32* const smem = (lds_u32*)smem_g;
  lds_u32* const stage = smem + kQ8StageOff;
  const int t = threadIdx.x;

  const __amdgpu_buffer_rsrc_t r_meta = q4_rsrc(v.base, (const uint8_t*)v.payload - v.base);
  const int so_w = (int)(v.width - v.base), so_q0 = (int)((const uint8_t*)v.q0 - v.base);
  const int so_co = (int)((const uint8_t*)v.chunk_off - v.base);
  const __amdgpu_buffer_rsrc_t r_pay = q4_rsrc(v.payload, v.payload_words * 4);
  const __amdgpu_buffer_rsrc_t r_rel = q4_rsrc(job.rel, 2 * (uint64_t)v.nb);
  const __amdgpu_buffer_rsrc_t r_out =
      q4_rsrc(job.out, 4 * (uint64_t)((b.z1 - b.z0) * (b.y1 - b.y0) * (b.x1 - b.x0)));

  const int64_t bx = b.x1 - b.x0, by = b.y1 - b.y0;
  const int64_t ntx = (bx + kQ8TXL - 1) / kQ8TXL, nty = (by + kQ8TY - 1) / kQ8TY;
  int64_t blk = tile;
  const int64_t tx = blk % ntx;
  blk /= ntx;
  const int64_t ty = blk % nty;
  const int64_t tzi = blk / nty;
  const int64_t x0 = b.x0 + tx * kQ8TXL, y0 = b.y0 + ty * kQ8TY, z0 = b.z0 + tzi * tz;
  const int xs = (int)min((int64_t)kQ8TXL, b.x1 - x0), ys = (int)min((int64_t)kQ8TY, b.y1 - y0);
  const int64_t zs = min((int64_t)tz, b.z1 - z0);
  const int64_t za = max((int64_t)0, z0 - 1), zb = min(d.z, z0 + zs + 1);
  const uint32_t bpr = (uint32_t)(d.x / S);

  // ---- decode item: block k of decoded row dr (consecutive lanes take
  // consecutive rows of one block column)
  // The tile's items (rows x blocks of a row) are spread evenly over as few
  // waves as hold them; the other waves neither fetch nor decode.
  const int lane = t % kWave, wv = __builtin_amdgcn_readfirstlane(t / kWave);
  const int64_t fb = x0 > 0 ? x0 / S - 1 : 0;
  const int64_t lb = min((int64_t)bpr - 1, (x0 + xs) / S);
  const int items = kQ8Rows * (int)(lb - fb + 1);
  const int ndw = (items + kWave - 1) / kWave, ipw = (items + ndw - 1) / ndw;
  const bool dwave = wv < ndw;
  const int item = wv * ipw + lane;
  const int dk = item / kQ8Rows, dr = item % kQ8Rows;
  const int64_t dy = y0 - 1 + dr;
  const bool decoder = dwave && lane < ipw && item < items && dr <= ys + 1 && dy >= 0 && dy < d.y;
  const int e0 = (int)((fb + dk) * S - x0 + S);
  const bool gl = decoder && x0 == 0 && dk == 0;
  const bool gr = decoder && x0 + xs == d.x && fb + dk == (int64_t)bpr - 1;
  const int drow = dr * P;
  lds_u32* const col = stage + (lane < ipw ? item : kQ8Items + (lane - ipw));
  const uint32_t bk0 = decoder ? (uint32_t)((za * d.y + dy) * (int64_t)bpr + fb + dk) : 0u;
  const uint32_t pstride = (uint32_t)(d.y * (int64_t)bpr);

  // a block's metadata: the loads are issued a plane ahead and their values
  // combined only when used (check), never right after the loads
  struct Meta {
    int w, q0;
    uint32_t cl, rel;  // chunk offset and offset in the chunk
  };
  auto valid_at = [&](int64_t p) { return decoder && p < zb; };
  auto meta_of = [&](int64_t p) {
    Meta m;
    const uint32_t bk = valid_at(p) ? bk0 + (uint32_t)(p - za) * pstride : 0u;
    m.w = (int)__builtin_amdgcn_raw_buffer_load_b8(r_meta, bk, so_w, 0);
    m.q0 = (int)__builtin_amdgcn_raw_buffer_load_b32(r_meta, 4 * bk, so_q0, 0);
    m.rel = __builtin_amdgcn_raw_buffer_load_b16(r_rel, 2 * bk, 0, 0);
    m.cl = __builtin_amdgcn_raw_buffer_load_b32(r_meta, 8 * (bk / kChunkBlocks), so_co, 0);
    return m;
  };
  // payload words of plane p's block (0 if it has none) and their offset; a
  // block whose metadata disagrees with the stream is reported and decoded
  // with width 0
  auto check = [&](Meta& m, int64_t p, uint32_t& off) -> int {
    off = m.cl + m.rel;
    const bool ok = valid_at(p);
    int words = ok ? block_words<S>(m.w) : 0;
    if (ok && (m.w > kQ4MaxW || words > kmax || (uint64_t)off + (uint64_t)words > v.payload_words)) {
      record_status(status, kErrBadStream);
      m.w = 0;
      words = 0;
    }
    return words;
  };
  auto fetch = [&](int words, uint32_t off, uint32_t (&pw)[kQ8PF]) {
    const uint32_t base = words ? 4 * off : 0x80000000u;
#pragma unroll
    for (int k = 0; k < kQ8PF; ++k) pw[k] = __builtin_amdgcn_raw_buffer_load_b32(r_pay, base + 4 * k, 0, 0);
  };
  auto stage_words = [&](const uint32_t (&pw)[kQ8PF]) {
#pragma unroll
    for (int k = 0; k < kQ8PF; ++k) col[k * kQ8NS] = pw[k];
  };

  // ---- stencil: wave wv owns rows 2 wv, 2 wv + 1 of the tile, lane the
  // column groups A = 4 lane .. 4 lane + 3 and B = 256 + 4 lane .. + 3
  // (halfwords S + .. of a row)
  const bool actA = 4 * lane < xs, actB = kQ8TXL / 2 + 4 * lane < xs;
  const int cwA = (S + 4 * lane) / 2, cwB = (S + kQ8TXL / 2 + 4 * lane) / 2;  // words of the groups
  const bool top = y0 == 0 && wv == 0;
  const int kb = (y0 + ys == d.y) ? ys + 1 - kQ8RY * wv : -1;  // window row of the ghost below
  const bool y2 = d.y >= 2, z2 = d.z >= 2;
  int nrows = ys - kQ8RY * wv;
  nrows = nrows < 0 ? 0 : (nrows > kQ8RY ? kQ8RY : nrows);
  const uint32_t ocol = 4u * (uint32_t)((x0 - b.x0) + 4 * lane);  // group A; group B 1 KiB further
  const int64_t orow0 = (y0 + kQ8RY * wv - b.y0) * bx;

  int Q[3][kQ8RY][4];        // q of three consecutive planes, 16-bit pairs
  uint32_t G[kQ8RY][8];      // nx^2 + ny^2 of the previous plane
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int i = 0; i < kQ8RY; ++i)
#pragma unroll
      for (int m = 0; m < 4; ++m) Q[r][i][m] = 0;
#pragma unroll
  for (int i = 0; i < kQ8RY; ++i)
#pragma unroll
    for (int e = 0; e < 8; ++e) G[i][e] = 0u;
  int as1 = 0;
  uint64_t as2 = 0;

  // output row i of plane o from its numerators (G of the row, nz) and its
  // stores; sums of its q.  Rows are emitted one at a time between the
  // stencil's arithmetic, which spreads a wave's stores over the plane.
  // The stores are issued on every path (a row or group with nothing to
  // write gets an offset past the end of the output, and the hardware
  // discards buffer stores out of range): with the same stores on every
  // path the compiler counts them exactly, and never waits for a step's
  // stores before the next step's metadata.
  auto emit_row = [&](int64_t o, int i, const int (&qo)[4], const int (&nzr)[4], bool live) {
    live = live && i < nrows;
    const int64_t orow = ((o - b.z0) * by) * bx + orow0;
    f4 r0, r1;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      r0[2 * m] = __builtin_amdgcn_sqrtf((float)sq1lo(nzr[m], G[i][2 * m])) * h;
      r0[2 * m + 1] = __builtin_amdgcn_sqrtf((float)sq1hi(nzr[m], G[i][2 * m + 1])) * h;
      r1[2 * m] = __builtin_amdgcn_sqrtf((float)sq1lo(nzr[m + 2], G[i][2 * m + 4])) * h;
      r1[2 * m + 1] = __builtin_amdgcn_sqrtf((float)sq1hi(nzr[m + 2], G[i][2 * m + 5])) * h;
    }
    const uint32_t so = ocol + (uint32_t)(4 * (orow + i * bx));
    store_b128(r0, r_out, live && actA ? so : kNoStore);
    store_b128(r1, r_out, live && actB ? so + 2 * kQ8TXL : kNoStore);
    if constexpr (ACC == 1) {
      // per row and lane 8 values of |q| < 2^13: both sums exact in 32 bits
      int s1p = 0, s2p = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int qm = (live && (m < 2 ? actA : actB)) ? qo[m] : 0;
        s1p = dot2(qm, 0x00010001, s1p);
        s2p = dot2(qm, qm, s2p);
      }
      as1 += s1p;
      as2 += (uint32_t)s2p;
    }
  };

  auto stencil = [&](auto RC, int64_t p, const lds_u32* buf) {
    constexpr int C = decltype(RC)::value, M1 = (C + 2) % 3, M2 = (C + 1) % 3;
    const lds_u32* rb = buf + kQ8RY * wv * P;
    typedef int i2 __attribute__((ext_vector_type(2)));
    int A[4][4];  // per window row: group A's two pairs, then group B's
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const i2 a = *(const __attribute__((address_space(3))) i2*)(rb + k * P + cwA);
      const i2 c = *(const __attribute__((address_space(3))) i2*)(rb + k * P + cwB);
      A[k][0] = a.x; A[k][1] = a.y; A[k][2] = c.x; A[k][3] = c.y;
    }
    // the columns beside each group: from the neighbouring lanes; the wave's
    // outer ones from LDS (the high half of word S/2 - 1 is column x0 - 1,
    // the low half of word S/2 + 128 column x0 + 256, the high half of the
    // word before it column x0 + 255, the low half of word S/2 + 256 column
    // x0 + 512)
    int XM[kQ8RY][2], XP[kQ8RY][2];
#pragma unroll
    for (int i = 0; i < kQ8RY; ++i) {
      const lds_u32* r = rb + (i + 1) * P;
      const int emA = (int)r[S / 2 - 1], epA = (int)r[S / 2 + kQ8TXL / 4];
      const int emB = (int)r[S / 2 + kQ8TXL / 4 - 1], epB = (int)r[S / 2 + kQ8TXL / 2];
      XM[i][0] = __builtin_amdgcn_update_dpp(emA, A[i + 1][1], 0x138, 0xf, 0xf, false);  // wave_shr:1
      XP[i][0] = __builtin_amdgcn_update_dpp(epA, A[i + 1][0], 0x130, 0xf, 0xf, false);  // wave_shl:1
      XM[i][1] = __builtin_amdgcn_update_dpp(emB, A[i + 1][3], 0x138, 0xf, 0xf, false);
      XP[i][1] = __builtin_amdgcn_update_dpp(epB, A[i + 1][2], 0x130, 0xf, 0xf, false);
    }
    if (top) {
#pragma unroll
      for (int m = 0; m < 4; ++m) A[0][m] = y2 ? pk_sub(pk_add(A[1][m], A[1][m]), A[2][m]) : A[1][m];
    }
    if (kb >= 2 && kb <= 3) {
#pragma unroll
      for (int k = 2; k < 4; ++k)
        if (k == kb) {
#pragma unroll
          for (int m = 0; m < 4; ++m) A[k][m] = y2 ? pk_sub(pk_add(A[k - 1][m], A[k - 1][m]), A[k - 2][m]) : A[k - 1][m];
        }
    }
    const int64_t o = p - 1;
    if (o == 0) {  // ghost plane q_{-1} = 2 q_0 - q_1 (q_0 on a length-1 axis)
#pragma unroll
      for (int i = 0; i < kQ8RY; ++i)
#pragma unroll
        for (int m = 0; m < 4; ++m)
          Q[M2][i][m] = z2 ? pk_sub(pk_add(Q[M1][i][m], Q[M1][i][m]), A[i + 1][m]) : Q[M1][i][m];
    }
    const bool out_plane = o >= z0 && o < z0 + zs;
    int nz[kQ8RY][4];
#pragma unroll
    for (int i = 0; i < kQ8RY; ++i)
#pragma unroll
      for (int m = 0; m < 4; ++m) nz[i][m] = pk_sub(A[i + 1][m], Q[M2][i][m]);
#pragma unroll
    for (int i = 0; i < kQ8RY; ++i) {
      emit_row(o, i, Q[M1][i], nz[i], out_plane);  // before G[i] is replaced
      const int* a = A[i + 1];
      // per group g: (x-1, x), (x+1, x+2), (x+3, x+4) for its columns x .. x+3
      int T[2][3];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        T[g][0] = (int)__builtin_amdgcn_alignbit((uint32_t)a[2 * g], (uint32_t)XM[i][g], 16u);
        T[g][1] = (int)__builtin_amdgcn_alignbit((uint32_t)a[2 * g + 1], (uint32_t)a[2 * g], 16u);
        T[g][2] = (int)__builtin_amdgcn_alignbit((uint32_t)XP[i][g], (uint32_t)a[2 * g + 1], 16u);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int nx = pk_sub(T[m / 2][m % 2 + 1], T[m / 2][m % 2]), ny = pk_sub(A[i + 2][m], A[i][m]);
        G[i][2 * m] = sq2lo(nx, ny, 0u);
        G[i][2 * m + 1] = sq2hi(nx, ny, 0u);
        Q[C][i][m] = a[m];
      }
    }
  };

  // One plane: decode waves fetch plane p+2's payload (into registers) and
  // plane p+3's metadata and decode plane p+1 into the other buffer; every
  // wave then runs the stencil on plane p; the fetched words are staged last,
  // so the loads have the decode and the stencil to land.  The metadata of
  // plane q lives in M[(q - za) % 3], so no loaded value is ever copied
  // (a copy would have to wait for its load, and with it for every store
  // issued before).
  Meta M[3];
  uint32_t pw[kQ8PF];
  auto step = [&](auto RC, int64_t p) {
    constexpr int C = decltype(RC)::value, N1 = (C + 1) % 3, N2 = (C + 2) % 3;
    const bool odd = ((p - za) & 1) != 0;
    const lds_u32* buf = smem + (odd ? kQ8Plane : 0);
    lds_u32* nbuf = smem + (odd ? 0 : kQ8Plane);
    if (dwave) {
      uint32_t off;
      const int words = check(M[N2], p + 2, off);
      fetch(words, off, pw);
      M[C] = meta_of(p + 3);
      if (valid_at(p + 1)) decode_q8(col, M[N1].w, M[N1].q0, (lds_i16*)(nbuf + drow), e0, gl, gr);
    }
    stencil(RC, p, buf);
    if (dwave) stage_words(pw);
    lds_barrier();
  };

  // prologue: plane za decoded into buffer 0, plane za+1's words staged,
  // plane za+2's metadata in flight
  if (dwave) {
    M[0] = meta_of(za);
    M[1] = meta_of(za + 1);
    uint32_t off;
    int words = check(M[0], za, off);
    fetch(words, off, pw);
    stage_words(pw);
    if (valid_at(za)) decode_q8(col, M[0].w, M[0].q0, (lds_i16*)(smem + drow), e0, gl, gr);
    words = check(M[1], za + 1, off);
    fetch(words, off, pw);
    stage_words(pw);
    M[2] = meta_of(za + 2);
  }
  lds_barrier();

  // the march, unrolled by three (plane p's values go to register set (p - za) % 3)
  int64_t p = za;
  for (; p + 3 <= zb; p += 3) {
    step(std::integral_constant<int, 0>{}, p);
    step(std::integral_constant<int, 1>{}, p + 1);
    step(std::integral_constant<int, 2>{}, p + 2);
  }
  const int rem = (int)(zb - p);
  if (rem >= 1) step(std::integral_constant<int, 0>{}, p);
  if (rem >= 2) step(std::integral_constant<int, 1>{}, p + 1);

  if (z0 + zs == zb) {
    const int64_t o = zb - 1;
    const int last = rem == 0 ? 2 : rem - 1;
    auto tail = [&](auto RC) {
      constexpr int C = decltype(RC)::value, M1 = (C + 2) % 3;
      int nz[kQ8RY][4];
#pragma unroll
      for (int i = 0; i < kQ8RY; ++i)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int dlt = pk_sub(Q[C][i][m], Q[M1][i][m]);
          nz[i][m] = z2 ? pk_add(dlt, dlt) : 0;
        }
#pragma unroll
      for (int i = 0; i < kQ8RY; ++i) emit_row(o, i, Q[C][i], nz[i], true);
    };
    if (last == 0) tail(std::integral_constant<int, 0>{});
    else if (last == 1) tail(std::integral_constant<int, 1>{});
    else tail(std::integral_constant<int, 2>{});
  }
  if constexpr (ACC == 1) {
    const int64_t cnt = (int64_t)nrows * 4 * ((int)actA + (int)actB) * zs;
    U128 s2v = {as2, 0};
    acc_add_group((BatchAcc*)job.acc, (int64_t)as1, cnt, s2v, (BatchAcc*)(smem_g + kQ8LdsWords), kQ8Threads / kWave);
  }
}

// Tiles handed out so that the workgroups of one XCD (launch order modulo 8)
// take consecutive tiles -- neighbours in y, sharing their halo rows in that
// XCD's L2 -- in every full round of the grid.
__device__ __forceinline__ int64_t xcd_tile(int64_t base, int64_t total) {
  const int64_t g = gridDim.x;
  if ((g & 7) == 0 && base + g <= total) return base + (int64_t)(blockIdx.x & 7) * (g >> 3) + (blockIdx.x >> 3);
  return base + blockIdx.x;
}

template <int S, int TXL>
__global__ void __launch_bounds__(kQ4Threads, 2) k_gradmag_q4(GradJob job, int* status) {
  extern __shared__ uint32_t smem[];
  gradmag_tile_q4<S, TXL, 0>(job, xcd_tile(0, gridDim.x), smem, status);
}

template <int S, int TXL, int ACC>
__global__ void __launch_bounds__(kQ4Threads, 2) k_batch_gradmag_q4(const GradJob* __restrict__ jobs,
                                                                      const int64_t* __restrict__ tile_start,
                                                                      const int64_t* __restrict__ counts, int* status) {
  extern __shared__ uint32_t smem[];
  const int n = (int)counts[0];
  const int64_t total = counts[1];
  for (int64_t base = 0; base < total; base += gridDim.x) {
    const int64_t tile = xcd_tile(base, total);
    if (tile >= total) break;
    int lo = 0, hi = n - 1;  // last job whose first tile is <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (tile_start[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    const GradJob job = load_job(jobs, lo);
    gradmag_tile_q4<S, TXL, ACC>(job, tile - tile_start[lo], smem, status);
  }
}

__global__ void __launch_bounds__(kQ8Threads, 4) k_gradmag_q8(GradJob job, int* status) {
  extern __shared__ uint32_t smem[];
  gradmag_tile_q8<0>(job, xcd_tile(0, gridDim.x), smem, status);
}

template <int ACC>
__global__ void __launch_bounds__(kQ8Threads, 4) k_batch_gradmag_q8(const GradJob* __restrict__ jobs,
                                                                   const int64_t* __restrict__ tile_start,
                                                                   const int64_t* __restrict__ counts, int* status) {
  extern __shared__ uint32_t smem[];
  const int n = (int)counts[0];
  const int64_t total = counts[1];
  for (int64_t base = 0; base < total; base += gridDim.x) {
    const int64_t tile = xcd_tile(base, total);
    if (tile >= total) break;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (tile_start[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    const GradJob job = load_job(jobs, lo);
    gradmag_tile_q8<ACC>(job, tile - tile_start[lo], smem, status);
  }
}

// The batch's statistics summed in these tiles and finished by the last
// workgroup (errors recorded in the tail's live word)
__global__ void __launch_bounds__(kQ8Threads, 4) k_batch_gradmag_q8_tail(const GradJob* __restrict__ jobs,
                                                                        const int64_t* __restrict__ tile_start,
                                                                        const int64_t* __restrict__ counts,
                                                                        BatchTail tail) {
  extern __shared__ uint32_t smem[];
  const int n = (int)counts[0];
  const int64_t total = counts[1];
  for (int64_t base = 0; base < total; base += gridDim.x) {
    const int64_t tile = xcd_tile(base, total);
    if (tile >= total) break;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (tile_start[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    const GradJob job = load_job(jobs, lo);
    gradmag_tile_q8<1>(job, tile - tile_start[lo], smem, tail.live);
  }
  // the flag in the workgroup-sum words past the tile (free after the tiles)
  batch_tail(tail, (int*)(smem + kQ8LdsWords));
}

template <int S, int TXL>
size_t q4_lds() {
  return (size_t)Q4<S, TXL>::kLdsWords * sizeof(uint32_t) + (kQ4Threads / kWave) * sizeof(BatchAcc);
}
// the tile's LDS, then one BatchAcc per wave for the workgroup's sums
size_t q8_lds() { return (size_t)kQ8LdsWords * sizeof(uint32_t) + (kQ8Threads / kWave) * sizeof(BatchAcc); }

hipError_t run_q4(const GradJob& job, int* status, hipStream_t s) {
  const int txl = q4_txl(job.b);
  const int64_t grid = q4_tiles(job.b, job.tz, txl);
  if (txl == 512)
    hipLaunchKernelGGL(k_gradmag_q8, dim3((unsigned)grid), dim3(kQ8Threads), q8_lds(), s, job, status);
  else
    hipLaunchKernelGGL((k_gradmag_q4<32, 256>), dim3((unsigned)grid), dim3(kQ4Threads), (q4_lds<32, 256>()), s, job,
                       status);
  return hipGetLastError();
}

}  // namespace

// Column tile: 512 (the sixteen-bit tile) for boxes wider than 256 columns
// whose width is a multiple of 8, else 256.
int q4_txl(const Box3& b) {
  const int64_t bx = b.x1 - b.x0;
  return (bx > 256 && bx % 8 == 0) ? 512 : 256;
}

bool q4_eligible(const StreamView& v, int via, int op, const Dims3& d, const Box3& b) {
  // 32-bit offsets: every section and the result below 2 GiB
  return via == 3 && op == 4 && v.dtype == 1 && v.flags == 0 && v.max_abs_q < 8192u && v.block == 32 &&
         d.x % 32 == 0 && b.x0 % 32 == 0 && (b.x1 - b.x0) % 4 == 0 && v.payload_words < (1ull << 29) &&
         v.nb < (1ll << 29) && b.volume() < (1ll << 29);
}

int64_t q4_tiles(const Box3& b, int tz, int txl) {
  const int ty = txl == 512 ? kQ8TY : Q4<32, 256>::kTY;
  const int64_t ntx = (b.x1 - b.x0 + txl - 1) / txl, nty = (b.y1 - b.y0 + ty - 1) / ty;
  return ntx * nty * ((b.z1 - b.z0 + tz - 1) / tz);
}

int q4_kmax(int S) { return (S / 32) * (1 + kQ4MaxW); }

// Planes per tile for a single launch: long runs along z, but enough tiles to
// fill the chip.
int q4_tz(const Box3& b) {
  const int txl = q4_txl(b);
  const int ty = txl == 512 ? kQ8TY : Q4<32, 256>::kTY;
  const int64_t ntx = (b.x1 - b.x0 + txl - 1) / txl, nty = (b.y1 - b.y0 + ty - 1) / ty;
  const int64_t bz = b.z1 - b.z0;
  int64_t tz = bz;
  while (tz > 8 && ntx * nty * ((bz + tz - 1) / tz) < 1024) tz = (tz + 1) / 2;
  return (int)tz;
}

hipError_t launch_gradmag_q4(const GradJob& job, int* status, hipStream_t s) { return run_q4(job, status, s); }

hipError_t launch_batch_gradmag_q4(int S, int txl, int acc, const GradJob* jobs, const int64_t* tile_start,
                                   const int64_t* counts, int grid, int* status, hipStream_t s) {
  if (S != 32) return hipErrorInvalidValue;
  if (txl == 512) {
    if (acc == 1)
      hipLaunchKernelGGL(k_batch_gradmag_q8<1>, dim3(grid), dim3(kQ8Threads), q8_lds(), s, jobs, tile_start, counts,
                         status);
    else
      hipLaunchKernelGGL(k_batch_gradmag_q8<0>, dim3(grid), dim3(kQ8Threads), q8_lds(), s, jobs, tile_start, counts,
                         status);
  } else {
    if (acc == 1)
      hipLaunchKernelGGL((k_batch_gradmag_q4<32, 256, 1>), dim3(grid), dim3(kQ4Threads), (q4_lds<32, 256>()), s, jobs,
                         tile_start, counts, status);
    else
      hipLaunchKernelGGL((k_batch_gradmag_q4<32, 256, 0>), dim3(grid), dim3(kQ4Threads), (q4_lds<32, 256>()), s, jobs,
                         tile_start, counts, status);
  }
  return hipGetLastError();
}

hipError_t launch_batch_gradmag_q8_tail(const GradJob* jobs, const int64_t* tile_start, const int64_t* counts,
                                        int grid, const BatchTail& tail, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_gradmag_q8_tail, dim3(grid), dim3(kQ8Threads), q8_lds(), s, jobs, tile_start, counts,
                     tail);
  return hipGetLastError();
}

size_t batch_gradmag_q4_lds(int S, int txl) {
  if (S != 32) return 0;
  return txl == 512 ? q8_lds() : q4_lds<32, 256>();
}

}  // namespace hsz
