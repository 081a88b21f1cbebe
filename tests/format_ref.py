"""A second, pure-Python reading of the compressed byte format, used only by
tests to pin the oracle's encoder (and, on the GPU, to read streams the
library wrote).  It parses the stream field by field from the format rules
and shares no code with the oracle's C encoder/decoder.

Format (little-endian):
  header, 256 bytes:  "HSZ1", u16 version, u8 dtype, u8 ndim, u64 dims[3]
  (slow->fast, leading ones), u64 n, u32 S, u32 chunk_blocks (=64),
  f64 eps, f64 quantum, f64 1/quantum, f64 vmin, f64 vmax, u32 max|q|,
  u32 flags, u64 nb, u64 nchunks, u64 section offsets (chunk table, q0,
  widths, payload), u64 payload words, u64 total bytes.
  sections, each 256-byte aligned: u64 chunk_off[nchunks+1] (payload word
  index of each 64-block chunk's first block, then the total);
  i32 q0[nb] (absent when flags bit 1, HSZp-nd, is set); u8 width[nb];
  u32 payload[].  'pblocks' returns every block's S values of p in slot
  order; p and q read the blocks in order (the 1D partition).
  block with width w > 0: ceil(S/32) sign words (bit i set iff p_i < 0),
  then ceil(S*w/32) magnitude words, element i in stream bits
  [i*w, i*w+w), bit k = bit k%32 of word k//32.  w = 0: no words.
"""
from __future__ import annotations

import struct

import numpy as np


def parse(buf: bytes):
    buf = bytes(buf)
    assert buf[:4] == b"HSZ1"
    (version,) = struct.unpack_from("<H", buf, 4)
    dtype, ndim = buf[6], buf[7]
    dims = struct.unpack_from("<3Q", buf, 8)
    (n,) = struct.unpack_from("<Q", buf, 32)
    S, chunk_blocks = struct.unpack_from("<2I", buf, 40)
    eps, quantum, inv_quantum, vmin, vmax = struct.unpack_from("<5d", buf, 48)
    max_abs_q, flags = struct.unpack_from("<2I", buf, 88)
    nb, nchunks, off_chunk, off_q0, off_width, off_payload, pwords, total = struct.unpack_from("<8Q", buf, 96)
    chunk_off = struct.unpack_from(f"<{nchunks + 1}Q", buf, off_chunk)
    nd = bool(flags & 2)  # HSZp-nd: no q0 section, blocks of the nd partition
    q0 = [] if nd else list(struct.unpack_from(f"<{nb}i", buf, off_q0))
    width = list(buf[off_width:off_width + nb])
    payload = struct.unpack_from(f"<{pwords}I", buf, off_payload)
    p = [0] * (nb * S)
    pos = 0
    for b in range(nb):
        if b % chunk_blocks == 0:
            assert chunk_off[b // chunk_blocks] == pos, "chunk table disagrees with widths"
        w = width[b]
        if w == 0:
            continue
        nsign = -(-S // 32)
        nmag = -(-S * w // 32)
        words = payload[pos:pos + nsign + nmag]
        stream = 0
        for k, word in enumerate(words[nsign:]):
            stream |= word << (32 * k)
        for i in range(S):
            mag = (stream >> (i * w)) & ((1 << w) - 1)
            neg = (words[i // 32] >> (i % 32)) & 1
            p[b * S + i] = -mag if neg else mag
        pos += nsign + nmag
    assert chunk_off[nchunks] == pos == pwords
    assert total == off_payload + 4 * pwords
    pblocks = np.array(p, dtype=np.int64).reshape(nb, S)
    p = p[:n]
    q = []
    if not nd:
        for e in range(n):
            q.append(q0[e // S] if e % S == 0 else q[-1] + p[e])
    return dict(version=version, dtype=dtype, ndim=ndim, dims=dims, n=n, S=S, eps=eps,
                quantum=quantum, inv_quantum=inv_quantum, vmin=vmin, vmax=vmax,
                max_abs_q=max_abs_q, flags=flags, nb=nb, nchunks=nchunks, q0=q0, width=width,
                payload=list(payload), p=np.array(p, dtype=np.int64), q=np.array(q, dtype=np.int64),
                total=total, pblocks=pblocks, off_q0=off_q0, off_width=off_width)
