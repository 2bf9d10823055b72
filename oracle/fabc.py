"""FaBC walk-corpus codec -- TEST INFRASTRUCTURE ONLY (plain numpy).

Frequency-aware bitmap compression, Section 5.2.2 of the FeLoG paper:
  * profile: normalised symbol frequencies p(1) >= p(2) >= ... of a sampled
    corpus; F_k = p(1) + ... + p(k);
  * size model: S(k) = 4NL(1 - F_k) + 4Nk + Nk L/8 bytes (Eq. 6), ratio
    g(k) = S(k) / 4NL = 1 - F_k + k/L + k/32 (Eq. 7);
  * target set: grow k while the next symbol still cuts the ratio by at
    least a tenth, p(k+1) >= c + 0.1 g(k) with c = 1/L + 1/32 (Eq. 8);
  * encoding: one L-bit bitmap per selected symbol per walk, the other
    positions' node ids kept in order.

Readings (stated once here, and in the design notes):
  * The corpus is the library's fixed-length walk array: a walk from an
    isolated node holds one node and -1 after it.  -1 is a symbol like any
    node id, so padded positions are profiled and may be selected.
  * Ties in frequency rank by symbol value, ascending (-1 first).
  * The selection stops at the first symbol that fails Eq. (8); k is capped at
    K_MAX.  Eq. (8) is evaluated in FP64 as written: p = count / total,
    c = 1/L + 1/32, the test p >= c + 0.1 g, then F += p, k += 1,
    g = (1 - F) + k c.
  * The selected symbols are stored once per corpus, not once per walk (the
    4Nk term of Eq. 6 becomes 4k).

Byte format (little endian), for W walks of L positions and k symbols:
  header   u32 magic 0x43426146 ("FaBC"), u32 k, u32 L, u32 0,
           u64 W, i64 id_base of the walks                         32 B
  symbols  i32[k]                                                  4k B
  bitmaps  u8[k][ceil(L/8)][W]: bit j%8 of byte j/8 of symbol b's
           bitmap of walk w is set iff position j of walk w holds
           symbol b                                                k ceil(L/8) W B
  padding  zero bytes up to a multiple of 8
  offsets  u64[ceil(W/256)]: residuals before walk 256 i           8 ceil(W/256) B
  residual i32[R]: the positions holding no selected symbol; walks in
           blocks of 256, and within a block position by position,
           walk ascending                                            4R B
The paper fixes neither the order of the residual ids nor a layout; this one
lets 256 GPU threads (one per walk) read and write both coalesced.
"""
from __future__ import annotations

import numpy as np

MAGIC = 0x43426146
K_MAX = 16
BLOCK_WALKS = 256
HEADER_BYTES = 32


def ranked_symbols(walks: np.ndarray):
    """All symbols of a walk-major corpus [W][L] with their counts, ranked by
    count descending, then symbol ascending."""
    vals, cnt = np.unique(walks.astype(np.int64), return_counts=True)
    order = np.lexsort((vals, -cnt))
    return vals[order].astype(np.int64), cnt[order].astype(np.int64)


def ratio_g(F: float, k: int, L: int) -> float:
    """Eq. (7): g(k) = 1 - F_k + k/L + k/32."""
    return 1.0 - F + k / L + k / 32.0


def size_model(N: int, L: int, F: float, k: int) -> float:
    """Eq. (6): S(k) = 4NL(1 - F_k) + 4Nk + Nk L/8 bytes."""
    return 4.0 * N * L * (1.0 - F) + 4.0 * N * k + N * k * L / 8.0


def select_k(counts, total: int, L: int, k_max: int = K_MAX) -> int:
    """Eq. (8): the number of leading symbols taken, each while
    p(k+1) >= c + 0.1 g(k)."""
    c = 1.0 / L + 1.0 / 32.0
    F = 0.0
    g = 1.0
    k = 0
    while k < min(k_max, len(counts)):
        p = float(counts[k]) / float(total)
        if not (p >= c + 0.1 * g):
            break
        F = F + p
        k += 1
        g = (1.0 - F) + k * c
    return k


def profile(walks: np.ndarray, k_max: int = K_MAX):
    """(k, the k_max top symbols, their counts, total positions)."""
    sym, cnt = ranked_symbols(walks)
    total = int(walks.size)
    k = select_k(cnt, total, walks.shape[1], k_max)
    return k, sym[:k_max], cnt[:k_max], total


def encode(walks: np.ndarray, symbols, id_base: int = 0) -> bytes:
    """The byte format above for a walk-major corpus [W][L]."""
    walks = np.asarray(walks, dtype=np.int32)
    W, L = walks.shape
    symbols = np.asarray(symbols, dtype=np.int32)
    k = len(symbols)
    B8 = (L + 7) // 8
    parts = [np.array([MAGIC, k, L, 0], dtype="<u4").tobytes(),
             np.array([W], dtype="<u8").tobytes(), np.array([id_base], dtype="<i8").tobytes(),
             symbols.astype("<i4").tobytes()]
    hit = np.zeros(walks.shape, dtype=bool)
    for b in range(k):
        bits = walks == symbols[b]
        hit |= bits
        padded = np.zeros((W, B8 * 8), dtype=bool)
        padded[:, :L] = bits
        by = np.packbits(padded, axis=1, bitorder="little")   # [W][B8]
        parts.append(np.ascontiguousarray(by.T).tobytes())     # [B8][W]
    used = HEADER_BYTES + 4 * k + k * B8 * W
    parts.append(b"\0" * ((-used) % 8))
    per_walk = (~hit).sum(axis=1).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(per_walk)])
    nblk = (W + BLOCK_WALKS - 1) // BLOCK_WALKS
    parts.append(starts[np.arange(nblk) * BLOCK_WALKS].astype("<u8").tobytes())
    for b0 in range(0, W, BLOCK_WALKS):
        blk = walks[b0:b0 + BLOCK_WALKS].T                        # [L][walks of the block]
        parts.append(blk[~hit[b0:b0 + BLOCK_WALKS].T].astype("<i4").tobytes())
    return b"".join(parts)


def decode(buf: bytes):
    """(walk-major corpus [W][L], id_base) from the byte format."""
    hdr = np.frombuffer(buf, dtype="<u4", count=4)
    assert int(hdr[0]) == MAGIC and int(hdr[3]) == 0
    k, L = int(hdr[1]), int(hdr[2])
    W = int(np.frombuffer(buf, dtype="<u8", count=1, offset=16)[0])
    id_base = int(np.frombuffer(buf, dtype="<i8", count=1, offset=24)[0])
    symbols = np.frombuffer(buf, dtype="<i4", count=k, offset=HEADER_BYTES)
    B8 = (L + 7) // 8
    pos = HEADER_BYTES + 4 * k
    out = np.zeros((W, L), dtype=np.int32)
    hit = np.zeros((W, L), dtype=bool)
    for b in range(k):
        by = np.frombuffer(buf, dtype=np.uint8, count=B8 * W, offset=pos).reshape(B8, W)
        pos += B8 * W
        bits = np.unpackbits(np.ascontiguousarray(by.T), axis=1, bitorder="little")[:, :L]
        bits = bits.astype(bool)
        assert not (bits & hit).any(), "two symbols claim one position"
        out[bits] = symbols[b]
        hit |= bits
    pos += (-pos) % 8
    nblk = (W + BLOCK_WALKS - 1) // BLOCK_WALKS
    offsets = np.frombuffer(buf, dtype="<u8", count=nblk, offset=pos)
    pos += 8 * nblk
    R = int((~hit).sum())
    res = np.frombuffer(buf, dtype="<i4", count=R, offset=pos)
    assert pos + 4 * R == len(buf)
    per_walk = (~hit).sum(axis=1)
    starts = np.concatenate([[0], np.cumsum(per_walk)])
    assert np.array_equal(offsets, starts[np.arange(nblk) * BLOCK_WALKS])
    for i, b0 in enumerate(range(0, W, BLOCK_WALKS)):
        seg = res[starts[b0]:starts[min(b0 + BLOCK_WALKS, W)]]
        view = out[b0:b0 + BLOCK_WALKS].T                         # writes through
        view[~hit[b0:b0 + BLOCK_WALKS].T] = seg
    return out, id_base


def packed_bytes(W: int, L: int, k: int, residuals: int) -> int:
    """Size of the byte format."""
    used = HEADER_BYTES + 4 * k + k * ((L + 7) // 8) * W
    used += (-used) % 8
    return used + 8 * ((W + BLOCK_WALKS - 1) // BLOCK_WALKS) + 4 * residuals
