"""Pins of the FaBC oracle (Section 5.2.2, Eq. 6-8) against closed forms, the
paper's worked example and brute force."""
import numpy as np
import pytest

from oracle import fabc


def _corpus(W, L, freqs, seed, pad_walks=0, n_rare=100000):
    """A walk-major corpus whose symbols 0..len(freqs)-1 fill exactly the given
    fractions of the positions (each rounded to whole positions); the rest are
    distinct-enough rare ids 1000..1000+n_rare, and pad_walks walks hold one
    node and -1 after it."""
    rng = np.random.default_rng(seed)
    total = W * L
    cells = rng.permutation(total)
    out = np.empty(total, np.int64)
    at = 0
    for s, f in enumerate(freqs):
        m = int(round(f * total))
        out[cells[at:at + m]] = s
        at += m
    out[cells[at:]] = 1000 + rng.integers(0, n_rare, total - at)
    out = out.reshape(W, L).astype(np.int32)
    out[:pad_walks, 1:] = -1
    return out


def test_worked_example_sizes():
    """Top-2 symbols covering 60% of the positions: bitmaps of 0.25 NL bytes and
    residual ids of 1.6 NL bytes, as in the paper's example (k N L / 8 + 4 N L_c
    with L_c = 0.4 L)."""
    N, L = 512, 80
    w = _corpus(N, L, [0.35, 0.25], seed=1)
    k, sym, cnt, total = fabc.profile(w)
    assert k == 2 and list(sym[:2]) == [0, 1]
    assert cnt[0] + cnt[1] == int(0.6 * N * L)
    buf = fabc.encode(w, sym[:k])
    B8 = L // 8
    bitmap_bytes = k * B8 * N
    R = N * L - int(cnt[0] + cnt[1])
    assert bitmap_bytes == 0.25 * N * L
    assert 4 * R == 1.6 * N * L
    assert len(buf) == fabc.packed_bytes(N, L, k, R)
    dec, _ = fabc.decode(buf)
    assert np.array_equal(dec, w)


def test_size_model_eq6_eq7():
    """The format's bytes equal Eq. (6) with the symbols stored once instead of
    once per walk, plus the header, the alignment and the block offsets; Eq. (7)
    is Eq. (6) over the 4NL-byte baseline."""
    for (N, L, freqs, seed) in [(300, 40, [0.3, 0.2, 0.1], 2), (257, 80, [0.5], 3),
                                (64, 16, [0.25, 0.25], 4)]:
        w = _corpus(N, L, freqs, seed)
        sym, cnt = fabc.ranked_symbols(w)
        for k in range(0, 4):
            F = float(cnt[:k].sum()) / (N * L)
            buf = fabc.encode(w, sym[:k])
            R = N * L - int(cnt[:k].sum())
            model = fabc.size_model(N, L, F, k)
            used = fabc.HEADER_BYTES + 4 * k + k * (L // 8) * N
            extra = used % 8 and 8 - used % 8
            mine = model - 4 * N * k + 4 * k + fabc.HEADER_BYTES + extra + \
                8 * ((N + 255) // 256)
            assert len(buf) == pytest.approx(mine, abs=1e-6)
            assert model / (4 * N * L) == pytest.approx(fabc.ratio_g(F, k, L), rel=1e-12)
            assert np.array_equal(fabc.decode(buf)[0], w)


def test_stop_rule_example_and_closed_form():
    """The example's shape: the top two symbols hold over half of the corpus and
    the third adds little, so Eq. (8) keeps exactly two.  By hand, at L = 80:
    c = 0.04375; p1 = .35 >= c + .1 = .14375; g(1) = .69375; p2 = .25 >=
    c + .069375; g(2) = .4875; p3 = .08 < c + .04875 = .0925."""
    L, total = 80, 100000
    counts = [35000, 25000, 8000, 7000, 1000]
    assert fabc.select_k(counts, total, L) == 2
    # p3 just above the threshold is taken, p4 then fails
    assert fabc.select_k([35000, 25000, 9300, 100], total, L) == 3
    # between c + 0.1 (1 - F_2) = .08375 and c + 0.1 g(2) = .0925: the k c term
    # of g keeps the third symbol out
    assert fabc.select_k([35000, 25000, 9000], total, L) == 2
    # equality takes the symbol (L = 32: c = 1/16, and 1625 / 10000 equals
    # 1/16 + 0.1 in FP64)
    assert fabc.select_k([1625, 10], 10000, 32) == 1
    # nothing reaches c + 0.1 = 0.14375 at k = 0
    assert fabc.select_k([14000, 13000], total, L) == 0
    # the cap
    assert fabc.select_k([1] * 40, 1, 10, k_max=16) == 16


def test_stop_rule_brute_force():
    """Every expansion up to k satisfies Eq. (8) with g from Eq. (7), and the
    next one fails (random profiles, away from exact ties)."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        L = int(rng.integers(4, 120))
        m = int(rng.integers(1, 30))
        counts = np.sort(rng.integers(1, 10 ** 6, m))[::-1]
        total = int(counts.sum() + rng.integers(0, 10 ** 7))
        k = fabc.select_k(counts, total, L, k_max=64)
        p = counts / total
        for i in range(k + 1):
            if i >= m:
                break
            gi = fabc.ratio_g(p[:i].sum(), i, L)
            ok = p[i] >= (1 / L + 1 / 32) + 0.1 * gi
            if abs(p[i] - ((1 / L + 1 / 32) + 0.1 * gi)) < 1e-12:
                continue
            assert ok == (i < k), (i, k)


def test_ranking_ties_and_pads():
    """Ties rank by symbol, -1 first; padded positions are symbols."""
    w = np.array([[5, 3, -1, -1], [3, 5, -1, -1], [7, 7, 9, 9]], np.int32)
    sym, cnt = fabc.ranked_symbols(w)
    assert list(sym) == [-1, 3, 5, 7, 9] and list(cnt) == [4, 2, 2, 2, 2]
    # a corpus of mostly one-node walks selects the pad symbol
    w = _corpus(400, 80, [0.02], seed=6, pad_walks=300)
    k, sym, cnt, total = fabc.profile(w)
    assert k >= 1 and sym[0] == -1
    assert cnt[0] == 300 * 79
    buf = fabc.encode(w, sym[:k], id_base=1 << 40)
    dec, base = fabc.decode(buf)
    assert np.array_equal(dec, w) and base == 1 << 40


@pytest.mark.parametrize("W,L,k", [(1, 1, 0), (1, 9, 1), (255, 7, 2), (256, 8, 3),
                                   (513, 33, 5), (1000, 80, 16)])
def test_round_trip_edges(W, L, k):
    """Decode inverts encode for ragged walk counts and lengths, k from 0 to
    the cap, and symbols that never occur."""
    rng = np.random.default_rng(W * 131 + L)
    w = rng.integers(-1, 20, (W, L)).astype(np.int32)
    sym = np.arange(-1, -1 + k, dtype=np.int32)[::-1] if k else np.zeros(0, np.int32)
    buf = fabc.encode(w, sym, id_base=W)
    dec, base = fabc.decode(buf)
    assert np.array_equal(dec, w) and base == W
    R = int(np.isin(w, sym, invert=True).sum())
    assert len(buf) == fabc.packed_bytes(W, L, k, R)


def test_bit_layout():
    """Bit j%8 of byte j/8, bytes [symbol][byte][walk]."""
    w = np.array([[4, 0, 4, 4, 0, 0, 0, 0, 0, 4], [0, 4, 0, 0, 0, 0, 0, 0, 4, 0]], np.int32)
    buf = fabc.encode(w, [4])
    by = np.frombuffer(buf, np.uint8, count=4, offset=fabc.HEADER_BYTES + 4)
    # walk 0: positions 0,2,3 -> 0b1101 = 13 in byte 0, position 9 -> bit 1 of byte 1
    # walk 1: position 1 -> 2 in byte 0, position 8 -> bit 0 of byte 1
    assert list(by) == [13, 2, 2, 1]


def test_residual_order():
    """Residuals run position by position within a block of 256 walks, walk
    ascending, and block after block."""
    w = np.array([[10, 4, 11], [4, 12, 13]], np.int32)
    buf = fabc.encode(w, [4])
    assert list(np.frombuffer(buf, "<i4", count=4, offset=len(buf) - 16)) == [10, 12, 11, 13]
    w = np.arange(300 * 2, dtype=np.int32).reshape(300, 2)
    buf = fabc.encode(w, [])
    res = np.frombuffer(buf, "<i4", count=600, offset=len(buf) - 2400)
    first = w[:256].T.reshape(-1)
    second = w[256:].T.reshape(-1)
    assert np.array_equal(res, np.concatenate([first, second]))
    offs = np.frombuffer(buf, "<u8", count=2, offset=len(buf) - 2400 - 16)
    assert list(offs) == [0, 512]
