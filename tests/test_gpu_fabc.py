"""GPU parity of the FaBC walk-corpus codec (Section 5.2.2, Eq. 6-8) against
the oracle: the profile, k and the packed bytes must be identical, and
unpacking must give the corpus back bit for bit.

Corpora are the oracle's: its uniform walks (checked equal to the library's
first), or oracle-encoded corpora uploaded with felog_packed_from_host and
unpacked on the device."""
import numpy as np
import pytest

import synth
from oracle import fabc

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def fl():
    from paper_2606_22180_amd import build, felog
    import os
    if not os.path.exists(build.LIB):
        build.build()
    felog.load()
    return felog


@pytest.fixture(scope="module")
def ctx(fl):
    return fl.Context(0)


def _check_codec(fl, W, corpus, id_base):
    """Profile, pack and unpack W (holding `corpus`, walk-major) on the device
    and compare each step with the oracle."""
    k, sym, cnt, total = W.fabc_profile()
    ok, osym, ocnt, ototal = fabc.profile(corpus)
    m = len(osym)
    assert (k, total) == (ok, ototal)
    assert np.array_equal(sym, osym[:m]) and np.array_equal(cnt, ocnt[:m].astype(np.uint64))
    P = W.pack(sym[:k])
    ref = fabc.encode(corpus, osym[:ok], id_base)
    by = P.read()
    assert len(by) == len(ref) == P.info()[0]
    assert by == ref
    R = corpus.size - int(ocnt[:ok].sum())
    assert P.info()[4] == R
    U = P.unpack()
    assert U.info() == W.info()
    assert np.array_equal(U.read(), corpus)
    return k, P


def test_codec_sbm_walks(fl, ctx):
    g = synth.build_graph("sbm1k").train
    from oracle import walks_uniform
    _say("fabc sbm1k walks")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=40, seed=3, id_base=77)
    ow = walks_uniform(g, np.arange(g.n), 10, 40, 3, 77)
    assert np.array_equal(W.read(), ow)
    k, P = _check_codec(fl, W, ow, 77)
    # forced symbol sets, from none to the cap
    for ks in (0, 1, 5, 16):
        sym = np.arange(-1, ks - 1, dtype=np.int32)
        assert W.pack(sym).read() == fabc.encode(ow, sym, 77)


def test_codec_worked_example_corpus(fl, ctx):
    """The example's shape (top two symbols on 60% of the positions) through an
    upload of its raw (k = 0) packing."""
    from test_oracle_fabc import _corpus
    N, L = 512, 80
    w = _corpus(N, L, [0.35, 0.25], seed=1, n_rare=900)
    w = np.where(w >= 1000, w - 1000 + 2, w).astype(np.int32)   # node ids below 1000
    _say("fabc worked-example corpus")
    indptr = np.zeros(1001, np.int64)
    G = fl.Graph.from_csr(ctx, indptr, np.zeros(0, np.int32))   # 1000 isolated nodes
    W = fl.Packed.from_host(G, fabc.encode(w, [], 5)).unpack()
    assert np.array_equal(W.read(), w)
    k, P = _check_codec(fl, W, w, 5)
    assert k == 2
    by, kk, NW, LL, R = P.info()
    assert 4 * R == 1.6 * N * L and kk * (L // 8) * N == 0.25 * N * L


@pytest.mark.parametrize("Wn,L,k,pads", [(1, 1, 0, 0), (1, 9, 1, 0), (255, 7, 2, 100),
                                         (256, 8, 3, 256), (257, 33, 5, 10),
                                         (1000, 80, 16, 400)])
def test_codec_ragged(fl, ctx, Wn, L, k, pads):
    """Ragged walk counts and lengths, padding, k up to the cap."""
    rng = np.random.default_rng(Wn * 7 + L)
    n = 50
    w = rng.integers(0, n, (Wn, L)).astype(np.int32)
    w[:pads, 1:] = -1
    G = fl.Graph.from_csr(ctx, np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
    _say("fabc ragged W=%d L=%d k=%d" % (Wn, L, k))
    W = fl.Packed.from_host(G, fabc.encode(w, [], 1 << 33)).unpack()
    assert np.array_equal(W.read(), w) and W.info()[2] == 1 << 33
    _check_codec(fl, W, w, 1 << 33)
    sym = np.arange(-1, k - 1, dtype=np.int32)
    assert W.pack(sym).read() == fabc.encode(w, sym, 1 << 33)


def test_codec_rmat_corpus(fl, ctx):
    """A larger corpus: R-MAT scale 16, r = 10, L = 80 (655,360 walks)."""
    e = synth.rmat_edges(16, 1 << 20, seed=5)
    g = synth.csr_from_edges(1 << 16, e)
    from oracle import walks_uniform
    _say("fabc rmat16 walks")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=80, seed=9)
    ow = walks_uniform(g, np.arange(g.n), 10, 80, 9)
    assert np.array_equal(W.read(), ow)
    k, P = _check_codec(fl, W, ow, 0)
    _say("rmat16: k=%d, %d of %d bytes" % (k, P.info()[0], 4 * ow.size))


def test_unpacked_corpus_trains_identically(fl, ctx):
    """Training on the unpacked corpus equals training on the original (the
    walk ids travel in the header)."""
    g = synth.build_graph("sbm1k").train
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=2, L=40, seed=4, id_base=123)
    k, sym, _, _ = W.fabc_profile()
    U = W.pack(sym[:max(k, 1)]).unpack()
    prm = fl.train_params(window=5, negatives=5, minibatch_pairs=1024, seed=2)
    out = []
    for C in (W, U):
        M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=1)
        st = M.train_steps(C, prm, 3, 40)
        out.append((M.read(fl.TABLE_IN), M.read(fl.TABLE_OUT), st.loss))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_corrupt_packed_corpus_is_rejected(fl, ctx):
    """Bad headers fail on the host; bitmaps, offsets and residuals that do not
    agree fail in the unpacking launch's own checks (every read there is
    bounds-checked first)."""
    n = 30
    G = fl.Graph.from_csr(ctx, np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
    rng = np.random.default_rng(1)
    w = rng.integers(-1, n, (300, 12)).astype(np.int32)
    good = fabc.encode(w, [3, -1], 0)
    fl.Packed.from_host(G, good).unpack()
    bad_magic = b"XXXX" + good[4:]
    with pytest.raises(fl.FelogError):
        fl.Packed.from_host(G, bad_magic)
    with pytest.raises(fl.FelogError):
        fl.Packed.from_host(G, good[:-2])
    bad_sym = bytearray(good)
    bad_sym[32:36] = np.int32(n).tobytes()          # symbol outside [-1, n)
    with pytest.raises(fl.FelogError):
        fl.Packed.from_host(G, bytes(bad_sym))
    # the second offsets entry moved: its blocks disagree with the bitmaps
    B8 = 2
    off_at = 32 + 8 + 2 * B8 * 300
    off_at += (-off_at) % 8
    tampered = bytearray(good)
    v = int(np.frombuffer(good, "<u8", count=1, offset=off_at + 8)[0])
    tampered[off_at + 8:off_at + 16] = np.uint64(v + 5).tobytes()
    with pytest.raises(fl.FelogError):
        fl.Packed.from_host(G, bytes(tampered)).unpack()
    # a residual outside [-1, n)
    tampered = bytearray(good)
    tampered[-4:] = np.int32(n + 7).tobytes()
    with pytest.raises(fl.FelogError):
        fl.Packed.from_host(G, bytes(tampered)).unpack()
    # two symbols claiming one position: set symbol 0's bit where symbol 1's is
    tampered = bytearray(good)
    bm0 = 32 + 8
    bm1 = bm0 + B8 * 300
    for i in range(B8 * 300):
        tampered[bm0 + i] |= tampered[bm1 + i]
    with pytest.raises(fl.FelogError):
        fl.Packed.from_host(G, bytes(tampered)).unpack()
    # the device is still usable afterwards
    assert np.array_equal(fl.Packed.from_host(G, good).unpack().read(), w)
