"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Every oracle input is the oracle's own (its walks, noise table and tables;
teacher forcing writes the oracle's tables into the library, never the other
way round).  Integer work (walks, noise tables, active lists) must be
bit-exact.  SGNS deltas are computed in FP64 over the FP32 tables on both
sides (they differ in summation order and the final rounding); per updated row
  ||d_gpu - d_orc|| <= 1e-5 ||d_orc|| + 1e-12,
and the tests print the rows' |term| mass as the scale of the rounding the
bar leaves room for.  Psi (FP64 on both sides) within 1e-12 and identical
decisions; Algorithm 1's next active sets equal except for nodes whose
oracle score lies within 1e-3 of mu (counted and printed).
"""
import numpy as np
import pytest

import synth
from conftest import link_auc_of

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


@pytest.fixture(scope="module")
def sbm():
    return synth.build_graph("sbm1k")


def _rmat(scale, edges, seed, weighted=False):
    e = synth.rmat_edges(scale, edges, seed=seed)
    w = synth.edge_weights(e.shape[0], seed + 1) if weighted else None
    return synth.csr_from_edges(1 << scale, e, w)


# ------------------------------------------------------------------ walks
@pytest.mark.parametrize("kind", ["path", "star", "house", "k8"])
def test_uniform_walks_tiny(fl, ctx, orc, kind):
    g = synth.tiny_graph(kind)
    _say("uniform walks tiny", kind)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=33, L=17, seed=7, id_base=3)
    assert np.array_equal(W.read(), orc.walks_uniform(g, np.arange(g.n), 33, 17, 7, 3))


def test_uniform_walks_sbm_and_starts(fl, ctx, orc, sbm):
    g = sbm.train
    _say("uniform walks sbm1k")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=40, seed=11)
    assert np.array_equal(W.read(), orc.walks_uniform(g, np.arange(g.n), 10, 40, 11))
    starts = np.arange(3, g.n, 7, dtype=np.int32)
    A = fl.Active.from_host(G, starts)
    W2 = fl.Walks.generate(G, r=3, L=25, seed=11, id_base=10000, starts=A)
    assert np.array_equal(W2.read(), orc.walks_uniform(g, starts, 3, 25, 11, 10000))


def test_uniform_walks_rmat(fl, ctx, orc):
    g = _rmat(16, 1 << 20, seed=5)
    _say("uniform walks rmat16 n=%d nnz=%d" % (g.n, g.nnz))
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=2, L=80, seed=3, id_base=1 << 33)   # ids above 2^32
    gw = W.read()
    ow = orc.walks_uniform(g, np.arange(g.n), 2, 80, 3, 1 << 33)
    assert np.array_equal(gw, ow)


@pytest.mark.parametrize("p,q", [(0.5, 2.0), (2.0, 0.5), (1.0, 1.0)])
def test_node2vec_walks(fl, ctx, orc, p, q):
    g = _rmat(12, 40000, seed=9, weighted=True)
    _say("node2vec walks rmat12 weighted p=%g q=%g" % (p, q))
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices, g.weights)
    W = fl.Walks.generate(G, r=2, L=30, seed=13, id_base=77, kind=fl.WALK_NODE2VEC, p=p, q=q)
    ow, capped = orc.walks_node2vec(g, np.arange(g.n), 2, 30, p, q, 13, 77)
    assert np.array_equal(W.read(), ow)
    assert W.capped() == capped == 0


@pytest.mark.parametrize("p,q", [(0.5, 2.0), (2.0, 0.5)])
def test_node2vec_dense_weighted(fl, ctx, orc, p, q):
    """A dense weighted graph (96 nodes, each pair an edge with probability
    0.6, plus a 400-node sparse tail hanging off it): proposals are often
    adjacent to the previous node and rows of equal length are common, so the
    adjacency search of the shorter row and the paired attempts are
    exercised; bit-exact against the oracle."""
    rng = np.random.default_rng(21)
    nd, nt = 96, 400
    iu, ju = np.triu_indices(nd, 1)
    keep = rng.random(iu.shape[0]) < 0.6
    dense = np.stack([iu[keep], ju[keep]], 1)
    tail_u = nd + np.arange(nt)
    # each tail node hangs off a dense node (every third) or the previous tail node
    tail_v = np.where(np.arange(nt) % 3 == 0, rng.integers(0, nd, nt),
                      nd + np.maximum(np.arange(nt) - 1, 0))
    tail = np.stack([np.minimum(tail_u, tail_v), np.maximum(tail_u, tail_v)], 1)
    tail = tail[tail[:, 0] != tail[:, 1]]
    e = np.unique(np.concatenate([dense, tail]), axis=0)
    g = synth.csr_from_edges(nd + nt, e, synth.edge_weights(e.shape[0], 5))
    _say("node2vec walks dense weighted n=%d nnz=%d p=%g q=%g" % (g.n, g.nnz, p, q))
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices, g.weights)
    W = fl.Walks.generate(G, r=4, L=40, seed=29, id_base=5, kind=fl.WALK_NODE2VEC, p=p, q=q)
    ow, capped = orc.walks_node2vec(g, np.arange(g.n), 4, 40, p, q, 29, 5)
    assert np.array_equal(W.read(), ow)
    assert W.capped() == capped == 0


def test_node2vec_unweighted(fl, ctx, orc, sbm):
    g = sbm.train
    _say("node2vec walks sbm1k unweighted")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=2, L=40, seed=1, kind=fl.WALK_NODE2VEC, p=0.5, q=2.0)
    ow, _ = orc.walks_node2vec(g, np.arange(g.n), 2, 40, 0.5, 2.0, 1)
    assert np.array_equal(W.read(), ow)


# ------------------------------------------------------- tables and noise
def test_init_and_noise_tables(fl, ctx, orc, sbm):
    g = sbm.train
    _say("init + degree noise table")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=42)
    tin, tout = orc.init_tables(g.n, 64, 42)
    assert np.array_equal(M.read(fl.TABLE_IN), tin)
    assert np.array_equal(M.read(fl.TABLE_OUT), tout)
    assert np.array_equal(M.read_cdf(), orc.neg_cdf(g.degrees().astype(np.uint64)))


def test_unigram_noise_table(fl, ctx, orc):
    g = _rmat(15, 1 << 19, seed=2)
    _say("unigram noise table rmat15")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=4, L=30, seed=8)
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_UNIGRAM, seed=1)
    M.set_unigram(W)
    ow = orc.walks_uniform(g, np.arange(g.n), 4, 30, 8)
    assert np.array_equal(W.read(), ow)
    counts = orc.corpus_counts(ow, g.n)
    assert np.array_equal(M.read_cdf(), orc.neg_cdf(counts))


# ------------------------------------------------------------------ SGNS
def _dense(rows, vals, n, d):
    out = np.zeros((n, d))
    out[rows] = vals
    return out


def _mass(tin, tout, ctx_, ctr, neg, lr, orc):
    """Per-row sum of |term| vectors of a minibatch (the FP32 error scale)."""
    n, d = tin.shape
    ain = np.zeros((n, d))
    aout = np.zeros((n, d))
    a = tin.astype(np.float64)
    b = tout.astype(np.float64)
    for p in range(len(ctx_)):
        c = ctx_[p]
        ts = [ctr[p]] + [t for t in neg[p] if t != ctr[p]]
        for k, t in enumerate(ts):
            s = a[c] @ b[t]
            g = lr * (1 - 1 / (1 + np.exp(-s))) if k == 0 else lr / (1 + np.exp(-s))
            ain[c] += np.abs(g * b[t])
            aout[t] += np.abs(g * a[c])
    return ain, aout


def _check_delta(gpu, ref, mass, what):
    """The per-step bar: every row's delta within 1e-5 of the oracle's in
    norm, plus 1e-12 absolute.  (mass, the row's sum of |term| vectors, is
    printed as the scale of the FP rounding the bar leaves room for.)"""
    num = np.linalg.norm(gpu - ref, axis=1)
    nref = np.linalg.norm(ref, axis=1)
    tol = 1e-5 * nref + 1e-12
    bad = np.nonzero(num > tol)[0]
    rel = num / np.maximum(nref, 1e-30)
    canc = np.linalg.norm(mass, axis=1) / np.maximum(nref, 1e-30)
    _say("%s: rows=%d max rel=%.3e misses of 1e-5|d|+1e-12: %d (max |mass|/|d| %.1f)"
         % (what, int((np.abs(ref).sum(1) > 0).sum()), rel.max(), len(bad),
            canc[nref > 0].max() if (nref > 0).any() else 0.0))
    assert len(bad) == 0, (what, bad[:5], num[bad[:5]], tol[bad[:5]])


def _sgns_step_parity(fl, ctx, orc, g, *, dim, K, P, window, L, neg, mbs, seed=3, pre_mb=0):
    """Teacher-forced per-step parity: the oracle runs from its own walks, noise
    table and tables (trained by the oracle for pre_mb minibatches), and the
    library gets the oracle's tables written in before every checked step."""
    r = 10 if g.n < 5000 else 1
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=r, L=L, seed=11)
    M = fl.Model.create(G, dim=dim, neg_dist=neg, seed=5)
    walks = orc.walks_uniform(g, np.arange(g.n), r, L, 11)
    assert np.array_equal(W.read(), walks)
    if neg == fl.NEG_UNIGRAM:
        M.set_unigram(W)
        cdf = orc.neg_cdf(orc.corpus_counts(walks, g.n))
    else:
        cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    assert np.array_equal(M.read_cdf(), cdf)
    prm = fl.train_params(window=window, negatives=K, minibatch_pairs=P, seed=seed)
    B, _ = orc.count_minibatches(walks, window, P)
    tin, tout = orc.init_tables(g.n, dim, 5)
    if pre_mb:                                    # move away from the initial state
        orc.train_epoch(tin, tout, walks, window=window, K=K, lr0=prm.lr_start,
                        lr_end=prm.lr_end, P=P, seed=seed, cdf=cdf, mb_end=pre_mb)
    for b in mbs:
        b = b % B
        M.write(fl.TABLE_IN, tin)
        M.write(fl.TABLE_OUT, tout)
        ri, di, ro, do, loss = M.train_delta(W, prm, b)
        mb = orc.minibatch_pairs(walks, window, P, b)
        ng = orc.draw_negatives(mb, 0, K, seed, cdf)
        lr = orc.lr_at(b, B, prm.lr_start, prm.lr_end)
        ref = orc.sgns_step(tin.copy(), tout.copy(), mb.ctx, mb.ctr, ng, lr, apply=False)
        assert sorted(ri.tolist()) == sorted(ref.rows_in.tolist())
        assert sorted(ro.tolist()) == sorted(ref.rows_out.tolist())
        ain, aout = _mass(tin, tout, mb.ctx, mb.ctr, ng, lr, orc)
        _check_delta(_dense(ri, di, g.n, dim), _dense(ref.rows_in, ref.d_in, g.n, dim), ain,
                     "mb %d in" % b)
        _check_delta(_dense(ro, do, g.n, dim), _dense(ref.rows_out, ref.d_out, g.n, dim), aout,
                     "mb %d out" % b)
        assert abs(loss - ref.loss) <= 1e-5 * abs(ref.loss)
        # the oracle applies its own step, so the next check starts elsewhere
        orc.sgns_step(tin, tout, mb.ctx, mb.ctr, ng, lr, apply=True)
    return M


def test_sgns_step_parity_sbm(fl, ctx, orc, sbm):
    _say("sgns per-step parity sbm1k d=64 K=5 P=1024")
    _sgns_step_parity(fl, ctx, orc, sbm.train, dim=64, K=5, P=1024, window=5, L=40,
                      neg=fl.NEG_DEGREE, mbs=[0, 1, 1800, 3613], pre_mb=0)


def test_sgns_step_parity_trained_state(fl, ctx, orc, sbm):
    _say("sgns per-step parity sbm1k after 2000 minibatches")
    _sgns_step_parity(fl, ctx, orc, sbm.train, dim=64, K=5, P=1024, window=5, L=40,
                      neg=fl.NEG_DEGREE, mbs=[2000, 3000], pre_mb=2000)


def test_sgns_step_parity_rmat_d128(fl, ctx, orc):
    g = _rmat(14, 1 << 18, seed=4)
    _say("sgns per-step parity rmat14 d=128 K=5 P=8192 w=10 unigram")
    _sgns_step_parity(fl, ctx, orc, g, dim=128, K=5, P=8192, window=10, L=80,
                      neg=fl.NEG_UNIGRAM, mbs=[0, 7, 123], pre_mb=64)


def test_sgns_step_parity_k_and_dims(fl, ctx, orc, sbm):
    for dim, K in ((256, 3), (128, 20), (64, 1)):
        _say("sgns per-step parity sbm1k d=%d K=%d" % (dim, K))
        _sgns_step_parity(fl, ctx, orc, sbm.train, dim=dim, K=K, P=777, window=3, L=12,
                          neg=fl.NEG_DEGREE, mbs=[0, 5], pre_mb=20)


def test_sgns_epoch_is_deterministic(fl, ctx, sbm):
    """Row sums are exact, so two epochs from the same state give identical tables."""
    g = sbm.train
    _say("sgns determinism sbm1k, P=1024 and P=16384")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=40, seed=5)
    for P in (1024, 16384):
        out = []
        for _ in range(2):
            M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=1)
            st = M.train_epoch(W, fl.train_params(window=5, negatives=5, minibatch_pairs=P, seed=2))
            out.append((M.read(fl.TABLE_IN), M.read(fl.TABLE_OUT), st.loss))
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
        assert out[0][2] == out[1][2]


def test_minibatch_size_switch_keeps_counters_clean(fl, ctx, sbm):
    """Large minibatches zero the row counters before their ids and leave them
    dirty; small ones reset rows as they go and need clean counters at the
    start.  Training a model at P = 4096 and then at P = 1024 (and back) gives
    the same tables as a fresh model given the same tables at each switch."""
    g = sbm.train
    _say("counter state across minibatch sizes")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=40, seed=5)
    big = fl.train_params(window=5, negatives=5, minibatch_pairs=4096, seed=2)
    small = fl.train_params(window=5, negatives=5, minibatch_pairs=1024, seed=2)
    M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=1)
    for prm, first, n in ((big, 10, 6), (small, 50, 9), (big, 30, 5), (small, 200, 3)):
        tin, tout = M.read(fl.TABLE_IN), M.read(fl.TABLE_OUT)
        F = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=1)
        F.write(fl.TABLE_IN, tin)
        F.write(fl.TABLE_OUT, tout)
        a = M.train_steps(W, prm, first, n)
        b = F.train_steps(W, prm, first, n)
        assert a.loss == b.loss and a.rows_out == b.rows_out
        assert np.array_equal(M.read(fl.TABLE_IN), F.read(fl.TABLE_IN))
        assert np.array_equal(M.read(fl.TABLE_OUT), F.read(fl.TABLE_OUT))
        F.close()


def test_sgns_epoch_auc_matches_oracle(fl, ctx, orc, sbm):
    """Free-running epoch on sbm1k: AUC within 0.005 of the oracle's."""
    g = sbm.train
    _say("sgns free-running epoch sbm1k")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=40, seed=11)
    M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=0)
    prm = fl.train_params(window=5, negatives=5, minibatch_pairs=1024, seed=3)
    st = M.train_epoch(W, prm)
    tin, tout = orc.init_tables(g.n, 64, 0)
    ow = orc.walks_uniform(g, np.arange(g.n), 10, 40, 11)
    assert np.array_equal(W.read(), ow)
    ref = orc.train_epoch(tin, tout, ow, window=5, K=5, lr0=prm.lr_start,
                          lr_end=prm.lr_end, P=1024, seed=3,
                          cdf=orc.neg_cdf(g.degrees().astype(np.uint64)))
    a_gpu = link_auc_of(M.read(fl.TABLE_IN), sbm)
    a_orc = orc.link_auc(tin, sbm)
    _say("AUC gpu=%.5f oracle=%.5f loss gpu=%.6e oracle=%.6e" % (a_gpu, a_orc, st.loss,
                                                                 ref.loss))
    assert st.pairs == ref.pairs == 3_700_000
    assert abs(a_gpu - a_orc) <= 0.005
    assert abs(st.loss - ref.loss) <= 1e-4 * ref.loss
    emb = M.read(fl.TABLE_IN)
    assert np.abs(emb - tin).max() <= 1e-3 * np.abs(tin).max()


# -------------------------------------------------------------- feedback
def test_psi_and_active_set(fl, ctx, orc, sbm):
    g = sbm.train
    _say("psi teacher-forced sbm1k")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=2)
    rng = np.random.default_rng(0)
    tin = rng.normal(0, 1, (g.n, 128)).astype(np.float32)
    tin[::97] += tin[1::97][: tin[::97].shape[0]]          # correlated neighbours
    tin[5] = 0.0                                            # zero vector
    M.write(fl.TABLE_IN, tin)
    for rnd, k_s, mu in ((0, 10, 0.02), (3, 4, 0.0), (1, 64, -0.01)):
        act, psi = M.feedback(mu=mu, k_s=k_s, seed=9, round=rnd, want_psi=True)
        opsi = orc.psi(tin, g, np.arange(g.n), k_s, 9, rnd)
        fin = np.isfinite(opsi)
        assert np.array_equal(np.isfinite(psi), fin)
        assert np.abs(psi[fin] - opsi[fin]).max() <= 1e-12
        assert np.array_equal(act.read(), orc.next_active(np.arange(g.n, dtype=np.int32),
                                                          opsi, mu))
    # monotone mode scores only the given list
    sub = fl.Active.from_host(G, np.arange(0, g.n, 3, dtype=np.int32))
    act, psi = M.feedback(mu=0.01, k_s=10, seed=9, round=1, active=sub, want_psi=True)
    nodes = np.arange(0, g.n, 3, dtype=np.int32)
    opsi = orc.psi(tin, g, nodes, 10, 9, 1)
    assert np.array_equal(act.read(), orc.next_active(nodes, opsi, 0.01))


def _algorithm1_guard_band(fl, ctx, orc, split, *, mode, mu, rounds, d=64, r=10, L=40,
                           window=5, K=5, P=1024, k_s=10, seeds=(1, 2, 3, 4)):
    """Algorithm 1 round by round on both sides (Eq. (4)-(5)), free-running
    tables.  Each round starts both sides from the same active list (the
    oracle's, handed to the library through felog_active_from_host), so walks
    and pair counts must be equal; the next active sets may differ only by
    nodes whose oracle score lies within 1e-3 of mu.  Returns the per-round
    flip counts."""
    g = split.train
    seed_walk, seed_model, seed_train, seed_psi = seeds
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    M = fl.Model.create(G, dim=d, neg_dist=fl.NEG_DEGREE, seed=seed_model)
    prm = fl.train_params(window=window, negatives=K, minibatch_pairs=P, seed=seed_train)
    tin, tout = orc.init_tables(g.n, d, seed_model)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    gmode = fl.FEEDBACK_MONOTONE if mode == "monotone" else fl.FEEDBACK_RECOMPUTE_ALL
    active = np.arange(g.n, dtype=np.int32)
    id_base = 0
    flips = []
    for rnd in range(rounds):
        if active.shape[0] == 0:
            break
        starts = None if rnd == 0 else fl.Active.from_host(G, active)
        W = fl.Walks.generate(G, r=r, L=L, seed=seed_walk, id_base=id_base, starts=starts)
        ow = orc.walks_uniform(g, active, r, L, seed_walk, id_base)
        assert np.array_equal(W.read(), ow), ("walks", rnd)
        st = M.train_epoch(W, prm)
        tr = orc.train_epoch(tin, tout, ow, window=window, K=K, lr0=prm.lr_start,
                             lr_end=prm.lr_end, P=P, seed=seed_train, cdf=cdf, id_base=id_base)
        assert st.pairs == tr.pairs, ("pairs", rnd)
        assert abs(st.loss - tr.loss) <= 1e-5 * abs(tr.loss), ("loss", rnd, st.loss, tr.loss)
        id_base += ow.shape[0]
        cand = active if mode == "monotone" else np.arange(g.n, dtype=np.int32)
        nxt, _ = M.feedback(mu=mu, k_s=k_s, seed=seed_psi, round=rnd, mode=gmode,
                            active=starts, want_psi=True)
        ps = orc.psi(tin, g, cand, k_s, seed_psi, rnd)
        o_next = orc.next_active(cand, ps, mu)
        g_next = nxt.read()
        diff = np.setxor1d(g_next, o_next)
        band = np.abs(ps[np.searchsorted(cand, diff)] - mu)
        _say("round %d (%s): active %d, next gpu %d oracle %d, flips %d (max |psi-mu| %.2e)"
             % (rnd, mode, active.shape[0], g_next.shape[0], o_next.shape[0], diff.shape[0],
                band.max() if diff.shape[0] else 0.0))
        assert np.all(band <= 1e-3), ("flip outside the guard band", rnd, diff[band > 1e-3])
        flips.append(int(diff.shape[0]))
        active = o_next
    a_gpu = link_auc_of(M.read(fl.TABLE_IN), split)
    a_orc = orc.link_auc(tin, split)
    _say("AUC gpu=%.5f oracle=%.5f" % (a_gpu, a_orc))
    assert abs(a_gpu - a_orc) <= 0.005
    return flips


def test_algorithm1_guard_band_monotone(fl, ctx, orc, sbm):
    """Algorithm 1 on sbm1k, MONOTONE (Eq. (5)), mu = 0.7, 3 rounds."""
    _say("algorithm 1 guard band sbm1k monotone mu=0.7")
    _algorithm1_guard_band(fl, ctx, orc, sbm, mode="monotone", mu=0.7, rounds=3)


def test_algorithm1_guard_band_recompute_all(fl, ctx, orc, sbm):
    """The same with every node rescored each round (RECOMPUTE_ALL, the
    reactivation reading of Section 5.1), mu = 0.7, 3 rounds."""
    _say("algorithm 1 guard band sbm1k recompute-all mu=0.7")
    _algorithm1_guard_band(fl, ctx, orc, sbm, mode="recompute_all", mu=0.7, rounds=3)


def test_run_matches_separate_calls(fl, ctx, orc, sbm):
    """felog_run (walks beside training on their own stream) against the
    oracle's Algorithm 1 on sbm1k: the same active sets round by round up to
    guard-band flips, the same pairs, and AUC within 0.005."""
    g = sbm.train
    _say("felog_run sbm1k 3 rounds mu=0.7")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=2)
    rp = fl.felog_run_params()
    rp.walk = fl.felog_walk_params(fl.WALK_UNIFORM, 10, 40, 1.0, 1.0, 1, 0)
    rp.train = fl.train_params(window=5, negatives=5, minibatch_pairs=1024, seed=3)
    rp.feedback = fl.felog_feedback_params(0.7, 10, fl.FEEDBACK_MONOTONE, 4, 0)
    rp.max_rounds = 3
    st = M.run(rp)
    tin, tout, ostats = orc.run(g, d=64, r=10, L=40, window=5, K=5, lr0=rp.train.lr_start,
                                lr_end=rp.train.lr_end, P=1024, mu=0.7, k_s=10, r_max=3,
                                seed_walk=1, seed_model=2, seed_train=3, seed_psi=4,
                                neg="degree")
    gpu_act = list(st.active[:st.rounds])
    orc_act = [s.active for s in ostats]
    _say("rounds gpu=%d oracle=%d active gpu=%s oracle=%s" % (st.rounds, len(ostats), gpu_act,
                                                               orc_act))
    assert st.rounds == len(ostats) == 3
    assert gpu_act[0] == orc_act[0] == 1000
    for r in range(st.rounds):
        # a flip within the guard band (checked node by node in the lockstep
        # tests) carries into the next round here
        assert abs(gpu_act[r] - orc_act[r]) <= 2
        if gpu_act[r] == orc_act[r]:
            assert st.train[r].pairs == ostats[r].pairs
            assert abs(st.train[r].loss - ostats[r].loss) <= 1e-5 * ostats[r].loss
    a_gpu = link_auc_of(M.read(fl.TABLE_IN), sbm)
    a_orc = orc.link_auc(tin, sbm)
    _say("AUC gpu=%.5f oracle=%.5f" % (a_gpu, a_orc))
    assert abs(a_gpu - a_orc) <= 0.005


# ---------------------------------------------------------- error paths
def test_invalid_graphs_rejected(fl, ctx):
    _say("invalid CSR")
    bad = {
        "asymmetric": ([0, 1, 1], [1]),
        "self loop": ([0, 1, 2], [0, 0]),
        "unsorted": ([0, 2, 3, 4], [2, 1, 0, 0]),
        "out of range": ([0, 1, 2], [5, 0]),
    }
    for what, (ip, ix) in bad.items():
        with pytest.raises(fl.FelogError) as e:
            fl.Graph.from_csr(ctx, np.array(ip), np.array(ix))
        assert e.value.status == fl.FELOG_EINVAL, what
    g = synth.tiny_graph("path")
    w = np.ones(g.nnz, np.float32)
    w[0] = 2.0                                    # reverse edge has weight 1
    with pytest.raises(fl.FelogError):
        fl.Graph.from_csr(ctx, g.indptr, g.indices, w)


def test_budget_and_bad_params(fl):
    _say("budget / params")
    small = fl.Context(0, hbm_budget=1 << 14)
    g = synth.tiny_graph("k8")
    G = fl.Graph.from_csr(small, g.indptr, g.indices)
    with pytest.raises(fl.FelogError) as e:
        fl.Model.create(G, dim=256)
    assert e.value.status in (fl.FELOG_ENOMEM, fl.FELOG_EINVAL)
    with pytest.raises(fl.FelogError) as e:
        fl.Walks.generate(G, r=0, L=5, seed=1)
    assert e.value.status == fl.FELOG_EINVAL


def test_context_closed_before_its_objects(fl):
    """The C library needs a context's objects destroyed before it; the
    binding defers a context's destruction until they are gone, whatever
    order the garbage collector finalises a reference cycle in."""
    import gc
    _say("context closed before its objects")
    g = synth.tiny_graph("k8")
    c = fl.Context(0)
    G = fl.Graph.from_csr(c, g.indptr, g.indices)
    M = fl.Model.create(G, dim=64)
    W = fl.Walks.generate(G, r=1, L=5, seed=1)
    c.close()                                    # objects alive: deferred
    assert c.handle is not None
    cycle = [c, G, M, W]
    cycle.append(cycle)
    del G, M, W, cycle
    gc.collect()
    assert c.handle is None                      # destroyed with the last object
    # no stale HIP error reaches the next calls
    c2 = fl.Context(0)
    G2 = fl.Graph.from_csr(c2, g.indptr, g.indices)
    assert np.array_equal(fl.Walks.generate(G2, r=1, L=5, seed=1).read()[:, 0], np.arange(g.n))
