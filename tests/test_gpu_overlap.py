"""Walks beside training (the one-GPU form of Section 5.3's overlap of sampling
and training): felog_run writes a round's walks chunk by chunk on a third
stream while the SGNS of earlier chunks runs.  The walks read no embeddings,
so the run must equal, bit for bit, the same rounds driven through the
separate calls (walk the whole corpus, then train, then feedback).  Runs cover
ragged chunks, chunks without a single walk that yields pairs, both stream
modes of the FP32 path, node2vec with unigram noise (round 1 walks first, the
later rounds overlap) and the BF16 form (one round; its per-row sums in
touch order make it bit-reproducible too)."""
import numpy as np
import pytest

import synth

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


def _rmat12(weighted):
    e = synth.rmat_edges(12, 1 << 15, seed=21)
    w = synth.edge_weights(e.shape[0], 22) if weighted else None
    return synth.csr_from_edges(1 << 12, e, w)


def _ring_with_isolated(n_ring=40, n_iso=24):
    """A ring on the first n_ring nodes, then n_iso isolated nodes."""
    n = n_ring + n_iso
    nbr = [[(i - 1) % n_ring, (i + 1) % n_ring] for i in range(n_ring)] + [[] for _ in range(n_iso)]
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum([len(x) for x in nbr])
    indices = np.array([v for x in nbr for v in sorted(x)], np.int32)
    return indptr, indices


def _sequential(fl, G, M, rp, neg):
    """Algorithm 1 through the separate calls, in felog_run's order."""
    act, n_active, id_base, rounds = None, G.n, 0, []
    wk, fb = rp.walk, rp.feedback
    for r in range(rp.max_rounds):
        if n_active == 0:
            break
        W = fl.Walks.generate(G, r=wk.walks_per_node, L=wk.length, seed=wk.seed,
                              id_base=id_base, kind=wk.kind, p=wk.p, q=wk.q, starts=act)
        if neg == fl.NEG_UNIGRAM and r == 0:
            M.set_unigram(W)
        st = M.train_epoch(W, rp.train)
        rounds.append((n_active, W.info()[0], st.pairs, st.minibatches, st.loss))
        id_base += W.info()[0]
        act = M.feedback(mu=fb.mu, k_s=fb.k_s, seed=fb.seed, round=r, mode=fb.mode,
                         active=act)
        n_active = act.count()
    return rounds, n_active


def _compare(fl, G, rp, neg, dim, prec=None):
    """Bit for bit, in both forms: the FP32 path and the BF16 form (whose
    apply sums each row's terms in touch order, without atomics) give the
    same rounds, losses and tables whether the walks overlap training or
    not."""
    kw = dict(dim=dim, neg_dist=neg, seed=7)
    if prec is not None:
        kw["precision"] = prec
    Ma = fl.Model.create(G, **kw)
    st = Ma.run(rp)
    Mb = fl.Model.create(G, **kw)
    rounds, final = _sequential(fl, G, Mb, rp, neg)
    got = [(st.active[r], st.walks[r], st.train[r].pairs, st.train[r].minibatches,
            st.train[r].loss) for r in range(st.rounds)]
    _say("rounds", got)
    for r in range(st.rounds):
        assert st.ms_walk[r] > 0.0
    assert got == rounds
    assert st.final_active == final
    for t in (fl.TABLE_IN, fl.TABLE_OUT):
        assert np.array_equal(Ma.read(t), Mb.read(t))
    return st


@pytest.mark.parametrize("P", [1024, 4096])
def test_overlapped_rounds_equal_sequential_fp32(fl, ctx, P):
    g = _rmat12(False)
    _say("overlap rmat12 uniform degree-noise P=%d chunk 777" % P)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    rp = fl.felog_run_params()
    rp.walk = fl.felog_walk_params(fl.WALK_UNIFORM, 5, 20, 1.0, 1.0, 3, 0)
    rp.train = fl.train_params(window=4, negatives=5, minibatch_pairs=P, chunk_walks=777,
                               seed=5)
    rp.feedback = fl.felog_feedback_params(0.7, 8, fl.FEEDBACK_MONOTONE, 6, 0)
    rp.max_rounds = 3
    st = _compare(fl, G, rp, fl.NEG_DEGREE, 64)
    assert st.rounds >= 2


def test_overlapped_rounds_with_empty_chunks(fl, ctx):
    """Chunks 5 to 7 and 13 to 15 of eight walks start at isolated nodes only:
    they yield no pairs, and their events are never waited for."""
    indptr, indices = _ring_with_isolated()
    _say("overlap ring+isolated chunk 8")
    G = fl.Graph.from_csr(ctx, indptr, indices)
    rp = fl.felog_run_params()
    rp.walk = fl.felog_walk_params(fl.WALK_UNIFORM, 2, 12, 1.0, 1.0, 9, 0)
    rp.train = fl.train_params(window=3, negatives=3, minibatch_pairs=64, chunk_walks=8, seed=1)
    rp.feedback = fl.felog_feedback_params(2.0, 4, fl.FEEDBACK_MONOTONE, 2, 0)
    rp.max_rounds = 2
    st = _compare(fl, G, rp, fl.NEG_DEGREE, 64)
    assert st.rounds == 2 and st.walks[0] == 128


def test_overlapped_rounds_node2vec_unigram(fl, ctx):
    g = _rmat12(True)
    _say("overlap rmat12 weighted node2vec unigram-noise chunk 1000")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices, g.weights)
    rp = fl.felog_run_params()
    rp.walk = fl.felog_walk_params(fl.WALK_NODE2VEC, 4, 16, 0.5, 2.0, 11, 0)
    rp.train = fl.train_params(window=3, negatives=4, minibatch_pairs=4096, chunk_walks=1000,
                               seed=12)
    rp.feedback = fl.felog_feedback_params(0.8, 6, fl.FEEDBACK_RECOMPUTE_ALL, 13, 0)
    rp.max_rounds = 3
    _compare(fl, G, rp, fl.NEG_UNIGRAM, 64)


def test_overlapped_rounds_bf16(fl, ctx):
    g = _rmat12(False)
    _say("overlap rmat12 bf16 chunk 2000")
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    rp = fl.felog_run_params()
    rp.walk = fl.felog_walk_params(fl.WALK_UNIFORM, 4, 20, 1.0, 1.0, 14, 0)
    rp.train = fl.train_params(window=4, negatives=5, minibatch_pairs=1024, chunk_walks=2000,
                               seed=15, shared_negatives=256)
    rp.feedback = fl.felog_feedback_params(0.7, 8, fl.FEEDBACK_MONOTONE, 16, 0)
    rp.max_rounds = 1
    _compare(fl, G, rp, fl.NEG_DEGREE, 64, fl.PREC_BF16)
