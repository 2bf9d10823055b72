"""The persistent small-minibatch SGNS update (plan launches + one cooperative
update launch per group of minibatches) against the per-minibatch launches
and against the oracle.

- Bit-identical tables and equal row counts and losses (up to the FP64 loss
  summation order) against path 1, the per-minibatch launches, over ragged
  ranges of minibatches, at d = 64/128/256, K = 1/5/6, P = 333/1024 and on
  graphs with rows touched many times per minibatch (the exact-sum rows).
- Against the oracle from a teacher-forced state: the tables after a few
  minibatches, every row's change within 1e-5 of the oracle's (norm) plus
  1e-12 absolute.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def fl():
    import os
    from paper_2606_22180_amd import build, felog
    if not os.path.exists(build.LIB):
        build.build()
    felog.load()
    return felog


@pytest.fixture(scope="module")
def sbm():
    return synth.build_graph("sbm1k")


def _rmat(scale, edges, seed):
    e = synth.rmat_edges(scale, edges, seed=seed)
    return synth.csr_from_edges(1 << scale, e)


def _both_paths(fl, g, *, dim, K, P, window, L, r, first, n, neg=None, blocks=0, seed=3):
    """Train minibatches [first, first + n) from the same state on both paths;
    return the two models' tables and stats."""
    out = []
    for path in (1, 0):
        ctx = fl.Context(0)
        ctx.set_sgns_path(path, blocks)
        G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
        W = fl.Walks.generate(G, r=r, L=L, seed=11)
        M = fl.Model.create(G, dim=dim, neg_dist=neg if neg is not None else fl.NEG_DEGREE,
                            seed=5)
        if neg == fl.NEG_UNIGRAM:
            M.set_unigram(W)
        prm = fl.train_params(window=window, negatives=K, minibatch_pairs=P, seed=seed)
        if first:
            # a trained state first, on the per-minibatch path for both
            ctx.set_sgns_path(1)
            M.train_steps(W, prm, 0, first)
            ctx.set_sgns_path(path, blocks)
        st = M.train_steps(W, prm, first, n)
        out.append((M.read(fl.TABLE_IN), M.read(fl.TABLE_OUT), st))
        M.close()
        W.close()
        G.close()
        ctx.close()
    return out


def _check_identical(res, what):
    (i1, o1, s1), (i0, o0, s0) = res
    assert s1.path == 0 and s0.path == 1, (s1.path, s0.path)
    assert s1.minibatches == s0.minibatches and s1.pairs == s0.pairs
    assert (s1.rows_in, s1.rows_out, s1.rows_out_single) == (s0.rows_in, s0.rows_out,
                                                             s0.rows_out_single), what
    assert abs(s1.loss - s0.loss) <= 1e-12 * abs(s1.loss), (what, s1.loss, s0.loss)
    di = int((i1.view(np.uint32) != i0.view(np.uint32)).sum())
    do = int((o1.view(np.uint32) != o0.view(np.uint32)).sum())
    _say("%s: %d minibatches, %d pairs, rows in %d out %d (once %d), differing words in %d "
         "out %d, blocks %d" % (what, s0.minibatches, s0.pairs, s0.rows_in, s0.rows_out,
                                s0.rows_out_single, di, do, s0.update_blocks))
    assert di == 0 and do == 0, what


@pytest.mark.parametrize("dim,K,P", [(64, 5, 1024), (128, 1, 333), (256, 6, 1024)])
def test_small_update_equals_launches_sbm(fl, sbm, dim, K, P):
    """sbm1k: 1,000 nodes, so rows take many touches per minibatch (exact-sum
    rows of more than 16 touches, in and out tables)."""
    res = _both_paths(fl, sbm.train, dim=dim, K=K, P=P, window=5, L=40, r=10, first=0, n=600)
    _check_identical(res, "sbm1k d=%d K=%d P=%d" % (dim, K, P))


@pytest.mark.parametrize("n", [777, 1500])
def test_small_update_equals_launches_rmat(fl, n):
    """R-MAT 2^14, d = 128, K = 5, P = 1,024, unigram noise: a ragged range of
    minibatches that crosses launch groups of 64, from a trained state (777
    and 1,500 minibatches)."""
    g = _rmat(14, 1 << 18, seed=4)
    res = _both_paths(fl, g, dim=128, K=5, P=1024, window=10, L=80, r=2, first=300, n=n,
                      neg=fl.NEG_UNIGRAM)
    _check_identical(res, "rmat14 d=128 K=5 P=1024 n=%d" % n)


def test_small_update_block_counts(fl, sbm):
    """The grid size does not change the result (64 and 512 workgroups, the
    latter capped at what is resident)."""
    base = _both_paths(fl, sbm.train, dim=128, K=5, P=1024, window=5, L=40, r=10, first=0,
                       n=300)
    for blocks in (64, 512):
        res = _both_paths(fl, sbm.train, dim=128, K=5, P=1024, window=5, L=40, r=10, first=0,
                          n=300, blocks=blocks)
        assert np.array_equal(res[1][0], base[1][0]) and np.array_equal(res[1][1], base[1][1])
        _say("blocks %d: tables equal to the default grid's (%d workgroups)"
             % (blocks, res[1][2].update_blocks))


def test_small_update_matches_oracle(fl, orc, sbm):
    """Teacher-forced: the oracle's tables in, eight minibatches on the small
    path, every row's change against the oracle's."""
    g = sbm.train
    P, K, dim = 1024, 5, 64
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=40, seed=11)
    walks = orc.walks_uniform(g, np.arange(g.n), 10, 40, 11)
    assert np.array_equal(W.read(), walks)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    prm = fl.train_params(window=5, negatives=K, minibatch_pairs=P, seed=3)
    tin, tout = orc.init_tables(g.n, dim, 5)
    orc.train_epoch(tin, tout, walks, window=5, K=K, lr0=prm.lr_start, lr_end=prm.lr_end, P=P,
                    seed=3, cdf=cdf, mb_end=500)
    M = fl.Model.create(G, dim=dim, neg_dist=fl.NEG_DEGREE, seed=5)
    M.write(fl.TABLE_IN, tin)
    M.write(fl.TABLE_OUT, tout)
    st = M.train_steps(W, prm, 500, 8)
    assert st.path == 1
    ref_in, ref_out = tin.copy(), tout.copy()
    res = orc.train_epoch(ref_in, ref_out, walks, window=5, K=K, lr0=prm.lr_start,
                          lr_end=prm.lr_end, P=P, seed=3, cdf=cdf, mb_begin=500, mb_end=508)
    assert st.pairs == res.pairs
    assert abs(st.loss - res.loss) <= 1e-5 * abs(res.loss)
    for what, a, b, before in (("in", M.read(fl.TABLE_IN), ref_in, tin),
                               ("out", M.read(fl.TABLE_OUT), ref_out, tout)):
        dg = a.astype(np.float64) - before
        dr = b.astype(np.float64) - before
        num = np.linalg.norm(dg - dr, axis=1)
        nref = np.linalg.norm(dr, axis=1)
        bad = int((num > 1e-5 * nref + 1e-12).sum())
        _say("oracle, 8 minibatches, %s rows changed %d, max rel %.2e, misses %d"
             % (what, int((nref > 0).sum()), (num / np.maximum(nref, 1e-30)).max(), bad))
        assert bad == 0, what


def test_single_stream_identical(fl, sbm):
    """One stream for every launch (plans in issue order after the updates
    they would overlap) gives the same tables and loss as two streams, on the
    persistent path and on the per-minibatch launches."""
    g = sbm.train
    for path in (0, 1):
        res = []
        for single in (False, True):
            ctx = fl.Context(0)
            ctx.set_sgns_path(path)
            ctx.set_single_stream(single)
            G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
            W = fl.Walks.generate(G, r=10, L=40, seed=11)
            M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=5)
            prm = fl.train_params(window=5, negatives=5, minibatch_pairs=1024, seed=3)
            st = M.train_steps(W, prm, 0, 200)
            res.append((M.read(fl.TABLE_IN), M.read(fl.TABLE_OUT), st.loss))
            for o in (M, W, G, ctx):
                o.close()
        (i0, o0, l0), (i1, o1, l1) = res
        _say("path %d: one stream vs two, tables equal %s, loss %.9e %.9e"
             % (path, np.array_equal(i0, i1) and np.array_equal(o0, o1), l0, l1))
        assert np.array_equal(i0, i1) and np.array_equal(o0, o1)
        assert l0 == l1


def test_small_update_wide_k_at_d64_uses_launches(fl, sbm):
    """d = 64 with K = 15: four pairs of 17 touches do not fit the 64 lanes the
    persistent forward gives a wave's pairs, so the per-minibatch launches
    serve the call on path 0 too, with the same tables."""
    (i1, o1, s1), (i0, o0, s0) = _both_paths(fl, sbm.train, dim=64, K=15, P=256, window=5,
                                             L=40, r=10, first=0, n=40)
    _say("d=64 K=15 P=256: paths %d and %d" % (s1.path, s0.path))
    assert s1.path == 0 and s0.path == 0
    assert np.array_equal(i1, i0) and np.array_equal(o1, o0)


def test_phase_clocks(fl, sbm):
    """With timing on, the persistent update reports its four phases (forward,
    barrier, apply, barrier) per minibatch from the device wall clock; they add
    up to the launches' HIP-event time per minibatch, and timing leaves the
    tables unchanged."""
    g = sbm.train
    res = []
    for timing in (0, 1):
        ctx = fl.Context(0)
        ctx.set_timing(timing)
        G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
        W = fl.Walks.generate(G, r=10, L=40, seed=11)
        M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=5)
        prm = fl.train_params(window=5, negatives=5, minibatch_pairs=1024, seed=3)
        st = M.train_steps(W, prm, 0, 300)
        res.append((M.read(fl.TABLE_IN), M.read(fl.TABLE_OUT), st))
        for o in (M, W, G, ctx):
            o.close()
    (i0, o0, s0), (i1, o1, s1) = res
    assert np.array_equal(i0, i1) and np.array_equal(o0, o1)
    ph = list(s1.us_phase)
    ev = 1e3 * s1.ms_update / s1.timed_minibatches
    _say("phases per minibatch: forward %.2f barrier %.2f apply %.2f barrier %.2f us "
         "(sum %.2f); events %.2f us" % (*ph, sum(ph), ev))
    assert s1.path == 1 and s1.timed_minibatches == 300
    assert all(p > 0 for p in ph) and list(s0.us_phase) == [0.0] * 4
    assert 0.7 * ev <= sum(ph) <= 1.1 * ev


@pytest.mark.parametrize("dim,K,P", [(128, 12, 512), (64, 13, 512), (256, 10, 512),
                                     (256, 20, 256)])
def test_small_update_register_spilling_instantiations(fl, sbm, dim, K, P):
    """Instantiations of the persistent update whose registers spill to
    scratch (K >= 11 at d = 64 and 128, every K at d = 256) against the
    per-minibatch launches, which do not spill at these sizes: bit-identical
    tables over 200 minibatches."""
    res = _both_paths(fl, sbm.train, dim=dim, K=K, P=P, window=5, L=40, r=10, first=0, n=200)
    _check_identical(res, "spilling instantiation d=%d K=%d P=%d" % (dim, K, P))
