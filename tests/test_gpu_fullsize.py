"""GPU parity at the full sizes of the measured configurations, on outputs the
oracle computes one by one (sampled walks, one minibatch, sampled Psi) and on
properties that hold at any size.

- R-MAT 2^20 (the bench's workload and launch configuration: P = 65,536,
  d = 128, K = 5, w = 10): all walks bit-exact, the unigram noise table
  bit-exact, one teacher-forced minibatch within the per-step tolerance, Psi of
  2,000 sampled nodes, and a minibatch's update bit-identical when repeated.
- R-MAT 2^22 (FP32 and BF16 shared-negative forms, P = M = 1,024) and weighted
  R-MAT 2^23 (node2vec p = 0.5, q = 2, the step at P = 1,024): sampled walks,
  the first 2^20-walk chunk and one minibatch of each form.
- The whole round-1 corpus of R-MAT 2^20 and its unigram table need minutes
  of oracle time and run only with FELOG_FULL_SIZE=1.

Every oracle input is the oracle's own; teacher forcing writes the oracle's
tables into the library.
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FULL = os.environ.get("FELOG_FULL_SIZE") == "1"


def _say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def fl():
    from paper_2606_22180_amd import build, felog
    if not os.path.exists(build.LIB):
        build.build()
    felog.load()
    return felog


def _rows_mass(tin, tout, ctx_, ctr, neg, lr):
    """Per-row sums of |term| vectors of one minibatch (FP64), as dicts row ->
    vector, for the in and out tables."""
    A = tin[ctx_].astype(np.float64)
    targets = [ctr] + [neg[:, k] for k in range(neg.shape[1])]
    in_rows, in_inv = np.unique(ctx_, return_inverse=True)
    m_in = np.zeros((in_rows.shape[0], tin.shape[1]))
    outs = np.concatenate(targets)
    out_rows, out_inv = np.unique(outs, return_inverse=True)
    m_out = np.zeros((out_rows.shape[0], tin.shape[1]))
    P = ctx_.shape[0]
    for k, t in enumerate(targets):
        T = tout[t].astype(np.float64)
        s = (A * T).sum(1)
        if k == 0:
            g = lr / (1 + np.exp(s))
            keep = np.ones(P, bool)
        else:
            g = lr / (1 + np.exp(-s))
            keep = t != ctr
        np.add.at(m_in, in_inv[keep], np.abs(g[keep, None] * T[keep]))
        np.add.at(m_out, out_inv[k * P:(k + 1) * P][keep], np.abs(g[keep, None] * A[keep]))
    return in_rows, m_in, out_rows, m_out


def _check_sparse(rows_gpu, d_gpu, rows_ref, d_ref, mrows, mass, what):
    """The per-step bar on every touched row: |d_gpu - d_orc| <= 1e-5 |d_orc|
    + 1e-12 (norms over the row).  The rows' |term| mass is printed as the
    cancellation scale."""
    assert np.array_equal(np.sort(rows_gpu), np.sort(rows_ref)), what
    og = np.argsort(rows_gpu)
    orf = np.argsort(rows_ref)
    g = d_gpu[og].astype(np.float64)
    r = d_ref[orf]
    rows = rows_gpu[og]
    m = mass[np.searchsorted(mrows, rows)]
    num = np.linalg.norm(g - r, axis=1)
    nref = np.linalg.norm(r, axis=1)
    tol = 1e-5 * nref + 1e-12
    rel = num / np.maximum(nref, 1e-30)
    bad = np.nonzero(num > tol)[0]
    canc = np.linalg.norm(m, axis=1) / np.maximum(nref, 1e-30)
    _say("%s: rows %d, max rel %.3e, misses of 1e-5|d|+1e-12: %d (max |mass|/|d| %.1f)"
         % (what, rows.shape[0], rel.max(), len(bad), canc.max()))
    assert len(bad) == 0, (what, rows[bad[:5]], num[bad[:5]], tol[bad[:5]])


def _sampled_walks(W, orc, g, L, seed, n_sample, rng, p=None, q=None):
    n_walks = W.info()[0]
    ids = np.sort(rng.choice(n_walks, n_sample, replace=False))
    for i in ids:
        gw = W.read_range(int(i), 1)[0]
        start = np.array([i % g.n], np.int32)
        if p is None:
            ow = orc.walks_uniform(g, start, 1, L, seed, int(i))[0]
        else:
            ow, _ = orc.walks_node2vec(g, start, 1, L, p, q, seed, int(i))
            ow = ow[0]
        assert np.array_equal(gw, ow), ("walk", int(i))
    return ids


def _step(fl, orc, M, W, walks, cdf, tin, tout, *, P, K, window, b, seed, what,
          lr0=0.025, lr1=1e-4):
    """Teacher-forced parity of minibatch b from the oracle's tables."""
    prm = fl.train_params(window=window, negatives=K, minibatch_pairs=P, seed=seed,
                          lr_start=lr0, lr_end=lr1)
    # with a constant rate the corpus' minibatch count does not enter
    B = 1 if lr0 == lr1 else orc.count_minibatches(walks, window, P)[0]
    M.write(fl.TABLE_IN, tin)
    M.write(fl.TABLE_OUT, tout)
    ri, di, ro, do, loss = M.train_delta(W, prm, b)
    mb = orc.minibatch_pairs(walks, window, P, b)
    ng = orc.draw_negatives(mb, 0, K, seed, cdf)
    lr = orc.lr_at(b, B, prm.lr_start, prm.lr_end)
    ref = orc.sgns_step(tin.copy(), tout.copy(), mb.ctx, mb.ctr, ng, lr, apply=False)
    in_rows, m_in, out_rows, m_out = _rows_mass(tin, tout, mb.ctx, mb.ctr, ng, lr)
    _check_sparse(ri, di, ref.rows_in, ref.d_in, in_rows, m_in, what + " in")
    _check_sparse(ro, do, ref.rows_out, ref.d_out, out_rows, m_out, what + " out")
    assert abs(loss - ref.loss) <= 1e-5 * abs(ref.loss)
    return prm, (ri, di, ro, do, loss)


def test_rmat20_bench_configuration(fl, orc):
    """The bench's graph and launch configuration.  The oracle's brute-force
    pair counting takes about 20 s per 2^20-walk chunk on one core, so the
    checks stay inside the first chunk: its walks bit-exact, 48 walks of the
    other chunks, and minibatch 9001 (in the first chunk) with a constant
    learning rate."""
    sp = synth.build_graph("rmat20")
    g = sp.train
    _say("rmat20 n=%d nnz=%d: walks r=10 L=80, P=65536 step, psi" % (g.n, g.nnz))
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=80, seed=1)
    chunk = orc.walks_uniform(g, np.arange(1 << 20) % g.n, 1, 80, 1)
    assert np.array_equal(W.read_range(0, 1 << 20), chunk)
    _sampled_walks(W, orc, g, 80, 1, 48, np.random.default_rng(3))
    _say("first chunk and 48 sampled walks bit-exact")
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=2)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    assert np.array_equal(M.read_cdf(), cdf)
    tin, tout = orc.init_tables(g.n, 128, 2)
    rng = np.random.default_rng(4)            # a state away from the initial one
    tout += rng.normal(0, 0.05, tout.shape).astype(np.float32)
    b = 9001
    prm, first = _step(fl, orc, M, W, chunk, cdf, tin, tout, P=65536, K=5, window=10, b=b,
                       seed=3, what="rmat20 mb %d" % b, lr0=0.0125, lr1=0.0125)
    # the same minibatch again: bit-identical update
    M.write(fl.TABLE_IN, tin)
    M.write(fl.TABLE_OUT, tout)
    again = M.train_delta(W, prm, b)
    # the touched-row lists come in the atomics' order; each row's delta does not
    for r0, d0, r1, d1 in ((first[0], first[1], again[0], again[1]),
                           (first[2], first[3], again[2], again[3])):
        o0, o1 = np.argsort(r0), np.argsort(r1)
        assert np.array_equal(r0[o0], r1[o1])
        assert np.array_equal(d0[o0], d1[o1])
    assert first[4] == again[4]
    _say("minibatch %d repeated: every row's delta bit-identical" % b)
    # Psi of sampled nodes on the oracle's table
    act, psi = M.feedback(mu=0.65, k_s=10, seed=4, round=0, want_psi=True)
    nodes = np.sort(np.random.default_rng(5).choice(g.n, 2000, replace=False)).astype(np.int32)
    opsi = orc.psi(tin, g, nodes, 10, 4, 0)
    fin = np.isfinite(opsi)
    assert np.array_equal(np.isfinite(psi[nodes]), fin)
    assert np.abs(psi[nodes][fin] - opsi[fin]).max() <= 1e-12
    keep = set(act.read().tolist())
    assert all((int(v) in keep) == bool(f and p < 0.65) for v, p, f in zip(nodes, opsi, fin))
    _say("psi of 2000 sampled nodes within 1e-12, decisions equal")


@pytest.mark.slow
@pytest.mark.skipif(not FULL, reason="the oracle's full corpus takes minutes; FELOG_FULL_SIZE=1")
def test_rmat20_unigram_table(fl, orc):
    """The unigram^0.75 table of the whole round-1 corpus of R-MAT 2^20."""
    g = synth.build_graph("rmat20").train
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=80, seed=1)
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_UNIGRAM, seed=2)
    M.set_unigram(W)
    _say("oracle corpus of 10,485,760 walks")
    walks = orc.walks_uniform(g, np.arange(g.n), 10, 80, 1)
    assert np.array_equal(W.read(), walks)
    assert np.array_equal(M.read_cdf(), orc.neg_cdf(orc.corpus_counts(walks, g.n)))
    _say("all walks and the unigram table bit-exact")


def _bf16_step(fl, orc, G, W, chunk, cdf, tin, tout, b, what):
    """One BF16 shared-negative minibatch (P = M = 1,024, d = 128, K = 5, w =
    10) from the tables (tin, tout) against the oracle's BF16 emulation:
    every row's delta within 2^-8 of its |term| mass (one BF16 rounding of G
    per entry) plus 1e-5 of its norm; the loss within 1e-3."""
    B = 1
    Mb = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=2, precision=fl.PREC_BF16)
    Mb.write(fl.TABLE_IN, tin)
    Mb.write(fl.TABLE_OUT, tout)
    prm = fl.train_params(window=10, negatives=5, minibatch_pairs=1024, seed=3,
                          shared_negatives=1024, lr_start=0.0125, lr_end=0.0125)
    _say("bf16 shared-negative step, minibatch %d" % b)
    ri, di, ro, do, loss = Mb.train_delta(W, prm, b)
    Mb.close()
    mb = orc.minibatch_pairs(chunk, 10, 1024, b)
    neg = orc.shared_negatives(b, 0, 1024, 3, cdf)
    lr = orc.lr_at(b, B, prm.lr_start, prm.lr_end)
    dctx, dneg, dctr, oloss = orc.shared_neg_step(tin, tout, mb.ctx, mb.ctr, neg, 5, lr,
                                                  bf16=True)
    # reference sums and |term| mass per row (BF16-rounded operands, FP64 sums)
    rows_in, inv_in = np.unique(mb.ctx, return_inverse=True)
    outs = np.concatenate([neg, mb.ctr])
    rows_out, inv_out = np.unique(outs, return_inverse=True)
    ref_in = np.zeros((rows_in.shape[0], 128))
    np.add.at(ref_in, inv_in, dctx)
    ref_out = np.zeros((rows_out.shape[0], 128))
    np.add.at(ref_out, inv_out, np.concatenate([dneg, dctr]))
    Cm = orc.bf16_round(tin[mb.ctx]).astype(np.float64)
    Om = orc.bf16_round(tout[mb.ctr]).astype(np.float64)
    Nm = orc.bf16_round(tout[neg]).astype(np.float64)
    S = Cm @ Nm.T
    Gm = lr * 5 / 1024 / (1 + np.exp(-S)) * (neg[None, :] != mb.ctr[:, None])
    g0 = lr / (1 + np.exp((Cm * Om).sum(1)))
    m_in = np.zeros_like(ref_in)
    np.add.at(m_in, inv_in, Gm @ np.abs(Nm) + g0[:, None] * np.abs(Om))
    m_out = np.zeros_like(ref_out)
    np.add.at(m_out, inv_out, np.concatenate([Gm.T @ np.abs(Cm), g0[:, None] * np.abs(Cm)]))
    for side, gr, gd, rr, rd, mm in (("in", ri, di, rows_in, ref_in, m_in),
                                     ("out", ro, do, rows_out, ref_out, m_out)):
        assert np.array_equal(np.sort(gr), rr)
        gv = gd[np.argsort(gr)].astype(np.float64)
        err = np.linalg.norm(gv - rd, axis=1)
        tol = 2.0 ** -8 * np.linalg.norm(mm, axis=1) + 1e-5 * np.linalg.norm(rd, axis=1)
        rel = err / np.maximum(np.linalg.norm(rd, axis=1), 1e-30)
        _say("%s bf16 mb %d %s: rows %d, max rel %.3e, bad %d" % (
            what, b, side, rr.shape[0], rel.max(), int((err > tol + 1e-30).sum())))
        assert (err <= tol + 1e-30).all()
    assert abs(loss - oloss) <= 1e-3 * abs(oloss)


def test_rmat22_fp32_and_bf16_forms(fl, orc):
    """R-MAT 2^22: the FP32 per-pair and BF16 shared-negative forms on one
    minibatch of the first chunk (degree^0.75 noise: the oracle's corpus of
    42M walks would take it many minutes; the unigram table is checked on
    R-MAT 2^20)."""
    sp = synth.build_graph("rmat22")
    g = sp.train
    _say("rmat22 n=%d nnz=%d: sampled walks, FP32 and BF16 steps at P=M=1024" % (g.n, g.nnz))
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=80, seed=1)
    rng = np.random.default_rng(11)
    _sampled_walks(W, orc, g, 80, 1, 48, rng)
    chunk = orc.walks_uniform(g, np.arange(1 << 20) % g.n, 1, 80, 1)
    assert np.array_equal(W.read_range(0, 1 << 20), chunk)
    _say("first chunk and 48 sampled walks bit-exact")
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=2)
    assert np.array_equal(M.read_cdf(), cdf)
    tin, tout = orc.init_tables(g.n, 128, 2)
    tout += np.random.default_rng(4).normal(0, 0.05, tout.shape).astype(np.float32)
    b = 123457                                # inside the first chunk
    _say("fp32 step, minibatch %d" % b)
    _step(fl, orc, M, W, chunk, cdf, tin, tout, P=1024, K=5, window=10, b=b, seed=3,
          what="rmat22 fp32 mb %d" % b, lr0=0.0125, lr1=0.0125)
    _bf16_step(fl, orc, G, W, chunk, cdf, tin, tout, b, "rmat22")


def test_rmat23w_node2vec(fl, orc):
    """Weighted R-MAT 2^23, node2vec p = 0.5, q = 2: sampled walks and the
    first 2^20-walk chunk bit-exact, then one FP32 step and one BF16
    shared-negative step on that chunk's pairs against the oracle."""
    sp = synth.build_graph("rmat23w")
    g = sp.train
    _say("rmat23w n=%d nnz=%d: node2vec p=0.5 q=2, r=10 L=80" % (g.n, g.nnz))
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices, g.weights)
    W = fl.Walks.generate(G, r=10, L=80, seed=1, kind=fl.WALK_NODE2VEC, p=0.5, q=2.0)
    assert W.capped() == 0
    rng = np.random.default_rng(13)
    _sampled_walks(W, orc, g, 80, 1, 48, rng, p=0.5, q=2.0)
    # one FP32 step on the first chunk's walks (degree^0.75 noise: the unigram
    # counts of 84M node2vec walks would take the oracle many minutes)
    first = W.read_range(0, 1 << 20)
    ow = orc.walks_node2vec(g, np.arange(1 << 20, dtype=np.int32) % g.n, 1, 80, 0.5, 2.0, 1, 0)[0]
    assert np.array_equal(first, ow)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=2)
    assert np.array_equal(M.read_cdf(), cdf)
    tin, tout = orc.init_tables(g.n, 128, 2)
    _say("first chunk bit-exact; step at minibatch 777 of its pairs")
    # the first chunk alone is a corpus whose minibatch 777 is the library's 777;
    # a constant learning rate keeps lr independent of the corpus' minibatch count
    _step(fl, orc, M, W, ow, cdf, tin, tout, P=1024, K=5, window=10, b=777, seed=3,
          what="rmat23w fp32 mb 777", lr0=0.025, lr1=0.025)
    M.close()
    # the BF16 shared-negative form on the same walks, from the oracle's
    # initial tables with out rows moved off zero
    tout += np.random.default_rng(4).normal(0, 0.05, tout.shape).astype(np.float32)
    _bf16_step(fl, orc, G, W, ow, cdf, tin, tout, 777, "rmat23w")


def test_rmat23w_persistent_update(fl, orc):
    """The headline launch configuration on weighted R-MAT 2^23: the
    persistent update (64 workgroups, P = 1,024, d = 128, K = 5, w = 10) runs
    minibatches 777-780 of the first 2^20-walk chunk in one call from the
    oracle's tables; the oracle runs the same four minibatches in order.

    Every row the minibatches touch must change by the oracle's change within
    1e-5 of its norm plus 1e-12, or else every entry of the row must lie
    within m FP32 spacings of the oracle's entry, m the number of the four
    minibatches that stored the row: both sides store each entry as the FP32
    rounding of an FP64 value, and where the two FP64 values straddle a
    rounding boundary the stored entries differ by exactly one spacing (the
    per-step delta tests compare unrounded deltas and need no such case).
    The rows of the second kind are counted and printed."""
    sp = synth.build_graph("rmat23w")
    g = sp.train
    _say("rmat23w persistent update, minibatches 777-780")
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices, g.weights)
    starts = fl.Active.from_host(G, np.arange(1 << 20, dtype=np.int32))
    W = fl.Walks.generate(G, r=1, L=80, seed=1, kind=fl.WALK_NODE2VEC, p=0.5, q=2.0,
                          starts=starts)
    ow = orc.walks_node2vec(g, np.arange(1 << 20, dtype=np.int32), 1, 80, 0.5, 2.0, 1, 0)[0]
    assert np.array_equal(W.read(), ow)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=2)
    tin, tout = orc.init_tables(g.n, 128, 2)
    # a state away from the initial one (out = 0 would zero every in-row delta)
    tout += np.float32(0.05) * np.random.default_rng(4).standard_normal(tout.shape,
                                                                         dtype=np.float32)
    M.write(fl.TABLE_IN, tin)
    M.write(fl.TABLE_OUT, tout)
    prm = fl.train_params(window=10, negatives=5, minibatch_pairs=1024, seed=3,
                          lr_start=0.0125, lr_end=0.0125)
    st = M.train_steps(W, prm, 777, 4)
    assert st.path == 1 and st.update_blocks == 64 and st.minibatches == 4
    # rows touched, with the number of minibatches that touch each
    m_in, m_out = {}, {}
    for b in range(777, 781):
        mb = orc.minibatch_pairs(ow, 10, 1024, b)
        ng = orc.draw_negatives(mb, 0, 5, 3, cdf)
        for r in set(mb.ctx.tolist()):
            m_in[r] = m_in.get(r, 0) + 1
        for r in set(mb.ctr.tolist()) | set(int(x) for x in ng.ravel().tolist() if x >= 0):
            m_out[r] = m_out.get(r, 0) + 1
    ref_in, ref_out = tin.copy(), tout.copy()
    res = orc.train_epoch(ref_in, ref_out, ow, window=10, K=5, lr0=0.0125, lr_end=0.0125,
                          P=1024, seed=3, cdf=cdf, mb_begin=777, mb_end=781)
    assert st.pairs == res.pairs
    assert abs(st.loss - res.loss) <= 1e-5 * abs(res.loss)
    for what, which, ref, before, touched in (("in", fl.TABLE_IN, ref_in, tin, m_in),
                                              ("out", fl.TABLE_OUT, ref_out, tout, m_out)):
        r = np.array(sorted(touched), dtype=np.int64)
        m = np.array([touched[x] for x in r.tolist()], dtype=np.float64)
        got = M.read(which)[r].astype(np.float64)
        dr = ref[r].astype(np.float64) - before[r]
        dg = got - before[r]
        num = np.linalg.norm(dg - dr, axis=1)
        nref = np.linalg.norm(dr, axis=1)
        out = np.nonzero(num > 1e-5 * nref + 1e-12)[0]
        ok = True
        for i in out.tolist():
            sp_ = np.spacing(np.abs(ref[r[i]])).astype(np.float64)
            steps = np.abs(got[i] - ref[r[i]].astype(np.float64)) / sp_
            _say("  %s row %d (stored by %d minibatches): rel %.2e, %d entries differ, by at "
                 "most %.3g FP32 spacings" % (what, r[i], m[i], num[i] / nref[i],
                                             int((steps > 0).sum()), steps.max()))
            ok = ok and steps.max() <= m[i]
        _say("%s: %d touched rows, max rel %.2e, outside the plain bar %d" % (
            what, r.shape[0], (num / np.maximum(nref, 1e-30)).max(), out.shape[0]))
        assert ok, what
    for o in (M, W, starts, G, ctx):
        o.close()
