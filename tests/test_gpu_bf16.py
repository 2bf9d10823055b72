"""GPU parity of the BF16 shared-negative form against the oracle's emulation.

The oracle rounds rows and the coefficients G to BF16 exactly as the form
defines and sums in FP64; the GPU sums in FP32 on MFMA.  A G entry whose FP32
and FP64 values round to different BF16 neighbours differs by one BF16 ulp
(2^-8 relative), so per updated row
  ||d_gpu - d_orc|| <= 2^-8 ||m|| + 1e-5 ||d_orc||,
with m the row's sum of |term| vectors.  The FP32 masters and BF16 copies are
checked bit-exactly (copy = round-to-nearest-even of the master).  Every
oracle input is the oracle's own: its walks, noise table and tables, which
are written into the library before each checked step.
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
    import os
    from paper_2606_22180_amd import build, felog
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


def _bf16_bits(orc, x):
    return orc.bf16_round(x).view(np.uint32) >> 16


def _rne16(x):
    """Round-to-nearest-even to the upper 16 bits of float32 (finite values)."""
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32)


def _setup(fl, ctx, g, *, dim, P, M, K, L=40, window=5, r=10, seed=3):
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=r, L=L, seed=11)
    Mo = fl.Model.create(G, dim=dim, neg_dist=fl.NEG_DEGREE, seed=5, precision=fl.PREC_BF16)
    prm = fl.train_params(window=window, negatives=K, minibatch_pairs=P, seed=seed,
                          shared_negatives=M)
    return G, W, Mo, prm


def test_bf16_copies_track_masters(fl, ctx, orc, sbm):
    g = sbm.train
    _say("bf16 copies = rne(masters)")
    G, W, Mo, prm = _setup(fl, ctx, g, dim=64, P=1024, M=1024, K=5)
    rng = np.random.default_rng(3)
    tin = rng.normal(0, 0.3, (g.n, 64)).astype(np.float32)
    tout = rng.normal(0, 0.3, (g.n, 64)).astype(np.float32)
    Mo.write(fl.TABLE_IN, tin)
    Mo.write(fl.TABLE_OUT, tout)
    assert np.array_equal(Mo.read_bf16(fl.TABLE_IN).astype(np.uint32), _bf16_bits(orc, tin))
    assert np.array_equal(Mo.read_bf16(fl.TABLE_OUT).astype(np.uint32), _bf16_bits(orc, tout))
    # after training steps the copies still equal the rounded masters (a property
    # of the library's own state, checked without the oracle)
    for step in range(2):
        Mo.train_steps(W, prm, step * 100, 100)
        for which in (fl.TABLE_IN, fl.TABLE_OUT):
            assert np.array_equal(Mo.read_bf16(which).astype(np.uint32), _rne16(Mo.read(which)))


def _agg(n, d, rows, vals):
    out = np.zeros((n, d))
    np.add.at(out, rows, vals)
    return out


@pytest.mark.parametrize("dim,pre,P,M", [(64, 0, 1024, 1024), (128, 300, 1024, 1024),
                                         (256, 50, 1024, 1024), (128, 20, 4096, 1024)])
def test_bf16_step_parity(fl, ctx, orc, sbm, dim, pre, P, M):
    """P = 4096, M = 1024: 9,216 touches, more than an LDS plan sorts, so the
    rows are grouped by the radix-sort plan."""
    g = sbm.train
    K = 5
    _say("bf16 step parity sbm1k d=%d P=%d M=%d after %d minibatches" % (dim, P, M, pre))
    G, W, Mo, prm = _setup(fl, ctx, g, dim=dim, P=P, M=M, K=K)
    walks = orc.walks_uniform(g, np.arange(g.n), 10, 40, 11)
    assert np.array_equal(W.read(), walks)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    assert np.array_equal(Mo.read_cdf(), cdf)
    B, _ = orc.count_minibatches(walks, 5, P)
    tin, tout = orc.init_tables(g.n, dim, 5)
    if pre:   # a trained state, made by the oracle
        orc.train_epoch(tin, tout, walks, window=5, K=K, lr0=prm.lr_start, lr_end=prm.lr_end,
                        P=P, seed=prm.seed, cdf=cdf, mb_end=pre)
    for b in (pre, pre + 1, B - 1):
        Mo.write(fl.TABLE_IN, tin)
        Mo.write(fl.TABLE_OUT, tout)
        ri, di, ro, do, loss = Mo.train_delta(W, prm, b)
        mb = orc.minibatch_pairs(walks, 5, P, b)
        neg = orc.shared_negatives(b, 0, M, prm.seed, cdf)
        lr = orc.lr_at(b, B, prm.lr_start, prm.lr_end)
        dctx, dneg, dctr, oloss = orc.shared_neg_step(tin, tout, mb.ctx, mb.ctr, neg, K, lr,
                                                      bf16=True)
        n = g.n
        assert set(ri.tolist()) == set(mb.ctx.tolist())
        assert set(ro.tolist()) == set(mb.ctr.tolist()) | set(neg.tolist())
        ref_in = _agg(n, dim, mb.ctx, dctx)
        ref_out = _agg(n, dim, neg, dneg) + _agg(n, dim, mb.ctr, dctr)
        # |term| mass per row, from the same BF16-rounded operands
        C = orc.bf16_round(tin[mb.ctx]).astype(np.float64)
        O = orc.bf16_round(tout[mb.ctr]).astype(np.float64)
        N = orc.bf16_round(tout[neg]).astype(np.float64)
        S = C @ N.T
        Gm = lr * K / M / (1 + np.exp(-S)) * (neg[None, :] != mb.ctr[:, None])
        s0 = (C * O).sum(1)
        g0 = lr / (1 + np.exp(s0))
        m_in = _agg(n, dim, mb.ctx, Gm @ np.abs(N) + g0[:, None] * np.abs(O))
        m_out = _agg(n, dim, neg, Gm.T @ np.abs(C)) + _agg(n, dim, mb.ctr, g0[:, None] * np.abs(C))
        for what, gpu_rows, gpu_vals, ref, mass in (("in", ri, di, ref_in, m_in),
                                                   ("out", ro, do, ref_out, m_out)):
            gpu = np.zeros((n, dim))
            gpu[gpu_rows] = gpu_vals
            err = np.linalg.norm(gpu - ref, axis=1)
            tol = 2.0 ** -8 * np.linalg.norm(mass, axis=1) + 1e-5 * np.linalg.norm(ref, axis=1)
            rel = err / np.maximum(np.linalg.norm(ref, axis=1), 1e-30)
            nz = np.abs(ref).sum(1) > 0
            _say("mb %d %s: rows %d, max rel err vs bf16 emulation %.3e, max abs %.3e, bad %d" % (
                b, what, int(nz.sum()), rel[nz].max() if nz.any() else 0.0, err.max(),
                int((err > tol + 1e-30).sum())))
            assert (err <= tol + 1e-30).all()
        assert abs(loss - oloss) <= 1e-4 * abs(oloss)
        # the same step without BF16 rounding (FP64 throughout): the form's error
        f_ctx, f_neg, f_ctr, _ = orc.shared_neg_step(tin, tout, mb.ctx, mb.ctr, neg, K, lr,
                                                     bf16=False)
        f_out = _agg(n, dim, neg, f_neg) + _agg(n, dim, mb.ctr, f_ctr)
        gpu = np.zeros((n, dim))
        gpu[ro] = do
        e64 = np.linalg.norm(gpu - f_out) / max(np.linalg.norm(f_out), 1e-30)
        _say("mb %d: relative error of the BF16 step vs FP64: %.3e" % (b, e64))
        # the oracle applies its own step, so the next check starts elsewhere
        tin = (tin + ref_in).astype(np.float32)
        tout = (tout + ref_out).astype(np.float32)


def test_bf16_epoch_auc(fl, ctx, orc, sbm):
    """One epoch of the BF16 shared-negative form on sbm1k next to the FP32
    per-pair form (same walks): link-prediction AUC within 0.01 (the two forms
    differ in their negative estimator, so this is a matched-quality check,
    not a parity bound)."""
    g = sbm.train
    G, W, Mo, prm = _setup(fl, ctx, g, dim=64, P=1024, M=1024, K=5)
    st = Mo.train_epoch(W, prm)
    a16 = link_auc_of(Mo.read(fl.TABLE_IN), sbm)
    M32 = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=5)
    st32 = M32.train_epoch(W, fl.train_params(window=5, negatives=5, minibatch_pairs=1024,
                                              seed=3))
    a32 = link_auc_of(M32.read(fl.TABLE_IN), sbm)
    _say("epoch sbm1k: AUC bf16 shared=%.4f fp32 per-pair=%.4f; ms bf16=%.1f fp32=%.1f" % (
        a16, a32, st.ms, st32.ms))
    assert st.pairs == st32.pairs
    assert abs(a16 - a32) <= 0.01


@pytest.mark.parametrize("P,M", [(1024, 1024), (4096, 1024), (64, 4096)])
def test_bf16_bit_reproducible(fl, ctx, sbm, P, M):
    """The same minibatches from the same state give bit-identical masters:
    every row's terms are summed in touch order, never with atomics.  sbm1k
    has 1,000 nodes, so a minibatch touches most rows several times (hub rows
    dozens of times) through contexts, centres and negatives alike.  P = 4096
    takes the radix-sort plan, the others the LDS plan; (64, 4096) has far
    more negatives than pairs."""
    g = sbm.train
    tabs = []
    for run in range(2):
        G, W, Mo, prm = _setup(fl, ctx, g, dim=128, P=P, M=M, K=5)
        st = Mo.train_steps(W, prm, 0, 60)
        tabs.append((Mo.read(fl.TABLE_IN), Mo.read(fl.TABLE_OUT), st.loss))
        Mo.close()
        W.close()
        G.close()
    (i0, o0, l0), (i1, o1, l1) = tabs
    di = int((i0.view(np.uint32) != i1.view(np.uint32)).sum())
    do = int((o0.view(np.uint32) != o1.view(np.uint32)).sum())
    _say("bf16 P=%d M=%d, 60 minibatches twice: differing words in %d out %d, loss %.9e %.9e"
         % (P, M, di, do, l0, l1))
    assert di == 0 and do == 0
    assert l0 == l1
