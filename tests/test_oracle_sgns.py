"""Pins for the oracle's training step (Train in Algorithm 1, Eq. (1)-(2)).

The SGD update of one minibatch is pinned by
  * central finite differences of the FP64 minibatch loss (Eq. (2), negated);
  * torch autograd on the same loss written with torch's logsigmoid;
  * the closed-form loss at the initial state (out = 0 gives s = 0, so every
    term is log 2);
  * minibatch semantics: every pair reads the state at minibatch start, so a
    minibatch's delta is the sum of its pairs' single-pair deltas;
and the pair enumeration and noise distribution by brute force and closed
forms.
"""
import math

import numpy as np
import pytest
from scipy.stats import chisquare

import synth


def _rand_problem(rng, n=9, d=6, P=7, K=3, dtype=np.float64):
    tin = rng.normal(0, 0.5, (n, d)).astype(dtype)
    tout = rng.normal(0, 0.5, (n, d)).astype(dtype)
    ctx = rng.integers(0, n, P).astype(np.int32)
    ctx[1] = ctx[0]                                   # repeated context row
    ctr = rng.integers(0, n, P).astype(np.int32)
    neg = rng.integers(0, n, (P, K)).astype(np.int32)
    neg[2, 1] = ctr[2]                                # negative equal to the centre: dropped
    neg[3, 0] = ctx[3]                                # negative equal to the context: kept
    neg[4, K - 1] = neg[4, 0]                         # repeated negative in one pair
    return tin, tout, ctx, ctr, neg


def _dense(delta_rows, delta_vals, n, d):
    out = np.zeros((n, d))
    out[delta_rows] = delta_vals
    return out


def test_sgns_delta_matches_finite_differences(orc):
    rng = np.random.default_rng(0)
    tin, tout, ctx, ctr, neg = _rand_problem(rng)
    n, d = tin.shape
    lr = 0.3
    dl = orc.sgns_step(tin.copy(), tout.copy(), ctx, ctr, neg, lr, apply=False)
    din = _dense(dl.rows_in, dl.d_in, n, d)
    dout = _dense(dl.rows_out, dl.d_out, n, d)
    h = 1e-6
    for table, delta in ((tin, din), (tout, dout)):
        for v in range(n):
            for e in range(d):
                old = table[v, e]
                table[v, e] = old + h
                lp = orc.sgns_loss_f64(tin, tout, ctx, ctr, neg)
                table[v, e] = old - h
                lm = orc.sgns_loss_f64(tin, tout, ctx, ctr, neg)
                table[v, e] = old
                grad = (lp - lm) / (2 * h)
                assert abs(delta[v, e] - (-lr * grad)) <= 1e-6 * (abs(lr * grad) + 1e-3), (v, e)


def test_sgns_delta_matches_torch_autograd(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    tin, tout, ctx, ctr, neg = _rand_problem(rng, n=30, d=16, P=40, K=5)
    n, d = tin.shape
    lr = 0.05
    dl = orc.sgns_step(tin.copy(), tout.copy(), ctx, ctr, neg, lr, apply=False)
    a = torch.tensor(tin, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(tout, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(ctx, dtype=torch.long)
    t0 = torch.tensor(ctr, dtype=torch.long)
    nk = torch.tensor(neg, dtype=torch.long)
    pos = (a[c] * b[t0]).sum(-1)
    s_neg = (a[c][:, None, :] * b[nk]).sum(-1)
    keep = (nk != t0[:, None]).to(torch.float64)
    loss = -(torch.nn.functional.logsigmoid(pos).sum()
             + (keep * torch.nn.functional.logsigmoid(-s_neg)).sum())
    loss.backward()
    assert abs(loss.item() - dl.loss) <= 1e-12 * abs(dl.loss)
    np.testing.assert_allclose(_dense(dl.rows_in, dl.d_in, n, d), -lr * a.grad.numpy(),
                               rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(_dense(dl.rows_out, dl.d_out, n, d), -lr * b.grad.numpy(),
                               rtol=1e-12, atol=1e-15)


def test_sgns_minibatch_is_sum_of_single_pairs(orc):
    rng = np.random.default_rng(2)
    tin, tout, ctx, ctr, neg = _rand_problem(rng, n=12, d=8, P=9, K=4)
    n, d = tin.shape
    lr = 0.1
    full = orc.sgns_step(tin.copy(), tout.copy(), ctx, ctr, neg, lr, apply=False)
    acc_in = np.zeros((n, d))
    acc_out = np.zeros((n, d))
    loss = 0.0
    for p in range(len(ctx)):
        one = orc.sgns_step(tin.copy(), tout.copy(), ctx[p:p + 1], ctr[p:p + 1], neg[p:p + 1],
                            lr, apply=False)
        acc_in += _dense(one.rows_in, one.d_in, n, d)
        acc_out += _dense(one.rows_out, one.d_out, n, d)
        loss += one.loss
    np.testing.assert_allclose(_dense(full.rows_in, full.d_in, n, d), acc_in, rtol=1e-13,
                               atol=1e-16)
    np.testing.assert_allclose(_dense(full.rows_out, full.d_out, n, d), acc_out, rtol=1e-13,
                               atol=1e-16)
    assert abs(full.loss - loss) < 1e-12 * loss


def test_sgns_apply_adds_delta_in_fp32(orc):
    rng = np.random.default_rng(3)
    tin, tout, ctx, ctr, neg = _rand_problem(rng, n=10, d=8, P=6, K=2, dtype=np.float32)
    a, b = tin.copy(), tout.copy()
    dl = orc.sgns_step(a, b, ctx, ctr, neg, 0.2, apply=True)
    exp_in = tin.copy()
    exp_in[dl.rows_in] = (tin[dl.rows_in].astype(np.float64) + dl.d_in).astype(np.float32)
    exp_out = tout.copy()
    exp_out[dl.rows_out] = (tout[dl.rows_out].astype(np.float64) + dl.d_out).astype(np.float32)
    assert np.array_equal(a, exp_in) and np.array_equal(b, exp_out)


def test_sgns_loss_at_zero_out_table(orc):
    """out = 0 gives s = 0 for every term: loss = log 2 per kept term."""
    rng = np.random.default_rng(4)
    n, d, P, K = 20, 8, 30, 5
    tin = rng.normal(0, 1, (n, d)).astype(np.float32)
    tout = np.zeros((n, d), np.float32)
    ctx = rng.integers(0, n, P).astype(np.int32)
    ctr = rng.integers(0, n, P).astype(np.int32)
    neg = rng.integers(0, n, (P, K)).astype(np.int32)
    kept = P + int((neg != ctr[:, None]).sum())
    dl = orc.sgns_step(tin, tout, ctx, ctr, neg, 0.1, apply=False)
    assert abs(dl.loss - kept * math.log(2.0)) < 1e-12 * dl.loss
    # at s = 0: g0 = lr/2, g_k = -lr/2; the in-row delta is zero because out = 0
    assert np.all(dl.d_in == 0.0)


def test_log_sigmoid_stable(orc):
    for x in (-800.0, -40.0, -1.5, 0.0, 2.0, 40.0, 800.0):
        v = orc.lib().orc_log_sigmoid(x)
        exact = -math.log1p(math.exp(-x)) if x > -700 else x
        assert math.isfinite(v) and abs(v - exact) <= 1e-15 * max(1.0, abs(exact))


def _pairs_brute(walks, w, P, chunk):
    """All minibatches by the definition, in pure Python."""
    W, L = walks.shape
    mbs = []
    for c0 in range(0, W, chunk):
        seq = []
        for j in range(L):
            for s in range(2 * w):
                i = s - w if s < w else s - w + 1
                if not 0 <= j + i < L:
                    continue
                for col in range(c0, min(W, c0 + chunk)):
                    a, c = walks[col, j + i], walks[col, j]
                    if a >= 0 and c >= 0:
                        seq.append((a, c, col, j, s))
        mbs += [seq[k:k + P] for k in range(0, len(seq), P)]
    return mbs


@pytest.mark.parametrize("P,chunk", [(7, 1 << 20), (16, 5), (1, 3), (1000, 4)])
def test_pair_enumeration_brute_force(orc, P, chunk):
    g = synth.tiny_graph("star")                     # node 5 isolated: a one-node walk
    walks = orc.walks_uniform(g, np.arange(g.n), r=2, L=6, seed=9)
    w = 2
    ref = _pairs_brute(walks, w, P, chunk)
    B, tp = orc.count_minibatches(walks, w, P, chunk)
    assert B == len(ref) and tp == sum(len(m) for m in ref)
    for b, m in enumerate(ref):
        mb = orc.minibatch_pairs(walks, w, P, b, chunk)
        got = list(zip(mb.ctx, mb.ctr, mb.col, mb.j, mb.slot))
        assert [tuple(int(x) for x in t) for t in got] == [tuple(int(x) for x in t) for t in m]


def test_pair_count_closed_form(orc):
    """Full-length walks give W * sum_j #{i : 0 < |i| <= w, 0 <= j+i < L} pairs."""
    sp = synth.build_graph("sbm1k")
    walks = orc.walks_uniform(sp.train, np.arange(1000), r=10, L=40, seed=1)
    full = (walks >= 0).all(1).sum()
    per_walk = sum(min(5, j) + min(5, 39 - j) for j in range(40))
    assert per_walk == 370
    B, tp = orc.count_minibatches(walks, 5, 1024)
    assert tp == full * per_walk
    assert B == math.ceil(tp / 1024)


def test_negatives_do_not_depend_on_minibatch_size(orc):
    """Negatives are keyed by (walk, j, slot, k), not by a pair's minibatch."""
    g = synth.tiny_graph("k8")
    walks = orc.walks_uniform(g, np.arange(8), r=3, L=7, seed=4)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    got = {}
    for P in (5, 64):
        B, _ = orc.count_minibatches(walks, 3, P)
        for b in range(B):
            mb = orc.minibatch_pairs(walks, 3, P, b)
            neg = orc.draw_negatives(mb, 100, 5, 77, cdf)
            for k in range(len(mb.ctx)):
                key = (int(mb.col[k]), int(mb.j[k]), int(mb.slot[k]))
                if key in got:
                    assert np.array_equal(got[key], neg[k])
                got[key] = neg[k]


def test_inverse_cdf_boundaries(orc):
    counts = np.array([0, 3, 0, 1, 10, 0], np.uint64)
    cdf = orc.neg_cdf(counts)
    w = np.diff(cdf.astype(object))
    assert w[0] == 0 and w[2] == 0 and w[5] == 0
    assert cdf[-1] == sum(w)
    xs = np.array([0, 2 ** 64 - 1, 2 ** 63], np.uint64)
    d = orc.inverse_cdf(cdf, xs)
    assert d[0] == 1 and d[1] == 4
    # every threshold maps exactly: x just below / at the start of each bucket
    T = int(cdf[-1])
    for i in (1, 3, 4):
        lo = int(cdf[i])
        x = -(-(lo << 64) // T)               # smallest x with floor(x*T/2^64) >= lo
        if x < 2 ** 64:
            assert orc.inverse_cdf(cdf, np.array([x], np.uint64))[0] == i
        if x > 0 and lo > 0:
            assert orc.inverse_cdf(cdf, np.array([x - 1], np.uint64))[0] < i


def test_noise_distribution_chi_square(orc):
    """Draws follow count^0.75 (Pn(u) in Eq. (2)); zero counts are never drawn."""
    rng = np.random.default_rng(7)
    counts = rng.integers(0, 60, 40).astype(np.uint64)
    counts[[3, 9]] = 0
    counts[5] = 5000
    cdf = orc.neg_cdf(counts)
    xs = rng.integers(0, 2 ** 64, size=1_000_000, dtype=np.uint64)
    d = orc.inverse_cdf(cdf, xs)
    obs = np.bincount(d, minlength=40)
    assert obs[3] == 0 and obs[9] == 0
    p = counts.astype(np.float64) ** 0.75
    p /= p.sum()
    nz = counts > 0
    assert chisquare(obs[nz], p[nz] * obs.sum()).pvalue > 1e-3
    # weights are the FP64 value of c^0.75 at 2^-16 resolution
    w = orc.neg_weights(counts).astype(np.float64)
    np.testing.assert_allclose(w / 65536.0, counts.astype(np.float64) ** 0.75, rtol=1e-12,
                               atol=2 ** -16)


def test_init_tables(orc):
    tin, tout = orc.init_tables(3000, 64, seed=0)
    assert np.all(tout == 0)
    assert tin.min() >= -0.5 / 64 and tin.max() < 0.5 / 64
    # 24-bit grid: (k * 2^-24 - 0.5) / 64
    k = (tin.astype(np.float64) * 64 + 0.5) * 2 ** 24
    assert np.all(k == np.round(k))
    hist = np.histogram(tin.ravel(), bins=32, range=(-0.5 / 64, 0.5 / 64))[0]
    assert chisquare(hist).pvalue > 1e-3
    t2, _ = orc.init_tables(3000, 64, seed=0)
    assert np.array_equal(tin, t2)


def test_lr_schedule(orc):
    assert orc.lr_at(0, 10, 0.025, 1e-4) == np.float32(0.025)
    assert orc.lr_at(9, 10, 0.025, 1e-4) == np.float32(1e-4)
    assert orc.lr_at(0, 1, 0.025, 1e-4) == np.float32(0.025)


def test_sbm_epoch_learns(orc):
    """One epoch on the 1,000-node SBM lowers the loss of fixed minibatches and
    raises held-out AUC.

    The 0.70 floor is a sanity bound for this homophilous graph, not a number
    from the paper (the paper's AUCs are on datasets that are not available).
    """
    sp = synth.build_graph("sbm1k")
    g = sp.train
    walks = orc.walks_uniform(g, np.arange(g.n), r=10, L=40, seed=11)
    tin, tout = orc.init_tables(g.n, 64, 0)
    cdf = orc.neg_cdf(g.degrees().astype(np.uint64))
    auc0 = orc.link_auc(tin, sp)
    B, _ = orc.count_minibatches(walks, 5, 1024)
    probe = [orc.minibatch_pairs(walks, 5, 1024, b) for b in range(0, B, 97)]
    probe_neg = [orc.draw_negatives(mb, 0, 5, 3, cdf) for mb in probe]

    def probe_loss(a, b):
        return sum(orc.sgns_step(a, b, mb.ctx, mb.ctr, ng, 0.0, apply=False).loss
                   for mb, ng in zip(probe, probe_neg))

    before = probe_loss(tin, tout)
    orc.train_epoch(tin, tout, walks, window=5, K=5, lr0=0.025, lr_end=1e-4, P=1024, seed=3,
                    cdf=cdf)
    assert probe_loss(tin, tout) < before
    assert orc.link_auc(tin, sp) > max(0.70, auc0 + 0.1)


def _noise_case():
    rng = np.random.default_rng(17)
    counts = rng.integers(1, 80, 24).astype(np.uint64)
    counts[4] = 3000                                   # one heavy node
    p = counts.astype(np.float64) ** 0.75
    return counts, p / p.sum()


def _mass_groups(p, groups=4):
    """Nodes grouped into `groups` classes of roughly equal noise mass (for
    contingency tables with well-filled cells)."""
    order = np.argsort(-p)
    cls = np.zeros(p.shape[0], np.int64)
    acc, g = 0.0, 0
    for i in order:
        cls[i] = g
        acc += p[i]
        if acc >= (g + 1) / groups and g < groups - 1:
            g += 1
    return cls


def _draw_negatives_raw(orc, wid, j, slot, K, seed, cdf):
    n = cdf.shape[0] - 1
    out = np.zeros((wid.shape[0], K), np.int32)
    orc.lib().orc_draw_negatives(wid.shape[0], orc._ptr(np.ascontiguousarray(wid, np.int64)),
                                 orc._ptr(np.ascontiguousarray(j, np.int32)),
                                 orc._ptr(np.ascontiguousarray(slot, np.int32)), K, seed, n,
                                 orc._ptr(cdf), orc._ptr(out))
    return out


def test_pair_negatives_marginal_and_independent(orc):
    """Negatives of Eq. (2): each of a pair's K draws is an independent draw
    from Pn(u) ~ c^0.75.  Marginals by chi-square per slot k; independence by
    chi-square on the joint class counts of every (k, k') of a pair, of the
    same k across the two window slots of one (walk, j), and across walks at
    the same (j, slot).  A plausible wiring mistake (two k sharing words, the
    slot or the walk left out of the counter) makes a joint table diagonal."""
    from scipy.stats import chi2_contingency
    counts, p = _noise_case()
    cdf = orc.neg_cdf(counts)
    cls = _mass_groups(p)
    K = 6
    n_pairs = 200_000
    rng = np.random.default_rng(5)
    wid = rng.integers(0, 2 ** 40, n_pairs, dtype=np.int64)
    j = rng.integers(0, 80, n_pairs).astype(np.int32)
    slot = rng.integers(0, 19, n_pairs).astype(np.int32)
    neg = _draw_negatives_raw(orc, wid, j, slot, K, 123, cdf)
    for k in range(K):
        obs = np.bincount(neg[:, k], minlength=p.shape[0])
        assert chisquare(obs, p * n_pairs).pvalue > 1e-4, k
    pooled = np.bincount(neg.ravel(), minlength=p.shape[0])
    assert chisquare(pooled, p * neg.size).pvalue > 1e-4

    def independent(a, b, what):
        tab = np.zeros((4, 4))
        np.add.at(tab, (cls[a], cls[b]), 1)
        assert chi2_contingency(tab).pvalue > 1e-4, (what, tab)

    for k in range(K):
        for k2 in range(k + 1, K):
            independent(neg[:, k], neg[:, k2], ("k", k, k2))
    # the next window slot of the same (walk, j), and the next walk
    neg_s = _draw_negatives_raw(orc, wid, j, slot + 1, K, 123, cdf)
    neg_w = _draw_negatives_raw(orc, wid + 1, j, slot, K, 123, cdf)
    neg_j = _draw_negatives_raw(orc, wid, j + 1, slot, K, 123, cdf)
    for k in (0, 1, K - 1):
        independent(neg[:, k], neg_s[:, k], ("slot", k))
        independent(neg[:, k], neg_w[:, k], ("walk", k))
        independent(neg[:, k], neg_j[:, k], ("j", k))


def test_shared_negatives_marginal_and_independent(orc):
    """The shared-negative form's M draws per minibatch: marginally c^0.75,
    independent between neighbouring draws m, m+1 (which share one Philox
    call) and between minibatches."""
    from scipy.stats import chi2_contingency
    counts, p = _noise_case()
    cdf = orc.neg_cdf(counts)
    cls = _mass_groups(p)
    M = 1024
    draws = np.stack([orc.shared_negatives(b, 0, M, 31, cdf) for b in range(400)])
    obs = np.bincount(draws.ravel(), minlength=p.shape[0])
    assert chisquare(obs, p * draws.size).pvalue > 1e-4
    for what, a, b in (("m, m+1", draws[:, 0::2], draws[:, 1::2]),
                       ("m, m+2", draws[:, 0:-2:4], draws[:, 2::4]),
                       ("b, b+1", draws[:-1], draws[1:])):
        tab = np.zeros((4, 4))
        np.add.at(tab, (cls[a.ravel()], cls[b.ravel()]), 1)
        assert chi2_contingency(tab).pvalue > 1e-4, (what, tab)
    # another round gives other draws
    other = orc.shared_negatives(0, 1, M, 31, cdf)
    assert not np.array_equal(other, draws[0])
