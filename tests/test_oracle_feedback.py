"""Pins for the oracle's feedback step (Eq. (4), Eq. (5)), the round loop of
Algorithm 1, the link-prediction AUC and the shared-negative (BF16) form.
"""
import math
from collections import Counter

import numpy as np
import pytest
from scipy.stats import chisquare

import synth


def _star_tables(d=8, mode="same"):
    g = synth.tiny_graph("star")          # hub 0, leaves 1..4, isolated 5
    rng = np.random.default_rng(0)
    base = rng.normal(0, 1, d).astype(np.float32)
    tin = np.zeros((g.n, d), np.float32)
    tin[0] = base
    for v in range(1, 5):
        if mode == "same":
            tin[v] = base * (v + 1)                         # parallel, any length
        elif mode == "anti":
            tin[v] = -base * v
        elif mode == "orth":
            x = rng.normal(0, 1, d)
            x -= x @ base.astype(np.float64) / (base.astype(np.float64) @ base) * base
            tin[v] = x.astype(np.float32)
    tin[5] = rng.normal(0, 1, d)
    return g, tin


@pytest.mark.parametrize("mode,expect", [("same", 1.0), ("anti", -1.0), ("orth", 0.0)])
def test_psi_closed_forms(orc, mode, expect):
    g, tin = _star_tables(mode=mode)
    ps = orc.psi(tin, g, np.array([0, 1, 2]), k_s=10, seed=1, rnd=0)
    assert abs(ps[0] - expect) < 1e-6
    # a leaf's only neighbour is the hub
    if mode != "orth":
        assert abs(ps[1] - expect) < 1e-6


def test_psi_isolated_is_nan_and_inactive(orc):
    g, tin = _star_tables()
    ps = orc.psi(tin, g, np.array([5]), k_s=10, seed=1, rnd=0)
    assert math.isnan(ps[0])
    assert orc.next_active(np.array([5], np.int32), ps, 2.0).shape[0] == 0


def test_psi_full_neighbourhood_brute_force(orc):
    """k_s >= deg(v): Psi is the exact mean cosine over all neighbours."""
    sp = synth.build_graph("sbm1k")
    g = sp.train
    rng = np.random.default_rng(3)
    tin = rng.normal(0, 1, (g.n, 16)).astype(np.float32)
    nodes = np.arange(0, g.n, 7, dtype=np.int32)
    ps = orc.psi(tin, g, nodes, k_s=1000, seed=0, rnd=0)
    e = tin.astype(np.float64)
    for v, p in zip(nodes, ps):
        nb = g.indices[g.indptr[v]:g.indptr[v + 1]]
        if len(nb) == 0:
            assert math.isnan(p)
            continue
        cos = (e[nb] @ e[v]) / (np.linalg.norm(e[nb], axis=1) * np.linalg.norm(e[v]))
        assert abs(p - cos.mean()) < 1e-13


def test_psi_zero_vector_gives_zero_cosine(orc):
    g, tin = _star_tables()
    tin[2] = 0.0
    ps = orc.psi(tin, g, np.array([2]), k_s=10, seed=0, rnd=0)
    assert ps[0] == 0.0


def test_floyd_subset_is_uniform(orc):
    """Floyd's algorithm: k distinct positions, each included with probability k/deg."""
    deg, k = 13, 4
    # a star whose hub has 13 leaves
    e = np.array([[0, i] for i in range(1, deg + 1)])
    g = synth.csr_from_edges(deg + 1, e)
    incl = Counter()
    R = 20000
    for rnd in range(R):
        s = orc.neighbour_subset(g, 0, k, seed=5, rnd=rnd)
        assert len(s) == k and len(set(s.tolist())) == k
        assert s.min() >= 0 and s.max() < deg
        incl.update(s.tolist())
    obs = np.array([incl[i] for i in range(deg)])
    assert chisquare(obs, np.full(deg, R * k / deg)).pvalue > 1e-3
    # small-degree nodes take the whole neighbourhood in CSR order
    assert orc.neighbour_subset(g, 3, 10, 5, 0).tolist() == [0]


def test_next_active_strict(orc):
    nodes = np.array([1, 2, 3, 4, 5], np.int32)
    ps = np.array([0.64, 0.65, 0.66, float("nan"), -1.0])
    assert orc.next_active(nodes, ps, 0.65).tolist() == [1, 5]


def _run_small(orc, mu, r_max=3, mode="monotone"):
    sp = synth.build_graph("sbm1k")
    return orc.run(sp.train, d=16, r=2, L=10, window=3, K=3, lr0=0.025, lr_end=1e-4, P=512,
                   mu=mu, k_s=10, r_max=r_max, seed_walk=1, seed_model=2, seed_train=3,
                   seed_psi=4, neg="degree", mode=mode)


def test_algorithm1_monotone_shrinks(orc):
    tin, tout, stats = _run_small(orc, mu=0.05, r_max=4)
    act = [s.active for s in stats]
    assert act[0] == 1000
    assert all(a >= b for a, b in zip(act, act[1:]))
    for s in stats:
        assert s.walks == 2 * s.active


def test_algorithm1_mu_above_one_is_without_feedback(orc):
    """mu > 1 keeps every node with neighbours: the w/o-FeeST setting."""
    sp = synth.build_graph("sbm1k")
    non_isolated = int((sp.train.degrees() > 0).sum())
    _, _, stats = _run_small(orc, mu=1.5, r_max=3)
    assert [s.active for s in stats] == [1000, non_isolated, non_isolated]


def test_algorithm1_mu_minus_one_stops_after_round_one(orc):
    _, _, stats = _run_small(orc, mu=-1.0, r_max=5)
    assert len(stats) == 1


def test_algorithm1_recompute_mode_can_reactivate(orc):
    _, _, mono = _run_small(orc, mu=0.05, r_max=3)
    _, _, rec = _run_small(orc, mu=0.05, r_max=3, mode="recompute")
    assert rec[0].active == mono[0].active
    assert all(r.active >= m.active for r, m in zip(rec, mono))


def test_auc_matches_sklearn_and_brute_force(orc):
    from sklearn.metrics import roc_auc_score
    rng = np.random.default_rng(0)
    pos = np.round(rng.normal(1, 1, 300), 1)          # rounding makes ties
    neg = np.round(rng.normal(0, 1, 250), 1)
    a = orc.auc(pos, neg)
    y = np.r_[np.ones(300), np.zeros(250)]
    assert abs(a - roc_auc_score(y, np.r_[pos, neg])) < 1e-12
    brute = ((pos[:, None] > neg[None, :]).sum() + 0.5 * (pos[:, None] == neg[None, :]).sum())
    assert abs(a - brute / (300 * 250)) < 1e-12


def test_bf16_round_matches_torch(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.r_[rng.normal(0, 1, 2000), rng.normal(0, 1e-30, 100), [0.0, -0.0, 1.0,
              1.00390625, 1.01171875, 65504.0, 3.4e38, -3.4e38]].astype(np.float32)
    # values exactly halfway between bf16 neighbours (ties to even)
    half = (np.arange(200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.r_[x, half, -half]
    got = orc.bf16_round(x)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_shared_negative_form_equals_per_pair_when_m_equals_k(orc):
    """M = K shared negatives with weight K/M = 1 is Eq. (2) with those K
    negatives given to every pair."""
    rng = np.random.default_rng(5)
    n, d, P, K = 25, 8, 12, 4
    tin = rng.normal(0, 0.5, (n, d)).astype(np.float32)
    tout = rng.normal(0, 0.5, (n, d)).astype(np.float32)
    ctx = rng.integers(0, n, P).astype(np.int32)
    ctr = rng.integers(0, n, P).astype(np.int32)
    neg = rng.integers(0, n, K).astype(np.int32)
    ctr[3] = neg[1]                                  # masked term
    lr = 0.1
    dctx, dneg, dctr, loss = orc.shared_neg_step(tin, tout, ctx, ctr, neg, K, lr, bf16=False)
    ref = orc.sgns_step(tin.copy(), tout.copy(), ctx, ctr, np.tile(neg, (P, 1)), lr,
                        apply=False)
    din = np.zeros((n, d))
    np.add.at(din, ctx, dctx)
    dout = np.zeros((n, d))
    np.add.at(dout, neg, dneg)
    np.add.at(dout, ctr, dctr)
    rin = np.zeros((n, d))
    rin[ref.rows_in] = ref.d_in
    rout = np.zeros((n, d))
    rout[ref.rows_out] = ref.d_out
    np.testing.assert_allclose(din, rin, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(dout, rout, rtol=1e-12, atol=1e-15)
    assert abs(loss - ref.loss) < 1e-12 * ref.loss


def test_shared_negative_form_autograd(orc):
    """General M: deltas are -lr times the gradient of the weighted loss."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    n, d, P, M, K = 40, 16, 20, 32, 5
    tin = rng.normal(0, 0.5, (n, d)).astype(np.float32)
    tout = rng.normal(0, 0.5, (n, d)).astype(np.float32)
    ctx = rng.integers(0, n, P).astype(np.int32)
    ctr = rng.integers(0, n, P).astype(np.int32)
    neg = rng.integers(0, n, M).astype(np.int32)
    ctr[0] = neg[0]
    lr = 0.07
    dctx, dneg, dctr, loss = orc.shared_neg_step(tin, tout, ctx, ctr, neg, K, lr, bf16=False)
    C = torch.tensor(tin[ctx], dtype=torch.float64, requires_grad=True)
    O = torch.tensor(tout[ctr], dtype=torch.float64, requires_grad=True)
    N = torch.tensor(tout[neg], dtype=torch.float64, requires_grad=True)
    mask = torch.tensor((neg[None, :] != ctr[:, None]).astype(np.float64))
    S = C @ N.T
    F = torch.nn.functional
    L = -(F.logsigmoid((C * O).sum(1)).sum() + (K / M) * (mask * F.logsigmoid(-S)).sum())
    L.backward()
    assert abs(L.item() - loss) < 1e-12 * abs(loss)
    np.testing.assert_allclose(dctx, -lr * C.grad.numpy(), rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(dneg, -lr * N.grad.numpy(), rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(dctr, -lr * O.grad.numpy(), rtol=1e-11, atol=1e-15)


def test_shared_negative_bf16_mode_rounds_inputs(orc):
    """bf16 mode equals the FP64 mode run on bf16-rounded tables, up to the
    rounding of the coefficients G, which moves deltas by at most 2^-8 relative."""
    rng = np.random.default_rng(8)
    n, d, P, M, K = 30, 16, 10, 16, 5
    tin = rng.normal(0, 0.5, (n, d)).astype(np.float32)
    tout = rng.normal(0, 0.5, (n, d)).astype(np.float32)
    ctx = rng.integers(0, n, P).astype(np.int32)
    ctr = rng.integers(0, n, P).astype(np.int32)
    neg = rng.integers(0, n, M).astype(np.int32)
    a = orc.shared_neg_step(tin, tout, ctx, ctr, neg, K, 0.05, bf16=True)
    b = orc.shared_neg_step(orc.bf16_round(tin), orc.bf16_round(tout), ctx, ctr, neg, K, 0.05,
                            bf16=False)
    np.testing.assert_allclose(a[2], b[2], rtol=1e-15)          # positive term: exact
    assert abs(a[3] - b[3]) < 1e-12 * abs(b[3])                # loss uses unrounded G
    for x, y in ((a[0], b[0]), (a[1], b[1])):
        assert np.abs(x - y).max() <= 2 ** -8 * np.abs(y).max() + 1e-12


def test_shared_negative_draws(orc):
    rng = np.random.default_rng(0)
    counts = rng.integers(1, 50, 64).astype(np.uint64)
    cdf = orc.neg_cdf(counts)
    a = orc.shared_negatives(3, 0, 1024, 9, cdf)
    b = orc.shared_negatives(3, 0, 1024, 9, cdf)
    c = orc.shared_negatives(4, 0, 1024, 9, cdf)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0 and a.max() < 64
