"""Checks of the seeded input generators (they hold none of the method)."""
import numpy as np

import synth


def _check_csr(g):
    assert g.indptr[0] == 0 and g.indptr[-1] == g.nnz
    assert np.all(np.diff(g.indptr) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(g.indptr))
    dst = g.indices.astype(np.int64)
    assert np.all(src != dst)                                    # no self loops
    key = src * g.n + dst
    assert np.all(np.diff(key) > 0)                              # sorted rows, no duplicates
    rev = np.sort(dst * g.n + src)
    assert np.array_equal(rev, key)                              # symmetric
    if g.weights is not None:
        order = np.argsort(dst * g.n + src)
        assert np.array_equal(g.weights, g.weights[order][np.argsort(np.argsort(key))])


def test_sbm_edge_count_and_csr():
    e = synth.sbm_edges(1000, 4, 0.035, 0.002, seed=0)
    # E[edges] = 4 * C(250,2) * 0.035 + (C(1000,2) - 4 C(250,2)) * 0.002
    pin = 4 * 250 * 249 / 2
    pout = 1000 * 999 / 2 - pin
    mean = pin * 0.035 + pout * 0.002
    var = pin * 0.035 * 0.965 + pout * 0.002 * 0.998
    assert abs(e.shape[0] - mean) < 4 * np.sqrt(var)
    assert abs(mean - 5107.5) < 1e-9
    g = synth.csr_from_edges(1000, e)
    _check_csr(g)
    blocks = np.arange(1000) // 250
    same = blocks[e[:, 0]] == blocks[e[:, 1]]
    assert same.mean() > 0.7                                     # homophilous


def test_rmat_unique_and_symmetric():
    e = synth.rmat_edges(12, 30000, seed=3)
    assert e.shape[0] == 30000
    assert np.all(e[:, 0] < e[:, 1])
    assert np.unique(e[:, 0] * 4096 + e[:, 1]).shape[0] == 30000
    g = synth.csr_from_edges(4096, e, synth.edge_weights(30000, 1))
    _check_csr(g)
    deg = g.degrees()
    assert deg.max() > 20 * deg.mean()                           # power-law hubs
    w = g.weights
    assert w.min() > 0 and w.max() <= 1


def test_holdout_split():
    e = synth.sbm_edges(1000, seed=0)
    sp = synth.holdout_split(1000, e, 0.1, seed=7)
    m = e.shape[0]
    assert sp.test_pos.shape[0] == round(0.1 * m) == sp.test_neg.shape[0]
    full = set(map(tuple, e.tolist()))
    assert all(tuple(p) in full for p in sp.test_pos.tolist())
    assert not any(tuple(p) in full for p in sp.test_neg.tolist())
    assert len(set(map(tuple, sp.test_neg.tolist()))) == sp.test_neg.shape[0]
    assert sp.train.nnz == 2 * (m - sp.test_pos.shape[0])
    _check_csr(sp.train)


def test_job_mix_ranges():
    jobs = synth.job_mix(500, seed=4)
    n = np.array([j["n"] for j in jobs])
    assert n.min() >= 200 and n.max() <= 200_000
    assert 3000 < np.median(n) < 12000                           # log-uniform median ~ 6,325
    assert set(j["dim"] for j in jobs) == {64, 128}
    g = synth.job_graph(jobs[0])
    _check_csr(g)
