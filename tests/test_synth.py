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


def test_edge_weight_hash_matches_library():
    """The numpy and C++ forms of the per-edge hash weight agree, and a weight
    does not depend on the direction of the edge."""
    rng = np.random.default_rng(0)
    u = rng.integers(0, 1 << 23, 2000)
    v = rng.integers(0, 1 << 23, 2000)
    w = synth.edge_weight_hash(u, v, 103)
    lib = synth._gg()
    assert all(lib.gg_edge_weight(int(a), int(b), 103) == x for a, b, x in zip(u, v, w))
    assert np.array_equal(w, synth.edge_weight_hash(v, u, 103))
    assert w.min() > 0 and w.max() <= 1


def test_rmat_independent_of_thread_count():
    """Counter-based draws: one thread and all threads give the same graph."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); import synth, hashlib; "
            "sp = synth.holdout_split(1 << 14, synth.rmat_edges(14, 1 << 17, seed=9), 0.1, seed=3, "
            "weight_seed=4); g = sp.train; "
            "print(hashlib.sha256(g.indptr.tobytes() + g.indices.tobytes() + g.weights.tobytes() "
            "+ sp.test_pos.tobytes() + sp.test_neg.tobytes()).hexdigest())"
            % __import__("os").path.dirname(__import__("os").path.dirname(__file__)))
    out = []
    for threads in ("1", "8"):
        env = dict(__import__("os").environ, OMP_NUM_THREADS=threads)
        out.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                  text=True, check=True).stdout.strip())
    assert out[0] == out[1]


def test_holdout_weighted_split_keeps_mirrored_weights():
    sp = synth.holdout_split(1 << 12, synth.rmat_edges(12, 20000, seed=5), 0.1, seed=2,
                             weight_seed=11)
    g = sp.train
    _check_csr(g)
    src = np.repeat(np.arange(g.n), np.diff(g.indptr))
    assert np.array_equal(g.weights, synth.edge_weight_hash(src, g.indices.astype(np.int64), 11))
    assert sp.test_pos.shape == sp.test_neg.shape == (2000, 2)
