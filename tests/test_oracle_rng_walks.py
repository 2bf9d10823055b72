"""Pins for the oracle's random numbers and walks (Sample in Algorithm 1).

The walks are pinned by what the method fixes independently of the oracle:
every transition is an edge; a uniform walk leaves v for each neighbour with
probability 1/deg(v) (DeepWalk, Section 2); a node2vec walk leaves v, having
come from t, for x with probability w(v,x) alpha(t,x) / sum_y w(v,y) alpha(t,y)
(return/in-out bias p, q); and the generator is Philox4x32-10, checked against
rocRAND's independent implementation.
"""
import os
import shutil
import subprocess
from collections import Counter, defaultdict

import numpy as np
import pytest
from scipy.stats import chisquare

import synth

PIN_SRC = os.path.join(os.path.dirname(__file__), "pins", "philox_rocrand.cpp")


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("pin") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe,
                           PIN_SRC], cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def test_philox_matches_rocrand(orc, rocrand_philox):
    rng = np.random.default_rng(5)
    N = 3000
    c = rng.integers(0, 2 ** 32, size=(N, 4), dtype=np.uint64)
    c[:, 1] %= 2 ** 30            # rocRAND's offset argument reaches counter word 1 < 2^30
    c[:7] = [[0, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 1 << 24], [0xFFFFFFFF, 0, 0, 0],
             [0, 0, 0xFFFFFFFF, 0xFFFFFFFF], [3, 1, 4, 1], [2 ** 30 - 1, 2 ** 30 - 1, 9, 9]]
    seeds = [int(s) for s in rng.integers(0, 2 ** 63, size=N, dtype=np.uint64)]
    seeds[0] = 0
    seeds[1] = 2 ** 64 - 1
    inp = "\n".join(f"{a} {b} {x} {d} {s}" for (a, b, x, d), s in zip(c.tolist(), seeds))
    out = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True,
                         check=True).stdout
    ref = np.array([list(map(int, ln.split())) for ln in out.strip().split("\n")], np.uint64)
    mine = np.array([orc.philox(cc.astype(np.uint32),
                                np.array([s & 0xFFFFFFFF, s >> 32], np.uint64).astype(np.uint32))
                     for cc, s in zip(c, seeds)], np.uint64)
    assert np.array_equal(ref, mine)


def test_philox_batch_equals_single(orc):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(50, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x1234_5678_9ABC_DEF0
    b = orc.philox_batch(ctr, seed)
    for i in range(50):
        assert np.array_equal(b[i], orc.philox(ctr[i], [seed & 0xFFFFFFFF, seed >> 32]))


def _edge_set(g):
    s = set()
    for v in range(g.n):
        for u in g.indices[g.indptr[v]:g.indptr[v + 1]]:
            s.add((v, int(u)))
    return s


@pytest.mark.parametrize("kind", ["path", "star", "house", "k8"])
def test_uniform_walks_are_edges(orc, kind):
    g = synth.tiny_graph(kind)
    edges = _edge_set(g)
    w = orc.walks_uniform(g, np.arange(g.n), r=7, L=9, seed=3, id_base=11)
    deg = g.degrees()
    for row, start in zip(w, np.tile(np.arange(g.n), 7)):
        assert row[0] == start
        if deg[start] == 0:                      # isolated start: one node, then padding
            assert (row[1:] == -1).all()
            continue
        assert (row >= 0).all()
        for a, b in zip(row[:-1], row[1:]):
            assert (int(a), int(b)) in edges


def test_uniform_walk_ids_and_determinism(orc):
    g = synth.tiny_graph("k8")
    a = orc.walks_uniform(g, np.arange(8), r=3, L=12, seed=5, id_base=0)
    b = orc.walks_uniform(g, np.arange(8), r=3, L=12, seed=5, id_base=0)
    assert np.array_equal(a, b)
    # walk number i of a call with id_base B is the walk with id B + i
    c = orc.walks_uniform(g, np.arange(8), r=3, L=12, seed=5, id_base=8)
    assert np.array_equal(a[8:], c[:16])
    d = orc.walks_uniform(g, np.arange(8), r=3, L=12, seed=6, id_base=0)
    assert not np.array_equal(a, d)


@pytest.mark.parametrize("kind", ["house", "k8", "star"])
def test_uniform_transition_chi_square(orc, kind):
    """Each transition out of v is uniform over N(v): P = 1/deg(v)."""
    g = synth.tiny_graph(kind)
    starts = np.arange(g.n)
    w = orc.walks_uniform(g, starts, r=40000, L=6, seed=17)
    a = w[:, :-1].ravel()
    b = w[:, 1:].ravel()
    ok = b >= 0
    a, b = a[ok], b[ok]
    for v in range(g.n):
        nb = g.indices[g.indptr[v]:g.indptr[v + 1]]
        if len(nb) < 2:
            continue
        sel = b[a == v]
        obs = np.array([(sel == u).sum() for u in nb])
        assert obs.sum() == sel.shape[0]          # no transition leaves N(v)
        exp = np.full(len(nb), sel.shape[0] / len(nb))
        assert chisquare(obs, exp).pvalue > 1e-3


def _weighted_tiny(seed=0):
    g = synth.tiny_graph("k8")
    e = []
    for v in range(g.n):
        for u in g.indices[g.indptr[v]:g.indptr[v + 1]]:
            if v < u:
                e.append((v, int(u)))
    e = np.array(e, np.int64)
    wts = synth.edge_weights(e.shape[0], seed)
    return synth.csr_from_edges(g.n, e, wts)


def _weight(g, a, b):
    lo, hi = g.indptr[a], g.indptr[a + 1]
    k = np.searchsorted(g.indices[lo:hi], b)
    return float(g.weights[lo + k])


@pytest.mark.parametrize("p,q", [(0.5, 2.0), (2.0, 0.5), (1.0, 1.0)])
def test_node2vec_transition_chi_square(orc, p, q):
    """Second-order transition t -> v -> x is proportional to w(v,x) alpha(t,x)."""
    g = _weighted_tiny()
    w, capped = orc.walks_node2vec(g, np.arange(g.n), r=12000, L=8, p=p, q=q, seed=23)
    assert capped == 0
    edges = _edge_set(g)
    cnt = defaultdict(Counter)
    first = defaultdict(Counter)
    for row in w:
        first[int(row[0])][int(row[1])] += 1
        for t, v, x in zip(row[:-2], row[1:-1], row[2:]):
            assert (int(v), int(x)) in edges
            cnt[(int(t), int(v))][int(x)] += 1
    nbrs = {v: [int(u) for u in g.indices[g.indptr[v]:g.indptr[v + 1]]] for v in range(g.n)}
    tested = 0
    for (t, v), c in cnt.items():
        xs = nbrs[v]
        if len(xs) < 2 or sum(c.values()) < 2000:
            continue
        alpha = [1 / p if x == t else (1.0 if x in nbrs[t] else 1 / q) for x in xs]
        wts = np.array([_weight(g, v, x) * a for x, a in zip(xs, alpha)])
        obs = np.array([c[x] for x in xs])
        exp = wts / wts.sum() * obs.sum()
        assert chisquare(obs, exp).pvalue > 1e-4, (t, v)
        tested += 1
    assert tested >= 10
    # first transition: proportional to w(v, x) alone
    for v, c in first.items():
        xs = nbrs[v]
        if len(xs) < 2:
            continue
        wts = np.array([_weight(g, v, x) for x in xs])
        obs = np.array([c[x] for x in xs])
        assert chisquare(obs, wts / wts.sum() * obs.sum()).pvalue > 1e-4


def test_node2vec_unweighted_p_q_one_is_uniform(orc):
    """With p = q = 1 and unit weights node2vec is the uniform walk's law."""
    g = synth.tiny_graph("house")
    w, capped = orc.walks_node2vec(g, np.arange(g.n), r=30000, L=4, p=1.0, q=1.0, seed=2)
    assert capped == 0
    a = w[:, 1:-1].ravel()
    b = w[:, 2:].ravel()
    for v in range(g.n):
        nb = g.indices[g.indptr[v]:g.indptr[v + 1]]
        sel = b[a == v]
        obs = np.array([(sel == u).sum() for u in nb])
        assert chisquare(obs, np.full(len(nb), sel.shape[0] / len(nb))).pvalue > 1e-3


def test_node2vec_isolated_and_cap(orc):
    g = synth.tiny_graph("star")            # node 5 is isolated
    w, _ = orc.walks_node2vec(g, np.array([5, 0]), r=2, L=5, p=0.5, q=2.0, seed=1)
    assert (w[0] == [5, -1, -1, -1, -1]).all()
    assert (w[1] >= 0).all()
    # with one attempt allowed every proposal is taken: identical to 'accept first proposal'
    w1, capped = orc.walks_node2vec(g, np.array([0, 1]), r=50, L=6, p=0.01, q=100.0, seed=1,
                                    max_attempts=1)
    assert capped > 0
    edges = _edge_set(g)
    for row in w1:
        for a, b in zip(row[:-1], row[1:]):
            assert (int(a), int(b)) in edges


def test_oracle_independent_of_thread_count():
    """The oracle's loops over independent items run under OpenMP; tables,
    walks, Psi and a training epoch are bit-identical with one thread and
    with several."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r'''
import sys, hashlib; sys.path.insert(0, %r)
import numpy as np, oracle, synth
g = synth.build_graph("sbm1k").train
tin, tout = oracle.init_tables(g.n, 64, 3)
w = oracle.walks_uniform(g, np.arange(g.n), 2, 20, 5)
gw = synth.csr_from_edges(1 << 10, synth.rmat_edges(10, 1 << 12, seed=41), weight_seed=42)
w2, c2 = oracle.walks_node2vec(gw, np.arange(gw.n), 2, 20, 0.5, 2.0, 5)
cdf = oracle.neg_cdf(g.degrees().astype(np.uint64))
r = oracle.train_epoch(tin, tout, w, window=3, K=5, lr0=0.025, lr_end=1e-4, P=1024, seed=9,
                       cdf=cdf, mb_end=60)
ps = oracle.psi(tin, g, np.arange(g.n), 10, 4, 0)
h = hashlib.sha256()
for a in (tin, tout, w, w2, ps, np.array([r.loss, c2])):
    h.update(np.ascontiguousarray(a).tobytes())
print(h.hexdigest())
''' % root
    out = []
    for threads in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        out.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                  text=True, check=True).stdout.strip())
    assert out[0] == out[1]
