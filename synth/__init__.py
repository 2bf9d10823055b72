"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only builds *inputs*: graphs, edge weights, link-prediction splits
and serving job mixes. It holds none of the embedding method's arithmetic (no
walks, no negative sampling, no SGNS, no feedback score), so both the CPU
oracle and the HIP path may use it without sharing any of the method's code.

Stand-ins for the paper's data:
  * the paper's real graphs (Flickr, YouTube, LiveJournal, ...) are not
    available, so a stochastic block model (small, homophilous) and R-MAT
    graphs (power-law, as used by the paper's own scalability study, Section
    6.3) stand in for them;
  * the link-prediction protocol of Section 6.4 (hide edges, score pairs by
    the inner product of embeddings, measure AUC) is kept, with a 10% holdout
    and one split per seed.

Every generator takes an explicit seed.  The R-MAT graphs, CSR assembly, edge
weights and link-prediction splits come from graphgen.cpp (C++ with OpenMP,
built in-tree by ``build()``), whose random numbers are counter based, so a
call returns the same arrays on every machine and for any thread count; the
SBM and the serving mix use numpy's PCG64.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

__all__ = [
    "Graph", "sbm_edges", "rmat_edges", "csr_from_edges", "edge_weights", "edge_weight_hash",
    "holdout_split", "LinkSplit", "build_graph", "tiny_graph", "job_mix",
    "CONFIGS",
]


@dataclasses.dataclass
class Graph:
    """Symmetric CSR graph (undirected, no self loops, no duplicate edges).

    indptr  int64[n+1], indices int32[nnz] sorted ascending within each row,
    weights float32[nnz] or None (mirrored: w(u,v) == w(v,u)).
    """
    n: int
    indptr: np.ndarray
    indices: np.ndarray
    weights: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.indptr)


@dataclasses.dataclass
class LinkSplit:
    """Link-prediction split: the training graph plus scored test pairs."""
    train: Graph
    test_pos: np.ndarray   # int64 [m, 2], held-out edges (u < v)
    test_neg: np.ndarray   # int64 [m, 2], node pairs with no edge in the full graph


def _canon(u: np.ndarray, v: np.ndarray):
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    keep = a != b
    return a[keep], b[keep]


def sbm_edges(n: int = 1000, blocks: int = 4, p_in: float = 0.035,
              p_out: float = 0.002, seed: int = 0) -> np.ndarray:
    """Undirected SBM edge list (u < v), equal contiguous blocks.

    Each unordered pair is an edge independently with probability p_in inside
    a block and p_out across blocks.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, k=1)
    bsz = n // blocks
    bi = np.minimum(iu // bsz, blocks - 1)
    bj = np.minimum(ju // bsz, blocks - 1)
    p = np.where(bi == bj, p_in, p_out)
    keep = rng.random(iu.shape[0]) < p
    return np.stack([iu[keep], ju[keep]], axis=1).astype(np.int64)


_LIB_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib")
_LIB = os.path.join(_LIB_DIR, "libgraphgen.so")
_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "graphgen.cpp")
_lib_handle = None


def build(force: bool = False) -> str:
    """Compile the graph-input library (g++, OpenMP) in-tree."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(_LIB_DIR, exist_ok=True)
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("g++ failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
        os.replace(tmp, _LIB)
    return _LIB


def _gg():
    global _lib_handle
    if _lib_handle is None:
        lib = ctypes.CDLL(build())
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, i64p, i64p]
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, i64p, i64p, i64p,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                               ctypes.c_uint64]
        lib.gg_csr.restype = ctypes.c_int
        lib.gg_holdout.argtypes = [ctypes.c_int64, ctypes.c_int64, i64p, i64p, ctypes.c_int64,
                                   ctypes.c_uint64, i64p, i64p, i64p]
        lib.gg_holdout.restype = ctypes.c_int
        lib.gg_edge_weight.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64]
        lib.gg_edge_weight.restype = ctypes.c_float
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def rmat_edges(scale: int, n_edges: int, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1, permute: bool = True) -> np.ndarray:
    """R-MAT edge list with ``n_edges`` distinct undirected edges (u < v),
    sorted by (u, v).

    Each candidate edge takes ``scale`` quadrant choices with probabilities
    (a, b, c, 1-a-b-c), each from a 16-bit uniform draw (the probabilities are
    rounded to multiples of 2^-16).  Self loops are dropped; candidates are
    made until the distinct edges number at least ``n_edges`` and the surplus
    is dropped uniformly at random.  A seeded random vertex permutation is
    applied at the end (the Graph500 convention), so that vertex id does not
    encode degree.  All draws are counter based (graphgen.cpp), so the graph
    depends on the arguments alone.
    """
    ta, tab, tabc = (int(round(x * 65536)) for x in (a, a + b, a + b + c))
    u = np.empty(n_edges, dtype=np.int64)
    v = np.empty(n_edges, dtype=np.int64)
    rc = _gg().gg_rmat(scale, n_edges, ta, tab, tabc, seed & (2**64 - 1), int(permute),
                       _ptr(u, ctypes.c_int64), _ptr(v, ctypes.c_int64))
    if rc != 0:
        raise ValueError("rmat_edges: scale %d with %d edges is out of range" % (scale, n_edges))
    return np.stack([u, v], axis=1)


def _splitmix64(z):
    z = z + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def edge_weight_hash(u: np.ndarray, v: np.ndarray, seed: int) -> np.ndarray:
    """Weight of undirected edge {u, v}, uniform on (0, 1] with 2^-24 spacing,
    as a function of the edge alone, so that both directions and every subset
    of the edges agree without an array riding along: ((h >> 40) + 1) 2^-24,
    h = word 0 of the SplitMix64 stream of the edge key (min << 32 | max), as
    graphgen.cpp computes it."""
    with np.errstate(over="ignore"):
        a = np.minimum(u, v).astype(np.uint64)
        b = np.maximum(u, v).astype(np.uint64)
        key = (a << np.uint64(32)) | b
        s = _splitmix64(np.uint64(seed & (2**64 - 1)) ^ np.uint64(0xD1B54A32D192ED03))
        h = _splitmix64(s ^ (key * np.uint64(16)))
    k = (h >> np.uint64(40)).astype(np.int64) + 1
    return (k.astype(np.float64) * 2.0 ** -24).astype(np.float32)


def edge_weights(n_edges: int, seed: int) -> np.ndarray:
    """One weight per undirected edge, uniform on (0, 1] with 24-bit spacing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(0, 1 << 24, size=n_edges, dtype=np.int64) + 1
    return (k.astype(np.float64) * 2.0 ** -24).astype(np.float32)


def csr_from_edges(n: int, edges: np.ndarray, weights: np.ndarray | None = None,
                   weight_seed: int | None = None) -> Graph:
    """Symmetric CSR from an undirected edge list (u != v, no repeated edge).

    Weights: ``weights`` aligned with ``edges`` (one per undirected edge), or
    ``weight_seed`` for the per-edge hash weights of ``edge_weight_hash`` (a
    function of the edge, so no array rides along with the sort), or neither
    for an unweighted graph.
    """
    m = edges.shape[0]
    if weights is None:
        u = np.ascontiguousarray(edges[:, 0], dtype=np.int64)
        v = np.ascontiguousarray(edges[:, 1], dtype=np.int64)
        indptr = np.empty(n + 1, dtype=np.int64)
        indices = np.empty(2 * m, dtype=np.int32)
        w = None if weight_seed is None else np.empty(2 * m, dtype=np.float32)
        rc = _gg().gg_csr(n, m, _ptr(u, ctypes.c_int64), _ptr(v, ctypes.c_int64),
                          _ptr(indptr, ctypes.c_int64), _ptr(indices, ctypes.c_int32),
                          None if w is None else _ptr(w, ctypes.c_float),
                          0 if weight_seed is None else weight_seed & (2**64 - 1))
        if rc != 0:
            raise ValueError("csr_from_edges: an edge is a self loop or leaves [0, n)")
        return Graph(n=n, indptr=indptr, indices=indices, weights=w)
    u = edges[:, 0].astype(np.int64)
    v = edges[:, 1].astype(np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.argsort(src * n + dst)
    src = src[order]
    dst = dst[order]
    w = np.concatenate([weights, weights])[order].astype(np.float32)
    counts = np.bincount(src, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return Graph(n=n, indptr=indptr, indices=dst.astype(np.int32), weights=w)


def holdout_split(n: int, edges: np.ndarray, frac: float = 0.1, seed: int = 7,
                  weights: np.ndarray | None = None,
                  weight_seed: int | None = None) -> LinkSplit:
    """Hide ``frac`` of the undirected edges (uniformly, without replacement)
    for link prediction.  Test negatives: as many distinct node pairs (u < v)
    as held-out edges, uniform over the pairs that are not edges of the *full*
    graph.  Draws are counter based (graphgen.cpp)."""
    m = edges.shape[0]
    n_test = int(round(frac * m))
    u = np.ascontiguousarray(edges[:, 0], dtype=np.int64)
    v = np.ascontiguousarray(edges[:, 1], dtype=np.int64)
    test_idx = np.empty(n_test, dtype=np.int64)
    nu = np.empty(n_test, dtype=np.int64)
    nv = np.empty(n_test, dtype=np.int64)
    rc = _gg().gg_holdout(n, m, _ptr(u, ctypes.c_int64), _ptr(v, ctypes.c_int64), n_test,
                          seed & (2**64 - 1), _ptr(test_idx, ctypes.c_int64),
                          _ptr(nu, ctypes.c_int64), _ptr(nv, ctypes.c_int64))
    if rc != 0:
        raise ValueError("holdout_split: %d test pairs do not fit a graph on %d nodes" % (n_test, n))
    train_mask = np.ones(m, dtype=bool)
    train_mask[test_idx] = False
    tw = None if weights is None else weights[train_mask]
    train = csr_from_edges(n, edges[train_mask], tw, weight_seed=weight_seed)
    return LinkSplit(train=train, test_pos=edges[test_idx].astype(np.int64),
                     test_neg=np.stack([nu, nv], axis=1))


def tiny_graph(kind: str = "path") -> Graph:
    """Small hand-made graphs for exact and chi-square tests."""
    if kind == "path":          # 0-1-2-3
        e = np.array([[0, 1], [1, 2], [2, 3]])
        n = 4
    elif kind == "star":        # hub 0 with 4 leaves, plus isolated node 5
        e = np.array([[0, 1], [0, 2], [0, 3], [0, 4]])
        n = 6
    elif kind == "house":       # 5-cycle with a chord (triangles + square)
        e = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [0, 4], [1, 4], [2, 4]])
        n = 5
    elif kind == "k8":          # a sparse 8-node graph with mixed degrees
        e = np.array([[0, 1], [0, 2], [0, 3], [1, 2], [2, 3], [3, 4], [4, 5],
                      [4, 6], [5, 6], [6, 7], [1, 7], [2, 5]])
        n = 8
    else:
        raise ValueError(kind)
    e = np.sort(e, axis=1).astype(np.int64)
    return csr_from_edges(n, e)


# Workload presets, in the order the configurations are listed for this method:
# a small homophilous graph sized for the CPU oracle, an R-MAT graph with the
# feedback loop, a larger R-MAT for the precision form, a weighted R-MAT for
# second-order walks, and a serving mix.
CONFIGS = {
    "sbm1k": dict(kind="sbm", n=1000, blocks=4, p_in=0.035, p_out=0.002,
                  seed=0, holdout=0.1, r=10, L=40, window=5, K=5, dim=64,
                  neg="degree", lr0=0.025, lr_end=1e-4, minibatch=1024),
    "rmat20": dict(kind="rmat", scale=20, edges=1 << 24, seed=1, holdout=0.1,
                   r=10, L=80, window=10, K=5, dim=128, neg="unigram",
                   lr0=0.025, lr_end=1e-4, minibatch=65536, mu=0.65, k_s=10,
                   r_max=4),
    "rmat22": dict(kind="rmat", scale=22, edges=1 << 26, seed=2, holdout=0.1,
                   r=10, L=80, window=10, K=5, dim=128, neg="unigram",
                   lr0=0.025, lr_end=1e-4, minibatch=1024, shared_neg=1024),
    "rmat23w": dict(kind="rmat", scale=23, edges=1 << 27, seed=3, holdout=0.1,
                    weighted=True, r=10, L=80, window=10, K=5, dim=128,
                    neg="unigram", p=0.5, q=2.0, lr0=0.025, lr_end=1e-4,
                    minibatch=1024),
}


def build_graph(name: str, scale_override: int | None = None,
                edges_override: int | None = None) -> LinkSplit:
    """Build a preset's graph and its link-prediction split."""
    cfg = CONFIGS[name]
    if cfg["kind"] == "sbm":
        n = cfg["n"]
        e = sbm_edges(n, cfg["blocks"], cfg["p_in"], cfg["p_out"], cfg["seed"])
        w = None
    else:
        scale = scale_override or cfg["scale"]
        ne = edges_override or cfg["edges"]
        n = 1 << scale
        e = rmat_edges(scale, ne, seed=cfg["seed"])
        ws = cfg["seed"] + 100 if cfg.get("weighted") else None
        return holdout_split(n, e, cfg["holdout"], seed=cfg["seed"] + 7, weight_seed=ws)
    return holdout_split(n, e, cfg["holdout"], seed=cfg["seed"] + 7)


def job_mix(n_jobs: int, seed: int = 4, n_min: int = 200, n_max: int = 200_000):
    """Serving job descriptors: graph kind, size, degree, dim, walk and window.

    Sizes are log-uniform in [n_min, n_max], average degree uniform in
    [8, 32], dim 64 or 128, walk length uniform in [40, 80], window in
    [5, 10]; every job asks for 10 walks per node and one epoch.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for j in range(n_jobs):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        jobs.append(dict(
            job=j, kind="sbm" if rng.random() < 0.5 else "rmat", n=n,
            avg_deg=int(rng.integers(8, 33)), dim=int(rng.choice([64, 128])),
            r=10, L=int(rng.integers(40, 81)), window=int(rng.integers(5, 11)),
            K=5, seed=j))
    return jobs


def job_graph(job: dict) -> Graph:
    """The graph a serving job embeds, sized by the job descriptor."""
    n = job["n"]
    m = max(1, n * job["avg_deg"] // 2)
    if job["kind"] == "sbm":
        blocks = 4
        bsz = n / blocks
        # p_in / p_out = 17.5 as in the small SBM preset, scaled to the degree
        pairs_in = blocks * bsz * (bsz - 1) / 2
        pairs_out = n * (n - 1) / 2 - pairs_in
        p_out = m / (17.5 * pairs_in + pairs_out)
        p_in = min(1.0, 17.5 * p_out)
        rng = np.random.Generator(np.random.PCG64(1000 + job["seed"]))
        blk = np.minimum((np.arange(n) // max(1, int(bsz))), blocks - 1)
        # sample an expected m edges without the O(n^2) pair list
        ein = rng.binomial(int(pairs_in), p_in)
        eout = rng.binomial(int(pairs_out), p_out)
        u = rng.integers(0, n, size=(ein + eout) * 3 + 64)
        v = rng.integers(0, n, size=u.shape[0])
        same = blk[u] == blk[v]
        cand_in = np.stack([u[same], v[same]], 1)[: ein * 2 + 32]
        cand_out = np.stack([u[~same], v[~same]], 1)[: eout * 2 + 32]
        e = np.concatenate([cand_in, cand_out])
        a, b = _canon(e[:, 0], e[:, 1])
        k = np.unique(a * n + b)
        rng.shuffle(k)
        k = k[:m]
        e = np.stack([k // n, k % n], axis=1)
    else:
        scale = max(1, math.ceil(math.log2(n)))
        cap = (1 << scale) * ((1 << scale) - 1) // 2
        e = rmat_edges(scale, min(m * 2, cap), seed=2000 + job["seed"], permute=False)
        e = e[(e[:, 0] < n) & (e[:, 1] < n)]
        if e.shape[0] > m:
            rng = np.random.Generator(np.random.PCG64(3000 + job["seed"]))
            e = e[np.sort(rng.choice(e.shape[0], m, replace=False))]
    return csr_from_edges(n, e.astype(np.int64))
