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

Every generator takes an explicit seed and uses numpy's PCG64, so the same
call returns the same arrays on every machine.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pandas as pd

__all__ = [
    "Graph", "sbm_edges", "rmat_edges", "csr_from_edges", "edge_weights",
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


def rmat_edges(scale: int, n_edges: int, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1, batch: int = 1 << 22,
               permute: bool = True) -> np.ndarray:
    """R-MAT edge list with ``n_edges`` unique undirected edges (u < v).

    Edges are drawn in batches by recursive quadrant choice with probabilities
    (a, b, c, 1-a-b-c); self loops and duplicates are dropped and the first
    ``n_edges`` unique edges in generation order are kept. A seeded random
    vertex permutation is applied at the end (the Graph500 convention) so
    that vertex id does not encode degree.
    """
    n = 1 << scale
    rng = np.random.Generator(np.random.PCG64(seed))
    ab = a + b
    abc = a + b + c
    keys_all = []
    have = 0
    uniq = None
    while True:
        src = np.zeros(batch, dtype=np.int64)
        dst = np.zeros(batch, dtype=np.int64)
        for lvl in range(scale):
            r = rng.random(batch, dtype=np.float32)
            bit = np.int64(1) << (scale - 1 - lvl)
            right = ((r >= a) & (r < ab)) | (r >= abc)
            down = r >= ab
            src |= np.where(down, bit, 0)
            dst |= np.where(right, bit, 0)
        u, v = _canon(src, dst)
        keys_all.append(u * n + v)
        have += u.shape[0]
        if have >= n_edges:
            # distinct keys in order of first appearance (a hash pass)
            keys = pd.unique(np.concatenate(keys_all))
            if keys.shape[0] >= n_edges:
                keys = keys[:n_edges]
                break
            keys_all = [keys]
    u = keys // n
    v = keys % n
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        u, v = perm[u], perm[v]
        u, v = np.minimum(u, v), np.maximum(u, v)
    return np.stack([u, v], axis=1)


def edge_weights(n_edges: int, seed: int) -> np.ndarray:
    """One weight per undirected edge, uniform on (0, 1] with 24-bit spacing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(0, 1 << 24, size=n_edges, dtype=np.int64) + 1
    return (k.astype(np.float64) * 2.0 ** -24).astype(np.float32)


def csr_from_edges(n: int, edges: np.ndarray,
                   weights: np.ndarray | None = None) -> Graph:
    """Symmetric CSR from an undirected edge list (u < v, unique)."""
    u = edges[:, 0].astype(np.int64)
    v = edges[:, 1].astype(np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = src * n + dst
    w = None
    if weights is None:
        key = np.sort(key)   # keys are distinct: no order among equals to keep
        src = key // n
        dst = key - src * n
    else:
        order = np.argsort(key)
        src = src[order]
        dst = dst[order]
        w = np.concatenate([weights, weights])[order].astype(np.float32)
    counts = np.bincount(src, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return Graph(n=n, indptr=indptr, indices=dst.astype(np.int32), weights=w)


def holdout_split(n: int, edges: np.ndarray, frac: float = 0.1, seed: int = 7,
                  weights: np.ndarray | None = None) -> LinkSplit:
    """Hide ``frac`` of the undirected edges (uniformly) for link prediction.

    Test negatives: as many node pairs (u < v) as held-out edges, uniform over
    pairs that are not edges of the *full* graph, drawn without replacement.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m = edges.shape[0]
    n_test = int(round(frac * m))
    perm = rng.permutation(m)
    test_idx = np.sort(perm[:n_test])
    train_mask = np.ones(m, dtype=bool)
    train_mask[test_idx] = False
    full_keys = edges[:, 0].astype(np.int64) * n + edges[:, 1]
    full_sorted = np.sort(full_keys)
    neg = np.zeros((0, 2), dtype=np.int64)
    seen = np.zeros(0, dtype=np.int64)
    while neg.shape[0] < n_test:
        want = (n_test - neg.shape[0]) * 2 + 16
        a = rng.integers(0, n, size=want, dtype=np.int64)
        b = rng.integers(0, n, size=want, dtype=np.int64)
        a, b = _canon(a, b)
        k = a * n + b
        pos = np.searchsorted(full_sorted, k)
        pos = np.minimum(pos, full_sorted.shape[0] - 1)
        ok = full_sorted[pos] != k
        k = k[ok]
        k = pd.unique(k)   # distinct, in order of first appearance
        k = k[~np.isin(k, seen)]
        seen = np.concatenate([seen, k])
        take = k[: n_test - neg.shape[0]]
        neg = np.concatenate([neg, np.stack([take // n, take % n], axis=1)])
    tw = None if weights is None else weights[train_mask]
    train = csr_from_edges(n, edges[train_mask], tw)
    return LinkSplit(train=train, test_pos=edges[test_idx].astype(np.int64),
                     test_neg=neg.astype(np.int64))


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
        w = edge_weights(e.shape[0], cfg["seed"] + 100) if cfg.get("weighted") else None
    return holdout_split(n, e, cfg["holdout"], seed=cfg["seed"] + 7, weights=w)


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
        e = rmat_edges(scale, m * 2, seed=2000 + job["seed"], batch=max(1024, m * 4),
                       permute=False)
        e = e[(e[:, 0] < n) & (e[:, 1] < n)][:m]
    return csr_from_edges(n, e.astype(np.int64))
