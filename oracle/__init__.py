"""CPU oracle for the FeLoG hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2606_22180_amd``) and never imports it; the product path never
imports this package.

The heavy loops are plain C in ``felog_oracle.c`` (built with gcc, no fast
math, no FP contraction).  This module adds the glue that is clearer in
Python: the epoch loop with its learning-rate schedule, the noise
distribution, the round loop of Algorithm 1 and the link-prediction AUC.

Paper passages (FeLoG, arxiv 2606.22180):
  * Sample(v, theta) -> walks: Section 2 ("Sampling process") and Section 5.1
    ("Implementation"); uniform and node2vec walks.
  * Train(walks, model) -> embeddings: Eq. (1), Eq. (2) (skip-gram with
    negative sampling, K negatives from Pn(u), sigma(x) = 1/(1+exp(-x))).
  * Feedback: Eq. (4) (Psi, neighbourhood cosine consistency on a subsampled
    neighbourhood), Eq. (5) (next active set = nodes with Psi < mu).
  * Algorithm 1: sample from the active set, train, score, shrink, until the
    active set is empty.
  * Link prediction (Section 6.4): score a node pair by phi(u) . phi(v), AUC.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "felog_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

TAG_WALK, TAG_N2V, TAG_NEG, TAG_INIT, TAG_PSI, TAG_SHNEG = 1, 2, 3, 4, 5, 6
DEFAULT_CHUNK = 1 << 20
N2V_MAX_ATTEMPTS = 1 << 16


def build(force: bool = False) -> str:
    """Compile the oracle's C file with gcc (plain IEEE arithmetic)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-fno-fast-math",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int
_dbl = ctypes.c_double
_flt = ctypes.c_float
_p = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        sig = {
            "orc_set_threads": (None, [_int]),
            "orc_max_threads": (_int, []),
            "orc_philox": (None, [_p, _p, _p]),
            "orc_philox_batch": (None, [_i64, _p, _u64, _p]),
            "orc_init_tables": (None, [_i64, _int, _u64, _p, _p]),
            "orc_neg_weights": (None, [_i64, _p, _p]),
            "orc_cdf": (None, [_i64, _p, _p]),
            "orc_inverse_cdf": (_i32, [_i64, _p, _u64]),
            "orc_draw_batch": (None, [_i64, _p, _i64, _p, _p]),
            "orc_walks_uniform": (None, [_i64, _p, _p, _p, _i64, _int, _int, _u64, _i64, _p]),
            "orc_walks_node2vec": (_i64, [_i64, _p, _p, _p, _p, _i64, _int, _int, _flt, _flt,
                                          _int, _u64, _i64, _p]),
            "orc_count_minibatches": (_i64, [_p, _i64, _int, _int, _i64, _i64, _p]),
            "orc_minibatch_pairs": (_i64, [_p, _i64, _int, _int, _i64, _i64, _i64,
                                           _p, _p, _p, _p, _p]),
            "orc_slice_counts": (None, [_p, _i64, _i64, _int, _int, _p]),
            "orc_chunk_pairs_range": (_i64, [_p, _i64, _i64, _int, _int, _p, _i64, _i64,
                                             _p, _p, _p, _p, _p]),
            "orc_draw_negatives": (None, [_i64, _p, _p, _p, _int, _u64, _i64, _p, _p]),
            "orc_log_sigmoid": (_dbl, [_dbl]),
            "orc_sigmoid": (_dbl, [_dbl]),
            "orc_sgns_step_f32": (_dbl, [_p, _p, _i64, _int, _i64, _p, _p, _p, _int, _dbl, _int,
                                         _p, _p, _p, _p, _p, _p]),
            "orc_sgns_step_f64": (_dbl, [_p, _p, _i64, _int, _i64, _p, _p, _p, _int, _dbl, _int,
                                         _p, _p, _p, _p, _p, _p]),
            "orc_sgns_loss_f64": (_dbl, [_p, _p, _int, _i64, _p, _p, _p, _int]),
            "orc_neighbour_subset": (_int, [_p, _i32, _int, _u64, _u32, _p]),
            "orc_psi": (None, [_p, _int, _p, _p, _p, _i64, _int, _u64, _u32, _p]),
            "orc_bf16_round": (_flt, [_flt]),
            "orc_shared_neg_draw": (None, [_i64, _u32, _int, _u64, _i64, _p, _p]),
            "orc_shared_neg_step": (_dbl, [_p, _p, _int, _int, _int, _int, _p, _p, _p, _dbl,
                                           _int, _p, _p, _p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous"
    return a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# Random numbers: Philox4x32-10 (Salmon et al., SC'11)
# --------------------------------------------------------------------------
def set_threads(k: int) -> None:
    """Threads of the oracle's OpenMP loops (independent items only)."""
    lib().orc_set_threads(int(k))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def philox(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_batch(ctrs: np.ndarray, seed: int) -> np.ndarray:
    c = _c(ctrs, np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    lib().orc_philox_batch(c.shape[0], _ptr(c), seed, _ptr(out))
    return out


# --------------------------------------------------------------------------
# Tables and noise distribution
# --------------------------------------------------------------------------
def init_tables(n: int, d: int, seed: int):
    """in ~ U(-0.5/d, 0.5/d) (24-bit uniform), out = 0; both FP32 [n, d]."""
    tin = np.zeros((n, d), np.float32)
    tout = np.zeros((n, d), np.float32)
    lib().orc_init_tables(n, d, seed, _ptr(tin), _ptr(tout))
    return tin, tout


def neg_weights(counts: np.ndarray) -> np.ndarray:
    c = _c(counts, np.uint64)
    w = np.zeros_like(c)
    lib().orc_neg_weights(c.shape[0], _ptr(c), _ptr(w))
    return w


def neg_cdf(counts: np.ndarray) -> np.ndarray:
    """Integer CDF of the noise distribution Pn(u) ~ counts^0.75."""
    w = neg_weights(counts)
    cdf = np.zeros(w.shape[0] + 1, np.uint64)
    lib().orc_cdf(w.shape[0], _ptr(w), _ptr(cdf))
    return cdf


def inverse_cdf(cdf: np.ndarray, xs: np.ndarray) -> np.ndarray:
    x = _c(xs, np.uint64)
    out = np.zeros(x.shape[0], np.int32)
    lib().orc_draw_batch(cdf.shape[0] - 1, _ptr(cdf), x.shape[0], _ptr(x), _ptr(out))
    return out


def corpus_counts(walks: np.ndarray, n: int) -> np.ndarray:
    """Occurrences of every node in a walk corpus (the unigram counts)."""
    w = walks[walks >= 0]
    return np.bincount(w, minlength=n).astype(np.uint64)


# --------------------------------------------------------------------------
# Walks (Sample)
# --------------------------------------------------------------------------
def walks_uniform(g, starts, r: int, L: int, seed: int, id_base: int = 0) -> np.ndarray:
    s = _c(starts, np.int32)
    out = np.zeros((s.shape[0] * r, L), np.int32)
    lib().orc_walks_uniform(g.n, _ptr(_c(g.indptr, np.int64)), _ptr(_c(g.indices, np.int32)),
                            _ptr(s), s.shape[0], r, L, seed, id_base, _ptr(out))
    return out


def walks_node2vec(g, starts, r: int, L: int, p: float, q: float, seed: int,
                   id_base: int = 0, max_attempts: int = N2V_MAX_ATTEMPTS):
    s = _c(starts, np.int32)
    out = np.zeros((s.shape[0] * r, L), np.int32)
    w = None if g.weights is None else _c(g.weights, np.float32)
    capped = lib().orc_walks_node2vec(g.n, _ptr(_c(g.indptr, np.int64)),
                                      _ptr(_c(g.indices, np.int32)), _ptr(w), _ptr(s),
                                      s.shape[0], r, L, p, q, max_attempts, seed, id_base,
                                      _ptr(out))
    return out, int(capped)


# --------------------------------------------------------------------------
# Skip-gram with negative sampling (Train)
# --------------------------------------------------------------------------
def count_minibatches(walks: np.ndarray, window: int, P: int, chunk: int = DEFAULT_CHUNK):
    w = _c(walks, np.int32)
    tp = np.zeros(1, np.int64)
    B = lib().orc_count_minibatches(_ptr(w), w.shape[0], w.shape[1], window, P, chunk, _ptr(tp))
    return int(B), int(tp[0])


@dataclasses.dataclass
class Minibatch:
    ctx: np.ndarray
    ctr: np.ndarray
    col: np.ndarray
    j: np.ndarray
    slot: np.ndarray


def minibatch_pairs(walks: np.ndarray, window: int, P: int, b: int,
                    chunk: int = DEFAULT_CHUNK) -> Minibatch:
    w = _c(walks, np.int32)
    ctx = np.zeros(P, np.int32)
    ctr = np.zeros(P, np.int32)
    col = np.zeros(P, np.int64)
    j = np.zeros(P, np.int32)
    slot = np.zeros(P, np.int32)
    k = lib().orc_minibatch_pairs(_ptr(w), w.shape[0], w.shape[1], window, P, chunk, b,
                                  _ptr(ctx), _ptr(ctr), _ptr(col), _ptr(j), _ptr(slot))
    return Minibatch(ctx[:k].copy(), ctr[:k].copy(), col[:k].copy(), j[:k].copy(),
                     slot[:k].copy())


def draw_negatives(mb: Minibatch, id_base: int, K: int, seed: int, cdf: np.ndarray):
    wid = _c(mb.col + id_base, np.int64)
    neg = np.zeros((mb.ctx.shape[0], K), np.int32)
    lib().orc_draw_negatives(mb.ctx.shape[0], _ptr(wid), _ptr(_c(mb.j, np.int32)),
                             _ptr(_c(mb.slot, np.int32)), K, seed,
                             cdf.shape[0] - 1, _ptr(cdf), _ptr(neg))
    return neg


def lr_at(b: int, B: int, lr0: float, lr_end: float) -> float:
    """Linear decay over the B minibatches of one training call, as an FP32 value."""
    lr = lr0 - (lr0 - lr_end) * b / max(1, B - 1)
    return float(np.float32(lr))


@dataclasses.dataclass
class Delta:
    rows_in: np.ndarray
    d_in: np.ndarray
    rows_out: np.ndarray
    d_out: np.ndarray
    loss: float


def sgns_step(tin: np.ndarray, tout: np.ndarray, ctx, ctr, neg, lr: float,
              apply: bool = True) -> Delta:
    """One minibatch of Eq. (2) SGD (see felog_oracle.c); FP32 or FP64 tables."""
    assert tin.dtype == tout.dtype and tin.flags["C_CONTIGUOUS"] and tout.flags["C_CONTIGUOUS"]
    n, d = tin.shape
    ctx = _c(ctx, np.int32)
    ctr = _c(ctr, np.int32)
    neg = _c(neg, np.int32)
    np_ = ctx.shape[0]
    K = neg.shape[1] if neg.ndim == 2 else 0
    ri = np.zeros(max(1, np_), np.int32)
    di = np.zeros((max(1, np_), d), np.float64)
    ro = np.zeros(max(1, np_ * (K + 1)), np.int32)
    do = np.zeros((max(1, np_ * (K + 1)), d), np.float64)
    ni = np.zeros(1, np.int64)
    no = np.zeros(1, np.int64)
    f = lib().orc_sgns_step_f32 if tin.dtype == np.float32 else lib().orc_sgns_step_f64
    loss = f(_ptr(tin), _ptr(tout), n, d, np_, _ptr(ctx), _ptr(ctr), _ptr(neg), K, lr,
             1 if apply else 0, _ptr(ri), _ptr(di), _ptr(ni), _ptr(ro), _ptr(do), _ptr(no))
    a, b = int(ni[0]), int(no[0])
    return Delta(ri[:a], di[:a], ro[:b], do[:b], float(loss))


def sgns_loss_f64(tin, tout, ctx, ctr, neg) -> float:
    n, d = tin.shape
    neg = _c(neg, np.int32)
    return float(lib().orc_sgns_loss_f64(_ptr(tin), _ptr(tout), d, len(ctx),
                                         _ptr(_c(ctx, np.int32)), _ptr(_c(ctr, np.int32)),
                                         _ptr(neg), neg.shape[1]))


@dataclasses.dataclass
class TrainResult:
    minibatches: int
    pairs: int
    loss: float


def _chunk_minibatches(walks, window, P, chunk):
    """Yield (chunk start, chunk end, slice counts, pairs in chunk) per chunk."""
    W, L = walks.shape
    for c0 in range(0, W, chunk):
        c1 = min(W, c0 + chunk)
        counts = np.zeros(L * 2 * window, np.int64)
        lib().orc_slice_counts(_ptr(walks), c0, c1, L, window, _ptr(counts))
        yield c0, c1, counts, int(counts.sum())


def train_epoch(tin, tout, walks, *, window, K, lr0, lr_end, P, seed, cdf,
                id_base=0, chunk=DEFAULT_CHUNK, mb_begin=0, mb_end=None) -> TrainResult:
    """One Train() call over a walk corpus: minibatches in pair order with lr decay.

    ``mb_begin``/``mb_end`` restrict the call to a minibatch range (the tables
    must then hold the state at the start of ``mb_begin``); the learning-rate
    schedule is always that of the whole corpus.
    """
    walks = _c(walks, np.int32)
    B, total = count_minibatches(walks, window, P, chunk)
    end = B if mb_end is None else min(B, mb_end)
    loss = 0.0
    pairs = 0
    b = 0
    ctx = np.zeros(P, np.int32)
    ctr = np.zeros(P, np.int32)
    col = np.zeros(P, np.int64)
    jj = np.zeros(P, np.int32)
    slot = np.zeros(P, np.int32)
    L = walks.shape[1]
    for c0, c1, counts, npairs in _chunk_minibatches(walks, window, P, chunk):
        nb = (npairs + P - 1) // P
        if b + nb <= mb_begin:
            b += nb
            continue
        for m in range(nb):
            if b >= end:
                break
            if b >= mb_begin:
                k = lib().orc_chunk_pairs_range(_ptr(walks), c0, c1, L, window, _ptr(counts),
                                                m * P, P, _ptr(ctx), _ptr(ctr), _ptr(col),
                                                _ptr(jj), _ptr(slot))
                mb = Minibatch(ctx[:k], ctr[:k], col[:k], jj[:k], slot[:k])
                neg = draw_negatives(mb, id_base, K, seed, cdf)
                d = sgns_step(tin, tout, mb.ctx, mb.ctr, neg, lr_at(b, B, lr0, lr_end))
                loss += d.loss
                pairs += k
            b += 1
        if b >= end:
            break
    return TrainResult(end - mb_begin, pairs, loss)


# --------------------------------------------------------------------------
# Feedback: Eq. (4) and Eq. (5)
# --------------------------------------------------------------------------
def neighbour_subset(g, v: int, k_s: int, seed: int, rnd: int) -> np.ndarray:
    pick = np.zeros(max(1, k_s), np.int64)
    m = lib().orc_neighbour_subset(_ptr(_c(g.indptr, np.int64)), v, k_s, seed, rnd, _ptr(pick))
    return pick[:m].copy()


def psi(tin: np.ndarray, g, nodes, k_s: int, seed: int, rnd: int) -> np.ndarray:
    nodes = _c(nodes, np.int32)
    out = np.zeros(nodes.shape[0], np.float64)
    lib().orc_psi(_ptr(_c(tin, np.float32)), tin.shape[1], _ptr(_c(g.indptr, np.int64)),
                  _ptr(_c(g.indices, np.int32)), _ptr(nodes), nodes.shape[0], k_s, seed, rnd,
                  _ptr(out))
    return out


def next_active(nodes: np.ndarray, psi_vals: np.ndarray, mu: float) -> np.ndarray:
    """Eq. (5): keep v with Psi(v) < mu (strict; NaN, i.e. no neighbours, drops)."""
    keep = psi_vals < mu
    return np.ascontiguousarray(nodes[keep], dtype=np.int32)


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
@dataclasses.dataclass
class RoundStats:
    round: int
    active: int
    walks: int
    pairs: int
    loss: float


def run(g, *, d, r, L, window, K, lr0, lr_end, P, mu, k_s, r_max, seed_walk, seed_model,
        seed_train, seed_psi, neg="unigram", walk="uniform", p=1.0, q=1.0,
        mode="monotone", chunk=DEFAULT_CHUNK, tables=None):
    """Algorithm 1: sample from V_a, train, score Psi, keep Psi < mu; stop when
    V_a is empty or after r_max rounds.  Returns (in, out, per-round stats)."""
    tin, tout = tables if tables is not None else init_tables(g.n, d, seed_model)
    active = np.arange(g.n, dtype=np.int32)
    stats = []
    cdf = None
    id_base = 0
    if neg == "degree":
        cdf = neg_cdf(g.degrees().astype(np.uint64))
    for rnd in range(r_max):
        if active.shape[0] == 0:
            break
        if walk == "uniform":
            walks = walks_uniform(g, active, r, L, seed_walk, id_base)
        else:
            walks, _ = walks_node2vec(g, active, r, L, p, q, seed_walk, id_base)
        if cdf is None:
            cdf = neg_cdf(corpus_counts(walks, g.n))
        tr = train_epoch(tin, tout, walks, window=window, K=K, lr0=lr0, lr_end=lr_end, P=P,
                         seed=seed_train, cdf=cdf, id_base=id_base, chunk=chunk)
        stats.append(RoundStats(rnd, int(active.shape[0]), int(walks.shape[0]), tr.pairs,
                                tr.loss))
        id_base += walks.shape[0]
        cand = active if mode == "monotone" else np.arange(g.n, dtype=np.int32)
        ps = psi(tin, g, cand, k_s, seed_psi, rnd)
        active = next_active(cand, ps, mu)
    return tin, tout, stats


# --------------------------------------------------------------------------
# Link prediction (Section 6.4)
# --------------------------------------------------------------------------
def link_scores(emb: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    e = emb.astype(np.float64)
    return np.einsum("ij,ij->i", e[pairs[:, 0]], e[pairs[:, 1]])


def auc(pos_scores: np.ndarray, neg_scores: np.ndarray) -> float:
    """Mann-Whitney AUC: P(score_pos > score_neg) + 0.5 P(tie)."""
    from scipy.stats import rankdata
    s = np.concatenate([pos_scores, neg_scores])
    ranks = rankdata(s, method="average")
    n1 = pos_scores.shape[0]
    n0 = neg_scores.shape[0]
    return float((ranks[:n1].sum() - n1 * (n1 + 1) / 2.0) / (n1 * n0))


def link_auc(emb: np.ndarray, split) -> float:
    return auc(link_scores(emb, split.test_pos), link_scores(emb, split.test_neg))


# --------------------------------------------------------------------------
# Shared-negative minibatch (BF16 systems form)
# --------------------------------------------------------------------------
def bf16_round(x: np.ndarray) -> np.ndarray:
    f = lib().orc_bf16_round
    flat = np.ascontiguousarray(x, np.float32).ravel()
    return np.array([f(float(v)) for v in flat], np.float32).reshape(np.shape(x))


def shared_negatives(b: int, rnd: int, M: int, seed: int, cdf: np.ndarray) -> np.ndarray:
    out = np.zeros(M, np.int32)
    lib().orc_shared_neg_draw(b, rnd, M, seed, cdf.shape[0] - 1, _ptr(cdf), _ptr(out))
    return out


def shared_neg_step(tin, tout, ctx, ctr, neg, K: int, lr: float, bf16: bool):
    """Deltas of one shared-negative minibatch; returns (dctx, dneg, dctr, loss)."""
    P = len(ctx)
    M = len(neg)
    d = tin.shape[1]
    dctx = np.zeros((P, d), np.float64)
    dneg = np.zeros((M, d), np.float64)
    dctr = np.zeros((P, d), np.float64)
    loss = lib().orc_shared_neg_step(_ptr(_c(tin, np.float32)), _ptr(_c(tout, np.float32)), d,
                                     P, M, K, _ptr(_c(ctx, np.int32)), _ptr(_c(ctr, np.int32)),
                                     _ptr(_c(neg, np.int32)), lr, 1 if bf16 else 0, _ptr(dctx),
                                     _ptr(dneg), _ptr(dctr))
    return dctx, dneg, dctr, float(loss)
