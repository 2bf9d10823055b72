"""Benchmark of the FeLoG hot path on one MI355X.

Headline workload (timed steps): second-order node2vec walks (p = 0.5,
q = 2) on a weighted R-MAT graph with 2^23 nodes and 2^27 undirected edges
(10% held out), feeding FP32 skip-gram with negative sampling at d = 128,
window 10, 5 negatives from unigram^0.75, 1,024 pairs per minibatch.  This is
the largest single-GPU configuration of the method's benchmark set.

One step is a fixed slice of that workload's epoch: the node2vec walks of one
2^20-walk chunk of the corpus (chunk s mod 80 at step s, the same walk ids
and start nodes as in the full corpus), then the first --mb-per-step
minibatches (default 16,384, i.e. 16.8M pair-updates) of that chunk's pairs.
The graph, the model and the unigram noise distribution (from the whole
r = 10 corpus, walked once before the timed region) are resident in HBM
before the timed region; nothing inside a step is skipped or cached.  Every
library call returns after its stream completes, so the timed region is
bracketed by device synchronisations.

After the timed steps the JSON line also carries, measured outside them:
  - roofline: the dominant SGNS kernel by HIP-event time, algorithmic bytes
    per launch over its average launch duration, against 8 TB/s;
  - c2_algorithm1: Algorithm 1 end to end on R-MAT 2^20 (uniform walks,
    P = 65,536, FeeST mu = 0.65, at most 4 rounds): per-round active set,
    pairs, walk steps/s, and link-prediction AUC;
  - c4_minibatch_65536, c4_bf16_shared_negative: the headline graph and
    corpus trained at 65,536 pairs per minibatch, and in the BF16
    shared-negative form (P = M = 1,024) against the FP32 form's time per
    minibatch;
  - c3_forms: FP32 per-pair against BF16 shared-negative minibatches
    (P = M = 1,024) on R-MAT 2^22, their error against the FP64 oracle on one
    minibatch, and the AUC of both forms after one epoch on the small SBM;
  - walk_codec, serving: the FaBC corpus codec and the serving loop's latency
    sample;
  - cpu_baseline: the CPU oracle on a bounded sample of the headline
    workload, at one thread and at all host cores.

`--gpus N` with N > 1 is refused: this build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SGNS pair-updates/s + walk steps/s at matched link-pred AUC; p99 job latency"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0     # dense BF16 MFMA
CHUNK = 1 << 20               # walks per training chunk


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def host_info():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def auc_score(emb: np.ndarray, pos: np.ndarray, neg: np.ndarray) -> float:
    """Link-prediction AUC (Section 6.4): score phi(u).phi(v), Mann-Whitney."""
    from sklearn.metrics import roc_auc_score
    e = emb.astype(np.float64)
    sp = np.einsum("ij,ij->i", e[pos[:, 0]], e[pos[:, 1]])
    sn = np.einsum("ij,ij->i", e[neg[:, 0]], e[neg[:, 1]])
    y = np.r_[np.ones(sp.shape[0]), np.zeros(sn.shape[0])]
    return float(roc_auc_score(y, np.r_[sp, sn]))


# ----------------------------------------------------------------- CPU oracle
def cpu_baseline(g, cfg, n_walks: int, n_mb: int, cores: int, model: str):
    """The CPU oracle as it stands, on a bounded sample of the headline
    workload: node2vec walks 0 .. n_walks-1 of the corpus, then the first n_mb
    minibatches of SGNS over those walks (unigram^0.75 noise of the sample),
    once with one thread and once with every host core (the oracle's OpenMP
    loops run over independent walks and over a minibatch's pair
    coefficients; its row sums stay sequential)."""
    import oracle
    oracle.build()
    out = {"unit": "pair-updates/s", "kind": "oracle", "cpu_model": model, "nproc": cores}
    legs = {}
    tin0 = None
    for threads in (1, cores):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        walks, _ = oracle.walks_node2vec(g, np.arange(n_walks, dtype=np.int32), 1, cfg["L"],
                                         cfg["p"], cfg["q"], cfg["seed_walk"], 0)
        t_walk = time.perf_counter() - t0
        steps = int((walks[:, 1:] >= 0).sum())
        if tin0 is None:
            cdf = oracle.neg_cdf(oracle.corpus_counts(walks, g.n))
            tin0, tout0 = oracle.init_tables(g.n, cfg["dim"], cfg["seed_model"])
        tin, tout = tin0.copy(), tout0.copy()
        t1 = time.perf_counter()
        tr = oracle.train_epoch(tin, tout, walks, window=cfg["window"], K=cfg["K"],
                                lr0=float(np.float32(cfg["lr0"])),
                                lr_end=float(np.float32(cfg["lr_end"])), P=cfg["minibatch"],
                                seed=cfg["seed_train"], cdf=cdf, mb_end=n_mb)
        t_train = time.perf_counter() - t1
        legs[threads] = {"pair_updates_per_s": tr.pairs / t_train,
                         "walk_steps_per_s": steps / t_walk, "threads": threads,
                         "walk_s": t_walk, "train_s": t_train, "pairs": int(tr.pairs),
                         "walk_steps": steps}
        log("cpu oracle, %d thread(s): %.3g walk steps/s, %.3g pair-updates/s"
            % (threads, steps / t_walk, tr.pairs / t_train))
        del tin, tout
    oracle.set_threads(cores)
    allc = legs[cores]
    out.update({"value": allc["pair_updates_per_s"], "cores": cores,
                "walk_steps_per_s": allc["walk_steps_per_s"],
                "single_thread": legs[1], "all_cores": allc,
                "sample": "node2vec walks 0..%d of the weighted R-MAT 2^23 corpus (%d steps) and "
                          "the first %d minibatches of %d pairs over them (%d pairs); unigram "
                          "noise of the sample; at 1 thread and at %d threads (%s)"
                          % (n_walks - 1, allc["walk_steps"], n_mb, cfg["minibatch"],
                             allc["pairs"], cores, model)})
    return out


# --------------------------------------------------------------- side legs
def c2_algorithm1(felog, max_rounds: int, per_round: bool = True):
    """Algorithm 1 end to end on R-MAT 2^20 (the feedback-loop workload) through
    felog_run, timed; with per_round, the same rounds again through the
    separate calls for the per-round AUC and hub-row norms."""
    import synth
    pre = synth.CONFIGS["rmat20"]
    t = time.perf_counter()
    split = synth.build_graph("rmat20")
    g = split.train
    log("c2: graph n=%d nnz=%d (%.1f s)" % (g.n, g.nnz, time.perf_counter() - t))
    ctx = felog.Context(0)
    G = felog.Graph.from_csr(ctx, g.indptr, g.indices)
    M = felog.Model.create(G, dim=pre["dim"], neg_dist=felog.NEG_UNIGRAM, seed=2)
    rp = felog.felog_run_params()
    rp.walk = felog.felog_walk_params(felog.WALK_UNIFORM, pre["r"], pre["L"], 1.0, 1.0, 1, 0)
    rp.train = felog.train_params(window=pre["window"], negatives=pre["K"], lr_start=pre["lr0"],
                                  lr_end=pre["lr_end"], minibatch_pairs=pre["minibatch"], seed=3)
    rp.feedback = felog.felog_feedback_params(pre["mu"], pre["k_s"], felog.FEEDBACK_MONOTONE,
                                              4, 0)
    rp.max_rounds = max_rounds
    t0 = time.perf_counter()
    st = M.run(rp)
    wall = time.perf_counter() - t0
    auc = auc_score(M.read(felog.TABLE_IN), split.test_pos, split.test_neg)
    rounds = []
    pairs = steps = 0
    walk_ms = 0.0
    for r in range(st.rounds):
        tr = st.train[r]
        pairs += tr.pairs
        steps += st.walk_steps[r]
        walk_ms += st.ms_walk[r]
        rounds.append(dict(active=int(st.active[r]), walks=int(st.walks[r]),
                           walk_steps=int(st.walk_steps[r]), pairs=int(tr.pairs),
                           loss_per_pair=tr.loss / max(1, tr.pairs), ms_walk=st.ms_walk[r],
                           ms_train=tr.ms, ms_feedback=st.ms_feedback[r],
                           minibatches=int(tr.minibatches)))
    out = {"workload": "R-MAT scale 20 (a,b,c = .57,.19,.19), 2^24 undirected edges, 10%% held "
                       "out; uniform walks r=10 L=80; SGNS d=128 w=10 K=5 unigram^0.75 P=65536; "
                       "FeeST mu=0.65 k_s=10 monotone, at most %d rounds" % max_rounds,
           "rounds": rounds, "final_active": int(st.final_active), "wall_s": wall,
           "pair_updates_per_s": pairs / wall, "pairs": int(pairs),
           "walk_steps_per_s": steps / (walk_ms / 1e3) if walk_ms > 0 else None,
           "link_pred_auc": auc}
    log("c2: %d rounds, active %s, %.2f s, %.3g pair-updates/s, AUC %.4f"
        % (st.rounds, [r["active"] for r in rounds], wall, pairs / wall, auc))
    if per_round:
        # the same rounds through the separate calls, with the AUC and the
        # hub-row norms after each round; their active sets equal felog_run's
        pr = feest_rounds(felog, G, split, pre, mu=pre["mu"], mode="monotone",
                          rounds=max_rounds)
        out["per_round"] = pr["rounds"]
        out["per_round_matches_felog_run"] = \
            [r["active"] for r in pr["rounds"]] == [r["active"] for r in rounds]
    W = felog.Walks.generate(G, r=pre["r"], L=pre["L"], seed=1)
    out_codec = codec_sample(felog, W)
    W.close()
    M.close()
    G.close()
    return out, out_codec


def hub_norms(emb: np.ndarray, deg: np.ndarray, top: int = 100):
    """Row norms of the in-table: the top-degree nodes (the rows that take the
    most summed terms per minibatch) against the median non-isolated node."""
    norms = np.linalg.norm(emb, axis=1)
    hubs = np.argsort(deg)[::-1][:top]
    live = deg > 0
    return {"hub_top%d_mean_norm" % top: float(norms[hubs].mean()),
            "median_norm": float(np.median(norms[live])), "max_norm": float(norms[live].max())}


def feest_rounds(felog, G, split, cfg, *, mu, mode, rounds, lr_span=False, seed_psi=4):
    """Algorithm 1 round by round through the separate calls (walks from the
    active set, one training call, feedback): per round the active set, pairs,
    walk steps, times, link-prediction AUC, hub-row norms and, in
    RECOMPUTE_ALL mode, the reactivated nodes.  lr_span: one learning-rate
    decay over all rounds (round r decays from lr(r / R) to lr((r + 1) / R))
    instead of a restart per round."""
    g = split.train
    deg = g.degrees()
    M = felog.Model.create(G, dim=cfg["dim"], neg_dist=felog.NEG_UNIGRAM, seed=2)
    fmode = felog.FEEDBACK_MONOTONE if mode == "monotone" else felog.FEEDBACK_RECOMPUTE_ALL
    active, prev = None, None
    id_base = 0
    out = []
    t_all = time.perf_counter()
    for rnd in range(rounds):
        n_act = g.n if active is None else active.count()
        if n_act == 0:
            break
        lr0, lr1 = cfg["lr0"], cfg["lr_end"]
        if lr_span:
            span = lr0 - lr1
            lr0, lr1 = cfg["lr0"] - span * rnd / rounds, cfg["lr0"] - span * (rnd + 1) / rounds
        prm = felog.train_params(window=cfg["window"], negatives=cfg["K"], lr_start=lr0,
                                 lr_end=lr1, minibatch_pairs=cfg["minibatch"], seed=3)
        t0 = time.perf_counter()
        W = felog.Walks.generate(G, r=cfg["r"], L=cfg["L"], seed=1, id_base=id_base,
                                 starts=active)
        walks = W.info()[0]
        t1 = time.perf_counter()
        if rnd == 0:
            M.set_unigram(W)
        st = M.train_epoch(W, prm)
        t2 = time.perf_counter()
        id_base += walks
        W.close()
        # a walk from a node with neighbours takes L - 1 transitions, one from
        # an isolated node none
        starts_live = int((deg > 0).sum()) if active is None else int((deg[active.read()] > 0).sum())
        steps = cfg["r"] * (cfg["L"] - 1) * starts_live
        nxt = M.feedback(mu=mu, k_s=cfg["k_s"], seed=seed_psi, round=rnd, mode=fmode,
                         active=active)
        t3 = time.perf_counter()
        emb = M.read(felog.TABLE_IN)
        auc = auc_score(emb, split.test_pos, split.test_neg)
        r = {"round": rnd + 1, "active": int(n_act), "walks": int(walks), "pairs": int(st.pairs),
             "walk_steps": steps, "s_walk": t1 - t0, "s_train": t2 - t1, "s_feedback": t3 - t2,
             "pair_updates_per_s": st.pairs / max(1e-9, t2 - t1), "auc": auc,
             "next_active": int(nxt.count())}
        r.update(hub_norms(emb, deg))
        del emb
        if fmode == felog.FEEDBACK_RECOMPUTE_ALL and active is not None:
            new = nxt.read()
            r["reactivated"] = int(np.isin(new, active.read(), invert=True).sum())
            r["reactivated_frac"] = r["reactivated"] / max(1, new.shape[0])
        if prev is not None:
            prev.close()
        prev = active
        active = nxt
        out.append(r)
        log("  mu %.2f %s round %d: active %d, pairs %.4g, AUC %.4f, hub norm %.3f, median %.3f"
            % (mu, mode, rnd + 1, n_act, st.pairs, auc, r["hub_top100_mean_norm"],
               r["median_norm"]))
    for a in (prev, active):
        if a is not None:
            a.close()
    M.close()
    return {"mu": mu, "mode": mode, "lr": "one decay over the rounds" if lr_span else
            "restart per round", "rounds": out, "pairs": int(sum(r["pairs"] for r in out)),
            "wall_s": time.perf_counter() - t_all, "final_auc": out[-1]["auc"] if out else None}


def ablation(felog, mus, rounds, extra=True):
    """FeeST ablation on R-MAT 2^20 (the Algorithm 1 workload): MONOTONE at each
    mu (mu = 2 keeps every node with neighbours active: training without
    FeeST), RECOMPUTE_ALL at mu = 0.65 with the reactivated share of each new
    active set, and mu = 0.65 with one learning-rate decay over the rounds."""
    import synth
    pre = synth.CONFIGS["rmat20"]
    split = synth.build_graph("rmat20")
    ctx = felog.Context(0)
    G = felog.Graph.from_csr(ctx, split.train.indptr, split.train.indices)
    runs = []
    for mu in mus:
        runs.append(feest_rounds(felog, G, split, pre, mu=mu, mode="monotone", rounds=rounds))
    if extra:
        runs.append(feest_rounds(felog, G, split, pre, mu=0.65, mode="recompute_all",
                                 rounds=rounds))
        runs.append(feest_rounds(felog, G, split, pre, mu=0.65, mode="monotone", rounds=rounds,
                                 lr_span=True))
    G.close()
    ctx.close()
    return {"workload": "R-MAT scale 20, 2^24 undirected edges, 10% held out; uniform walks "
                        "r=10 L=80; SGNS d=128 w=10 K=5 unigram^0.75 P=65536; k_s=10",
            "runs": runs}


def codec_sample(felog, W, reps: int = 3):
    """The FaBC walk-corpus codec (Section 5.2.2) on a round-1 corpus: profile,
    the Eq. (8) target set, pack and unpack on the device, best of reps, with a
    sampled round-trip check."""
    n_walks, L, _ = W.info()
    raw = 4 * n_walks * L
    best = None
    for _ in range(reps):
        k, sym, cnt, total = W.fabc_profile()
        P = W.pack(sym[:k])
        U = P.unpack()
        by, _, _, _, R = P.info()
        for first in (0, n_walks // 2, max(0, n_walks - 4096)):
            c = min(4096, n_walks - first)
            assert np.array_equal(U.read_range(first, c), W.read_range(first, c))
        pack_ms = P.ms[0] + P.ms[1]
        if best is None or pack_ms + U.unpack_ms < best[0] + best[1]:
            best = (pack_ms, U.unpack_ms, P.ms)
        U.close()
        P.close()
    F = float(cnt[:k].sum()) / total
    moved = raw + by
    pack_gbs = moved / (best[0] * 1e-3) / 1e9
    unpack_gbs = moved / (best[1] * 1e-3) / 1e9
    out = {"walks": int(n_walks), "length": int(L), "k": int(k),
           "symbols": [int(x) for x in sym[:k]], "top_shares": [float(c) / total for c in cnt[:4]],
           "raw_bytes": int(raw), "packed_bytes": int(by), "residuals": int(R),
           "ratio": by / raw, "g_eq7": 1.0 - F + k / L + k / 32.0,
           "pack_ms": best[0], "unpack_ms": best[1], "pack_gbs": pack_gbs,
           "unpack_gbs": unpack_gbs, "pack_frac": pack_gbs / HBM_PEAK_GBS,
           "unpack_frac": unpack_gbs / HBM_PEAK_GBS}
    log("codec: k=%d, %.3f of raw, pack %.2f ms, unpack %.2f ms"
        % (k, by / raw, best[0], best[1]))
    return out


def c3_forms(felog, n_mb: int):
    """FP32 per-pair against BF16 shared-negative minibatches at P = M = 1,024
    (d = 128, K = 5, w = 10, degree^0.75 noise) on R-MAT 2^22: time per
    minibatch over n_mb minibatches from the middle of the first 2^20-walk
    chunk; each form's error against the FP64 oracle on one minibatch from the
    same teacher-forced state; and the AUC of both forms after one epoch on
    the small SBM graph (the R-MAT epoch is 62.5G pairs)."""
    import oracle
    import synth
    t = time.perf_counter()
    split = synth.build_graph("rmat22")
    g = split.train
    log("c3: graph n=%d nnz=%d (%.1f s)" % (g.n, g.nnz, time.perf_counter() - t))
    ctx = felog.Context(0)
    G = felog.Graph.from_csr(ctx, g.indptr, g.indices)
    starts = felog.Active.from_host(G, np.arange(CHUNK, dtype=np.int32))
    W = felog.Walks.generate(G, r=1, L=80, seed=1, starts=starts)
    out = {"workload": "R-MAT scale 22, 2^26 undirected edges, 10% held out; uniform walks "
                       "L=80; SGNS d=128 w=10 K=5 degree^0.75; P = M = 1024",
           "minibatches": n_mb}
    first = 300000
    for prec, msh, name in ((felog.PREC_FP32, 0, "fp32_per_pair"),
                            (felog.PREC_BF16, 1024, "bf16_shared_negative")):
        M = felog.Model.create(G, dim=128, neg_dist=felog.NEG_DEGREE, seed=2, precision=prec)
        prm = felog.train_params(window=10, negatives=5, minibatch_pairs=1024, seed=3,
                                 shared_negatives=msh)
        M.train_steps(W, prm, first - 200, 200)
        st = M.train_steps(W, prm, first, n_mb)
        us = st.ms / st.minibatches * 1e3
        r = {"us_per_minibatch": us, "pair_updates_per_s": st.pairs / (st.ms / 1e3)}
        if msh:
            flops = 3 * 2 * 1024 * 1024 * 128   # S = C N^T, dC = G N, dN = G^T C
            r["mfma_tflops"] = flops / (us * 1e-6) / 1e12
            r["mfma_frac"] = r["mfma_tflops"] / BF16_PEAK_TFLOPS
        out[name] = r
        log("c3 %s: %.1f us/minibatch" % (name, us))
        M.close()
    out["bf16_speedup"] = (out["fp32_per_pair"]["us_per_minibatch"]
                           / out["bf16_shared_negative"]["us_per_minibatch"])
    # error of each form against the FP64 oracle, one minibatch, same state
    oracle.build()
    ow = oracle.walks_uniform(g, np.arange(CHUNK, dtype=np.int32), 1, 80, 1, 0)
    assert np.array_equal(W.read_range(0, 4096), ow[:4096])
    cdf = oracle.neg_cdf(g.degrees().astype(np.uint64))
    tin, tout = oracle.init_tables(g.n, 128, 2)
    tout += np.random.default_rng(4).normal(0, 0.05, tout.shape).astype(np.float32)
    b = first
    mb = oracle.minibatch_pairs(ow, 10, 1024, b)
    lr = 0.0125
    errs = {}
    for prec, msh, name in ((felog.PREC_FP32, 0, "fp32_per_pair"),
                            (felog.PREC_BF16, 1024, "bf16_shared_negative")):
        M = felog.Model.create(G, dim=128, neg_dist=felog.NEG_DEGREE, seed=2, precision=prec)
        M.write(felog.TABLE_IN, tin)
        M.write(felog.TABLE_OUT, tout)
        prm = felog.train_params(window=10, negatives=5, minibatch_pairs=1024, seed=3,
                                 shared_negatives=msh, lr_start=lr, lr_end=lr)
        ri, di, ro, do, loss = M.train_delta(W, prm, b)
        M.close()
        if msh:
            neg = oracle.shared_negatives(b, 0, 1024, 3, cdf)
            dctx, dneg, dctr, oloss = oracle.shared_neg_step(tin, tout, mb.ctx, mb.ctr, neg, 5,
                                                             lr, bf16=False)
            rows_in, inv_in = np.unique(mb.ctx, return_inverse=True)
            ref_in = np.zeros((rows_in.shape[0], 128))
            np.add.at(ref_in, inv_in, dctx)
            outs = np.concatenate([neg, mb.ctr])
            rows_out, inv_out = np.unique(outs, return_inverse=True)
            ref_out = np.zeros((rows_out.shape[0], 128))
            np.add.at(ref_out, inv_out, np.concatenate([dneg, dctr]))
        else:
            ng = oracle.draw_negatives(mb, 0, 5, 3, cdf)
            ref = oracle.sgns_step(tin.copy(), tout.copy(), mb.ctx, mb.ctr, ng, lr, apply=False)
            o = np.argsort(ref.rows_in)
            rows_in, ref_in = ref.rows_in[o], ref.d_in[o]
            o = np.argsort(ref.rows_out)
            rows_out, ref_out = ref.rows_out[o], ref.d_out[o]
            oloss = ref.loss
        rel = []
        for gr, gd, rr, rd in ((ri, di, rows_in, ref_in), (ro, do, rows_out, ref_out)):
            assert np.array_equal(np.sort(gr), rr)
            gv = gd[np.argsort(gr)].astype(np.float64)
            rel.append(np.linalg.norm(gv - rd, axis=1) / np.maximum(np.linalg.norm(rd, axis=1),
                                                                  1e-30))
        rel = np.concatenate(rel)
        errs[name] = {"rows": int(rel.shape[0]), "median_rel_err": float(np.median(rel)),
                      "p99_rel_err": float(np.percentile(rel, 99)),
                      "max_rel_err": float(rel.max()),
                      "loss_rel_err": abs(loss - oloss) / abs(oloss)}
        log("c3 %s vs FP64 oracle: median %.2e, max %.2e" % (name, np.median(rel), rel.max()))
    out["error_vs_fp64_oracle"] = errs
    W.close()
    starts.close()
    G.close()
    # AUC of both forms after one epoch on the small SBM (d = 128)
    sbm = synth.build_graph("sbm1k")
    Gs = felog.Graph.from_csr(ctx, sbm.train.indptr, sbm.train.indices)
    Ws = felog.Walks.generate(Gs, r=10, L=40, seed=11)
    aucs = {}
    for prec, msh, name in ((felog.PREC_FP32, 0, "fp32_per_pair"),
                            (felog.PREC_BF16, 1024, "bf16_shared_negative")):
        M = felog.Model.create(Gs, dim=128, neg_dist=felog.NEG_DEGREE, seed=0, precision=prec)
        M.train_epoch(Ws, felog.train_params(window=5, negatives=5, minibatch_pairs=1024,
                                             seed=3, shared_negatives=msh))
        aucs[name] = auc_score(M.read(felog.TABLE_IN), sbm.test_pos, sbm.test_neg)
        M.close()
    out["sbm_epoch_auc"] = aucs
    out["sbm_auc_delta"] = aucs["bf16_shared_negative"] - aucs["fp32_per_pair"]
    log("c3: sbm epoch AUC fp32 %.4f bf16 %.4f" % (aucs["fp32_per_pair"],
                                                    aucs["bf16_shared_negative"]))
    return out


def serving_sample(felog, n_jobs: int, slots: int, seed: int = 4, n_max: int = 200_000,
                   minibatch: int = 65536, update_mode: int = 0):
    """p50/p99 job latency of the serving loop on a sample of the serving mix
    (job sizes log-uniform in [200, n_max]): capacity = 1 / mean service time
    of the jobs run alone, then the same jobs arrive as a seeded Poisson
    process at 0.5, 0.8 and 0.95 x capacity."""
    import synth
    if update_mode == 1:
        slots = 1   # the persistent mode runs one job at a time
    t0 = time.perf_counter()
    mix = synth.job_mix(n_jobs, seed=seed, n_max=n_max)
    graphs = [synth.job_graph(j) for j in mix]
    log("serving: %d jobs, n in [200, %d] (graphs %.1f s)" % (n_jobs, n_max,
                                                             time.perf_counter() - t0))

    def submit(S, j, g, at=0.0):
        return S.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                        window=j["window"], seed=j["seed"], arrival_time=at)

    def server(n_slots):
        return felog.Server(0, 0, slots=n_slots, minibatch_pairs=minibatch, negatives=5,
                            update_mode=update_mode)

    S = server(1)
    service, pairs = [], []
    for j, g in zip(mix, graphs):
        st = S.wait(submit(S, j, g), -1.0)
        service.append(st.t_done - st.t_admit)
        pairs.append(st.pairs)
    S.close()
    capacity = 1.0 / float(np.mean(service))
    out = {"jobs": n_jobs, "slots": slots, "n_max": n_max, "minibatch_cap": minibatch,
           "update_mode": ["per-minibatch launches", "persistent per job",
                           "shared persistent launches"][update_mode],
           "capacity_jobs_per_s": capacity, "mean_service_s": 1.0 / capacity,
           "pairs_per_job": float(np.mean(pairs)), "rates": []}
    log("serving: alone %.3f s per job on average, %.4g pairs per job" % (1.0 / capacity,
                                                                         np.mean(pairs)))
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    for frac in (0.5, 0.8, 0.95):
        lam = frac * capacity
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_jobs))
        S = server(slots)
        base = S.stats()[0] + 0.05
        ids = []
        for (j, g), at in zip(zip(mix, graphs), arrivals):
            while S.stats()[0] < base + at:
                time.sleep(min(0.002, max(0.0, base + at - S.stats()[0])))
            ids.append(submit(S, j, g, base + at))
        states = [S.wait(i, -1.0) for i in ids]
        S.close()
        lat = np.array([s.t_done - s.t_arrive for s in states])
        span = max(s.t_done for s in states) - (base + arrivals[0])
        r = {"load": frac, "arrival_rate_jobs_per_s": lam,
             "p50_latency_s": float(np.percentile(lat, 50)),
             "p99_latency_s": float(np.percentile(lat, 99)), "jobs_per_s": n_jobs / span,
             "pair_updates_per_s": float(np.sum(pairs)) / span}
        log("serving: load %.2f p50 %.3f s p99 %.3f s" % (frac, r["p50_latency_s"],
                                                          r["p99_latency_s"]))
        out["rates"].append(r)
    return out


# ----------------------------------------------------------------- roofline
def sgns_roofline(sts, d: int, K: int, pairs: int):
    """Roofline of the dominant SGNS kernel by HIP-event time.

    Algorithmic bytes of a minibatch: each touched row read once and written
    once (d * 4 bytes each way), the pair's ids and one 8-byte cumulative
    weight per negative draw, and the 8-byte touch descriptor the update
    reads per touch.  Intermediates that a kernel writes and reads back
    (entries, per-pair deltas, context copies) are not counted.

    Persistent path (stats.path == 1): every plan and update launch is timed;
    a launch covers timed_minibatches / timed_launches minibatches.
    Per-minibatch launches (path 0): every timing_every-th minibatch's
    forward and two apply launches are timed."""
    mbs = sum(s.minibatches for s in sts)
    timed = sum(s.timed_launches for s in sts)
    rows_in = sum(s.rows_in for s in sts)
    rows_out = sum(s.rows_out for s in sts)
    single = sum(s.rows_out_single for s in sts)
    touches = pairs * (K + 2)
    row_bytes = (rows_in + rows_out) * d * 4
    upd_bytes = (2 * row_bytes + pairs * (8 + 8 * K)) / mbs
    upd_us = sum(s.ms for s in sts) / mbs * 1e3
    kern = {}
    if sts[0].path == 1:
        tmb = sum(s.timed_minibatches for s in sts)
        per_launch_mb = tmb / max(1, timed)
        per_mb_update = (2 * row_bytes + touches * 8) / mbs
        per_mb_plan = (pairs * (8 + 8 * K) + touches * 8) / mbs
        for name, per, ms in (("sgns_small_update_kernel<%d, %d>" % (d, K), per_mb_update,
                               sum(s.ms_update for s in sts)),
                              ("sgns_plan_kernel<%d>" % K, per_mb_plan,
                               sum(s.ms_prep for s in sts))):
            avg = ms / 1e3 / max(1, timed)
            byt = per * per_launch_mb
            ach = byt / avg / 1e9 if avg > 0 else None
            kern[name] = {"algorithmic_bytes_per_launch": byt, "avg_launch_us": avg * 1e6,
                          "minibatches_per_launch": per_launch_mb,
                          "us_per_minibatch": avg * 1e6 / max(1e-30, per_launch_mb),
                          "achieved_gbs": ach, "frac": ach / HBM_PEAK_GBS if ach else None}
        blocks = sts[0].update_blocks
        # device wall-clock phases of the update (per minibatch and workgroup)
        ph = [sum(s.us_phase[i] * s.timed_minibatches for s in sts) / max(1, tmb)
              for i in range(4)]
        kern["sgns_small_update_kernel<%d, %d>" % (d, K)]["phases_us_per_minibatch"] = {
            "forward": ph[0], "barrier_1": ph[1], "apply": ph[2], "barrier_2": ph[3]}
    else:
        multi_out = rows_out - single
        out_touches = pairs * (K + 1)
        per = {"sgns_forward_kernel<%d, %d>" % (d, K):
                   (row_bytes + single * d * 4 + pairs * (8 + 8 * K)) / mbs,
               "sgns_apply_kernel<%d, 0>" % d:
                   (multi_out * d * 8 + rows_in * d * 4 + (out_touches - single) * 16) / mbs,
               "sgns_apply_kernel<%d, 1>" % d: (rows_in * d * 8 + pairs * d * 4) / mbs}
        ms = {"sgns_forward_kernel<%d, %d>" % (d, K): sum(s.ms_forward for s in sts),
              "sgns_apply_kernel<%d, 0>" % d: sum(s.ms_apply_first for s in sts),
              "sgns_apply_kernel<%d, 1>" % d: sum(s.ms_apply - s.ms_apply_first for s in sts)}
        for name in per:
            avg = ms[name] / 1e3 / max(1, timed)
            ach = per[name] / avg / 1e9 if avg > 0 else None
            kern[name] = {"algorithmic_bytes_per_launch": per[name], "avg_launch_us": avg * 1e6,
                          "achieved_gbs": ach, "frac": ach / HBM_PEAK_GBS if ach else None}
        blocks = None
    dom = max(kern, key=lambda k: kern[k]["avg_launch_us"])
    return {"bound": "hbm", "kernel": dom, "achieved": kern[dom]["achieved_gbs"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kern[dom]["frac"], "traffic": None,
            "algorithmic_bytes_per_launch": kern[dom]["algorithmic_bytes_per_launch"],
            "avg_launch_us": kern[dom]["avg_launch_us"], "timed_launches": timed,
            "update_path": "persistent" if sts[0].path == 1 else "per-minibatch launches",
            "update_blocks": blocks, "kernels": kern,
            "touched_rows_per_minibatch": (rows_in + rows_out) / mbs,
            "sgns_update": {"algorithmic_bytes": upd_bytes, "us_per_minibatch": upd_us,
                            "achieved_gbs": upd_bytes / upd_us / 1e3,
                            "frac": upd_bytes / upd_us / 1e3 / HBM_PEAK_GBS}}


# --------------------------------------------------------------- counters
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "sgns_small_update_rmat23w_counters.md")
COUNTER_SOURCES = ("paper_2606_22180_amd/csrc/sgns_small.hip",
                   "paper_2606_22180_amd/csrc/sgns_device.h", "paper_2606_22180_amd/csrc/noise.h",
                   "paper_2606_22180_amd/csrc/common.h")


def kernel_sources_digest() -> str:
    """SHA-256 over the sources the persistent update kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for rel in COUNTER_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per persistent update launch from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters' reading of
    a copy of known size), or None when the summary is missing or was taken
    on other kernel sources."""
    try:
        with open(COUNTER_SUMMARY) as f:
            kv = dict(line.split(":", 1) for line in f.read().splitlines()
                      if line.startswith(("traffic_bytes_per_launch:", "kernel_sources_sha256:",
                                          "minibatches_per_launch:")))
    except OSError:
        return None
    if kv.get("kernel_sources_sha256", "").strip() != kernel_sources_digest():
        return None
    return {"bytes": float(kv["traffic_bytes_per_launch"]),
            "minibatches_per_launch": float(kv["minibatches_per_launch"])}


def counter_workload(args):
    """A short single-stream run of the headline kernels for counter passes
    (rocprofv3 --pmc takes one dispatch at a time): a 1 GiB elementwise copy
    (torch.neg, 1 GiB read + 1 GiB written) that calibrates the counters,
    then on the weighted R-MAT 2^23 graph with the unigram table of the full
    node2vec corpus, three persistent-update launch groups (192 minibatches
    of 1,024 pairs, d = 128, K = 5) and 64 BF16 shared-negative minibatches
    (P = M = 1,024).  The graph is cached at --graph-cache when given."""
    import synth
    import torch
    path = args.graph_cache
    t = time.perf_counter()
    if path and os.path.exists(path):
        z = np.load(path)
        g = synth.Graph(n=int(z["n"]), indptr=z["indptr"], indices=z["indices"],
                        weights=z["weights"])
    else:
        g = synth.build_graph("rmat23w").train
        if path:
            np.savez(path, n=g.n, indptr=g.indptr, indices=g.indices, weights=g.weights)
    log("counters: graph n=%d nnz=%d (%.1f s)" % (g.n, g.nnz, time.perf_counter() - t))
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y
    log("counters: calibration copies done (3 x 1 GiB read + 1 GiB written)")
    from paper_2606_22180_amd import felog
    ctx = felog.Context(0)
    ctx.set_single_stream(True)
    G = felog.Graph.from_csr(ctx, g.indptr, g.indices, g.weights)
    M = felog.Model.create(G, dim=128, neg_dist=felog.NEG_UNIGRAM, seed=2)
    Mb = felog.Model.create(G, dim=128, neg_dist=felog.NEG_UNIGRAM, seed=2,
                            precision=felog.PREC_BF16)
    Wf = felog.Walks.generate(G, r=10, L=80, seed=1, kind=felog.WALK_NODE2VEC, p=0.5, q=2.0)
    M.set_unigram(Wf)
    Mb.set_unigram(Wf)
    Wf.close()
    starts = felog.Active.from_host(G, np.arange(CHUNK, dtype=np.int32))
    W = felog.Walks.generate(G, r=1, L=80, seed=1, kind=felog.WALK_NODE2VEC, p=0.5, q=2.0,
                             starts=starts)
    log("counters: corpus, unigram table and one 2^20-walk chunk ready")
    prm = felog.train_params(window=10, negatives=5, lr_start=0.025, lr_end=1e-4,
                             minibatch_pairs=1024, seed=3)
    st = M.train_steps(W, prm, 0, 192)
    log("counters: fp32 persistent update, %d minibatches, path %d" % (st.minibatches,
                                                                         st.path))
    prm16 = felog.train_params(window=10, negatives=5, lr_start=0.025, lr_end=1e-4,
                               minibatch_pairs=1024, seed=3, shared_negatives=1024)
    st = Mb.train_steps(W, prm16, 0, 64)
    log("counters: bf16 shared-negative form, %d minibatches" % st.minibatches)
    for o in (W, starts, Mb, M, G, ctx):
        o.close()
    print(json.dumps({"counter_workload": "done", "kernel_sources_sha256":
                      kernel_sources_digest()}), flush=True)


# ------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mb-per-step", type=int, default=16384,
                    help="minibatches of a walk chunk's pairs per step")
    ap.add_argument("--timing-every", type=int, default=16,
                    help="time every n-th minibatch's launches with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walks", type=int, default=1 << 15)
    ap.add_argument("--cpu-minibatches", type=int, default=12)
    ap.add_argument("--c2-rounds", type=int, default=4, help="0 skips the Algorithm 1 leg")
    ap.add_argument("--c3-minibatches", type=int, default=20000, help="0 skips the C3 leg")
    ap.add_argument("--c4-bf16-minibatches", type=int, default=2048,
                    help="BF16 shared-negative minibatches on the headline graph (0 skips)")
    ap.add_argument("--serving-jobs", type=int, default=8, help="0 skips the serving sample")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--large-minibatches", type=int, default=1024,
                    help="minibatches of 65,536 pairs on the headline graph after the timed "
                         "steps (0 skips)")
    ap.add_argument("--no-c2-per-round", action="store_true",
                    help="skip the per-round AUC / hub-norm rerun of the Algorithm 1 leg")
    ap.add_argument("--ablation", action="store_true",
                    help="run the FeeST ablation and mu sweep instead of the benchmark")
    ap.add_argument("--ablation-mus", default="0.5,0.6,0.65,0.7,1.0,2.0")
    ap.add_argument("--ablation-rounds", type=int, default=4)
    ap.add_argument("--ablation-no-extra", action="store_true",
                    help="only the mu sweep (no RECOMPUTE_ALL and learning-rate runs)")
    ap.add_argument("--serving-nmax", type=int, default=20_000,
                    help="largest job of the serving sample (log-uniform sizes from 200)")
    ap.add_argument("--serving-minibatch", type=int, default=65536,
                    help="serving jobs' largest minibatch")
    ap.add_argument("--serving-mode", type=int, default=0,
                    help="serving update mode: 0 per-minibatch launches, 1 persistent per job, "
                         "2 shared persistent launches")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving sample and print it")
    ap.add_argument("--counters", action="store_true",
                    help="run the short single-stream workload for counter passes instead")
    ap.add_argument("--graph-cache", default=None, help="--counters: graph cache file (.npz)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported by this build" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.counters:
        counter_workload(args)
        return
    if args.ablation or args.serving_only:
        from paper_2606_22180_amd import build as hipbuild
        if not os.path.exists(hipbuild.LIB):
            hipbuild.build()
        from paper_2606_22180_amd import felog
        if args.ablation:
            mus = [float(x) for x in args.ablation_mus.split(",") if x]
            print(json.dumps({"ablation": ablation(felog, mus, args.ablation_rounds,
                                                   not args.ablation_no_extra)}), flush=True)
        else:
            print(json.dumps({"serving": serving_sample(
                felog, args.serving_jobs, args.serving_slots, n_max=args.serving_nmax,
                minibatch=args.serving_minibatch, update_mode=args.serving_mode)}),
                flush=True)
        return

    import synth
    cores, cpu_model = host_info()
    cfg = dict(L=80, r=10, p=0.5, q=2.0, window=10, K=5, dim=128, minibatch=1024, lr0=0.025,
               lr_end=1e-4, seed_walk=1, seed_model=2, seed_train=3)
    t = time.perf_counter()
    split = synth.build_graph("rmat23w")
    g = split.train
    deg = g.degrees()
    log("graph n=%d nnz=%d isolated=%d (%.1f s)" % (g.n, g.nnz, int((deg == 0).sum()),
                                                   time.perf_counter() - t))
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched
        cpu = cpu_baseline(g, cfg, args.cpu_walks, args.cpu_minibatches, cores, cpu_model)

    from paper_2606_22180_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    from paper_2606_22180_amd import felog
    ctx = felog.Context(0)
    G = felog.Graph.from_csr(ctx, g.indptr, g.indices, g.weights)
    M = felog.Model.create(G, dim=cfg["dim"], neg_dist=felog.NEG_UNIGRAM, seed=cfg["seed_model"])
    t = time.perf_counter()
    Wf = felog.Walks.generate(G, r=cfg["r"], L=cfg["L"], seed=cfg["seed_walk"],
                              kind=felog.WALK_NODE2VEC, p=cfg["p"], q=cfg["q"])
    full_walks = Wf.info()[0]
    full_s = time.perf_counter() - t
    capped = Wf.capped()
    M.set_unigram(Wf)
    Mb = None
    if args.c4_bf16_minibatches > 0:
        # the BF16 shared-negative form on the same graph and noise table
        Mb = felog.Model.create(G, dim=cfg["dim"], neg_dist=felog.NEG_UNIGRAM,
                                seed=cfg["seed_model"], precision=felog.PREC_BF16)
        Mb.set_unigram(Wf)
    Wf.close()
    full_steps = cfg["r"] * (cfg["L"] - 1) * int((deg > 0).sum())
    log("full node2vec corpus: %d walks, %d steps in %.3f s, capped %d; unigram table set"
        % (full_walks, full_steps, full_s, capped))
    n_chunks = full_walks // CHUNK
    offsets = {}
    prm = felog.train_params(window=cfg["window"], negatives=cfg["K"], lr_start=cfg["lr0"],
                             lr_end=cfg["lr_end"], minibatch_pairs=cfg["minibatch"],
                             seed=cfg["seed_train"])

    def chunk_starts(s):
        """Walk id base and start list of corpus chunk s mod 80."""
        first = (s % n_chunks) * CHUNK
        off = first % g.n
        if off not in offsets:
            offsets[off] = felog.Active.from_host(G, np.arange(off, off + CHUNK, dtype=np.int32))
        return first, off

    def chunk_walks(first, off):
        """The chunk's walks: the corpus's own walk ids and start nodes."""
        return felog.Walks.generate(G, r=1, L=cfg["L"], seed=cfg["seed_walk"], id_base=first,
                                    kind=felog.WALK_NODE2VEC, p=cfg["p"], q=cfg["q"],
                                    starts=offsets[off])

    def step(s):
        first, off = chunk_starts(s)
        t0 = time.perf_counter()
        W = chunk_walks(first, off)
        t1 = time.perf_counter()
        st = M.train_steps(W, prm, 0, args.mb_per_step)
        W.close()
        steps = (cfg["L"] - 1) * int((deg[off:off + CHUNK] > 0).sum())
        return st, t1 - t0, steps

    for i in range(args.warmup):
        st, _, _ = step(i)
        log("warmup %d: %d minibatches" % (i, st.minibatches))
    ctx.set_timing(args.timing_every)
    walk_s = 0.0
    walk_steps = pairs = 0
    sts = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        st, ws, steps = step(args.warmup + i)
        walk_s += ws
        walk_steps += steps
        pairs += st.pairs
        sts.append(st)
    total = time.perf_counter() - t0
    ctx.set_timing(0)
    value = pairs / total
    log("timed: %d steps, %.3f s, %.4g pair-updates/s, walks %.3g steps/s"
        % (args.steps, total, value, walk_steps / walk_s))

    roof = sgns_roofline(sts, cfg["dim"], cfg["K"], pairs)
    tr = measured_traffic()
    if tr is not None and roof["kernel"].startswith("sgns_small_update_kernel"):
        # counters were taken on launches of tr["minibatches_per_launch"] minibatches
        roof["traffic"] = tr["bytes"] / tr["minibatches_per_launch"] * \
            roof["kernels"][roof["kernel"]]["minibatches_per_launch"]
        roof["traffic_over_algorithmic"] = roof["traffic"] / roof["algorithmic_bytes_per_launch"]
    out = {
        "metric": METRIC, "value": value, "unit": "pair-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "weighted R-MAT scale 23 (a,b,c = .57,.19,.19), 2^27 undirected "
                               "edges, 10%% held out, weights U(0,1]; node2vec p=0.5 q=2, "
                               "r=10 L=80; SGNS FP32 d=128 w=10 K=5 unigram^0.75, minibatch "
                               "1024; one step = the walks of one 2^20-walk chunk + its first "
                               "%d minibatches" % args.mb_per_step,
                   "nodes": g.n, "csr_entries": g.nnz, "minibatches_per_step": args.mb_per_step},
        "walk_steps_per_s": walk_steps / walk_s,
        "walk_steps_per_s_full_corpus": full_steps / full_s,
        "pairs_per_step": pairs / args.steps, "node2vec_capped": int(capped),
        "roofline": roof,
    }
    if args.large_minibatches > 0:
        # the same graph, walks and model at the plain FP32 configuration's
        # minibatch of 65,536 pairs (per-minibatch launches), outside the
        # timed steps: the rate at which the C4 graph trains in large minibatches
        W = chunk_walks(*chunk_starts(args.steps + args.warmup))
        prm_l = felog.train_params(window=cfg["window"], negatives=cfg["K"], lr_start=cfg["lr0"],
                                   lr_end=cfg["lr_end"], minibatch_pairs=65536,
                                   seed=cfg["seed_train"])
        M.train_steps(W, prm_l, 0, 4)
        ctx.set_timing(4)
        st = M.train_steps(W, prm_l, 4, args.large_minibatches)
        ctx.set_timing(0)
        W.close()
        lr_roof = sgns_roofline([st], cfg["dim"], cfg["K"], st.pairs)
        out["c4_minibatch_65536"] = {
            "minibatches": int(st.minibatches), "pairs": int(st.pairs),
            "pair_updates_per_s": st.pairs / (st.ms / 1e3),
            "us_per_minibatch": st.ms / st.minibatches * 1e3,
            "dominant_kernel": lr_roof["kernel"], "achieved_gbs": lr_roof["achieved"],
            "frac": lr_roof["frac"], "sgns_update": lr_roof["sgns_update"]}
        log("c4 at P = 65536: %.4g pair-updates/s, %.1f us per minibatch, %s at %.3f of HBM"
            % (st.pairs / (st.ms / 1e3), st.ms / st.minibatches * 1e3, lr_roof["kernel"],
               lr_roof["frac"]))
    if Mb is not None:
        # BF16 shared-negative minibatches (P = M = 1,024) on one chunk of the
        # same corpus, outside the timed steps, against the FP32 form's rate
        W = chunk_walks(*chunk_starts(args.steps + args.warmup + 1))
        prm16 = felog.train_params(window=cfg["window"], negatives=cfg["K"],
                                   lr_start=cfg["lr0"], lr_end=cfg["lr_end"],
                                   minibatch_pairs=cfg["minibatch"], seed=cfg["seed_train"],
                                   shared_negatives=1024)
        Mb.train_steps(W, prm16, 0, 64)
        st = Mb.train_steps(W, prm16, 64, args.c4_bf16_minibatches)
        W.close()
        us = st.ms / st.minibatches * 1e3
        flop = 2.0 * 3 * cfg["minibatch"] * 1024 * cfg["dim"]   # S = C N^T, dC = G N, dN = G^T C
        fp32_us = roof["sgns_update"]["us_per_minibatch"]   # device time per minibatch, FP32 form
        out["c4_bf16_shared_negative"] = {
            "minibatches": int(st.minibatches), "us_per_minibatch": us,
            "pair_updates_per_s": st.pairs / (st.ms / 1e3),
            "mfma_tflops": flop / (us * 1e-6) / 1e12,
            "mfma_frac": flop / (us * 1e-6) / 1e12 / BF16_PEAK_TFLOPS,
            "fp32_us_per_minibatch": fp32_us, "bf16_speedup": fp32_us / us}
        log("c4 bf16 shared-negative: %.1f us per minibatch (fp32 %.1f), %.3g pair-updates/s"
            % (us, fp32_us, st.pairs / (st.ms / 1e3)))
        Mb.close()
    G.close()
    M.close()
    for a in offsets.values():
        a.close()
    if args.c2_rounds > 0:
        out["c2_algorithm1"], out["walk_codec"] = c2_algorithm1(felog, args.c2_rounds,
                                                                not args.no_c2_per_round)
    if args.c3_minibatches > 0:
        out["c3_forms"] = c3_forms(felog, args.c3_minibatches)
    if args.serving_jobs > 0:
        out["serving"] = serving_sample(felog, args.serving_jobs, args.serving_slots,
                                        n_max=args.serving_nmax,
                                        minibatch=args.serving_minibatch,
                                        update_mode=args.serving_mode)
        out["p99_job_latency_s"] = out["serving"]["rates"][1]["p99_latency_s"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
