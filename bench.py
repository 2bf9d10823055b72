"""Benchmark of the FeLoG hot path on one MI355X.

One step = Algorithm 1 end to end on the R-MAT 2^20 workload: walks from the
active set, one SGNS training call per round, the Psi feedback and the
active-set compaction, until the active set is empty or 4 rounds ran.  The
graph is resident in HBM before the timed region; each step re-initialises the
embedding tables so that every step does the same work.

Prints one JSON line (see the keys below).  `--gpus N` with N > 1 is refused:
this build measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
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
COUNTERS = os.path.join(ROOT, "profiles", "sgns_rmat20_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2606_22180_amd", "csrc", "sgns.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def auc_score(emb: np.ndarray, pos: np.ndarray, neg: np.ndarray) -> float:
    """Link-prediction AUC (Section 6.4): score phi(u).phi(v), Mann-Whitney."""
    from sklearn.metrics import roc_auc_score
    e = emb.astype(np.float64)
    sp = np.einsum("ij,ij->i", e[pos[:, 0]], e[pos[:, 1]])
    sn = np.einsum("ij,ij->i", e[neg[:, 0]], e[neg[:, 1]])
    y = np.r_[np.ones(sp.shape[0]), np.zeros(sn.shape[0])]
    return float(roc_auc_score(y, np.r_[sp, sn]))


def kernel_traffic(kernel: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counters,
    if they were taken on the current kernel source; else None."""
    if not os.path.exists(COUNTERS):
        return None
    rec = json.load(open(COUNTERS))
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if rec.get("source_sha256") != src or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(g, cfg, n_walks: int, n_mb: int):
    """The CPU oracle as it stands, on a bounded sample of the same workload:
    the first n_walks walks of round 1 and the first n_mb minibatches of SGNS
    over that sub-corpus.  Single-threaded C."""
    import oracle
    t0 = time.perf_counter()
    walks = oracle.walks_uniform(g, np.arange(n_walks, dtype=np.int32), 1, cfg["L"], cfg["seed_walk"])
    t_walk = time.perf_counter() - t0
    steps = int((walks[:, 1:] >= 0).sum())
    cdf = oracle.neg_cdf(oracle.corpus_counts(walks, g.n))
    tin, tout = oracle.init_tables(g.n, cfg["dim"], cfg["seed_model"])
    t1 = time.perf_counter()
    tr = oracle.train_epoch(tin, tout, walks, window=cfg["window"], K=cfg["K"],
                            lr0=float(np.float32(cfg["lr0"])), lr_end=float(np.float32(cfg["lr_end"])),
                            P=cfg["minibatch"], seed=cfg["seed_train"], cdf=cdf, mb_end=n_mb)
    t_train = time.perf_counter() - t1
    return {
        "value": tr.pairs / t_train, "unit": "pair-updates/s", "cores": 1, "kind": "oracle",
        "walk_steps_per_s": steps / t_walk,
        "sample": "first %d round-1 walks (%d steps, %.1f s) and the first %d minibatches "
                  "of %d pairs over that sub-corpus (%d pairs, %.1f s), single thread"
                  % (n_walks, steps, t_walk, n_mb, cfg["minibatch"], tr.pairs, t_train),
    }


def serving_sample(felog, n_jobs: int, slots: int, seed: int = 4):
    """p50/p99 job latency of the serving loop on a bounded sample of the serving
    mix: capacity = 1 / mean service time of the jobs run alone, then the same
    jobs arrive as a seeded Poisson process at 0.5, 0.8 and 0.95 x capacity."""
    import synth
    t0 = time.perf_counter()
    mix = synth.job_mix(n_jobs, seed=seed)
    graphs = [synth.job_graph(j) for j in mix]
    log("serving: %d jobs, n = %s (graphs %.1f s)" % (n_jobs, [j["n"] for j in mix],
                                                     time.perf_counter() - t0))

    def submit(S, j, g, at=0.0):
        return S.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                        window=j["window"], seed=j["seed"], arrival_time=at)

    S = felog.Server(0, 0, slots=1, minibatch_pairs=65536, negatives=5)
    service, pairs = [], []
    for j, g in zip(mix, graphs):
        st = S.wait(submit(S, j, g), -1.0)
        service.append(st.t_done - st.t_admit)
        pairs.append(st.pairs)
    S.close()
    capacity = 1.0 / float(np.mean(service))
    log("serving: mean service %.3f s, capacity %.3f jobs/s" % (1.0 / capacity, capacity))
    out = {"jobs": n_jobs, "slots": slots, "capacity_jobs_per_s": capacity,
           "mean_service_s": 1.0 / capacity, "pairs_per_job": float(np.mean(pairs)), "rates": []}
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    for frac in (0.5, 0.8, 0.95):
        lam = frac * capacity
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_jobs))
        S = felog.Server(0, 0, slots=slots, minibatch_pairs=65536, negatives=5)
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
        r = {"load": frac, "arrival_rate_jobs_per_s": lam, "p50_latency_s": float(np.percentile(lat, 50)),
             "p99_latency_s": float(np.percentile(lat, 99)), "jobs_per_s": n_jobs / span,
             "pair_updates_per_s": float(np.sum(pairs)) / span}
        log("serving: load %.2f p50 %.3f s p99 %.3f s" % (frac, r["p50_latency_s"], r["p99_latency_s"]))
        out["rates"].append(r)
    return out


def small_minibatch_sample(felog, G, n_mb: int, seed: int = 3):
    """The FP32 per-pair form against the BF16 shared-negative form at P = M = 1024
    (d = 128, K = 5, w = 10, degree noise) on the bench graph: time per minibatch
    over n_mb minibatches from the middle of the corpus."""
    W = felog.Walks.generate(G, r=10, L=80, seed=1)
    out = {"minibatch_pairs": 1024, "shared_negatives": 1024, "dim": 128, "negatives": 5,
           "window": 10, "minibatches": n_mb}
    for prec, msh, name in ((felog.PREC_FP32, 0, "fp32_per_pair"),
                            (felog.PREC_BF16, 1024, "bf16_shared_negative")):
        M = felog.Model.create(G, dim=128, neg_dist=felog.NEG_DEGREE, seed=2, precision=prec)
        prm = felog.train_params(window=10, negatives=5, minibatch_pairs=1024, seed=seed,
                                 shared_negatives=msh)
        M.train_steps(W, prm, 0, 200)
        st = M.train_steps(W, prm, 300000, n_mb)
        us = st.ms / st.minibatches * 1e3
        r = {"us_per_minibatch": us, "pair_updates_per_s": st.pairs / (st.ms / 1e3)}
        if msh:
            flops = 3 * 2 * 1024 * 1024 * 128   # S, dC and dN
            r["mfma_tflops"] = flops / (us * 1e-6) / 1e12
            r["mfma_frac"] = r["mfma_tflops"] / BF16_PEAK_TFLOPS
        out[name] = r
        log("%s at P=1024: %.1f us/minibatch" % (name, us))
        M.close()
    W.close()
    return out


def codec_sample(felog, G, reps: int = 3):
    """The FaBC walk-corpus codec (Section 5.2.2) on the round-1 corpus of the
    bench graph (r = 10, L = 80): profile, the Eq. (8) target set, pack and
    unpack on the device, best of reps, with a sampled round-trip check."""
    W = felog.Walks.generate(G, r=10, L=80, seed=1)
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
    W.close()
    F = float(cnt[:k].sum()) / total
    moved = raw + by                      # read the corpus once, write the packed bytes
    pack_gbs = moved / (best[0] * 1e-3) / 1e9
    unpack_gbs = moved / (best[1] * 1e-3) / 1e9
    out = {"walks": int(n_walks), "length": int(L), "k": int(k),
           "symbols": [int(x) for x in sym[:k]], "top_shares": [float(c) / total for c in cnt[:4]],
           "raw_bytes": int(raw), "packed_bytes": int(by), "residuals": int(R),
           "ratio": by / raw, "g_eq7": 1.0 - F + k / L + k / 32.0,
           "pack_ms": best[0], "pack_count_ms": best[2][0], "pack_write_ms": best[2][1],
           "unpack_ms": best[1], "pack_gbs": pack_gbs, "unpack_gbs": unpack_gbs,
           "pack_frac": pack_gbs / HBM_PEAK_GBS, "unpack_frac": unpack_gbs / HBM_PEAK_GBS}
    log("codec: k=%d, %d of %d bytes (%.3f; Eq. (7) g = %.3f), pack %.2f ms, unpack %.2f ms" % (
        k, by, raw, by / raw, out["g_eq7"], best[0], best[1]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--max-rounds", type=int, default=4)
    ap.add_argument("--timing-every", type=int, default=16,
                    help="time every n-th forward/apply launch with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walks", type=int, default=1 << 17)
    ap.add_argument("--cpu-minibatches", type=int, default=30)
    ap.add_argument("--progress-every", type=int, default=0,
                    help="drive the rounds from Python (same ABI calls and kernels as "
                         "felog_run) and print a line every N minibatches; for profiler runs")
    ap.add_argument("--serving-jobs", type=int, default=8,
                    help="jobs in the serving-latency sample (0: skip)")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--no-codec", action="store_true",
                    help="skip the walk-corpus codec sample")
    ap.add_argument("--small-minibatches", type=int, default=20000,
                    help="minibatches of the FP32 vs BF16 comparison at P = 1024 (0 = skip)")
    ap.add_argument("--calibrate", action="store_true",
                    help="after the run, build a BF16 model once: its two table conversions "
                         "read n*d*4 and write n*d*2 bytes each (known sizes, for HBM "
                         "counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported by this build" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import synth
    from paper_2606_22180_amd import build as hipbuild
    from paper_2606_22180_amd import felog
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()

    preset = synth.CONFIGS["rmat20"]
    cfg = dict(L=preset["L"], r=preset["r"], window=preset["window"], K=preset["K"],
               dim=preset["dim"], minibatch=preset["minibatch"], lr0=preset["lr0"],
               lr_end=preset["lr_end"], mu=preset["mu"], k_s=preset["k_s"],
               r_max=args.max_rounds, seed_walk=1, seed_model=2, seed_train=3, seed_psi=4)
    t = time.perf_counter()
    split = synth.build_graph("rmat20")
    g = split.train
    log("graph n=%d nnz=%d isolated=%d (%.1f s)" % (g.n, g.nnz, int((g.degrees() == 0).sum()),
                                                   time.perf_counter() - t))

    ctx = felog.Context(0)
    G = felog.Graph.from_csr(ctx, g.indptr, g.indices)
    M = felog.Model.create(G, dim=cfg["dim"], neg_dist=felog.NEG_UNIGRAM, seed=cfg["seed_model"])
    rp = felog.felog_run_params()
    rp.walk = felog.felog_walk_params(felog.WALK_UNIFORM, cfg["r"], cfg["L"], 1.0, 1.0,
                                      cfg["seed_walk"], 0)
    rp.train = felog.train_params(window=cfg["window"], negatives=cfg["K"], lr_start=cfg["lr0"],
                                  lr_end=cfg["lr_end"], minibatch_pairs=cfg["minibatch"],
                                  seed=cfg["seed_train"])
    rp.feedback = felog.felog_feedback_params(cfg["mu"], cfg["k_s"], felog.FEEDBACK_MONOTONE,
                                              cfg["seed_psi"], 0)
    rp.max_rounds = cfg["r_max"]

    deg = g.degrees()

    def run_rounds_python():
        """Algorithm 1 through the separate ABI calls (what felog_run does), with a
        progress line every --progress-every minibatches."""
        st = felog.felog_run_stats()
        act = None
        n_active = g.n
        id_base = 0
        for r in range(cfg["r_max"]):
            if n_active == 0:
                break
            t0 = time.perf_counter()
            W = felog.Walks.generate(G, r=cfg["r"], L=cfg["L"], seed=cfg["seed_walk"],
                                     id_base=id_base, starts=act)
            if r == 0:
                M.set_unigram(W)
            st.ms_walk[r] = (time.perf_counter() - t0) * 1e3
            B = M.train_steps(W, rp.train, 0, 0).minibatches_total
            tr = felog.felog_train_stats()
            for b0 in range(0, B, args.progress_every):
                s = M.train_steps(W, rp.train, b0, args.progress_every)
                for f in ("minibatches", "pairs", "rows_in", "rows_out", "rows_out_single",
                          "timed_launches"):
                    setattr(tr, f, getattr(tr, f) + getattr(s, f))
                for f in ("loss", "ms", "ms_forward", "ms_apply", "ms_prep", "ms_apply_first"):
                    setattr(tr, f, getattr(tr, f) + getattr(s, f))
                log("round %d: minibatches %d/%d" % (r, min(B, b0 + args.progress_every), B))
            st.train[r] = tr
            st.active[r] = n_active
            st.walks[r] = W.info()[0]
            starts = np.arange(g.n) if act is None else act.read()
            st.walk_steps[r] = int(cfg["r"] * (cfg["L"] - 1) * (deg[starts] > 0).sum())
            id_base += st.walks[r]
            t1 = time.perf_counter()
            act = M.feedback(mu=cfg["mu"], k_s=cfg["k_s"], seed=cfg["seed_psi"], round=r,
                             active=act)
            st.ms_feedback[r] = (time.perf_counter() - t1) * 1e3
            n_active = act.count()
            st.rounds = r + 1
        st.final_active = n_active
        return st

    def step():
        M.reset(cfg["seed_model"])
        t0 = time.perf_counter()
        st = run_rounds_python() if args.progress_every else M.run(rp)
        return st, time.perf_counter() - t0

    for i in range(args.warmup):
        st, dt = step()
        log("warmup %d: %.2f s, rounds=%d" % (i, dt, st.rounds))

    ctx.set_timing(args.timing_every)
    times = []
    st = None
    for i in range(args.steps):
        st, dt = step()
        times.append(dt)
        log("step %d: %.2f s, rounds=%d active=%s" % (i, dt, st.rounds,
                                                       list(st.active[:st.rounds])))
    ctx.set_timing(0)
    total = float(np.sum(times))
    R = st.rounds
    rounds = []
    pairs = walk_steps = 0
    fwd_ms = apply_ms = prep_ms = apply0_ms = 0.0
    timed = 0
    mbs = rows = rows_in = rows_out = rows_single = 0
    ms_walk = 0.0
    for r in range(R):
        tr = st.train[r]
        pairs += tr.pairs
        walk_steps += st.walk_steps[r]
        fwd_ms += tr.ms_forward
        apply_ms += tr.ms_apply
        prep_ms += tr.ms_prep
        apply0_ms += tr.ms_apply_first
        timed += tr.timed_launches
        mbs += tr.minibatches
        rows += tr.rows_in + tr.rows_out
        rows_in += tr.rows_in
        rows_out += tr.rows_out
        rows_single += tr.rows_out_single
        ms_walk += st.ms_walk[r]
        rounds.append(dict(active=int(st.active[r]), walks=int(st.walks[r]),
                           walk_steps=int(st.walk_steps[r]), pairs=int(tr.pairs),
                           loss_per_pair=tr.loss / max(1, tr.pairs), ms_walk=st.ms_walk[r],
                           ms_train=tr.ms, ms_feedback=st.ms_feedback[r],
                           minibatches=int(tr.minibatches)))
    pairs_per_step = pairs
    value = pairs_per_step * len(times) / total
    if args.calibrate:
        Mb = felog.Model.create(G, dim=cfg["dim"], neg_dist=felog.NEG_DEGREE,
                                seed=cfg["seed_model"], precision=felog.PREC_BF16)
        log("calibration: 2 conversions of %d bytes read, %d bytes written" % (
            g.n * cfg["dim"] * 4, g.n * cfg["dim"] * 2))
        Mb.close()
    emb = M.read(felog.TABLE_IN)
    auc = auc_score(emb, split.test_pos, split.test_neg)
    log("pairs/step=%d walk_steps/step=%d value=%.4g pairs/s auc=%.4f" % (
        pairs_per_step, walk_steps, value, auc))

    # Roofline of the dominant kernel by time (the events decide): the forward
    # or the first apply launch.  Algorithmic bytes per launch:
    #  - forward: every distinct touched row read once (d*4 B), the out rows
    #    touched once in their minibatch written once (d*4 B; the forward
    #    applies them), the pair's two node ids (8 B) and one 8 B cumulative
    #    weight per negative;
    #  - first apply launch (sgns_apply_kernel<d, 0>, the other out rows' sums):
    #    those out rows read and written once (d*8 B), each distinct in row (a
    #    pair's context) read once (d*4 B) and 12 B per out touch it sums (its
    #    coefficient, context id and pair-order key).  Rows with more than 16
    #    touches are summed here and written by the second launch; their writes
    #    are counted here.
    # The whole minibatch update (ids, the destination sort, forward, both apply
    # launches) reads and writes each touched row once: rows*d*8 + pairs*(8 + 8K).
    # Durations come from HIP events on every timing_every-th minibatch, on the
    # stream the kernels run on; the id work of later minibatches runs
    # concurrently on a second stream, so the durations include that contention.
    d = cfg["dim"]
    K = cfg["K"]
    row_bytes = rows * d * 4
    id_bytes = pairs * (8 + 8 * K)
    multi_out = rows_out - rows_single
    out_touches = pairs * (K + 1)
    per_apply0 = (multi_out * d * 8 + rows_in * d * 4 + (out_touches - rows_single) * 12) / max(1, mbs)
    per_fwd = (row_bytes + rows_single * d * 4 + id_bytes) / max(1, mbs)
    per_update = (2 * row_bytes + id_bytes) / max(1, mbs)
    avg_apply0_s = apply0_ms / 1e3 / max(1, timed)
    avg_fwd_s = fwd_ms / 1e3 / max(1, timed)
    # the next minibatches' ids overlap this one's update, so the update's cost is
    # the training wall time per minibatch
    avg_upd_s = sum(st.train[r].ms for r in range(R)) / 1e3 / max(1, mbs)

    def kernel_roof(name, per, avg_s):
        ach = per / avg_s / 1e9 if timed else None
        return {"kernel": name, "algorithmic_bytes_per_launch": per, "avg_launch_us": avg_s * 1e6,
                "achieved": ach, "frac": (ach / HBM_PEAK_GBS) if ach else None}

    fwd = kernel_roof("sgns_forward_kernel<%d, %d>" % (d, K), per_fwd, avg_fwd_s)
    ap0 = kernel_roof("sgns_apply_kernel<%d, 0>" % d, per_apply0, avg_apply0_s)
    dom, other = (fwd, ap0) if avg_fwd_s >= avg_apply0_s else (ap0, fwd)
    upd_achieved = per_update / avg_upd_s / 1e9 if timed else None
    roof = {"bound": "hbm", "kernel": dom["kernel"],
            "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["frac"], "traffic": kernel_traffic(dom["kernel"]),
            "algorithmic_bytes_per_launch": dom["algorithmic_bytes_per_launch"],
            "avg_launch_us": dom["avg_launch_us"], "timed_launches": timed,
            "touched_rows_per_minibatch": rows / max(1, mbs),
            "in_rows_per_minibatch": rows_in / max(1, mbs),
            "out_rows_per_minibatch": rows_out / max(1, mbs),
            "out_rows_touched_once_per_minibatch": rows_single / max(1, mbs),
            "other_kernel": other,
            "sgns_update": {"kernels": "prep and scan (second stream), forward, two apply "
                                       "launches",
                            "avg_prep_us": prep_ms / 1e3 / max(1, timed) * 1e6,
                            "avg_reduce_us": apply_ms / 1e3 / max(1, timed) * 1e6,
                            "algorithmic_bytes": per_update, "avg_us": avg_upd_s * 1e6,
                            "achieved": upd_achieved,
                            "frac": (upd_achieved / HBM_PEAK_GBS) if upd_achieved else None}}

    out = {
        "metric": METRIC, "value": value, "unit": "pair-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / len(times) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rmat20: R-MAT scale 20 (a,b,c = .57,.19,.19), 2^24 undirected "
                               "edges with 10%% held out, uniform walks r=10 L=80, SGNS d=128 "
                               "w=10 K=5 unigram^0.75 minibatch 65536, FeeST mu=0.65 k_s=10 "
                               "monotone, at most %d rounds" % cfg["r_max"],
                   "nodes": g.n, "csr_entries": g.nnz},
        "walk_steps_per_s": walk_steps * len(times) / (ms_walk / 1e3 * len(times)),
        "walk_steps_per_step": int(walk_steps), "pairs_per_step": int(pairs_per_step),
        "link_pred_auc": auc, "rounds": rounds, "roofline": roof,
    }
    if not args.no_codec:
        out["walk_codec"] = codec_sample(felog, G)
    if args.small_minibatches > 0:
        out["small_minibatch_forms"] = small_minibatch_sample(felog, G, args.small_minibatches)
    if args.serving_jobs > 0:
        out["serving"] = serving_sample(felog, args.serving_jobs, args.serving_slots)
        out["p99_job_latency_s"] = out["serving"]["rates"][1]["p99_latency_s"]   # at 0.8 x capacity
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, cfg, args.cpu_walks, args.cpu_minibatches)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
