"""GPU tests of the serving loop (felog_server_*).

A serving job is the plain path (uniform walks, degree^0.75 noise, one SGNS
epoch) with job-local seeds, so its result must not depend on the other jobs
in flight.  The SGNS row sums are exact (terms on a 2^-40 grid, added in
FP64), so a job's embeddings are bit-identical alone and in a mix.
"""
import numpy as np
import pytest

import synth
from conftest import link_auc_of

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def fl():
    import os
    from paper_2606_22180_amd import build, felog
    if not os.path.exists(build.LIB):
        build.build()
    felog.load()
    return felog


def _jobs():
    mix = synth.job_mix(12, seed=9, n_min=200, n_max=6000)
    out = []
    for j in mix:
        g = synth.job_graph(j)
        out.append((j, g))
    return out


def test_serving_job_matches_oracle(fl, orc):
    """A job on the sbm1k training graph reaches the oracle's AUC."""
    sp = synth.build_graph("sbm1k")
    g = sp.train
    _say("serving job sbm1k vs oracle")
    S = fl.Server(0, 0, slots=2, minibatch_pairs=65536, negatives=5)
    jid = S.submit(g.indptr, g.indices, dim=64, r=10, L=40, window=5, seed=21)
    st = S.wait(jid, 120.0)
    emb = S.fetch(jid)
    S.close()
    walks = orc.walks_uniform(g, np.arange(g.n), 10, 40, 21)
    tin, tout = orc.init_tables(g.n, 64, 21)
    ref = orc.train_epoch(tin, tout, walks, window=5, K=5, lr0=float(np.float32(0.025)),
                          lr_end=float(np.float32(1e-4)), P=1024, seed=21,
                          cdf=orc.neg_cdf(g.degrees().astype(np.uint64)))
    a_gpu, a_orc = link_auc_of(emb, sp), orc.link_auc(tin, sp)
    _say("AUC serving=%.5f oracle=%.5f pairs %d/%d latency %.3f s" % (
        a_gpu, a_orc, st.pairs, ref.pairs, st.t_done - st.t_arrive))
    assert st.state == fl.JOB_DONE and st.pairs == ref.pairs and st.minibatch_pairs == 1024
    assert abs(a_gpu - a_orc) <= 0.005
    assert abs(st.loss - ref.loss) <= 1e-4 * ref.loss


@pytest.mark.parametrize("mode", [0, 2])
def test_serving_job_equals_direct_path(fl, mode):
    """A serving job's embeddings equal, bit for bit, those of the same job run
    through the library's own calls (uniform walks, degree^0.75 noise, one
    epoch, the job's seed for walks, tables and negatives), whose minibatch
    steps the parity tests hold to the oracle row by row: per-minibatch
    launches (mode 0) and shared persistent launches (mode 2)."""
    sp = synth.build_graph("sbm1k")
    g = sp.train
    S = fl.Server(0, 0, slots=2, minibatch_pairs=65536, negatives=5, update_mode=mode)
    jid = S.submit(g.indptr, g.indices, dim=64, r=10, L=40, window=5, seed=21)
    st = S.wait(jid, 120.0)
    emb = S.fetch(jid)
    S.close()
    assert st.state == fl.JOB_DONE and st.minibatch_pairs == 1024
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    W = fl.Walks.generate(G, r=10, L=40, seed=21)
    M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=21)
    ds = M.train_epoch(W, fl.train_params(window=5, negatives=5, minibatch_pairs=1024, seed=21))
    ref = M.read(fl.TABLE_IN)
    for o in (M, W, G, ctx):
        o.close()
    diff = int((emb.view(np.uint32) != ref.view(np.uint32)).sum())
    _say("mode %d: serving job vs direct calls: pairs %d/%d, differing words %d of %d"
         % (mode, st.pairs, ds.pairs, diff, ref.size))
    assert st.pairs == ds.pairs and diff == 0


def test_serving_alone_equals_mix(fl):
    jobs = _jobs()
    _say("serving alone vs mix: %d jobs, n = %s" % (len(jobs), [j["n"] for j, _ in jobs]))
    alone = {}
    S1 = fl.Server(0, 0, slots=1, minibatch_pairs=4096, negatives=5)
    for j, g in jobs[:4]:
        jid = S1.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                        window=j["window"], seed=j["seed"])
        S1.wait(jid, 300.0)
        alone[j["job"]] = (S1.fetch(jid), S1.poll(jid).loss)
    S1.close()
    S4 = fl.Server(0, 0, slots=4, minibatch_pairs=4096, negatives=5)
    ids = []
    for j, g in jobs:
        ids.append((j, S4.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                                 window=j["window"], seed=j["seed"])))
    for j, jid in ids:
        st = S4.wait(jid, 300.0)
        assert st.state == fl.JOB_DONE and np.isfinite(st.loss)
        if j["job"] in alone:
            emb, loss = alone[j["job"]]
            mixed = S4.fetch(jid)
            assert np.isfinite(mixed).all() and np.isfinite(emb).all()
            rel = np.abs(mixed - emb).max() / np.abs(emb).max()
            _say("job %d n=%d: max |mix - alone| / max|alone| = %.2e, loss %.9e vs %.9e" % (
                j["job"], j["n"], rel, st.loss, loss))
            assert np.array_equal(mixed, emb)
            assert st.loss == loss
    S4.close()


def test_serving_budget_and_fifo(fl):
    jobs = _jobs()[:8]
    # a budget that fits the largest job but not two of them at once
    sizes = []
    probe = fl.Server(0, 0, slots=1, minibatch_pairs=4096, negatives=5)
    for j, g in jobs:
        jid = probe.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                           window=j["window"], seed=j["seed"])
        sizes.append(probe.poll(jid).device_bytes)
    probe.close()
    budget = max(sizes) + min(sizes) // 2
    _say("budget %d bytes, job estimates %s" % (budget, sizes))
    S = fl.Server(0, budget, slots=4, minibatch_pairs=4096, negatives=5)
    ids = [S.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"], window=j["window"],
                    seed=j["seed"]) for j, g in jobs]
    states = [S.wait(i, 300.0) for i in ids]
    _, peak, queued = S.stats()
    assert queued == 0 and all(s.state == fl.JOB_DONE for s in states)
    assert peak <= budget
    admits = [s.t_admit for s in states]
    assert admits == sorted(admits)                      # FIFO admission
    for s_, size in zip(states, sizes):
        assert s_.device_bytes == size and 0 < s_.peak_bytes <= size
    # running intervals: the estimates of overlapping jobs fit the budget
    for a in states:
        live = [b.device_bytes for b in states if b.t_admit <= a.t_admit < b.t_done]
        assert sum(live) <= budget
    g = jobs[0][1]
    big = fl.Server(0, 1 << 20, slots=1, minibatch_pairs=4096, negatives=5)
    try:
        with pytest.raises(fl.FelogError):
            big.submit(g.indptr, g.indices, dim=256, r=10, L=80, window=5, seed=1)
    finally:
        big.close()
    S.close()


@pytest.mark.skip(reason="several jobs' cooperative launches in flight at once on separate "
                         "streams: the test ran for more than 180 s without output once in a "
                         "full-suite run (it had passed three times); the cause was not found, "
                         "and the persistent serving mode now takes one slot only")
def test_serving_persistent_jobs_concurrent(fl):
    """Four slots of jobs on the persistent update (minibatches of at most
    1,024 pairs, each job's launch on a quarter of the compute units) give the
    same embeddings and losses as the jobs alone on the per-minibatch
    launches."""
    jobs = _jobs()[:8]
    alone = {}
    S1 = fl.Server(0, 0, slots=1, minibatch_pairs=1024, negatives=5,
                   update_mode=fl.SERVE_LAUNCHES)
    for j, g in jobs:
        jid = S1.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                        window=j["window"], seed=j["seed"])
        st = S1.wait(jid, 300.0)
        alone[j["job"]] = (S1.fetch(jid), st.loss, st.t_done - st.t_admit)
    S1.close()
    S4 = fl.Server(0, 0, slots=4, minibatch_pairs=1024, negatives=5,
                   update_mode=fl.SERVE_PERSISTENT)
    ids = [(j, S4.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                         window=j["window"], seed=j["seed"])) for j, g in jobs]
    for j, jid in ids:
        st = S4.wait(jid, 300.0)
        emb, loss, t_alone = alone[j["job"]]
        same = np.array_equal(S4.fetch(jid), emb)
        _say("job %d n=%d P=%d: persistent in a mix equal to per-minibatch alone: %s, "
             "service %.3f s (alone, per-minibatch %.3f s)" % (
                 j["job"], j["n"], st.minibatch_pairs, same, st.t_done - st.t_admit, t_alone))
        # the two paths sum the loss terms in different orders
        assert st.state == fl.JOB_DONE and same and abs(st.loss - loss) <= 1e-12 * abs(loss)
    S4.close()


def test_serving_persistent_one_slot(fl):
    """The persistent mode takes one slot (one cooperative launch in flight);
    its jobs give the same embeddings and losses as the jobs alone on the
    per-minibatch launches.  More slots are refused."""
    with pytest.raises(fl.FelogError):
        fl.Server(0, 0, slots=2, minibatch_pairs=1024, negatives=5,
                  update_mode=fl.SERVE_PERSISTENT)
    jobs = _jobs()[:4]
    alone = {}
    S1 = fl.Server(0, 0, slots=1, minibatch_pairs=1024, negatives=5,
                   update_mode=fl.SERVE_LAUNCHES)
    try:
        for j, g in jobs:
            jid = S1.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                            window=j["window"], seed=j["seed"])
            st = S1.wait(jid, 120.0)
            alone[j["job"]] = (S1.fetch(jid), st.loss, st.t_done - st.t_admit)
    finally:
        S1.close()
    SP = fl.Server(0, 0, slots=1, minibatch_pairs=1024, negatives=5,
                   update_mode=fl.SERVE_PERSISTENT)
    try:
        ids = [(j, SP.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                             window=j["window"], seed=j["seed"])) for j, g in jobs]
        for j, jid in ids:
            st = SP.wait(jid, 120.0)
            emb, loss, t_alone = alone[j["job"]]
            same = np.array_equal(SP.fetch(jid), emb)
            _say("job %d n=%d P=%d: persistent (one slot) equal to per-minibatch alone: %s, "
                 "service %.3f s (per-minibatch %.3f s)" % (
                     j["job"], j["n"], st.minibatch_pairs, same, st.t_done - st.t_admit,
                     t_alone))
            assert st.state == fl.JOB_DONE and same and abs(st.loss - loss) <= 1e-12 * abs(loss)
    finally:
        SP.close()


def test_serving_shared_launches(fl):
    """Jobs training in shared persistent launches (up to 8 running jobs of
    equal d per launch; here 3 slots, jobs of d = 64 and 128, minibatches of
    at most 1,024 pairs, and one job whose P is 2,048, which keeps its
    per-minibatch launches) give the same embeddings as each job alone on the
    per-minibatch launches, and every job's loss within 1e-12."""
    jobs = [jg for jg in _jobs() if jg[0]["n"] <= 1024][:6]
    extra = synth.job_mix(1, seed=5, n_min=1500, n_max=1800)[0]
    jobs.append((extra, synth.job_graph(extra)))
    _say("shared launches: jobs n = %s, d = %s" % ([j["n"] for j, _ in jobs],
                                                     [j["dim"] for j, _ in jobs]))
    alone = {}
    S1 = fl.Server(0, 0, slots=1, minibatch_pairs=2048, negatives=5,
                   update_mode=fl.SERVE_LAUNCHES)
    for j, g in jobs:
        jid = S1.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                        window=j["window"], seed=j["seed"])
        st = S1.wait(jid, 300.0)
        alone[j["job"], j["n"]] = (S1.fetch(jid), st.loss, st.t_done - st.t_admit,
                                   st.minibatch_pairs)
    S1.close()
    S3 = fl.Server(0, 0, slots=3, minibatch_pairs=2048, negatives=5,
                   update_mode=fl.SERVE_SHARED)
    ids = [(j, S3.submit(g.indptr, g.indices, dim=j["dim"], r=j["r"], L=j["L"],
                         window=j["window"], seed=j["seed"])) for j, g in jobs]
    for j, jid in ids:
        st = S3.wait(jid, 300.0)
        emb, loss, t_alone, P = alone[j["job"], j["n"]]
        same = np.array_equal(S3.fetch(jid), emb)
        _say("job %d n=%d d=%d P=%d: shared launches equal to alone: %s, service %.3f s "
             "(alone %.3f s)" % (j["job"], j["n"], j["dim"], st.minibatch_pairs, same,
                                 st.t_done - st.t_admit, t_alone))
        assert st.state == fl.JOB_DONE and same and st.minibatch_pairs == P
        assert abs(st.loss - loss) <= 1e-12 * abs(loss)
    S3.close()
    with pytest.raises(fl.FelogError):
        fl.Server(0, 0, slots=4, minibatch_pairs=1024, negatives=5, update_mode=fl.SERVE_SHARED)
