"""Persist(S, V) (Section 5.4): model checkpoints through felog_model_save and
felog_model_load.  A loaded model equals the saved one bit for bit (tables,
noise table, active list, round metadata); Algorithm 1 resumed from a
checkpoint after round 1 equals the uninterrupted run bit for bit; malformed
files are rejected with an error, never loaded."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def fl():
    from paper_2606_22180_amd import build, felog
    if not os.path.exists(build.LIB):
        build.build()
    felog.load()
    return felog


@pytest.fixture(scope="module")
def ctx(fl):
    return fl.Context(0)


@pytest.fixture(scope="module")
def rmat12(fl, ctx):
    e = synth.rmat_edges(12, 1 << 15, seed=31)
    g = synth.csr_from_edges(1 << 12, e)
    return g, fl.Graph.from_csr(ctx, g.indptr, g.indices)


def _state(fl, M):
    return (M.read(fl.TABLE_IN), M.read(fl.TABLE_OUT), M.read_cdf())


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_save_load_round_trip(fl, ctx, rmat12, tmp_path, prec):
    g, G = rmat12
    _say("checkpoint round trip rmat12", prec)
    P = fl.PREC_FP32 if prec == "fp32" else fl.PREC_BF16
    M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_UNIGRAM, seed=3, precision=P)
    W = fl.Walks.generate(G, r=2, L=20, seed=4)
    M.set_unigram(W)
    prm = fl.train_params(window=3, negatives=4, minibatch_pairs=1024, seed=5,
                          shared_negatives=256 if P == fl.PREC_BF16 else 0)
    M.train_steps(W, prm, 0, 20)
    act = M.feedback(mu=0.5, k_s=8, seed=6, round=0)
    path = str(tmp_path / "m.felog")
    M.save(path, active=act, round=1, walk_id_base=W.info()[0])
    L, lact, rnd, base = fl.Model.load(G, path)
    assert (L.n, L.dim, L.neg_dist, L.precision) == (g.n, 64, fl.NEG_UNIGRAM, P)
    assert (rnd, base) == (1, W.info()[0])
    for a, b in zip(_state(fl, M), _state(fl, L)):
        assert np.array_equal(a, b)
    assert np.array_equal(lact.read(), act.read())
    if P == fl.PREC_BF16:
        for t in (fl.TABLE_IN, fl.TABLE_OUT):
            assert np.array_equal(L.read_bf16(t), M.read_bf16(t))
    # the loaded model trains like the original
    st_a = M.train_steps(W, prm, 20, 5)
    st_b = L.train_steps(W, prm, 20, 5)
    if P == fl.PREC_FP32:
        assert st_a.loss == st_b.loss
        assert np.array_equal(M.read(fl.TABLE_IN), L.read(fl.TABLE_IN))
    else:
        assert abs(st_a.loss - st_b.loss) <= 1e-6 * abs(st_a.loss)
    assert os.path.getsize(path) == 64 + 2 * 4 * g.n * 64 + 8 * (g.n + 1) + 4 * act.count()


def test_checkpoint_without_noise_or_list(fl, ctx, rmat12, tmp_path):
    g, G = rmat12
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_UNIGRAM, seed=8)
    path = str(tmp_path / "fresh.felog")
    M.save(path)
    L, act, rnd, base = fl.Model.load(G, path)
    assert act is None and (rnd, base) == (0, 0)
    assert np.array_equal(L.read(fl.TABLE_IN), M.read(fl.TABLE_IN))
    with pytest.raises(fl.FelogError):      # the unigram table is not set yet
        L.read_cdf()
    W = fl.Walks.generate(G, r=1, L=10, seed=1)
    with pytest.raises(fl.FelogError):
        L.train_steps(W, fl.train_params(window=2, negatives=2, minibatch_pairs=512), 0, 1)
    assert os.path.getsize(path) == 64 + 2 * 4 * g.n * 128


def _rounds(fl, G, M, rp, first_round, act, id_base, n_rounds):
    wk, fb = rp.walk, rp.feedback
    losses = []
    for r in range(first_round, first_round + n_rounds):
        W = fl.Walks.generate(G, r=wk.walks_per_node, L=wk.length, seed=wk.seed,
                              id_base=id_base, starts=act)
        if r == 0:
            M.set_unigram(W)
        losses.append(M.train_epoch(W, rp.train).loss)
        id_base += W.info()[0]
        act = M.feedback(mu=fb.mu, k_s=fb.k_s, seed=fb.seed, round=r, mode=fb.mode,
                         active=act)
    return act, id_base, losses


def test_resume_equals_uninterrupted(fl, ctx, rmat12, tmp_path):
    """Three rounds straight, against one round, a checkpoint, a new model
    loaded from it and two more rounds: bit for bit."""
    g, G = rmat12
    _say("checkpoint resume rmat12 3 rounds")
    rp = fl.felog_run_params()
    rp.walk = fl.felog_walk_params(fl.WALK_UNIFORM, 3, 20, 1.0, 1.0, 11, 0)
    rp.train = fl.train_params(window=4, negatives=5, minibatch_pairs=4096, seed=12)
    rp.feedback = fl.felog_feedback_params(0.7, 8, fl.FEEDBACK_MONOTONE, 13, 0)
    A = fl.Model.create(G, dim=64, neg_dist=fl.NEG_UNIGRAM, seed=14)
    act_a, base_a, loss_a = _rounds(fl, G, A, rp, 0, None, 0, 3)
    B = fl.Model.create(G, dim=64, neg_dist=fl.NEG_UNIGRAM, seed=14)
    act_b, base_b, loss_b = _rounds(fl, G, B, rp, 0, None, 0, 1)
    path = str(tmp_path / "r1.felog")
    B.save(path, active=act_b, round=1, walk_id_base=base_b)
    del B
    C, act_c, rnd, base_c = fl.Model.load(G, path)
    act_c, base_c, loss_c = _rounds(fl, G, C, rp, rnd, act_c, base_c, 2)
    assert loss_b + loss_c == loss_a and base_c == base_a
    assert np.array_equal(act_c.read(), act_a.read())
    for t in (fl.TABLE_IN, fl.TABLE_OUT):
        assert np.array_equal(C.read(t), A.read(t))


@pytest.mark.parametrize("P", [1024, 4096])
def test_injected_failure_then_resume(fl, ctx, rmat12, tmp_path, monkeypatch, P):
    """FELOG_DEBUG_FAIL_AFTER_MINIBATCHES=N stops an epoch after N minibatches
    with FELOG_EFAULT_INJECTED; the tables then hold exactly those N
    minibatches, and both recoveries (the rest of the epoch from minibatch N,
    or the whole epoch again from the checkpoint taken before it) equal the
    uninterrupted epoch bit for bit.  P = 1,024 takes the persistent update,
    P = 4,096 the per-minibatch launches."""
    g, G = rmat12
    W = fl.Walks.generate(G, r=2, L=20, seed=21)
    prm = fl.train_params(window=4, negatives=5, minibatch_pairs=P, seed=22)

    def fresh():
        M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_UNIGRAM, seed=23)
        M.set_unigram(W)
        return M

    A = fresh()
    st_a = A.train_epoch(W, prm)
    B_total = st_a.minibatches_total
    cut = B_total // 3
    _say("injected failure rmat12 P=%d: %d minibatches, fail after %d" % (P, B_total, cut))
    assert 0 < cut < B_total
    B = fresh()
    path = str(tmp_path / "before.felog")
    B.save(path, round=0, walk_id_base=0)
    monkeypatch.setenv("FELOG_DEBUG_FAIL_AFTER_MINIBATCHES", str(cut))
    with pytest.raises(fl.FelogError) as err:
        B.train_epoch(W, prm)
    assert err.value.status == fl.FELOG_EFAULT_INJECTED
    # a range the count covers is not cut short
    Cm = fresh()
    Cm.train_steps(W, prm, 0, cut)
    monkeypatch.delenv("FELOG_DEBUG_FAIL_AFTER_MINIBATCHES")
    for t in (fl.TABLE_IN, fl.TABLE_OUT):
        assert np.array_equal(B.read(t), Cm.read(t))
    B.train_steps(W, prm, cut, B_total - cut)
    L, _, rnd, _ = fl.Model.load(G, path)
    assert rnd == 0
    L.train_epoch(W, prm)
    for t in (fl.TABLE_IN, fl.TABLE_OUT):
        a = A.read(t)
        assert np.array_equal(B.read(t), a)
        assert np.array_equal(L.read(t), a)


def test_bad_checkpoints_rejected(fl, ctx, rmat12, tmp_path):
    g, G = rmat12
    M = fl.Model.create(G, dim=64, neg_dist=fl.NEG_DEGREE, seed=1)
    act = fl.Active.from_host(G, np.arange(0, g.n, 5, dtype=np.int32))
    path = str(tmp_path / "ok.felog")
    M.save(path, active=act, round=2, walk_id_base=99)
    good = open(path, "rb").read()
    fl.Model.load(G, path)

    def rejected(data, status=None):
        p = str(tmp_path / "bad.felog")
        open(p, "wb").write(data)
        with pytest.raises(fl.FelogError) as e:
            fl.Model.load(G, p)
        if status is not None:
            assert e.value.status == status

    rejected(b"XXXX" + good[4:], fl.FELOG_EINVAL)                  # magic
    rejected(good[:-4], fl.FELOG_EINVAL)                           # size disagrees
    rejected(good[:40], fl.FELOG_EIO)                              # header cut short
    bad = bytearray(good)
    bad[8:12] = np.int32(g.n + 1).tobytes()                        # another graph
    rejected(bytes(bad), fl.FELOG_EINVAL)
    bad = bytearray(good)
    bad[12:16] = np.int32(48).tobytes()                            # dimension
    rejected(bytes(bad))
    cdf_at = 64 + 2 * 4 * g.n * 64
    bad = bytearray(good)
    bad[cdf_at + 8 * 5:cdf_at + 8 * 6] = np.uint64(1 << 62).tobytes()   # cdf decreases after 5
    rejected(bytes(bad), fl.FELOG_EINVAL)
    bad = bytearray(good)
    bad[-8:-4], bad[-4:] = bad[-4:], bad[-8:-4]                    # list out of order
    rejected(bytes(bad), fl.FELOG_EINVAL)
    with pytest.raises(fl.FelogError) as e:
        fl.Model.load(G, str(tmp_path / "missing.felog"))
    assert e.value.status == fl.FELOG_EIO
    with pytest.raises(fl.FelogError) as e:
        M.save(str(tmp_path / "no_such_dir" / "x.felog"))
    assert e.value.status == fl.FELOG_EIO
    # the context is still usable
    L, a, rnd, base = fl.Model.load(G, path)
    assert (rnd, base) == (2, 99) and np.array_equal(a.read(), act.read())
