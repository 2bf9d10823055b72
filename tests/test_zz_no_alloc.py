"""felog_feedback_noalloc, the feedback step without device allocation,
against felog_feedback through the C ABI: the same Psi (bit for bit) and the
same next active set, on two calls in a row, the second with a smaller input
list; all nodes and RECOMPUTE_ALL; an invalid list and the size limit
rejected.  Device buffers are the caller's, allocated here with hipMalloc on
the HIP runtime the library uses."""
import ctypes as C
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
def hip(fl):
    """The HIP runtime the library loaded (its path from /proc/self/maps)."""
    path = None
    for line in open("/proc/self/maps"):
        if "libamdhip64.so" in line:
            path = line.split()[-1]
            break
    assert path, "libamdhip64 not loaded"
    h = C.CDLL(path)
    h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    h.hipFree.argtypes = [C.c_void_p]
    h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    h.hipDeviceSynchronize.argtypes = []
    return h


class DevArray:
    """A caller-owned device buffer (hipMalloc / hipFree)."""

    def __init__(self, hip, nbytes):
        self.hip = hip
        self.ptr = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.ptr), max(8, nbytes)) == 0
        self.nbytes = nbytes

    def put(self, a: np.ndarray):
        a = np.ascontiguousarray(a)
        assert a.nbytes <= self.nbytes
        assert self.hip.hipMemcpy(self.ptr, a.ctypes.data, a.nbytes, 1) == 0   # host to device

    def get(self, dtype, count) -> np.ndarray:
        out = np.zeros(max(1, count), dtype)
        assert self.hip.hipMemcpy(out.ctypes.data, self.ptr, out.itemsize * count, 2) == 0
        return out[:count]

    def free(self):
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = None


def test_feedback_noalloc_matches_feedback(fl, hip):
    sp = synth.build_graph("sbm1k")
    g = sp.train
    _say("feedback_noalloc vs feedback on sbm1k")
    ctx = fl.Context(0)
    G = fl.Graph.from_csr(ctx, g.indptr, g.indices)
    M = fl.Model.create(G, dim=128, neg_dist=fl.NEG_DEGREE, seed=2)
    rng = np.random.default_rng(0)
    tin = rng.normal(0, 1, (g.n, 128)).astype(np.float32)
    tin[::97] += tin[1::97][: tin[::97].shape[0]]
    M.write(fl.TABLE_IN, tin)
    din = DevArray(hip, 4 * g.n)
    dout = DevArray(hip, 4 * g.n)
    dpsi = DevArray(hip, 8 * g.n)
    try:
        # two calls in a row, the second on a smaller list; then all nodes
        lists = [np.arange(0, g.n, 2, dtype=np.int32), np.arange(5, 400, 7, dtype=np.int32)]
        for i, (nodes, mu, rnd) in enumerate(((lists[0], 0.02, 1), (lists[1], 0.05, 2),
                                              (None, 0.02, 3))):
            ref_act, ref_psi = M.feedback(mu=mu, k_s=10, seed=9, round=rnd,
                                          active=None if nodes is None else fl.Active.from_host(G, nodes),
                                          want_psi=True)
            ref = ref_act.read()
            count = g.n if nodes is None else nodes.shape[0]
            if nodes is not None:
                din.put(nodes)
            # stale values in the outputs from the previous call must not leak
            dout.put(np.full(g.n, -7, np.int32))
            kept = M.feedback_noalloc(mu=mu, k_s=10, seed=9, round=rnd,
                                      in_nodes_dev=None if nodes is None else din.ptr.value,
                                      count=count, out_nodes_dev=dout.ptr.value, out_cap=g.n,
                                      psi_dev=dpsi.ptr.value, psi_cap=g.n)
            got = dout.get(np.int32, kept)
            psi = dpsi.get(np.float64, count)
            _say("call %d: scored %d, kept %d (reference %d)" % (i, count, kept, ref.shape[0]))
            assert kept == ref.shape[0]
            assert np.array_equal(got, ref)
            assert np.array_equal(psi.view(np.uint64), ref_psi.view(np.uint64))
        # RECOMPUTE_ALL scores every node whatever the list
        ref_act, ref_psi = M.feedback(mu=0.02, k_s=10, seed=9, round=4,
                                      mode=fl.FEEDBACK_RECOMPUTE_ALL,
                                      active=fl.Active.from_host(G, lists[1]), want_psi=True)
        din.put(lists[1])
        kept = M.feedback_noalloc(mu=0.02, k_s=10, seed=9, round=4, in_nodes_dev=din.ptr.value,
                                  count=lists[1].shape[0], out_nodes_dev=dout.ptr.value,
                                  out_cap=g.n, psi_dev=dpsi.ptr.value, psi_cap=g.n,
                                  mode=fl.FEEDBACK_RECOMPUTE_ALL)
        assert np.array_equal(dout.get(np.int32, kept), ref_act.read())
        assert np.array_equal(dpsi.get(np.float64, g.n).view(np.uint64), ref_psi.view(np.uint64))
        # an unsorted list and a list past the node range are rejected
        for bad in (np.array([3, 2, 9], np.int32), np.array([1, g.n], np.int32)):
            din.put(bad)
            with pytest.raises(fl.FelogError) as e:
                M.feedback_noalloc(mu=0.1, k_s=10, seed=9, round=0, in_nodes_dev=din.ptr.value,
                                   count=bad.shape[0], out_nodes_dev=dout.ptr.value, out_cap=g.n,
                                   psi_dev=dpsi.ptr.value, psi_cap=g.n)
            assert e.value.status == fl.FELOG_EINVAL
        # more nodes than the scratch covers: rejected before any device work
        with pytest.raises(fl.FelogError) as e:
            M.feedback_noalloc(mu=0.1, k_s=10, seed=9, round=0, in_nodes_dev=din.ptr.value,
                               count=(1 << 24) + 1, out_nodes_dev=dout.ptr.value,
                               out_cap=(1 << 24) + 1, psi_dev=dpsi.ptr.value, psi_cap=(1 << 24) + 1)
        assert e.value.status == fl.FELOG_EINVAL
        # small output buffers are rejected
        with pytest.raises(fl.FelogError):
            M.feedback_noalloc(mu=0.1, k_s=10, seed=9, round=0, in_nodes_dev=None, count=g.n,
                               out_nodes_dev=dout.ptr.value, out_cap=10, psi_dev=dpsi.ptr.value,
                               psi_cap=g.n)
    finally:
        din.free()
        dout.free()
        dpsi.free()
