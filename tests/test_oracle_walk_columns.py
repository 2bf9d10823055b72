"""The fact that lets a round's training schedule be planned before its walks
exist (walks beside training, Section 5.3 on one GPU): a walk has a second
node exactly when its start node has a neighbour.  Checked on the oracle's
walks, uniform and node2vec, including node2vec with an attempt cap so small
that proposals are taken capped."""
import numpy as np
import pytest

import synth
import oracle


def _ring_with_isolated():
    """A ring on nodes 0..11, then 7 isolated nodes."""
    e = np.array([[i, i + 1] for i in range(11)] + [[0, 11]], dtype=np.int64)
    return synth.csr_from_edges(19, e)


def _graphs():
    yield "ring+isolated", _ring_with_isolated()
    e = synth.rmat_edges(10, 1 << 12, seed=41)
    yield "rmat10 weighted", synth.csr_from_edges(1 << 10, e, synth.edge_weights(e.shape[0], 42))


def _check(walks, g, starts, r):
    assert np.array_equal(walks[:, 0], np.tile(starts, r))
    deg = np.diff(g.indptr)
    assert np.array_equal(walks[:, 1] >= 0, deg[walks[:, 0]] > 0)


@pytest.mark.parametrize("which", [0, 1])
def test_second_node_iff_start_has_neighbour(which):
    name, g = list(_graphs())[which]
    starts = np.arange(g.n, dtype=np.int32)
    _check(oracle.walks_uniform(g, starts, 3, 6, 5), g, starts, 3)
    for p, q in ((0.5, 2.0), (4.0, 0.25)):
        _check(oracle.walks_node2vec(g, starts, 3, 6, p, q, 7)[0], g, starts, 3)
    # an attempt cap of 1: proposals are taken capped, and the walk goes on
    w, capped = oracle.walks_node2vec(g, starts, 3, 6, 0.1, 10.0, 7, max_attempts=1)
    _check(w, g, starts, 3)
    if g.weights is not None:
        assert capped > 0
    sub = starts[::3]
    _check(oracle.walks_uniform(g, sub, 2, 4, 9, id_base=100), g, sub, 2)
