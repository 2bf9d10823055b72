import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


def link_auc_of(emb, split) -> float:
    """Link-prediction AUC of embeddings produced by the library, by sklearn
    (scores phi(u).phi(v) of held-out edges against non-edges), so that no
    oracle function ever takes the library's output as its input."""
    import numpy as np
    from sklearn.metrics import roc_auc_score
    e = emb.astype(np.float64)
    pos, neg = split.test_pos, split.test_neg
    sp = np.einsum("ij,ij->i", e[pos[:, 0]], e[pos[:, 1]])
    sn = np.einsum("ij,ij->i", e[neg[:, 0]], e[neg[:, 1]])
    y = np.r_[np.ones(sp.shape[0]), np.zeros(sn.shape[0])]
    return float(roc_auc_score(y, np.r_[sp, sn]))
