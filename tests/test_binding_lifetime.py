"""Handle lifetime in the Python binding, on the CPU with a stand-in library:
a context closed (or finalised) while objects made on it are alive is
destroyed only after the last of them, since the C library needs a context's
objects destroyed first."""
import gc

import pytest

from paper_2606_22180_amd import felog


class _FakeLib:
    def __init__(self):
        self.calls = []

    def felog_ctx_destroy(self, h):
        self.calls.append(("ctx", h))

    def felog_graph_destroy(self, h):
        self.calls.append(("graph", h))

    def felog_model_destroy(self, h):
        self.calls.append(("model", h))


@pytest.fixture
def fake(monkeypatch):
    lib = _FakeLib()
    monkeypatch.setattr(felog, "load", lambda: lib)
    return lib


def _ctx(handle):
    c = felog.Context.__new__(felog.Context)      # no device: set the fields by hand
    c.handle, c._live, c._close_pending = handle, 0, False
    return c


def test_context_waits_for_its_objects(fake):
    c = _ctx(1)
    g = felog.Graph(2, c)
    m = felog.Model(3, g)
    c.close()
    assert fake.calls == [] and c.handle == 1       # deferred: two objects alive
    m.close()
    assert fake.calls == [("model", 3)]
    g.close()
    assert fake.calls == [("model", 3), ("graph", 2), ("ctx", 1)]
    assert c.handle is None
    c.close()                                       # a second close is a no-op
    assert len(fake.calls) == 3


def test_cycle_finalised_in_any_order(fake):
    c = _ctx(7)
    g = felog.Graph(8, c)
    m = felog.Model(9, g)
    cycle = [c, g, m]
    cycle.append(cycle)
    del c, g, m, cycle
    gc.collect()
    names = [k for k, _ in fake.calls]
    assert sorted(names) == ["ctx", "graph", "model"]
    assert names[-1] == "ctx"                       # the context goes last


def test_close_without_objects_is_immediate(fake):
    c = _ctx(5)
    c.close()
    assert fake.calls == [("ctx", 5)] and c.handle is None
