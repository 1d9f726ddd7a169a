"""Host logic of the solve server, without a GPU: the latency percentile
(against NumPy's linear interpolation), and admission by device bytes --
engines are created while the budget allows, idle engines are evicted least
recently used first, busy engines never are, and a request whose engine
does not fit waits."""
import contextlib
import types

import numpy as np
import pytest

from paper_1512_04629_amd import amg
from paper_1512_04629_amd import serve


def test_percentile_matches_numpy_linear():
    rng = np.random.default_rng(3)
    for n in (1, 2, 7, 100):
        v = rng.exponential(size=n).tolist()
        for q in (0, 1, 50, 90, 99, 100):
            assert serve.percentile(v, q) == pytest.approx(np.percentile(v, q, method="linear"), rel=1e-15)
    assert np.isnan(serve.percentile([], 50))


class FakeEngine:
    def __init__(self, owner):
        self.owner = owner
        self.state = [amg.Batch.FREE] * 4
        self.closed = False

    def states(self):
        return self.state

    def close(self):
        self.closed = True
        self.owner.engine_bytes -= self.owner.eng


class FakeHierarchy:
    """Resident bytes `base`, plus `eng` while an engine exists."""

    def __init__(self, base, eng):
        self.base, self.eng, self.engine_bytes = base, eng, 0

    def device_bytes(self):
        return self.base + self.engine_bytes

    def batch_bytes(self, slots, precision):
        return self.eng

    def batch(self, slots, precision, tol, maxit, graphs):
        self.engine_bytes += self.eng
        return FakeEngine(self)


@pytest.fixture(autouse=True)
def no_device(monkeypatch):
    """The library refuses to run without a ROCm GPU; these tests drive only
    the scheduler, so its stream contexts become no-ops."""
    fake = types.SimpleNamespace(cuda=types.SimpleNamespace(stream=lambda s: contextlib.nullcontext()))
    monkeypatch.setattr(amg, "_torch", lambda: fake)


def _server(budget, hiers):
    s = serve.SolveServer.__new__(serve.SolveServer)
    s.slots, s.precision, s.tol, s.maxit, s.graphs = 4, 32, 1e-10, 100, False
    s.budget = budget
    s.hier = hiers
    s.streams = {k: None for k in hiers}
    s.engines, s.last_used = {}, {}
    s.stats = serve.ServeStats()
    return s


def test_admission_by_bytes_evicts_idle_engines_lru_first():
    hs = {k: FakeHierarchy(100, 50) for k in ("a", "b", "c")}
    s = _server(400, hs)              # three hierarchies (300 B) and at most two engines
    ea, eb = s._admit("a"), s._admit("b")
    assert ea is not None and eb is not None and s.stats.engines_created == 2
    assert s._admit("a") is ea        # an existing engine is reused
    ec = s._admit("c")                # evicts the least recently used idle engine: a
    assert ec is not None and ea.closed and not eb.closed
    assert set(s.engines) == {"b", "c"} and s.stats.engines_evicted == 1
    assert s.device_bytes() <= s.budget and s.stats.peak_bytes == 400


def test_busy_engines_are_not_evicted_and_requests_wait():
    hs = {k: FakeHierarchy(100, 50) for k in ("a", "b", "c")}
    s = _server(400, hs)
    ea, eb = s._admit("a"), s._admit("b")
    ea.state[1] = amg.Batch.ITERATING
    eb.state[0] = amg.Batch.SUBMITTED
    assert s._admit("c") is None
    assert s.stats.waits_for_budget == 1 and s.stats.engines_evicted == 0
    assert not ea.closed and not eb.closed
    eb.state[0] = amg.Batch.FREE      # b goes idle: c can now take its place
    assert s._admit("c") is not None and eb.closed and not ea.closed
