"""Host logic of the request loop (queueing, batching, admission, latency
statistics) with a stand-in engine: no GPU."""
import threading
import time

import numpy as np
import pytest

from paper_2412_06347_amd.serve import Server, AdmissionError, poisson_arrivals


class FakeEngine:
    def __init__(self, name, wl):
        self.name, self.V, self.resident = name, wl["V"], wl["resident"]
        self.calls = []
        self.lock = threading.Lock()

    def run(self, reqs):
        with self.lock:
            self.calls.append([r.rid for r in reqs])
        time.sleep(0.02)
        if any(r.seed < 0 for r in reqs):
            raise RuntimeError("failing batch")
        return [dict(G=np.full(4, r.seed, dtype=float), n=r.n_src) for r in reqs]


def per_rhs(V):
    return V * 10.0


def test_batching_and_stats():
    srv = Server(hbm_budget=1e9, max_batch_rhs=16, engine_factory=FakeEngine, bytes_per_rhs=per_rhs)
    assert srv.add_ensemble("a", dict(V=1000, resident=1e6)) == 16
    assert srv.add_ensemble("b", dict(V=2000, resident=1e6)) == 16
    srv.start()
    reqs = [srv.submit("a" if i % 3 else "b", 1 + i % 2, i) for i in range(20)]
    for r in reqs:
        res = r.wait(10)
        assert res["G"][0] == r.seed          # each request gets its own result
    srv.stop()
    st = srv.stats()
    assert st["n"] == 20 and st["solves"] == sum(r.nrhs for r in reqs)
    assert 0 < st["p50_s"] <= st["p99_s"]
    # batches never exceed the slot count and queued requests joined batches
    for b in srv.batches:
        assert sum(next(r for r in reqs if r.rid == i).nrhs for i in b) <= 16
    assert len(srv.batches) < 20


def test_admission_by_hbm_budget():
    srv = Server(hbm_budget=1.0e6, max_batch_rhs=48, engine_factory=FakeEngine, bytes_per_rhs=per_rhs)
    # resident 0.5 MB, 10 kB per rhs -> at most 48 slots fit
    assert srv.add_ensemble("a", dict(V=1000, resident=5e5)) == 48
    # the second ensemble gets the slots that are left (0.02 MB -> none)
    with pytest.raises(AdmissionError):
        srv.add_ensemble("b", dict(V=1000, resident=4.8e5))
    with pytest.raises(AdmissionError):
        srv.submit("a", 13, 1)                # 52 right-hand sides > 48 slots


def test_failure_is_per_request():
    srv = Server(hbm_budget=1e9, max_batch_rhs=4, engine_factory=FakeEngine, bytes_per_rhs=per_rhs)
    srv.add_ensemble("a", dict(V=10, resident=1))
    srv.start()
    bad = srv.submit("a", 1, -1)
    good = srv.submit("a", 1, 3)
    with pytest.raises(RuntimeError):
        bad.wait(5)
    assert good.wait(5)["G"][0] == 3
    srv.stop()


def test_poisson_arrivals_seeded():
    a = poisson_arrivals(100, 5.0, 7)
    assert np.all(np.diff(a) > 0) and np.array_equal(a, poisson_arrivals(100, 5.0, 7))
    assert abs(100 / a[-1] - 5.0) < 2.0
