"""Host logic of the request loop (queueing, batching, admission, latency
statistics) with a stand-in engine: no GPU."""
import threading
import time

import numpy as np
import pytest

from paper_2412_06347_amd.serve import Server, AdmissionError, poisson_arrivals


class FakeEngine:
    """Stand-in for the GPU side: a part of a request needs as many outer
    cycles as the request has sources; a cycle takes 5 ms; a negative seed
    fails at completion."""

    def __init__(self, name, wl):
        self.name, self.V, self.resident = name, wl["V"], wl["resident"]
        self.lock = threading.Lock()

    def open_pool(self, nslots):
        self.nslots = nslots
        self.left = {}
        self.nid = 0
        self.in_use = 0
        self.max_in_use = 0

    def admit(self, parts):
        out = []
        for r, a, b in parts:
            self.nid += 1
            self.left[self.nid] = r.n_src
            self.in_use += 4 * (b - a)
            self.max_in_use = max(self.max_in_use, self.in_use)
            assert self.in_use <= self.nslots
            out.append(dict(req=r, a=a, b=b, pid=self.nid))
        return out

    def step(self):
        time.sleep(0.005)
        for pid in list(self.left):
            self.left[pid] -= 1
        return dict(self.left)

    def done(self, part, status):
        return status[part["pid"]] <= 0

    def finish(self, part):
        del self.left[part["pid"]]
        r = part["req"]
        self.in_use -= 4 * (part["b"] - part["a"])
        r.done_src += part["b"] - part["a"]
        if r.seed < 0:
            raise RuntimeError("failing request")
        if r.done_src < r.n_src:
            return None
        return dict(G=np.full(4, r.seed, dtype=float), n=r.n_src)


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
    # the right-hand sides in the pool never exceed the slot count, and
    # requests shared cycles
    assert all(e.max_in_use <= 16 and e.in_use == 0 for e in srv.engines.values())
    assert any(len(b) > 1 for b in srv.batches)


def test_request_joins_running_solve():
    """A short request submitted while a long one runs starts at the next
    cycle and finishes first (continuous batching, not batch at a time)."""
    srv = Server(hbm_budget=1e9, max_batch_rhs=32, engine_factory=FakeEngine, bytes_per_rhs=per_rhs)
    srv.add_ensemble("a", dict(V=1000, resident=1e6))
    srv.start()
    long = srv.submit("a", 6, 1)               # 24 right-hand sides, 6 cycles
    time.sleep(0.007)                          # inside its first or second cycle
    short = srv.submit("a", 1, 2)              # 4 right-hand sides, 1 cycle
    short.wait(5)
    long.wait(5)
    srv.stop()
    assert short.t_start < long.t_done and short.joined_running == 1
    assert short.t_done < long.t_done


def test_admission_by_hbm_budget():
    srv = Server(hbm_budget=1.0e6, max_batch_rhs=48, engine_factory=FakeEngine, bytes_per_rhs=per_rhs)
    # resident 0.5 MB, 10 kB per rhs -> at most 48 slots fit
    assert srv.add_ensemble("a", dict(V=1000, resident=5e5)) == 48
    # the second ensemble gets the slots that are left (0.02 MB -> none)
    with pytest.raises(AdmissionError):
        srv.add_ensemble("b", dict(V=1000, resident=4.8e5))


def test_request_larger_than_the_pool_runs_in_parts():
    srv = Server(hbm_budget=1e9, max_batch_rhs=8, engine_factory=FakeEngine, bytes_per_rhs=per_rhs)
    srv.add_ensemble("a", dict(V=1000, resident=1e6))
    srv.start()
    big = srv.submit("a", 5, 4)               # 20 right-hand sides, 8 slots: three parts
    small = srv.submit("a", 1, 5)
    assert big.wait(5)["n"] == 5 and small.wait(5)["n"] == 1
    srv.stop()
    eng = srv.engines["a"]
    assert eng.max_in_use <= 8 and eng.in_use == 0


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
