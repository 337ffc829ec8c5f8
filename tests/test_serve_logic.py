"""Host logic of the serving loop (serve.py) on the CPU, with a stand-in for
the library: FIFO admission, the byte budget, window accounting and the
records.  The stand-in advances each resident replica by min(K, steps left)
per window, as dpd_batch_advance does."""
import numpy as np
import pytest

from paper_1804_06205_amd import serve
from paper_1804_06205_amd import workloads as W


class FakeSystem:
    live = 0

    def __init__(self, n, bytes_):
        self.n, self.bytes, self.t, self.closed = n, bytes_, 0, False
        FakeSystem.live += 1

    def step(self, k):
        self.t += k

    def sync(self):
        pass

    def close(self):
        if not self.closed:
            self.closed = True
            FakeSystem.live -= 1

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class FakeBatch:
    instances = []

    def __init__(self, budget, max_replicas, stream=None, variant=-1):
        self.budget, self.max = budget, max_replicas
        self.slots, self.used, self.peak, self.windows, self.order = {}, 0, 0, 0, []
        FakeBatch.instances.append(self)

    def admit(self, sysm, nsteps):
        if self.used + sysm.bytes > self.budget or len(self.slots) >= self.max:
            raise RuntimeError("EBUSY")
        slot = min(set(range(self.max)) - set(self.slots))
        self.slots[slot] = [sysm, sysm.t + nsteps, False]
        self.used += sysm.bytes
        self.peak = max(self.peak, self.used)
        self.order.append(sysm.rid)
        return slot

    def advance(self, K):
        self.windows += 1
        for s in self.slots.values():
            s[0].t = min(s[0].t + K, s[1])

    def autotune(self, K):
        self.advance(K)
        return 1, 0.01

    def poll(self):
        done = []
        for k, s in self.slots.items():
            if s[0].t >= s[1] and not s[2]:
                s[2] = True
                done.append(k)
        return done

    def retire(self, slot):
        sysm = self.slots.pop(slot)[0]
        self.used -= sysm.bytes
        return sysm

    def info(self):
        return {"resident": len(self.slots), "bytes_used": self.used, "budget": self.budget,
                "captures": 1, "windows": self.windows, "variant": 1}

    def close(self):
        pass


class FakeDPD:
    Batch = FakeBatch

    class System:
        @staticmethod
        def from_workload(w, cell_capacity=0):
            s = FakeSystem(w.n, 1000 * w.L)
            s.rid = w.rid
            return s

    @staticmethod
    def footprint_bytes(L, n, nb, precision, cell_capacity):
        return 1000 * L


class FakeWorkload:
    def __init__(self, req):
        self.rid, self.L, self.n, self.nbonds, self.precision = req.rid, req.L, 3 * req.L ** 3, 0, "mixed"


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(serve, "dpd", FakeDPD)
    FakeBatch.instances.clear()
    FakeSystem.live = 0
    yield


def test_fifo_admission_under_budget_and_all_complete(fake):
    reqs = W.replica_stream(nreq=40, rate=1e6, seed=3, steps_range=(10, 300))
    budget = 3 * 1000 * 12          # at most three of the largest boxes at once
    recs, summ = serve.serve_batched(reqs, budget, window=25, make=FakeWorkload, realtime=False)
    b = FakeBatch.instances[0]
    assert [r.rid for r in recs] == [q.rid for q in reqs]
    assert b.order == [q.rid for q in reqs]             # admitted first come first served
    assert b.peak <= budget and b.peak > 2 * 1000 * 6   # the budget binds and holds
    assert all(np.isfinite(r.done) and r.done >= r.admitted for r in recs)
    assert summ["requests"] == 40
    assert summ["particle_steps"] == sum(3 * q.L ** 3 * q.steps for q in reqs)
    assert FakeSystem.live == 0                         # every system freed


def test_autotune_runs_once_when_the_batch_fills(fake):
    reqs = W.replica_stream(nreq=12, rate=1e6, seed=5, steps_range=(200, 400))
    recs, summ = serve.serve_batched(reqs, 10 ** 9, window=50, make=FakeWorkload,
                                     realtime=False, autotune_at=8, autotune_window=20)
    assert summ["autotuned"]["variant"] == 1
    assert len(recs) == 12 and all(np.isfinite(r.done) for r in recs)


def test_windows_cover_the_longest_request(fake):
    reqs = [W.Request(k, 0.0, 6, 10, s, 1000 + k) for k, s in enumerate((7, 50, 120))]
    recs, summ = serve.serve_batched(reqs, 10 ** 9, window=20, make=FakeWorkload, realtime=False)
    assert summ["windows"] == 6                          # ceil(120 / 20)
    assert [r.steps for r in recs] == [7, 50, 120]


def test_one_at_a_time_steps_each_request_once(fake):
    reqs = W.replica_stream(nreq=5, rate=1e6, seed=4, steps_range=(10, 20))
    recs, summ = serve.serve_one_at_a_time(reqs, make=FakeWorkload, realtime=False)
    assert [r.rid for r in recs] == [q.rid for q in reqs]
    assert summ["replica_steps_per_s"] > 0 and FakeSystem.live == 0
