"""Serving scheduler logic on the CPU with a simulated executor (no GPU)."""
import pytest

from paper_2606_24647_amd.serve import Query, Scheduler, make_workload, summarize


class VirtualClock:
    def __init__(self, tick=1e-4):
        self.t = 0.0
        self.tick = tick

    def __call__(self):
        self.t += self.tick
        return self.t


class FakeExecutor:
    """Each query takes a fixed service time from its start; footprints per kind."""

    SERVICE = {"agg": 0.004, "join": 0.030, "part": 0.020}
    FOOT = {"agg": 1, "join": 10, "part": 25}

    def __init__(self, clock, nslots):
        self.clock, self.nslots = clock, nslots
        self.in_use = 0
        self.max_in_use = 0
        self.active = 0
        self.max_active = 0
        self.starts = []

    def footprint(self, q):
        return self.FOOT[q.kind]

    def rows(self, q):
        return 100

    def start(self, q, slot):
        self.in_use += self.FOOT[q.kind]
        self.max_in_use = max(self.max_in_use, self.in_use)
        self.active += 1
        self.max_active = max(self.max_active, self.active)
        self.starts.append(q.qid)
        return {"q": q, "end": self.clock.t + self.SERVICE[q.kind], "done": False}

    def step(self, job):
        if not job["done"] and self.clock.t >= job["end"]:
            job["done"] = True
            self.in_use -= self.FOOT[job["q"].kind]
            self.active -= 1
        return job["done"]

    def result(self, job):
        return job["q"].qid


def run(qps, nslots, budget, n=300):
    clock = VirtualClock()
    ex = FakeExecutor(clock, nslots)
    qs = make_workload(n, qps, seed=1)
    recs = Scheduler(ex, budget, clock=clock, idle_sleep=0).run(qs, keep_results=True)
    return ex, qs, recs


def test_all_complete_fifo_and_limits():
    ex, qs, recs = run(qps=200, nslots=4, budget=40)
    assert sorted(r.qid for r in recs) == [q.qid for q in qs]
    assert ex.starts == sorted(ex.starts)                 # admitted in arrival order
    assert ex.max_active <= 4 and ex.max_in_use <= 40
    for r in recs:
        assert r.admitted >= r.arrival - 1e-9
        assert r.latency >= FakeExecutor.SERVICE[r.kind] - 1e-9
        assert r.result == r.qid


def test_budget_blocks_admission():
    ex, qs, recs = run(qps=500, nslots=8, budget=26)
    assert ex.max_in_use <= 26                           # two partition queries never overlap
    assert ex.max_active <= 8


def test_served_beats_plain_under_load():
    _, _, served = run(qps=120, nslots=4, budget=1000)
    _, _, plain = run(qps=120, nslots=1, budget=1000)
    s, p = summarize(served), summarize(plain)
    assert s["p99_ms"] < p["p99_ms"]
    assert s["rows_per_s"] >= p["rows_per_s"]


def test_over_budget_query_is_rejected():
    clock = VirtualClock()
    ex = FakeExecutor(clock, 2)
    with pytest.raises(ValueError):
        Scheduler(ex, 5, clock=clock, idle_sleep=0).run([Query(0, "part", 0.0, {"b": 1, "P": 64})])


def test_workload_is_seeded_poisson():
    a = make_workload(2000, 50.0, seed=5)
    b = make_workload(2000, 50.0, seed=5)
    assert [(q.kind, q.arrival, q.params) for q in a] == [(q.kind, q.arrival, q.params) for q in b]
    gaps = [y.arrival - x.arrival for x, y in zip(a, a[1:])]
    mean = sum(gaps) / len(gaps)
    assert abs(mean - 1 / 50.0) < 0.002
    kinds = {k: sum(q.kind == k for q in a) for k in ("agg", "join", "part")}
    assert all(500 < v < 830 for v in kinds.values())
