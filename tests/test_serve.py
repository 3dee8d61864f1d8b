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


class SharingExecutor(FakeExecutor):
    max_share = 8

    def share_key(self, q):
        return "agg" if q.kind == "agg" else None

    def start_group(self, qs, slot):
        self.groups = getattr(self, "groups", []) + [[q.qid for q in qs]]
        job = self.start(qs[0], slot)
        for q in qs[1:]:
            self.in_use += self.FOOT[q.kind]
        job["extra"] = qs[1:]
        return job

    def step(self, job):
        was = job["done"]
        done = super().step(job)
        if done and not was:
            for q in job.get("extra", []):
                self.in_use -= self.FOOT[q.kind]
        return done

    def result_of(self, job, j):
        return "shared"


def test_shared_scans_group_waiting_aggregations():
    clock = VirtualClock()
    ex = SharingExecutor(clock, 1)
    qs = [Query(i, "agg" if i % 3 else "join", 0.001 * i, {"b": 5}) for i in range(30)]
    recs = Scheduler(ex, 100, clock=clock, idle_sleep=0).run(qs, keep_results=True)
    assert sorted(r.qid for r in recs) == list(range(30))
    groups = getattr(ex, "groups", [])
    assert groups and max(len(g) for g in groups) > 1
    assert all(len(g) <= 8 for g in groups)
    for g in groups:                                   # only aggregation queries share
        assert all(i % 3 for i in g)
    assert ex.in_use == 0


class CappedExecutor(FakeExecutor):
    """Joins and partitions are heavy; at most max_heavy of them run at once."""

    def __init__(self, clock, nslots, max_heavy):
        super().__init__(clock, nslots)
        self.max_heavy = max_heavy
        self.heavy_now = 0
        self.max_heavy_seen = 0
        self.heavy_starts = []

    @staticmethod
    def heavy(q):
        return q.kind != "agg"

    def start(self, q, slot):
        job = super().start(q, slot)
        if self.heavy(q):
            self.heavy_now += 1
            self.max_heavy_seen = max(self.max_heavy_seen, self.heavy_now)
            self.heavy_starts.append(q.qid)
        return job

    def step(self, job):
        was = job["done"]
        done = super().step(job)
        if done and not was and self.heavy(job["q"]):
            self.heavy_now -= 1
        return done


@pytest.mark.parametrize("max_heavy", [1, 2])
def test_heavy_cap_light_queries_overtake(max_heavy):
    clock = VirtualClock()
    ex = CappedExecutor(clock, 4, max_heavy)
    qs = make_workload(300, 150, seed=3)
    recs = Scheduler(ex, 1000, clock=clock, idle_sleep=0).run(qs, keep_results=True)
    assert sorted(r.qid for r in recs) == [q.qid for q in qs]
    assert all(r.result == r.qid for r in recs)
    assert ex.max_heavy_seen == max_heavy                # the cap binds and holds
    assert ex.heavy_starts == sorted(ex.heavy_starts)    # heavy queries stay in arrival order
    assert ex.starts != sorted(ex.starts)                # some light query went ahead
    assert ex.max_active <= 4


def test_heavy_cap_lowers_light_latency():
    def light_p99(ex):
        qs = make_workload(300, 150, seed=3)
        recs = Scheduler(ex, 1000, clock=ex.clock, idle_sleep=0).run(qs)
        return summarize([r for r in recs if r.kind == "agg"])["p99_ms"]
    free = light_p99(FakeExecutor(VirtualClock(), 2))
    capped = light_p99(CappedExecutor(VirtualClock(), 2, 1))
    assert capped < free
