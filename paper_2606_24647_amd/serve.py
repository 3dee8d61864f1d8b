"""Serving loop: continuous batching of analytical queries over device-resident tables.

The paper keeps the working set in GPU memory for the whole query (Section 2,
hypothesis 2), lets pipelines run concurrently on their own streams with
synchronisation only at pipeline boundaries (Section 3), and blocks senders
when queues exceed thresholds because the working set must fit in GPU memory
(Section 3.3).  This module applies the same ideas to a request loop:

* tables stay resident in HBM; queries only read them;
* a single host thread drives everything asynchronously: it admits arriving
  queries as soon as a slot (a stream with its own library context) and the
  HBM budget allow, enqueues their kernels, and polls completion events;
* each query is a small state machine (for example filter, then partition the
  filtered rows once their count is known), advanced when its stage's event
  completes, so no query ever blocks the loop;
* queries that arrive while others run are admitted between their stages:
  their work overlaps on the device;
* over-budget queries wait in FIFO order; nothing is spilled.

"plain" mode runs the same queries one at a time, in arrival order, on one
stream: the baseline that serving must beat on throughput at a given p99.

The scheduler is written against a small executor interface so that it can be
tested on the CPU with a simulated executor (tests/test_serve.py).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

# Resident fact columns: fkey, qty, price, disc, date, flag, status.
F_FKEY, F_QTY, F_PRICE, F_DISC, F_DATE, F_FLAG, F_STATUS = range(7)
# Resident dimension columns: pkey, date, ckey.
D_PKEY, D_DATE, D_CKEY = range(3)

REV = [("col", F_PRICE), ("k-col", 100, F_DISC)]
AGG_AGGS = [("sum", [("col", F_QTY)]), ("sum", [("col", F_PRICE)]), ("sum", [("col", F_DISC)]), ("sum", REV),
            ("count*",)]
JOIN_AGGS = [("sum", REV), ("count*",)]
PART_COLS = [F_FKEY, F_PRICE, F_DATE, F_FLAG]   # 8 + 8 + 4 + 1 = 21 B per row


# Radix group-join sizing of the library (a build side of at least 2^20 rows
# is partitioned into 2^k regions of about 3,500 rows, k in 8..12; partition
# tiles of 4,096 to 32,768 rows, about 2,048 of them), used to bound a join
# query's memory.
RADIX_MIN_BUILD = 1 << 20


def radix_regions(build_rows: int) -> int:
    k = 8
    while k < 12 and (1 << k) * 3500 < build_rows:
        k += 1
    return 1 << k


def radix_tiles(rows: int) -> int:
    t = 4096
    while t < 32768 and t * 2048 < rows:
        t *= 2
    return rows // t + 1


@dataclass
class Query:
    qid: int
    kind: str            # "agg", "join" or "part"
    arrival: float       # seconds after the start of the run
    params: dict = field(default_factory=dict)


def make_workload(n: int, qps: float, seed: int = 5, kinds=("agg", "join", "part")) -> list:
    """Open-loop Poisson arrivals at `qps`, kinds uniform, random filter bounds."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind == "agg":
            p = {"b": int(rng.integers(0, 2556))}
        elif kind == "join":
            p = {"b_dim": int(rng.integers(0, 2406)), "b_fact": int(rng.integers(0, 2556))}
        else:
            p = {"b": int(rng.integers(0, 2556)), "P": int(rng.choice([64, 256]))}
        out.append(Query(i, kind, float(t[i]), p))
    return out


# ---------------------------------------------------------------------------
# Scheduler
# ---------------------------------------------------------------------------

@dataclass
class Record:
    qid: int
    kind: str
    arrival: float
    admitted: float
    done: float
    rows: int
    result: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """Admission by slots and HBM budget, FIFO queue, non-blocking polling.

    executor: object with nslots, footprint(q) -> bytes, start(q, slot) -> job,
    step(job) -> bool (advance the job's state machine if its current stage has
    finished; True once the query is complete), result(job), rows(q).
    """

    def __init__(self, executor, budget_bytes: int, nslots: int | None = None, clock=time.perf_counter,
                 idle_sleep: float = 20e-6):
        self.ex = executor
        self.budget = budget_bytes
        self.nslots = nslots if nslots is not None else executor.nslots
        self.clock = clock
        self.idle_sleep = idle_sleep

    def run(self, queries: list, keep_results: bool = False) -> list:
        pending = sorted(queries, key=lambda q: q.arrival)
        queue: list = []
        running: dict = {}      # slot -> (query, job, admitted, footprint)
        free = list(range(self.nslots))
        used = 0
        records = []
        i = 0
        t0 = self.clock()
        while i < len(pending) or queue or running:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            # Admit in FIFO order while a slot and the budget allow.  A query that
            # can share its scan takes queued queries of the same kind along
            # (shared scan), up to the executor's limit.  With an executor that
            # marks queries heavy (each one alone fills the device), at most
            # max_heavy of them run at once: while that many do, the first light
            # query in the queue is admitted instead (heavy ones stay FIFO).
            max_heavy = getattr(self.ex, "max_heavy", None)
            while queue and free:
                q = queue[0]
                if max_heavy is not None and self.ex.heavy(q):
                    nheavy = sum(1 for grp, _, _, _ in running.values() if self.ex.heavy(grp[0]))
                    if nheavy >= max_heavy:
                        light = next((x for x in queue if not self.ex.heavy(x)), None)
                        if light is None:
                            break
                        q = light
                fp = self.ex.footprint(q)
                if fp > self.budget:
                    raise ValueError(f"query {q.qid} needs {fp} bytes, more than the whole budget")
                if used + fp > self.budget:
                    break
                group = [q]
                key = self.ex.share_key(q) if hasattr(self.ex, "share_key") else None
                if key is not None:
                    for other in queue:
                        if other is q:
                            continue
                        limit = self.ex.share_limit(q) if hasattr(self.ex, "share_limit") else self.ex.max_share
                        if len(group) >= limit:
                            break
                        if self.ex.share_key(other) == key and used + fp + self.ex.footprint(other) <= self.budget:
                            group.append(other)
                            fp += self.ex.footprint(other)
                for g in group:
                    queue.remove(g)
                slot = free.pop(0)
                used += fp
                job = self.ex.start(q, slot) if len(group) == 1 else self.ex.start_group(group, slot)
                running[slot] = (group, job, self.clock() - t0, fp)
            # Advance running queries.
            progressed = False
            for slot in list(running):
                group, job, adm, fp = running[slot]
                if self.ex.step(job):
                    done = self.clock() - t0
                    for j, q in enumerate(group):
                        res = None
                        if keep_results:
                            res = self.ex.result(job) if len(group) == 1 else self.ex.result_of(job, j)
                        records.append(Record(q.qid, q.kind, q.arrival, adm, done, self.ex.rows(q), res))
                    del running[slot]
                    free.append(slot)
                    free.sort()
                    used -= fp
                    progressed = True
            if not progressed and self.idle_sleep:
                if i < len(pending) and not queue and not running:
                    wait = pending[i].arrival - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                else:
                    time.sleep(self.idle_sleep)
        return records


def summarize(records: list, wall: float | None = None) -> dict:
    if not records:
        return {"queries": 0}
    lat = np.array([r.latency for r in records]) * 1e3
    first = min(r.arrival for r in records)
    last = max(r.done for r in records)
    span = wall if wall is not None else (last - first)
    rows = sum(r.rows for r in records)
    out = {"queries": len(records), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "rows_per_s": rows / span if span > 0 else float("nan"),
           "wall_s": span}
    for kind in sorted({r.kind for r in records}):
        kl = np.array([r.latency for r in records if r.kind == kind]) * 1e3
        out[f"{kind}_p50_ms"] = float(np.percentile(kl, 50))
        out[f"{kind}_p99_ms"] = float(np.percentile(kl, 99))
    return out


# ---------------------------------------------------------------------------
# Device executor (the real one)
# ---------------------------------------------------------------------------

class DeviceExecutor:
    """Runs queries on a pool of streams, one library context per stream."""

    def __init__(self, gq, torch, fact, dim, nslots: int = 4, share: bool = True, max_heavy: int | None = None):
        self.gq, self.torch = gq, torch
        self.fact, self.dim = fact, dim
        self.nslots = nslots
        self.share = share
        self.max_share = 8        # aggregation queries sharing one scan
        self.max_share_join = 3   # join queries sharing one fact partition: all of a group complete together
        if max_heavy is not None:
            self.max_heavy = max_heavy
        self.streams = [torch.cuda.Stream() for _ in range(nslots)]
        self.ctxs = [gq.Context(allocator="torch") for _ in range(nslots)]
        self.nf, self.nd = fact.nrows, dim.nrows

    # Upper bounds of the device memory a query allocates (tables, outputs, workspaces).
    def footprint(self, q: Query) -> int:
        if q.kind == "agg":
            return 64 << 20
        if q.kind == "join":
            out = self.nd * 24 + (self.nd // 8 + 64) * 2      # key, sum, count per group; bitmaps
            if self.nd >= RADIX_MIN_BUILD:
                # Radix group-join: the build side's (hash, row) pairs and its
                # per-(tile, region) counts, starts and chunk sums; the probe
                # side's (hash, value) tuples at 16 B per fact row, twice (the
                # first level's slots and the final regions), the same count
                # arrays and the first level's run offsets; work items.  (Joins
                # sharing one fact partition have 24-byte tuples, once for the
                # group: the sum of their footprints bounds it.)
                P = radix_regions(self.nd)
                tf, td = radix_tiles(self.nf), radix_tiles(self.nd)
                build = self.nd * 16 + td * P * 4 * 3 + P * 8
                probe = self.nf * 32 + tf * P * 4 * 3 + (self.nf // 1024 + 1) * 66 + (P + self.nd) * 8
                return build + probe + out + (64 << 20)
            cap = 2 * self.nd + 1       # load factor 0.5 over every dimension row
            # keys, meta, 2 accumulators, run cursors per slot; rows and merge
            # buffer per build row; the output at one group per build row.
            return cap * (8 + 8 + 16 + 4) + self.nd * 8 + out + (64 << 20)
        # filter output and partition output at 21 B per row, plus workspace
        return 2 * self.nf * 21 + (self.nf // 4096 + 1) * 256 * 12 + (256 << 20)

    @staticmethod
    def heavy(q: Query) -> bool:
        """Joins and partitions each fill the device; aggregations are short."""
        return q.kind != "agg"

    def rows(self, q: Query) -> int:
        return self.nf + (self.nd if q.kind == "join" else 0)

    def share_key(self, q: Query):
        """Aggregation queries over the fact table share one scan; join queries
        (radix group-joins against the dimension) share the fact side's
        partition, each applying its own date range to the date carried in
        the partitioned tuples."""
        if not self.share:
            return None
        if q.kind == "agg":
            return "agg"
        if q.kind == "join" and self.nd >= RADIX_MIN_BUILD:
            return "join"
        return None

    def share_limit(self, q: Query) -> int:
        return self.max_share_join if q.kind == "join" else self.max_share

    def start_group(self, qs: list, slot: int):
        s, ctx = self.streams[slot], self.ctxs[slot]
        job = {"qs": qs, "slot": slot, "stage": 9, "q": qs[0]}
        with self.torch.cuda.stream(s):
            if qs[0].kind == "join":
                tables = [ctx.join_build(self.dim, [D_PKEY], [("range", D_DATE, 0, q.params["b_dim"])], stream=s)
                          for q in qs]
                res = ctx.pipeline_shared(self.fact, [], F_FKEY, JOIN_AGGS, tables,
                                          [("range", F_DATE, q.params["b_fact"], 2555) for q in qs],
                                          capacity=self.nd, stream=s)
                for jt in tables:
                    jt.free(stream=s)
                job.update(outs=[o for o, _ in res], cnts=[c for _, c in res])
            else:
                outs, cnt = ctx.groupby_shared(self.fact, [F_FLAG, F_STATUS],
                                               [[("range", F_DATE, 0, q.params["b"])] for q in qs], AGG_AGGS,
                                               capacity=16, expected_groups=6, stream=s)
                job.update(outs=outs, cnts=[cnt[j:j + 1] for j in range(len(qs))])
            job["ev"] = self._event(s)
        return job

    def result_of(self, job, j: int):
        self.ctxs[job["slot"]].raise_status(stream=self.streams[job["slot"]])
        n = int(job["cnts"][j].item())
        return ("groups", self.gq.read_table(job["outs"][j], n))

    def _event(self, s):
        e = self.torch.cuda.Event()
        e.record(s)
        return e

    def start(self, q: Query, slot: int):
        s, ctx = self.streams[slot], self.ctxs[slot]
        job = {"q": q, "slot": slot, "stage": 0, "keep": []}
        with self.torch.cuda.stream(s):
            if q.kind == "agg":
                out, cnt = ctx.groupby_agg(self.fact, [F_FLAG, F_STATUS], [("range", F_DATE, 0, q.params["b"])],
                                           AGG_AGGS, capacity=16, strategy="lds", expected_groups=6, stream=s)
                job.update(out=out, cnt=cnt, stage=9)
            elif q.kind == "join":
                jt = ctx.join_build(self.dim, [D_PKEY], [("range", D_DATE, 0, q.params["b_dim"])], acc_slots=2,
                                    stream=s)
                out, cnt = ctx.pipeline(self.fact, [("range", F_DATE, q.params["b_fact"], 2555)], [F_FKEY],
                                        JOIN_AGGS, join=jt, probe_key=F_FKEY, capacity=self.nd, stream=s)
                jt.free(stream=s)
                job.update(out=out, cnt=cnt, stage=9)
            else:
                fout, fcnt = ctx.filter(self.fact, [("range", F_DATE, 0, q.params["b"])], PART_COLS, stream=s)
                job.update(fout=fout, fcnt=fcnt, stage=1)
            job["ev"] = self._event(s)
        return job

    def step(self, job) -> bool:
        if not job["ev"].query():
            return False
        if job["stage"] == 9:
            return True
        # Partition query: the filter finished, so its row count can be read
        # without waiting; partition the filtered rows.
        s, ctx = self.streams[job["slot"]], self.ctxs[job["slot"]]
        n = int(job["fcnt"].item())
        fout = job["fout"]
        for c in fout.cols:
            c.length = n
        with self.torch.cuda.stream(s):
            out, offs = ctx.hash_partition(fout, [0], job["q"].params["P"], stream=s)
            job.update(out=out, offs=offs, stage=9, n=n)
            job["ev"] = self._event(s)
        return False

    def result(self, job):
        """Host copy of the query's result, for checking (small runs only)."""
        gq = self.gq
        q = job["q"]
        ctx = self.ctxs[job["slot"]]
        ctx.raise_status(stream=self.streams[job["slot"]])
        if q.kind in ("agg", "join"):
            n = int(job["cnt"].item())
            return ("groups", gq.read_table(job["out"], n))
        n = job["n"]
        return ("partition", job["offs"].cpu().numpy(), gq.read_table(job["out"], n))


def canonical(result):
    """Order-independent form of a group result (partition results are already canonical)."""
    if result[0] != "groups":
        return result
    cols = result[1]
    if not cols or len(cols[0][0]) == 0:
        return ("groups", [])
    keys = np.stack([c[0].astype(np.int64) for c in cols], axis=1)
    order = np.lexsort(keys.T[::-1])
    return ("groups", keys[order])


def same_result(a, b) -> bool:
    a, b = canonical(a), canonical(b)
    if a[0] != b[0]:
        return False
    if a[0] == "groups":
        return np.array_equal(a[1], b[1]) if len(a[1]) or len(b[1]) else True
    if not np.array_equal(a[1], b[1]):
        return False
    return all(np.array_equal(x[0], y[0]) for x, y in zip(a[2], b[2]))
