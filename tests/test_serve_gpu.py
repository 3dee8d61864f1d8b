"""Serving on the GPU: every query's result is the same alone and in the mix
(tolerance 0: integer results), and matches the oracle on small tables."""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from paper_2606_24647_amd import serve

pytestmark = pytest.mark.gpu

# A dimension of more than 2^20 rows: every join query takes the radix
# group-join (two-level probe partition, build on its own stream, LDS join),
# the path the full-size serving run takes.
NF, ND = 3_000_000, 1_200_000


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2606_24647_amd import devgen, gq
    fact = devgen.fact_c5(NF, nkeys=ND)
    dim = devgen.dim_c5(ND)
    torch.cuda.synchronize()
    return gq, torch, fact, dim


@pytest.mark.parametrize("max_heavy", [None, 1])
def test_alone_equals_mix(env, max_heavy):
    gq, torch, fact, dim = env
    qs = serve.make_workload(36, qps=2000.0, seed=3)
    mixed_ex = serve.DeviceExecutor(gq, torch, fact, dim, nslots=4, max_heavy=max_heavy)
    for c in mixed_ex.ctxs:
        c.set_timing(True)
    mixed = serve.Scheduler(mixed_ex, budget_bytes=1 << 40).run(qs, keep_results=True)
    assert len(mixed) == len(qs)
    launched = set()
    for c in mixed_ex.ctxs:
        launched |= set(c.timing_report())
        c.set_timing(False)
    assert "rj_join" in launched and "rp1_probe" in launched, sorted(launched)
    alone_ex = serve.DeviceExecutor(gq, torch, fact, dim, nslots=1)
    by_id = {r.qid: r for r in mixed}
    for q in qs:
        q0 = serve.Query(q.qid, q.kind, 0.0, q.params)
        rec = serve.Scheduler(alone_ex, budget_bytes=1 << 40).run([q0], keep_results=True)[0]
        assert serve.same_result(rec.result, by_id[q.qid].result), (q.qid, q.kind)


def test_agg_and_join_match_oracle(env):
    gq, torch, fact, dim = env
    hf = dg.fact_c5(NF, nkeys=ND)
    hd = dg.dim_c5(ND)
    ex = serve.DeviceExecutor(gq, torch, fact, dim, nslots=2)
    qs = [serve.Query(0, "agg", 0.0, {"b": 1700}),
          serve.Query(1, "join", 0.0, {"b_dim": 900, "b_fact": 1400}),
          serve.Query(2, "part", 0.0, {"b": 300, "P": 64})]
    recs = {r.qid: r for r in serve.Scheduler(ex, 1 << 40).run(qs, keep_results=True)}
    exp = oracle.groupby(hf, [serve.F_FLAG, serve.F_STATUS], [("range", serve.F_DATE, 0, 1700)], serve.AGG_AGGS)
    got = serve.canonical(recs[0].result)[1]
    assert np.array_equal(got, np.stack([c[0] for c in exp.keys + exp.aggs], axis=1)[np.lexsort(
        np.stack([c[0] for c in exp.keys + exp.aggs], axis=1).T[::-1])])
    expj = oracle.pipeline(hf, [("range", serve.F_DATE, 1400, 2555)], [serve.F_FKEY], serve.JOIN_AGGS,
                           join_spec=(hd, [serve.D_PKEY], [("range", serve.D_DATE, 0, 900)], [serve.F_FKEY]))
    gj = serve.canonical(recs[1].result)[1]
    ej = np.stack([c[0] for c in expj.keys + expj.aggs], axis=1)
    assert np.array_equal(gj, ej)
    # partition: filter then partition of the projected rows
    rows = oracle.filter_rows(hf, [("range", serve.F_DATE, 0, 300)])
    sub = dg.Table([dg.Column(hf.cols[c].name, hf.cols[c].data[rows]) for c in serve.PART_COLS])
    perm, off = oracle.partition(sub, [0], 64)
    kind, offs, cols = recs[2].result
    assert np.array_equal(offs, off)
    for j, c in enumerate(sub.cols):
        assert np.array_equal(cols[j][0], c.data[perm])
