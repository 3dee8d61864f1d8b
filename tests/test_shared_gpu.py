"""gq_pipeline_shared: several group-join pipelines over one probe input, the
probe side partitioned once with the hull of the queries' ranges and each
query's range applied to the value carried in the tuples.  Every query must
equal its own gq_pipeline call (bit for bit) and the oracle."""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import canon_groups, tbl

pytestmark = pytest.mark.gpu

REV = [("col", 1), ("k-col", 100, 2)]
MIN_BUILD = 1 << 20


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def host_groups(gq, out, cnt):
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    return n, canon_groups([(cols[0][0].astype(np.int64), cols[0][1])], cols[1:])


def check_shared(gq, ctx, probe, build, ppreds, ranges, bpreds_list, aggs, sorted_out=False, oracle_every=1):
    pdv, bdv = gq.to_device(probe), gq.to_device(build)
    tables = [ctx.join_build(bdv, [0], bp) for bp in bpreds_list]
    res = ctx.pipeline_shared(pdv, ppreds, 0, aggs, tables, ranges, sorted=sorted_out)
    assert ctx.sync_status() == 0
    for i, (jt, rng_pred, bp) in enumerate(zip(tables, ranges, bpreds_list)):
        n, (gk, ga) = host_groups(gq, *res[i])
        # The same query alone.
        out1, cnt1 = ctx.pipeline(pdv, list(ppreds) + [rng_pred], [0], aggs, join=jt, probe_key=0,
                                  sorted=sorted_out)
        assert ctx.sync_status() == 0
        n1, (gk1, ga1) = host_groups(gq, out1, cnt1)
        assert n == n1, (i, n, n1)
        for (gv, gok), (ev, eok) in zip(gk + ga, gk1 + ga1):
            assert np.array_equal(gok, eok) and np.array_equal(gv, ev), i
        if sorted_out and n > 1:
            keys = gq.read_table(res[i][0], n)[0][0].astype(np.int64)
            assert np.all(np.diff(keys) > 0)
        if i % oracle_every == 0:
            exp = oracle.pipeline(probe, list(ppreds) + [rng_pred], [0], aggs, join_spec=(build, [0], bp, [0]))
            assert n == exp.nrows, (i, n, exp.nrows)
            ek, ea = canon_groups(exp.keys, exp.aggs)
            for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
                assert np.array_equal(gok, eok) and np.array_equal(gv, ev), i
    for jt in tables:
        jt.free()


def test_shared_config2_shape(gq, ctx):
    # Four queries: each its own dimension bound (its own table) and fact date
    # range, ranges overlapping, one of them empty (lo > hi: no groups).
    n_dim, n_fact = MIN_BUILD + 4321, 2_500_003
    dim = dg.dim_c2(n_dim, seed=51)
    fact = dg.fact_c2(n_fact, nkeys=n_dim, seed=51)
    ranges = [("range", 3, 1278, 2555), ("range", 3, 0, 900), ("range", 3, 600, 2000), ("range", 3, 50, 40)]
    bpreds = [[("range", 1, 0, 1202)], [("range", 1, 0, 2405)], [("range", 1, 300, 700)], [("range", 1, 0, 1202)]]
    check_shared(gq, ctx, fact, dim, [], ranges, bpreds, [("sum", REV), ("count*",)])


def test_shared_nulls_duplicates_two_values_sorted(gq, ctx):
    # Duplicate build keys (multiplicities), NULL probe keys and values, a
    # nullable int16 range column, a common predicate, two value words, sorted
    # output.
    rng = np.random.default_rng(52)
    nb, npr = MIN_BUILD + 99, 1_600_007
    build = tbl(k=rng.integers(0, 400_000, nb), d=rng.integers(0, 10, nb).astype(np.int32))
    probe = tbl(k=(rng.integers(0, 450_000, npr), rng.random(npr) > 0.04),
                v=(rng.integers(-1000, 1000, npr), rng.random(npr) > 0.1),
                w=rng.integers(-5, 6, npr).astype(np.int8),
                r=(rng.integers(-300, 300, npr).astype(np.int16), rng.random(npr) > 0.05))
    aggs = [("sum", [("col", 1)]), ("count*",), ("max", [("col", 1)])]
    ranges = [("range", 3, -300, 0), ("range", 3, -20, 250), ("range", 3, 100, 299)]
    bpreds = [[("range", 1, 0, 6)], [("range", 1, 3, 9)], [("range", 1, 0, 9)]]
    check_shared(gq, ctx, probe, build, [("range", 2, -4, 4)], ranges, bpreds, aggs, sorted_out=True)


def test_shared_rejects_unpartitioned_table(gq, ctx):
    # A small build side is not partitioned: nothing is enqueued, UNSUPPORTED.
    rng = np.random.default_rng(53)
    build = tbl(k=rng.integers(0, 1000, 5000), d=rng.integers(0, 10, 5000).astype(np.int32))
    probe = tbl(k=rng.integers(0, 1000, 20000), r=rng.integers(0, 10, 20000).astype(np.int32))
    jt = ctx.join_build(gq.to_device(build), [0], [])
    with pytest.raises(gq.GqError) as e:
        ctx.pipeline_shared(gq.to_device(probe), [], 0, [("count*",)], [jt], [("range", 1, 0, 5)])
    assert e.value.code == gq.GQ_ERR_UNSUPPORTED
    assert ctx.sync_status() == 0
    jt.free()
