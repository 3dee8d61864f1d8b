"""Late materialisation (gq_join_groupby): key-only join -> gather maps ->
gather of the columns the group-by needs from either side -> group-by, against
the oracle's join + group-by over build- and probe-side columns."""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import canon_groups, random_table

pytestmark = pytest.mark.gpu

REV = [("col", 1), ("k-col", 100, 2)]


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def check(gq, ctx, build, bkeys, bpreds, probe, pkeys, ppreds, gkeys, aggs, pair_capacity=0):
    bd, pd_ = gq.to_device(build), gq.to_device(probe)
    jt = ctx.join_build(bd, bkeys, bpreds)
    out, cnt = ctx.join_groupby(jt, bd, pd_, pkeys, ppreds, gkeys, aggs, pair_capacity=pair_capacity)
    ctx.raise_status()
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    jt.free()
    exp = oracle.join_groupby(probe, ppreds, pkeys, build, bpreds, bkeys, gkeys, aggs)
    assert n == exp.nrows, (n, exp.nrows)
    nk = len(gkeys)
    gk, ga = canon_groups([(v.astype(np.int64), ok) for v, ok in cols[:nk]], cols[nk:])
    ek, ea = canon_groups(exp.keys, exp.aggs)
    for j, ((gv, gok), (ev, eok)) in enumerate(zip(gk + ga, ek + ea)):
        assert np.array_equal(gok, eok), (j, "validity")
        assert np.array_equal(gv, ev), (j, "values")
    return n


@pytest.mark.parametrize("seed", range(3))
def test_small_duplicates_nulls_both_sides(gq, ctx, seed):
    rng = np.random.default_rng(seed)
    # build: c0 key (dups, NULLs), c1 int32 payload, c2 int8 payload
    build = random_table(rng, 3_000, (np.int64, np.int32, np.int8), null_frac=0.05, lo=-200, hi=200)
    probe = random_table(rng, 20_000, (np.int64, np.int64, np.int16, np.int32), null_frac=0.05, lo=-200, hi=200)
    np_ = len(probe.cols)
    aggs = [("sum", [("col", 1)]), ("count*",), ("count", [("col", np_ + 1)]), ("min", [("col", np_ + 1)]),
            ("max", [("col", 2)]), ("sum", [("col", 1), ("col", np_ + 2)])]
    bpreds = [("range", 1, -150, 150)]
    ppreds = [("range", 3, -180, 190)]
    # group by a build column, a probe column, both, and none
    for gkeys in ([np_ + 2], [2], [2, np_ + 2], []):
        check(gq, ctx, build, [0], bpreds, probe, [0], ppreds, gkeys, aggs, pair_capacity=400_000)


def test_dim_payload_groups_at_full_partitioned_scale(gq, ctx):
    # 2^20 dimension rows: the table is stored partitioned and its probe index
    # is built on first use.  Group by the dimension's ckey (a build column
    # reached only through the gather map), revenue from the fact side.
    nd = 1 << 20
    dim = dg.dim_c2(nd, seed=31)
    fact = dg.fact_c2(3_000_000, nkeys=nd, seed=31)
    nfc = len(fact.cols)
    ckey = nfc + 2
    aggs = [("sum", REV), ("count*",), ("max", [("col", nfc + 1)])]
    n = check(gq, ctx, dim, [0], [("range", 1, 0, 1202)], fact, [0], [("range", 3, 1278, 2555)], [ckey], aggs)
    assert n > 100_000


def test_pair_capacity_overflow_reported(gq, ctx):
    rng = np.random.default_rng(9)
    build = random_table(rng, 500, (np.int64, np.int32), lo=0, hi=10)     # heavy duplicates
    probe = random_table(rng, 2_000, (np.int64, np.int32), lo=0, hi=10)
    bd, pd_ = gq.to_device(build), gq.to_device(probe)
    jt = ctx.join_build(bd, [0], [])
    ctx.join_groupby(jt, bd, pd_, [0], [], [3], [("count*",)], pair_capacity=100)
    assert ctx.sync_status() & gq.DEV_CAPACITY
    jt.free()


def test_two_key_columns(gq, ctx):
    # Join on (int32, int16) key tuples with NULLs in either column; group by
    # a build column and a probe column.
    rng = np.random.default_rng(11)
    build = random_table(rng, 4_000, (np.int32, np.int16, np.int8), null_frac=0.05, lo=-20, hi=20)
    probe = random_table(rng, 30_000, (np.int32, np.int16, np.int32), null_frac=0.05, lo=-20, hi=20)
    np_ = len(probe.cols)
    aggs = [("count*",), ("sum", [("col", 2)]), ("max", [("col", np_ + 2)])]
    check(gq, ctx, build, [0, 1], [], probe, [0, 1], [("range", 2, -15, 15)], [np_ + 2, 2], aggs,
          pair_capacity=600_000)
