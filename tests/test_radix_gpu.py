"""Radix group-join (large build inputs, partitioned by key hash, LDS aggregation)
and the index built on first use for such tables, against the oracle.

Build inputs here have at least 2^20 rows, the size from which gq_join_build
partitions the build side.  Sizes span several hist tiles (16384 rows) with a
ragged tail on both sides.
"""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import canon_groups, tbl
from tests.test_join_gpu import check_join, check_pipeline

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


@pytest.mark.parametrize("acc_slots", [0, 2])
def test_radix_config2_shape(gq, ctx, acc_slots):
    n_dim, n_fact = MIN_BUILD + 12_345, 3_000_017
    dim = dg.dim_c2(n_dim, seed=31)
    fact = dg.fact_c2(n_fact, nkeys=n_dim, seed=31)
    check_pipeline(gq, ctx, fact, [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)],
                   join_spec=(dim, [0], [("range", 1, 0, 1202)], 0), acc_slots=acc_slots)


def test_radix_duplicates_nulls(gq, ctx):
    # About 3.5 build rows per key (multiplicities weight the matches), NULL
    # probe keys and NULL values; two value words (SUM, MAX) and a non-NULL mask.
    rng = np.random.default_rng(32)
    nb, npr = MIN_BUILD + 777, 2_000_003
    build = tbl(k=rng.integers(0, 300_000, nb), d=rng.integers(0, 10, nb).astype(np.int32))
    probe = tbl(k=(rng.integers(0, 400_000, npr), rng.random(npr) > 0.05),
                v=(rng.integers(-1000, 1000, npr), rng.random(npr) > 0.1),
                w=rng.integers(-5, 5, npr).astype(np.int16))
    aggs = [("sum", [("col", 1)]), ("count*",), ("count", [("col", 1)]), ("max", [("col", 1)])]
    check_pipeline(gq, ctx, probe, [("range", 2, -4, 4)], [0], aggs,
                   join_spec=(build, [0], [("range", 1, 0, 6)], 0))


def test_radix_three_values_falls_back(gq, ctx):
    # Three value words exceed the radix tuple: the pipeline takes the index path,
    # building the index of the partitioned table on first use.
    rng = np.random.default_rng(33)
    nb, npr = MIN_BUILD + 5, 1_500_000
    build = tbl(k=rng.integers(0, 200_000, nb))
    probe = tbl(k=rng.integers(0, 250_000, npr), v=(rng.integers(-50, 50, npr), rng.random(npr) > 0.2))
    aggs = [("sum", [("col", 1)]), ("min", [("col", 1)]), ("max", [("col", 1)]), ("count*",)]
    check_pipeline(gq, ctx, probe, [], [0], aggs, join_spec=(build, [0], [], 0), acc_slots=6)


def test_radix_special_keys(gq, ctx):
    lo, hi = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    rng = np.random.default_rng(34)
    nb, npr = MIN_BUILD + 3, 600_001
    bk = rng.integers(-1_000_000, 1_000_000, nb)
    bk[:6] = [lo, hi, -1, 0, -1, hi]
    pk = rng.integers(-1_000_000, 1_000_000, npr)
    pk[::1000] = -1
    pk[1::1000] = lo
    pk[2::1000] = hi
    build = tbl(k=bk)
    probe = tbl(k=pk, v=rng.integers(0, 100, npr))
    check_pipeline(gq, ctx, probe, [], [0], [("sum", [("col", 1)]), ("count*",)], join_spec=(build, [0], [], 0))


def test_radix_int32_keys(gq, ctx):
    rng = np.random.default_rng(35)
    nb, npr = MIN_BUILD + 100, 1_000_003
    build = tbl(k=rng.integers(-2**31, 2**31 - 1, nb).astype(np.int32))
    pk = build.cols[0].data[rng.integers(0, nb, npr)].copy()
    pk[::3] = rng.integers(-2**31, 2**31 - 1, len(pk[::3]))
    probe = tbl(k=pk.astype(np.int32), v=rng.integers(-9, 9, npr).astype(np.int8))
    check_pipeline(gq, ctx, probe, [], [0], [("sum", [("col", 1), ("const", 3)]), ("count*",)],
                   join_spec=(build, [0], [], 0))


def test_radix_sorted_output(gq, ctx):
    n_dim, n_fact = MIN_BUILD + 1, 2_000_000
    dim = dg.dim_c2(n_dim, seed=36)
    fact = dg.fact_c2(n_fact, nkeys=n_dim, seed=36)
    jt = ctx.join_build(gq.to_device(dim), [0], [("range", 1, 0, 1202)])
    out, cnt = ctx.pipeline(gq.to_device(fact), [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)],
                            join=jt, probe_key=0, sorted=True)
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    jt.free()
    exp = oracle.pipeline(fact, [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)],
                          join_spec=(dim, [0], [("range", 1, 0, 1202)], [0]))
    ek, ea = canon_groups(exp.keys, exp.aggs)
    assert n == exp.nrows
    # Already in key order: no canonicalisation of the device output.
    assert np.array_equal(cols[0][0].astype(np.int64), ek[0][0])
    for (gv, _), (ev, _) in zip(cols[1:], ea):
        assert np.array_equal(gv, ev)


def test_radix_table_probe_pairs(gq, ctx):
    # gq_join_probe on a partitioned table builds its index first.
    dim = dg.dim_c2(MIN_BUILD + 9, seed=37)
    fact = dg.fact_c2(700_001, nkeys=MIN_BUILD + 9, seed=37)
    check_join(gq, ctx, dim, [0], [("range", 1, 0, 1202)], fact, [0], [("range", 3, 1278, 2555)])


def test_radix_table_duplicate_pairs(gq, ctx):
    rng = np.random.default_rng(38)
    nb = MIN_BUILD + 4000
    build = tbl(k=(rng.integers(0, 50_000, nb), rng.random(nb) > 0.02))
    probe = tbl(k=rng.integers(0, 60_000, 30_000))
    check_join(gq, ctx, build, [0], [], probe, [0], [])


def test_radix_table_other_group_key(gq, ctx):
    # Group by a probe column other than the join key: index path on a partitioned table.
    rng = np.random.default_rng(39)
    nb, npr = MIN_BUILD + 11, 800_000
    build = tbl(k=rng.integers(0, 400_000, nb))
    probe = tbl(k=rng.integers(0, 500_000, npr), g=rng.integers(0, 9, npr).astype(np.int8),
                v=rng.integers(0, 1000, npr))
    check_pipeline(gq, ctx, probe, [], [1], [("sum", [("col", 2)]), ("count*",)], join_spec=(build, [0], [], 0))


@pytest.mark.parametrize("case", ["build_filtered_out", "empty_probe", "probe_filtered_out"])
def test_radix_empty(gq, ctx, case):
    rng = np.random.default_rng(40)
    nb = MIN_BUILD + 17
    build = tbl(k=rng.integers(0, 1000, nb), d=rng.integers(0, 10, nb))
    npr = 0 if case == "empty_probe" else 100_000
    probe = tbl(k=rng.integers(0, 1000, npr), v=rng.integers(0, 10, npr))
    bpred = [("range", 1, 100, 200)] if case == "build_filtered_out" else []
    ppred = [("range", 1, 100, 200)] if case == "probe_filtered_out" else []
    check_pipeline(gq, ctx, probe, ppred, [0], [("sum", [("col", 1)]), ("count*",)],
                   join_spec=(build, [0], bpred, 0))


def test_radix_reuse_table(gq, ctx):
    # One partitioned table serves two group-joins and then a pairs probe.
    dim = dg.dim_c2(MIN_BUILD + 2, seed=41)
    fact = dg.fact_c2(500_000, nkeys=MIN_BUILD + 2, seed=41)
    bd, fd = gq.to_device(dim), gq.to_device(fact)
    jt = ctx.join_build(bd, [0], [("range", 1, 0, 1202)])
    spec = (dim, [0], [("range", 1, 0, 1202)], [0])
    for preds in ([("range", 3, 1278, 2555)], [("range", 3, 0, 1000)]):
        out, cnt = ctx.pipeline(fd, preds, [0], [("sum", REV), ("count*",)], join=jt, probe_key=0)
        assert ctx.sync_status() == 0
        n = int(cnt.item())
        exp = oracle.pipeline(fact, preds, [0], [("sum", REV), ("count*",)], join_spec=spec)
        assert n == exp.nrows
        cols = gq.read_table(out, n)
        gk, ga = canon_groups([(cols[0][0].astype(np.int64), cols[0][1])], cols[1:])
        ek, ea = canon_groups(exp.keys, exp.aggs)
        for (gv, _), (ev, _) in zip(gk + ga, ek + ea):
            assert np.array_equal(gv, ev)
    pi, bi, cnt = ctx.join_probe(jt, fd, [0], [("range", 3, 1278, 2555)], capacity=600_000)
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    epi, ebi = oracle.join(dim, [0], [("range", 1, 0, 1202)], fact, [0], [("range", 3, 1278, 2555)])
    assert n == len(epi)
    assert np.array_equal(pi[:n].cpu().numpy(), epi) and np.array_equal(bi[:n].cpu().numpy(), ebi)
    jt.free()


@pytest.mark.parametrize("rlog", [4, 9, 12])
def test_radix_region_counts(gq, ctx, rlog):
    # 16 regions (two per XCD queue), 512, and 4096 (about 256 build keys each).
    n_dim, n_fact = MIN_BUILD + 4097, 1_200_007
    dim = dg.dim_c2(n_dim, seed=42)
    fact = dg.fact_c2(n_fact, nkeys=n_dim, seed=42)
    jt = ctx.join_build(gq.to_device(dim), [0], [("range", 1, 0, 1202)], regions_log2=rlog)
    out, cnt = ctx.pipeline(gq.to_device(fact), [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)],
                            join=jt, probe_key=0)
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    jt.free()
    exp = oracle.pipeline(fact, [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)],
                          join_spec=(dim, [0], [("range", 1, 0, 1202)], [0]))
    assert n == exp.nrows
    gk, ga = canon_groups([(cols[0][0].astype(np.int64), cols[0][1])], cols[1:])
    ek, ea = canon_groups(exp.keys, exp.aggs)
    for (gv, _), (ev, _) in zip(gk + ga, ek + ea):
        assert np.array_equal(gv, ev)


@pytest.mark.parametrize("rlog", [3, 13])
def test_radix_region_count_out_of_range(gq, ctx, rlog):
    dim = dg.dim_c2(1000, seed=43)
    with pytest.raises(gq.GqError):
        ctx.join_build(gq.to_device(dim), [0], [], regions_log2=rlog)


@pytest.mark.parametrize("radix,alloc", [(True, None), (False, None), (True, "torch")])
def test_build_on_another_stream(gq, ctx, radix, alloc):
    # The build is enqueued on a second stream behind a long kernel; the
    # pipeline on the current stream must wait for it where it reads the table
    # (radix path: after partitioning its probe side; index path: before it).
    import torch
    if alloc:
        ctx = gq.Context(allocator=alloc)   # the table is freed on another stream than its allocation
    n_dim = MIN_BUILD + 3 if radix else 200_000
    dim = dg.dim_c2(n_dim, seed=44)
    fact = dg.fact_c2(900_001, nkeys=n_dim, seed=44)
    bd, fd = gq.to_device(dim), gq.to_device(fact)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        x = torch.ones(1 << 24, device="cuda")
        for _ in range(20):
            x = x * 1.0001                     # delays the build on this stream
    jt = ctx.join_build(bd, [0], [("range", 1, 0, 1202)], acc_slots=2, stream=s)
    out, cnt = ctx.pipeline(fd, [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)], join=jt, probe_key=0)
    jt.free()
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    exp = oracle.pipeline(fact, [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)],
                          join_spec=(dim, [0], [("range", 1, 0, 1202)], [0]))
    assert n == exp.nrows
    gk, ga = canon_groups([(cols[0][0].astype(np.int64), cols[0][1])], cols[1:])
    ek, ea = canon_groups(exp.keys, exp.aggs)
    for (gv, _), (ev, _) in zip(gk + ga, ek + ea):
        assert np.array_equal(gv, ev)


def test_radix_register_path_column_types(gq, ctx):
    # The register-path histogram loads its columns as 16-byte chunks and
    # extracts two rows per lane: int8 and int16 predicate columns and an
    # int16 key on the probe side (with int32 and nullable int64 values for the
    # scatter), an int8 predicate on the build side; both sides end in a
    # ragged tail.
    rng = np.random.default_rng(41)
    nb, npr = MIN_BUILD + 13, 1_700_009
    build = tbl(k=rng.integers(-30_000, 30_000, nb).astype(np.int16),
                f=rng.integers(-3, 4, nb).astype(np.int8))
    probe = tbl(k=rng.integers(-32_000, 32_000, npr).astype(np.int16),
                p8=rng.integers(-100, 100, npr).astype(np.int8),
                p16=rng.integers(-1000, 1000, npr).astype(np.int16),
                v32=rng.integers(-10**9, 10**9, npr).astype(np.int32),
                v64=(rng.integers(-10**15, 10**15, npr), rng.random(npr) > 0.07))
    aggs = [("sum", [("col", 3), ("k-col", 7, 1)]), ("max", [("col", 4)]), ("count*",), ("count", [("col", 4)])]
    check_pipeline(gq, ctx, probe, [("range", 1, -60, 90), ("ne", 2, 5)], [0], aggs,
                   join_spec=(build, [0], [("range", 1, -2, 3)], 0))


def test_radix_staged_path_unaligned_and_wide(gq, ctx):
    # Columns that are not 16-byte aligned (slices starting at row 1): the
    # histogram stages them through LDS like the scatter, on both sides.
    rng = np.random.default_rng(42)
    nb, npr = MIN_BUILD + 3, 1_200_001
    build = tbl(k=rng.integers(0, 500_000, nb + 1), d=rng.integers(0, 10, nb + 1).astype(np.int32))
    probe = tbl(k=rng.integers(0, 600_000, npr + 1), a=rng.integers(0, 9, npr + 1).astype(np.int8),
                b=rng.integers(0, 9, npr + 1).astype(np.int16), c=rng.integers(0, 9, npr + 1).astype(np.int32),
                d=rng.integers(0, 9, npr + 1), v=rng.integers(-99, 99, npr + 1))
    # Row-1 slices on the device, and the matching host tables for the oracle.
    from paper_2606_24647_amd.datagen import Column, Table
    hb = Table([Column(c.name, c.data[1:]) for c in build.cols])
    hp = Table([Column(c.name, c.data[1:]) for c in probe.cols])
    bd, pd_ = gq.to_device(build), gq.to_device(probe)
    for c in bd.cols + pd_.cols:
        c.offset = 1
    preds = [("range", 1, 1, 8), ("range", 2, 0, 7), ("ne", 3, 4), ("range", 4, 1, 8)]
    aggs = [("sum", [("col", 5)]), ("max", [("col", 5), ("col", 4)]), ("count*",)]
    jt = ctx.join_build(bd, [0], [("range", 1, 0, 7)], acc_slots=2)
    out, cnt = ctx.pipeline(pd_, preds, [0], aggs, join=jt, probe_key=0)
    ctx.raise_status()
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    jt.free()
    exp = oracle.pipeline(hp, preds, [0], aggs, join_spec=(hb, [0], [("range", 1, 0, 7)], [0]))
    assert n == exp.nrows
    gk, ga = canon_groups([(cols[0][0].astype(np.int64), cols[0][1])], cols[1:])
    ek, ea = canon_groups(exp.keys, exp.aggs)
    for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
        assert np.array_equal(gok, eok) and np.array_equal(gv, ev)
