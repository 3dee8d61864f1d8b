"""gq_groupby_agg on the GPU against the oracle, bit-exact after canonical ordering."""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import canon_groups, random_table, tbl

pytestmark = pytest.mark.gpu

REV = [("col", 1), ("k-col", 100, 2)]
C1_AGGS = [("sum", [("col", 0)]), ("sum", [("col", 1)]), ("sum", [("col", 2)]), ("sum", REV), ("count*",)]


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def gpu_groupby(gq, ctx, table, keys, preds, aggs, **kw):
    dev = gq.to_device(table)
    out, cnt = ctx.groupby_agg(dev, keys, preds, aggs, **kw)
    bits = ctx.sync_status()
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    return cols[:len(keys)], cols[len(keys):], n, bits


def check(gq, ctx, table, keys, preds, aggs, **kw):
    gk, ga, n, bits = gpu_groupby(gq, ctx, table, keys, preds, aggs, **kw)
    assert bits == 0, bits
    exp = oracle.groupby(table, keys, preds, aggs)
    assert n == exp.nrows
    gk = [(v.astype(np.int64), ok) for v, ok in gk]
    gk, ga = canon_groups(gk, ga)
    ek, ea = canon_groups(exp.keys, exp.aggs)
    for j, ((gv, gok), (ev, eok)) in enumerate(zip(gk, ek)):
        assert np.array_equal(gok, eok), f"key {j} validity"
        assert np.array_equal(gv, ev), f"key {j} values"
    for j, ((gv, gok), (ev, eok)) in enumerate(zip(ga, ea)):
        assert np.array_equal(gok, eok), f"agg {j} validity"
        assert np.array_equal(gv, ev), f"agg {j} values"


@pytest.mark.parametrize("strategy", ["lds", "global"])
def test_config1_full(gq, ctx, strategy):
    t = dg.fact_c1(1_000_000)
    check(gq, ctx, t, [4, 5], [("range", 3, -(1 << 31), 2466)], C1_AGGS, strategy=strategy, expected_groups=6)


@pytest.mark.parametrize("strategy", ["lds", "global", "auto"])
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1023, 1024, 1025, 50_001])
def test_sizes(gq, ctx, strategy, n):
    rng = np.random.default_rng(n + 7)
    t = random_table(rng, n, lo=-3, hi=3)
    check(gq, ctx, t, [3, 2], [("range", 1, -2, 2)], [("count*",), ("sum", [("col", 0)]),
                                                       ("min", [("col", 0)]), ("max", [("col", 1)])],
          strategy=strategy)


@pytest.mark.parametrize("strategy", ["lds", "global"])
def test_nulls_everywhere(gq, ctx, strategy):
    rng = np.random.default_rng(11)
    t = random_table(rng, 80_000, null_frac=0.2, lo=-4, hi=4)
    aggs = [("count*",), ("count", [("col", 0)]), ("sum", [("col", 0), ("k-col", 10, 1)]),
            ("min", [("col", 2)]), ("max", [("k+col", 5, 3)]), ("sum", [("const", 7)])]
    check(gq, ctx, t, [3, 1], [("ne", 2, 0)], aggs, strategy=strategy)


@pytest.mark.parametrize("strategy", ["lds", "global"])
def test_int64_key_high_cardinality(gq, ctx, strategy):
    rng = np.random.default_rng(12)
    n = 200_000
    k = rng.integers(-50_000, 50_000, n)
    k[::97] = -1                          # the key value that equals the empty-slot pattern
    k[::101] = np.iinfo(np.int64).min
    k[::103] = np.iinfo(np.int64).max
    valid = rng.random(n) > 0.05
    v = rng.integers(-(1 << 40), 1 << 40, n)
    t = tbl(k=(k, valid), v=v)
    check(gq, ctx, t, [0], [], [("sum", [("col", 1)]), ("count*",), ("min", [("col", 1)])], strategy=strategy)


def test_wrapping_sums(gq, ctx):
    big = np.iinfo(np.int64).max
    n = 30_000
    t = tbl(g=(np.arange(n) % 3).astype(np.int8), x=np.full(n, big - 5, dtype=np.int64))
    check(gq, ctx, t, [0], [], [("sum", [("col", 1)]), ("sum", [("col", 1), ("col", 1)])], strategy="lds")


def test_all_equal_keys_high_contention(gq, ctx):
    n = 500_000
    t = tbl(g=np.zeros(n, dtype=np.int32), x=np.arange(n, dtype=np.int64))
    for strategy in ("lds", "global"):
        check(gq, ctx, t, [0], [], [("sum", [("col", 1)]), ("count*",), ("max", [("col", 1)])],
              strategy=strategy)


def test_global_aggregate(gq, ctx):
    rng = np.random.default_rng(3)
    t = random_table(rng, 10_000, null_frac=0.1)
    check(gq, ctx, t, [], [("range", 0, 0, 20)], [("count*",), ("sum", [("col", 1)]), ("min", [("col", 2)])])
    e = random_table(rng, 0, null_frac=0.1)
    check(gq, ctx, e, [], [], [("count*",), ("sum", [("col", 1)]), ("min", [("col", 2)])])


def test_capacity_and_table_full(gq, ctx):
    rng = np.random.default_rng(4)
    t = tbl(k=rng.integers(0, 10_000, 100_000), v=np.ones(100_000, dtype=np.int64))
    dev = gq.to_device(t)
    out, cnt = ctx.groupby_agg(dev, [0], [], [("count*",)], capacity=10)
    assert ctx.sync_status() & 1
    exp = oracle.groupby(t, [0], [], [("count*",)])
    assert int(cnt.item()) == exp.nrows
    out, cnt = ctx.groupby_agg(dev, [0], [], [("count*",)], expected_groups=100, load_factor=0.9)
    assert ctx.sync_status() & 2


def test_unsupported_wide_keys(gq, ctx):
    t = gq.to_device(tbl(a=np.zeros(4, dtype=np.int64), b=np.zeros(4, dtype=np.int32)))
    with pytest.raises(gq.GqError) as e:
        ctx.groupby_agg(t, [0, 1], [], [("count*",)])
    assert e.value.code == gq.GQ_ERR_UNSUPPORTED


@pytest.mark.parametrize("nq", [1, 3, 8])
def test_shared_scan_equals_separate_queries(gq, ctx, nq):
    t = dg.fact_c1(300_001, seed=31, null_permille=20)
    rng = np.random.default_rng(nq)
    qpreds = [[("range", 3, int(rng.integers(0, 1000)), int(rng.integers(1000, 2600))), ("ne", 0, int(q))]
              for q in range(nq)]
    aggs = C1_AGGS + [("min", [("col", 1)]), ("count", [("col", 2)])]
    outs, cnt = ctx.groupby_shared(gq.to_device(t), [4, 5], qpreds, aggs, capacity=64, expected_groups=16)
    assert ctx.sync_status() == 0
    for q in range(nq):
        n = int(cnt[q].item())
        cols = gq.read_table(outs[q], n)
        exp = oracle.groupby(t, [4, 5], qpreds[q], aggs)
        assert n == exp.nrows
        gk = [(v.astype(np.int64), ok) for v, ok in cols[:2]]
        gk, ga = canon_groups(gk, cols[2:])
        ek, ea = canon_groups(exp.keys, exp.aggs)
        for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
            assert np.array_equal(gok, eok) and np.array_equal(gv, ev)


def test_shared_scan_rejects_mixed_columns(gq, ctx):
    t = gq.to_device(dg.fact_c1(1000))
    with pytest.raises(gq.GqError):
        ctx.groupby_shared(t, [4], [[("range", 3, 0, 5)], [("range", 0, 0, 5)]], [("count*",)])


def check_sorted(gq, cols, exp, nk):
    """GQ_SORTED output equals the oracle's canonical order directly (no host sort)."""
    for j, (g, e) in enumerate(zip(cols, exp.keys + exp.aggs)):
        gv, gok = g
        ev, eok = e
        gok = np.ones(len(gv), dtype=bool) if gok is None else gok
        assert np.array_equal(gok, eok), f"col {j} validity"
        assert np.array_equal(np.where(gok, gv.astype(np.int64), 0), np.where(eok, ev, 0)), f"col {j} values"


@pytest.mark.parametrize("strategy", ["lds", "global"])
def test_sorted_output_packed_keys(gq, ctx, strategy):
    rng = np.random.default_rng(41)
    t = random_table(rng, 60_000, null_frac=0.15, lo=-40, hi=40)
    aggs = [("count*",), ("sum", [("col", 0)])]
    out, cnt = ctx.groupby_agg(gq.to_device(t), [2, 3], [], aggs, strategy=strategy, sorted=True)
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    exp = oracle.groupby(t, [2, 3], [], aggs)
    assert n == exp.nrows
    check_sorted(gq, gq.read_table(out, n), exp, 2)


def test_sorted_output_raw64_keys(gq, ctx):
    rng = np.random.default_rng(42)
    n = 100_000
    k = rng.integers(-3_000, 3_000, n)
    k[::89] = -1
    k[::97] = np.iinfo(np.int64).min
    k[::101] = np.iinfo(np.int64).max
    t = tbl(k=(k, rng.random(n) > 0.05), v=rng.integers(0, 100, n))
    aggs = [("sum", [("col", 1)]), ("count*",)]
    out, cnt = ctx.groupby_agg(gq.to_device(t), [0], [], aggs, sorted=True)
    assert ctx.sync_status() == 0
    m = int(cnt.item())
    exp = oracle.groupby(t, [0], [], aggs)
    assert m == exp.nrows
    check_sorted(gq, gq.read_table(out, m), exp, 1)


def test_sorted_groupjoin_and_shared(gq, ctx):
    dim = dg.dim_c2(50_000, seed=44)
    fact = dg.fact_c2(200_000, nkeys=50_000, seed=44)
    aggs = [("sum", REV), ("count*",)]
    jt = ctx.join_build(gq.to_device(dim), [0], [("range", 1, 0, 1202)], acc_slots=2)
    out, cnt = ctx.pipeline(gq.to_device(fact), [("range", 3, 1278, 2555)], [0], aggs, join=jt, probe_key=0,
                            sorted=True)
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    exp = oracle.pipeline(fact, [("range", 3, 1278, 2555)], [0], aggs, join_spec=(dim, [0], [("range", 1, 0, 1202)], [0]))
    assert n == exp.nrows
    check_sorted(gq, gq.read_table(out, n), exp, 1)
    t = dg.fact_c1(100_000, seed=45)
    qp = [[("range", 3, 0, 1000)], [("range", 3, 500, 2555)]]
    outs, cnts = ctx.groupby_shared(gq.to_device(t), [4, 5], qp, C1_AGGS, capacity=16, expected_groups=6,
                                    sorted=True)
    assert ctx.sync_status() == 0
    for q in range(2):
        m = int(cnts[q].item())
        check_sorted(gq, gq.read_table(outs[q], m), oracle.groupby(t, [4, 5], qp[q], C1_AGGS), 2)


@pytest.mark.parametrize("keys", [[0], [3, 4]])
@pytest.mark.parametrize("sorted_out", [False, True])
def test_few_groups_over_many_tiles(gq, ctx, keys, sorted_out):
    """A large HBM table (sized for every row to be its own group) holding a
    few hundred groups: every compaction tile has a handful of occupied slots,
    at arbitrary output offsets, with NULL keys and NULL aggregate inputs."""
    rng = np.random.default_rng(31 + len(keys) + 2 * sorted_out)
    t = random_table(rng, 200_000, types=(np.int64, np.int64, np.int32, np.int16, np.int8), null_frac=0.3,
                     lo=-150, hi=150)
    aggs = [("sum", [("col", 1)]), ("count", [("col", 1)]), ("min", [("col", 2)]), ("max", [("col", 2)]),
            ("count*",)]
    check(gq, ctx, t, keys, [], aggs, strategy="global", expected_groups=200_000, sorted=sorted_out)


# Two-launch small group-by (a hint of at most 256 groups, packed keys,
# unsorted output): every block's partial merged by the last block.
@pytest.mark.parametrize("n", [1, 777, 2048, 65_537, 1_000_003])
def test_small_path_nulls_minmax(gq, ctx, n):
    rng = np.random.default_rng(n + 91)
    t = tbl(g=(rng.integers(-3, 4, n).astype(np.int8), rng.random(n) > 0.1),
            h=rng.integers(0, 5, n).astype(np.int16),
            v=(rng.integers(-10**12, 10**12, n), rng.random(n) > 0.2),
            w=rng.integers(-100, 100, n).astype(np.int32))
    aggs = [("sum", [("col", 2)]), ("min", [("col", 2)]), ("max", [("col", 3)]), ("count", [("col", 2)]),
            ("count*",), ("sum", [("col", 3), ("k-col", 7, 3)])]
    check(gq, ctx, t, [0, 1], [("range", 3, -90, 95)], aggs, strategy="lds", expected_groups=40)
    check(gq, ctx, t, [1, 0], [], aggs, expected_groups=256)


def test_small_path_capacity_and_table_full(gq, ctx):
    rng = np.random.default_rng(92)
    n = 300_000
    # 40 groups into an output of 16 rows: the count is still the group count.
    t = tbl(a=rng.integers(0, 8, n).astype(np.int8), b=rng.integers(0, 5, n).astype(np.int8),
            v=np.ones(n, dtype=np.int64))
    dev = gq.to_device(t)
    out, cnt = ctx.groupby_agg(dev, [0, 1], [], [("count*",)], capacity=16, expected_groups=40)
    assert ctx.sync_status() == 1
    assert int(cnt.item()) == 40
    # More groups than the table the hint sizes (as for the HBM table of the
    # general path): reported as a full table, never a wrong result without a
    # status.
    out, cnt = ctx.groupby_agg(dev, [0, 1], [], [("count*",)], capacity=64, expected_groups=10)
    assert ctx.sync_status() & 2
    t2 = tbl(a=rng.integers(0, 200, n).astype(np.int16), b=rng.integers(0, 200, n).astype(np.int16))
    out, cnt = ctx.groupby_agg(gq.to_device(t2), [0, 1], [], [("count*",)], expected_groups=100)
    assert ctx.sync_status() & 2


def test_small_path_equals_global(gq, ctx):
    rng = np.random.default_rng(93)
    t = dg.fact_c1(500_000, seed=93)
    a_small = gpu_groupby(gq, ctx, t, [4, 5], [("range", 3, 100, 2000)], C1_AGGS, expected_groups=6)
    a_glob = gpu_groupby(gq, ctx, t, [4, 5], [("range", 3, 100, 2000)], C1_AGGS, strategy="global",
                         expected_groups=6)
    assert a_small[2] == a_glob[2] and a_small[3] == 0 and a_glob[3] == 0
    gk, ga = canon_groups([(v.astype(np.int64), ok) for v, ok in a_small[0]], a_small[1])
    hk, ha = canon_groups([(v.astype(np.int64), ok) for v, ok in a_glob[0]], a_glob[1])
    for (gv, gok), (hv, hok) in zip(gk + ga, hk + ha):
        assert np.array_equal(gv, hv) and np.array_equal(gok, hok)
