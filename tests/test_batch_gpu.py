"""Batched fragments (one graph-captured persistent launch) against the oracle
and against one plain gq_groupby_agg call per fragment."""
import numpy as np
import pytest
import torch

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import canon_groups, tbl

pytestmark = pytest.mark.gpu

REV = [("col", 1), ("k-col", 100, 2)]
AGGS = [("sum", [("col", 0)]), ("sum", [("col", 1)]), ("sum", [("col", 2)]), ("sum", REV), ("count*",)]


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def make_fragments(nf, seed, rows_hi=30_000, card_hi=5_000):
    rng = np.random.default_rng(seed)
    rows = np.exp(rng.uniform(np.log(1), np.log(rows_hi), nf)).astype(np.int64)
    rows[0], rows[1] = 0, 1                       # empty and single-row fragments
    card = np.exp(rng.uniform(np.log(1), np.log(card_hi), nf)).astype(np.int64)
    bound = rng.integers(0, dg.DATE_DAYS, nf)
    frags = [dg.fragment_c4(f, int(rows[f]), int(card[f]), seed=seed) for f in range(nf)]
    return frags, rows, card, bound


def canon(cols, nk):
    keys = [(v.astype(np.int64), ok) for v, ok in cols[:nk]]
    return canon_groups(keys, cols[nk:])


@pytest.mark.parametrize("lds_max", [-1, 0, 4096])
def test_batch_vs_oracle_and_plain(gq, ctx, lds_max):
    frags, rows, card, bound = make_fragments(48, seed=7)
    dev = [gq.to_device(t) for t in frags]
    preds = [[("range", 3, 0, int(b))] for b in bound]
    plan = gq.BatchPlan(ctx, [(d, p, int(c)) for d, p, c in zip(dev, preds, card)], [4], AGGS,
                        lds_max_groups=lds_max, tile_rows=2048)
    info = plan.info()
    assert info["total_rows"] == int(rows.sum())
    results = []
    for rep in range(3):
        plan.launch()
        ctx.raise_status()
        results.append([plan.result(f) for f in range(len(frags))])
        # eager work between graph replays
        _ = torch.arange(1000, device="cuda").sum().item()
    for f, t in enumerate(frags):
        exp = oracle.groupby(t, [4], preds[f], AGGS)
        ek, ea = canon_groups(exp.keys, exp.aggs)
        for rep in range(3):
            cols, n = results[rep][f]
            assert n == exp.nrows, (f, rep)
            gk, ga = canon(cols, 1)
            for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
                assert np.array_equal(gv, ev) and np.array_equal(gok, eok), (f, rep)
        # plain path, same fragment
        out, cnt = ctx.groupby_agg(dev[f], [4], preds[f], AGGS, expected_groups=int(card[f]))
        ctx.raise_status()
        pk, pa = canon(gq.read_table(out, int(cnt.item())), 1)
        for (gv, gok), (ev, eok) in zip(pk + pa, ek + ea):
            assert np.array_equal(gv, ev)
    plan.free()


def test_batch_large_fragments_multi_tile(gq, ctx):
    frags, rows, card, bound = make_fragments(6, seed=9, rows_hi=400_000, card_hi=70_000)
    rows_big = [300_000, 150_000, 9_000, 1, 0, 77_777]
    frags = [dg.fragment_c4(f, rows_big[f], int(card[f]) + 2, seed=9) for f in range(6)]
    dev = [gq.to_device(t) for t in frags]
    preds = [[("range", 3, 0, int(b))] for b in bound]
    plan = gq.BatchPlan(ctx, [(d, p, int(card[f]) + 2) for f, (d, p) in enumerate(zip(dev, preds))], [4], AGGS)
    plan.launch()
    ctx.raise_status()
    for f, t in enumerate(frags):
        exp = oracle.groupby(t, [4], preds[f], AGGS)
        cols, n = plan.result(f)
        assert n == exp.nrows
        gk, ga = canon(cols, 1)
        ek, ea = canon_groups(exp.keys, exp.aggs)
        for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
            assert np.array_equal(gv, ev)
    plan.free()


def test_batch_rejects_mismatched_shapes(gq, ctx):
    a = gq.to_device(dg.fragment_c4(0, 100, 5))
    t = dg.fragment_c4(1, 100, 5)
    t.cols[4].data = t.cols[4].data.astype(np.int64)      # key type differs
    b = gq.to_device(t)
    with pytest.raises(gq.GqError):
        gq.BatchPlan(ctx, [(a, [], 5), (b, [], 5)], [4], AGGS)


def test_batch_rejects_mismatched_nullable_inputs(gq, ctx):
    # SUM(qty), MIN(price): qty nullable in fragment 0 only, price in fragment 1
    # only; the accumulator words of the two fragments would not line up.
    aggs = [("sum", [("col", 0)]), ("min", [("col", 1)]), ("count*",)]
    t0 = dg.fragment_c4(0, 200, 5)
    t1 = dg.fragment_c4(1, 200, 5)
    t0.cols[0].valid = np.arange(200) % 3 != 0
    t1.cols[1].valid = np.arange(200) % 5 != 0
    a, b = gq.to_device(t0), gq.to_device(t1)
    with pytest.raises(gq.GqError):
        gq.BatchPlan(ctx, [(a, [], 5), (b, [], 5)], [4], aggs)
    # The same nullability in every fragment is accepted and matches the oracle.
    t1.cols[0].valid = np.arange(200) % 7 != 0
    t0.cols[1].valid = np.arange(200) % 2 != 0
    a, b = gq.to_device(t0), gq.to_device(t1)
    plan = gq.BatchPlan(ctx, [(a, [], 5), (b, [], 5)], [4], aggs)
    _check_plan(gq, plan, [t0, t1], [4], [[], []], aggs)
    plan.free()


# Fragments expecting at least radix_min_groups groups are partitioned by key
# hash and aggregated region by region in LDS; these cases force that path.

def _check_plan(gq, plan, frags, keys, preds, aggs, reps=1):
    results = []
    for _ in range(reps):
        plan.launch()
        gq_ctx = plan.ctx
        gq_ctx.raise_status()
        results.append([plan.result(f) for f in range(len(frags))])
        _ = torch.arange(1000, device="cuda").sum().item()
    for f, t in enumerate(frags):
        exp = oracle.groupby(t, keys, preds[f], aggs)
        ek, ea = canon_groups(exp.keys, exp.aggs)
        for rep in range(reps):
            cols, n = results[rep][f]
            assert n == exp.nrows, (f, rep, n, exp.nrows)
            gk, ga = canon(cols, len(keys))
            for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
                assert np.array_equal(gv, ev) and np.array_equal(gok, eok), (f, rep)


@pytest.mark.parametrize("radix_min", [1, 500])
def test_batch_radix_vs_oracle(gq, ctx, radix_min):
    # Mixed cardinalities: with radix_min=500 some fragments take the tile
    # path (LDS or HBM table) and the rest the radix path, in one graph.
    frags, rows, card, bound = make_fragments(40, seed=13, rows_hi=80_000, card_hi=30_000)
    dev = [gq.to_device(t) for t in frags]
    preds = [[("range", 3, 0, int(b))] for b in bound]
    plan = gq.BatchPlan(ctx, [(d, p, int(c)) for d, p, c in zip(dev, preds, card)], [4], AGGS,
                        radix_min_groups=radix_min)
    _check_plan(gq, plan, frags, [4], preds, AGGS, reps=3)
    plan.free()


def _raw_key_hashing_to_empty():
    # The one 64-bit key whose region hash is all ones (inverse of fmix64 of
    # ~0, then the seed), computed here from the hash's definition.
    m = (1 << 64) - 1
    h = m
    h ^= h >> 33
    h = (h * pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)) & m
    h ^= h >> 33
    h = (h * pow(0xFF51AFD7ED558CCD, -1, 1 << 64)) & m
    h ^= h >> 33
    k = h ^ 0x2545F4914F6CDD1D
    # forward check
    x = k ^ 0x2545F4914F6CDD1D
    x ^= x >> 33
    x = (x * 0xFF51AFD7ED558CCD) & m
    x ^= x >> 33
    x = (x * 0xC4CEB9FE1A85EC53) & m
    x ^= x >> 33
    assert x == m
    return np.array([k], dtype=np.uint64).view(np.int64)[0]


def test_batch_radix_raw_keys_nulls(gq, ctx):
    # Nullable int64 keys (raw key mode) with the EMPTY key (-1), NULL keys and
    # the key hashing to the LDS empty marker; nullable values under SUM, MIN,
    # MAX and COUNT(col).
    rng = np.random.default_rng(21)
    special = _raw_key_hashing_to_empty()
    frags, preds = [], []
    # Every fragment holds a NULL key and a NULL value (all fragments of a plan
    # share their column shapes, nullability included).
    for f, n in enumerate([50_000, 7_000, 2, 33_333, 120_001]):
        k = rng.integers(-2**62, 2**62, n)
        k = np.where(rng.random(n) < 0.5, rng.integers(0, 4000, n), k)
        k[::97] = -1
        k[5::101] = special
        kv, vv = rng.random(n) > 0.03, rng.random(n) > 0.1
        kv[0], vv[-1] = False, False
        frags.append(tbl(k=(k, kv), v=(rng.integers(-1000, 1000, n), vv),
                         w=rng.integers(0, 50, n).astype(np.int16)))
        preds.append([("range", 2, 0, 40)] if f % 2 else [])
    aggs = [("sum", [("col", 1)]), ("min", [("col", 1)]), ("max", [("col", 1)]), ("count", [("col", 1)]),
            ("count*",)]
    dev = [gq.to_device(t) for t in frags]
    plan = gq.BatchPlan(ctx, [(d, p, max(t.nrows, 1)) for d, p, t in zip(dev, preds, frags)], [0], aggs,
                        radix_min_groups=1)
    _check_plan(gq, plan, frags, [0], preds, aggs, reps=2)
    plan.free()


def test_batch_radix_packed_keys(gq, ctx):
    # Two keys packed into one word, one of them nullable.
    rng = np.random.default_rng(22)
    frags, preds = [], []
    for n in [90_000, 20_000, 3]:
        frags.append(tbl(a=rng.integers(-3000, 3000, n).astype(np.int32),
                         b=(rng.integers(-100, 100, n).astype(np.int8), rng.random(n) > 0.05),
                         v=rng.integers(0, 10**9, n)))
        preds.append([("ne", 1, 7)])
    aggs = [("sum", [("col", 2)]), ("max", [("col", 2)]), ("count*",)]
    dev = [gq.to_device(t) for t in frags]
    plan = gq.BatchPlan(ctx, [(d, p, t.nrows) for d, p, t in zip(dev, preds, frags)], [0, 1], aggs,
                        radix_min_groups=1)
    _check_plan(gq, plan, frags, [0, 1], preds, aggs, reps=2)
    plan.free()


def test_batch_radix_underestimated_groups(gq, ctx):
    # Three times more groups than expected: regions outgrow their LDS tables
    # and the excess goes to the fragment's HBM table.
    n, card, expected = 400_000, 60_000, 20_000
    t = dg.fragment_c4(0, n, card, seed=23)
    d = gq.to_device(t)
    plan = gq.BatchPlan(ctx, [(d, [], expected, n)], [4], AGGS, radix_min_groups=1)
    _check_plan(gq, plan, [t], [4], [[]], AGGS, reps=2)
    plan.free()


def test_batch_radix_too_many_columns_falls_back(gq, ctx):
    # Ten distinct columns to stage (key, predicate, eight SUM inputs) exceed
    # the radix path's staging: every fragment takes the tile path.
    rng = np.random.default_rng(24)
    frags, preds = [], []
    for n in [40_000, 5_000]:
        cols = {"k": rng.integers(0, 20_000, n), "p": rng.integers(0, 10, n).astype(np.int8)}
        for j in range(8):
            cols[f"v{j}"] = rng.integers(-1000, 1000, n)
        frags.append(tbl(**cols))
        preds.append([("range", 1, 0, 6)])
    aggs = [("sum", [("col", 2 + j)]) for j in range(7)] + [("count*",)]
    dev = [gq.to_device(t) for t in frags]
    plan = gq.BatchPlan(ctx, [(d, p, t.nrows) for d, p, t in zip(dev, preds, frags)], [0], aggs,
                        radix_min_groups=1)
    _check_plan(gq, plan, frags, [0], preds, aggs, reps=2)
    plan.free()
