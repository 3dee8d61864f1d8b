"""Batched fragments (one graph-captured persistent launch) against the oracle
and against one plain gq_groupby_agg call per fragment."""
import numpy as np
import pytest
import torch

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import canon_groups

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
