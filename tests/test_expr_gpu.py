"""Expression programs (gq_compute_column, gq_filter_expr, gq_groupby_expr)
and ORDER BY / top-k (gq_order_by) on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
from tests.helpers import canon_groups, random_table

pytestmark = pytest.mark.gpu

TYPES = (np.int64, np.int32, np.int16, np.int8, np.int64)
BIN = ["add", "sub", "mul", "lt", "le", "eq", "ne", "gt", "ge"]


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def random_tree(rng, ncols, depth):
    if depth == 0 or rng.random() < 0.25:
        if rng.random() < 0.7:
            return ("col", int(rng.integers(ncols)))
        return ("const", int(rng.integers(-20, 21)))
    r = rng.random()
    if r < 0.1:
        return ("neg", random_tree(rng, ncols, depth - 1))
    if r < 0.25:
        return ("case", random_tree(rng, ncols, depth - 1), random_tree(rng, ncols, depth - 1),
                random_tree(rng, ncols, depth - 1))
    return (BIN[int(rng.integers(len(BIN)))], random_tree(rng, ncols, depth - 1), random_tree(rng, ncols, depth - 1))


def table(seed, n, null_frac=0.1):
    rng = np.random.default_rng(seed)
    t = random_table(rng, n, TYPES, null_frac=null_frac, lo=-30, hi=30)
    t.cols[4].data = rng.integers(-(1 << 62), 1 << 62, n).astype(np.int64)   # wrapping products
    return t


@pytest.mark.parametrize("seed", range(6))
def test_compute_column_random_trees(gq, ctx, seed):
    rng = np.random.default_rng(100 + seed)
    t = table(seed, 70_001)
    d = gq.to_device(t)
    for _ in range(8):
        tree = random_tree(rng, len(t.cols), 5)
        if len(gq.compile_expr(tree)) > 32:
            continue
        out = ctx.compute_column(d, tree)
        ctx.raise_status()
        (gv, gok), = gq.read_table(out, t.nrows)
        ev, eok = oracle.eval_expr(t, tree)
        assert np.array_equal(gok, eok), tree
        assert np.array_equal(gv[eok], ev[eok]), tree


def test_filter_expr(gq, ctx):
    t = table(7, 100_003)
    d = gq.to_device(t)
    exprs = [("gt", ("mul", ("col", 0), ("col", 1)), ("const", -100)),
             ("case", ("lt", ("col", 2), ("const", 0)), ("ne", ("col", 3), ("const", 5)), ("const", 1))]
    preds = [("range", 0, -25, 28)]
    proj = [4, 1, 3]
    out, cnt = ctx.filter_expr(d, preds, exprs, proj)
    ctx.raise_status()
    n = int(cnt.item())
    rows, cols = oracle.filter_expr(t, preds, exprs, proj)
    assert n == len(rows)
    got = gq.read_table(out, n)
    for (gv, gok), (ev, eok) in zip(got, cols):
        ok = np.ones(n, bool) if eok is None else eok
        if gok is not None:
            assert np.array_equal(gok, ok)
        assert np.array_equal(gv[ok], ev[ok])


@pytest.mark.parametrize("keys", [[3], [3, 2], []])
def test_groupby_expr(gq, ctx, keys):
    t = table(9, 80_000)
    d = gq.to_device(t)
    exprs = [("ne", ("col", 1), ("const", 0))]
    aggs = [("sum", ("mul", ("col", 4), ("sub", ("const", 100), ("col", 2)))), ("count*",),
            ("count", ("case", ("gt", ("col", 0), ("const", 0)), ("col", 1), ("col", 2))),
            ("min", ("add", ("col", 0), ("col", 3))), ("max", ("neg", ("col", 4)))]
    preds = [("range", 2, -25, 30)]
    out, cnt = ctx.groupby_expr(d, keys, preds, exprs, aggs)
    ctx.raise_status()
    n = int(cnt.item())
    exp = oracle.groupby_expr(t, keys, preds, exprs, aggs)
    assert n == exp.nrows
    cols = gq.read_table(out, n)
    nk = len(keys)
    gk, ga = canon_groups([(v.astype(np.int64), ok) for v, ok in cols[:nk]], cols[nk:])
    ek, ea = canon_groups(exp.keys, exp.aggs)
    for j, ((gv, gok), (ev, eok)) in enumerate(zip(gk + ga, ek + ea)):
        assert np.array_equal(gok, eok), j
        assert np.array_equal(gv, ev), j


@pytest.mark.parametrize("spec", [
    ([3], None, None, None),
    ([3, 2], [True, False], [False, True], None),
    ([1, 3, 0], [False, True, True], [True, False, True], 100),
    ([4], [True], None, 17),
    ([2, 1], None, [True, True], 0),
])
def test_order_by_vs_oracle(gq, ctx, spec):
    keys, desc, nf, limit = spec
    t = table(11, 40_000, null_frac=0.15)
    d = gq.to_device(t)
    got = ctx.order_by(d, keys, desc, nf, limit)
    ctx.raise_status()
    exp = oracle.order_by(t, keys, desc, nf, limit)
    assert np.array_equal(got.cpu().numpy(), exp)


def test_order_by_large_is_sorted_and_stable(gq, ctx):
    # 3M rows: the permutation is checked against numpy's stable lexsort.
    rng = np.random.default_rng(5)
    n = 3_000_000
    t = random_table(rng, n, (np.int64, np.int16), lo=-1000, hi=1000)
    d = gq.to_device(t)
    got = ctx.order_by(d, [1, 0], [True, False], None, None).cpu().numpy()
    exp = np.lexsort((t.cols[0].data, -t.cols[1].data.astype(np.int64)))
    assert np.array_equal(got, exp)
    top = ctx.order_by(d, [1, 0], [True, False], None, 1000).cpu().numpy()
    assert np.array_equal(top, exp[:1000])
