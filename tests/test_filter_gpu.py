"""gq_filter on the GPU against the oracle, bit-exact (values, validity, order, count)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import assert_col_equal, random_table, tbl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def run_filter(gq, ctx, table, preds, proj, capacity=None, dev=None):
    dev = dev if dev is not None else gq.to_device(table)
    out, cnt = ctx.filter(dev, preds, proj, capacity=capacity)
    bits = ctx.sync_status()
    n = int(cnt.item())
    return out, n, bits


def check_filter(gq, ctx, table, preds, proj):
    out, n, bits = run_filter(gq, ctx, table, preds, proj)
    assert bits == 0
    rows, exp = oracle.filter(table, preds, proj)
    assert n == len(rows)
    got = gq.read_table(out, n)
    for j, (g, (ev, eok)) in enumerate(zip(got, exp)):
        assert_col_equal(g, ev, eok, f"proj {j}")


@pytest.mark.parametrize("n", [0, 1, 7, 8, 63, 64, 65, 2047, 2048, 2049, 4097, 100_003])
def test_filter_sizes(gq, ctx, n):
    rng = np.random.default_rng(n)
    t = random_table(rng, n)
    check_filter(gq, ctx, t, [("range", 0, -20, 30), ("ne", 3, 5)], [0, 1, 2, 3])


@pytest.mark.parametrize("null_frac", [0.1, 0.9])
def test_filter_nulls(gq, ctx, null_frac):
    rng = np.random.default_rng(5)
    t = random_table(rng, 70_001, null_frac=null_frac)
    check_filter(gq, ctx, t, [("range", 1, -40, 40)], [3, 2, 1, 0, 1])


def test_filter_no_predicates_and_no_projection(gq, ctx):
    rng = np.random.default_rng(6)
    t = random_table(rng, 5000)
    check_filter(gq, ctx, t, [], [2, 0])
    out, n, bits = run_filter(gq, ctx, t, [("range", 0, 0, 10)], [])
    assert n == len(oracle.filter_rows(t, [("range", 0, 0, 10)]))


def test_filter_all_and_none(gq, ctx):
    t = tbl(x=np.arange(10_000, dtype=np.int32), y=np.arange(10_000, dtype=np.int64))
    check_filter(gq, ctx, t, [("range", 0, -1, 10_000)], [0, 1])
    check_filter(gq, ctx, t, [("range", 0, 5, 4)], [0, 1])


def test_filter_int64_extremes(gq, ctx):
    lo, hi = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    v = np.array([lo, -1, 0, 1, hi] * 1000, dtype=np.int64)
    t = tbl(x=v)
    check_filter(gq, ctx, t, [("range", 0, int(lo), -1)], [0])
    check_filter(gq, ctx, t, [("range", 0, 0, int(hi))], [0])
    check_filter(gq, ctx, t, [("ne", 0, int(lo))], [0])


@pytest.mark.parametrize("offset", [1, 3, 5, 13])
def test_filter_unaligned_slice(gq, ctx, offset):
    rng = np.random.default_rng(offset)
    full = random_table(rng, 30_000, null_frac=0.2)
    dev = gq.to_device(full)
    n = 30_000 - offset - 7
    for c in dev.cols:
        c.offset, c.length = offset, n
    sl = dg.Table([dg.Column(c.name, c.data[offset:offset + n], c.valid[offset:offset + n])
                   for c in full.cols])
    preds, proj = [("range", 0, -25, 25)], [0, 1, 2, 3]
    out, cnt = ctx.filter(dev, preds, proj)
    assert ctx.sync_status() == 0
    rows, exp = oracle.filter(sl, preds, proj)
    assert int(cnt.item()) == len(rows)
    for j, (g, (ev, eok)) in enumerate(zip(gq.read_table(out, len(rows)), exp)):
        assert_col_equal(g, ev, eok, f"proj {j}")


def test_filter_capacity_error(gq, ctx):
    t = tbl(x=np.arange(50_000, dtype=np.int64))
    out, n, bits = run_filter(gq, ctx, t, [("range", 0, 0, 39_999)], [0], capacity=1000)
    assert bits & 1                       # GQ_DEV_CAPACITY
    assert n == 40_000                    # required size still reported
    v, _ = gq.read_column(out.cols[0], 1000)
    assert np.array_equal(v, np.arange(1000))


def test_filter_bad_descriptor(gq, ctx):
    t = gq.to_device(tbl(x=np.arange(10, dtype=np.int64)))
    with pytest.raises(gq.GqError) as e:
        ctx.filter(t, [("range", 3, 0, 1)], [0])
    assert e.value.code == gq.GQ_ERR_INVALID


def test_filter_config1_shape(gq, ctx):
    t = dg.fact_c1(1_000_000)
    check_filter(gq, ctx, t, [("range", 3, -(1 << 31), 2466)], [0, 1, 2, 3, 4, 5])
