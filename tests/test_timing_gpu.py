"""Per-kernel timing of a context: every launch, or only the launches of one
kernel name (the form bench.py uses inside its timed region)."""
import pytest

from paper_2606_24647_amd import datagen as dg

pytestmark = pytest.mark.gpu

AGGS = [("sum", [("col", 0)]), ("count*",)]
PRED = [("range", 3, 0, 1800)]


def run_ops(gq, ctx, t):
    ctx.filter(t, PRED, [0, 3])
    ctx.groupby_agg(t, [4, 5], PRED, AGGS, capacity=16, expected_groups=6)


def test_timing_all_and_only():
    from paper_2606_24647_amd import gq
    ctx = gq.Context()
    t = gq.to_device(dg.fact_c1(100_000))
    ctx.set_timing(True)
    run_ops(gq, ctx, t)
    ctx.set_timing(False)
    everything = ctx.timing_report()
    assert "filter" in everything and len(everything) >= 3
    assert all(ms >= 0 and n >= 1 for ms, n in everything.values())

    ctx.set_timing(True, only="filter")
    run_ops(gq, ctx, t)
    run_ops(gq, ctx, t)
    ctx.set_timing(False)
    only = ctx.timing_report()
    assert set(only) == {"filter"} and only["filter"][1] == 2

    ctx.set_timing(True)                  # the filter is cleared again
    run_ops(gq, ctx, t)
    ctx.set_timing(False)
    assert set(ctx.timing_report()) == set(everything)
    assert ctx.timing_report() == {}      # a report clears the records
    ctx.raise_status()
