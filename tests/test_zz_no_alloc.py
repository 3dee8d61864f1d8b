"""gq_filter_noalloc (the entry point for callers that cannot allocate): its
output equals gq_filter's on two calls in a row, the second with a smaller
input, through the C ABI; inputs beyond its fixed workspace are rejected."""
import numpy as np
import pytest
import torch

from paper_2606_24647_amd import datagen as dg
from tests.helpers import random_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def compare(gq, ctx, t, preds, proj):
    d = gq.to_device(t)
    ref, rcnt = ctx.filter(d, preds, proj)
    out = gq.empty_like_cols([d.cols[j].type for j in proj], t.nrows, [d.cols[j].valid is not None for j in proj])
    # Poison the outputs so that a row the call does not write shows up.
    for c in out.cols:
        c.data.fill_(-77)
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ctx.filter_noalloc(d, preds, proj, out, cnt, t.nrows)
    ctx.raise_status()
    n = int(rcnt.item())
    assert int(cnt.item()) == n
    got, exp = gq.read_table(out, n), gq.read_table(ref, n)
    for (gv, gok), (ev, eok) in zip(got, exp):
        assert np.array_equal(gv, ev)
        assert (gok is None) == (eok is None)
        if gok is not None:
            assert np.array_equal(gok, eok)
    return n


def test_noalloc_filter_matches_filter_twice(gq, ctx):
    rng = np.random.default_rng(41)
    big = random_table(rng, 3_000_017, (np.int64, np.int32, np.int8, np.int16), null_frac=0.05, lo=-100, hi=100)
    n1 = compare(gq, ctx, big, [("range", 1, -60, 70), ("ne", 2, 3)], [0, 3, 1, 2])
    small = random_table(rng, 70_001, (np.int64, np.int32, np.int8, np.int16), null_frac=0.2, lo=-100, hi=100)
    n2 = compare(gq, ctx, small, [("range", 0, -10, 90)], [2, 0])
    assert n1 > n2 > 0
    # The 1M-row workload's table, projected and filtered as the filter + group-by query does.
    t1 = dg.fact_c1(1_000_000)
    compare(gq, ctx, t1, [("range", 3, -(1 << 31), 2466)], [0, 1, 2, 4, 5])


def test_noalloc_filter_rejects_oversized_input(gq, ctx):
    n = (1 << 28) + 1
    d = gq.DevTable([gq.DevColumn(torch.zeros(n, dtype=torch.int8, device="cuda"))])
    out = gq.empty_like_cols([gq.GQ_I8], 16, [False])
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(gq.GqError):
        ctx.filter_noalloc(d, [("range", 0, 1, 1)], [0], out, cnt, 16)
    del d
    torch.cuda.empty_cache()


def test_noalloc_filter_on_a_context_whose_allocator_fails(gq):
    calls = {"alloc": 0}

    def alloc(nbytes, stream):
        calls["alloc"] += 1
        return None

    def free(ptr, nbytes, stream):
        raise AssertionError("nothing was allocated, so nothing is freed")

    ctx = gq.Context(allocator=gq.make_allocator(alloc, free))
    t = dg.fact_c1(60_000)
    d = gq.to_device(t)
    out = gq.empty_like_cols([d.cols[j].type for j in (0, 3)], t.nrows, [False, False])
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.filter_noalloc(d, [("range", 3, 0, 1000)], [0, 3], out, cnt, t.nrows)
    ctx.raise_status()
    assert calls["alloc"] == 0
    keep = (t.cols[3].data >= 0) & (t.cols[3].data <= 1000)
    n = int(cnt.item())
    assert n == int(keep.sum())
    assert np.array_equal(out.cols[0].data[:n].cpu().numpy(), t.cols[0].data[keep])
    assert np.array_equal(out.cols[1].data[:n].cpu().numpy(), t.cols[3].data[keep])
