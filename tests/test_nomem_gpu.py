"""Allocation failure: with an allocator that returns NULL, every call that
needs device memory returns GQ_ERR_NOMEM and enqueues nothing (its outputs
and device counts stay as they were)."""
import numpy as np
import pytest
import torch

from paper_2606_24647_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def failing(gq):
    calls = {"alloc": 0}

    def alloc(nbytes, stream):
        calls["alloc"] += 1
        return None

    def free(ptr, nbytes, stream):
        raise AssertionError("nothing was allocated, so nothing is freed")

    ctx = gq.Context(allocator=gq.make_allocator(alloc, free))
    return ctx, calls


def _untouched(t: torch.Tensor, value: int):
    torch.cuda.synchronize()
    assert bool((t == value).all())


def test_filter_nomem(gq, failing):
    ctx, calls = failing
    t = gq.to_device(dg.fact_c1(50_000))
    out = gq.empty_like_cols([c.type for c in t.cols], t.nrows, [False] * len(t.cols))
    for c in out.cols:
        c.data.fill_(-7)
    cnt = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    ib, ob = gq._BatchArg(t), gq._BatchArg(out, t.nrows)
    p, np_ = gq._preds([("range", 3, 0, 1000)])
    pj, npj = gq._ints(list(range(len(t.cols))))
    before = calls["alloc"]
    rc = gq.lib().gq_filter(ctx.h, ib.ref, p, np_, pj, npj, ob.ref, gq.C.c_void_p(cnt.data_ptr()),
                            gq._stream(None))
    assert rc == gq.GQ_ERR_NOMEM and calls["alloc"] > before
    _untouched(cnt, -5)
    for c in out.cols:
        _untouched(c.data, -7)


def test_groupby_join_partition_sort_stream_nomem(gq, failing):
    ctx, _ = failing
    t = gq.to_device(dg.fact_c1(50_000))
    with pytest.raises(gq.GqError) as e:
        ctx.groupby_agg(t, [4, 5], [], [("count*",)])
    assert e.value.code == gq.GQ_ERR_NOMEM
    dim = gq.to_device(dg.dim_c2(10_000, seed=3))
    with pytest.raises(gq.GqError) as e:
        ctx.join_build(dim, [0], [])
    assert e.value.code == gq.GQ_ERR_NOMEM
    with pytest.raises(gq.GqError) as e:
        ctx.hash_partition(t, [0], 64)
    assert e.value.code == gq.GQ_ERR_NOMEM
    with pytest.raises(gq.GqError) as e:
        ctx.order_by(t, [0])
    assert e.value.code == gq.GQ_ERR_NOMEM
    with pytest.raises(gq.GqError) as e:
        gq.AggStream(ctx, "single", [4], [gq.GQ_I8], [False], [("count*",)], 16)
    assert e.value.code == gq.GQ_ERR_NOMEM

