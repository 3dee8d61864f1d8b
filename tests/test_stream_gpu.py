"""Aggregation modes and streaming aggregation (gq_agg_stream_*) on the GPU
against the oracle: one-shot Partial / Intermediate / Final calls, streams over
many uneven batches with NULL keys and inputs, early emission at a group-count
threshold, and a Partial -> Final chain equal to one Single aggregation."""
import numpy as np
import pytest
import torch

import oracle
from paper_2606_24647_amd.datagen import Column, Table
from tests.helpers import canon_groups, random_table

pytestmark = pytest.mark.gpu

# Columns of the raw batches: c0 int64 key, c1 int8 key, c2 int64 value, c3 int32 value
AGGS = [("sum", [("col", 2)]), ("count*",), ("count", [("col", 3)]), ("min", [("col", 3)]),
        ("max", [("col", 2)]), ("sum", [("col", 2), ("k-col", 100, 3)])]
TYPES = (np.int64, np.int8, np.int64, np.int32)


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def raw_batches(seed, nb=9, nkey=40):
    """nb batches of uneven sizes (0 .. 20,000 rows), NULLs in keys and values."""
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.integers(0, 20_000, nb)]
    sizes[2] = 0
    sizes[5] = 1
    out = []
    for n in sizes:
        t = random_table(rng, n, TYPES, null_frac=0.1, lo=-nkey, hi=nkey)
        t.cols[2].data = rng.integers(-10**12, 10**12, n).astype(np.int64)
        out.append(t)
    return out


def canon_res(res):
    return canon_groups(res.keys, res.aggs)


def canon_dev(gq, out, n, nk):
    cols = gq.read_table(out, n)
    keys = [(v.astype(np.int64), ok) for v, ok in cols[:nk]]
    return canon_groups(keys, cols[nk:])


def assert_same(got, exp, what):
    (gk, ga), (ek, ea) = got, exp
    assert len(gk) == len(ek) and len(ga) == len(ea), what
    for j, ((gv, gok), (ev, eok)) in enumerate(zip(gk + ga, ek + ea)):
        assert np.array_equal(gok, eok), (what, j, "validity")
        assert np.array_equal(gv, ev), (what, j, "values")


def state_table(res, key_types):
    """A group result as a state batch: key columns in their original types,
    then one int64 state column per aggregate (oracle.result_table keeps
    every key as int64)."""
    t = oracle.result_table(res)
    for j, dt in enumerate(key_types):
        t.cols[j].data = t.cols[j].data.astype(dt)
    return t


def state_aggs(aggs, nk):
    return [(a[0], [("col", nk + i)]) for i, a in enumerate(aggs)]


def key_nullable(batches, keys):
    return [any(b.cols[k].valid is not None for b in batches) for k in keys]


@pytest.mark.parametrize("keys", [[0], [1], [1, 3], []])
def test_one_shot_modes(gq, ctx, keys):
    rng = np.random.default_rng(3)
    t = random_table(rng, 30_000, TYPES, null_frac=0.1, lo=-30, hi=30)
    preds = [("range", 3, -20, 25)]
    d = gq.to_device(t)
    exp = oracle.groupby_mode(t, keys, preds, AGGS, "single")
    for mode in ("single", "partial"):
        out, cnt = ctx.groupby_agg(d, keys, preds, AGGS, mode=mode)
        ctx.raise_status()
        assert_same(canon_dev(gq, out, int(cnt.item()), len(keys)), canon_res(exp), mode)
    # State rows of two halves, concatenated, merged by the intermediate and
    # final modes: equal to the single aggregation of all rows.
    half = t.nrows // 2
    parts = []
    for lo, hi in ((0, half), (half, t.nrows)):
        sub = Table()
        for c in t.cols:
            sub.cols.append(Column(c.name, c.data[lo:hi], None if c.valid is None else c.valid[lo:hi]))
        parts.append(state_table(oracle.groupby_mode(sub, keys, preds, AGGS, "partial"), [TYPES[k] for k in keys]))
    states = oracle.concat_tables(parts)
    nk = len(keys)
    sd = gq.to_device(states)
    for mode in ("intermediate", "final"):
        out, cnt = ctx.groupby_agg(sd, list(range(nk)), [], state_aggs(AGGS, nk), mode=mode)
        ctx.raise_status()
        assert_same(canon_dev(gq, out, int(cnt.item()), nk), canon_res(exp), mode)
    with pytest.raises(gq.GqError):
        ctx.groupby_agg(sd, list(range(nk)), [("range", 0, 0, 1)], state_aggs(AGGS, nk), mode="final")


def run_stream(gq, ctx, batches, keys, preds, aggs, mode, emit_groups, max_groups=16384):
    types = [int(gq.np_to_type(b.cols[k].data.dtype)) for b in batches[:1] for k in keys]
    st = gq.AggStream(ctx, mode, keys, types, key_nullable(batches, keys), aggs, max_groups, emit_groups)
    emitted = []
    for i, b in enumerate(batches):
        r = st.push(gq.to_device(b), preds[i] if preds else ())
        if r is not None:
            out, cnt = r
            n = int(cnt.item())
            if n:
                emitted.append(canon_dev(gq, out, n, len(keys)))
    out, cnt = st.finish()
    ctx.raise_status()
    n, held = (int(x) for x in cnt.cpu().numpy())
    if held:
        emitted.append(canon_dev(gq, out, n, len(keys)))
    st.free()
    return emitted


@pytest.mark.parametrize("keys", [[0], [1, 3], []])
@pytest.mark.parametrize("mode,emit", [("single", 0), ("partial", 0), ("partial", 60), ("partial", 1)])
def test_stream_raw_batches(gq, ctx, keys, mode, emit):
    batches = raw_batches(11)
    preds = [[("range", 3, -30, 30 - i)] for i in range(len(batches))]
    got = run_stream(gq, ctx, batches, keys, preds, AGGS, mode, emit)
    exp = oracle.agg_stream(batches, keys, preds, AGGS, mode=mode, emit_groups=emit or None)
    assert len(got) == len(exp), (len(got), len(exp))
    for i, (g, e) in enumerate(zip(got, exp)):
        assert_same(g, canon_res(e), f"emission {i}")


@pytest.mark.parametrize("mode,emit", [("intermediate", 0), ("intermediate", 50), ("final", 0)])
def test_stream_state_batches(gq, ctx, mode, emit):
    # State batches: each the partial aggregation of one raw batch (oracle).
    raw = raw_batches(17, nb=10)
    keys = [1, 3]
    states = [state_table(oracle.groupby_mode(b, keys, [], AGGS, "partial"), [TYPES[k] for k in keys]) for b in raw]
    saggs = state_aggs(AGGS, 2)
    got = run_stream(gq, ctx, states, [0, 1], None, saggs, mode, emit)
    exp = oracle.agg_stream(states, [0, 1], None, saggs, mode=mode, emit_groups=emit or None)
    assert len(got) == len(exp)
    for i, (g, e) in enumerate(zip(got, exp)):
        assert_same(g, canon_res(e), f"emission {i}")


def test_partial_to_final_chain_equals_single(gq, ctx):
    # GPU Partial stream emitting every ~40 groups, its emissions fed to a GPU
    # Final stream: the result equals one Single aggregation of all raw rows.
    raw = raw_batches(23, nb=12, nkey=60)
    keys = [0]
    nullable = key_nullable(raw, keys)
    types = [int(gq.np_to_type(raw[0].cols[0].data.dtype))]
    part = gq.AggStream(ctx, "partial", keys, types, nullable, AGGS, 8192, emit_groups=40)
    fin = gq.AggStream(ctx, "final", [0], types, [True], state_aggs(AGGS, 1), 8192)
    pending = []
    for b in raw:
        out, cnt = part.push(gq.to_device(b))
        pending.append((out, cnt))
    out, cnt = part.finish()
    pending.append((out, cnt[:1]))
    nstates = 0
    for out, cnt in pending:
        n = int(cnt[0].item())
        if n:
            fin.push(out.head(n))
            nstates += 1
    assert nstates >= 3
    out, cnt = fin.finish()
    ctx.raise_status()
    n = int(cnt[0].item())
    alls = Table()
    for j, c in enumerate(raw[0].cols):
        data = np.concatenate([b.cols[j].data for b in raw])
        valid = np.concatenate([np.ones(b.nrows, bool) if b.cols[j].valid is None else b.cols[j].valid for b in raw])
        alls.cols.append(Column(c.name, data, valid))
    exp = oracle.groupby(alls, keys, [], AGGS)
    assert_same(canon_dev(gq, out, n, 1), canon_res(exp), "final")
    part.free()
    fin.free()


def test_stream_table_full_reported(gq, ctx):
    raw = raw_batches(5, nb=6, nkey=1000)
    st = gq.AggStream(ctx, "single", [0], [int(gq.np_to_type(np.int64))], [True], AGGS, max_groups=16)
    for b in raw:
        st.push(gq.to_device(b))
    st.finish()
    bits = ctx.sync_status()
    assert bits & gq.DEV_TABLE_FULL
    st.free()
