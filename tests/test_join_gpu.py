"""Join build/probe, gather and the fused pipeline on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import assert_col_equal, canon_groups, random_table, tbl

pytestmark = pytest.mark.gpu

REV = [("col", 1), ("k-col", 100, 2)]


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def gpu_join(gq, ctx, build, bkeys, bpreds, probe, pkeys, ppreds, lf=0.0, capacity=None):
    bd, pd_ = gq.to_device(build), gq.to_device(probe)
    jt = ctx.join_build(bd, bkeys, bpreds, load_factor=lf)
    if capacity is None:
        # Two-phase use: a count-only probe (capacity 0), then the sized one.
        _, _, cnt0 = ctx.join_probe(jt, pd_, pkeys, ppreds, capacity=0)
        ctx.sync_status()
        cap = int(cnt0.item())
    else:
        cap = capacity
    pi, bi, cnt = ctx.join_probe(jt, pd_, pkeys, ppreds, capacity=cap)
    bits = ctx.sync_status()
    n = int(cnt.item())
    out = (pi[:min(n, cap)].cpu().numpy(), bi[:min(n, cap)].cpu().numpy(), n, bits)
    jt.free()
    return out


def check_join(gq, ctx, build, bkeys, bpreds, probe, pkeys, ppreds, lf=0.0):
    pi, bi, n, bits = gpu_join(gq, ctx, build, bkeys, bpreds, probe, pkeys, ppreds, lf)
    assert bits == 0
    epi, ebi = oracle.join(build, bkeys, bpreds, probe, pkeys, ppreds)
    assert n == len(epi)
    assert np.array_equal(pi, epi) and np.array_equal(bi, ebi)


@pytest.mark.parametrize("lf", [0.25, 0.5, 0.9])
def test_join_unique_keys(gq, ctx, lf):
    dim = dg.dim_c2(100_000, seed=5)
    fact = dg.fact_c2(400_003, nkeys=100_000, seed=5)
    check_join(gq, ctx, dim, [0], [("range", 1, 0, 1202)], fact, [0], [("range", 3, 1278, 2555)], lf)


@pytest.mark.parametrize("seed", range(4))
def test_join_duplicates_and_nulls(gq, ctx, seed):
    rng = np.random.default_rng(seed)
    nb, npr = int(rng.integers(1, 30_000)), int(rng.integers(1, 60_000))
    dom = int(rng.integers(1, 5_000))
    bk = rng.integers(-dom, dom, nb)
    pk = rng.integers(-dom, dom, npr).astype(np.int32)
    build = tbl(k=(bk, rng.random(nb) > 0.1), d=rng.integers(0, 100, nb).astype(np.int8))
    probe = tbl(k=(pk, rng.random(npr) > 0.1), d=rng.integers(0, 100, npr).astype(np.int16))
    check_join(gq, ctx, build, [0], [("range", 1, 0, 70)], probe, [0], [("ne", 1, 3)])


def test_join_long_runs(gq, ctx):
    # One key with 5000 build rows, one with 40; every probe row matches one of them.
    bk = np.concatenate([np.full(5000, 7), np.full(40, 9), np.arange(100, 200)])
    rng = np.random.default_rng(1)
    rng.shuffle(bk)
    pk = np.array([7, 9, 150, 7, 3, 9], dtype=np.int64)
    check_join(gq, ctx, tbl(k=bk.astype(np.int64)), [0], [], tbl(k=pk), [0], [])


def test_join_special_keys(gq, ctx):
    lo, hi = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    b = tbl(k=np.array([lo, hi, -1, 0, -1, 5], dtype=np.int64))
    p = tbl(k=np.array([hi, lo, -1, 5, 6, -1, 0], dtype=np.int64))
    check_join(gq, ctx, b, [0], [], p, [0], [])


@pytest.mark.parametrize("nb,np_", [(0, 10), (10, 0), (0, 0), (1, 1), (64, 65)])
def test_join_tiny(gq, ctx, nb, np_):
    rng = np.random.default_rng(nb * 100 + np_)
    b = tbl(k=rng.integers(0, 5, nb))
    p = tbl(k=rng.integers(0, 5, np_))
    check_join(gq, ctx, b, [0], [], p, [0], [])


def test_join_capacity(gq, ctx):
    b = tbl(k=np.arange(1000, dtype=np.int64))
    p = tbl(k=np.arange(1000, dtype=np.int64))
    pi, bi, n, bits = gpu_join(gq, ctx, b, [0], [], p, [0], [], capacity=100)
    assert bits & 1 and n == 1000
    assert np.array_equal(pi, np.arange(100))


def test_gather(gq, ctx):
    rng = np.random.default_rng(9)
    t = random_table(rng, 5000, null_frac=0.3)
    idx = rng.integers(0, 5000, 7777).astype(np.int32)
    import torch
    out = ctx.gather(gq.to_device(t), [0, 1, 2, 3], torch.from_numpy(idx).cuda())
    ctx.raise_status()
    got = gq.read_table(out, len(idx))
    for j, c in enumerate(t.cols):
        assert_col_equal(got[j], c.data[idx], c.valid[idx], f"col {j}")


def check_pipeline(gq, ctx, probe, ppreds, gkeys, aggs, join_spec=None, acc_slots=0, **kw):
    pdv = gq.to_device(probe)
    jt = None
    if join_spec is not None:
        build, bkeys, bpreds, pkey = join_spec
        jt = ctx.join_build(gq.to_device(build), bkeys, bpreds, acc_slots=acc_slots)
    out, cnt = ctx.pipeline(pdv, ppreds, gkeys, aggs, join=jt, probe_key=join_spec[3] if join_spec else 0, **kw)
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    cols = gq.read_table(out, n)
    if jt:
        jt.free()
    spec = None if join_spec is None else (join_spec[0], join_spec[1], join_spec[2], [join_spec[3]])
    exp = oracle.pipeline(probe, ppreds, gkeys, aggs, join_spec=spec)
    assert n == exp.nrows
    gk = [(v.astype(np.int64), ok) for v, ok in cols[:len(gkeys)]]
    gk, ga = canon_groups(gk, cols[len(gkeys):])
    ek, ea = canon_groups(exp.keys, exp.aggs)
    for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
        assert np.array_equal(gok, eok) and np.array_equal(gv, ev)


@pytest.mark.parametrize("acc_slots", [0, 2])
def test_pipeline_config2_shape(gq, ctx, acc_slots):
    n_dim, n_fact = 150_000, 600_000
    dim = dg.dim_c2(n_dim, seed=8)
    fact = dg.fact_c2(n_fact, nkeys=n_dim, seed=8)
    check_pipeline(gq, ctx, fact, [("range", 3, 1278, 2555)], [0], [("sum", REV), ("count*",)],
                   join_spec=(dim, [0], [("range", 1, 0, 1202)], 0), acc_slots=acc_slots)


@pytest.mark.parametrize("acc_slots", [0, 6])
def test_pipeline_duplicates_minmax(gq, ctx, acc_slots):
    rng = np.random.default_rng(21)
    nb, npr = 20_000, 90_000
    build = tbl(k=rng.integers(0, 3000, nb), d=rng.integers(0, 10, nb).astype(np.int32))
    probe = tbl(k=(rng.integers(0, 3500, npr), rng.random(npr) > 0.05),
                v=(rng.integers(-1000, 1000, npr), rng.random(npr) > 0.1),
                g=rng.integers(0, 7, npr).astype(np.int8))
    # 2 + 0 + 2 + 1 accumulator words after the hidden count: fits a 6-word group-join slot
    aggs = [("sum", [("col", 1)]), ("count*",), ("min", [("col", 1)]), ("max", [("col", 2)])]
    # group by the probe key (group-join when acc_slots allows) and by another column
    check_pipeline(gq, ctx, probe, [], [0], aggs, join_spec=(build, [0], [("range", 1, 0, 6)], 0),
                   acc_slots=acc_slots)
    check_pipeline(gq, ctx, probe, [], [2], aggs, join_spec=(build, [0], [("range", 1, 0, 6)], 0),
                   acc_slots=acc_slots)


def test_pipeline_general_aggs_with_join(gq, ctx):
    rng = np.random.default_rng(22)
    build = tbl(k=rng.integers(0, 500, 3000))
    probe = tbl(k=rng.integers(0, 600, 20_000), v=(rng.integers(-9, 9, 20_000), rng.random(20_000) > 0.2))
    aggs = [("sum", [("col", 1)]), ("count*",), ("count", [("col", 1)]), ("min", [("col", 1)]),
            ("max", [("col", 1)])]
    check_pipeline(gq, ctx, probe, [], [0], aggs, join_spec=(build, [0], [], 0), acc_slots=6)


def test_pipeline_without_join(gq, ctx):
    t = dg.fact_c1(300_000, seed=4)
    check_pipeline(gq, ctx, t, [("range", 3, 0, 2466)], [4, 5],
                   [("sum", [("col", 0)]), ("sum", REV), ("count*",)], strategy="lds")


def test_partitioned_table_index_from_two_streams(gq, ctx):
    # A build side of 2^20 rows is stored partitioned; the first probe builds
    # its index lazily on its own stream.  A second probe, enqueued on another
    # stream right after, must see the complete index (the table's event is
    # re-recorded after the index build), and both must equal the oracle.
    import torch
    nd = 1 << 20
    dim = dg.dim_c2(nd, seed=21)
    fact = dg.fact_c2(600_000, nkeys=nd, seed=21)
    bpred, ppred = [("range", 1, 0, 1202)], [("range", 3, 1278, 2555)]
    bd, pd_ = gq.to_device(dim), gq.to_device(fact)
    epi, ebi = oracle.join(dim, [0], bpred, fact, [0], ppred)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    jt = ctx.join_build(bd, [0], bpred)
    cap = len(epi) + 16
    with torch.cuda.stream(s1):
        r1 = ctx.join_probe(jt, pd_, [0], ppred, capacity=cap, stream=s1)
    with torch.cuda.stream(s2):
        r2 = ctx.join_probe(jt, pd_, [0], ppred, capacity=cap, stream=s2)
    torch.cuda.synchronize()
    assert ctx.sync_status() == 0
    for pi, bi, cnt in (r1, r2):
        n = int(cnt.item())
        assert n == len(epi)
        assert np.array_equal(pi[:n].cpu().numpy(), epi) and np.array_equal(bi[:n].cpu().numpy(), ebi)
    torch.cuda.current_stream().wait_stream(s1)
    torch.cuda.current_stream().wait_stream(s2)
    jt.free()
