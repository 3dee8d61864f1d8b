"""Full-size parity in the launch configuration bench.py times.

The 60M x 15M pipeline and the 60M-row partition are too large for the oracle
to recompute whole in seconds, so these tests check
  * properties that hold at any size (key uniqueness and range, total counts
    against a hash-free dense formulation, offsets against the oracle; for the
    pipeline, every group's SUM and COUNT against per-key totals of the joined
    rows), and
  * sampled outputs the oracle computes exactly: the oracle runs on the subset
    of input rows that can contribute to the sampled groups / positions.
Inputs are generated on the device by the seeded generator (equal to the host
generator, see test_devgen_gpu.py); the host side regenerates only the columns
and rows the checks need.
"""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from paper_2606_24647_amd.datagen import Column, Table

pytestmark = pytest.mark.gpu

FACT, DIM = 60_000_000, 15_000_000
REV = [("col", 1), ("k-col", 100, 2)]
AGGS = [("sum", REV), ("count*",)]
FPRED, DPRED = [("range", 3, 1278, 2555)], [("range", 1, 0, 1202)]


@pytest.fixture(scope="module")
def mods():
    from paper_2606_24647_amd import devgen, gq
    return gq, devgen


def test_pipeline_fact60m_dim15m(mods):
    gq, devgen = mods
    import torch
    ctx = gq.Context()
    dim = devgen.dim_c2(DIM)
    fact = devgen.fact_c2(FACT, DIM)
    jt = ctx.join_build(dim, [0], DPRED, load_factor=0.5, acc_slots=2)
    out, cnt = ctx.pipeline(fact, FPRED, [0], AGGS, join=jt, probe_key=0, capacity=DIM)
    ctx.raise_status()
    n = int(cnt.item())
    gk, gsum, gcnt = (c.data[:n].cpu().numpy() for c in out.cols)
    jt.free()
    del dim, fact, out
    torch.cuda.empty_cache()

    # Properties at full size.
    assert len(np.unique(gk)) == n and gk.min() >= 1 and gk.max() <= DIM
    fkey = dg.uniform(2, 0, 0, FACT, 1, DIM)
    fdate = dg.uniform(2, 3, 0, FACT, 0, dg.DATE_DAYS - 1, np.int32)
    pkey = dg.permutation(2, 16, 0, DIM, DIM) + 1
    ddate = dg.uniform(2, 17, 0, DIM, 0, dg.DIM_DATE_DAYS - 1, np.int32)
    inv = np.empty(DIM + 1, dtype=np.int64)
    inv[pkey] = np.arange(DIM)
    ok = (fdate >= 1278) & (ddate[inv[fkey]] <= 1202)
    assert int(gcnt.sum()) == int(ok.sum())
    assert n == len(np.unique(fkey[ok]))
    # Complete and hash-free: the revenue sums of all groups add up to the
    # revenue of all joined rows (int64, wrapping as the device does).
    price = dg.uniform(2, 1, 0, FACT, dg.PRICE_LO, dg.PRICE_HI)
    disc = dg.uniform(2, 2, 0, FACT, 0, 10)
    rev = price[ok] * (100 - disc[ok])
    assert int(np.sum(gsum, dtype=np.int64)) == int(np.sum(rev, dtype=np.int64))
    # Complete: every group's SUM and COUNT against per-key totals of the
    # joined rows.  The float64 per-key sums are exact: each partial sum is an
    # integer below 2^53 (bounded by the largest revenue times the largest
    # group).
    ecnt = np.bincount(fkey[ok], minlength=DIM + 1)
    assert int(rev.max()) * int(ecnt.max()) < 2**53
    esum = np.bincount(fkey[ok], weights=rev.astype(np.float64), minlength=DIM + 1)
    assert np.array_equal(ecnt[gk], gcnt)
    assert np.array_equal(esum[gk].astype(np.int64), gsum)
    del price, disc, rev, ecnt, esum

    # Sampled groups, exactly, by the oracle on the rows that can reach them.
    rng = np.random.default_rng(0)
    pick = rng.choice(n, 2000, replace=False)
    absent = np.setdiff1d(rng.integers(1, DIM + 1, 400), gk)[:200]
    sample = np.concatenate([gk[pick], absent])
    frows = np.flatnonzero(np.isin(fkey, sample))
    drows = inv[sample]
    sub_fact = Table([Column("fkey", fkey[frows]),
                      Column("price", dg.uniform_at(2, 1, frows, dg.PRICE_LO, dg.PRICE_HI)),
                      Column("disc", dg.uniform_at(2, 2, frows, 0, 10)),
                      Column("date", fdate[frows])])
    sub_dim = Table([Column("pkey", pkey[drows]), Column("date", ddate[drows])])
    exp = oracle.pipeline(sub_fact, FPRED, [0], AGGS, join_spec=(sub_dim, [0], DPRED, [0]))
    got = dict(zip(gk[pick].tolist(), zip(gsum[pick].tolist(), gcnt[pick].tolist())))
    expd = dict(zip(exp.keys[0][0].tolist(), zip(exp.aggs[0][0].tolist(), exp.aggs[1][0].tolist())))
    assert set(expd) == set(got), "sampled groups present on one side only"
    assert all(expd[k] == got[k] for k in got)
    assert not (set(absent.tolist()) & set(expd)), "a group missing from the GPU output exists"


@pytest.fixture(scope="module")
def c3_keys():
    return dg.zipf(3, 0, 0, FACT, DIM)


@pytest.mark.parametrize("P", [64, 256])
def test_partition_60m(mods, c3_keys, P):
    gq, devgen = mods
    import torch
    ctx = gq.Context()
    t = devgen.batch_c3(FACT, DIM)
    out, offs = ctx.hash_partition(t, [0], P)
    ctx.raise_status()
    okey = out.cols[0].data.cpu().numpy()
    offs = offs.cpu().numpy()
    pos = np.sort(np.random.default_rng(P).choice(FACT, 20_000, replace=False))
    osamp = [c.data[torch.from_numpy(pos).cuda()].cpu().numpy() for c in out.cols[1:]]
    del t, out
    torch.cuda.empty_cache()

    key = c3_keys
    perm, eoff = oracle.partition(Table([Column("key", key)]), [0], P, 0)
    assert np.array_equal(offs, eoff)
    assert np.array_equal(okey, key[perm])
    rows = perm[pos]
    exp = [dg.uniform_at(3, 1, rows, dg.PRICE_LO, dg.PRICE_HI),
           dg.uniform_at(3, 2, rows, 0, dg.DATE_DAYS - 1, np.int32),
           dg.uniform_at(3, 3, rows, 0, 2, np.int8)]
    for g, e in zip(osamp, exp):
        assert np.array_equal(g, e)


C1_AGGS = [("sum", [("col", 0)]), ("sum", [("col", 1)]), ("sum", [("col", 2)]), ("sum", REV), ("count*",)]


def test_batched_4096_fragments(mods):
    """The whole batched workload (4,096 fragments, about 2e9 rows resident) in
    one plan with the default configuration, as the bench launches it: every
    fragment's COUNT(*) total and group count against properties computed on
    the device, and sampled fragments (the largest, the one with the most
    groups, LDS- and radix-routed ones) against the oracle exactly."""
    gq, devgen = mods
    import torch
    from tests.helpers import canon_groups
    ctx = gq.Context()
    spec, tables, cols, starts = devgen.fragments_c4_resident(4096)
    preds = [[("range", 3, 0, int(b))] for b in spec.bound]
    plan = gq.BatchPlan(ctx, [(t, p, int(c)) for t, p, c in zip(tables, preds, spec.card)], [4], C1_AGGS)
    plan.launch()
    plan.launch()          # a replay reproduces the first launch's results
    ctx.raise_status()
    ng = plan.d_groups.cpu().numpy()
    assert (ng >= 0).all() and (ng <= np.minimum(spec.rows, spec.card)).all()
    # COUNT(*) summed per fragment equals the rows that pass its filter.
    got_cnt, exp_cnt, nonempty = [], [], []
    for f, t in enumerate(tables):
        n = int(spec.rows[f])
        exp_cnt.append((cols[3][int(starts[f]):int(starts[f]) + n] <= int(spec.bound[f])).sum())
        got_cnt.append(plan.outs[f].cols[-1].data[:int(ng[f])].sum())
    got_cnt = torch.stack(got_cnt).cpu().numpy()
    exp_cnt = torch.stack(exp_cnt).cpu().numpy()
    assert np.array_equal(got_cnt, exp_cnt)
    assert ((ng > 0) == (exp_cnt > 0)).all()

    rng = np.random.default_rng(11)
    lds = np.flatnonzero(spec.card <= 256)
    rad = np.flatnonzero(spec.card > 256)
    pick = {int(np.argmax(spec.rows)), int(np.argmax(spec.card)), int(np.argmin(spec.rows))}
    pick |= set(rng.choice(lds, 4, replace=False).tolist()) | set(rng.choice(rad, 6, replace=False).tolist())
    for f in sorted(pick):
        host = dg.fragment_c4(f, int(spec.rows[f]), int(spec.card[f]))
        exp = oracle.groupby(host, [4], preds[f], C1_AGGS)
        ek, ea = canon_groups(exp.keys, exp.aggs)
        res, n = plan.result(f)
        assert n == exp.nrows, f
        gk, ga = canon_groups([(v.astype(np.int64), ok) for v, ok in res[:1]], res[1:])
        for (gv, gok), (ev, eok) in zip(gk + ga, ek + ea):
            assert np.array_equal(gv, ev) and np.array_equal(gok, eok), f
    plan.free()
    del tables, cols
    torch.cuda.empty_cache()
