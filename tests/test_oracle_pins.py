"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: a brute-force
loop on tiny inputs, a numpy/pandas library routine, a closed form, an
independently written inverse, or an invariant.  The choices are such that a
plausible slip in the oracle (a dropped hash step, a wrong shift or constant,
a flipped comparison, a lost NULL rule, a reordered output) fails at least one.
"""
import itertools
import json
import os
import random

import numpy as np
import pandas as pd
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from paper_2606_24647_amd.datagen import Column, Table

M64 = (1 << 64) - 1
HERE = os.path.dirname(os.path.abspath(__file__))


def tbl(**cols):
    out = Table()
    for name, v in cols.items():
        if isinstance(v, tuple):
            out.cols.append(Column(name, np.asarray(v[0]), np.asarray(v[1], dtype=bool)))
        else:
            out.cols.append(Column(name, np.asarray(v)))
    return out


# ---------------------------------------------------------------------------
# Hash (the partitioning hash reading: MurmurHash3 fmix64 chain)
# ---------------------------------------------------------------------------

def _inv_fmix64(h: int) -> int:
    """Inverse of the finaliser, written from its structure, not its code.

    Each of the five steps is a bijection of Z/2^64: x ^= x >> 33 is its own
    inverse (33 >= 32, so the shifted part never overlaps itself), and
    multiplication by an odd constant is undone by its modular inverse.
    """
    c1, c2 = 0xFF51AFD7ED558CCD, 0xC4CEB9FE1A85EC53
    x = h
    x ^= x >> 33
    x = (x * pow(c2, -1, 1 << 64)) & M64
    x ^= x >> 33
    x = (x * pow(c1, -1, 1 << 64)) & M64
    x ^= x >> 33
    return x


def test_fmix64_closed_form_zero():
    assert oracle.fmix64(0) == 0


def test_fmix64_inverts():
    rng = random.Random(7)
    xs = [0, 1, 2, M64, 1 << 63, 0x0123456789ABCDEF] + [rng.getrandbits(64) for _ in range(2000)]
    for x in xs:
        assert _inv_fmix64(oracle.fmix64(x)) == x


def test_fmix64_avalanche():
    # Every input bit flips each output bit with probability close to 1/2.
    rng = random.Random(11)
    n = 400
    flips = np.zeros((64, 64))
    for _ in range(n):
        x = rng.getrandbits(64)
        hx = oracle.fmix64(x)
        for b in range(64):
            d = hx ^ oracle.fmix64(x ^ (1 << b))
            for o in range(64):
                flips[b, o] += (d >> o) & 1
    p = flips / n
    assert p.min() > 0.35 and p.max() < 0.65


def test_row_hash_chain_and_nulls():
    rng = np.random.default_rng(3)
    a = rng.integers(-(1 << 62), 1 << 62, 500)
    b = rng.integers(-100, 100, 500).astype(np.int8)
    valid_b = rng.random(500) > 0.3
    seed = 0x1234_5678_9ABC_DEF0
    t = tbl(a=a, b=(b, valid_b))
    h = oracle.hash_rows(t, [0, 1], seed)
    for i in range(500):
        # Undo the chain with the independent inverse: h = f(f(seed ^ a) ^ b').
        bv = int(b[i]) & M64 if valid_b[i] else 0          # int8 sign-extended; NULL hashes as 0
        inner = _inv_fmix64(int(h[i])) ^ bv
        assert _inv_fmix64(inner) ^ seed == int(a[i]) & M64
    # Order of key columns matters.
    h2 = oracle.hash_rows(t, [1, 0], seed)
    assert (h != h2).mean() > 0.99


def test_row_hash_sign_extension():
    v = np.array([-1, -128, 127, 0], dtype=np.int8)
    h8 = oracle.hash_rows(tbl(x=v), [0], 0)
    h64 = oracle.hash_rows(tbl(x=v.astype(np.int64)), [0], 0)
    h32 = oracle.hash_rows(tbl(x=v.astype(np.int32)), [0], 0)
    assert np.array_equal(h8, h64) and np.array_equal(h32, h64)


@pytest.mark.parametrize("P", [1, 2, 4, 64, 256, 65536])
def test_partition_of_power_of_two_is_top_bits(P):
    rng = random.Random(P)
    shift = 64 - (P.bit_length() - 1)
    for _ in range(500):
        h = rng.getrandbits(64)
        expect = 0 if P == 1 else h >> shift
        assert oracle.partition_of(h, P) == expect


def test_partition_of_general_P():
    # floor(h * P / 2^64) equals the integer division of the exact product.
    rng = random.Random(5)
    for P in [3, 7, 1000, 65535]:
        for _ in range(200):
            h = rng.getrandbits(64)
            assert oracle.partition_of(h, P) == (h * P) >> 64
        assert oracle.partition_of(M64, P) == P - 1 and oracle.partition_of(0, P) == 0


# ---------------------------------------------------------------------------
# Filter
# ---------------------------------------------------------------------------

def test_filter_matches_flatnonzero():
    t = dg.fact_c1(50_000, seed=9, null_permille=50)
    preds = [("range", 3, 100, 2000), ("ne", 4, 1), ("range", 0, 5, 45)]
    rows = oracle.filter_rows(t, preds)
    sd, fl, q = t["shipdate"], t["flag"], t["qty"]
    mask = (sd.valid & (sd.data >= 100) & (sd.data <= 2000) & fl.valid & (fl.data != 1)
            & q.valid & (q.data >= 5) & (q.data <= 45))
    assert np.array_equal(rows, np.flatnonzero(mask))
    assert len(rows) == int(mask.sum())


def test_filter_empty_and_trivial():
    t = tbl(x=np.arange(10, dtype=np.int32))
    assert np.array_equal(oracle.filter_rows(t, []), np.arange(10))
    assert len(oracle.filter_rows(t, [("range", 0, 5, 4)])) == 0
    e = tbl(x=np.zeros(0, dtype=np.int64))
    assert len(oracle.filter_rows(e, [("range", 0, 0, 1)])) == 0
    # Inclusive bounds at both ends; NE drops only the value.
    assert list(oracle.filter_rows(t, [("range", 0, 3, 5)])) == [3, 4, 5]
    assert list(oracle.filter_rows(t, [("ne", 0, 7)])) == [0, 1, 2, 3, 4, 5, 6, 8, 9]


def test_filter_int64_extremes():
    v = np.array([np.iinfo(np.int64).min, -1, 0, 1, np.iinfo(np.int64).max], dtype=np.int64)
    t = tbl(x=v)
    lo, hi = int(np.iinfo(np.int64).min), int(np.iinfo(np.int64).max)
    assert list(oracle.filter_rows(t, [("range", 0, lo, -1)])) == [0, 1]
    assert list(oracle.filter_rows(t, [("range", 0, 0, hi)])) == [2, 3, 4]


# ---------------------------------------------------------------------------
# Hash partition
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("P", [1, 2, 3, 64, 256])
def test_partition_matches_stable_argsort(P):
    t = dg.batch_c3(20_000, nkeys=5_000, seed=13, null_permille=20)
    perm, off = oracle.partition(t, [0], P, seed=0)
    h = oracle.hash_rows(t, [0], 0)
    p = np.array([(int(x) * P) >> 64 for x in h], dtype=np.int64)
    assert np.array_equal(perm, np.argsort(p, kind="stable"))
    counts = np.bincount(p, minlength=P)
    assert np.array_equal(np.diff(off), counts)
    assert off[0] == 0 and off[-1] == t.nrows
    for q in range(P):
        seg = perm[off[q]:off[q + 1]]
        assert (p[seg] == q).all()
        assert (np.diff(seg) > 0).all()          # stable: row ids increase
    if P == 1:
        assert np.array_equal(perm, np.arange(t.nrows))


def test_partition_multikey_and_empty():
    t = tbl(a=np.array([1, 2, 1, 2, 1], dtype=np.int64), b=np.array([5, 5, 5, 6, 5], dtype=np.int16))
    perm, off = oracle.partition(t, [0, 1], 8, seed=99)
    # Equal key tuples land in the same partition, in input order.
    where = {}
    for q in range(8):
        for r in perm[off[q]:off[q + 1]]:
            where[int(r)] = q
    assert where[0] == where[2] == where[4]
    e = tbl(a=np.zeros(0, dtype=np.int64))
    perm, off = oracle.partition(e, [0], 4)
    assert len(perm) == 0 and list(off) == [0, 0, 0, 0, 0]


# ---------------------------------------------------------------------------
# Join
# ---------------------------------------------------------------------------

def _brute_join(bk, bv, bpass, pk, pv, ppass):
    out = []
    for i in range(len(pk)):
        if not (ppass[i] and pv[i]):
            continue
        for j in range(len(bk)):
            if bpass[j] and bv[j] and bk[j] == pk[i]:
                out.append((i, j))
    return out


@pytest.mark.parametrize("seed", range(4))
def test_join_two_keys_brute_force(seed):
    # Key tuples: a pair matches when both columns are non-NULL and equal.
    rng = np.random.default_rng(100 + seed)
    nb, npr = int(rng.integers(1, 200)), int(rng.integers(1, 300))
    ba, bb = rng.integers(-4, 4, nb), rng.integers(-3, 3, nb).astype(np.int16)
    pa, pb = rng.integers(-4, 4, npr).astype(np.int32), rng.integers(-3, 3, npr).astype(np.int8)
    bva, bvb = rng.random(nb) > 0.1, rng.random(nb) > 0.1
    pva, pvb = rng.random(npr) > 0.1, rng.random(npr) > 0.1
    build, probe = tbl(a=(ba, bva), b=(bb, bvb)), tbl(a=(pa, pva), b=(pb, pvb))
    pi, bi = oracle.join(build, [0, 1], [], probe, [0, 1], [])
    expect = [(i, j) for i in range(npr) for j in range(nb)
              if pva[i] and pvb[i] and bva[j] and bvb[j] and pa[i] == ba[j] and pb[i] == bb[j]]
    assert list(zip(pi.tolist(), bi.tolist())) == expect
    # The key order is the caller's: swapping both sides' key lists changes nothing.
    pi2, bi2 = oracle.join(build, [1, 0], [], probe, [1, 0], [])
    assert np.array_equal(pi, pi2) and np.array_equal(bi, bi2)


@pytest.mark.parametrize("seed", range(6))
def test_join_brute_force(seed):
    rng = np.random.default_rng(seed)
    nb, npr = int(rng.integers(0, 300)), int(rng.integers(0, 400))
    dom = int(rng.integers(1, 60))
    bk = rng.integers(-dom, dom, nb)
    pk = rng.integers(-dom, dom, npr).astype(np.int32)
    bvalid = rng.random(nb) > 0.1
    pvalid = rng.random(npr) > 0.1
    bd = rng.integers(0, 100, nb).astype(np.int32)
    pd_ = rng.integers(0, 100, npr).astype(np.int32)
    build = tbl(k=(bk, bvalid), d=bd)
    probe = tbl(k=(pk, pvalid), d=pd_)
    pi, bi = oracle.join(build, [0], [("range", 1, 0, 59)], probe, [0], [("range", 1, 30, 99)])
    expect = _brute_join(bk, bvalid, (bd >= 0) & (bd <= 59), pk, pvalid, (pd_ >= 30) & (pd_ <= 99))
    assert list(zip(pi.tolist(), bi.tolist())) == expect


def test_join_pandas_and_cardinality():
    rng = np.random.default_rng(42)
    bk = rng.integers(0, 2000, 20_000)
    pk = rng.integers(0, 2500, 50_000)
    pi, bi = oracle.join(tbl(k=bk), [0], [], tbl(k=pk), [0], [])
    m = pd.merge(pd.DataFrame({"k": pk, "i": np.arange(len(pk))}),
                 pd.DataFrame({"k": bk, "j": np.arange(len(bk))}), on="k")
    m = m.sort_values(["i", "j"], kind="stable")
    assert np.array_equal(pi, m["i"].to_numpy()) and np.array_equal(bi, m["j"].to_numpy())
    ub, cb = np.unique(bk, return_counts=True)
    up, cp = np.unique(pk, return_counts=True)
    common, ib, ip = np.intersect1d(ub, up, return_indices=True)
    assert len(pi) == int((cb[ib] * cp[ip]).sum())


def test_join_permutation_closed_form():
    # Dim keys are a permutation of 1..n: the match of fact row i is inv[fkey[i]].
    n, m = 40_000, 160_000
    dim = dg.dim_c2(n, seed=21)
    fact = dg.fact_c2(m, nkeys=n, seed=21)
    pi, bi = oracle.join(dim, [0], [("range", 1, 0, 1202)], fact, [0], [("range", 3, 1278, 2555)])
    inv = np.empty(n + 1, dtype=np.int64)
    inv[dim["pkey"].data] = np.arange(n)
    j = inv[fact["fkey"].data]
    ok = (fact["date"].data >= 1278) & (dim["date"].data[j] <= 1202)
    assert np.array_equal(pi, np.flatnonzero(ok))
    assert np.array_equal(bi, j[ok])


def test_join_int64_extremes_and_empty():
    lo, hi = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    b = tbl(k=np.array([lo, hi, 0, lo], dtype=np.int64))
    p = tbl(k=np.array([hi, lo, 5], dtype=np.int64))
    pi, bi = oracle.join(b, [0], [], p, [0], [])
    assert list(zip(pi, bi)) == [(0, 1), (1, 0), (1, 3)]
    e = tbl(k=np.zeros(0, dtype=np.int64))
    assert len(oracle.join(e, [0], [], p, [0], [])[0]) == 0
    assert len(oracle.join(b, [0], [], e, [0], [])[0]) == 0


# ---------------------------------------------------------------------------
# Group-by
# ---------------------------------------------------------------------------

def test_groupby_hand_worked_example():
    # Six rows worked by hand.
    #   g: 2 1 2 - 1 2     (- = NULL)
    #   x: 5 7 - 4 1 3     (- = NULL)
    # groups in canonical order: NULL, 1, 2
    #   NULL: rows {3}    sum x = 4,  count* = 1, count x = 1, min 4, max 4
    #   1:    rows {1,4}  sum x = 8,  count* = 2, count x = 2, min 1, max 7
    #   2:    rows {0,2,5} sum x = 8, count* = 3, count x = 2, min 3, max 5
    g = (np.array([2, 1, 2, 9, 1, 2], dtype=np.int8), [1, 1, 1, 0, 1, 1])
    x = (np.array([5, 7, 0, 4, 1, 3], dtype=np.int64), [1, 1, 0, 1, 1, 1])
    t = tbl(g=g, x=x)
    X = [("col", 1)]
    r = oracle.groupby(t, [0], [], [("sum", X), ("count*",), ("count", X), ("min", X), ("max", X)])
    assert r.nrows == 3
    assert list(r.keys[0][1]) == [False, True, True]
    assert list(r.keys[0][0][1:]) == [1, 2]
    assert [list(a[0]) for a in r.aggs] == [[4, 8, 8], [1, 2, 3], [1, 2, 2], [4, 1, 3], [4, 7, 5]]
    assert all(a[1].all() for a in r.aggs)
    # Filter g >= 2 leaves one group; SUM over only NULL inputs is NULL.
    r2 = oracle.groupby(tbl(g=g, x=(x[0], [1, 1, 0, 1, 1, 0])), [0], [("range", 0, 2, 2)],
                        [("sum", X), ("count*",)])
    assert r2.nrows == 1 and list(r2.aggs[0][0]) == [5] and list(r2.aggs[1][0]) == [3]
    r3 = oracle.groupby(tbl(g=g, x=(x[0], [0, 1, 0, 1, 1, 0])), [0], [("range", 0, 2, 2)],
                        [("sum", X), ("count*",), ("min", X)])
    assert list(r3.aggs[0][1]) == [False] and list(r3.aggs[1][0]) == [3] and list(r3.aggs[2][1]) == [False]


def _brute_groupby(keys_cols, preds_mask, factor_fn, n):
    groups = {}
    for i in range(n):
        if not preds_mask[i]:
            continue
        k = tuple((1, int(v[i])) if ok[i] else (0, 0) for v, ok in keys_cols)
        acc = groups.setdefault(k, [0, 0])
        val = factor_fn(i)
        acc[0] += 1
        if val is not None:
            acc[1] = (acc[1] + val) & M64
    return dict(sorted(groups.items()))


@pytest.mark.parametrize("seed", range(5))
def test_groupby_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(0, 600))
    a = rng.integers(-3, 3, n).astype(np.int16)
    av = rng.random(n) > 0.15
    b = rng.integers(0, 4, n).astype(np.int64)
    bv = rng.random(n) > 0.05
    p = rng.integers(-(1 << 40), 1 << 40, n)
    pv = rng.random(n) > 0.1
    d = rng.integers(0, 11, n)
    t = tbl(a=(a, av), b=(b, bv), p=(p, pv), d=d)
    keep = rng.integers(0, 100, n)
    t.cols.append(Column("f", keep.astype(np.int32)))
    expr = [("col", 2), ("k-col", 100, 3), ("const", 3)]
    r = oracle.groupby(t, [0, 1], [("range", 4, 10, 89)], [("count*",), ("sum", expr)])
    mask = (keep >= 10) & (keep <= 89)

    def val(i):
        if not pv[i]:
            return None
        return (int(p[i]) * (100 - int(d[i])) * 3) & M64

    exp = _brute_groupby([(a, av), (b, bv)], mask, val, n)
    got_keys = []
    for gi in range(r.nrows):
        got_keys.append(tuple((1, int(r.keys[j][0][gi])) if r.keys[j][1][gi] else (0, 0) for j in range(2)))
    assert got_keys == list(exp.keys())
    assert list(r.aggs[0][0]) == [v[0] for v in exp.values()]
    assert [int(x) & M64 for x in r.aggs[1][0]] == [v[1] for v in exp.values()]


def test_groupby_sorted_reduceat_and_invariants():
    t = dg.fact_c1(200_000, seed=17)
    keys = [4, 5]
    preds = [("range", 3, 0, 2466)]
    rev = [("col", 1), ("k-col", 100, 2)]
    aggs = [("sum", [("col", 0)]), ("sum", [("col", 1)]), ("sum", [("col", 2)]), ("sum", rev),
            ("count*",)]
    r = oracle.groupby(t, keys, preds, aggs)
    m = t["shipdate"].data <= 2466
    fl, st = t["flag"].data[m].astype(np.int64), t["status"].data[m].astype(np.int64)
    order = np.lexsort((st, fl))
    fl, st = fl[order], st[order]
    starts = np.flatnonzero(np.r_[True, (np.diff(fl) != 0) | (np.diff(st) != 0)])
    assert np.array_equal(r.keys[0][0], fl[starts]) and np.array_equal(r.keys[1][0], st[starts])
    cols = [t["qty"].data[m], t["price"].data[m], t["disc"].data[m],
            t["price"].data[m] * (100 - t["disc"].data[m])]
    for a, c in enumerate(cols):
        assert np.array_equal(r.aggs[a][0], np.add.reduceat(c[order], starts))
    assert r.aggs[4][0].sum() == m.sum()
    assert r.aggs[3][0].sum() == cols[3].sum()
    assert not r.overflow


def test_groupby_wrapping_sums_and_overflow_flag():
    big = np.iinfo(np.int64).max
    t = tbl(g=np.array([0, 0, 0, 1], dtype=np.int8), x=np.array([big, big, 3, -5], dtype=np.int64))
    r = oracle.groupby(t, [0], [], [("sum", [("col", 1)])])
    assert list(r.aggs[0][0]) == [np.array([big, big, 3]).sum(), -5]   # numpy wraps the same way
    assert r.overflow


def test_groupby_global_aggregate_on_empty():
    e = tbl(x=np.zeros(0, dtype=np.int64))
    r = oracle.groupby(e, [], [], [("count*",), ("sum", [("col", 0)])])
    assert r.nrows == 1
    assert r.aggs[0][0][0] == 0 and r.aggs[0][1][0]
    assert not r.aggs[1][1][0]
    r = oracle.groupby(e, [0], [], [("count*",)])
    assert r.nrows == 0


def test_pipeline_c2_dense_formulation():
    n, m = 30_000, 120_000
    dim = dg.dim_c2(n, seed=33)
    fact = dg.fact_c2(m, nkeys=n, seed=33)
    rev = [("col", 1), ("k-col", 100, 2)]
    r = oracle.pipeline(fact, [("range", 3, 1278, 2555)], [0], [("sum", rev), ("count*",)],
                        join_spec=(dim, [0], [("range", 1, 0, 1202)], [0]))
    # Hash-free: dense per-key accumulation over matching fact rows.
    inv = np.empty(n + 1, dtype=np.int64)
    inv[dim["pkey"].data] = np.arange(n)
    fk = fact["fkey"].data
    ok = (fact["date"].data >= 1278) & (dim["date"].data[inv[fk]] <= 1202)
    term = fact["price"].data * (100 - fact["disc"].data)
    acc = np.zeros(n + 1, dtype=np.int64)
    cnt = np.zeros(n + 1, dtype=np.int64)
    np.add.at(acc, fk[ok], term[ok])
    np.add.at(cnt, fk[ok], 1)
    keys = np.flatnonzero(cnt)
    assert np.array_equal(r.keys[0][0], keys)
    assert np.array_equal(r.aggs[0][0], acc[keys]) and np.array_equal(r.aggs[1][0], cnt[keys])


def test_golden_c1_fixture():
    """Stored full-size config-1 result (written by tests/golden/make_golden.py)."""
    with open(os.path.join(HERE, "golden", "c1_filter_groupby.json")) as f:
        g = json.load(f)
    t = dg.fact_c1(g["rows"], seed=g["seed"])
    m = t["shipdate"].data <= g["bound"]
    # Independent of the oracle: six masked numpy sums per aggregate.
    for row in g["groups"]:
        sel = m & (t["flag"].data == row["flag"]) & (t["status"].data == row["status"])
        q, p, d = t["qty"].data[sel], t["price"].data[sel], t["disc"].data[sel]
        assert row["sum_qty"] == int(q.sum()) and row["sum_price"] == int(p.sum())
        assert row["sum_disc"] == int(d.sum()) and row["sum_rev"] == int((p * (100 - d)).sum())
        assert row["count"] == int(sel.sum())
    assert sum(r["count"] for r in g["groups"]) == int(m.sum())


# ---------------------------------------------------------------------------
# Aggregation modes and streaming aggregation (Section 3.2): pinned by brute
# force over the raw rows, independent of the concatenate / re-aggregate steps
# ---------------------------------------------------------------------------

STREAM_AGGS = [("sum", [("col", 2)]), ("count*",), ("count", [("col", 2)]), ("min", [("col", 3)]),
               ("max", [("col", 2), ("k-col", 10, 3)])]


def _stream_batch(rng, n):
    k = rng.integers(0, 9, n).astype(np.int32)
    kv = rng.random(n) > 0.1
    k2 = rng.integers(-1, 2, n).astype(np.int8)
    x = rng.integers(-(1 << 40), 1 << 40, n)
    xv = rng.random(n) > 0.3
    y = rng.integers(0, 7, n).astype(np.int16)
    yv = rng.random(n) > 0.2
    f = rng.integers(0, 100, n).astype(np.int32)
    return tbl(k=(k, kv), k2=k2, x=(x, xv), y=(y, yv), f=f)


def _brute_aggs(batches, preds):
    """{key: [sum, count*, count, min, max]} over the kept raw rows, None = NULL."""
    groups = {}
    for t, pr in zip(batches, preds):
        k, kv = t.cols[0].data, t.cols[0].valid
        k2 = t.cols[1].data
        x, xv = t.cols[2].data, t.cols[2].valid
        y, yv = t.cols[3].data, t.cols[3].valid
        f = t.cols[4].data
        lo, hi = pr[0][2], pr[0][3]
        for i in range(len(k)):
            if not (lo <= f[i] <= hi):
                continue
            key = ((1, int(k[i])) if kv[i] else (0, 0), (1, int(k2[i])))
            g = groups.setdefault(key, [None, 0, 0, None, None])
            g[1] += 1
            if xv[i]:
                g[0] = ((g[0] or 0) + int(x[i])) & M64
                g[2] += 1
            if yv[i]:
                g[3] = int(y[i]) if g[3] is None else min(g[3], int(y[i]))
            if xv[i] and yv[i]:
                v = (int(x[i]) * (10 - int(y[i]))) & M64
                v = v - (1 << 64) if v >= (1 << 63) else v
                g[4] = v if g[4] is None else max(g[4], v)
    return dict(sorted(groups.items()))


def _as_dict(res):
    out = {}
    for gi in range(res.nrows):
        key = tuple((1, int(res.keys[j][0][gi])) if res.keys[j][1][gi] else (0, 0) for j in range(len(res.keys)))
        vals = []
        for a, (v, ok) in enumerate(res.aggs):
            if not ok[gi]:
                vals.append(None)
            else:
                vals.append(int(v[gi]) & M64 if a == 0 else int(v[gi]))
        out[key] = vals
    return out


@pytest.mark.parametrize("seed,emit", [(0, 1), (1, 3), (2, 10), (3, None), (4, 6)])
def test_stream_partial_emissions_brute_force(seed, emit):
    """Every emission of a partial stream equals the brute-force aggregate of the
    raw rows pushed since the previous one; it comes after the first batch at
    which the distinct kept keys since the previous emission reach the
    threshold; the final merge of all emissions equals the single-step result."""
    rng = np.random.default_rng(700 + seed)
    sizes = [0, 1, 57, 3, 250, 0, 19, 400, 2, 75]
    batches = [_stream_batch(rng, n) for n in sizes]
    preds = [[("range", 4, int(rng.integers(0, 30)), int(rng.integers(60, 100)))] for _ in sizes]
    em = oracle.agg_stream(batches, [0, 1], preds, STREAM_AGGS, mode="partial", emit_groups=emit)
    # Emission points by counting distinct keys (a set) since the last emission.
    bounds, start, seen = [], 0, set()
    for b, t in enumerate(batches):
        k, kv, k2, f = t.cols[0].data, t.cols[0].valid, t.cols[1].data, t.cols[4].data
        lo, hi = preds[b][0][2], preds[b][0][3]
        for i in range(len(k)):
            if lo <= f[i] <= hi:
                seen.add(((1, int(k[i])) if kv[i] else (0, 0), int(k2[i])))
        if emit is not None and len(seen) >= emit:
            bounds.append((start, b + 1))
            start, seen = b + 1, set()
    if start < len(batches):
        bounds.append((start, len(batches)))
    assert len(em) == len(bounds)
    for res, (b0, b1) in zip(em, bounds):
        assert _as_dict(res) == _brute_aggs(batches[b0:b1], preds[b0:b1])
    # Final over the concatenated emissions (as state batches) == single over every row.
    states = [oracle.result_table(r) for r in em]
    nk = 2
    final_aggs = [(a[0], [("col", nk + i)]) for i, a in enumerate(STREAM_AGGS)]
    fin = oracle.agg_stream(states, list(range(nk)), None, final_aggs, mode="final")
    assert len(fin) == 1
    assert _as_dict(fin[0]) == _brute_aggs(batches, preds)
    single = oracle.agg_stream(batches, [0, 1], preds, STREAM_AGGS, mode="single", emit_groups=emit)
    assert len(single) == 1 and _as_dict(single[0]) == _brute_aggs(batches, preds)


def test_merge_modes_all_null_groups_and_counts():
    """Intermediate over two partial results: SUM/MIN/MAX of a group whose inputs
    are NULL in both halves stay NULL; COUNT(*) and COUNT add up and are never NULL."""
    a = tbl(k=np.array([1, 1, 2], dtype=np.int64), x=(np.array([5, 0, 0]), np.array([True, False, False])),
            f=np.zeros(3, dtype=np.int32))
    b = tbl(k=np.array([2, 3], dtype=np.int64), x=(np.array([0, 7]), np.array([False, True])),
            f=np.zeros(2, dtype=np.int32))
    aggs = [("sum", [("col", 1)]), ("count*",), ("count", [("col", 1)]), ("min", [("col", 1)])]
    pa = oracle.groupby_mode(a, [0], [], aggs, "partial")
    pb = oracle.groupby_mode(b, [0], [], aggs, "partial")
    both = oracle.concat_tables([oracle.result_table(pa), oracle.result_table(pb)])
    st = [(x[0], [("col", 1 + i)]) for i, x in enumerate(aggs)]
    m = oracle.groupby_mode(both, [0], [], st, "intermediate")
    assert list(m.keys[0][0]) == [1, 2, 3]
    assert list(m.aggs[0][1]) == [True, False, True] and m.aggs[0][0][0] == 5 and m.aggs[0][0][2] == 7
    assert list(m.aggs[1][0]) == [2, 2, 1] and m.aggs[1][1].all()
    assert list(m.aggs[2][0]) == [1, 0, 1] and m.aggs[2][1].all()
    assert list(m.aggs[3][1]) == [True, False, True]


# ---------------------------------------------------------------------------
# Late materialisation: group-by over a build-side payload column
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_join_groupby_build_payload_brute_force(seed):
    """Nested loops over (probe, build) pairs, then a dict keyed by the build
    side's payload column (NULL its own group), summing a probe-side product."""
    rng = np.random.default_rng(900 + seed)
    nb, npr = int(rng.integers(1, 120)), int(rng.integers(0, 300))
    bk = rng.integers(0, 25, nb)
    bkv = rng.random(nb) > 0.1
    bd = rng.integers(0, 10, nb).astype(np.int32)
    bc = rng.integers(0, 6, nb)
    bcv = rng.random(nb) > 0.2
    pk = rng.integers(0, 25, npr)
    pkv = rng.random(npr) > 0.1
    pp = rng.integers(1, 1000, npr)
    pdisc = rng.integers(0, 11, npr)
    pdate = rng.integers(0, 10, npr).astype(np.int32)
    build = tbl(k=(bk, bkv), d=bd, c=(bc, bcv))
    probe = tbl(k=(pk, pkv), p=pp, disc=pdisc, date=pdate)
    bpred, ppred = [("range", 1, 0, 6)], [("range", 3, 3, 9)]
    aggs = [("sum", [("col", 1), ("k-col", 100, 2)]), ("count*",), ("max", [("col", 1)])]
    r = oracle.join_groupby(probe, ppred, [0], build, bpred, [0], [4 + 2], aggs)
    groups = {}
    for i in range(npr):
        if not (pkv[i] and 3 <= pdate[i] <= 9):
            continue
        for j in range(nb):
            if bkv[j] and 0 <= bd[j] <= 6 and bk[j] == pk[i]:
                key = (1, int(bc[j])) if bcv[j] else (0, 0)
                g = groups.setdefault(key, [0, 0, None])
                g[0] = (g[0] + int(pp[i]) * (100 - int(pdisc[i]))) & M64
                g[1] += 1
                g[2] = int(pp[i]) if g[2] is None else max(g[2], int(pp[i]))
    exp = dict(sorted(groups.items()))
    got = {}
    for gi in range(r.nrows):
        key = (1, int(r.keys[0][0][gi])) if r.keys[0][1][gi] else (0, 0)
        got[key] = [int(r.aggs[0][0][gi]) & M64, int(r.aggs[1][0][gi]), int(r.aggs[2][0][gi])]
    assert got == {k: v for k, v in exp.items()}


def test_join_groupby_dense_build_payload():
    """C2-shaped tables grouped by the dimension's ckey: pkey is a permutation,
    so fact row i joins dim row inv[fkey[i]] (if that row passes), and the
    revenue per ckey is a dense np.add.at -- no hashing, no join."""
    nd, nf = 3000, 20000
    dim = dg.dim_c2(nd, seed=17, ckeys=50)
    fact = dg.fact_c2(nf, nkeys=nd, seed=17)
    dpred, fpred = [("range", 1, 0, 1202)], [("range", 3, 1278, 2555)]
    rev = [("col", 1), ("k-col", 100, 2)]
    r = oracle.join_groupby(fact, fpred, [0], dim, dpred, [0], [4 + 2], [("sum", rev), ("count*",)])
    pkey, ddate, ckey = (dim.cols[j].data for j in range(3))
    inv = np.empty(nd + 1, dtype=np.int64)
    inv[pkey] = np.arange(nd)
    fkey, price, disc, fdate = (fact.cols[j].data for j in range(4))
    j = inv[fkey]
    m = (fdate >= 1278) & (ddate[j] <= 1202)
    tot = np.zeros(51, dtype=np.int64)
    cnt = np.zeros(51, dtype=np.int64)
    np.add.at(tot, ckey[j[m]], (price * (100 - disc))[m])
    np.add.at(cnt, ckey[j[m]], 1)
    nz = np.flatnonzero(cnt)
    assert np.array_equal(r.keys[0][0], nz)
    assert np.array_equal(r.aggs[0][0], tot[nz]) and np.array_equal(r.aggs[1][0], cnt[nz])


# ---------------------------------------------------------------------------
# Expression programs
# ---------------------------------------------------------------------------

def _expr_table(rng, n):
    a = rng.integers(-(1 << 62), 1 << 62, n)
    av = rng.random(n) > 0.2
    b = rng.integers(-50, 50, n).astype(np.int32)
    bv = rng.random(n) > 0.1
    c = rng.integers(0, 3, n).astype(np.int8)
    return tbl(a=(a, av), b=(b, bv), c=c)


def _rand_expr(rng, depth):
    if depth == 0 or rng.random() < 0.25:
        return ("col", int(rng.integers(0, 3))) if rng.random() < 0.7 else ("const", int(rng.integers(-9, 9)))
    op = ["add", "sub", "mul", "neg", "lt", "le", "eq", "ne", "gt", "ge", "case"][int(rng.integers(0, 11))]
    if op == "neg":
        return (op, _rand_expr(rng, depth - 1))
    if op == "case":
        return (op, _rand_expr(rng, depth - 1), _rand_expr(rng, depth - 1), _rand_expr(rng, depth - 1))
    return (op, _rand_expr(rng, depth - 1), _rand_expr(rng, depth - 1))


def _scalar_eval(t, e, i):
    """One row, Python integers: None for NULL; arithmetic reduced modulo 2^64
    into the signed range after every step."""
    def s64(x):
        x &= M64
        return x - (1 << 64) if x >= (1 << 63) else x
    op = e[0]
    if op == "col":
        c = t.cols[e[1]]
        if c.valid is not None and not c.valid[i]:
            return None
        return int(c.data[i])
    if op == "const":
        return e[1]
    if op == "neg":
        x = _scalar_eval(t, e[1], i)
        return None if x is None else s64(-x)
    if op == "case":
        c = _scalar_eval(t, e[1], i)
        return _scalar_eval(t, e[2], i) if (c is not None and c != 0) else _scalar_eval(t, e[3], i)
    x, y = _scalar_eval(t, e[1], i), _scalar_eval(t, e[2], i)
    if x is None or y is None:
        return None
    return {"add": lambda: s64(x + y), "sub": lambda: s64(x - y), "mul": lambda: s64(x * y),
            "lt": lambda: int(x < y), "le": lambda: int(x <= y), "eq": lambda: int(x == y),
            "ne": lambda: int(x != y), "gt": lambda: int(x > y), "ge": lambda: int(x >= y)}[op]()


@pytest.mark.parametrize("seed", range(6))
def test_expr_eval_against_scalar_rows(seed):
    rng = np.random.default_rng(1200 + seed)
    t = _expr_table(rng, 200)
    for _ in range(25):
        e = _rand_expr(rng, 4)
        v, ok = oracle.eval_expr(t, e)
        for i in range(t.nrows):
            x = _scalar_eval(t, e, i)
            assert ok[i] == (x is not None), (e, i)
            if x is not None:
                assert int(v[i]) == x, (e, i)


def test_expr_product_equals_factor_form_and_identities():
    """price*(100-disc) as an expression equals the factor-list aggregate (pinned
    above); (a+b)-b == a and a*(b+c) == a*b + a*c modulo 2^64."""
    t1 = dg.fact_c1(5000, seed=3)
    rev_e = ("mul", ("col", 1), ("sub", ("const", 100), ("col", 2)))
    r_e = oracle.groupby_expr(t1, [4, 5], [("range", 3, 0, 2466)], [], [("sum", rev_e), ("count*",)])
    r_f = oracle.groupby(t1, [4, 5], [("range", 3, 0, 2466)], [("sum", [("col", 1), ("k-col", 100, 2)]), ("count*",)])
    assert np.array_equal(r_e.aggs[0][0], r_f.aggs[0][0]) and np.array_equal(r_e.aggs[1][0], r_f.aggs[1][0])
    rng = np.random.default_rng(5)
    t = _expr_table(rng, 500)
    a, b, c = ("col", 0), ("col", 1), ("col", 2)
    v1, ok1 = oracle.eval_expr(t, ("sub", ("add", a, b), b))
    v0, ok0 = oracle.eval_expr(t, a)
    assert np.array_equal(v1[ok1], v0[ok1]) and np.array_equal(ok1, ok0 & t.cols[1].valid)
    l, lok = oracle.eval_expr(t, ("mul", a, ("add", b, c)))
    r, rok = oracle.eval_expr(t, ("add", ("mul", a, b), ("mul", a, c)))
    assert np.array_equal(lok, rok) and np.array_equal(l[lok], r[rok])


def test_filter_expr_case_condition_null_takes_else():
    t = tbl(x=(np.array([5, 5, 5, 0]), np.array([True, False, True, True])), y=np.array([1, 0, 0, 0]))
    # CASE WHEN x > 3 THEN y ELSE 1 - y: row 1 (x NULL) takes the ELSE branch (1 - 0).
    e = ("case", ("gt", ("col", 0), ("const", 3)), ("col", 1), ("sub", ("const", 1), ("col", 1)))
    rows, _ = oracle.filter_expr(t, [], [e], [0])
    assert list(rows) == [0, 1, 3]
    # A comparison with a NULL operand is NULL, so the row is dropped.
    rows, _ = oracle.filter_expr(t, [], [("gt", ("col", 0), ("const", -1))], [0])
    assert list(rows) == [0, 2, 3]


# ---------------------------------------------------------------------------
# ORDER BY / top-k
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_order_by_matches_pandas_stable_sort(seed):
    rng = np.random.default_rng(1300 + seed)
    n = int(rng.integers(0, 400))
    k1 = rng.integers(-3, 3, n)
    k1v = rng.random(n) > 0.2
    k2 = rng.integers(-1000, 1000, n).astype(np.int32)
    k2v = rng.random(n) > 0.1
    t = tbl(k1=(k1, k1v), k2=(k2, k2v), row=np.arange(n))
    for desc in ([False, False], [True, False], [False, True], [True, True]):
        for nf in (False, True):
            got = oracle.order_by(t, [0, 1], desc=desc, nulls_first=[nf, nf])
            df = pd.DataFrame({"k1": pd.array(np.where(k1v, k1, 0), dtype="Int64"),
                               "k2": pd.array(np.where(k2v, k2, 0), dtype="Int64")})
            df.loc[~k1v, "k1"] = pd.NA
            df.loc[~k2v, "k2"] = pd.NA
            exp = df.sort_values(["k1", "k2"], ascending=[not d for d in desc], kind="stable",
                                 na_position="first" if nf else "last").index.to_numpy()
            assert np.array_equal(got, exp), (desc, nf)
            top = oracle.order_by(t, [0, 1], desc=desc, nulls_first=[nf, nf], limit=7)
            assert np.array_equal(top, exp[:7])
