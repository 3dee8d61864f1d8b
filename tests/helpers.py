"""Shared test helpers: host tables, device upload and result comparison."""
import numpy as np

from paper_2606_24647_amd.datagen import Column, Table


def tbl(**cols):
    out = Table()
    for name, v in cols.items():
        if isinstance(v, tuple):
            out.cols.append(Column(name, np.asarray(v[0]), np.asarray(v[1], dtype=bool)))
        else:
            out.cols.append(Column(name, np.asarray(v)))
    return out


def random_table(rng, n, types=(np.int64, np.int32, np.int16, np.int8), null_frac=0.0, lo=-50, hi=50):
    t = Table()
    for i, dt in enumerate(types):
        info = np.iinfo(dt)
        a, b = max(lo, info.min), min(hi, info.max)
        v = rng.integers(a, b + 1, n).astype(dt)
        valid = (rng.random(n) >= null_frac) if null_frac > 0 else None
        t.cols.append(Column(f"c{i}", v, valid))
    return t


def assert_col_equal(got, exp_vals, exp_valid, what=""):
    """got = (values, valid-or-None) from the device; exp_valid None = all valid."""
    gv, gok = got
    exp_vals = np.asarray(exp_vals)
    assert len(gv) == len(exp_vals), f"{what}: length {len(gv)} != {len(exp_vals)}"
    if exp_valid is None:
        if gok is not None:
            assert gok.all(), f"{what}: unexpected NULLs"
        assert np.array_equal(gv, exp_vals.astype(gv.dtype)), f"{what}: values differ"
        return
    assert gok is not None, f"{what}: missing validity"
    assert np.array_equal(gok, exp_valid), f"{what}: validity differs"
    assert np.array_equal(gv[exp_valid], exp_vals.astype(gv.dtype)[exp_valid]), f"{what}: values differ"


def canon_groups(keys, aggs):
    """Sort group-by output rows canonically: keys ascending, NULL first.

    keys/aggs: lists of (values, valid bool array or None).  Returns the same
    lists reordered, NULL values zeroed.
    """
    n = len(keys[0][0]) if keys else (len(aggs[0][0]) if aggs else 0)
    sort_cols = []
    norm = []
    for v, ok in keys:
        ok = np.ones(n, dtype=bool) if ok is None else ok
        vv = np.where(ok, v.astype(np.int64), 0)
        norm.append((vv, ok))
    for vv, ok in reversed(norm):
        sort_cols.append(vv)
        sort_cols.append(ok.astype(np.int8))
    order = np.lexsort(sort_cols) if sort_cols else np.arange(n)
    ok_keys = [(vv[order], ok[order]) for vv, ok in norm]
    ok_aggs = []
    for v, ok in aggs:
        ok = np.ones(n, dtype=bool) if ok is None else ok
        ok_aggs.append((np.where(ok, v, 0)[order], ok[order]))
    return ok_keys, ok_aggs
