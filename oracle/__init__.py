"""CPU oracle for the columnar operator path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It loads ``liboracle.so`` (plain C++, built from ``oracle.cpp`` by
``build()`` below with g++) through ctypes and takes host numpy columns.  It shares no
code with the GPU library.

Operator specs are plain tuples, the same ones the GPU binding accepts:

* predicate: ``("range", col, lo, hi)`` keeps ``lo <= x <= hi``;
  ``("ne", col, v)`` keeps ``x != v``.  NULL never passes.
* factor: ``("col", c)``, ``("k-col", k, c)``, ``("k+col", k, c)``, ``("const", k)``.
* aggregate: ``("sum", factors)``, ``("count*",)``, ``("count", factors)``,
  ``("min", factors)``, ``("max", factors)``.

Beyond the single-step operators it holds the aggregation modes and the
streaming aggregation of Section 3.2 (``groupby_mode``, ``agg_stream``), the
late-materialisation join + group-by over either side's columns of Section 2.3
(``join_groupby``), expression programs (``eval_expr``, ``filter_expr``,
``groupby_expr``) and ORDER BY / top-k (``order_by``).

Parity status: every function here is pinned by the not-gpu tests in
``tests/test_oracle_pins.py`` (brute force, library routines, closed forms and
invariants); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

T_CODES = {np.dtype(np.int8): 1, np.dtype(np.int16): 2, np.dtype(np.int32): 3,
           np.dtype(np.int64): 4}
PRED_OPS = {"range": 1, "ne": 2}
FACTOR_KINDS = {"col": 1, "k-col": 2, "k+col": 3, "const": 4}
AGG_OPS = {"sum": 1, "count*": 2, "count": 3, "min": 4, "max": 5}


class OrcCol(C.Structure):
    _fields_ = [("type", C.c_int32), ("pad", C.c_int32), ("length", C.c_int64),
                ("data", C.c_void_p), ("validity", C.c_void_p)]


class OrcPred(C.Structure):
    _fields_ = [("col", C.c_int32), ("op", C.c_int32), ("lo", C.c_int64), ("hi", C.c_int64)]


class OrcFactor(C.Structure):
    _fields_ = [("kind", C.c_int32), ("col", C.c_int32), ("k", C.c_int64)]


class OrcAgg(C.Structure):
    _fields_ = [("op", C.c_int32), ("nf", C.c_int32), ("f", OrcFactor * 3)]


_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ -O2 (plain host C++)."""
    src = os.path.join(_HERE, "oracle.cpp")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_fmix64.restype = C.c_uint64
        L.orc_fmix64.argtypes = [C.c_uint64]
        L.orc_partition_of.restype = C.c_uint64
        L.orc_partition_of.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_hash_rows.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_uint64, C.c_int64, C.c_void_p]
        L.orc_filter.restype = C.c_int64
        L.orc_filter.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p]
        L.orc_partition.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_int64,
                                    C.c_uint64, C.c_void_p, C.c_void_p]
        L.orc_join.restype = C.c_void_p
        L.orc_join.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                               C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int]
        L.orc_pairs_count.restype = C.c_int64
        L.orc_pairs_count.argtypes = [C.c_void_p]
        L.orc_pairs_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_pairs_free.argtypes = [C.c_void_p]
        L.orc_groupby.restype = C.c_void_p
        L.orc_groupby.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                  C.c_void_p, C.c_int]
        L.orc_groups_rows.restype = C.c_int64
        L.orc_groups_rows.argtypes = [C.c_void_p]
        L.orc_groups_overflow.restype = C.c_int
        L.orc_groups_overflow.argtypes = [C.c_void_p]
        L.orc_groups_copy.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_groups_free.argtypes = [C.c_void_p]
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# Marshalling
# ---------------------------------------------------------------------------

class _Cols:
    """ctypes column array over a table; keeps the numpy buffers alive."""

    def __init__(self, table):
        self.keep = []
        cols = table.cols
        self.arr = (OrcCol * max(1, len(cols)))()
        for i, c in enumerate(cols):
            d = np.ascontiguousarray(c.data)
            self.keep.append(d)
            bm = c.bitmap()
            if bm is not None:
                self.keep.append(bm)
            self.arr[i].type = T_CODES[d.dtype]
            self.arr[i].length = len(d)
            self.arr[i].data = d.ctypes.data if len(d) else None
            self.arr[i].validity = bm.ctypes.data if bm is not None else None
        self.n = table.nrows

    @property
    def ptr(self):
        return C.cast(self.arr, C.c_void_p)


def _preds(preds):
    preds = list(preds or [])
    arr = (OrcPred * max(1, len(preds)))()
    for i, p in enumerate(preds):
        arr[i].op = PRED_OPS[p[0]]
        arr[i].col = p[1]
        if p[0] == "range":
            arr[i].lo, arr[i].hi = p[2], p[3]
        else:
            arr[i].lo = arr[i].hi = p[2]
    return arr, len(preds)


def _int32s(xs):
    xs = list(xs or [])
    arr = (C.c_int32 * max(1, len(xs)))(*xs)
    return arr, len(xs)


def _aggs(aggs):
    arr = (OrcAgg * max(1, len(aggs)))()
    for i, a in enumerate(aggs):
        arr[i].op = AGG_OPS[a[0]]
        factors = a[1] if len(a) > 1 else []
        assert len(factors) <= 3
        arr[i].nf = len(factors)
        for j, f in enumerate(factors):
            kind = FACTOR_KINDS[f[0]]
            arr[i].f[j].kind = kind
            if f[0] == "col":
                arr[i].f[j].col = f[1]
            elif f[0] == "const":
                arr[i].f[j].k = f[1]
            else:
                arr[i].f[j].k, arr[i].f[j].col = f[1], f[2]
    return arr, len(aggs)


# ---------------------------------------------------------------------------
# Public functions
# ---------------------------------------------------------------------------

def fmix64(x: int) -> int:
    return int(lib().orc_fmix64(x & 0xFFFFFFFFFFFFFFFF))


def partition_of(h: int, P: int) -> int:
    return int(lib().orc_partition_of(h, P))


def hash_rows(table, keys, seed: int = 0) -> np.ndarray:
    cols = _Cols(table)
    k, nk = _int32s(keys)
    out = np.empty(table.nrows, dtype=np.uint64)
    lib().orc_hash_rows(cols.ptr, k, nk, seed, table.nrows, out.ctypes.data)
    return out


def filter_rows(table, preds) -> np.ndarray:
    cols = _Cols(table)
    p, np_ = _preds(preds)
    out = np.empty(max(1, table.nrows), dtype=np.int64)
    k = lib().orc_filter(cols.ptr, table.nrows, p, np_, out.ctypes.data)
    return out[:k].copy()


def _take(col, rows):
    vals = col.data[rows]
    valid = None if col.valid is None else col.valid[rows]
    return vals, valid


def filter(table, preds, proj):
    """Stable filter then projection: (kept rows, [(values, valid-or-None)])."""
    rows = filter_rows(table, preds)
    return rows, [_take(table.cols[j], rows) for j in proj]


def partition(table, keys, P: int, seed: int = 0):
    """(perm, offsets): perm[r] = input row at output position r."""
    cols = _Cols(table)
    k, nk = _int32s(keys)
    perm = np.empty(max(1, table.nrows), dtype=np.int64)
    offsets = np.empty(P + 1, dtype=np.int64)
    lib().orc_partition(cols.ptr, table.nrows, k, nk, P, seed, perm.ctypes.data, offsets.ctypes.data)
    return perm[: table.nrows].copy(), offsets


def join(build, bkeys, bpreds, probe, pkeys, ppreds):
    """Inner equi-join pairs (probe_row, build_row), ordered (probe asc, build asc)."""
    bc, pc = _Cols(build), _Cols(probe)
    bk, nk = _int32s(bkeys)
    pk, nk2 = _int32s(pkeys)
    assert nk == nk2
    bp, nbp = _preds(bpreds)
    pp, npp = _preds(ppreds)
    L = lib()
    h = L.orc_join(bc.ptr, build.nrows, bk, nk, bp, nbp, pc.ptr, probe.nrows, pk, pp, npp)
    try:
        n = L.orc_pairs_count(h)
        pi = np.empty(max(1, n), dtype=np.int64)
        bi = np.empty(max(1, n), dtype=np.int64)
        L.orc_pairs_copy(h, pi.ctypes.data, bi.ctypes.data)
        return pi[:n].copy(), bi[:n].copy()
    finally:
        L.orc_pairs_free(h)


class GroupResult:
    """Group-by result in canonical order (keys ascending, NULL first)."""

    def __init__(self, keys, aggs, overflow):
        self.keys = keys          # list of (values int64, valid bool)
        self.aggs = aggs          # list of (values int64, valid bool)
        self.overflow = overflow  # True if any exact sum or product left int64

    @property
    def nrows(self) -> int:
        if self.keys:
            return len(self.keys[0][0])
        return len(self.aggs[0][0]) if self.aggs else 0


def groupby(table, keys, preds, aggs) -> GroupResult:
    cols = _Cols(table)
    k, nk = _int32s(keys)
    p, np_ = _preds(preds)
    a, na = _aggs(aggs)
    L = lib()
    h = L.orc_groupby(cols.ptr, table.nrows, k, nk, p, np_, a, na)
    try:
        n = L.orc_groups_rows(h)
        out = []
        for j in range(nk + na):
            v = np.empty(max(1, n), dtype=np.int64)
            ok = np.empty(max(1, n), dtype=np.uint8)
            L.orc_groups_copy(h, j, v.ctypes.data, ok.ctypes.data)
            out.append((v[:n].copy(), ok[:n].astype(bool)))
        return GroupResult(out[:nk], out[nk:], bool(L.orc_groups_overflow(h)))
    finally:
        L.orc_groups_free(h)


def pipeline(probe, ppreds, gkeys, aggs, join_spec=None) -> GroupResult:
    """Group-by over filter(probe) [joined with filter(build)].

    ``join_spec`` = (build_table, build_keys, build_preds, probe_keys) or None.
    Group keys and aggregate inputs are probe-side columns.  The join is
    materialised (one row per matching pair) and then aggregated, exactly as the
    composition of the relational operators reads.
    """
    if join_spec is None:
        return groupby(probe, gkeys, ppreds, aggs)
    build, bkeys, bpreds, pkeys = join_spec
    pi, _ = join(build, bkeys, bpreds, probe, pkeys, ppreds)
    joined = _Table([_Column(c.data[pi], None if c.valid is None else c.valid[pi])
                     for c in probe.cols])
    return groupby(joined, gkeys, [], aggs)


class _Column:
    def __init__(self, data, valid):
        self.data, self.valid = data, valid

    def bitmap(self):
        if self.valid is None:
            return None
        n = len(self.valid)
        out = np.zeros(((n + 63) // 64) * 8, dtype=np.uint8)
        if n:
            b = np.packbits(self.valid.astype(np.uint8), bitorder="little")
            out[: len(b)] = b
        return out


class _Table:
    def __init__(self, cols):
        self.cols = cols

    @property
    def nrows(self):
        return len(self.cols[0].data) if self.cols else 0


# ---------------------------------------------------------------------------
# Aggregation modes and streaming aggregation (Section 3.2, HashAggregation)
# ---------------------------------------------------------------------------
# The paper's aggregation operator runs in one of four modes so that an
# aggregation can be split across exchange stages: Partial turns input rows
# into per-group partial states, Intermediate merges partial states into
# partial states, Final merges partial states into final values, Single goes
# from rows to final values in one step.  For the aggregates here a partial
# state is one int64 value with validity:
#   SUM      sum of the non-NULL inputs, NULL if there is none
#   COUNT(*) number of rows;  COUNT  number of non-NULL inputs (never NULL)
#   MIN/MAX  over the non-NULL inputs, NULL if there is none
# so a partial state holds the same value as the aggregate itself, and merging
# states is SUM for SUM, COUNT(*) and COUNT, and MIN or MAX for MIN and MAX.
# In the merge modes an aggregate names its state column with one factor
# ("col", c); its factor list is otherwise unused.

MODES = {"single": 0, "partial": 1, "intermediate": 2, "final": 3}
_MERGE_OP = {"sum": "sum", "count*": "sum", "count": "sum", "min": "min", "max": "max"}


def merge_aggs(aggs):
    """Aggregates over state columns that merge the states of `aggs`: the state of
    aggregate i is column i of the aggregate block (column nk + i of a state batch)."""
    return [(_MERGE_OP[a[0]],) + (a[1:] if len(a) > 1 else ()) for a in aggs]


def groupby_mode(table, keys, preds, aggs, mode):
    """One group-by step in the given mode.  Raw input (single, partial): `aggs`
    read raw columns.  State input (intermediate, final): `aggs` are the
    original aggregates, each with one factor ("col", c) naming its state
    column, and no predicates apply."""
    if mode in ("single", "partial"):
        return groupby(table, keys, preds, aggs)
    assert not preds, "merge modes take no predicates"
    for a in aggs:
        assert len(a) == 2 and len(a[1]) == 1 and a[1][0][0] == "col", "merge-mode aggregates name one state column"
    return groupby(table, keys, [], merge_aggs(aggs))


def result_table(res):
    """A group result as a table: key columns, then one column per aggregate."""
    return _Table([_Column(v, ok.copy()) for v, ok in res.keys + res.aggs])


def concat_tables(tables):
    """Row-wise concatenation of tables of equal column count."""
    ncols = len(tables[0].cols)
    cols = []
    for j in range(ncols):
        data = np.concatenate([t.cols[j].data for t in tables])
        valid = None
        if any(t.cols[j].valid is not None for t in tables):
            valid = np.concatenate([np.ones(len(t.cols[j].data), dtype=bool) if t.cols[j].valid is None
                                    else np.asarray(t.cols[j].valid, dtype=bool) for t in tables])
        cols.append(_Column(data, valid))
    return _Table(cols)


def agg_stream(batches, keys, preds, aggs, mode="partial", emit_groups=None):
    """Streaming aggregation over a sequence of batches, in the paper's order of
    steps: each batch is aggregated on its own (Partial over raw rows, or a
    merge over state rows), the result is concatenated with the results held
    so far and the concatenation is aggregated again (Intermediate), and once
    the held result reaches `emit_groups` groups it is emitted and the
    operator starts over.  Only partial and intermediate streams emit early;
    single and final streams emit once, after the last batch.

    batches  list of tables (raw rows, or state rows for intermediate/final)
    preds    one predicate list per batch (raw input only)
    Returns the emitted results (GroupResult, canonical order each), in order;
    a stream that received no batch emits nothing.
    """
    nk = len(keys)
    raw = mode in ("single", "partial")
    state_aggs = [(a[0], [("col", nk + i)]) for i, a in enumerate(aggs)]
    held = None
    emitted = []
    for b, batch in enumerate(batches):
        if raw:
            part = groupby_mode(batch, keys, preds[b] if preds else [], aggs, "partial")
        else:
            part = groupby_mode(batch, keys, [], aggs, "intermediate")
        if held is None:
            held = part
        else:
            both = concat_tables([result_table(held), result_table(part)])
            held = groupby_mode(both, list(range(nk)), [], state_aggs, "intermediate")
        if mode in ("partial", "intermediate") and emit_groups is not None and held.nrows >= emit_groups:
            emitted.append(held)
            held = None
    if held is not None:
        emitted.append(held)
    return emitted


# ---------------------------------------------------------------------------
# Late materialisation (Section 2.3): a key-only join gives gather maps, the
# payload columns of both sides are gathered through them, then grouped
# ---------------------------------------------------------------------------

def join_groupby(probe, ppreds, pkeys, build, bpreds, bkeys, gkeys, aggs):
    """Group-by over the materialised inner join of filter(probe) and
    filter(build).  Column c of the joined rows is probe column c for
    c < len(probe.cols), else build column c - len(probe.cols); group keys and
    aggregate inputs may come from either side.  The steps are the paper's
    late materialisation: the join on the key columns alone (pairs of row
    ids), then the gather of every payload column through those ids, then
    the group-by."""
    pi, bi = join(build, bkeys, bpreds, probe, pkeys, ppreds)
    cols = [_Column(c.data[pi], None if c.valid is None else np.asarray(c.valid, dtype=bool)[pi]) for c in probe.cols]
    cols += [_Column(c.data[bi], None if c.valid is None else np.asarray(c.valid, dtype=bool)[bi]) for c in build.cols]
    return groupby(_Table(cols), gkeys, [], aggs)


# ---------------------------------------------------------------------------
# Expression programs (Section 3.2: expressions evaluated fused, as cuDF's AST
# compute_column) and ORDER BY / top-k (Section 3.1 names OrderBy among the
# operators moved to the GPU)
# ---------------------------------------------------------------------------
# An expression is a tree of tuples:
#   ("col", c)  ("const", k)  ("add", a, b)  ("sub", a, b)  ("mul", a, b)  ("neg", a)
#   ("lt"|"le"|"eq"|"ne"|"gt"|"ge", a, b)      1 or 0
#   ("case", cond, a, b)                        a where cond is non-NULL and non-zero, else b
# Integer arithmetic wraps modulo 2^64.  An operand that is NULL makes add, sub,
# mul, neg and the comparisons NULL; a CASE whose condition is NULL takes its
# ELSE branch (SQL's CASE WHEN).  A predicate ("expr", e) keeps a row when e
# is non-NULL and non-zero.

_CMP = {"lt": np.less, "le": np.less_equal, "eq": np.equal, "ne": np.not_equal,
        "gt": np.greater, "ge": np.greater_equal}


def eval_expr(table, e):
    """(values int64, valid bool) of expression e over every row of table."""
    n = table.nrows
    op = e[0]
    if op == "col":
        c = table.cols[e[1]]
        v = np.asarray(c.data).astype(np.int64)
        ok = np.ones(n, dtype=bool) if c.valid is None else np.asarray(c.valid, dtype=bool).copy()
        return v, ok
    if op == "const":
        return np.full(n, np.int64(e[1]), dtype=np.int64), np.ones(n, dtype=bool)
    if op == "neg":
        a, ok = eval_expr(table, e[1])
        with np.errstate(over="ignore"):
            return (np.uint64(0) - a.astype(np.uint64)).astype(np.int64), ok
    if op == "case":
        c, cok = eval_expr(table, e[1])
        a, aok = eval_expr(table, e[2])
        b, bok = eval_expr(table, e[3])
        take = cok & (c != 0)
        return np.where(take, a, b), np.where(take, aok, bok)
    a, aok = eval_expr(table, e[1])
    b, bok = eval_expr(table, e[2])
    ok = aok & bok
    if op in _CMP:
        return _CMP[op](a, b).astype(np.int64), ok
    ua, ub = a.astype(np.uint64), b.astype(np.uint64)
    with np.errstate(over="ignore"):
        r = {"add": ua + ub, "sub": ua - ub, "mul": ua * ub}[op]
    return r.astype(np.int64), ok


def filter_expr(table, preds, exprs, proj):
    """Filter where every range/ne predicate holds and every expression predicate
    is non-NULL and non-zero; stable; projected columns."""
    keep = np.zeros(table.nrows, dtype=bool)
    keep[filter_rows(table, preds)] = True
    for e in exprs:
        v, ok = eval_expr(table, e)
        keep &= ok & (v != 0)
    rows = np.flatnonzero(keep)
    return rows, [_take(table.cols[j], rows) for j in proj]


def groupby_expr(table, keys, preds, exprs, aggs):
    """Group-by whose aggregates read expression programs: aggs are
    (op, expr) with op in sum/count/min/max, or ("count*",).  Each expression
    is evaluated into a column first, then the plain group-by runs over them."""
    keep = np.zeros(table.nrows, dtype=bool)
    keep[filter_rows(table, preds)] = True
    for e in exprs:
        v, ok = eval_expr(table, e)
        keep &= ok & (v != 0)
    rows = np.flatnonzero(keep)
    cols = [_Column(np.asarray(c.data)[rows], None if c.valid is None else np.asarray(c.valid, dtype=bool)[rows])
            for c in table.cols]
    plain = []
    for a in aggs:
        if a[0] == "count*":
            plain.append(("count*",))
            continue
        v, ok = eval_expr(_Table(cols), a[1])
        cols.append(_Column(v, ok))
        plain.append((a[0], [("col", len(cols) - 1)]))
    return groupby(_Table(cols), keys, [], plain)


def order_by(table, keys, desc=None, nulls_first=None, limit=None):
    """Row ids of `table` in ORDER BY order: key columns compared in turn, each
    ascending unless desc[j], NULLs first or last per nulls_first[j] (default:
    NULLs last, Presto's default); ties keep input order (a stable sort).  With
    `limit`, the first `limit` of them (top-k)."""
    nk = len(keys)
    desc = list(desc or [False] * nk)
    nulls_first = list(nulls_first or [False] * nk)
    n = table.nrows
    cols = []
    for j, c in enumerate(keys):
        col = table.cols[c]
        v = [int(x) for x in np.asarray(col.data)]
        ok = [True] * n if col.valid is None else [bool(x) for x in np.asarray(col.valid)]
        cols.append((v, ok))

    def sort_key(i):
        parts = []
        for j, (v, ok) in enumerate(cols):
            null_rank = 0 if nulls_first[j] else 1
            if not ok[i]:
                parts.append((null_rank, 0))
            else:
                parts.append((1 - null_rank, -v[i] if desc[j] else v[i]))
        return tuple(parts) + (i,)

    rows = sorted(range(n), key=sort_key)
    if limit is not None:
        rows = rows[:limit]
    return np.asarray(rows, dtype=np.int64)
