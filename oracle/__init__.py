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
