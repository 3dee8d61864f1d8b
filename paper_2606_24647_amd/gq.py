"""Python binding of libgq.so (include/gq.h): argument marshalling only.

Device memory comes from torch tensors and streams from ``torch.cuda`` (HIP
streams under ROCm); every step of every operator runs in the HIP kernels of
libgq.so.  There is no fallback: if the library is missing, importing this
module raises.

Operator specs are plain tuples:

* predicate ``("range", col, lo, hi)`` (lo <= x <= hi) or ``("ne", col, v)``;
* factor ``("col", c)``, ``("k-col", k, c)``, ``("k+col", k, c)``, ``("const", k)``;
* aggregate ``("sum", factors)``, ``("count*",)``, ``("count", factors)``,
  ``("min", factors)``, ``("max", factors)``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgq.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2606_24647_amd.build` "
                      "(there is no CPU fallback)")

_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------------------
# ABI structures (mirror include/gq.h)
# ---------------------------------------------------------------------------
GQ_OK = 0
GQ_ERR_INVALID, GQ_ERR_UNSUPPORTED, GQ_ERR_NOMEM, GQ_ERR_HIP = -1, -2, -3, -4
GQ_ERR_CAPACITY, GQ_ERR_TABLE_FULL = -5, -6
GQ_I8, GQ_I16, GQ_I32, GQ_I64 = 1, 2, 3, 4
GQ_RANGE, GQ_NE = 1, 2
GQ_SUM, GQ_COUNT_STAR, GQ_COUNT, GQ_MIN, GQ_MAX = 1, 2, 3, 4, 5
GQ_SORTED = 1
GQ_DEV_CAPACITY, GQ_DEV_TABLE_FULL = 1, 2
DEV_CAPACITY, DEV_TABLE_FULL = GQ_DEV_CAPACITY, GQ_DEV_TABLE_FULL
STRATEGY = {"auto": 0, "lds": 1, "global": 2}

_STATUS_NAMES = {0: "GQ_OK", -1: "GQ_ERR_INVALID", -2: "GQ_ERR_UNSUPPORTED", -3: "GQ_ERR_NOMEM",
                 -4: "GQ_ERR_HIP", -5: "GQ_ERR_CAPACITY", -6: "GQ_ERR_TABLE_FULL"}

_TORCH_TYPE = {torch.int8: GQ_I8, torch.int16: GQ_I16, torch.int32: GQ_I32, torch.int64: GQ_I64}
_TYPE_TORCH = {v: k for k, v in _TORCH_TYPE.items()}
_NP_TYPE = {np.dtype(np.int8): GQ_I8, np.dtype(np.int16): GQ_I16, np.dtype(np.int32): GQ_I32,
            np.dtype(np.int64): GQ_I64}


def np_to_type(dtype) -> int:
    """gq column type of a numpy integer dtype."""
    return _NP_TYPE[np.dtype(dtype)]
_PRED_OPS = {"range": GQ_RANGE, "ne": GQ_NE}
_FACTORS = {"col": 1, "k-col": 2, "k+col": 3, "const": 4}
_AGGS = {"sum": GQ_SUM, "count*": GQ_COUNT_STAR, "count": GQ_COUNT, "min": GQ_MIN, "max": GQ_MAX}


class GqColumn(C.Structure):
    _fields_ = [("type", C.c_int32), ("scale", C.c_int32), ("length", C.c_int64),
                ("offset", C.c_int64), ("data", C.c_void_p), ("validity", C.c_void_p)]


class GqBatch(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int32), ("reserved", C.c_int32),
                ("cols", C.POINTER(GqColumn))]


class GqPred(C.Structure):
    _fields_ = [("col", C.c_int32), ("op", C.c_int32), ("lo", C.c_int64), ("hi", C.c_int64)]


class GqFactor(C.Structure):
    _fields_ = [("kind", C.c_int32), ("col", C.c_int32), ("k", C.c_int64)]


class GqAgg(C.Structure):
    _fields_ = [("op", C.c_int32), ("nfactors", C.c_int32), ("f", GqFactor * 3)]


class GqJoinOpts(C.Structure):
    _fields_ = [("load_factor", C.c_float), ("acc_slots", C.c_int32), ("regions_log2", C.c_int32)]


class GqGroupbyOpts(C.Structure):
    _fields_ = [("load_factor", C.c_float), ("strategy", C.c_int32), ("flags", C.c_int32),
                ("block_size", C.c_int32), ("expected_groups", C.c_int64), ("mode", C.c_int32),
                ("reserved", C.c_int32)]


MODES = {"single": 0, "partial": 1, "intermediate": 2, "final": 3}


class GqExprInstr(C.Structure):
    _fields_ = [("op", C.c_int32), ("a", C.c_int32), ("b", C.c_int32), ("c", C.c_int32), ("k", C.c_int64)]


class GqExpr(C.Structure):
    _fields_ = [("ninstr", C.c_int32), ("reserved", C.c_int32), ("instr", C.POINTER(GqExprInstr))]


_EXPR_OPS = {"col": 1, "const": 2, "add": 3, "sub": 4, "mul": 5, "neg": 6, "lt": 7, "le": 8, "eq": 9,
             "ne": 10, "gt": 11, "ge": 12, "case": 13}


def compile_expr(tree):
    """An expression tree (("col", c), ("const", k), ("add", x, y), ...,
    ("case", cond, then, else)) as the postfix instruction list of gq_expr:
    operands are the indices of earlier instructions."""
    prog = []

    def emit(e):
        op = e[0]
        if op == "col":
            prog.append((1, int(e[1]), 0, 0, 0))
        elif op == "const":
            prog.append((2, 0, 0, 0, int(e[1])))
        else:
            args = [emit(x) for x in e[1:]] + [0, 0]
            prog.append((_EXPR_OPS[op], args[0], args[1], args[2], 0))
        return len(prog) - 1

    emit(tree)
    return prog


class _ExprArg:
    """A list of expression trees as gq_expr structs kept alive for one call."""

    def __init__(self, trees):
        self.progs = []
        self.arr = (GqExpr * max(1, len(trees)))()
        for i, t in enumerate(trees):
            prog = compile_expr(t)
            ins = (GqExprInstr * len(prog))(*[GqExprInstr(*q) for q in prog])
            self.progs.append(ins)
            self.arr[i] = GqExpr(len(prog), 0, C.cast(ins, C.POINTER(GqExprInstr)))

    @property
    def ptr(self):
        return C.cast(self.arr, C.POINTER(GqExpr))


class GqAggStreamSpec(C.Structure):
    _fields_ = [("mode", C.c_int32), ("nkeys", C.c_int32), ("keys", C.POINTER(C.c_int32)),
                ("key_nullable", C.POINTER(C.c_int32)), ("aggs", C.POINTER(GqAgg)), ("naggs", C.c_int32),
                ("reserved", C.c_int32), ("max_groups", C.c_int64), ("emit_groups", C.c_int64),
                ("load_factor", C.c_float), ("reserved2", C.c_int32)]


class GqPlan(C.Structure):
    _fields_ = [("preds", C.POINTER(GqPred)), ("npreds", C.c_int32), ("probe_key", C.c_int32),
                ("join", C.c_void_p), ("group_keys", C.POINTER(C.c_int32)),
                ("ngroup_keys", C.c_int32), ("naggs", C.c_int32), ("aggs", C.POINTER(GqAgg)),
                ("opts", GqGroupbyOpts)]


class GqFragment(C.Structure):
    _fields_ = [("inp", GqBatch), ("preds", C.POINTER(GqPred)), ("npreds", C.c_int32),
                ("reserved", C.c_int32), ("expected_groups", C.c_int64), ("out", GqBatch),
                ("d_groups", C.c_void_p)]


class GqBatchSpec(C.Structure):
    _fields_ = [("keys", C.POINTER(C.c_int32)), ("nkeys", C.c_int32), ("naggs", C.c_int32),
                ("aggs", C.POINTER(GqAgg)), ("load_factor", C.c_float), ("lds_max_groups", C.c_int32),
                ("tile_rows", C.c_int32), ("blocks_per_cu", C.c_int32), ("radix_min_groups", C.c_int32)]


class GqAllocator(C.Structure):
    _fields_ = [("alloc", C.c_void_p), ("free", C.c_void_p), ("user", C.c_void_p)]


_P = C.c_void_p
_SIGS = {
    "gq_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "gq_ctx_destroy": (C.c_int, [_P]),
    "gq_last_error": (C.c_char_p, [_P]),
    "gq_ctx_sync_status": (C.c_int, [_P, _P, C.POINTER(C.c_int32)]),
    "gq_ctx_status_ptr": (_P, [_P]),
    "gq_ctx_set_timing": (C.c_int, [_P, C.c_int]),
    "gq_ctx_set_timing_only": (C.c_int, [_P, C.c_char_p]),
    "gq_ctx_timing_report": (C.c_int, [_P, C.c_char_p, C.c_int, _P, _P, C.c_int]),
    "gq_filter": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(GqPred), C.c_int,
                            C.POINTER(C.c_int32), C.c_int, C.POINTER(GqBatch), _P, _P]),
    "gq_filter_noalloc": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(GqPred), C.c_int,
                                    C.POINTER(C.c_int32), C.c_int, C.POINTER(GqBatch), _P, _P]),
    "gq_hash_partition": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int,
                                    C.c_int32, C.c_uint64, C.POINTER(GqBatch), _P, _P]),
    "gq_join_build": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int,
                                C.POINTER(GqPred), C.c_int, C.POINTER(GqJoinOpts), _P,
                                C.POINTER(_P)]),
    "gq_join_probe": (C.c_int, [_P, _P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int,
                                C.POINTER(GqPred), C.c_int, _P, _P, C.c_int64, _P, _P]),
    "gq_join_table_count_ptr": (_P, [_P]),
    "gq_join_table_free": (C.c_int, [_P, _P, _P]),
    "gq_gather": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int, _P,
                            C.c_int64, C.POINTER(GqBatch), _P]),
    "gq_groupby_agg": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int,
                                 C.POINTER(GqPred), C.c_int, C.POINTER(GqAgg), C.c_int,
                                 C.POINTER(GqGroupbyOpts), C.POINTER(GqBatch), _P, _P]),
    "gq_pipeline": (C.c_int, [_P, C.POINTER(GqPlan), C.POINTER(GqBatch), C.POINTER(GqBatch),
                              _P, _P]),
    "gq_pipeline_shared": (C.c_int, [_P, C.POINTER(GqPlan), C.POINTER(GqBatch), C.c_int32, C.POINTER(_P),
                                     C.POINTER(GqPred), C.POINTER(C.POINTER(GqBatch)), C.POINTER(_P), _P]),
    "gq_groupby_shared": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int, C.POINTER(GqPred),
                                    C.c_int, C.c_int, C.POINTER(GqAgg), C.c_int, C.POINTER(GqGroupbyOpts),
                                    C.POINTER(GqBatch), _P, _P]),
    "gq_batch_plan_create": (C.c_int, [_P, C.POINTER(GqFragment), C.c_int, C.POINTER(GqBatchSpec), _P,
                                       C.POINTER(_P)]),
    "gq_batch_plan_launch": (C.c_int, [_P, _P]),
    "gq_batch_plan_info": (C.c_int, [_P, _P, _P, _P, _P]),
    "gq_batch_plan_free": (C.c_int, [_P]),
    "gq_join_groupby": (C.c_int, [_P, _P, C.POINTER(GqBatch), C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int,
                                  C.POINTER(GqPred), C.c_int, C.POINTER(C.c_int32), C.c_int, C.POINTER(GqAgg),
                                  C.c_int, C.POINTER(GqGroupbyOpts), C.c_int64, C.POINTER(GqBatch), _P, _P]),
    "gq_compute_column": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(GqExpr), C.POINTER(GqColumn), _P]),
    "gq_filter_expr": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(GqPred), C.c_int, C.POINTER(GqExpr), C.c_int,
                                 C.POINTER(C.c_int32), C.c_int, C.POINTER(GqBatch), _P, _P]),
    "gq_groupby_expr": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int, C.POINTER(GqPred), C.c_int,
                                  C.POINTER(GqExpr), C.c_int, C.POINTER(C.c_int32), C.POINTER(GqExpr), C.c_int,
                                  C.POINTER(GqGroupbyOpts), C.POINTER(GqBatch), _P, _P]),
    "gq_order_by": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), C.c_int64, _P, _P]),
    "gq_agg_stream_create": (C.c_int, [_P, C.POINTER(GqAggStreamSpec), _P, C.POINTER(_P)]),
    "gq_agg_stream_push": (C.c_int, [_P, C.POINTER(GqBatch), C.POINTER(GqPred), C.c_int, C.POINTER(GqBatch),
                                     _P, _P]),
    "gq_agg_stream_finish": (C.c_int, [_P, C.POINTER(GqBatch), _P, _P]),
    "gq_agg_stream_free": (C.c_int, [_P, _P]),
}
EXPORTS = tuple(_SIGS)

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def lib():
    return _lib


class GqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# Device tables
# ---------------------------------------------------------------------------

def bitmap_bytes(n: int) -> int:
    return ((n + 63) // 64) * 8


@dataclass
class DevColumn:
    data: torch.Tensor                   # 1-D int8/16/32/64 on the device
    valid: torch.Tensor | None = None    # uint8 LSB-first bitmap, or None = all valid
    offset: int = 0                      # Arrow slice offset (rows)
    length: int | None = None            # rows (defaults to len(data) - offset)
    scale: int = 0

    @property
    def type(self) -> int:
        return _TORCH_TYPE[self.data.dtype]

    @property
    def nrows(self) -> int:
        return self.data.numel() - self.offset if self.length is None else self.length

    def abi(self) -> GqColumn:
        return GqColumn(self.type, self.scale, self.nrows, self.offset,
                        self.data.data_ptr() if self.data.numel() else None,
                        self.valid.data_ptr() if self.valid is not None else None)


@dataclass
class DevTable:
    cols: list = field(default_factory=list)
    nrows_override: int | None = None

    @property
    def nrows(self) -> int:
        if self.nrows_override is not None:
            return self.nrows_override
        return self.cols[0].nrows if self.cols else 0

    def head(self, n: int) -> "DevTable":
        """The first n rows (a view: columns and bitmaps are shared)."""
        return DevTable([DevColumn(c.data, c.valid, c.offset, n, c.scale) for c in self.cols])


def to_device(table, device="cuda") -> DevTable:
    """Upload a host table (objects with .data numpy array and .valid bool array)."""
    out = DevTable()
    for c in table.cols:
        d = torch.from_numpy(np.ascontiguousarray(c.data)).to(device)
        v = None
        if c.valid is not None:
            bm = np.zeros(bitmap_bytes(len(c.data)), dtype=np.uint8)
            if len(c.data):
                b = np.packbits(np.asarray(c.valid, dtype=np.uint8), bitorder="little")
                bm[: len(b)] = b
            v = torch.from_numpy(bm).to(device)
        out.cols.append(DevColumn(d, v, scale=getattr(c, "scale", 0)))
    return out


def empty_like_cols(types, capacity, nullable, device="cuda") -> DevTable:
    t = DevTable()
    for ty, nl in zip(types, nullable):
        d = torch.empty(max(1, capacity), dtype=_TYPE_TORCH[ty], device=device)[:capacity] \
            if capacity > 0 else torch.empty(0, dtype=_TYPE_TORCH[ty], device=device)
        v = torch.zeros(max(8, bitmap_bytes(capacity)), dtype=torch.uint8, device=device) if nl else None
        t.cols.append(DevColumn(d, v))
    return t


class _BatchArg:
    """Keeps the ctypes column array of a DevTable alive for one call."""

    def __init__(self, table: DevTable, capacity: int | None = None):
        n = len(table.cols)
        self.arr = (GqColumn * max(1, n))()
        for i, c in enumerate(table.cols):
            self.arr[i] = c.abi()
            if capacity is not None:
                self.arr[i].length = capacity
        nrows = table.nrows if capacity is None else capacity
        self.batch = GqBatch(nrows, n, 0, C.cast(self.arr, C.POINTER(GqColumn)))

    @property
    def ref(self):
        return C.byref(self.batch)


def _preds(preds):
    preds = list(preds or [])
    arr = (GqPred * max(1, len(preds)))()
    for i, p in enumerate(preds):
        arr[i].op = _PRED_OPS[p[0]]
        arr[i].col = p[1]
        if p[0] == "range":
            arr[i].lo, arr[i].hi = int(p[2]), int(p[3])
        else:
            arr[i].lo = arr[i].hi = int(p[2])
    return arr, len(preds)


def _ints(xs):
    xs = list(xs or [])
    return (C.c_int32 * max(1, len(xs)))(*xs), len(xs)


def _aggs(aggs):
    aggs = list(aggs or [])
    arr = (GqAgg * max(1, len(aggs)))()
    for i, a in enumerate(aggs):
        arr[i].op = _AGGS[a[0]]
        fs = a[1] if len(a) > 1 else []
        arr[i].nfactors = len(fs)
        for j, f in enumerate(fs):
            arr[i].f[j].kind = _FACTORS[f[0]]
            if f[0] == "col":
                arr[i].f[j].col = f[1]
            elif f[0] == "const":
                arr[i].f[j].k = int(f[1])
            else:
                arr[i].f[j].k, arr[i].f[j].col = int(f[1]), f[2]
    return arr, len(aggs)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def agg_nullable(table: DevTable, agg) -> bool:
    if agg[0] in ("count*", "count"):
        return False
    return True


# ---------------------------------------------------------------------------
# Context
# ---------------------------------------------------------------------------

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class GqAllocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


def make_allocator(alloc, free) -> GqAllocator:
    """A gq_allocator from two Python callables: alloc(nbytes, stream) -> int
    device pointer or None, free(ptr, nbytes, stream)."""
    return GqAllocator(_ALLOC_FN(lambda n, s, u: alloc(n, s)), _FREE_FN(lambda p, n, s, u: free(p, n, s)), None)


def _torch_allocator(device: int) -> GqAllocator:
    """gq_allocator over torch's caching allocator (stream-ordered per stream):
    one cache for the library's scratch and the caller's tensors.

    torch reuses a freed block for later allocations on the stream it was
    allocated on.  A block freed on another stream (a join table built on one
    stream and freed on the stream that used it) first makes the allocation
    stream wait for the freeing stream's work, so that reuse is ordered after
    every use."""
    owner = {}

    def alloc(nbytes, stream, user):
        try:
            ptr = torch.cuda.caching_allocator_alloc(max(1, int(nbytes)), device, stream or 0)
        except Exception:  # noqa: BLE001 - reported by the library as GQ_ERR_NOMEM
            return None
        owner[ptr] = stream or 0
        return ptr

    def free(ptr, nbytes, stream, user):
        if not ptr:
            return
        home = owner.pop(ptr, None)
        if home is not None and (stream or 0) != home:
            ev = torch.cuda.Event()
            ev.record(torch.cuda.ExternalStream(stream or 0, device=device) if stream else
                      torch.cuda.default_stream(device))
            (torch.cuda.ExternalStream(home, device=device) if home else torch.cuda.default_stream(device)).wait_event(ev)
        torch.cuda.caching_allocator_delete(ptr)

    return GqAllocator(_ALLOC_FN(alloc), _FREE_FN(free), None)


class Context:
    """A library context.  allocator=None: hipMallocAsync on the device's pool;
    allocator="torch": the library allocates through torch's caching allocator
    (for callers that also hold large torch tensors: one cache instead of two);
    a GqAllocator: the caller's own callbacks (see make_allocator)."""

    def __init__(self, device: int | None = None, allocator=None):
        self.device = torch.cuda.current_device() if device is None else device
        h = C.c_void_p()
        self._alloc = None
        if isinstance(allocator, GqAllocator):
            self._alloc = allocator          # caller-built callbacks (kept alive here)
            rc = _lib.gq_ctx_create(self.device, C.byref(self._alloc), C.byref(h))
        elif allocator == "torch":
            self._alloc = _torch_allocator(self.device)
            rc = _lib.gq_ctx_create(self.device, C.byref(self._alloc), C.byref(h))
        elif allocator is None:
            rc = _lib.gq_ctx_create(self.device, None, C.byref(h))
        else:
            raise ValueError(f"unknown allocator {allocator!r}")
        if rc != GQ_OK:
            raise GqError(rc, "gq_ctx_create failed")
        self.h = h

    def close(self):
        if self.h:
            _lib.gq_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc):
        if rc != GQ_OK:
            raise GqError(rc, _lib.gq_last_error(self.h).decode())

    def sync_status(self, stream=None) -> int:
        """Synchronise the stream; return the device status bits (and clear them)."""
        bits = C.c_int32(0)
        rc = _lib.gq_ctx_sync_status(self.h, _stream(stream), C.byref(bits))
        if rc not in (GQ_OK, GQ_ERR_CAPACITY, GQ_ERR_TABLE_FULL):
            self.check(rc)
        return int(bits.value)

    def set_timing(self, enable: bool, only: str | None = None):
        """Per-kernel events on (every launch, or only launches named `only`) or off."""
        self.check(_lib.gq_ctx_set_timing_only(self.h, only.encode() if only else None))
        self.check(_lib.gq_ctx_set_timing(self.h, 1 if enable else 0))

    def timing_report(self) -> dict:
        """{kernel name: (total ms, launches)} since the last report (synchronises)."""
        cap, nl = 64, 64
        names = C.create_string_buffer(cap * nl)
        ms = np.zeros(cap, dtype=np.float64)
        ln = np.zeros(cap, dtype=np.int64)
        n = _lib.gq_ctx_timing_report(self.h, names, nl, ms.ctypes.data, ln.ctypes.data, cap)
        if n < 0:
            self.check(n)
        out = {}
        for i in range(min(n, cap)):
            nm = names.raw[i * nl:(i + 1) * nl].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(ln[i]))
        return out

    def raise_status(self, stream=None):
        bits = C.c_int32(0)
        self.check(_lib.gq_ctx_sync_status(self.h, _stream(stream), C.byref(bits)))

    # -- operators ---------------------------------------------------------
    def filter(self, table: DevTable, preds, proj, capacity: int | None = None, stream=None):
        """Returns (output DevTable, device int64 count tensor)."""
        cap = table.nrows if capacity is None else capacity
        out = empty_like_cols([table.cols[j].type for j in proj], cap,
                              [table.cols[j].valid is not None for j in proj])
        cnt = torch.zeros(1, dtype=torch.int64, device=table.cols[0].data.device if table.cols else "cuda")
        p, np_ = _preds(preds)
        pj, npj = _ints(proj)
        ib, ob = _BatchArg(table), _BatchArg(out, cap)
        self.check(_lib.gq_filter(self.h, ib.ref, p, np_, pj, npj, ob.ref,
                                  C.c_void_p(cnt.data_ptr()), _stream(stream)))
        return out, cnt

    def filter_noalloc(self, table: DevTable, preds, proj, out: DevTable, cnt: torch.Tensor, capacity: int,
                       stream=None):
        """gq_filter_noalloc into caller-provided outputs (no allocation in the
        library): out must have the projected columns' types and `capacity`
        rows; cnt is a device int64 tensor of one element."""
        p, np_ = _preds(preds)
        pj, npj = _ints(proj)
        ib, ob = _BatchArg(table), _BatchArg(out, capacity)
        self.check(_lib.gq_filter_noalloc(self.h, ib.ref, p, np_, pj, npj, ob.ref,
                                          C.c_void_p(cnt.data_ptr()), _stream(stream)))

    def hash_partition(self, table: DevTable, keys, nparts: int, seed: int = 0, stream=None):
        """Returns (output DevTable of all columns, device int64 offsets[nparts+1])."""
        n = table.nrows
        out = empty_like_cols([c.type for c in table.cols], n, [c.valid is not None for c in table.cols])
        offs = torch.empty(nparts + 1, dtype=torch.int64, device="cuda")
        k, nk = _ints(keys)
        ib, ob = _BatchArg(table), _BatchArg(out, n)
        self.check(_lib.gq_hash_partition(self.h, ib.ref, k, nk, nparts, seed & 0xFFFFFFFFFFFFFFFF,
                                          ob.ref, C.c_void_p(offs.data_ptr()), _stream(stream)))
        return out, offs

    def join_build(self, table: DevTable, keys, preds=(), load_factor: float = 0.0,
                   acc_slots: int = 0, regions_log2: int = 0, stream=None) -> "JoinTable":
        k, nk = _ints(keys)
        p, np_ = _preds(preds)
        opts = GqJoinOpts(load_factor, acc_slots, regions_log2)
        h = C.c_void_p()
        ib = _BatchArg(table)
        self.check(_lib.gq_join_build(self.h, ib.ref, k, nk, p, np_, C.byref(opts),
                                      _stream(stream), C.byref(h)))
        return JoinTable(self, h)

    def join_probe(self, jt: "JoinTable", table: DevTable, keys, preds=(), capacity: int | None = None,
                   stream=None):
        """Returns (probe_idx int32, build_idx int32, device count)."""
        cap = table.nrows if capacity is None else capacity
        pi = torch.empty(max(1, cap), dtype=torch.int32, device="cuda")
        bi = torch.empty(max(1, cap), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        k, nk = _ints(keys)
        p, np_ = _preds(preds)
        ib = _BatchArg(table)
        self.check(_lib.gq_join_probe(self.h, jt.h, ib.ref, k, nk, p, np_,
                                      C.c_void_p(pi.data_ptr()), C.c_void_p(bi.data_ptr()), cap,
                                      C.c_void_p(cnt.data_ptr()), _stream(stream)))
        return pi, bi, cnt

    def gather(self, table: DevTable, cols, idx: torch.Tensor, n: int | None = None, stream=None):
        n = idx.numel() if n is None else n
        out = empty_like_cols([table.cols[j].type for j in cols], n,
                              [table.cols[j].valid is not None for j in cols])
        cs, nc = _ints(cols)
        ib, ob = _BatchArg(table), _BatchArg(out, n)
        self.check(_lib.gq_gather(self.h, ib.ref, cs, nc, C.c_void_p(idx.data_ptr()), n, ob.ref,
                                  _stream(stream)))
        return out

    def compute_column(self, table: DevTable, tree, stream=None):
        """(int64 values, bitmap) of an expression tree over every row."""
        out = empty_like_cols([GQ_I64], table.nrows, [True])
        e = _ExprArg([tree])
        ib, ob = _BatchArg(table), _BatchArg(out, table.nrows)
        self.check(_lib.gq_compute_column(self.h, ib.ref, e.ptr, ob.arr, _stream(stream)))
        return out

    def filter_expr(self, table: DevTable, preds, exprs, proj, capacity: int | None = None, stream=None):
        """Filter by predicates and expression trees (non-NULL, non-zero);
        returns (output DevTable, device count)."""
        cap = table.nrows if capacity is None else capacity
        out = empty_like_cols([table.cols[j].type for j in proj], cap, [table.cols[j].valid is not None for j in proj])
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        p, np_ = _preds(preds)
        e = _ExprArg(exprs)
        pj, npj = _ints(proj)
        ib, ob = _BatchArg(table), _BatchArg(out, cap)
        self.check(_lib.gq_filter_expr(self.h, ib.ref, p, np_, e.ptr, len(exprs), pj, npj, ob.ref,
                                       C.c_void_p(cnt.data_ptr()), _stream(stream)))
        return out, cnt

    def groupby_expr(self, table: DevTable, keys, preds, exprs, aggs, capacity: int | None = None,
                     expected_groups=0, stream=None):
        """Group-by with expression aggregates: aggs are (op, tree) with op in
        sum/count/min/max, or ("count*",).  Returns (output, device count)."""
        cap = max(1, table.nrows) if capacity is None else capacity
        types = [table.cols[j].type for j in keys] + [GQ_I64] * len(aggs)
        nullable = [table.cols[j].valid is not None for j in keys] + [a[0] not in ("count*", "count") for a in aggs]
        out = empty_like_cols(types, cap, nullable)
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        k, nk = _ints(keys)
        p, np_ = _preds(preds)
        e = _ExprArg(exprs)
        ops, _ = _ints([_AGGS[a[0]] for a in aggs])
        ae = _ExprArg([a[1] if len(a) > 1 else ("const", 0) for a in aggs])
        opts = self._opts(0.0, "auto", False, 0, expected_groups)
        ib, ob = _BatchArg(table), _BatchArg(out, cap)
        self.check(_lib.gq_groupby_expr(self.h, ib.ref, k, nk, p, np_, e.ptr, len(exprs), ops, ae.ptr, len(aggs),
                                        C.byref(opts), ob.ref, C.c_void_p(cnt.data_ptr()), _stream(stream)))
        return out, cnt

    def order_by(self, table: DevTable, keys, desc=None, nulls_first=None, limit=None, stream=None):
        """Row ids (device int32) in ORDER BY order; the first `limit` with a limit."""
        n = table.nrows
        take = n if limit is None else min(int(limit), n)
        out = torch.empty(max(1, take), dtype=torch.int32, device="cuda")
        k, nk = _ints(keys)
        d, _ = _ints([1 if x else 0 for x in (desc or [False] * nk)])
        nf, _ = _ints([1 if x else 0 for x in (nulls_first or [False] * nk)])
        ib = _BatchArg(table)
        self.check(_lib.gq_order_by(self.h, ib.ref, k, nk, d, nf, -1 if limit is None else int(limit),
                                    C.c_void_p(out.data_ptr()), _stream(stream)))
        return out[:take]

    def join_groupby(self, jt: "JoinTable", build: DevTable, probe: DevTable, probe_keys, probe_preds, group_keys,
                     aggs, capacity: int | None = None, pair_capacity: int = 0, load_factor=0.0, strategy="auto",
                     expected_groups=0, stream=None):
        """Group-by over the joined rows (late materialisation).  Column c of a
        joined row is probe column c for c < len(probe.cols), else build column
        c - len(probe.cols).  Returns (output DevTable, device group count)."""
        joined = DevTable(list(probe.cols) + list(build.cols))
        cap = max(1, pair_capacity or probe.nrows) if capacity is None else capacity
        out = self._groupby_out(joined, group_keys, aggs, cap)
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        pk, npk = _ints(probe_keys)
        p, np_ = _preds(probe_preds)
        gk, ngk = _ints(group_keys)
        a, na = _aggs(aggs)
        opts = self._opts(load_factor, strategy, False, 0, expected_groups)
        bb, pb, ob = _BatchArg(build), _BatchArg(probe), _BatchArg(out, cap)
        self.check(_lib.gq_join_groupby(self.h, jt.h, bb.ref, pb.ref, pk, npk, p, np_, gk, ngk, a, na,
                                        C.byref(opts), int(pair_capacity), ob.ref, C.c_void_p(cnt.data_ptr()),
                                        _stream(stream)))
        return out, cnt

    def _groupby_out(self, table, keys, aggs, capacity, merge=False):
        types = [table.cols[j].type for j in keys] + [GQ_I64] * len(aggs)
        nullable = [table.cols[j].valid is not None for j in keys] + [merge or agg_nullable(table, a) for a in aggs]
        return empty_like_cols(types, capacity, nullable)

    @staticmethod
    def _opts(load_factor=0.0, strategy="auto", sorted=False, block_size=0, expected_groups=0, mode="single"):
        return GqGroupbyOpts(load_factor, STRATEGY[strategy], GQ_SORTED if sorted else 0, block_size,
                             expected_groups, MODES[mode], 0)

    def groupby_agg(self, table: DevTable, keys, preds, aggs, capacity: int | None = None,
                    load_factor=0.0, strategy="auto", sorted=False, block_size=0, expected_groups=0,
                    stream=None, mode="single"):
        """Returns (output DevTable: keys then aggregates, device int64 group count).
        mode: "single" / "partial" (raw rows), "intermediate" / "final" (state
        rows: each aggregate names its state column with one ("col", c) factor)."""
        cap = max(1, table.nrows) if capacity is None else capacity
        out = self._groupby_out(table, keys, aggs, cap, merge=mode in ("intermediate", "final"))
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        k, nk = _ints(keys)
        p, np_ = _preds(preds)
        a, na = _aggs(aggs)
        opts = self._opts(load_factor, strategy, sorted, block_size, expected_groups, mode)
        ib, ob = _BatchArg(table), _BatchArg(out, cap)
        self.check(_lib.gq_groupby_agg(self.h, ib.ref, k, nk, p, np_, a, na, C.byref(opts), ob.ref,
                                       C.c_void_p(cnt.data_ptr()), _stream(stream)))
        return out, cnt

    def groupby_shared(self, table: DevTable, keys, query_preds, aggs, capacity: int | None = None,
                       load_factor=0.0, expected_groups=0, sorted=False, stream=None):
        """Several filter + group-by queries in one pass (query_preds: one predicate
        list per query, same columns and ops).  Returns (list of outputs, device counts)."""
        nq = len(query_preds)
        npreds = len(query_preds[0]) if nq else 0
        cap = max(1, table.nrows) if capacity is None else capacity
        outs = [self._groupby_out(table, keys, aggs, cap) for _ in range(nq)]
        cnt = torch.zeros(max(1, nq), dtype=torch.int64, device="cuda")
        flat = [p for q in query_preds for p in q]
        p, _ = _preds(flat)
        k, nk = _ints(keys)
        a, na = _aggs(aggs)
        obs = [_BatchArg(o, cap) for o in outs]
        oarr = (GqBatch * max(1, nq))(*[ob.batch for ob in obs])
        opts = self._opts(load_factor, "auto", sorted, 0, expected_groups)
        ib = _BatchArg(table)
        self.check(_lib.gq_groupby_shared(self.h, ib.ref, k, nk, p, npreds, nq, a, na, C.byref(opts), oarr,
                                          C.c_void_p(cnt.data_ptr()), _stream(stream)))
        return outs, cnt

    def pipeline(self, table: DevTable, preds, group_keys, aggs, join: "JoinTable | None" = None,
                 probe_key: int = 0, capacity: int | None = None, load_factor=0.0,
                 strategy="auto", sorted=False, block_size=0, expected_groups=0, stream=None):
        cap = max(1, table.nrows) if capacity is None else capacity
        out = self._groupby_out(table, group_keys, aggs, cap)
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        p, np_ = _preds(preds)
        k, nk = _ints(group_keys)
        a, na = _aggs(aggs)
        plan = GqPlan(C.cast(p, C.POINTER(GqPred)), np_, probe_key, join.h if join else None,
                      C.cast(k, C.POINTER(C.c_int32)), nk, na, C.cast(a, C.POINTER(GqAgg)),
                      self._opts(load_factor, strategy, sorted, block_size, expected_groups))
        ib, ob = _BatchArg(table), _BatchArg(out, cap)
        self.check(_lib.gq_pipeline(self.h, C.byref(plan), ib.ref, ob.ref, C.c_void_p(cnt.data_ptr()),
                                    _stream(stream)))
        return out, cnt

    def pipeline_shared(self, table: DevTable, preds, probe_key, aggs, joins, ranges, capacity: int | None = None,
                        sorted=False, stream=None):
        """gq_pipeline_shared: one group-join pipeline per (join table, range)
        pair, the probe side partitioned once.  ranges: ("range", col, lo, hi)
        tuples on one column.  Returns a list of (out, device count)."""
        joins, ranges = list(joins), list(ranges)
        nq = len(joins)
        cap = max(1, table.nrows) if capacity is None else capacity
        outs = [self._groupby_out(table, [probe_key], aggs, cap) for _ in range(nq)]
        cnt = torch.zeros(max(1, nq), dtype=torch.int64, device="cuda")
        p, np_ = _preds(preds)
        r, nr = _preds(ranges)
        k, nk = _ints([probe_key])
        a, na = _aggs(aggs)
        plan = GqPlan(C.cast(p, C.POINTER(GqPred)), np_, probe_key, None, C.cast(k, C.POINTER(C.c_int32)), nk, na,
                      C.cast(a, C.POINTER(GqAgg)), self._opts(0.0, "auto", sorted, 0, 0))
        ib = _BatchArg(table)
        obs = [_BatchArg(o, cap) for o in outs]
        oarr = (C.POINTER(GqBatch) * max(1, nq))(*[C.pointer(ob.batch) for ob in obs])
        tarr = (_P * max(1, nq))(*[j.h.value if isinstance(j.h, C.c_void_p) else j.h for j in joins])
        carr = (_P * max(1, nq))(*[cnt.data_ptr() + 8 * i for i in range(nq)])
        self.check(_lib.gq_pipeline_shared(self.h, C.byref(plan), ib.ref, nq, tarr, C.cast(r, C.POINTER(GqPred)),
                                           oarr, carr, _stream(stream)))
        return [(outs[i], cnt[i:i + 1]) for i in range(nq)]


class AggStream:
    """Streaming aggregation over a sequence of batches (gq_agg_stream_*).

    mode: "single", "partial", "intermediate" or "final"; keys: key column
    indices of every batch; key_types: their gq types; key_nullable: which key
    columns may be NULL; aggs: as for groupby_agg in that mode; max_groups:
    table size; emit_groups: Partial / Intermediate emit once this many
    groups are held (0: only at finish).  push() returns (out, device emitted
    count) for a stream that can emit early, else None; finish() returns
    (out, device int64[2]: groups, emitted flag).  Call free() to release the
    stream's table (there is no implicit release)."""

    def __init__(self, ctx: "Context", mode, keys, key_types, key_nullable, aggs, max_groups, emit_groups=0,
                 load_factor=0.0, stream=None):
        self.ctx = ctx
        self.h = None
        self.mode = mode
        self.keys = list(keys)
        self.key_types = list(key_types)
        self.key_nullable = [bool(x) for x in key_nullable]
        self.aggs = list(aggs)
        self.max_groups = int(max_groups) if self.keys else 1
        self.emit_groups = int(emit_groups)
        self._k, nk = _ints(self.keys)
        self._kn, _ = _ints([1 if x else 0 for x in self.key_nullable])
        self._a, na = _aggs(self.aggs)
        spec = GqAggStreamSpec(MODES[mode], nk, C.cast(self._k, C.POINTER(C.c_int32)),
                               C.cast(self._kn, C.POINTER(C.c_int32)), C.cast(self._a, C.POINTER(GqAgg)), na, 0,
                               self.max_groups, self.emit_groups, load_factor, 0)
        h = C.c_void_p()
        ctx.check(_lib.gq_agg_stream_create(ctx.h, C.byref(spec), _stream(stream), C.byref(h)))
        self.h = h

    def _out(self):
        types = self.key_types + [GQ_I64] * len(self.aggs)
        return empty_like_cols(types, max(1, self.max_groups), self.key_nullable + [True] * len(self.aggs))

    @property
    def emits_early(self):
        return self.mode in ("partial", "intermediate") and self.emit_groups > 0

    def push(self, table: DevTable, preds=(), stream=None):
        p, np_ = _preds(preds)
        ib = _BatchArg(table)
        if self.emits_early:
            out = self._out()
            ob = _BatchArg(out, max(1, self.max_groups))
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            self.ctx.check(_lib.gq_agg_stream_push(self.h, ib.ref, p, np_, ob.ref, C.c_void_p(cnt.data_ptr()),
                                                   _stream(stream)))
            return out, cnt
        self.ctx.check(_lib.gq_agg_stream_push(self.h, ib.ref, p, np_, None, None, _stream(stream)))
        return None

    def finish(self, stream=None):
        out = self._out()
        ob = _BatchArg(out, max(1, self.max_groups))
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        self.ctx.check(_lib.gq_agg_stream_finish(self.h, ob.ref, C.c_void_p(cnt.data_ptr()), _stream(stream)))
        return out, cnt

    def free(self, stream=None):
        if self.h:
            self.ctx.check(_lib.gq_agg_stream_free(self.h, _stream(stream)))
            self.h = None


class BatchPlan:
    """Many filter + group-by fragments in one graph-captured persistent launch.

    fragments: list of (DevTable, preds, expected_groups[, out_capacity]);
    every fragment uses the same key columns and aggregates.  Outputs are
    allocated here, one DevTable per fragment with capacity out_capacity, by
    default min(rows, expected_groups).
    """

    def __init__(self, ctx: "Context", fragments, keys, aggs, load_factor=0.0, lds_max_groups=0,
                 tile_rows=0, blocks_per_cu=0, radix_min_groups=0, stream=None):
        self.ctx = ctx
        self.h = None
        nf = len(fragments)
        self._keep = []
        self.outs = []
        self.d_groups = torch.zeros(nf, dtype=torch.int64, device="cuda")
        farr = (GqFragment * nf)()
        for f, fr in enumerate(fragments):
            tab, preds, expected = fr[:3]
            cap = tab.nrows if not expected else min(tab.nrows, int(expected))
            if len(fr) > 3 and fr[3] is not None:
                cap = int(fr[3])
            cap = max(cap, 1)
            out = ctx._groupby_out(tab, keys, aggs, cap)
            ib, ob = _BatchArg(tab), _BatchArg(out, cap)
            p, np_ = _preds(preds)
            self._keep += [ib, ob, p, out, tab]
            self.outs.append(out)
            farr[f].inp = ib.batch
            farr[f].preds = C.cast(p, C.POINTER(GqPred))
            farr[f].npreds = np_
            farr[f].expected_groups = int(expected or 0)
            farr[f].out = ob.batch
            farr[f].d_groups = self.d_groups.data_ptr() + 8 * f
        k, nk = _ints(keys)
        a, na = _aggs(aggs)
        self._keep += [k, a, farr]
        spec = GqBatchSpec(C.cast(k, C.POINTER(C.c_int32)), nk, na, C.cast(a, C.POINTER(GqAgg)),
                           load_factor, lds_max_groups, tile_rows, blocks_per_cu, radix_min_groups)
        h = C.c_void_p()
        ctx.check(_lib.gq_batch_plan_create(ctx.h, farr, nf, C.byref(spec), _stream(stream), C.byref(h)))
        self.h = h

    def launch(self, stream=None):
        self.ctx.check(_lib.gq_batch_plan_launch(self.h, _stream(stream)))

    def info(self) -> dict:
        v = [C.c_int64() for _ in range(4)]
        self.ctx.check(_lib.gq_batch_plan_info(self.h, *[C.byref(x) for x in v]))
        return dict(zip(["total_rows", "tiles", "table_slots", "bytes"], [x.value for x in v]))

    def result(self, f: int):
        """Output columns of fragment f as [(values, valid)] and its group count (synchronises)."""
        n = int(self.d_groups[f].item())
        return read_table(self.outs[f], n), n

    def free(self):
        if self.h:
            _lib.gq_batch_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class JoinTable:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def count_tensor(self):
        """Device int64 with the number of inserted build rows (a 1-element view)."""
        ptr = _lib.gq_join_table_count_ptr(self.h)
        return ptr

    def free(self, stream=None):
        if self.h:
            self.ctx.check(_lib.gq_join_table_free(self.ctx.h, self.h, _stream(stream)))
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Host-side readers (after a synchronisation)
# ---------------------------------------------------------------------------

def read_column(col: DevColumn, n: int):
    """(values numpy, valid bool numpy or None) of the first n rows."""
    v = col.data[:n].cpu().numpy()
    if col.valid is None:
        return v, None
    bm = col.valid.cpu().numpy()
    valid = np.unpackbits(bm, bitorder="little")[:n].astype(bool)
    return v, valid


def read_table(t: DevTable, n: int):
    return [read_column(c, n) for c in t.cols]
