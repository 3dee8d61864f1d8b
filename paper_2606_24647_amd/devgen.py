"""Device twin of the seeded input generator (libgqgen.so, csrc/gen.hip).

Produces the same columns as ``datagen`` directly in device memory, for
workloads too large to generate on the host and upload.  Input generation only.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import datagen as dg
from .gq import DevColumn, DevTable

_PKG = os.path.dirname(os.path.abspath(__file__))
GEN_PATH = os.path.join(_PKG, "libgqgen.so")
if not os.path.exists(GEN_PATH):
    raise ImportError(f"{GEN_PATH} is not built; run `python -m paper_2606_24647_amd.build`")
_gen = C.CDLL(GEN_PATH)
_P = C.c_void_p
_gen.gqgen_uniform.argtypes = [_P, C.c_int, C.c_int64, C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_int64, _P]
_gen.gqgen_zipf.argtypes = [_P, C.c_int64, C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, _P, _P]
_gen.gqgen_permutation.argtypes = [_P, C.c_int64, C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_int64, _P]

_WIDTH = {torch.int8: 1, torch.int16: 2, torch.int32: 4, torch.int64: 8}
_NP2T = {"int8": torch.int8, "int16": torch.int16, "int32": torch.int32, "int64": torch.int64}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"device generator failed: {what}")


def uniform(seed, col, start, n, lo, hi, dtype=torch.int64, out=None):
    t = out if out is not None else torch.empty(max(1, n), dtype=dtype, device="cuda")[:n]
    _check(_gen.gqgen_uniform(t.data_ptr() if n else None, _WIDTH[t.dtype], n, seed, col, start, lo, hi, _stream()),
           "uniform")
    return t


_ZIPF_DEV = {}


def zipf(seed, col, start, n, N):
    """Device twin of datagen.zipf: the host's threshold table, uploaded once
    per N, searched on the device."""
    thr = _ZIPF_DEV.get(N)
    if thr is None:
        _ZIPF_DEV.clear()
        thr = torch.from_numpy(dg.zipf_thresholds(N).view(np.int64)).cuda() if N > 1 else None
        _ZIPF_DEV[N] = thr
    t = torch.empty(max(1, n), dtype=torch.int64, device="cuda")[:n]
    _check(_gen.gqgen_zipf(t.data_ptr() if n else None, n, seed, col, start, N,
                           thr.data_ptr() if thr is not None else None, _stream()), "zipf")
    return t


def permutation(seed, col, start, n, N, add=0):
    t = torch.empty(max(1, n), dtype=torch.int64, device="cuda")[:n]
    _check(_gen.gqgen_permutation(t.data_ptr() if n else None, n, seed, col, start, N, add, _stream()), "permutation")
    return t


def _table(cols):
    return DevTable([DevColumn(d, None, scale=sc) for d, sc in cols])


def fact_c1(n=1_000_000, start=0, seed=1) -> DevTable:
    return _table([
        (uniform(seed, 0, start, n, 1, 50), 0),
        (uniform(seed, 1, start, n, dg.PRICE_LO, dg.PRICE_HI), 2),
        (uniform(seed, 2, start, n, 0, 10), 2),
        (uniform(seed, 3, start, n, 0, dg.DATE_DAYS - 1, torch.int32), 0),
        (uniform(seed, 4, start, n, 0, 2, torch.int8), 0),
        (uniform(seed, 5, start, n, 0, 1, torch.int8), 0),
    ])


def fact_c2(n=60_000_000, nkeys=15_000_000, start=0, seed=2) -> DevTable:
    return _table([
        (uniform(seed, 0, start, n, 1, nkeys), 0),
        (uniform(seed, 1, start, n, dg.PRICE_LO, dg.PRICE_HI), 2),
        (uniform(seed, 2, start, n, 0, 10), 2),
        (uniform(seed, 3, start, n, 0, dg.DATE_DAYS - 1, torch.int32), 0),
    ])


def dim_c2(n=15_000_000, start=0, seed=2, ckeys=None) -> DevTable:
    ckeys = ckeys if ckeys is not None else max(1, n // 10)
    m = n - start
    return _table([
        (permutation(seed, 16, start, m, n, add=1), 0),
        (uniform(seed, 17, start, m, 0, dg.DIM_DATE_DAYS - 1, torch.int32), 0),
        (uniform(seed, 18, start, m, 1, ckeys), 0),
    ])


def batch_c3(n=60_000_000, nkeys=15_000_000, start=0, seed=3) -> DevTable:
    return _table([
        (zipf(seed, 0, start, n, nkeys), 0),
        (uniform(seed, 1, start, n, dg.PRICE_LO, dg.PRICE_HI), 0),
        (uniform(seed, 2, start, n, 0, dg.DATE_DAYS - 1, torch.int32), 0),
        (uniform(seed, 3, start, n, 0, 2, torch.int8), 0),
    ])


def fact_c5(n=dg.C5_FACT_ROWS, nkeys=dg.C5_DIM_ROWS, start=0, seed=5) -> DevTable:
    return _table([
        (uniform(seed, 0, start, n, 1, nkeys), 0),
        (uniform(seed, 1, start, n, 1, 50), 0),
        (uniform(seed, 2, start, n, dg.PRICE_LO, dg.PRICE_HI), 2),
        (uniform(seed, 3, start, n, 0, 10), 2),
        (uniform(seed, 4, start, n, 0, dg.DATE_DAYS - 1, torch.int32), 0),
        (uniform(seed, 5, start, n, 0, 2, torch.int8), 0),
        (uniform(seed, 6, start, n, 0, 1, torch.int8), 0),
    ])


def dim_c5(n=dg.C5_DIM_ROWS, start=0, seed=5) -> DevTable:
    return dim_c2(n, start=start, seed=seed, ckeys=max(1, n // 10))


def fragment_c4(f, rows, card, seed=4) -> DevTable:
    s = dg.fragment_seed(f, seed)
    return _table([
        (uniform(s, 0, 0, rows, 1, 50), 0),
        (uniform(s, 1, 0, rows, dg.PRICE_LO, dg.PRICE_HI), 2),
        (uniform(s, 2, 0, rows, 0, 10), 2),
        (uniform(s, 3, 0, rows, 0, dg.DATE_DAYS - 1, torch.int32), 0),
        (uniform(s, 4, 0, rows, 0, card - 1, torch.int32), 0),
    ])


def fragments_c4_resident(nfrag=4096, seed=4, align=16):
    """Every fragment of the batched workload resident at once: five device
    columns holding all fragments back to back, fragment f starting on an
    `align`-row boundary (so its 128-bit loads stay aligned).  Fragment f's
    rows equal fragment_c4(f, ...).  Returns (spec, tables, cols, starts):
    the host spec (rows, cardinality, filter bound per fragment), one DevTable
    view per fragment, the five backing tensors and the fragment starts."""
    import numpy as np
    spec = dg.fragments_c4(nfrag, seed)
    starts = np.zeros(nfrag + 1, dtype=np.int64)
    for f in range(nfrag):
        starts[f + 1] = starts[f] + (int(spec.rows[f]) + align - 1) // align * align
    total = int(starts[-1])
    layout = [(torch.int64, 1, 50, 0), (torch.int64, dg.PRICE_LO, dg.PRICE_HI, 2), (torch.int64, 0, 10, 2),
              (torch.int32, 0, dg.DATE_DAYS - 1, 0), (torch.int32, 0, None, 0)]
    cols = [torch.empty(max(1, total), dtype=dt, device="cuda") for dt, _, _, _ in layout]
    tables = []
    for f in range(nfrag):
        n, card, s0 = int(spec.rows[f]), int(spec.card[f]), int(starts[f])
        s = dg.fragment_seed(f, seed)
        views = []
        for c, (col, (_, lo, hi, sc)) in enumerate(zip(cols, layout)):
            v = col[s0:s0 + n]
            uniform(s, c, 0, n, lo, card - 1 if hi is None else hi, out=v)
            views.append(DevColumn(v, None, scale=sc))
        tables.append(DevTable(views))
    return spec, tables, cols, starts
