"""Seeded synthetic column generators (host side, numpy).

This module is the only code shared by the oracle side and the GPU side of the
tests and the benchmark: it makes input columns and nothing else.  It holds none
of the operators' arithmetic (no predicate, hash, join or aggregation).

Every value is a pure function of (seed, column id, row index), so any row range
can be regenerated on its own and a device generator can reproduce the same
values bit for bit.  Column values use integer arithmetic only; the one use of
floating point is the host-only fragment table of the batched workload.

Building blocks (all mod 2**64):

* ``mix``: the SplitMix64 output finaliser (Steele, Lea and Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014):
  ``z ^= z >> 30; z *= 0xbf58476d1ce4e5b9; z ^= z >> 27; z *= 0x94d049bb133111eb;
  z ^= z >> 31``.
* stream of column ``c`` under ``seed``:
  ``s_c = mix(seed ^ (c * GAMMA))`` and ``r(row) = mix(s_c + (row + 1) * GAMMA)``
  with ``GAMMA = 0x9e3779b97f4a7c15``.
* uniform integer on ``[lo, hi]``: ``lo + mulhi64(r, hi - lo + 1)`` (Lemire's
  multiply-shift range reduction; the range is at most 2**32 here).
* Zipf keys on ``1..N`` with P(k) proportional to ``k**-0.5`` (exponent
  s = 0.5), by inversion: the thresholds ``T[k-1] = floor(2**63 * F(k))`` for
  k = 1..N-1, F the distribution function (float64 cumulative sums, computed
  once per N on the host and handed to the device generator as a table), and
  a 63-bit draw ``r >> 1`` maps to ``1 + #{k : T[k] <= r >> 1}``.  Host and
  device search the same table, so they agree bit for bit.
* permutation of ``0..N-1``: a 4-round balanced Feistel network over the
  smallest even bit width covering N, with cycle walking until the value falls
  below N (Black and Rogaway, "Ciphers with arbitrary finite domains", 2002).

The workload recipes (column order and ranges) are the synthetic stand-ins for
the TPC-H-like tables the paper measures on (Section 2 and Section 3.4): a
lineitem-like fact table, an orders-like dimension and date-range filters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

_U64 = np.uint64

# Arrow-style type codes used everywhere in this repository.
I8, I16, I32, I64 = 1, 2, 3, 4
NP_DTYPE = {I8: np.int8, I16: np.int16, I32: np.int32, I64: np.int64}
TYPE_OF_DTYPE = {np.dtype(np.int8): I8, np.dtype(np.int16): I16,
                 np.dtype(np.int32): I32, np.dtype(np.int64): I64}


def mix_int(z: int) -> int:
    """SplitMix64 finaliser on a Python int (used for per-column stream seeds)."""
    z &= MASK64
    z ^= z >> 30
    z = (z * M1) & MASK64
    z ^= z >> 27
    z = (z * M2) & MASK64
    z ^= z >> 31
    return z


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser, vectorised over a uint64 array (in place)."""
    z ^= z >> _U64(30)
    z *= _U64(M1)
    z ^= z >> _U64(27)
    z *= _U64(M2)
    z ^= z >> _U64(31)
    return z


def stream_seed(seed: int, col: int) -> int:
    return mix_int((seed ^ ((col * GAMMA) & MASK64)) & MASK64)


def raw(seed: int, col: int, start: int, n: int) -> np.ndarray:
    """r(row) for rows start..start+n-1 of column ``col`` (uint64)."""
    s = stream_seed(seed, col)
    with np.errstate(over="ignore"):
        z = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z *= _U64(GAMMA)
        z += _U64(s)
        return _mix(z)


def raw_at(seed: int, col: int, rows: np.ndarray) -> np.ndarray:
    """r(row) for arbitrary row indices (uint64)."""
    s = stream_seed(seed, col)
    with np.errstate(over="ignore"):
        z = np.asarray(rows, dtype=np.uint64) + np.uint64(1)
        z *= _U64(GAMMA)
        z += _U64(s)
        return _mix(z)


def _mulhi_small(r: np.ndarray, m: int) -> np.ndarray:
    """floor(r * m / 2**64) for uint64 r and 0 < m <= 2**32, exact."""
    assert 0 < m <= (1 << 32)
    with np.errstate(over="ignore"):
        if m == (1 << 32):
            return r >> _U64(32)
        mm = _U64(m)
        hi = r >> _U64(32)
        lo = r & _U64(0xFFFFFFFF)
        t = hi * mm + ((lo * mm) >> _U64(32))
        return t >> _U64(32)


def uniform(seed: int, col: int, start: int, n: int, lo: int, hi: int,
            dtype=np.int64) -> np.ndarray:
    """Uniform integers on [lo, hi] (inclusive)."""
    assert hi >= lo and hi - lo + 1 <= (1 << 32)
    r = raw(seed, col, start, n)
    v = _mulhi_small(r, hi - lo + 1).astype(np.int64)
    v += lo
    return v.astype(dtype, copy=False)


def uniform_at(seed: int, col: int, rows: np.ndarray, lo: int, hi: int, dtype=np.int64) -> np.ndarray:
    """Uniform integers on [lo, hi] at arbitrary row indices (same values as uniform())."""
    assert hi >= lo and hi - lo + 1 <= (1 << 32)
    v = _mulhi_small(raw_at(seed, col, rows), hi - lo + 1).astype(np.int64)
    v += lo
    return v.astype(dtype, copy=False)


_ZIPF_THRESHOLDS = {}


def zipf_thresholds(N: int) -> np.ndarray:
    """uint64 T[0..N-2]: T[k-1] = floor(2**63 * F(k)), F the distribution
    function of P(k) proportional to k**-0.5 on 1..N (cached per N)."""
    t = _ZIPF_THRESHOLDS.get(N)
    if t is None:
        w = 1.0 / np.sqrt(np.arange(1, N + 1, dtype=np.float64))
        cdf = np.cumsum(w)
        t = np.floor(cdf[:-1] / cdf[-1] * 2.0 ** 63).astype(np.uint64)
        _ZIPF_THRESHOLDS.clear()
        _ZIPF_THRESHOLDS[N] = t
    return t


def zipf(seed: int, col: int, start: int, n: int, N: int) -> np.ndarray:
    """Keys on 1..N with P(k) proportional to k**-0.5 (Zipf, s = 0.5).  The
    draws are searched in sorted order (the table is 8 N bytes; random probes
    into it would be memory-latency bound) and the keys put back in row order."""
    t = zipf_thresholds(N)
    r = raw(seed, col, start, n) >> _U64(1)
    order = np.argsort(r)
    k = np.empty(n, dtype=np.int64)
    k[order] = np.searchsorted(t, r[order], side="right") + 1
    return k


def _feistel_bits(N: int) -> int:
    b = max(2, (N - 1).bit_length())
    return b + (b & 1)


def feistel_keys(seed: int, col: int):
    return [mix_int(stream_seed(seed, col) ^ ((r + 1) * GAMMA & MASK64)) for r in range(4)]


def permutation(seed: int, col: int, start: int, n: int, N: int) -> np.ndarray:
    """Value pi(row) of a seeded permutation of 0..N-1 for rows start..start+n-1."""
    bits = _feistel_bits(N)
    half = bits // 2
    hmask = _U64((1 << half) - 1)
    keys = [_U64(k) for k in feistel_keys(seed, col)]

    def enc(x: np.ndarray) -> np.ndarray:
        left = x >> _U64(half)
        right = x & hmask
        with np.errstate(over="ignore"):
            for k in keys:
                f = _mix(right ^ k) & hmask
                left, right = right, left ^ f
        return (left << _U64(half)) | right

    x = np.arange(start, start + n, dtype=np.uint64)
    y = enc(x)
    bad = y >= _U64(N)
    while bad.any():
        y[bad] = enc(y[bad])
        bad = y >= _U64(N)
    return y.astype(np.int64)


def validity(seed: int, col: int, start: int, n: int, null_permille: int) -> np.ndarray:
    """Boolean validity (True = valid) with about null_permille/1000 nulls."""
    if null_permille <= 0:
        return np.ones(n, dtype=bool)
    r = raw(seed, 1000 + col, start, n)
    return _mulhi_small(r, 1000) >= _U64(null_permille)


def pack_validity(valid: np.ndarray) -> np.ndarray:
    """Arrow LSB-first validity bitmap (uint8), padded to a multiple of 8 bytes."""
    n = len(valid)
    nbytes = ((n + 63) // 64) * 8
    out = np.zeros(nbytes, dtype=np.uint8)
    if n:
        packed = np.packbits(valid.astype(np.uint8), bitorder="little")
        out[: len(packed)] = packed
    return out


def unpack_validity(bitmap: np.ndarray, n: int) -> np.ndarray:
    if bitmap is None:
        return np.ones(n, dtype=bool)
    return np.unpackbits(np.asarray(bitmap, dtype=np.uint8), bitorder="little")[:n].astype(bool)


# ---------------------------------------------------------------------------
# Host-side column container
# ---------------------------------------------------------------------------

@dataclass
class Column:
    name: str
    data: np.ndarray                      # int8/16/32/64
    valid: np.ndarray | None = None       # bool, None = all valid
    scale: int = 0                        # fixed-point decimal digits (metadata)

    @property
    def type(self) -> int:
        return TYPE_OF_DTYPE[self.data.dtype]

    def bitmap(self) -> np.ndarray | None:
        return None if self.valid is None else pack_validity(self.valid)


@dataclass
class Table:
    cols: list = field(default_factory=list)

    @property
    def nrows(self) -> int:
        return len(self.cols[0].data) if self.cols else 0

    def index(self, name: str) -> int:
        for i, c in enumerate(self.cols):
            if c.name == name:
                return i
        raise KeyError(name)

    def __getitem__(self, name: str) -> Column:
        return self.cols[self.index(name)]


# ---------------------------------------------------------------------------
# Workload recipes.  Column ids within a seed follow the schema order below.
# ---------------------------------------------------------------------------

DATE_DAYS = 2556          # shipdate / fact date domain [0, 2556)
DIM_DATE_DAYS = 2406      # dim date domain [0, 2406)
PRICE_LO, PRICE_HI = 90_000, 10_500_000   # cents (scale 2)


def fact_c1(n: int = 1_000_000, start: int = 0, seed: int = 1,
            null_permille: int = 0) -> Table:
    """Lineitem-like fact: qty, price (cents), disc (percent), shipdate, flag, status."""
    spec = [("qty", 0, 1, 50, np.int64, 0), ("price", 1, PRICE_LO, PRICE_HI, np.int64, 2),
            ("disc", 2, 0, 10, np.int64, 2), ("shipdate", 3, 0, DATE_DAYS - 1, np.int32, 0),
            ("flag", 4, 0, 2, np.int8, 0), ("status", 5, 0, 1, np.int8, 0)]
    t = Table()
    for name, c, lo, hi, dt, sc in spec:
        v = uniform(seed, c, start, n, lo, hi, dt)
        val = validity(seed, c, start, n, null_permille) if null_permille else None
        t.cols.append(Column(name, v, val, sc))
    return t


def fact_c2(n: int = 60_000_000, nkeys: int = 15_000_000, start: int = 0, seed: int = 2,
            null_permille: int = 0) -> Table:
    """Fact for the join workload: fkey U[1,nkeys], price, disc, date."""
    spec = [("fkey", 0, 1, nkeys, np.int64, 0), ("price", 1, PRICE_LO, PRICE_HI, np.int64, 2),
            ("disc", 2, 0, 10, np.int64, 2), ("date", 3, 0, DATE_DAYS - 1, np.int32, 0)]
    t = Table()
    for name, c, lo, hi, dt, sc in spec:
        v = uniform(seed, c, start, n, lo, hi, dt)
        val = validity(seed, c, start, n, null_permille) if null_permille else None
        t.cols.append(Column(name, v, val, sc))
    return t


def dim_c2(n: int = 15_000_000, start: int = 0, seed: int = 2, ckeys: int | None = None,
           null_permille: int = 0) -> Table:
    """Dimension: pkey = a permutation of 1..n, date U[0,2406), ckey U[1,n/10]."""
    ckeys = ckeys if ckeys is not None else max(1, n // 10)
    pkey = permutation(seed, 16, start, min(n, n - start), n) + 1
    t = Table()
    t.cols.append(Column("pkey", pkey.astype(np.int64), None, 0))
    t.cols.append(Column("date", uniform(seed, 17, start, len(pkey), 0, DIM_DATE_DAYS - 1, np.int32),
                         validity(seed, 17, start, len(pkey), null_permille) if null_permille else None, 0))
    t.cols.append(Column("ckey", uniform(seed, 18, start, len(pkey), 1, ckeys, np.int64), None, 0))
    return t


def batch_c3(n: int = 60_000_000, nkeys: int = 15_000_000, start: int = 0, seed: int = 3,
             null_permille: int = 0) -> Table:
    """Exchange batch: Zipf (s = 0.5) int64 key, int64, int32, int8."""
    t = Table()
    t.cols.append(Column("key", zipf(seed, 0, start, n, nkeys),
                         validity(seed, 0, start, n, null_permille) if null_permille else None))
    spec = [("v64", 1, PRICE_LO, PRICE_HI, np.int64), ("v32", 2, 0, DATE_DAYS - 1, np.int32),
            ("v8", 3, 0, 2, np.int8)]
    for name, c, lo, hi, dt in spec:
        t.cols.append(Column(name, uniform(seed, c, start, n, lo, hi, dt),
                             validity(seed, c, start, n, null_permille) if null_permille else None))
    return t


# Serving tables: the join fact with the 1M-row fact's columns, 10x the keys --

C5_FACT_ROWS, C5_DIM_ROWS = 600_000_000, 150_000_000


def fact_c5(n: int = C5_FACT_ROWS, nkeys: int = C5_DIM_ROWS, start: int = 0, seed: int = 5) -> Table:
    """Resident fact: fkey U[1,nkeys], qty, price, disc (int64), date int32, flag, status int8."""
    spec = [("fkey", 0, 1, nkeys, np.int64, 0), ("qty", 1, 1, 50, np.int64, 0),
            ("price", 2, PRICE_LO, PRICE_HI, np.int64, 2), ("disc", 3, 0, 10, np.int64, 2),
            ("date", 4, 0, DATE_DAYS - 1, np.int32, 0), ("flag", 5, 0, 2, np.int8, 0),
            ("status", 6, 0, 1, np.int8, 0)]
    t = Table()
    for name, c, lo, hi, dt, sc in spec:
        t.cols.append(Column(name, uniform(seed, c, start, n, lo, hi, dt), None, sc))
    return t


def dim_c5(n: int = C5_DIM_ROWS, start: int = 0, seed: int = 5) -> Table:
    """Resident dimension: the join dimension's recipe at the serving scale."""
    return dim_c2(n, start=start, seed=seed, ckeys=max(1, n // 10))


# Config-4 fragments -------------------------------------------------------

FRAG_ROWS_LO, FRAG_ROWS_HI = 1_000, 4_000_000
FRAG_CARD_LO, FRAG_CARD_HI = 2, 65_536


def _log_uniform_int(seed: int, col: int, nfrag: int, lo: int, hi: int) -> np.ndarray:
    """floor(lo * (hi/lo)**u) with u = j / 2**32, j uniform on [0, 2**32).

    Evaluated on the host only (the fragment table is passed to the device), in
    IEEE double through the C library's correctly rounded pow.
    """
    j = uniform(seed, col, 0, nfrag, 0, (1 << 32) - 1, np.int64)
    ratio = hi / lo
    out = np.empty(nfrag, dtype=np.int64)
    for f in range(nfrag):
        u = int(j[f]) / 4294967296.0
        out[f] = min(hi, max(lo, int(math.floor(lo * ratio ** u))))
    return out


@dataclass
class FragmentSpec:
    rows: np.ndarray     # int64[nf]
    card: np.ndarray     # int64[nf]
    bound: np.ndarray    # int64[nf]  keep shipdate <= bound

    @property
    def nfrag(self) -> int:
        return len(self.rows)


def fragments_c4(nfrag: int = 4096, seed: int = 4) -> FragmentSpec:
    rows = _log_uniform_int(seed, 100, nfrag, FRAG_ROWS_LO, FRAG_ROWS_HI)
    card = _log_uniform_int(seed, 101, nfrag, FRAG_CARD_LO, FRAG_CARD_HI)
    bound = uniform(seed, 102, 0, nfrag, 0, DATE_DAYS - 1, np.int64)
    return FragmentSpec(rows, card, bound)


def fragment_seed(f: int, seed: int = 4) -> int:
    return (seed << 32) | f


def fragment_c4(f: int, rows: int, card: int, start: int = 0, n: int | None = None,
                seed: int = 4) -> Table:
    """Rows start..start+n-1 of fragment f: qty, price, disc, shipdate, gkey U[0,card)."""
    n = rows - start if n is None else n
    s = fragment_seed(f, seed)
    spec = [("qty", 0, 1, 50, np.int64), ("price", 1, PRICE_LO, PRICE_HI, np.int64),
            ("disc", 2, 0, 10, np.int64), ("shipdate", 3, 0, DATE_DAYS - 1, np.int32),
            ("gkey", 4, 0, card - 1, np.int32)]
    t = Table()
    for name, c, lo, hi, dt in spec:
        t.cols.append(Column(name, uniform(s, c, start, n, lo, hi, dt)))
    return t
