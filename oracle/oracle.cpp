// Plain, slow CPU oracle for the columnar operator path.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no code,
// header, table or constant with the GPU library: every definition below is
// written out here on its own.
//
// What it follows.  The paper ("Accelerating Presto with GPUs") names the
// operators but defines none of them: filter and projection (Section 3.2,
// CudfFilterProject), equi-join (Section 3.1 lists Join among the relational
// operators; Section 3.2 states cuDF covers all standard SQL operations),
// hash aggregation (Section 3.2, HashAggregation), and partitioned output into
// per-destination packed buffers (Section 3.3).  Their meaning is therefore
// SQL's, as Presto implements it.  Where SQL leaves a choice open (output order,
// the partitioning hash), the reading chosen is stated at each function.
//
// Style: std containers, sort- and ordered-map-based algorithms, no hashing
// structure of any kind, no blocking or reordering.  Every loop visits rows in
// input order.
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

namespace {

// Column type codes (Arrow fixed-width signed integers).
enum { T_I8 = 1, T_I16 = 2, T_I32 = 3, T_I64 = 4 };
// Predicate kinds.
enum { P_RANGE = 1, P_NE = 2 };
// Factor kinds of an aggregate input expression.
enum { F_COL = 1, F_K_MINUS_COL = 2, F_K_PLUS_COL = 3, F_CONST = 4 };
// Aggregate kinds.
enum { A_SUM = 1, A_COUNT_STAR = 2, A_COUNT = 3, A_MIN = 4, A_MAX = 5 };

}  // namespace

extern "C" {

struct orc_col {
  int32_t type;
  int32_t pad;
  int64_t length;
  const void* data;
  const uint8_t* validity;  // Arrow LSB-first bitmap, 1 = valid; NULL = all valid
};

struct orc_pred {
  int32_t col;
  int32_t op;
  int64_t lo;
  int64_t hi;
};

struct orc_factor {
  int32_t kind;
  int32_t col;
  int64_t k;
};

struct orc_agg {
  int32_t op;
  int32_t nf;
  orc_factor f[3];
};

}  // extern "C"

namespace {

// Value of row i of a column, sign-extended to int64.
int64_t value_at(const orc_col& c, int64_t i) {
  switch (c.type) {
    case T_I8: return (int64_t)((const int8_t*)c.data)[i];
    case T_I16: return (int64_t)((const int16_t*)c.data)[i];
    case T_I32: return (int64_t)((const int32_t*)c.data)[i];
    default: return ((const int64_t*)c.data)[i];
  }
}

// Arrow validity: bit (i mod 8) of byte i/8, least significant bit first.
bool valid_at(const orc_col& c, int64_t i) {
  if (c.validity == nullptr) return true;
  return ((c.validity[i / 8] >> (i % 8)) & 1) != 0;
}

// SQL WHERE over a conjunction: a row is kept only when every predicate is
// TRUE.  A comparison involving NULL is UNKNOWN, so the row is dropped.
bool row_passes(const orc_col* cols, const orc_pred* p, int np, int64_t i) {
  for (int j = 0; j < np; ++j) {
    const orc_col& c = cols[p[j].col];
    if (!valid_at(c, i)) return false;
    int64_t v = value_at(c, i);
    if (p[j].op == P_RANGE) {
      if (v < p[j].lo || v > p[j].hi) return false;
    } else {  // P_NE
      if (v == p[j].lo) return false;
    }
  }
  return true;
}

// MurmurHash3's 64-bit finaliser (Appleby, public domain): three xor-shifts by
// 33 separated by multiplications with two fixed odd constants.
uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

// Row hash over key columns: h = seed, then for each key column in order
// h = fmix64(h xor x) with x the sign-extended value (0 for NULL).
uint64_t row_hash(const orc_col* cols, const int32_t* keys, int nk, uint64_t seed, int64_t i) {
  uint64_t h = seed;
  for (int j = 0; j < nk; ++j) {
    const orc_col& c = cols[keys[j]];
    uint64_t x = valid_at(c, i) ? (uint64_t)value_at(c, i) : 0;
    h = fmix64(h ^ x);
  }
  return h;
}

// Partition of a hash: floor(h * P / 2^64) (multiply-shift range reduction).
uint64_t partition_of(uint64_t h, uint64_t P) {
  return (uint64_t)(((unsigned __int128)h * P) >> 64);
}

// Aggregate input expression: product of its factors, int64 arithmetic modulo
// 2^64.  NULL if any referenced column is NULL.  `exact` receives the same
// product in 128-bit arithmetic and `ovf` is set when it leaves int64.
bool eval_expr(const orc_col* cols, const orc_agg& a, int64_t i, uint64_t* wrapped,
               __int128* exact, bool* ovf) {
  uint64_t w = 1;
  __int128 e = 1;
  for (int j = 0; j < a.nf; ++j) {
    const orc_factor& f = a.f[j];
    int64_t x = 0;
    if (f.kind != F_CONST) {
      const orc_col& c = cols[f.col];
      if (!valid_at(c, i)) return false;
      x = value_at(c, i);
    }
    uint64_t fw;
    __int128 fe;
    switch (f.kind) {
      case F_COL: fw = (uint64_t)x; fe = x; break;
      case F_K_MINUS_COL: fw = (uint64_t)f.k - (uint64_t)x; fe = (__int128)f.k - x; break;
      case F_K_PLUS_COL: fw = (uint64_t)f.k + (uint64_t)x; fe = (__int128)f.k + x; break;
      default: fw = (uint64_t)f.k; fe = f.k; break;
    }
    w *= fw;
    __int128 prod;
    if (__builtin_mul_overflow(e, fe, &prod)) *ovf = true;
    e = prod;
  }
  if (e > (__int128)INT64_MAX || e < (__int128)INT64_MIN) *ovf = true;
  *wrapped = w;
  *exact = e;
  return true;
}

// Per-group accumulator for one aggregate.
struct Acc {
  uint64_t sum = 0;       // wrapping int64 sum
  __int128 exact = 0;     // the same sum in 128-bit arithmetic
  int64_t count = 0;      // non-null inputs (or rows, for COUNT(*))
  int64_t minv = INT64_MAX;
  int64_t maxv = INT64_MIN;
};

// A group key: one (is_valid, value) pair per key column.  Comparing these
// lexicographically orders NULL before every value, then values ascending.
typedef std::vector<std::pair<int, int64_t>> GroupKey;

struct GroupResult {
  int nk = 0, na = 0;
  std::vector<int64_t> keyval;   // nrows * nk
  std::vector<uint8_t> keyok;    // nrows * nk
  std::vector<int64_t> aggval;   // nrows * na
  std::vector<uint8_t> aggok;    // nrows * na
  int64_t nrows = 0;
  bool overflow = false;
};

struct PairResult {
  std::vector<int64_t> probe, build;
};

typedef std::vector<int64_t> KeyTuple;

// Key tuple of row i; false if any component is NULL (NULL never joins).
bool key_tuple(const orc_col* cols, const int32_t* keys, int nk, int64_t i, KeyTuple* out) {
  out->clear();
  for (int j = 0; j < nk; ++j) {
    const orc_col& c = cols[keys[j]];
    if (!valid_at(c, i)) return false;
    out->push_back(value_at(c, i));
  }
  return true;
}

}  // namespace

extern "C" {

uint64_t orc_fmix64(uint64_t k) { return fmix64(k); }

uint64_t orc_partition_of(uint64_t h, uint64_t P) { return partition_of(h, P); }

void orc_hash_rows(const orc_col* cols, const int32_t* keys, int nk, uint64_t seed, int64_t n,
                   uint64_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = row_hash(cols, keys, nk, seed, i);
}

// Filter: the kept row ids in input order (stable).  Returns their number.
int64_t orc_filter(const orc_col* cols, int64_t n, const orc_pred* p, int np, int64_t* out_rows) {
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    if (row_passes(cols, p, np, i)) out_rows[k++] = i;
  return k;
}

// Hash partition: counting sort of rows by partition id, stable.  out_perm[r]
// is the input row placed at output position r; out_offsets has P+1 entries,
// partition q occupying [out_offsets[q], out_offsets[q+1]).
void orc_partition(const orc_col* cols, int64_t n, const int32_t* keys, int nk, int64_t P,
                   uint64_t seed, int64_t* out_perm, int64_t* out_offsets) {
  std::vector<int64_t> part(n);
  std::vector<int64_t> count(P, 0);
  for (int64_t i = 0; i < n; ++i) {
    part[i] = (int64_t)partition_of(row_hash(cols, keys, nk, seed, i), (uint64_t)P);
    count[part[i]] += 1;
  }
  out_offsets[0] = 0;
  for (int64_t q = 0; q < P; ++q) out_offsets[q + 1] = out_offsets[q] + count[q];
  std::vector<int64_t> next(out_offsets, out_offsets + P);
  for (int64_t i = 0; i < n; ++i) out_perm[next[part[i]]++] = i;
}

// Inner equi-join.  Build rows that pass their predicates and have no NULL key
// go into an ordered multimap (equal keys keep insertion order, hence ascending
// build row).  Probe rows are visited in ascending order; each emits one pair
// per matching build row.  Output order: (probe row, build row) ascending.
void* orc_join(const orc_col* bcols, int64_t nb, const int32_t* bkeys, int nk, const orc_pred* bp,
               int nbp, const orc_col* pcols, int64_t npr, const int32_t* pkeys, const orc_pred* pp,
               int npp) {
  std::multimap<KeyTuple, int64_t> table;
  KeyTuple k;
  for (int64_t j = 0; j < nb; ++j) {
    if (!row_passes(bcols, bp, nbp, j)) continue;
    if (!key_tuple(bcols, bkeys, nk, j, &k)) continue;
    table.insert(std::make_pair(k, j));
  }
  PairResult* r = new PairResult;
  for (int64_t i = 0; i < npr; ++i) {
    if (!row_passes(pcols, pp, npp, i)) continue;
    if (!key_tuple(pcols, pkeys, nk, i, &k)) continue;
    auto range = table.equal_range(k);
    for (auto it = range.first; it != range.second; ++it) {
      r->probe.push_back(i);
      r->build.push_back(it->second);
    }
  }
  return r;
}

int64_t orc_pairs_count(void* h) { return (int64_t)((PairResult*)h)->probe.size(); }

void orc_pairs_copy(void* h, int64_t* probe, int64_t* build) {
  PairResult* r = (PairResult*)h;
  if (!r->probe.empty()) {
    std::memcpy(probe, r->probe.data(), r->probe.size() * sizeof(int64_t));
    std::memcpy(build, r->build.data(), r->build.size() * sizeof(int64_t));
  }
}

void orc_pairs_free(void* h) { delete (PairResult*)h; }

// Hash aggregation in SQL GROUP BY semantics over the rows that pass the
// predicates.  Groups are kept in an ordered map, so the result comes out in
// canonical order: keys ascending, NULL first in each key column.
//   SUM(e)    wrapping int64 sum of non-NULL e; NULL if there is none
//   COUNT(*)  rows in the group
//   COUNT(e)  non-NULL e
//   MIN/MAX   over non-NULL e; NULL if there is none
// With no key columns the input forms one group, present even when empty.
void* orc_groupby(const orc_col* cols, int64_t n, const int32_t* keys, int nk, const orc_pred* p,
                  int np, const orc_agg* aggs, int na) {
  std::map<GroupKey, std::vector<Acc>> groups;
  GroupResult* res = new GroupResult;
  res->nk = nk;
  res->na = na;
  if (nk == 0) groups[GroupKey()] = std::vector<Acc>(na);
  GroupKey key;
  for (int64_t i = 0; i < n; ++i) {
    if (!row_passes(cols, p, np, i)) continue;
    key.clear();
    for (int j = 0; j < nk; ++j) {
      const orc_col& c = cols[keys[j]];
      if (valid_at(c, i))
        key.push_back(std::make_pair(1, value_at(c, i)));
      else
        key.push_back(std::make_pair(0, (int64_t)0));
    }
    auto it = groups.find(key);
    if (it == groups.end()) it = groups.insert(std::make_pair(key, std::vector<Acc>(na))).first;
    std::vector<Acc>& acc = it->second;
    for (int a = 0; a < na; ++a) {
      if (aggs[a].op == A_COUNT_STAR) {
        acc[a].count += 1;
        continue;
      }
      uint64_t w;
      __int128 e;
      bool ovf = false;
      if (!eval_expr(cols, aggs[a], i, &w, &e, &ovf)) continue;
      if (ovf) res->overflow = true;
      acc[a].count += 1;
      acc[a].sum += w;
      acc[a].exact += e;
      int64_t v = (int64_t)w;
      if (v < acc[a].minv) acc[a].minv = v;
      if (v > acc[a].maxv) acc[a].maxv = v;
    }
  }
  for (auto& g : groups) {
    for (int j = 0; j < nk; ++j) {
      res->keyok.push_back((uint8_t)g.first[j].first);
      res->keyval.push_back(g.first[j].second);
    }
    for (int a = 0; a < na; ++a) {
      const Acc& acc = g.second[a];
      int64_t v = 0;
      uint8_t ok = 1;
      switch (aggs[a].op) {
        case A_SUM:
          v = (int64_t)acc.sum;
          ok = acc.count > 0;
          if (acc.exact > (__int128)INT64_MAX || acc.exact < (__int128)INT64_MIN) res->overflow = true;
          break;
        case A_COUNT_STAR:
        case A_COUNT: v = acc.count; break;
        case A_MIN: v = acc.count > 0 ? acc.minv : 0; ok = acc.count > 0; break;
        default: v = acc.count > 0 ? acc.maxv : 0; ok = acc.count > 0; break;
      }
      if (!ok) v = 0;
      res->aggval.push_back(v);
      res->aggok.push_back(ok);
    }
    res->nrows += 1;
  }
  return res;
}

int64_t orc_groups_rows(void* h) { return ((GroupResult*)h)->nrows; }

int orc_groups_overflow(void* h) { return ((GroupResult*)h)->overflow ? 1 : 0; }

// Column j of the result: key columns first (j < nk), then aggregates.
void orc_groups_copy(void* h, int j, int64_t* values, uint8_t* valid) {
  GroupResult* r = (GroupResult*)h;
  for (int64_t g = 0; g < r->nrows; ++g) {
    if (j < r->nk) {
      values[g] = r->keyval[g * r->nk + j];
      valid[g] = r->keyok[g * r->nk + j];
    } else {
      int a = j - r->nk;
      values[g] = r->aggval[g * r->na + a];
      valid[g] = r->aggok[g * r->na + a];
    }
  }
}

void orc_groups_free(void* h) { delete (GroupResult*)h; }

}  // extern "C"
