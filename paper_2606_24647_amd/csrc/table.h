// Hash-table building blocks shared by the join, group-by and pipeline
// kernels: key encodings, table layouts, aggregate plans and the compaction of
// a table into an output batch.
//
// Every table is open addressing with linear probing over `cap` slots in HBM,
// stored as separate arrays:
//   keys[s]  one 64-bit word per slot, EMPTY (all ones) when unused.  Probing
//            touches only this array: 16 keys per 128-byte cache line, and at
//            the sizes used here it stays resident in the Infinity Cache.
//   meta[s]  (join tables) count << 32 | row: the number of build rows with the
//            key, and the build row of a unique key or the start of the key's
//            run of rows once duplicates were found.
//   acc[s*aw .. s*aw+aw)  accumulator words, touched only when a row lands in
//            the slot (group-by), i.e. once per aggregated row.
//   kv[2s], kv[2s+1]  (join tables) keys[s] and meta[s] side by side, copied
//            once the index is complete: the pair probe reads a slot's key
//            and its match count and row with one 16-byte load, where the two
//            arrays cost two random cache lines per match.
// Slot index = floor(fmix64(key ^ kTableSeed) * cap / 2^64): a different seed
// from the partitioning hash, so a table built over one partition still spreads
// over all of its slots.  Slots past the hashed range (index cap_alloc and
// cap_alloc + 1) hold the key whose encoding equals EMPTY and the NULL key,
// where such keys can occur.
#pragma once

#include "common.h"

namespace gq {

constexpr uint64_t kEmpty = ~0ull;
constexpr uint64_t kTableSeed = 0x5bd1e9955bd1e995ull;

__host__ __device__ __forceinline__ uint64_t slot_of(uint64_t key, uint64_t cap) {
#ifdef __HIP_DEVICE_COMPILE__
  return __umul64hi(fmix64(key ^ kTableSeed), cap);
#else
  return (uint64_t)(((unsigned __int128)fmix64(key ^ kTableSeed) * cap) >> 64);
#endif
}

// ---------------------------------------------------------------------------
// Group keys
// ---------------------------------------------------------------------------
// Packed mode: key columns are packed into one 64-bit word, first column most
// significant; each field is the value with its sign bit flipped (so unsigned
// order is signed order), preceded by a validity bit for nullable columns (0 =
// NULL, field value 0, which orders NULL first).  At most 63 bits are used, so
// a packed key never equals EMPTY.  Raw mode: one int64 column, key = value;
// the value EMPTY (-1) and NULL go to the two extra slots.
enum { KEY_PACKED = 0, KEY_RAW64 = 1 };

struct KeyPlan {
  int32_t mode;
  int32_t nk;
  int32_t shift[GQ_MAX_KEYS];
  int32_t bits[GQ_MAX_KEYS];
  int32_t nullable[GQ_MAX_KEYS];
  DCol cols[GQ_MAX_KEYS];
};

// Decode key column j of a packed key (value, valid).
template <class KP>
__device__ __forceinline__ int64_t decode_field(const KP& kp, uint64_t key, int j, bool* valid) {
  const int w = kp.bits[j];
  const uint64_t mask = (w == 64) ? ~0ull : ((1ull << w) - 1);
  uint64_t f = key >> kp.shift[j];
  *valid = kp.nullable[j] ? ((f >> w) & 1ull) != 0 : true;
  uint64_t x = (f & mask) ^ (1ull << (w - 1));
  int64_t s = (int64_t)(x << (64 - w)) >> (64 - w);  // sign-extend w bits
  return *valid ? s : 0;
}

// ---------------------------------------------------------------------------
// Aggregates
// ---------------------------------------------------------------------------
// Accumulator words of a group: word 0 the weighted row count (COUNT(*), and
// the occupancy of the extra slots), then one word per aggregate value and one
// more per aggregate whose input can be NULL (its non-NULL count, which decides
// the validity of SUM/MIN/MAX).
constexpr int kMaxVals = 8;  // distinct value columns referenced by aggregates
constexpr int kMaxAcc = 1 + 2 * GQ_MAX_AGGS;

struct DFactor {
  int32_t kind;
  int32_t v;  // index into the value-column list
  int64_t k;
};

struct DAgg {
  int32_t op;
  int32_t nf;
  int32_t word;   // accumulator word (COUNT(*): 0)
  int32_t cword;  // non-NULL count word, -1 if the input cannot be NULL
  DFactor f[3];
};

// Word update kinds, for initialising and merging accumulators.
enum { WOP_ADD = 0, WOP_MIN = 1, WOP_MAX = 2 };

struct AggPlan {
  int32_t naggs;
  int32_t nvals;
  int32_t nacc;  // accumulator words per group
  int32_t pad;
  DAgg aggs[GQ_MAX_AGGS];
  DCol vals[kMaxVals];
  int8_t wop[kMaxAcc];
};

__host__ __device__ __forceinline__ uint64_t word_identity(int8_t wop) {
  return (uint64_t)(wop == WOP_MIN ? INT64_MAX : wop == WOP_MAX ? INT64_MIN : 0);
}

struct GlobalAtomics {
  static __device__ __forceinline__ void add(uint64_t* p, uint64_t v) {
    atomicAdd((unsigned long long*)p, (unsigned long long)v);
  }
  static __device__ __forceinline__ void min(uint64_t* p, int64_t v) { atomicMin((long long*)p, (long long)v); }
  static __device__ __forceinline__ void max(uint64_t* p, int64_t v) { atomicMax((long long*)p, (long long)v); }
};

// LDS accumulators (same instructions, LDS address space after inlining).
using SharedAtomics = GlobalAtomics;

// ---------------------------------------------------------------------------
// Probing
// ---------------------------------------------------------------------------
// A key word only ever changes once, from EMPTY to its key, so a stale plain
// read can only show EMPTY, and the CAS that follows returns the true value.
// Returns the slot of `key` (inserting it), or -1 when all cap slots are taken.
// `start` is slot_of(key, cap) and `first` the key word read there.
__device__ __forceinline__ int64_t find_insert_from(uint64_t* keys, uint64_t cap, uint64_t key, uint64_t start,
                                                    uint64_t first, bool* inserted) {
  uint64_t s = start;
  uint64_t k = first;
  *inserted = false;
  for (uint64_t probes = 0; probes < cap; ++probes) {
    if (k == key) return (int64_t)s;
    if (k == kEmpty) {
      const uint64_t prev =
          atomicCAS((unsigned long long*)&keys[s], (unsigned long long)kEmpty, (unsigned long long)key);
      if (prev == kEmpty) {
        *inserted = true;
        return (int64_t)s;
      }
      if (prev == key) return (int64_t)s;
    }
    if (++s == cap) s = 0;
    k = keys[s];
  }
  return -1;
}

__device__ __forceinline__ int64_t find_insert(uint64_t* keys, uint64_t cap, uint64_t key, bool* inserted) {
  const uint64_t s = slot_of(key, cap);
  return find_insert_from(keys, cap, key, s, keys[s], inserted);
}

// Read-only lookup continuing from a first probe; -1 when absent.
__device__ __forceinline__ int64_t find_from(const uint64_t* keys, uint64_t cap, uint64_t key, uint64_t start,
                                             uint64_t first) {
  uint64_t s = start;
  uint64_t k = first;
  for (uint64_t probes = 0; probes < cap; ++probes) {
    if (k == key) return (int64_t)s;
    if (k == kEmpty) return -1;
    if (++s == cap) s = 0;
    k = keys[s];
  }
  return -1;
}

__device__ __forceinline__ int64_t find(const uint64_t* keys, uint64_t cap, uint64_t key) {
  if (cap == 0) return -1;
  const uint64_t s = slot_of(key, cap);
  return find_from(keys, cap, key, s, keys[s]);
}

// ---------------------------------------------------------------------------
// Join table
// ---------------------------------------------------------------------------
struct JoinHdr {
  uint64_t cap;      // hashed slots in use (computed on the device)
  int64_t nrows;     // build rows inserted
  int32_t has_dups;  // some key occurs more than once
  int32_t full;      // insertion failed for lack of space
  int64_t nlong;     // runs too long for one thread to sort (duplicates only)
  int64_t pad[4];
};

__device__ __forceinline__ uint32_t meta_count(uint64_t m) { return (uint32_t)(m >> 32); }
__device__ __forceinline__ uint32_t meta_row(uint64_t m) { return (uint32_t)(m & 0xffffffffu); }

// ---------------------------------------------------------------------------
// Table -> output batch compaction
// ---------------------------------------------------------------------------
struct CompactArgs {
  const uint64_t* keys;    // hashed slots, then the extra slots
  const uint64_t* acc;     // aw words per slot
  const uint64_t* d_cap;   // device cap (join tables); NULL = use cap
  uint64_t cap;
  uint64_t cap_alloc;      // slots allocated in the hashed range (extras follow)
  int32_t aw;              // accumulator words per slot
  int32_t key_kind;        // 0 packed, 1 raw64, 2 join key (raw int64)
  int32_t extra;           // number of extra slots to visit (1 or 2)
  int32_t naggs;
  int32_t global_agg;      // no key columns: one row even when nothing is occupied
  int32_t extras_first;    // visit the extra slots first, NULL key first (sorted output)
  KeyPlan kp;
  DAgg aggs[GQ_MAX_AGGS];
  OCol out[GQ_MAX_KEYS + GQ_MAX_AGGS];
  OCol sortkey;            // if data != NULL: an unsigned sort key per output row
  int64_t out_cap;
  int64_t ntiles;
  uint32_t* ticket;
  uint64_t* status;
  int64_t* d_count;
  int32_t* dev_status;
  const int64_t* gate;     // if set and *gate == 0: write nothing (d_count stays 0)
};

}  // namespace gq

// Host-side join table object (the opaque gq_join_table of the C-ABI).
struct gq_join_table {
  gq_ctx* ctx = nullptr;
  void* mem = nullptr;        // one allocation from the context allocator
  size_t bytes = 0;
  void* imem = nullptr;       // partitioned tables: the probe index, allocated on first use
  size_t ibytes = 0;
  gq::JoinHdr* hdr = nullptr;
  uint64_t* keys = nullptr;   // cap_alloc + 1 words; slot cap_alloc holds the key EMPTY
  uint64_t* meta = nullptr;   // cap_alloc + 1 words
  uint64_t* kv = nullptr;     // cap_alloc + 1 pairs (keys[s], meta[s]), written once the index is complete
  uint64_t* acc = nullptr;    // (cap_alloc + 1) * acc_slots words, or NULL
  int32_t* rows = nullptr;    // build rows grouped by key once duplicates were found
  uint32_t* aux = nullptr;    // cap_alloc + 1 words: fill cursors, then the long-run list
  int32_t* tmp = nullptr;     // nrows words, merge-sort buffer for long runs
  uint64_t cap_alloc = 0;
  int32_t acc_slots = 0;
  int64_t build_rows = 0;
  int32_t key_type = GQ_I64;
  int32_t nkeys = 1;          // key columns; above 1 the table holds their packed word
  int32_t key_types[GQ_MAX_KEYS] = {GQ_I64, GQ_I64, GQ_I64, GQ_I64};  // the build side's key types
  int32_t device = 0;
  bool acc_dirty = false;     // accumulators used by an earlier group-join
  // Probe index (keys/meta/rows): built by gq_join_build for small build
  // inputs, else on first use from the partitioned rows below.
  bool index_built = false;
  int32_t lf_milli = 500;     // load factor of the index, times 1000
  // Partitioned build side (large build inputs): kept rows as (region hash,
  // row id) pairs of 64-bit words, grouped by region (top rj_pbits bits of
  // the region hash), region r in pairs [rj_off[r], rj_off[r + 1]).  NULL when
  // the build input is small.
  int32_t rj_pbits = 0;
  uint64_t* rj_kr = nullptr;
  int64_t* rj_off = nullptr;
  // Recorded on the build stream once the build work is enqueued; every call
  // that reads the table waits for it on its own stream.
  hipEvent_t ready = nullptr;
};
