// Hash-table building blocks shared by the join, group-by and pipeline
// kernels: key encodings, slot layouts, aggregate plans and the compaction of a
// table into an output batch.
//
// Tables are open-addressing with linear probing over `cap` slots in HBM; a
// slot's first 8-byte word is its key, EMPTY (all ones) when unused.  Slot
// index = floor(fmix64(key ^ kTableSeed) * cap / 2^64): a different seed from
// the partitioning hash, so a table built over one partition still spreads over
// all of its slots.  Two extra slots after the hashed range hold the key whose
// encoding equals EMPTY and the NULL key, where such keys can occur.
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

// Encode one row's key; *special = 0 (hashed), 1 (EMPTY-valued raw key) or
// 2 (NULL raw key).
__device__ __forceinline__ uint64_t encode_key(const KeyPlan& kp, const int64_t* v, uint32_t validmask,
                                               int* special) {
  *special = 0;
  if (kp.mode == KEY_RAW64) {
    if (!(validmask & 1u)) {
      *special = 2;
      return 0;
    }
    uint64_t k = (uint64_t)v[0];
    if (k == kEmpty) *special = 1;
    return k;
  }
  uint64_t key = 0;
  for (int j = 0; j < kp.nk; ++j) {
    const int w = kp.bits[j];
    const uint64_t mask = (w == 64) ? ~0ull : ((1ull << w) - 1);
    uint64_t f = ((uint64_t)v[j] ^ (1ull << (w - 1))) & mask;
    if (kp.nullable[j]) f = ((validmask >> j) & 1u) ? (f | (1ull << w)) : 0ull;
    key |= f << kp.shift[j];
  }
  return key;
}

// Decode key column j of a packed key (value, valid).
__device__ __forceinline__ int64_t decode_field(const KeyPlan& kp, uint64_t key, int j, bool* valid) {
  const int w = kp.bits[j];
  const uint64_t mask = (w == 64) ? ~0ull : ((1ull << w) - 1);
  uint64_t f = key >> kp.shift[j];
  *valid = kp.nullable[j] ? ((f >> w) & 1ull) != 0 : true;
  uint64_t x = (f & mask) ^ (1ull << (w - 1));
  // sign-extend w bits
  int64_t s = (int64_t)(x << (64 - w)) >> (64 - w);
  return *valid ? s : 0;
}

// ---------------------------------------------------------------------------
// Aggregates
// ---------------------------------------------------------------------------
// Accumulator words of a group slot: word 0 key, word 1 the weighted row count
// (COUNT(*), also the occupancy of the extra slots), then one word per
// aggregate value and one more per aggregate whose input can be NULL (its
// non-NULL count, which decides the validity of SUM/MIN/MAX).
constexpr int kMaxVals = 8;  // distinct value columns referenced by aggregates

struct DFactor {
  int32_t kind;
  int32_t v;  // index into the value-column list
  int64_t k;
};

struct DAgg {
  int32_t op;
  int32_t nf;
  int32_t word;   // value word (COUNT(*): 1)
  int32_t cword;  // non-NULL count word, -1 if the input cannot be NULL
  DFactor f[3];
};

struct AggPlan {
  int32_t naggs;
  int32_t nvals;
  int32_t nwords;  // words per slot including the key word
  int32_t pad;
  DAgg aggs[GQ_MAX_AGGS];
  DCol vals[kMaxVals];
  int8_t wop[2 + 2 * GQ_MAX_AGGS];  // update kind of each word (index 0 unused)
};

// Word update kinds, for merging one table's accumulators into another.
enum { WOP_ADD = 0, WOP_MIN = 1, WOP_MAX = 2 };

__host__ __device__ __forceinline__ int64_t agg_init_word(int op) {
  return op == GQ_MIN ? INT64_MAX : op == GQ_MAX ? INT64_MIN : 0;
}

struct GlobalAtomics {
  static __device__ __forceinline__ void add(uint64_t* p, uint64_t v) {
    atomicAdd((unsigned long long*)p, (unsigned long long)v);
  }
  static __device__ __forceinline__ void min(uint64_t* p, int64_t v) { atomicMin((long long*)p, (long long)v); }
  static __device__ __forceinline__ void max(uint64_t* p, int64_t v) { atomicMax((long long*)p, (long long)v); }
};

// LDS accumulators (same instructions, LDS address space).
struct SharedAtomics {
  static __device__ __forceinline__ void add(uint64_t* p, uint64_t v) {
    atomicAdd((unsigned long long*)p, (unsigned long long)v);
  }
  static __device__ __forceinline__ void min(uint64_t* p, int64_t v) { atomicMin((long long*)p, (long long)v); }
  static __device__ __forceinline__ void max(uint64_t* p, int64_t v) { atomicMax((long long*)p, (long long)v); }
};

// Find or insert `key` in a global table with `cap` hashed slots of `stride`
// words; returns the slot's word pointer or nullptr when the table is full.
// A key word only ever changes once, from EMPTY to its key, so a stale plain
// read can only show EMPTY, and the CAS that follows returns the true value.
__device__ __forceinline__ uint64_t* table_find_insert(uint64_t* slots, uint64_t cap, int stride, uint64_t key) {
  uint64_t s = slot_of(key, cap);
  for (uint64_t probes = 0; probes < cap; ++probes) {
    uint64_t* slot = slots + s * stride;
    const uint64_t k = slot[0];
    if (k == key) return slot;
    if (k == kEmpty) {
      uint64_t prev = atomicCAS((unsigned long long*)slot, (unsigned long long)kEmpty, (unsigned long long)key);
      if (prev == kEmpty || prev == key) return slot;
    }
    if (++s == cap) s = 0;
  }
  return nullptr;
}

// Read-only lookup.
__device__ __forceinline__ const uint64_t* table_find(const uint64_t* slots, uint64_t cap, int stride, uint64_t key) {
  if (cap == 0) return nullptr;
  uint64_t s = slot_of(key, cap);
  for (uint64_t probes = 0; probes < cap; ++probes) {
    const uint64_t* slot = slots + s * stride;
    const uint64_t k = slot[0];
    if (k == key) return slot;
    if (k == kEmpty) return nullptr;
    if (++s == cap) s = 0;
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// Join table layout
// ---------------------------------------------------------------------------
// Slot (stride 2 + acc words): word 0 key, word 1 = (row:int32 low, count:int32
// high) where row is the build row of a unique key or the start of the key's
// run in the row array once duplicates were found; then acc words for a fused
// group-by.  Header (device): see JoinHdr.
struct JoinHdr {
  uint64_t cap;         // hashed slots in use (computed on the device)
  int64_t nrows;        // build rows inserted
  int32_t has_dups;     // some key occurs more than once
  int32_t full;         // insertion failed for lack of space
  int64_t pad[5];
};

__device__ __forceinline__ uint32_t slot_count(const uint64_t* slot) { return (uint32_t)(slot[1] >> 32); }
__device__ __forceinline__ uint32_t slot_row(const uint64_t* slot) { return (uint32_t)(slot[1] & 0xffffffffu); }

// ---------------------------------------------------------------------------
// Table -> output batch compaction
// ---------------------------------------------------------------------------
struct CompactArgs {
  const uint64_t* slots;   // hashed slots followed by the two extra slots
  const uint64_t* d_cap;   // device cap (join tables); NULL = use cap
  uint64_t cap;
  uint64_t max_cap;        // slots allocated in the hashed range
  int32_t stride;          // words per slot
  int32_t acc_base;        // word index of the hidden row count
  int32_t key_kind;        // 0 packed, 1 raw64, 2 join key (word 0, raw int64)
  int32_t extra;           // number of extra slots to visit (1 or 2)
  KeyPlan kp;
  int32_t naggs;
  int32_t global_agg;      // no key columns: one row even when nothing is occupied
  DAgg aggs[GQ_MAX_AGGS];  // word/cword relative to acc_base - 1
  OCol out[GQ_MAX_KEYS + GQ_MAX_AGGS];
  int64_t out_cap;
  int64_t ntiles;
  uint32_t* ticket;
  uint64_t* status;
  int64_t* d_count;
  int32_t* dev_status;
};

}  // namespace gq

// Host-side join table object (the opaque gq_join_table of the C-ABI).
struct gq_join_table {
  gq_ctx* ctx = nullptr;
  void* mem = nullptr;      // one allocation from the context allocator
  size_t bytes = 0;
  gq::JoinHdr* hdr = nullptr;
  uint64_t* slots = nullptr;  // (max_cap + 1) * stride words; slot max_cap holds the key EMPTY
  int32_t* rows = nullptr;    // build rows grouped by key once duplicates were found
  uint32_t* aux = nullptr;    // max_cap + 1 words: fill cursors, then the long-run list
  int32_t* tmp = nullptr;     // nrows words, merge-sort buffer for long runs
  uint64_t max_cap = 0;
  int32_t stride = 2;         // words per slot
  int32_t acc_slots = 0;
  int64_t build_rows = 0;
  int32_t key_type = GQ_I64;
  int32_t device = 0;
  bool acc_dirty = false;     // accumulator words used by an earlier group-join
};
