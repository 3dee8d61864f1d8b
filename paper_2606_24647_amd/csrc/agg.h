// Device-side aggregation helpers shared by the group-by, pipeline and
// batched-fragment kernels: predicate evaluation, join lookups with
// read-ahead, group-key encoding, aggregate inputs, and the atomic updates of
// LDS or HBM accumulators.
#pragma once

#include "table.h"

#include <functional>

namespace gq {

struct JoinRef {
  const JoinHdr* hdr;
  const uint64_t* keys;
  const uint64_t* meta;
  uint64_t* acc;
  uint64_t cap_alloc;
  int32_t acc_slots;
  int32_t pad;
  DCol key;  // probe key column
};

struct GbArgs {
  int64_t n;
  int64_t ntiles;
  int32_t npreds;
  int32_t lcap;      // LDS table slots (power of two), LDS strategy only
  DPred preds[GQ_MAX_PREDS];
  DCol pcols[GQ_MAX_PREDS];
  KeyPlan kp;
  AggPlan ap;
  uint64_t* keys;    // HBM group table: cap hashed slots, then 2 extra slots
  uint64_t* acc;     // ap.nacc words per slot
  uint64_t cap;
  JoinRef join;
  int32_t* dev_status;
  int64_t tile_rows;  // batched plans: rows per work item of this fragment
  int32_t nrep;       // LDS strategy: replicas of the HBM table the blocks merge into
  int32_t pad_rep;
  int64_t rep_slots;  // slots per replica (cap + 2)
  int64_t* d_inserted;  // if set: counts the groups inserted into the HBM table (streaming aggregation)
  const int64_t* d_nrows;  // if set: rows at or past *d_nrows (a device count) are not read
};

// Rows of a group-by input: n, or fewer when a device-side count bounds it.
template <class GA>
__device__ __forceinline__ int64_t rows_of(const GA& a) {
  if (!a.d_nrows) return a.n;
  const int64_t d = *a.d_nrows;
  return d < a.n ? d : a.n;
}

template <int ITEMS, class C>
__device__ __forceinline__ void load_col(const C& c, int64_t r0, int64_t n, int64_t (&v)[ITEMS]) {
  if (c.nt) load_items<ITEMS, true>(c, r0, n, v);
  else load_items<ITEMS, false>(c, r0, n, v);
}

// ---------------------------------------------------------------------------
// Per-tile row evaluation shared by the kernels
// ---------------------------------------------------------------------------
template <int ITEMS, class GA>
__device__ __forceinline__ uint32_t eval_preds(const GA& a, int64_t r0, int64_t n) {
  uint32_t keep = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (r0 + k < n) keep |= 1u << k;
  for (int p = 0; p < a.npreds; ++p) {
    int64_t v[ITEMS];
    load_col<ITEMS>(a.pcols[p], r0, n, v);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (!pred_pass(a.preds[p], v[k])) keep &= ~(1u << k);
    if (a.pcols[p].valid) keep &= valid_items<ITEMS>(a.pcols[p], r0, n);
  }
  return keep;
}

// Join slots of the kept rows' probe keys (-1: no match), all first probes
// issued before any is resolved.  Rows without a match are dropped from keep.
template <int ITEMS>
__device__ __forceinline__ void join_lookup(const JoinRef& j, int64_t r0, int64_t n, uint32_t& keep,
                                            int64_t (&slot)[ITEMS]) {
  int64_t kv[ITEMS];
  load_col<ITEMS>(j.key, r0, n, kv);
  if (j.key.valid) keep &= valid_items<ITEMS>(j.key, r0, n);
  const uint64_t cap = j.hdr->cap;
  uint64_t start[ITEMS], first[ITEMS];
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    start[k] = slot_of((uint64_t)kv[k], cap);
    first[k] = ((keep >> k) & 1u) ? j.keys[start[k]] : kEmpty;
  });
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    slot[k] = -1;
    if (!((keep >> k) & 1u)) return;
    const uint64_t key = (uint64_t)kv[k];
    if (key == kEmpty) {
      if (meta_count(j.meta[j.cap_alloc])) slot[k] = (int64_t)j.cap_alloc;
    } else {
      slot[k] = find_from(j.keys, cap, key, start[k], opaque_copy(first[k]));
    }
    if (slot[k] < 0) keep &= ~(1u << k);
  });
}

// Match counts of found slots: 1 unless the build side had duplicate keys.
template <int ITEMS>
__device__ __forceinline__ void join_weights(const JoinRef& j, uint32_t keep, const int64_t (&slot)[ITEMS],
                                             uint32_t (&w)[ITEMS]) {
  const bool dups = j.hdr->has_dups != 0;
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    w[k] = 1;
    if (((keep >> k) & 1u) && (dups || slot[k] == (int64_t)j.cap_alloc)) w[k] = meta_count(j.meta[slot[k]]);
  });
}

// Group keys of ITEMS rows.  special: 0 hashed, 1 EMPTY-valued raw key, 2 NULL raw key.
template <int ITEMS, class KP>
__device__ __forceinline__ void make_keys(const KP& kp, int64_t r0, int64_t n, uint64_t (&key)[ITEMS],
                                          uint8_t (&special)[ITEMS]) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    key[k] = 0;
    special[k] = 0;
  }
#pragma unroll
  for (int j = 0; j < GQ_MAX_KEYS; ++j) {
    if (j < kp.nk) {
      int64_t v[ITEMS];
      load_col<ITEMS>(kp.cols[j], r0, n, v);
      const uint32_t vm = kp.cols[j].valid ? valid_items<ITEMS>(kp.cols[j], r0, n) : 0xffffffffu;
      if (kp.mode == KEY_RAW64) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          key[k] = (uint64_t)v[k];
          special[k] = !((vm >> k) & 1u) ? 2 : (key[k] == kEmpty ? 1 : 0);
        }
      } else {
        const int w = kp.bits[j];
        const uint64_t mask = (w == 64) ? ~0ull : ((1ull << w) - 1);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          uint64_t f = ((uint64_t)v[k] ^ (1ull << (w - 1))) & mask;
          if (kp.nullable[j]) f = ((vm >> k) & 1u) ? (f | (1ull << w)) : 0ull;
          key[k] |= f << kp.shift[j];
        }
      }
    }
  }
}

// Input of aggregate `ag` for ITEMS rows: x[k] = product of its factors
// (wrapping).  Returns the mask of rows whose input is non-NULL.  A column used
// by several aggregates is re-read from cache (such columns use temporal loads).
template <int ITEMS, class AG, class AP>
__device__ __forceinline__ uint32_t agg_values(const AG& ag, const AP& ap, int64_t r0, int64_t n,
                                               uint64_t (&x)[ITEMS]) {
  uint32_t nn = 0xffffffffu;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) x[k] = 1;
  for (int f = 0; f < ag.nf; ++f) {
    const auto& fa = ag.f[f];
    if (fa.kind == GQ_F_CONST) {
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) x[k] *= (uint64_t)fa.k;
      continue;
    }
    const auto& c = ap.vals[fa.v];
    int64_t v[ITEMS];
    load_col<ITEMS>(c, r0, n, v);
    if (c.valid) nn &= valid_items<ITEMS>(c, r0, n);
    const uint64_t kk = (uint64_t)fa.k;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t cv = (uint64_t)v[k];
      const uint64_t t = fa.kind == GQ_F_COL ? cv : fa.kind == GQ_F_K_MINUS_COL ? kk - cv : kk + cv;
      x[k] *= t;
    }
  }
  return nn;
}

// Apply all aggregates of ITEMS rows.  Row k's accumulators are in LDS at
// lds + loff[k] (loff[k] >= 0) or in HBM at gsp[k]; word 0 is the row count.
template <int ITEMS, class AP>
__device__ __forceinline__ void apply_rows(const AP& ap, int64_t r0, int64_t n, uint32_t keep,
                                           const uint32_t (&w)[ITEMS], uint64_t* lds, const int (&loff)[ITEMS],
                                           uint64_t* const (&gsp)[ITEMS]) {
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    if (!((keep >> k) & 1u)) return;
    if (loff[k] >= 0) SharedAtomics::add(&lds[loff[k]], w[k]);
    else GlobalAtomics::add(&gsp[k][0], w[k]);
  });
  for (int i = 0; i < ap.naggs; ++i) {
    const auto& ag = ap.aggs[i];
    if (ag.op == GQ_COUNT_STAR) continue;
    uint64_t x[ITEMS];
    const uint32_t nn = agg_values<ITEMS>(ag, ap, r0, n, x) & keep;
    static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
      constexpr int k = decltype(kk)::value;
      if (!((nn >> k) & 1u)) return;
      const uint64_t wk = w[k];
      if (loff[k] >= 0) {
        uint64_t* s = lds + loff[k];
        switch (ag.op) {
          case GQ_SUM: SharedAtomics::add(&s[ag.word], x[k] * wk); break;
          case GQ_COUNT: SharedAtomics::add(&s[ag.word], wk); break;
          case GQ_MIN: SharedAtomics::min(&s[ag.word], (int64_t)x[k]); break;
          default: SharedAtomics::max(&s[ag.word], (int64_t)x[k]); break;
        }
        if (ag.cword >= 0) SharedAtomics::add(&s[ag.cword], wk);
      } else {
        uint64_t* s = gsp[k];
        switch (ag.op) {
          case GQ_SUM: GlobalAtomics::add(&s[ag.word], x[k] * wk); break;
          case GQ_COUNT: GlobalAtomics::add(&s[ag.word], wk); break;
          case GQ_MIN: GlobalAtomics::min(&s[ag.word], (int64_t)x[k]); break;
          default: GlobalAtomics::max(&s[ag.word], (int64_t)x[k]); break;
        }
        if (ag.cword >= 0) GlobalAtomics::add(&s[ag.cword], wk);
      }
    });
  }
}

// HBM accumulators of a row's group (hashed or extra), or nullptr if the table is full.
template <class GA>
__device__ __forceinline__ uint64_t* global_acc(const GA& a, uint64_t key, int special) {
  int64_t s;
  if (special) {
    s = (int64_t)(a.cap + (uint64_t)(special - 1));
  } else {
    bool ins;
    s = find_insert(a.keys, a.cap, key, &ins);
    if (s < 0) {
      atomicOr(a.dev_status, GQ_DEV_TABLE_FULL);
      return nullptr;
    }
    if (ins && a.d_inserted) atomicAdd((unsigned long long*)a.d_inserted, 1ull);
  }
  return a.acc + (uint64_t)s * a.ap.nacc;
}

// Merge one group's accumulators into HBM.
template <class AP>
__device__ __forceinline__ void merge_words(const AP& ap, uint64_t* dst, const uint64_t* src) {
  for (int w = 0; w < ap.nacc; ++w) {
    const uint64_t v = src[w];
    switch (ap.wop[w]) {
      case WOP_ADD:
        if (v) atomicAdd((unsigned long long*)&dst[w], (unsigned long long)v);
        break;
      case WOP_MIN:
        if ((int64_t)v != INT64_MAX) atomicMin((long long*)&dst[w], (long long)v);
        break;
      default:
        if ((int64_t)v != INT64_MIN) atomicMax((long long*)&dst[w], (long long)v);
        break;
    }
  }
}

// Slot of `key` in a block's LDS table (lcap slots of sw words: key, then
// accumulators), inserting it; returns the word offset of the slot's
// accumulators or -1 after kLdsProbes occupied probes.
constexpr int kLdsProbes = 16;

__device__ __forceinline__ int lds_find_insert(uint64_t* s_tab, int lcap, int sw, uint64_t key) {
  uint32_t s = (uint32_t)slot_of(key, (uint64_t)lcap);
  for (int p = 0; p < kLdsProbes; ++p) {
    const int off = (int)s * sw;
    const uint64_t kv = s_tab[off];
    if (kv == key) return off + 1;
    if (kv == kEmpty) {
      const uint64_t prev =
          atomicCAS((unsigned long long*)&s_tab[off], (unsigned long long)kEmpty, (unsigned long long)key);
      if (prev == kEmpty || prev == key) return off + 1;
    }
    s = (s + 1) & (uint32_t)(lcap - 1);
  }
  return -1;
}

// Host-side plan builders (groupby.hip), shared with the batched path.
int make_preds(gq_ctx* ctx, GbArgs& a, const gq_batch* in, const gq_pred* preds, int npreds);
// force_nullable (nk flags): the key packing reserves a NULL bit exactly for
// the flagged columns whatever this batch's bitmaps say (a key column with a
// bitmap must be flagged), so that batches of a stream pack keys alike.
int make_key_plan(gq_ctx* ctx, KeyPlan& kp, const gq_batch* in, const int32_t* keys, int nk,
                  const int32_t* force_nullable = nullptr);
// all_nullable: every SUM/MIN/MAX gets a non-NULL count word, so that the
// accumulator layout does not depend on which input columns have bitmaps.
int make_agg_plan(gq_ctx* ctx, AggPlan& ap, const gq_batch* in, const gq_agg* aggs, int na,
                  bool all_nullable = false);
// Aggregates that merge partial states (the Intermediate and Final modes of
// Section 3.2): each of `aggs` names its state column with one GQ_F_COL
// factor; SUM, COUNT(*) and COUNT states merge by SUM, MIN and MAX by MIN and
// MAX.  Writes na aggregates to merged.
int merge_aggs(gq_ctx* ctx, const gq_agg* aggs, int na, int ncols, gq_agg* merged);
// gq_groupby_agg over the first min(in->nrows, *d_nrows) rows of `in` (the
// row count known only on the device), no predicates and no join.
int groupby_rows(gq_ctx* ctx, const gq_batch* in, const int64_t* d_nrows, const int32_t* keys, int nkeys,
                 const gq_agg* aggs, int naggs, const gq_groupby_opts* opts, gq_batch* out, int64_t* d_groups,
                 hipStream_t stream);
// Aggregate the rows of a.n (no join) into the HBM table a.keys / a.acc
// (strategy GQ_STRATEGY_LDS or GQ_STRATEGY_GLOBAL); the table is not reset.
int aggregate_into(gq_ctx* ctx, GbArgs& a, int strategy, hipStream_t stream);
// Output validation and table compaction (groupby.hip).
int check_outputs(gq_ctx* ctx, int nk_out, int na, gq_batch* out, CompactArgs& ca, const int* key_types);
int compact_launch(gq_ctx* ctx, CompactArgs& ca, int64_t* d_groups, hipStream_t stream);
// Compaction into `out`, key-sorted through a radix sort when `sorted` is set.
// `emit`, when given, writes the groups into a CompactArgs' outputs in place
// of the compaction of its table.
int finish_groups(gq_ctx* ctx, CompactArgs& ca, const gq_batch* out, int64_t* d_groups, bool sorted,
                  hipStream_t stream, const std::function<int(CompactArgs&)>* emit = nullptr);
// Stable LSD radix sort by the unsigned int64 key in column 0 (partition.hip).
int radix_sort_rows(gq_ctx* ctx, const gq_batch* in, gq_batch* const bufs[2], gq_batch* out, int bits, int64_t n,
                    const int64_t* d_n, hipStream_t stream);

}  // namespace gq
