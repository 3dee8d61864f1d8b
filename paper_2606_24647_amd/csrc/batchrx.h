// Radix aggregation of high-cardinality fragments in a batched plan
// (batchrx.hip), shared with the plan builder (batch.hip).
#pragma once

#include "agg.h"

namespace gq {

// Output of one fragment of a batched plan.
struct BatchOut {
  OCol out[GQ_MAX_KEYS + GQ_MAX_AGGS];
  int64_t out_cap;
  int64_t* d_groups;
  int32_t append;  // the compaction appends after groups already written (radix fragments)
  int32_t pad;
};

constexpr int kBrxMaxStage = 8;

// One radix fragment: its regions, tiles, and the LDS staging of its columns.
struct BrxFrag {
  int32_t f;        // fragment index in the plan
  int32_t rbits;    // 2^rbits regions
  int64_t tiles;    // hist tiles (16384 rows)
  int64_t tile0;    // first global radix tile
  int64_t cbase;    // first entry of its (region, tile) counts
  int64_t item0;    // first global region item
  int32_t nst;      // staged columns: predicates and keys first, then values
  int32_t nst_hist;
  int32_t in_bytes;
  int32_t pad;
  DCol st[kBrxMaxStage];
  int32_t st_off[kBrxMaxStage];
  int32_t pred_st[GQ_MAX_PREDS];
  int32_t key_st[GQ_MAX_KEYS];
  int32_t val_st[kMaxVals];
};

struct BrxArgs {
  const GbArgs* frags;     // every fragment's plan (device)
  const BatchOut* outs;    // every fragment's output (device)
  const BrxFrag* rf;       // radix fragments (device)
  const int32_t* tile_frag;  // radix fragment of every hist tile
  const int32_t* item_frag;  // radix fragment of every region item
  int32_t nrf;
  int32_t lcap;            // LDS table slots of k_brx_agg
  int32_t nacc;
  int32_t nv;              // value words per tuple
  int32_t need_nn;         // tuples carry a non-NULL mask
  int32_t nk;
  int32_t vagg[GQ_MAX_AGGS];   // aggregate of value word v
  int32_t vword[GQ_MAX_AGGS];  // value word of aggregate i, -1 if none
  uint32_t* counts;        // (region, tile) counts of every radix fragment
  int64_t* starts;         // their exclusive scan, plus the total
  uint32_t* scan_ticket;
  uint64_t* scan_status;
  int64_t nscan;
  uint64_t* tup;           // tuples: key hash, then nv value words
  uint8_t* tnn;
  unsigned long long* item_ticket;
  int64_t nitems;          // region items of all radix fragments
};

size_t brx_lds_budget();
int brx_lcap(int nacc);
int64_t brx_tile_rows();
// Dynamic LDS of the scatter and hist kernels for one radix fragment.
size_t brx_scatter_lds_bytes(const BrxFrag& x);
size_t brx_hist_lds_bytes(const BrxFrag& x);
// LDS staging of a fragment's columns; -1 if they exceed kBrxMaxStage.
int brx_stage_plan(BrxFrag& x, const GbArgs& g, int nv, const int32_t* vagg, bool need_nn);
// Enqueue init, histogram, scan, scatter and aggregation (graph-capturable).
int brx_enqueue(const BrxArgs& a, int64_t ntiles, int64_t m, size_t max_scatter_lds, size_t max_hist_lds,
                int grid_agg, hipStream_t stream);

}  // namespace gq
