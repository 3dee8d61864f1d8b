// Host-side entry points of the radix group-join (radix.hip), used by the join
// build (join.hip) and the pipeline (groupby.hip).
#pragma once

#include "table.h"

namespace gq {

// Seed of the region hash; differs from the table-slot seed so that the slot
// of a key inside a region's LDS table is independent of its region.
constexpr uint64_t kRegionSeed = 0x2545f4914f6cdd1dull;
// Region hash of a join key and its inverse.  fmix64 is a bijection on 64-bit
// words (xor-shifts by 33 and odd multipliers), so partitioned rows carry the
// hash in place of the key: equal hashes are equal keys, and the key is
// recovered for output.
__host__ __device__ __forceinline__ uint64_t region_hash(uint64_t key) { return fmix64(key ^ kRegionSeed); }
__host__ __device__ __forceinline__ uint64_t region_unhash(uint64_t h) {
  h ^= h >> 33;
  h *= 0x9cb4b2f8129337dbull;  // inverse of 0xc4ceb9fe1a85ec53 modulo 2^64
  h ^= h >> 33;
  h *= 0x4f74430c22a54005ull;  // inverse of 0xff51afd7ed558ccd modulo 2^64
  h ^= h >> 33;
  return h ^ kRegionSeed;
}
// LDS of the join workgroup: table keys, accumulators, multiplicities and the
// staging words of an output validity bitmap.
constexpr size_t kRjLdsBytes = 150 * 1024;
// Build rows per sub-region assumed when the regions are laid out (two
// accumulator words: a count and one sum; about the kpr of such a table).
constexpr int64_t kRjNominalKpr = 3500;
// Build inputs from this many rows on are partitioned for the radix path.
constexpr int64_t kRjMinBuild = 1 << 20;

struct AggPlan;
struct CompactArgs;

// log2 of the number of regions for a build side of build_rows rows.
int rj_choose_pbits(int64_t build_rows);
// LDS table slots for nacc accumulator words, and the build rows one
// sub-region may hold (load factor 0.65).
int rj_lcap(int nacc);
int rj_kpr(int lcap);
// Partition the kept build rows (predicates pass, key non-NULL) by region into
// t->rj_kr / t->rj_off; the kept count goes to t->hdr->nrows.
int rj_build(gq_ctx* ctx, const gq_batch* build, int32_t key_col, const gq_pred* preds, int npreds,
             gq_join_table* t, hipStream_t stream);
// Whether a group-join of `in` with this aggregate plan can take the radix
// path (carry_col: a column whose value every probe tuple carries, or -1).
bool rj_usable(const gq_join_table* t, const gq_batch* in, int32_t probe_key, const gq_pred* preds, int npreds,
               const AggPlan& ap, int32_t carry_col = -1);
// Whether the build side's partition pass fits its staging limits.
bool rj_build_fits(const gq_batch* build, int32_t key_col, const gq_pred* preds, int npreds, int pbits);
// Group-join of `in` (rows passing preds, keyed by column probe_key) with the
// partitioned build side of t, writing the groups into ca.out (and ca.sortkey
// when set); *d_groups receives the group count.
int rj_groupjoin(gq_ctx* ctx, const gq_batch* in, int32_t probe_key, const gq_pred* preds, int npreds,
                 const AggPlan& ap, const gq_join_table* t, const CompactArgs& ca, int64_t* d_groups,
                 hipStream_t stream);

// A probe side partitioned once and joined with several tables (every table
// built over an input of the same row count, hence the same region count):
// rj_part_create partitions the rows of `in` that pass preds, each tuple
// carrying the value of column carry_col when carry_col >= 0; rj_part_join
// group-joins it with t, only tuples whose carried value lies in
// [carry_lo, carry_hi] taking part (bounds ignored without a carried column);
// rj_part_destroy releases the workspace, stream-ordered on the creating
// stream, so joins enqueued on that stream may still read it.
struct RjPart;
int rj_part_create(gq_ctx* ctx, const gq_batch* in, int32_t probe_key, const gq_pred* preds, int npreds,
                   int32_t carry_col, const AggPlan& ap, int pbits, hipStream_t stream, RjPart** out);
int rj_part_join(gq_ctx* ctx, const RjPart* part, const AggPlan& ap, const gq_join_table* t, int64_t carry_lo,
                 int64_t carry_hi, const CompactArgs& ca, int64_t* d_groups, hipStream_t stream);
void rj_part_destroy(RjPart* part);

// Build the probe index of a table whose build side was partitioned, if not
// built yet (on `stream`; later users on other streams must be ordered after it).
int join_ensure_index(gq_ctx* ctx, const gq_join_table* t, hipStream_t stream);
// Make `stream` wait until the table's build work has run (join.hip).
int join_wait_ready(gq_ctx* ctx, const gq_join_table* t, hipStream_t stream);

}  // namespace gq
