// Hash group-by (gq_groupby_agg) and the fused filter -> probe -> group-by
// pipeline (gq_pipeline).
//
// Strategies (chosen per call, see gq_groupby_opts):
//  - LDS-privatised: each block owns a small open-addressing table in LDS and
//    aggregates its rows there with LDS atomics; at the end it merges every
//    group it saw into the HBM table with one device-scope atomic per
//    accumulator word.  Rows whose key finds no LDS slot within a few probes go
//    straight to HBM.  For low-cardinality keys this turns one HBM atomic per
//    row and aggregate into one per block and group.
//  - Global: every row updates the HBM table directly (high cardinality).
//  - Group-join (pipeline only): when the only group key is the probe key and
//    the join table reserved accumulator words, a matching row accumulates into
//    the accumulators of the join slot it found, so the probe and the
//    aggregation share one lookup.
// In the pipeline a probe row that matches m build rows is accumulated with
// weight m (SUM adds m*x, COUNT adds m), which equals aggregating the
// materialised join.  All sums wrap modulo 2^64 and are therefore independent
// of the order in which atomics land.
#include "agg.h"
#include "radix.h"

#include <functional>

namespace gq {
namespace {

constexpr int kGbBlock = 256;
constexpr int kGbItems = 4;
constexpr int kGbLdsItems = 8;   // rows per thread per tile of the LDS strategy
constexpr int kGbReplicas = 16;  // HBM table replicas of a small LDS-strategy table
constexpr uint64_t kGbRepMaxCap = 1024;
constexpr int kGbLdsBlocksPerCu = 4;
constexpr int kGjItems = 8;
constexpr size_t kLdsBudget = 32 * 1024;

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Initialise `nslots` HBM slots: key EMPTY, accumulators at their identity.
__global__ void k_gt_init(uint64_t* keys, uint64_t* acc, int64_t nslots, AggPlan ap) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < nslots; i += step) {
    keys[i] = kEmpty;
    for (int w = 0; w < ap.nacc; ++w) acc[i * ap.nacc + w] = word_identity(ap.wop[w]);
  }
}

// Group-join accumulator init in a join table: occupied slots of [0, cap) and
// the extra slot.
__global__ void k_gj_init(JoinRef j, AggPlan ap) {
  const uint64_t cap = j.hdr->cap;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i <= (int64_t)cap; i += step) {
    const uint64_t s = (i == (int64_t)cap) ? j.cap_alloc : (uint64_t)i;
    if (s != j.cap_alloc && j.keys[s] == kEmpty) continue;
    for (int w = 0; w < ap.nacc; ++w) j.acc[s * j.acc_slots + w] = word_identity(ap.wop[w]);
  }
}

template <int BLOCK, int ITEMS, bool JOIN>
__global__ __launch_bounds__(BLOCK) void k_gb_global(const GbArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  const int64_t n = rows_of(a);
  const int64_t r0 = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * ITEMS;
  uint32_t keep = eval_preds<ITEMS>(a, r0, n);
  uint32_t w[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) w[k] = 1;
  if (JOIN) {
    int64_t js[ITEMS];
    join_lookup<ITEMS>(a.join, r0, n, keep, js);
    join_weights<ITEMS>(a.join, keep, js, w);
  }
  if (!keep) return;
  uint64_t key[ITEMS];
  uint8_t special[ITEMS];
  make_keys<ITEMS>(a.kp, r0, n, key, special);
  int loff[ITEMS];
  uint64_t* gsp[ITEMS];
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    loff[k] = -1;
    gsp[k] = nullptr;
    if ((keep >> k) & 1u) {
      gsp[k] = global_acc(a, key[k], special[k]);
      if (!gsp[k]) keep &= ~(1u << k);
    }
  });
  apply_rows<ITEMS>(a.ap, r0, n, keep, w, nullptr, loff, gsp);
}

template <int BLOCK, int ITEMS, bool JOIN>
__global__ __launch_bounds__(BLOCK) void k_gb_lds(const GbArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  extern __shared__ uint64_t s_tab[];
  const int sw = 1 + a.ap.nacc;  // LDS slot: key, then accumulators
  const int lcap = a.lcap;
  for (int i = threadIdx.x; i < lcap * sw; i += BLOCK) {
    const int wi = i % sw;
    s_tab[i] = wi == 0 ? kEmpty : word_identity(a.ap.wop[wi - 1]);
  }
  __syncthreads();

  const int64_t n = rows_of(a);
  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;
    uint32_t keep = eval_preds<ITEMS>(a, r0, n);
    uint32_t w[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) w[k] = 1;
    if (JOIN) {
      int64_t js[ITEMS];
      join_lookup<ITEMS>(a.join, r0, n, keep, js);
      join_weights<ITEMS>(a.join, keep, js, w);
    }
    if (!keep) continue;
    uint64_t key[ITEMS];
    uint8_t special[ITEMS];
    make_keys<ITEMS>(a.kp, r0, n, key, special);
    int loff[ITEMS];
    uint64_t* gsp[ITEMS];
    static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
      constexpr int k = decltype(kk)::value;
      loff[k] = -1;
      gsp[k] = nullptr;
      if (!((keep >> k) & 1u)) return;
      if (!special[k]) loff[k] = lds_find_insert(s_tab, lcap, sw, key[k]);
      if (loff[k] < 0) {
        gsp[k] = global_acc(a, key[k], special[k]);
        if (!gsp[k]) keep &= ~(1u << k);
      }
    });
    apply_rows<ITEMS>(a.ap, r0, n, keep, w, s_tab, loff, gsp);
  }
  __syncthreads();
  // Block b merges into replica b % nrep of the HBM table (device-wide
  // atomics on few group slots contend less); k_gb_rep_merge folds the
  // replicas into the first.
  const int rep = a.nrep > 1 ? (int)(blockIdx.x % a.nrep) : 0;
  uint64_t* rkeys = a.keys + (size_t)rep * a.rep_slots;
  uint64_t* racc = a.acc + (size_t)rep * a.rep_slots * a.ap.nacc;
  for (int i = threadIdx.x; i < lcap; i += BLOCK) {
    const uint64_t* ls = s_tab + (size_t)i * sw;
    if (ls[0] == kEmpty) continue;
    bool ins;
    const int64_t sl = find_insert(rkeys, a.cap, ls[0], &ins);
    if (sl < 0) {
      atomicOr(a.dev_status, GQ_DEV_TABLE_FULL);
      continue;
    }
    merge_words(a.ap, racc + (size_t)sl * a.ap.nacc, ls + 1);
  }
}

// Fold replicas 1..nrep-1 of the HBM table into replica 0.
__global__ void k_gb_rep_merge(const GbArgs a) {
  const int64_t total = (int64_t)(a.nrep - 1) * a.rep_slots;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += step) {
    const int64_t r = 1 + idx / a.rep_slots, sl = idx % a.rep_slots;
    const uint64_t* src = a.acc + ((size_t)r * a.rep_slots + sl) * a.ap.nacc;
    uint64_t* dst;
    if (sl < (int64_t)a.cap) {
      const uint64_t key = a.keys[(size_t)r * a.rep_slots + sl];
      if (key == kEmpty) continue;
      dst = global_acc(a, key, 0);
    } else {
      if (src[0] == 0) continue;  // extra slot never used in this replica
      dst = global_acc(a, 0, (int)(sl - (int64_t)a.cap) + 1);
    }
    if (dst) merge_words(a.ap, dst, src);
  }
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_groupjoin(const GbArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  const int64_t r0 = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * ITEMS;
  uint32_t keep = eval_preds<ITEMS>(a, r0, a.n);
  if (!keep) return;
  int64_t js[ITEMS];
  join_lookup<ITEMS>(a.join, r0, a.n, keep, js);
  uint32_t w[ITEMS];
  join_weights<ITEMS>(a.join, keep, js, w);
  int loff[ITEMS];
  uint64_t* gsp[ITEMS];
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    loff[k] = -1;
    gsp[k] = ((keep >> k) & 1u) ? a.join.acc + (uint64_t)js[k] * a.join.acc_slots : nullptr;
  });
  if (!keep) return;
  apply_rows<ITEMS>(a.ap, r0, a.n, keep, w, nullptr, loff, gsp);
}

__device__ __forceinline__ void put_value(uint8_t* out, int64_t g, int64_t v, int type) {
  switch (type) {
    case GQ_I8: reinterpret_cast<int8_t*>(out)[g] = (int8_t)v; break;
    case GQ_I16: reinterpret_cast<int16_t*>(out)[g] = (int16_t)v; break;
    case GQ_I32: reinterpret_cast<int32_t*>(out)[g] = (int32_t)v; break;
    default: reinterpret_cast<int64_t*>(out)[g] = v; break;
  }
}

// ---------------------------------------------------------------------------
// Small group-by in two launches
// ---------------------------------------------------------------------------
// For a cardinality hint of at most kGbSmallMax groups (packed keys, unsorted
// output): every block aggregates its tiles in an LDS table and stores its
// groups as a partial (no HBM table, no atomics outside LDS); the last block
// to finish, found with a ticket, merges all partials in its LDS and writes
// the output rows and the group count.  One launch zeroes the ticket, one does
// everything else, instead of table init, aggregation, replica merge and two
// compaction passes.
// The table has as many slots as the HBM table the hint would size (so the
// same inputs overflow it), and each slot's accumulators are replicated R
// times, lane l updating replica l % R: with a handful of groups, the lanes of
// a wave would otherwise serialise on the same few LDS words.
constexpr int64_t kGbSmallMax = 256;
constexpr int kGbSmallItems = 8;       // rows per thread per tile
constexpr int kGbSmallGrid = 256;      // blocks at most (each stores one partial; at most the block size)
constexpr size_t kGbSmallLds = 64 * 1024;
constexpr int kGbSmallVw = 1024 / 32;  // validity staging words (tables of at most 1024 slots)

struct SmallArgs {
  uint64_t* part;       // per block: word 0 the entry count, then entries of 1 + nacc words (key, accumulators)
  int64_t part_words;   // words per block
  uint32_t* ticket;     // zeroed by k_gb_small_init
  int32_t lcap;         // table slots (power of two, at most 1024)
  int32_t reps;         // accumulator replicas per slot (power of two)
  CompactArgs ca;       // output columns, key plan, aggregates, out_cap, d_count, dev_status
};

__global__ void k_gb_small_init(uint32_t* ticket) {
  if (threadIdx.x == 0) *ticket = 0;
}

// Slot of `key` in a key array of lcap slots, inserting it; -1 when full.
__device__ __forceinline__ int small_insert(uint64_t* s_keys, int lcap, uint64_t key) {
  uint32_t s = (uint32_t)slot_of(key, (uint64_t)lcap);
  for (int p = 0; p < lcap; ++p) {
    const uint64_t kv = s_keys[s];
    if (kv == key) return (int)s;
    if (kv == kEmpty) {
      const uint64_t prev =
          atomicCAS((unsigned long long*)&s_keys[s], (unsigned long long)kEmpty, (unsigned long long)key);
      if (prev == kEmpty || prev == key) return (int)s;
    }
    s = (s + 1) & (uint32_t)(lcap - 1);
  }
  return -1;
}

template <int BLOCK>
__device__ __forceinline__ void small_table_init(uint64_t* s_keys, uint64_t* s_acc, int lcap, int reps,
                                                 const AggPlan& ap) {
  for (int i = threadIdx.x; i < lcap; i += BLOCK) s_keys[i] = kEmpty;
  const int nw = lcap * reps * ap.nacc;
  for (int i = threadIdx.x; i < nw; i += BLOCK) s_acc[i] = word_identity(ap.wop[i % ap.nacc]);
}

// Word w of slot i, its replicas combined.
__device__ __forceinline__ uint64_t small_word(const uint64_t* s_acc, int i, int reps, const AggPlan& ap, int w) {
  const uint64_t* p = s_acc + (size_t)i * reps * ap.nacc + w;
  uint64_t v = p[0];
  for (int r = 1; r < reps; ++r) {
    const uint64_t x = p[(size_t)r * ap.nacc];
    switch (ap.wop[w]) {
      case WOP_ADD: v += x; break;
      case WOP_MIN: v = (int64_t)x < (int64_t)v ? x : v; break;
      default: v = (int64_t)x > (int64_t)v ? x : v; break;
    }
  }
  return v;
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_gb_small(const GbArgs a, const SmallArgs sa) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  extern __shared__ uint64_t s_mem[];
  __shared__ uint32_t s_n;
  __shared__ uint32_t s_last;
  __shared__ uint32_t s_wave[NW];
  __shared__ uint32_t s_vw[kGbSmallVw];
  __shared__ uint32_t s_pbase[kGbSmallGrid + 1];
  const int lcap = sa.lcap, reps = sa.reps, nacc = a.ap.nacc;
  uint64_t* s_keys = s_mem;
  uint64_t* s_acc = s_mem + lcap;
  const int rep = (int)(threadIdx.x & (uint32_t)(reps - 1));
  small_table_init<BLOCK>(s_keys, s_acc, lcap, reps, a.ap);
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();

  // 1. This block's tiles into its LDS table.
  const int64_t n = a.n;
  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;
    uint32_t keep = eval_preds<ITEMS>(a, r0, n);
    if (!keep) continue;
    uint32_t w[ITEMS];
    uint64_t key[ITEMS];
    uint8_t special[ITEMS];
    make_keys<ITEMS>(a.kp, r0, n, key, special);
    int loff[ITEMS];
    uint64_t* gsp[ITEMS];
    static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
      constexpr int k = decltype(kk)::value;
      w[k] = 1;
      gsp[k] = nullptr;
      loff[k] = -1;
      if (!((keep >> k) & 1u)) return;
      const int sl = small_insert(s_keys, lcap, key[k]);
      if (sl < 0) {
        atomicOr(a.dev_status, GQ_DEV_TABLE_FULL);
        keep &= ~(1u << k);
        return;
      }
      loff[k] = (sl * reps + rep) * nacc;
    });
    apply_rows<ITEMS>(a.ap, r0, n, keep, w, s_acc, loff, gsp);
  }
  __syncthreads();

  // 2. Its groups as a partial; the last block to get here merges them all.
  const int ew = 1 + nacc;
  uint64_t* part = sa.part + (size_t)blockIdx.x * sa.part_words;
  // The partial's words are agent-scope stores (written through to where
  // every XCD reads them) and complete (vmcnt 0) before the block's ticket is
  // taken; the last block reads them with agent-scope loads.  No device-wide
  // fence: on this GPU that would write back or invalidate whole L2 caches.
  for (int i = threadIdx.x; i < lcap; i += BLOCK) {
    if (s_keys[i] == kEmpty) continue;
    uint64_t* dst = part + 1 + (size_t)atomicAdd(&s_n, 1u) * ew;
    status_store(&dst[0], s_keys[i]);
    for (int k = 0; k < nacc; ++k) status_store(&dst[1 + k], small_word(s_acc, i, reps, a.ap, k));
  }
  __syncthreads();
  if (threadIdx.x == 0) status_store(&part[0], (uint64_t)s_n);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(sa.ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;

  // 3. Last block: every partial merged into a fresh LDS table.  The
  // partials' counts are read at once (a thread each) and scanned, then the
  // entries are spread over the threads, every word of an entry loaded before
  // the first is used (one round trip per entry, not one per word).
  small_table_init<BLOCK>(s_keys, s_acc, lcap, reps, a.ap);
  const int nb = (int)gridDim.x;  // <= kGbSmallGrid <= BLOCK
  const uint32_t pc = threadIdx.x < (uint32_t)nb
                          ? (uint32_t)status_load(sa.part + (size_t)threadIdx.x * sa.part_words) : 0u;
  {
    uint32_t wt;
    const uint32_t wp = wave_prefix_small<11>(pc, &wt);  // counts <= lcap <= 1024
    if (lane_id() == 0) s_wave[threadIdx.x / kWave] = wt;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      before += k < (int)(threadIdx.x / kWave) ? s_wave[k] : 0;
      total += s_wave[k];
    }
    if (threadIdx.x < (uint32_t)nb) s_pbase[threadIdx.x] = before + wp;
    if (threadIdx.x == 0) {
      s_pbase[nb] = total;
      s_n = total;
    }
  }
  __syncthreads();
  const uint32_t nent = s_n;
  for (uint32_t e = threadIdx.x; e < nent; e += BLOCK) {
    int lo = 0, hi = nb - 1;  // the partial b with s_pbase[b] <= e < s_pbase[b + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pbase[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    uint64_t* src = sa.part + (size_t)lo * sa.part_words + 1 + (size_t)(e - s_pbase[lo]) * ew;
    uint64_t v[1 + kMaxAcc];
#pragma unroll
    for (int k = 0; k <= kMaxAcc; ++k) v[k] = k <= nacc ? status_load(&src[k]) : 0;
    const int sl = small_insert(s_keys, lcap, v[0]);
    if (sl < 0) {
      atomicOr(a.dev_status, GQ_DEV_TABLE_FULL);
      continue;
    }
    uint64_t* dst = s_acc + ((size_t)sl * reps + rep) * nacc;
#pragma unroll
    for (int k = 0; k < kMaxAcc; ++k) {
      if (k >= nacc) break;
      switch (a.ap.wop[k]) {
        case WOP_ADD: SharedAtomics::add(&dst[k], v[1 + k]); break;
        case WOP_MIN: SharedAtomics::min(&dst[k], (int64_t)v[1 + k]); break;
        default: SharedAtomics::max(&dst[k], (int64_t)v[1 + k]); break;
      }
    }
  }
  __syncthreads();

  // 4. Occupied slots in slot order to the output rows, and the validity
  // bits of the first min(groups, out_cap) rows staged in LDS.
  const CompactArgs& ca = sa.ca;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nk = ca.kp.nk, ncol = nk + ca.naggs;
  int64_t base = 0;
  for (int c0 = 0; c0 < lcap; c0 += BLOCK) {
    const int i = c0 + (int)threadIdx.x;
    const bool occ = i < lcap && s_keys[i] != kEmpty;
    const uint64_t m = ballot(occ);
    if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      wpre += k < wave ? s_wave[k] : 0;
      tot += s_wave[k];
    }
    if (occ) {
      const int64_t g = base + wpre + rank_in(m);
      if (g < ca.out_cap) {
        for (int j = 0; j < ncol; ++j) {
          bool ok = true;
          int64_t v;
          if (j < nk) {
            v = decode_field(ca.kp, s_keys[i], j, &ok);
          } else {
            const DAgg& ag = ca.aggs[j - nk];
            v = (int64_t)small_word(s_acc, i, reps, a.ap, ag.word);
            if ((ag.op == GQ_SUM || ag.op == GQ_MIN || ag.op == GQ_MAX) && ag.cword >= 0)
              ok = small_word(s_acc, i, reps, a.ap, ag.cword) != 0;
            if (!ok) v = 0;
          }
          put_value(ca.out[j].data, g, v, ca.out[j].type);
        }
      }
    }
    base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ca.d_count = base;
    if (base > ca.out_cap) atomicOr(a.dev_status, GQ_DEV_CAPACITY);
  }
  // 5. Validity bitmaps of the rows [0, min(groups, out_cap)), word by word
  // (the last word's bits past the rows are 0).
  const int64_t rows = base < ca.out_cap ? base : ca.out_cap;
  const int vw = (int)((rows + 31) / 32);
  for (int j = 0; j < ncol; ++j) {
    if (!ca.out[j].valid) continue;
    for (int k = threadIdx.x; k < vw; k += BLOCK) s_vw[k] = 0;
    __syncthreads();
    int64_t run = 0;
    for (int c0 = 0; c0 < lcap; c0 += BLOCK) {
      const int i = c0 + (int)threadIdx.x;
      const bool occ = i < lcap && s_keys[i] != kEmpty;
      const uint64_t m = ballot(occ);
      if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
      __syncthreads();
      uint32_t wpre = 0, tot = 0;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        wpre += k < wave ? s_wave[k] : 0;
        tot += s_wave[k];
      }
      if (occ) {
        const int64_t g = run + wpre + rank_in(m);
        bool ok = true;
        if (j < nk) {
          (void)decode_field(ca.kp, s_keys[i], j, &ok);
        } else {
          const DAgg& ag = ca.aggs[j - nk];
          if ((ag.op == GQ_SUM || ag.op == GQ_MIN || ag.op == GQ_MAX) && ag.cword >= 0)
            ok = small_word(s_acc, i, reps, a.ap, ag.cword) != 0;
        }
        if (ok && g < rows) atomicOr(&s_vw[g >> 5], 1u << (g & 31));
      }
      run += tot;
      __syncthreads();
    }
    for (int k = threadIdx.x; k < vw; k += BLOCK) ca.out[j].valid[k] = s_vw[k];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Compaction of a table into the output batch
// ---------------------------------------------------------------------------
__global__ void k_compact_init(uint32_t* ticket, uint64_t* status, int64_t ntiles, int64_t* d_count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i == 0) {
    *ticket = 0;
    *d_count = 0;
  }
  for (; i < ntiles; i += stride) status[i] = 0;
}

// Output value of column j for occupied slot s (keys first, then aggregates,
// then the optional unsigned sort key); *ok = false for NULL.
__device__ __forceinline__ int64_t compact_value(const CompactArgs& a, int j, int nk, uint64_t s, bool* ok) {
  const bool extra = s >= a.cap_alloc;
  int64_t v = 0;
  *ok = true;
  if (j == nk + a.naggs) {
    // Sort key: unsigned order = key order, NULL first.
    constexpr uint64_t kSign = 1ull << 63;
    if (a.key_kind == 0) v = (int64_t)a.keys[s];
    else if (!extra) v = (int64_t)(a.keys[s] ^ kSign);
    else if (a.key_kind == 1 && s == a.cap_alloc + 1) v = 0;  // NULL
    else v = (int64_t)(~0ull ^ kSign);                         // the key -1
  } else if (j < nk) {
    if (a.key_kind == 2) {
      v = extra ? -1 : (int64_t)a.keys[s];
    } else if (a.kp.mode == KEY_RAW64) {
      if (extra) {
        const bool is_null = s == a.cap_alloc + 1;
        v = is_null ? 0 : -1;
        *ok = !is_null;
      } else {
        v = (int64_t)a.keys[s];
      }
    } else {
      v = decode_field(a.kp, a.keys[s], j, ok);
    }
  } else {
    const DAgg& ag = a.aggs[j - nk];
    const uint64_t* acc = a.acc + s * a.aw;
    v = (int64_t)acc[ag.word];
    if ((ag.op == GQ_SUM || ag.op == GQ_MIN || ag.op == GQ_MAX) && ag.cword >= 0) *ok = acc[ag.cword] != 0;
    if (!*ok) v = 0;
  }
  return v;
}


template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_compact(const CompactArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_wave[NW];
  __shared__ int64_t s_excl;
  __shared__ __attribute__((aligned(16))) uint8_t s_stage[TILE * 8];
  __shared__ uint8_t s_vbyte[TILE];
  __shared__ uint64_t s_slot[TILE];   // the tile's occupied slots in output order

  if (a.gate && *a.gate == 0) return;  // conditional compaction (streaming aggregation): nothing to emit
  if (threadIdx.x == 0) s_tile = atomicAdd(a.ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const uint64_t cap = a.d_cap ? *a.d_cap : a.cap;
  const int64_t total_idx = (int64_t)cap + a.extra;
  const int64_t i0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;
  int64_t sl[ITEMS];
  uint32_t keep = 0;
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    const int64_t i = i0 + k;
    sl[k] = -1;
    if (i >= total_idx) return;
    bool extra;
    uint64_t s;
    if (a.extras_first) {  // extras in reverse (NULL key, then the EMPTY-valued key), then hashed slots
      extra = i < a.extra;
      s = extra ? a.cap_alloc + (uint64_t)(a.extra - 1 - i) : (uint64_t)(i - a.extra);
    } else {
      extra = i >= (int64_t)cap;
      s = extra ? a.cap_alloc + (uint64_t)(i - (int64_t)cap) : (uint64_t)i;
    }
    bool occ;
    if (extra) occ = a.acc[s * a.aw] != 0;                       // extra slots: row count
    else if (a.key_kind == 2) occ = a.keys[s] != kEmpty && a.acc[s * a.aw] != 0;  // group-join: matched
    else occ = a.keys[s] != kEmpty;
    if (occ) {
      keep |= 1u << k;
      sl[k] = (int64_t)s;
    }
  });
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t wtot;
  const uint32_t wpre = wave_prefix_small<4>((uint32_t)__popc(keep), &wtot);
  if (lane == 0) s_wave[wave] = wtot;
  __syncthreads();
  uint32_t bpre = 0, btot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if (i < wave) bpre += s_wave[i];
    btot += s_wave[i];
  }
  const int local = (int)(bpre + wpre);
  {
    int pos = local;
    static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
      constexpr int k = decltype(kk)::value;
      if ((keep >> k) & 1u) s_slot[pos++] = (uint64_t)sl[k];
    });
  }
  if (wave == 0) {
    int64_t e = lookback_exclusive(a.status, tile, (int64_t)btot);
    if (lane == 0) s_excl = e;
  }
  __syncthreads();
  const int64_t goff = s_excl;
  const int nk = a.key_kind == 2 ? 1 : a.kp.nk;
  const int ncols = nk + a.naggs + (a.sortkey.data ? 1 : 0);
  if (tile == a.ntiles - 1 && threadIdx.x == 0) {
    int64_t total = goff + btot;
    if (total == 0 && a.global_agg) {
      // SQL: an aggregate without GROUP BY returns one row even for no input.
      for (int j = 0; j < a.naggs; ++j) {
        const OCol& o = a.out[j];
        const bool cnt = a.aggs[j].op == GQ_COUNT || a.aggs[j].op == GQ_COUNT_STAR;
        if (a.out_cap >= 1) {
          reinterpret_cast<int64_t*>(o.data)[0] = 0;
          if (o.valid) o.valid[0] = cnt ? (o.valid[0] | 1u) : (o.valid[0] & ~1u);
        }
      }
      total = 1;
    }
    *a.d_count = total;
    if (total > a.out_cap) atomicOr(a.dev_status, GQ_DEV_CAPACITY);
  }
  if (btot == 0) return;

  if ((int)btot * ncols <= TILE) {
    // Few groups: every (row, column) value of the tile is read in one round,
    // one per thread, so that the reads of all columns are in flight together
    // (the general path below reads one column per round).
    int64_t* s_val = reinterpret_cast<int64_t*>(s_stage);
    const int nb = (int)btot;
    for (int q = threadIdx.x; q < nb * ncols; q += BLOCK) {
      const int j = q / nb;
      bool ok;
      s_val[q] = compact_value(a, j, nk, s_slot[q - j * nb], &ok);
      s_vbyte[q] = ok ? 1 : 0;
    }
    __syncthreads();
    for (int j = 0; j < ncols; ++j) {
      const OCol& o = j < nk + a.naggs ? a.out[j] : a.sortkey;
      for (int i = threadIdx.x; i < nb; i += BLOCK) {
        const int64_t g = goff + i;
        if (g < a.out_cap) put_value(o.data, g, s_val[j * nb + i], o.type);
      }
      if (o.valid) write_valid_bits<BLOCK>(o.valid, s_vbyte + j * nb, goff, nb, a.out_cap);
    }
    return;
  }

  for (int j = 0; j < ncols; ++j) {
    const OCol& o = j < nk + a.naggs ? a.out[j] : a.sortkey;
    int pos = local;
    static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
      constexpr int k = decltype(kk)::value;
      if (!((keep >> k) & 1u)) return;
      bool ok;
      const int64_t v = compact_value(a, j, nk, (uint64_t)sl[k], &ok);
      stage_put(s_stage, pos, v, o.type);
      s_vbyte[pos] = ok ? 1 : 0;
      ++pos;
    });
    __syncthreads();
    for (int i = threadIdx.x; i < (int)btot; i += BLOCK) {
      const int64_t g = goff + i;
      if (g < a.out_cap) copy_out(s_stage, i, o.data, g, o.type);
    }
    if (o.valid) write_valid_bits<BLOCK>(o.valid, s_vbyte, goff, (int)btot, a.out_cap);
    __syncthreads();
  }
}

constexpr int kCBlock = 256, kCItems = 8;

// ---------------------------------------------------------------------------
// Host-side plans
// ---------------------------------------------------------------------------
template <bool JOIN>
int launch_aggregate(gq_ctx* ctx, GbArgs& a, int strategy, hipStream_t stream) {
  if (a.n == 0) return GQ_OK;
  if (strategy == GQ_STRATEGY_LDS) {
    constexpr int LTILE = kGbBlock * kGbLdsItems;
    a.ntiles = (a.n + LTILE - 1) / LTILE;
    const int sw = 1 + a.ap.nacc;
    int lcap = 1;
    while ((size_t)(lcap * 2) * sw * 8 <= kLdsBudget) lcap *= 2;
    a.lcap = lcap;
    const size_t lds = (size_t)lcap * sw * 8;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    const int64_t max_grid = (int64_t)cus * kGbLdsBlocksPerCu;
    int64_t grid = a.ntiles < max_grid ? a.ntiles : max_grid;
    GQ_LAUNCH(ctx, "gb_lds", (k_gb_lds<kGbBlock, kGbLdsItems, JOIN>), dim3((unsigned)grid), dim3(kGbBlock), lds,
              stream, a);
  } else {
    constexpr int TILE = kGbBlock * kGbItems;
    a.ntiles = (a.n + TILE - 1) / TILE;
    GQ_LAUNCH(ctx, "gb_global", (k_gb_global<kGbBlock, kGbItems, JOIN>), dim3((unsigned)a.ntiles), dim3(kGbBlock), 0,
              stream, a);
  }
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

static_assert(sizeof(GbArgs) + sizeof(SmallArgs) <= 4000, "k_gb_small kernel arguments exceed the kernarg limit");

// Table slots and accumulator replicas of a small group-by for this hint and
// load factor (the slots of the HBM table the hint would size, rounded up to
// a power of two); false when it does not fit the small path's LDS.
static bool small_shape(int64_t expected, float lf, int nacc, int* lcap, int* reps) {
  uint64_t cap = (uint64_t)((double)expected / lf) + 1;
  if (cap < 16) cap = 16;
  int l = 16;
  while ((uint64_t)l < cap) l *= 2;
  if (l > kGbSmallVw * 32) return false;
  int r = 8;
  while (r > 1 && (size_t)l * 8 * (1 + (size_t)r * nacc) > kGbSmallLds) r /= 2;
  if ((size_t)l * 8 * (1 + (size_t)r * nacc) > kGbSmallLds) return false;
  *lcap = l;
  *reps = r;
  return true;
}

static_assert(sizeof(GbArgs) + sizeof(SmallArgs) <= 4000, "k_gb_small kernel arguments exceed the kernarg limit");

// The two launches of a small group-by (k_gb_small); ca holds the checked
// outputs and the aggregate list.
static int run_small(gq_ctx* ctx, GbArgs& a, CompactArgs& ca, int lcap, int reps, int64_t* d_groups,
                     hipStream_t stream) {
  constexpr int LTILE = kGbBlock * kGbSmallItems;
  a.ntiles = (a.n + LTILE - 1) / LTILE;
  const int64_t grid = a.ntiles < kGbSmallGrid ? a.ntiles : kGbSmallGrid;
  SmallArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.lcap = lcap;
  sa.reps = reps;
  sa.part_words = 1 + (int64_t)lcap * (1 + a.ap.nacc);
  Scratch ws(ctx, stream);
  if (!ws.get(256 + (size_t)grid * (size_t)sa.part_words * 8))
    return set_error(ctx, GQ_ERR_NOMEM, "group-by: partial table allocation failed");
  sa.ticket = ws.as<uint32_t>(0);
  sa.part = ws.as<uint64_t>(256);
  ca.kp = a.kp;
  ca.d_count = d_groups;
  ca.dev_status = ctx->d_status;
  sa.ca = ca;
  const size_t lds = (size_t)lcap * 8 * (1 + (size_t)reps * a.ap.nacc);
  GQ_LAUNCH(ctx, "gb_small_init", k_gb_small_init, dim3(1), dim3(64), 0, stream, sa.ticket);
  GQ_LAUNCH_CHECK(ctx);
  GQ_LAUNCH(ctx, "gb_small", (k_gb_small<kGbBlock, kGbSmallItems>), dim3((unsigned)grid), dim3(kGbBlock), lds,
            stream, a, sa);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

int run_groupby(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys, const gq_pred* preds, int npreds,
                const gq_agg* aggs, int naggs, const gq_groupby_opts* opts, const gq_join_table* join,
                int32_t probe_key, gq_batch* out, int64_t* d_groups, hipStream_t stream,
                const int64_t* d_nrows = nullptr) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "group-by input");
  if (rc) return rc;
  if (!d_groups) return set_error(ctx, GQ_ERR_INVALID, "group-by: NULL group count");
  gq_groupby_opts o{};
  if (opts) o = *opts;
  if (o.mode < GQ_MODE_SINGLE || o.mode > GQ_MODE_FINAL) return set_error(ctx, GQ_ERR_INVALID, "group-by: unknown mode");
  gq_agg merged[GQ_MAX_AGGS];
  if (o.mode == GQ_MODE_INTERMEDIATE || o.mode == GQ_MODE_FINAL) {
    // Partial states in, merged states out: no predicates (the rows are
    // groups already) and no join.
    if (npreds != 0 || join)
      return set_error(ctx, GQ_ERR_INVALID, "group-by: the intermediate and final modes take no predicates or join");
    rc = merge_aggs(ctx, aggs, naggs, in->ncols, merged);
    if (rc) return rc;
    aggs = merged;
  }
  const float lf = o.load_factor > 0.f ? o.load_factor : 0.5f;
  if (!(lf > 0.f && lf <= 0.9f)) return set_error(ctx, GQ_ERR_INVALID, "group-by: load factor outside (0, 0.9]");
  if (o.strategy < GQ_STRATEGY_AUTO || o.strategy > GQ_STRATEGY_GLOBAL)
    return set_error(ctx, GQ_ERR_INVALID, "group-by: unknown strategy");

  GbArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = in->nrows;
  a.d_nrows = d_nrows;
  a.dev_status = ctx->d_status;
  rc = make_preds(ctx, a, in, preds, npreds);
  if (rc) return rc;
  rc = make_key_plan(ctx, a.kp, in, keys, nkeys);
  if (rc) return rc;
  rc = make_agg_plan(ctx, a.ap, in, aggs, naggs);
  if (rc) return rc;
  if (join) {
    if (probe_key < 0 || probe_key >= in->ncols) return set_error(ctx, GQ_ERR_INVALID, "pipeline: probe key out of range");
    if (join->device != ctx->device) return set_error(ctx, GQ_ERR_INVALID, "pipeline: join table on another device");
    a.join.hdr = join->hdr;
    a.join.keys = join->keys;
    a.join.meta = join->meta;
    a.join.acc = join->acc;
    a.join.cap_alloc = join->cap_alloc;
    a.join.acc_slots = join->acc_slots;
    a.join.key = make_dcol(in->cols[probe_key]);
    a.join.key.nt = 1;
    // A group key that is also the probe key is read twice; keep it cached.
    for (int j = 0; j < nkeys; ++j)
      if (keys[j] == probe_key) a.kp.cols[j].nt = 0;
  }

  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  CompactArgs ca;
  std::memset(&ca, 0, sizeof(ca));
  ca.naggs = naggs;
  for (int i = 0; i < naggs; ++i) ca.aggs[i] = a.ap.aggs[i];
  ca.global_agg = nkeys == 0;

  // Group-join of a partitioned (large) build side: radix path, no HBM table.
  const bool gj_shape = join && nkeys == 1 && keys[0] == probe_key;
  if (gj_shape && rj_usable(join, in, probe_key, preds, npreds, a.ap)) {
    int kt[1] = {in->cols[probe_key].type};
    rc = check_outputs(ctx, 1, naggs, out, ca, kt);
    if (rc) return rc;
    ca.key_kind = 2;
    ca.extra = 1;
    const std::function<int(CompactArgs&)> emit = [&](CompactArgs& target) {
      return rj_groupjoin(ctx, in, probe_key, preds, npreds, a.ap, join, target, d_groups, stream);
    };
    return finish_groups(ctx, ca, out, d_groups, (o.flags & GQ_SORTED) != 0, stream, &emit);
  }
  if (join) {
    rc = join_ensure_index(ctx, join, stream);
    if (rc) return rc;
    // A partitioned table's index arrays exist from here on.
    a.join.keys = join->keys;
    a.join.meta = join->meta;
    a.join.acc = join->acc;
  }
  // Group-join: the only key is the probe key and the table has room.
  const bool groupjoin = gj_shape && join->acc_slots >= a.ap.nacc;
  if (groupjoin) {
    int kt[1] = {in->cols[probe_key].type};
    rc = check_outputs(ctx, 1, naggs, out, ca, kt);
    if (rc) return rc;
    // A fresh table has zeroed accumulators; MIN/MAX identities or a table
    // already used by a group-join need the init pass.
    bool need_init = join->acc_dirty;
    for (int w = 0; w < a.ap.nacc; ++w) need_init |= a.ap.wop[w] != WOP_ADD;
    if (need_init) {
      int64_t blocks = (int64_t)((join->cap_alloc + 1 + 255) / 256);
      if (blocks > 8192) blocks = 8192;
      GQ_LAUNCH(ctx, "gj_init", k_gj_init, dim3((unsigned)blocks), dim3(256), 0, stream, a.join, a.ap);
      GQ_LAUNCH_CHECK(ctx);
    }
    const_cast<gq_join_table*>(join)->acc_dirty = true;
    constexpr int TILE = kGbBlock * kGjItems;
    a.ntiles = (a.n + TILE - 1) / TILE;
    if (a.ntiles > 0) {
      GQ_LAUNCH(ctx, "groupjoin", (k_groupjoin<kGbBlock, kGjItems>), dim3((unsigned)a.ntiles), dim3(kGbBlock), 0,
                stream, a);
      GQ_LAUNCH_CHECK(ctx);
    }
    ca.keys = join->keys;
    ca.acc = join->acc;
    ca.d_cap = &join->hdr->cap;
    ca.cap_alloc = join->cap_alloc;
    ca.aw = join->acc_slots;
    ca.key_kind = 2;
    ca.extra = 1;
    ca.global_agg = 0;
    return finish_groups(ctx, ca, out, d_groups, (o.flags & GQ_SORTED) != 0, stream);
  }

  int key_types[GQ_MAX_KEYS];
  for (int j = 0; j < nkeys; ++j) key_types[j] = in->cols[keys[j]].type;
  rc = check_outputs(ctx, nkeys, naggs, out, ca, key_types);
  if (rc) return rc;

  int strategy = o.strategy;
  if (strategy == GQ_STRATEGY_AUTO) {
    // LDS privatisation unless the caller expects more groups than a block's
    // LDS table holds comfortably; with no estimate, LDS first (rows that find
    // no LDS slot fall through to HBM).
    strategy = (o.expected_groups == 0 || o.expected_groups <= 256) ? GQ_STRATEGY_LDS : GQ_STRATEGY_GLOBAL;
  }

  // A small group-by (a hint of at most kGbSmallMax groups, packed keys,
  // unsorted output) takes two launches.
  int small_lcap = 0, small_reps = 0;
  if (strategy == GQ_STRATEGY_LDS && !join && nkeys > 0 && a.kp.mode != KEY_RAW64 && o.expected_groups > 0 &&
      o.expected_groups <= kGbSmallMax && (o.flags & GQ_SORTED) == 0 && !d_nrows && o.mode == GQ_MODE_SINGLE &&
      a.n > 0 && small_shape(o.expected_groups, lf, a.ap.nacc, &small_lcap, &small_reps)) {
    GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return run_small(ctx, a, ca, small_lcap, small_reps, d_groups, stream);
  }

  // Table sizing.  A small table under the LDS strategy gets replicas for the
  // blocks' merges.
  int64_t expected = o.expected_groups > 0 ? o.expected_groups : in->nrows;
  if (nkeys == 0) expected = 1;
  uint64_t cap = (uint64_t)((double)expected / lf) + 1;
  if (cap < 16) cap = 16;
  a.cap = cap;
  const size_t nslot = (size_t)cap + 2;
  a.nrep = strategy == GQ_STRATEGY_LDS && cap <= kGbRepMaxCap ? kGbReplicas : 1;
  a.rep_slots = (int64_t)nslot;
  const size_t nslot_all = nslot * (size_t)a.nrep;
  const size_t off_acc = align_up(nslot_all * 8, 256);
  const size_t bytes = off_acc + nslot_all * 8 * (size_t)a.ap.nacc;
  Scratch table(ctx, stream);
  if (!table.get(bytes)) return set_error(ctx, GQ_ERR_NOMEM, "group-by: table allocation failed");
  a.keys = table.as<uint64_t>(0);
  a.acc = table.as<uint64_t>(off_acc);
  int64_t iblocks = (int64_t)((nslot_all + 255) / 256);
  if (iblocks > 8192) iblocks = 8192;
  GQ_LAUNCH(ctx, "gt_init", k_gt_init, dim3((unsigned)iblocks), dim3(256), 0, stream, a.keys, a.acc,
            (int64_t)nslot_all, a.ap);
  GQ_LAUNCH_CHECK(ctx);

  rc = join ? launch_aggregate<true>(ctx, a, strategy, stream) : launch_aggregate<false>(ctx, a, strategy, stream);
  if (rc) return rc;
  if (a.nrep > 1 && a.n > 0) {
    const int64_t mblocks = ((int64_t)(a.nrep - 1) * a.rep_slots + 255) / 256;
    GQ_LAUNCH(ctx, "gb_rep_merge", k_gb_rep_merge, dim3((unsigned)mblocks), dim3(256), 0, stream, a);
    GQ_LAUNCH_CHECK(ctx);
  }

  ca.keys = a.keys;
  ca.acc = a.acc;
  ca.d_cap = nullptr;
  ca.cap = cap;
  ca.cap_alloc = cap;
  ca.aw = a.ap.nacc;
  ca.key_kind = a.kp.mode == KEY_RAW64 ? 1 : 0;
  ca.kp = a.kp;
  ca.extra = 2;
  return finish_groups(ctx, ca, out, d_groups, (o.flags & GQ_SORTED) != 0 && nkeys > 0, stream);
}

}  // namespace

int check_outputs(gq_ctx* ctx, int nk_out, int na, gq_batch* out, CompactArgs& ca, const int* key_types) {
  if (!out || out->ncols < nk_out + na || (nk_out + na > 0 && !out->cols))
    return set_error(ctx, GQ_ERR_INVALID, "group-by: output needs key and aggregate columns");
  int64_t cap = INT64_MAX;
  for (int j = 0; j < nk_out + na; ++j) {
    const gq_column& oc = out->cols[j];
    const int want = j < nk_out ? key_types[j] : GQ_I64;
    if (oc.type != want) return set_error(ctx, GQ_ERR_INVALID, "group-by: output column type mismatch");
    if (oc.length < 0 || (oc.length > 0 && !oc.data)) return set_error(ctx, GQ_ERR_INVALID, "group-by: bad output column");
    if (oc.validity && (reinterpret_cast<uintptr_t>(oc.validity) & 3))
      return set_error(ctx, GQ_ERR_INVALID, "group-by: output bitmap must be 4-byte aligned");
    if (oc.offset != 0) return set_error(ctx, GQ_ERR_INVALID, "group-by: output offset must be 0");
    ca.out[j] = OCol{static_cast<uint8_t*>(oc.data), reinterpret_cast<uint32_t*>(oc.validity), oc.type, 0};
    if (oc.length < cap) cap = oc.length;
  }
  ca.out_cap = cap;
  return GQ_OK;
}

int compact_launch(gq_ctx* ctx, CompactArgs& ca, int64_t* d_groups, hipStream_t stream) {
  constexpr int TILE = kCBlock * kCItems;
  const int64_t nidx = (int64_t)ca.cap_alloc + ca.extra;
  const int64_t ntiles = (nidx + TILE - 1) / TILE;
  ca.ntiles = ntiles;
  ca.d_count = d_groups;
  ca.dev_status = ctx->d_status;
  Scratch ws(ctx, stream);
  if (!ws.get(256 + align_up((size_t)ntiles * 8, 256)))
    return set_error(ctx, GQ_ERR_NOMEM, "group-by: compaction workspace allocation failed");
  ca.ticket = ws.as<uint32_t>(0);
  ca.status = ws.as<uint64_t>(256);
  int64_t iblocks = (ntiles + 255) / 256;
  if (iblocks < 1) iblocks = 1;
  if (iblocks > 4096) iblocks = 4096;
  GQ_LAUNCH(ctx, "compact_init", k_compact_init, dim3((unsigned)iblocks), dim3(256), 0, stream, ca.ticket, ca.status,
            ntiles, d_groups);
  GQ_LAUNCH_CHECK(ctx);
  GQ_LAUNCH(ctx, "compact", (k_compact<kCBlock, kCItems>), dim3((unsigned)ntiles), dim3(kCBlock), 0, stream, ca);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

int finish_groups(gq_ctx* ctx, CompactArgs& ca, const gq_batch* out, int64_t* d_groups, bool sorted,
                  hipStream_t stream, const std::function<int(CompactArgs&)>* emit) {
  if (!sorted) return emit ? (*emit)(ca) : compact_launch(ctx, ca, d_groups, stream);
  // Compact into two scratch batches [sort key, keys..., aggregates...], then
  // radix-sort by the key into [scratch key, caller's columns].
  const int nk = ca.key_kind == 2 ? 1 : ca.kp.nk;
  const int nc = nk + ca.naggs;
  const int64_t cap = ca.out_cap;
  int bits = 64;
  if (ca.key_kind == 0) {
    bits = 0;
    for (int j = 0; j < ca.kp.nk; ++j) bits += ca.kp.bits[j] + ca.kp.nullable[j];
  }
  size_t bytes = 0;
  size_t off[2][1 + GQ_MAX_KEYS + GQ_MAX_AGGS], voff[2][1 + GQ_MAX_KEYS + GQ_MAX_AGGS];
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j <= nc; ++j) {
      const int w = j == 0 ? 8 : type_width(ca.out[j - 1].type);
      off[b][j] = bytes;
      bytes = align_up(bytes + (size_t)(cap > 0 ? cap : 1) * w, 256);
      voff[b][j] = bytes;
      if (j > 0 && ca.out[j - 1].valid) bytes = align_up(bytes + (size_t)((cap + 63) / 64) * 8, 256);
    }
  const size_t key3 = bytes;
  bytes = align_up(bytes + (size_t)(cap > 0 ? cap : 1) * 8, 256);
  Scratch ws(ctx, stream);
  if (!ws.get(bytes)) return set_error(ctx, GQ_ERR_NOMEM, "group-by: sort workspace allocation failed");
  gq_column cols[3][1 + GQ_MAX_KEYS + GQ_MAX_AGGS];
  std::memset(cols, 0, sizeof(cols));
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j <= nc; ++j) {
      gq_column& c = cols[b][j];
      c.type = j == 0 ? GQ_I64 : ca.out[j - 1].type;
      c.length = cap;
      c.data = ws.as<void>(off[b][j]);
      c.validity = (j > 0 && ca.out[j - 1].valid) ? ws.as<uint8_t>(voff[b][j]) : nullptr;
    }
  cols[2][0].type = GQ_I64;
  cols[2][0].length = cap;
  cols[2][0].data = ws.as<void>(key3);
  for (int j = 1; j <= nc; ++j) cols[2][j] = out->cols[j - 1];
  gq_batch bt[3];
  for (int b = 0; b < 3; ++b) bt[b] = gq_batch{cap, nc + 1, 0, cols[b]};
  // Compaction into buffer 0.
  CompactArgs c2 = ca;
  c2.sortkey = OCol{static_cast<uint8_t*>(cols[0][0].data), nullptr, GQ_I64, 0};
  for (int j = 0; j < nc; ++j)
    c2.out[j] = OCol{static_cast<uint8_t*>(cols[0][j + 1].data), reinterpret_cast<uint32_t*>(cols[0][j + 1].validity),
                     cols[0][j + 1].type, 0};
  c2.extras_first = 1;
  int rc = emit ? (*emit)(c2) : compact_launch(ctx, c2, d_groups, stream);
  if (rc) return rc;
  gq_batch* bufs[2] = {&bt[1], &bt[0]};
  return radix_sort_rows(ctx, &bt[0], bufs, &bt[2], bits, cap, d_groups, stream);
}


int make_preds(gq_ctx* ctx, GbArgs& a, const gq_batch* in, const gq_pred* preds, int npreds) {
  if (npreds < 0 || npreds > GQ_MAX_PREDS || (npreds > 0 && !preds))
    return set_error(ctx, GQ_ERR_INVALID, "group-by: bad predicate list");
  a.npreds = npreds;
  for (int p = 0; p < npreds; ++p) {
    if (preds[p].col < 0 || preds[p].col >= in->ncols)
      return set_error(ctx, GQ_ERR_INVALID, "group-by: predicate column out of range");
    if (preds[p].op != GQ_RANGE && preds[p].op != GQ_NE)
      return set_error(ctx, GQ_ERR_INVALID, "group-by: unknown predicate op");
    a.preds[p] = DPred{preds[p].col, preds[p].op, preds[p].lo, preds[p].hi};
    a.pcols[p] = make_dcol(in->cols[preds[p].col]);
    a.pcols[p].nt = 1;
  }
  return GQ_OK;
}

int make_key_plan(gq_ctx* ctx, KeyPlan& kp, const gq_batch* in, const int32_t* keys, int nk,
                  const int32_t* force_nullable) {
  if (nk < 0 || nk > GQ_MAX_KEYS || (nk > 0 && !keys))
    return set_error(ctx, GQ_ERR_INVALID, "group-by: bad key list");
  kp.nk = nk;
  for (int j = 0; j < nk; ++j) {
    if (keys[j] < 0 || keys[j] >= in->ncols) return set_error(ctx, GQ_ERR_INVALID, "group-by: key column out of range");
    kp.cols[j] = make_dcol(in->cols[keys[j]]);
    kp.cols[j].nt = 1;
  }
  if (nk == 1 && in->cols[keys[0]].type == GQ_I64) {
    kp.mode = KEY_RAW64;
    kp.bits[0] = 64;
    kp.shift[0] = 0;
    kp.nullable[0] = in->cols[keys[0]].validity != nullptr;
    if (force_nullable) {
      if (kp.nullable[0] && !force_nullable[0])
        return set_error(ctx, GQ_ERR_INVALID, "group-by: key column has a bitmap but was declared non-nullable");
      kp.nullable[0] = force_nullable[0] != 0;
    }
    return GQ_OK;
  }
  kp.mode = KEY_PACKED;
  int shift = 0;
  for (int j = nk - 1; j >= 0; --j) {
    const gq_column& c = in->cols[keys[j]];
    kp.bits[j] = 8 * type_width(c.type);
    kp.nullable[j] = c.validity != nullptr;
    if (force_nullable) {
      if (kp.nullable[j] && !force_nullable[j])
        return set_error(ctx, GQ_ERR_INVALID, "group-by: key column has a bitmap but was declared non-nullable");
      kp.nullable[j] = force_nullable[j] != 0;
    }
    kp.shift[j] = shift;
    shift += kp.bits[j] + kp.nullable[j];
  }
  if (shift > 63)
    return set_error(ctx, GQ_ERR_UNSUPPORTED,
                     "group-by: key columns wider than 63 bits together (use one int64 key column)");
  return GQ_OK;
}

int make_agg_plan(gq_ctx* ctx, AggPlan& ap, const gq_batch* in, const gq_agg* aggs, int na, bool all_nullable) {
  if (na < 0 || na > GQ_MAX_AGGS || (na > 0 && !aggs))
    return set_error(ctx, GQ_ERR_INVALID, "group-by: bad aggregate list");
  ap.naggs = na;
  ap.nvals = 0;
  int cols[kMaxVals];
  int uses[kMaxVals] = {0};
  int word = 1;
  ap.wop[0] = WOP_ADD;
  for (int i = 0; i < na; ++i) {
    const gq_agg& g = aggs[i];
    DAgg& d = ap.aggs[i];
    d.op = g.op;
    d.nf = 0;
    d.cword = -1;
    if (g.op < GQ_SUM || g.op > GQ_MAX) return set_error(ctx, GQ_ERR_INVALID, "group-by: unknown aggregate");
    if (g.op == GQ_COUNT_STAR) {
      d.word = 0;
      continue;
    }
    if (g.nfactors < 0 || g.nfactors > 3) return set_error(ctx, GQ_ERR_INVALID, "group-by: 0..3 factors");
    bool nullable = false;
    d.nf = g.nfactors;
    for (int f = 0; f < g.nfactors; ++f) {
      const gq_factor& fa = g.f[f];
      if (fa.kind < GQ_F_COL || fa.kind > GQ_F_CONST) return set_error(ctx, GQ_ERR_INVALID, "group-by: bad factor");
      d.f[f].kind = fa.kind;
      d.f[f].k = fa.k;
      d.f[f].v = 0;
      if (fa.kind == GQ_F_CONST) continue;
      if (fa.col < 0 || fa.col >= in->ncols) return set_error(ctx, GQ_ERR_INVALID, "group-by: factor column out of range");
      int vi = -1;
      for (int q = 0; q < ap.nvals; ++q)
        if (cols[q] == fa.col) vi = q;
      if (vi < 0) {
        if (ap.nvals == kMaxVals) return set_error(ctx, GQ_ERR_UNSUPPORTED, "group-by: more than 8 value columns");
        vi = ap.nvals++;
        cols[vi] = fa.col;
        ap.vals[vi] = make_dcol(in->cols[fa.col]);
      }
      uses[vi] += 1;
      d.f[f].v = vi;
      if (in->cols[fa.col].validity) nullable = true;
    }
    d.word = word++;
    ap.wop[d.word] = g.op == GQ_MIN ? WOP_MIN : g.op == GQ_MAX ? WOP_MAX : WOP_ADD;
    if ((nullable || all_nullable) && g.op != GQ_COUNT) {
      d.cword = word++;
      ap.wop[d.cword] = WOP_ADD;
    }
  }
  // A value column read by one factor only is streamed with non-temporal loads.
  for (int q = 0; q < ap.nvals; ++q) ap.vals[q].nt = uses[q] == 1 ? 1 : 0;
  ap.nacc = word;
  return GQ_OK;
}

int groupby_rows(gq_ctx* ctx, const gq_batch* in, const int64_t* d_nrows, const int32_t* keys, int nkeys,
                 const gq_agg* aggs, int naggs, const gq_groupby_opts* opts, gq_batch* out, int64_t* d_groups,
                 hipStream_t stream) {
  return run_groupby(ctx, in, keys, nkeys, nullptr, 0, aggs, naggs, opts, nullptr, 0, out, d_groups, stream, d_nrows);
}

int aggregate_into(gq_ctx* ctx, GbArgs& a, int strategy, hipStream_t stream) {
  return launch_aggregate<false>(ctx, a, strategy, stream);
}

int merge_aggs(gq_ctx* ctx, const gq_agg* aggs, int na, int ncols, gq_agg* merged) {
  if (na < 0 || na > GQ_MAX_AGGS || (na > 0 && !aggs))
    return set_error(ctx, GQ_ERR_INVALID, "group-by: bad aggregate list");
  for (int i = 0; i < na; ++i) {
    const gq_agg& g = aggs[i];
    if (g.nfactors != 1 || g.f[0].kind != GQ_F_COL || g.f[0].col < 0 || g.f[0].col >= ncols)
      return set_error(ctx, GQ_ERR_INVALID,
                       "group-by: in the intermediate and final modes each aggregate names its state column "
                       "(one GQ_F_COL factor)");
    gq_agg m = g;
    switch (g.op) {
      case GQ_SUM: case GQ_COUNT_STAR: case GQ_COUNT: m.op = GQ_SUM; break;
      case GQ_MIN: m.op = GQ_MIN; break;
      case GQ_MAX: m.op = GQ_MAX; break;
      default: return set_error(ctx, GQ_ERR_INVALID, "group-by: unknown aggregate");
    }
    merged[i] = m;
  }
  return GQ_OK;
}

}  // namespace gq

using namespace gq;

extern "C" {

int gq_groupby_agg(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys, const gq_pred* preds, int npreds,
                   const gq_agg* aggs, int naggs, const gq_groupby_opts* opts, gq_batch* out, int64_t* d_groups,
                   hipStream_t stream) {
  return run_groupby(ctx, in, keys, nkeys, preds, npreds, aggs, naggs, opts, nullptr, 0, out, d_groups, stream);
}

int gq_pipeline(gq_ctx* ctx, const gq_plan* plan, const gq_batch* in, gq_batch* out, int64_t* d_groups,
                hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  if (!plan) return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline: NULL plan");
  if (plan->join && plan->join->nkeys != 1)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "gq_pipeline: the join table must have one key column");
  return run_groupby(ctx, in, plan->group_keys, plan->ngroup_keys, plan->preds, plan->npreds, plan->aggs, plan->naggs,
                     &plan->opts, plan->join, plan->probe_key, out, d_groups, stream);
}

int gq_pipeline_shared(gq_ctx* ctx, const gq_plan* plan, const gq_batch* in, int32_t nq,
                       const gq_join_table* const* tables, const gq_pred* ranges, gq_batch* const* outs,
                       int64_t* const* d_groups, hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  if (!plan || nq < 1 || !tables || !ranges || !outs || !d_groups)
    return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline_shared: NULL argument or no query");
  int rc = check_batch(ctx, in, "shared pipeline input");
  if (rc) return rc;
  if (plan->join) return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline_shared: the tables are passed per query");
  const int32_t pk = plan->probe_key;
  if (pk < 0 || pk >= in->ncols) return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline_shared: probe key out of range");
  if (plan->ngroup_keys != 1 || !plan->group_keys || plan->group_keys[0] != pk)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "gq_pipeline_shared: the only group key must be the probe key");
  if (plan->opts.mode != GQ_MODE_SINGLE)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "gq_pipeline_shared: single-mode aggregation only");
  if (plan->npreds < 0 || plan->npreds + 1 > GQ_MAX_PREDS || (plan->npreds > 0 && !plan->preds))
    return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline_shared: too many predicates");
  const int32_t rcol = ranges[0].col;
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  for (int i = 0; i < nq; ++i) {
    if (ranges[i].op != GQ_RANGE || ranges[i].col != rcol)
      return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline_shared: every query range is a GQ_RANGE on one column");
    if (ranges[i].lo < lo) lo = ranges[i].lo;
    if (ranges[i].hi > hi) hi = ranges[i].hi;
    const gq_join_table* t = tables[i];
    if (!t || !d_groups[i]) return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline_shared: NULL table or group count");
    if (t->device != ctx->device) return set_error(ctx, GQ_ERR_INVALID, "gq_pipeline_shared: table on another device");
    if (t->nkeys != 1)
      return set_error(ctx, GQ_ERR_UNSUPPORTED, "gq_pipeline_shared: every table must have one key column");
    if (!t->rj_kr || t->rj_pbits != tables[0]->rj_pbits)
      return set_error(ctx, GQ_ERR_UNSUPPORTED,
                       "gq_pipeline_shared: every table must be partitioned with the same region count");
  }
  // The probe side keeps the rows of the hull of the ranges.
  gq_pred preds[GQ_MAX_PREDS];
  for (int p = 0; p < plan->npreds; ++p) preds[p] = plan->preds[p];
  preds[plan->npreds] = gq_pred{rcol, GQ_RANGE, lo, hi};
  const int npreds = plan->npreds + 1;
  GbArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = in->nrows;
  rc = make_preds(ctx, a, in, preds, npreds);
  if (rc) return rc;
  rc = make_agg_plan(ctx, a.ap, in, plan->aggs, plan->naggs);
  if (rc) return rc;
  if (!rj_usable(tables[0], in, pk, preds, npreds, a.ap, rcol))
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "gq_pipeline_shared: the radix group-join does not take this input");
  std::vector<CompactArgs> ca(nq);
  const int kt[1] = {in->cols[pk].type};
  for (int i = 0; i < nq; ++i) {
    std::memset(&ca[i], 0, sizeof(CompactArgs));
    ca[i].naggs = plan->naggs;
    for (int g = 0; g < plan->naggs; ++g) ca[i].aggs[g] = a.ap.aggs[g];
    rc = check_outputs(ctx, 1, plan->naggs, outs[i], ca[i], kt);
    if (rc) return rc;
    ca[i].key_kind = 2;
    ca[i].extra = 1;
  }
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  RjPart* part = nullptr;
  rc = rj_part_create(ctx, in, pk, preds, npreds, rcol, a.ap, tables[0]->rj_pbits, stream, &part);
  if (rc) return rc;
  const bool sorted = (plan->opts.flags & GQ_SORTED) != 0;
  for (int i = 0; i < nq && rc == GQ_OK; ++i) {
    const std::function<int(CompactArgs&)> emit = [&](CompactArgs& target) {
      return rj_part_join(ctx, part, a.ap, tables[i], ranges[i].lo, ranges[i].hi, target, d_groups[i], stream);
    };
    rc = finish_groups(ctx, ca[i], outs[i], d_groups[i], sorted, stream, &emit);
  }
  rj_part_destroy(part);
  return rc;
}

}  // extern "C"
