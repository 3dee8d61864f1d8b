// Hash join: gq_join_build, gq_join_probe, gq_gather.
//
// Build (all on the caller's stream, no host synchronisation):
//  1. k_jcount       count build rows that pass the predicates with a non-NULL key
//  2. k_jinit        size the table on the device from that count
//                    (cap = ceil(count / load factor)) and clear keys and meta
//  3. k_jinsert      CAS the key into the key array; one atomic add on the slot's
//                    meta word records the count and, from the inserting row,
//                    the row; a second inserter of a key marks duplicates.  The
//                    inserting row also zeroes the slot's accumulator words.
//  4. duplicates only (every kernel below returns at once otherwise):
//     k_jdup_scan    exclusive scan of slot counts -> start of each key's run
//     k_jdup_fill    place every build row in its key's run (atomic cursor)
//     k_jdup_sort    sort each run by row: short runs in one thread, long runs
//                    by a block-wide merge sort, so runs hold ascending rows
//  5. k_jpack        copy keys and meta side by side (the probe's layout)
// Probe: per probe row, the match count from the table, a decoupled look-back
// scan of the counts, then (probe row, build row) pairs in canonical order.
// Each thread issues the first probe of all its rows before resolving any of
// them, so the random reads of a thread overlap; a probe step is one 16-byte
// load of a (key, meta) pair.
#include <vector>

#include "agg.h"
#include "radix.h"

namespace gq {
namespace {

constexpr int kJBlock = 256;
constexpr int kJItems = 8;
constexpr int kShortRun = 32;

struct JoinBuildArgs {
  int64_t n;
  DCol key;
  int32_t npreds;
  int32_t lf_milli;  // load factor * 1000
  DPred preds[GQ_MAX_PREDS];
  DCol pcols[GQ_MAX_PREDS];
  JoinHdr* hdr;
  uint64_t* keys;
  uint64_t* meta;
  uint64_t* acc;
  int32_t* rows;
  uint32_t* aux;
  int32_t* tmp;
  uint64_t cap_alloc;
  int32_t acc_slots;
  int32_t pad;
  int32_t* dev_status;
  const int64_t* d_n;     // device row count (NULL: n); n is then an upper bound
  int32_t key_hashed;     // the key column holds (region hash, row) pairs of a partitioned table
  int32_t pad2;
};

__device__ __forceinline__ int64_t jb_rows(const JoinBuildArgs& a) {
  if (!a.d_n) return a.n;
  const int64_t d = *a.d_n;
  return d < a.n ? d : a.n;
}
__device__ __forceinline__ int64_t jb_row(const JoinBuildArgs& a, int64_t r) {
  if (a.key_hashed) return (int64_t)reinterpret_cast<const uint64_t*>(a.key.data)[2 * r + 1];
  return r;
}

// Keep mask of rows r0..r0+ITEMS-1 (predicates and a non-NULL key); key values.
template <int ITEMS>
__device__ __forceinline__ uint32_t build_rows_keep(const JoinBuildArgs& a, int64_t r0, int64_t (&key)[ITEMS]) {
  const int64_t n = jb_rows(a);
  uint32_t keep = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (r0 + k < n) keep |= 1u << k;
  for (int p = 0; p < a.npreds; ++p) {
    int64_t v[ITEMS];
    load_items<ITEMS, true>(a.pcols[p], r0, n, v);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (!pred_pass(a.preds[p], v[k])) keep &= ~(1u << k);
    if (a.pcols[p].valid) keep &= valid_items<ITEMS>(a.pcols[p], r0, n);
  }
  if (a.key_hashed) {
    const uint64_t* kr = reinterpret_cast<const uint64_t*>(a.key.data);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) key[k] = r0 + k < n ? (int64_t)region_unhash(kr[2 * (r0 + k)]) : 0;
    return keep;
  }
  load_items<ITEMS, true>(a.key, r0, n, key);
  if (a.key.valid) keep &= valid_items<ITEMS>(a.key, r0, n);
  return keep;
}

__global__ void k_jhdr_init(JoinHdr* hdr) {
  if (threadIdx.x == 0) {
    hdr->cap = 0;
    hdr->nrows = 0;
    hdr->has_dups = 0;
    hdr->full = 0;
    hdr->nlong = 0;
  }
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_jcount(const JoinBuildArgs a) {
  __shared__ uint32_t s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const int64_t r0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * ITEMS;
  uint32_t keep = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (r0 + k < a.n) keep |= 1u << k;
  for (int p = 0; p < a.npreds; ++p) {
    int64_t v[ITEMS];
    load_items<ITEMS>(a.pcols[p], r0, a.n, v);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (!pred_pass(a.preds[p], v[k])) keep &= ~(1u << k);
    if (a.pcols[p].valid) keep &= valid_items<ITEMS>(a.pcols[p], r0, a.n);
  }
  if (a.key.valid) keep &= valid_items<ITEMS>(a.key, r0, a.n);
  uint32_t tot;
  wave_prefix_small<5>((uint32_t)__popc(keep), &tot);
  if ((threadIdx.x & (kWave - 1)) == 0 && tot) atomicAdd(&s_cnt, tot);
  __syncthreads();
  if (threadIdx.x == 0 && s_cnt) atomicAdd((unsigned long long*)&a.hdr->nrows, (unsigned long long)s_cnt);
}

__device__ __forceinline__ uint64_t cap_for(int64_t n, int lf_milli, uint64_t cap_alloc) {
  uint64_t c = ((uint64_t)n * 1000 + lf_milli - 1) / (uint64_t)lf_milli;
  if (c < 1) c = 1;
  if (c > cap_alloc) c = cap_alloc;
  return c;
}

// Clear keys and meta of slots [0, cap) and of the extra slot (index
// cap_alloc), plus the extra slot's accumulators.
__global__ void k_jinit(const JoinBuildArgs a) {
  const uint64_t cap = cap_for(a.hdr->nrows, a.lf_milli, a.cap_alloc);
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i0 == 0) {
    a.hdr->cap = cap;
    a.keys[a.cap_alloc] = kEmpty;
    a.meta[a.cap_alloc] = 0;
    for (int w = 0; w < a.acc_slots; ++w) a.acc[a.cap_alloc * a.acc_slots + w] = 0;
  }
  for (int64_t i = i0; i < (int64_t)cap; i += stride) {
    a.keys[i] = kEmpty;
    a.meta[i] = 0;
  }
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_jinsert(const JoinBuildArgs a) {
  const int64_t r0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * ITEMS;
  int64_t key[ITEMS];
  const uint32_t keep = build_rows_keep<ITEMS>(a, r0, key);
  if (!keep) return;
  const uint64_t cap = a.hdr->cap;
  uint64_t start[ITEMS], first[ITEMS];
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    start[k] = slot_of((uint64_t)key[k], cap);
    first[k] = ((keep >> k) & 1u) ? a.keys[start[k]] : kEmpty;
  });
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    if (!((keep >> k) & 1u)) return;
    const uint64_t kv = (uint64_t)key[k];
    const uint64_t row = (uint64_t)jb_row(a, r0 + k);
    int64_t s;
    bool inserted = false;
    if (kv == kEmpty) {
      s = (int64_t)a.cap_alloc;
    } else {
      s = find_insert_from(a.keys, cap, kv, start[k], opaque_copy(first[k]), &inserted);
      if (s < 0) {
        a.hdr->full = 1;
        atomicOr(a.dev_status, GQ_DEV_TABLE_FULL);
        return;
      }
    }
    if (inserted) {
      for (int w = 0; w < a.acc_slots; ++w) a.acc[(uint64_t)s * a.acc_slots + w] = 0;
      // Count and row in one atomic.  Another inserter of the same key may have
      // landed first; then the row sum is meaningless, but duplicates are
      // flagged and the run construction below rewrites the word.
      const uint64_t old = atomicAdd((unsigned long long*)&a.meta[s], (1ull << 32) | row);
      if (meta_count(old) != 0) a.hdr->has_dups = 1;
    } else {
      // An existing key (or the extra slot): the first to arrive records its row.
      const uint64_t old = atomicAdd((unsigned long long*)&a.meta[s], 1ull << 32);
      if (meta_count(old) == 0)
        atomicAdd((unsigned long long*)&a.meta[s], row);
      else
        a.hdr->has_dups = 1;
    }
  });
}

// kv[2s], kv[2s+1] = keys[s], meta[s] for the hashed slots [0, cap) and the
// extra slot (index cap_alloc), once meta holds its final count and row.
__global__ void k_jpack(const JoinBuildArgs a, uint64_t* kv) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  const uint64_t cap = a.hdr->cap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= (int64_t)a.cap_alloc; i += stride) {
    if ((uint64_t)i >= cap && (uint64_t)i != a.cap_alloc) continue;
    *reinterpret_cast<u64x2*>(kv + 2 * i) = u64x2{a.keys[i], a.meta[i]};
  }
}

// Exclusive scan of slot counts over [0, cap) and the extra slot (entry cap).
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_jdup_scan(const JoinBuildArgs a, uint32_t* ticket, uint64_t* status) {
  if (!a.hdr->has_dups) return;
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t s_tile;
  __shared__ int64_t s_wave[NW];
  __shared__ int64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const uint64_t cap = a.hdr->cap;
  const int64_t i0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;
  uint32_t c[ITEMS];
  int64_t tsum = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t i = i0 + k;
    c[k] = 0;
    if (i <= (int64_t)cap) {
      const uint64_t s = (i == (int64_t)cap) ? a.cap_alloc : (uint64_t)i;
      if (s == a.cap_alloc || a.keys[s] != kEmpty) c[k] = meta_count(a.meta[s]);
    }
    tsum += c[k];
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int64_t incl = tsum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int64_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  int64_t bpre = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wave) bpre += s_wave[w];
    btot += s_wave[w];
  }
  if (wave == 0) {
    int64_t e = lookback_exclusive(status, tile, btot);
    if (lane == 0) s_excl = e;
  }
  __syncthreads();
  int64_t run = s_excl + bpre + incl - tsum;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t i = i0 + k;
    if (i <= (int64_t)cap && c[k] > 0) {
      const uint64_t s = (i == (int64_t)cap) ? a.cap_alloc : (uint64_t)i;
      a.meta[s] = ((uint64_t)c[k] << 32) | (uint64_t)(uint32_t)run;  // run start replaces the row
      a.aux[s == a.cap_alloc ? cap : s] = (uint32_t)run;             // fill cursor
    }
    run += c[k];
  }
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_jdup_fill(const JoinBuildArgs a) {
  if (!a.hdr->has_dups) return;
  const int64_t r0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * ITEMS;
  int64_t key[ITEMS];
  const uint32_t keep = build_rows_keep<ITEMS>(a, r0, key);
  const uint64_t cap = a.hdr->cap;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    if (!((keep >> k) & 1u)) continue;
    const uint64_t kv = (uint64_t)key[k];
    uint64_t idx;
    if (kv == kEmpty) {
      idx = cap;
    } else {
      const int64_t s = find(a.keys, cap, kv);
      if (s < 0) continue;  // only after a full table, already reported
      idx = (uint64_t)s;
    }
    const uint32_t pos = atomicAdd(&a.aux[idx], 1u);
    a.rows[pos] = (int32_t)jb_row(a, r0 + k);
  }
}

// Short runs: insertion sort by one thread.  Long runs go to a list in aux.
__global__ void k_jdup_sort(const JoinBuildArgs a) {
  if (!a.hdr->has_dups) return;
  const uint64_t cap = a.hdr->cap;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i <= (int64_t)cap; i += stride) {
    const uint64_t s = (i == (int64_t)cap) ? a.cap_alloc : (uint64_t)i;
    if (s != a.cap_alloc && a.keys[s] == kEmpty) continue;
    const uint64_t m = a.meta[s];
    const uint32_t cnt = meta_count(m);
    if (cnt < 2) continue;
    int32_t* r = a.rows + meta_row(m);
    if (cnt <= (uint32_t)kShortRun) {
      for (uint32_t x = 1; x < cnt; ++x) {
        const int32_t v = r[x];
        int32_t y = (int32_t)x - 1;
        while (y >= 0 && r[y] > v) {
          r[y + 1] = r[y];
          --y;
        }
        r[y + 1] = v;
      }
    } else {
      const unsigned long long pos = atomicAdd((unsigned long long*)&a.hdr->nlong, 1ull);
      a.aux[pos] = (uint32_t)s;
    }
  }
}

// Long runs: one block per run, bottom-up merge sort between the run and tmp.
// Each element finds its output place by binary search in the other half.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_jdup_sort_long(const JoinBuildArgs a) {
  if (!a.hdr->has_dups) return;
  const int64_t nlong = a.hdr->nlong;
  for (int64_t li = blockIdx.x; li < nlong; li += gridDim.x) {
    const uint64_t m = a.meta[a.aux[li]];
    const uint32_t cnt = meta_count(m);
    const uint32_t start = meta_row(m);
    int32_t* src = a.rows + start;
    int32_t* dst = a.tmp + start;
    for (uint32_t w = 1; w < cnt; w <<= 1) {
      for (uint32_t i = threadIdx.x; i < cnt; i += BLOCK) {
        const uint32_t blk = i / (2 * w);
        const uint32_t lo = blk * 2 * w;
        const uint32_t mid = lo + w < cnt ? lo + w : cnt;
        const uint32_t hi = lo + 2 * w < cnt ? lo + 2 * w : cnt;
        const int32_t v = src[i];
        uint32_t pos;
        if (i < mid) {
          uint32_t l = mid, h = hi;  // right-half elements smaller than v
          while (l < h) {
            const uint32_t q = (l + h) >> 1;
            if (src[q] < v) l = q + 1; else h = q;
          }
          pos = lo + (i - lo) + (l - mid);
        } else {
          uint32_t l = lo, h = mid;  // left-half elements smaller than v
          while (l < h) {
            const uint32_t q = (l + h) >> 1;
            if (src[q] < v) l = q + 1; else h = q;
          }
          pos = lo + (i - mid) + (l - lo);
        }
        dst[pos] = v;
      }
      __syncthreads();
      int32_t* t = src;
      src = dst;
      dst = t;
    }
    if (src != a.rows + start) {
      for (uint32_t i = threadIdx.x; i < cnt; i += BLOCK) dst[i] = src[i];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Probe
// ---------------------------------------------------------------------------
struct ProbeArgs {
  int64_t n;
  int64_t ntiles;
  int64_t out_cap;
  DCol key;
  int32_t npreds;
  int32_t pad;
  DPred preds[GQ_MAX_PREDS];
  DCol pcols[GQ_MAX_PREDS];
  const JoinHdr* hdr;
  const uint64_t* kv;       // (key, meta) pairs
  const int32_t* rows;
  uint64_t cap_alloc;
  int32_t* probe_idx;
  int32_t* build_idx;
  uint32_t* ticket;
  uint64_t* status;
  int64_t* d_count;
  int32_t* dev_status;
};

__global__ void k_probe_init(uint32_t* ticket, uint64_t* status, int64_t ntiles, int64_t* d_count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i == 0) {
    *ticket = 0;
    *d_count = 0;
  }
  for (; i < ntiles; i += stride) status[i] = 0;
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_jprobe(const ProbeArgs a) {
  constexpr int NW = BLOCK / kWave;
  constexpr int TILE = BLOCK * ITEMS;
  __shared__ uint32_t s_tile;
  __shared__ int64_t s_wave[NW];
  __shared__ int64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(a.ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t r0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;

  uint32_t keep = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (r0 + k < a.n) keep |= 1u << k;
  for (int p = 0; p < a.npreds; ++p) {
    int64_t v[ITEMS];
    load_items<ITEMS, true>(a.pcols[p], r0, a.n, v);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (!pred_pass(a.preds[p], v[k])) keep &= ~(1u << k);
    if (a.pcols[p].valid) keep &= valid_items<ITEMS>(a.pcols[p], r0, a.n);
  }
  int64_t key[ITEMS];
  load_items<ITEMS, true>(a.key, r0, a.n, key);
  if (a.key.valid) keep &= valid_items<ITEMS>(a.key, r0, a.n);

  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  const uint64_t cap = a.hdr->cap;
  const bool dups = a.hdr->has_dups != 0;
  const u64x2* kv = reinterpret_cast<const u64x2*>(a.kv);
  // First probe of every row (the key EMPTY lives in the extra slot).
  uint64_t pos0[ITEMS];
  u64x2 e[ITEMS];
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    pos0[k] = (uint64_t)key[k] == kEmpty ? a.cap_alloc : slot_of((uint64_t)key[k], cap);
    e[k] = ((keep >> k) & 1u) ? kv[pos0[k]] : u64x2{kEmpty, 0};
  });
  uint32_t cnt[ITEMS], srow[ITEMS];
  int64_t tsum = 0;
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    cnt[k] = 0;
    srow[k] = 0;
    if ((keep >> k) & 1u) {
      const uint64_t kx = (uint64_t)key[k];
      uint64_t meta = 0;
      if (kx == kEmpty) {
        meta = opaque_copy(e[k].y);
      } else {
        // Linear probing from the home slot: a hit gives the meta word with
        // the key; an empty slot ends the search.
        uint64_t s = pos0[k];
        u64x2 x = u64x2{opaque_copy(e[k].x), opaque_copy(e[k].y)};
        for (uint64_t n = 0; n < cap; ++n) {
          if (x.x == kx) {
            meta = x.y;
            break;
          }
          if (x.x == kEmpty) break;
          if (++s == cap) s = 0;
          x = kv[s];
        }
      }
      cnt[k] = meta_count(meta);
      srow[k] = meta_row(meta);
    }
    tsum += cnt[k];
  });
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int64_t incl = tsum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int64_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  int64_t bpre = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wave) bpre += s_wave[w];
    btot += s_wave[w];
  }
  if (wave == 0) {
    int64_t e = lookback_exclusive(a.status, tile, btot);
    if (lane == 0) s_excl = e;
  }
  __syncthreads();
  if (tile == a.ntiles - 1 && threadIdx.x == 0) {
    const int64_t total = s_excl + btot;
    *a.d_count = total;
    if (total > a.out_cap) atomicOr(a.dev_status, GQ_DEV_CAPACITY);
  }
  int64_t pos = s_excl + bpre + incl - tsum;
  static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
    constexpr int k = decltype(kk)::value;
    for (uint32_t j = 0; j < cnt[k]; ++j, ++pos) {
      if (pos >= a.out_cap) break;
      a.probe_idx[pos] = (int32_t)(r0 + k);
      a.build_idx[pos] = dups ? a.rows[srow[k] + j] : (int32_t)srow[k];
    }
  });
}

// ---------------------------------------------------------------------------
// Gather
// ---------------------------------------------------------------------------
struct GatherArgs {
  int64_t n;
  int32_t ncols;
  int32_t pad;
  const int32_t* idx;
  const int64_t* d_n;      // if set: only the first min(n, *d_n) rows (a device count)
  DCol cols[GQ_MAX_COLS];
  OCol out[GQ_MAX_COLS];
};

__global__ void k_gather(GatherArgs a) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (a.d_n && *a.d_n < a.n) a.n = *a.d_n > 0 ? *a.d_n : 0;
  for (int64_t r = i0; r < a.n; r += stride) {
    const int64_t src = a.idx[r];
    for (int j = 0; j < a.ncols; ++j) {
      const int64_t v = load_one(a.cols[j], src);
      switch (a.out[j].type) {
        case GQ_I8: a.out[j].data[r] = (uint8_t)v; break;
        case GQ_I16: reinterpret_cast<int16_t*>(a.out[j].data)[r] = (int16_t)v; break;
        case GQ_I32: reinterpret_cast<int32_t*>(a.out[j].data)[r] = (int32_t)v; break;
        default: reinterpret_cast<int64_t*>(a.out[j].data)[r] = v; break;
      }
    }
  }
  // Validity: one thread per 32-row output word.
  const int64_t nwords = (a.n + 31) / 32;
  for (int64_t w = i0; w < nwords; w += stride) {
    for (int j = 0; j < a.ncols; ++j) {
      if (!a.out[j].valid) continue;
      uint32_t bits = 0;
      for (int b = 0; b < 32; ++b) {
        const int64_t r = w * 32 + b;
        if (r < a.n && valid_one(a.cols[j], a.idx[r])) bits |= 1u << b;
      }
      a.out[j].valid[w] = bits;
    }
  }
}

int fill_build_args(gq_ctx* ctx, JoinBuildArgs& a, const gq_batch* b, const int32_t* keys, int nkeys,
                    const gq_pred* preds, int npreds) {
  if (nkeys != 1 || !keys)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "join: exactly one key column is supported");
  if (keys[0] < 0 || keys[0] >= b->ncols) return set_error(ctx, GQ_ERR_INVALID, "join: key column out of range");
  if (npreds < 0 || npreds > GQ_MAX_PREDS || (npreds > 0 && !preds))
    return set_error(ctx, GQ_ERR_INVALID, "join: bad predicate list");
  a.n = b->nrows;
  a.key = make_dcol(b->cols[keys[0]]);
  a.npreds = npreds;
  for (int p = 0; p < npreds; ++p) {
    if (preds[p].col < 0 || preds[p].col >= b->ncols)
      return set_error(ctx, GQ_ERR_INVALID, "join: predicate column out of range");
    if (preds[p].op != GQ_RANGE && preds[p].op != GQ_NE)
      return set_error(ctx, GQ_ERR_INVALID, "join: unknown predicate op");
    a.preds[p] = DPred{preds[p].col, preds[p].op, preds[p].lo, preds[p].hi};
    a.pcols[p] = make_dcol(b->cols[preds[p].col]);
  }
  return GQ_OK;
}

// Probe index (keys/meta, and rows for duplicate keys) of t from the rows
// described by a: the build input itself (count = true: count the kept rows
// first), or the partitioned kept rows of a large build input.
int build_index(gq_ctx* ctx, JoinBuildArgs& a, gq_join_table* t, bool count, hipStream_t stream) {
  a.hdr = t->hdr;
  a.keys = t->keys;
  a.meta = t->meta;
  a.acc = t->acc;
  a.rows = t->rows;
  a.aux = t->aux;
  a.tmp = t->tmp;
  a.cap_alloc = t->cap_alloc;
  a.acc_slots = t->acc_slots;
  a.lf_milli = t->lf_milli;
  a.dev_status = ctx->d_status;
  constexpr int TILE = kJBlock * kJItems;
  const int64_t nblk = (a.n + TILE - 1) / TILE;
  if (count && nblk > 0) {
    GQ_LAUNCH(ctx, "jcount", (k_jcount<kJBlock, kJItems>), dim3((unsigned)nblk), dim3(kJBlock), 0, stream, a);
    GQ_LAUNCH_CHECK(ctx);
  }
  int64_t iblocks = (int64_t)((t->cap_alloc + 1 + 255) / 256);
  if (iblocks > 8192) iblocks = 8192;
  GQ_LAUNCH(ctx, "jinit", k_jinit, dim3((unsigned)iblocks), dim3(256), 0, stream, a);
  GQ_LAUNCH_CHECK(ctx);
  if (nblk > 0) {
    GQ_LAUNCH(ctx, "jinsert", (k_jinsert<kJBlock, kJItems>), dim3((unsigned)nblk), dim3(kJBlock), 0, stream, a);
    GQ_LAUNCH_CHECK(ctx);
    // Duplicate handling (kernels return at once when every key is unique).
    constexpr int STILE = 256 * 16;
    const int64_t nscan = (int64_t)((t->cap_alloc + 1 + STILE - 1) / STILE);
    Scratch ws(ctx, stream);
    if (!ws.get(256 + align_up((size_t)nscan * 8, 256)))
      return set_error(ctx, GQ_ERR_NOMEM, "join: index workspace allocation failed");
    int rc = launch_fill_u32(ctx, ws.p, 0u, 64 + 2 * nscan, stream);
    if (rc) return rc;
    GQ_LAUNCH(ctx, "jdup_scan", (k_jdup_scan<256, 16>), dim3((unsigned)nscan), dim3(256), 0, stream, a,
              ws.as<uint32_t>(0), ws.as<uint64_t>(256));
    GQ_LAUNCH_CHECK(ctx);
    GQ_LAUNCH(ctx, "jdup_fill", (k_jdup_fill<kJBlock, kJItems>), dim3((unsigned)nblk), dim3(kJBlock), 0, stream, a);
    GQ_LAUNCH_CHECK(ctx);
    GQ_LAUNCH(ctx, "jdup_sort", k_jdup_sort, dim3((unsigned)iblocks), dim3(256), 0, stream, a);
    GQ_LAUNCH_CHECK(ctx);
    GQ_LAUNCH(ctx, "jdup_sort_long", (k_jdup_sort_long<1024>), dim3(64), dim3(1024), 0, stream, a);
    GQ_LAUNCH_CHECK(ctx);
  }
  GQ_LAUNCH(ctx, "jpack", k_jpack, dim3((unsigned)iblocks), dim3(256), 0, stream, a, t->kv);
  GQ_LAUNCH_CHECK(ctx);
  t->index_built = true;
  return GQ_OK;
}

}  // namespace

// Probe index arrays of a table: keys and meta (cap_alloc + 1 slots), the
// accumulators of a fused group-join, build rows, fill cursors and the merge
// buffer, in one block.
struct IndexLayout {
  size_t meta, kv, acc, rows, aux, tmp, bytes;
};
IndexLayout index_layout(uint64_t cap_alloc, int64_t n, int acc) {
  const size_t nslot = (size_t)cap_alloc + 1;
  IndexLayout l;
  l.meta = align_up(nslot * 8, 256);
  l.kv = align_up(l.meta + nslot * 8, 256);
  l.acc = align_up(l.kv + nslot * 16, 256);
  l.rows = align_up(l.acc + nslot * 8 * (size_t)acc, 256);
  l.aux = align_up(l.rows + (size_t)n * 4, 256);
  l.tmp = align_up(l.aux + nslot * 4, 256);
  l.bytes = align_up(l.tmp + (size_t)n * 4, 256);
  return l;
}
void set_index(gq_join_table* t, char* base, const IndexLayout& l, int acc) {
  t->keys = reinterpret_cast<uint64_t*>(base);
  t->meta = reinterpret_cast<uint64_t*>(base + l.meta);
  t->kv = reinterpret_cast<uint64_t*>(base + l.kv);
  t->acc = acc ? reinterpret_cast<uint64_t*>(base + l.acc) : nullptr;
  t->rows = reinterpret_cast<int32_t*>(base + l.rows);
  t->aux = reinterpret_cast<uint32_t*>(base + l.aux);
  t->tmp = reinterpret_cast<int32_t*>(base + l.tmp);
}

int join_wait_ready(gq_ctx* ctx, const gq_join_table* t, hipStream_t stream) {
  if (t && t->ready) GQ_HIP_CHECK(ctx, hipStreamWaitEvent(stream, t->ready, 0));
  return GQ_OK;
}

int join_ensure_index(gq_ctx* ctx, const gq_join_table* table, hipStream_t stream) {
  gq_join_table* t = const_cast<gq_join_table*>(table);
  int rc = join_wait_ready(ctx, t, stream);
  if (rc) return rc;
  if (t->index_built) return GQ_OK;
  if (!t->keys) {
    // Allocated through the table's own context, which also frees it.
    const IndexLayout il = index_layout(t->cap_alloc, t->build_rows, t->acc_slots);
    t->imem = ctx_alloc(t->ctx ? t->ctx : ctx, il.bytes, stream);
    if (!t->imem) return set_error(ctx, GQ_ERR_NOMEM, "join: probe index allocation failed");
    t->ibytes = il.bytes;
    set_index(t, static_cast<char*>(t->imem), il, t->acc_slots);
  }
  JoinBuildArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = t->build_rows;
  a.key.data = reinterpret_cast<const uint8_t*>(t->rj_kr);
  a.key.type = GQ_I64;
  a.key.align = 16;
  a.npreds = 0;
  a.d_n = &t->hdr->nrows;
  a.key_hashed = 1;
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  rc = build_index(ctx, a, t, false, stream);
  if (rc) return rc;
  // Readers on other streams wait for the table's ready event: from now on
  // it also covers the index built here.
  if (t->ready) GQ_HIP_CHECK(ctx, hipEventRecord(t->ready, stream));
  return GQ_OK;
}

// Gather of gq_gather; with d_n, only rows below the device count *d_n.
int gather_rows(gq_ctx* ctx, const gq_batch* in, const int32_t* cols, int ncols, const int32_t* idx, int64_t n,
                const int64_t* d_n, gq_batch* out, hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_gather input");
  if (rc) return rc;
  if (ncols < 0 || ncols > GQ_MAX_COLS || (ncols > 0 && !cols) || n < 0 || (n > 0 && !idx) || !out ||
      out->ncols < ncols)
    return set_error(ctx, GQ_ERR_INVALID, "gq_gather: bad arguments");
  GatherArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.ncols = ncols;
  a.idx = idx;
  a.d_n = d_n;
  for (int j = 0; j < ncols; ++j) {
    if (cols[j] < 0 || cols[j] >= in->ncols) return set_error(ctx, GQ_ERR_INVALID, "gq_gather: column out of range");
    const gq_column& ic = in->cols[cols[j]];
    const gq_column& oc = out->cols[j];
    if (oc.type != ic.type || oc.length < n || (n > 0 && !oc.data))
      return set_error(ctx, GQ_ERR_INVALID, "gq_gather: bad output column");
    if (ic.validity && !oc.validity)
      return set_error(ctx, GQ_ERR_INVALID, "gq_gather: nullable input needs an output bitmap");
    if (oc.validity && (reinterpret_cast<uintptr_t>(oc.validity) & 3))
      return set_error(ctx, GQ_ERR_INVALID, "gq_gather: output bitmap must be 4-byte aligned");
    a.cols[j] = make_dcol(ic);
    a.out[j] = OCol{static_cast<uint8_t*>(oc.data), reinterpret_cast<uint32_t*>(oc.validity), oc.type, 0};
  }
  if (n == 0 || ncols == 0) return GQ_OK;
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  GQ_LAUNCH(ctx, "gather", k_gather, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

// Composite join keys.  The key columns of a row are packed into one 64-bit
// word, first column most significant, each field as wide as the build
// side's column type (the value's low bits, two's complement), so two rows'
// words are equal exactly when every key column is.  A row with a NULL key
// column, or a probe value that does not fit its field (it cannot equal any
// build value), gets a NULL word and matches nothing.  The tables and kernels
// of the single-key join then run on that word.
struct JKeyPack {
  int32_t nk;
  int32_t shift[GQ_MAX_KEYS];
  int32_t bits[GQ_MAX_KEYS];
  DCol cols[GQ_MAX_KEYS];
};

constexpr int kJPackBlock = 256;

__global__ __launch_bounds__(kJPackBlock) void k_jpack_keys(const JKeyPack p, int64_t n, int64_t* out,
                                                           uint32_t* valid) {
  const int64_t r = (int64_t)blockIdx.x * kJPackBlock + threadIdx.x;
  bool ok = r < n;
  uint64_t key = 0;
  for (int j = 0; j < p.nk && ok; ++j) {
    const DCol& c = p.cols[j];
    if (!valid_one(c, r)) {
      ok = false;
      break;
    }
    const int64_t v = load_one(c, r);
    const int w = p.bits[j];
    if (w < 64 && (v < -(1ll << (w - 1)) || v > (1ll << (w - 1)) - 1)) {
      ok = false;
      break;
    }
    const uint64_t mask = w == 64 ? ~0ull : (1ull << w) - 1;
    key |= ((uint64_t)v & mask) << p.shift[j];
  }
  // Rows r..r+31 of a 32-aligned group give one validity word (every lane
  // takes part in the ballot).
  const uint64_t m = ballot(ok);
  if (r < n) {
    out[r] = ok ? (int64_t)key : 0;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    if ((lane & 31) == 0) valid[r >> 5] = (uint32_t)(m >> lane);
  }
}

// Field layout of the key columns `types` (the build side's): widths of the
// types, first column most significant.  False if they need more than 64 bits.
bool jkey_layout(const int32_t* types, int nk, JKeyPack& p) {
  int total = 0;
  for (int j = 0; j < nk; ++j) total += 8 * type_width(types[j]);
  if (total > 64) return false;
  p.nk = nk;
  int sh = total;
  for (int j = 0; j < nk; ++j) {
    p.bits[j] = 8 * type_width(types[j]);
    sh -= p.bits[j];
    p.shift[j] = sh;
  }
  return true;
}

// The batch `b` with one more column: the packed key words of its columns
// keys[0..nk) in the layout of `types`, in workspace memory of `ws`.  `cols`
// receives the column list of the new batch (ncols + 1 entries).
int jkey_pack_batch(gq_ctx* ctx, const gq_batch* b, const int32_t* keys, int nk, const int32_t* types, Scratch& ws,
                    std::vector<gq_column>& cols, gq_batch& packed, hipStream_t stream) {
  JKeyPack p;
  std::memset(&p, 0, sizeof(p));
  if (!jkey_layout(types, nk, p))
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "join: the key columns need more than 64 bits together");
  for (int j = 0; j < nk; ++j) {
    if (keys[j] < 0 || keys[j] >= b->ncols) return set_error(ctx, GQ_ERR_INVALID, "join: key column out of range");
    p.cols[j] = make_dcol(b->cols[keys[j]]);
  }
  const int64_t n = b->nrows;
  const size_t vbytes = align_up((size_t)((n + 31) / 32) * 4, 256);
  if (!ws.get(vbytes + align_up((size_t)n * 8, 256)))
    return set_error(ctx, GQ_ERR_NOMEM, "join: key packing workspace allocation failed");
  uint32_t* valid = ws.as<uint32_t>(0);
  int64_t* words = ws.as<int64_t>(vbytes);
  if (n > 0) {
    GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    GQ_LAUNCH(ctx, "jpack_keys", k_jpack_keys, dim3((unsigned)((n + kJPackBlock - 1) / kJPackBlock)),
              dim3(kJPackBlock), 0, stream, p, n, words, valid);
    GQ_LAUNCH_CHECK(ctx);
  }
  cols.assign(b->cols, b->cols + b->ncols);
  gq_column c;
  std::memset(&c, 0, sizeof(c));
  c.type = GQ_I64;
  c.length = n;
  c.offset = 0;
  c.data = words;
  c.validity = reinterpret_cast<uint8_t*>(valid);
  cols.push_back(c);
  packed = *b;
  packed.ncols = b->ncols + 1;
  packed.cols = cols.data();
  return GQ_OK;
}

int join_build_one(gq_ctx* ctx, const gq_batch* build, const int32_t* keys, int nkeys, const gq_pred* preds,
                   int npreds, const gq_join_opts* opts, hipStream_t stream, gq_join_table** out);
int join_probe_one(gq_ctx* ctx, const gq_join_table* table, const gq_batch* probe, const int32_t* keys, int nkeys,
                   const gq_pred* preds, int npreds, int32_t* probe_idx, int32_t* build_idx, int64_t out_cap,
                   int64_t* d_count, hipStream_t stream);

}  // namespace gq

using namespace gq;

extern "C" {

int gq_join_build(gq_ctx* ctx, const gq_batch* build, const int32_t* keys, int nkeys, const gq_pred* preds,
                  int npreds, const gq_join_opts* opts, hipStream_t stream, gq_join_table** out) {
  if (!ctx || !out) return GQ_ERR_INVALID;
  *out = nullptr;
  if (nkeys <= 1 || !keys) return join_build_one(ctx, build, keys, nkeys, preds, npreds, opts, stream, out);
  if (nkeys > GQ_MAX_KEYS) return set_error(ctx, GQ_ERR_UNSUPPORTED, "gq_join_build: more than GQ_MAX_KEYS key columns");
  int rc = check_batch(ctx, build, "gq_join_build input");
  if (rc) return rc;
  int32_t types[GQ_MAX_KEYS];
  for (int j = 0; j < nkeys; ++j) {
    if (keys[j] < 0 || keys[j] >= build->ncols) return set_error(ctx, GQ_ERR_INVALID, "join: key column out of range");
    types[j] = build->cols[keys[j]].type;
  }
  Scratch ws(ctx, stream);
  std::vector<gq_column> cols;
  gq_batch packed;
  rc = jkey_pack_batch(ctx, build, keys, nkeys, types, ws, cols, packed, stream);
  if (rc) return rc;
  const int32_t kp = build->ncols;
  rc = join_build_one(ctx, &packed, &kp, 1, preds, npreds, opts, stream, out);
  if (rc) return rc;
  (*out)->nkeys = nkeys;
  for (int j = 0; j < nkeys; ++j) (*out)->key_types[j] = types[j];
  return GQ_OK;
}

int gq_join_probe(gq_ctx* ctx, const gq_join_table* table, const gq_batch* probe, const int32_t* keys, int nkeys,
                  const gq_pred* preds, int npreds, int32_t* probe_idx, int32_t* build_idx, int64_t out_cap,
                  int64_t* d_count, hipStream_t stream) {
  if (!ctx || !table) return GQ_ERR_INVALID;
  if (nkeys != table->nkeys || !keys)
    return set_error(ctx, GQ_ERR_INVALID, "gq_join_probe: the key count differs from the table's");
  if (nkeys == 1)
    return join_probe_one(ctx, table, probe, keys, 1, preds, npreds, probe_idx, build_idx, out_cap, d_count, stream);
  int rc = check_batch(ctx, probe, "gq_join_probe input");
  if (rc) return rc;
  Scratch ws(ctx, stream);
  std::vector<gq_column> cols;
  gq_batch packed;
  rc = jkey_pack_batch(ctx, probe, keys, nkeys, table->key_types, ws, cols, packed, stream);
  if (rc) return rc;
  const int32_t kp = probe->ncols;
  return join_probe_one(ctx, table, &packed, &kp, 1, preds, npreds, probe_idx, build_idx, out_cap, d_count, stream);
}

}  // extern "C"

namespace gq {

int join_build_one(gq_ctx* ctx, const gq_batch* build, const int32_t* keys, int nkeys, const gq_pred* preds,
                   int npreds, const gq_join_opts* opts, hipStream_t stream, gq_join_table** out) {
  if (!ctx || !out) return GQ_ERR_INVALID;
  *out = nullptr;
  int rc = check_batch(ctx, build, "gq_join_build input");
  if (rc) return rc;
  JoinBuildArgs a;
  std::memset(&a, 0, sizeof(a));
  rc = fill_build_args(ctx, a, build, keys, nkeys, preds, npreds);
  if (rc) return rc;
  float lf = opts && opts->load_factor > 0.f ? opts->load_factor : 0.5f;
  if (!(lf > 0.f && lf <= 0.9f)) return set_error(ctx, GQ_ERR_INVALID, "gq_join_build: load factor outside (0, 0.9]");
  const int acc = opts ? opts->acc_slots : 0;
  if (acc != 0 && acc != 2 && acc != 6)
    return set_error(ctx, GQ_ERR_INVALID, "gq_join_build: acc_slots must be 0, 2 or 6");
  a.lf_milli = (int)(lf * 1000.f + 0.5f);
  if (a.lf_milli < 1) a.lf_milli = 1;
  const int64_t n = build->nrows;
  uint64_t cap_alloc = ((uint64_t)n * 1000 + a.lf_milli - 1) / (uint64_t)a.lf_milli;
  if (cap_alloc < 1) cap_alloc = 1;
  a.cap_alloc = cap_alloc;
  a.acc_slots = acc;
  // Large build inputs are partitioned by region (radix group-join); their
  // probe index is built from the partitioned rows when first needed.
  const int rlog = opts ? opts->regions_log2 : 0;
  if (rlog != 0 && (rlog < 4 || rlog > 12))
    return set_error(ctx, GQ_ERR_INVALID, "gq_join_build: regions_log2 must be 0 or in [4, 12]");
  const int pbits = rlog ? rlog : rj_choose_pbits(n);
  const bool radix = n >= kRjMinBuild && n < ((int64_t)1 << 31) && rj_build_fits(build, keys[0], preds, npreds, pbits);

  // Partitioned tables allocate their probe index (keys ... tmp) on first use.
  const size_t off_keys = 256;
  IndexLayout il = index_layout(cap_alloc, n, acc);
  const size_t off_rjkey = radix ? off_keys : align_up(off_keys + il.bytes, 256);
  const size_t off_rjoff = align_up(off_rjkey + (radix ? (size_t)n * 16 : 0), 256);
  const size_t total = align_up(off_rjoff + (radix ? ((size_t)1 << pbits) * 8 + 8 : 0), 256);

  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  gq_join_table* t = new (std::nothrow) gq_join_table;
  if (!t) return GQ_ERR_NOMEM;
  t->ctx = ctx;
  t->mem = ctx_alloc(ctx, total, stream);
  if (!t->mem) {
    delete t;
    return set_error(ctx, GQ_ERR_NOMEM, "gq_join_build: table allocation failed");
  }
  t->bytes = total;
  char* base = static_cast<char*>(t->mem);
  t->hdr = reinterpret_cast<JoinHdr*>(base);
  if (!radix) set_index(t, base + off_keys, il, acc);
  t->cap_alloc = cap_alloc;
  t->acc_slots = acc;
  t->build_rows = n;
  t->key_type = build->cols[keys[0]].type;
  t->device = ctx->device;
  t->lf_milli = a.lf_milli;
  if (radix) {
    t->rj_pbits = pbits;
    t->rj_kr = reinterpret_cast<uint64_t*>(base + off_rjkey);
    t->rj_off = reinterpret_cast<int64_t*>(base + off_rjoff);
  }
  auto fail = [&](int code) {
    gq_join_table_free(ctx, t, stream);
    return code;
  };
  GQ_LAUNCH(ctx, "jhdr_init", k_jhdr_init, dim3(1), dim3(64), 0, stream, t->hdr);
  GQ_LAUNCH_CHECK(ctx);
  if (radix) {
    rc = rj_build(ctx, build, keys[0], preds, npreds, t, stream);
    if (rc) return fail(rc);
    t->index_built = false;
  } else {
    rc = build_index(ctx, a, t, true, stream);
    if (rc) return fail(rc);
  }
  if (hipEventCreateWithFlags(&t->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(t->ready, stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(set_error(ctx, GQ_ERR_HIP, "gq_join_build: event creation failed"));
  }
  *out = t;
  return GQ_OK;
}

int join_probe_one(gq_ctx* ctx, const gq_join_table* table, const gq_batch* probe, const int32_t* keys, int nkeys,
                   const gq_pred* preds, int npreds, int32_t* probe_idx, int32_t* build_idx, int64_t out_cap,
                   int64_t* d_count, hipStream_t stream) {
  if (!ctx || !table) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, probe, "gq_join_probe input");
  if (rc) return rc;
  if (!d_count || out_cap < 0 || (out_cap > 0 && (!probe_idx || !build_idx)))
    return set_error(ctx, GQ_ERR_INVALID, "gq_join_probe: bad output");
  JoinBuildArgs b;
  std::memset(&b, 0, sizeof(b));
  rc = fill_build_args(ctx, b, probe, keys, nkeys, preds, npreds);
  if (rc) return rc;
  ProbeArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = probe->nrows;
  a.out_cap = out_cap;
  a.key = b.key;
  a.npreds = b.npreds;
  for (int p = 0; p < b.npreds; ++p) {
    a.preds[p] = b.preds[p];
    a.pcols[p] = b.pcols[p];
  }
  rc = join_ensure_index(ctx, table, stream);
  if (rc) return rc;
  a.hdr = table->hdr;
  a.kv = table->kv;
  a.rows = table->rows;
  a.cap_alloc = table->cap_alloc;
  a.probe_idx = probe_idx;
  a.build_idx = build_idx;
  a.d_count = d_count;
  a.dev_status = ctx->d_status;
  constexpr int TILE = kJBlock * kJItems;
  const int64_t ntiles = (a.n + TILE - 1) / TILE;
  a.ntiles = ntiles;
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  Scratch ws(ctx, stream);
  if (!ws.get(256 + align_up((size_t)(ntiles > 0 ? ntiles : 1) * 8, 256)))
    return set_error(ctx, GQ_ERR_NOMEM, "gq_join_probe: workspace allocation failed");
  a.ticket = ws.as<uint32_t>(0);
  a.status = ws.as<uint64_t>(256);
  int64_t iblocks = (ntiles + 255) / 256;
  if (iblocks < 1) iblocks = 1;
  if (iblocks > 4096) iblocks = 4096;
  GQ_LAUNCH(ctx, "probe_init", k_probe_init, dim3((unsigned)iblocks), dim3(256), 0, stream, a.ticket, a.status,
            ntiles, d_count);
  GQ_LAUNCH_CHECK(ctx);
  if (ntiles > 0) {
    GQ_LAUNCH(ctx, "jprobe", (k_jprobe<kJBlock, kJItems>), dim3((unsigned)ntiles), dim3(kJBlock), 0, stream, a);
    GQ_LAUNCH_CHECK(ctx);
  }
  return GQ_OK;
}

}  // namespace gq

extern "C" {

const int64_t* gq_join_table_count_ptr(const gq_join_table* table) {
  return table ? &table->hdr->nrows : nullptr;
}

int gq_join_table_free(gq_ctx* ctx, gq_join_table* table, hipStream_t stream) {
  if (!table) return GQ_OK;
  if (!ctx) ctx = table->ctx;
  if (table->ready) {
    (void)hipStreamWaitEvent(stream, table->ready, 0);
    (void)hipEventDestroy(table->ready);
  }
  // Both allocations came from the building context's allocator.
  gq_ctx* actx = table->ctx ? table->ctx : ctx;
  if (table->imem) ctx_free(actx, table->imem, table->ibytes, stream);
  ctx_free(actx, table->mem, table->bytes, stream);
  delete table;
  return GQ_OK;
}

int gq_gather(gq_ctx* ctx, const gq_batch* in, const int32_t* cols, int ncols, const int32_t* idx, int64_t n,
              gq_batch* out, hipStream_t stream) {
  return gather_rows(ctx, in, cols, ncols, idx, n, nullptr, out, stream);
}

int gq_join_groupby(gq_ctx* ctx, const gq_join_table* table, const gq_batch* build, const gq_batch* probe,
                    const int32_t* probe_keys, int nprobe_keys, const gq_pred* probe_preds, int nprobe_preds,
                    const int32_t* group_keys, int ngroup_keys, const gq_agg* aggs, int naggs,
                    const gq_groupby_opts* opts, int64_t pair_capacity, gq_batch* out, int64_t* d_groups,
                    hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  if (!table || !build || !probe || !d_groups) return set_error(ctx, GQ_ERR_INVALID, "gq_join_groupby: NULL argument");
  int rc = check_batch(ctx, probe, "gq_join_groupby probe");
  if (rc) return rc;
  rc = check_batch(ctx, build, "gq_join_groupby build");
  if (rc) return rc;
  if (build->nrows != table->build_rows)
    return set_error(ctx, GQ_ERR_INVALID, "gq_join_groupby: build batch is not the table's build input");
  const int np = probe->ncols, nb = build->ncols;
  if (np + nb > GQ_MAX_COLS) return set_error(ctx, GQ_ERR_UNSUPPORTED, "gq_join_groupby: more than 16 joined columns");
  if (ngroup_keys < 0 || ngroup_keys > GQ_MAX_KEYS || (ngroup_keys > 0 && !group_keys) || naggs < 0 ||
      naggs > GQ_MAX_AGGS || (naggs > 0 && !aggs))
    return set_error(ctx, GQ_ERR_INVALID, "gq_join_groupby: bad key or aggregate list");
  if (opts && opts->mode != GQ_MODE_SINGLE && opts->mode != GQ_MODE_PARTIAL)
    return set_error(ctx, GQ_ERR_INVALID, "gq_join_groupby: aggregates read joined rows (single or partial mode)");
  const int64_t cap = pair_capacity > 0 ? pair_capacity : probe->nrows;
  // The joined columns the group-by reads: remap them to a gathered batch.
  int used[GQ_MAX_COLS];
  int nused = 0;
  int remap[GQ_MAX_COLS];
  for (int c = 0; c < GQ_MAX_COLS; ++c) remap[c] = -1;
  auto use = [&](int c) -> int {
    if (c < 0 || c >= np + nb) return -1;
    if (remap[c] < 0) {
      remap[c] = nused;
      used[nused++] = c;
    }
    return remap[c];
  };
  int32_t gk[GQ_MAX_KEYS];
  for (int j = 0; j < ngroup_keys; ++j) {
    gk[j] = use(group_keys[j]);
    if (gk[j] < 0) return set_error(ctx, GQ_ERR_INVALID, "gq_join_groupby: group key column out of range");
  }
  gq_agg ga[GQ_MAX_AGGS];
  for (int i = 0; i < naggs; ++i) {
    ga[i] = aggs[i];
    if (aggs[i].nfactors < 0 || aggs[i].nfactors > 3) return set_error(ctx, GQ_ERR_INVALID, "gq_join_groupby: 0..3 factors");
    for (int f = 0; f < aggs[i].nfactors; ++f) {
      if (aggs[i].f[f].kind == GQ_F_CONST) continue;
      ga[i].f[f].col = use(aggs[i].f[f].col);
      if (ga[i].f[f].col < 0) return set_error(ctx, GQ_ERR_INVALID, "gq_join_groupby: factor column out of range");
    }
  }
  // Workspace: the gather maps, their device count, the gathered columns.
  size_t off = 256;
  const size_t off_pi = off;
  off = align_up(off + (size_t)(cap > 0 ? cap : 1) * 4, 256);
  const size_t off_bi = off;
  off = align_up(off + (size_t)(cap > 0 ? cap : 1) * 4, 256);
  size_t coff[GQ_MAX_COLS], voff[GQ_MAX_COLS];
  for (int u = 0; u < nused; ++u) {
    const gq_column& src = used[u] < np ? probe->cols[used[u]] : build->cols[used[u] - np];
    coff[u] = off;
    off = align_up(off + (size_t)(cap > 0 ? cap : 1) * type_width(src.type), 256);
    voff[u] = off;
    if (src.validity) off = align_up(off + (size_t)((cap + 63) / 64) * 8, 256);
  }
  Scratch ws(ctx, stream);
  if (!ws.get(off)) return set_error(ctx, GQ_ERR_NOMEM, "gq_join_groupby: workspace allocation failed");
  int64_t* d_pairs = ws.as<int64_t>(0);
  int32_t* pi = ws.as<int32_t>(off_pi);
  int32_t* bi = ws.as<int32_t>(off_bi);
  // 1. Key-only join: the (probe row, build row) gather maps.
  rc = gq_join_probe(ctx, table, probe, probe_keys, nprobe_keys, probe_preds, nprobe_preds, pi, bi, cap, d_pairs,
                     stream);
  if (rc) return rc;
  // 2. Gather the columns the group-by reads, each from its side.
  gq_column gcols[GQ_MAX_COLS];
  std::memset(gcols, 0, sizeof(gcols));
  for (int u = 0; u < nused; ++u) {
    const bool from_probe = used[u] < np;
    const gq_batch* side = from_probe ? probe : build;
    const int32_t col = from_probe ? used[u] : used[u] - np;
    const gq_column& src = side->cols[col];
    gq_column& g = gcols[u];
    g.type = src.type;
    g.scale = src.scale;
    g.length = cap;
    g.data = ws.as<void>(coff[u]);
    g.validity = src.validity ? ws.as<uint8_t>(voff[u]) : nullptr;
    gq_batch gb{cap, 1, 0, &g};
    rc = gather_rows(ctx, side, &col, 1, from_probe ? pi : bi, cap, d_pairs, &gb, stream);
    if (rc) return rc;
  }
  // 3. Group-by over the gathered rows (their number is the device count).
  gq_batch joined{cap, nused, 0, gcols};
  return groupby_rows(ctx, &joined, d_pairs, gk, ngroup_keys, ga, naggs, opts, out, d_groups, stream);
}

}  // extern "C"
