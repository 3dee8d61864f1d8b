// gq_hash_partition: hash rows to partitions and write every partition
// contiguously, rows in input order within each partition.
//
// Three kernels on the caller's stream, over hist tiles of 16384 rows cut into
// sub-tiles of 1024 rows; each sub-tile's columns are first copied into LDS
// with 16-byte global-to-LDS loads (every load of the sub-tile in flight at
// once), and all row work reads LDS:
//  1. k_part_hist    per hist tile, an LDS histogram of partition ids, stored
//                    partition-major: counts[p * ntiles + tile].
//  2. k_scan_counts  single-pass exclusive scan of that array (decoupled
//                    look-back); entry (p, tile) becomes the output row where
//                    tile's rows of partition p start.  Also writes offsets[].
//  3. k_part_scatter per sub-tile, a stable rank of each row within its
//                    partition: wave w owns rows [256w, 256w + 256) of the
//                    sub-tile in four steps of 64; lanes with the same partition
//                    find each other with one ballot per bit of the partition
//                    id and the lowest of them bumps the wave's LDS counter, so
//                    ranks follow row order.  Then every column is written in
//                    partitioned order from the staged copy, consecutive lanes
//                    writing consecutive rows of a partition.
// Consecutive hist tiles run on the same XCD (blocks are mapped to tiles per
// XCD), so partial output lines of neighbouring tiles meet in its L2.
#include "common.h"

namespace gq {
namespace {

constexpr int kPartMax = 1024;

struct PartArgs {
  int64_t n;             // rows (an upper bound when d_n is set)
  const int64_t* d_n;    // device row count, or NULL
  int64_t ntiles;
  uint64_t seed;
  uint64_t nparts;
  int32_t nkeys;
  int32_t ncols;
  int32_t digit;         // 0: hash partition; 1: radix digit (key >> shift) & (nparts - 1)
  int32_t shift;
  DCol keys[GQ_MAX_KEYS];
  DCol cols[GQ_MAX_COLS];
  OCol out[GQ_MAX_COLS];
  uint32_t* counts;  // nparts * ntiles
  int64_t* starts;   // nparts * ntiles, exclusive scan of counts
  int32_t key_col[GQ_MAX_KEYS];   // column of cols[] holding key j
  int32_t st_off[GQ_MAX_COLS];    // LDS offset of staged column j (scatter)
  int32_t kst_off[GQ_MAX_KEYS];   // LDS offset of staged key j (histogram)
  int32_t in_bytes;               // LDS bytes of the scatter's staged sub-tile
  int32_t kin_bytes;              // LDS bytes of the histogram's staged keys
};

constexpr int kPBlock = 256;
constexpr int kPSub = 1024;                  // rows per sub-tile
constexpr int kPSubs = 16;                   // sub-tiles per hist tile
constexpr int kPTile = kPSub * kPSubs;       // rows per hist tile
constexpr int kPSteps = kPSub / kPBlock;     // rows per thread per sub-tile
constexpr int kPWBlock = 1024;               // wide scatter variant: workgroup
constexpr int kPWSub = kPSteps * kPWBlock;   // and sub-tile rows
constexpr size_t kPWMaxLds = 150 * 1024;

// Staged rows r0 + i * stride, i < kPSteps, of one column: one type dispatch.
__device__ __forceinline__ void lds_rows_at(const uint8_t* base, int type, int r0, int stride,
                                            int64_t (&v)[kPSteps]) {
  switch (type) {
    case GQ_I8:
#pragma unroll
      for (int i = 0; i < kPSteps; ++i) v[i] = reinterpret_cast<const int8_t*>(base)[r0 + i * stride];
      break;
    case GQ_I16:
#pragma unroll
      for (int i = 0; i < kPSteps; ++i) v[i] = reinterpret_cast<const int16_t*>(base)[r0 + i * stride];
      break;
    case GQ_I32:
#pragma unroll
      for (int i = 0; i < kPSteps; ++i) v[i] = reinterpret_cast<const int32_t*>(base)[r0 + i * stride];
      break;
    default:
#pragma unroll
      for (int i = 0; i < kPSteps; ++i) v[i] = reinterpret_cast<const int64_t*>(base)[r0 + i * stride];
      break;
  }
}

__device__ __forceinline__ int64_t rows_of(const PartArgs& a) {
  if (!a.d_n) return a.n;
  const int64_t d = *a.d_n;
  return d < a.n ? d : a.n;
}

// Partitions of the kPSteps staged rows r0 + i * stride (rows >= nrows get 0):
// one type dispatch per key column for all of them.
template <class KeyBase>
__device__ __forceinline__ void part_of_rows(const PartArgs& a, int64_t sbase, int r0, int stride, int nrows,
                                             KeyBase kbase, uint32_t (&p)[kPSteps]) {
  uint64_t h[kPSteps];
  if (a.digit) {
    int64_t v[kPSteps];
    lds_rows_at(kbase(0), a.keys[0].type, r0, stride, v);
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) p[i] = (uint32_t)(((uint64_t)v[i] >> a.shift) & (a.nparts - 1));
    return;
  }
#pragma unroll
  for (int i = 0; i < kPSteps; ++i) h[i] = a.seed;
  for (int j = 0; j < a.nkeys; ++j) {
    const DCol& c = a.keys[j];
    int64_t v[kPSteps];
    lds_rows_at(kbase(j), c.type, r0, stride, v);
    if (c.valid) {
#pragma unroll
      for (int i = 0; i < kPSteps; ++i) {
        const int r = r0 + i * stride;
        if (r < nrows && !valid_one(c, sbase + r)) v[i] = 0;
      }
    }
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) h[i] = fmix64(h[i] ^ (uint64_t)v[i]);
  }
#pragma unroll
  for (int i = 0; i < kPSteps; ++i) p[i] = (uint32_t)mulhi64(h[i], a.nparts);
}

__global__ __launch_bounds__(kPBlock) void k_part_hist(const PartArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int P = (int)a.nparts;
  uint32_t* s_hist = reinterpret_cast<uint32_t*>(s_raw);
  uint8_t* s_in = s_raw + align_up((size_t)P * 4, 16);
  for (int i = threadIdx.x; i < P; i += kPBlock) s_hist[i] = 0;
  const int64_t tile = blockIdx.x;
  const int64_t n = rows_of(a);
  auto kbase = [&](int j) { return (const uint8_t*)(s_in + a.kst_off[j]); };
  for (int sub = 0; sub < kPSubs; ++sub) {
    const int64_t sbase = tile * kPTile + (int64_t)sub * kPSub;
    if (sbase >= n) break;
    const int nrows = n - sbase < kPSub ? (int)(n - sbase) : kPSub;
    __syncthreads();  // the previous sub-tile's keys are read
    const int nk = a.digit ? 1 : a.nkeys;
    for (int j = 0; j < nk; ++j) stage_col_lds<kPBlock>(a.keys[j], sbase, nrows, s_in + a.kst_off[j]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    uint32_t pid[kPSteps];
    part_of_rows(a, sbase, threadIdx.x, kPBlock, nrows, kbase, pid);
#pragma unroll
    for (int i = 0; i < kPSteps; ++i)
      if (i * kPBlock + (int)threadIdx.x < nrows) atomicAdd(&s_hist[pid[i]], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += kPBlock) a.counts[(int64_t)i * a.ntiles + tile] = s_hist[i];
}

// Exclusive scan of counts[0..m) into starts[], with offsets[q] = starts[q * ntiles]
// and offsets[nparts] = total.
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_scan_counts(const uint32_t* counts, int64_t m, int64_t* starts,
                                                       int64_t ntiles, int64_t nparts, int64_t* offsets,
                                                       uint32_t* ticket, uint64_t* status, int64_t nblocks) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t s_tile;
  __shared__ int64_t s_wave[NW];
  __shared__ int64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t i0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;
  uint32_t c[ITEMS];
  int64_t tsum = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    c[k] = (i0 + k < m) ? counts[i0 + k] : 0u;
    tsum += c[k];
  }
  // Wave inclusive scan of per-thread sums.
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
    if (i < m) {
      starts[i] = run;
      if (i % ntiles == 0) offsets[i / ntiles] = run;
    }
    run += c[k];
  }
  if (tile == nblocks - 1 && threadIdx.x == 0) offsets[nparts] = s_excl + btot;
}

// LDS of k_part_scatter (dynamic): staged columns (in_bytes), per-wave
// counts [4][P] (u32), sub-tile starts [P + 1] (u32), write positions [P]
// (i64), then per sorted position its partition and source row (u16 each).
template <int BLOCK, int SUB>
__host__ inline size_t part_scatter_lds(int P, int in_bytes) {
  return align_up((size_t)in_bytes, 16) + align_up((size_t)(BLOCK / kWave) * P * 4, 16) +
         align_up((size_t)(P + 1) * 4, 16) + (size_t)P * 8 + (size_t)SUB * 4;
}

// BLOCK threads stage SUB = 4 * BLOCK rows per sub-tile: the wide variant
// (1024 threads, 4096 rows) writes longer runs per partition; the narrow one
// (256, 1024) serves column sets too wide to stage 4096 rows.
template <int BLOCK, int SUB>
__global__ __launch_bounds__(BLOCK) void k_part_scatter(const PartArgs a) {
  static_assert(SUB == kPSteps * BLOCK, "four rows per thread per sub-tile");
  constexpr int NW = BLOCK / kWave;
  constexpr int SUBS = kPTile / SUB;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int P = (int)a.nparts;
  uint8_t* s_in = s_raw;
  uint32_t* s_whist = reinterpret_cast<uint32_t*>(s_raw + align_up((size_t)a.in_bytes, 16));
  uint32_t* s_sub = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(s_whist) + align_up((size_t)NW * P * 4, 16));
  int64_t* s_base = reinterpret_cast<int64_t*>(reinterpret_cast<uint8_t*>(s_sub) + align_up((size_t)(P + 1) * 4, 16));
  uint16_t* s_pid = reinterpret_cast<uint16_t*>(s_base + P);
  uint16_t* s_src = s_pid + SUB;
  __shared__ uint32_t s_wsum[NW];

  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t n = rows_of(a);
  for (int q = threadIdx.x; q < P; q += BLOCK) s_base[q] = a.starts[(int64_t)q * a.ntiles + tile];
  int nbits = 0;
  while ((1 << nbits) < P) ++nbits;
  auto kbase = [&](int j) { return (const uint8_t*)(s_in + a.st_off[a.key_col[j]]); };
  const int per = (P + BLOCK - 1) / BLOCK;

  for (int sub = 0; sub < SUBS; ++sub) {
    const int64_t sbase = tile * kPTile + (int64_t)sub * SUB;
    if (sbase >= n) break;
    const int nrows = n - sbase < SUB ? (int)(n - sbase) : SUB;
    for (int i = threadIdx.x; i < NW * P; i += BLOCK) s_whist[i] = 0;
    for (int j = 0; j < a.ncols; ++j) stage_col_lds<BLOCK>(a.cols[j], sbase, nrows, s_in + a.st_off[j]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // Stable ranks: wave w owns rows 256w + 64i + lane, i = 0..3, in order.
    uint32_t pid[kPSteps], rank[kPSteps];
    part_of_rows(a, sbase, wave * (SUB / NW) + lane, kWave, nrows, kbase, pid);
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) {
      const int r = wave * (SUB / NW) + i * kWave + lane;
      const bool in = r < nrows;
      const uint32_t p = in ? pid[i] : 0u;
      uint64_t peers = ballot(in);
      for (int b = 0; b < nbits; ++b) {
        const bool bit = (p >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
      }
      pid[i] = p;
      rank[i] = 0;
      if (in) {
        uint32_t* cnt = s_whist + wave * P + p;
        const uint32_t before = *cnt;
        rank[i] = before + rank_in(peers);
        // The lowest lane of the peer group advances the counter after every
        // lane of the wave has read it (same wave, program order).
        if (rank_in(peers) == 0) *cnt = before + (uint32_t)__popcll(peers);
      }
    }
    __syncthreads();
    // Per partition: wave-exclusive counts, and the sub-tile total.
    uint32_t mysum = 0;
    uint32_t cnt_own[4] = {0u, 0u, 0u, 0u};  // per <= 4 for P <= 1024
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < P) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = s_whist[w * P + q];
          s_whist[w * P + q] = run;
          run += c;
        }
        cnt_own[j] = run;
        mysum += run;
      }
    }
    // Exclusive scan over partitions of the sub-tile totals.
    uint32_t incl = mysum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) s_wsum[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if (w < wave) wpre += s_wsum[w];
      tot += s_wsum[w];
    }
    uint32_t run = wpre + incl - mysum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < P) {
        s_sub[q] = run;
        run += cnt_own[j];
      }
    }
    if (threadIdx.x == 0) s_sub[P] = tot;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) {
      const int r = wave * (SUB / NW) + i * kWave + lane;
      if (r < nrows) {
        const uint32_t pos = s_sub[pid[i]] + s_whist[wave * P + pid[i]] + rank[i];
        s_src[pos] = (uint16_t)r;
        s_pid[pos] = (uint16_t)pid[i];
      }
    }
    __syncthreads();
    const int total = (int)tot;
    // Source row and output row of the sorted positions k = t + 256 i, once
    // for all columns.
    int srow[kPSteps];
    int64_t grow[kPSteps];
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) {
      const int k = i * BLOCK + threadIdx.x;
      srow[i] = 0;
      grow[i] = -1;
      if (k < total) {
        const uint32_t q = s_pid[k];
        srow[i] = s_src[k];
        grow[i] = s_base[q] + (k - (int)s_sub[q]);
      }
    }
    for (int j = 0; j < a.ncols; ++j) {
      const OCol& o = a.out[j];
      const uint8_t* col = s_in + a.st_off[j];
      switch (a.cols[j].type) {
        case GQ_I8:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0) o.data[grow[i]] = col[srow[i]];
          break;
        case GQ_I16:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0)
              reinterpret_cast<int16_t*>(o.data)[grow[i]] = reinterpret_cast<const int16_t*>(col)[srow[i]];
          break;
        case GQ_I32:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0)
              reinterpret_cast<int32_t*>(o.data)[grow[i]] = reinterpret_cast<const int32_t*>(col)[srow[i]];
          break;
        default:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0)
              reinterpret_cast<int64_t*>(o.data)[grow[i]] = reinterpret_cast<const int64_t*>(col)[srow[i]];
          break;
      }
      if (o.valid) {
        const DCol& c = a.cols[j];
#pragma unroll
        for (int i = 0; i < kPSteps; ++i) {
          if (grow[i] < 0) continue;
          const uint32_t bit = 1u << (grow[i] & 31);
          if (valid_one(c, sbase + srow[i])) atomicOr(&o.valid[grow[i] >> 5], bit);
          else atomicAnd(&o.valid[grow[i] >> 5], ~bit);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < P) s_base[q] += cnt_own[j];
    }
    __syncthreads();
  }
}

// Prefetching form of the scatter (both shapes), for every column 16-byte
// aligned and without a bitmap, at most kPPfMax columns, the row count known
// on the host.  The next sub-tile's columns are loaded into
// registers (at most two 16-byte chunks per column and thread) while the
// current one is ranked, and written to LDS once its rows have left.
// Barriers order LDS only, so the loads and the row stores stay in flight
// across them (a full barrier also waits for every outstanding global access
// of the wave).
constexpr int kPPfMax = 4;

template <int BLOCK, int SUB, int NPF>
__global__ __launch_bounds__(BLOCK) void k_part_scatter_pf(const PartArgs a) {
  static_assert(SUB == kPSteps * BLOCK, "four rows per thread per sub-tile");
  constexpr int NW = BLOCK / kWave, SUBS = kPTile / SUB;
  constexpr int CH = SUB * 8 / 16 / BLOCK;  // 16-byte chunks per thread of an 8-byte column
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int P = (int)a.nparts;
  uint8_t* s_in = s_raw;
  uint32_t* s_whist = reinterpret_cast<uint32_t*>(s_raw + align_up((size_t)a.in_bytes, 16));
  uint32_t* s_sub = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(s_whist) + align_up((size_t)NW * P * 4, 16));
  int64_t* s_base = reinterpret_cast<int64_t*>(reinterpret_cast<uint8_t*>(s_sub) + align_up((size_t)(P + 1) * 4, 16));
  uint16_t* s_pid = reinterpret_cast<uint16_t*>(s_base + P);
  uint16_t* s_src = s_pid + SUB;
  __shared__ uint32_t s_wsum[NW];

  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t n = a.n;
  const int64_t tbase = tile * kPTile;
  for (int q = threadIdx.x; q < P; q += BLOCK) s_base[q] = a.starts[(int64_t)q * a.ntiles + tile];
  for (int i = threadIdx.x; i < NW * P; i += BLOCK) s_whist[i] = 0;
  int nbits = 0;
  while ((1 << nbits) < P) ++nbits;
  auto kbase = [&](int j) { return (const uint8_t*)(s_in + a.st_off[a.key_col[j]]); };
  const int per = (P + BLOCK - 1) / BLOCK;
  {
    const int nrows0 = n - tbase < SUB ? (int)(n - tbase) : SUB;
    for (int j = 0; j < a.ncols; ++j) stage_col_lds<BLOCK>(a.cols[j], tbase, nrows0, s_in + a.st_off[j]);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int sub = 0; sub < SUBS; ++sub) {
    const int64_t sbase = tbase + (int64_t)sub * SUB;
    if (sbase >= n) break;
    const int nrows = n - sbase < SUB ? (int)(n - sbase) : SUB;
    const int64_t nbase = sbase + SUB;
    const bool has_next = sub + 1 < SUBS && nbase < n;
    const bool pf = has_next && n - nbase >= SUB;
    u32x4 pfv[NPF][CH];
#pragma unroll
    for (int j = 0; j < NPF; ++j)
#pragma unroll
      for (int c = 0; c < CH; ++c) pfv[j][c] = u32x4{0u, 0u, 0u, 0u};
    if (pf) {
#pragma unroll
      for (int j = 0; j < NPF; ++j) {
        const int w = type_width(a.cols[j].type);
        const int nch = SUB * w / 16;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int idx = (int)threadIdx.x + c * BLOCK;
          if (idx < nch)
            pfv[j][c] = *reinterpret_cast<const u32x4*>(a.cols[j].data + nbase * w + (int64_t)idx * 16);
        }
      }
    }
    // Stable ranks: wave w owns rows 256w + 64i + lane, i = 0..3, in order;
    // lanes of one partition find each other with one ballot per bit of its
    // id, and the lowest of them advances the wave's counter.
    uint32_t pid[kPSteps], rank[kPSteps];
    part_of_rows(a, sbase, wave * (SUB / NW) + lane, kWave, nrows, kbase, pid);
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) {
      const int r = wave * (SUB / NW) + i * kWave + lane;
      const bool in = r < nrows;
      const uint32_t p = in ? pid[i] : 0u;
      uint64_t peers = ballot(in);
      for (int b = 0; b < nbits; ++b) {
        const bool bit = (p >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
      }
      pid[i] = p;
      rank[i] = 0;
      if (in) {
        uint32_t* cnt = s_whist + wave * P + p;
        const uint32_t before = *cnt;
        rank[i] = before + rank_in(peers);
        if (rank_in(peers) == 0) *cnt = before + (uint32_t)__popcll(peers);
      }
    }
    lds_barrier();
    // Per partition: wave-exclusive counts and the sub-tile total; then the
    // exclusive scan of the totals over partitions.
    uint32_t mysum = 0;
    uint32_t cnt_own[4] = {0u, 0u, 0u, 0u};  // per <= 4 for P <= 1024
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < P) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = s_whist[w * P + q];
          s_whist[w * P + q] = run;
          run += c;
        }
        cnt_own[j] = run;
        mysum += run;
      }
    }
    uint32_t incl = mysum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) s_wsum[wave] = incl;
    lds_barrier();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if (w < wave) wpre += s_wsum[w];
      tot += s_wsum[w];
    }
    uint32_t run = wpre + incl - mysum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < P) {
        s_sub[q] = run;
        run += cnt_own[j];
      }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) {
      const int r = wave * (SUB / NW) + i * kWave + lane;
      if (r < nrows) {
        const uint32_t pos = s_sub[pid[i]] + s_whist[wave * P + pid[i]] + rank[i];
        s_src[pos] = (uint16_t)r;
        s_pid[pos] = (uint16_t)pid[i];
      }
    }
    lds_barrier();
    const int total = (int)tot;
    int srow[kPSteps];
    int64_t grow[kPSteps];
#pragma unroll
    for (int i = 0; i < kPSteps; ++i) {
      const int k = i * BLOCK + threadIdx.x;
      srow[i] = 0;
      grow[i] = -1;
      if (k < total) {
        const uint32_t q = s_pid[k];
        srow[i] = s_src[k];
        grow[i] = s_base[q] + (k - (int)s_sub[q]);
      }
    }
    // The next sub-tile's loads have landed (and the previous sub-tile's
    // stores left) before this one's stores are issued, so that refilling LDS
    // below waits for nothing.
    __builtin_amdgcn_s_waitcnt(0);
    for (int j = 0; j < a.ncols; ++j) {
      const OCol& o = a.out[j];
      const uint8_t* col = s_in + a.st_off[j];
      switch (a.cols[j].type) {
        case GQ_I8:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0) o.data[grow[i]] = col[srow[i]];
          break;
        case GQ_I16:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0)
              reinterpret_cast<int16_t*>(o.data)[grow[i]] = reinterpret_cast<const int16_t*>(col)[srow[i]];
          break;
        case GQ_I32:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0)
              reinterpret_cast<int32_t*>(o.data)[grow[i]] = reinterpret_cast<const int32_t*>(col)[srow[i]];
          break;
        default:
#pragma unroll
          for (int i = 0; i < kPSteps; ++i)
            if (grow[i] >= 0)
              reinterpret_cast<int64_t*>(o.data)[grow[i]] = reinterpret_cast<const int64_t*>(col)[srow[i]];
          break;
      }
    }
    // Every row has left the staged input; the next sub-tile replaces it.
    lds_barrier();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < P) s_base[q] += cnt_own[j];
    }
    for (int i = threadIdx.x; i < NW * P; i += BLOCK) s_whist[i] = 0;
    if (pf) {
#pragma unroll
      for (int j = 0; j < NPF; ++j) {
        const int nch = SUB * type_width(a.cols[j].type) / 16;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int idx = (int)threadIdx.x + c * BLOCK;
          if (idx < nch) *reinterpret_cast<u32x4*>(s_in + a.st_off[j] + (int64_t)idx * 16) = pfv[j][c];
        }
      }
    } else if (has_next) {
      const int nr = n - nbase < SUB ? (int)(n - nbase) : SUB;
      for (int j = 0; j < a.ncols; ++j) stage_col_lds<BLOCK>(a.cols[j], nbase, nr, s_in + a.st_off[j]);
      __builtin_amdgcn_s_waitcnt(0);
    }
    lds_barrier();
  }
}

constexpr int kScanBlock = 256, kScanItems = 16;

template <int BLOCK, int SUB>
int launch_scatter_pf(gq_ctx* ctx, const PartArgs& a, int64_t ntiles, size_t lds, hipStream_t stream) {
  const dim3 g((unsigned)ntiles), b(BLOCK);
  switch (a.ncols) {
    case 1: GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter_pf<BLOCK, SUB, 1>), g, b, lds, stream, a); break;
    case 2: GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter_pf<BLOCK, SUB, 2>), g, b, lds, stream, a); break;
    case 3: GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter_pf<BLOCK, SUB, 3>), g, b, lds, stream, a); break;
    default: GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter_pf<BLOCK, SUB, 4>), g, b, lds, stream, a); break;
  }
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

// Histogram, scan and scatter for the rows of `a` (a.n, or at most a.n rows
// counted on the device when a.d_n is set).  d_offsets receives nparts + 1
// partition starts.
int launch_partition(gq_ctx* ctx, PartArgs& a, int64_t* d_offsets, hipStream_t stream) {
  const int64_t nparts = (int64_t)a.nparts;
  int rc;
  if (a.n == 0) return launch_fill_u32(ctx, d_offsets, 0u, 2 * (nparts + 1), stream);
  const int64_t ntiles = (a.n + kPTile - 1) / kPTile;
  a.ntiles = ntiles;
  const int64_t m = ntiles * nparts;
  constexpr int STILE = kScanBlock * kScanItems;
  const int64_t nscan = (m + STILE - 1) / STILE;
  // LDS layouts: every column for the scatter (4096-row sub-tiles when they
  // fit two workgroups' worth of LDS, else 1024), the key columns for the
  // histogram.
  int lds_max = 0;
  GQ_HIP_CHECK(ctx, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
  size_t row_bytes = 0;
  for (int j = 0; j < a.ncols; ++j) row_bytes += (size_t)type_width(a.cols[j].type);
  // The wide shape (4096-row sub-tiles, longer runs per partition) where its
  // LDS fits, else the narrow one; each in its prefetching form where that
  // applies.
  bool pf = !a.d_n && a.ncols >= 1 && a.ncols <= kPPfMax;
  for (int j = 0; j < a.ncols; ++j) pf = pf && a.cols[j].align >= 16 && !a.cols[j].valid;
  const size_t wide_lds = part_scatter_lds<kPWBlock, kPWSub>((int)nparts, (int)(row_bytes * kPWSub + 16 * a.ncols));
  const bool wide = wide_lds <= kPWMaxLds && wide_lds + 256 <= (size_t)lds_max;
  const int ssub = wide ? kPWSub : kPSub;
  a.in_bytes = 0;
  for (int j = 0; j < a.ncols; ++j) {
    a.st_off[j] = a.in_bytes;
    a.in_bytes += (int)align_up((size_t)ssub * type_width(a.cols[j].type), 16);
  }
  a.kin_bytes = 0;
  const int nk = a.digit ? 1 : a.nkeys;
  for (int j = 0; j < nk; ++j) {
    a.kst_off[j] = a.kin_bytes;
    a.kin_bytes += (int)align_up((size_t)kPSub * type_width(a.keys[j].type), 16);
  }
  const size_t lds_hist = align_up((size_t)nparts * 4, 16) + (size_t)a.kin_bytes;
  const size_t lds_scat = wide ? part_scatter_lds<kPWBlock, kPWSub>((int)nparts, a.in_bytes)
                               : part_scatter_lds<kPBlock, kPSub>((int)nparts, a.in_bytes);
  if (lds_scat + 256 > (size_t)lds_max || lds_hist + 256 > (size_t)lds_max)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "partition: too many or too wide columns for one staged sub-tile");

  Scratch ws(ctx, stream);
  const size_t off_counts = 256;
  const size_t off_starts = off_counts + align_up((size_t)m * 4, 256);
  const size_t off_status = off_starts + align_up((size_t)m * 8, 256);
  const size_t total = off_status + align_up((size_t)nscan * 8, 256);
  if (!ws.get(total)) return set_error(ctx, GQ_ERR_NOMEM, "partition: workspace allocation failed");
  a.counts = ws.as<uint32_t>(off_counts);
  a.starts = ws.as<int64_t>(off_starts);
  uint32_t* ticket = ws.as<uint32_t>(0);
  uint64_t* status = ws.as<uint64_t>(off_status);

  // ticket (one word) and the scan status words start at zero.
  rc = launch_fill_u32(ctx, ticket, 0u, 1, stream);
  if (rc) return rc;
  rc = launch_fill_u32(ctx, status, 0u, 2 * nscan, stream);
  if (rc) return rc;

  GQ_LAUNCH(ctx, "part_hist", k_part_hist, dim3((unsigned)ntiles), dim3(kPBlock), lds_hist, stream, a);
  GQ_LAUNCH_CHECK(ctx);
  GQ_LAUNCH(ctx, "scan_counts", (k_scan_counts<kScanBlock, kScanItems>), dim3((unsigned)nscan), dim3(kScanBlock), 0,
            stream, (const uint32_t*)a.counts, m, a.starts, ntiles, nparts, d_offsets, ticket, status, nscan);
  GQ_LAUNCH_CHECK(ctx);
  if (pf) {
    int rc2 = wide ? launch_scatter_pf<kPWBlock, kPWSub>(ctx, a, ntiles, lds_scat, stream)
                   : launch_scatter_pf<kPBlock, kPSub>(ctx, a, ntiles, lds_scat, stream);
    if (rc2) return rc2;
  } else if (wide)
    GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter<kPWBlock, kPWSub>), dim3((unsigned)ntiles), dim3(kPWBlock), lds_scat,
              stream, a);
  else
    GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter<kPBlock, kPSub>), dim3((unsigned)ntiles), dim3(kPBlock), lds_scat,
              stream, a);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

}  // namespace

// Stable LSD radix sort of rows by an unsigned key (column 0 of `a`, int64):
// one partition pass per 8-bit digit of the `bits` low key bits, ping-ponging
// between `bufs[0]` and `bufs[1]` (both laid out like the output, every column
// including the key); the result lands in `out`.  Row count: at most `n`,
// exactly *d_n when d_n is set.
int radix_sort_rows(gq_ctx* ctx, const gq_batch* in, gq_batch* const bufs[2], gq_batch* out, int bits, int64_t n,
                    const int64_t* d_n, hipStream_t stream) {
  if (bits < 1) bits = 1;
  const int passes = (bits + 7) / 8;
  Scratch offs(ctx, stream);
  if (!offs.get(8 * 257)) return set_error(ctx, GQ_ERR_NOMEM, "radix sort: workspace allocation failed");
  const gq_batch* src = in;
  for (int pass = 0; pass < passes; ++pass) {
    const bool last = pass == passes - 1;
    gq_batch* dst = last ? out : bufs[pass & 1];
    const int dbits = (pass == passes - 1) ? bits - 8 * pass : 8;
    PartArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.d_n = d_n;
    a.nparts = 1ull << dbits;
    a.digit = 1;
    a.shift = 8 * pass;
    a.nkeys = 1;
    a.ncols = src->ncols;
    a.keys[0] = make_dcol(src->cols[0]);
    a.key_col[0] = 0;
    for (int j = 0; j < src->ncols; ++j) {
      a.cols[j] = make_dcol(src->cols[j]);
      const gq_column& oc = dst->cols[j];
      a.out[j] = OCol{static_cast<uint8_t*>(oc.data), reinterpret_cast<uint32_t*>(oc.validity), oc.type, 0};
    }
    int rc = launch_partition(ctx, a, offs.as<int64_t>(0), stream);
    if (rc) return rc;
    src = dst;
  }
  return GQ_OK;
}

namespace {
}  // namespace
}  // namespace gq

using namespace gq;

extern "C" int gq_hash_partition(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys,
                                 int32_t nparts, uint64_t seed, gq_batch* out, int64_t* d_offsets,
                                 hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_hash_partition input");
  if (rc) return rc;
  if (nparts < 1 || nparts > kPartMax)
    return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: nparts outside [1, 1024]");
  if (nkeys < 0 || nkeys > GQ_MAX_KEYS || (nkeys > 0 && !keys))
    return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: bad key list");
  if (!d_offsets) return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: NULL offsets");
  if (!out || out->ncols != in->ncols || (in->ncols > 0 && !out->cols))
    return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: output must have the input's columns");

  PartArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = in->nrows;
  a.seed = seed;
  a.nparts = (uint64_t)nparts;
  a.nkeys = nkeys;
  a.ncols = in->ncols;
  for (int j = 0; j < nkeys; ++j) {
    if (keys[j] < 0 || keys[j] >= in->ncols)
      return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: key column out of range");
    a.keys[j] = make_dcol(in->cols[keys[j]]);
    a.key_col[j] = keys[j];
  }
  for (int j = 0; j < in->ncols; ++j) {
    const gq_column& ic = in->cols[j];
    const gq_column& oc = out->cols[j];
    if (oc.type != ic.type) return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: output type mismatch");
    if (oc.length < in->nrows || (in->nrows > 0 && !oc.data))
      return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: output capacity below the row count");
    if (ic.validity && !oc.validity)
      return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: nullable input needs an output bitmap");
    if (oc.validity && (reinterpret_cast<uintptr_t>(oc.validity) & 3))
      return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: output bitmap must be 4-byte aligned");
    if (oc.offset != 0) return set_error(ctx, GQ_ERR_INVALID, "gq_hash_partition: output offset must be 0");
    a.cols[j] = make_dcol(ic);
    a.out[j] = OCol{static_cast<uint8_t*>(oc.data), reinterpret_cast<uint32_t*>(oc.validity), oc.type, 0};
  }
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  return launch_partition(ctx, a, d_offsets, stream);
}
