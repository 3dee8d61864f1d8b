// gq_hash_partition: hash rows to partitions and write every partition
// contiguously, rows in input order within each partition.
//
// Three kernels on the caller's stream:
//  1. k_part_hist    per tile, an LDS histogram of partition ids, stored
//                    partition-major: counts[p * ntiles + tile].
//  2. k_scan_counts  single-pass exclusive scan of that array (decoupled
//                    look-back); entry (p, tile) becomes the output row where
//                    tile's rows of partition p start.  Also writes offsets[].
//  3. k_part_scatter per tile, a stable rank of each row within its partition:
//                    rows are visited wave by wave in row order, lanes of a wave
//                    holding 64 consecutive rows; lanes with the same partition
//                    find each other with one ballot per bit of the partition id
//                    and the lowest of them bumps the wave's LDS counter.  Every
//                    column is then staged in LDS in partitioned order and
//                    written out, consecutive lanes writing consecutive rows of
//                    a partition.
// The hash is recomputed in kernel 3 rather than stored: the key columns are
// read again anyway because they are part of the output.
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
};

__device__ __forceinline__ int64_t rows_of(const PartArgs& a) {
  if (!a.d_n) return a.n;
  const int64_t d = *a.d_n;
  return d < a.n ? d : a.n;
}

__device__ __forceinline__ uint32_t part_of_row(const PartArgs& a, int64_t r) {
  if (a.digit) return (uint32_t)(((uint64_t)load_one(a.keys[0], r) >> a.shift) & (a.nparts - 1));
  uint64_t h = a.seed;
  for (int j = 0; j < a.nkeys; ++j) {
    const DCol& c = a.keys[j];
    uint64_t x = valid_one(c, r) ? (uint64_t)load_one(c, r) : 0;
    h = fmix64(h ^ x);
  }
  return (uint32_t)mulhi64(h, a.nparts);
}

template <int ITEMS>
__device__ __forceinline__ void part_of_items(const PartArgs& a, int64_t r0, int64_t n, uint32_t (&p)[ITEMS]) {
  if (a.digit) {
    int64_t v[ITEMS];
    load_items<ITEMS>(a.keys[0], r0, n, v);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) p[k] = (uint32_t)(((uint64_t)v[k] >> a.shift) & (a.nparts - 1));
    return;
  }
  uint64_t h[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) h[k] = a.seed;
  for (int j = 0; j < a.nkeys; ++j) {
    const DCol& c = a.keys[j];
    int64_t v[ITEMS];
    load_items<ITEMS>(c, r0, n, v);
    uint32_t vm = c.valid ? valid_items<ITEMS>(c, r0, n) : 0xffffffffu;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) h[k] = fmix64(h[k] ^ (((vm >> k) & 1u) ? (uint64_t)v[k] : 0ull));
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) p[k] = (uint32_t)mulhi64(h[k], a.nparts);
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_part_hist(const PartArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  __shared__ uint32_t s_hist[kPartMax];
  const int P = (int)a.nparts;
  for (int i = threadIdx.x; i < P; i += BLOCK) s_hist[i] = 0;
  __syncthreads();
  const int64_t tile = blockIdx.x;
  const int64_t n = rows_of(a);
  const int64_t r0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;
  uint32_t p[ITEMS];
  part_of_items<ITEMS>(a, r0, n, p);
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (r0 + k < n) atomicAdd(&s_hist[p[k]], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += BLOCK) a.counts[(int64_t)i * a.ntiles + tile] = s_hist[i];
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

template <int BLOCK, int ITEMS, int PMAX>
__global__ __launch_bounds__(BLOCK) void k_part_scatter(const PartArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t s_whist[NW][PMAX];   // per-wave running counts, then wave-exclusive
  __shared__ uint32_t s_pstart[PMAX];      // tile-local start of each partition
  __shared__ int64_t s_gstart[PMAX];       // output row of the tile's first row of each partition
  __shared__ __attribute__((aligned(16))) uint8_t s_stage[TILE * 8];
  __shared__ uint16_t s_pid[TILE];
  __shared__ uint32_t s_scan[BLOCK];

  const int P = (int)a.nparts;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t tbase = tile * TILE;
  const int64_t n = rows_of(a);
  for (int i = threadIdx.x; i < NW * PMAX; i += BLOCK) (&s_whist[0][0])[i] = 0;
  __syncthreads();

  int nbits = 0;
  while ((1 << nbits) < P) ++nbits;

  // Rank pass: item k of lane l in wave w is row tbase + (w * ITEMS + k) * 64 + l.
  uint32_t pid[ITEMS];
  uint32_t rank[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t r = tbase + ((int64_t)wave * ITEMS + k) * kWave + lane;
    const bool in = r < n;
    const uint32_t p = in ? part_of_row(a, r) : 0u;
    uint64_t peers = ballot(in);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (p >> b) & 1u;
      const uint64_t m = ballot(bit);
      peers &= bit ? m : ~m;
    }
    pid[k] = p;
    rank[k] = 0;
    if (in) {
      const uint32_t before = s_whist[wave][p];
      rank[k] = before + rank_in(peers);
      // Lowest lane of the peer group advances the counter.  All lanes have
      // read the old value above (same wave, program order).
      if (rank_in(peers) == 0) s_whist[wave][p] = before + (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();

  // Per partition: wave-exclusive counts and the tile total.
  for (int q = threadIdx.x; q < P; q += BLOCK) {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      uint32_t c = s_whist[w][q];
      s_whist[w][q] = run;
      run += c;
    }
    s_pstart[q] = run;  // tile total for now
    s_gstart[q] = a.starts[(int64_t)q * a.ntiles + tile];
  }
  __syncthreads();
  // Exclusive scan of tile totals over partitions (BLOCK threads, PMAX/BLOCK each).
  {
    constexpr int PER = (PMAX + BLOCK - 1) / BLOCK;
    uint32_t loc[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int q = threadIdx.x * PER + j;
      loc[j] = q < P ? s_pstart[q] : 0u;
      sum += loc[j];
    }
    s_scan[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < BLOCK; o <<= 1) {
      uint32_t y = threadIdx.x >= (unsigned)o ? s_scan[threadIdx.x - o] : 0u;
      __syncthreads();
      s_scan[threadIdx.x] += y;
      __syncthreads();
    }
    uint32_t run = s_scan[threadIdx.x] - sum;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int q = threadIdx.x * PER + j;
      if (q < P) s_pstart[q] = run;
      run += loc[j];
    }
  }
  __syncthreads();

  int lpos[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t r = tbase + ((int64_t)wave * ITEMS + k) * kWave + lane;
    lpos[k] = -1;
    if (r < n) {
      lpos[k] = (int)(s_pstart[pid[k]] + s_whist[wave][pid[k]] + rank[k]);
      s_pid[lpos[k]] = (uint16_t)pid[k];
    }
  }
  const int tn = (int)((n - tbase) < TILE ? (n - tbase) : TILE);
  __syncthreads();

  for (int j = 0; j < a.ncols; ++j) {
    const DCol& c = a.cols[j];
    const OCol& o = a.out[j];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      if (lpos[k] >= 0) {
        const int64_t r = tbase + ((int64_t)wave * ITEMS + k) * kWave + lane;
        stage_put(s_stage, lpos[k], load_one(c, r), c.type);
        if (o.valid) {
          // Nullable column: set or clear the row's output bit directly.
          const uint32_t q = pid[k];
          const int64_t g = s_gstart[q] + (lpos[k] - (int)s_pstart[q]);
          const uint32_t bit = 1u << (g & 31);
          if (valid_one(c, r))
            atomicOr(&o.valid[g >> 5], bit);
          else
            atomicAnd(&o.valid[g >> 5], ~bit);
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < tn; i += BLOCK) {
      const uint32_t q = s_pid[i];
      const int64_t g = s_gstart[q] + (i - (int)s_pstart[q]);
      copy_out(s_stage, i, o.data, g, c.type);
    }
    __syncthreads();
  }
}

constexpr int kHistBlock = 256, kHistItems = 16;
constexpr int kScatBlock = 256, kScatItems = 16;
constexpr int kScanBlock = 256, kScanItems = 16;

// Histogram, scan and scatter for the rows of `a` (a.n, or at most a.n rows
// counted on the device when a.d_n is set).  d_offsets receives nparts + 1
// partition starts.
int launch_partition(gq_ctx* ctx, PartArgs& a, int64_t* d_offsets, hipStream_t stream) {
  const int64_t nparts = (int64_t)a.nparts;
  int rc;
  if (a.n == 0) return launch_fill_u32(ctx, d_offsets, 0u, 2 * (nparts + 1), stream);
  constexpr int TILE = kScatBlock * kScatItems;
  static_assert(TILE == kHistBlock * kHistItems, "histogram and scatter tiles must agree");
  const int64_t ntiles = (a.n + TILE - 1) / TILE;
  a.ntiles = ntiles;
  const int64_t m = ntiles * nparts;
  constexpr int STILE = kScanBlock * kScanItems;
  const int64_t nscan = (m + STILE - 1) / STILE;

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

  GQ_LAUNCH(ctx, "part_hist", (k_part_hist<kHistBlock, kHistItems>), dim3((unsigned)ntiles), dim3(kHistBlock), 0,
            stream, a);
  GQ_LAUNCH_CHECK(ctx);
  GQ_LAUNCH(ctx, "scan_counts", (k_scan_counts<kScanBlock, kScanItems>), dim3((unsigned)nscan), dim3(kScanBlock), 0,
            stream, (const uint32_t*)a.counts, m, a.starts, ntiles, nparts, d_offsets, ticket, status, nscan);
  GQ_LAUNCH_CHECK(ctx);
  if (nparts <= 256) {
    GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter<kScatBlock, kScatItems, 256>), dim3((unsigned)ntiles),
              dim3(kScatBlock), 0, stream, a);
  } else {
    GQ_LAUNCH(ctx, "part_scatter", (k_part_scatter<kScatBlock, kScatItems, kPartMax>), dim3((unsigned)ntiles),
              dim3(kScatBlock), 0, stream, a);
  }
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
