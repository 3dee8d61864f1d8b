// Radix group-join: a join whose only group key is the join key, evaluated
// without any HBM hash table.  Both sides are partitioned by a hash of the key
// into P regions; every (region, sub-region) is then joined and aggregated by
// one workgroup in an LDS hash table.
//
// Why this shape: on gfx950 a device-wide atomic add is served by one
// chip-wide path (about 24 G atomics/s measured, independent of the table
// size, even for a table that fits one XCD's L2), so a group-join that adds
// into an HBM table pays two atomics per matched row and is bound by them, not
// by HBM bandwidth.  Here every row is read and written with coalesced
// streaming accesses, and the per-row atomics are LDS atomics.
//
// Build side (gq_join_build, large build inputs):
//   k_rp_hist_r   per tile (4,096 to 32,768 rows, about 2,048 tiles),
//                 histogram of the region ids of the kept rows (predicates
//                 pass, key non-NULL); region = top pbits of
//                 fmix64(key ^ kRegionSeed); columns read straight into
//                 registers (k_rp_hist stages them through LDS where one is
//                 not 16-byte aligned)
//   k_cs_*        column scan of the (tile, region) counts, stored tile-major
//                 so that every tile reads and writes its P counts coalesced:
//                 per-chunk column sums and region totals, then the start of
//                 every (tile, region), each block deriving its regions'
//                 offsets from the totals
//   k_rp_scatter  each tile in sub-tiles of 2048 rows staged in LDS (one
//                 1024-thread workgroup per tile); a
//                 kept row takes the next position of its region in the tile's
//                 range with an LDS atomic and is written there: (key hash,
//                 build row) pairs of 64-bit words grouped by region, one
//                 16-byte store each (order inside a region is unspecified;
//                 with thousands of regions a tile holds only a few rows per
//                 region, so there is no run of stores to coalesce)
// Probe side (gq_pipeline when the only group key is the probe key): the
// payload of a row is its aggregate inputs (one 64-bit product expression per
// SUM/MIN/MAX, and a non-NULL mask where an input can be NULL).  Without a
// mask it is partitioned in two levels (k_rp1, k_cs_*, k_rp2, described with
// the kernels below: a sort into 32 first-level regions inside every
// sub-tile, written out whole, then every first-level region moved to its
// final regions), else by the same three kernels as the build side; then
//   k_rj_plan     per region p, the number of sub-regions S_p so that each holds
//                 at most kpr build rows, and per-XCD work lists of
//                 (region, sub-region) items
//   k_rj_join     persistent, one workgroup per CU: a workgroup takes an item
//                 (p, s), inserts the build keys of region p that fall in
//                 sub-region s into an LDS table (with their multiplicities),
//                 streams the probe tuples of region p through it, accumulating
//                 the matches of sub-region s in LDS (unweighted; a key's build
//                 multiplicity scales its sums and counts at emission), and
//                 writes its matched groups to the output (one atomic per item
//                 for the output range; validity words stored whole).
// Region p is queued on XCD p % 8 (workgroups are dispatched to XCDs
// round-robin), so the S_p workgroups that re-read region p's tuples share one
// L2.  A workgroup whose queue is empty takes items from the other queues, so
// every item is processed whatever the placement.
#include "agg.h"
#include "radix.h"

namespace gq {
namespace {

constexpr int kRpBlock = 256;                    // hist workgroup
constexpr int kRpSBlock = 1024;                  // scatter workgroup
constexpr int kRpSub = 2048;                     // rows per scatter sub-tile (unit of the staging layout)
constexpr int kRpRows = kRpSub / kRpSBlock;      // rows per thread per scatter sub-tile
constexpr int kRpMinTile = 4096;                 // rows per tile: a power of two in [kRpMinTile, kRpMaxTile],
constexpr int kRpMaxTile = 32768;                //   a multiple of both sub-tiles
constexpr int kRpHSub = 2048;                    // rows per hist sub-tile
constexpr int kRpHRows = kRpHSub / kRpBlock;
constexpr int kRpHScale = kRpHSub / kRpSub;      // hist staging offsets = layout offsets * kRpHScale
constexpr int kRpMaxStage = 8;                   // distinct input columns staged in LDS

constexpr int kRjBlock = 1024;
constexpr int kRjPerCu = 1;                      // join workgroups per CU (the LDS table takes the CU)
constexpr int kRjMaxVals = 2;                    // value words per probe tuple
constexpr int kRjUnroll = 4;                     // build keys per thread per round in k_rj_join
constexpr int kRjProbeUnroll = 4;                // probe tuples per thread per round in k_rj_join

__device__ __forceinline__ uint32_t region_of(uint64_t h, int pbits) {
  return pbits ? (uint32_t)(h >> (64 - pbits)) : 0u;
}
__device__ __forceinline__ uint32_t subregion_of(uint64_t h, int pbits, uint32_t S) {
  return S > 1 ? (uint32_t)__umul64hi(h << pbits, (uint64_t)S) : 0u;
}

struct RpArgs {
  int64_t n;               // input rows
  int64_t ntiles;          // hist tiles
  int64_t tile_rows;       // rows per tile (histogram and scatter alike)
  int32_t pbits;           // P = 1 << pbits regions
  int32_t npreds;
  int32_t probe;           // 0: build side (payload = row id), 1: probe side (aggregate inputs)
  int32_t nv;              // probe: value words per tuple
  int32_t need_nn;         // probe: tuples carry a non-NULL mask
  int32_t naggs;
  int32_t nst;             // staged input columns (predicates and key first, then values)
  int32_t nst_hist;        // of which the histogram pass needs the first nst_hist
  int32_t key_st;          // staged index of the key column
  int32_t in_bytes;        // LDS bytes of the staged input of one sub-tile
  DCol st[kRpMaxStage];
  int32_t st_off[kRpMaxStage];   // LDS byte offset of staged column j
  int32_t pred_st[GQ_MAX_PREDS];
  int32_t val_st[kMaxVals];      // staged index of aggregate value column v
  DPred preds[GQ_MAX_PREDS];
  AggPlan ap;
  int32_t vagg[kRjMaxVals];      // probe: aggregate whose input is value word j
  int32_t carry_st;              // probe: staged column whose value is the tuple's last word (-1: none)
  int32_t pad_carry;
  uint32_t* counts;        // [p * ntiles + tile]
  uint32_t* starts;        // exclusive scan of counts
  uint32_t* rtot;          // region totals of the column scan, zeroed by the histogram
  uint64_t* okey;          // build: (region hash, row) pairs; probe: tuples
  int32_t tw;              // probe: words per tuple (hash, then nv values), tuple i at okey[i * tw]
  int32_t pad_tw;
  uint8_t* onn;            // probe: non-NULL mask (bit i = aggregate i)
  int64_t ocap;
  // Two-level probe partition (k_rp1, k_rp2): the first level's tuples, a
  // slot of kRp1Sub tuples per sub-tile, and every sub-tile's run offsets.
  uint64_t* slots;
  uint16_t* roff;          // per sub-tile: kR1 + 1 offsets (the last the total)
};

// Copy rows [sbase, sbase + kRpSub) (those below n) of the first nst staged
// columns into LDS with 16-byte global-to-LDS loads (no register round trip:
// every load of the sub-tile is in flight at once); slices that are not
// 16-byte aligned, and the ragged end of a column, are copied byte by byte.
// The caller waits and synchronises the block before reading.
template <int BLOCK>
__device__ __forceinline__ void rp_stage(const RpArgs& a, int nst, int scale, int64_t sbase, int nrows,
                                         uint8_t* s_in) {
  for (int j = 0; j < nst; ++j) stage_col_lds<BLOCK>(a.st[j], sbase, nrows, s_in + a.st_off[j] * scale);
}

// The ROWS rows r = i * 256 + threadIdx.x of a staged column; one type
// dispatch for all of them.
template <int ROWS, int BLOCK>
__device__ __forceinline__ void lds_rows(const uint8_t* base, int type, int64_t (&v)[ROWS]) {
  const int t = threadIdx.x;
  switch (type) {
    case GQ_I8:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int8_t*>(base)[i * BLOCK + t];
      break;
    case GQ_I16:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int16_t*>(base)[i * BLOCK + t];
      break;
    case GQ_I32:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int32_t*>(base)[i * BLOCK + t];
      break;
    default:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int64_t*>(base)[i * BLOCK + t];
      break;
  }
}

// Rows r = i * 256 + threadIdx.x of the staged sub-tile at sbase: mask of the
// kept ones (predicates pass, key non-NULL) and their keys.  Column-major: each
// predicate is applied to all rows of the thread before the next.
template <int ROWS, int BLOCK>
__device__ __forceinline__ uint32_t rp_rows_keep(const RpArgs& a, const uint8_t* s_in, int scale, int64_t sbase,
                                                 int nrows, int64_t (&key)[ROWS]) {
  uint32_t keep = 0;
#pragma unroll
  for (int i = 0; i < ROWS; ++i)
    if (i * BLOCK + (int)threadIdx.x < nrows) keep |= 1u << i;
  for (int p = 0; p < a.npreds; ++p) {
    const int j = a.pred_st[p];
    const DCol& c = a.st[j];
    int64_t v[ROWS];
    lds_rows<ROWS, BLOCK>(s_in + a.st_off[j] * scale, c.type, v);
    const int64_t lo = a.preds[p].lo, hi = a.preds[p].hi;
    if (a.preds[p].op == GQ_RANGE) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (v[i] < lo || v[i] > hi) keep &= ~(1u << i);
    } else {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (v[i] == lo) keep &= ~(1u << i);
    }
    if (c.valid) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (((keep >> i) & 1u) && !valid_one(c, sbase + i * BLOCK + threadIdx.x)) keep &= ~(1u << i);
    }
  }
  const DCol& kc = a.st[a.key_st];
  lds_rows<ROWS, BLOCK>(s_in + a.st_off[a.key_st] * scale, kc.type, key);
  if (kc.valid) {
#pragma unroll
    for (int i = 0; i < ROWS; ++i)
      if (((keep >> i) & 1u) && !valid_one(kc, sbase + i * BLOCK + threadIdx.x)) keep &= ~(1u << i);
  }
  return keep;
}

// Aggregate input (product expression) of aggregate ag for staged row r; *nn
// is cleared when a referenced column is NULL (global row grow).
__device__ __forceinline__ uint64_t rp_value_row(const RpArgs& a, const DAgg& ag, const uint8_t* s_in, int r,
                                                 int64_t grow, bool* nn) {
  uint64_t x = 1;
  for (int f = 0; f < ag.nf; ++f) {
    const DFactor& fa = ag.f[f];
    const uint64_t k = (uint64_t)fa.k;
    if (fa.kind == GQ_F_CONST) {
      x *= k;
      continue;
    }
    const int j = a.val_st[fa.v];
    const uint64_t v = (uint64_t)lds_value(s_in + a.st_off[j], r, a.st[j].type);
    if (a.ap.vals[fa.v].valid && !valid_one(a.ap.vals[fa.v], grow)) *nn = false;
    if (fa.kind == GQ_F_COL) x *= v;
    else if (fa.kind == GQ_F_K_MINUS_COL) x *= k - v;
    else x *= k + v;
  }
  return x;
}

template <bool PROBE>  // a.probe; only names each side apart in kernel traces
__global__ __launch_bounds__(kRpBlock) void k_rp_hist(const RpArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int P = 1 << a.pbits;
  uint32_t* s_hist = reinterpret_cast<uint32_t*>(s_raw);
  uint8_t* s_in = s_raw + align_up((size_t)P * 4, 16);
  for (int i = threadIdx.x; i < P; i += kRpBlock) s_hist[i] = 0;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < P; i += kRpBlock) a.rtot[i] = 0;
  const int64_t tile = blockIdx.x;
  for (int64_t sub = 0; sub < a.tile_rows / kRpHSub; ++sub) {
    const int64_t sbase = tile * a.tile_rows + sub * kRpHSub;
    if (sbase >= a.n) break;
    const int nrows = a.n - sbase < kRpHSub ? (int)(a.n - sbase) : kRpHSub;
    __syncthreads();  // previous sub-tile's rows read
    rp_stage<kRpBlock>(a, a.nst_hist, kRpHScale, sbase, nrows, s_in);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int64_t key[kRpHRows];
    const uint32_t keep = rp_rows_keep<kRpHRows, kRpBlock>(a, s_in, kRpHScale, sbase, nrows, key);
#pragma unroll
    for (int i = 0; i < kRpHRows; ++i)
      if ((keep >> i) & 1u) atomicAdd(&s_hist[region_of(region_hash((uint64_t)key[i]), a.pbits)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += kRpBlock) a.counts[tile * P + i] = s_hist[i];
}

// Column scan of the tile-major counts (count of region q in tile t at
// counts[t * P + q]; all of them fit 32 bits since a batch has fewer than 2^32
// rows): starts[t * P + q] = offsets[q] + the counts of region q in tiles
// before t, offsets[q] = the counts of all regions before q.
constexpr int kCsChunk = 64;  // tiles per chunk

// Per chunk of tiles and region: the sum of the chunk's counts, also added to
// the region's total (zeroed before).
__global__ __launch_bounds__(256) void k_cs_chunk(const uint32_t* counts, int64_t ntiles, int P, uint32_t* csum,
                                                  uint32_t* tot) {
  const int q = blockIdx.y * 256 + threadIdx.x;
  if (q >= P) return;
  const int64_t t0 = (int64_t)blockIdx.x * kCsChunk;
  const int64_t t1 = t0 + kCsChunk < ntiles ? t0 + kCsChunk : ntiles;
  uint32_t sum = 0;
#pragma unroll 8
  for (int64_t t = t0; t < t1; ++t) sum += counts[t * P + q];
  csum[(int64_t)blockIdx.x * P + q] = sum;
  if (sum) atomicAdd(&tot[q], sum);
}

// Per chunk of tiles and region: the start of the region's rows in each tile.
// Every block first derives its regions' offsets from the region totals (the
// totals of the regions before its 256, then a block scan of its own); the
// blocks of the first chunk also store offsets[0..P] and the total.
__global__ __launch_bounds__(256) void k_cs_fill(const uint32_t* counts, const uint32_t* csum, const uint32_t* rtot,
                                                 int64_t ntiles, int P, uint32_t* starts, int64_t* offsets,
                                                 int64_t* total) {
  constexpr int NW = 256 / kWave;
  __shared__ int64_t s_before[NW];
  __shared__ int64_t s_wave[NW];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int q0 = blockIdx.y * 256;
  const int q = q0 + (int)threadIdx.x;
  int64_t before = 0;
  for (int i = threadIdx.x; i < q0; i += 256) before += rtot[i];
  const int64_t mine = q < P ? (int64_t)rtot[q] : 0;
  int64_t incl = mine;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
    before += __shfl_xor(before, o, kWave);
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  if (lane == 0) s_before[wave] = before;
  __syncthreads();
  int64_t base = 0, wpre = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    base += s_before[w];
    if (w < wave) wpre += s_wave[w];
    btot += s_wave[w];
  }
  const int64_t off = base + wpre + incl - mine;
  if (blockIdx.x == 0) {
    if (q < P) offsets[q] = off;
    if (blockIdx.y == gridDim.y - 1 && threadIdx.x == 0) {
      offsets[P] = base + btot;
      if (total) *total = base + btot;
    }
  }
  if (q >= P) return;
  const int64_t c = blockIdx.x;
  uint32_t run = (uint32_t)off;
#pragma unroll 8
  for (int64_t k = 0; k < c; ++k) run += csum[k * P + q];
  const int64_t t0 = c * kCsChunk;
  const int64_t t1 = t0 + kCsChunk < ntiles ? t0 + kCsChunk : ntiles;
#pragma unroll 8
  for (int64_t t = t0; t < t1; ++t) {
    const uint32_t v = counts[t * P + q];
    starts[t * P + q] = run;
    run += v;
  }
}

// LDS layout of k_rp_scatter (dynamic): the tile's next write position of
// every region (u32), then two buffers of staged input (in_bytes each).
__host__ __device__ inline size_t rp_scatter_lds(int P, int in_bytes) {
  return align_up((size_t)P * 4, 16) + 2 * align_up((size_t)in_bytes, 16);
}

// Per tile, sub-tiles of kRpSub rows staged in LDS, double-buffered: the
// global-to-LDS loads of sub-tile k + 1 are issued before sub-tile k is
// processed, so they are in flight during its LDS atomics and scattered
// stores; one wait and one barrier per sub-tile.
// PROBE is a.probe fixed at compile time: each side gets its own code (and
// its own name in kernel traces).
template <bool PROBE>
__global__ __launch_bounds__(kRpSBlock) void k_rp_scatter(const RpArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int P = 1 << a.pbits;
  uint32_t* s_pos = reinterpret_cast<uint32_t*>(s_raw);
  uint8_t* s_buf0 = s_raw + align_up((size_t)P * 4, 16);
  const size_t bstride = align_up((size_t)a.in_bytes, 16);
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t tbase = tile * a.tile_rows;
  const int64_t trows = a.n - tbase < a.tile_rows ? a.n - tbase : a.tile_rows;
  const int64_t nsub = (trows + kRpSub - 1) / kRpSub;
  for (int q = threadIdx.x; q < P; q += kRpSBlock) s_pos[q] = a.starts[tile * P + q];
  rp_stage<kRpSBlock>(a, a.nst, 1, tbase, trows < kRpSub ? (int)trows : kRpSub, s_buf0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t sub = 0; sub < nsub; ++sub) {
    const int64_t sbase = tbase + sub * kRpSub;
    const int nrows = a.n - sbase < kRpSub ? (int)(a.n - sbase) : kRpSub;
    const uint8_t* s_in = s_buf0 + (sub & 1) * bstride;
    if (sub + 1 < nsub) {
      const int64_t nbase = sbase + kRpSub;
      rp_stage<kRpSBlock>(a, a.nst, 1, nbase, a.n - nbase < kRpSub ? (int)(a.n - nbase) : kRpSub,
                          s_buf0 + ((sub + 1) & 1) * bstride);
    }
    int64_t key[kRpRows];
    const uint32_t keep = rp_rows_keep<kRpRows, kRpSBlock>(a, s_in, 1, sbase, nrows, key);
#pragma unroll
    for (int i = 0; i < kRpRows; ++i) {
      if (!((keep >> i) & 1u)) continue;
      const int r = i * kRpSBlock + threadIdx.x;
      const uint64_t h = region_hash((uint64_t)key[i]);
      const int64_t g = atomicAdd(&s_pos[region_of(h, a.pbits)], 1u);
      if (g >= a.ocap) continue;
      if constexpr (PROBE) {
        // The tuple (hash and values side by side) is one contiguous store;
        // values come from the staged input.
        uint64_t* t = a.okey + (size_t)g * a.tw;
        uint64_t x[kRjMaxVals] = {0, 0};
#pragma unroll
        for (int v = 0; v < kRjMaxVals; ++v) {
          if (v >= a.nv) break;
          bool nn = true;
          x[v] = rp_value_row(a, a.ap.aggs[a.vagg[v]], s_in, r, sbase + r, &nn);
        }
        if (a.carry_st >= 0) {
          // Hash, values, then the carried column's value.
          t[0] = h;
#pragma unroll
          for (int v = 0; v < kRjMaxVals; ++v)
            if (v < a.nv) t[1 + v] = x[v];
          t[1 + a.nv] = (uint64_t)lds_value(s_in + a.st_off[a.carry_st], r, a.st[a.carry_st].type);
        } else if (a.nv == 1) {
          typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
          *reinterpret_cast<u64x2*>(t) = u64x2{h, x[0]};
        } else {
          t[0] = h;
#pragma unroll
          for (int v = 0; v < kRjMaxVals; ++v)
            if (v < a.nv) t[1 + v] = x[v];
        }
        if (a.need_nn) {
          uint32_t nnm = 0;
          for (int gi = 0; gi < a.naggs; ++gi) {
            const DAgg& ag = a.ap.aggs[gi];
            if (ag.op == GQ_COUNT_STAR) continue;
            bool ok = true;
            for (int f = 0; f < ag.nf; ++f) {
              if (ag.f[f].kind == GQ_F_CONST) continue;
              const DCol& c = a.ap.vals[ag.f[f].v];
              if (c.valid && !valid_one(c, sbase + r)) ok = false;
            }
            nnm |= (ok ? 1u : 0u) << gi;
          }
          a.onn[g] = (uint8_t)nnm;
        }
      } else {
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
        *reinterpret_cast<u64x2*>(a.okey + 2 * (size_t)g) = u64x2{h, (uint64_t)(sbase + r)};
      }
    }
    // The next sub-tile's loads have landed (every thread's), and every thread
    // is done with this buffer before it is refilled.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Two-level probe partition
// ---------------------------------------------------------------------------
// With thousands of regions a sub-tile of the single-level scatter holds a row
// or two per region, so it writes one 16-byte tuple per region and sub-tile,
// and those scattered stores, not the bytes, set its time; its histogram pass
// also re-reads the key and predicate columns.  The probe side (tuples without
// a non-NULL mask, P >= 256) instead sorts by kR1 = 32 first-level regions
// (the top 5 bits of the region hash) inside each sub-tile, and then moves
// every first-level region's tuples to their final regions:
//   k_rp1      per tile, sub-tiles of SUB = 1024 rows staged in LDS (512
//              threads, several workgroups per CU): the kept rows' tuples
//              sorted by first-level region in LDS and written out whole, one
//              contiguous store stream per sub-tile, into the sub-tile's own
//              slot of SUB tuples, with the sub-tile's kR1 + 1 run offsets;
//              the tile's tuple count per final region is counted in LDS on
//              the way and stored at the end.  No device atomics and no
//              histogram pass.
//   k_cs_*     the column scan of those (tile, region) counts (as for the
//              single-level path): the start of every (tile, region) and the
//              region offsets.
//   k_rp2      one workgroup per (first-level region, group of G tiles): the
//              group's runs of that region (one per sub-tile, about 16 tuples
//              each) gathered in rounds of up to kRp2Round tuples, ranked by
//              final region in LDS and written out sorted: the group's tuples
//              of final region q go to [start(first tile, q), ...), so every
//              position is exact (no atomics) and the stores form runs.
// The order of tuples inside a region is unspecified, as with the
// single-level scatter.
constexpr int kR1Bits = 5;
constexpr int kR1 = 1 << kR1Bits;       // first-level regions
constexpr int kRp1Block = 512;
constexpr int kRp1Sub = 2 * kRp1Block;   // rows per sub-tile (and tuples per slot)
constexpr int kRp2Block = 256;
constexpr int kRp2Round = 2048;          // tuples per round of k_rp2
constexpr int kRp2Items = kRp2Round / kRp2Block;
constexpr int kRp2MaxRuns = kRp2Block;   // runs per k_rp2 workgroup (G * sub-tiles per tile): one per thread

// A probe tuple of up to four words (named fields: no indexed array, so it
// stays in registers).
struct Tup4 {
  uint64_t w0, w1, w2, w3;
};

// The tuples carry no non-NULL mask, so a value's NULL inputs are not looked
// up (its value is then unspecified and never aggregated).
__device__ __forceinline__ uint64_t rp_value_nn(const RpArgs& a, const DAgg& ag, const uint8_t* s_in, int r) {
  uint64_t x = 1;
  for (int f = 0; f < ag.nf; ++f) {
    const DFactor& fa = ag.f[f];
    const uint64_t k = (uint64_t)fa.k;
    if (fa.kind == GQ_F_CONST) {
      x *= k;
      continue;
    }
    const int j = a.val_st[fa.v];
    const uint64_t v = (uint64_t)lds_value(s_in + a.st_off[j], r, a.st[j].type);
    if (fa.kind == GQ_F_COL) x *= v;
    else if (fa.kind == GQ_F_K_MINUS_COL) x *= k - v;
    else x *= k + v;
  }
  return x;
}

// Tuple words of staged row r: hash, value words, carried value.
__device__ __forceinline__ Tup4 rp_tuple(const RpArgs& a, const uint8_t* s_in, int r, uint64_t h) {
  Tup4 t{h, 0, 0, 0};
  if (a.nv >= 1) t.w1 = rp_value_nn(a, a.ap.aggs[a.vagg[0]], s_in, r);
  if (a.nv >= 2) t.w2 = rp_value_nn(a, a.ap.aggs[a.vagg[1]], s_in, r);
  if (a.carry_st >= 0) {
    const uint64_t cv = (uint64_t)lds_value(s_in + a.st_off[a.carry_st], r, a.st[a.carry_st].type);
    if (a.nv == 0) t.w1 = cv;
    else if (a.nv == 1) t.w2 = cv;
    else t.w3 = cv;
  }
  return t;
}

__device__ __forceinline__ void rp_put_tuple(uint64_t* dst, const Tup4& t, int tw) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  *reinterpret_cast<u64x2*>(dst) = u64x2{t.w0, t.w1};
  if (tw >= 3) dst[2] = t.w2;
  if (tw >= 4) dst[3] = t.w3;
}

__device__ __forceinline__ Tup4 rp_get_tuple(const uint64_t* src, int tw) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  const u64x2 v = *reinterpret_cast<const u64x2*>(src);
  Tup4 t{v.x, v.y, 0, 0};
  if (tw >= 3) t.w2 = src[2];
  if (tw >= 4) t.w3 = src[3];
  return t;
}

// The same with the tuple width known at compile time (unused words stay 0
// and take no registers).
template <int TW>
__device__ __forceinline__ Tup4 rp_get_tuple_t(const uint64_t* src) {
  return rp_get_tuple(src, TW);
}
template <int TW>
__device__ __forceinline__ void rp_put_tuple_t(uint64_t* dst, const Tup4& t) {
  rp_put_tuple(dst, t, TW);
}

// Kept rows (predicates pass, key non-NULL) of the staged sub-tile and their
// keys, as rp_rows_keep; NULLABLE = false drops the bitmap lookups (no staged
// column has one).
template <int ROWS, int BLOCK, bool NULLABLE>
__device__ __forceinline__ uint32_t rp1_keep(const RpArgs& a, const uint8_t* s_in, int64_t sbase, int nrows,
                                             int64_t (&key)[ROWS]) {
  if constexpr (NULLABLE) return rp_rows_keep<ROWS, BLOCK>(a, s_in, 1, sbase, nrows, key);
  uint32_t keep = 0;
#pragma unroll
  for (int i = 0; i < ROWS; ++i)
    if (i * BLOCK + (int)threadIdx.x < nrows) keep |= 1u << i;
  for (int p = 0; p < a.npreds; ++p) {
    const int j = a.pred_st[p];
    int64_t v[ROWS];
    lds_rows<ROWS, BLOCK>(s_in + a.st_off[j], a.st[j].type, v);
    const int64_t lo = a.preds[p].lo, hi = a.preds[p].hi;
    if (a.preds[p].op == GQ_RANGE) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (v[i] < lo || v[i] > hi) keep &= ~(1u << i);
    } else {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (v[i] == lo) keep &= ~(1u << i);
    }
  }
  lds_rows<ROWS, BLOCK>(s_in + a.st_off[a.key_st], a.st[a.key_st].type, key);
  return keep;
}

// Dynamic LDS of k_rp1: packed 16-bit tuple counts of the P final regions,
// the staged input (laid out for kRp1Sub rows) and the sorted tuples.
__host__ __device__ inline size_t rp1_lds(int P, int in_bytes, int tw) {
  return align_up((size_t)P * 2, 16) + align_up((size_t)in_bytes, 16) + (size_t)kRp1Sub * tw * 8;
}

// With NPF > 0 (every staged column 16-byte aligned, NPF of them) the next
// sub-tile is loaded into registers while the current one is processed (a column of a
// sub-tile is at most kRp1Block 16-byte chunks: one per thread) and written
// to LDS once the current input is no longer read, before any store of the
// sub-tile is issued.  (Global-to-LDS loads would not overlap: every LDS write
// or atomic issued after one waits for it.)  Barriers order LDS only, so the
// stores of a sub-tile stay in flight while the next one is processed.
constexpr int kRp1MaxPf = 5;  // staged columns prefetched through registers at most

template <bool NULLABLE, int NPF>  // NPF: staged columns (all 16-byte aligned) prefetched; 0: none
__global__ __launch_bounds__(kRp1Block) __attribute__((amdgpu_waves_per_eu(6))) void k_rp1(const RpArgs a) {
  constexpr int BLOCK = kRp1Block, SUB = kRp1Sub, ROWS = 2;
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  __shared__ uint32_t s_cnt[kR1], s_off[kR1 + 1];
  const int P = 1 << a.pbits;
  const int tw = a.tw;
  uint32_t* s_fin = reinterpret_cast<uint32_t*>(s_raw);
  uint8_t* s_in = s_raw + align_up((size_t)P * 2, 16);
  uint64_t* s_tup = reinterpret_cast<uint64_t*>(s_in + align_up((size_t)a.in_bytes, 16));
  const int64_t tile = blockIdx.x;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t tbase = tile * a.tile_rows;
  const int64_t trows = a.n - tbase < a.tile_rows ? a.n - tbase : a.tile_rows;
  const int64_t nsub = (trows + SUB - 1) / SUB;
  const int64_t subs = a.tile_rows / SUB;
  for (int i = threadIdx.x; i < P / 2; i += BLOCK) s_fin[i] = 0;
  if (threadIdx.x < kR1) s_cnt[threadIdx.x] = 0;
  if (tile == 0)
    for (int q = threadIdx.x; q < P; q += BLOCK) a.rtot[q] = 0;
  rp_stage<BLOCK>(a, a.nst, 1, tbase, trows < SUB ? (int)trows : SUB, s_in);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t sub = 0; sub < nsub; ++sub) {
    const int64_t sbase = tbase + sub * SUB;
    const int nrows = a.n - sbase < SUB ? (int)(a.n - sbase) : SUB;
    const int64_t nbase = sbase + SUB;
    const bool has_next = sub + 1 < nsub;
    const bool pf = NPF > 0 && has_next && a.n - nbase >= SUB;
    u32x4 pfv[NPF > 0 ? NPF : 1];
#pragma unroll
    for (int j = 0; j < (NPF > 0 ? NPF : 1); ++j) pfv[j] = u32x4{0u, 0u, 0u, 0u};
    if (pf) {
#pragma unroll
      for (int j = 0; j < NPF; ++j) {
        const int w = type_width(a.st[j].type);
        if ((int)threadIdx.x < SUB * w / 16)
          pfv[j] = *reinterpret_cast<const u32x4*>(a.st[j].data + nbase * w + (int64_t)threadIdx.x * 16);
      }
    }
    int64_t key[ROWS];
    const uint32_t keep = rp1_keep<ROWS, BLOCK, NULLABLE>(a, s_in, sbase, nrows, key);
    uint64_t h[ROWS];
    uint32_t rank[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      h[i] = 0;
      rank[i] = 0;
      if (!((keep >> i) & 1u)) continue;
      h[i] = region_hash((uint64_t)key[i]);
      const uint32_t q = region_of(h[i], a.pbits);
      atomicAdd(&s_fin[q >> 1], 1u << ((q & 1u) << 4));
      rank[i] = atomicAdd(&s_cnt[(uint32_t)(h[i] >> (64 - kR1Bits))], 1u);
    }
    lds_barrier();
    // Run offsets of the sub-tile (kR1 + 1 of them, the last the total).
    if (wave == 0) {
      const uint32_t c = lane < kR1 ? s_cnt[lane] : 0u;
      uint32_t tot;
      const uint32_t pre = wave_prefix_small<12>(c, &tot);
      if (lane <= kR1) s_off[lane] = lane < kR1 ? pre : tot;
      if (lane < kR1) s_cnt[lane] = 0;
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      if (!((keep >> i) & 1u)) continue;
      const int r = i * BLOCK + threadIdx.x;
      const uint32_t pos = s_off[(uint32_t)(h[i] >> (64 - kR1Bits))] + rank[i];
      // Probe: hash and aggregate inputs; build: hash and row.
      const Tup4 tup = a.probe ? rp_tuple(a, s_in, r, h[i]) : Tup4{h[i], (uint64_t)(sbase + r), 0, 0};
      rp_put_tuple(s_tup + (size_t)pos * tw, tup, tw);
    }
    // The sorted tuples are complete and the staged input is no longer read.
    lds_barrier();
    if (pf) {
#pragma unroll
      for (int j = 0; j < NPF; ++j) {
        const int w = type_width(a.st[j].type);
        if ((int)threadIdx.x < SUB * w / 16)
          *reinterpret_cast<u32x4*>(s_in + a.st_off[j] + (int64_t)threadIdx.x * 16) = pfv[j];
      }
    } else if (has_next) {
      rp_stage<BLOCK>(a, a.nst, 1, nbase, a.n - nbase < SUB ? (int)(a.n - nbase) : SUB, s_in);
    }
    // The sorted tuples leave as one contiguous stream into the slot.
    const int64_t slot = tile * subs + sub;
    const int total = (int)s_off[kR1];
    if ((int)threadIdx.x <= kR1) a.roff[slot * (kR1 + 1) + threadIdx.x] = (uint16_t)s_off[threadIdx.x];
    uint64_t* dst = a.slots + (size_t)slot * SUB * tw;
    if (tw == 2) {
      typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
      for (int k = threadIdx.x; k < total; k += BLOCK)
        reinterpret_cast<u64x2*>(dst)[k] = reinterpret_cast<const u64x2*>(s_tup)[k];
    } else {
      for (int k = threadIdx.x; k < total * tw; k += BLOCK) dst[k] = s_tup[k];
    }
    if (!pf && has_next) __builtin_amdgcn_s_waitcnt(0);
    // The next sub-tile is in LDS and the sorted buffer is free.
    lds_barrier();
  }
  // Sub-tiles past the end of the input: empty runs.
  for (int64_t sub = nsub; sub < subs; ++sub)
    if (threadIdx.x <= kR1) a.roff[(tile * subs + sub) * (kR1 + 1) + threadIdx.x] = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < P; q += BLOCK)
    a.counts[tile * P + q] = (s_fin[q >> 1] >> ((q & 1) << 4)) & 0xffffu;
}

// Dynamic LDS of k_rp2: the sorted tuples of a round and their sub-regions.
__host__ __device__ inline size_t rp2_lds(int tw) { return (size_t)kRp2Round * tw * 8 + kRp2Round; }

// Workgroup b: first-level region r1 = b % kR1, tiles [g G, g G + G) with
// g = b / kR1.  Its tuples of final region q = r1 * S2 + s go to consecutive
// positions from start(first tile, q): within a region, tuples are ordered by
// tile, and the group's tiles are consecutive.
template <int TW>
__global__ __launch_bounds__(kRp2Block) void k_rp2(const RpArgs a, int32_t group) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  __shared__ uint32_t s_rbeg[kRp2MaxRuns];      // first tuple of every run (slot index * SUB + offset)
  __shared__ uint32_t s_rpre[kRp2MaxRuns + 1];  // exclusive prefix of the run lengths
  __shared__ uint32_t s_cnt[1 << (12 - kR1Bits)], s_off[1 << (12 - kR1Bits)];
  __shared__ uint32_t s_cur[1 << (12 - kR1Bits)];
  __shared__ uint32_t s_wsum[kRp2Block / kWave];
  constexpr int tw = TW;
  const int S2 = 1 << (a.pbits - kR1Bits);
  const int P = 1 << a.pbits;
  uint64_t* s_tup = reinterpret_cast<uint64_t*>(s_raw);
  uint8_t* s_sid = reinterpret_cast<uint8_t*>(s_tup + (size_t)kRp2Round * tw);
  // The kR1 workgroups of a tile group are dispatched together, one XCD
  // after another; the kR1 / kXcds first-level regions that share an XCD are
  // adjacent, so the lines their runs share in a slot are read once into that
  // XCD's L2.
  static_assert(kR1 % kXcds == 0, "first-level regions spread evenly over the XCDs");
  const int k = (int)(blockIdx.x % kR1);
  const int r1 = (k % kXcds) * (kR1 / kXcds) + k / kXcds;
  const int64_t t0 = (int64_t)(blockIdx.x / kR1) * group;
  const int64_t t1 = t0 + group < a.ntiles ? t0 + group : a.ntiles;
  const int64_t subs = a.tile_rows / kRp1Sub;
  const int nruns = (int)((t1 - t0) * subs);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  // Runs: lengths, then their prefix (one run per thread).
  uint32_t len = 0;
  if ((int)threadIdx.x < nruns) {
    const int64_t slot = t0 * subs + threadIdx.x;
    const uint16_t* ro = a.roff + slot * (kR1 + 1) + r1;
    const uint32_t b = ro[0];
    len = (uint32_t)ro[1] - b;
    s_rbeg[threadIdx.x] = (uint32_t)(slot * kRp1Sub) + b;
  }
  uint32_t incl = len;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) s_wsum[wave] = incl;
  for (int s = threadIdx.x; s < S2; s += kRp2Block) {
    s_cnt[s] = 0;
    s_cur[s] = a.starts[t0 * P + r1 * S2 + s];
  }
  __syncthreads();
  uint32_t wpre = 0, total = 0;
  for (int w = 0; w < kRp2Block / kWave; ++w) {
    if (w < wave) wpre += s_wsum[w];
    total += s_wsum[w];
  }
  if ((int)threadIdx.x < nruns) s_rpre[threadIdx.x] = wpre + incl - len;
  if (threadIdx.x == 0) s_rpre[nruns] = total;
  __syncthreads();
  for (uint32_t base = 0; base < total; base += kRp2Round) {
    const uint32_t nr = total - base < (uint32_t)kRp2Round ? total - base : (uint32_t)kRp2Round;
    Tup4 t[kRp2Items];
    uint32_t sid[kRp2Items], rk[kRp2Items];
#pragma unroll
    for (int i = 0; i < kRp2Items; ++i) {
      const uint32_t k = (uint32_t)(i * kRp2Block + threadIdx.x);
      t[i] = Tup4{0, 0, 0, 0};
      if (k < nr) {
        // The run holding tuple base + k: the last run starting at or before it.
        const uint32_t x = base + k;
        int lo = 0, hi = nruns - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_rpre[mid] <= x) lo = mid;
          else hi = mid - 1;
        }
        t[i] = rp_get_tuple_t<TW>(a.slots + (size_t)(s_rbeg[lo] + (x - s_rpre[lo])) * tw);
      }
    }
#pragma unroll
    for (int i = 0; i < kRp2Items; ++i) {
      const uint32_t k = (uint32_t)(i * kRp2Block + threadIdx.x);
      sid[i] = 0;
      rk[i] = 0;
      if (k >= nr) continue;
      sid[i] = region_of(t[i].w0, a.pbits) & (uint32_t)(S2 - 1);
      rk[i] = atomicAdd(&s_cnt[sid[i]], 1u);
    }
    __syncthreads();
    if (wave == 0) {
      // Exclusive prefix of the S2 <= 128 counts, two per lane.
      const uint32_t c0 = 2 * lane < S2 ? s_cnt[2 * lane] : 0u;
      const uint32_t c1 = 2 * lane + 1 < S2 ? s_cnt[2 * lane + 1] : 0u;
      uint32_t tot;
      const uint32_t pre = wave_prefix_small<14>(c0 + c1, &tot);
      if (2 * lane < S2) s_off[2 * lane] = pre;
      if (2 * lane + 1 < S2) s_off[2 * lane + 1] = pre + c0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRp2Items; ++i) {
      const uint32_t k = (uint32_t)(i * kRp2Block + threadIdx.x);
      if (k >= nr) continue;
      const uint32_t pos = s_off[sid[i]] + rk[i];
      rp_put_tuple_t<TW>(s_tup + (size_t)pos * tw, t[i]);
      s_sid[pos] = (uint8_t)sid[i];
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nr; k += kRp2Block) {
      const uint32_t s = s_sid[k];
      const int64_t dst = (int64_t)s_cur[s] + (int64_t)(k - s_off[s]);
      if (dst >= a.ocap) continue;
      rp_put_tuple_t<TW>(a.okey + (size_t)dst * tw, rp_get_tuple_t<TW>(s_tup + (size_t)k * tw));
    }
    __syncthreads();
    for (int s = threadIdx.x; s < S2; s += kRp2Block) {
      s_cur[s] += s_cnt[s];
      s_cnt[s] = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Register-path histogram (every column it reads 16-byte aligned)
// ---------------------------------------------------------------------------
// A lane takes two consecutive rows per step and loads, for every column, the
// aligned 16-byte chunk that holds both (one load instruction per column
// whatever its width; no type-dependent branch before the loads, so the loads
// of all columns are in flight together), then extracts the two values.  The
// next step's chunks are loaded before the current step is processed, and
// there is no barrier inside the row loop: the waves of a workgroup stream
// through their tile independently, so the loads and LDS atomics of many
// waves overlap.  Rows within 16 of the end of the input are loaded one by one
// (a chunk there could pass the column's end).  The same scheme for the
// scatter measured slower than staging through LDS (its scattered stores then
// compete with the loads of every wave), so the scatter keeps the staged form.
constexpr int kRpItems = 2;

// Raw chunks of the NS staged columns for one step: halves lo[j], hi[j] of
// column j's chunk, or (in the tail) the two rows' values.  Two plain arrays
// rather than an array of structs, so that they stay in registers.
template <int NS>
struct RawStep {
  uint64_t lo[NS];
  uint64_t hi[NS];
};

// One branch around all loads (not one per column): on the usual path every
// chunk load is issued back to back with no wait in between.
template <int NS>
__device__ __forceinline__ void rp_raw(const RpArgs& a, int64_t r0, bool full, RawStep<NS>& raw) {
  if (full) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const DCol& c = a.st[j];
      const int w = type_width(c.type);
      const uint8_t* p = c.data + ((r0 * w) & ~(int64_t)15);
      const gq_v4i x = __builtin_nontemporal_load(reinterpret_cast<const gq_v4i*>(p));
      raw.lo[j] = ((uint64_t)(uint32_t)x.y << 32) | (uint32_t)x.x;
      raw.hi[j] = ((uint64_t)(uint32_t)x.w << 32) | (uint32_t)x.z;
    }
  } else {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const DCol& c = a.st[j];
      raw.lo[j] = r0 < a.n ? (uint64_t)load_one(c, r0) : 0;
      raw.hi[j] = r0 + 1 < a.n ? (uint64_t)load_one(c, r0 + 1) : 0;
    }
  }
}

// The two rows' values of staged column j (sign-extended).
__device__ __forceinline__ void rp_decode(const DCol& c, int64_t r0, bool full, uint64_t lo, uint64_t hi,
                                          int64_t (&v)[2]) {
  if (!full || c.type == GQ_I64) {
    v[0] = (int64_t)lo;
    v[1] = (int64_t)hi;
    return;
  }
  const int w = type_width(c.type);
  const int off = (int)((r0 * w) & 15);
  const uint64_t u = ((off & 8) ? hi : lo) >> ((off & 7) * 8);
  switch (c.type) {
    case GQ_I8: v[0] = (int8_t)u; v[1] = (int8_t)(u >> 8); break;
    case GQ_I16: v[0] = (int16_t)u; v[1] = (int16_t)(u >> 16); break;
    default: v[0] = (int32_t)u; v[1] = (int32_t)(u >> 32); break;
  }
}

// Rows r0, r0 + 1: the kept mask (below t1, predicates pass, key non-NULL)
// and the region hashes of their keys.  The staged columns are visited in a
// static loop and each role (predicate, key) tests whether it reads column j,
// so that the register arrays are only ever indexed by compile-time constants
// (an array indexed at run time would be placed in scratch memory).
template <int NS>
__device__ __forceinline__ uint32_t rp_eval_r(const RpArgs& a, int64_t r0, int64_t t1, bool full,
                                              const RawStep<NS>& raw, uint64_t (&h)[2]) {
  uint32_t keep = (r0 < t1 ? 1u : 0u) | (r0 + 1 < t1 ? 2u : 0u);
  int64_t kv[2] = {0, 0};
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const DCol& c = a.st[j];
    int64_t v[2];
    rp_decode(c, r0, full, raw.lo[j], raw.hi[j], v);
    for (int p = 0; p < a.npreds; ++p) {
      if (a.pred_st[p] != j) continue;
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (!pred_pass(a.preds[p], v[k])) keep &= ~(1u << k);
      if (c.valid) keep &= valid_items<2>(c, r0, a.n);
    }
    if (a.key_st == j) {
      kv[0] = v[0];
      kv[1] = v[1];
      if (c.valid) keep &= valid_items<2>(c, r0, a.n);
    }
  }
  h[0] = region_hash((uint64_t)kv[0]);
  h[1] = region_hash((uint64_t)kv[1]);
  return keep;
}

// One step of the histogram: the two rows' regions counted in LDS.
template <int NS>
__device__ __forceinline__ void rp_hist_step(const RpArgs& a, int64_t r0, int64_t t1, bool full,
                                             const RawStep<NS>& raw, uint32_t* s_hist) {
  uint64_t h[2];
  const uint32_t keep = rp_eval_r<NS>(a, r0, t1, full, raw, h);
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if ((keep >> k) & 1u) atomicAdd(&s_hist[region_of(h[k], a.pbits)], 1u);
}

// The row loop of a tile: a lane's steps r0 = t0 + 2 * lane + k * 512.  In
// every tile but the one that ends within 16 rows of the input's end, every
// step reads whole chunks, and two register sets alternate: the loads of
// step k + 1 (unconditional: past the tile they re-read step k's chunks, so
// the number in flight is fixed and the wait before step k's use covers step
// k's loads only) are issued before step k is processed, and no register copy
// waits for loads in flight.  The last tile takes its steps one at a time.
template <int NS>
__device__ __forceinline__ void rp_hist_tile(const RpArgs& a, int64_t t0, int64_t t1, uint32_t* s_hist) {
  constexpr int64_t STEP = (int64_t)kRpBlock * kRpItems;
  int64_t r0 = t0 + (int64_t)threadIdx.x * kRpItems;
  if (t1 + 16 > a.n) {
    RawStep<NS> raw;
    for (; r0 < t1; r0 += STEP) {
      const bool full = r0 + 16 <= a.n;
      rp_raw<NS>(a, r0, full, raw);
      rp_hist_step<NS>(a, r0, t1, full, raw, s_hist);
    }
    return;
  }
  RawStep<NS> ra, rb;
  if (r0 >= t1) return;
  rp_raw<NS>(a, r0, true, ra);
  for (;;) {
    int64_t rn = r0 + STEP;
    rp_raw<NS>(a, rn < t1 ? rn : r0, true, rb);
    rp_hist_step<NS>(a, r0, t1, true, ra, s_hist);
    if (rn >= t1) break;
    r0 = rn;
    rn = r0 + STEP;
    rp_raw<NS>(a, rn < t1 ? rn : r0, true, ra);
    rp_hist_step<NS>(a, r0, t1, true, rb, s_hist);
    if (rn >= t1) break;
    r0 = rn;
  }
}

// Per tile, the histogram of the kept rows' regions (see k_rp_hist).
template <int NS, bool PROBE>  // PROBE = a.probe; only names each side apart in kernel traces
__global__ __launch_bounds__(kRpBlock) void k_rp_hist_r(const RpArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t s_hist[];
  const int P = 1 << a.pbits;
  for (int i = threadIdx.x; i < P; i += kRpBlock) s_hist[i] = 0;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < P; i += kRpBlock) a.rtot[i] = 0;
  __syncthreads();
  const int64_t tile = blockIdx.x;
  const int64_t t0 = tile * a.tile_rows;
  const int64_t t1 = t0 + a.tile_rows < a.n ? t0 + a.tile_rows : a.n;
  rp_hist_tile<NS>(a, t0, t1, s_hist);
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += kRpBlock) a.counts[tile * P + i] = s_hist[i];
}

// ---------------------------------------------------------------------------
// Join and aggregation of (region, sub-region) items
// ---------------------------------------------------------------------------
struct RjJoinArgs {
  int32_t pbits;
  int32_t P;
  int32_t lcap;             // LDS table slots; slot lcap holds the hash EMPTY
  int32_t kpr;              // build rows per sub-region at most
  int32_t nacc;
  int32_t naggs;
  int32_t nv;
  int32_t need_nn;
  AggPlan ap;
  int32_t vword[GQ_MAX_AGGS];   // value word of aggregate i in the tuple, -1 if none
  int32_t sums_only;            // every aggregate is COUNT(*) or a SUM of a non-NULL input
  int32_t sum_word[kRjMaxVals]; // then: accumulator word of value word v
  // Emission of aggregate i (all output columns 8 bytes wide: emit64): its
  // accumulator word, whether the build multiplicity scales it (SUM, COUNT,
  // COUNT(*)), and the count word that makes it NULL when zero (-1: never).
  // Plain arrays read at constant offsets, so that they stay in scalar
  // registers for the whole item instead of being re-read per slot.
  int32_t emit64;
  int32_t e_word[GQ_MAX_AGGS];
  int32_t e_mul[GQ_MAX_AGGS];
  int32_t e_cword[GQ_MAX_AGGS];
  uint64_t ident[kMaxAcc];      // initial value of every accumulator word (word_identity of its wop)
  const uint64_t* bkey;     // build (key hash, row) pairs grouped by region
  const int64_t* boff;      // P + 1
  const uint64_t* tkey;     // probe tuple key hashes grouped by region
  int32_t tw;               // words per probe tuple: hash, then nv values (then the carried value)
  int32_t pad_tw;
  int64_t carry_lo;         // with a carried value: only tuples whose value lies in
  int64_t carry_hi;         //   [carry_lo, carry_hi] take part
  const uint8_t* tnn;
  const int64_t* toff;      // P + 1
  uint64_t* items;          // work items of all queues: region | sub-region << 16 | S << 40
  uint32_t* qoff;           // kXcds + 1: queue q's items are items[qoff[q] .. qoff[q + 1])
  uint32_t* qticket;        // per queue: next item
  int32_t sorted;           // write the unsigned sort key column
  int32_t key_type;
  OCol out[1 + GQ_MAX_AGGS];
  OCol sortkey;
  int64_t out_cap;
  int64_t* d_count;
  int32_t* dev_status;
};

constexpr uint64_t kNoItem = ~0ull;
__device__ __forceinline__ uint32_t item_region(uint64_t it) { return (uint32_t)(it & 0xffffu); }
__device__ __forceinline__ uint32_t item_sub(uint64_t it) { return (uint32_t)((it >> 16) & 0xffffffu); }
__device__ __forceinline__ uint32_t item_nsub(uint64_t it) { return (uint32_t)(it >> 40); }

// Per region, the number of sub-regions S_p, and the work items: region p's
// S_p items in queue p % 8, queues one after another.  One block of 1024
// threads: regions are ordered queue by queue (index q * P/8 + k for region
// q + 8k), each thread takes up to four consecutive ones, and a block scan of
// their S_p gives every region's first item.
__global__ __launch_bounds__(1024) void k_rj_plan(const RjJoinArgs a) {
  constexpr int NW = 1024 / kWave;
  __shared__ uint32_t s_wave[NW];
  const int P = a.P;
  const int Q = P / kXcds;                        // regions per queue (P >= 16)
  const int per = (P + 1023) / 1024;              // <= 4
  uint32_t S[4];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int idx = (int)threadIdx.x * per + j;
    S[j] = 0;
    if (j < per && idx < P) {
      const int p = (idx % Q) * kXcds + idx / Q;
      const int64_t nb = a.boff[p + 1] - a.boff[p];
      S[j] = (uint32_t)((nb + a.kpr - 1) / a.kpr);
      if (S[j] < 1) S[j] = 1;
    }
    sum += S[j];
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint32_t base = incl - sum, total = 0;
  for (int w = 0; w < NW; ++w) {
    if (w < wave) base += s_wave[w];
    total += s_wave[w];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int idx = (int)threadIdx.x * per + j;
    if (j < per && idx < P) {
      const int q = idx / Q, k = idx % Q;
      const int p = k * kXcds + q;
      if (k == 0) a.qoff[q] = base;
      for (uint32_t u = 0; u < S[j]; ++u)
        a.items[base + u] = (uint64_t)p | ((uint64_t)u << 16) | ((uint64_t)S[j] << 40);
      base += S[j];
    }
  }
  if (threadIdx.x == 0) {
    a.qoff[kXcds] = total;
    *a.d_count = 0;
  }
  if (threadIdx.x < kXcds) a.qticket[threadIdx.x] = 0;
}

// The LDS table is probed linearly in buckets of four slots: a hash starts at
// the first slot of its bucket (its low 32 bits scaled to the lcap / 4
// buckets; the high bits chose the region and sub-region), and one probe step
// reads a whole bucket (two 16-byte LDS reads).  Slots only go from empty to
// taken, so a bucket with the key decides a hit, and one with an empty slot
// and no key decides a miss.
constexpr int kRjBucket = 4;
__device__ __forceinline__ uint32_t rj_bucket0(uint64_t h, int lcap) {
  return (uint32_t)(((uint64_t)(uint32_t)h * (uint64_t)(lcap / kRjBucket)) >> 32) * kRjBucket;
}

__device__ __forceinline__ int rj_find_insert(uint64_t* s_keys, int lcap, uint64_t key) {
  uint32_t s = rj_bucket0(key, lcap);
  for (int probe = 0; probe < lcap; ++probe) {
    const uint64_t kv = s_keys[s];
    if (kv == key) return (int)s;
    if (kv == kEmpty) {
      const uint64_t prev =
          atomicCAS((unsigned long long*)&s_keys[s], (unsigned long long)kEmpty, (unsigned long long)key);
      if (prev == kEmpty || prev == key) return (int)s;
    }
    s = (s + 1 == (uint32_t)lcap) ? 0u : s + 1;
  }
  return -1;
}

// LDS of k_rj_join: keys, accumulators and build multiplicities of lcap table
// slots, the slot of the hash EMPTY (index lcap) and 64 dump slots (one per
// lane: updates of tuples without a match go there, so the update code has no
// branches), then the staging words of one output validity bitmap.
__host__ __device__ inline int rj_slots(int lcap) { return lcap + 1 + kWave; }
__host__ __device__ inline int rj_vwords(int lcap) { return (lcap + 1) / 32 + 3; }
__host__ __device__ inline size_t rj_join_lds(int lcap, int nacc) {
  return (size_t)rj_slots(lcap) * (8 + 8 * (size_t)nacc + 4) + 4 * (size_t)rj_vwords(lcap);
}

__device__ __forceinline__ void rj_write(const OCol& o, int64_t g, int64_t v) {
  switch (o.type) {
    case GQ_I8: o.data[g] = (uint8_t)v; break;
    case GQ_I16: reinterpret_cast<int16_t*>(o.data)[g] = (int16_t)v; break;
    case GQ_I32: reinterpret_cast<int32_t*>(o.data)[g] = (int32_t)v; break;
    default: reinterpret_cast<int64_t*>(o.data)[g] = v; break;
  }
}

constexpr int kRjChunks = 8;  // emission chunks of kRjBlock slots: lcap + 1 <= kRjChunks * kRjBlock

// Next work item: queue q's ticket t (already taken) or, once q is used up,
// tickets from the following queues.  Called by one thread.
__device__ uint64_t rj_next(const RjJoinArgs& a, const uint32_t* s_qoff, int home, int& qi, uint32_t t) {
  while (qi < kXcds) {
    const int q = (home + qi) % kXcds;
    if (t < s_qoff[q + 1] - s_qoff[q]) return a.items[s_qoff[q] + t];
    if (++qi == kXcds) break;
    t = atomicAdd(&a.qticket[(home + qi) % kXcds], 1u);
  }
  return kNoItem;
}

// One round of probe tuples held in registers: kRjProbeUnroll per thread,
// NV value words each.
template <int NV>
struct RjRound {
  uint64_t h[kRjProbeUnroll];
  uint64_t x[kRjProbeUnroll][NV > 0 ? NV : 1];
  uint32_t nn[kRjProbeUnroll];
  uint32_t act;
};

// Issue the loads of the tuples base + u * kRjBlock + tid (u < kRjProbeUnroll)
// that lie below t1; the others re-read the last tuple (tuple 0 of the
// buffer when t1 is 0) and are inactive.  With CARRY the tuple's last word is
// a carried column value, and a tuple whose value lies outside
// [carry_lo, carry_hi] is inactive too.
// Straight-line code (NV, NN and CARRY fixed at compile time), so that every
// load of the round is in flight before the first is used.
template <int NV, bool NN, bool CARRY>
__device__ __forceinline__ void rj_load_round(const RjJoinArgs& a, int64_t base, int64_t t1, RjRound<NV>& r) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  r.act = 0;
  int64_t cv[kRjProbeUnroll];
#pragma unroll
  for (int u = 0; u < kRjProbeUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kRjBlock + threadIdx.x;
    const int64_t ic = i < t1 ? i : (t1 > 0 ? t1 - 1 : 0);
    const uint64_t* tp = a.tkey + (size_t)ic * (1 + NV + (CARRY ? 1 : 0));
    if constexpr (NV == 0) {
      r.h[u] = tp[0];
      r.x[u][0] = 0;
    } else if constexpr (NV == 1) {
      const u64x2 tv = *reinterpret_cast<const u64x2*>(tp);
      r.h[u] = tv.x;
      r.x[u][0] = tv.y;
    } else {
      r.h[u] = tp[0];
#pragma unroll
      for (int v = 0; v < NV; ++v) r.x[u][v] = tp[1 + v];
    }
    cv[u] = CARRY ? (int64_t)tp[1 + NV] : 0;
    if constexpr (NN) r.nn[u] = a.tnn[ic];
    else r.nn[u] = 0xffu;
  }
#pragma unroll
  for (int u = 0; u < kRjProbeUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kRjBlock + threadIdx.x;
    bool on = i < t1;
    if constexpr (CARRY) on = on && cv[u] >= a.carry_lo && cv[u] <= a.carry_hi;
    if (on) r.act |= 1u << u;
  }
}

// Probe one round of tuples in the table and apply their updates.  A tuple
// adds 1 to its group's row count and its plain (unweighted) inputs to the
// SUM and COUNT words; the build multiplicity of the key multiplies these at
// emission (every joined row of a probe tuple carries the same inputs).
template <int NV>
__device__ __forceinline__ void rj_probe_round(const RjJoinArgs& a, RjRound<NV>& r, const uint64_t* s_keys,
                                               uint64_t* s_acc, const uint32_t* s_mult, int L, uint32_t s,
                                               uint32_t S, uint32_t dump) {
  uint32_t act = r.act;
  uint32_t pos[kRjProbeUnroll];
  int32_t res[kRjProbeUnroll];
#pragma unroll
  for (int u = 0; u < kRjProbeUnroll; ++u) {
    res[u] = -1;
    pos[u] = rj_bucket0(r.h[u], L);
    if (subregion_of(r.h[u], a.pbits, S) != s) act &= ~(1u << u);
    if (((act >> u) & 1u) && r.h[u] == kEmpty) {
      res[u] = s_mult[L] ? L : -1;
      act &= ~(1u << u);
    }
  }
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  // First bucket of every tuple, all reads in flight together; it decides
  // almost every lookup (a hit, or an empty slot: a miss).
  {
    u64x2 k01[kRjProbeUnroll], k23[kRjProbeUnroll];
#pragma unroll
    for (int u = 0; u < kRjProbeUnroll; ++u) {
      k01[u] = *reinterpret_cast<const u64x2*>(&s_keys[pos[u]]);
      k23[u] = *reinterpret_cast<const u64x2*>(&s_keys[pos[u] + 2]);
    }
#pragma unroll
    for (int u = 0; u < kRjProbeUnroll; ++u) {
      const bool on = (act >> u) & 1u;
      const uint64_t h = r.h[u];
      const bool m0 = k01[u].x == h, m1 = k01[u].y == h, m2 = k23[u].x == h, m3 = k23[u].y == h;
      const bool hit = m0 | m1 | m2 | m3;
      const bool empty = (k01[u].x == kEmpty) | (k01[u].y == kEmpty) | (k23[u].x == kEmpty) |
                         (k23[u].y == kEmpty);
      const int32_t at = (int32_t)pos[u] + (m0 ? 0 : m1 ? 1 : m2 ? 2 : 3);
      res[u] = on && hit ? at : res[u];
      if (on && (hit || empty)) act &= ~(1u << u);
      pos[u] = pos[u] + kRjBucket == (uint32_t)L ? 0u : pos[u] + kRjBucket;
    }
  }
  // The rest walk on, one tuple at a time, reading buckets only for the
  // lanes still searching.
#pragma unroll
  for (int u = 0; u < kRjProbeUnroll; ++u) {
    for (int it = 1; ((act >> u) & 1u) && it < L / kRjBucket; ++it) {
      const u64x2 k01 = *reinterpret_cast<const u64x2*>(&s_keys[pos[u]]);
      const u64x2 k23 = *reinterpret_cast<const u64x2*>(&s_keys[pos[u] + 2]);
      const uint64_t h = r.h[u];
      const bool m0 = k01.x == h, m1 = k01.y == h, m2 = k23.x == h, m3 = k23.y == h;
      const bool hit = m0 | m1 | m2 | m3;
      const bool empty = (k01.x == kEmpty) | (k01.y == kEmpty) | (k23.x == kEmpty) | (k23.y == kEmpty);
      if (hit) res[u] = (int32_t)pos[u] + (m0 ? 0 : m1 ? 1 : m2 ? 2 : 3);
      if (hit || empty) act &= ~(1u << u);
      pos[u] = pos[u] + kRjBucket == (uint32_t)L ? 0u : pos[u] + kRjBucket;
    }
  }
  uint32_t slot[kRjProbeUnroll];
#pragma unroll
  for (int u = 0; u < kRjProbeUnroll; ++u) {
    slot[u] = res[u] >= 0 ? (uint32_t)res[u] : dump;
    atomicAdd((unsigned long long*)&s_acc[(size_t)slot[u] * a.nacc], 1ull);
  }
  if (a.sums_only) {
    // Accumulator words at fixed kernel-argument offsets: no per-aggregate
    // descriptor reads (whose waits would also wait for the updates).
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int word = a.sum_word[v];
#pragma unroll
      for (int u = 0; u < kRjProbeUnroll; ++u)
        atomicAdd((unsigned long long*)&s_acc[(size_t)slot[u] * a.nacc + word], (unsigned long long)r.x[u][v]);
    }
    return;
  }
  for (int g = 0; g < a.naggs; ++g) {
    const DAgg& ag = a.ap.aggs[g];
    const int op = ag.op;
    if (op == GQ_COUNT_STAR) continue;
    const int vw = a.vword[g];
    const int word = ag.word, cword = ag.cword;
    if (op == GQ_SUM || op == GQ_COUNT) {
#pragma unroll
      for (int u = 0; u < kRjProbeUnroll; ++u) {
        const uint64_t ok = (r.nn[u] >> g) & 1u;
        const uint64_t x = vw <= 0 ? r.x[u][0] : r.x[u][NV > 1 ? NV - 1 : 0];
        uint64_t* acc = s_acc + (size_t)slot[u] * a.nacc;
        atomicAdd((unsigned long long*)&acc[word], (unsigned long long)(op == GQ_SUM ? (ok ? x : 0) : ok));
        if (cword >= 0) atomicAdd((unsigned long long*)&acc[cword], (unsigned long long)ok);
      }
    } else {
#pragma unroll
      for (int u = 0; u < kRjProbeUnroll; ++u) {
        const bool ok = (r.nn[u] >> g) & 1u;
        const uint32_t sl = ok ? slot[u] : dump;
        const uint64_t x = vw <= 0 ? r.x[u][0] : r.x[u][NV > 1 ? NV - 1 : 0];
        uint64_t* acc = s_acc + (size_t)sl * a.nacc;
        if (op == GQ_MIN) atomicMin((long long*)&acc[word], (long long)x);
        else atomicMax((long long*)&acc[word], (long long)x);
        if (cword >= 0) atomicAdd((unsigned long long*)&acc[cword], (unsigned long long)(ok ? 1 : 0));
      }
    }
  }
}

// Validity bits of output rows [obase, obase + tot) (clipped to out_cap) of
// one output column: bit rel of the staging words (rel = row - (obase & ~31))
// is the bit of row obase - (obase & 31) + rel (s_vw NULL: every row valid).
// Words wholly inside the range are stored; the first and last words, shared
// with the neighbouring items' rows, are updated with an atomic AND of the
// range's bits and an OR.
__device__ __forceinline__ void rj_store_valid(uint32_t* words, const uint32_t* s_vw, int64_t obase, int64_t tot,
                                               int64_t out_cap) {
  int64_t end = obase + tot;
  if (end > out_cap) end = out_cap;
  if (end <= obase) return;
  const int64_t w0 = obase >> 5, w1 = (end - 1) >> 5;
  for (int64_t w = w0 + threadIdx.x; w <= w1; w += kRjBlock) {
    const int64_t lo = w * 32 > obase ? w * 32 : obase;
    const int64_t hi = w * 32 + 32 < end ? w * 32 + 32 : end;
    const uint32_t mask = (hi - lo == 32) ? ~0u : (((1u << (uint32_t)(hi - lo)) - 1u) << (uint32_t)(lo - w * 32));
    const uint32_t bits = (s_vw ? s_vw[w - w0] : ~0u) & mask;
    if (mask == ~0u) {
      words[w] = bits;
    } else {
      atomicAnd(&words[w], ~mask);
      if (bits) atomicOr(&words[w], bits);
    }
  }
}

// Persistent: workgroups (one per CU: the table takes the CU's LDS) take
// (region, sub-region) items from their XCD's queue.  Per item: the loads of
// the first build keys and probe tuples are issued, the table is cleared while
// they are in flight, the build keys of the sub-region are inserted with their
// multiplicities, the probe tuples streamed through the table in rounds (the
// next round's loads issued before the current round is probed), and the
// matched groups written in slot order to one output range per item.
template <int NV, bool NN, bool CARRY>
__global__ __launch_bounds__(kRjBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_rj_join(const RjJoinArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int L = a.lcap;
  const int NS = rj_slots(L);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  constexpr int NW = kRjBlock / kWave;
  const uint32_t dump = (uint32_t)(L + 1 + lane);
  uint64_t* s_keys = reinterpret_cast<uint64_t*>(s_raw);
  uint64_t* s_acc = s_keys + NS;
  uint32_t* s_mult = reinterpret_cast<uint32_t*>(s_acc + (size_t)NS * a.nacc);
  uint32_t* s_vw = s_mult + NS;
  const int VW = rj_vwords(L);
  __shared__ uint64_t s_item;
  __shared__ uint32_t s_qoff[kXcds + 1];
  __shared__ uint32_t s_cc[kRjChunks][NW];
  __shared__ int64_t s_obase;
  __shared__ int64_t s_tot;
  const int home = (int)(blockIdx.x % kXcds);
  if (threadIdx.x <= kXcds) s_qoff[threadIdx.x] = a.qoff[threadIdx.x];
  lds_barrier();
  int qi = 0;
  uint64_t cur = kNoItem;
  if (threadIdx.x == 0) cur = rj_next(a, s_qoff, home, qi, atomicAdd(&a.qticket[home], 1u));
  const int nchunks = (L + kRjBlock) / kRjBlock;  // chunks covering slots 0..L
  if (threadIdx.x == 0) s_item = cur;
  lds_barrier();
  uint64_t item = s_item;
  // An empty table for the first item; each later item finds its table
  // cleared by the threads that emitted the previous one.
  for (int i = threadIdx.x; i < NS; i += kRjBlock) {
    s_keys[i] = kEmpty;
    s_mult[i] = 0;
  }
  // The loads of an item (its region's offsets, its first build keys and its
  // first probe round) are issued as soon as the item is known: for the first
  // item here, for every later one right after the previous item's probe, so
  // that they are in flight while that item's groups are written out.
  // (Indices past the region re-read its last pair: unconditional loads stay
  // in flight together.)
  uint64_t bh[kRjUnroll];
  RjRound<NV> ra, rb;
  int64_t b0 = 0, b1 = 0, t0 = 0, t1 = 0;
  if (item != kNoItem) {
    const uint32_t p = item_region(item);
    b0 = a.boff[p];
    b1 = a.boff[p + 1];
    t0 = a.toff[p];
    t1 = a.toff[p + 1];
#pragma unroll
    for (int u = 0; u < kRjUnroll; ++u) {
      const int64_t i = b0 + (int64_t)u * kRjBlock + threadIdx.x;
      bh[u] = a.bkey[2 * (i < b1 ? i : (b1 > 0 ? b1 - 1 : 0))];
    }
    rj_load_round<NV, NN, CARRY>(a, t0, t1, ra);
  }
  while (item != kNoItem) {
    const uint32_t s = item_sub(item), S = item_nsub(item);
    uint32_t tnext = 0;
    if (threadIdx.x == 0 && qi < kXcds) tnext = atomicAdd(&a.qticket[(home + qi) % kXcds], 1u);

    // 1. The table's keys and multiplicities are clear (see the end of the
    // loop).  A slot's accumulator words are set when its first build key
    // arrives; the other slots' (and the dump slots') are never read.
    lds_barrier();
    // 2. Build keys of sub-region s, counting duplicates.
    for (int64_t base = b0; base < b1; base += (int64_t)kRjBlock * kRjUnroll) {
      if (base != b0) {
#pragma unroll
        for (int u = 0; u < kRjUnroll; ++u) {
          const int64_t i = base + (int64_t)u * kRjBlock + threadIdx.x;
          bh[u] = a.bkey[2 * (i < b1 ? i : b1 - 1)];
        }
      }
#pragma unroll
      for (int u = 0; u < kRjUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kRjBlock + threadIdx.x;
        if (i >= b1 || subregion_of(bh[u], a.pbits, S) != s) continue;
        const int slot = bh[u] == kEmpty ? L : rj_find_insert(s_keys, L, bh[u]);
        if (slot < 0) {
          atomicOr(a.dev_status, GQ_DEV_TABLE_FULL);
          continue;
        }
        if (atomicAdd(&s_mult[slot], 1u) == 0u)
          for (int w = 0; w < a.nacc; ++w) s_acc[(size_t)slot * a.nacc + w] = a.ident[w];
      }
    }
    lds_barrier();
    // The next item, resolved while this one is probed (every thread reads it
    // after the barrier that ends the probe).
    if (threadIdx.x == 0) {
      cur = rj_next(a, s_qoff, home, qi, tnext);
      s_item = cur;
    }
    // 3. Probe rounds, two register sets alternating: the loads of the next
    // round are in flight while the current one is probed.
    constexpr int64_t R = (int64_t)kRjBlock * kRjProbeUnroll;
    for (int64_t base = t0; base < t1; base += 2 * R) {
      if (base + R < t1) rj_load_round<NV, NN, CARRY>(a, base + R, t1, rb);
      else rb.act = 0;
      rj_probe_round<NV>(a, ra, s_keys, s_acc, s_mult, L, s, S, dump);
      if (base + 2 * R < t1) rj_load_round<NV, NN, CARRY>(a, base + 2 * R, t1, ra);
      else ra.act = 0;
      if (base + R < t1) rj_probe_round<NV>(a, rb, s_keys, s_acc, s_mult, L, s, S, dump);
    }
    lds_barrier();
    // The next item's loads, in flight while this item's groups are written.
    item = s_item;
    if (item != kNoItem) {
      const uint32_t p = item_region(item);
      b0 = a.boff[p];
      b1 = a.boff[p + 1];
      t0 = a.toff[p];
      t1 = a.toff[p + 1];
#pragma unroll
      for (int u = 0; u < kRjUnroll; ++u) {
        const int64_t i = b0 + (int64_t)u * kRjBlock + threadIdx.x;
        bh[u] = a.bkey[2 * (i < b1 ? i : (b1 > 0 ? b1 - 1 : 0))];
      }
      rj_load_round<NV, NN, CARRY>(a, t0, t1, ra);
    }
    // 4. Matched groups (row count non-zero) to the output, in slot order:
    // per chunk of kRjBlock slots the wave counts, one output range per item.
    uint32_t occm = 0;
    for (int c = 0; c < nchunks; ++c) {
      const int i = c * kRjBlock + threadIdx.x;
      const bool occ = i <= L && s_mult[i] != 0u && s_acc[(size_t)i * a.nacc] != 0;
      const uint64_t m = ballot(occ);
      if (occ) occm |= 1u << c;
      if (lane == 0) s_cc[c][wave] = (uint32_t)__popcll(m);
    }
    lds_barrier();
    // Wave 0 turns the (chunk, wave) counts, in emission order, into their
    // exclusive prefix (two entries per lane) and reserves the item's output
    // range.
    if (wave == 0) {
      static_assert(kRjChunks * NW <= 2 * kWave, "two (chunk, wave) counts per lane");
      uint32_t* flat = &s_cc[0][0];
      const int ne = nchunks * NW, e0 = 2 * lane, e1 = 2 * lane + 1;
      const uint32_t x0 = e0 < ne ? flat[e0] : 0u, x1 = e1 < ne ? flat[e1] : 0u;
      uint32_t tot;
      const uint32_t pre = wave_prefix_small<8>(x0 + x1, &tot);  // x0 + x1 <= 128
      if (e0 < ne) flat[e0] = pre;
      if (e1 < ne) flat[e1] = pre + x0;
      if (lane == 0) {
        const int64_t base = tot ? (int64_t)atomicAdd((unsigned long long*)a.d_count, (unsigned long long)tot) : 0;
        if (tot && base + tot > a.out_cap) atomicOr(a.dev_status, GQ_DEV_CAPACITY);
        s_obase = base;
        s_tot = tot;
      }
    }
    lds_barrier();
    const int64_t obase = s_obase, otot = s_tot;
    for (int c = 0; c < nchunks; ++c) {
      const int i = c * kRjBlock + threadIdx.x;
      const bool occ = (occm >> c) & 1u;
      const uint64_t m = ballot(occ);
      if (occ) {
        const int64_t rel = (int64_t)s_cc[c][wave] + rank_in(m);
        const int64_t g = obase + rel;
        const uint64_t mult = s_mult[i];
        s_mult[i] = (uint32_t)rel;  // the slot's output row, for the validity bits below
        if (g < a.out_cap && a.emit64) {
          // Slot L holds the key whose region hash is all ones.
          const uint64_t key = region_unhash(s_keys[i]);
          reinterpret_cast<uint64_t*>(a.out[0].data)[g] = key;
          if (a.sorted) reinterpret_cast<uint64_t*>(a.sortkey.data)[g] = key ^ (1ull << 63);
          const uint64_t* acc = s_acc + (size_t)i * a.nacc;
#pragma unroll
          for (int j = 0; j < GQ_MAX_AGGS; ++j) {
            if (j >= a.naggs) break;
            uint64_t v = acc[a.e_word[j]];
            if (a.e_mul[j]) v *= mult;
            if (a.e_cword[j] >= 0 && acc[a.e_cword[j]] == 0) v = 0;
            reinterpret_cast<uint64_t*>(a.out[1 + j].data)[g] = v;
          }
        } else if (g < a.out_cap) {
          const uint64_t key = region_unhash(s_keys[i]);
          rj_write(a.out[0], g, (int64_t)key);
          if (a.sorted) reinterpret_cast<uint64_t*>(a.sortkey.data)[g] = key ^ (1ull << 63);
          const uint64_t* acc = s_acc + (size_t)i * a.nacc;
          for (int j = 0; j < a.naggs; ++j) {
            const DAgg& ag = a.ap.aggs[j];
            int64_t v = (int64_t)acc[ag.word];
            if (ag.op == GQ_SUM || ag.op == GQ_COUNT || ag.op == GQ_COUNT_STAR) v = (int64_t)((uint64_t)v * mult);
            bool ok = true;
            if ((ag.op == GQ_SUM || ag.op == GQ_MIN || ag.op == GQ_MAX) && ag.cword >= 0) ok = acc[ag.cword] != 0;
            if (!ok) v = 0;
            rj_write(a.out[1 + j], g, v);
          }
        }
      }
    }
    // 5. Validity bitmaps of the nullable output columns: the item's bits are
    // gathered in LDS, then stored word by word.
    const int64_t shift = obase & 31;
    for (int oc = 0; oc <= a.naggs; ++oc) {
      if (!a.out[oc].valid || otot == 0) continue;
      const int aop = oc ? a.ap.aggs[oc - 1].op : GQ_COUNT_STAR;
      const int cword = oc ? a.ap.aggs[oc - 1].cword : -1;
      const bool maybe_null = (aop == GQ_SUM || aop == GQ_MIN || aop == GQ_MAX) && cword >= 0;
      if (!maybe_null) {
        // Every row of the item valid: the words are written directly.
        rj_store_valid(a.out[oc].valid, nullptr, obase, otot, a.out_cap);
        continue;
      }
      lds_barrier();
      for (int w = threadIdx.x; w < VW; w += kRjBlock) s_vw[w] = 0;
      lds_barrier();
      for (int c = 0; c < nchunks; ++c) {
        const int i = c * kRjBlock + threadIdx.x;
        if (!((occm >> c) & 1u)) continue;
        if (s_acc[(size_t)i * a.nacc + cword] == 0) continue;
        const int64_t b = shift + (int64_t)s_mult[i];
        atomicOr(&s_vw[b >> 5], 1u << (b & 31));
      }
      lds_barrier();
      rj_store_valid(a.out[oc].valid, s_vw, obase, otot, a.out_cap);
    }
    // Slots 0..L are read after the probe only by the thread that owns them
    // (slot c * kRjBlock + thread of every chunk c), which clears them for
    // the next item once its groups and validity bits are out; the dump
    // slots' keys and multiplicities are never read.
    for (int c = 0; c < nchunks; ++c) {
      const int i = c * kRjBlock + threadIdx.x;
      if (i <= L) {
        s_keys[i] = kEmpty;
        s_mult[i] = 0;
      }
    }
    // (The barrier at the top of the loop orders these clears before the
    // next item's inserts.)
  }
}

// Staged input columns: predicate columns and the key first (the histogram
// pass reads only those), then aggregate value columns; each distinct column
// once.  ok turns false when they do not fit the staging limits.
struct StageBuilder {
  RpArgs& a;
  bool ok = true;
  int add(const DCol& c) {
    for (int j = 0; j < a.nst; ++j)
      if (a.st[j].data == c.data && a.st[j].type == c.type && a.st[j].valid == c.valid && a.st[j].voff == c.voff)
        return j;
    if (a.nst == kRpMaxStage) {
      ok = false;
      return 0;
    }
    a.st[a.nst] = c;
    a.st_off[a.nst] = a.in_bytes;
    a.in_bytes += (int)align_up((size_t)kRpSub * type_width(c.type), 16);
    return a.nst++;
  }
};

constexpr size_t kRpMaxLds = 160 * 1024;  // LDS of one workgroup


// Histogram, scan and scatter of one side; a.counts/starts/okey... set by the
// caller except the workspace, allocated here.  offsets: P + 1 int64.
constexpr int kRpMaxReg = 5;  // columns of the register-path histogram

template <int NS>
int rp_launch_hist_reg(gq_ctx* ctx, const RpArgs& a, size_t lds, hipStream_t stream) {
  if (a.probe)
    GQ_LAUNCH(ctx, "rp_hist_probe", (k_rp_hist_r<NS, true>), dim3((unsigned)a.ntiles), dim3(kRpBlock), lds, stream, a);
  else
    GQ_LAUNCH(ctx, "rp_hist_build", (k_rp_hist_r<NS, false>), dim3((unsigned)a.ntiles), dim3(kRpBlock), lds, stream,
              a);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

int rp_launch_hist_reg_n(gq_ctx* ctx, const RpArgs& a, int ns, size_t lds, hipStream_t stream) {
  switch (ns) {
    case 1: return rp_launch_hist_reg<1>(ctx, a, lds, stream);
    case 2: return rp_launch_hist_reg<2>(ctx, a, lds, stream);
    case 3: return rp_launch_hist_reg<3>(ctx, a, lds, stream);
    case 4: return rp_launch_hist_reg<4>(ctx, a, lds, stream);
    default: return rp_launch_hist_reg<5>(ctx, a, lds, stream);
  }
}

int rp_run(gq_ctx* ctx, RpArgs& a, int64_t* offsets, int64_t* total, hipStream_t stream) {
  const int64_t P = 1ll << a.pbits;
  // Tiles sized for about 2,048 workgroups.  The histogram reads its columns
  // straight into registers when every one of them is 16-byte aligned (the
  // usual case), else through LDS like the scatter.
  int64_t t = kRpMinTile;
  while (t < kRpMaxTile && t * 2048 < a.n) t *= 2;
  a.tile_rows = t;
  bool reg = a.nst_hist <= kRpMaxReg;
  for (int j = 0; j < a.nst_hist; ++j) reg = reg && a.st[j].align >= 16;
  a.ntiles = (a.n + a.tile_rows - 1) / a.tile_rows;
  if (a.ntiles == 0) {
    // No rows: every offset 0.
    int rc = launch_fill_u32(ctx, offsets, 0u, 2 * (P + 1), stream);
    if (rc) return rc;
    if (total) rc = launch_fill_u32(ctx, total, 0u, 2, stream);
    return rc;
  }
  const int64_t m = a.ntiles * P;
  const int64_t nchunks = (a.ntiles + kCsChunk - 1) / kCsChunk;
  Scratch ws(ctx, stream);
  const size_t off_counts = 256;
  const size_t off_starts = off_counts + align_up((size_t)m * 4, 256);
  const size_t off_csum = off_starts + align_up((size_t)m * 4, 256);
  const size_t off_tot = off_csum + align_up((size_t)nchunks * P * 4, 256);
  const size_t bytes = off_tot + align_up((size_t)P * 4, 256);
  if (!ws.get(bytes)) return set_error(ctx, GQ_ERR_NOMEM, "radix join: partition workspace allocation failed");
  a.counts = ws.as<uint32_t>(off_counts);
  a.starts = ws.as<uint32_t>(off_starts);
  uint32_t* csum = ws.as<uint32_t>(off_csum);
  uint32_t* rtot = ws.as<uint32_t>(off_tot);
  a.rtot = rtot;
  if (reg) {
    int rc = rp_launch_hist_reg_n(ctx, a, a.nst_hist, (size_t)P * 4, stream);
    if (rc) return rc;
  } else {
    const size_t lds_hist = align_up((size_t)P * 4, 16) +
                           ((size_t)a.st_off[a.nst_hist - 1] +
                            align_up((size_t)kRpSub * type_width(a.st[a.nst_hist - 1].type), 16)) * kRpHScale;
    if (a.probe)
      GQ_LAUNCH(ctx, "rp_hist_probe", k_rp_hist<true>, dim3((unsigned)a.ntiles), dim3(kRpBlock), lds_hist, stream, a);
    else
      GQ_LAUNCH(ctx, "rp_hist_build", k_rp_hist<false>, dim3((unsigned)a.ntiles), dim3(kRpBlock), lds_hist, stream, a);
    GQ_LAUNCH_CHECK(ctx);
  }
  const dim3 cgrid((unsigned)nchunks, (unsigned)((P + 255) / 256));
  GQ_LAUNCH(ctx, a.probe ? "rp_scan_probe" : "rp_scan_build", k_cs_chunk, cgrid, dim3(256), 0, stream,
            (const uint32_t*)a.counts, a.ntiles, (int)P, csum, rtot);
  GQ_LAUNCH_CHECK(ctx);
  GQ_LAUNCH(ctx, a.probe ? "rp_scan_probe" : "rp_scan_build", k_cs_fill, cgrid, dim3(256), 0, stream,
            (const uint32_t*)a.counts, (const uint32_t*)csum, (const uint32_t*)rtot, a.ntiles, (int)P, a.starts,
            offsets, total);
  GQ_LAUNCH_CHECK(ctx);
  const size_t lds = rp_scatter_lds((int)P, a.in_bytes);
  if (a.probe)
    GQ_LAUNCH(ctx, "rp_scatter_probe", k_rp_scatter<true>, dim3((unsigned)a.ntiles), dim3(kRpSBlock), lds, stream, a);
  else
    GQ_LAUNCH(ctx, "rp_scatter_build", k_rp_scatter<false>, dim3((unsigned)a.ntiles), dim3(kRpSBlock), lds, stream, a);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}


// Two-level partition: tuples without a non-NULL mask, 256 to 4096 regions,
// first-level slots of at most kRp2MaxSlots bytes (they come on top of the
// final tuples: above that size, as for the 600M-row fact and 150M-row
// dimension sides of concurrent serving queries, each slot's stream caching
// such workspaces, the single-level path's smaller workspace wins), LDS room for
// both kernels (k_rp1 stages its columns for kRp1Sub rows, half the layout
// built for kRpSub).
constexpr size_t kRp2MaxSlots = (size_t)2 << 30;

static bool rp2_applies(const RpArgs& a) {
  if (a.need_nn || a.pbits < 8 || a.pbits > 12 || a.tw < 2 || a.tw > 4 || (!a.probe && a.tw != 2)) return false;
  if ((size_t)(a.n + kRp1Sub) * a.tw * 8 > kRp2MaxSlots) return false;
  const int P = 1 << a.pbits;
  return rp1_lds(P, a.in_bytes / 2, a.tw) + 512 <= kRpMaxLds && rp2_lds(a.tw) + 6144 <= kRpMaxLds;
}

template <bool NULLABLE>
static int rp1_launch(gq_ctx* ctx, const RpArgs& h, int npf, size_t lds, hipStream_t stream) {
  const dim3 grid((unsigned)h.ntiles), block(kRp1Block);
  const char* nm = h.probe ? "rp1_probe" : "rp1_build";
  switch (npf) {
    case 1: GQ_LAUNCH(ctx, nm, (k_rp1<NULLABLE, 1>), grid, block, lds, stream, h); break;
    case 2: GQ_LAUNCH(ctx, nm, (k_rp1<NULLABLE, 2>), grid, block, lds, stream, h); break;
    case 3: GQ_LAUNCH(ctx, nm, (k_rp1<NULLABLE, 3>), grid, block, lds, stream, h); break;
    case 4: GQ_LAUNCH(ctx, nm, (k_rp1<NULLABLE, 4>), grid, block, lds, stream, h); break;
    case 5: GQ_LAUNCH(ctx, nm, (k_rp1<NULLABLE, 5>), grid, block, lds, stream, h); break;
    default: GQ_LAUNCH(ctx, nm, (k_rp1<NULLABLE, 0>), grid, block, lds, stream, h); break;
  }
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

// k_rp1, the column scan and k_rp2 for the probe side; offsets: P + 1 int64.
int rp_run2(gq_ctx* ctx, RpArgs& a, int64_t* offsets, int64_t* total, hipStream_t stream) {
  const int64_t P = 1ll << a.pbits;
  // Tiles of at most kRpMaxTile rows (a multiple of kRp1Sub), as many as fill
  // whole rounds of the workgroups resident at once (three per CU), so that
  // the last round is not mostly idle.
  int dev_cus = 256;
  (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  const int64_t resident = (int64_t)dev_cus * 3;
  int64_t rounds = (a.n + resident * kRpMaxTile - 1) / (resident * kRpMaxTile);
  if (rounds < 1) rounds = 1;
  int64_t t = (a.n + resident * rounds - 1) / (resident * rounds);
  t = (t + kRp1Sub - 1) / kRp1Sub * kRp1Sub;
  if (t < kRpMinTile) t = kRpMinTile;
  a.tile_rows = t;
  a.ntiles = (a.n + a.tile_rows - 1) / a.tile_rows;
  if (a.ntiles == 0) {
    int rc = launch_fill_u32(ctx, offsets, 0u, 2 * (P + 1), stream);
    if (!rc && total) rc = launch_fill_u32(ctx, total, 0u, 2, stream);
    return rc;
  }
  const int64_t subs = t / kRp1Sub;
  // k_rp2 workgroups of about 2 * kRp2Round * kR1 input rows (a round of
  // tuples when half the rows are kept), at most kRp2MaxRuns runs.
  int64_t group = (int64_t)2 * kRp2Round * kR1 / t;
  if (group < 1) group = 1;
  if (group * subs > kRp2MaxRuns) group = kRp2MaxRuns / subs;
  const int64_t ngroups = (a.ntiles + group - 1) / group;
  const int64_t m = a.ntiles * P;
  const int64_t nchunks = (a.ntiles + kCsChunk - 1) / kCsChunk;
  const int64_t nslots = a.ntiles * subs;
  Scratch ws(ctx, stream);
  const size_t off_counts = 256;
  const size_t off_starts = off_counts + align_up((size_t)m * 4, 256);
  const size_t off_csum = off_starts + align_up((size_t)m * 4, 256);
  const size_t off_tot = off_csum + align_up((size_t)nchunks * P * 4, 256);
  const size_t off_roff = off_tot + align_up((size_t)P * 4, 256);
  const size_t off_slots = off_roff + align_up((size_t)nslots * (kR1 + 1) * 2, 256);
  const size_t bytes = off_slots + (size_t)nslots * kRp1Sub * a.tw * 8;
  if (!ws.get(bytes)) return set_error(ctx, GQ_ERR_NOMEM, "radix join: probe workspace allocation failed");
  a.counts = ws.as<uint32_t>(off_counts);
  a.starts = ws.as<uint32_t>(off_starts);
  uint32_t* csum = ws.as<uint32_t>(off_csum);
  a.rtot = ws.as<uint32_t>(off_tot);
  a.roff = ws.as<uint16_t>(off_roff);
  a.slots = ws.as<uint64_t>(off_slots);
  // k_rp1 stages kRp1Sub rows: every column in half the space.
  RpArgs h = a;
  for (int j = 0; j < h.nst; ++j) h.st_off[j] = a.st_off[j] / 2;
  h.in_bytes = a.in_bytes / 2;
  bool nullable = false, aligned = true;
  for (int j = 0; j < a.nst; ++j) {
    nullable = nullable || a.st[j].valid != nullptr;
    aligned = aligned && a.st[j].align >= 16;
  }
  const int npf = aligned && a.nst <= kRp1MaxPf ? a.nst : 0;
  const size_t lds1 = rp1_lds((int)P, h.in_bytes, a.tw);
  int rc = nullable ? rp1_launch<true>(ctx, h, npf, lds1, stream) : rp1_launch<false>(ctx, h, npf, lds1, stream);
  if (rc) return rc;
  const dim3 cgrid((unsigned)nchunks, (unsigned)((P + 255) / 256));
  GQ_LAUNCH(ctx, a.probe ? "rp_scan_probe" : "rp_scan_build", k_cs_chunk, cgrid, dim3(256), 0, stream,
            (const uint32_t*)a.counts, a.ntiles, (int)P, csum, a.rtot);
  GQ_LAUNCH_CHECK(ctx);
  GQ_LAUNCH(ctx, a.probe ? "rp_scan_probe" : "rp_scan_build", k_cs_fill, cgrid, dim3(256), 0, stream, (const uint32_t*)a.counts,
            (const uint32_t*)csum, (const uint32_t*)a.rtot, a.ntiles, (int)P, a.starts, offsets, total);
  GQ_LAUNCH_CHECK(ctx);
  const dim3 g2((unsigned)(kR1 * ngroups)), b2(kRp2Block);
  const char* nm2 = a.probe ? "rp2_probe" : "rp2_build";
  if (a.tw == 2) GQ_LAUNCH(ctx, nm2, k_rp2<2>, g2, b2, rp2_lds(2), stream, a, (int32_t)group);
  else if (a.tw == 3) GQ_LAUNCH(ctx, nm2, k_rp2<3>, g2, b2, rp2_lds(3), stream, a, (int32_t)group);
  else GQ_LAUNCH(ctx, nm2, k_rp2<4>, g2, b2, rp2_lds(4), stream, a, (int32_t)group);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

}  // namespace

int rj_choose_pbits(int64_t build_rows) {
  // Regions of at most about kRjNominalKpr build rows, so that one LDS table
  // holds a region's kept rows (one sub-region) even when most rows are kept:
  // each probe tuple is then read once.  Between 256 and 4096 regions.
  int pbits = 8;
  while (pbits < 12 && ((int64_t)1 << pbits) * kRjNominalKpr < build_rows) ++pbits;
  return pbits;
}

// Staging plan of the build side; false when it does not fit.
static bool rj_build_plan(RpArgs& a, const gq_batch* build, int32_t key_col, const gq_pred* preds, int npreds,
                          int pbits) {
  std::memset(&a, 0, sizeof(a));
  a.carry_st = -1;
  a.n = build->nrows;
  a.pbits = pbits;
  a.npreds = npreds;
  a.probe = 0;
  StageBuilder sb{a};
  for (int p = 0; p < npreds; ++p) {
    a.preds[p] = DPred{preds[p].col, preds[p].op, preds[p].lo, preds[p].hi};
    a.pred_st[p] = sb.add(make_dcol(build->cols[preds[p].col]));
  }
  a.key_st = sb.add(make_dcol(build->cols[key_col]));
  a.nst_hist = a.nst;
  return sb.ok && rp_scatter_lds(1 << pbits, a.in_bytes) <= kRpMaxLds;
}

bool rj_build_fits(const gq_batch* build, int32_t key_col, const gq_pred* preds, int npreds, int pbits) {
  RpArgs a;
  return rj_build_plan(a, build, key_col, preds, npreds, pbits);
}

int rj_build(gq_ctx* ctx, const gq_batch* build, int32_t key_col, const gq_pred* preds, int npreds,
             gq_join_table* t, hipStream_t stream) {
  RpArgs a;
  if (!rj_build_plan(a, build, key_col, preds, npreds, t->rj_pbits))
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "radix join: build staging does not fit");
  a.okey = t->rj_kr;
  a.ocap = build->nrows;
  a.tw = 2;
  return rp2_applies(a) ? rp_run2(ctx, a, t->rj_off, &t->hdr->nrows, stream)
                        : rp_run(ctx, a, t->rj_off, &t->hdr->nrows, stream);
}

// Staging plan and value words of the probe side; false when it does not fit.
static bool rj_probe_plan(RpArgs& r, int32_t (&vword)[GQ_MAX_AGGS], const gq_batch* in, int32_t probe_key,
                          const gq_pred* preds, int npreds, const AggPlan& ap, int pbits, int32_t carry_col = -1) {
  std::memset(&r, 0, sizeof(r));
  r.carry_st = -1;
  r.n = in->nrows;
  r.pbits = pbits;
  r.npreds = npreds;
  r.probe = 1;
  r.ap = ap;
  r.naggs = ap.naggs;
  StageBuilder sb{r};
  for (int p = 0; p < npreds; ++p) {
    r.preds[p] = DPred{preds[p].col, preds[p].op, preds[p].lo, preds[p].hi};
    r.pred_st[p] = sb.add(make_dcol(in->cols[preds[p].col]));
  }
  r.key_st = sb.add(make_dcol(in->cols[probe_key]));
  r.nst_hist = r.nst;
  for (int v = 0; v < ap.nvals; ++v) r.val_st[v] = sb.add(ap.vals[v]);
  for (int i = 0; i < ap.naggs; ++i) {
    vword[i] = -1;
    const int op = ap.aggs[i].op;
    if (op == GQ_SUM || op == GQ_MIN || op == GQ_MAX) {
      if (r.nv == kRjMaxVals) return false;
      r.vagg[r.nv] = i;
      vword[i] = r.nv++;
    }
    if (op != GQ_COUNT_STAR)
      for (int f = 0; f < ap.aggs[i].nf; ++f)
        if (ap.aggs[i].f[f].kind != GQ_F_CONST && ap.vals[ap.aggs[i].f[f].v].valid) r.need_nn = 1;
  }
  if (carry_col >= 0) r.carry_st = sb.add(make_dcol(in->cols[carry_col]));
  return sb.ok && rp_scatter_lds(1 << pbits, r.in_bytes) <= kRpMaxLds;
}

bool rj_usable(const gq_join_table* t, const gq_batch* in, int32_t probe_key, const gq_pred* preds, int npreds,
               const AggPlan& ap, int32_t carry_col) {
  if (!t || !t->rj_kr) return false;
  if (in->nrows >= ((int64_t)1 << 32)) return false;
  RpArgs r;
  int32_t vword[GQ_MAX_AGGS];
  if (!rj_probe_plan(r, vword, in, probe_key, preds, npreds, ap, t->rj_pbits, carry_col)) return false;
  const int lcap = rj_lcap(ap.nacc);
  if (lcap < 1024) return false;
  // Sub-regions per region stay few when every build row is kept.
  const int64_t per_region = t->build_rows >> t->rj_pbits;
  return per_region <= (int64_t)16 * rj_kpr(lcap);
}

int rj_lcap(int nacc) {
  const size_t per = 8 + 8 * (size_t)nacc + 4;
  int l = (int)(kRjLdsBytes / per) - 1 - kWave;
  if (l > kRjChunks * kRjBlock - 1) l = kRjChunks * kRjBlock - 1;
  l &= ~(kRjBucket - 1);  // whole buckets
  while (l > 0 && rj_join_lds(l, nacc) > kRjLdsBytes) l -= kRjBucket;
  return l;
}

int rj_kpr(int lcap) { return (int)((int64_t)lcap * 13 / 20); }  // load factor 0.65

// A partitioned probe side: its tuples, region offsets and plan, in a
// workspace released (stream-ordered) with it.
struct RjPart {
  Scratch ws;
  RpArgs r;
  int32_t vword[GQ_MAX_AGGS];
  int64_t* toff;
  int pbits;
  RjPart(gq_ctx* ctx, hipStream_t stream) : ws(ctx, stream) {}
};

int rj_part_create(gq_ctx* ctx, const gq_batch* in, int32_t probe_key, const gq_pred* preds, int npreds,
                   int32_t carry_col, const AggPlan& ap, int pbits, hipStream_t stream, RjPart** out) {
  *out = nullptr;
  RjPart* part = new RjPart(ctx, stream);
  RpArgs& r = part->r;
  if (!rj_probe_plan(r, part->vword, in, probe_key, preds, npreds, ap, pbits, carry_col)) {
    delete part;
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "radix join: probe staging does not fit");
  }
  const int64_t P = 1ll << pbits;
  const int64_t cap = in->nrows > 0 ? in->nrows : 1;
  r.tw = 1 + r.nv + (carry_col >= 0 ? 1 : 0);
  const size_t off_key = 256;
  const size_t off_nn = off_key + align_up((size_t)cap * 8 * r.tw, 256);
  const size_t off_toff = off_nn + align_up(r.need_nn ? (size_t)cap : 1, 256);
  const size_t bytes = off_toff + align_up((size_t)(P + 1) * 8, 256);
  if (!part->ws.get(bytes)) {
    delete part;
    return set_error(ctx, GQ_ERR_NOMEM, "radix join: probe workspace allocation failed");
  }
  r.okey = part->ws.as<uint64_t>(off_key);
  r.onn = part->ws.as<uint8_t>(off_nn);
  r.ocap = cap;
  part->toff = part->ws.as<int64_t>(off_toff);
  part->pbits = pbits;
  const int rc = rp2_applies(r) ? rp_run2(ctx, r, part->toff, nullptr, stream) : rp_run(ctx, r, part->toff, nullptr, stream);
  if (rc) {
    delete part;
    return rc;
  }
  *out = part;
  return GQ_OK;
}

void rj_part_destroy(RjPart* part) { delete part; }

template <int NV, bool NN, bool CARRY>
static int rj_launch_join(gq_ctx* ctx, const RjJoinArgs& j, dim3 grid, size_t lds, hipStream_t stream) {
  GQ_LAUNCH(ctx, "rj_join", (k_rj_join<NV, NN, CARRY>), grid, dim3(kRjBlock), lds, stream, j);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

template <bool CARRY>
static int rj_launch_join_nv(gq_ctx* ctx, const RjJoinArgs& j, dim3 grid, size_t lds, hipStream_t stream) {
  if (j.nv == 0) return j.need_nn ? rj_launch_join<0, true, CARRY>(ctx, j, grid, lds, stream)
                                  : rj_launch_join<0, false, CARRY>(ctx, j, grid, lds, stream);
  if (j.nv == 1) return j.need_nn ? rj_launch_join<1, true, CARRY>(ctx, j, grid, lds, stream)
                                  : rj_launch_join<1, false, CARRY>(ctx, j, grid, lds, stream);
  return j.need_nn ? rj_launch_join<2, true, CARRY>(ctx, j, grid, lds, stream)
                   : rj_launch_join<2, false, CARRY>(ctx, j, grid, lds, stream);
}

int rj_part_join(gq_ctx* ctx, const RjPart* part, const AggPlan& ap, const gq_join_table* t, int64_t carry_lo,
                 int64_t carry_hi, const CompactArgs& ca, int64_t* d_groups, hipStream_t stream) {
  const RpArgs& r = part->r;
  if (t->rj_pbits != part->pbits)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "radix join: table and probe side have different region counts");
  const int64_t P = 1ll << part->pbits;
  RjJoinArgs j;
  std::memset(&j, 0, sizeof(j));
  for (int i = 0; i < GQ_MAX_AGGS; ++i) j.vword[i] = part->vword[i];
  // Work items: S_p = max(1, ceil(rows_p / kpr)) per region, so at most
  // P + build_rows / kpr + 1 in all.
  const int lcap = rj_lcap(ap.nacc);
  const int64_t max_items = P + t->build_rows / rj_kpr(lcap) + 2;
  Scratch ws(ctx, stream);
  const size_t off_items = 256;
  const size_t off_q = off_items + align_up((size_t)max_items * 8, 256);
  if (!ws.get(off_q + 256)) return set_error(ctx, GQ_ERR_NOMEM, "radix join: work item allocation failed");

  j.pbits = part->pbits;
  j.P = (int32_t)P;
  j.nacc = ap.nacc;
  j.lcap = lcap;
  j.kpr = rj_kpr(lcap);
  j.naggs = ap.naggs;
  j.nv = r.nv;
  j.need_nn = r.need_nn;
  j.ap = ap;
  for (int w = 0; w < ap.nacc; ++w) j.ident[w] = word_identity(ap.wop[w]);
  j.sums_only = 1;
  for (int i = 0; i < ap.naggs; ++i) {
    const DAgg& ag = ap.aggs[i];
    if (ag.op == GQ_COUNT_STAR) continue;
    if (ag.op != GQ_SUM || ag.cword >= 0 || j.vword[i] < 0) j.sums_only = 0;
    else j.sum_word[j.vword[i]] = ag.word;
  }
  j.emit64 = type_width(ca.out[0].type) == 8;
  for (int i = 0; i < ap.naggs; ++i) {
    const DAgg& ag = ap.aggs[i];
    j.emit64 = j.emit64 && type_width(ca.out[1 + i].type) == 8;
    j.e_word[i] = ag.word;
    j.e_mul[i] = ag.op == GQ_SUM || ag.op == GQ_COUNT || ag.op == GQ_COUNT_STAR;
    j.e_cword[i] = (ag.op == GQ_SUM || ag.op == GQ_MIN || ag.op == GQ_MAX) ? ag.cword : -1;
  }
  j.bkey = t->rj_kr;
  j.boff = t->rj_off;
  j.tkey = r.okey;
  j.tw = r.tw;
  j.tnn = r.onn;
  j.toff = part->toff;
  j.carry_lo = carry_lo;
  j.carry_hi = carry_hi;
  j.items = ws.as<uint64_t>(off_items);
  j.qoff = ws.as<uint32_t>(off_q);
  j.qticket = ws.as<uint32_t>(off_q + 64);
  j.sorted = ca.sortkey.data != nullptr;
  j.sortkey = ca.sortkey;
  j.key_type = ca.out[0].type;
  for (int i = 0; i <= ap.naggs; ++i) j.out[i] = ca.out[i];
  j.out_cap = ca.out_cap;
  j.d_count = d_groups;
  j.dev_status = ctx->d_status;
  // The probe side is partitioned; from here on the build side is read.
  int rc = join_wait_ready(ctx, t, stream);
  if (rc) return rc;
  GQ_LAUNCH(ctx, "rj_plan", k_rj_plan, dim3(1), dim3(1024), 0, stream, j);
  GQ_LAUNCH_CHECK(ctx);
  int lds_max = 0;
  GQ_HIP_CHECK(ctx, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
  if ((size_t)lds_max < rj_join_lds(j.lcap, j.nacc) + 256)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "radix join: device LDS per workgroup too small");
  int dev_cus = 256;
  (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  const dim3 jgrid((unsigned)(dev_cus * kRjPerCu));
  const size_t jlds = rj_join_lds(j.lcap, j.nacc);
  return r.carry_st >= 0 ? rj_launch_join_nv<true>(ctx, j, jgrid, jlds, stream)
                         : rj_launch_join_nv<false>(ctx, j, jgrid, jlds, stream);
}

int rj_groupjoin(gq_ctx* ctx, const gq_batch* in, int32_t probe_key, const gq_pred* preds, int npreds,
                 const AggPlan& ap, const gq_join_table* t, const CompactArgs& ca, int64_t* d_groups,
                 hipStream_t stream) {
  RjPart* part = nullptr;
  int rc = rj_part_create(ctx, in, probe_key, preds, npreds, -1, ap, t->rj_pbits, stream, &part);
  if (rc) return rc;
  rc = rj_part_join(ctx, part, ap, t, 0, 0, ca, d_groups, stream);
  rj_part_destroy(part);
  return rc;
}

}  // namespace gq
