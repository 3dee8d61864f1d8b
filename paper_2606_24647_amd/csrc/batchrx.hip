// Radix aggregation of the high-cardinality fragments of a batched plan.
//
// A fragment expecting more groups than one LDS table holds would otherwise
// add every row into its HBM table with device-wide atomics (one per
// accumulator word), and those run at about 24 G/s for the whole GPU.  Here
// such fragments are aggregated without per-row HBM atomics:
//   k_brx_hist     per hist tile (16384 rows) of any radix fragment: the tile's
//                  rows staged in LDS per 1024-row sub-tile, kept rows
//                  (predicates) counted per region, region = top bits of
//                  fmix64(group key ^ seed), 2^rbits_f regions of about half an
//                  LDS table each;
//   k_brx_scan     exclusive scan of all the counts, laid out fragment by
//                  fragment, region-major: a global position per (fragment,
//                  region, tile);
//   k_brx_scatter  the same tiles again: each kept row becomes a tuple (key hash,
//                  aggregate inputs) written at its region's position;
//   k_brx_agg      persistent: a workgroup takes a (fragment, region) item,
//                  aggregates the region's tuples in an LDS table and appends the
//                  groups to the fragment's output (one atomic for the range).
// Rows whose group key is the raw key EMPTY or NULL, or hashes to the LDS
// table's empty marker, go to the fragment's HBM table at scatter time, as do the tuples of a region that holds more groups
// than its LDS table (only when the expected cardinality was too low); the
// plan's compaction then appends the HBM table's groups after the radix ones.
#include "agg.h"
#include "batchrx.h"
#include "radix.h"

namespace gq {
namespace {

constexpr int kXBlock = 256;
constexpr int kXSub = 512;                // scatter sub-tile; unit of the staging layout
constexpr int kXRows = kXSub / kXBlock;
constexpr int kXTile = 16384;             // hist tile (one count per region)
constexpr int kXSubs = kXTile / kXSub;
constexpr int kHSub = 2048;               // hist sub-tile
constexpr int kHRows = kHSub / kXBlock;
constexpr int kHScale = kHSub / kXSub;    // hist staging offsets = layout offsets * kHScale
constexpr int kXJoinBlock = 1024;
constexpr int kXU = 4;                    // tuples per thread and round of k_brx_agg
constexpr int kXV = 4;                    // value words held in registers

__device__ __forceinline__ uint32_t bx_region(uint64_t h, int rbits) {
  return rbits ? (uint32_t)(h >> (64 - rbits)) : 0u;
}

// Rows r = i * 256 + t (i < ROWS) of a staged column: one type dispatch.
template <int ROWS>
__device__ __forceinline__ void bx_rows(const uint8_t* base, int type, int64_t (&v)[ROWS]) {
  const int t = threadIdx.x;
  switch (type) {
    case GQ_I8:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int8_t*>(base)[i * kXBlock + t];
      break;
    case GQ_I16:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int16_t*>(base)[i * kXBlock + t];
      break;
    case GQ_I32:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int32_t*>(base)[i * kXBlock + t];
      break;
    default:
#pragma unroll
      for (int i = 0; i < ROWS; ++i) v[i] = reinterpret_cast<const int64_t*>(base)[i * kXBlock + t];
      break;
  }
}

// Stage the sub-tile's columns (the first nst of the fragment's list); column
// j lands at s_in + st_off[j] * scale.
typedef const GQ_CONST_AS BrxFrag CFrag;
typedef const GQ_CONST_AS GbArgs CArgs;
typedef const GQ_CONST_AS DAgg CAgg;

__device__ __forceinline__ void bx_stage(CFrag& x, int nst, int scale, int64_t sbase, int nrows,
                                         uint8_t* s_in) {
  for (int j = 0; j < nst; ++j) stage_col_lds<kXBlock>(x.st[j], sbase, nrows, s_in + x.st_off[j] * scale);
}

// Kept rows of the staged sub-tile and their group keys (packed or raw, with
// the special kinds of make_keys: 0 hashed, 1 raw key EMPTY, 2 NULL raw key).
template <int ROWS>
__device__ __forceinline__ uint32_t bx_keep_keys(CFrag& x, CArgs& g, const uint8_t* s_in, int scale,
                                                 int64_t sbase, int nrows, uint64_t (&key)[ROWS],
                                                 uint8_t (&special)[ROWS]) {
  uint32_t keep = 0;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    if (i * kXBlock + (int)threadIdx.x < nrows) keep |= 1u << i;
    key[i] = 0;
    special[i] = 0;
  }
  for (int p = 0; p < g.npreds; ++p) {
    const int j = x.pred_st[p];
    int64_t v[ROWS];
    bx_rows<ROWS>(s_in + x.st_off[j] * scale, x.st[j].type, v);
    const int64_t lo = g.preds[p].lo, hi = g.preds[p].hi;
    if (g.preds[p].op == GQ_RANGE) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (v[i] < lo || v[i] > hi) keep &= ~(1u << i);
    } else {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (v[i] == lo) keep &= ~(1u << i);
    }
    if (x.st[j].valid) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (((keep >> i) & 1u) && !valid_one(x.st[j], sbase + i * kXBlock + threadIdx.x)) keep &= ~(1u << i);
    }
  }
  const GQ_CONST_AS KeyPlan& kp = g.kp;
  for (int j = 0; j < kp.nk; ++j) {
    const int c = x.key_st[j];
    int64_t v[ROWS];
    bx_rows<ROWS>(s_in + x.st_off[c] * scale, x.st[c].type, v);
    uint32_t vm = 0xffffffffu;
    if (kp.cols[j].valid) {
      vm = 0;
#pragma unroll
      for (int i = 0; i < ROWS; ++i)
        if (((keep >> i) & 1u) && valid_one(kp.cols[j], sbase + i * kXBlock + threadIdx.x)) vm |= 1u << i;
    }
    if (kp.mode == KEY_RAW64) {
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        key[i] = (uint64_t)v[i];
        special[i] = !((vm >> i) & 1u) ? 2 : (key[i] == kEmpty ? 1 : 0);
      }
    } else {
      const int w = kp.bits[j];
      const uint64_t mask = (w == 64) ? ~0ull : ((1ull << w) - 1);
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        uint64_t f = ((uint64_t)v[i] ^ (1ull << (w - 1))) & mask;
        if (kp.nullable[j]) f = ((vm >> i) & 1u) ? (f | (1ull << w)) : 0ull;
        key[i] |= f << kp.shift[j];
      }
    }
  }
  return keep;
}

// Input of aggregate ag for staged row r (global row grow): the product of its
// factors; *nn is cleared when a referenced column is NULL.
__device__ __forceinline__ uint64_t bx_value_row(CFrag& x, CArgs& g, CAgg& ag,
                                                 const uint8_t* s_in, int r, int64_t grow, bool* nn) {
  uint64_t xv = 1;
  for (int f = 0; f < ag.nf; ++f) {
    const GQ_CONST_AS DFactor& fa = ag.f[f];
    const uint64_t k = (uint64_t)fa.k;
    if (fa.kind == GQ_F_CONST) {
      xv *= k;
      continue;
    }
    const int j = x.val_st[fa.v];
    const uint64_t v = (uint64_t)lds_value(s_in + x.st_off[j], r, x.st[j].type);
    if (g.ap.vals[fa.v].valid && !valid_one(g.ap.vals[fa.v], grow)) *nn = false;
    if (fa.kind == GQ_F_COL) xv *= v;
    else if (fa.kind == GQ_F_K_MINUS_COL) xv *= k - v;
    else xv *= k + v;
  }
  return xv;
}

// The aggregate inputs of staged row r as a tuple's value words (dst[vword])
// and the mask of aggregates whose input is non-NULL.
__device__ __forceinline__ uint32_t bx_tuple_values(const BrxArgs& a, CFrag& x, CArgs& g,
                                                    const uint8_t* s_in, int r, int64_t grow, uint64_t* dst) {
  uint32_t nnm = 0xffu;
  for (int gi = 0; gi < g.ap.naggs; ++gi) {
    CAgg& ag = g.ap.aggs[gi];
    const int vw = a.vword[gi];
    if (vw < 0 && !(a.need_nn && ag.op == GQ_COUNT)) continue;
    bool nn = true;
    const uint64_t xv = bx_value_row(x, g, ag, s_in, r, grow, &nn);
    if (vw >= 0) dst[vw] = xv;
    if (!nn) nnm &= ~(1u << gi);
  }
  return nnm;
}

// Add one row into the fragment's HBM table (special keys and overflow); tv
// holds the tuple's value words.
__device__ void bx_global_row(const GbArgs& g, const int32_t* vword, uint64_t key, int special, const uint64_t* tv,
                              uint32_t nn) {
  uint64_t* acc = global_acc(g, key, special);
  if (!acc) return;
  GlobalAtomics::add(&acc[0], 1);
  for (int i = 0; i < g.ap.naggs; ++i) {
    const DAgg& ag = g.ap.aggs[i];
    if (ag.op == GQ_COUNT_STAR || !((nn >> i) & 1u)) continue;
    const uint64_t xv = vword[i] >= 0 ? tv[vword[i]] : 0;
    switch (ag.op) {
      case GQ_SUM: GlobalAtomics::add(&acc[ag.word], xv); break;
      case GQ_COUNT: GlobalAtomics::add(&acc[ag.word], 1); break;
      case GQ_MIN: GlobalAtomics::min(&acc[ag.word], (int64_t)xv); break;
      default: GlobalAtomics::max(&acc[ag.word], (int64_t)xv); break;
    }
    if (ag.cword >= 0) GlobalAtomics::add(&acc[ag.cword], 1);
  }
}

// The same for staged row r of a sub-tile, its inputs read from LDS.
__device__ void bx_global_row_staged(CFrag& x, CArgs& g, uint64_t key, int special,
                                     const uint8_t* s_in, int r, int64_t grow) {
  uint64_t* acc = global_acc(gref(g), key, special);
  if (!acc) return;
  GlobalAtomics::add(&acc[0], 1);
  for (int i = 0; i < g.ap.naggs; ++i) {
    CAgg& ag = g.ap.aggs[i];
    if (ag.op == GQ_COUNT_STAR) continue;
    bool nn = true;
    const uint64_t xv = bx_value_row(x, g, ag, s_in, r, grow, &nn);
    if (!nn) continue;
    switch (ag.op) {
      case GQ_SUM: GlobalAtomics::add(&acc[ag.word], xv); break;
      case GQ_COUNT: GlobalAtomics::add(&acc[ag.word], 1); break;
      case GQ_MIN: GlobalAtomics::min(&acc[ag.word], (int64_t)xv); break;
      default: GlobalAtomics::max(&acc[ag.word], (int64_t)xv); break;
    }
    if (ag.cword >= 0) GlobalAtomics::add(&acc[ag.cword], 1);
  }
}

// Reset the counters of one replay: scan status and tickets, item ticket, and
// the group counts of the radix fragments.
__global__ void k_brx_init(const BrxArgs a) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  if (i0 == 0) {
    *a.scan_ticket = 0;
    *a.item_ticket = 0;
  }
  for (int64_t i = i0; i < a.nscan; i += step) a.scan_status[i] = 0;
  for (int64_t i = i0; i < a.nrf; i += step) *a.outs[a.rf[i].f].d_groups = 0;
}

// Region counts of one hist tile, from 2048-row sub-tiles of the predicate and
// key columns.
__global__ __launch_bounds__(kXBlock) void k_brx_hist(const BrxArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int64_t t = blockIdx.x;
  const int fi = a.tile_frag[t];
  CFrag& x = cref(a.rf + fi);
  CArgs& g = cref(a.frags + x.f);
  const int R = 1 << x.rbits;
  uint32_t* s_hist = reinterpret_cast<uint32_t*>(s_raw);
  uint8_t* s_in = s_raw + align_up((size_t)R * 4, 16);
  for (int i = threadIdx.x; i < R; i += kXBlock) s_hist[i] = 0;
  const int64_t tl = t - x.tile0;
  for (int sub = 0; sub < kXTile / kHSub; ++sub) {
    const int64_t sbase = tl * kXTile + (int64_t)sub * kHSub;
    if (sbase >= g.n) break;
    const int nrows = g.n - sbase < kHSub ? (int)(g.n - sbase) : kHSub;
    __syncthreads();
    bx_stage(x, x.nst_hist, kHScale, sbase, nrows, s_in);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    uint64_t key[kHRows];
    uint8_t special[kHRows];
    const uint32_t keep = bx_keep_keys<kHRows>(x, g, s_in, kHScale, sbase, nrows, key, special);
#pragma unroll
    for (int i = 0; i < kHRows; ++i) {
      const uint64_t h = region_hash(key[i]);
      if (((keep >> i) & 1u) && !special[i] && h != kEmpty) atomicAdd(&s_hist[bx_region(h, x.rbits)], 1u);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += kXBlock) a.counts[x.cbase + (int64_t)r * x.tiles + tl] = s_hist[r];
}

// Exclusive scan of counts[0..m) into starts[0..m]; starts[m] = total.
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_brx_scan(const uint32_t* counts, int64_t m, int64_t* starts,
                                                    uint32_t* ticket, uint64_t* status, int64_t nblocks) {
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t s_tile;
  __shared__ int64_t s_wave[NW];
  __shared__ int64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t i0 = (tile * BLOCK + threadIdx.x) * ITEMS;
  uint32_t c[ITEMS];
  int64_t tsum = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    c[k] = (i0 + k < m) ? counts[i0 + k] : 0u;
    tsum += c[k];
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int64_t incl = tsum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(incl, o, kWave);
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
    const int64_t e = lookback_exclusive(status, tile, btot);
    if (lane == 0) s_excl = e;
  }
  __syncthreads();
  int64_t run = s_excl + bpre + incl - tsum;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    if (i0 + k < m) starts[i0 + k] = run;
    run += c[k];
  }
  if (tile == nblocks - 1 && threadIdx.x == 0) starts[m] = s_excl + btot;
}

// LDS of k_brx_scatter: R region bases (int64) and counters (u32), the staged
// sub-tile, then per row: pp (u32: region << 16 | rank, ~0 = no tuple), src
// (u16, rows in tuple order) and the key hash.
__host__ __device__ inline size_t bx_scatter_lds(int R, int in_bytes) {
  return align_up((size_t)R * 12, 16) + align_up((size_t)in_bytes, 16) + (size_t)kXSub * (4 + 2 + 8);
}

// With every staged column 16-byte aligned (at most kXPfMax of them) the next
// sub-tile is loaded into registers while the current one is counted and
// ranked (a column of a sub-tile is at most kXBlock 16-byte chunks), waited
// for before the current tuples are stored, and written to LDS once they have
// left.  Barriers inside the loop order LDS only: a full barrier waits for
// every outstanding load and store of the wave, and every LDS write after a
// global-to-LDS load waits for it, so neither would let loads overlap the row
// work.
constexpr int kXPfMax = 5;

__global__ __launch_bounds__(kXBlock) void k_brx_scatter(const BrxArgs a) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int64_t t = blockIdx.x;
  const int fi = a.tile_frag[t];
  CFrag& x = cref(a.rf + fi);
  CArgs& g = cref(a.frags + x.f);
  const int R = 1 << x.rbits;
  int64_t* s_base = reinterpret_cast<int64_t*>(s_raw);
  uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_base + R);
  uint8_t* s_in = s_raw + align_up((size_t)R * 12, 16);
  uint64_t* s_h = reinterpret_cast<uint64_t*>(s_in + align_up((size_t)x.in_bytes, 16));
  uint32_t* s_pp = reinterpret_cast<uint32_t*>(s_h + kXSub);
  uint16_t* s_src = reinterpret_cast<uint16_t*>(s_pp + kXSub);
  __shared__ uint32_t s_wsum[kXBlock / kWave];
  __shared__ uint32_t s_total;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t tl = t - x.tile0;
  const int tw = 1 + a.nv;
  for (int r = threadIdx.x; r < R; r += kXBlock) {
    s_base[r] = a.starts[x.cbase + (int64_t)r * x.tiles + tl];
    s_cnt[r] = 0;
  }
  const int per = (R + kXBlock - 1) / kXBlock;  // <= 4
  bool pf_ok = x.nst <= kXPfMax;
  for (int j = 0; j < x.nst; ++j) pf_ok = pf_ok && x.st[j].align >= 16;
  {
    const int64_t sbase = tl * kXTile;
    if (sbase < g.n) bx_stage(x, x.nst, 1, sbase, g.n - sbase < kXSub ? (int)(g.n - sbase) : kXSub, s_in);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int sub = 0; sub < kXSubs; ++sub) {
    const int64_t sbase = tl * kXTile + (int64_t)sub * kXSub;
    if (sbase >= g.n) break;
    const int nrows = g.n - sbase < kXSub ? (int)(g.n - sbase) : kXSub;
    const int64_t nbase = sbase + kXSub;
    const bool has_next = sub + 1 < kXSubs && nbase < g.n;
    const bool pf = pf_ok && has_next && g.n - nbase >= kXSub;
    u32x4 pfv[kXPfMax];
#pragma unroll
    for (int j = 0; j < kXPfMax; ++j) pfv[j] = u32x4{0u, 0u, 0u, 0u};
    if (pf) {
#pragma unroll
      for (int j = 0; j < kXPfMax; ++j) {
        if (j >= x.nst) continue;
        const int w = type_width(x.st[j].type);
        if ((int)threadIdx.x < kXSub * w / 16)
          pfv[j] = *reinterpret_cast<const u32x4*>(x.st[j].data + nbase * w + (int64_t)threadIdx.x * 16);
      }
    }
    uint64_t key[kXRows];
    uint8_t special[kXRows];
    const uint32_t keep = bx_keep_keys<kXRows>(x, g, s_in, 1, sbase, nrows, key, special);
#pragma unroll
    for (int i = 0; i < kXRows; ++i) {
      const int r = i * kXBlock + threadIdx.x;
      s_pp[r] = 0xffffffffu;
      if (!((keep >> i) & 1u)) continue;
      const uint64_t h = region_hash(key[i]);
      if (special[i] || h == kEmpty) {
        // Raw key EMPTY or NULL, or the one key whose hash is the LDS table's
        // empty marker: straight into the fragment's HBM table.
        bx_global_row_staged(x, g, key[i], special[i], s_in, r, sbase + r);
        continue;
      }
      s_pp[r] = (bx_region(h, x.rbits) << 16) | atomicAdd(&s_cnt[bx_region(h, x.rbits)], 1u);
      s_h[r] = h;
    }
    lds_barrier();
    // Exclusive scan of the region counts.
    uint32_t mysum = 0;
    uint32_t cnt_own[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < R) {
        cnt_own[j] = s_cnt[q];
        mysum += cnt_own[j];
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
    for (int w = 0; w < kXBlock / kWave; ++w) {
      if (w < wave) wpre += s_wsum[w];
      tot += s_wsum[w];
    }
    uint32_t run = wpre + incl - mysum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < R) {
        s_cnt[q] = run;
        run += cnt_own[j];
      }
    }
    if (threadIdx.x == 0) s_total = tot;
    lds_barrier();
#pragma unroll
    for (int i = 0; i < kXRows; ++i) {
      const int r = i * kXBlock + threadIdx.x;
      const uint32_t pp = s_pp[r];
      if (pp != 0xffffffffu) s_src[s_cnt[pp >> 16] + (pp & 0xffffu)] = (uint16_t)r;
    }
    lds_barrier();
    // The next sub-tile's loads have landed (and the previous sub-tile's
    // stores left) before this one's tuples are stored, so that refilling LDS
    // below waits for nothing.
    __builtin_amdgcn_s_waitcnt(0);
    // Tuples in region order: consecutive threads write consecutive tuples of
    // a region's run; value words are computed here from the staged columns.
    const int total = (int)s_total;
    for (int k = threadIdx.x; k < total; k += kXBlock) {
      const int r = s_src[k];
      const uint32_t q = s_pp[r] >> 16;
      const int64_t pos = s_base[q] + (k - (int)s_cnt[q]);
      uint64_t* dst = a.tup + (size_t)pos * tw;
      dst[0] = s_h[r];
      const uint32_t nnm = bx_tuple_values(a, x, g, s_in, r, sbase + r, dst + 1);
      if (a.need_nn) a.tnn[pos] = (uint8_t)nnm;
    }
    // Every tuple has left the staged input; the next sub-tile replaces it.
    lds_barrier();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = threadIdx.x * per + j;
      if (j < per && q < R) {
        s_base[q] += cnt_own[j];
        s_cnt[q] = 0;
      }
    }
    if (pf) {
#pragma unroll
      for (int j = 0; j < kXPfMax; ++j) {
        if (j >= x.nst) continue;
        if ((int)threadIdx.x < kXSub * type_width(x.st[j].type) / 16)
          *reinterpret_cast<u32x4*>(s_in + x.st_off[j] + (int64_t)threadIdx.x * 16) = pfv[j];
      }
    } else if (has_next) {
      bx_stage(x, x.nst, 1, nbase, g.n - nbase < kXSub ? (int)(g.n - nbase) : kXSub, s_in);
      __builtin_amdgcn_s_waitcnt(0);
    }
    lds_barrier();
  }
}

// LDS slot of a key hash (its low 32 bits; the high bits chose the region).
__device__ __forceinline__ uint32_t bx_slot(uint64_t h, int lcap) {
  return (uint32_t)(((uint64_t)(uint32_t)h * (uint64_t)lcap) >> 32);
}

// Find or insert h in the LDS table; -1 when kLdsProbes slots are taken by
// other keys.
__device__ __forceinline__ int bx_find_insert(uint64_t* s_keys, int lcap, uint64_t h) {
  uint32_t s = bx_slot(h, lcap);
  for (int probe = 0; probe < kLdsProbes; ++probe) {
    const uint64_t kv = s_keys[s];
    if (kv == h) return (int)s;
    if (kv == kEmpty) {
      const uint64_t prev =
          atomicCAS((unsigned long long*)&s_keys[s], (unsigned long long)kEmpty, (unsigned long long)h);
      if (prev == kEmpty || prev == h) return (int)s;
    }
    s = (s + 1 == (uint32_t)lcap) ? 0u : s + 1;
  }
  return -1;
}

__device__ __forceinline__ int bx_find(const uint64_t* s_keys, int lcap, uint64_t h) {
  uint32_t s = bx_slot(h, lcap);
  for (int probe = 0; probe < kLdsProbes; ++probe) {
    const uint64_t kv = s_keys[s];
    if (kv == h) return (int)s;
    if (kv == kEmpty) return -1;
    s = (s + 1 == (uint32_t)lcap) ? 0u : s + 1;
  }
  return -1;
}

__device__ __forceinline__ void bx_write(const GQ_CONST_AS OCol& o, int64_t g, int64_t v) {
  switch (o.type) {
    case GQ_I8: o.data[g] = (uint8_t)v; break;
    case GQ_I16: reinterpret_cast<int16_t*>(o.data)[g] = (int16_t)v; break;
    case GQ_I32: reinterpret_cast<int32_t*>(o.data)[g] = (int32_t)v; break;
    default: reinterpret_cast<int64_t*>(o.data)[g] = v; break;
  }
}

__device__ __forceinline__ void bx_valid(const GQ_CONST_AS OCol& o, int64_t g, bool ok) {
  if (!o.valid) return;
  const uint32_t bit = 1u << (g & 31);
  if (ok) atomicOr(&o.valid[g >> 5], bit);
  else atomicAnd(&o.valid[g >> 5], ~bit);
}

__global__ __launch_bounds__(kXJoinBlock) void k_brx_agg(const BrxArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  const int L = a.lcap;
  const int nacc = a.nacc;
  uint64_t* s_keys = reinterpret_cast<uint64_t*>(s_raw);
  uint64_t* s_acc = s_keys + L;
  __shared__ int64_t s_it;
  __shared__ int64_t s_obase;
  __shared__ uint32_t s_cc[8][kXJoinBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int tw = 1 + a.nv;
  for (;;) {
    if (threadIdx.x == 0) s_it = (int64_t)atomicAdd((unsigned long long*)a.item_ticket, 1ull);
    __syncthreads();
    const int64_t it = s_it;
    if (it >= a.nitems) break;
    const int fi = a.item_frag[it];
    CFrag& x = cref(a.rf + fi);
    CArgs& g = cref(a.frags + x.f);
    const GQ_CONST_AS BatchOut& bo = cref(a.outs + x.f);
    const int r = (int)(it - x.item0);
    const int64_t e0 = x.cbase + (int64_t)r * x.tiles;
    const int64_t t0 = a.starts[e0], t1 = a.starts[e0 + x.tiles];
    // 1. Clear.
    for (int i = threadIdx.x; i < L; i += kXJoinBlock) s_keys[i] = kEmpty;
    for (int w = 0; w < nacc; ++w) {
      const uint64_t id = word_identity(g.ap.wop[w]);
      for (int i = threadIdx.x; i < L; i += kXJoinBlock) s_acc[(size_t)i * nacc + w] = id;
    }
    __syncthreads();
    // 2. Tuples: insert or find in LDS, accumulate; a tuple whose key finds no
    // slot is retried after the round's barrier (another lane may have taken
    // the slot for the same key) and otherwise goes to the HBM table.
    // kXU tuples per thread and round, all loads issued first; value words
    // are held in registers when there are at most kXV of them.
    const int nv = a.nv;
    const bool regs = nv <= kXV;
    for (int64_t base = t0; base < t1; base += (int64_t)kXJoinBlock * kXU) {
      uint64_t h[kXU];
      uint64_t v[kXU][kXV];
      uint32_t nnm[kXU];
      int slot[kXU];
#pragma unroll
      for (int u = 0; u < kXU; ++u) {
        const int64_t i = base + (int64_t)u * kXJoinBlock + threadIdx.x;
        h[u] = 0;
        nnm[u] = 0xffu;
#pragma unroll
        for (int w = 0; w < kXV; ++w) v[u][w] = 0;
        if (i < t1) {
          const uint64_t* tp = a.tup + (size_t)i * tw;
          h[u] = tp[0];
          if (regs) {
#pragma unroll
            for (int w = 0; w < kXV; ++w)
              if (w < nv) v[u][w] = tp[1 + w];
          }
          if (a.need_nn) nnm[u] = a.tnn[i];
        }
      }
#pragma unroll
      for (int u = 0; u < kXU; ++u) {
        const int64_t i = base + (int64_t)u * kXJoinBlock + threadIdx.x;
        slot[u] = i < t1 ? bx_find_insert(s_keys, L, h[u]) : L;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kXU; ++u) {
        if (slot[u] < 0) slot[u] = bx_find(s_keys, L, h[u]);
        if (slot[u] == L) continue;  // no tuple
        const int64_t i = base + (int64_t)u * kXJoinBlock + threadIdx.x;
        const uint64_t* tv = a.tup + (size_t)i * tw + 1;
        if (slot[u] < 0) {
          bx_global_row(gref(g), a.vword, region_unhash(h[u]), 0, tv, nnm[u]);
          continue;
        }
        uint64_t* acc = s_acc + (size_t)slot[u] * nacc;
        atomicAdd((unsigned long long*)&acc[0], 1ull);
        if (regs) {
#pragma unroll
          for (int w = 0; w < kXV; ++w) {
            if (w >= nv) break;
            CAgg& ag = g.ap.aggs[a.vagg[w]];
            if (!((nnm[u] >> a.vagg[w]) & 1u)) continue;
            const uint64_t xv = v[u][w];
            switch (ag.op) {
              case GQ_SUM: atomicAdd((unsigned long long*)&acc[ag.word], (unsigned long long)xv); break;
              case GQ_MIN: atomicMin((long long*)&acc[ag.word], (long long)xv); break;
              default: atomicMax((long long*)&acc[ag.word], (long long)xv); break;
            }
          }
        }
        for (int gi = 0; gi < g.ap.naggs; ++gi) {
          CAgg& ag = g.ap.aggs[gi];
          if (ag.op == GQ_COUNT_STAR || !((nnm[u] >> gi) & 1u)) continue;
          if (ag.op == GQ_COUNT) {
            atomicAdd((unsigned long long*)&acc[ag.word], 1ull);
          } else if (!regs) {
            const uint64_t xv = tv[a.vword[gi]];
            switch (ag.op) {
              case GQ_SUM: atomicAdd((unsigned long long*)&acc[ag.word], (unsigned long long)xv); break;
              case GQ_MIN: atomicMin((long long*)&acc[ag.word], (long long)xv); break;
              default: atomicMax((long long*)&acc[ag.word], (long long)xv); break;
            }
          }
          if (ag.cword >= 0) atomicAdd((unsigned long long*)&acc[ag.cword], 1ull);
        }
      }
    }
    __syncthreads();
    // 3. Groups to the fragment's output, in slot order.
    const int nchunks = (L + kXJoinBlock - 1) / kXJoinBlock;
    uint32_t occm = 0;
    for (int c = 0; c < nchunks; ++c) {
      const int i = c * kXJoinBlock + threadIdx.x;
      const bool occ = i < L && s_keys[i] != kEmpty;
      const uint64_t m = ballot(occ);
      if (occ) occm |= 1u << c;
      if (lane == 0) s_cc[c][wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (int c = 0; c < nchunks; ++c)
        for (int w = 0; w < kXJoinBlock / kWave; ++w) tot += s_cc[c][w];
      const int64_t b = tot ? (int64_t)atomicAdd((unsigned long long*)bo.d_groups, (unsigned long long)tot) : 0;
      if (tot && b + tot > bo.out_cap) atomicOr(g.dev_status, GQ_DEV_CAPACITY);
      s_obase = b;
    }
    __syncthreads();
    int64_t run = s_obase;
    for (int c = 0; c < nchunks; ++c) {
      uint32_t wpre = 0, ctot = 0;
      for (int w = 0; w < kXJoinBlock / kWave; ++w) {
        const uint32_t v = s_cc[c][w];
        wpre += w < wave ? v : 0;
        ctot += v;
      }
      const int i = c * kXJoinBlock + threadIdx.x;
      const bool occ = (occm >> c) & 1u;
      const uint64_t m = ballot(occ);
      if (occ) {
        const int64_t gpos = run + wpre + rank_in(m);
        if (gpos < bo.out_cap) {
          const uint64_t key = region_unhash(s_keys[i]);
          for (int j = 0; j < a.nk; ++j) {
            bool ok = true;
            const int64_t v = g.kp.mode == KEY_RAW64 ? (int64_t)key : decode_field(g.kp, key, j, &ok);
            bx_write(bo.out[j], gpos, v);
            bx_valid(bo.out[j], gpos, ok);
          }
          const uint64_t* acc = s_acc + (size_t)i * nacc;
          for (int j = 0; j < g.ap.naggs; ++j) {
            CAgg& ag = g.ap.aggs[j];
            int64_t v = (int64_t)acc[ag.word];
            bool ok = true;
            if ((ag.op == GQ_SUM || ag.op == GQ_MIN || ag.op == GQ_MAX) && ag.cword >= 0) ok = acc[ag.cword] != 0;
            if (!ok) v = 0;
            bx_write(bo.out[a.nk + j], gpos, v);
            bx_valid(bo.out[a.nk + j], gpos, ok);
          }
        }
      }
      run += ctot;
    }
    __syncthreads();
  }
}

constexpr int kXScanBlock = 256, kXScanItems = 16;

}  // namespace

size_t brx_lds_budget() { return 150 * 1024; }

int brx_lcap(int nacc) {
  int l = (int)(brx_lds_budget() / (8 + 8 * (size_t)nacc));
  if (l > 8 * kXJoinBlock) l = 8 * kXJoinBlock;
  return l;
}

int64_t brx_tile_rows() { return kXTile; }

size_t brx_scatter_lds_bytes(const BrxFrag& x) { return bx_scatter_lds(1 << x.rbits, x.in_bytes); }

size_t brx_hist_lds_bytes(const BrxFrag& x) {
  const int hist_in = x.nst_hist < x.nst ? x.st_off[x.nst_hist] : x.in_bytes;
  return align_up((size_t)4 << x.rbits, 16) + (size_t)hist_in * kHScale;
}

int brx_stage_plan(BrxFrag& x, const GbArgs& g, int nv, const int32_t* vagg, bool need_nn) {
  std::memset(x.st_off, 0, sizeof(x.st_off));
  x.nst = 0;
  x.in_bytes = 0;
  auto add = [&](const DCol& c) -> int {
    for (int j = 0; j < x.nst; ++j)
      if (x.st[j].data == c.data && x.st[j].type == c.type && x.st[j].valid == c.valid && x.st[j].voff == c.voff)
        return j;
    if (x.nst == kBrxMaxStage) return -1;
    x.st[x.nst] = c;
    x.st_off[x.nst] = x.in_bytes;
    x.in_bytes += (int)align_up((size_t)kXSub * type_width(c.type), 16);
    return x.nst++;
  };
  for (int p = 0; p < g.npreds; ++p)
    if ((x.pred_st[p] = add(g.pcols[p])) < 0) return -1;
  for (int j = 0; j < g.kp.nk; ++j)
    if ((x.key_st[j] = add(g.kp.cols[j])) < 0) return -1;
  x.nst_hist = x.nst;
  for (int v = 0; v < g.ap.nvals; ++v)
    if ((x.val_st[v] = add(g.ap.vals[v])) < 0) return -1;
  (void)nv;
  (void)vagg;
  (void)need_nn;
  return 0;
}

int brx_enqueue(const BrxArgs& a, int64_t ntiles, int64_t m, size_t max_scatter_lds, size_t max_hist_lds,
                int grid_agg, hipStream_t stream) {
  constexpr int STILE = kXScanBlock * kXScanItems;
  const int64_t nscan = (m + STILE - 1) / STILE;
  int64_t iblocks = (nscan + a.nrf + 255) / 256;
  if (iblocks < 1) iblocks = 1;
  if (iblocks > 4096) iblocks = 4096;
  hipLaunchKernelGGL(k_brx_init, dim3((unsigned)iblocks), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_brx_hist, dim3((unsigned)ntiles), dim3(kXBlock), max_hist_lds, stream, a);
  hipLaunchKernelGGL((k_brx_scan<kXScanBlock, kXScanItems>), dim3((unsigned)(nscan > 0 ? nscan : 1)),
                     dim3(kXScanBlock), 0, stream, (const uint32_t*)a.counts, m, a.starts, a.scan_ticket,
                     a.scan_status, nscan > 0 ? nscan : 1);
  hipLaunchKernelGGL(k_brx_scatter, dim3((unsigned)ntiles), dim3(kXBlock), max_scatter_lds, stream, a);
  hipLaunchKernelGGL(k_brx_agg, dim3((unsigned)grid_agg), dim3(kXJoinBlock),
                     (size_t)a.lcap * (8 + 8 * (size_t)a.nacc), stream, a);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GQ_OK : GQ_ERR_HIP;
}

}  // namespace gq
