// Batched fragments: thousands of independent filter + group-by fragments of
// very different sizes in one persistent launch, captured in a HIP graph.
//
// The paper finds the largest batch that fits GPU memory to be the fastest
// (Section 2.3) and reports that millions of small vectors degrade GPU
// libraries until they are merged (Section 3.3).  Here small and large
// fragments share one launch instead: the plan cuts every fragment into tiles
// of `tile_rows` rows, and a persistent grid takes tiles from one ticket
// counter until none is left, so a 1,000-row fragment costs one tile and a
// 4,000,000-row fragment is spread over every CU.
//
// Graph (built once per plan, replayed by gq_batch_plan_launch):
//   1. k_batch_init     every fragment's HBM table in one arena: keys EMPTY,
//                       accumulators at their identity; resets the ticket.
//   2. k_batch_agg      persistent: take a tile, filter its rows, aggregate
//                       into an LDS table (fragments expecting few groups,
//                       merged into HBM at the end of the tile) or straight into
//                       the fragment's HBM table.
//   3. k_batch_compact  one block per fragment: stable compaction of its table
//                       into the fragment's output batch, in slot order.
#include "agg.h"
#include "batchrx.h"

#include <vector>

namespace gq {
namespace {

constexpr int kBBlock = 256;
constexpr int kBItems = 4;
constexpr int kBCItems = 8;
constexpr int kBLdsTileMul = 4;  // work item of an LDS fragment: this many tiles


struct BatchArgs {
  const GbArgs* frags;        // per-fragment plan, in device memory
  const BatchOut* outs;       // per-fragment output, in device memory
  const int64_t* tile_start;  // nfrag + 1 prefix sums of tiles per fragment
  int64_t ntiles;
  int32_t nfrag;
  int32_t tile_rows;
  int32_t lcap;               // LDS table slots for LDS fragments
  int32_t nacc;
  int32_t nk;
  int32_t naggs;
  uint64_t* keys;             // arena: every fragment's keys
  uint64_t* acc;              // arena: every fragment's accumulators
  int64_t nslots;             // arena slots
  AggPlan ap;                 // shared aggregate plan (word kinds)
  uint32_t* ticket;
};

__global__ void k_batch_init(const BatchArgs a) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  if (i0 == 0) *a.ticket = 0;
  for (int64_t i = i0; i < a.nslots; i += step) {
    a.keys[i] = kEmpty;
    for (int w = 0; w < a.nacc; ++w) a.acc[i * a.nacc + w] = word_identity(a.ap.wop[w]);
  }
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_batch_agg(const BatchArgs a) {
  extern __shared__ uint64_t s_tab[];
  __shared__ int64_t s_t;
  __shared__ int32_t s_f;
  const int sw = 1 + a.nacc;
  for (;;) {
    if (threadIdx.x == 0) {
      const int64_t t = (int64_t)atomicAdd(a.ticket, 1u);
      int f = 0;
      if (t < a.ntiles) {
        int lo = 0, hi = a.nfrag;  // last fragment with tile_start <= t
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (a.tile_start[mid] <= t) lo = mid; else hi = mid;
        }
        f = lo;
      }
      s_t = t;
      s_f = f;
    }
    __syncthreads();
    const int64_t t = s_t;
    if (t >= a.ntiles) break;
    const int f = __builtin_amdgcn_readfirstlane(s_f);
    const GQ_CONST_AS GbArgs& g = cref(a.frags + f);
    const int64_t tr = g.tile_rows;
    const int64_t row0 = (t - cref(a.tile_start + f)) * tr;
    const int64_t row1 = row0 + tr < g.n ? row0 + tr : g.n;
    const bool lds = g.lcap > 0;
    if (lds) {
      for (int i = threadIdx.x; i < a.lcap * sw; i += BLOCK) {
        const int wi = i % sw;
        s_tab[i] = wi == 0 ? kEmpty : word_identity(a.ap.wop[wi - 1]);
      }
      __syncthreads();
    }
    for (int64_t r0 = row0 + (int64_t)threadIdx.x * ITEMS; r0 < row1; r0 += BLOCK * ITEMS) {
      uint32_t keep = eval_preds<ITEMS>(g, r0, row1);
      if (!keep) continue;
      uint32_t w[ITEMS];
      uint64_t key[ITEMS];
      uint8_t special[ITEMS];
      make_keys<ITEMS>(g.kp, r0, row1, key, special);
      int loff[ITEMS];
      uint64_t* gsp[ITEMS];
      static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
        constexpr int k = decltype(kk)::value;
        w[k] = 1;
        loff[k] = -1;
        gsp[k] = nullptr;
        if (!((keep >> k) & 1u)) return;
        if (lds && !special[k]) loff[k] = lds_find_insert(s_tab, a.lcap, sw, key[k]);
        if (loff[k] < 0) {
          gsp[k] = global_acc(g, key[k], special[k]);
          if (!gsp[k]) keep &= ~(1u << k);
        }
      });
      apply_rows<ITEMS>(g.ap, r0, row1, keep, w, s_tab, loff, gsp);
    }
    __syncthreads();
    if (lds) {
      for (int i = threadIdx.x; i < a.lcap; i += BLOCK) {
        const uint64_t* ls = s_tab + (size_t)i * sw;
        if (ls[0] == kEmpty) continue;
        uint64_t* gs = global_acc(g, ls[0], 0);
        if (gs) merge_words(g.ap, gs, ls + 1);
      }
      __syncthreads();
    }
  }
}

// One block per fragment: compact its table (cap hashed slots, then the two
// extra slots) into its output, in slot order.
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_batch_compact(const BatchArgs a) {
  constexpr int NW = BLOCK / kWave;
  constexpr int TILE = BLOCK * ITEMS;
  __shared__ uint32_t s_wave[NW];
  const int f = blockIdx.x;
  const GQ_CONST_AS GbArgs& g = cref(a.frags + f);
  const GQ_CONST_AS BatchOut& bo = cref(a.outs + f);
  const int64_t total = (int64_t)g.cap + 2;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  // Radix fragments: the groups of the HBM table (special keys, overflow)
  // follow those the radix aggregation already wrote.
  int64_t run = bo.append ? *bo.d_groups : 0;
  for (int64_t c0 = 0; c0 < total; c0 += TILE) {
    const int64_t i0 = c0 + (int64_t)threadIdx.x * ITEMS;
    uint32_t keep = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = i0 + k;
      if (i >= total) continue;
      const bool extra = i >= (int64_t)g.cap;
      const bool occ = extra ? g.acc[i * a.nacc] != 0 : g.keys[i] != kEmpty;
      if (occ) keep |= 1u << k;
    }
    uint32_t wtot;
    const uint32_t wpre = wave_prefix_small<4>((uint32_t)__popc(keep), &wtot);
    if (lane == 0) s_wave[wave] = wtot;
    __syncthreads();
    uint32_t bpre = 0, btot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      if (q < wave) bpre += s_wave[q];
      btot += s_wave[q];
    }
    __syncthreads();
    int64_t pos = run + bpre + wpre;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      if (!((keep >> k) & 1u)) continue;
      const int64_t s = i0 + k;
      if (pos < bo.out_cap) {
        const bool extra = s >= (int64_t)g.cap;
        for (int j = 0; j < a.nk + a.naggs; ++j) {
          const auto& o = bo.out[j];
          int64_t v = 0;
          bool ok = true;
          if (j < a.nk) {
            if (g.kp.mode == KEY_RAW64) {
              if (extra) {
                ok = s != (int64_t)g.cap + 1;
                v = ok ? -1 : 0;
              } else {
                v = (int64_t)g.keys[s];
              }
            } else {
              v = decode_field(g.kp, g.keys[s], j, &ok);
            }
          } else {
            const auto& ag = g.ap.aggs[j - a.nk];
            const uint64_t* acc = g.acc + s * a.nacc;
            v = (int64_t)acc[ag.word];
            if ((ag.op == GQ_SUM || ag.op == GQ_MIN || ag.op == GQ_MAX) && ag.cword >= 0) ok = acc[ag.cword] != 0;
            if (!ok) v = 0;
          }
          switch (o.type) {
            case GQ_I8: o.data[pos] = (uint8_t)v; break;
            case GQ_I16: reinterpret_cast<int16_t*>(o.data)[pos] = (int16_t)v; break;
            case GQ_I32: reinterpret_cast<int32_t*>(o.data)[pos] = (int32_t)v; break;
            default: reinterpret_cast<int64_t*>(o.data)[pos] = v; break;
          }
          if (o.valid) {
            const uint32_t bit = 1u << (pos & 31);
            if (ok) atomicOr(&o.valid[pos >> 5], bit);
            else atomicAnd(&o.valid[pos >> 5], ~bit);
          }
        }
      }
      ++pos;
    }
    run += btot;
  }
  if (threadIdx.x == 0) {
    *bo.d_groups = run;
    if (run > bo.out_cap) atomicOr(g.dev_status, GQ_DEV_CAPACITY);
  }
}

}  // namespace
}  // namespace gq

using namespace gq;

struct gq_batch_plan {
  gq_ctx* ctx = nullptr;
  void* mem = nullptr;  // arena + descriptors, one allocation
  size_t bytes = 0;
  hipStream_t cap_stream = nullptr;
  hipStream_t side_stream = nullptr;  // capture only: the tile path beside the radix path
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t total_rows = 0;
  int64_t ntiles = 0;
  int64_t nslots = 0;
  int32_t nfrag = 0;
  int32_t grid = 0;
};

namespace {

void plan_release(gq_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) {
    (void)hipStreamSynchronize(p->cap_stream);
    (void)hipStreamDestroy(p->cap_stream);
  }
  if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->mem) {
    (void)hipDeviceSynchronize();
    gq::ctx_free(p->ctx, p->mem, p->bytes, nullptr);
    (void)hipDeviceSynchronize();
  }
  delete p;
}

}  // namespace

extern "C" {

int gq_batch_plan_create(gq_ctx* ctx, const gq_fragment* frags, int nfrags, const gq_batch_spec* spec,
                         hipStream_t stream, gq_batch_plan** out) {
  if (!ctx || !out) return GQ_ERR_INVALID;
  *out = nullptr;
  if (nfrags < 1 || !frags || !spec) return set_error(ctx, GQ_ERR_INVALID, "gq_batch_plan_create: bad arguments");
  const float lf = spec->load_factor > 0.f ? spec->load_factor : 0.5f;
  if (!(lf > 0.f && lf <= 0.9f)) return set_error(ctx, GQ_ERR_INVALID, "gq_batch_plan_create: load factor outside (0, 0.9]");
  const int tile_rows = spec->tile_rows > 0 ? spec->tile_rows : 8192;
  if (tile_rows % (kBBlock * kBItems) != 0)
    return set_error(ctx, GQ_ERR_INVALID, "gq_batch_plan_create: tile_rows must be a multiple of 1024");
  const int lds_max = spec->lds_max_groups >= 0 ? (spec->lds_max_groups ? spec->lds_max_groups : 256) : 0;
  const int bpc = spec->blocks_per_cu > 0 ? spec->blocks_per_cu : 4;
  const int64_t radix_min = spec->radix_min_groups >= 0
                                ? (spec->radix_min_groups ? spec->radix_min_groups : (int64_t)lds_max + 1)
                                : INT64_MAX;

  std::vector<GbArgs> plans((size_t)nfrags);
  std::vector<BatchOut> outs((size_t)nfrags);
  std::vector<int64_t> tstart((size_t)nfrags + 1, 0);
  std::vector<char> is_radix((size_t)nfrags, 0);
  int64_t nslots = 0, total_rows = 0;
  int nacc = 0;
  for (int f = 0; f < nfrags; ++f) {
    const gq_fragment& fr = frags[f];
    int rc = check_batch(ctx, &fr.in, "gq_batch_plan_create fragment");
    if (rc) return rc;
    GbArgs& g = plans[f];
    std::memset(&g, 0, sizeof(g));
    g.n = fr.in.nrows;
    g.dev_status = ctx->d_status;
    rc = make_preds(ctx, g, &fr.in, fr.preds, fr.npreds);
    if (rc) return rc;
    rc = make_key_plan(ctx, g.kp, &fr.in, spec->keys, spec->nkeys);
    if (rc) return rc;
    rc = make_agg_plan(ctx, g.ap, &fr.in, spec->aggs, spec->naggs);
    if (rc) return rc;
    if (f == 0) nacc = g.ap.nacc;
    if (g.ap.nacc != nacc || g.kp.mode != plans[0].kp.mode)
      return set_error(ctx, GQ_ERR_INVALID, "gq_batch_plan_create: fragments must share key and aggregate shapes");
    // Every fragment's accumulators are initialised and merged with one word
    // layout (the first fragment's), so the layouts must agree word for word:
    // an aggregate input that can be NULL in one fragment and not in another
    // moves the words that follow it.
    bool same_words = true;
    for (int w = 0; w < nacc; ++w) same_words &= g.ap.wop[w] == plans[0].ap.wop[w];
    for (int i = 0; i < g.ap.naggs; ++i)
      same_words &= g.ap.aggs[i].word == plans[0].ap.aggs[i].word && g.ap.aggs[i].cword == plans[0].ap.aggs[i].cword;
    if (!same_words)
      return set_error(ctx, GQ_ERR_INVALID,
                       "gq_batch_plan_create: fragments must agree on which aggregate inputs can be NULL");
    for (int j = 0; j < spec->nkeys; ++j)
      if (g.kp.bits[j] != plans[0].kp.bits[j] || g.kp.nullable[j] != plans[0].kp.nullable[j])
        return set_error(ctx, GQ_ERR_INVALID, "gq_batch_plan_create: fragments must share key column types");
    const int64_t expected = fr.expected_groups > 0 ? fr.expected_groups : (fr.in.nrows > 0 ? fr.in.nrows : 1);
    uint64_t cap = (uint64_t)((double)(spec->nkeys == 0 ? 1 : expected) / lf) + 1;
    if (cap < 16) cap = 16;
    g.cap = cap;
    g.lcap = expected <= lds_max ? 1 : 0;  // LDS flag; the size is set below
    // LDS fragments merge their table into HBM after every work item, with
    // device-wide atomics that contend on few slots: larger items, fewer merges.
    g.tile_rows = g.lcap ? (int64_t)tile_rows * kBLdsTileMul : tile_rows;
    g.keys = reinterpret_cast<uint64_t*>((uintptr_t)nslots);  // offset for now
    nslots += (int64_t)cap + 2;
    total_rows += g.n;
    is_radix[f] = spec->nkeys > 0 && expected >= radix_min && g.n > 0 && g.n < ((int64_t)1 << 31);
    tstart[f + 1] = tstart[f] + (is_radix[f] ? 0 : (g.n + g.tile_rows - 1) / g.tile_rows);
    // outputs
    BatchOut& bo = outs[f];
    std::memset(&bo, 0, sizeof(bo));
    const int ncols = spec->nkeys + spec->naggs;
    if (fr.out.ncols < ncols || (ncols > 0 && !fr.out.cols) || !fr.d_groups)
      return set_error(ctx, GQ_ERR_INVALID, "gq_batch_plan_create: fragment output needs key and aggregate columns");
    bo.out_cap = INT64_MAX;
    for (int j = 0; j < ncols; ++j) {
      const gq_column& oc = fr.out.cols[j];
      const int want = j < spec->nkeys ? fr.in.cols[spec->keys[j]].type : GQ_I64;
      if (oc.type != want || oc.length < 0 || (oc.length > 0 && !oc.data) || oc.offset != 0 ||
          (oc.validity && (reinterpret_cast<uintptr_t>(oc.validity) & 3)))
        return set_error(ctx, GQ_ERR_INVALID, "gq_batch_plan_create: bad fragment output column");
      bo.out[j] = OCol{static_cast<uint8_t*>(oc.data), reinterpret_cast<uint32_t*>(oc.validity), oc.type, 0};
      if (oc.length < bo.out_cap) bo.out_cap = oc.length;
    }
    bo.d_groups = fr.d_groups;
  }

  // Radix fragments: regions of about half an LDS table each, tiles, counts.
  BrxArgs rx;
  std::memset(&rx, 0, sizeof(rx));
  std::vector<BrxFrag> rfs;
  std::vector<int32_t> tile_frag, item_frag;
  int64_t rx_tiles = 0, rx_counts = 0, rx_items = 0, rx_rows = 0;
  size_t rx_scatter_lds = 0, rx_hist_lds = 0;
  {
    const AggPlan& ap0 = plans[0].ap;
    for (int i = 0; i < ap0.naggs; ++i) {
      rx.vword[i] = -1;
      const int op = ap0.aggs[i].op;
      if (op == GQ_SUM || op == GQ_MIN || op == GQ_MAX) {
        rx.vagg[rx.nv] = i;
        rx.vword[i] = rx.nv++;
      }
    }
    const int lcap_x = brx_lcap(nacc);
    const int64_t per_region = lcap_x / 2;
    for (int f = 0; f < nfrags; ++f) {
      if (!is_radix[f]) continue;
      const GbArgs& g = plans[f];
      bool nullable = false;
      for (int v = 0; v < g.ap.nvals; ++v) nullable |= g.ap.vals[v].valid != nullptr;
      rx.need_nn |= nullable ? 1 : 0;
      BrxFrag x;
      std::memset(&x, 0, sizeof(x));
      if (brx_stage_plan(x, g, rx.nv, rx.vagg, nullable) != 0) {
        // Too many distinct columns to stage: this fragment stays on the tile path.
        is_radix[f] = 0;
        continue;
      }
      const int64_t expected = frags[f].expected_groups > 0 ? frags[f].expected_groups : g.n;
      int rbits = 0;
      while (rbits < 10 && ((int64_t)1 << rbits) * per_region < expected) ++rbits;
      x.f = f;
      x.rbits = rbits;
      x.tiles = (g.n + brx_tile_rows() - 1) / brx_tile_rows();
      x.tile0 = rx_tiles;
      x.cbase = rx_counts;
      x.item0 = rx_items;
      rx_tiles += x.tiles;
      rx_counts += x.tiles << rbits;
      rx_items += (int64_t)1 << rbits;
      rx_rows += g.n;
      tile_frag.insert(tile_frag.end(), (size_t)x.tiles, (int32_t)rfs.size());
      item_frag.insert(item_frag.end(), (size_t)1 << rbits, (int32_t)rfs.size());
      const size_t sl = brx_scatter_lds_bytes(x);
      const size_t hl = brx_hist_lds_bytes(x);
      if (sl > rx_scatter_lds) rx_scatter_lds = sl;
      if (hl > rx_hist_lds) rx_hist_lds = hl;
      rfs.push_back(x);
    }
    // Fragments that fell back to the tile path need tiles again.
    for (int f = 0; f < nfrags; ++f) {
      const int64_t t = is_radix[f] ? 0 : (plans[f].n + plans[f].tile_rows - 1) / plans[f].tile_rows;
      tstart[f + 1] = tstart[f] + t;
    }
    for (int f = 0; f < nfrags; ++f) outs[f].append = is_radix[f] ? 1 : 0;
    rx.nrf = (int32_t)rfs.size();
    rx.lcap = lcap_x;
    rx.nacc = nacc;
    rx.nk = spec->nkeys;
    rx.nitems = rx_items;
    if (rx_scatter_lds > 150 * 1024 || rx_hist_lds > 150 * 1024) {
      // A staging layout this wide does not fit: every fragment takes the tile path.
      rfs.clear();
      tile_frag.clear();
      item_frag.clear();
      rx.nrf = 0;
      rx_tiles = rx_counts = rx_items = rx_rows = 0;
      for (int f = 0; f < nfrags; ++f) {
        is_radix[f] = 0;
        outs[f].append = 0;
        tstart[f + 1] = tstart[f] + (plans[f].n + plans[f].tile_rows - 1) / plans[f].tile_rows;
      }
    }
  }
  const int sw = 1 + nacc;
  int lcap = 1;
  while ((size_t)(lcap * 2) * sw * 8 <= 32 * 1024) lcap *= 2;

  // One allocation: keys, accumulators, plans, outputs, tile starts, ticket.
  const size_t off_keys = 0;
  const size_t off_acc = align_up((size_t)nslots * 8, 256);
  const size_t off_plans = align_up(off_acc + (size_t)nslots * nacc * 8, 256);
  const size_t off_outs = align_up(off_plans + sizeof(GbArgs) * nfrags, 256);
  const size_t off_ts = align_up(off_outs + sizeof(BatchOut) * nfrags, 256);
  const size_t off_ticket = align_up(off_ts + 8 * ((size_t)nfrags + 1), 256);
  // Radix path: fragment descriptors, counts, starts, scan status, tuples.
  const int64_t rx_nscan = (rx_counts + 4095) / 4096;
  const size_t off_rf = off_ticket + 256;
  const size_t off_tf = align_up(off_rf + sizeof(BrxFrag) * rfs.size(), 256);
  const size_t off_if = align_up(off_tf + 4 * tile_frag.size(), 256);
  const size_t off_cnt = align_up(off_if + 4 * item_frag.size(), 256);
  const size_t off_st = align_up(off_cnt + 4 * (size_t)rx_counts, 256);
  const size_t off_ss = align_up(off_st + 8 * ((size_t)rx_counts + 1), 256);
  const size_t off_tup = align_up(off_ss + 8 * (size_t)(rx_nscan + 1), 256);
  const size_t off_tnn = align_up(off_tup + 8 * (size_t)(1 + rx.nv) * (size_t)rx_rows, 256);
  const size_t total = align_up(off_tnn + (rx.need_nn ? (size_t)rx_rows : 0), 256) + 256;

  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  gq_batch_plan* p = new (std::nothrow) gq_batch_plan;
  if (!p) return GQ_ERR_NOMEM;
  p->ctx = ctx;
  p->mem = ctx_alloc(ctx, total, stream);
  if (!p->mem) {
    delete p;
    const std::string msg = "gq_batch_plan_create: allocation of " + std::to_string(total) + " bytes failed (" +
                            std::to_string(nslots) + " table slots, " + std::to_string(rx_rows) + " radix rows)";
    return set_error(ctx, GQ_ERR_NOMEM, msg.c_str());
  }
  p->bytes = total;
  char* base = static_cast<char*>(p->mem);
  uint64_t* keys = reinterpret_cast<uint64_t*>(base + off_keys);
  uint64_t* acc = reinterpret_cast<uint64_t*>(base + off_acc);
  for (int f = 0; f < nfrags; ++f) {
    GbArgs& g = plans[f];
    const uint64_t off = (uint64_t)reinterpret_cast<uintptr_t>(g.keys);
    g.keys = keys + off;
    g.acc = acc + off * nacc;
    g.lcap = g.lcap ? lcap : 0;
  }
  BatchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.frags = reinterpret_cast<const GbArgs*>(base + off_plans);
  a.outs = reinterpret_cast<const BatchOut*>(base + off_outs);
  a.tile_start = reinterpret_cast<const int64_t*>(base + off_ts);
  a.ntiles = tstart[nfrags];
  a.nfrag = nfrags;
  a.tile_rows = tile_rows;
  a.lcap = lcap;
  a.nacc = nacc;
  a.nk = spec->nkeys;
  a.naggs = spec->naggs;
  a.keys = keys;
  a.acc = acc;
  a.nslots = nslots;
  a.ap = plans[0].ap;
  a.ticket = reinterpret_cast<uint32_t*>(base + off_ticket);
  rx.frags = a.frags;
  rx.outs = a.outs;
  rx.rf = reinterpret_cast<const BrxFrag*>(base + off_rf);
  rx.tile_frag = reinterpret_cast<const int32_t*>(base + off_tf);
  rx.item_frag = reinterpret_cast<const int32_t*>(base + off_if);
  rx.counts = reinterpret_cast<uint32_t*>(base + off_cnt);
  rx.starts = reinterpret_cast<int64_t*>(base + off_st);
  rx.scan_status = reinterpret_cast<uint64_t*>(base + off_ss);
  rx.scan_ticket = reinterpret_cast<uint32_t*>(base + off_ticket + 64);
  rx.item_ticket = reinterpret_cast<unsigned long long*>(base + off_ticket + 128);
  rx.nscan = rx_nscan;
  rx.tup = reinterpret_cast<uint64_t*>(base + off_tup);
  rx.tnn = rx.need_nn ? reinterpret_cast<uint8_t*>(base + off_tnn) : nullptr;
  p->total_rows = total_rows;
  p->ntiles = a.ntiles;
  p->nslots = nslots;
  p->nfrag = nfrags;

  auto fail = [&](int code, const char* what) {
    set_error(ctx, code, what);
    plan_release(p);
    return code;
  };
  if (hipMemcpyAsync(base + off_plans, plans.data(), sizeof(GbArgs) * nfrags, hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipMemcpyAsync(base + off_outs, outs.data(), sizeof(BatchOut) * nfrags, hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipMemcpyAsync(base + off_ts, tstart.data(), 8 * ((size_t)nfrags + 1), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      (!rfs.empty() && (hipMemcpyAsync(base + off_rf, rfs.data(), sizeof(BrxFrag) * rfs.size(),
                                       hipMemcpyHostToDevice, stream) != hipSuccess ||
                        hipMemcpyAsync(base + off_tf, tile_frag.data(), 4 * tile_frag.size(),
                                       hipMemcpyHostToDevice, stream) != hipSuccess ||
                        hipMemcpyAsync(base + off_if, item_frag.data(), 4 * item_frag.size(),
                                       hipMemcpyHostToDevice, stream) != hipSuccess)) ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(GQ_ERR_HIP, "gq_batch_plan_create: descriptor upload failed");

  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return fail(GQ_ERR_HIP, "device properties");
  p->grid = prop.multiProcessorCount * bpc;
  const size_t lds_bytes = (size_t)lcap * sw * 8;

  // Capture the kernels on a private stream (and a second one for the branch
  // of the tile path when radix fragments exist).
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess)
    return fail(GQ_ERR_HIP, "gq_batch_plan_create: stream creation failed");
  if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(GQ_ERR_HIP, "gq_batch_plan_create: graph capture failed");
  int64_t iblocks = (nslots + 255) / 256;
  if (iblocks > 8192) iblocks = 8192;
  hipLaunchKernelGGL(k_batch_init, dim3((unsigned)iblocks), dim3(256), 0, p->cap_stream, a);
  if (rx.nrf > 0) {
    // The tile path (k_batch_agg) and the radix path touch disjoint fragments
    // and counters: the graph runs them as two branches between the init and
    // the compaction.
    if (hipEventRecord(p->ev_fork, p->cap_stream) != hipSuccess ||
        hipStreamWaitEvent(p->side_stream, p->ev_fork, 0) != hipSuccess) {
      hipGraph_t g0 = nullptr;
      (void)hipStreamEndCapture(p->cap_stream, &g0);
      if (g0) (void)hipGraphDestroy(g0);
      return fail(GQ_ERR_HIP, "gq_batch_plan_create: graph fork failed");
    }
    hipLaunchKernelGGL((k_batch_agg<kBBlock, kBItems>), dim3((unsigned)p->grid), dim3(kBBlock), lds_bytes,
                       p->side_stream, a);
    const bool rx_ok = brx_enqueue(rx, rx_tiles, rx_counts, rx_scatter_lds, rx_hist_lds, prop.multiProcessorCount,
                                   p->cap_stream) == GQ_OK;
    if (!rx_ok || hipEventRecord(p->ev_join, p->side_stream) != hipSuccess ||
        hipStreamWaitEvent(p->cap_stream, p->ev_join, 0) != hipSuccess) {
      hipGraph_t g0 = nullptr;
      (void)hipStreamEndCapture(p->cap_stream, &g0);
      if (g0) (void)hipGraphDestroy(g0);
      return fail(GQ_ERR_HIP, "gq_batch_plan_create: radix kernels failed to enqueue");
    }
  } else {
    hipLaunchKernelGGL((k_batch_agg<kBBlock, kBItems>), dim3((unsigned)p->grid), dim3(kBBlock), lds_bytes,
                       p->cap_stream, a);
  }
  hipLaunchKernelGGL((k_batch_compact<kBBlock, kBCItems>), dim3((unsigned)nfrags), dim3(kBBlock), 0, p->cap_stream, a);
  const hipError_t le = hipGetLastError();
  const hipError_t ce = hipStreamEndCapture(p->cap_stream, &p->graph);
  if (le != hipSuccess || ce != hipSuccess) return fail(GQ_ERR_HIP, "gq_batch_plan_create: graph capture failed");
  if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
    return fail(GQ_ERR_HIP, "gq_batch_plan_create: graph instantiation failed");
  *out = p;
  return GQ_OK;
}

int gq_batch_plan_launch(gq_batch_plan* plan, hipStream_t stream) {
  if (!plan || !plan->exec) return GQ_ERR_INVALID;
  hipError_t e = hipGraphLaunch(plan->exec, stream);
  if (e != hipSuccess) return hip_error(plan->ctx, e, "gq_batch_plan_launch");
  return GQ_OK;
}

int gq_batch_plan_info(const gq_batch_plan* plan, int64_t* total_rows, int64_t* tiles, int64_t* table_slots,
                       int64_t* bytes) {
  if (!plan) return GQ_ERR_INVALID;
  if (total_rows) *total_rows = plan->total_rows;
  if (tiles) *tiles = plan->ntiles;
  if (table_slots) *table_slots = plan->nslots;
  if (bytes) *bytes = (int64_t)plan->bytes;
  return GQ_OK;
}

int gq_batch_plan_free(gq_batch_plan* plan) {
  plan_release(plan);
  return GQ_OK;
}

}  // extern "C"
