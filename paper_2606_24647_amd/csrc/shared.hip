// gq_groupby_shared: several filter + group-by queries over the same batch in
// one pass (a shared scan).
//
// Queries that differ only in their predicate bounds read the same columns;
// each tile loads every column once, evaluates every query's predicates on the
// loaded values, and aggregates each query's kept rows into that query's own
// LDS table (spilling to its HBM table when the LDS table has no room).  The
// column bytes are read once for up to GQ_MAX_SHARED queries instead of once
// per query.  Each query's table is then compacted into its own output.
#include "agg.h"

namespace gq {
namespace {

constexpr int kSBlock = 256;
constexpr int kSItems = 4;
constexpr size_t kSLdsBudget = 48 * 1024;

struct SharedArgs {
  int64_t n;
  int64_t ntiles;
  int32_t nq;
  int32_t npreds;
  int32_t lcap;  // LDS slots per query (power of two)
  int32_t pad;
  int32_t op[GQ_MAX_PREDS];
  DCol pcols[GQ_MAX_PREDS];
  int64_t lo[GQ_MAX_SHARED][GQ_MAX_PREDS];
  int64_t hi[GQ_MAX_SHARED][GQ_MAX_PREDS];
  KeyPlan kp;
  AggPlan ap;
  uint64_t* keys[GQ_MAX_SHARED];
  uint64_t* acc[GQ_MAX_SHARED];
  uint64_t cap;
  int32_t* dev_status;
};

__device__ __forceinline__ uint64_t* shared_global_acc(const SharedArgs& a, int q, uint64_t key, int special) {
  int64_t s;
  if (special) {
    s = (int64_t)(a.cap + (uint64_t)(special - 1));
  } else {
    bool ins;
    s = find_insert(a.keys[q], a.cap, key, &ins);
    if (s < 0) {
      atomicOr(a.dev_status, GQ_DEV_TABLE_FULL);
      return nullptr;
    }
  }
  return a.acc[q] + (uint64_t)s * a.ap.nacc;
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_gb_shared(const SharedArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int Q = GQ_MAX_SHARED;
  extern __shared__ uint64_t s_tab[];
  const int sw = 1 + a.ap.nacc;
  const int per_q = a.lcap * sw;
  for (int i = threadIdx.x; i < a.nq * per_q; i += BLOCK) {
    const int wi = (i % per_q) % sw;
    s_tab[i] = wi == 0 ? kEmpty : word_identity(a.ap.wop[wi - 1]);
  }
  __syncthreads();

  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;
    uint32_t inrange = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (r0 + k < a.n) inrange |= 1u << k;
    uint32_t keep[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) keep[q] = q < a.nq ? inrange : 0u;
    for (int p = 0; p < a.npreds; ++p) {
      int64_t v[ITEMS];
      load_items<ITEMS, true>(a.pcols[p], r0, a.n, v);
      const uint32_t vm = a.pcols[p].valid ? valid_items<ITEMS>(a.pcols[p], r0, a.n) : 0xffffffffu;
      static_for<0, Q>([&](auto qq) __attribute__((always_inline)) {
        constexpr int q = decltype(qq)::value;
        if (q >= a.nq) return;
        const DPred pr{0, a.op[p], a.lo[q][p], a.hi[q][p]};
        uint32_t m = vm;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
          if (!pred_pass(pr, v[k])) m &= ~(1u << k);
        keep[q] &= m;
      });
    }
    uint32_t any = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) any |= keep[q];
    if (!any) continue;
    uint64_t key[ITEMS];
    uint8_t special[ITEMS];
    make_keys<ITEMS>(a.kp, r0, a.n, key, special);
    // Slots of every (query, row): LDS word offset, else the HBM accumulators.
    int loff[Q][ITEMS];
    uint64_t* gsp[Q][ITEMS];
    static_for<0, Q>([&](auto qq) __attribute__((always_inline)) {
      constexpr int q = decltype(qq)::value;
      static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
        constexpr int k = decltype(kk)::value;
        loff[q][k] = -1;
        gsp[q][k] = nullptr;
        if (!((keep[q] >> k) & 1u)) return;
        if (!special[k]) {
          const int o = lds_find_insert(s_tab + q * per_q, a.lcap, sw, key[k]);
          if (o >= 0) loff[q][k] = q * per_q + o;
        }
        if (loff[q][k] < 0) {
          gsp[q][k] = shared_global_acc(a, q, key[k], special[k]);
          if (!gsp[q][k]) keep[q] &= ~(1u << k);
        }
        if (loff[q][k] >= 0) SharedAtomics::add(&s_tab[loff[q][k]], 1);
        else if (gsp[q][k]) GlobalAtomics::add(&gsp[q][k][0], 1);
      });
    });
    for (int i = 0; i < a.ap.naggs; ++i) {
      const DAgg& ag = a.ap.aggs[i];
      if (ag.op == GQ_COUNT_STAR) continue;
      uint64_t x[ITEMS];
      const uint32_t nn = agg_values<ITEMS>(ag, a.ap, r0, a.n, x);
      static_for<0, Q>([&](auto qq) __attribute__((always_inline)) {
        constexpr int q = decltype(qq)::value;
        const uint32_t m = keep[q] & nn;
        static_for<0, ITEMS>([&](auto kk) __attribute__((always_inline)) {
          constexpr int k = decltype(kk)::value;
          if (!((m >> k) & 1u)) return;
          if (loff[q][k] >= 0) {
            uint64_t* s = s_tab + loff[q][k];
            switch (ag.op) {
              case GQ_SUM: SharedAtomics::add(&s[ag.word], x[k]); break;
              case GQ_COUNT: SharedAtomics::add(&s[ag.word], 1); break;
              case GQ_MIN: SharedAtomics::min(&s[ag.word], (int64_t)x[k]); break;
              default: SharedAtomics::max(&s[ag.word], (int64_t)x[k]); break;
            }
            if (ag.cword >= 0) SharedAtomics::add(&s[ag.cword], 1);
          } else {
            uint64_t* s = gsp[q][k];
            switch (ag.op) {
              case GQ_SUM: GlobalAtomics::add(&s[ag.word], x[k]); break;
              case GQ_COUNT: GlobalAtomics::add(&s[ag.word], 1); break;
              case GQ_MIN: GlobalAtomics::min(&s[ag.word], (int64_t)x[k]); break;
              default: GlobalAtomics::max(&s[ag.word], (int64_t)x[k]); break;
            }
            if (ag.cword >= 0) GlobalAtomics::add(&s[ag.cword], 1);
          }
        });
      });
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.nq * a.lcap; i += BLOCK) {
    const int q = i / a.lcap;
    const uint64_t* ls = s_tab + (size_t)i * sw;
    if (ls[0] == kEmpty) continue;
    uint64_t* gs = shared_global_acc(a, q, ls[0], 0);
    if (gs) merge_words(a.ap, gs, ls + 1);
  }
}

__global__ void k_shared_init(SharedArgs a, int64_t nslots) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int q = 0; q < a.nq; ++q)
    for (int64_t i = i0; i < nslots; i += step) {
      a.keys[q][i] = kEmpty;
      for (int w = 0; w < a.ap.nacc; ++w) a.acc[q][i * a.ap.nacc + w] = word_identity(a.ap.wop[w]);
    }
}

}  // namespace
}  // namespace gq

using namespace gq;

extern "C" int gq_groupby_shared(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys,
                                 const gq_pred* preds, int npreds, int nqueries, const gq_agg* aggs, int naggs,
                                 const gq_groupby_opts* opts, gq_batch* outs, int64_t* d_groups,
                                 hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_groupby_shared input");
  if (rc) return rc;
  if (nqueries < 1 || nqueries > GQ_MAX_SHARED || !outs || !d_groups)
    return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_shared: 1..8 queries with outputs and counts");
  if (npreds < 0 || npreds > GQ_MAX_PREDS || (npreds > 0 && !preds))
    return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_shared: bad predicate list");
  gq_groupby_opts o{};
  if (opts) o = *opts;
  const float lf = o.load_factor > 0.f ? o.load_factor : 0.5f;
  if (!(lf > 0.f && lf <= 0.9f)) return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_shared: load factor outside (0, 0.9]");

  SharedArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = in->nrows;
  a.nq = nqueries;
  a.npreds = npreds;
  a.dev_status = ctx->d_status;
  for (int p = 0; p < npreds; ++p) {
    const gq_pred& p0 = preds[p];
    if (p0.col < 0 || p0.col >= in->ncols || (p0.op != GQ_RANGE && p0.op != GQ_NE))
      return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_shared: bad predicate");
    a.op[p] = p0.op;
    a.pcols[p] = make_dcol(in->cols[p0.col]);
    for (int q = 0; q < nqueries; ++q) {
      const gq_pred& pq = preds[q * npreds + p];
      if (pq.col != p0.col || pq.op != p0.op)
        return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_shared: queries must share predicate columns and ops");
      a.lo[q][p] = pq.lo;
      a.hi[q][p] = pq.hi;
    }
  }
  rc = make_key_plan(ctx, a.kp, in, keys, nkeys);
  if (rc) return rc;
  for (int j = 0; j < nkeys; ++j) a.kp.cols[j].nt = 1;
  rc = make_agg_plan(ctx, a.ap, in, aggs, naggs);
  if (rc) return rc;
  for (int v = 0; v < a.ap.nvals; ++v) a.ap.vals[v].nt = 0;  // re-read by every aggregate that uses it

  int key_types[GQ_MAX_KEYS];
  for (int j = 0; j < nkeys; ++j) key_types[j] = in->cols[keys[j]].type;
  CompactArgs ca[GQ_MAX_SHARED];
  for (int q = 0; q < nqueries; ++q) {
    std::memset(&ca[q], 0, sizeof(CompactArgs));
    rc = check_outputs(ctx, nkeys, naggs, &outs[q], ca[q], key_types);
    if (rc) return rc;
  }
  int64_t expected = o.expected_groups > 0 ? o.expected_groups : in->nrows;
  if (nkeys == 0) expected = 1;
  uint64_t cap = (uint64_t)((double)expected / lf) + 1;
  if (cap < 16) cap = 16;
  a.cap = cap;
  const size_t nslot = (size_t)cap + 2;
  const size_t per_keys = align_up(nslot * 8, 256);
  const size_t per_acc = align_up(nslot * 8 * (size_t)a.ap.nacc, 256);
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  Scratch tables(ctx, stream);
  if (!tables.get((per_keys + per_acc) * nqueries))
    return set_error(ctx, GQ_ERR_NOMEM, "gq_groupby_shared: table allocation failed");
  for (int q = 0; q < nqueries; ++q) {
    a.keys[q] = tables.as<uint64_t>((per_keys + per_acc) * q);
    a.acc[q] = tables.as<uint64_t>((per_keys + per_acc) * q + per_keys);
  }
  const int sw = 1 + a.ap.nacc;
  int lcap = 1;
  while ((size_t)(lcap * 2) * sw * 8 * nqueries <= kSLdsBudget) lcap *= 2;
  a.lcap = lcap;
  int64_t iblocks = (int64_t)((nslot + 255) / 256);
  if (iblocks > 4096) iblocks = 4096;
  GQ_LAUNCH(ctx, "shared_init", k_shared_init, dim3((unsigned)iblocks), dim3(256), 0, stream, a, (int64_t)nslot);
  GQ_LAUNCH_CHECK(ctx);
  constexpr int TILE = kSBlock * kSItems;
  a.ntiles = (a.n + TILE - 1) / TILE;
  if (a.ntiles > 0) {
    const size_t lds = (size_t)lcap * sw * 8 * nqueries;
    int64_t grid = a.ntiles < 1024 ? a.ntiles : 1024;
    GQ_LAUNCH(ctx, "gb_shared", (k_gb_shared<kSBlock, kSItems>), dim3((unsigned)grid), dim3(kSBlock), lds, stream, a);
    GQ_LAUNCH_CHECK(ctx);
  }
  for (int q = 0; q < nqueries; ++q) {
    ca[q].naggs = naggs;
    for (int i = 0; i < naggs; ++i) ca[q].aggs[i] = a.ap.aggs[i];
    ca[q].global_agg = nkeys == 0;
    ca[q].keys = a.keys[q];
    ca[q].acc = a.acc[q];
    ca[q].d_cap = nullptr;
    ca[q].cap = cap;
    ca[q].cap_alloc = cap;
    ca[q].aw = a.ap.nacc;
    ca[q].key_kind = a.kp.mode == KEY_RAW64 ? 1 : 0;
    ca[q].kp = a.kp;
    ca[q].extra = 2;
    rc = finish_groups(ctx, ca[q], &outs[q], d_groups + q, (o.flags & GQ_SORTED) != 0 && nkeys > 0, stream);
    if (rc) return rc;
  }
  return GQ_OK;
}
