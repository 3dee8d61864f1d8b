// Streaming aggregation (gq_agg_stream_*): one aggregation over a sequence of
// batches in one of the four modes of Section 3.2, holding its groups in an
// HBM hash table between batches.
//
// The paper's operator aggregates each batch, concatenates the result with the
// groups held so far and aggregates the concatenation again, emitting once the
// held result reaches a size threshold.  The held groups here stay in one
// open-addressing table that every batch is aggregated into directly (merging
// a batch into the held groups and aggregating the concatenation give the same
// groups and values: SUM, COUNT and MIN/MAX are associative and commutative,
// and wrapping int64 sums make the order of additions irrelevant).  The
// number of held groups is counted on the device (one atomic per inserted
// group), and the emission that follows a batch is a compaction and a table
// reset gated by a device flag, so no call waits for the device.
//
// Per push: k_gt/k_gb (the group-by kernels) aggregate the batch; k_as_after
// updates the counters and sets the emission flag; a gated compaction writes
// the held groups; k_as_init, gated by the same flag, empties the table.
#include "agg.h"

namespace gq {
namespace {

enum { ST_INSERTED = 0, ST_BATCHES = 1, ST_HELD = 2, ST_EMIT = 3, ST_FIN = 4, ST_WORDS = 8 };

struct AsWords {
  int32_t nacc;
  int32_t pad;
  uint64_t ident[kMaxAcc];  // initial value of every accumulator word
};

// Empty the held table (keys EMPTY, accumulators at their identity) and reset
// the counters; with a gate, only when *gate != 0.
__global__ void k_as_init(uint64_t* keys, uint64_t* acc, int64_t nslots, AsWords w, int64_t* st,
                          const int64_t* gate) {
  if (gate && *gate == 0) return;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < nslots; i += step) {
    keys[i] = kEmpty;
    for (int k = 0; k < w.nacc; ++k) acc[i * w.nacc + k] = w.ident[k];
  }
  if (i0 == 0) {
    st[ST_INSERTED] = 0;
    st[ST_BATCHES] = 0;
    st[ST_HELD] = 0;
  }
}

// After a batch: one more batch held; the held group count (hashed groups
// inserted so far plus the two extra slots when used; one global group when
// there are no keys); the emission flag.
__global__ void k_as_after(int64_t* st, const uint64_t* acc, uint64_t cap, int nacc, int nkeys, int64_t emit_groups,
                           int can_emit, int64_t* d_emitted) {
  st[ST_BATCHES] += 1;
  int64_t g = 1;
  if (nkeys > 0)
    g = st[ST_INSERTED] + (acc[cap * (uint64_t)nacc] != 0 ? 1 : 0) + (acc[(cap + 1) * (uint64_t)nacc] != 0 ? 1 : 0);
  st[ST_HELD] = g;
  st[ST_EMIT] = (can_emit && emit_groups > 0 && g >= emit_groups) ? 1 : 0;
  if (d_emitted) *d_emitted = 0;
}

// Before finish: emit iff a batch is held.
__global__ void k_as_fin(int64_t* st, int64_t* d_groups) {
  st[ST_FIN] = st[ST_BATCHES] > 0 ? 1 : 0;
  d_groups[0] = 0;
  d_groups[1] = st[ST_FIN];
}

}  // namespace
}  // namespace gq

struct gq_agg_stream {
  gq_ctx* ctx = nullptr;
  int32_t mode = 0;
  int32_t nkeys = 0;
  int32_t naggs = 0;
  int32_t keys[GQ_MAX_KEYS] = {};
  int32_t key_nullable[GQ_MAX_KEYS] = {};
  int32_t key_types[GQ_MAX_KEYS] = {};
  gq_agg aggs[GQ_MAX_AGGS] = {};   // the aggregates applied to every batch (merge modes: merging ops)
  int64_t max_groups = 0;
  int64_t emit_groups = 0;
  uint64_t cap = 0;                // hashed slots; two extra slots follow
  void* mem = nullptr;
  size_t bytes = 0;
  uint64_t* keys_tab = nullptr;
  uint64_t* acc = nullptr;
  int64_t* st = nullptr;
  bool have_layout = false;        // set by the first push: accumulator layout and key plan
  gq::AsWords words{};
  gq::KeyPlan kp{};
  gq::AggPlan ap{};
  int strategy = GQ_STRATEGY_GLOBAL;
};

namespace gq {
namespace {

int as_compact(gq_ctx* ctx, gq_agg_stream* s, gq_batch* out, int64_t* d_count, const int64_t* gate,
               hipStream_t stream) {
  CompactArgs ca;
  std::memset(&ca, 0, sizeof(ca));
  ca.naggs = s->naggs;
  for (int i = 0; i < s->naggs; ++i) ca.aggs[i] = s->ap.aggs[i];
  ca.global_agg = s->nkeys == 0;
  int rc = check_outputs(ctx, s->nkeys, s->naggs, out, ca, s->key_types);
  if (rc) return rc;
  ca.keys = s->keys_tab;
  ca.acc = s->acc;
  ca.d_cap = nullptr;
  ca.cap = s->cap;
  ca.cap_alloc = s->cap;
  ca.aw = s->words.nacc;
  ca.key_kind = s->kp.mode == KEY_RAW64 ? 1 : 0;
  ca.kp = s->kp;
  ca.extra = 2;
  ca.gate = gate;
  return compact_launch(ctx, ca, d_count, stream);
}

int as_reset(gq_ctx* ctx, gq_agg_stream* s, const int64_t* gate, hipStream_t stream) {
  const int64_t nslots = (int64_t)s->cap + 2;
  int64_t blocks = (nslots + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  GQ_LAUNCH(ctx, "as_init", k_as_init, dim3((unsigned)blocks), dim3(256), 0, stream, s->keys_tab, s->acc, nslots,
            s->words, s->st, gate);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

}  // namespace
}  // namespace gq

using namespace gq;

extern "C" {

int gq_agg_stream_create(gq_ctx* ctx, const gq_agg_stream_spec* spec, hipStream_t stream, gq_agg_stream** out) {
  if (!ctx || !spec || !out) return GQ_ERR_INVALID;
  *out = nullptr;
  if (spec->mode < GQ_MODE_SINGLE || spec->mode > GQ_MODE_FINAL)
    return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_create: unknown mode");
  if (spec->nkeys < 0 || spec->nkeys > GQ_MAX_KEYS || (spec->nkeys > 0 && !spec->keys))
    return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_create: bad key list");
  if (spec->naggs < 0 || spec->naggs > GQ_MAX_AGGS || (spec->naggs > 0 && !spec->aggs))
    return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_create: bad aggregate list");
  if (spec->emit_groups < 0) return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_create: emit_groups < 0");
  const int64_t maxg = spec->nkeys == 0 ? 1 : spec->max_groups;
  if (maxg < 1) return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_create: max_groups must be positive");
  const float lf = spec->load_factor > 0.f ? spec->load_factor : 0.5f;
  if (!(lf > 0.f && lf <= 0.9f)) return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_create: load factor outside (0, 0.9]");
  gq_agg_stream* s = new (std::nothrow) gq_agg_stream;
  if (!s) return GQ_ERR_NOMEM;
  s->ctx = ctx;
  s->mode = spec->mode;
  s->nkeys = spec->nkeys;
  s->naggs = spec->naggs;
  for (int j = 0; j < spec->nkeys; ++j) {
    s->keys[j] = spec->keys[j];
    s->key_nullable[j] = spec->key_nullable ? (spec->key_nullable[j] != 0) : 0;
  }
  for (int i = 0; i < spec->naggs; ++i) s->aggs[i] = spec->aggs[i];
  if (spec->mode == GQ_MODE_INTERMEDIATE || spec->mode == GQ_MODE_FINAL) {
    int rc = merge_aggs(ctx, spec->aggs, spec->naggs, GQ_MAX_COLS, s->aggs);
    if (rc) {
      delete s;
      return rc;
    }
  }
  s->max_groups = maxg;
  s->emit_groups = spec->emit_groups;
  uint64_t cap = (uint64_t)((double)maxg / lf) + 1;
  if (cap < 16) cap = 16;
  s->cap = cap;
  s->strategy = maxg <= 256 ? GQ_STRATEGY_LDS : GQ_STRATEGY_GLOBAL;
  // Accumulators: at most one count word plus two words per aggregate.
  const size_t nslot = (size_t)cap + 2;
  const size_t off_acc = align_up(nslot * 8, 256);
  const size_t off_st = align_up(off_acc + nslot * 8 * (size_t)(1 + 2 * spec->naggs), 256);
  s->bytes = off_st + ST_WORDS * 8;
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  s->mem = ctx_alloc(ctx, s->bytes, stream);
  if (!s->mem) {
    delete s;
    return set_error(ctx, GQ_ERR_NOMEM, "gq_agg_stream_create: table allocation failed");
  }
  char* base = static_cast<char*>(s->mem);
  s->keys_tab = reinterpret_cast<uint64_t*>(base);
  s->acc = reinterpret_cast<uint64_t*>(base + off_acc);
  s->st = reinterpret_cast<int64_t*>(base + off_st);
  int rc = launch_fill_u32(ctx, s->st, 0u, 2 * ST_WORDS, stream);
  if (rc) {
    gq_agg_stream_free(s, stream);
    return rc;
  }
  *out = s;
  return GQ_OK;
}

int gq_agg_stream_push(gq_agg_stream* s, const gq_batch* in, const gq_pred* preds, int npreds, gq_batch* out,
                       int64_t* d_emitted, hipStream_t stream) {
  if (!s) return GQ_ERR_INVALID;
  gq_ctx* ctx = s->ctx;
  int rc = check_batch(ctx, in, "gq_agg_stream_push input");
  if (rc) return rc;
  const bool merge = s->mode == GQ_MODE_INTERMEDIATE || s->mode == GQ_MODE_FINAL;
  if (merge && npreds != 0)
    return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_push: the intermediate and final modes take no predicates");
  const bool can_emit = (s->mode == GQ_MODE_PARTIAL || s->mode == GQ_MODE_INTERMEDIATE) && s->emit_groups > 0;
  if (can_emit && (!out || !d_emitted))
    return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_push: a stream that emits early needs an output");
  GbArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = in->nrows;
  a.dev_status = ctx->d_status;
  rc = make_preds(ctx, a, in, preds, npreds);
  if (rc) return rc;
  rc = make_key_plan(ctx, a.kp, in, s->keys, s->nkeys, s->key_nullable);
  if (rc) return rc;
  rc = make_agg_plan(ctx, a.ap, in, s->aggs, s->naggs, true);
  if (rc) return rc;
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  if (!s->have_layout) {
    s->words.nacc = a.ap.nacc;
    for (int w = 0; w < a.ap.nacc; ++w) s->words.ident[w] = word_identity(a.ap.wop[w]);
    for (int j = 0; j < s->nkeys; ++j) s->key_types[j] = in->cols[s->keys[j]].type;
    s->kp = a.kp;
    s->ap = a.ap;
    s->have_layout = true;
    rc = as_reset(ctx, s, nullptr, stream);
    if (rc) return rc;
  } else {
    bool same = a.ap.nacc == s->words.nacc && a.kp.mode == s->kp.mode;
    for (int j = 0; j < s->nkeys; ++j)
      same &= in->cols[s->keys[j]].type == s->key_types[j] && a.kp.shift[j] == s->kp.shift[j];
    if (!same) return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_push: key column types differ from the first batch");
  }
  a.keys = s->keys_tab;
  a.acc = s->acc;
  a.cap = s->cap;
  a.nrep = 1;
  a.rep_slots = (int64_t)s->cap + 2;
  a.d_inserted = &s->st[ST_INSERTED];
  rc = aggregate_into(ctx, a, s->strategy, stream);
  if (rc) return rc;
  GQ_LAUNCH(ctx, "as_after", k_as_after, dim3(1), dim3(1), 0, stream, s->st, (const uint64_t*)s->acc, s->cap,
            s->words.nacc, s->nkeys, s->emit_groups, can_emit ? 1 : 0, d_emitted);
  GQ_LAUNCH_CHECK(ctx);
  if (!can_emit) return GQ_OK;
  rc = as_compact(ctx, s, out, d_emitted, &s->st[ST_EMIT], stream);
  if (rc) return rc;
  return as_reset(ctx, s, &s->st[ST_EMIT], stream);
}

int gq_agg_stream_finish(gq_agg_stream* s, gq_batch* out, int64_t* d_groups, hipStream_t stream) {
  if (!s) return GQ_ERR_INVALID;
  gq_ctx* ctx = s->ctx;
  if (!d_groups) return set_error(ctx, GQ_ERR_INVALID, "gq_agg_stream_finish: NULL group count");
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  if (!s->have_layout) {
    // Nothing was ever pushed: nothing to emit.
    return launch_fill_u32(ctx, d_groups, 0u, 4, stream);
  }
  GQ_LAUNCH(ctx, "as_fin", k_as_fin, dim3(1), dim3(1), 0, stream, s->st, d_groups);
  GQ_LAUNCH_CHECK(ctx);
  int rc = as_compact(ctx, s, out, d_groups, &s->st[ST_FIN], stream);
  if (rc) return rc;
  return as_reset(ctx, s, &s->st[ST_FIN], stream);
}

int gq_agg_stream_free(gq_agg_stream* s, hipStream_t stream) {
  if (!s) return GQ_OK;
  if (s->mem) ctx_free(s->ctx, s->mem, s->bytes, stream);
  delete s;
  return GQ_OK;
}

}  // extern "C"
