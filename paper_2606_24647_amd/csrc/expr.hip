// Expression programs (gq_compute_column, gq_filter_expr, gq_groupby_expr)
// and ORDER BY / top-k (gq_order_by).
//
// An expression program is evaluated for every row by one kernel (k_expr):
// each thread takes a row and keeps the program's intermediate values in its
// own column of an LDS array (value i of row r at s_v[i][r]: consecutive
// threads touch consecutive words, so there are no bank conflicts and no
// barriers), the instruction stream being uniform across the wave.  The
// filter and group-by forms evaluate their expressions into int64 columns
// and run the filter and group-by kernels over the input extended by them.
//
// ORDER BY is a stable LSD radix sort of (sort word, row id) pairs, one key at
// a time from the last to the first: a key's value pass orders by the value
// biased to unsigned (complemented for DESC), over the key's width in bytes,
// and a nullable key's flag pass then orders NULLs first or last; stability
// keeps the order of the passes before.  Each pass uses the partition
// kernels with the digit of the sort word in place of the hash.
#include "agg.h"

namespace gq {
namespace {

constexpr int kExBlock = 256;

struct ExInstr {
  int32_t op, a, b, c;
  int64_t k;
};

struct ExprArgs {
  int64_t n;
  int32_t ninstr;
  int32_t pad;
  DCol cols[GQ_MAX_COLS];
  ExInstr ins[GQ_MAX_EXPR];
  int64_t* out;
  uint32_t* out_valid;  // may be NULL
};

// One row per thread per step; rows of a wave are 64 consecutive rows starting
// at a multiple of 64, so the wave writes whole validity words.
__global__ __launch_bounds__(kExBlock) void k_expr(const ExprArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t s_raw[];
  int64_t* s_v = reinterpret_cast<int64_t*>(s_raw);
  uint8_t* s_ok = s_raw + (size_t)a.ninstr * kExBlock * 8;
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int64_t step = (int64_t)gridDim.x * kExBlock;
  for (int64_t base = (int64_t)blockIdx.x * kExBlock; base < a.n; base += step) {
    const int64_t r = base + t;
    const bool in = r < a.n;
    for (int i = 0; i < a.ninstr; ++i) {
      const ExInstr& q = a.ins[i];
      int64_t v = 0;
      bool ok = true;
      switch (q.op) {
        case GQ_E_COL: {
          const DCol& c = a.cols[q.a];
          v = in ? load_one(c, r) : 0;
          ok = in ? valid_one(c, r) : false;
          break;
        }
        case GQ_E_CONST:
          v = q.k;
          break;
        case GQ_E_NEG: {
          v = (int64_t)(0ull - (uint64_t)s_v[q.a * kExBlock + t]);
          ok = s_ok[q.a * kExBlock + t];
          break;
        }
        case GQ_E_CASE: {
          const bool take = s_ok[q.a * kExBlock + t] && s_v[q.a * kExBlock + t] != 0;
          const int src = take ? q.b : q.c;
          v = s_v[src * kExBlock + t];
          ok = s_ok[src * kExBlock + t];
          break;
        }
        default: {
          const int64_t x = s_v[q.a * kExBlock + t], y = s_v[q.b * kExBlock + t];
          ok = s_ok[q.a * kExBlock + t] && s_ok[q.b * kExBlock + t];
          const uint64_t ux = (uint64_t)x, uy = (uint64_t)y;
          switch (q.op) {
            case GQ_E_ADD: v = (int64_t)(ux + uy); break;
            case GQ_E_SUB: v = (int64_t)(ux - uy); break;
            case GQ_E_MUL: v = (int64_t)(ux * uy); break;
            case GQ_E_LT: v = x < y; break;
            case GQ_E_LE: v = x <= y; break;
            case GQ_E_EQ: v = x == y; break;
            case GQ_E_NE: v = x != y; break;
            case GQ_E_GT: v = x > y; break;
            default: v = x >= y; break;
          }
          break;
        }
      }
      s_v[i * kExBlock + t] = v;
      s_ok[i * kExBlock + t] = ok ? 1 : 0;
    }
    const int last = a.ninstr - 1;
    const bool ok = in && s_ok[last * kExBlock + t];
    if (in) a.out[r] = ok ? s_v[last * kExBlock + t] : 0;
    if (a.out_valid) {
      const uint64_t m = ballot(ok);
      const int64_t w = (base + (t - lane)) >> 5;  // first of the wave's two words
      if (lane == 0 && (w << 5) < a.n) a.out_valid[w] = (uint32_t)m;
      if (lane == 32 && ((w + 1) << 5) < a.n) a.out_valid[w + 1] = (uint32_t)(m >> 32);
    }
  }
}

int check_expr(gq_ctx* ctx, const gq_batch* in, const gq_expr* e, ExprArgs& a) {
  if (!e || e->ninstr < 1 || e->ninstr > GQ_MAX_EXPR || !e->instr)
    return set_error(ctx, GQ_ERR_INVALID, "expression: 1..32 instructions");
  a.ninstr = e->ninstr;
  for (int i = 0; i < e->ninstr; ++i) {
    const gq_expr_instr& q = e->instr[i];
    a.ins[i] = ExInstr{q.op, q.a, q.b, q.c, q.k};
    switch (q.op) {
      case GQ_E_COL:
        if (q.a < 0 || q.a >= in->ncols) return set_error(ctx, GQ_ERR_INVALID, "expression: column out of range");
        break;
      case GQ_E_CONST:
        break;
      case GQ_E_NEG:
        if (q.a < 0 || q.a >= i) return set_error(ctx, GQ_ERR_INVALID, "expression: operand must precede its use");
        break;
      case GQ_E_CASE:
        if (q.a < 0 || q.a >= i || q.b < 0 || q.b >= i || q.c < 0 || q.c >= i)
          return set_error(ctx, GQ_ERR_INVALID, "expression: operand must precede its use");
        break;
      default:
        if (q.op < GQ_E_ADD || q.op > GQ_E_GE) return set_error(ctx, GQ_ERR_INVALID, "expression: unknown op");
        if (q.a < 0 || q.a >= i || q.b < 0 || q.b >= i)
          return set_error(ctx, GQ_ERR_INVALID, "expression: operand must precede its use");
        break;
    }
  }
  for (int j = 0; j < in->ncols && j < GQ_MAX_COLS; ++j) a.cols[j] = make_dcol(in->cols[j]);
  return GQ_OK;
}

int launch_expr(gq_ctx* ctx, const gq_batch* in, const gq_expr* e, int64_t* out, uint32_t* out_valid,
                hipStream_t stream) {
  ExprArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = in->nrows;
  int rc = check_expr(ctx, in, e, a);
  if (rc) return rc;
  a.out = out;
  a.out_valid = out_valid;
  if (a.n == 0) return GQ_OK;
  int64_t blocks = (a.n + kExBlock - 1) / kExBlock;
  if (blocks > 8192) blocks = 8192;
  const size_t lds = (size_t)a.ninstr * kExBlock * 9;
  GQ_LAUNCH(ctx, "expr", k_expr, dim3((unsigned)blocks), dim3(kExBlock), lds, stream, a);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

// The input extended by nexprs computed int64 columns (with bitmaps) in a
// workspace; cols must hold in->ncols + nexprs entries.
int extend_with_exprs(gq_ctx* ctx, const gq_batch* in, const gq_expr* exprs, int nexprs, Scratch& ws,
                      gq_column* cols, gq_batch* ext, hipStream_t stream) {
  if (nexprs < 0 || (nexprs > 0 && !exprs)) return set_error(ctx, GQ_ERR_INVALID, "expression: bad list");
  if (in->ncols + nexprs > GQ_MAX_COLS)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "expression: more than 16 input and computed columns");
  const int64_t n = in->nrows;
  const size_t vbytes = align_up((size_t)((n + 63) / 64) * 8 + 8, 256);
  const size_t per = align_up((size_t)(n > 0 ? n : 1) * 8, 256) + vbytes;
  if (nexprs > 0 && !ws.get(per * (size_t)nexprs)) return set_error(ctx, GQ_ERR_NOMEM, "expression: workspace allocation failed");
  for (int j = 0; j < in->ncols; ++j) cols[j] = in->cols[j];
  for (int e = 0; e < nexprs; ++e) {
    gq_column& c = cols[in->ncols + e];
    std::memset(&c, 0, sizeof(c));
    c.type = GQ_I64;
    c.length = n;
    c.data = ws.as<void>(per * e);
    c.validity = ws.as<uint8_t>(per * e + align_up((size_t)(n > 0 ? n : 1) * 8, 256));
    int rc = launch_expr(ctx, in, &exprs[e], static_cast<int64_t*>(c.data), reinterpret_cast<uint32_t*>(c.validity),
                         stream);
    if (rc) return rc;
  }
  *ext = gq_batch{n, in->ncols + nexprs, 0, cols};
  return GQ_OK;
}

// ---------------------------------------------------------------------------
// ORDER BY
// ---------------------------------------------------------------------------
struct ObWordArgs {
  int64_t n;
  DCol key;
  const int32_t* rows_in;  // row id of each position (NULL: identity)
  uint64_t* word;          // sort word of each position
  int32_t* rows_out;       // identity row ids written here when rows_in is NULL
  int32_t flag_pass;       // 0: value pass, 1: NULL-flag pass
  int32_t desc;
  int32_t nulls_first;
  int32_t bits;            // value width in bits
};

__global__ void k_ob_word(const ObWordArgs a) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const uint64_t mask = a.bits >= 64 ? ~0ull : ((1ull << a.bits) - 1);
  for (int64_t i = i0; i < a.n; i += step) {
    const int64_t r = a.rows_in ? a.rows_in[i] : i;
    if (!a.rows_in) a.rows_out[i] = (int32_t)i;
    const bool ok = valid_one(a.key, r);
    uint64_t w;
    if (a.flag_pass) {
      w = ok ? (a.nulls_first ? 1u : 0u) : (a.nulls_first ? 0u : 1u);
    } else {
      const int64_t v = ok ? load_one(a.key, r) : 0;
      w = ((uint64_t)v + (1ull << (a.bits - 1))) & mask;  // order-preserving bias to unsigned
      if (a.desc) w = mask - w;
    }
    a.word[i] = w;
  }
}

__global__ void k_ob_take(const int32_t* rows, int64_t n, int32_t* out) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) out[i] = rows[i];
}

}  // namespace
}  // namespace gq

using namespace gq;

extern "C" {

int gq_compute_column(gq_ctx* ctx, const gq_batch* in, const gq_expr* expr, gq_column* out, hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_compute_column input");
  if (rc) return rc;
  if (!out || out->type != GQ_I64 || out->length < in->nrows || (in->nrows > 0 && !out->data) || out->offset != 0)
    return set_error(ctx, GQ_ERR_INVALID, "gq_compute_column: output must be int64 with capacity >= nrows");
  if (out->validity && (reinterpret_cast<uintptr_t>(out->validity) & 3))
    return set_error(ctx, GQ_ERR_INVALID, "gq_compute_column: output bitmap must be 4-byte aligned");
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  return launch_expr(ctx, in, expr, static_cast<int64_t*>(out->data), reinterpret_cast<uint32_t*>(out->validity),
                     stream);
}

int gq_filter_expr(gq_ctx* ctx, const gq_batch* in, const gq_pred* preds, int npreds, const gq_expr* exprs,
                   int nexprs, const int32_t* proj, int nproj, gq_batch* out, int64_t* d_count, hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_filter_expr input");
  if (rc) return rc;
  if (npreds < 0 || npreds + nexprs > GQ_MAX_PREDS || (npreds > 0 && !preds))
    return set_error(ctx, GQ_ERR_INVALID, "gq_filter_expr: at most 8 predicates and expressions together");
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  Scratch ws(ctx, stream);
  gq_column cols[GQ_MAX_COLS];
  gq_batch ext;
  rc = extend_with_exprs(ctx, in, exprs, nexprs, ws, cols, &ext, stream);
  if (rc) return rc;
  gq_pred p[GQ_MAX_PREDS];
  for (int i = 0; i < npreds; ++i) p[i] = preds[i];
  for (int e = 0; e < nexprs; ++e) p[npreds + e] = gq_pred{in->ncols + e, GQ_NE, 0, 0};
  return gq_filter(ctx, &ext, p, npreds + nexprs, proj, nproj, out, d_count, stream);
}

int gq_groupby_expr(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys, const gq_pred* preds,
                    int npreds, const gq_expr* exprs, int nexprs, const int32_t* agg_ops, const gq_expr* agg_exprs,
                    int naggs, const gq_groupby_opts* opts, gq_batch* out, int64_t* d_groups, hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_groupby_expr input");
  if (rc) return rc;
  if (npreds < 0 || nexprs < 0 || npreds + nexprs > GQ_MAX_PREDS || (npreds > 0 && !preds))
    return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_expr: at most 8 predicates and expressions together");
  if (naggs < 0 || naggs > GQ_MAX_AGGS || (naggs > 0 && (!agg_ops || !agg_exprs)))
    return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_expr: bad aggregate list");
  if (opts && opts->mode != GQ_MODE_SINGLE && opts->mode != GQ_MODE_PARTIAL)
    return set_error(ctx, GQ_ERR_INVALID, "gq_groupby_expr: single or partial mode");
  // Filter expressions first, then one computed column per aggregate input.
  gq_expr all[2 * GQ_MAX_AGGS + GQ_MAX_PREDS];
  int ne = 0;
  for (int e = 0; e < nexprs; ++e) all[ne++] = exprs[e];
  int acol[GQ_MAX_AGGS];
  for (int i = 0; i < naggs; ++i) {
    acol[i] = -1;
    if (agg_ops[i] == GQ_COUNT_STAR) continue;
    acol[i] = in->ncols + ne;
    all[ne++] = agg_exprs[i];
  }
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  Scratch ws(ctx, stream);
  gq_column cols[GQ_MAX_COLS];
  gq_batch ext;
  rc = extend_with_exprs(ctx, in, all, ne, ws, cols, &ext, stream);
  if (rc) return rc;
  gq_pred p[GQ_MAX_PREDS];
  for (int i = 0; i < npreds; ++i) p[i] = preds[i];
  for (int e = 0; e < nexprs; ++e) p[npreds + e] = gq_pred{in->ncols + e, GQ_NE, 0, 0};
  gq_agg aggs[GQ_MAX_AGGS];
  for (int i = 0; i < naggs; ++i) {
    std::memset(&aggs[i], 0, sizeof(gq_agg));
    aggs[i].op = agg_ops[i];
    if (acol[i] >= 0) {
      aggs[i].nfactors = 1;
      aggs[i].f[0] = gq_factor{GQ_F_COL, acol[i], 0};
    }
  }
  return gq_groupby_agg(ctx, &ext, keys, nkeys, p, npreds + nexprs, aggs, naggs, opts, out, d_groups, stream);
}

int gq_order_by(gq_ctx* ctx, const gq_batch* in, const int32_t* keys, int nkeys, const int32_t* desc,
                const int32_t* nulls_first, int64_t limit, int32_t* out_rows, hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_order_by input");
  if (rc) return rc;
  if (nkeys < 1 || nkeys > GQ_MAX_KEYS || !keys) return set_error(ctx, GQ_ERR_INVALID, "gq_order_by: 1..4 key columns");
  for (int j = 0; j < nkeys; ++j)
    if (keys[j] < 0 || keys[j] >= in->ncols) return set_error(ctx, GQ_ERR_INVALID, "gq_order_by: key column out of range");
  const int64_t n = in->nrows;
  if (n >= ((int64_t)1 << 31)) return set_error(ctx, GQ_ERR_INVALID, "gq_order_by: more than 2^31 - 1 rows");
  const int64_t take = limit < 0 || limit > n ? n : limit;
  if (take > 0 && !out_rows) return set_error(ctx, GQ_ERR_INVALID, "gq_order_by: NULL output");
  if (take == 0) return GQ_OK;
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  // Three (word, row id) buffers: the pass's input, output and scratch.
  const size_t wbytes = align_up((size_t)n * 8, 256), rbytes = align_up((size_t)n * 4, 256);
  Scratch ws(ctx, stream);
  if (!ws.get(3 * (wbytes + rbytes))) return set_error(ctx, GQ_ERR_NOMEM, "gq_order_by: workspace allocation failed");
  gq_column cols[3][2];
  gq_batch bt[3];
  std::memset(cols, 0, sizeof(cols));
  for (int b = 0; b < 3; ++b) {
    cols[b][0].type = GQ_I64;
    cols[b][0].length = n;
    cols[b][0].data = ws.as<void>(b * (wbytes + rbytes));
    cols[b][1].type = GQ_I32;
    cols[b][1].length = n;
    cols[b][1].data = ws.as<void>(b * (wbytes + rbytes) + wbytes);
    bt[b] = gq_batch{n, 2, 0, cols[b]};
  }
  int cur = 0;
  bool first = true;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  for (int j = nkeys - 1; j >= 0; --j) {
    const gq_column& kc = in->cols[keys[j]];
    const int npasses = kc.validity ? 2 : 1;
    for (int pass = 0; pass < npasses; ++pass) {
      ObWordArgs w;
      std::memset(&w, 0, sizeof(w));
      w.n = n;
      w.key = make_dcol(kc);
      w.rows_in = first ? nullptr : static_cast<const int32_t*>(cols[cur][1].data);
      w.rows_out = static_cast<int32_t*>(cols[cur][1].data);
      w.word = static_cast<uint64_t*>(cols[cur][0].data);
      w.flag_pass = pass;
      w.desc = desc ? desc[j] != 0 : 0;
      w.nulls_first = nulls_first ? nulls_first[j] != 0 : 0;
      w.bits = 8 * type_width(kc.type);
      first = false;
      GQ_LAUNCH(ctx, "ob_word", k_ob_word, dim3((unsigned)blocks), dim3(256), 0, stream, w);
      GQ_LAUNCH_CHECK(ctx);
      const int nxt = (cur + 1) % 3, tmp = (cur + 2) % 3;
      gq_batch* bufs[2] = {&bt[tmp], &bt[cur]};
      rc = radix_sort_rows(ctx, &bt[cur], bufs, &bt[nxt], pass ? 1 : w.bits, n, nullptr, stream);
      if (rc) return rc;
      cur = nxt;
    }
  }
  GQ_LAUNCH(ctx, "ob_take", k_ob_take, dim3((unsigned)((take + 255) / 256 < 8192 ? (take + 255) / 256 : 8192)),
            dim3(256), 0, stream, static_cast<const int32_t*>(cols[cur][1].data), take, out_rows);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

}  // extern "C"
