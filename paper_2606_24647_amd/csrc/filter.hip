// gq_filter: conjunctive predicate + stable stream compaction of the projected
// columns and their validity, in one pass over the input.
//
// Per tile of BLOCK * ITEMS rows (thread t owns ITEMS consecutive rows, loaded
// with 128-bit loads): predicates give a keep mask in registers; ranks come from
// one wave ballot per bit of the per-thread count plus a block scan of the wave
// totals; the tile's output offset comes from a decoupled look-back over tiles
// in ticket order.  Kept values are staged in LDS in output order and written
// out with consecutive lanes writing consecutive rows.
#include "common.h"

#include <mutex>

namespace gq {
namespace {

struct FilterArgs {
  int64_t n;
  int64_t ntiles;
  int64_t out_cap;
  int32_t npreds;
  int32_t nproj;
  DPred preds[GQ_MAX_PREDS];
  DCol cols[GQ_MAX_COLS];  // projected input columns, in output order
  DCol pcols[GQ_MAX_PREDS];  // predicate columns
  OCol out[GQ_MAX_COLS];
  uint32_t* ticket;
  uint64_t* status;
  int64_t* d_count;
  int32_t* dev_status;
};

__global__ void k_filter_init(uint32_t* ticket, uint64_t* status, int64_t ntiles, int64_t* d_count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i == 0) {
    *ticket = 0;
    *d_count = 0;
  }
  for (; i < ntiles; i += stride) status[i] = 0;
}

template <int ITEMS>
struct CountBits {
  static constexpr int value = ITEMS < 2 ? 1 : ITEMS < 4 ? 2 : ITEMS < 8 ? 3 : ITEMS < 16 ? 4 : ITEMS < 32 ? 5 : 6;
};

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_filter(const FilterArgs a) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_wave[NW];
  __shared__ int64_t s_excl;
  __shared__ __attribute__((aligned(16))) uint8_t s_stage[TILE * 8];
  __shared__ uint8_t s_vbyte[TILE];

  if (threadIdx.x == 0) s_tile = atomicAdd(a.ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t r0 = tile * TILE + (int64_t)threadIdx.x * ITEMS;

  uint32_t keep = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (r0 + k < a.n) keep |= 1u << k;
  for (int p = 0; p < a.npreds; ++p) {
    const DCol& c = a.pcols[p];
    int64_t v[ITEMS];
    load_items<ITEMS>(c, r0, a.n, v);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (!pred_pass(a.preds[p], v[k])) keep &= ~(1u << k);
    if (c.valid) keep &= valid_items<ITEMS>(c, r0, a.n);
  }

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  uint32_t wtot;
  const uint32_t wpre = wave_prefix_small<CountBits<ITEMS>::value>((uint32_t)__popc(keep), &wtot);
  if (lane == 0) s_wave[wave] = wtot;
  __syncthreads();
  uint32_t bpre = 0, btot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if (i < wave) bpre += s_wave[i];
    btot += s_wave[i];
  }
  const int local = (int)(bpre + wpre);

  if (wave == 0) {
    int64_t e = lookback_exclusive(a.status, tile, (int64_t)btot);
    if (lane == 0) s_excl = e;
  }
  __syncthreads();
  const int64_t goff = s_excl;
  if (tile == a.ntiles - 1 && threadIdx.x == 0) {
    const int64_t total = goff + btot;
    *a.d_count = total;
    if (total > a.out_cap) atomicOr(a.dev_status, GQ_DEV_CAPACITY);
  }
  if (btot == 0) return;

  for (int j = 0; j < a.nproj; ++j) {
    const DCol& c = a.cols[j];
    if (keep) {
      int64_t v[ITEMS];
      load_items<ITEMS>(c, r0, a.n, v);
      uint32_t vm = c.valid ? valid_items<ITEMS>(c, r0, a.n) : 0xffffffffu;
      int pos = local;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if ((keep >> k) & 1u) {
          stage_put(s_stage, pos, v[k], c.type);
          s_vbyte[pos] = (uint8_t)((vm >> k) & 1u);
          ++pos;
        }
      }
    }
    __syncthreads();
    const OCol& o = a.out[j];
    for (int i = threadIdx.x; i < (int)btot; i += BLOCK) {
      const int64_t g = goff + i;
      if (g < a.out_cap) copy_out(s_stage, i, o.data, g, c.type);
    }
    if (o.valid) write_valid_bits<BLOCK>(o.valid, s_vbyte, goff, (int)btot, a.out_cap);
    __syncthreads();
  }
}

constexpr int kFilterBlock = 256;
constexpr int kFilterItems = 16;
constexpr int64_t kFilterTile = (int64_t)kFilterBlock * kFilterItems;

// Workspace of gq_filter_noalloc: the ticket word (first 256 bytes) and the
// look-back status words of up to kScratchTiles tiles, in a file-scope device
// array: each device holds its own copy for the life of the process.  Host
// code never passes the array's name to a kernel (on the host it stands for a
// host-side shadow, not the device address); it passes the address that
// hipGetSymbolAddress returned for the device.
constexpr int64_t kScratchTiles = 65536;
constexpr size_t kScratchBytes = 256 + (size_t)kScratchTiles * 8;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

// Filter of `in` with the given workspace (256 + ntiles * 8 bytes), or one
// allocated through the context allocator when ws is NULL.
int filter_run(gq_ctx* ctx, const gq_batch* in, const gq_pred* preds, int npreds, const int32_t* proj, int nproj,
               gq_batch* out, int64_t* d_count, hipStream_t stream, void* ws_fixed) {
  if (!ctx) return GQ_ERR_INVALID;
  int rc = check_batch(ctx, in, "gq_filter input");
  if (rc) return rc;
  if (npreds < 0 || npreds > GQ_MAX_PREDS || (npreds > 0 && !preds))
    return set_error(ctx, GQ_ERR_INVALID, "gq_filter: bad predicate list");
  if (nproj < 0 || nproj > GQ_MAX_COLS || (nproj > 0 && (!proj || !out)))
    return set_error(ctx, GQ_ERR_INVALID, "gq_filter: bad projection list");
  if (!d_count) return set_error(ctx, GQ_ERR_INVALID, "gq_filter: NULL count");
  if (nproj > 0 && (!out->cols || out->ncols < nproj))
    return set_error(ctx, GQ_ERR_INVALID, "gq_filter: output has fewer columns than the projection");

  FilterArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = in->nrows;
  a.npreds = npreds;
  a.nproj = nproj;
  a.out_cap = INT64_MAX;
  for (int p = 0; p < npreds; ++p) {
    if (preds[p].col < 0 || preds[p].col >= in->ncols)
      return set_error(ctx, GQ_ERR_INVALID, "gq_filter: predicate column out of range");
    if (preds[p].op != GQ_RANGE && preds[p].op != GQ_NE)
      return set_error(ctx, GQ_ERR_INVALID, "gq_filter: unknown predicate op");
    a.preds[p] = DPred{preds[p].col, preds[p].op, preds[p].lo, preds[p].hi};
    a.pcols[p] = make_dcol(in->cols[preds[p].col]);
  }
  for (int j = 0; j < nproj; ++j) {
    if (proj[j] < 0 || proj[j] >= in->ncols)
      return set_error(ctx, GQ_ERR_INVALID, "gq_filter: projection column out of range");
    const gq_column& ic = in->cols[proj[j]];
    const gq_column& oc = out->cols[j];
    if (oc.type != ic.type) return set_error(ctx, GQ_ERR_INVALID, "gq_filter: output type mismatch");
    if (oc.length < 0 || (oc.length > 0 && !oc.data))
      return set_error(ctx, GQ_ERR_INVALID, "gq_filter: bad output column");
    if (ic.validity && !oc.validity)
      return set_error(ctx, GQ_ERR_INVALID, "gq_filter: nullable input needs an output bitmap");
    if (oc.validity && (reinterpret_cast<uintptr_t>(oc.validity) & 3))
      return set_error(ctx, GQ_ERR_INVALID, "gq_filter: output bitmap must be 4-byte aligned");
    if (oc.offset != 0) return set_error(ctx, GQ_ERR_INVALID, "gq_filter: output offset must be 0");
    a.cols[j] = make_dcol(ic);
    a.out[j] = OCol{static_cast<uint8_t*>(oc.data), reinterpret_cast<uint32_t*>(oc.validity), oc.type, 0};
    if (oc.length < a.out_cap) a.out_cap = oc.length;
  }

  const int64_t ntiles = (a.n + kFilterTile - 1) / kFilterTile;
  a.ntiles = ntiles;
  GQ_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  Scratch ws(ctx, stream);
  char* wbase = static_cast<char*>(ws_fixed);
  if (!wbase) {
    if (!ws.get(256 + align_up((size_t)(ntiles > 0 ? ntiles : 1) * 8, 256)))
      return set_error(ctx, GQ_ERR_NOMEM, "gq_filter: workspace allocation failed");
    wbase = ws.as<char>(0);
  }
  a.ticket = reinterpret_cast<uint32_t*>(wbase);
  a.status = reinterpret_cast<uint64_t*>(wbase + 256);
  a.d_count = d_count;
  a.dev_status = ctx->d_status;

  int64_t iblocks = (ntiles + 255) / 256;
  if (iblocks < 1) iblocks = 1;
  if (iblocks > 4096) iblocks = 4096;
  GQ_LAUNCH(ctx, "filter_init", k_filter_init, dim3((unsigned)iblocks), dim3(256), 0, stream, a.ticket, a.status,
                     ntiles, d_count);
  GQ_LAUNCH_CHECK(ctx);
  if (ntiles > 0) {
    GQ_LAUNCH(ctx, "filter", (k_filter<kFilterBlock, kFilterItems>), dim3((unsigned)ntiles), dim3(kFilterBlock), 0,
                       stream, a);
    GQ_LAUNCH_CHECK(ctx);
  }
  return GQ_OK;
}

}  // namespace

// Looks up the device address of `scratch` on `device` (current), once per
// device; called by gq_ctx_create.
int filter_scratch_init(gq_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_error(ctx, GQ_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[ctx->device]) return GQ_OK;
  void* p = nullptr;
  GQ_HIP_CHECK(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return set_error(ctx, GQ_ERR_HIP, "hipGetSymbolAddress returned no address for the filter scratch");
  g_scratch_ptr[ctx->device] = p;
  return GQ_OK;
}

}  // namespace gq

using namespace gq;

extern "C" int gq_filter(gq_ctx* ctx, const gq_batch* in, const gq_pred* preds, int npreds,
                         const int32_t* proj, int nproj, gq_batch* out, int64_t* d_count,
                         hipStream_t stream) {
  return filter_run(ctx, in, preds, npreds, proj, nproj, out, d_count, stream, nullptr);
}

extern "C" int gq_filter_noalloc(gq_ctx* ctx, const gq_batch* in, const gq_pred* preds, int npreds,
                                 const int32_t* proj, int nproj, gq_batch* out, int64_t* d_count,
                                 hipStream_t stream) {
  if (!ctx) return GQ_ERR_INVALID;
  if (!in) return set_error(ctx, GQ_ERR_INVALID, "gq_filter_noalloc: NULL input");
  if (in->nrows > kScratchTiles * kFilterTile)
    return set_error(ctx, GQ_ERR_INVALID,
                     "gq_filter_noalloc: more than 268,435,456 rows (the fixed workspace's limit); use gq_filter");
  void* ws = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch_ptr[ctx->device] : nullptr;
  if (!ws) return set_error(ctx, GQ_ERR_HIP, "gq_filter_noalloc: the device's scratch address was not looked up");
  return filter_run(ctx, in, preds, npreds, proj, nproj, out, d_count, stream, ws);
}
