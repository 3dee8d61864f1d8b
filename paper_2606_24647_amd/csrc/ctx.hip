// Context, allocator, device status word and shared host helpers of libgq.
#include "common.h"

#include <algorithm>
#include <cstdio>
#include <map>

namespace gq {

int set_error(gq_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_error(gq_ctx* ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_error(ctx, e == hipErrorOutOfMemory ? GQ_ERR_NOMEM : GQ_ERR_HIP, m);
}

void* ctx_alloc(gq_ctx* ctx, size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  if (!ctx->default_alloc) return ctx->alloc.alloc(bytes, s, ctx->alloc.user);
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void ctx_free(gq_ctx* ctx, void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (bytes == 0) bytes = 256;
  if (!ctx->default_alloc) {
    ctx->alloc.free(p, bytes, s, ctx->alloc.user);
    return;
  }
  (void)hipFreeAsync(p, s);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

int launch_fill_u32(gq_ctx* ctx, void* p, uint32_t v, int64_t nwords, hipStream_t s) {
  if (nwords <= 0) return GQ_OK;
  int64_t blocks = (nwords + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  GQ_LAUNCH(ctx, "fill_u32", k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, v, nwords);
  GQ_LAUNCH_CHECK(ctx);
  return GQ_OK;
}

int check_batch(gq_ctx* ctx, const gq_batch* b, const char* what) {
  if (!b) return set_error(ctx, GQ_ERR_INVALID, std::string(what) + ": NULL batch");
  if (b->nrows < 0 || b->nrows > INT32_MAX)
    return set_error(ctx, GQ_ERR_INVALID, std::string(what) + ": row count outside [0, 2^31-1]");
  if (b->ncols < 0 || b->ncols > GQ_MAX_COLS)
    return set_error(ctx, GQ_ERR_INVALID, std::string(what) + ": column count outside [0, 16]");
  if (b->ncols > 0 && !b->cols) return set_error(ctx, GQ_ERR_INVALID, std::string(what) + ": NULL columns");
  for (int i = 0; i < b->ncols; ++i) {
    const gq_column& c = b->cols[i];
    if (c.type < GQ_I8 || c.type > GQ_I64)
      return set_error(ctx, GQ_ERR_INVALID, std::string(what) + ": bad column type");
    if (c.offset < 0) return set_error(ctx, GQ_ERR_INVALID, std::string(what) + ": negative offset");
    if (b->nrows > 0 && !c.data) return set_error(ctx, GQ_ERR_INVALID, std::string(what) + ": NULL data");
  }
  return GQ_OK;
}

int timing_begin(gq_ctx* ctx, hipStream_t s, const char* name) {
  if (!ctx || !ctx->timing) return -1;
  if (!ctx->timing_only.empty() && ctx->timing_only != name) return -1;
  hipEvent_t ev[2];
  for (int i = 0; i < 2; ++i) {
    if (!ctx->pool.empty()) {
      ev[i] = ctx->pool.back();
      ctx->pool.pop_back();
    } else if (hipEventCreate(&ev[i]) != hipSuccess) {
      return -1;
    }
  }
  if (hipEventRecord(ev[0], s) != hipSuccess) return -1;
  ctx->recs.push_back(gq_ctx::TimingRec{name, ev[0], ev[1]});
  return (int)ctx->recs.size() - 1;
}

void timing_end(gq_ctx* ctx, hipStream_t s, int idx) {
  if (!ctx || idx < 0 || idx >= (int)ctx->recs.size()) return;
  (void)hipEventRecord(ctx->recs[idx].b, s);
}

DCol make_dcol(const gq_column& c) {
  DCol d;
  const int w = type_width(c.type);
  d.data = static_cast<const uint8_t*>(c.data) + c.offset * w;
  d.valid = c.validity;
  d.voff = c.offset;
  d.type = c.type;
  d.align = addr_align(d.data);
  d.nt = 0;
  d.pad = 0;
  return d;
}

}  // namespace gq

using namespace gq;

extern "C" {

int gq_ctx_create(int device, const gq_allocator* alloc, gq_ctx** out) {
  if (!out) return GQ_ERR_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return GQ_ERR_INVALID;
  if (alloc && (!alloc->alloc || !alloc->free)) return GQ_ERR_INVALID;
  gq_ctx* ctx = new (std::nothrow) gq_ctx;
  if (!ctx) return GQ_ERR_NOMEM;
  ctx->device = device;
  if (alloc) {
    ctx->alloc = *alloc;
    ctx->default_alloc = false;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return GQ_ERR_HIP;
  }
  if (!alloc) {
    // Keep up to 8 GiB of freed blocks in the device's default pool, so that
    // repeated stream-ordered allocations cost no driver call; larger amounts
    // go back to the device at the next synchronisation, where other
    // allocators (the caller's) can use them.
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      uint64_t threshold = 8ull << 30;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
  }
  if (hipMalloc(&ctx->d_status, 256) != hipSuccess) {
    delete ctx;
    return GQ_ERR_NOMEM;
  }
  if (hipMemset(ctx->d_status, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(ctx->d_status);
    delete ctx;
    return GQ_ERR_HIP;
  }
  // Set-up of gq_filter_noalloc's fixed workspace on this device.
  const int src = filter_scratch_init(ctx);
  if (src != GQ_OK) {
    (void)hipFree(ctx->d_status);
    delete ctx;
    return src;
  }
  *out = ctx;
  return GQ_OK;
}

int gq_ctx_destroy(gq_ctx* ctx) {
  if (!ctx) return GQ_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(ctx->d_status);
  for (auto& r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
  return GQ_OK;
}

const char* gq_last_error(gq_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int32_t* gq_ctx_status_ptr(gq_ctx* ctx) { return ctx ? ctx->d_status : nullptr; }

int gq_ctx_sync_status(gq_ctx* ctx, hipStream_t stream, int32_t* bits) {
  if (!ctx) return GQ_ERR_INVALID;
  int32_t h = 0;
  GQ_HIP_CHECK(ctx, hipMemcpyAsync(&h, ctx->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  GQ_HIP_CHECK(ctx, hipStreamSynchronize(stream));
  if (h != 0) {
    const int32_t zero = 0;
    GQ_HIP_CHECK(ctx, hipMemcpyAsync(ctx->d_status, &zero, sizeof(int32_t), hipMemcpyHostToDevice, stream));
    GQ_HIP_CHECK(ctx, hipStreamSynchronize(stream));
  }
  if (bits) *bits = h;
  if (h & GQ_DEV_CAPACITY) return set_error(ctx, GQ_ERR_CAPACITY, "output capacity exceeded");
  if (h & GQ_DEV_TABLE_FULL) return set_error(ctx, GQ_ERR_TABLE_FULL, "hash table full");
  return GQ_OK;
}

int gq_ctx_set_timing(gq_ctx* ctx, int enable) {
  if (!ctx) return GQ_ERR_INVALID;
  ctx->timing = enable != 0;
  return GQ_OK;
}

int gq_ctx_set_timing_only(gq_ctx* ctx, const char* name) {
  if (!ctx) return GQ_ERR_INVALID;
  ctx->timing_only = name ? name : "";
  return GQ_OK;
}

int gq_ctx_timing_report(gq_ctx* ctx, char* names, int name_len, double* total_ms, int64_t* launches, int cap) {
  if (!ctx || cap < 0 || (cap > 0 && (!names || !total_ms || !launches || name_len < 2))) return GQ_ERR_INVALID;
  std::map<std::string, std::pair<double, int64_t>> acc;
  int rc = GQ_OK;
  for (auto& r : ctx->recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      rc = set_error(ctx, GQ_ERR_HIP, "gq_ctx_timing_report: event query failed");
      ms = 0.f;
    }
    auto& e = acc[r.name];
    e.first += ms;
    e.second += 1;
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->recs.clear();
  if (rc != GQ_OK) return rc;
  std::vector<std::pair<std::string, std::pair<double, int64_t>>> v(acc.begin(), acc.end());
  std::sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.second.first > y.second.first; });
  const int n = (int)v.size() < cap ? (int)v.size() : cap;
  for (int i = 0; i < n; ++i) {
    std::snprintf(names + (size_t)i * name_len, (size_t)name_len, "%s", v[i].first.c_str());
    total_ms[i] = v[i].second.first;
    launches[i] = v[i].second.second;
  }
  return (int)v.size();
}

}  // extern "C"
