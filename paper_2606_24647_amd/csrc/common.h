// Shared device and host helpers of libgq (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/gq.h"

namespace gq {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
}  // namespace gq

struct gq_ctx {
  int device = 0;
  gq_allocator alloc{};
  bool default_alloc = true;
  int32_t* d_status = nullptr;
  std::string err;
  // Per-kernel event timing (gq_ctx_set_timing).
  struct TimingRec {
    const char* name;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::string timing_only;   // non-empty: time only launches of this name
  std::vector<TimingRec> recs;
  std::vector<hipEvent_t> pool;
};

namespace gq {

int set_error(gq_ctx* ctx, int code, const std::string& msg);
int hip_error(gq_ctx* ctx, hipError_t e, const char* what);
void* ctx_alloc(gq_ctx* ctx, size_t bytes, hipStream_t s);
void ctx_free(gq_ctx* ctx, void* p, size_t bytes, hipStream_t s);

#define GQ_HIP_CHECK(ctx, expr)                                    \
  do {                                                             \
    hipError_t e_ = (expr);                                        \
    if (e_ != hipSuccess) return ::gq::hip_error((ctx), e_, #expr); \
  } while (0)

// Per-kernel timing: when enabled on the context, every launch is bracketed by
// two events recorded on its stream.
int timing_begin(gq_ctx* ctx, hipStream_t s, const char* name);
void timing_end(gq_ctx* ctx, hipStream_t s, int idx);

#define GQ_LAUNCH(ctx, name, kern, grid, block, shm, stream, ...)          \
  do {                                                                     \
    const int ti_ = ::gq::timing_begin((ctx), (stream), (name));           \
    hipLaunchKernelGGL(kern, grid, block, shm, stream, __VA_ARGS__);       \
    ::gq::timing_end((ctx), (stream), ti_);                                \
  } while (0)

// Launch check: kernel launches report errors through hipGetLastError.
#define GQ_LAUNCH_CHECK(ctx)                                                    \
  do {                                                                          \
    hipError_t e_ = hipGetLastError();                                          \
    if (e_ != hipSuccess) return ::gq::hip_error((ctx), e_, "kernel launch");   \
  } while (0)

// Stream-ordered scratch memory released when the owning call returns (the
// release is ordered after the work the call enqueued on the same stream).
struct Scratch {
  gq_ctx* ctx;
  hipStream_t s;
  void* p = nullptr;
  size_t bytes = 0;
  Scratch(gq_ctx* c, hipStream_t st) : ctx(c), s(st) {}
  bool get(size_t n) {
    bytes = n < 256 ? 256 : n;
    p = ctx_alloc(ctx, bytes, s);
    return p != nullptr;
  }
  ~Scratch() {
    if (p) ctx_free(ctx, p, bytes, s);
  }
  template <class T>
  T* as(size_t byte_offset = 0) const {
    return reinterpret_cast<T*>(static_cast<char*>(p) + byte_offset);
  }
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Column descriptors as kernels see them
// ---------------------------------------------------------------------------

// Input column: data points at row 0 of the slice; validity bits start at voff.
struct DCol {
  const uint8_t* data;
  const uint8_t* valid;  // NULL = all valid
  int64_t voff;
  int32_t type;          // GQ_I8..GQ_I64
  int32_t align;         // largest power of two (<= 16) dividing the data address
  int32_t nt;            // read once per kernel: use non-temporal loads
  int32_t pad;
};

// Read-only descriptors in device memory (plans of batched fragments) are read
// through the constant address space: uniform loads from it are scalar loads,
// also after the kernel's own global stores, which would otherwise turn every
// descriptor read into a vector load with a full memory round trip.
#define GQ_CONST_AS __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const GQ_CONST_AS T& cref(const T* p) {
  return *(const GQ_CONST_AS T*)p;
}
// Back to a generic reference, for rarely taken paths.
template <class T>
__device__ __forceinline__ const T& gref(const GQ_CONST_AS T& r) {
  return *(const T*)&r;
}

// Output column.
struct OCol {
  uint8_t* data;
  uint32_t* valid;  // 32-bit words of the output bitmap, NULL = not written
  int32_t type;
  int32_t pad;
};

struct DPred {
  int32_t col;
  int32_t op;
  int64_t lo;
  int64_t hi;
};

__host__ __device__ inline int type_width(int t) { return 1 << (t - 1); }

inline int addr_align(const void* p) {
  uintptr_t a = reinterpret_cast<uintptr_t>(p);
  int al = 16;
  while (al > 1 && (a % al) != 0) al >>= 1;
  return al;
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Tile handled by block b of an nblocks grid such that every XCD works
// through one contiguous range of tiles: workgroups are dispatched to the 8
// XCDs round-robin (block b runs on XCD b % 8), so XCD x takes tiles
// [x * per + min(x, rem), ...) in order.  Neighbouring tiles then run on the
// same XCD at about the same time and their partial output lines meet in
// that XCD's L2.  A bijection on [0, nblocks).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nblocks) {
  const int64_t x = b % kXcds, i = b / kXcds;
  const int64_t per = nblocks / kXcds, rem = nblocks % kXcds;
  return x * per + (x < rem ? x : rem) + i;
}

template <class C>
__device__ __forceinline__ int64_t load_one(const C& c, int64_t i) {
  switch (c.type) {
    case GQ_I8: return (int64_t)((const int8_t*)c.data)[i];
    case GQ_I16: return (int64_t)((const int16_t*)c.data)[i];
    case GQ_I32: return (int64_t)((const int32_t*)c.data)[i];
    default: return ((const int64_t*)c.data)[i];
  }
}

template <class C>
__device__ __forceinline__ bool valid_one(const C& c, int64_t i) {
  if (c.valid == nullptr) return true;
  int64_t b = c.voff + i;
  return (c.valid[b >> 3] >> (b & 7)) & 1;
}

// 16-, 8- and 4-byte loads; NT = non-temporal (streamed once: hint the caches
// not to keep the line, so hash tables stay resident).
typedef int gq_v4i __attribute__((ext_vector_type(4)));
typedef int gq_v2i __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ gq_v4i ld16(const uint8_t* p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const gq_v4i*>(p));
  else return *reinterpret_cast<const gq_v4i*>(p);
}
template <bool NT>
__device__ __forceinline__ gq_v2i ld8(const uint8_t* p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const gq_v2i*>(p));
  else return *reinterpret_cast<const gq_v2i*>(p);
}
template <bool NT>
__device__ __forceinline__ int ld4(const uint8_t* p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const int*>(p));
  else return *reinterpret_cast<const int*>(p);
}

// Blocked load of ITEMS consecutive rows r0..r0+ITEMS-1 into int64 registers,
// sign-extended.  Uses 128-bit loads (or the widest that covers ITEMS*width
// bytes) when the whole group is in range and the slice is aligned for it;
// rows past n read as 0.
template <int ITEMS, bool NT = false, class C = DCol>
__device__ __forceinline__ void load_items(const C& c, int64_t r0, int64_t n, int64_t (&v)[ITEMS]) {
  const int w = type_width(c.type);
  const int need = ITEMS * w < 16 ? ITEMS * w : 16;
  if (r0 + ITEMS <= n && c.align >= need) {
    const uint8_t* p = c.data + r0 * w;
    switch (c.type) {
      case GQ_I64: {
        if constexpr (ITEMS % 2 == 0) {
#pragma unroll
          for (int k = 0; k < ITEMS; k += 2) {
            gq_v4i x = ld16<NT>(p + k * 8);
            v[k] = (int64_t)(((uint64_t)(uint32_t)x.y << 32) | (uint32_t)x.x);
            v[k + 1] = (int64_t)(((uint64_t)(uint32_t)x.w << 32) | (uint32_t)x.z);
          }
          return;
        }
        break;
      }
      case GQ_I32: {
        if constexpr (ITEMS % 4 == 0) {
#pragma unroll
          for (int k = 0; k < ITEMS; k += 4) {
            gq_v4i x = ld16<NT>(p + k * 4);
            v[k] = x.x; v[k + 1] = x.y; v[k + 2] = x.z; v[k + 3] = x.w;
          }
          return;
        } else if constexpr (ITEMS == 2) {
          gq_v2i x = ld8<NT>(p);
          v[0] = x.x; v[1] = x.y;
          return;
        }
        break;
      }
      case GQ_I16: {
        if constexpr (ITEMS % 8 == 0) {
#pragma unroll
          for (int k = 0; k < ITEMS; k += 8) {
            gq_v4i x = ld16<NT>(p + k * 2);
            int32_t q[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              v[k + 2 * j] = (int16_t)(q[j] & 0xffff);
              v[k + 2 * j + 1] = (int16_t)((uint32_t)q[j] >> 16);
            }
          }
          return;
        } else if constexpr (ITEMS == 4) {
          gq_v2i x = ld8<NT>(p);
          v[0] = (int16_t)(x.x & 0xffff); v[1] = (int16_t)((uint32_t)x.x >> 16);
          v[2] = (int16_t)(x.y & 0xffff); v[3] = (int16_t)((uint32_t)x.y >> 16);
          return;
        } else if constexpr (ITEMS == 2) {
          int32_t x = ld4<NT>(p);
          v[0] = (int16_t)(x & 0xffff); v[1] = (int16_t)((uint32_t)x >> 16);
          return;
        }
        break;
      }
      default: {  // GQ_I8
        if constexpr (ITEMS % 16 == 0) {
#pragma unroll
          for (int k = 0; k < ITEMS; k += 16) {
            gq_v4i x = ld16<NT>(p + k);
            int32_t q[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int j = 0; j < 16; ++j) v[k + j] = (int8_t)((uint32_t)q[j >> 2] >> (8 * (j & 3)));
          }
          return;
        } else if constexpr (ITEMS == 8) {
          gq_v2i x = ld8<NT>(p);
#pragma unroll
          for (int j = 0; j < 8; ++j)
            v[j] = (int8_t)((uint32_t)(j < 4 ? x.x : x.y) >> (8 * (j & 3)));
          return;
        } else if constexpr (ITEMS == 4) {
          int32_t x = ld4<NT>(p);
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (int8_t)((uint32_t)x >> (8 * j));
          return;
        }
        break;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) v[k] = (r0 + k < n) ? load_one(c, r0 + k) : 0;
}

// Validity bits of rows r0..r0+ITEMS-1 as a bit mask (bit k = row r0+k).
template <int ITEMS, class C>
__device__ __forceinline__ uint32_t valid_items(const C& c, int64_t r0, int64_t n) {
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (r0 + k < n && valid_one(c, r0 + k)) m |= 1u << k;
  return m;
}

template <class P>
__device__ __forceinline__ bool pred_pass(const P& p, int64_t v) {
  return p.op == GQ_RANGE ? (v >= p.lo && v <= p.hi) : (v != p.lo);
}

// Copy rows [sbase, sbase + nrows) of column c (nrows * width bytes) into LDS
// at dst with 16-byte global-to-LDS loads issued by the whole block: no
// register round trip, so every load of the block is in flight at once.
// Slices that are not 16-byte aligned, and the bytes after the last whole
// 16-byte chunk, are copied byte by byte.  dst is 16-byte aligned.  Returns
// without waiting: the caller waits (s_waitcnt) and synchronises the block.
template <int BLOCK, class C>
__device__ __forceinline__ void stage_col_lds(const C& c, int64_t sbase, int nrows, uint8_t* dst) {
  const int w = type_width(c.type);
  const uint8_t* src = c.data + sbase * w;
  const int nb = nrows * w;
  const int wave = threadIdx.x / 64, lane = threadIdx.x & 63;
  int done = 0;
  if (c.align >= 16) {
    const int nfull = nb >> 4;
    for (int ch0 = wave * 64; ch0 < nfull; ch0 += BLOCK) {
      if (ch0 + lane < nfull)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void*)(src + (size_t)(ch0 + lane) * 16),
            (__attribute__((address_space(3))) void*)(dst + (size_t)ch0 * 16), 16, 0, 2 /* non-temporal */);
    }
    done = nfull << 4;
  }
  for (int b = done + threadIdx.x; b < nb; b += BLOCK) dst[b] = src[b];
}

// Value of row r of a column staged in LDS.
__device__ __forceinline__ int64_t lds_value(const uint8_t* base, int r, int type) {
  switch (type) {
    case GQ_I8: return (int64_t)reinterpret_cast<const int8_t*>(base)[r];
    case GQ_I16: return (int64_t)reinterpret_cast<const int16_t*>(base)[r];
    case GQ_I32: return (int64_t)reinterpret_cast<const int32_t*>(base)[r];
    default: return reinterpret_cast<const int64_t*>(base)[r];
  }
}

// MurmurHash3 64-bit finaliser.
__host__ __device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// Compile-time loop: f(std::integral_constant<int, K>) for K = B..E-1, so that
// register arrays indexed by K stay in registers.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// A copy of a register value that the optimiser cannot see through.  Used on
// hash-table words read ahead for several rows: without it the compiler may
// merge the "first probe" value and the "next probe" load into one load
// through a pointer chosen at run time, which moves the read-ahead array to
// scratch memory.  Applied where the value is consumed, after all read-ahead
// loads were issued, so they still overlap.
__device__ __forceinline__ uint64_t opaque_copy(uint64_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits for every global load and store the wave has in flight (its release
// fence); this one waits for LDS operations (lgkmcnt 0) and leaves global
// loads in flight across the barrier, so loads issued before a phase that
// only works in LDS overlap it.  The signal fences keep the compiler from
// moving memory operations across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0); vmcnt and expcnt unconstrained
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Lane helpers (wave64).
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive prefix over the wave of small per-lane counts c (0 <= c < 2^BITS),
// from one ballot per bit.  Returns the lane's prefix; *total gets the wave sum.
template <int BITS>
__device__ __forceinline__ uint32_t wave_prefix_small(uint32_t c, uint32_t* total) {
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    uint64_t m = ballot((c >> b) & 1u);
    pre += rank_in(m) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  *total = tot;
  return pre;
}

// ---------------------------------------------------------------------------
// Single-pass device-wide exclusive prefix by decoupled look-back
// (Merrill and Garland, "Single-pass Parallel Prefix Scan with Decoupled
// Look-back", NVIDIA TR 2016).  One 64-bit status word per tile: the top two
// bits say "nothing yet" (0), "tile aggregate" (1) or "inclusive prefix" (2),
// the low 62 bits hold the value.  Flag and value travel in one atomic word,
// so relaxed device-scope atomics suffice (no other data is published).
// Tiles are numbered in the order blocks start (a global ticket), so a tile
// only ever waits for tiles whose blocks are already running.
// ---------------------------------------------------------------------------
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPre = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of one wave.  Returns the exclusive prefix of `tile`.
__device__ inline int64_t lookback_exclusive(uint64_t* status, int64_t tile, int64_t agg) {
  const int lane = lane_id();
  if (tile == 0) {
    if (lane == 0) status_store(&status[0], kFlagPre | (uint64_t)agg);
    return 0;
  }
  if (lane == 0) status_store(&status[tile], kFlagAgg | (uint64_t)agg);
  int64_t excl = 0;
  int64_t hi = tile - 1;
  while (true) {
    const int64_t idx = hi - lane;
    uint64_t s = kFlagPre;  // before tile 0: an inclusive prefix of 0
    if (idx >= 0) {
      s = status_load(&status[idx]);
      while ((s >> 62) == 0) {
        __builtin_amdgcn_s_sleep(1);
        s = status_load(&status[idx]);
      }
    }
    const uint64_t pre = ballot((s >> 62) == 2);
    const int first = pre ? (__ffsll((unsigned long long)pre) - 1) : 64;
    int64_t v = lane <= first ? (int64_t)(s & kValMask) : 0;
    excl += wave_sum(v);
    if (pre) break;
    hi -= 64;
  }
  if (lane == 0) status_store(&status[tile], kFlagPre | (uint64_t)(excl + agg));
  return excl;
}

// ---------------------------------------------------------------------------
// LDS staging of output rows
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stage_put(uint8_t* stage, int pos, int64_t v, int type) {
  switch (type) {
    case GQ_I8: stage[pos] = (uint8_t)v; break;
    case GQ_I16: reinterpret_cast<int16_t*>(stage)[pos] = (int16_t)v; break;
    case GQ_I32: reinterpret_cast<int32_t*>(stage)[pos] = (int32_t)v; break;
    default: reinterpret_cast<int64_t*>(stage)[pos] = v; break;
  }
}

__device__ __forceinline__ void copy_out(const uint8_t* stage, int i, uint8_t* out, int64_t g, int type) {
  switch (type) {
    case GQ_I8: out[g] = stage[i]; break;
    case GQ_I16: reinterpret_cast<int16_t*>(out)[g] = reinterpret_cast<const int16_t*>(stage)[i]; break;
    case GQ_I32: reinterpret_cast<int32_t*>(out)[g] = reinterpret_cast<const int32_t*>(stage)[i]; break;
    default: reinterpret_cast<int64_t*>(out)[g] = reinterpret_cast<const int64_t*>(stage)[i]; break;
  }
}

// Write the validity bits of output rows [g0, g0 + cnt) (clipped to cap) from
// one byte per row in LDS.  Whole 32-bit words are stored; words shared with a
// neighbouring tile are updated with an atomic AND (clear own bits) and OR.
template <int BLOCK>
__device__ void write_valid_bits(uint32_t* words, const uint8_t* vbytes, int64_t g0, int cnt, int64_t cap) {
  int64_t g1 = g0 + cnt;
  if (g1 > cap) g1 = cap;
  if (g1 <= g0) return;
  const int64_t w0 = g0 >> 5, w1 = (g1 - 1) >> 5;
  for (int64_t w = w0 + threadIdx.x; w <= w1; w += BLOCK) {
    uint32_t bits = 0, mask = 0;
    for (int b = 0; b < 32; ++b) {
      int64_t pos = w * 32 + b;
      if (pos >= g0 && pos < g1) {
        mask |= 1u << b;
        bits |= (uint32_t)(vbytes[pos - g0] & 1) << b;
      }
    }
    if (mask == 0xffffffffu) {
      words[w] = bits;
    } else {
      atomicAnd(&words[w], ~mask);
      atomicOr(&words[w], bits);
    }
  }
}

// Fill kernel (graph-capture safe replacement for hipMemsetAsync).
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n);

int launch_fill_u32(gq_ctx* ctx, void* p, uint32_t v, int64_t nwords, hipStream_t s);

// Device address of gq_filter_noalloc's fixed workspace on ctx's (current)
// device, looked up once per device (filter.hip).
int filter_scratch_init(gq_ctx* ctx);

// Host-side validation helpers.
int check_batch(gq_ctx* ctx, const gq_batch* b, const char* what);
DCol make_dcol(const gq_column& c);

}  // namespace gq
