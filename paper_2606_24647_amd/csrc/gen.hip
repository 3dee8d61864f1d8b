// libgqgen: device twin of the seeded input generator (paper_2606_24647_amd/datagen.py).
//
// Input generation only; no operator arithmetic.  Every value is a pure
// function of (seed, column id, row), computed with the same integer formulas
// as the host generator, so any chunk can be checked against it bit for bit:
//   mix     SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014)
//   stream  s_c = mix(seed ^ c*GAMMA), r(row) = mix(s_c + (row+1)*GAMMA)
//   uniform lo + mulhi64(r, hi-lo+1)
//   zipf     k = 1 + #{j : T[j] <= r >> 1}, T the host's table of 63-bit
//            thresholds of the distribution function (P(k) ~ k^-0.5)
//   permutation  4-round Feistel over an even bit width, cycle walking
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ uint64_t mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ uint64_t draw(uint64_t s, int64_t row) { return mix(s + (uint64_t)(row + 1) * kGamma); }

template <class T>
__global__ void k_uniform(T* out, int64_t n, uint64_t s, int64_t start, int64_t lo, uint64_t range) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += step) {
    const uint64_t r = draw(s, start + i);
    out[i] = (T)(lo + (int64_t)__umul64hi(r, range));
  }
}

// Zipf keys by inversion: the number of thresholds at or below the 63-bit
// draw (binary search over the nthr ascending thresholds), plus one.
__global__ void k_zipf(int64_t* out, int64_t n, uint64_t s, int64_t start, const uint64_t* thr, int64_t nthr) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += step) {
    const uint64_t r = draw(s, start + i) >> 1;
    int64_t lo = 0, hi = nthr;  // first index with thr[index] > r
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (thr[mid] <= r) lo = mid + 1;
      else hi = mid;
    }
    out[i] = lo + 1;
  }
}

struct FeistelKeys {
  uint64_t k[4];
};

__device__ __forceinline__ uint64_t feistel(uint64_t x, int half, FeistelKeys fk) {
  const uint64_t mask = (1ull << half) - 1;
  uint64_t l = x >> half, r = x & mask;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t f = mix(r ^ fk.k[i]) & mask;
    const uint64_t nl = r;
    r = l ^ f;
    l = nl;
  }
  return (l << half) | r;
}

__global__ void k_permutation(int64_t* out, int64_t n, int64_t start, int64_t N, int half, FeistelKeys fk,
                              int64_t add) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n; i += step) {
    uint64_t y = feistel((uint64_t)(start + i), half, fk);
    while (y >= (uint64_t)N) y = feistel(y, half, fk);  // cycle walking ends: the orbit returns below N
    out[i] = (int64_t)y + add;
  }
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

uint64_t stream_seed(uint64_t seed, uint64_t col) { return mix(seed ^ (col * kGamma)); }

}  // namespace

extern "C" {

// Uniform integers on [lo, hi] for rows start..start+n-1 of column `col`;
// width = 1, 2, 4 or 8 bytes.  Returns 0, or -1 on bad arguments / launch error.
int gqgen_uniform(void* out, int width, int64_t n, uint64_t seed, uint64_t col, int64_t start, int64_t lo,
                  int64_t hi, hipStream_t stream) {
  if (n < 0 || hi < lo || (uint64_t)(hi - lo) >= (1ull << 32)) return -1;
  if (n == 0) return 0;
  const uint64_t s = stream_seed(seed, col);
  const uint64_t range = (uint64_t)(hi - lo) + 1;
  switch (width) {
    case 1: hipLaunchKernelGGL(k_uniform<int8_t>, dim3(grid_for(n)), dim3(256), 0, stream, (int8_t*)out, n, s, start, lo, range); break;
    case 2: hipLaunchKernelGGL(k_uniform<int16_t>, dim3(grid_for(n)), dim3(256), 0, stream, (int16_t*)out, n, s, start, lo, range); break;
    case 4: hipLaunchKernelGGL(k_uniform<int32_t>, dim3(grid_for(n)), dim3(256), 0, stream, (int32_t*)out, n, s, start, lo, range); break;
    case 8: hipLaunchKernelGGL(k_uniform<int64_t>, dim3(grid_for(n)), dim3(256), 0, stream, (int64_t*)out, n, s, start, lo, range); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Zipf keys on 1..N (int64); thr: the N - 1 thresholds (device memory).
int gqgen_zipf(int64_t* out, int64_t n, uint64_t seed, uint64_t col, int64_t start, int64_t N, const uint64_t* thr,
               hipStream_t stream) {
  if (n < 0 || N < 1 || (N > 1 && !thr)) return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_zipf, dim3(grid_for(n)), dim3(256), 0, stream, out, n, stream_seed(seed, col), start, thr,
                     N - 1);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// pi(row) + add for rows start..start+n-1 of the seeded permutation of 0..N-1.
int gqgen_permutation(int64_t* out, int64_t n, uint64_t seed, uint64_t col, int64_t start, int64_t N, int64_t add,
                      hipStream_t stream) {
  if (n < 0 || N < 1 || start < 0 || start + n > N) return -1;
  if (n == 0) return 0;
  int b = 2;
  while ((1ll << b) < N) ++b;
  b += b & 1;
  FeistelKeys fk;
  const uint64_t sc = stream_seed(seed, col);
  for (int r = 0; r < 4; ++r) fk.k[r] = mix(sc ^ ((uint64_t)(r + 1) * kGamma));
  hipLaunchKernelGGL(k_permutation, dim3(grid_for(n)), dim3(256), 0, stream, out, n, start, N, b / 2, fk, add);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
