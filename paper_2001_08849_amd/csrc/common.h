// Internal helpers shared by the library's HIP sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/sfem.h"

namespace sfem {

constexpr int kWave = 64;

struct Error {
  int code;
  std::string msg;
};

#define SFEM_HIP(x)                                                              \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess)                                                        \
      throw ::sfem::Error{SFEM_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define SFEM_REQUIRE(cond, code, msg)                 \
  do {                                                \
    if (!(cond)) throw ::sfem::Error{(code), (msg)};  \
  } while (0)

// Owning device buffer (hipMalloc / hipFree), grown on demand.
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  // Ensure capacity for `count` elements (contents not preserved on growth).
  T* reserve(size_t count) {
    if (count <= n && p) return p;
    release();
    size_t bytes = (count ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{SFEM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    n = count;
    return p;
  }
  T* get() const { return p; }
};

// Stream-ordered temporary (hipMallocAsync / hipFreeAsync on one stream),
// freed when it goes out of scope, on error paths too; release() frees it
// earlier.
template <typename T>
struct TmpBuf {
  T* p = nullptr;
  hipStream_t s = nullptr;
  TmpBuf(size_t count, hipStream_t stream) : s(stream) {
    const size_t bytes = (count ? count : 1) * sizeof(T);
    if (hipMallocAsync(reinterpret_cast<void**>(&p), bytes, s) != hipSuccess) {
      p = nullptr;
      throw Error{SFEM_ENOMEM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed"};
    }
  }
  TmpBuf(const TmpBuf&) = delete;
  TmpBuf& operator=(const TmpBuf&) = delete;
  ~TmpBuf() { release(); }
  void release() {
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
  }
  T* get() const { return p; }
};

inline int div_up(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// ------------------------------------------------------------ device helpers
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o);
    v = v > w ? v : w;
  }
  return v;
}

// Inclusive scan across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T w = __shfl_up(v, o);
    if (lane >= o) v += w;
  }
  return v;
}

// ------------------------------------------------------------ primitives
// Exclusive scan of n int32 values into out[0..n]; out[n] is the total.
// `in` and `out` may not alias.
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);

// Counting sort of n items by bucket (0 <= bucket < n_buckets), then a sort
// of the values inside each of the first n_sorted buckets (all if < 0;
// values must be distinct within a bucket).  ptr gets n_buckets+1 offsets;
// out the values, bucket by bucket.
void bucket_sort_u64(const int32_t* bucket, const uint64_t* vals, int64_t n, int n_buckets,
                     int32_t* ptr, uint64_t* out, hipStream_t s, int n_sorted = -1);
void bucket_sort_u32(const int32_t* bucket, const uint32_t* vals, int64_t n, int n_buckets,
                     int32_t* ptr, uint32_t* out, hipStream_t s, int n_sorted = -1);

// Sort the values of every segment [ptr[i], ptr[i+1]) of `in` into `out`.
void segmented_sort_u64(const int32_t* ptr, int n_seg, const uint64_t* in, uint64_t* out,
                        hipStream_t s);
void segmented_sort_u32(const int32_t* ptr, int n_seg, const uint32_t* in, uint32_t* out,
                        hipStream_t s);

}  // namespace sfem
