// Device-wide primitives used by the topology build: exclusive scan,
// counting sort into buckets and a per-segment rank sort.  All results are
// deterministic: the only atomics are integer counters, and every segment is
// fully sorted afterwards (values are distinct within a segment).
#include "common.h"

namespace sfem {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the prefix and
// writes the block total to *total.
template <typename T>
__device__ T block_exclusive_scan(T v, T* total) {
  __shared__ T wsum[kScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  T inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) wsum[wid] = inc;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    T s = wsum[w];
    if (w < wid) before += s;
    tot += s;
  }
  *total = tot;
  __syncthreads();
  return before + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const T* in, int64_t n, T* sums) {
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  T acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) acc += in[base + i];
  T tot;
  (void)block_exclusive_scan(acc, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = offs[tile] + exclusive prefix inside the tile (offs == nullptr:
// a single tile, offset 0); the last tile also writes out[n] = grand total.
template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const T* in, int64_t n, const T* offs,
                                                            T* out) {
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  T v[kScanItems];
  T acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : T(0);
    acc += v[i];
  }
  T tot;
  const T off = offs ? offs[blockIdx.x] : T(0);
  T pre = block_exclusive_scan(acc, &tot) + off;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = pre;
    pre += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + tot;
}

template <typename T>
void exclusive_scan_impl(const T* in, T* out, int64_t n, hipStream_t s) {
  if (n <= 0) {
    SFEM_HIP(hipMemsetAsync(out, 0, sizeof(T), s));
    return;
  }
  const int nt = div_up(n, kScanTile);
  if (nt == 1) {  // one tile: no tile offsets to scan (ends the recursion)
    k_tile_scan<T><<<1, kScanThreads, 0, s>>>(in, n, nullptr, out);
    SFEM_HIP(hipGetLastError());
    return;
  }
  TmpBuf<T> sums(nt, s), offs(nt + 1, s);
  k_tile_sums<T><<<nt, kScanThreads, 0, s>>>(in, n, sums.get());
  SFEM_HIP(hipGetLastError());
  exclusive_scan_impl<T>(sums.get(), offs.get(), nt, s);
  k_tile_scan<T><<<nt, kScanThreads, 0, s>>>(in, n, offs.get(), out);
  SFEM_HIP(hipGetLastError());
}

// ------------------------------------------------------------ bucket sort
__global__ void k_count(const int32_t* bucket, int64_t n, int32_t* cnt) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[bucket[i]], 1);
}

template <typename V>
__global__ void k_scatter(const int32_t* bucket, const V* vals, int64_t n, int32_t* cursor,
                          V* out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    int pos = atomicAdd(&cursor[bucket[i]], 1);
    out[pos] = vals[i];
  }
}

// One wave per segment.  rank(v) = #{w in segment : w < v}; values are
// distinct, so ranks are a permutation.  Short segments are staged in LDS.
constexpr int kSegWaves = 4;
constexpr int kSegLds = 512;  // values per wave held in LDS

template <typename V>
__global__ void __launch_bounds__(kSegWaves * kWave)
    k_segsort(const int32_t* ptr, int n_seg, const V* in, V* out) {
  __shared__ V lds[kSegWaves][kSegLds];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int seg = blockIdx.x * kSegWaves + wid;
  int b = 0, m = 0;
  if (seg < n_seg) {
    b = ptr[seg];
    m = ptr[seg + 1] - b;
  }
  const bool staged = m > 1 && m <= kSegLds;
  V* s = lds[wid];
  if (staged)
    for (int i = lane; i < m; i += kWave) s[i] = in[b + i];
  __syncthreads();  // every wave of the block reaches this barrier
  if (m == 1) {
    if (lane == 0) out[b] = in[b];
  } else if (staged) {
    for (int i = lane; i < m; i += kWave) {
      V v = s[i];
      int r = 0;
      for (int j = 0; j < m; ++j) r += (s[j] < v);
      out[b + r] = v;
    }
  } else if (m > 1) {
    for (int i = lane; i < m; i += kWave) {
      V v = in[b + i];
      int r = 0;
      for (int j = 0; j < m; ++j) r += (in[b + j] < v);
      out[b + r] = v;
    }
  }
}

template <typename V>
void segmented_sort_impl(const int32_t* ptr, int n_seg, const V* in, V* out, hipStream_t s) {
  // (segments are sorted independently; callers may pass fewer segments
  // than the buckets they counted to leave trailing buckets unsorted)
  if (n_seg <= 0) return;
  k_segsort<V><<<div_up(n_seg, kSegWaves), kSegWaves * kWave, 0, s>>>(ptr, n_seg, in, out);
  SFEM_HIP(hipGetLastError());
}

template <typename V>
void bucket_sort_impl(const int32_t* bucket, const V* vals, int64_t n, int n_buckets, int32_t* ptr,
                      V* out, hipStream_t s, int n_sorted) {
  TmpBuf<int32_t> cnt(n_buckets + 1, s), cursor(n_buckets + 1, s);
  TmpBuf<V> tmp(n, s);
  SFEM_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int32_t) * (n_buckets + 1), s));
  if (n > 0) {
    k_count<<<div_up(n, 256), 256, 0, s>>>(bucket, n, cnt.get());
    SFEM_HIP(hipGetLastError());
  }
  exclusive_scan_impl<int32_t>(cnt.get(), ptr, n_buckets, s);
  SFEM_HIP(hipMemcpyAsync(cursor.get(), ptr, sizeof(int32_t) * (n_buckets + 1),
                          hipMemcpyDeviceToDevice, s));
  if (n > 0) {
    k_scatter<V><<<div_up(n, 256), 256, 0, s>>>(bucket, vals, n, cursor.get(), tmp.get());
    SFEM_HIP(hipGetLastError());
  }
  segmented_sort_impl<V>(ptr, n_sorted, tmp.get(), out, s);
  if (n_sorted < n_buckets) {  // unsorted trailing buckets: plain copy
    int32_t first = 0;
    SFEM_HIP(hipMemcpyAsync(&first, ptr + n_sorted, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SFEM_HIP(hipStreamSynchronize(s));
    if (n > first)
      SFEM_HIP(hipMemcpyAsync(out + first, tmp.get() + first, sizeof(V) * (n - first),
                              hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  exclusive_scan_impl<int32_t>(in, out, n, s);
}

void bucket_sort_u64(const int32_t* bucket, const uint64_t* vals, int64_t n, int n_buckets,
                     int32_t* ptr, uint64_t* out, hipStream_t s, int n_sorted) {
  bucket_sort_impl<uint64_t>(bucket, vals, n, n_buckets, ptr, out, s,
                             n_sorted < 0 ? n_buckets : n_sorted);
}

void bucket_sort_u32(const int32_t* bucket, const uint32_t* vals, int64_t n, int n_buckets,
                     int32_t* ptr, uint32_t* out, hipStream_t s, int n_sorted) {
  bucket_sort_impl<uint32_t>(bucket, vals, n, n_buckets, ptr, out, s,
                             n_sorted < 0 ? n_buckets : n_sorted);
}

void segmented_sort_u64(const int32_t* ptr, int n_seg, const uint64_t* in, uint64_t* out,
                        hipStream_t s) {
  segmented_sort_impl<uint64_t>(ptr, n_seg, in, out, s);
}

void segmented_sort_u32(const int32_t* ptr, int n_seg, const uint32_t* in, uint32_t* out,
                        hipStream_t s) {
  segmented_sort_impl<uint32_t>(ptr, n_seg, in, out, s);
}

}  // namespace sfem
