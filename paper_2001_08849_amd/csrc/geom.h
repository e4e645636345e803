// Device helpers shared by the assembly kernels of the face- and
// edge-based smoothing domains (not part of the ABI).
#pragma once
#include "common.h"

namespace sfem {

struct Vec3 {
  double x, y, z;
};
__device__ __forceinline__ Vec3 sub(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Vec3 cross(Vec3 a, Vec3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ Vec3 load3(const double* __restrict__ xyz, int n) {
  const double* p = xyz + 3 * int64_t(n);
  return {p[0], p[1], p[2]};
}

// Gradients of the barycentric shape functions of tet (P0, P1, P2, P3) and
// its volume (Eq. 10, orientation-free).
__device__ __forceinline__ void tet_grads(Vec3 P0, Vec3 P1, Vec3 P2, Vec3 P3, Vec3 g[4],
                                          double& vol) {
  Vec3 e1 = sub(P1, P0), e2 = sub(P2, P0), e3 = sub(P3, P0);
  Vec3 c23 = cross(e2, e3), c31 = cross(e3, e1), c12 = cross(e1, e2);
  double det = dot(e1, c23);
  double inv = 1.0 / det;
  g[1] = {c23.x * inv, c23.y * inv, c23.z * inv};
  g[2] = {c31.x * inv, c31.y * inv, c31.z * inv};
  g[3] = {c12.x * inv, c12.y * inv, c12.z * inv};
  g[0] = {-(g[1].x + g[2].x + g[3].x), -(g[1].y + g[2].y + g[3].y), -(g[1].z + g[2].z + g[3].z)};
  vol = fabs(det) * (1.0 / 6.0);
}

// Fixed-point accumulation (see the face assembly): contributions in units
// of a power-of-two u are accumulated onto kShift by FMAs, which round them
// to integers held in the low mantissa bits.
constexpr double kShift = 0x1.8p52;

// Integer value of t - kShift for t in [2^52, 2^53) (two's complement).
__device__ __forceinline__ unsigned long long unshift(double t) {
  return static_cast<unsigned long long>(__double_as_longlong(t)) - 0x4338000000000000ull;
}

// Largest index i in [0, n) with a[i] <= v (a ascending, a[0] <= v).
__device__ __forceinline__ int upper_index(const int32_t* a, int n, int v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace sfem
