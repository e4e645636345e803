// Many meshes and load cases in one solve.
//
// The meshes are concatenated into one mesh with disjoint node ranges, so
// the single-mesh pipeline (face adjacency, pattern, assembly, loads, BCs)
// builds all of them in one pass and K is block diagonal.  Up to four load
// cases per mesh share K: vectors are stored [3N][4] (the four right-hand
// sides of a DOF side by side) and one product reads K once for all four.
//
// CG runs one independent system per (mesh, load case): workgroups own runs
// of node rows inside one mesh and write per-workgroup partial sums per load
// case; a one-thread-per-system kernel adds the partials of its mesh in a
// fixed order (bit-reproducible) and updates that system's scalars.  A
// system leaves the iteration once its FP64 true residual, recomputed every
// `check_every` iterations, meets the tolerance (or stagnates, or breaks
// down).  The iterations of a check period are captured once in a hipGraph
// and replayed until every system has finished.
//
// Autotuner: meshes fall into size buckets; for each bucket the lanes per
// node row and the node rows per workgroup are timed over a candidate set
// (the bucket's own product launch) and the choice is cached per bucket
// shape for the rest of the process.
#include <map>
#include <mutex>
#include <tuple>

#include "handles.h"

namespace sfem {

namespace {

constexpr int kNR = 4;             // right-hand sides per product
constexpr int kBThreads = 256;
constexpr int kNumBuckets = 3;     // mesh sizes: < 8192, < 32768, >= 32768 nodes
constexpr int kNumLpr = 3;
constexpr int kLprs[kNumLpr] = {8, 16, 32};
constexpr int kCU = 4;                       // columns per step in the CSR-order product
constexpr int kNumPLpr = 2;                  // packed layout (FP64 values)
constexpr int kPLprs[kNumPLpr] = {4, 8};
constexpr int kNumRw = 3;
constexpr int kRws[kNumRw] = {16, 64, 256};

struct BScal {
  double rz, pq, alpha, beta, rr, rr_true, ff, tol2, best;
  int active, iters, breakdown, stale;
  int need64, pad;  // stagnated with FP32 products: the batch continues with FP64 ones
};

enum BOp { kBStart = 0, kBAlpha = 1, kBBeta = 2, kBReplace = 3 };

template <int LPR>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Block sum of 8 doubles; thread j < 8 stores sum j at out[j].
__device__ __forceinline__ void block_store8(double (&v)[8], double* out) {
  __shared__ double sm[kBThreads / 64][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = wave_sum(v[j]);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[wid][j] = v[j];
  __syncthreads();
  if (threadIdx.x < 8) {
    double s = 0.0;
    for (int q = 0; q < kBThreads / 64; ++q) s += sm[q][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// True when every system of the workgroup's mesh has finished (then the
// workgroup has nothing to do; a block-uniform test).
__device__ __forceinline__ bool mesh_done(const BScal* __restrict__ sc, int m) {
  if (!sc) return false;
  const BScal* s = sc + m * kNR;
  return !(s[0].active | s[1].active | s[2].active | s[3].active);
}

// The work items a launch walks: with a list, the compacted items
// list[base + i], i < *cnt (those of meshes still active when the list was
// made); without one, the items base + i, i < n.  A workgroup takes items
// blockIdx.x, blockIdx.x + gridDim.x, ...
struct Work {
  const int32_t* __restrict__ list;
  const int32_t* __restrict__ cnt;
  int base, n;
  __device__ __forceinline__ int count() const { return list ? *cnt : n; }
  __device__ __forceinline__ int item(int i) const { return list ? list[base + i] : base + i; }
};

// Product of K with a [3N][4] panel over the node rows [wr[w].x, wr[w].y)
// of each work item w.
//   EPI 0: Y = K X, partials (x.y) per load case.
//   EPI 1: residual replacement Y = F - K X, Z = dinv Y, partials (y.y),
//          (y.z) per load case.
// Partials: part[w][k][2].
// CORR: the translation form's value in the corrected form, Y_I = sum_J
// K32_IJ X_J + C_I X_I with rsum = C = R - R32 (R the FP64 block row sums,
// R32 those of the FP32 values): the FP32 values' rounding then meets
// neighbour differences only (see the single-system product).
// 128 VGPRs at most: 4 waves per SIMD (the 8-lane FP32 form otherwise
// takes 130 and 3 waves).
template <typename VT, int LPR, int EPI, bool CORR = false>
__global__ void __launch_bounds__(kBThreads) __attribute__((amdgpu_waves_per_eu(4)))
    k_bspmm(Work wk, const int2* __restrict__ wr, const int32_t* __restrict__ wmesh,
            const BScal* __restrict__ sc, const int32_t* __restrict__ bptr,
            const int32_t* __restrict__ bcol, const VT* __restrict__ val,
            const double* __restrict__ X, const double* __restrict__ F, double* __restrict__ Y,
            double* __restrict__ Z, const double* __restrict__ dinv, double* __restrict__ part,
            const double* __restrict__ rsum = nullptr) {
  constexpr int G = kBThreads / LPR;
  const int n_items = wk.count();
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int w = wk.item(it);
    if (mesh_done(sc, wmesh[w])) continue;
    const int2 rr = wr[w];
    const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
    double pv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int I0 = rr.x; I0 < rr.y; I0 += G) {
      const int I = I0 + g;
      const bool valid = I < rr.y;
      int rb = 0, deg = 0;
      if (valid) {
        rb = bptr[I];
        deg = bptr[I + 1] - rb;
      }
      const int td = 3 * deg;
      const VT* v = val + 9 * int64_t(rb);
      double acc[3][kNR];
  #pragma unroll
      for (int a = 0; a < 3; ++a)
  #pragma unroll
        for (int k = 0; k < kNR; ++k) acc[a][k] = 0.0;
      // kCU columns per step (masked past the row), so each lane keeps kCU
      // columns' loads in flight
      for (int c0 = sub; c0 < td; c0 += kCU * LPR) {
  #pragma unroll
        for (int h = 0; h < kCU; ++h) {
          const int c = c0 + h * LPR;
          const bool in = c < td;
          const int cc = in ? c : c0;
          const int jj = cc / 3;
          const int comp = cc - 3 * jj;
          const int64_t col = 3 * int64_t(bcol[rb + jj]) + comp;
          const double2 xa = *reinterpret_cast<const double2*>(X + col * kNR);
          const double2 xb = *reinterpret_cast<const double2*>(X + col * kNR + 2);
          const double x4[kNR] = {xa.x, xa.y, xb.x, xb.y};
          const double m = in ? 1.0 : 0.0;
          const double a3[3] = {m * double(v[cc]), m * double(v[td + cc]),
                                m * double(v[2 * td + cc])};
  #pragma unroll
          for (int a = 0; a < 3; ++a)
  #pragma unroll
            for (int k = 0; k < kNR; ++k) acc[a][k] += a3[a] * x4[k];
        }
      }
  #pragma unroll
      for (int a = 0; a < 3; ++a)
  #pragma unroll
        for (int k = 0; k < kNR; ++k) acc[a][k] = gsum<LPR>(acc[a][k]);
      if (valid && sub == 0) {
        if constexpr (CORR) {
          const double* C = rsum + 9 * int64_t(I);
  #pragma unroll
          for (int k = 0; k < kNR; ++k) {
            const double x0 = X[(3 * int64_t(I)) * kNR + k];
            const double x1 = X[(3 * int64_t(I) + 1) * kNR + k];
            const double x2 = X[(3 * int64_t(I) + 2) * kNR + k];
  #pragma unroll
            for (int a = 0; a < 3; ++a) acc[a][k] += C[3 * a] * x0 + C[3 * a + 1] * x1 + C[3 * a + 2] * x2;
          }
        }
  #pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int64_t i = 3 * int64_t(I) + a;
  #pragma unroll
          for (int k = 0; k < kNR; ++k) {
            const int64_t e = i * kNR + k;
            if constexpr (EPI == 0) {
              Y[e] = acc[a][k];
              pv[2 * k] += X[e] * acc[a][k];
            } else {
              const double r = F[e] - acc[a][k];
              const double z = dinv[i] * r;
              Y[e] = r;
              Z[e] = z;
              pv[2 * k] += r * r;
              pv[2 * k + 1] += r * z;
            }
          }
        }
      }
    }
    block_store8(pv, part + int64_t(w) * 8);
    __syncthreads();  // the next item reuses block_store8's shared array
  }
}

// The same product on the packed layout of the single-system row kernels
// (node row I: a [9][d4] array at 9 ptr4[I], d4 = degree rounded up to 4,
// block columns col4 padded with I and zero values).  A lane takes 4 blocks
// per step: one int4 of columns, 18 double2 value loads and, per block, the
// 12 panel entries of its node (6 double2 loads) for 144 FMAs.
template <int LPR, int EPI>
__global__ void __launch_bounds__(kBThreads)
    k_bspmm_p(Work wk, const int2* __restrict__ wr, const int32_t* __restrict__ wmesh,
              const BScal* __restrict__ sc, const int32_t* __restrict__ ptr4,
              const int32_t* __restrict__ col4, const double* __restrict__ valp,
              const double* __restrict__ X, const double* __restrict__ F, double* __restrict__ Y,
              double* __restrict__ Z, const double* __restrict__ dinv, double* __restrict__ part) {
  constexpr int G = kBThreads / LPR;
  const int n_items = wk.count();
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int w = wk.item(it);
    if (mesh_done(sc, wmesh[w])) continue;
    const int2 rr = wr[w];
    const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
    double pv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int I0 = rr.x; I0 < rr.y; I0 += G) {
      const int I = I0 + g;
      const bool valid = I < rr.y;
      int r4 = 0, d4 = 0;
      if (valid) {
        r4 = ptr4[I];
        d4 = ptr4[I + 1] - r4;
      }
      const double* wv = valp + 9 * int64_t(r4);
      double acc[3][kNR];
  #pragma unroll
      for (int a = 0; a < 3; ++a)
  #pragma unroll
        for (int k = 0; k < kNR; ++k) acc[a][k] = 0.0;
      for (int jb = 4 * sub; jb < d4; jb += 4 * LPR) {
        const int4 J = *reinterpret_cast<const int4*>(col4 + r4 + jb);
        double m[9][4];
  #pragma unroll
        for (int q = 0; q < 9; ++q) {
          const double2 lo = *reinterpret_cast<const double2*>(wv + q * d4 + jb);
          const double2 hi = *reinterpret_cast<const double2*>(wv + q * d4 + jb + 2);
          m[q][0] = lo.x;
          m[q][1] = lo.y;
          m[q][2] = hi.x;
          m[q][3] = hi.y;
        }
        const int Js[4] = {J.x, J.y, J.z, J.w};
  #pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double2* xp = reinterpret_cast<const double2*>(X + 12 * int64_t(Js[t]));
          double x[3][kNR];
  #pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            const double2 a = xp[2 * cc], b = xp[2 * cc + 1];
            x[cc][0] = a.x;
            x[cc][1] = a.y;
            x[cc][2] = b.x;
            x[cc][3] = b.y;
          }
  #pragma unroll
          for (int a = 0; a < 3; ++a)
  #pragma unroll
            for (int cc = 0; cc < 3; ++cc)
  #pragma unroll
              for (int k = 0; k < kNR; ++k) acc[a][k] += m[3 * a + cc][t] * x[cc][k];
        }
      }
  #pragma unroll
      for (int a = 0; a < 3; ++a)
  #pragma unroll
        for (int k = 0; k < kNR; ++k) acc[a][k] = gsum<LPR>(acc[a][k]);
      if (valid && sub == 0) {
  #pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int64_t i = 3 * int64_t(I) + a;
  #pragma unroll
          for (int k = 0; k < kNR; ++k) {
            const int64_t e = i * kNR + k;
            if constexpr (EPI == 0) {
              Y[e] = acc[a][k];
              pv[2 * k] += X[e] * acc[a][k];
            } else {
              const double r = F[e] - acc[a][k];
              const double z = dinv[i] * r;
              Y[e] = r;
              Z[e] = z;
              pv[2 * k] += r * r;
              pv[2 * k + 1] += r * z;
            }
          }
        }
      }
    }
    block_store8(pv, part + int64_t(w) * 8);
    __syncthreads();  // the next item reuses block_store8's shared array
  }
}

// p = z + beta p on active systems.
__global__ void __launch_bounds__(kBThreads)
    k_bp(Work wk, const int2* __restrict__ wr, const int32_t* __restrict__ wmesh,
         const BScal* __restrict__ sc, const double* __restrict__ Z, double* __restrict__ P) {
  const int n_items = wk.count();
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int w = wk.item(it);
    if (mesh_done(sc, wmesh[w])) continue;
    const int64_t e0 = int64_t(wr[w].x) * 3 * kNR, e1 = int64_t(wr[w].y) * 3 * kNR;
    const BScal* s = sc + wmesh[w] * kNR;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBThreads) {
      const BScal& q = s[e % kNR];
      if (q.active) P[e] = Z[e] + q.beta * P[e];
    }
  }
}

// x += alpha p; r -= alpha q; z = dinv r on active systems; partials (r.z),
// (r.r) per load case.
__global__ void __launch_bounds__(kBThreads)
    k_bupdate(Work wk, const int2* __restrict__ wr, const int32_t* __restrict__ wmesh,
              const BScal* __restrict__ sc, const double* __restrict__ dinv,
              double* __restrict__ X, double* __restrict__ R, double* __restrict__ Z,
              const double* __restrict__ P, const double* __restrict__ Q,
              double* __restrict__ part) {
  const int n_items = wk.count();
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int w = wk.item(it);
    if (mesh_done(sc, wmesh[w])) continue;
    const int64_t e0 = int64_t(wr[w].x) * 3 * kNR, e1 = int64_t(wr[w].y) * 3 * kNR;
    const BScal* s = sc + wmesh[w] * kNR;
    double pv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBThreads) {
      const int k = int(e % kNR);
      const BScal& q = s[k];
      if (!q.active) continue;
      const double r = R[e] - q.alpha * Q[e];
      const double z = dinv[e / kNR] * r;
      X[e] += q.alpha * P[e];
      R[e] = r;
      Z[e] = z;
      pv[2 * k] += r * z;
      pv[2 * k + 1] += r * r;
    }
    block_store8(pv, part + int64_t(w) * 8);
    __syncthreads();  // the next item reuses block_store8's shared array
  }
}

// Compacted work lists of the meshes still active, one per block j: j <
// kNumBuckets lists the product items of bucket j's active meshes (ranges
// mw), j = kNumBuckets the elementwise items (ranges mv), j = kNumBuckets + 1
// the product items of every active mesh (for one launch over all buckets
// when they share a schedule).  List j starts at list[base.b[j]] and has
// cnt[j] entries.  Meshes in ascending order, so each list is a fixed
// function of the masks.
constexpr int kNumLists = kNumBuckets + 2;
struct ListBase {
  int b[kNumLists];
};

__global__ void __launch_bounds__(kBThreads)
    k_bcompact(int n_meshes, const int32_t* __restrict__ mbucket, const int2* __restrict__ mw,
               const int2* __restrict__ mv, const BScal* __restrict__ sc, ListBase base,
               int32_t* __restrict__ list, int32_t* __restrict__ cnt) {
  const int j = blockIdx.x;
  const int ob = base.b[j];
  __shared__ int wsum[kBThreads / 64];
  __shared__ int off;
  if (threadIdx.x == 0) off = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int m0 = 0; m0 < n_meshes; m0 += kBThreads) {
    const int m = m0 + threadIdx.x;
    int2 rg = {0, 0};
    if (m < n_meshes && !mesh_done(sc, m) && (j >= kNumBuckets || mbucket[m] == j))
      rg = j == kNumBuckets ? mv[m] : mw[m];
    const int len = rg.y - rg.x;
    const int inc = wave_inclusive_scan(len);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int pre = off;
    for (int q = 0; q < wid; ++q) pre += wsum[q];
    const int ex = pre + inc - len;
    for (int t = 0; t < len; ++t) list[ob + ex + t] = rg.x + t;
    __syncthreads();
    if (threadIdx.x == kBThreads - 1) off = ex + len;
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[j] = off;
}

// Start from x = 0: r = f, z = dinv f, p = 0; partials (r.z), (r.r).
__global__ void __launch_bounds__(kBThreads)
    k_bstart(const int2* __restrict__ wr, const double* __restrict__ dinv,
             const double* __restrict__ F, double* __restrict__ X, double* __restrict__ R,
             double* __restrict__ Z, double* __restrict__ P, double* __restrict__ part) {
  const int w = blockIdx.x;
  const int64_t e0 = int64_t(wr[w].x) * 3 * kNR, e1 = int64_t(wr[w].y) * 3 * kNR;
  double pv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kBThreads) {
    const int k = int(e % kNR);
    const double f = F[e];
    const double z = dinv[e / kNR] * f;
    X[e] = 0.0;
    R[e] = f;
    Z[e] = z;
    P[e] = 0.0;
    pv[2 * k] += f * z;
    pv[2 * k + 1] += f * f;
  }
  block_store8(pv, part + int64_t(w) * 8);
}

// One workgroup per mesh: sums the partials of the mesh's workgroups
// [mw[m].x, mw[m].y) (thread t takes workgroups t, t + 256, ... in order,
// then a fixed-shape tree) and updates the scalars of its 4 systems.
// Finished systems are final and left untouched.
__global__ void __launch_bounds__(kBThreads)
    k_bfinal(int op, const int2* __restrict__ mw, const double* __restrict__ part,
             BScal* __restrict__ sc, double rtol2, int max_stale, int f32) {
  const int m = blockIdx.x;
  BScal* sys = sc + m * kNR;
  if (op != kBStart && mesh_done(sc, m)) return;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int w = mw[m].x + threadIdx.x; w < mw[m].y; w += kBThreads)
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] += part[int64_t(w) * 8 + j];
  __shared__ double tot[8];
  block_store8(v, tot);
  __syncthreads();
  if (threadIdx.x >= kNR) return;
  const int k = threadIdx.x;
  const double v0 = tot[2 * k], v1 = tot[2 * k + 1];
  BScal& c = sys[k];
  switch (op) {
    case kBStart:  // v0 = f.dinv f, v1 = f.f
      c.rz = v0;
      c.rr = v1;
      c.rr_true = v1;
      c.ff = v1;
      c.tol2 = rtol2 * v1;
      c.best = v1;
      c.beta = 0.0;
      c.alpha = 0.0;
      c.pq = 0.0;
      c.iters = 0;
      c.breakdown = 0;
      c.stale = 0;
      c.need64 = 0;
      c.active = (v1 > 0.0 && v1 > c.tol2) ? 1 : 0;
      break;
    case kBAlpha:  // v0 = p.K p
      if (!c.active) return;
      c.pq = v0;
      c.alpha = c.rz / v0;
      if (!(v0 > 0.0) || !isfinite(c.alpha)) {
        c.alpha = 0.0;
        c.active = 0;
        c.breakdown = 1;
      }
      break;
    case kBBeta:  // v0 = r.z, v1 = r.r
      if (!c.active) return;
      c.beta = c.rz > 0.0 ? v0 / c.rz : 0.0;
      if (!isfinite(c.beta)) c.beta = 0.0;
      c.rz = v0;
      c.rr = v1;
      c.iters += 1;
      break;
    case kBReplace:  // replaced residual: v0 = r.r, v1 = r.z
      if (!c.active) return;
      c.rr_true = v0;
      c.rr = v0;
      c.rz = v1;
      if (v0 <= c.tol2) {
        c.active = 0;
      } else if (v0 < c.best) {
        c.best = v0;
        c.stale = 0;
      } else if (f32 && c.best <= 1e-6 * c.ff) {
        // past relres 1e-3 with no new minimum for max_stale / 4 checks:
        // FP32 products cannot take this system further (too ill-conditioned
        // for their rounding).  It stays active and the host moves the batch
        // to FP64 products (k_brestart) before the next period.
        if (++c.stale >= max_stale / 4) {
          c.need64 = 1;
          c.stale = 0;
        }
      } else if (c.best <= 1e4 * c.tol2 && ++c.stale >= max_stale) {
        // stagnation counts only near the tolerance: CG residual norms may
        // rise far above their start before they fall
        c.active = 0;
      }
      break;
  }
}

// Column k of a [3N][4] panel (rows [i0, i0 + n)) into a contiguous vector.
__global__ void k_bcolumn(int64_t n, const double* __restrict__ X, int k, double* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = X[i * kNR + k];
}

__global__ void k_bset_column(int64_t n, const double* __restrict__ f, int k,
                              double* __restrict__ F) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) F[i * kNR + k] = f[i];
}

__global__ void k_bzero(int64_t n, double* __restrict__ x) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// Autotuner cache: (bucket, log2 of the bucket's node rows, mean block
// degree) -> (lanes per row, rows per workgroup).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, std::pair<int, int>> g_tune_cache;

int bucket_of(int64_t nodes) { return nodes < 8192 ? 0 : (nodes < 32768 ? 1 : 2); }

}  // namespace

// ------------------------------------------------------------- host state
struct BatchState {
  int n_meshes = 0;
  std::vector<int64_t> node0;        // [n_meshes + 1] first node of each mesh
  std::vector<int> bucket;           // per mesh
  int lpr[kNumBuckets] = {16, 16, 16};
  int rw[kNumBuckets] = {64, 64, 64};
  bool packed[kNumBuckets] = {false, false, false};  // FP64 products on the packed layout
  bool from_cache[kNumBuckets] = {false, false, false};
  // workgroup table, bucket-major (a mesh's workgroups are contiguous)
  std::vector<int2> h_wr;            // node rows [x, y) per workgroup
  std::vector<int32_t> h_wmesh;      // mesh per workgroup
  std::vector<int2> h_mw;            // workgroups [x, y) per mesh
  int bw0[kNumBuckets + 1] = {0, 0, 0, 0};
  DBuf<int2> wr, mw;
  DBuf<int32_t> wmesh;
  // the elementwise kernels' own table (fixed kVRows-row chunks per mesh),
  // so that their workgroup count does not follow the product schedule
  std::vector<int2> h_vr, h_mv;
  std::vector<int32_t> h_vmesh;
  int n_vw = 0;
  DBuf<int2> vr, mv;
  DBuf<int32_t> vmesh;
  // compacted lists of the items of meshes still active (products by bucket
  // at bw0[bk], elementwise at n_wg()), remade at the start of each period
  DBuf<int32_t> mbucket, alist, acnt;
  DBuf<double> F, X, R, Z, P, Q, part;
  DBuf<BScal> sc;
  BScal* sc_host = nullptr;          // two slots of n_sys: period p's flags in slot p % 2
  hipEvent_t flags_ready[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_key[2] = {-1, -1};       // (mode, check_every) of the captured period
  ~BatchState() {
    drop_graph();
    if (sc_host) (void)hipHostFree(sc_host);
    for (hipEvent_t e : flags_ready)
      if (e) (void)hipEventDestroy(e);
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    graph_key[0] = graph_key[1] = -1;
  }
  int n_wg() const { return bw0[kNumBuckets]; }
};

namespace {

// Rows per workgroup of the elementwise kernels (p update, x/r/z update,
// start), 12 values per row: small enough that a lone large mesh still
// spreads over the CUs late in a solve.
constexpr int kVRows = 64;

void build_table(Ctx& c, BatchState& b) {
  b.h_vr.clear();
  b.h_vmesh.clear();
  b.h_mv.assign(b.n_meshes, int2{0, 0});
  int v = 0;
  for (int m = 0; m < b.n_meshes; ++m) {
    const int first = v;
    for (int64_t r = b.node0[m]; r < b.node0[m + 1]; r += kVRows) {
      const int64_t r1 = std::min<int64_t>(r + kVRows, b.node0[m + 1]);
      b.h_vr.push_back(int2{int(r), int(r1)});
      b.h_vmesh.push_back(m);
      ++v;
    }
    b.h_mv[m] = int2{first, v};
  }
  b.n_vw = v;
  b.vr.reserve(std::max(1, v));
  b.vmesh.reserve(std::max(1, v));
  b.mv.reserve(std::max(1, b.n_meshes));
  b.h_wr.clear();
  b.h_wmesh.clear();
  b.h_mw.assign(b.n_meshes, int2{0, 0});
  int w = 0;
  for (int bk = 0; bk < kNumBuckets; ++bk) {
    b.bw0[bk] = w;
    for (int m = 0; m < b.n_meshes; ++m) {
      if (b.bucket[m] != bk) continue;
      const int first = w;
      for (int64_t r = b.node0[m]; r < b.node0[m + 1]; r += b.rw[bk]) {
        const int64_t r1 = std::min<int64_t>(r + b.rw[bk], b.node0[m + 1]);
        b.h_wr.push_back(int2{int(r), int(r1)});
        b.h_wmesh.push_back(m);
        ++w;
      }
      b.h_mw[m] = int2{first, w};
    }
  }
  b.bw0[kNumBuckets] = w;
  b.wr.reserve(std::max(1, w));
  b.wmesh.reserve(std::max(1, w));
  b.mw.reserve(std::max(1, b.n_meshes));
  b.part.reserve(size_t(std::max(std::max(1, w), v)) * 8);  // either table's partials
  b.alist.reserve(size_t(std::max(1, 2 * w + v)));
  b.acnt.reserve(kNumLists);
  b.mbucket.reserve(std::max(1, b.n_meshes));
  SFEM_HIP(hipMemcpyAsync(b.mbucket.get(), b.bucket.data(), sizeof(int32_t) * b.n_meshes,
                          hipMemcpyHostToDevice, c.stream));
  SFEM_HIP(hipMemcpyAsync(b.wr.get(), b.h_wr.data(), sizeof(int2) * w, hipMemcpyHostToDevice,
                          c.stream));
  SFEM_HIP(hipMemcpyAsync(b.wmesh.get(), b.h_wmesh.data(), sizeof(int32_t) * w,
                          hipMemcpyHostToDevice, c.stream));
  SFEM_HIP(hipMemcpyAsync(b.mw.get(), b.h_mw.data(), sizeof(int2) * b.n_meshes,
                          hipMemcpyHostToDevice, c.stream));
  SFEM_HIP(hipMemcpyAsync(b.vr.get(), b.h_vr.data(), sizeof(int2) * v, hipMemcpyHostToDevice,
                          c.stream));
  SFEM_HIP(hipMemcpyAsync(b.vmesh.get(), b.h_vmesh.data(), sizeof(int32_t) * v,
                          hipMemcpyHostToDevice, c.stream));
  SFEM_HIP(hipMemcpyAsync(b.mv.get(), b.h_mv.data(), sizeof(int2) * b.n_meshes,
                          hipMemcpyHostToDevice, c.stream));
  SFEM_HIP(hipStreamSynchronize(c.stream));
  b.drop_graph();
}

// One product of K (FP64 or FP32 values) with a panel, bucket by bucket,
// each with its own lanes-per-row; only_bucket >= 0 restricts to one.
// Workgroups of a list-driven launch, at most: enough to fill the chip while
// every mesh is active, few enough that the late iterations of a solve do
// not pay for dispatching the retired meshes' items.
constexpr int kBGridCap = 4096;

// Remakes the lists of the items of meshes still active (kernel only:
// capturable).
void compact(Ctx& c, BatchState& b) {
  const ListBase base = {{b.bw0[0], b.bw0[1], b.bw0[2], b.n_wg(), b.n_wg() + b.n_vw}};
  k_bcompact<<<kNumLists, kBThreads, 0, c.stream>>>(b.n_meshes, b.mbucket.get(),
                                                         b.mw.get(), b.mv.get(), b.sc.get(), base,
                                                         b.alist.get(), b.acnt.get());
  SFEM_HIP(hipGetLastError());
}

// One product, bucket by bucket.  use_sc: over the compacted lists (made by
// compact() from the current masks; retired meshes skipped); otherwise over
// every item with no masks.
template <int EPI>
void bspmm(Ctx& c, BatchState& b, bool f32, const double* X, const double* F, double* Y,
           double* Z, int only_bucket = -1, bool use_sc = true) {
  // every non-empty bucket on one schedule: one launch over the merged list
  int first = -1;
  bool uniform = true;
  for (int bk = 0; bk < kNumBuckets; ++bk) {
    if (b.bw0[bk + 1] == b.bw0[bk]) continue;
    if (first < 0) first = bk;
    else uniform = uniform && b.lpr[bk] == b.lpr[first] && b.packed[bk] == b.packed[first];
  }
  const bool merged = use_sc && only_bucket < 0 && uniform && first >= 0;
  for (int bk = 0; bk < kNumBuckets; ++bk) {
    if (only_bucket >= 0 && bk != only_bucket) continue;
    if (merged && bk != first) continue;
    const int nw = merged ? b.n_wg() : b.bw0[bk + 1] - b.bw0[bk];
    if (nw == 0) continue;
    const Work wk = merged ? Work{b.alist.get(), b.acnt.get() + kNumBuckets + 1,
                                  b.n_wg() + b.n_vw, nw}
                           : Work{use_sc ? b.alist.get() : nullptr,
                                  use_sc ? b.acnt.get() + bk : nullptr, b.bw0[bk], nw};
    const int grid = use_sc ? std::min(nw, kBGridCap) : nw;
#define L_(VT, VAL, LPR)                                                                   \
  k_bspmm<VT, LPR, EPI><<<grid, kBThreads, 0, c.stream>>>(                                \
      wk, b.wr.get(), b.wmesh.get(), use_sc ? b.sc.get() : nullptr, c.topo.bptr.get(),     \
      c.topo.bcol.get(), VAL, X, F, Y, Z, c.dinv.get(), b.part.get())
  // FP32 values: the corrected form (C made with the assembly)
#define T_(LPR)                                                                             \
  k_bspmm<float, LPR, EPI, true><<<grid, kBThreads, 0, c.stream>>>(                       \
      wk, b.wr.get(), b.wmesh.get(), use_sc ? b.sc.get() : nullptr, c.topo.bptr.get(),     \
      c.topo.bcol.get(), c.val32.get(), X, F, Y, Z, c.dinv.get(), b.part.get(), c.rcorr.get())
#define P_(LPR)                                                                              \
  k_bspmm_p<LPR, EPI><<<grid, kBThreads, 0, c.stream>>>(                                    \
      wk, b.wr.get(), b.wmesh.get(), use_sc ? b.sc.get() : nullptr, c.ptr4.get(),           \
      c.col4.get(), c.valp.get(), X, F, Y, Z, c.dinv.get(), b.part.get())
    if (f32) SFEM_REQUIRE(c.have_rcorr, SFEM_ESTATE, "row sums of the FP32 rounding missing");
    if (f32 && b.packed[bk]) {
      T_(16);  // FP32 values keep the CSR order
    } else if (b.packed[bk]) {
      SFEM_REQUIRE(c.packed64, SFEM_ESTATE, "packed copy of K missing");
      if (b.lpr[bk] == 4) P_(4);
      else P_(8);
    } else if (f32) {
      switch (b.lpr[bk]) {
        case 8: T_(8); break;
        case 16: T_(16); break;
        default: T_(32); break;
      }
    } else {
      switch (b.lpr[bk]) {
        case 8: L_(double, c.val.get(), 8); break;
        case 16: L_(double, c.val.get(), 16); break;
        default: L_(double, c.val.get(), 32); break;
      }
    }
#undef L_
#undef T_
#undef P_
    SFEM_HIP(hipGetLastError());
  }
}

// The partials of kBAlpha / kBReplace come from the product's table, those
// of kBStart / kBBeta from the elementwise one.
// Every active system restarts CG from its x and true residual (beta = 0):
// on the move from FP32 to FP64 products.  Directions made with the FP32
// products and the residual jumps of their replacements have lost the
// conjugacy that continuing them in FP64 would assume (on the most
// ill-conditioned meshes continuing them converged far slower than a
// restart).
__global__ void k_brestart(int n_sys, BScal* __restrict__ sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n_sys && sc[s].active) {
    sc[s].beta = 0.0;
    sc[s].stale = 0;
  }
}

void bfinal(Ctx& c, BatchState& b, BOp op, double rtol2, int max_stale, bool f32 = false) {
  const int2* map = (op == kBAlpha || op == kBReplace) ? b.mw.get() : b.mv.get();
  k_bfinal<<<b.n_meshes, kBThreads, 0, c.stream>>>(int(op), map, b.part.get(), b.sc.get(), rtol2,
                                                   max_stale, int(f32));
  SFEM_HIP(hipGetLastError());
}

// One check period: `iters` CG iterations, then the FP64 residual
// replacement and the convergence test (kernel launches only: capturable).
void period(Ctx& c, BatchState& b, bool f32, int iters, double rtol2, int max_stale) {
  const int V = b.n_vw;
  const Work vk{b.alist.get(), b.acnt.get() + kNumBuckets, b.n_wg(), V};
  const int vgrid = std::min(V, kBGridCap);
  compact(c, b);
  for (int k = 0; k < iters; ++k) {
    k_bp<<<vgrid, kBThreads, 0, c.stream>>>(vk, b.vr.get(), b.vmesh.get(), b.sc.get(), b.Z.get(),
                                            b.P.get());
    bspmm<0>(c, b, f32, b.P.get(), nullptr, b.Q.get(), nullptr);
    bfinal(c, b, kBAlpha, rtol2, max_stale);
    k_bupdate<<<vgrid, kBThreads, 0, c.stream>>>(vk, b.vr.get(), b.vmesh.get(), b.sc.get(),
                                             c.dinv.get(), b.X.get(), b.R.get(), b.Z.get(),
                                             b.P.get(), b.Q.get(), b.part.get());
    bfinal(c, b, kBBeta, rtol2, max_stale);
  }
  bspmm<1>(c, b, false, b.X.get(), b.F.get(), b.R.get(), b.Z.get());
  bfinal(c, b, kBReplace, rtol2, max_stale, f32);
  SFEM_HIP(hipGetLastError());
}

}  // namespace

// ------------------------------------------------------------ host driver
void batch_prepare(Ctx& c, BatchState& b) {
  const int64_t n = c.n_dof();
  b.bucket.resize(b.n_meshes);
  for (int m = 0; m < b.n_meshes; ++m) {
    b.bucket[m] = bucket_of(b.node0[m + 1] - b.node0[m]);
  }
  for (auto* v : {&b.F, &b.X, &b.R, &b.Z, &b.P, &b.Q}) v->reserve(size_t(n) * kNR);
  b.sc.reserve(size_t(b.n_meshes) * kNR);
  if (!b.sc_host)
    SFEM_HIP(hipHostMalloc((void**)&b.sc_host, 2 * sizeof(BScal) * b.n_meshes * kNR,
                           hipHostMallocDefault));
  for (hipEvent_t& e : b.flags_ready)
    if (!e) SFEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  k_bzero<<<div_up(n * kNR, 256), 256, 0, c.stream>>>(n * kNR, b.F.get());
  SFEM_HIP(hipGetLastError());
  build_table(c, b);
}

// Right-hand side k from the context's current f_bc.
void batch_set_column(Ctx& c, BatchState& b, int k) {
  const int64_t n = c.n_dof();
  k_bset_column<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.f_bc.get(), k, b.F.get());
  SFEM_HIP(hipGetLastError());
}

static std::tuple<int, int, int> tune_key(Ctx& c, BatchState& b, int bk) {
  int64_t rows = 0, blocks = 0;
  std::vector<int32_t> bp;
  for (int m = 0; m < b.n_meshes; ++m)
    if (b.bucket[m] == bk) rows += b.node0[m + 1] - b.node0[m];
  // mean block degree of the bucket from the host copy of the row pointers
  for (int m = 0; m < b.n_meshes; ++m) {
    if (b.bucket[m] != bk) continue;
    int32_t lohi[2];
    SFEM_HIP(hipMemcpy(&lohi[0], c.topo.bptr.get() + b.node0[m], sizeof(int32_t),
                       hipMemcpyDeviceToHost));
    SFEM_HIP(hipMemcpy(&lohi[1], c.topo.bptr.get() + b.node0[m + 1], sizeof(int32_t),
                       hipMemcpyDeviceToHost));
    blocks += lohi[1] - lohi[0];
  }
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= rows) ++lg;
  const int deg = rows ? int((blocks + rows / 2) / rows) : 0;
  return {bk, lg, deg};
}

// Times every (lanes per row, rows per workgroup) candidate for each
// non-empty bucket unless the bucket's shape is cached (use_cache).  A
// candidate's cost is its product time with every system active plus its
// time with only the bucket's largest mesh active: most iterations of a
// batched solve run with the easy meshes already retired, where the
// workgroups of finished meshes still cost their dispatch.  Returns the
// tuned product time in microseconds (all buckets, all active).
// Uploads per-system scalars whose only meaningful field is the active flag
// (tuning; a solve's start resets every system's scalars).
static void set_masks(Ctx& c, BatchState& b, const std::vector<BScal>& mask) {
  SFEM_HIP(hipMemcpyAsync(b.sc.get(), mask.data(), sizeof(BScal) * mask.size(),
                          hipMemcpyHostToDevice, c.stream));
}

double batch_autotune(Ctx& c, BatchState& b, int reps, bool use_cache, bool f32) {
  if (reps <= 0) reps = 5;
  std::vector<BScal> all_mask(size_t(b.n_meshes) * kNR, BScal{});
  for (auto& q : all_mask) q.active = 1;
  pack_values64(c);  // the packed candidates read it
  SFEM_HIP(hipStreamSynchronize(c.stream));
  for (int bk = 0; bk < kNumBuckets; ++bk) {
    bool any = false;
    for (int m = 0; m < b.n_meshes; ++m) any = any || b.bucket[m] == bk;
    if (!any) continue;
    const auto key = tune_key(c, b, bk);
    if (use_cache) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        b.packed[bk] = it->second.first < 0;   // packed schedules are cached negated
        b.lpr[bk] = std::abs(it->second.first);
        b.rw[bk] = it->second.second;
        b.from_cache[bk] = true;
        continue;
      }
    }
    // the tail state: only the bucket's largest mesh active
    std::vector<BScal> tail_mask(size_t(b.n_meshes) * kNR, BScal{});
    {
      int big = -1;
      int64_t rows = -1;
      for (int m = 0; m < b.n_meshes; ++m)
        if (b.bucket[m] == bk && b.node0[m + 1] - b.node0[m] > rows) {
          rows = b.node0[m + 1] - b.node0[m];
          big = m;
        }
      for (int k = 0; k < kNR; ++k) tail_mask[size_t(big) * kNR + k].active = 1;
    }
    // the bucket's product over the lists compacted from a mask, as in a solve
    auto time_product = [&](const std::vector<BScal>& mask) {
      set_masks(c, b, mask);
      compact(c, b);
      bspmm<0>(c, b, f32, b.F.get(), nullptr, b.Q.get(), nullptr, bk);  // warm
      SFEM_HIP(hipEventRecord(c.ev0, c.stream));
      for (int r = 0; r < reps; ++r)
        bspmm<0>(c, b, f32, b.F.get(), nullptr, b.Q.get(), nullptr, bk);
      SFEM_HIP(hipEventRecord(c.ev1, c.stream));
      SFEM_HIP(hipEventSynchronize(c.ev1));
      float ms = 0;
      SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
      return double(ms);
    };
    double best = 1e30;
    int bl = b.lpr[bk], br = b.rw[bk];
    bool bp = b.packed[bk];
    const int n_cand = kNumLpr + (f32 ? 0 : kNumPLpr);
    for (int li = 0; li < n_cand; ++li)
      for (int ri = 0; ri < kNumRw; ++ri) {
        const bool pk = li >= kNumLpr;
        const int lpr = pk ? kPLprs[li - kNumLpr] : kLprs[li];
        // a workgroup has kBThreads / lpr row groups: fewer rows would idle some
        if (kRws[ri] < kBThreads / lpr) continue;
        b.packed[bk] = pk;
        b.lpr[bk] = lpr;
        b.rw[bk] = kRws[ri];
        build_table(c, b);
        const double ms = time_product(all_mask) + time_product(tail_mask);
        if (ms < best) {
          best = ms;
          bl = b.lpr[bk];
          br = kRws[ri];
          bp = pk;
        }
      }
    b.lpr[bk] = bl;
    b.rw[bk] = br;
    b.packed[bk] = bp;
    b.from_cache[bk] = false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {bp ? -bl : bl, br};
  }
  build_table(c, b);
  // time the tuned product over all buckets, every system active
  set_masks(c, b, all_mask);
  compact(c, b);
  bspmm<0>(c, b, f32, b.F.get(), nullptr, b.Q.get(), nullptr, -1);
  SFEM_HIP(hipEventRecord(c.ev0, c.stream));
  for (int r = 0; r < reps; ++r)
    bspmm<0>(c, b, f32, b.F.get(), nullptr, b.Q.get(), nullptr, -1);
  SFEM_HIP(hipEventRecord(c.ev1, c.stream));
  SFEM_HIP(hipEventSynchronize(c.ev1));
  float ms = 0;
  SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
  return 1e3 * ms / reps;
}

// Solves every (mesh, load case) system.  Returns the number of check
// periods run; the per-system scalars are left in b.sc_host.
int batch_solve(Ctx& c, BatchState& b, bool f32, double rtol, int max_iter, int check_every,
                bool use_graph, double* ms_out, int* fp64_from) {
  SFEM_REQUIRE(!f32 || c.have_f32, SFEM_ESTATE, "the FP32 mode needs an FP32 copy of K");
  const int V = b.n_vw;
  const double rtol2 = rtol * rtol;
  const int max_stale = 40;
  const int n_sys = b.n_meshes * kNR;
  if (b.packed[0] || b.packed[1] || b.packed[2]) pack_values64(c);  // before any capture
  if (fp64_from) *fp64_from = 0;
  SFEM_HIP(hipEventRecord(c.ev0, c.stream));
  k_bstart<<<V, kBThreads, 0, c.stream>>>(b.vr.get(), c.dinv.get(), b.F.get(), b.X.get(),
                                          b.R.get(), b.Z.get(), b.P.get(), b.part.get());
  SFEM_HIP(hipGetLastError());
  bfinal(c, b, kBStart, rtol2, max_stale);
  auto capture = [&](bool prec32) {
    if (!use_graph || (b.graph_key[0] == int(prec32) && b.graph_key[1] == check_every)) return;
    b.drop_graph();
    SFEM_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    try {
      period(c, b, prec32, check_every, rtol2, max_stale);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    SFEM_HIP(hipStreamEndCapture(c.stream, &b.graph));
    SFEM_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    b.graph_key[0] = int(prec32);
    b.graph_key[1] = check_every;
  };
  capture(f32);
  // Period p copies the systems' flags into host slot p % 2 and records
  // flags_ready[p % 2].  Period p + 1 is enqueued before the host waits for
  // period p's flags, so the GPU never idles while the host reads them; a
  // period enqueued after every system has finished walks empty work lists.
  const size_t slot_bytes = sizeof(BScal) * n_sys;
  auto enqueue = [&](int p) {
    if (use_graph) SFEM_HIP(hipGraphLaunch(b.exec, c.stream));
    else period(c, b, f32, check_every, rtol2, max_stale);
    SFEM_HIP(hipMemcpyAsync(b.sc_host + (p & 1) * n_sys, b.sc.get(), slot_bytes,
                            hipMemcpyDeviceToHost, c.stream));
    SFEM_HIP(hipEventRecord(b.flags_ready[p & 1], c.stream));
  };
  const int max_periods = std::max(1, div_up(max_iter, check_every));
  int periods = 0;
  enqueue(periods++);
  for (int p = 0; p < max_periods; ++p) {
    if (periods < max_periods) enqueue(periods++);
    SFEM_HIP(hipEventSynchronize(b.flags_ready[p & 1]));
    const BScal* fl = b.sc_host + (p & 1) * n_sys;
    bool any = false, need64 = false;
    for (int s = 0; s < n_sys; ++s) {
      any = any || fl[s].active;
      need64 = need64 || (fl[s].active && fl[s].need64);
    }
    if (!any) break;
    if (f32 && need64) {
      // a system stagnated with FP32 products: the rest of the solve runs
      // FP64 products, every active system restarted from its x (after the
      // period already enqueued, whose graph must finish before the
      // recapture)
      f32 = false;
      if (fp64_from) *fp64_from = periods;
      SFEM_HIP(hipStreamSynchronize(c.stream));
      k_brestart<<<div_up(n_sys, 256), 256, 0, c.stream>>>(n_sys, b.sc.get());
      SFEM_HIP(hipGetLastError());
      capture(false);
    }
  }
  // the final per-system scalars, for the info calls
  SFEM_HIP(hipMemcpyAsync(b.sc_host, b.sc.get(), slot_bytes, hipMemcpyDeviceToHost, c.stream));
  SFEM_HIP(hipEventRecord(c.ev1, c.stream));
  SFEM_HIP(hipEventSynchronize(c.ev1));
  float ms = 0;
  SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
  if (ms_out) *ms_out = ms;
  return periods;
}

void batch_column(Ctx& c, BatchState& b, int m, int k, double* out_dev) {
  const int64_t i0 = 3 * b.node0[m], n = 3 * (b.node0[m + 1] - b.node0[m]);
  k_bcolumn<<<div_up(n, 256), 256, 0, c.stream>>>(n, b.X.get() + i0 * kNR, k, out_dev);
  SFEM_HIP(hipGetLastError());
}

void batch_system(const BatchState& b, int s, int* iters, int* converged, double* relres,
                  int* breakdown) {
  const BScal& q = b.sc_host[s];
  *iters = q.iters;
  *converged = q.rr_true <= q.tol2 ? 1 : 0;
  *relres = q.ff > 0 ? std::sqrt(q.rr_true / q.ff) : 0.0;
  *breakdown = q.breakdown;
}

void batch_rebuild_table(Ctx& c, BatchState& b) {
  build_table(c, b);
  if (b.packed[0] || b.packed[1] || b.packed[2]) pack_values64(c);
}

void batch_set_schedule(BatchState& b, int bk, int lanes, int rows, bool packed) {
  b.lpr[bk] = lanes;
  b.rw[bk] = rows;
  b.packed[bk] = packed;
  b.from_cache[bk] = false;
}

int batch_bucket_info(const BatchState& b, int bk, int* lanes, int* rows, int* cached,
                      int* packed) {
  *packed = b.packed[bk] ? 1 : 0;
  *lanes = b.lpr[bk];
  *rows = b.rw[bk];
  *cached = b.from_cache[bk] ? 1 : 0;
  int n = 0;
  for (int m = 0; m < b.n_meshes; ++m) n += b.bucket[m] == bk;
  return n;
}

}  // namespace sfem

// ================================================================ C ABI
struct sfem_batch {
  sfem_ctx* ctx = nullptr;
  int device = 0;
  std::string err;
  struct Mesh {
    std::vector<double> xyz;
    std::vector<int32_t> tets;
    double E, nu;
    std::vector<int32_t> fixed;
  };
  struct Trac {
    int mesh, rhs;
    std::vector<int32_t> tri;
    double t[3];
  };
  std::vector<Mesh> meshes;
  std::vector<Trac> trac;
  bool built = false;
  std::unique_ptr<sfem::BatchState> st = std::make_unique<sfem::BatchState>();
};

namespace {

template <typename F>
int bguarded(sfem_batch* h, F&& fn) {
  if (!h) return SFEM_EINVAL;
  h->err.clear();
  try {
    SFEM_HIP(hipSetDevice(h->device));
    return fn(*h);
  } catch (const sfem::Error& e) {
    h->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    h->err = e.what();
    return SFEM_EINVAL;
  }
}

int check(sfem_batch& h, int st) {
  if (st != SFEM_OK) throw sfem::Error{st, std::string("batch build: ") + sfem_last_error(h.ctx)};
  return st;
}

}  // namespace

extern "C" {

int sfem_batch_create(sfem_batch** out, int device) {
  if (!out) return SFEM_EINVAL;
  *out = nullptr;
  sfem_batch* h = new (std::nothrow) sfem_batch;
  if (!h) return SFEM_ENOMEM;
  h->device = device;
  const int st = sfem_create(&h->ctx, device, nullptr);
  if (st != SFEM_OK) {
    delete h;
    return st;
  }
  *out = h;
  return SFEM_OK;
}

void sfem_batch_destroy(sfem_batch* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  if (h->ctx) (void)hipStreamSynchronize(h->ctx->c.stream);
  h->st.reset();  // graph and device buffers before the context's stream
  sfem_destroy(h->ctx);
  delete h;
}

const char* sfem_batch_last_error(const sfem_batch* h) { return h ? h->err.c_str() : "null batch"; }

int sfem_batch_add_mesh(sfem_batch* h, int64_t n_nodes, const double* xyz, int64_t n_tets,
                        const int32_t* tets, double E, double nu, int64_t n_fixed,
                        const int32_t* fixed_dofs, int* mesh_index) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(!b.built, SFEM_ESTATE, "the batch is already built");
    SFEM_REQUIRE(n_nodes > 0 && n_tets > 0 && xyz && tets, SFEM_EINVAL, "empty mesh");
    SFEM_REQUIRE(n_fixed >= 0 && (fixed_dofs || n_fixed == 0), SFEM_EINVAL, "bad fixed DOFs");
    SFEM_REQUIRE(E > 0.0 && nu > -1.0 && nu < 0.5, SFEM_EINVAL, "need E > 0, -1 < nu < 0.5");
    int64_t total = 0;
    for (const auto& m : b.meshes) total += int64_t(m.xyz.size() / 3);
    SFEM_REQUIRE(total + n_nodes < (int64_t(1) << 30), SFEM_EINVAL, "batch too large");
    sfem_batch::Mesh m;
    m.xyz.assign(xyz, xyz + 3 * n_nodes);
    m.tets.assign(tets, tets + 4 * n_tets);
    for (int32_t v : m.tets)
      SFEM_REQUIRE(v >= 0 && v < n_nodes, SFEM_EINVAL, "tet node index out of range");
    m.fixed.assign(fixed_dofs, fixed_dofs + n_fixed);
    for (int32_t d : m.fixed)
      SFEM_REQUIRE(d >= 0 && d < 3 * n_nodes, SFEM_EINVAL, "fixed DOF out of range");
    m.E = E;
    m.nu = nu;
    b.meshes.push_back(std::move(m));
    if (mesh_index) *mesh_index = int(b.meshes.size()) - 1;
    return SFEM_OK;
  });
}

int sfem_batch_add_traction(sfem_batch* h, int mesh, int rhs, int64_t n_tri, const int32_t* tri,
                            const double t[3]) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(!b.built, SFEM_ESTATE, "the batch is already built");
    SFEM_REQUIRE(mesh >= 0 && mesh < int(b.meshes.size()), SFEM_EINVAL, "bad mesh index");
    SFEM_REQUIRE(rhs >= 0 && rhs < 4, SFEM_EINVAL, "rhs must be in [0, 4)");
    SFEM_REQUIRE(n_tri >= 0 && t && (tri || n_tri == 0), SFEM_EINVAL, "bad traction");
    const int64_t nn = int64_t(b.meshes[mesh].xyz.size() / 3);
    sfem_batch::Trac tr{mesh, rhs, std::vector<int32_t>(tri, tri + 3 * n_tri), {t[0], t[1], t[2]}};
    for (int32_t v : tr.tri) SFEM_REQUIRE(v >= 0 && v < nn, SFEM_EINVAL, "triangle node out of range");
    b.trac.push_back(std::move(tr));
    return SFEM_OK;
  });
}

int sfem_batch_build(sfem_batch* h, int flags) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(!b.built, SFEM_ESTATE, "the batch is already built");
    SFEM_REQUIRE(!b.meshes.empty(), SFEM_ESTATE, "add meshes first");
    std::vector<double> xyz, E, nu;
    std::vector<int32_t> tets, fixed;
    std::vector<int64_t> node0{0};
    for (const auto& m : b.meshes) {
      const int64_t off = node0.back();
      xyz.insert(xyz.end(), m.xyz.begin(), m.xyz.end());
      for (int32_t v : m.tets) tets.push_back(int32_t(v + off));
      E.insert(E.end(), m.tets.size() / 4, m.E);
      nu.insert(nu.end(), m.tets.size() / 4, m.nu);
      for (int32_t d : m.fixed) fixed.push_back(int32_t(d + 3 * off));
      node0.push_back(off + int64_t(m.xyz.size() / 3));
    }
    sfem_ctx* ch = b.ctx;
    check(b, sfem_set_mesh(ch, node0.back(), xyz.data(), int64_t(tets.size() / 4), tets.data(),
                           SFEM_PTR_HOST));
    check(b, sfem_set_material_per_tet(ch, E.data(), nu.data(), SFEM_PTR_HOST));
    if (!fixed.empty())
      check(b, sfem_set_dirichlet(ch, int64_t(fixed.size()), fixed.data(), nullptr, SFEM_PTR_HOST));
    check(b, sfem_assemble(ch, flags));
    sfem::Ctx& c = ch->c;
    sfem::ensure_csr64(c);  // the batched products read the CSR order
    if (c.have_f32) sfem::ensure_rowcorr(c);  // FP32 products in the corrected form
    sfem::BatchState& s = *b.st;
    s.n_meshes = int(b.meshes.size());
    s.node0 = node0;
    sfem::batch_prepare(c, s);
    // load cases: f_user := tractions of case k, f_bc := BCs applied, column k
    const int64_t n = c.n_dof();
    for (int k = 0; k < 4; ++k) {
      SFEM_HIP(hipMemsetAsync(c.f_user.get(), 0, sizeof(double) * n, c.stream));
      bool any = false;
      for (const auto& tr : b.trac) {
        if (tr.rhs != k || tr.tri.empty()) continue;
        const int64_t off = node0[tr.mesh];
        std::vector<int32_t> g(tr.tri.size());
        for (size_t i = 0; i < g.size(); ++i) g[i] = int32_t(tr.tri[i] + off);
        sfem::DBuf<int32_t> dt;
        dt.reserve(g.size());
        SFEM_HIP(hipMemcpyAsync(dt.get(), g.data(), sizeof(int32_t) * g.size(),
                                hipMemcpyHostToDevice, c.stream));
        sfem::traction_load(c, int64_t(g.size() / 3), dt.get(), tr.t);
        SFEM_HIP(hipStreamSynchronize(c.stream));
        any = true;
      }
      if (!any) continue;
      sfem::rhs_with_bc(c);
      sfem::batch_set_column(c, s, k);
    }
    SFEM_HIP(hipStreamSynchronize(c.stream));
    b.built = true;
    return SFEM_OK;
  });
}

int sfem_batch_sizes(sfem_batch* h, int* n_meshes, int64_t* n_nodes, int64_t* n_tets,
                     int64_t* n_faces, int64_t* nnz) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(b.built, SFEM_ESTATE, "build the batch first");
    const sfem::Ctx& c = b.ctx->c;
    if (n_meshes) *n_meshes = b.st->n_meshes;
    if (n_nodes) *n_nodes = c.N;
    if (n_tets) *n_tets = c.T;
    if (n_faces) *n_faces = c.topo.nf;
    if (nnz) *nnz = 9 * c.topo.nb;
    return SFEM_OK;
  });
}

int sfem_batch_autotune(sfem_batch* h, int reps, int use_cache, int precision, double* us) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(b.built, SFEM_ESTATE, "build the batch first");
    const bool f32 = precision == SFEM_ASM_F32_COPY;
    SFEM_REQUIRE(!f32 || b.ctx->c.have_f32, SFEM_ESTATE, "no FP32 copy of K");
    const double t = sfem::batch_autotune(b.ctx->c, *b.st, reps, use_cache != 0, f32);
    if (us) *us = t;
    return SFEM_OK;
  });
}

int sfem_batch_set_schedule(sfem_batch* h, int bucket, int lanes_per_row, int rows_per_wg,
                            int packed) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(b.built, SFEM_ESTATE, "build the batch first");
    SFEM_REQUIRE(bucket >= 0 && bucket < 3, SFEM_EINVAL, "bucket must be in [0, 3)");
    const bool ok_l = packed ? (lanes_per_row == 4 || lanes_per_row == 8)
                             : (lanes_per_row == 8 || lanes_per_row == 16 || lanes_per_row == 32);
    SFEM_REQUIRE(ok_l && (rows_per_wg == 16 || rows_per_wg == 64 || rows_per_wg == 256),
                 SFEM_EINVAL, "not one of the tuner's schedules");
    sfem::batch_set_schedule(*b.st, bucket, lanes_per_row, rows_per_wg, packed != 0);
    sfem::batch_rebuild_table(b.ctx->c, *b.st);
    return SFEM_OK;
  });
}

int sfem_batch_get_schedule(sfem_batch* h, int bucket, int* lanes_per_row, int* rows_per_wg,
                            int* n_meshes, int* from_cache, int* packed) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(b.built, SFEM_ESTATE, "build the batch first");
    SFEM_REQUIRE(bucket >= 0 && bucket < 3, SFEM_EINVAL, "bucket must be in [0, 3)");
    int l = 0, r = 0, fc = 0, pk = 0;
    const int n = sfem::batch_bucket_info(*b.st, bucket, &l, &r, &fc, &pk);
    if (packed) *packed = pk;
    if (lanes_per_row) *lanes_per_row = l;
    if (rows_per_wg) *rows_per_wg = r;
    if (n_meshes) *n_meshes = n;
    if (from_cache) *from_cache = fc;
    return SFEM_OK;
  });
}

int sfem_batch_solve(sfem_batch* h, const sfem_batch_opts* o, sfem_batch_info* info) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(b.built, SFEM_ESTATE, "build the batch first");
    SFEM_REQUIRE(o && o->rtol > 0.0, SFEM_EINVAL, "need opts with rtol > 0");
    SFEM_REQUIRE(o->mode == SFEM_MODE_F64 || o->mode == SFEM_MODE_F32_RR, SFEM_EINVAL,
                 "batch modes: SFEM_MODE_F64 or SFEM_MODE_F32_RR");
    const int every = o->check_every > 0 ? o->check_every : 50;
    const int max_iter = o->max_iter > 0 ? o->max_iter : 100000;
    double ms = 0;
    int fp64_from = 0;
    const int periods = sfem::batch_solve(b.ctx->c, *b.st, o->mode == SFEM_MODE_F32_RR, o->rtol,
                                          max_iter, every, o->use_graph != 0, &ms, &fp64_from);
    int all = 1, worst_it = 0;
    double worst = 0.0;
    for (int s = 0; s < b.st->n_meshes * 4; ++s) {
      int it, conv, brk;
      double rr;
      sfem::batch_system(*b.st, s, &it, &conv, &rr, &brk);
      all = all && conv;
      worst = std::max(worst, rr);
      worst_it = std::max(worst_it, it);
    }
    if (info) {
      info->ms_solve = ms;
      info->periods = periods;
      info->all_converged = all;
      info->max_iters = worst_it;
      info->worst_relres = worst;
      info->fp64_from_period = fp64_from;
    }
    return all ? SFEM_OK : SFEM_ENOCONV;
  });
}

int sfem_batch_get_solution(sfem_batch* h, int mesh, int rhs, double* u, int ptr_kind) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(b.built, SFEM_ESTATE, "build the batch first");
    SFEM_REQUIRE(mesh >= 0 && mesh < b.st->n_meshes && rhs >= 0 && rhs < 4 && u, SFEM_EINVAL,
                 "bad mesh / rhs / output");
    SFEM_REQUIRE(ptr_kind == SFEM_PTR_HOST || ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL,
                 "bad ptr_kind");
    sfem::Ctx& c = b.ctx->c;
    const int64_t n = 3 * (b.st->node0[mesh + 1] - b.st->node0[mesh]);
    if (ptr_kind == SFEM_PTR_DEVICE) {
      sfem::batch_column(c, *b.st, mesh, rhs, u);
    } else {
      sfem::DBuf<double> tmp;
      tmp.reserve(n);
      sfem::batch_column(c, *b.st, mesh, rhs, tmp.get());
      SFEM_HIP(hipMemcpyAsync(u, tmp.get(), sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    }
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

int sfem_batch_get_system_info(sfem_batch* h, int32_t* iters, int32_t* converged, double* relres,
                               int32_t* breakdown) {
  return bguarded(h, [&](sfem_batch& b) {
    SFEM_REQUIRE(b.built, SFEM_ESTATE, "build the batch first");
    for (int s = 0; s < b.st->n_meshes * 4; ++s) {
      int it, conv, brk;
      double rr;
      sfem::batch_system(*b.st, s, &it, &conv, &rr, &brk);
      if (iters) iters[s] = it;
      if (converged) converged[s] = conv;
      if (relres) relres[s] = rr;
      if (breakdown) breakdown[s] = brk;
    }
    return SFEM_OK;
  });
}

}  // extern "C"
