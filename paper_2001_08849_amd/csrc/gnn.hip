// Learned preconditioner: a message-passing network over the 3x3-block
// pattern of K outputs a symmetric block correction S', and
//   M = D^-1/2 (I + S') D^-1/2
// is applied inside flexible PCG (not part of the paper; the network and the
// loss are defined in the library header).
//
// Dense layers run on MFMA (v_mfma_f32_16x16x32_bf16): BF16 operands staged
// in LDS, FP32 accumulation.  A workgroup of 4 waves computes 64 x 64 output
// tiles; wave w owns rows 16w..16w+15 and all four 16-column tiles.  Lane
// layout of the 16x16x32 BF16 MFMA (checked on the device): lane l holds
// A[l%16][8(l/16)+t], B[8(l/16)+t][l%16] (t = 0..7) and C[4(l/16)+v][l%16]
// (v = 0..3).
//
// Three GEMM shapes cover training and inference:
//   k_gemm_xwT   Y[rows x 64]  = X[rows x KD] W^T       (layer forward)
//   k_gemm_xw    Y[rows x KO]  = G[rows x 64] W          (input gradients)
//   k_gemm_wgrad P[64 x KD]   += G[tile]^T X[tile]       (weight gradients,
//                split over row tiles; partials summed in a fixed order)
// Rows are edges (blocks of the pattern) or nodes.  Edge inputs [h_I; h_J; e]
// are gathered while staging, never stored.  Scatter-adds of the backward
// pass go through the transposed-edge map (edge (J,I) of edge (I,J)), so
// every output has one writer and results are reproducible.
#include <limits>

#include "gnn.h"

namespace sfem {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;          // rows (edges or nodes) per GEMM tile
constexpr int kGemmThreads = 256;  // 4 waves
constexpr int kGemmGrid = 2048;    // cap of the row-tile GEMM grids
constexpr int kWgradGrid = 256;    // workgroups (partials) of a weight gradient
constexpr int kRedGrid = 256;      // partials of the small reductions
// workgroups of the column-sum and small weight-gradient reductions over the
// edges / nodes (memory-bound: enough workgroups to fill the chip)
constexpr int kColGrid = 2048;
constexpr int kMaxBatch = 64;      // pairs per minibatch

__device__ __forceinline__ float relu(float v) { return v > 0.f ? v : 0.f; }

// acc[jt] += A[16w.., :KD] * Bt[16jt.., :KD]^T on the 16x16 tiles of wave w.
// A, Bt: BF16 in LDS with row strides lda, ldb (elements); row j of Bt is
// column j of B.
template <int KD>
__device__ __forceinline__ void mfma_tile(const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                          f32x4 (&acc)[4]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = l & 15, kq = (l >> 4) * 8;
#pragma unroll
  for (int ks = 0; ks < KD; ks += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(A + (16 * w + r) * lda + ks + kq);
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bt + (16 * jt + r) * ldb + ks + kq);
      acc[jt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[jt], 0, 0, 0);
    }
  }
}

// Visits this lane's outputs of a 64 x 64 tile: f(row, col, value).
template <class F>
__device__ __forceinline__ void tile_out(const f32x4 (&acc)[4], F&& f) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v) f(16 * w + 4 * (l >> 4) + v, 16 * jt + (l & 15), acc[jt][v]);
}

// ------------------------------------------------------------- row loaders
// get4(row, k): four consecutive FP32 inputs of a GEMM row (k % 4 == 0).
struct EdgeX {  // [h_I; h_J; e] of edge b = (I, J)
  const int32_t* __restrict__ erow;
  const int32_t* __restrict__ bcol;
  const float* __restrict__ h;
  const float* __restrict__ e;
  __device__ __forceinline__ float4 get4(int64_t b, int k) const {
    const float* src = k < kH       ? h + int64_t(erow[b]) * kH + k
                       : k < 2 * kH ? h + int64_t(bcol[b]) * kH + (k - kH)
                                    : e + b * kH + (k - 2 * kH);
    return *reinterpret_cast<const float4*>(src);
  }
};

struct NodeY {  // [h_I; a_I]
  const float* __restrict__ h;
  const float* __restrict__ a;
  __device__ __forceinline__ float4 get4(int64_t I, int k) const {
    const float* src = k < kH ? h + I * kH + k : a + I * kH + (k - kH);
    return *reinterpret_cast<const float4*>(src);
  }
};

struct Rows64 {  // a plain [rows][64] array
  const float* __restrict__ p;
  __device__ __forceinline__ float4 get4(int64_t r, int k) const {
    return *reinterpret_cast<const float4*>(p + r * kH + k);
  }
};

// Row-major BF16 tile staging, split in two for software pipelining:
// fetch() loads the inputs L(r0 + r, k) of a tile into registers (zero past
// `rows`), store() writes them to LDS at dst[r * ld + k].  Each row is split
// over TPR consecutive threads, each taking a contiguous run of the row (one
// row's gather indices per thread).
template <int KD, class Ld>
struct RowsPrefetch {
  static constexpr int Q = KD / 4;
  static constexpr int TPR = kGemmThreads / kTile;
  static constexpr int PER = Q / TPR;
  float4 v[PER];
  __device__ __forceinline__ void fetch(const Ld& L, int64_t r0, int64_t rows) {
    const int r = threadIdx.x / TPR, k0 = 4 * PER * (threadIdx.x % TPR);
    const int64_t row = r0 + r;
#pragma unroll
    for (int j = 0; j < PER; ++j)
      v[j] = row < rows ? L.get4(row, k0 + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __device__ __forceinline__ void store(__bf16* dst, int ld) const {
    const int r = threadIdx.x / TPR, k0 = 4 * PER * (threadIdx.x % TPR);
#pragma unroll
    for (int j = 0; j < PER; ++j)
      *reinterpret_cast<bf16x4*>(dst + r * ld + k0 + 4 * j) =
          bf16x4{__bf16(v[j].x), __bf16(v[j].y), __bf16(v[j].z), __bf16(v[j].w)};
  }
};

// Transposed BF16 tile staging, split the same way: dst[k * ld + r] =
// L(r0 + r, k) (consecutive lanes take consecutive rows, so the 2-byte LDS
// writes do not collide).
template <int KD, class Ld>
struct ColsPrefetch {
  static constexpr int PER = kTile * (KD / 4) / kGemmThreads;
  static_assert(kTile * (KD / 4) % kGemmThreads == 0, "tile inputs must split evenly");
  float4 v[PER];
  __device__ __forceinline__ void fetch(const Ld& L, int64_t r0, int64_t rows) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = threadIdx.x + j * kGemmThreads;
      const int r = i % kTile, k = 4 * (i / kTile);
      v[j] = (r0 + r < rows) ? L.get4(r0 + r, k) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  __device__ __forceinline__ void store(__bf16* dst, int ld) const {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = threadIdx.x + j * kGemmThreads;
      const int r = i % kTile, k = 4 * (i / kTile);
      dst[(k + 0) * ld + r] = __bf16(v[j].x);
      dst[(k + 1) * ld + r] = __bf16(v[j].y);
      dst[(k + 2) * ld + r] = __bf16(v[j].z);
      dst[(k + 3) * ld + r] = __bf16(v[j].w);
    }
  }
};

// ------------------------------------------------------------------ GEMMs
// Y = X W^T, W: [64][KD] BF16 (row o = output feature).
// epi.pre(row, o): the output's residual input, loaded before the MFMA;
// epi(row, o, y, pre).
// Software-pipelined over the workgroup's row tiles: the next tile's rows are
// loaded into registers (and this tile's residual inputs, issued first so
// that waiting for them does not wait for the prefetch) while this tile's
// MFMA runs; the registers go to LDS after the tile is done.
template <int KD, class Ld, class Epi>
__global__ void __launch_bounds__(kGemmThreads)
    k_gemm_xwT(int64_t rows, Ld L, const __bf16* __restrict__ W, Epi epi) {
  constexpr int LD = KD + 8;  // padded LDS row (bank spread), 16-byte multiple
  __shared__ __align__(16) __bf16 sW[kH * LD];
  __shared__ __align__(16) __bf16 sX[kTile * LD];
  for (int i = threadIdx.x; i < kH * KD / 8; i += kGemmThreads) {
    const int o = i / (KD / 8), k = 8 * (i % (KD / 8));
    *reinterpret_cast<bf16x8*>(sW + o * LD + k) = *reinterpret_cast<const bf16x8*>(W + o * KD + k);
  }
  const int64_t ntiles = (rows + kTile - 1) / kTile;
  RowsPrefetch<KD, Ld> pf;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t tile = blockIdx.x;
  if (tile < ntiles) pf.fetch(L, tile * kTile, rows);
  for (; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * kTile;
    __syncthreads();  // the previous tile's MFMA reads of sX are done
    pf.store(sX, LD);
    __syncthreads();
    float res[16];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + 4 * (l >> 4) + v, o = 16 * jt + (l & 15);
        res[4 * jt + v] = r0 + r < rows ? epi.pre(r0 + r, o) : 0.f;
      }
    if (tile + gridDim.x < ntiles) pf.fetch(L, (tile + gridDim.x) * kTile, rows);
    f32x4 acc[4] = {};
    mfma_tile<KD>(sX, LD, sW, LD, acc);
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + 4 * (l >> 4) + v, o = 16 * jt + (l & 15);
        if (r0 + r < rows) epi(r0 + r, o, acc[jt][v], res[4 * jt + v]);
      }
  }
}

// Y = G W, G: [rows][64] FP32 (loader), W: [64][KO] BF16.  epi(row, j, y).
template <int KO, class Ld, class Epi>
__global__ void __launch_bounds__(kGemmThreads)
    k_gemm_xw(int64_t rows, Ld L, const __bf16* __restrict__ W, Epi epi) {
  constexpr int LD = kH + 8;
  __shared__ __align__(16) __bf16 sWt[KO * LD];  // W^T: row j = column j of W
  __shared__ __align__(16) __bf16 sA[kTile * LD];
  for (int i = threadIdx.x; i < kH * KO; i += kGemmThreads) {
    const int k = i / KO, j = i % KO;
    sWt[j * LD + k] = W[i];
  }
  const int64_t ntiles = (rows + kTile - 1) / kTile;
  // the next tile's rows load into registers during this tile's MFMA
  RowsPrefetch<kH, Ld> pf;
  if (int64_t(blockIdx.x) < ntiles) pf.fetch(L, int64_t(blockIdx.x) * kTile, rows);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * kTile;
    __syncthreads();
    pf.store(sA, LD);
    __syncthreads();
    if (tile + gridDim.x < ntiles) pf.fetch(L, (tile + gridDim.x) * kTile, rows);
#pragma unroll
    for (int jc = 0; jc < KO / 64; ++jc) {
      f32x4 acc[4] = {};
      mfma_tile<kH>(sA, LD, sWt + jc * 64 * LD, LD, acc);
      tile_out(acc, [&](int r, int j, float v) {
        if (r0 + r < rows) epi(r0 + r, jc * 64 + j, v);
      });
    }
  }
}

// part[block][i][j] = sum over this block's row tiles of G[r][i] X[r][j]
// (i < 64, j < KD): the split-K partials of a weight gradient.
template <int KD, class LG, class LX>
__global__ void __launch_bounds__(kGemmThreads)
    k_gemm_wgrad(int64_t rows, LG G, LX X, float* __restrict__ part) {
  constexpr int LD = kTile + 8;
  __shared__ __align__(16) __bf16 sGt[kH * LD];
  __shared__ __align__(16) __bf16 sXt[KD * LD];
  f32x4 acc[KD / 64][4];
#pragma unroll
  for (int jc = 0; jc < KD / 64; ++jc)
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) acc[jc][jt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t ntiles = (rows + kTile - 1) / kTile;
  // the next tile's columns load into registers during this tile's MFMA
  ColsPrefetch<kH, LG> pg;
  ColsPrefetch<KD, LX> px;
  if (int64_t(blockIdx.x) < ntiles) {
    pg.fetch(G, int64_t(blockIdx.x) * kTile, rows);
    px.fetch(X, int64_t(blockIdx.x) * kTile, rows);
  }
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    pg.store(sGt, LD);
    px.store(sXt, LD);
    __syncthreads();
    if (tile + gridDim.x < ntiles) {
      pg.fetch(G, (tile + gridDim.x) * kTile, rows);
      px.fetch(X, (tile + gridDim.x) * kTile, rows);
    }
#pragma unroll
    for (int jc = 0; jc < KD / 64; ++jc) mfma_tile<kTile>(sGt, LD, sXt + jc * 64 * LD, LD, acc[jc]);
  }
  float* out = part + int64_t(blockIdx.x) * kH * KD;
#pragma unroll
  for (int jc = 0; jc < KD / 64; ++jc)
    tile_out(acc[jc], [&](int i, int j, float v) { out[i * KD + jc * 64 + j] = v; });
}

// out[j] = sum_b part[b * len + j], b ascending.
__global__ void k_reduce_part(int nparts, int64_t len, const float* __restrict__ part,
                              float* __restrict__ out) {
  int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= len) return;
  float acc = 0.f;
  for (int b = 0; b < nparts; ++b) acc += part[b * len + j];
  out[j] = acc;
}

// out[j] = sum_b part[b * len + j] for few outputs and many partials: one
// workgroup per output, a fixed-order strided sum and tree (deterministic).
// With split (NI >= 0), the partials of a small weight gradient with bias:
// outputs j = o * (NI + 1) + i go to W[o * NI + i] (i < NI) and b[o]
// (i == NI).
__global__ void __launch_bounds__(256)
    k_reduce_wide(int nparts, int64_t len, const float* __restrict__ part, float* __restrict__ out,
                  int NI, float* __restrict__ W, float* __restrict__ bias) {
  __shared__ float sm[256];
  const int64_t j = blockIdx.x;
  float acc = 0.f;
  for (int b = threadIdx.x; b < nparts; b += 256) acc += part[int64_t(b) * len + j];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (NI < 0) {
    out[j] = sm[0];
  } else {
    const int o = int(j) / (NI + 1), i = int(j) % (NI + 1);
    if (i < NI) W[o * NI + i] = sm[0];
    else bias[o] = sm[0];
  }
}

// Column sums of a [rows][64] array (bias gradients): partials per block.
__global__ void __launch_bounds__(256)
    k_colsum64(int64_t rows, const float* __restrict__ g, float* __restrict__ part) {
  const int o = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * per, hi = lo + per < rows ? lo + per : rows;
  float acc = 0.f;
  for (int64_t r = lo + q; r < hi; r += 4) acc += g[r * kH + o];
  __shared__ float sm[4][64];
  sm[q][o] = acc;
  __syncthreads();
  if (q == 0) part[blockIdx.x * kH + o] = sm[0][o] + sm[1][o] + sm[2][o] + sm[3][o];
}

// Small weight gradients (encoders, decoder): out[o][i] = sum_r G[r][o] IN[r][i]
// for o < NO, i < NI, plus out[o][NI] = sum_r G[r][o] when BIAS.  Partials
// per block ([NO][NI + BIAS] each).
template <int NO, int NI, bool BIAS>
__global__ void __launch_bounds__(256)
    k_wgrad_small(int64_t rows, const float* __restrict__ G, const float* __restrict__ IN,
                  float* __restrict__ part) {
  constexpr int NC = NI + (BIAS ? 1 : 0);
  constexpr int NOUT = NO * NC;
  constexpr int PER = (NOUT + 255) / 256;
  constexpr int CH = 32;  // rows staged per step
  __shared__ float sG[CH * NO];
  __shared__ float sI[CH * NI];
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * per, hi = lo + per < rows ? lo + per : rows;
  float acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = 0.f;
  for (int64_t r0 = lo; r0 < hi; r0 += CH) {
    const int nr = int(hi - r0 < CH ? hi - r0 : CH);
    __syncthreads();
    for (int i = threadIdx.x; i < CH * NO; i += 256)
      sG[i] = i / NO < nr ? G[(r0 + i / NO) * NO + i % NO] : 0.f;
    for (int i = threadIdx.x; i < CH * NI; i += 256)
      sI[i] = i / NI < nr ? IN[(r0 + i / NI) * NI + i % NI] : 0.f;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = threadIdx.x + 256 * u;
      if (t < NOUT) {
        const int o = t / NC, i = t % NC;
        float s = 0.f;
        for (int r = 0; r < CH; ++r) s += sG[r * NO + o] * (i < NI ? sI[r * NI + i] : 1.f);
        acc[u] += s;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + 256 * u;
    if (t < NOUT) part[int64_t(blockIdx.x) * NOUT + t] = acc[u];
  }
}

// ----------------------------------------------------------------- features
// Per edge (block b of row I, column J): row node, transposed edge.
__global__ void k_edge_index(int64_t N, const int32_t* __restrict__ bptr,
                             const int32_t* __restrict__ bcol, int32_t* __restrict__ erow,
                             int32_t* __restrict__ etr) {
  int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  for (int b = bptr[I]; b < bptr[I + 1]; ++b) {
    erow[b] = int(I);
    const int J = bcol[b];
    int lo = bptr[J], hi = bptr[J + 1] - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (bcol[mid] < I) lo = mid + 1;
      else hi = mid;
    }
    etr[b] = lo;
  }
}

// Position of K entry (3I+a, 3 bcol[b] + c) in the scalar-CSR value layout.
__device__ __forceinline__ int64_t kval_index(const int32_t* bptr, int I, int b, int a, int c) {
  const int rb = bptr[I], deg = bptr[I + 1] - rb;
  return 9 * int64_t(rb) + a * 3 * deg + 3 * (b - rb) + c;
}

// Block of the diagonal (I, I) in row I (every row has one: a node belongs
// to at least one face; the search stays inside the row regardless).
__device__ __forceinline__ int diag_slot(const int32_t* bptr, const int32_t* bcol, int I) {
  const int rb = bptr[I], deg = bptr[I + 1] - rb;
  int jj = 0;
  while (jj < deg - 1 && bcol[rb + jj] != I) ++jj;
  return rb + jj;
}

// Sum and count of the free diagonal entries (per-block partials).
__global__ void __launch_bounds__(256)
    k_diag_mean(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                const double* __restrict__ val, const uint8_t* __restrict__ fixed,
                double* __restrict__ part) {
  double v[2] = {0.0, 0.0};
  for (int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; I < N;
       I += int64_t(gridDim.x) * blockDim.x) {
    const int b = diag_slot(bptr, bcol, int(I));
    for (int a = 0; a < 3; ++a) {
      if (fixed && fixed[3 * I + a]) continue;
      v[0] += val[kval_index(bptr, int(I), b, a, a)];
      v[1] += 1.0;
    }
  }
  __shared__ double sm[2][4];
  for (int k = 0; k < 2; ++k) {
    const double s = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 2; ++k) part[2 * blockIdx.x + k] = sm[k][0] + sm[k][1] + sm[k][2] + sm[k][3];
}

// Sum of the off-diagonal edge lengths (per-block partials).
__global__ void __launch_bounds__(256)
    k_edge_length(int64_t nb, const int32_t* __restrict__ erow, const int32_t* __restrict__ bcol,
                  const double* __restrict__ xyz, double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < nb;
       b += int64_t(gridDim.x) * blockDim.x) {
    const int I = erow[b], J = bcol[b];
    if (I == J) continue;
    const double dx = xyz[3 * J] - xyz[3 * I], dy = xyz[3 * J + 1] - xyz[3 * I + 1],
                 dz = xyz[3 * J + 2] - xyz[3 * I + 2];
    acc += sqrt(dx * dx + dy * dy + dz * dz);
  }
  __shared__ double sm[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

// s = diag(K)^-1/2 and node features x [N][8].
__global__ void k_node_features(int64_t N, const int32_t* __restrict__ bptr,
                                const int32_t* __restrict__ bcol, const double* __restrict__ val,
                                const uint8_t* __restrict__ fixed, double dbar,
                                float* __restrict__ x, double* __restrict__ s,
                                float* __restrict__ s32) {
  int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int b = diag_slot(bptr, bcol, int(I));
  double K[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) K[a][c] = val[kval_index(bptr, int(I), b, a, c)];
  float* o = x + kFNode * I;
  o[0] = float(K[0][1] / sqrt(K[0][0] * K[1][1]));
  o[1] = float(K[0][2] / sqrt(K[0][0] * K[2][2]));
  o[2] = float(K[1][2] / sqrt(K[1][1] * K[2][2]));
  for (int a = 0; a < 3; ++a) {
    o[3 + a] = float(log(K[a][a] / dbar));
    const double si = 1.0 / sqrt(K[a][a]);
    s[3 * I + a] = si;
    s32[3 * I + a] = float(si);
  }
  o[6] = (fixed && (fixed[3 * I] || fixed[3 * I + 1] || fixed[3 * I + 2])) ? 1.f : 0.f;
  o[7] = 1.f;
}

// Edge features y [nb][12]: s_I K_IJ s_J (row-major), (p_J - p_I) / hbar.
__global__ void k_edge_features(int64_t nb, const int32_t* __restrict__ erow,
                                const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                                const double* __restrict__ val, const double* __restrict__ s,
                                const double* __restrict__ xyz, double inv_hbar,
                                float* __restrict__ y) {
  int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int I = erow[b], J = bcol[b];
  float* o = y + kFEdge * b;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c)
      o[3 * a + c] = float(s[3 * I + a] * val[kval_index(bptr, I, int(b), a, c)] * s[3 * J + c]);
  for (int a = 0; a < 3; ++a) o[9 + a] = float((xyz[3 * J + a] - xyz[3 * I + a]) * inv_hbar);
}

// ------------------------------------------------------------------ forward
// out[r][o] = relu(sum_i W[o][i] in[r][i] + b[o]), fan-in F (FP32: the
// encoders are too narrow for the matrix cores).
// Workgroups of the encoders: 16 rows each, up to 8,192.
inline int enc_grid(int64_t rows) {
  return int(std::max<int64_t>(1, std::min<int64_t>(div_up(rows, 16), 8192)));
}

// A thread computes four consecutive outputs of a row (one 16-byte store),
// its weights held in registers across a grid-stride loop over rows.
template <int F>
__global__ void __launch_bounds__(256)
    k_encode(int64_t rows, const float* __restrict__ in, const float* __restrict__ W,
             const float* __restrict__ b, float* __restrict__ out) {
  constexpr int kQ = kH / 4;  // threads per row
  const int o0 = 4 * (threadIdx.x % kQ);
  float w[4][F], bias[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    bias[c] = b[o0 + c];
#pragma unroll
    for (int i = 0; i < F; ++i) w[c][i] = W[(o0 + c) * F + i];
  }
  const int64_t stride = int64_t(gridDim.x) * (blockDim.x / kQ);
  for (int64_t r = int64_t(blockIdx.x) * (blockDim.x / kQ) + threadIdx.x / kQ; r < rows;
       r += stride) {
    float x[F];
#pragma unroll
    for (int i = 0; i < F; ++i) x[i] = in[r * F + i];
    float acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      acc[c] = bias[c];
#pragma unroll
      for (int i = 0; i < F; ++i) acc[c] += w[c][i] * x[i];
    }
    *reinterpret_cast<float4*>(out + r * kH + o0) =
        make_float4(relu(acc[0]), relu(acc[1]), relu(acc[2]), relu(acc[3]));
  }
}

// Edge layer epilogue: z = y + b;  e_out = e_in + relu(z).
struct EdgeFwdEpi {
  const float* __restrict__ bias;
  const float* __restrict__ e_in;
  float* __restrict__ z;
  float* __restrict__ e_out;
  __device__ __forceinline__ float pre(int64_t b, int o) const { return e_in[b * kH + o]; }
  __device__ __forceinline__ void operator()(int64_t b, int o, float v, float ein) const {
    const float zz = v + bias[o];
    z[b * kH + o] = zz;
    e_out[b * kH + o] = ein + relu(zz);
  }
};

// Node layer epilogue: t = y + c;  h_out = h_in + relu(t).
struct NodeFwdEpi {
  const float* __restrict__ bias;
  const float* __restrict__ h_in;
  float* __restrict__ t;
  float* __restrict__ h_out;
  __device__ __forceinline__ float pre(int64_t I, int o) const { return h_in[I * kH + o]; }
  __device__ __forceinline__ void operator()(int64_t I, int o, float v, float hin) const {
    const float tt = v + bias[o];
    t[I * kH + o] = tt;
    h_out[I * kH + o] = hin + relu(tt);
  }
};

// a_I = mean over the edges of row I of relu(z).  One wave per node.
__global__ void k_aggregate(int64_t N, const int32_t* __restrict__ bptr,
                            const float* __restrict__ z, float* __restrict__ a) {
  const int lane = threadIdx.x & 63;
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
  if (I >= N) return;
  float acc = 0.f;
  for (int b = bptr[I]; b < bptr[I + 1]; ++b) acc += relu(z[int64_t(b) * kH + lane]);
  a[I * kH + lane] = acc / float(bptr[I + 1] - bptr[I]);
}

// R_IJ = Wo e_IJ (3x3 row-major per edge): a thread per edge, its row of e
// read once with 16-byte loads, Wo from LDS.
__global__ void __launch_bounds__(256)
    k_decode(int64_t nb, const float* __restrict__ e, const float* __restrict__ Wo,
             float* __restrict__ R) {
  __shared__ float sWo[9 * kH];
  for (int i = threadIdx.x; i < 9 * kH; i += blockDim.x) sWo[i] = Wo[i];
  __syncthreads();
  for (int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < nb;
       b += int64_t(gridDim.x) * blockDim.x) {
    float acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.f;
    const float4* row = reinterpret_cast<const float4*>(e + b * kH);
#pragma unroll 4
    for (int i4 = 0; i4 < kH / 4; ++i4) {
      const float4 v = row[i4];
      const float ev[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[q] += sWo[q * kH + 4 * i4 + u] * ev[u];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) R[b * 9 + q] = acc[q];
  }
}

// S'_IJ = (R_IJ + R_JI^T) / 2, zero on fixed DOFs, into the scalar-CSR layout.
__global__ void k_symmetrize(int64_t nb, const int32_t* __restrict__ erow,
                             const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                             const int32_t* __restrict__ etr, const uint8_t* __restrict__ fixed,
                             const float* __restrict__ R, float* __restrict__ mval) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nb * 9) return;
  const int64_t b = t / 9;
  const int a = int(t % 9) / 3, c = int(t % 9) % 3;
  const int I = erow[b], J = bcol[b];
  float v = 0.5f * (R[t] + R[int64_t(etr[b]) * 9 + 3 * c + a]);
  if (fixed && (fixed[3 * I + a] || fixed[3 * J + c])) v = 0.f;
  mval[kval_index(bptr, I, int(b), a, c)] = v;
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ in, __bf16* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = __bf16(in[i]);
}

// ----------------------------------------------------------------- the loss
// Minibatch panels [3N][B]: r, e of the pairs ids[p], and rh = s r.
__global__ void k_gather_pairs(int64_t n, int B, const int32_t* __restrict__ ids,
                               const float* __restrict__ pr, const float* __restrict__ pe,
                               const double* __restrict__ s, float* __restrict__ br,
                               float* __restrict__ be, float* __restrict__ brh) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * B) return;
  const int64_t i = t / B;
  const int p = int(t % B);
  const int64_t src = int64_t(ids[p]) * n + i;
  const float r = pr[src];
  br[t] = r;
  be[t] = pe[src];
  brh[t] = float(s[i] * double(r));
}

// out = A in for a [3N][B] panel; A in the scalar-CSR value layout of K.
template <typename VT>
__global__ void k_spmm(int64_t N, const int32_t* __restrict__ bptr,
                       const int32_t* __restrict__ bcol, const VT* __restrict__ val, int B,
                       const float* __restrict__ in, float* __restrict__ out) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 3 * N * B) return;
  const int64_t i = t / B;
  const int p = int(t % B);
  const int64_t I = i / 3;
  const int a = int(i % 3);
  const int rb = bptr[I], deg = bptr[I + 1] - rb;
  const VT* v = val + 9 * int64_t(rb) + a * 3 * deg;
  double acc = 0.0;
  for (int jj = 0; jj < deg; ++jj) {
    const int64_t J = bcol[rb + jj];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc += double(v[3 * jj + c]) * double(in[(3 * J + c) * B + p]);
  }
  out[t] = float(acc);
}

// w = s (rh + S' rh) - e   (M r - e), in place of the S' rh panel.
__global__ void k_loss_w(int64_t n, int B, const double* __restrict__ s,
                         const float* __restrict__ brh, const float* __restrict__ be,
                         float* __restrict__ w) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * B) return;
  const int64_t i = t / B;
  w[t] = float(s[i] * (double(brh[t]) + double(w[t])) - double(be[t]));
}

// Per-pair partial dot products sum_i x[i][p] y[i][p] (per block).
__global__ void __launch_bounds__(256)
    k_panel_dot(int64_t n, int B, const float* __restrict__ x, const float* __restrict__ y,
                double* __restrict__ part) {
  __shared__ double sm[256];
  const int nq = 256 / B;
  const int p = threadIdx.x % B, q = threadIdx.x / B;
  double acc = 0.0;
  if (q < nq)
    for (int64_t i = int64_t(blockIdx.x) * nq + q; i < n; i += int64_t(gridDim.x) * nq)
      acc += double(x[i * B + p]) * double(y[i * B + p]);
  sm[threadIdx.x] = acc;
  __syncthreads();
  if (int(threadIdx.x) < B) {
    double s = 0.0;
    for (int k = 0; k < nq; ++k) s += sm[k * B + threadIdx.x];
    part[int64_t(blockIdx.x) * B + threadIdx.x] = s;
  }
}

// gh = s * 2 K w / (den_p B)   (dL/dy, y = rh + S' rh), in place of K w.
__global__ void k_loss_gh(int64_t n, int B, const double* __restrict__ s,
                          const double* __restrict__ den, float* __restrict__ kw) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * B) return;
  const int64_t i = t / B;
  const int p = int(t % B);
  kw[t] = float(s[i] * 2.0 * double(kw[t]) / (den[p] * double(B)));
}

// dS'_IJ[a][c] = sum_p gh[3I+a][p] rh[3J+c][p], zero on fixed DOFs.  One
// thread per (edge, a).
__global__ void k_dS(int64_t nb, int B, const int32_t* __restrict__ erow,
                     const int32_t* __restrict__ bcol, const uint8_t* __restrict__ fixed,
                     const float* __restrict__ gh, const float* __restrict__ rh,
                     float* __restrict__ dS) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nb * 3) return;
  const int64_t b = t / 3;
  const int a = int(t % 3);
  const int64_t I = erow[b], J = bcol[b];
  const float* g = gh + (3 * I + a) * B;
  const float* r0 = rh + (3 * J) * B;
  float acc[3] = {0.f, 0.f, 0.f};
  for (int p = 0; p < B; ++p) {
    const float gp = g[p];
    acc[0] += gp * r0[p];
    acc[1] += gp * r0[B + p];
    acc[2] += gp * r0[2 * B + p];
  }
  const bool fa = fixed && fixed[3 * I + a];
  for (int c = 0; c < 3; ++c) {
    const bool off = fa || (fixed && fixed[3 * J + c]);
    dS[b * 9 + 3 * a + c] = off ? 0.f : acc[c];
  }
}

// dR_IJ = (dS_IJ + dS_JI^T) / 2.
__global__ void k_dR(int64_t nb, const int32_t* __restrict__ etr, const float* __restrict__ dS,
                     float* __restrict__ dR) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nb * 9) return;
  const int64_t b = t / 9;
  const int a = int(t % 9) / 3, c = int(t % 9) % 3;
  dR[t] = 0.5f * (dS[t] + dS[int64_t(etr[b]) * 9 + 3 * c + a]);
}

// ----------------------------------------------------------------- backward
// de_L = dR Wo  ([nb][9] x [9][64]).
__global__ void k_decode_bwd(int64_t nb, const float* __restrict__ dR, const float* __restrict__ Wo,
                             float* __restrict__ de) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nb * kH) return;
  const int64_t b = t / kH;
  const int o = int(t % kH);
  float acc = 0.f;
#pragma unroll
  for (int q = 0; q < 9; ++q) acc += dR[b * 9 + q] * Wo[q * kH + o];
  de[t] = acc;
}

// out = g * (pre > 0)  (ReLU backward; pre = t, z, or a ReLU output).
__global__ void k_relu_bwd(int64_t n, const float* __restrict__ g, const float* __restrict__ pre,
                           float* __restrict__ out) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) out[t] = pre[t] > 0.f ? g[t] : 0.f;
}

// dz = (de + da_I / deg_I) * (z > 0)  for edge (I, J).
__global__ void k_dz(int64_t nb, const int32_t* __restrict__ erow, const int32_t* __restrict__ bptr,
                     const float* __restrict__ de, const float* __restrict__ da,
                     const float* __restrict__ z, float* __restrict__ dz) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nb * kH) return;
  const int64_t b = t / kH;
  const int o = int(t % kH);
  const int I = erow[b];
  const float inv_deg = 1.f / float(bptr[I + 1] - bptr[I]);
  dz[t] = z[t] > 0.f ? de[t] + da[int64_t(I) * kH + o] * inv_deg : 0.f;
}

// Node-layer backward epilogue of dY = dt U: dh += dY[:, :64]; da = dY[:, 64:].
struct NodeBwdEpi {
  float* __restrict__ dh;
  float* __restrict__ da;
  __device__ __forceinline__ void operator()(int64_t I, int j, float v) const {
    if (j < kH) dh[I * kH + j] += v;
    else da[I * kH + (j - kH)] = v;
  }
};

// Edge-layer backward epilogue of dX = dz W: the h_I, h_J parts go to dXh
// (summed per node afterwards); de += dX[:, 128:].
struct EdgeBwdEpi {
  float* __restrict__ dXh;
  float* __restrict__ de;
  __device__ __forceinline__ void operator()(int64_t b, int j, float v) const {
    if (j < 2 * kH) dXh[b * 2 * kH + j] = v;
    else de[b * kH + (j - 2 * kH)] += v;
  }
};

// dh_I += sum over the edges b of row I of dXh[b][:64] (I as the row end)
// + dXh[tr(b)][64:] (I as the column end of the transposed edge).
__global__ void k_dh_gather(int64_t N, const int32_t* __restrict__ bptr,
                            const int32_t* __restrict__ etr, const float* __restrict__ dXh,
                            float* __restrict__ dh) {
  const int lane = threadIdx.x & 63;
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
  if (I >= N) return;
  float acc = 0.f;
  for (int b = bptr[I]; b < bptr[I + 1]; ++b)
    acc += dXh[int64_t(b) * 2 * kH + lane] + dXh[int64_t(etr[b]) * 2 * kH + kH + lane];
  dh[I * kH + lane] += acc;
}

// ------------------------------------------------------------------- Adam
__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_fill_f32(int64_t n, float v, float* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

__global__ void k_fill_f64(int64_t n, double v, double* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

// ------------------------------------------------------------------ pairs
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// b_i = scale * u_i, u uniform in [-1, 1) from a counter hash; 0 if fixed.
__global__ void k_random_load(int64_t n, uint64_t key, double scale,
                              const uint8_t* __restrict__ fixed, double* __restrict__ b) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double u = double(mix64(key ^ mix64(uint64_t(i))) >> 11) * (1.0 / 9007199254740992.0);
  b[i] = (fixed && fixed[i]) ? 0.0 : scale * (2.0 * u - 1.0);
}

// x *= sqrt(dinv)  (dinv = 1 / diag(K)).
__global__ void k_scale_by(int64_t n, const double* __restrict__ dinv, double* __restrict__ x) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= sqrt(dinv[i]);
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ in, float* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = float(in[i]);
}

// Partial sums of a . b (FP64, per block); a and b FP64 or FP32.
template <typename A, typename B>
__global__ void __launch_bounds__(256)
    k_dot(int64_t n, const A* __restrict__ a, const B* __restrict__ b, double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    acc += double(a[i]) * double(b[i]);
  __shared__ double sm[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

// Lanczos step: w -= alpha v + beta u, then (separately) u = v, v = w / |w|.
__global__ void k_lanczos_w(int64_t n, double alpha, double beta, const double* __restrict__ v,
                            const double* __restrict__ u, double* __restrict__ w) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) w[i] -= alpha * v[i] + beta * u[i];
}

__global__ void k_lanczos_next(int64_t n, double inv_beta, const double* __restrict__ w,
                               double* __restrict__ v, double* __restrict__ u) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    u[i] = v[i];
    v[i] = w[i] * inv_beta;
  }
}

__global__ void k_scale_f64(int64_t n, double a, double* __restrict__ x) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= a;
}

__global__ void k_scale_f32(int64_t n, float a, float* __restrict__ x) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= a;
}

// Number of eigenvalues below x of the symmetric tridiagonal (a, b)
// (Sturm sequence; b[j] couples j-1 and j).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t j = 0; j < a.size(); ++j) {
    const double off = j ? b[j] * b[j] : 0.0;
    q = a[j] - x - (j ? off / q : 0.0);
    if (q == 0.0) q = 1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// Smallest (k = 0) or largest (k = n-1) eigenvalue of the tridiagonal, by
// bisection inside its Gershgorin interval.
double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
  double lo = 1e300, hi = -1e300;
  for (size_t j = 0; j < a.size(); ++j) {
    const double r = (j ? std::fabs(b[j]) : 0.0) + (j + 1 < a.size() ? std::fabs(b[j + 1]) : 0.0);
    lo = std::min(lo, a[j] - r);
    hi = std::max(hi, a[j] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, mid) > k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

int grid_for(int64_t items, int per_block, int cap) {
  const int64_t g = (items + per_block - 1) / per_block;
  return int(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

int tile_grid(int64_t rows, int cap) { return grid_for((rows + kTile - 1) / kTile, 1, cap); }

// Sums per-block double partials on the host (fixed order).
std::vector<double> host_sum(hipStream_t s, const double* dpart, int nblocks, int width) {
  std::vector<double> h(size_t(nblocks) * width), out(width, 0.0);
  SFEM_HIP(hipMemcpyAsync(h.data(), dpart, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  SFEM_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < nblocks; ++b)
    for (int k = 0; k < width; ++k) out[k] += h[size_t(b) * width + k];
  return out;
}

template <typename A, typename B>
double dot(Ctx& c, const A* a, const B* b, int64_t n) {
  GnnWork& w = gnn_work(c);
  w.part.reserve(2 * kRedGrid);
  const int g = grid_for(n, 256, kRedGrid);
  k_dot<A, B><<<g, 256, 0, c.stream>>>(n, a, b, w.part.get());
  SFEM_HIP(hipGetLastError());
  return host_sum(c.stream, w.part.get(), g, 1)[0];
}

}  // namespace

// ============================================================== host side
const ParamLayout& param_layout() {
  static const ParamLayout L = [] {
    ParamLayout p{};
    int64_t o = 0;
    auto put = [&](int64_t n) {
      const int64_t r = o;
      o += n;
      return r;
    };
    p.Wn = put(kH * kFNode);
    p.bn = put(kH);
    p.We = put(kH * kFEdge);
    p.be = put(kH);
    for (int l = 0; l < kLayers; ++l) {
      p.W[l] = put(kH * 3 * kH);
      p.b[l] = put(kH);
      p.U[l] = put(kH * 2 * kH);
      p.c[l] = put(kH);
    }
    p.Wo = put(9 * kH);
    p.total = o;
    return p;
  }();
  return L;
}

GnnWork& gnn_work(Ctx& c) {
  if (!c.gnn) c.gnn = std::make_shared<GnnWork>();
  return *c.gnn;
}

void gnn_features(Ctx& c) {
  ensure_csr64(c);  // the features read K in CSR order
  SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "assemble K first");
  GnnWork& w = gnn_work(c);
  const Topology& tp = c.topo;
  const int64_t N = c.N, nb = tp.nb;
  hipStream_t s = c.stream;
  if (w.have_features && w.N == N && w.nb == nb) return;
  SFEM_REQUIRE(nb > N, SFEM_EMESH, "the mesh has no edges");
  w.N = N;
  w.nb = nb;
  w.erow.reserve(nb);
  w.etr.reserve(nb);
  w.x.reserve(N * kFNode);
  w.y.reserve(nb * kFEdge);
  w.s.reserve(3 * N);
  w.part.reserve(2 * kRedGrid);
  c.msqrt.reserve(3 * N);
  c.msqrt32.reserve(3 * N);
  k_edge_index<<<div_up(N, 256), 256, 0, s>>>(N, tp.bptr.get(), tp.bcol.get(), w.erow.get(),
                                               w.etr.get());
  const uint8_t* fixed = c.any_fixed ? c.fixed.get() : nullptr;
  const int g1 = grid_for(N, 256, kRedGrid);
  k_diag_mean<<<g1, 256, 0, s>>>(N, tp.bptr.get(), tp.bcol.get(), c.val.get(), fixed,
                                 w.part.get());
  SFEM_HIP(hipGetLastError());
  const std::vector<double> dm = host_sum(s, w.part.get(), g1, 2);
  const double dbar = dm[1] > 0 ? dm[0] / dm[1] : 1.0;
  k_node_features<<<div_up(N, 256), 256, 0, s>>>(N, tp.bptr.get(), tp.bcol.get(), c.val.get(),
                                                 fixed, dbar, w.x.get(), c.msqrt.get(),
                                                 c.msqrt32.get());
  SFEM_HIP(hipMemcpyAsync(w.s.get(), c.msqrt.get(), sizeof(double) * 3 * N,
                          hipMemcpyDeviceToDevice, s));
  const int g2 = grid_for(nb, 256, kRedGrid);
  k_edge_length<<<g2, 256, 0, s>>>(nb, w.erow.get(), tp.bcol.get(), c.xyz.get(), w.part.get());
  SFEM_HIP(hipGetLastError());
  const double hbar = host_sum(s, w.part.get(), g2, 1)[0] / double(nb - N);
  k_edge_features<<<div_up(nb, 256), 256, 0, s>>>(nb, w.erow.get(), tp.bptr.get(), tp.bcol.get(),
                                                  c.val.get(), w.s.get(), c.xyz.get(),
                                                  1.0 / hbar, w.y.get());
  SFEM_HIP(hipGetLastError());
  w.have_features = true;
}

void gnn_forward(Ctx& c, Gnn& g, bool keep) {
  gnn_features(c);
  GnnWork& w = gnn_work(c);
  const Topology& tp = c.topo;
  const int64_t N = c.N, nb = tp.nb;
  hipStream_t s = c.stream;
  const ParamLayout& L = param_layout();
  const int nst = keep ? kLayers + 1 : 2;  // stored layer states
  const int nzl = keep ? kLayers : 1;
  w.h.reserve(nst * N * kH);
  w.e.reserve(nst * nb * kH);
  w.z.reserve(nzl * nb * kH);
  w.t.reserve(nzl * N * kH);
  w.a.reserve(nzl * N * kH);
  w.dS.reserve(nb * 9);  // holds R in the forward pass
  c.mval.reserve(9 * nb);
  const float* P = g.params.get();
  k_to_bf16<<<div_up(L.total, 256), 256, 0, s>>>(L.total, P, g.params_bf16.get());
  const __bf16* Pb = g.params_bf16.get();
  k_encode<kFNode><<<enc_grid(N), 256, 0, s>>>(N, w.x.get(), P + L.Wn, P + L.bn,
                                                       w.h.get());
  k_encode<kFEdge><<<enc_grid(nb), 256, 0, s>>>(nb, w.y.get(), P + L.We, P + L.be,
                                                        w.e.get());
  SFEM_HIP(hipGetLastError());
  const int ge = tile_grid(nb, kGemmGrid), gn = tile_grid(N, kGemmGrid);
  for (int l = 0; l < kLayers; ++l) {
    const int si = keep ? l : (l & 1), so = keep ? l + 1 : ((l + 1) & 1);
    const int zi = keep ? l : 0;
    float* h_in = w.h.get() + si * N * kH;
    float* h_out = w.h.get() + so * N * kH;
    float* e_in = w.e.get() + si * nb * kH;
    float* e_out = w.e.get() + so * nb * kH;
    float* z = w.z.get() + zi * nb * kH;
    float* t = w.t.get() + zi * N * kH;
    float* a = w.a.get() + zi * N * kH;
    k_gemm_xwT<3 * kH><<<ge, kGemmThreads, 0, s>>>(
        nb, EdgeX{w.erow.get(), tp.bcol.get(), h_in, e_in}, Pb + L.W[l],
        EdgeFwdEpi{P + L.b[l], e_in, z, e_out});
    k_aggregate<<<div_up(N * 64, 256), 256, 0, s>>>(N, tp.bptr.get(), z, a);
    k_gemm_xwT<2 * kH><<<gn, kGemmThreads, 0, s>>>(N, NodeY{h_in, a}, Pb + L.U[l],
                                                    NodeFwdEpi{P + L.c[l], h_in, t, h_out});
    SFEM_HIP(hipGetLastError());
  }
  const int sl = keep ? kLayers : (kLayers & 1);
  k_decode<<<int(std::max<int64_t>(1, std::min<int64_t>(div_up(nb, 256), 8192))), 256, 0, s>>>(
      nb, w.e.get() + sl * nb * kH, P + L.Wo,
                                               w.dS.get());
  k_symmetrize<<<div_up(nb * 9, 256), 256, 0, s>>>(
      nb, w.erow.get(), tp.bptr.get(), tp.bcol.get(), w.etr.get(),
      c.any_fixed ? c.fixed.get() : nullptr, w.dS.get(), c.mval.get());
  SFEM_HIP(hipGetLastError());
  c.have_learned = false;  // S is raw until gnn_precondition scales it
}

void gnn_precondition(Ctx& c, Gnn& g) {
  gnn_forward(c, g, false);
  const int64_t n = c.n_dof();
  hipStream_t s = c.stream;
  // Lanczos on the symmetric S from a fixed pseudo-random start
  DBuf<double> v, u, w;
  v.reserve(n);
  u.reserve(n);
  w.reserve(n);
  k_random_load<<<div_up(n, 256), 256, 0, s>>>(n, 0x5eedull, 1.0, nullptr, v.get());
  k_fill_f64<<<div_up(n, 256), 256, 0, s>>>(n, 0.0, u.get());
  SFEM_HIP(hipGetLastError());
  const double v0 = std::sqrt(dot(c, v.get(), v.get(), n));
  k_scale_f64<<<div_up(n, 256), 256, 0, s>>>(n, 1.0 / v0, v.get());
  std::vector<double> al, be{0.0};
  for (int j = 0; j < kLanczosSteps; ++j) {
    spmv_f32val(c, c.mval.get(), v.get(), w.get(), s);
    const double a = dot(c, w.get(), v.get(), n);
    k_lanczos_w<<<div_up(n, 256), 256, 0, s>>>(n, a, be.back(), v.get(), u.get(), w.get());
    SFEM_HIP(hipGetLastError());
    al.push_back(a);
    const double b = std::sqrt(dot(c, w.get(), w.get(), n));
    if (!(b > 1e-12 * std::fabs(a)) || !std::isfinite(b)) break;  // invariant subspace
    be.push_back(b);
    k_lanczos_next<<<div_up(n, 256), 256, 0, s>>>(n, 1.0 / b, w.get(), v.get(), u.get());
  }
  be.resize(al.size());
  bool finite = true;
  for (double a : al) finite = finite && std::isfinite(a);
  c.m_lmin = finite ? tridiag_eig(al, be, 0) : NAN;
  c.m_lmax = finite ? tridiag_eig(al, be, int(al.size()) - 1) : NAN;
  double theta = 1.0;
  if (finite && c.m_lmin < 0.0) theta = std::min(1.0, 0.9 / (1.05 * -c.m_lmin));
  c.m_theta = theta;
  if (theta < 1.0) {
    k_scale_f32<<<div_up(9 * c.topo.nb, 256), 256, 0, s>>>(9 * c.topo.nb, float(theta),
                                                            c.mval.get());
    SFEM_HIP(hipGetLastError());
  }
  // packed copy for the solver's M apply
  pack_pattern(c);
  c.mvalp.reserve(9 * c.nb4);
  pack_values_bf16(c, c.mval.get(), c.mvalp.get());
  build_mgroups(c);
  SFEM_HIP(hipStreamSynchronize(s));
  c.have_learned = true;
}

double gnn_loss_grad(Ctx& c, Gnn& g, const int32_t* ids, int B, bool grad) {
  ensure_csr64(c);  // K (M r - e) in CSR order
  GnnWork& w = gnn_work(c);
  SFEM_REQUIRE(w.n_pairs > 0, SFEM_ESTATE, "no training pairs on this context");
  SFEM_REQUIRE(B >= 1 && B <= kMaxBatch, SFEM_EINVAL, "batch size must be in [1, 64]");
  for (int p = 0; p < B; ++p)
    SFEM_REQUIRE(ids[p] >= 0 && ids[p] < w.n_pairs, SFEM_EINVAL, "pair index out of range");
  gnn_forward(c, g, grad);
  const Topology& tp = c.topo;
  const int64_t N = c.N, nb = tp.nb, n = 3 * N;
  hipStream_t s = c.stream;
  const ParamLayout& L = param_layout();
  const float* P = g.params.get();
  const __bf16* Pb = g.params_bf16.get();
  float* G = g.grad.get();

  // ---- loss: L = mean_p (Mr - e).K(Mr - e) / (e.K e)
  w.bidx.reserve(kMaxBatch);
  w.bpart.reserve(size_t(kRedGrid) * kMaxBatch + kMaxBatch);
  for (auto* b : {&w.br, &w.be, &w.bw, &w.bkw, &w.brh}) b->reserve(n * B);
  SFEM_HIP(hipMemcpyAsync(w.bidx.get(), ids, sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
  const int64_t nB = n * B;
  k_gather_pairs<<<div_up(nB, 256), 256, 0, s>>>(n, B, w.bidx.get(), w.pr.get(), w.pe.get(),
                                                 w.s.get(), w.br.get(), w.be.get(), w.brh.get());
  k_spmm<float><<<div_up(nB, 256), 256, 0, s>>>(N, tp.bptr.get(), tp.bcol.get(), c.mval.get(), B,
                                                w.brh.get(), w.bw.get());
  k_loss_w<<<div_up(nB, 256), 256, 0, s>>>(n, B, w.s.get(), w.brh.get(), w.be.get(), w.bw.get());
  k_spmm<double><<<div_up(nB, 256), 256, 0, s>>>(N, tp.bptr.get(), tp.bcol.get(), c.val.get(),
                                                 B, w.bw.get(), w.bkw.get());
  const int gd = grid_for(n, 256 / B, kRedGrid);
  k_panel_dot<<<gd, 256, 0, s>>>(n, B, w.bw.get(), w.bkw.get(), w.bpart.get());
  SFEM_HIP(hipGetLastError());
  const std::vector<double> num = host_sum(s, w.bpart.get(), gd, B);
  std::vector<double> den(B);
  double loss = 0.0;
  for (int p = 0; p < B; ++p) {
    den[p] = w.pden[ids[p]];
    loss += num[p] / den[p];
  }
  loss /= B;
  if (!grad) return loss;

  // ---- dL/dS' and the symmetrisation
  double* dden = w.bpart.get() + size_t(kRedGrid) * kMaxBatch;
  SFEM_HIP(hipMemcpyAsync(dden, den.data(), sizeof(double) * B, hipMemcpyHostToDevice, s));
  k_loss_gh<<<div_up(nB, 256), 256, 0, s>>>(n, B, w.s.get(), dden, w.bkw.get());
  w.dS.reserve(nb * 9);
  w.de.reserve(nb * kH);
  w.dz.reserve(nb * kH);
  w.dXh.reserve(nb * 2 * kH);
  w.dh.reserve(N * kH);
  w.dt.reserve(N * kH);
  w.da.reserve(N * kH);
  float* dR = w.dz.get();  // [nb][9] scratch before dz is needed
  k_dS<<<div_up(nb * 3, 256), 256, 0, s>>>(nb, B, w.erow.get(), tp.bcol.get(),
                                           c.any_fixed ? c.fixed.get() : nullptr, w.bkw.get(),
                                           w.brh.get(), w.dS.get());
  k_dR<<<div_up(nb * 9, 256), 256, 0, s>>>(nb, w.etr.get(), w.dS.get(), dR);
  SFEM_HIP(hipGetLastError());

  // ---- decoder
  static_assert(size_t(kColGrid) * kH * (kFEdge + 1) <= size_t(kWgradGrid) * kH * 3 * kH,
                "partials of the small reductions fit the weight-gradient buffer");
  g.wpart.reserve(size_t(kWgradGrid) * kH * 3 * kH);
  float* part = g.wpart.get();
  const float* eL = w.e.get() + kLayers * nb * kH;
  const int gs = grid_for(nb, 256, kColGrid);
  k_wgrad_small<9, kH, false><<<gs, 256, 0, s>>>(nb, dR, eL, part);
  k_reduce_wide<<<9 * kH, 256, 0, s>>>(gs, 9 * kH, part, G + L.Wo, -1, nullptr, nullptr);
  k_decode_bwd<<<div_up(nb * kH, 256), 256, 0, s>>>(nb, dR, P + L.Wo, w.de.get());
  k_fill_f32<<<div_up(N * kH, 256), 256, 0, s>>>(N * kH, 0.f, w.dh.get());
  SFEM_HIP(hipGetLastError());

  // ---- message-passing layers, last first
  const int ge = tile_grid(nb, kGemmGrid), gn = tile_grid(N, kGemmGrid);
  const int gwe = tile_grid(nb, kWgradGrid), gwn = tile_grid(N, kWgradGrid);
  const int gce = grid_for(nb, 256, kColGrid), gcn = grid_for(N, 256, kColGrid);
  for (int l = kLayers - 1; l >= 0; --l) {
    const float* h_l = w.h.get() + l * N * kH;
    const float* e_l = w.e.get() + l * nb * kH;
    const float* z_l = w.z.get() + l * nb * kH;
    const float* t_l = w.t.get() + l * N * kH;
    const float* a_l = w.a.get() + l * N * kH;
    // node update h += relu(U [h; a] + c)
    k_relu_bwd<<<div_up(N * kH, 256), 256, 0, s>>>(N * kH, w.dh.get(), t_l, w.dt.get());
    k_gemm_wgrad<2 * kH><<<gwn, kGemmThreads, 0, s>>>(N, Rows64{w.dt.get()}, NodeY{h_l, a_l},
                                                       part);
    k_reduce_part<<<div_up(kH * 2 * kH, 256), 256, 0, s>>>(gwn, kH * 2 * kH, part, G + L.U[l]);
    k_colsum64<<<gcn, 256, 0, s>>>(N, w.dt.get(), part);
    k_reduce_wide<<<kH, 256, 0, s>>>(gcn, kH, part, G + L.c[l], -1, nullptr, nullptr);
    k_gemm_xw<2 * kH><<<gn, kGemmThreads, 0, s>>>(N, Rows64{w.dt.get()}, Pb + L.U[l],
                                                   NodeBwdEpi{w.dh.get(), w.da.get()});
    // edge update e += relu(W [h_I; h_J; e] + b), a = mean relu(z)
    k_dz<<<div_up(nb * kH, 256), 256, 0, s>>>(nb, w.erow.get(), tp.bptr.get(), w.de.get(),
                                              w.da.get(), z_l, w.dz.get());
    k_gemm_wgrad<3 * kH><<<gwe, kGemmThreads, 0, s>>>(
        nb, Rows64{w.dz.get()}, EdgeX{w.erow.get(), tp.bcol.get(), h_l, e_l}, part);
    k_reduce_part<<<div_up(kH * 3 * kH, 256), 256, 0, s>>>(gwe, kH * 3 * kH, part, G + L.W[l]);
    k_colsum64<<<gce, 256, 0, s>>>(nb, w.dz.get(), part);
    k_reduce_wide<<<kH, 256, 0, s>>>(gce, kH, part, G + L.b[l], -1, nullptr, nullptr);
    k_gemm_xw<3 * kH><<<ge, kGemmThreads, 0, s>>>(nb, Rows64{w.dz.get()}, Pb + L.W[l],
                                                   EdgeBwdEpi{w.dXh.get(), w.de.get()});
    k_dh_gather<<<div_up(N * 64, 256), 256, 0, s>>>(N, tp.bptr.get(), w.etr.get(), w.dXh.get(),
                                                    w.dh.get());
    SFEM_HIP(hipGetLastError());
  }

  // ---- encoders
  k_relu_bwd<<<div_up(nb * kH, 256), 256, 0, s>>>(nb * kH, w.de.get(), w.e.get(), w.dz.get());
  k_wgrad_small<kH, kFEdge, true><<<gs, 256, 0, s>>>(nb, w.dz.get(), w.y.get(), part);
  k_reduce_wide<<<kH * (kFEdge + 1), 256, 0, s>>>(gs, kH * (kFEdge + 1), part, nullptr, kFEdge,
                                                  G + L.We, G + L.be);
  const int gsn = grid_for(N, 256, kColGrid);
  k_relu_bwd<<<div_up(N * kH, 256), 256, 0, s>>>(N * kH, w.dh.get(), w.h.get(), w.dt.get());
  k_wgrad_small<kH, kFNode, true><<<gsn, 256, 0, s>>>(N, w.dt.get(), w.x.get(), part);
  k_reduce_wide<<<kH * (kFNode + 1), 256, 0, s>>>(gsn, kH * (kFNode + 1), part, nullptr, kFNode,
                                                  G + L.Wn, G + L.bn);
  SFEM_HIP(hipGetLastError());
  return loss;
}

void gnn_init_params(Gnn& g, uint64_t seed) {
  const ParamLayout& L = param_layout();
  std::vector<float> h(L.total, 0.f);
  uint64_t st = seed;
  auto uni = [&]() {  // splitmix64 stream, 53-bit uniform in [0, 1)
    st += 0x9e3779b97f4a7c15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return double(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto glorot = [&](int64_t off, int fan_in, int fan_out) {
    const double lim = std::sqrt(6.0 / (fan_in + fan_out));
    for (int64_t i = 0; i < int64_t(fan_in) * fan_out; ++i)
      h[off + i] = float((2.0 * uni() - 1.0) * lim);
  };
  glorot(L.Wn, kFNode, kH);
  glorot(L.We, kFEdge, kH);
  for (int l = 0; l < kLayers; ++l) {
    glorot(L.W[l], 3 * kH, kH);
    glorot(L.U[l], 2 * kH, kH);
  }
  // biases and the decoder start at zero: the untrained M is Jacobi
  const std::vector<float> zero(L.total, 0.f);
  SFEM_HIP(hipMemcpy(g.params.get(), h.data(), sizeof(float) * L.total, hipMemcpyHostToDevice));
  SFEM_HIP(hipMemcpy(g.adam_m.get(), zero.data(), sizeof(float) * L.total, hipMemcpyHostToDevice));
  SFEM_HIP(hipMemcpy(g.adam_v.get(), zero.data(), sizeof(float) * L.total, hipMemcpyHostToDevice));
  g.adam_t = 0;
}

void gnn_adam(Gnn& g, hipStream_t s, double lr, double beta1, double beta2, double eps) {
  const int64_t n = param_layout().total;
  g.adam_t += 1;
  const float c1 = float(1.0 - std::pow(beta1, double(g.adam_t)));
  const float c2 = float(1.0 - std::pow(beta2, double(g.adam_t)));
  k_adam<<<div_up(n, 256), 256, 0, s>>>(n, g.params.get(), g.grad.get(), g.adam_m.get(),
                                        g.adam_v.get(), float(lr), float(beta1), float(beta2),
                                        float(eps), c1, c2);
  SFEM_HIP(hipGetLastError());
}

void gnn_set_pairs(Ctx& c, int64_t n_pairs, const float* r, const float* e) {
  GnnWork& w = gnn_work(c);
  const int64_t n = c.n_dof();
  w.n_pairs = 0;
  w.pr.reserve(n_pairs * n);
  w.pe.reserve(n_pairs * n);
  SFEM_HIP(hipMemcpyAsync(w.pr.get(), r, sizeof(float) * n_pairs * n, hipMemcpyDefault, c.stream));
  SFEM_HIP(hipMemcpyAsync(w.pe.get(), e, sizeof(float) * n_pairs * n, hipMemcpyDefault, c.stream));
  // e.K e = e.r, in FP64 from the stored FP32 values
  std::vector<double> den(n_pairs);
  for (int64_t p = 0; p < n_pairs; ++p) {
    den[p] = dot(c, w.pr.get() + p * n, w.pe.get() + p * n, n);
    SFEM_REQUIRE(den[p] > 0.0, SFEM_EINVAL, "a pair has e.r <= 0 (r must be K e, e nonzero)");
  }
  w.pden = den;
  w.n_pairs = n_pairs;
}

int64_t gnn_generate_pairs(Ctx& c, int n_rhs, int snaps, uint64_t seed) {
  SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "assemble K first");
  SFEM_REQUIRE(n_rhs >= 1 && snaps >= 1, SFEM_EINVAL, "need n_rhs >= 1 and snaps >= 1");
  GnnWork& w = gnn_work(c);
  const int64_t n = c.n_dof();
  hipStream_t s = c.stream;
  const int64_t total = int64_t(n_rhs) * snaps;
  w.n_pairs = 0;
  w.pr.reserve(total * n);
  w.pe.reserve(total * n);
  std::vector<double> den;
  DBuf<double> b, x0, xs, e, r;
  b.reserve(n);
  x0.reserve(n);
  xs.reserve(int64_t(snaps) * n);
  e.reserve(n);
  r.reserve(n);
  const uint8_t* fixed = c.any_fixed ? c.fixed.get() : nullptr;
  for (int k = 0; k < n_rhs; ++k) {
    if (k == 0) {
      // the load case itself: its error is smooth from the start
      SFEM_HIP(hipMemcpyAsync(b.get(), c.f_bc.get(), sizeof(double) * n, hipMemcpyDeviceToDevice,
                              s));
    } else {
      // b = K x0 for a rough target x0 = D^-1/2 u (u uniform in [-1, 1),
      // zero on fixed DOFs): the early errors of this solve carry the high
      // frequencies a sparse preconditioner can act on
      k_random_load<<<div_up(n, 256), 256, 0, s>>>(n, seed * 0x100000001b3ull + uint64_t(k), 1.0,
                                                    fixed, x0.get());
      k_scale_by<<<div_up(n, 256), 256, 0, s>>>(n, c.dinv.get(), x0.get());
      SFEM_HIP(hipGetLastError());
      spmv_f64(c, c.val.get(), x0.get(), b.get(), s);
    }
    const double bnorm = std::sqrt(dot(c, b.get(), b.get(), n));
    if (bnorm == 0.0) continue;
    const double tol = 1e-10 * bnorm;
    // pass 1: iterations to converge; pass 2: snapshots at iterations
    // its (j / snaps)^2, j = 0..snaps-1 (dense early, where errors are rough)
    const int its = jacobi_run(c, b.get(), tol, 50, 200000, [](int) {});
    std::vector<int> at;
    for (int j = 0; j < snaps; ++j) {
      const int t = int(double(its) * double(j) * double(j) / (double(snaps) * double(snaps)));
      if (at.empty() || t > at.back()) at.push_back(t);
    }
    int got = 0;
    auto grab = [&] {
      SFEM_HIP(hipMemcpyAsync(xs.get() + int64_t(got) * n, c.x.get(), sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
      ++got;
    };
    size_t next = 0;
    if (at[0] == 0) {  // x = 0: e = x*
      SFEM_HIP(hipMemsetAsync(xs.get(), 0, sizeof(double) * n, s));
      ++got;
      ++next;
    }
    // periods end at the snapshot iterations (and every 50 in between)
    const std::function<int(int)> stop = [&](int) {
      return next < at.size() ? at[next] : std::numeric_limits<int>::max();
    };
    jacobi_run(c, b.get(), tol, 50, 200000, [&](int done) {
      if (next < at.size() && done >= at[next]) {
        grab();
        ++next;
      }
    }, &stop);
    // c.x = x*; e_j = x* - x_j, r_j = K e_j
    for (int j = 0; j < got; ++j) {
      k_sub<<<div_up(n, 256), 256, 0, s>>>(n, c.x.get(), xs.get() + int64_t(j) * n, e.get());
      SFEM_HIP(hipGetLastError());
      spmv_f64(c, c.val.get(), e.get(), r.get(), s);
      const int64_t slot = int64_t(den.size());
      k_to_f32<<<div_up(n, 256), 256, 0, s>>>(n, e.get(), w.pe.get() + slot * n);
      k_to_f32<<<div_up(n, 256), 256, 0, s>>>(n, r.get(), w.pr.get() + slot * n);
      SFEM_HIP(hipGetLastError());
      const double d = dot(c, w.pr.get() + slot * n, w.pe.get() + slot * n, n);
      if (d > 0.0) den.push_back(d);
    }
  }
  SFEM_HIP(hipStreamSynchronize(s));
  w.pden = den;
  w.n_pairs = int64_t(den.size());
  return w.n_pairs;
}

}  // namespace sfem
