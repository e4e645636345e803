// Sparse matrix-vector products and the preconditioned conjugate-gradient
// solve of K u = f (the paper solves with a direct method; this library
// replaces it by PCG judged by the FP64 true residual).
//
// Products: a group of LPR lanes (4 to 64, a power of two) per node row I.
// The three scalar rows 3I..3I+2 share the row's block-column list, so one
// gather of x_J serves three sums, reduced across the group with shuffles.
// Two value layouts: the CSR order of the scalar matrix (row schedules 0-13:
// one or two rows per step, an unrolled column loop, nontemporal value
// loads), and a packed copy in which node row I is a [9][deg rounded up to
// 4] array read four blocks per lane with 16-byte loads (schedules 14-16;
// schedule 17 also stages the x entries a chunk of 128 rows gathers in
// LDS).  The autotuner times every schedule inside PCG iterations and keeps
// the fastest.  The learned M's apply has the same two forms (k_mapply,
// k_mapply_lds), the faster kept per mesh.  Grids are XCD-banded (for_rows).  The translation form
// (row3p's DIFF) multiplies neighbour differences x_J - x_I and adds
// R_I x_I, the FP64 block row sum: the true residual of every solve uses it.
// The FP32 products of SFEM_MODE_F32_TF take the same value in the
// corrected form: plain FP32 rows plus C_I x_I, C_I = sum_J (K_IJ - K32_IJ)
// (MODE bit 6).
//
// PCG: x0 = 0; each iteration is
//   p = z + beta p;   q = K p with (p.q) -> alpha;   x, r, z updates with
//   (r.z), (r.r) -> beta and a device-side convergence flag.
// Dot products are FP64 partial sums per workgroup, added in a fixed order
// by a separate one-workgroup k_finalize launch (no device-scope fences;
// results are bit-reproducible).  Every `check_every` iterations the
// residual is replaced by the true one, r = f - K x, whose norm the host
// reads; the iterations of a check period are replayed from a captured
// hipGraph after the first period.
#include "gnn.h"

namespace sfem {

namespace {

constexpr int kRowWaves = 4;               // waves per row-kernel workgroup
constexpr int kVecThreads = 256;

// The three sums of node row I, computed by a group of LPR lanes (a
// power of two dividing 64): lane c of the group takes column positions c,
// c+LPR, ... of the row and multiplies the SAME x entry with the values of
// all three scalar rows (one gather per column), then the group reduces with
// shuffles.  Rows with valid == false contribute zeros but still shuffle.
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Two rows per group at a time, column loop unrolled by kUnroll: all block
// column loads, then all x gathers and value loads are issued before any
// result is used, so each lane keeps many independent loads in flight.
constexpr int kUnroll = 3;

// Matrix-value load; NT: nontemporal (the value stream is read once per
// product and should not evict the gathered x from L2).
template <bool NT, typename T>
__device__ __forceinline__ T ldv(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <typename VT, int LPR, bool NT, class XF>
__device__ __forceinline__ void row3x2(const int (&I)[2], const bool (&valid)[2], int sub,
                                       const int32_t* __restrict__ bptr,
                                       const int32_t* __restrict__ bcol,
                                       const VT* __restrict__ val, const XF& x, double (&y)[2][3]) {
  using AT = double;  // row sums in FP64 for every matrix / vector precision
  int rb[2], td[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    int b = 0, e = 0;
    if (valid[r]) {
      b = bptr[I[r]];
      e = bptr[I[r] + 1];
    }
    rb[r] = b;
    td[r] = 3 * (e - b);
  }
  AT acc[2][3];
#pragma unroll
  for (int r = 0; r < 2; ++r) acc[r][0] = acc[r][1] = acc[r][2] = AT(0);
  const int tdmax = td[0] > td[1] ? td[0] : td[1];
  for (int c0 = 0; c0 < tdmax; c0 += kUnroll * LPR) {
    int col[2][kUnroll];
    bool on[2][kUnroll];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int c = c0 + u * LPR + sub;
        on[r][u] = c < td[r];
        const int jj = c / 3;
        col[r][u] = on[r][u] ? 3 * bcol[rb[r] + jj] + (c - 3 * jj) : 0;
      }
    AT xv[2][kUnroll], v0[2][kUnroll], v1[2][kUnroll], v2[2][kUnroll];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int c = c0 + u * LPR + sub;
        const VT* v = val + 9 * int64_t(rb[r]) + c;
        xv[r][u] = on[r][u] ? AT(x(int64_t(col[r][u]))) : AT(0);
        v0[r][u] = on[r][u] ? AT(ldv<NT>(v)) : AT(0);
        v1[r][u] = on[r][u] ? AT(ldv<NT>(v + td[r])) : AT(0);
        v2[r][u] = on[r][u] ? AT(ldv<NT>(v + 2 * td[r])) : AT(0);
      }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        acc[r][0] += v0[r][u] * xv[r][u];
        acc[r][1] += v1[r][u] * xv[r][u];
        acc[r][2] += v2[r][u] * xv[r][u];
      }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) y[r][a] = group_sum<LPR>(double(acc[r][a]));
}

template <typename VT, int LPR, bool NT, class XF>
__device__ __forceinline__ void row3(int I, bool valid, int sub, const int32_t* __restrict__ bptr,
                                     const int32_t* __restrict__ bcol,
                                     const VT* __restrict__ val, const XF& x, double& y0,
                                     double& y1, double& y2) {
  int rb = 0, deg = 0;
  if (valid) {
    rb = bptr[I];
    deg = bptr[I + 1] - rb;
  }
  const int td = 3 * deg;
  const VT* v = val + 9 * int64_t(rb);
  const int32_t* cols = bcol + rb;
  using AT = double;  // row sums in FP64 for every matrix / vector precision
  AT a0 = 0, a1 = 0, a2 = 0;
  for (int c = sub; c < td; c += LPR) {
    const int jj = c / 3;
    const int b = c - 3 * jj;
    const AT xv = AT(x(3 * int64_t(cols[jj]) + b));
    a0 += AT(ldv<NT>(v + c)) * xv;
    a1 += AT(ldv<NT>(v + td + c)) * xv;
    a2 += AT(ldv<NT>(v + 2 * td + c)) * xv;
  }
  y0 = group_sum<LPR>(double(a0));
  y1 = group_sum<LPR>(double(a1));
  y2 = group_sum<LPR>(double(a2));
}

// One row per group, column loop unrolled by kUnroll with every load of a
// step issued before any is used (more loads in flight per lane than row3).
template <typename VT, int LPR, bool NT, class XF>
__device__ __forceinline__ void row3u(int I, bool valid, int sub, const int32_t* __restrict__ bptr,
                                      const int32_t* __restrict__ bcol,
                                      const VT* __restrict__ val, const XF& x, double& y0,
                                      double& y1, double& y2) {
  int rb = 0, deg = 0;
  if (valid) {
    rb = bptr[I];
    deg = bptr[I + 1] - rb;
  }
  const int td = 3 * deg;
  const VT* v = val + 9 * int64_t(rb);
  const int32_t* cols = bcol + rb;
  double a0 = 0, a1 = 0, a2 = 0;
  for (int c0 = 0; c0 < td; c0 += kUnroll * LPR) {
    int col[kUnroll];
    bool on[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int c = c0 + u * LPR + sub;
      on[u] = c < td;
      const int jj = c / 3;
      col[u] = on[u] ? 3 * cols[jj] + (c - 3 * jj) : 0;
    }
    double xv[kUnroll], v0[kUnroll], v1[kUnroll], v2[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int c = c0 + u * LPR + sub;
      xv[u] = on[u] ? double(x(int64_t(col[u]))) : 0.0;
      v0[u] = on[u] ? double(ldv<NT>(v + c)) : 0.0;
      v1[u] = on[u] ? double(ldv<NT>(v + td + c)) : 0.0;
      v2[u] = on[u] ? double(ldv<NT>(v + 2 * td + c)) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      a0 += v0[u] * xv[u];
      a1 += v1[u] * xv[u];
      a2 += v2[u] * xv[u];
    }
  }
  y0 = group_sum<LPR>(a0);
  y1 = group_sum<LPR>(a1);
  y2 = group_sum<LPR>(a2);
}

template <typename T>
struct PlainX {
  const T* __restrict__ p;
  __device__ __forceinline__ T operator()(int64_t i) const { return p[i]; }
};

// Gathers s_i r_i (the Jacobi-scaled residual of the learned preconditioner).
template <typename T>
struct ScaledX {
  const T* __restrict__ r;
  const T* __restrict__ s;
  __device__ __forceinline__ T operator()(int64_t i) const { return r[i] * s[i]; }
};

// Row loop shared by the row kernels.  Workgroups are dealt round-robin to
// the 8 XCDs (block b runs on XCD b mod 8), so XCD x is given the x-th
// contiguous eighth of the node rows and its groups of LPR lanes sweep that
// range grid-stride: each XCD's L2 then holds the band of x entries its rows
// gather (neighbour node ids are close), while the rows in flight at any
// moment stay in one band per XCD.  body(I, valid, sub) runs in every lane
// (invalid rows still take part in the group shuffles).
constexpr int kXcds = 8;

template <int LPR, class Body>
__device__ __forceinline__ void for_rows(int64_t N, Body&& body) {
  constexpr int G = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane / LPR, sub = lane % LPR;
  const int xcd = blockIdx.x % kXcds;
  const int64_t groups_per_xcd = int64_t(gridDim.x / kXcds) * kRowWaves * G;  // grid % 8 == 0
  const int64_t lgroup = (int64_t(blockIdx.x / kXcds) * kRowWaves + threadIdx.x / kWave) * G + g;
  const int64_t span = (N + kXcds - 1) / kXcds;
  const int64_t lo = xcd * span;
  const int64_t hi = lo + span < N ? lo + span : N;
  const int64_t steps = (span + groups_per_xcd - 1) / groups_per_xcd;
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t I = lo + lgroup + k * groups_per_xcd;
    body(int(I < hi ? I : 0), I < hi, sub);
  }
}

// As for_rows, two rows per group per step (rows k and k + half of the
// group's sweep), handed to body2(I[2], valid[2], sub).
template <int LPR, class Body2>
__device__ __forceinline__ void for_rows2(int64_t N, Body2&& body2) {
  constexpr int G = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane / LPR, sub = lane % LPR;
  const int xcd = blockIdx.x % kXcds;
  const int64_t groups_per_xcd = int64_t(gridDim.x / kXcds) * kRowWaves * G;
  const int64_t lgroup = (int64_t(blockIdx.x / kXcds) * kRowWaves + threadIdx.x / kWave) * G + g;
  const int64_t span = (N + kXcds - 1) / kXcds;
  const int64_t lo = xcd * span;
  const int64_t hi = lo + span < N ? lo + span : N;
  const int64_t steps = (span + groups_per_xcd - 1) / groups_per_xcd;
  const int64_t half = (steps + 1) / 2;
  for (int64_t k = 0; k < half; ++k) {
    const int64_t I0 = lo + lgroup + k * groups_per_xcd;
    const int64_t I1 = lo + lgroup + (k + half) * groups_per_xcd;
    const bool v0 = I0 < hi, v1 = (k + half) < steps && I1 < hi;
    const int I[2] = {int(v0 ? I0 : 0), int(v1 ? I1 : 0)};
    const bool valid[2] = {v0, v1};
    body2(I, valid, sub);
  }
}

// Four consecutive values of a packed row (16-byte aligned).
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
__device__ __forceinline__ void load4(const __bf16* p, double (&v)[4]) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const bf16x4 a = *reinterpret_cast<const bf16x4*>(p);
  v[0] = float(a[0]);
  v[1] = float(a[1]);
  v[2] = float(a[2]);
  v[3] = float(a[3]);
}
__device__ __forceinline__ void load4(const float* p, double (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = a.z;
  v[3] = a.w;
}

// The three sums of node row I in the packed layout (ptr4 / col4 / values
// [9][d4] per row): a lane takes 4 blocks per step with one int4 column
// load and nine 4-wide value loads (36 entries; the CSR-order layout needs
// 60 loads for as many).
//
// DIFF: the translation form.  The row multiplies the neighbour differences
// x_J - x_I instead of x_J; the caller adds R_I x_I (R_I = sum_J K_IJ, the
// FP64 block row sum) to complete K x.  K maps rigid translations to
// (nearly) zero, so the plain sum cancels terms of size |K||x| down to a
// small result and keeps their rounding; here the matrix values only meet
// differences, and their rounding (FP64 arithmetic, or FP32 values) is
// relative to |x_J - x_I|, which is small wherever x is smooth.  Padding
// blocks (column I, value 0) give I - I = 0.
template <typename VT, int LPR, bool DIFF, class XF>
__device__ __forceinline__ void row3p(int I, bool valid, int sub, const int32_t* __restrict__ ptr4,
                                      const int32_t* __restrict__ col4,
                                      const VT* __restrict__ valp, const XF& x, double& y0,
                                      double& y1, double& y2) {
  int r4 = 0, d4 = 0;
  double xi0 = 0.0, xi1 = 0.0, xi2 = 0.0;
  if (valid) {
    r4 = ptr4[I];
    d4 = ptr4[I + 1] - r4;
    if constexpr (DIFF) {
      xi0 = double(x(3 * int64_t(I)));
      xi1 = double(x(3 * int64_t(I) + 1));
      xi2 = double(x(3 * int64_t(I) + 2));
    }
  }
  const VT* w = valp + 9 * int64_t(r4);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const auto blocks = [&](const int (&Js)[4], const double (&m)[9][4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t j3 = 3 * int64_t(Js[t]);
      double x0 = double(x(j3)), x1 = double(x(j3 + 1)), x2 = double(x(j3 + 2));
      if constexpr (DIFF) {
        x0 -= xi0;
        x1 -= xi1;
        x2 -= xi2;
      }
      a0 += m[0][t] * x0 + m[1][t] * x1 + m[2][t] * x2;
      a1 += m[3][t] * x0 + m[4][t] * x1 + m[5][t] * x2;
      a2 += m[6][t] * x0 + m[7][t] * x1 + m[8][t] * x2;
    }
  };
  if constexpr (sizeof(VT) == 8) {
    // FP64: four blocks are 32 bytes per component, two 16-byte loads.  A
    // lane takes the block pairs (jb, jb + 1) and (jb + 2 LPR, jb + 2 LPR +
    // 1), so that in each load the group's lanes read one contiguous run
    // (16 bytes apart) instead of every other 16 bytes of it.
    for (int jb = 2 * sub; jb < d4; jb += 4 * LPR) {
      const int jc = jb + 2 * LPR;
      const bool two = jc < d4;
      const int2 Ja = *reinterpret_cast<const int2*>(col4 + r4 + jb);
      int2 Jc = make_int2(I, I);  // no second pair: column I with zero values
      if (two) Jc = *reinterpret_cast<const int2*>(col4 + r4 + jc);
      double m[9][4];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const double2 a = *reinterpret_cast<const double2*>(w + q * d4 + jb);
        double2 b = make_double2(0.0, 0.0);
        if (two) b = *reinterpret_cast<const double2*>(w + q * d4 + jc);
        m[q][0] = a.x;
        m[q][1] = a.y;
        m[q][2] = b.x;
        m[q][3] = b.y;
      }
      const int Js[4] = {Ja.x, Ja.y, Jc.x, Jc.y};
      blocks(Js, m);
    }
  } else {
    for (int jb = 4 * sub; jb < d4; jb += 4 * LPR) {
      const int4 J = *reinterpret_cast<const int4*>(col4 + r4 + jb);
      double m[9][4];
#pragma unroll
      for (int q = 0; q < 9; ++q) load4(w + q * d4 + jb, m[q]);
      const int Js[4] = {J.x, J.y, J.z, J.w};
      blocks(Js, m);
    }
  }
  y0 = group_sum<LPR>(a0);
  y1 = group_sum<LPR>(a1);
  y2 = group_sum<LPR>(a2);
}

// Row schedule: LPR lanes per node row; MODE bit 0: two rows per group
// per step, bit 1: one row with the unrolled column loop, bit 2:
// nontemporal matrix-value loads, bit 3: the packed layout (bptr, bcol, val
// are then ptr4, col4 and the packed values), bit 4 (with bit 3): the
// translation form of row3p (the epilogue then adds R_I x_I).  epi(I, y)
// runs for each valid row in the group's first lane.
template <typename VT, int LPR, int MODE, class XF, class Epi>
__device__ __forceinline__ void row_apply(int64_t N, const int32_t* __restrict__ bptr,
                                          const int32_t* __restrict__ bcol,
                                          const VT* __restrict__ val, const XF& xf, Epi&& epi) {
  constexpr bool NT = (MODE & 4) != 0;
  if constexpr ((MODE & 8) != 0) {
    for_rows<LPR>(N, [&](int I, bool valid, int sub) {
      double y[3];
      row3p<VT, LPR, (MODE & 16) != 0>(I, valid, sub, bptr, bcol, val, xf, y[0], y[1], y[2]);
      if (valid && sub == 0) epi(I, y);
    });
  } else if constexpr ((MODE & 1) != 0) {
    for_rows2<LPR>(N, [&](const int (&I)[2], const bool (&valid)[2], int sub) {
      double yy[2][3];
      row3x2<VT, LPR, NT>(I, valid, sub, bptr, bcol, val, xf, yy);
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (valid[r] && sub == 0) epi(I[r], yy[r]);
    });
  } else if constexpr ((MODE & 2) != 0) {
    for_rows<LPR>(N, [&](int I, bool valid, int sub) {
      double y[3];
      row3u<VT, LPR, NT>(I, valid, sub, bptr, bcol, val, xf, y[0], y[1], y[2]);
      if (valid && sub == 0) epi(I, y);
    });
  } else {
    for_rows<LPR>(N, [&](int I, bool valid, int sub) {
      double y[3];
      row3<VT, LPR, NT>(I, valid, sub, bptr, bcol, val, xf, y[0], y[1], y[2]);
      if (valid && sub == 0) epi(I, y);
    });
  }
}

// Block reduction of NV doubles (thread 0 gets the block totals).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double lds[16 * NV];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[wid * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < nw; ++w)
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] += lds[w * NV + i];
}

// Each workgroup stores its NV partial sums; a one-workgroup k_finalize
// launched next adds them in a fixed order (no device-scope fences: the
// kernel boundary orders the writes).
template <int NV>
__device__ __forceinline__ void store_partials(double (&v)[NV], double* partials) {
  block_sum<NV>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[blockIdx.x * NV + i] = v[i];
}

// y += R_I x_I: the translation part of K x in the translation form
// (MODE bit 4; rsum holds R_I row-major per node), or y += C_I x_I in the
// corrected form (MODE bit 6; rsum holds C_I).
//
// The corrected form: sum_J K32_IJ (x_J - x_I) + R_I x_I equals
// sum_J K32_IJ x_J + C_I x_I with C_I = R_I - sum_J K32_IJ = sum_J (K_IJ -
// K32_IJ), the row sum of the FP32 values' rounding.  In exact arithmetic
// both are K x + sum_J (K32_IJ - K_IJ)(x_J - x_I): the FP32 rounding still
// meets only neighbour differences.  The rows then run as plain FP32
// products (no x_I held, no subtractions); what changes is the FP64
// accumulation's own rounding, now relative to |K||x| as in an FP64
// product.
template <int MODE, typename P>
__device__ __forceinline__ void add_translation(int I, const double* __restrict__ rsum,
                                                const P* __restrict__ x, double (&y)[3]) {
  if constexpr ((MODE & (16 | 64)) != 0) {
    const double* R = rsum + 9 * int64_t(I);
    const double x0 = double(x[3 * int64_t(I)]), x1 = double(x[3 * int64_t(I) + 1]),
                 x2 = double(x[3 * int64_t(I) + 2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) y[a] += R[3 * a] * x0 + R[3 * a + 1] * x1 + R[3 * a + 2] * x2;
  }
}

template <typename VT, typename XT, int LPR, int MODE>
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_spmv(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
           const VT* __restrict__ val, const XT* __restrict__ x, XT* __restrict__ y) {
  const PlainX<XT> xf{x};
  row_apply<VT, LPR, MODE>(N, bptr, bcol, val, xf, [&](int I, const double (&yy)[3]) {
    y[3 * int64_t(I) + 0] = XT(yy[0]);
    y[3 * int64_t(I) + 1] = XT(yy[1]);
    y[3 * int64_t(I) + 2] = XT(yy[2]);
  });
}

// ---------------------------------------------------------------- CG kernels
// p = z + beta p (beta = 0 on the first iteration)
template <typename P>
__global__ void __launch_bounds__(kVecThreads)
    k_cg_p(int64_t n, const P* __restrict__ z, P* __restrict__ p, const CgScalars* __restrict__ sc) {
  if (sc->converged) return;
  const P beta = P(sc->beta);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// q = K p, partial (p.q).  MODE bit 4: the translation form (rsum: R);
// bit 6: the corrected form (rsum: C).
template <typename VT, typename P, int LPR, int MODE>
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_cg_spmv(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
              const VT* __restrict__ val, const P* __restrict__ p, P* __restrict__ q,
              const CgScalars* __restrict__ sc, double* __restrict__ partials,
              const double* __restrict__ rsum) {
  if (sc->converged) return;
  const PlainX<P> xf{p};
  double v[1] = {0.0};
  row_apply<VT, LPR, MODE>(N, bptr, bcol, val, xf, [&](int I, const double (&yr)[3]) {
    double y[3] = {yr[0], yr[1], yr[2]};
    add_translation<MODE>(I, rsum, p, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t i = 3 * int64_t(I) + a;
      const P qi = P(y[a]);
      q[i] = qi;
      v[0] += double(p[i]) * double(qi);
    }
  });
  store_partials<1>(v, partials);
}

// ----------------------------------------------- LDS-staged CG product
// Window tables, one workgroup per chunk of kChunkRows node rows: the
// chunk's packed block columns are marked in an LDS bitmap over [min, max]
// of their ids; the set bits, in order, are the window (the x entries the
// chunk gathers) and a column's window index is the number of set bits
// below it.  A chunk whose id span exceeds kSpanBits, or whose window
// exceeds kWindow nodes, sets *fail.
constexpr int kSpanBits = 32768;

__global__ void __launch_bounds__(256)
    k_lds_tables(int64_t N, const int32_t* __restrict__ ptr4, const int32_t* __restrict__ col4,
                 int32_t* __restrict__ wcol, int32_t* __restrict__ wcnt,
                 uint16_t* __restrict__ lcol4, int32_t* __restrict__ fail) {
  __shared__ uint32_t bits[kSpanBits / 32];
  __shared__ int32_t wpre[kSpanBits / 32 + 1];
  __shared__ int32_t red[2][4];
  const int64_t r0 = int64_t(blockIdx.x) * kChunkRows;
  const int64_t r1 = r0 + kChunkRows < N ? r0 + kChunkRows : N;
  const int b0 = ptr4[r0], b1 = ptr4[r1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int lo = 0x7fffffff, hi = -1;
  for (int b = b0 + tid; b < b1; b += blockDim.x) {
    lo = min(lo, col4[b]);
    hi = max(hi, col4[b]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o));
    hi = max(hi, __shfl_xor(hi, o));
  }
  if (lane == 0) {
    red[0][wid] = lo;
    red[1][wid] = hi;
  }
  __syncthreads();
  lo = min(min(red[0][0], red[0][1]), min(red[0][2], red[0][3]));
  hi = max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3]));
  const int span = hi - lo + 1;
  if (span > kSpanBits) {
    if (tid == 0) {
      wcnt[blockIdx.x] = 0;
      atomicOr(fail, 1);
    }
    return;
  }
  const int nw = (span + 31) / 32;
  for (int w = tid; w < nw; w += blockDim.x) bits[w] = 0u;
  __syncthreads();
  for (int b = b0 + tid; b < b1; b += blockDim.x) {
    const int d = col4[b] - lo;
    atomicOr(&bits[d >> 5], 1u << (d & 31));
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) {
      wpre[w] = acc;
      acc += __popc(bits[w]);
    }
    wpre[nw] = acc;
  }
  __syncthreads();
  const int cnt = wpre[nw];
  if (cnt > kWindow) {
    if (tid == 0) {
      wcnt[blockIdx.x] = 0;
      atomicOr(fail, 1);
    }
    return;
  }
  int32_t* W = wcol + int64_t(blockIdx.x) * kWindow;
  for (int w = tid; w < nw; w += blockDim.x) {
    uint32_t word = bits[w];
    int k = wpre[w];
    while (word) {
      const int bit = __ffs(int(word)) - 1;
      W[k++] = lo + 32 * w + bit;
      word &= word - 1u;
    }
  }
  for (int b = b0 + tid; b < b1; b += blockDim.x) {
    const int d = col4[b] - lo;
    const int w = d >> 5, m = d & 31;
    lcol4[b] = uint16_t(wpre[w] + __popc(bits[w] & ((1u << m) - 1u)));
  }
  if (tid == 0) wcnt[blockIdx.x] = cnt;
}

// The three sums of node row I against the LDS window xs ([window][3],
// FP64): as row3p, with each lane's 4 block columns given by one 8-byte
// load of window indices.
template <typename VT, int LPR>
__device__ __forceinline__ void row3p_lds(int I, bool valid, int sub,
                                          const int32_t* __restrict__ ptr4,
                                          const uint16_t* __restrict__ lcol4,
                                          const VT* __restrict__ valp, const double* xs,
                                          double (&y)[3]) {
  int r4 = 0, d4 = 0;
  if (valid) {
    r4 = ptr4[I];
    d4 = ptr4[I + 1] - r4;
  }
  const VT* w = valp + 9 * int64_t(r4);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int jb = 4 * sub; jb < d4; jb += 4 * LPR) {
    const ushort4 J = *reinterpret_cast<const ushort4*>(lcol4 + r4 + jb);
    double m[9][4];
#pragma unroll
    for (int q = 0; q < 9; ++q) load4(w + q * d4 + jb, m[q]);
    const int Js[4] = {J.x, J.y, J.z, J.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double* xj = xs + 3 * Js[t];
      const double x0 = xj[0], x1 = xj[1], x2 = xj[2];
      a0 += m[0][t] * x0 + m[1][t] * x1 + m[2][t] * x2;
      a1 += m[3][t] * x0 + m[4][t] * x1 + m[5][t] * x2;
      a2 += m[6][t] * x0 + m[7][t] * x1 + m[8][t] * x2;
    }
  }
  y[0] = group_sum<LPR>(a0);
  y[1] = group_sum<LPR>(a1);
  y[2] = group_sum<LPR>(a2);
}

// q = K p, partial (p.q), with p staged in LDS per chunk of rows (schedule
// 17).  Chunks are dealt to the XCDs in contiguous ranges (workgroup b runs
// on XCD b mod 8), so neighbouring windows share an L2.  CORR: the
// corrected form (rsum: C).
constexpr int kLdsThreads = 256;

template <typename VT, typename P, int LPR, bool CORR>
__global__ void __launch_bounds__(kLdsThreads)
    k_cg_spmv_lds(int64_t N, const int32_t* __restrict__ ptr4,
                  const uint16_t* __restrict__ lcol4, const VT* __restrict__ valp,
                  const int32_t* __restrict__ wcol, const int32_t* __restrict__ wcnt,
                  const P* __restrict__ p, P* __restrict__ q, const CgScalars* __restrict__ sc,
                  double* __restrict__ partials, const double* __restrict__ rsum) {
  if (sc->converged) return;
  __shared__ double xs[3 * kWindow];
  constexpr int G = kLdsThreads / LPR;  // row groups per workgroup
  const int tid = threadIdx.x;
  const int g = tid / LPR, sub = tid % LPR;
  const int64_t n_chunks = (N + kChunkRows - 1) / kChunkRows;
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = gridDim.x / kXcds;  // grid % 8 == 0
  const int64_t span = (n_chunks + kXcds - 1) / kXcds;
  const int64_t c_lo = xcd * span;
  const int64_t c_hi = c_lo + span < n_chunks ? c_lo + span : n_chunks;
  double v[1] = {0.0};
  for (int64_t ch = c_lo + blockIdx.x / kXcds; ch < c_hi; ch += per_xcd) {
    const int cnt = wcnt[ch];
    const int32_t* W = wcol + ch * kWindow;
    for (int i = tid; i < 3 * cnt; i += kLdsThreads) {
      const int k = i / 3;
      xs[i] = double(p[3 * int64_t(W[k]) + (i - 3 * k)]);
    }
    __syncthreads();
    const int64_t r0 = ch * kChunkRows;
    for (int rr = 0; rr < kChunkRows; rr += G) {
      const int64_t I = r0 + rr + g;
      const bool valid = I < N;
      const int Ii = valid ? int(I) : 0;
      double y[3];
      row3p_lds<VT, LPR>(Ii, valid, sub, ptr4, lcol4, valp, xs, y);
      if (valid && sub == 0) {
        if constexpr (CORR) {
          const double* C = rsum + 9 * int64_t(Ii);
          const double xi[3] = {double(p[3 * int64_t(Ii)]), double(p[3 * int64_t(Ii) + 1]),
                                double(p[3 * int64_t(Ii) + 2])};
#pragma unroll
          for (int a = 0; a < 3; ++a)
            y[a] += C[3 * a] * xi[0] + C[3 * a + 1] * xi[1] + C[3 * a + 2] * xi[2];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int64_t i = 3 * int64_t(Ii) + a;
          const P qi = P(y[a]);
          q[i] = qi;
          v[0] += double(p[i]) * double(qi);
        }
      }
    }
    __syncthreads();  // the window is rewritten by the next chunk
  }
  store_partials<1>(v, partials);
}

// The learned M apply of k_mapply with rh staged in LDS per chunk of rows
// (the window tables of schedule 17; the same row sums in the same order).
template <typename P>
__global__ void __launch_bounds__(kLdsThreads)
    k_mapply_lds(int64_t N, const int32_t* __restrict__ ptr4, const uint16_t* __restrict__ lcol4,
                 const __bf16* __restrict__ mvalp, const int32_t* __restrict__ wcol,
                 const int32_t* __restrict__ wcnt, const P* __restrict__ s,
                 const P* __restrict__ r, const P* __restrict__ rh, P* __restrict__ z,
                 const CgScalars* __restrict__ sc, double* __restrict__ partials) {
  if (sc && sc->converged) return;
  __shared__ double xs[3 * kWindow];
  constexpr int LPR = 8;
  constexpr int G = kLdsThreads / LPR;
  const int tid = threadIdx.x;
  const int g = tid / LPR, sub = tid % LPR;
  const int64_t n_chunks = (N + kChunkRows - 1) / kChunkRows;
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = gridDim.x / kXcds;  // grid % 8 == 0
  const int64_t span = (n_chunks + kXcds - 1) / kXcds;
  const int64_t c_lo = xcd * span;
  const int64_t c_hi = c_lo + span < n_chunks ? c_lo + span : n_chunks;
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t ch = c_lo + blockIdx.x / kXcds; ch < c_hi; ch += per_xcd) {
    const int cnt = wcnt[ch];
    const int32_t* W = wcol + ch * kWindow;
    for (int i = tid; i < 3 * cnt; i += kLdsThreads) {
      const int k = i / 3;
      xs[i] = double(rh[3 * int64_t(W[k]) + (i - 3 * k)]);
    }
    __syncthreads();
    const int64_t r0 = ch * kChunkRows;
    for (int rr = 0; rr < kChunkRows; rr += G) {
      const int64_t I = r0 + rr + g;
      const bool valid = I < N;
      const int Ii = valid ? int(I) : 0;
      double y[3];
      row3p_lds<__bf16, LPR>(Ii, valid, sub, ptr4, lcol4, mvalp, xs, y);
      if (valid && sub == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int64_t i = 3 * int64_t(Ii) + a;
          const double ri = double(r[i]);
          const P zi = P(double(s[i]) * (double(rh[i]) + y[a]));
          v[0] += ri * double(zi);
          v[1] += ri * ri;
          v[2] += ri * double(z[i]);
          z[i] = zi;
        }
      }
    }
    __syncthreads();  // the window is rewritten by the next chunk
  }
  store_partials<3>(v, partials);
}

// x += alpha p; r -= alpha q; z = dinv r; partials (r.z), (r.r)
template <typename P>
__global__ void __launch_bounds__(kVecThreads)
    k_cg_update(int64_t n, P* __restrict__ x, P* __restrict__ r, P* __restrict__ z,
                const P* __restrict__ p, const P* __restrict__ q, const P* __restrict__ dinv,
                const CgScalars* __restrict__ sc, double* __restrict__ partials) {
  if (sc->converged) return;
  const P alpha = P(sc->alpha);
  double v[2] = {0.0, 0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const P xi = x[i] + alpha * p[i];
    const P ri = r[i] - alpha * q[i];
    const P zi = dinv[i] * ri;
    x[i] = xi;
    r[i] = ri;
    z[i] = zi;
    v[0] += double(ri) * double(zi);
    v[1] += double(ri) * double(ri);
  }
  store_partials<2>(v, partials);
}

// x += alpha p; r -= alpha q; rh = s r (the learned preconditioner applies
// z after, gathering rh).
template <typename P>
__global__ void __launch_bounds__(kVecThreads)
    k_cg_xr(int64_t n, P* __restrict__ x, P* __restrict__ r, const P* __restrict__ p,
            const P* __restrict__ q, const P* __restrict__ s, P* __restrict__ rh,
            const CgScalars* __restrict__ sc) {
  if (sc->converged) return;
  const P alpha = P(sc->alpha);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    const P ri = r[i] - alpha * q[i];
    r[i] = ri;
    rh[i] = s[i] * ri;
  }
}

// rh = s r (start and residual replacement).
template <typename P>
__global__ void k_rh(int64_t n, const P* __restrict__ s, const P* __restrict__ r,
                     P* __restrict__ rh) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) rh[i] = s[i] * r[i];
}

// Learned preconditioner z = M r = s (rh + S' rh), rh = s r, s =
// diag(K)^-1/2, with S' (BF16) in the packed layout: node row I holds a
// [9][d4] array (component q = 3a + c major, blocks minor, d4 = deg rounded
// up to 4) at 9 ptr4[I], block columns col4 padded with I and zero values.
// A lane takes 4 blocks per step: one int4 column load and nine float4 value
// loads for 36 entries (the row kernels' layout needs 60 loads).  Partials
// (r.z_new), (r.r), (r.z_old): the flexible (Polak-Ribiere) beta needs the
// previous z.  sc == nullptr: run unconditionally (start and replacement).
constexpr int kMLanes = 8;  // lanes per node row: 32 blocks per step

// 128 VGPRs at most: 4 waves per SIMD (unconstrained it takes 131, i.e. 3
// waves, and runs ~4% slower).
template <typename P>
__global__ void __launch_bounds__(kRowWaves * kWave) __attribute__((amdgpu_waves_per_eu(4)))
    k_mapply(int64_t N, const int32_t* __restrict__ ptr4, const int32_t* __restrict__ col4,
             const __bf16* __restrict__ mvalp, const P* __restrict__ s, const P* __restrict__ r,
             const P* __restrict__ rh, P* __restrict__ z, const CgScalars* __restrict__ sc,
             double* __restrict__ partials) {
  if (sc && sc->converged) return;
  const PlainX<P> xf{rh};
  double v[3] = {0.0, 0.0, 0.0};
  row_apply<__bf16, kMLanes, 8>(N, ptr4, col4, mvalp, xf, [&](int I, const double (&y)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t i = 3 * int64_t(I) + a;
      const double ri = double(r[i]);
      const P zi = P(double(s[i]) * (double(rh[i]) + y[a]));
      v[0] += ri * double(zi);
      v[1] += ri * ri;
      v[2] += ri * double(z[i]);
      z[i] = zi;
    }
  });
  store_partials<3>(v, partials);
}

// The three sums of node row I of S' in the grouped layout: a lane takes
// one group (4 blocks) per step with five 16-byte loads, the 36 BF16
// values [q][t] and the 4 int16 offsets J - I (the packed layout needs
// nine 8-byte value loads and a 16-byte column load for as many).  The
// sums are row3p's on the packed copy, term for term in the same order.
template <int LPR, class XF>
__device__ __forceinline__ void row3g(int I, bool valid, int sub, const int32_t* __restrict__ ptr4,
                                      const uint4* __restrict__ grp, const XF& x, double& y0,
                                      double& y1, double& y2) {
  int g0 = 0, ng = 0;
  if (valid) {
    const int r4 = ptr4[I];
    g0 = r4 >> 2;
    ng = (ptr4[I + 1] - r4) >> 2;
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int g = sub; g < ng; g += LPR) {
    const uint4* G = grp + 5 * (int64_t(g0) + g);
    uint32_t w[20];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint4 t = G[k];
      w[4 * k] = t.x;
      w[4 * k + 1] = t.y;
      w[4 * k + 2] = t.z;
      w[4 * k + 3] = t.w;
    }
    double m[9][4];
#pragma unroll
    for (int i = 0; i < 36; ++i) {
      // BF16 i is the low (even i) or high half of word i / 2
      const uint32_t bits = (i & 1) ? (w[i >> 1] & 0xffff0000u) : (w[i >> 1] << 16);
      m[i >> 2][i & 3] = double(__uint_as_float(bits));
    }
    const int Js[4] = {I + int(int16_t(w[18] & 0xffffu)), I + int(int16_t(w[18] >> 16)),
                       I + int(int16_t(w[19] & 0xffffu)), I + int(int16_t(w[19] >> 16))};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t j3 = 3 * int64_t(Js[t]);
      const double x0 = double(x(j3)), x1 = double(x(j3 + 1)), x2 = double(x(j3 + 2));
      a0 += m[0][t] * x0 + m[1][t] * x1 + m[2][t] * x2;
      a1 += m[3][t] * x0 + m[4][t] * x1 + m[5][t] * x2;
      a2 += m[6][t] * x0 + m[7][t] * x1 + m[8][t] * x2;
    }
  }
  y0 = group_sum<LPR>(a0);
  y1 = group_sum<LPR>(a1);
  y2 = group_sum<LPR>(a2);
}

// The learned M apply of k_mapply from the grouped layout (same sums, same
// order, same epilogue).
template <typename P>
__global__ void __launch_bounds__(kRowWaves * kWave) __attribute__((amdgpu_waves_per_eu(4)))
    k_mapply_grp(int64_t N, const int32_t* __restrict__ ptr4, const uint4* __restrict__ grp,
                 const P* __restrict__ s, const P* __restrict__ r, const P* __restrict__ rh,
                 P* __restrict__ z, const CgScalars* __restrict__ sc,
                 double* __restrict__ partials) {
  if (sc && sc->converged) return;
  const PlainX<P> xf{rh};
  double v[3] = {0.0, 0.0, 0.0};
  for_rows<kMLanes>(N, [&](int I, bool valid, int sub) {
    double y[3];
    row3g<kMLanes>(I, valid, sub, ptr4, grp, xf, y[0], y[1], y[2]);
    if (valid && sub == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int64_t i = 3 * int64_t(I) + a;
        const double ri = double(r[i]);
        const P zi = P(double(s[i]) * (double(rh[i]) + y[a]));
        v[0] += ri * double(zi);
        v[1] += ri * ri;
        v[2] += ri * double(z[i]);
        z[i] = zi;
      }
    }
  });
  store_partials<3>(v, partials);
}

// Packed BF16 S' and block columns -> the grouped layout, one thread per
// node row; bad is set if an offset J - I does not fit in int16.
__global__ void k_mgroup(int64_t N, const int32_t* __restrict__ ptr4,
                         const int32_t* __restrict__ col4, const __bf16* __restrict__ mvalp,
                         uint4* __restrict__ grp, int* __restrict__ bad) {
  const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int r4 = ptr4[I], d4 = ptr4[I + 1] - r4;
  const uint16_t* v = reinterpret_cast<const uint16_t*>(mvalp) + 9 * int64_t(r4);
  for (int jb = 0; jb < d4; jb += 4) {
    uint32_t w[20];
#pragma unroll
    for (int i = 0; i < 36; i += 2) {
      const int q = i >> 2, t = i & 3;  // t is 0 or 2: (q, t) and (q, t + 1)
      const int64_t o = int64_t(q) * d4 + jb + t;
      w[i >> 1] = uint32_t(v[o]) | (uint32_t(v[o + 1]) << 16);
    }
    uint32_t off[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int d = col4[r4 + jb + t] - int(I);
      if (d < -32768 || d > 32767) {
        atomicOr(bad, 1);
        d = 0;
      }
      off[t] = uint32_t(d) & 0xffffu;
    }
    w[18] = off[0] | (off[1] << 16);
    w[19] = off[2] | (off[3] << 16);
    uint4* G = grp + 5 * (int64_t(r4 + jb) >> 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) G[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
  }
}

// Residual replacement: r = b - K x, z = dinv r; partials (r.r), (r.z).
// MODE bit 4: K x in the translation form (rsum: R).
template <typename VT, typename P, int LPR, int MODE>
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_cg_replace(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                 const VT* __restrict__ val, const P* __restrict__ b, const P* __restrict__ x,
                 P* __restrict__ r, P* __restrict__ z, const P* __restrict__ dinv,
                 double* __restrict__ partials, const double* __restrict__ rsum) {
  const PlainX<P> xf{x};
  double v[2] = {0.0, 0.0};
  row_apply<VT, LPR, MODE>(N, bptr, bcol, val, xf, [&](int I, const double (&yr)[3]) {
    double y[3] = {yr[0], yr[1], yr[2]};
    add_translation<MODE>(I, rsum, x, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t i = 3 * int64_t(I) + a;
      const P ri = P(double(b[i]) - y[a]);
      const P zi = dinv[i] * ri;
      r[i] = ri;
      z[i] = zi;
      v[0] += double(ri) * double(ri);
      v[1] += double(ri) * double(zi);
    }
  });
  store_partials<2>(v, partials);
}

// FP64 residual of the outer problem: r = f - K u; partials ||r||^2, ||f||^2.
// MODE bit 4: K u in the translation form (rsum: R).
template <int LPR, int MODE>
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_resid64(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
              const double* __restrict__ val, const double* __restrict__ f,
              const double* __restrict__ u, double* __restrict__ r,
              double* __restrict__ partials, const double* __restrict__ rsum) {
  const PlainX<double> xf{u};
  double v[2] = {0.0, 0.0};
  row_apply<double, LPR, MODE>(N, bptr, bcol, val, xf, [&](int I, const double (&yr)[3]) {
    double y[3] = {yr[0], yr[1], yr[2]};
    add_translation<MODE>(I, rsum, u, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t i = 3 * int64_t(I) + a;
      const double ri = f[i] - y[a];
      if (r) r[i] = ri;
      v[0] += ri * ri;
      v[1] += f[i] * f[i];
    }
  });
  store_partials<2>(v, partials);
}

// CG start from x = 0 with right-hand side b (FP64, scaled by inv_scale and
// converted to P; bp receives the converted copy when non-null): x = 0,
// r = b, z = dinv b, p = 0; partials (r.z), (r.r).
template <typename P>
__global__ void __launch_bounds__(kVecThreads)
    k_cg_start(int64_t n, const double* __restrict__ b, double inv_scale, P* __restrict__ bp,
               P* __restrict__ x, P* __restrict__ r, P* __restrict__ z, P* __restrict__ p0,
               P* __restrict__ p1, const P* __restrict__ dinv, double* __restrict__ partials) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const P bi = P(b[i] * inv_scale);
    const P zi = dinv[i] * bi;
    if (bp) bp[i] = bi;
    x[i] = P(0);
    r[i] = bi;
    z[i] = zi;
    p0[i] = P(0);
    p1[i] = P(0);
    v[0] += double(bi) * double(zi);
    v[1] += double(bi) * double(bi);
  }
  store_partials<2>(v, partials);
}

enum FinalizeOp {
  kFinAlpha = 0,
  kFinBeta = 1,
  kFinReplace = 2,
  kFinResid = 3,
  kFinStart = 4,
  kFinBetaFlex = 5,   // learned M: (r.z_new, r.r, r.z_old)
  kFinStartM = 6,     // learned M at the start: r.z
  kFinReplaceM = 7    // learned M after a residual replacement: r.z
};

// One workgroup: adds the partials of the previous kernel in a fixed order
// and updates the CG scalars.  The flag and the scalars it reads are loaded
// together with the partials, so that the launch waits on one memory
// latency rather than three (flag, then partials, then scalars); a
// converged solve discards what it loaded.
__global__ void __launch_bounds__(1024)
    k_finalize(int op, const double* __restrict__ partials, int nparts, CgScalars* __restrict__ sc) {
  const int converged = sc->converged;
  const double rz = sc->rz, iters = sc->aux[0], tol2 = sc->aux[1];
  const int nv = op == kFinAlpha ? 1 : (op >= kFinBetaFlex ? 3 : 2);
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
    for (int i = 0; i < nv; ++i) v[i] += partials[b * nv + i];
  if ((op == kFinAlpha || op == kFinBeta || op == kFinBetaFlex) && converged) return;
  block_sum<3>(v);
  if (threadIdx.x != 0) return;
  switch (op) {
    case kFinAlpha:
      sc->pq = v[0];
      sc->alpha = rz / v[0];
      if (!(v[0] > 0.0) || !isfinite(sc->alpha)) sc->converged = 2;
      break;
    case kFinBeta:
      sc->beta = v[0] / rz;
      sc->rz = v[0];
      sc->rr = v[1];
      sc->aux[0] = iters + 1.0;                         // iteration count
      if (v[1] <= tol2) sc->converged = 1;  // aux[1]: tolerance^2 on r.r
      if (!isfinite(v[1])) sc->converged = 2;
      break;
    case kFinReplace:
      sc->rr_true = v[0];
      sc->rr = v[0];
      sc->rz = v[1];
      break;
    case kFinResid:
      sc->rr_true = v[0];
      sc->ff = v[1];
      break;
    case kFinStart:
      sc->rz = v[0];
      sc->rr = v[1];
      sc->rr_true = v[1];
      sc->beta = 0.0;
      sc->converged = 0;
      break;
    case kFinBetaFlex:
      // r.M r must stay positive: otherwise M is not positive definite
      // along r and the solve reports a breakdown (the host falls back)
      sc->beta = (v[0] - v[2]) / rz;
      sc->rz = v[0];
      sc->rr = v[1];
      sc->aux[0] = iters + 1.0;
      if (v[1] <= tol2) sc->converged = 1;
      else if (!(v[0] > 0.0) || !isfinite(v[0]) || !isfinite(sc->beta)) sc->converged = 2;
      break;
    case kFinStartM:
    case kFinReplaceM:
      sc->rz = v[0];
      if (v[1] > 0.0 && (!(v[0] > 0.0) || !isfinite(v[0]))) sc->converged = 2;
      break;
  }
}

// u += scale * d (refinement update)
__global__ void k_axpy_f32(int64_t n, double scale, const float* __restrict__ d,
                           double* __restrict__ u) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) u[i] += scale * double(d[i]);
}

__global__ void k_zero(int64_t n, double* __restrict__ u) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) u[i] = 0.0;
}

constexpr int kRowGridMax = 4096;
constexpr int kVecGridMax = 2048;

// Row-kernel schedules: lanes per row and the MODE bits of row_apply.
struct SchedShape {
  int lpr;
  int mode;
};
constexpr SchedShape kSched[kNumSched] = {
    {8, 0},  {16, 0}, {32, 0}, {64, 0},   // one row per step
    {8, 1},  {16, 1}, {32, 1}, {64, 1},   // two rows per step
    {16, 2}, {32, 2},                     // one row, unrolled columns
    {16, 6}, {32, 6}, {64, 6},            // unrolled, nontemporal values
    {32, 5},                              // two rows, nontemporal values
    {4, 8},  {8, 8},  {16, 8},            // packed layout, 4 blocks per lane
    {8, 8 | 32}};                         // packed, x staged in LDS per chunk

int row_grid(int64_t N, const RowSched& rs) {
  const SchedShape sh = kSched[rs.variant];
  const int64_t rows_per_block = int64_t(kRowWaves) * (kWave / sh.lpr) * ((sh.mode & 1) ? 2 : 1);
  int g = div_up(N, rows_per_block);
  const int cap = std::min(rs.grid_cap, kRowGridMax);
  g = g < cap ? g : cap;
  return div_up(g, kXcds) * kXcds;  // for_rows needs a multiple of kXcds
}

// Launch KERNEL<prefix..., LPR, MODE> for the schedule's variant.
#define SFEM_SCHED_SWITCH(variant, LAUNCH) \
  switch (variant) {                        \
    case 0: LAUNCH(8, 0); break;            \
    case 1: LAUNCH(16, 0); break;           \
    case 2: LAUNCH(32, 0); break;           \
    case 3: LAUNCH(64, 0); break;           \
    case 4: LAUNCH(8, 1); break;            \
    case 5: LAUNCH(16, 1); break;           \
    case 6: LAUNCH(32, 1); break;           \
    case 7: LAUNCH(64, 1); break;           \
    case 8: LAUNCH(16, 2); break;           \
    case 9: LAUNCH(32, 2); break;           \
    case 10: LAUNCH(16, 6); break;          \
    case 11: LAUNCH(32, 6); break;          \
    case 12: LAUNCH(64, 6); break;          \
    case 13: LAUNCH(32, 5); break;          \
    case 14: LAUNCH(4, 8); break;           \
    case 15: LAUNCH(8, 8); break;           \
    case 16: LAUNCH(16, 8); break;          \
    default: LAUNCH(8, 8); break;           \
  }
// (schedule 17, the LDS-staged CG product, launches its own kernel; every
// other row kernel runs the packed 8-lane path for it)

// Launch KERNEL<prefix..., LPR, 24> (packed layout, translation form) for
// a packed schedule's lanes per row.
#define SFEM_TF_SWITCH(lpr, LAUNCH) \
  switch (lpr) {                    \
    case 4: LAUNCH(4, 24); break;   \
    case 16: LAUNCH(16, 24); break; \
    default: LAUNCH(8, 24); break;  \
  }
// The same schedules in the corrected form (packed layout, MODE bit 6).
#define SFEM_CF_SWITCH(lpr, LAUNCH) \
  switch (lpr) {                    \
    case 4: LAUNCH(4, 72); break;   \
    case 16: LAUNCH(16, 72); break; \
    default: LAUNCH(8, 72); break;  \
  }

// The schedule the translation form runs with: rs itself if it is a packed
// schedule, else the packed one with 8 lanes per row (same grid cap).
RowSched tf_sched(const RowSched& rs) {
  return (kSched[rs.variant].mode & 8) ? rs : RowSched{15, rs.grid_cap};
}

// R_I = sum_J K_IJ per node row, one thread per (I, q = 3a + c): the
// row's d4 packed values of component q (the padding adds zeros),
// Neumaier-compensated (exact to one rounding of R plus O(deg eps^2)
// sum |K_IJ|).  CORR: C_I = sum_J (K_IJ - K32_IJ) from the packed FP32
// copy v32 (each difference is exact when K32 is K rounded to FP32).
template <bool CORR>
__global__ void k_rowsum(int64_t N, const int32_t* __restrict__ ptr4,
                         const double* __restrict__ valp, const float* __restrict__ valp32,
                         double* __restrict__ rsum) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 9 * N) return;
  const int64_t I = t / 9;
  const int q = int(t - 9 * I);
  const int r4 = ptr4[I], d4 = ptr4[I + 1] - r4;
  const int64_t off = 9 * int64_t(r4) + int64_t(q) * d4;
  const double* v = valp + off;
  double sum = 0.0, comp = 0.0;
  for (int j = 0; j < d4; ++j) {
    const double x = CORR ? v[j] - double(valp32[off + j]) : v[j];
    const double t2 = sum + x;
    comp += fabs(sum) >= fabs(x) ? (sum - t2) + x : (x - t2) + sum;
    sum = t2;
  }
  rsum[t] = sum + comp;
}

// Pattern tables of the packed layout (once per mesh).
__global__ void k_deg4(int64_t N, const int32_t* __restrict__ bptr, int32_t* __restrict__ d4) {
  int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I < N) d4[I] = (bptr[I + 1] - bptr[I] + 3) & ~3;
}

__global__ void k_col4(int64_t N, const int32_t* __restrict__ bptr,
                       const int32_t* __restrict__ bcol, const int32_t* __restrict__ p4,
                       int32_t* __restrict__ c4) {
  int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int rb = bptr[I], deg = bptr[I + 1] - rb, r4 = p4[I], d4 = p4[I + 1] - r4;
  for (int j = 0; j < d4; ++j) c4[r4 + j] = j < deg ? bcol[rb + j] : int(I);
}

// CSR-order values -> packed layout; one wave per node row.
template <typename T>
__global__ void k_pack(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ p4,
                       const T* __restrict__ csr, T* __restrict__ packed) {
  const int lane = threadIdx.x & 63;
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
  if (I >= N) return;
  const int rb = bptr[I], deg = bptr[I + 1] - rb, r4 = p4[I], d4 = p4[I + 1] - r4;
  const T* src = csr + 9 * int64_t(rb);
  T* dst = packed + 9 * int64_t(r4);
  for (int k = lane; k < 9 * d4; k += 64) {
    const int q = k / d4, j = k - q * d4;
    const int a = q / 3, c = q - 3 * a;
    dst[k] = j < deg ? src[a * 3 * deg + 3 * j + c] : T(0);
  }
}

// The arrays a schedule reads: the CSR-order layout or the packed one.
template <typename VT>
struct Lay {
  const int32_t* ptr;
  const int32_t* col;
  const VT* val;
};

void ensure_packed64(Ctx& c);
void ensure_packed32(Ctx& c);

template <typename VT>
Lay<VT> lay(Ctx& c, const RowSched& rs, const VT* csr_val) {
  if (!(kSched[rs.variant].mode & 8)) {
    if ((const void*)csr_val == (const void*)c.val.get()) ensure_csr64(c);
    return {c.topo.bptr.get(), c.topo.bcol.get(), csr_val};
  }
  const void* pv = nullptr;
  if ((const void*)csr_val == (const void*)c.val.get()) {
    ensure_packed64(c);
    pv = c.valp.get();
  } else if ((const void*)csr_val == (const void*)c.val32.get()) {
    ensure_packed32(c);
    pv = c.valp32.get();
  } else {
    throw Error{SFEM_EINVAL, "packed schedule for a matrix without a packed copy"};
  }
  return {c.ptr4.get(), c.col4.get(), static_cast<const VT*>(pv)};
}

int vec_grid(int64_t n) {
  int g = div_up(n, kVecThreads);
  return g < kVecGridMax ? g : kVecGridMax;
}

void finalize(Ctx& c, FinalizeOp op, int nparts) {
  k_finalize<<<1, 1024, 0, c.stream>>>(int(op), c.partials.get(), nparts, c.sc.get());
  SFEM_HIP(hipGetLastError());
}

// ------------------------------------------------------------- host driver
struct CgBuffers {
  const void* val;       // matrix of the iteration (FP64 or FP32 values)
  const void* val_true;  // FP64 matrix of the residual replacement
  const void* dinv;
  void *b, *x, *r, *z, *p0, *p1, *q;  // p0: search direction (p1 unused)
  const __bf16* mval = nullptr;       // learned S', packed BF16 (null: Jacobi)
  const int32_t* mptr4 = nullptr;
  const int32_t* mcol4 = nullptr;
  const void* msq = nullptr;          // its diag(K)^-1/2, typed like the vectors
  void* rh = nullptr;                 // s r, typed like the vectors
  const double* rsum = nullptr;       // set (FP32 values only): C of the corrected form
};

// Grid of the LDS-staged product: one workgroup per chunk up to the cap,
// a multiple of the XCD count.
int lds_grid(Ctx& c, const RowSched& rs) {
  const int64_t n_chunks = div_up(c.N, kChunkRows);
  int g = int(std::min<int64_t>(n_chunks, std::min(rs.grid_cap, kRowGridMax)));
  return div_up(g, kXcds) * kXcds;
}

}  // namespace

// Block row sums R of the FP64 K_bc (once per assembly).
void ensure_rowsum(Ctx& c) {
  if (c.have_rsum) return;
  ensure_packed64(c);
  c.rsum.reserve(9 * c.N);
  k_rowsum<false><<<div_up(9 * c.N, 256), 256, 0, c.stream>>>(c.N, c.ptr4.get(), c.valp.get(),
                                                               nullptr, c.rsum.get());
  SFEM_HIP(hipGetLastError());
  c.have_rsum = true;
}

// C = R - R32, the block row sums of the FP32 copy's rounding (once per
// assembly).
void ensure_rowcorr(Ctx& c) {
  if (c.have_rcorr) return;
  ensure_packed64(c);
  ensure_packed32(c);
  c.rcorr.reserve(9 * c.N);
  k_rowsum<true><<<div_up(9 * c.N, 256), 256, 0, c.stream>>>(c.N, c.ptr4.get(), c.valp.get(),
                                                              c.valp32.get(), c.rcorr.get());
  SFEM_HIP(hipGetLastError());
  c.have_rcorr = true;
}

namespace {

int lds_grid(Ctx& c, const RowSched& rs);

int mapply_parts(Ctx& c) {
  if (c.mapply_kernel == 1) return lds_grid(c, RowSched{17, kRowGridMax});
  const RowSched rs{0, kRowGridMax};
  const int64_t rows_per_block = int64_t(kRowWaves) * (kWave / kMLanes);
  int g = div_up(c.N, rows_per_block);
  g = g < rs.grid_cap ? g : rs.grid_cap;
  return div_up(g, kXcds) * kXcds;  // for_rows needs a multiple of kXcds
}

// z = M r; with fresh_rh the scaled residual rh = s r is formed first (it
// is otherwise maintained by k_cg_xr).
// partials: 3 mapply_parts(c) doubles (null: the context's).
template <typename P>
void mapply(Ctx& c, const CgBuffers& B, const P* r, P* z, bool guarded, bool fresh_rh,
            double* partials = nullptr) {
  const int64_t n = c.n_dof();
  if (fresh_rh) {
    k_rh<P><<<div_up(n, 256), 256, 0, c.stream>>>(n, (const P*)B.msq, r, (P*)B.rh);
    SFEM_HIP(hipGetLastError());
  }
  if (c.mapply_kernel == 1) {
    k_mapply_lds<P><<<mapply_parts(c), kLdsThreads, 0, c.stream>>>(
        c.N, B.mptr4, c.lcol4.get(), B.mval, c.wcol.get(), c.wcnt.get(), (const P*)B.msq, r,
        (const P*)B.rh, z, guarded ? c.sc.get() : nullptr, partials ? partials : c.partials.get());
  } else if (c.mapply_kernel == 2) {
    k_mapply_grp<P><<<mapply_parts(c), kRowWaves * kWave, 0, c.stream>>>(
        c.N, B.mptr4, c.mgrp.get(), (const P*)B.msq, r, (const P*)B.rh, z,
        guarded ? c.sc.get() : nullptr, partials ? partials : c.partials.get());
  } else {
    k_mapply<P><<<mapply_parts(c), kRowWaves * kWave, 0, c.stream>>>(
        c.N, B.mptr4, B.mcol4, B.mval, (const P*)B.msq, r, (const P*)B.rh, z,
        guarded ? c.sc.get() : nullptr, partials ? partials : c.partials.get());
  }
  SFEM_HIP(hipGetLastError());
}

// With c.profile set, every SpMV launch is bracketed by a pair of events;
// their elapsed times are summed once the chunk has finished.
template <typename VT, typename P>
void cg_iterations(Ctx& c, const CgBuffers& B, int iters, int& parity) {
  const int64_t N = c.N, n = c.n_dof();
  hipStream_t s = c.stream;
  const RowSched rs = sizeof(VT) == 8 ? c.sched64 : c.sched32;
  // schedule 17: the LDS-staged product (its tables were built when it
  // was chosen)
  const bool lds = (kSched[rs.variant].mode & 32) != 0 && c.lds_tables == 1;
  const int rg = lds ? lds_grid(c, rs) : row_grid(N, B.rsum ? tf_sched(rs) : rs);
  const int vg = vec_grid(n);
  if (c.profile)
    while (int(c.prof_ev.size()) < 4 * iters) {
      hipEvent_t e;
      SFEM_HIP(hipEventCreate(&e));
      c.prof_ev.push_back(e);
    }
  (void)parity;
  // the corrected form's C belongs to the FP32 copy
  SFEM_REQUIRE(!B.rsum || sizeof(VT) == 4, SFEM_ESTATE, "the corrected form is for FP32 values");
  P* p = (P*)B.p0;
  const RowSched rt = tf_sched(rs);
  const Lay<VT> LY = lay<VT>(c, B.rsum ? rt : rs, (const VT*)B.val);
  for (int k = 0; k < iters; ++k) {
    k_cg_p<P><<<vg, kVecThreads, 0, s>>>(n, (const P*)B.z, p, c.sc.get());
    if (c.profile) SFEM_HIP(hipEventRecord(c.prof_ev[4 * k], s));
#define L_(LPR, MODE)                                                                          \
  k_cg_spmv<VT, P, LPR, MODE><<<rg, kRowWaves * kWave, 0, s>>>(N, LY.ptr, LY.col, LY.val,       \
                                                                p, (P*)B.q, c.sc.get(),  \
                                                                c.partials.get(), B.rsum)
    if (lds) {
      if constexpr (sizeof(VT) == 4) {
        if (B.rsum)
          k_cg_spmv_lds<VT, P, 8, true><<<rg, kLdsThreads, 0, s>>>(
              N, LY.ptr, c.lcol4.get(), LY.val, c.wcol.get(), c.wcnt.get(), p, (P*)B.q,
              c.sc.get(), c.partials.get(), B.rsum);
        else
          k_cg_spmv_lds<VT, P, 8, false><<<rg, kLdsThreads, 0, s>>>(
              N, LY.ptr, c.lcol4.get(), LY.val, c.wcol.get(), c.wcnt.get(), p, (P*)B.q,
              c.sc.get(), c.partials.get(), nullptr);
      } else {
        k_cg_spmv_lds<VT, P, 8, false><<<rg, kLdsThreads, 0, s>>>(
            N, LY.ptr, c.lcol4.get(), LY.val, c.wcol.get(), c.wcnt.get(), p, (P*)B.q,
            c.sc.get(), c.partials.get(), nullptr);
      }
    } else if (B.rsum) {
      if constexpr (sizeof(VT) == 4) SFEM_CF_SWITCH(kSched[rt.variant].lpr, L_)
    } else {
      SFEM_SCHED_SWITCH(rs.variant, L_)
    }
#undef L_
    if (c.profile) SFEM_HIP(hipEventRecord(c.prof_ev[4 * k + 1], s));
    finalize(c, kFinAlpha, rg);
    if (B.mval) {
      k_cg_xr<P><<<vg, kVecThreads, 0, s>>>(n, (P*)B.x, (P*)B.r, p, (const P*)B.q,
                                            (const P*)B.msq, (P*)B.rh, c.sc.get());
      if (c.profile) SFEM_HIP(hipEventRecord(c.prof_ev[4 * k + 2], s));
      mapply<P>(c, B, (const P*)B.r, (P*)B.z, true, false);
      if (c.profile) SFEM_HIP(hipEventRecord(c.prof_ev[4 * k + 3], s));
      finalize(c, kFinBetaFlex, mapply_parts(c));
    } else {
      k_cg_update<P><<<vg, kVecThreads, 0, s>>>(n, (P*)B.x, (P*)B.r, (P*)B.z, p, (const P*)B.q,
                                                (const P*)B.dinv, c.sc.get(), c.partials.get());
      finalize(c, kFinBeta, vg);
    }
  }
  SFEM_HIP(hipGetLastError());
}

// One full check period of iterations replayed from a hipGraph (captured
// on first use and whenever an address, size or schedule it launched with
// has changed); the first period of a solve runs eagerly (it also builds
// any packed copy the schedule needs, which must not be captured).  Small
// meshes' iterations are launch-bound: five short kernels each.
template <typename VT, typename P>
void cg_period(Ctx& c, const CgBuffers& B, int iters, int& parity, bool eager) {
  if (eager || c.profile || !c.graph_replay) {
    cg_iterations<VT, P>(c, B, iters, parity);
    return;
  }
  const RowSched rs = sizeof(VT) == 8 ? c.sched64 : c.sched32;
  const Lay<VT> LY = lay<VT>(c, B.rsum ? tf_sched(rs) : rs, (const VT*)B.val);
  const std::vector<const void*> key = {
      B.val, B.dinv, B.x, B.r, B.z, B.p0, B.q, B.mval, B.mptr4, B.mcol4, B.msq, B.rh, B.rsum,
      c.lcol4.get(), c.wcol.get(),
      LY.ptr, LY.col, LY.val, c.sc.get(), c.partials.get(),
      reinterpret_cast<const void*>(intptr_t(c.N)), reinterpret_cast<const void*>(intptr_t(iters)),
      reinterpret_cast<const void*>(intptr_t(rs.variant * 100000 + rs.grid_cap)),
      reinterpret_cast<const void*>(intptr_t(sizeof(VT) * 16 + sizeof(P))),
      reinterpret_cast<const void*>(intptr_t(c.mapply_kernel)), c.mgrp.get()};
  if (!c.cg_exec || c.cg_key != key) {
    c.drop_cg_graph();
    SFEM_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    try {
      cg_iterations<VT, P>(c, B, iters, parity);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    SFEM_HIP(hipStreamEndCapture(c.stream, &c.cg_graph));
    SFEM_HIP(hipGraphInstantiate(&c.cg_exec, c.cg_graph, nullptr, nullptr, 0));
    c.cg_key = key;
  }
  SFEM_HIP(hipGraphLaunch(c.cg_exec, c.stream));
}

// Adds the SpMV (and learned M) launches of the last chunk that did work (a
// launch that returned at once because the solve had converged is not
// counted).
void collect_profile(Ctx& c, int iters, int done_before, int done_after, bool learned) {
  if (!c.profile) return;
  SFEM_HIP(hipStreamSynchronize(c.stream));
  const int worked = std::min(iters, done_after - done_before);
  for (int k = 0; k < worked; ++k) {
    float ms = 0;
    SFEM_HIP(hipEventElapsedTime(&ms, c.prof_ev[4 * k], c.prof_ev[4 * k + 1]));
    c.prof_ms += ms;
    c.prof_n += 1;
    if (learned) {
      SFEM_HIP(hipEventElapsedTime(&ms, c.prof_ev[4 * k + 2], c.prof_ev[4 * k + 3]));
      c.prof_mms += ms;
      c.prof_mn += 1;
    }
  }
}

// The replacement residual b - K x.  With the FP64 K_bc (every solve that
// replaces: VT = double) it is computed in the translation form, whose
// rounding is relative to the neighbour differences of x: the FP64 true
// residual then resolves levels far below eps || |K| |x| || / ||b||, the
// floor of the plain sum (3.7e-9 relative on the 1.92M-tet cantilever).
template <typename VT, typename P>
void cg_replace(Ctx& c, const CgBuffers& B) {
  const RowSched rs = sizeof(VT) == 8 ? c.sched64 : c.sched32;
  int rg = row_grid(c.N, rs);
#define L_(LPR, MODE)                                                                          \
  k_cg_replace<VT, P, LPR, MODE><<<rg, kRowWaves * kWave, 0, c.stream>>>(                     \
      c.N, LY.ptr, LY.col, LY.val, (const P*)B.b, (const P*)B.x, (P*)B.r, (P*)B.z,            \
      (const P*)B.dinv, c.partials.get(), c.rsum.get())
  if constexpr (sizeof(VT) == 8) {
    const bool own = (const void*)B.val_true == (const void*)c.val.get();
    if (own) ensure_rowsum(c);
    const RowSched rt = tf_sched(rs);
    const Lay<VT> LY = lay<VT>(c, own ? rt : rs, (const VT*)B.val_true);
    if (own) {
      rg = row_grid(c.N, rt);
      SFEM_TF_SWITCH(kSched[rt.variant].lpr, L_)
    } else {
      SFEM_SCHED_SWITCH(rs.variant, L_)
    }
  } else {
    const Lay<VT> LY = lay<VT>(c, rs, (const VT*)B.val_true);
    SFEM_SCHED_SWITCH(rs.variant, L_)
  }
#undef L_
  SFEM_HIP(hipGetLastError());
  finalize(c, kFinReplace, rg);
  if (B.mval) {
    mapply<P>(c, B, (const P*)B.r, (P*)B.z, false, true);
    finalize(c, kFinReplaceM, mapply_parts(c));
  }
}

void read_scalars(Ctx& c) {
  SFEM_HIP(hipMemcpyAsync(c.sc_host, c.sc.get(), sizeof(CgScalars), hipMemcpyDeviceToHost,
                          c.stream));
  SFEM_HIP(hipStreamSynchronize(c.stream));
}

// Iteration counter := 0 and the r.r convergence threshold.
__global__ void k_cg_arm(CgScalars* sc, double tol2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->aux[0] = 0.0;
    sc->aux[1] = tol2;
  }
}

__global__ void k_cg_clear(CgScalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc->converged = 0;
}

// One PCG solve of A x = b from x = 0.  With `replace` it stops when the
// true residual (the replacement residual, computed in the solve's own
// precision) satisfies ||r|| <= tol_abs, after max_iter iterations, or on
// stagnation near the tolerance.  Without it (inner solves of the
// refinement, whose accuracy the FP64 outer residual judges) it stops on the
// recursive residual, which keeps falling below the working precision's
// floor.  b is FP64 (scaled into P).  Returns the iterations done.
//
// late (with replace): once the true residual has reached sqrt(late_tol2),
// the remaining periods run late's products (FP32 values, VT = float) and
// continue the same recurrence: x, r, z, p and the scalars carry over (the
// product's rounding matters least late in the solve, when the updates are
// small; early in the solve it costs conjugacy).
template <typename VT, typename P, typename VTR = VT>
int pcg(Ctx& c, const CgBuffers& B, const double* b64, double inv_scale, double tol_abs,
        int max_iter, int check_every, bool& met, bool& breakdown, bool replace = true,
        const std::function<void(int)>* hook = nullptr,
        const std::function<int(int)>* next_stop = nullptr,
        const CgBuffers* late = nullptr, double late_tol2 = 0.0) {
  const int64_t n = c.n_dof();
  hipStream_t s = c.stream;
  const double tol2 = tol_abs * tol_abs;
  // B.b is the P-typed right-hand side the replacement uses; when it is b64
  // itself (FP64 solve) there is nothing to convert
  P* bconv = (static_cast<const void*>(B.b) == static_cast<const void*>(b64)) ? nullptr : (P*)B.b;
  const int vg = vec_grid(n);
  k_cg_start<P><<<vg, kVecThreads, 0, s>>>(n, b64, inv_scale, bconv, (P*)B.x, (P*)B.r, (P*)B.z,
                                           (P*)B.p0, (P*)B.p1, (const P*)B.dinv,
                                           c.partials.get());
  SFEM_HIP(hipGetLastError());
  finalize(c, kFinStart, vg);
  if (B.mval) {
    mapply<P>(c, B, (const P*)B.r, (P*)B.z, false, true);
    finalize(c, kFinStartM, mapply_parts(c));
  }
  k_cg_arm<<<1, 64, 0, s>>>(c.sc.get(), tol2);
  SFEM_HIP(hipGetLastError());
  read_scalars(c);
  met = c.sc_host->rr <= tol2;
  breakdown = c.sc_host->converged == 2;
  if (breakdown) return 0;
  int done = 0, parity = 0;
  double best = c.sc_host->rr;
  int stale = 0;  // checks without a new best, counted once near the tolerance
  bool in_late = false, late_eager = false;
  while (!met && done < max_iter && stale < 40) {
    int chunk = std::min(check_every, max_iter - done);
    // end the period at the caller's next stop (snapshots), if one is sooner
    if (next_stop) chunk = std::max(1, std::min(chunk, (*next_stop)(done) - done));
    if (in_late) {
      // the first late period runs eagerly: it builds the packed FP32 copy
      cg_period<float, P>(c, *late, chunk, parity, late_eager || chunk != check_every);
      late_eager = false;
    } else {
      cg_period<VT, P>(c, B, chunk, parity, done == 0 || chunk != check_every);
    }
    if (replace) cg_replace<VTR, P>(c, B);
    read_scalars(c);
    const int before = done;
    done = int(c.sc_host->aux[0]);
    collect_profile(c, chunk, before, done, B.mval != nullptr);
    if (hook && done > before) (*hook)(done);
    if (!replace) {
      met = c.sc_host->converged == 1;
      if (c.sc_host->converged == 2) breakdown = true;
      if (met || breakdown || done == before) break;
      continue;
    }
    met = c.sc_host->rr_true <= tol2;
    if (late && !in_late && c.sc_host->rr_true <= late_tol2) in_late = late_eager = true;
    if (c.sc_host->rr_true < best) {
      best = c.sc_host->rr_true;
      stale = 0;
    } else if (best <= 1e4 * tol2 || B.mval) {
      // Jacobi: stagnation counts only near the tolerance; the learned M
      // (not guaranteed positive definite) gets the same budget anywhere
      ++stale;
    }
    if (c.sc_host->converged == 2) {
      breakdown = true;
      break;
    }
    if (c.sc_host->converged == 1 && !met) {
      k_cg_clear<<<1, 64, 0, s>>>(c.sc.get());
      SFEM_HIP(hipGetLastError());
    }
    if (done == before && !met) break;  // no progress possible
  }
  return done;
}

}  // namespace

void spmv_f64_sched(Ctx& c, const RowSched& rs, const double* val, const double* x, double* y,
                    hipStream_t s) {
  const int rg = row_grid(c.N, rs);
  const Lay<double> LY = lay<double>(c, rs, val);
#define L_(LPR, MODE)                                                        \
  k_spmv<double, double, LPR, MODE><<<rg, kRowWaves * kWave, 0, s>>>(        \
      c.N, LY.ptr, LY.col, LY.val, x, y)
  SFEM_SCHED_SWITCH(rs.variant, L_)
#undef L_
  SFEM_HIP(hipGetLastError());
}

void spmv_f32_sched(Ctx& c, const RowSched& rs, const float* val, const float* x, float* y,
                    hipStream_t s) {
  const int rg = row_grid(c.N, rs);
  const Lay<float> LY = lay<float>(c, rs, val);
#define L_(LPR, MODE)                                                      \
  k_spmv<float, float, LPR, MODE><<<rg, kRowWaves * kWave, 0, s>>>(        \
      c.N, LY.ptr, LY.col, LY.val, x, y)
  SFEM_SCHED_SWITCH(rs.variant, L_)
#undef L_
  SFEM_HIP(hipGetLastError());
}

void spmv_f32val(Ctx& c, const float* val, const double* x, double* y, hipStream_t s) {
  // any FP32 matrix in the CSR-order layout (no packed copy): a fixed schedule
  const RowSched rs{2, 4096};
  const int rg = row_grid(c.N, rs);
  k_spmv<float, double, 32, 0><<<rg, kRowWaves * kWave, 0, s>>>(c.N, c.topo.bptr.get(),
                                                                 c.topo.bcol.get(), val, x, y);
  SFEM_HIP(hipGetLastError());
}

void spmv_f64(Ctx& c, const double* val, const double* x, double* y, hipStream_t s) {
  spmv_f64_sched(c, c.sched64, val, x, y, s);
}

void spmv_f32(Ctx& c, const float* val, const float* x, float* y, hipStream_t s) {
  spmv_f32_sched(c, c.sched32, val, x, y, s);
}

// Times every row schedule (variant x grid cap) on this context's matrix
// with HIP events and keeps the fastest for FP64 and, if present, FP32.
static void ensure_work(Ctx& c, bool f32);

__global__ void k_ones(int64_t n, double* __restrict__ u) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) u[i] = 1.0;
}

// Times every row schedule (variant x grid cap) and keeps the fastest.
// FP64: `reps` Jacobi-PCG iterations on the context's matrix from a fixed
// start (b = 1), i.e. the product inside the loop where the vector kernels
// share the caches (an isolated product favours other schedules); the time
// per iteration is reported.  FP32 (if present): the same iterations with
// the FP32 values in the translation form (FP64 vectors), the FP32 copy's
// main use, over the packed schedules (the only ones with that form).
void autotune_rows(Ctx& c, int reps, double* best_us64, double* best_us32) {
  const int64_t n = c.n_dof();
  ensure_work(c, false);
  k_zero<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.x.get());
  k_ones<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.w.get());
  SFEM_HIP(hipGetLastError());
  const bool prof = c.profile;
  c.profile = false;
  const int caps[] = {1024, 2048, 4096, 8192};
  const RowSched keep64 = c.sched64;
  for (int prec = 0; prec < (c.have_f32 ? 2 : 1); ++prec) {
    double best = 1e30;
    RowSched pick = prec ? c.sched32 : keep64;
    if (prec == 1) ensure_rowcorr(c);
    for (int v = 0; v < kNumSched; ++v)
      for (int cap : caps) {
        if ((kSched[v].mode & 32) && !ensure_lds_tables(c)) continue;
        if (prec == 1 && !(kSched[v].mode & 8)) continue;
        const RowSched rs{v, cap};
        double us = 0.0;
        (prec == 0 ? c.sched64 : c.sched32) = rs;
        CgBuffers B{prec == 0 ? (const void*)c.val.get() : (const void*)c.val32.get(),
                    c.val.get(), c.dinv.get(), c.w.get(), c.x.get(), c.r.get(),
                    c.z.get(), c.p.get(), c.p2.get(), c.q.get()};
        if (prec == 1) B.rsum = c.rcorr.get();
        const int vg = vec_grid(n);
        k_cg_start<double><<<vg, kVecThreads, 0, c.stream>>>(
            n, c.w.get(), 1.0, nullptr, c.x.get(), c.r.get(), c.z.get(), c.p.get(), c.p2.get(),
            c.dinv.get(), c.partials.get());
        finalize(c, kFinStart, vg);
        k_cg_arm<<<1, 64, 0, c.stream>>>(c.sc.get(), 0.0);
        int parity = 0;
        if (prec == 0) {
          cg_iterations<double, double>(c, B, 2, parity);  // warm
          SFEM_HIP(hipEventRecord(c.ev0, c.stream));
          cg_iterations<double, double>(c, B, reps, parity);
          SFEM_HIP(hipEventRecord(c.ev1, c.stream));
        } else {
          cg_iterations<float, double>(c, B, 2, parity);  // warm
          SFEM_HIP(hipEventRecord(c.ev0, c.stream));
          cg_iterations<float, double>(c, B, reps, parity);
          SFEM_HIP(hipEventRecord(c.ev1, c.stream));
        }
        SFEM_HIP(hipEventSynchronize(c.ev1));
        float ms = 0;
        SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
        us = 1e3 * ms / reps;
        if (us < best) {
          best = us;
          pick = rs;
        }
      }
    if (prec == 0) {
      c.sched64 = pick;
      if (best_us64) *best_us64 = best;
    } else {
      c.sched32 = pick;
      if (best_us32) *best_us32 = best;
    }
  }
  c.profile = prof;
}

// r = f - K u with the FP64 K_bc, in the translation form (see cg_replace).
void resid64(Ctx& c, const double* u, double* r) {
  ensure_rowsum(c);
  const RowSched rt = tf_sched(c.sched64);
  const int rg = row_grid(c.N, rt);
  const Lay<double> LY = lay<double>(c, rt, c.val.get());
#define L_(LPR, MODE)                                                                 \
  k_resid64<LPR, MODE><<<rg, kRowWaves * kWave, 0, c.stream>>>(                       \
      c.N, LY.ptr, LY.col, LY.val, c.f_bc.get(), u, r, c.partials.get(), c.rsum.get())
  SFEM_TF_SWITCH(kSched[rt.variant].lpr, L_)
#undef L_
  SFEM_HIP(hipGetLastError());
  finalize(c, kFinResid, rg);
}

double true_residual(Ctx& c, const double* u) {
  resid64(c, u, c.w.get());
  read_scalars(c);
  const double ff = c.sc_host->ff;
  return ff > 0 ? std::sqrt(c.sc_host->rr_true / ff) : std::sqrt(c.sc_host->rr_true);
}

static void ensure_work(Ctx& c, bool f32) {
  const int64_t n = c.n_dof();
  c.x.reserve(n);
  c.r.reserve(n);
  c.z.reserve(n);
  c.p.reserve(n);
  c.p2.reserve(n);
  c.q.reserve(n);
  c.w.reserve(n);
  c.xs.reserve(n);
  c.rh.reserve(n);
  if (f32) {
    c.rh32.reserve(n);
    c.x32.reserve(n);
    c.r32.reserve(n);
    c.z32.reserve(n);
    c.p32.reserve(n);
    c.p32b.reserve(n);
    c.q32.reserve(n);
    c.b32.reserve(n);
  }
  c.partials.reserve(3 * std::max(kRowGridMax, kVecGridMax) + 16);
}

__global__ void k_axpy64(int64_t n, const double* __restrict__ d, double* __restrict__ u) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) u[i] += d[i];
}

// From the current x: solve K d = f - K x by FP64 PCG with B's
// preconditioner and add d (the restart of SFEM_MODE_F32_RR).
static int refine64(Ctx& c, const CgBuffers& B, double tol_abs, int max_iter, int check_every,
                    bool& met, bool& brk) {
  const int64_t n = c.n_dof();
  SFEM_HIP(hipMemcpyAsync(c.xs.get(), c.x.get(), sizeof(double) * n, hipMemcpyDeviceToDevice,
                          c.stream));
  resid64(c, c.xs.get(), c.w.get());
  CgBuffers J = B;
  J.val = c.val.get();
  J.val_true = c.val.get();
  J.rsum = nullptr;  // plain FP64 products
  J.b = c.w.get();
  const int its = pcg<double, double>(c, J, c.w.get(), 1.0, tol_abs, max_iter, check_every, met,
                                      brk);
  k_axpy64<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.xs.get(), c.x.get());
  SFEM_HIP(hipGetLastError());
  return its;
}

// Jacobi fallback after a learned solve stopped short: from the current x,
// solve K d = f - K x with Jacobi PCG and add d.  Returns the iterations.
static int jacobi_fallback(Ctx& c, const CgBuffers& B, double tol_abs, int max_iter,
                           int check_every, bool& met) {
  const int64_t n = c.n_dof();
  SFEM_HIP(hipMemcpyAsync(c.xs.get(), c.x.get(), sizeof(double) * n, hipMemcpyDeviceToDevice,
                          c.stream));
  resid64(c, c.xs.get(), c.w.get());
  CgBuffers J = B;
  J.val = c.val.get();
  J.val_true = c.val.get();
  J.rsum = nullptr;  // plain FP64 products
  J.mval = nullptr;
  J.b = c.w.get();
  bool brk = false;
  const int its = pcg<double, double>(c, J, c.w.get(), 1.0, tol_abs, max_iter, check_every, met,
                                      brk);
  k_axpy64<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.xs.get(), c.x.get());
  SFEM_HIP(hipGetLastError());
  return its;
}

int solve(Ctx& c, const sfem_solve_opts& o, sfem_solve_info& info) {
  const int64_t n = c.n_dof();
  SFEM_REQUIRE(o.mode == SFEM_MODE_F64 || o.mode == SFEM_MODE_F32_IR ||
                   o.mode == SFEM_MODE_F32_RR || o.mode == SFEM_MODE_F32_TF,
               SFEM_EINVAL, "unknown solve mode");
  SFEM_REQUIRE(o.precond == SFEM_PRECOND_JACOBI || o.precond == SFEM_PRECOND_LEARNED,
               SFEM_EINVAL, "unknown preconditioner");
  const bool learned = o.precond == SFEM_PRECOND_LEARNED;
  SFEM_REQUIRE(!learned || c.have_learned, SFEM_ESTATE,
               "SFEM_PRECOND_LEARNED needs sfem_gnn_apply on this context first");
  const bool f32 = o.mode == SFEM_MODE_F32_IR;
  ensure_work(c, f32);
  // FP64 products: 100-iteration periods (fewer replacements and host
  // reads; measured 1-2% faster than 50 for Jacobi and learned M at 1.9M
  // tets).  FP32 products: 50, to bound their drift between replacements.
  const int check_every = o.check_every > 0 ? o.check_every : (o.mode == SFEM_MODE_F64 ? 100 : 50);
  const int max_iter = o.max_iter > 0 ? o.max_iter : 100000;
  c.profile = o.profile != 0;
  c.prof_ms = 0;
  c.prof_n = 0;
  c.prof_mms = 0;
  c.prof_mn = 0;
  SFEM_HIP(hipEventRecord(c.ev0, c.stream));

  // ||f||: the residual of u = 0
  k_zero<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.x.get());
  SFEM_HIP(hipGetLastError());
  (void)true_residual(c, c.x.get());
  const double fnorm = std::sqrt(c.sc_host->ff);
  info = sfem_solve_info{};
  int status = SFEM_OK;
  if (fnorm == 0.0) {
    info.converged = 1;
  } else if (o.mode == SFEM_MODE_F64 || o.mode == SFEM_MODE_F32_RR ||
             o.mode == SFEM_MODE_F32_TF) {
    // F32_RR: K32 products, FP64 vectors and dots; every check_every
    // iterations the residual is replaced by the FP64 one, f - K64 x, which
    // is the refinement step and the convergence test.
    // F32_TF: the same with the K32 products in the translation form,
    // q_I = sum_J K32_IJ (p_J - p_I) + R_I p_I (R_I the FP64 block row
    // sums of K64), to the end: no restart.  The kernels compute it as
    // sum_J K32_IJ p_J + C_I p_I (the corrected form, C = R - R32).
    const bool rr = o.mode == SFEM_MODE_F32_RR;
    const bool tf = o.mode == SFEM_MODE_F32_TF;
    SFEM_REQUIRE(!(rr || tf) || c.have_f32, SFEM_ESTATE,
                 "SFEM_MODE_F32_RR and SFEM_MODE_F32_TF need sfem_assemble(..., "
                 "SFEM_ASM_F32_COPY)");
    CgBuffers B{(rr || tf) ? (const void*)c.val32.get() : (const void*)c.val.get(),
                c.val.get(), c.dinv.get(), c.f_bc.get(), c.x.get(), c.r.get(),
                c.z.get(), c.p.get(), c.p2.get(), c.q.get()};
    if (tf) {
      ensure_rowcorr(c);
      B.rsum = c.rcorr.get();
    }
    if (learned) {
      B.mval = c.mvalp.get();
      B.mptr4 = c.ptr4.get();
      B.mcol4 = c.col4.get();
      B.msq = c.msqrt.get();
      B.rh = c.rh.get();
    }
    bool met = false, brk = false;
    if (rr) {
      // FP32 products while the FP64 true residual is above the switch
      // level, then FP64 products, continuing the same recurrence
      const double sw = std::max(o.rtol, o.f32_until > 0 ? o.f32_until : 1e-3);
      info.iters = pcg<float, double, double>(c, B, c.f_bc.get(), 1.0, sw * fnorm, max_iter,
                                              check_every, met, brk);
      // then FP64 products, restarted on the correction K d = f - K u from
      // the current u (search directions built with FP32 products are not
      // conjugate for the FP64 matrix, so continuing the recurrence stalls)
      if (!brk && info.iters < max_iter && sw > o.rtol) {
        B.val = c.val.get();
        bool met2 = false;
        info.iters += refine64(c, B, o.rtol * fnorm, max_iter - info.iters, check_every, met2,
                               brk);
        met = met2;
      }
    } else if (tf && o.f32_from > o.rtol && o.f32_from < 1.0) {
      // FP64 products down to f32_from, then FP32 translation-form ones
      CgBuffers B64 = B;
      B64.val = c.val.get();
      B64.rsum = nullptr;
      const double lt = o.f32_from * fnorm;
      info.iters = pcg<double, double>(c, B64, c.f_bc.get(), 1.0, o.rtol * fnorm, max_iter,
                                       check_every, met, brk, true, nullptr, nullptr, &B,
                                       lt * lt);
    } else if (tf) {
      info.iters = pcg<float, double, double>(c, B, c.f_bc.get(), 1.0, o.rtol * fnorm, max_iter,
                                              check_every, met, brk);
    } else {
      info.iters = pcg<double, double>(c, B, c.f_bc.get(), 1.0, o.rtol * fnorm, max_iter,
                                       check_every, met, brk);
    }
    if (learned && !met && info.iters < max_iter) {
      info.fell_back = 1;
      info.iters += jacobi_fallback(c, B, o.rtol * fnorm, max_iter - info.iters, check_every,
                                    met);
    }
    info.outer_steps = (rr || tf) ? info.iters / check_every + 1 : 1;
    info.true_relres = true_residual(c, c.x.get());
    info.converged = info.true_relres <= o.rtol;
  } else {
    SFEM_REQUIRE(c.have_f32, SFEM_ESTATE,
                 "SFEM_MODE_F32_IR needs sfem_assemble(..., SFEM_ASM_F32_COPY)");
    const double inner = o.inner_rtol > 0 ? o.inner_rtol : 1e-2;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 30;
    double* u = c.x.get();
    k_zero<<<div_up(n, 256), 256, 0, c.stream>>>(n, u);
    SFEM_HIP(hipGetLastError());
    // inner solve K32 d = r / scale in FP32; d accumulates in x32
    CgBuffers B{c.val32.get(), c.val32.get(), c.dinv32.get(), c.b32.get(), c.x32.get(),
                c.r32.get(), c.z32.get(), c.p32.get(), c.p32b.get(), c.q32.get()};
    bool use_learned = learned;
    double relres = 1.0;
    int iters = 0, outer = 0;
    double* r64 = c.w.get();
    while (outer < max_outer && iters < max_iter) {
      resid64(c, u, r64);
      read_scalars(c);
      const double rnorm = std::sqrt(c.sc_host->rr_true);
      relres = rnorm / fnorm;
      if (relres <= o.rtol) break;
      const double scale = rnorm / std::sqrt(double(n));  // keeps FP32 values O(1)
      bool met = false, brk = false;
      const double tol = inner * std::sqrt(double(n));  // ||r / scale|| = sqrt(n)
      B.mval = use_learned ? c.mvalp.get() : nullptr;
      B.mptr4 = c.ptr4.get();
      B.mcol4 = c.col4.get();
      B.msq = c.msqrt32.get();
      B.rh = c.rh32.get();
      iters += pcg<float, float>(c, B, r64, 1.0 / scale, tol, max_iter - iters,
                                 std::max(check_every, 200), met, brk, /*replace=*/false);
      k_axpy_f32<<<div_up(n, 256), 256, 0, c.stream>>>(n, scale, c.x32.get(), u);
      SFEM_HIP(hipGetLastError());
      ++outer;
      if (brk) {
        if (!use_learned) {
          status = SFEM_ENOCONV;
          break;
        }
        use_learned = false;  // M not positive definite here: Jacobi from now on
        info.fell_back = 1;
      }
    }
    info.iters = iters;
    info.outer_steps = outer;
    info.true_relres = true_residual(c, u);
    info.converged = info.true_relres <= o.rtol;
  }
  SFEM_HIP(hipEventRecord(c.ev1, c.stream));
  SFEM_HIP(hipEventSynchronize(c.ev1));
  float ms = 0;
  SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
  info.ms_solve = ms;
  info.n_spmv = c.prof_n;
  info.ms_spmv_avg = c.prof_n ? c.prof_ms / c.prof_n : 0.0;
  info.n_mapply = c.prof_mn;
  info.ms_mapply_avg = c.prof_mn ? c.prof_mms / c.prof_mn : 0.0;
  if (!info.converged && status == SFEM_OK) status = SFEM_ENOCONV;
  return status;
}

int jacobi_run(Ctx& c, const double* b, double tol_abs, int every, int max_iter,
               const std::function<void(int)>& hook,
               const std::function<int(int)>* next_stop) {
  ensure_work(c, false);
  c.profile = false;
  CgBuffers B{c.val.get(), c.val.get(), c.dinv.get(), (void*)b, c.x.get(), c.r.get(),
              c.z.get(), c.p.get(), c.p2.get(), c.q.get()};
  bool met = false, brk = false;
  return pcg<double, double>(c, B, b, 1.0, tol_abs, max_iter, every, met, brk, true, &hook,
                             next_stop);
}

void pack_pattern(Ctx& c) {
  if (c.nb4 > 0) return;
  const int64_t N = c.N;
  hipStream_t s = c.stream;
  c.ptr4.reserve(N + 1);
  DBuf<int32_t> d4;
  d4.reserve(N);
  k_deg4<<<div_up(N, 256), 256, 0, s>>>(N, c.topo.bptr.get(), d4.get());
  SFEM_HIP(hipGetLastError());
  exclusive_scan_i32(d4.get(), c.ptr4.get(), N, s);
  int32_t nb4 = 0;
  SFEM_HIP(hipMemcpyAsync(&nb4, c.ptr4.get() + N, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SFEM_HIP(hipStreamSynchronize(s));
  c.col4.reserve(nb4);
  k_col4<<<div_up(N, 256), 256, 0, s>>>(N, c.topo.bptr.get(), c.topo.bcol.get(), c.ptr4.get(),
                                         c.col4.get());
  SFEM_HIP(hipGetLastError());
  c.nb4 = nb4;
}

// CSR-order FP32 values -> packed BF16 (round to nearest even).
__global__ void k_pack_bf16(int64_t N, const int32_t* __restrict__ bptr,
                            const int32_t* __restrict__ p4, const float* __restrict__ csr,
                            __bf16* __restrict__ packed) {
  const int lane = threadIdx.x & 63;
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
  if (I >= N) return;
  const int rb = bptr[I], deg = bptr[I + 1] - rb, r4 = p4[I], d4 = p4[I + 1] - r4;
  const float* src = csr + 9 * int64_t(rb);
  __bf16* dst = packed + 9 * int64_t(r4);
  for (int k = lane; k < 9 * d4; k += 64) {
    const int q = k / d4, j = k - q * d4;
    const int a = q / 3, c = q - 3 * a;
    dst[k] = __bf16(j < deg ? src[a * 3 * deg + 3 * j + c] : 0.f);
  }
}

void pack_values_bf16(Ctx& c, const float* csr, __bf16* packed) {
  pack_pattern(c);
  k_pack_bf16<<<div_up(c.N * 64, 256), 256, 0, c.stream>>>(c.N, c.topo.bptr.get(),
                                                            c.ptr4.get(), csr, packed);
  SFEM_HIP(hipGetLastError());
}

void pack_values_f32(Ctx& c, const float* csr, float* packed) {
  pack_pattern(c);
  k_pack<float><<<div_up(c.N * 64, 256), 256, 0, c.stream>>>(c.N, c.topo.bptr.get(),
                                                              c.ptr4.get(), csr, packed);
  SFEM_HIP(hipGetLastError());
}

namespace {
// Packed layout -> CSR order; one wave per node row.
__global__ void k_unpack(int64_t N, const int32_t* __restrict__ bptr,
                         const int32_t* __restrict__ p4, const double* __restrict__ packed,
                         double* __restrict__ csr) {
  const int lane = threadIdx.x & 63;
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
  if (I >= N) return;
  const int rb = bptr[I], deg = bptr[I + 1] - rb, r4 = p4[I], d4 = p4[I + 1] - r4;
  const double* src = packed + 9 * int64_t(r4);
  double* dst = csr + 9 * int64_t(rb);
  const int three_deg = 3 * deg;
  for (int k = lane; k < 9 * deg; k += 64) {
    const int a = k / three_deg, r = k - a * three_deg;
    const int j = r / 3, cc = r - 3 * j;
    dst[k] = src[(3 * a + cc) * d4 + j];
  }
}

// diag(K) from the packed copy: the row's self block is its first block
// column equal to I (the padding repeats I after the real columns).
__global__ void k_diag_packed(int64_t N, const int32_t* __restrict__ p4,
                              const int32_t* __restrict__ c4, const double* __restrict__ packed,
                              double* __restrict__ diag) {
  const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int r4 = p4[I], d4 = p4[I + 1] - r4;
  int j = 0;
  while (j < d4 - 1 && c4[r4 + j] != int(I)) ++j;
  const double* row = packed + 9 * int64_t(r4);
  for (int a = 0; a < 3; ++a) diag[3 * I + a] = row[4 * a * d4 + j];
}
}  // namespace

bool ensure_lds_tables(Ctx& c) {
  if (c.lds_tables != 0) return c.lds_tables == 1;
  pack_pattern(c);
  const int64_t n_chunks = div_up(c.N, kChunkRows);
  c.wcol.reserve(n_chunks * kWindow);
  c.wcnt.reserve(n_chunks);
  c.lcol4.reserve(c.nb4);
  TmpBuf<int32_t> fail(1, c.stream);
  SFEM_HIP(hipMemsetAsync(fail.get(), 0, sizeof(int32_t), c.stream));
  k_lds_tables<<<int(n_chunks), 256, 0, c.stream>>>(c.N, c.ptr4.get(), c.col4.get(), c.wcol.get(),
                                                     c.wcnt.get(), c.lcol4.get(), fail.get());
  SFEM_HIP(hipGetLastError());
  int32_t f = 0;
  SFEM_HIP(hipMemcpyAsync(&f, fail.get(), sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  SFEM_HIP(hipStreamSynchronize(c.stream));
  c.lds_tables = f ? -1 : 1;
  return c.lds_tables == 1;
}

void ensure_csr64(Ctx& c) {
  if (c.csr64) return;
  SFEM_REQUIRE(c.packed64, SFEM_ESTATE, "no current copy of K");
  c.val.reserve(9 * c.topo.nb);
  k_unpack<<<div_up(c.N * 64, 256), 256, 0, c.stream>>>(c.N, c.topo.bptr.get(), c.ptr4.get(),
                                                          c.valp.get(), c.val.get());
  SFEM_HIP(hipGetLastError());
  c.csr64 = true;
}

namespace {
__global__ void k_diag_csr(int64_t N, const int32_t* __restrict__ bptr,
                           const int32_t* __restrict__ bcol, const double* __restrict__ val,
                           double* __restrict__ diag) {
  const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int rb = bptr[I], deg = bptr[I + 1] - rb;
  int jj = 0;
  while (jj < deg - 1 && bcol[rb + jj] != int(I)) ++jj;
  for (int a = 0; a < 3; ++a) diag[3 * I + a] = val[9 * int64_t(rb) + a * 3 * deg + 3 * jj + a];
}
}  // namespace

void matrix_diagonal(Ctx& c, double* diag) {
  if (c.csr64) {
    k_diag_csr<<<div_up(c.N, 256), 256, 0, c.stream>>>(c.N, c.topo.bptr.get(), c.topo.bcol.get(),
                                                        c.val.get(), diag);
  } else {
    SFEM_REQUIRE(c.packed64, SFEM_ESTATE, "no current copy of K");
    k_diag_packed<<<div_up(c.N, 256), 256, 0, c.stream>>>(c.N, c.ptr4.get(), c.col4.get(),
                                                           c.valp.get(), diag);
  }
  SFEM_HIP(hipGetLastError());
}

namespace {
void ensure_packed64(Ctx& c) {
  if (c.packed64) return;
  SFEM_REQUIRE(c.csr64, SFEM_ESTATE, "no current copy of K");
  pack_pattern(c);
  c.valp.reserve(9 * c.nb4);
  k_pack<double><<<div_up(c.N * 64, 256), 256, 0, c.stream>>>(c.N, c.topo.bptr.get(),
                                                               c.ptr4.get(), c.val.get(),
                                                               c.valp.get());
  SFEM_HIP(hipGetLastError());
  c.packed64 = true;
}

void ensure_packed32(Ctx& c) {
  if (c.packed32) return;
  SFEM_REQUIRE(c.have_f32, SFEM_ESTATE, "no FP32 copy of K to pack");
  c.valp32.reserve(9 * c.nb4 > 0 ? 9 * c.nb4 : 1);
  pack_pattern(c);
  c.valp32.reserve(9 * c.nb4);
  pack_values_f32(c, c.val32.get(), c.valp32.get());
  c.packed32 = true;
}
}  // namespace

void pack_values64(Ctx& c) { ensure_packed64(c); }


// z = M r with caller-provided work memory: rh (3 N doubles) and partials
// (learned_apply_partials(c) doubles).  Allocates nothing.
int64_t learned_apply_partials(Ctx& c) { return 3 * int64_t(mapply_parts(c)); }

void learned_apply_into(Ctx& c, const double* r, double* z, double* rh, double* partials) {
  SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "no learned preconditioner on this context");
  CgBuffers B{};
  B.mval = c.mvalp.get();
  B.mptr4 = c.ptr4.get();
  B.mcol4 = c.col4.get();
  B.msq = c.msqrt.get();
  B.rh = rh;
  mapply<double>(c, B, r, z, false, true, partials);
}

void tune_mapply(Ctx& c, int variant) {
  SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "no learned preconditioner on this context");
  SFEM_REQUIRE(variant >= -1 && variant <= 2, SFEM_EINVAL,
               "M apply variant must be -1, 0, 1 or 2");
  const bool lds_ok = ensure_lds_tables(c);
  SFEM_REQUIRE(variant != 1 || lds_ok, SFEM_EINVAL,
               "a chunk of rows gathers more than the LDS window holds");
  SFEM_REQUIRE(variant != 2 || c.mgrp_ok, SFEM_EINVAL,
               "a block column lies beyond the grouped layout's int16 offsets");
  ensure_work(c, false);
  const int64_t n = c.n_dof();
  CgBuffers B{};
  B.mval = c.mvalp.get();
  B.mptr4 = c.ptr4.get();
  B.mcol4 = c.col4.get();
  B.msq = c.msqrt.get();
  B.rh = c.rh.get();
  k_ones<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.r.get());
  SFEM_HIP(hipGetLastError());
  c.mapply_us[0] = c.mapply_us[1] = c.mapply_us[2] = 0.0;
  constexpr int kReps = 10;
  for (int v = 0; v < 3; ++v) {
    if ((v == 1 && !lds_ok) || (v == 2 && !c.mgrp_ok)) continue;
    if (variant >= 0 && v != variant) continue;
    c.mapply_kernel = v;
    mapply<double>(c, B, c.r.get(), c.z.get(), false, true);  // warm
    SFEM_HIP(hipEventRecord(c.ev0, c.stream));
    for (int k = 0; k < kReps; ++k) mapply<double>(c, B, c.r.get(), c.z.get(), false, false);
    SFEM_HIP(hipEventRecord(c.ev1, c.stream));
    SFEM_HIP(hipEventSynchronize(c.ev1));
    float ms = 0;
    SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    c.mapply_us[v] = 1e3 * ms / kReps;
  }
  if (variant >= 0) {
    c.mapply_kernel = variant;
  } else {
    c.mapply_kernel = 0;
    for (int v = 1; v < 3; ++v)
      if (c.mapply_us[v] > 0.0 && c.mapply_us[v] < c.mapply_us[c.mapply_kernel])
        c.mapply_kernel = v;
  }
}

// S' in the grouped layout (after every new packed copy of M).
void build_mgroups(Ctx& c) {
  c.mgrp.reserve(c.nb4 > 0 ? 5 * int64_t(c.nb4 / 4) : 1);
  DBuf<int> bad;
  bad.reserve(1);
  SFEM_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), c.stream));
  k_mgroup<<<div_up(c.N, 256), 256, 0, c.stream>>>(c.N, c.ptr4.get(), c.col4.get(),
                                                   c.mvalp.get(), c.mgrp.get(), bad.get());
  SFEM_HIP(hipGetLastError());
  int b = 0;
  SFEM_HIP(hipMemcpyAsync(&b, bad.get(), sizeof(int), hipMemcpyDeviceToHost, c.stream));
  SFEM_HIP(hipStreamSynchronize(c.stream));
  c.mgrp_ok = b == 0;
  // a kernel chosen on the previous M stays valid only if this one fits
  if (!c.mgrp_ok && c.mapply_kernel == 2) {
    c.mapply_kernel = 0;
    c.mapply_tuned = false;
  }
}

void learned_apply(Ctx& c, const double* r, double* z) {
  SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "no learned preconditioner on this context");
  ensure_work(c, false);
  CgBuffers B{};
  B.mval = c.mvalp.get();
  B.mptr4 = c.ptr4.get();
  B.mcol4 = c.col4.get();
  B.msq = c.msqrt.get();
  B.rh = c.rh.get();
  mapply<double>(c, B, r, z, false, true);
}

}  // namespace sfem
