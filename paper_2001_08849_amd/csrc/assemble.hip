// Numeric FS-FEM assembly and the right-hand side.
//
// Per face k (Sec. 2.1 STEP 2-4): the smoothing domain is the sub-tet (face
// + centroid) of each adjacent tet, holding a quarter of that tet's volume,
// so V_k = (V_1 + V_2)/4.  Because the shape functions are linear in each
// tet and the Table-1 centroid rule is exact on each boundary triangle, the
// boundary sum of Eq. 7 equals (divergence theorem) the volume-weighted mean
// of the tet gradients:  b_I = (V_1 grad N_I^1 + V_2 grad N_I^2)/(V_1+V_2).
// The kernel evaluates that closed form in FP64 registers (tet volumes and
// inverse Jacobians by cross products, Eq. 10), then the 3x3 blocks of
// K_k = V_k B^T c B (Eq. 9) for isotropic c:
//   K_IJ = V_k [ lam b_I b_J^T + mu b_J b_I^T + mu (b_I . b_J) I_3 ].
//
// Scatter-assembly (Eq. 12 summed into CSR) is owner-computes by tile: a
// workgroup owns a run of consecutive node rows and holds their CSR values in
// LDS (as 64-bit fixed-point integers, see below).  Its work items are the (row, face) incidences of those rows: each
// evaluates the face in registers and adds the row's blocks with LDS
// atomics at column slots precomputed with the topology.  The finished rows
// are streamed to HBM once, coalesced, with the essential BCs applied on the
// way out.
#include "ctx.h"
#include "geom.h"

namespace sfem {

namespace {

constexpr int kAsmThreads = 256;

// Smoothed gradients b[0..n-1] of the face's support nodes (A, B, C, D[, E]),
// V_k, and the domain's Lame constants.
template <bool HET>
__device__ __forceinline__ int face_geometry(const int32_t* __restrict__ row,
                                             const double* __restrict__ xyz, double lam0,
                                             double mu0, const double* __restrict__ lam_t,
                                             const double* __restrict__ mu_t, int sup[5],
                                             Vec3 b[5], double& Vk, double& lam, double& mu) {
  int4 r0 = *reinterpret_cast<const int4*>(row);
  int4 r1 = *reinterpret_cast<const int4*>(row + 4);
  sup[0] = r0.x;
  sup[1] = r0.y;
  sup[2] = r0.z;
  sup[3] = r0.w;
  sup[4] = r1.x;
  const bool interior = r1.x >= 0;
  Vec3 A = load3(xyz, r0.x), B = load3(xyz, r0.y), C = load3(xyz, r0.z), D = load3(xyz, r0.w);
  // the second tet's far node, gathered with the others (a valid node id on
  // exterior faces too, where it is not used)
  const Vec3 E = load3(xyz, interior ? r1.x : r0.w);
  // The two tets share the face (A, B, C): with e1 = B - A, e2 = C - A,
  // n = e1 x e2 and the far-node offsets f_t = D - A, E - A, tet t's
  // gradients are (e2 x f_t, f_t x e1, n) / det_t for B, C and its far node,
  // det_t = f_t . n, and its volume |det_t| / 6.  The weights V_t / (V_1 +
  // V_2) then give, with k_t = sgn(det_t) / (|det_1| + |det_2|) and
  // g = k_1 f_1 + k_2 f_2:  b_B = e2 x g,  b_C = g x e1,  b_D = k_1 n,
  // b_E = k_2 n,  b_A = -(b_B + b_C + b_D + b_E)  (each tet's gradients sum
  // to zero): one division per face.  An exterior face takes the same path
  // with k_2 = 0, so a wave mixing both kinds runs it once.
  const Vec3 e1 = sub(B, A), e2 = sub(C, A);
  const Vec3 n = cross(e1, e2);
  const Vec3 f1 = sub(D, A), f2 = sub(E, A);
  const double d1 = dot(f1, n), d2 = dot(f2, n);
  const double a1 = fabs(d1), a2 = interior ? fabs(d2) : 0.0;
  const double inv = 1.0 / (a1 + a2);
  const double k1 = copysign(inv, d1), k2 = interior ? copysign(inv, d2) : 0.0;
  const Vec3 g = {k1 * f1.x + k2 * f2.x, k1 * f1.y + k2 * f2.y, k1 * f1.z + k2 * f2.z};
  b[1] = cross(e2, g);
  b[2] = cross(g, e1);
  b[3] = {k1 * n.x, k1 * n.y, k1 * n.z};
  b[4] = {k2 * n.x, k2 * n.y, k2 * n.z};
  b[0] = {-(b[1].x + b[2].x + b[3].x + b[4].x), -(b[1].y + b[2].y + b[3].y + b[4].y),
          -(b[1].z + b[2].z + b[3].z + b[4].z)};
  Vk = (a1 + a2) * (1.0 / 24.0);
  if (HET) {
    const double w1 = a1 * inv, w2 = a2 * inv;
    lam = w1 * lam_t[r1.y] + w2 * lam_t[interior ? r1.z : r1.y];
    mu = w1 * mu_t[r1.y] + w2 * mu_t[interior ? r1.z : r1.y];
  } else {
    lam = lam0;
    mu = mu0;
  }
  return interior ? 5 : 4;
}

// The same smoothing domain with FP32 arithmetic after the tet volumes and
// inverse Jacobians: V_1, V_2 and the tet gradients come from tet_grads in
// FP64; the volume weights, the smoothed gradients b, V_k and the Lame
// constants are formed in FP32.
struct F3 {
  float x, y, z;
};

template <bool HET>
__device__ __forceinline__ int face_geometry32(const int32_t* __restrict__ row,
                                               const double* __restrict__ xyz, double lam0,
                                               double mu0, const double* __restrict__ lam_t,
                                               const double* __restrict__ mu_t, int sup[5],
                                               F3 b[5], float& Vk, float& lam, float& mu) {
  int4 r0 = *reinterpret_cast<const int4*>(row);
  int4 r1 = *reinterpret_cast<const int4*>(row + 4);
  sup[0] = r0.x;
  sup[1] = r0.y;
  sup[2] = r0.z;
  sup[3] = r0.w;
  sup[4] = r1.x;
  const bool interior = r1.x >= 0;
  Vec3 A = load3(xyz, r0.x), B = load3(xyz, r0.y), C = load3(xyz, r0.z), D = load3(xyz, r0.w);
  const Vec3 E = load3(xyz, interior ? r1.x : r0.w);
  Vec3 g1[4];
  double V1;
  tet_grads(A, B, C, D, g1, V1);
  if (!interior) {
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = {float(g1[i].x), float(g1[i].y), float(g1[i].z)};
    b[4] = {0.f, 0.f, 0.f};
    Vk = 0.25f * float(V1);
    lam = HET ? float(lam_t[r1.y]) : float(lam0);
    mu = HET ? float(mu_t[r1.y]) : float(mu0);
    return 4;
  }
  Vec3 g2[4];
  double V2;
  tet_grads(A, B, C, E, g2, V2);
  const float v1 = float(V1), v2 = float(V2);
  const float W = v1 + v2;
  const float iW = 1.0f / W;
  const float w1 = v1 * iW, w2 = v2 * iW;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    b[i] = {w1 * float(g1[i].x) + w2 * float(g2[i].x), w1 * float(g1[i].y) + w2 * float(g2[i].y),
            w1 * float(g1[i].z) + w2 * float(g2[i].z)};
  b[3] = {w1 * float(g1[3].x), w1 * float(g1[3].y), w1 * float(g1[3].z)};
  b[4] = {w2 * float(g2[3].x), w2 * float(g2[3].y), w2 * float(g2[3].z)};
  Vk = 0.25f * W;
  if (HET) {
    lam = w1 * float(lam_t[r1.y]) + w2 * float(lam_t[r1.z]);
    mu = w1 * float(mu_t[r1.y]) + w2 * float(mu_t[r1.z]);
  } else {
    lam = float(lam0);
    mu = float(mu0);
  }
  return 5;
}

// Exponent e of a row's unit 2^(e - 50): 0.5 bmax < 2^e (half the largest
// face bound bounds every contribution), clamped so that 2^(50 - e) stays a
// normal double (a larger e only coarsens the unit of absurdly small rows).
__device__ __forceinline__ int16_t row_exponent(double bmax) {
  const int e = bmax > 0.0 ? ilogb(0.5 * bmax) + 1 : 0;
  return int16_t(e < -973 ? -973 : e);
}

// Largest face bound max(V_i G_i) among the faces incident to each node.
__global__ void k_row_bound(int64_t N, const int32_t* __restrict__ inc_ptr,
                            const int32_t* __restrict__ inc, const int32_t* __restrict__ face,
                            float* __restrict__ row_vg) {
  const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  float m = 0.0f;
  for (int e = inc_ptr[I]; e < inc_ptr[I + 1]; ++e)
    m = fmaxf(m, __int_as_float(face[int64_t(inc[e]) * kFaceStride + 7]));
  row_vg[I] = m;
}


// ---------------------------------------------------------- fixed-point unit
// A tile accumulates in 64-bit integers (LDS integer atomics are about twice
// as fast as FP64 ones on this chip, and integer sums do not depend on the
// order of the additions, so the matrix is bit-reproducible).
//
// Bound of one contribution.  An entry of V_k [lam b_p b_q^T + mu b_q b_p^T
// + mu (b_p.b_q) I] is at most (|lam| + 2 mu)_k V_k |b_p| |b_q|.  The
// domain's constants are convex combinations of its tets' ones, and with
// b = (V_1 g_1 + V_2 g_2) / (V_1 + V_2), V_k = (V_1 + V_2) / 4 and
// G_i = max_a |grad N_a^i|^2, Cauchy-Schwarz gives
//   V_k |b_p| |b_q| <= (V_1 G_1 + V_2 G_2) / 4 <= max(V_1 G_1, V_2 G_2) / 2.
// The face record keeps max(V_i G_i) (rounded up to FP32) in its spare word;
// a row's unit u is the power of two with every contribution of its items
// below 2^50 u, so the rounding is relative to the row's own magnitude
// whatever the material contrast across the mesh.  A contribution (in units of u) is accumulated onto the shift
// 1.5 * 2^52 by FMAs: every intermediate lies in [2^52, 2^53), where the FP64
// spacing is 1, so each FMA rounds to an integer and the low mantissa bits
// hold the contribution's integer value (its two or three terms are rounded
// once each: error <= 1.5 u).  The partial sums of the <= max_inc (< 2^12)
// contributions an entry receives stay below 2^62 u; rounding costs at most
// 1.5 max_inc u per entry, about 2^-49 max_inc of the row's largest
// contribution.

// max(V_1 G_1, V_2 G_2) of every face, into the spare word of its record.
__global__ void __launch_bounds__(256)
    k_face_bound(const double* __restrict__ xyz, int64_t nf, int32_t* __restrict__ face) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int32_t* row = face + f * kFaceStride;
  const int4 r0 = *reinterpret_cast<const int4*>(row);
  const int e = row[4];
  const Vec3 A = load3(xyz, r0.x), B = load3(xyz, r0.y), C = load3(xyz, r0.z);
  double vg = 0.0;
  for (int t = 0; t < 2; ++t) {
    const int o = t == 0 ? r0.w : e;
    if (o < 0) break;
    Vec3 g[4];
    double vol;
    tet_grads(A, B, C, load3(xyz, o), g, vol);
    double gg = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) gg = fmax(gg, dot(g[a], g[a]));
    vg = fmax(vg, vol * gg);
  }
  float v32 = float(vg);
  if (double(v32) < vg) v32 = nextafterf(v32, INFINITY);
  row[7] = __float_as_int(v32);
}

// The essential-BC rule for the value v at (row, col) of a row that touches
// a prescribed DOF: penalty adds alpha on a fixed diagonal; elimination
// zeroes the off-diagonal entries of fixed rows and columns.
__device__ __forceinline__ double bc_value(double v, int row, int col,
                                           const uint8_t* __restrict__ fixed, double penalty) {
  const bool fr = fixed[row], fc = fixed[col];
  if (penalty > 0.0) {
    if (fr && row == col) v += penalty;
  } else if ((fr || fc) && row != col) {
    v = 0.0;
  }
  return v;
}

// One workgroup per tile of node rows.  Work item = incidence entry e of a
// row I in the tile, i.e. a (row, face) pair: the face's smoothed gradients
// are evaluated in registers and the row's 4 or 5 blocks K_{I,J} are added
// into the LDS copy of the rows with the column slots from the slot map.
// The finished rows are written in the CSR order of the scalar matrix and,
// with valp, also in the solver's packed layout (node row I as a [9][d4]
// array at 9 ptr4[I], component-major, zero padding past deg).
// F32: FP32 face arithmetic after the FP64 tet geometry (face_geometry32);
// each FP32 contribution is rounded to the row's unit once and summed
// exactly as in the FP64 kernel; only the FP32 outputs are written.
template <bool HET, bool F32>
__global__ void __launch_bounds__(kAsmThreads) __attribute__((amdgpu_waves_per_eu(6)))
    k_assemble(const double* __restrict__ xyz, const int32_t* __restrict__ face,
               const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
               const uint32_t* __restrict__ slot, const uint16_t* __restrict__ irow,
               const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
               const int32_t* __restrict__ tile_first, const float* __restrict__ row_vg,
               double lam0, double mu0,
               const double* __restrict__ lam_t, const double* __restrict__ mu_t,
               const uint8_t* __restrict__ fixed, const uint8_t* __restrict__ bc_row,
               double penalty, double* __restrict__ val, float* __restrict__ val32,
               const int32_t* __restrict__ ptr4, double* __restrict__ valp,
               float* __restrict__ valp32) {
  __shared__ unsigned long long sval[kTileBlocks * 9];  // fixed point, units of u
  __shared__ int32_t sptr[kTileBlocks + 1];  // block offsets of the tile's rows
  __shared__ int32_t sinc[kTileBlocks + 1];  // incidence offsets of the tile's rows
  __shared__ int16_t sexp[kTileBlocks];     // per row: its unit is 2^(sexp - 50)

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  const int nwaves = kAsmThreads / kWave;
  const int n0 = tile_first[blockIdx.x], n1 = tile_first[blockIdx.x + 1];
  const int nn = n1 - n0;
  const int b0 = bptr[n0];
  const int nblk = bptr[n1] - b0;
  const int e0 = inc_ptr[n0], e1 = inc_ptr[n1];

  for (int i = tid; i < 9 * nblk; i += kAsmThreads) sval[i] = 0ull;
  for (int i = tid; i <= nn; i += kAsmThreads) {
    sptr[i] = bptr[n0 + i] - b0;
    sinc[i] = inc_ptr[n0 + i] - e0;
  }
  const int n_items = e1 - e0;
  __syncthreads();
  // each row's unit, from the largest contribution bound of its items (one
  // material: the row's precomputed largest face bound)
  if (!HET) {
    for (int li = tid; li < nn; li += kAsmThreads) {
      const double bmax = (fabs(lam0) + 2.0 * mu0) * double(row_vg[n0 + li]);
      sexp[li] = row_exponent(bmax);
    }
  }
  for (int li = wid; HET && li < nn; li += nwaves) {
    double bmax = 0.0;
    for (int k = sinc[li] + lane; k < sinc[li + 1]; k += kWave) {
      const int4 r1 =
          *reinterpret_cast<const int4*>(face + int64_t(inc[e0 + k]) * kFaceStride + 4);
      double F = fabs(lam0) + 2.0 * mu0;
      if (HET) {
        F = fabs(lam_t[r1.y]) + 2.0 * mu_t[r1.y];
        if (r1.z >= 0) F = fmax(F, fabs(lam_t[r1.z]) + 2.0 * mu_t[r1.z]);
      }
      bmax = fmax(bmax, F * double(__int_as_float(r1.w)));
    }
    bmax = wave_max(bmax);
    if (lane == 0) sexp[li] = row_exponent(bmax);
  }
  __syncthreads();

  int stride = 1;
  if (n_items > 1)
    for (const int cand : {61, 59, 53, 47, 43, 41, 37, 31})
      if (n_items % cand != 0) {
        stride = cand;
        break;
      }
  // item k is (k * stride) mod n_items, advanced incrementally
  const int step = n_items > 0 ? int((int64_t(kAsmThreads) * stride) % n_items) : 0;
  int pos = n_items > 0 ? int((int64_t(tid) * stride) % n_items) : 0;
  for (int k = tid; k < n_items; k += kAsmThreads) {
    const int e = e0 + pos;
    pos += step;
    if (pos >= n_items) pos -= n_items;
    const int li = irow[e];
    const int I = n0 + li;
    const int rb = sptr[li];
    const int deg = sptr[li + 1] - rb;
    const uint32_t code = slot[e];
    int sup[5];
    // 2^(50 - sexp) built from its exponent bits (sexp is clamped to keep it normal)
    const double inv_u = __longlong_as_double((long long)(1023 + 50 - sexp[li]) << 52);
    if constexpr (F32) {
      F3 b[5];
      float Vk, lam, mu;
      const int n = face_geometry32<HET>(face + int64_t(inc[e]) * kFaceStride, xyz, lam0, mu0,
                                         lam_t, mu_t, sup, b, Vk, lam, mu);
      // in units of the row's u; the power of two is applied in FP64 (it
      // may lie outside the FP32 range), the products stay below 2^50
      const float lV = float(double(lam * Vk) * inv_u), mV = float(double(mu * Vk) * inv_u);
      F3 bp = b[0];
#pragma unroll
      for (int p = 1; p < 5; ++p)
        if (sup[p] == I) bp = b[p];
      const float lbp[3] = {lV * bp.x, lV * bp.y, lV * bp.z};
      const float mbp[3] = {mV * bp.x, mV * bp.y, mV * bp.z};
      unsigned long long* rowv = sval + 9 * rb;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        if (q >= n) continue;
        const int jj = int((code >> (6 * q)) & 63u);
        const float bqa[3] = {b[q].x, b[q].y, b[q].z};
        const float dS = mV * (bp.x * bqa[0] + bp.y * bqa[1] + bp.z * bqa[2]);
        unsigned long long* dst = rowv + 3 * jj;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float t = fmaf(lbp[a], bqa[c], fmaf(mbp[c], bqa[a], a == c ? dS : 0.0f));
            // one FP64 addition rounds the FP32 value to an integer number of units
            atomicAdd(dst + a * 3 * deg + c, unshift(double(t) + kShift));
          }
        }
      }
      continue;
    }
    Vec3 b[5];
    double Vk, lam, mu;
    const int n = face_geometry<HET>(face + int64_t(inc[e]) * kFaceStride, xyz, lam0, mu0, lam_t,
                                     mu_t, sup, b, Vk, lam, mu);
    const double lV = lam * Vk * inv_u, mV = mu * Vk * inv_u;  // in units of the row's u
    Vec3 bp = b[0];
#pragma unroll
    for (int p = 1; p < 5; ++p)
      if (sup[p] == I) bp = b[p];
    const double lbp[3] = {lV * bp.x, lV * bp.y, lV * bp.z};
    const double mbp[3] = {mV * bp.x, mV * bp.y, mV * bp.z};
    unsigned long long* rowv = sval + 9 * rb;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      if (q >= n) continue;
      const int jj = int((code >> (6 * q)) & 63u);
      const double bqa[3] = {b[q].x, b[q].y, b[q].z};
      // mu V_k (b_p . b_q) on the block's diagonal, already shifted
      const double dS = fma(mV, bp.x * bqa[0] + bp.y * bqa[1] + bp.z * bqa[2], kShift);
      unsigned long long* dst = rowv + 3 * jj;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double t = fma(lbp[a], bqa[c], fma(mbp[c], bqa[a], a == c ? dS : kShift));
          atomicAdd(dst + a * 3 * deg + c, unshift(t));
        }
      }
    }
  }

  // stream the finished rows out, applying the essential BCs (only rows
  // that touch a prescribed DOF can need them)
  __syncthreads();
  for (int li = wid; li < nn; li += nwaves) {
    const int I = n0 + li;
    const int rb = sptr[li];
    const int deg = sptr[li + 1] - rb;
    const int three_deg = 3 * deg;
    const float inv3d = 1.0f / float(three_deg);
    const int64_t gbase = 9 * (int64_t(b0) + rb);
    const double u = ldexp(1.0, sexp[li] - 50);
    const bool rbc = fixed && bc_row[I];
    for (int k = lane; (val || val32) && k < 9 * deg; k += kWave) {
      double v = double((long long)sval[9 * rb + k]) * u;
      if (rbc) {
        const int a = int((float(k) + 0.5f) * inv3d);
        const int r = k - a * three_deg;
        const int jj = r / 3;
        const int c = r - 3 * jj;
        v = bc_value(v, 3 * I + a, 3 * bcol[b0 + rb + jj] + c, fixed, penalty);
      }
      if (val) __builtin_nontemporal_store(v, val + gbase + k);
      if (val32) __builtin_nontemporal_store(float(v), val32 + gbase + k);
    }
    if (!valp && !valp32) continue;
    // the same row in the packed layout: entry (q = 3a + c, block j) at
    // q d4 + j, read back from LDS in that order so the stores coalesce
    const int r4 = ptr4[I], d4 = ptr4[I + 1] - r4;
    const float inv_d4 = 1.0f / float(d4);
    const int64_t pbase = 9 * int64_t(r4);
    for (int kp = lane; kp < 9 * d4; kp += kWave) {
      const int q = int((float(kp) + 0.5f) * inv_d4);
      const int j = kp - q * d4;
      double v = 0.0;
      if (j < deg) {
        const int a = q / 3, c = q - 3 * a;
        v = double((long long)sval[9 * rb + a * three_deg + 3 * j + c]) * u;
        if (rbc) v = bc_value(v, 3 * I + a, 3 * bcol[b0 + rb + j] + c, fixed, penalty);
      }
      if (valp) __builtin_nontemporal_store(v, valp + pbase + kp);
      if (valp32) __builtin_nontemporal_store(float(v), valp32 + pbase + kp);
    }
  }
}

// Rows that can need the BC rule: node I or a block column J of its row
// has a prescribed DOF.  One wave per row.
__global__ void k_bc_rows(int64_t N, const int32_t* __restrict__ bptr,
                          const int32_t* __restrict__ bcol, const uint8_t* __restrict__ fixed,
                          uint8_t* __restrict__ bc_row) {
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (I >= N) return;
  int any = 0;
  for (int j = bptr[I] + lane; j < bptr[I + 1]; j += kWave) {
    const int64_t J3 = 3 * int64_t(bcol[j]);
    any |= fixed[J3] | fixed[J3 + 1] | fixed[J3 + 2];
  }
  any = wave_max(any);
  if (lane == 0) bc_row[I] = uint8_t(any);
}

// In-place elimination on an assembled unconstrained matrix (used when the
// prescribed values are nonzero: K_unc ubar is needed first).
__global__ void k_bc_mask(int64_t N, const int32_t* __restrict__ bptr,
                          const int32_t* __restrict__ bcol, const uint8_t* __restrict__ fixed,
                          double penalty, double* __restrict__ val, float* __restrict__ val32) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (I >= N) return;
  const int rb = bptr[I];
  const int deg = bptr[I + 1] - rb;
  const int three_deg = 3 * deg;
  const float inv3d = 1.0f / float(three_deg);
  for (int k = lane; k < 9 * deg; k += kWave) {
    const int a = int((float(k) + 0.5f) * inv3d);
    const int r = k - a * three_deg;
    const int jj = r / 3;
    const int c = r - 3 * jj;
    const int row = 3 * int(I) + a;
    const int col = 3 * bcol[rb + jj] + c;
    const int64_t idx = 9 * int64_t(rb) + k;
    double v = val[idx];
    if (penalty > 0.0) {
      if (fixed[row] && row == col) v += penalty;
    } else if ((fixed[row] || fixed[col]) && row != col) {
      v = 0.0;
    }
    val[idx] = v;
    if (val32) val32[idx] = float(v);
  }
}

// f_bc: free rows f - (K_unc ubar) (kub may be null when ubar == 0), fixed
// rows K_ii ubar_i (elimination) or penalty * ubar_i.
__global__ void k_rhs_bc(int64_t n, const double* __restrict__ f, const double* __restrict__ kub,
                         const uint8_t* __restrict__ fixed, const double* __restrict__ ubar,
                         const double* __restrict__ diag_unc, double penalty,
                         double* __restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = f[i];
  if (fixed && fixed[i]) {
    v = penalty > 0.0 ? penalty * ubar[i] : diag_unc[i] * ubar[i];
  } else if (kub && penalty <= 0.0) {
    v -= kub[i];
  }
  out[i] = v;
}

// diag[3I+a] = K(3I+a, 3I+a) from the node's own block.
__global__ void k_invert(int64_t n, const double* __restrict__ d, double* __restrict__ inv,
                         float* __restrict__ inv32) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 1.0 / d[i];
  inv[i] = v;
  inv32[i] = float(v);
}

// Scalar CSR arrays implied by the block pattern.
__global__ void k_scalar_pattern(int64_t N, const int32_t* __restrict__ bptr,
                                 const int32_t* __restrict__ bcol, int32_t* __restrict__ row_ptr,
                                 int32_t* __restrict__ col_idx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (I >= N) return;
  const int rb = bptr[I];
  const int deg = bptr[I + 1] - rb;
  if (row_ptr && lane < 3) row_ptr[3 * I + lane] = 9 * rb + lane * 3 * deg;
  if (row_ptr && I == N - 1 && lane == 0) row_ptr[3 * N] = 9 * bptr[N];
  if (!col_idx) return;
  for (int k = lane; k < 9 * deg; k += kWave) {
    const int r = k % (3 * deg);
    col_idx[9 * int64_t(rb) + k] = 3 * bcol[rb + r / 3] + r % 3;
  }
}

__global__ void k_face_public(int64_t nf, const int32_t* __restrict__ face,
                              int32_t* __restrict__ out) {
  int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int32_t* r = face + f * kFaceStride;
  int32_t* o = out + 7 * f;
  o[0] = r[0];
  o[1] = r[1];
  o[2] = r[2];
  o[3] = r[5];
  o[4] = r[6];
  o[5] = r[3];
  o[6] = r[4];
}

// Traction load, deterministic: per node, the triangles touching it are
// visited in ascending order; each adds t * area / 3 (Eq. 11 area).
__global__ void k_tri_entries(int64_t n_tri, const int32_t* __restrict__ tri, int64_t N,
                              int32_t* __restrict__ bucket, uint32_t* __restrict__ vals,
                              int32_t* __restrict__ err) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 3 * n_tri) return;
  int v = tri[i];
  if (v < 0 || v >= N) {
    atomicOr(err, 1);
    v = 0;
  }
  bucket[i] = v;
  vals[i] = uint32_t(i / 3);
}

__global__ void k_traction_gather(int64_t N, const int32_t* __restrict__ ptr,
                                  const uint32_t* __restrict__ tris_of, const int32_t* __restrict__ tri,
                                  const double* __restrict__ xyz, double tx, double ty, double tz,
                                  double* __restrict__ f) {
  int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  double sx = 0, sy = 0, sz = 0;
  for (int k = ptr[I]; k < ptr[I + 1]; ++k) {
    const int32_t* t = tri + 3 * int64_t(tris_of[k]);
    Vec3 A = load3(xyz, t[0]), B = load3(xyz, t[1]), C = load3(xyz, t[2]);
    Vec3 n = cross(sub(B, A), sub(C, A));
    double area = 0.5 * sqrt(dot(n, n));
    sx += tx * area / 3.0;
    sy += ty * area / 3.0;
    sz += tz * area / 3.0;
  }
  f[3 * I + 0] += sx;
  f[3 * I + 1] += sy;
  f[3 * I + 2] += sz;
}

}  // namespace

const uint8_t* bc_rows(Ctx& c) {
  if (!c.bc_row_valid) {
    const Topology& tp = c.topo;
    c.bc_row.reserve(tp.N);
    k_bc_rows<<<div_up(tp.N * kWave, 256), 256, 0, c.stream>>>(tp.N, tp.bptr.get(),
                                                                tp.bcol.get(), c.fixed.get(),
                                                                c.bc_row.get());
    SFEM_HIP(hipGetLastError());
    c.bc_row_valid = true;
  }
  return c.bc_row.get();
}

void face_bounds(Ctx& c) {
  Topology& tp = c.topo;
  k_face_bound<<<div_up(tp.nf, 256), 256, 0, c.stream>>>(c.xyz.get(), tp.nf, tp.face.get());
  tp.row_vg.reserve(tp.N);
  k_row_bound<<<div_up(tp.N, 256), 256, 0, c.stream>>>(tp.N, tp.inc_ptr.get(), tp.inc.get(),
                                                      tp.face.get(), tp.row_vg.get());
  SFEM_HIP(hipGetLastError());
}

// With `packed` (face domains), the kernel also writes the packed copies
// c.valp (and c.valp32 with an FP32 copy) and marks them valid.  With
// f32_arith the FP32 copy comes from a second pass with FP32 face arithmetic
// instead of the rounded FP64 values.
//
// val_out == c.val: the CSR order is written and marked current; null: only
// the packed copy (packed must be set); another buffer: a scratch matrix
// (the unconstrained K for sfem_get_csr), nothing is marked.
void assemble_values(Ctx& c, double* val_out, float* val32_out, bool apply_mask, bool packed,
                     bool f32_arith) {
  if (val_out == c.val.get() && val_out) {
    c.csr64 = true;
    c.packed64 = c.packed32 = false;
  }
  if (c.domain == SFEM_DOMAIN_EDGE) {
    SFEM_REQUIRE(!f32_arith, SFEM_EINVAL,
                 "FP32 face arithmetic is for face-based smoothing domains");
    SFEM_REQUIRE(val_out != nullptr, SFEM_EINVAL, "the edge assembly writes the CSR order");
    assemble_edge_values(c, val_out, val32_out, apply_mask);
    return;
  }
  SFEM_REQUIRE(val_out != nullptr || packed, SFEM_EINVAL, "no output for the assembly");
  if (!val_out) {
    c.csr64 = false;
    c.packed64 = c.packed32 = false;
  }
  double* valp = nullptr;
  float* valp32 = nullptr;
  if (packed) {
    pack_pattern(c);
    valp = c.valp.reserve(9 * c.nb4);
    if (val32_out) valp32 = c.valp32.reserve(9 * c.nb4);
  }
  const Topology& tp = c.topo;
  const uint8_t* fixed = (apply_mask && c.any_fixed) ? c.fixed.get() : nullptr;
  const uint8_t* brow = fixed ? bc_rows(c) : nullptr;
  const double* lam_t = c.per_tet ? c.lam_t.get() : nullptr;
  const double* mu_t = c.per_tet ? c.mu_t.get() : nullptr;
  dim3 grid(tp.n_tiles), block(kAsmThreads);
#define L_(HET, F32, V, V32, VP, VP32)                                                             \
  k_assemble<HET, F32><<<grid, block, 0, c.stream>>>(                                             \
      c.xyz.get(), tp.face.get(), tp.inc_ptr.get(), tp.inc.get(), tp.slot.get(), tp.irow.get(),   \
      tp.bptr.get(), tp.bcol.get(), tp.tile_first.get(), tp.row_vg.get(), c.lam0, c.mu0, lam_t,  \
      mu_t, fixed, brow, c.penalty, V, V32, c.ptr4.get(), VP, VP32)
  if (!f32_arith) {
    if (c.per_tet) L_(true, false, val_out, val32_out, valp, valp32);
    else L_(false, false, val_out, val32_out, valp, valp32);
  } else {
    if (c.per_tet) {
      L_(true, false, val_out, nullptr, valp, nullptr);
      L_(true, true, nullptr, val32_out, nullptr, valp32);
    } else {
      L_(false, false, val_out, nullptr, valp, nullptr);
      L_(false, true, nullptr, val32_out, nullptr, valp32);
    }
  }
#undef L_
  SFEM_HIP(hipGetLastError());
  if (packed) {
    c.packed64 = true;
    c.packed32 = valp32 != nullptr;
  }
}

void bc_mask_values(Ctx& c) {
  const Topology& tp = c.topo;
  const int B = 256;
  k_bc_mask<<<div_up(tp.N * kWave, B), B, 0, c.stream>>>(
      tp.N, tp.bptr.get(), tp.bcol.get(), c.fixed.get(), c.penalty, c.val.get(),
      c.have_f32 ? c.val32.get() : nullptr);
  SFEM_HIP(hipGetLastError());
}

// Builds c.f_bc from c.f_user; c.val must hold the UNCONSTRAINED matrix when
// there are nonzero prescribed values (the caller orders the calls so).
void rhs_with_bc(Ctx& c) {
  const int64_t n = c.n_dof();
  const int B = 256;
  c.f_bc.reserve(n);
  if (!c.any_fixed) {
    SFEM_HIP(hipMemcpyAsync(c.f_bc.get(), c.f_user.get(), n * sizeof(double),
                            hipMemcpyDeviceToDevice, c.stream));
    return;
  }
  double* kub = nullptr;
  double* diag = c.w.reserve(n);  // unconstrained diagonal
  matrix_diagonal(c, diag);
  if (c.any_nonzero_bc && c.penalty <= 0.0) {
    kub = c.q.reserve(n);
    spmv_f64(c, c.val.get(), c.ubar.get(), kub, c.stream);
  }
  k_rhs_bc<<<div_up(n, B), B, 0, c.stream>>>(n, c.f_user.get(), kub, c.fixed.get(), c.ubar.get(),
                                            diag, c.penalty, c.f_bc.get());
  SFEM_HIP(hipGetLastError());
}

void extract_dinv(Ctx& c) {
  const int64_t n = c.n_dof();
  const int B = 256;
  c.dinv.reserve(n);
  c.dinv32.reserve(n);
  double* diag = c.w.reserve(n);
  matrix_diagonal(c, diag);
  SFEM_HIP(hipGetLastError());
  k_invert<<<div_up(n, B), B, 0, c.stream>>>(n, diag, c.dinv.get(), c.dinv32.get());
  SFEM_HIP(hipGetLastError());
}

void scalar_csr_pattern(Ctx& c, int32_t* row_ptr, int32_t* col_idx) {
  const int B = 256;
  k_scalar_pattern<<<div_up(c.N * kWave, B), B, 0, c.stream>>>(c.N, c.topo.bptr.get(),
                                                               c.topo.bcol.get(), row_ptr, col_idx);
  SFEM_HIP(hipGetLastError());
}

void face_table_public(Ctx& c, int32_t* out) {
  const int B = 256;
  k_face_public<<<div_up(c.topo.nf, B), B, 0, c.stream>>>(c.topo.nf, c.topo.face.get(), out);
  SFEM_HIP(hipGetLastError());
}

namespace {

// Post-processing: smoothed strain eps_k = B_k d_k and stress
// sigma_k = c_k eps_k of every smoothing domain (Voigt xx, yy, zz, yz, xz,
// xy; engineering shear), with the domain's b, V_k and Lame constants as in
// the stiffness.  One thread per face.
template <bool HET>
__global__ void __launch_bounds__(256)
    k_face_stress(int64_t nf, const int32_t* __restrict__ face, const double* __restrict__ xyz,
                  double lam0, double mu0, const double* __restrict__ lam_t,
                  const double* __restrict__ mu_t, const double* __restrict__ u,
                  double* __restrict__ eps, double* __restrict__ sig) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int sup[5];
  Vec3 b[5];
  double Vk, lam, mu;
  face_geometry<HET>(face + f * kFaceStride, xyz, lam0, mu0, lam_t, mu_t, sup, b, Vk, lam, mu);
  // displacement gradient G[a][c] = sum_I u_I[a] b_I[c], all five gathers
  // issued together (an exterior face's fifth gradient is zero: its slot
  // gathers a support node and adds exactly nothing)
  double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int I = 0; I < 5; ++I) {
    const double* uI = u + 3 * int64_t(sup[I] >= 0 ? sup[I] : sup[0]);
    const double ua[3] = {uI[0], uI[1], uI[2]};
    const double bc[3] = {b[I].x, b[I].y, b[I].z};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) G[a][c] += ua[a] * bc[c];
  }
  const double e[6] = {G[0][0], G[1][1], G[2][2], G[1][2] + G[2][1], G[0][2] + G[2][0],
                       G[0][1] + G[1][0]};
  const double tr = e[0] + e[1] + e[2];
  // 16-byte stores (a face's 6 values start at a multiple of 48 bytes)
  if (eps) {
    double2* o = reinterpret_cast<double2*>(eps + 6 * f);
    o[0] = make_double2(e[0], e[1]);
    o[1] = make_double2(e[2], e[3]);
    o[2] = make_double2(e[4], e[5]);
  }
  if (sig) {
    double2* o = reinterpret_cast<double2*>(sig + 6 * f);
    o[0] = make_double2(lam * tr + 2.0 * mu * e[0], lam * tr + 2.0 * mu * e[1]);
    o[1] = make_double2(lam * tr + 2.0 * mu * e[2], mu * e[3]);
    o[2] = make_double2(mu * e[4], mu * e[5]);
  }
}

}  // namespace

void face_stress(Ctx& c, const double* u, double* eps, double* sig) {
  const int64_t nf = c.topo.nf;
  if (nf == 0) return;
  const int B = 256;
  if (c.per_tet)
    k_face_stress<true><<<div_up(nf, B), B, 0, c.stream>>>(nf, c.topo.face.get(), c.xyz.get(),
                                                           0.0, 0.0, c.lam_t.get(), c.mu_t.get(),
                                                           u, eps, sig);
  else
    k_face_stress<false><<<div_up(nf, B), B, 0, c.stream>>>(nf, c.topo.face.get(), c.xyz.get(),
                                                            c.lam0, c.mu0, nullptr, nullptr, u,
                                                            eps, sig);
  SFEM_HIP(hipGetLastError());
}

void traction_load(Ctx& c, int64_t n_tri, const int32_t* tri_dev, const double t[3]) {
  if (n_tri <= 0) return;
  hipStream_t s = c.stream;
  const int B = 256;
  TmpBuf<int32_t> bucket(3 * n_tri, s), ptr(c.N + 1, s), err(1, s);
  TmpBuf<uint32_t> vals(3 * n_tri, s), sorted(3 * n_tri, s);
  SFEM_HIP(hipMemsetAsync(err.get(), 0, sizeof(int32_t), s));
  k_tri_entries<<<div_up(3 * n_tri, B), B, 0, s>>>(n_tri, tri_dev, c.N, bucket.get(), vals.get(),
                                                   err.get());
  SFEM_HIP(hipGetLastError());
  int32_t h_err = 0;
  SFEM_HIP(hipMemcpyAsync(&h_err, err.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SFEM_HIP(hipStreamSynchronize(s));
  if (!h_err) {
    bucket_sort_u32(bucket.get(), vals.get(), 3 * n_tri, int(c.N), ptr.get(), sorted.get(), s);
    k_traction_gather<<<div_up(c.N, B), B, 0, s>>>(c.N, ptr.get(), sorted.get(), tri_dev,
                                                   c.xyz.get(), t[0], t[1], t[2], c.f_user.get());
    SFEM_HIP(hipGetLastError());
  }
  SFEM_REQUIRE(!h_err, SFEM_EINVAL, "traction triangle node index out of range");
}

}  // namespace sfem
