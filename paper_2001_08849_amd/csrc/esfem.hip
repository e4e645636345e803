// Edge-based smoothing domains (ES-FEM), the member of the S-FEM family the
// paper names beside its face-based one, built the same way (Sec. 2.1
// STEP 2-4 with the edge in the role of the face):
//   domain of edge k = (a, b): in every tet e around the edge, the two
//   sub-tets (a, b, centroid of a face through the edge, centroid of e),
//   a sixth of e; V_k = sum V_e / 6;
//   smoothed gradients: the boundary integral of n N_I over the domain,
//   which (N linear per tet, divergence theorem) is
//   b_I = sum_e (V_e / 6) grad N_I^e / V_k;
//   support: every node of those tets; K_k = V_k B^T c B, c from the
//   volume-weighted Lame constants.
//
// Topology (once per mesh): edges by a bucket sort of the 6 T tet edges by
// their smaller node; supports per edge; the node -> edge incidence; the
// block pattern and tiles (shared with the face domains); per incidence the
// block slots of the support nodes in the row.  Assembly: one pass per edge
// for V_k, c and b (the edge record), then the face assembly's scheme: a
// workgroup owns a tile of rows in LDS, accumulates the (row, edge) items'
// blocks as 64-bit fixed point with per-row units, and streams the rows out
// with the BCs applied.
#include "ctx.h"
#include "geom.h"

namespace sfem {

namespace {

constexpr int kB = 256;
constexpr int kAsmThreads = 256;
constexpr uint8_t kNoSlot = 0xff;

__global__ void k_fill(int64_t n, int32_t* __restrict__ a, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// 6 edge entries per tet, bucketed by the smaller node: value (larger << 32
// | tet), distinct within a bucket.
__global__ void k_edge_entries(const int32_t* __restrict__ tets, int64_t T,
                               int32_t* __restrict__ bucket, uint64_t* __restrict__ vals) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 6 * T) return;
  const int64_t t = i / 6;
  const int k = int(i % 6);
  const int a = k < 3 ? 0 : (k < 5 ? 1 : 2);
  const int b = k < 3 ? k + 1 : (k < 5 ? k - 1 : 3);
  const int va = tets[4 * t + a], vb = tets[4 * t + b];
  bucket[i] = va < vb ? va : vb;
  vals[i] = (uint64_t(uint32_t(va < vb ? vb : va)) << 32) | uint32_t(t);
}

// Edges starting at each node (distinct larger nodes among its entries).
__global__ void k_edge_count(int64_t N, const int32_t* __restrict__ ptr,
                             const uint64_t* __restrict__ v, int32_t* __restrict__ cnt) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int n = 0;
  uint32_t prev = 0xffffffffu;
  for (int i = ptr[a]; i < ptr[a + 1]; ++i) {
    const uint32_t b = uint32_t(v[i] >> 32);
    n += b != prev;
    prev = b;
  }
  cnt[a] = n;
}

// Edge table rows (a, b, first entry, tet count), ascending (a, b).
__global__ void k_edge_write(int64_t N, const int32_t* __restrict__ ptr,
                             const uint64_t* __restrict__ v, const int32_t* __restrict__ ofs,
                             int32_t* __restrict__ etab) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int e = ofs[a];
  int i = ptr[a];
  const int end = ptr[a + 1];
  while (i < end) {
    const uint32_t b = uint32_t(v[i] >> 32);
    int j = i + 1;
    while (j < end && uint32_t(v[j] >> 32) == b) ++j;
    int32_t* row = etab + 4 * int64_t(e);
    row[0] = int32_t(a);
    row[1] = int32_t(b);
    row[2] = i;
    row[3] = j - i;
    ++e;
    i = j;
  }
}

// Support of every edge: the distinct nodes of its tets, ascending, padded
// with -1.  err |= 1: too many tets around an edge; 2: support too large.
__global__ void k_edge_support(int64_t ne, const int32_t* __restrict__ etab,
                               const uint64_t* __restrict__ ent, const int32_t* __restrict__ tets,
                               int32_t* __restrict__ esup, int32_t* __restrict__ err) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int first = etab[4 * e + 2], cnt = etab[4 * e + 3];
  int32_t* out = esup + e * kEdgeSup;
  if (cnt > kEdgeTets) {
    atomicOr(err, 1);
    for (int q = 0; q < kEdgeSup; ++q) out[q] = -1;
    return;
  }
  int n = 0;
  for (int q = 0; q < kEdgeSup; ++q) out[q] = -1;
  for (int i = 0; i < cnt; ++i) {
    const int64_t t = int64_t(uint32_t(ent[first + i]));
    for (int k = 0; k < 4; ++k) {
      const int v = tets[4 * t + k];
      // insert v into the ascending list out[0..n) unless present
      int pos = 0;
      while (pos < n && out[pos] < v) ++pos;
      if (pos < n && out[pos] == v) continue;
      if (n == kEdgeSup) {
        atomicOr(err, 2);
        return;
      }
      for (int q = n; q > pos; --q) out[q] = out[q - 1];
      out[pos] = v;
      ++n;
    }
  }
}

// Support size of every edge, and the largest (atomicMax into *max_sup).
__global__ void k_edge_nsup(int64_t ne, const int32_t* __restrict__ esup,
                            int32_t* __restrict__ nsup, int32_t* __restrict__ max_sup) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int n = 0;
  for (int q = 0; q < kEdgeSup; ++q) n += esup[e * kEdgeSup + q] >= 0;
  nsup[e] = n;
  atomicMax(max_sup, n);
}

// Incidence entries: one per support node, at ofs[e] + q (no padding
// entries, so no bucket collects the -1 slots).
__global__ void k_edge_inc_entries(int64_t ne, const int32_t* __restrict__ esup,
                                   const int32_t* __restrict__ ofs, int32_t* __restrict__ bucket,
                                   uint32_t* __restrict__ vals) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int o = ofs[e], n = ofs[e + 1] - o;
  for (int q = 0; q < n; ++q) {
    bucket[o + q] = esup[e * kEdgeSup + q];
    vals[o + q] = uint32_t(e);
  }
}

// Per incidence (row I, edge k): the block slot in row I of each support
// node of k (kNoSlot past the support).  One wave per node row.
__global__ void k_edge_slots(int64_t N, const int32_t* __restrict__ inc_ptr,
                             const int32_t* __restrict__ inc, const int32_t* __restrict__ esup,
                             const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                             uint8_t* __restrict__ slots) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (I >= N) return;
  const int rb = bptr[I], deg = bptr[I + 1] - rb;
  const int32_t* cols = bcol + rb;
  for (int e = inc_ptr[I] + lane; e < inc_ptr[I + 1]; e += kWave) {
    const int32_t* sup = esup + int64_t(inc[e]) * kEdgeSup;
    uint8_t* out = slots + int64_t(e) * kEdgeSup;
    for (int q = 0; q < kEdgeSup; ++q) {
      const int J = sup[q];
      if (J < 0) {
        out[q] = kNoSlot;
        continue;
      }
      int lo = 0, hi = deg - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < J) lo = mid + 1;
        else hi = mid;
      }
      out[q] = uint8_t(lo);
    }
  }
}

// Edge records: V_k, lam_k, mu_k, a spare word, and b of each support node
// (past the support the record is not written and never read); and in a
// compact array of its own the bound (|lam| + 2 mu) V_k max |b_q|^2 of one
// contribution of the edge.
template <bool HET, int SUP>
__global__ void __launch_bounds__(kB)
    k_edge_geometry(int64_t ne, const int32_t* __restrict__ etab,
                    const uint64_t* __restrict__ ent, const int32_t* __restrict__ esup,
                    const int32_t* __restrict__ tets, const double* __restrict__ xyz,
                    double lam0, double mu0, const double* __restrict__ lam_t,
                    const double* __restrict__ mu_t, double* __restrict__ rec,
                    double* __restrict__ ebound) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int first = etab[4 * e + 2], cnt = etab[4 * e + 3];
  int sup[SUP];
#pragma unroll
  for (int q = 0; q < SUP; ++q) sup[q] = esup[e * kEdgeSup + q];
  double b[SUP][3];
#pragma unroll
  for (int q = 0; q < SUP; ++q) b[q][0] = b[q][1] = b[q][2] = 0.0;
  double V = 0.0, lw = 0.0, mw = 0.0;
  for (int i = 0; i < cnt; ++i) {
    const int64_t t = int64_t(uint32_t(ent[first + i]));
    const int v0 = tets[4 * t], v1 = tets[4 * t + 1], v2 = tets[4 * t + 2], v3 = tets[4 * t + 3];
    Vec3 g[4];
    double vol;
    tet_grads(load3(xyz, v0), load3(xyz, v1), load3(xyz, v2), load3(xyz, v3), g, vol);
    const double w = vol * (1.0 / 6.0);
    V += w;
    if (HET) {
      lw += w * lam_t[t];
      mw += w * mu_t[t];
    }
    const int vv[4] = {v0, v1, v2, v3};
#pragma unroll
    for (int q = 0; q < SUP; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (sup[q] == vv[k]) {
          b[q][0] += w * g[k].x;
          b[q][1] += w * g[k].y;
          b[q][2] += w * g[k].z;
        }
  }
  const double iV = 1.0 / V;
  const double lam = HET ? lw * iV : lam0, mu = HET ? mw * iV : mu0;
  double* out = rec + e * kEdgeRec;
  double bb = 0.0;
#pragma unroll
  for (int q = 0; q < SUP; ++q) {
    const double x = b[q][0] * iV, y = b[q][1] * iV, z = b[q][2] * iV;
    if (sup[q] >= 0) {  // the support is -1 padded at its end
      out[4 + 3 * q] = x;
      out[4 + 3 * q + 1] = y;
      out[4 + 3 * q + 2] = z;
    }
    bb = fmax(bb, x * x + y * y + z * z);
  }
  out[0] = V;
  out[1] = lam;
  out[2] = mu;
  ebound[e] = (fabs(lam) + 2.0 * mu) * V * bb;
}

// Exponent e with bmax < 2^e, clamped so that 2^(50 - e) stays a normal
// double (a larger e only coarsens the unit of absurdly small rows).
__device__ __forceinline__ int16_t edge_exponent(double bmax) {
  const int ex = bmax > 0.0 ? ilogb(bmax) + 1 : 0;
  return int16_t(ex < -973 ? -973 : ex);
}

// Largest edge bound among each node row's edges (one wave per row): the
// row's unit exponent (per assembly, per-tet materials), or with the
// topology the geometric factor max V_k max |b_q|^2, rounded up to FP32 (one
// material: the bound is (|lam| + 2 mu) times it).
template <bool GEO>
__global__ void k_edge_row_bound(int64_t N, const int32_t* __restrict__ inc_ptr,
                                 const int32_t* __restrict__ inc,
                                 const double* __restrict__ ebound, int16_t* __restrict__ rexp,
                                 float* __restrict__ row_eg) {
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (I >= N) return;
  double bmax = 0.0;
  for (int k = inc_ptr[I] + lane; k < inc_ptr[I + 1]; k += kWave)
    bmax = fmax(bmax, ebound[inc[k]]);
  bmax = wave_max(bmax);
  if (lane != 0) return;
  if (GEO) {
    float v = float(bmax);
    if (double(v) < bmax) v = nextafterf(v, INFINITY);
    row_eg[I] = v;
  } else {
    rexp[I] = edge_exponent(bmax);
  }
}

// Tile assembly of the edge items (see the face assembly for the scheme and
// the fixed-point unit: here a row's unit comes from the edge records'
// bounds, every contribution of the row below 2^50 units).
__global__ void __launch_bounds__(kAsmThreads) __attribute__((amdgpu_waves_per_eu(6)))
    k_assemble_edge(const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
                    const uint8_t* __restrict__ slot, const double* __restrict__ rec,
                    const int16_t* __restrict__ rexp, const float* __restrict__ row_eg,
                    double F, const int32_t* __restrict__ bptr,
                    const int32_t* __restrict__ bcol, const int32_t* __restrict__ tile_first,
                    const uint8_t* __restrict__ fixed, const uint8_t* __restrict__ bc_row,
                    double penalty, double* __restrict__ val, float* __restrict__ val32) {
  __shared__ unsigned long long sval[kTileBlocks * 9];
  __shared__ int32_t sptr[kTileBlocks + 1];
  __shared__ int32_t sinc[kTileBlocks + 1];
  __shared__ int16_t sexp[kTileBlocks];
  __shared__ uint8_t sdpos[kTileBlocks];  // per row: slot of its own (diagonal) block

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
    if (i < nn) {
      // per-tet materials: the exponents of this assembly; one material:
      // F = |lam| + 2 mu times the row's geometric factor
      sexp[i] = row_eg ? edge_exponent(F * double(row_eg[n0 + i])) : rexp[n0 + i];
      // the row's own column among its ascending block columns
      const int I = n0 + i, rb = bptr[I];
      int lo = 0, hi = bptr[I + 1] - rb - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (bcol[rb + mid] < I) lo = mid + 1;
        else hi = mid;
      }
      sdpos[i] = uint8_t(lo);
    }
  }
  const int n_items = e1 - e0;
  __syncthreads();

  int stride = 1;
  if (n_items > 1)
    for (const int cand : {61, 59, 53, 47, 43, 41, 37, 31})
      if (n_items % cand != 0) {
        stride = cand;
        break;
      }
  const int step = n_items > 0 ? int((int64_t(kAsmThreads) * stride) % n_items) : 0;
  int pos = n_items > 0 ? int((int64_t(tid) * stride) % n_items) : 0;
  for (int k = tid; k < n_items; k += kAsmThreads) {
    const int e = e0 + pos;
    pos += step;
    if (pos >= n_items) pos -= n_items;
    const int li = upper_index(sinc, nn, e - e0);
    const int rb = sptr[li];
    const int deg = sptr[li + 1] - rb;
    const int64_t edge = inc[e];
    const double* r = rec + edge * kEdgeRec;
    // the item's 16 slot bytes: the support's size ns (slots past it are
    // kNoSlot) and the position p of row I in it (the slot of I's own block)
    const uint4 sl4 = *reinterpret_cast<const uint4*>(slot + int64_t(e) * kEdgeSup);
    const uint32_t sw[4] = {sl4.x, sl4.y, sl4.z, sl4.w};
    const uint32_t dp = sdpos[li];
    int p = 0, ns = 0;
#pragma unroll
    for (int q = 0; q < kEdgeSup; ++q) {
      const uint32_t jj = (sw[q >> 2] >> (8 * (q & 3))) & 0xffu;
      ns += jj != kNoSlot;
      if (jj == dp) p = q;
    }
    // gradients of four support nodes per step, the first four loaded
    // together with the row's own
    double bq[4][3];
    auto load_group = [&](int q0) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u < ns ? q0 + u : q0;
        bq[u][0] = r[4 + 3 * q];
        bq[u][1] = r[5 + 3 * q];
        bq[u][2] = r[6 + 3 * q];
      }
    };
    load_group(0);  // ns >= 1: the support holds I
    // 2^(50 - sexp) built from its exponent bits (sexp is clamped to keep it normal)
    const double inv_u = __longlong_as_double((long long)(1023 + 50 - sexp[li]) << 52);
    const double lV = r[1] * r[0] * inv_u, mV = r[2] * r[0] * inv_u;
    const Vec3 bp = {r[4 + 3 * p], r[5 + 3 * p], r[6 + 3 * p]};
    const double lbp[3] = {lV * bp.x, lV * bp.y, lV * bp.z};
    const double mbp[3] = {mV * bp.x, mV * bp.y, mV * bp.z};
    unsigned long long* rowv = sval + 9 * rb;
    for (int q0 = 0;;) {
      const uint32_t w4 = q0 == 0 ? sw[0] : q0 == 4 ? sw[1] : q0 == 8 ? sw[2] : sw[3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (q0 + u >= ns) break;
        const int jj = int((w4 >> (8 * u)) & 0xffu);
        const double* bqa = bq[u];
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
      q0 += 4;
      if (q0 >= ns) break;
      load_group(q0);
    }
  }

  __syncthreads();
  for (int li = wid; li < nn; li += nwaves) {
    const int I = n0 + li;
    const int rb = sptr[li];
    const int deg = sptr[li + 1] - rb;
    const int three_deg = 3 * deg;
    const float inv3d = 1.0f / float(three_deg);
    const int64_t gbase = 9 * (int64_t(b0) + rb);
    const double u = ldexp(1.0, sexp[li] - 50);
    const bool rbc = fixed && bc_row[I];  // only rows touching a prescribed DOF
    for (int k = lane; k < 9 * deg; k += kWave) {
      double v = double((long long)sval[9 * rb + k]) * u;
      if (rbc) {
        const int a = int((float(k) + 0.5f) * inv3d);
        const int rr = k - a * three_deg;
        const int jj = rr / 3;
        const int c = rr - 3 * jj;
        const int row = 3 * I + a;
        const int col = 3 * bcol[b0 + rb + jj] + c;
        const bool fr = fixed[row], fc = fixed[col];
        if (penalty > 0.0) {
          if (fr && row == col) v += penalty;
        } else if ((fr || fc) && row != col) {
          v = 0.0;
        }
      }
      __builtin_nontemporal_store(v, val + gbase + k);
      if (val32) __builtin_nontemporal_store(float(v), val32 + gbase + k);
    }
  }
}

template <typename T>
T read1(const T* d, hipStream_t s) {
  T h;
  SFEM_HIP(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, s));
  SFEM_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace

// Edge records and bounds (per-tet materials from c.lam_t / c.mu_t when
// het).  Every support of these meshes fits 8 slots, the kernel tracks
// only 8 (half the accumulators); otherwise all 16.
static void edge_geometry(Ctx& c, hipStream_t s, bool het, double lam0, double mu0) {
  EdgeTopo& et = c.et;
  const double* lt = het ? c.lam_t.get() : nullptr;
  const double* mt = het ? c.mu_t.get() : nullptr;
#define G_(H, S)                                                                                \
  k_edge_geometry<H, S><<<div_up(et.ne, kB), kB, 0, s>>>(et.ne, et.etab.get(), et.ent.get(),    \
                                                         et.esup.get(), c.tets.get(),          \
                                                         c.xyz.get(), lam0, mu0, lt, mt,       \
                                                         et.rec.get(), et.ebound.get())
  if (het) {
    if (et.max_sup <= 8) G_(true, 8);
    else G_(true, kEdgeSup);
  } else {
    if (et.max_sup <= 8) G_(false, 8);
    else G_(false, kEdgeSup);
  }
#undef G_
  SFEM_HIP(hipGetLastError());
}

void build_edge_topology(Ctx& c) {
  hipStream_t s = c.stream;
  EdgeTopo& et = c.et;
  Topology& tp = c.topo;
  const int64_t N = c.N, T = c.T;
  // 1. edges
  const int64_t n6 = 6 * T;
  DBuf<int32_t> bucket, eptr, cnt, ofs, err;
  DBuf<uint64_t> vals;
  bucket.reserve(n6);
  vals.reserve(n6);
  eptr.reserve(N + 1);
  et.ent.reserve(n6);
  k_edge_entries<<<div_up(n6, kB), kB, 0, s>>>(c.tets.get(), T, bucket.get(), vals.get());
  SFEM_HIP(hipGetLastError());
  bucket_sort_u64(bucket.get(), vals.get(), n6, int(N), eptr.get(), et.ent.get(), s);
  cnt.reserve(N + 1);
  ofs.reserve(N + 1);
  k_edge_count<<<div_up(N, kB), kB, 0, s>>>(N, eptr.get(), et.ent.get(), cnt.get());
  SFEM_HIP(hipGetLastError());
  exclusive_scan_i32(cnt.get(), ofs.get(), N, s);
  et.ne = read1(ofs.get() + N, s);
  et.etab.reserve(4 * et.ne);
  k_edge_write<<<div_up(N, kB), kB, 0, s>>>(N, eptr.get(), et.ent.get(), ofs.get(),
                                            et.etab.get());
  SFEM_HIP(hipGetLastError());
  // 2. supports
  err.reserve(1);
  k_fill<<<1, 64, 0, s>>>(1, err.get(), 0);
  et.esup.reserve(et.ne * kEdgeSup);
  k_edge_support<<<div_up(et.ne, kB), kB, 0, s>>>(et.ne, et.etab.get(), et.ent.get(),
                                                  c.tets.get(), et.esup.get(), err.get());
  SFEM_HIP(hipGetLastError());
  const int e_err = read1(err.get(), s);
  SFEM_REQUIRE(!(e_err & 1), SFEM_EMESH, "edge domains: more than 12 tets around an edge");
  SFEM_REQUIRE(!(e_err & 2), SFEM_EMESH, "edge domains: an edge support exceeds 16 nodes");
  // 3. node -> edge incidence
  DBuf<int32_t> nsup, sofs, ib;
  DBuf<uint32_t> iv;
  nsup.reserve(et.ne + 1);
  sofs.reserve(et.ne + 1);
  k_fill<<<1, 64, 0, s>>>(1, err.get(), 0);  // reused for the largest support
  k_edge_nsup<<<div_up(et.ne, kB), kB, 0, s>>>(et.ne, et.esup.get(), nsup.get(), err.get());
  SFEM_HIP(hipGetLastError());
  et.max_sup = read1(err.get(), s);
  exclusive_scan_i32(nsup.get(), sofs.get(), et.ne, s);
  const int64_t ni = read1(sofs.get() + et.ne, s);
  ib.reserve(ni);
  iv.reserve(ni);
  k_edge_inc_entries<<<div_up(et.ne, kB), kB, 0, s>>>(et.ne, et.esup.get(), sofs.get(), ib.get(),
                                                      iv.get());
  SFEM_HIP(hipGetLastError());
  et.inc_ptr.reserve(N + 1);
  et.inc.reserve(ni);
  bucket_sort_u32(ib.get(), iv.get(), ni, int(N), et.inc_ptr.get(),
                  reinterpret_cast<uint32_t*>(et.inc.get()), s);
  et.n_inc = ni;
  // 4. pattern, tiles, slots
  et.max_inc = build_pattern<kEdgeSup, kEdgeSup>(c, et.inc_ptr.get(), et.inc.get(),
                                                 et.esup.get());
  et.slot.reserve(et.n_inc * kEdgeSup);
  k_edge_slots<<<div_up(N * kWave, kB), kB, 0, s>>>(N, et.inc_ptr.get(), et.inc.get(),
                                                    et.esup.get(), tp.bptr.get(), tp.bcol.get(),
                                                    et.slot.get());
  SFEM_HIP(hipGetLastError());
  // geometric row factors of the one-material units: the edge geometry with
  // lam = 0, mu = 1/2 makes each edge bound V_k max |b_q|^2
  et.rec.reserve(et.ne * kEdgeRec);
  et.ebound.reserve(et.ne);
  edge_geometry(c, s, false, 0.0, 0.5);
  et.row_eg.reserve(N);
  k_edge_row_bound<true><<<div_up(N * kWave, kB), kB, 0, s>>>(
      N, et.inc_ptr.get(), et.inc.get(), et.ebound.get(), nullptr, et.row_eg.get());
  SFEM_HIP(hipGetLastError());
  SFEM_HIP(hipStreamSynchronize(s));
}

void assemble_edge_values(Ctx& c, double* val_out, float* val32_out, bool apply_mask) {
  const Topology& tp = c.topo;
  EdgeTopo& et = c.et;
  const uint8_t* fixed = (apply_mask && c.any_fixed) ? c.fixed.get() : nullptr;
  et.rec.reserve(et.ne * kEdgeRec);
  et.ebound.reserve(et.ne);
  edge_geometry(c, c.stream, c.per_tet, c.lam0, c.mu0);
  if (c.per_tet) {
    et.rexp.reserve(c.N);
    k_edge_row_bound<false><<<div_up(c.N * kWave, kB), kB, 0, c.stream>>>(
        c.N, et.inc_ptr.get(), et.inc.get(), et.ebound.get(), et.rexp.get(), nullptr);
    SFEM_HIP(hipGetLastError());
  }
  k_assemble_edge<<<tp.n_tiles, kAsmThreads, 0, c.stream>>>(
      et.inc_ptr.get(), et.inc.get(), et.slot.get(), et.rec.get(),
      c.per_tet ? et.rexp.get() : nullptr, c.per_tet ? nullptr : et.row_eg.get(),
      std::fabs(c.lam0) + 2.0 * c.mu0, tp.bptr.get(), tp.bcol.get(), tp.tile_first.get(), fixed,
      fixed ? bc_rows(c) : nullptr, c.penalty, val_out, val32_out);
  SFEM_HIP(hipGetLastError());
}

}  // namespace sfem
