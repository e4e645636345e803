// Sparse matrix-vector products and the preconditioned conjugate-gradient
// solve of K u = f (the paper solves with a direct method; this library
// replaces it by PCG judged by the FP64 true residual).
//
// SpMV: one wavefront per node row I.  The 3 scalar rows 3I..3I+2 are
// contiguous in the CSR values (9 deg(I) numbers), so the wave streams them
// with unit stride; the column of value k is 3*bcol[jj] + c, read from the
// node's block-column list (9 values share one entry), and the three row
// sums are reduced with wavefront shuffles.
//
// PCG: x0 = 0; each iteration is three kernels
//   p = z + beta p;   q = K p with (p.q) -> alpha;   x, r, z updates with
//   (r.z), (r.r) -> beta and a device-side convergence flag.
// Dot products are FP64 partial sums per workgroup; the last workgroup to
// finish (atomic ticket) reduces the partials in a fixed order, so results
// are bit-reproducible.  Every `check_every` iterations the residual is
// replaced by the true one, r = f - K x, whose norm the host reads.
#include "ctx.h"

namespace sfem {

namespace {

constexpr int kRowWaves = 4;               // node rows per workgroup
constexpr int kVecThreads = 256;

// The three sums of node row I (valid in every lane after the reduction).
template <typename VT, typename XT>
__device__ __forceinline__ void row_product(int I, int lane, const int32_t* __restrict__ bptr,
                                            const int32_t* __restrict__ bcol,
                                            const VT* __restrict__ val, const XT* __restrict__ x,
                                            double& y0, double& y1, double& y2) {
  const int rb = bptr[I];
  const int deg = bptr[I + 1] - rb;
  const int three_deg = 3 * deg;
  const float inv3d = 1.0f / float(three_deg);
  const VT* v = val + 9 * int64_t(rb);
  const int32_t* cols = bcol + rb;
  using AT = typename std::conditional<sizeof(VT) == 8, double, float>::type;
  AT a0 = 0, a1 = 0, a2 = 0;
  for (int k = lane; k < 9 * deg; k += kWave) {
    const int a = int((float(k) + 0.5f) * inv3d);
    const int r = k - a * three_deg;
    const int jj = r / 3;
    const int c = r - 3 * jj;
    const AT prod = AT(v[k]) * AT(x[3 * cols[jj] + c]);
    a0 += a == 0 ? prod : AT(0);
    a1 += a == 1 ? prod : AT(0);
    a2 += a == 2 ? prod : AT(0);
  }
  y0 = wave_sum(double(a0));
  y1 = wave_sum(double(a1));
  y2 = wave_sum(double(a2));
}

// Block reduction of NV doubles (each thread passes its values; thread 0
// gets the block totals).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
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

// Writes this block's partial sums; returns true (in every thread) for the
// last block to arrive, whose thread 0 then holds the grand totals in v.
template <int NV>
__device__ __forceinline__ bool last_block_reduce(double (&v)[NV], double* partials,
                                                  unsigned int* counter) {
  __shared__ double lds[16 * NV];
  __shared__ int is_last;
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[blockIdx.x * NV + i] = v[i];
    __threadfence();
    unsigned int ticket = atomicAdd(counter, 1u);
    is_last = (ticket == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int b = threadIdx.x; b < int(gridDim.x); b += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += partials[b * NV + i];
  block_sum<NV>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = acc[i];
    atomicExch(counter, 0u);
  }
  return true;
}

template <typename VT, typename XT>
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_spmv(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
           const VT* __restrict__ val, const XT* __restrict__ x, XT* __restrict__ y) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = int64_t(blockIdx.x) * kRowWaves + threadIdx.x / kWave;
  if (I >= N) return;
  double y0, y1, y2;
  row_product<VT, XT>(int(I), lane, bptr, bcol, val, x, y0, y1, y2);
  if (lane == 0) {
    y[3 * I + 0] = XT(y0);
    y[3 * I + 1] = XT(y1);
    y[3 * I + 2] = XT(y2);
  }
}

// ---------------------------------------------------------------- CG kernels
// p = z + beta p
template <typename P>
__global__ void k_cg_p(int64_t n, const P* __restrict__ z, P* __restrict__ p,
                       const CgScalars* __restrict__ sc) {
  if (sc->converged) return;
  const P beta = P(sc->beta);
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + beta * p[i];
}

// q = K p; alpha = rz / (p . q); breakdown (p.q <= 0 or not finite) sets
// converged = 2.
template <typename VT, typename P>
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_cg_spmv(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
              const VT* __restrict__ val, const P* __restrict__ p, P* __restrict__ q,
              CgScalars* __restrict__ sc, double* __restrict__ partials) {
  if (sc->converged) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = int64_t(blockIdx.x) * kRowWaves + threadIdx.x / kWave;
  double v[1] = {0.0};
  if (I < N) {
    double y0, y1, y2;
    row_product<VT, P>(int(I), lane, bptr, bcol, val, p, y0, y1, y2);
    const P q0 = P(y0), q1 = P(y1), q2 = P(y2);
    if (lane == 0) {
      q[3 * I + 0] = q0;
      q[3 * I + 1] = q1;
      q[3 * I + 2] = q2;
      v[0] = double(p[3 * I]) * double(q0) + double(p[3 * I + 1]) * double(q1) +
             double(p[3 * I + 2]) * double(q2);
    }
  }
  if (last_block_reduce<1>(v, partials, &sc->counter[0]) && threadIdx.x == 0) {
    sc->pq = v[0];
    sc->alpha = sc->rz / v[0];
    if (!(v[0] > 0.0) || !isfinite(sc->alpha)) sc->converged = 2;
  }
}

// x += alpha p; r -= alpha q; z = dinv r; (r.z), (r.r) -> beta, rz, rr
template <typename P>
__global__ void __launch_bounds__(kVecThreads)
    k_cg_update(int64_t n, P* __restrict__ x, P* __restrict__ r, P* __restrict__ z,
                const P* __restrict__ p, const P* __restrict__ q, const P* __restrict__ dinv,
                CgScalars* __restrict__ sc, double* __restrict__ partials) {
  if (sc->converged) return;
  const double alpha = sc->alpha;
  double v[2] = {0.0, 0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    P xi = x[i] + P(alpha) * p[i];
    P ri = r[i] - P(alpha) * q[i];
    P zi = dinv[i] * ri;
    x[i] = xi;
    r[i] = ri;
    z[i] = zi;
    v[0] += double(ri) * double(zi);
    v[1] += double(ri) * double(ri);
  }
  if (last_block_reduce<2>(v, partials, &sc->counter[1]) && threadIdx.x == 0) {
    sc->beta = v[0] / sc->rz;
    sc->rz = v[0];
    sc->rr = v[1];
    sc->aux[0] += 1.0;  // iteration count
    if (v[1] <= sc->aux[1]) sc->converged = 1;  // aux[1] = tolerance^2 on r.r
    if (!isfinite(v[1])) sc->converged = 2;
  }
}

// Residual replacement: r = b - K x, z = dinv r; (r.r) -> rr_true, (r.z) -> rz.
template <typename VT, typename P>
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_cg_replace(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                 const VT* __restrict__ val, const P* __restrict__ b, const P* __restrict__ x,
                 P* __restrict__ r, P* __restrict__ z, const P* __restrict__ dinv,
                 CgScalars* __restrict__ sc, double* __restrict__ partials) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = int64_t(blockIdx.x) * kRowWaves + threadIdx.x / kWave;
  double v[2] = {0.0, 0.0};
  if (I < N) {
    double y[3];
    row_product<VT, P>(int(I), lane, bptr, bcol, val, x, y[0], y[1], y[2]);
    if (lane == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int64_t i = 3 * I + a;
        const P ri = P(double(b[i]) - y[a]);
        const P zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        v[0] += double(ri) * double(ri);
        v[1] += double(ri) * double(zi);
      }
    }
  }
  if (last_block_reduce<2>(v, partials, &sc->counter[2]) && threadIdx.x == 0) {
    sc->rr_true = v[0];
    sc->rz = v[1];
    sc->rr = v[0];
  }
}

// FP64 residual of the outer problem: r = f - K u and ||r||^2 -> rr_true.
__global__ void __launch_bounds__(kRowWaves * kWave)
    k_resid64(int64_t N, const int32_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
              const double* __restrict__ val, const double* __restrict__ f,
              const double* __restrict__ u, double* __restrict__ r, CgScalars* __restrict__ sc,
              double* __restrict__ partials) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = int64_t(blockIdx.x) * kRowWaves + threadIdx.x / kWave;
  double v[2] = {0.0, 0.0};
  if (I < N) {
    double y[3];
    row_product<double, double>(int(I), lane, bptr, bcol, val, u, y[0], y[1], y[2]);
    if (lane == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int64_t i = 3 * I + a;
        const double ri = f[i] - y[a];
        if (r) r[i] = ri;
        v[0] += ri * ri;
        v[1] += f[i] * f[i];
      }
    }
  }
  if (last_block_reduce<2>(v, partials, &sc->counter[3]) && threadIdx.x == 0) {
    sc->rr_true = v[0];
    sc->ff = v[1];
  }
}

// CG start from x = 0 with right-hand side b: x = 0, r = b, z = dinv b,
// p = 0, beta = 0; (r.z) -> rz, (r.r) -> rr.  b may be FP64 while P is FP32
// (inner solve of the refinement), in which case b is scaled by 1/scale.
template <typename P>
__global__ void __launch_bounds__(kVecThreads)
    k_cg_start(int64_t n, const double* __restrict__ b, double inv_scale, P* __restrict__ bp,
               P* __restrict__ x, P* __restrict__ r, P* __restrict__ z, P* __restrict__ p,
               const P* __restrict__ dinv, CgScalars* __restrict__ sc,
               double* __restrict__ partials) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const P bi = P(b[i] * inv_scale);
    const P zi = dinv[i] * bi;
    if (bp) bp[i] = bi;
    x[i] = P(0);
    r[i] = bi;
    z[i] = zi;
    p[i] = P(0);
    v[0] += double(bi) * double(zi);
    v[1] += double(bi) * double(bi);
  }
  if (last_block_reduce<2>(v, partials, &sc->counter[4]) && threadIdx.x == 0) {
    sc->rz = v[0];
    sc->rr = v[1];
    sc->rr_true = v[1];
    sc->beta = 0.0;
    sc->converged = 0;
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

int vec_grid(int64_t n) {
  int g = div_up(n, kVecThreads);
  return g < 2048 ? g : 2048;
}

// ------------------------------------------------------------- host driver
struct CgBuffers {
  // P-typed vectors and matrix
  const void* val;
  const void* dinv;
  void *b, *x, *r, *z, *p, *q;
};

template <typename VT, typename P>
void cg_iterations(Ctx& c, const CgBuffers& B, int iters) {
  const int64_t N = c.N, n = c.n_dof();
  hipStream_t s = c.stream;
  const int rg = div_up(N, kRowWaves);
  const int vg = vec_grid(n);
  for (int k = 0; k < iters; ++k) {
    k_cg_p<P><<<div_up(n, kVecThreads), kVecThreads, 0, s>>>(n, (const P*)B.z, (P*)B.p,
                                                              c.sc.get());
    k_cg_spmv<VT, P><<<rg, kRowWaves * kWave, 0, s>>>(N, c.topo.bptr.get(), c.topo.bcol.get(),
                                                       (const VT*)B.val, (const P*)B.p, (P*)B.q,
                                                       c.sc.get(), c.partials.get());
    k_cg_update<P><<<vg, kVecThreads, 0, s>>>(n, (P*)B.x, (P*)B.r, (P*)B.z, (const P*)B.p,
                                              (const P*)B.q, (const P*)B.dinv, c.sc.get(),
                                              c.partials.get());
  }
  SFEM_HIP(hipGetLastError());
}

template <typename VT, typename P>
void cg_replace(Ctx& c, const CgBuffers& B) {
  const int64_t N = c.N;
  k_cg_replace<VT, P><<<div_up(N, kRowWaves), kRowWaves * kWave, 0, c.stream>>>(
      N, c.topo.bptr.get(), c.topo.bcol.get(), (const VT*)B.val, (const P*)B.b, (const P*)B.x,
      (P*)B.r, (P*)B.z, (const P*)B.dinv, c.sc.get(), c.partials.get());
  SFEM_HIP(hipGetLastError());
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

// One PCG solve of A x = b from x = 0, stopping when the true residual (the
// replacement residual, computed in the solve's own precision) satisfies
// ||r|| <= tol_abs, or after max_iter iterations.  b is FP64 (scaled into P).
// Returns the iterations done and whether the tolerance was met.
template <typename VT, typename P>
int pcg(Ctx& c, const CgBuffers& B, const double* b64, double inv_scale, double tol_abs,
        int max_iter, int check_every, bool& met, bool& breakdown) {
  const int64_t n = c.n_dof();
  hipStream_t s = c.stream;
  // B.b is the P-typed right-hand side the replacement uses; when it is b64
  // itself (FP64 solve) there is nothing to convert
  P* bconv = (static_cast<const void*>(B.b) == static_cast<const void*>(b64)) ? nullptr : (P*)B.b;
  k_cg_start<P><<<vec_grid(n), kVecThreads, 0, s>>>(
      n, b64, inv_scale, bconv, (P*)B.x, (P*)B.r, (P*)B.z, (P*)B.p, (const P*)B.dinv,
      c.sc.get(), c.partials.get());
  SFEM_HIP(hipGetLastError());
  const double tol2 = tol_abs * tol_abs;
  k_cg_arm<<<1, 64, 0, s>>>(c.sc.get(), tol2);
  SFEM_HIP(hipGetLastError());
  read_scalars(c);
  met = c.sc_host->rr <= tol2;
  breakdown = false;
  int done = 0;
  double best = c.sc_host->rr;
  int stale = 0;  // checks without a new best true residual
  while (!met && done < max_iter && stale < 40) {
    const int chunk = std::min(check_every, max_iter - done);
    cg_iterations<VT, P>(c, B, chunk);
    cg_replace<VT, P>(c, B);
    read_scalars(c);
    done = int(c.sc_host->aux[0]);
    met = c.sc_host->rr_true <= tol2;
    if (c.sc_host->rr_true < best) {
      best = c.sc_host->rr_true;
      stale = 0;
    } else {
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
  }
  return done;
}

}  // namespace

void spmv_f64(Ctx& c, const double* val, const double* x, double* y, hipStream_t s) {
  k_spmv<double, double><<<div_up(c.N, kRowWaves), kRowWaves * kWave, 0, s>>>(
      c.N, c.topo.bptr.get(), c.topo.bcol.get(), val, x, y);
  SFEM_HIP(hipGetLastError());
}

void spmv_f32(Ctx& c, const float* val, const float* x, float* y, hipStream_t s) {
  k_spmv<float, float><<<div_up(c.N, kRowWaves), kRowWaves * kWave, 0, s>>>(
      c.N, c.topo.bptr.get(), c.topo.bcol.get(), val, x, y);
  SFEM_HIP(hipGetLastError());
}

double true_residual(Ctx& c, const double* u) {
  const int64_t N = c.N;
  k_resid64<<<div_up(N, kRowWaves), kRowWaves * kWave, 0, c.stream>>>(
      N, c.topo.bptr.get(), c.topo.bcol.get(), c.val.get(), c.f_bc.get(), u, c.w.get(),
      c.sc.get(), c.partials.get());
  SFEM_HIP(hipGetLastError());
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
  c.q.reserve(n);
  c.w.reserve(n);
  if (f32) {
    c.x32.reserve(n);
    c.r32.reserve(n);
    c.z32.reserve(n);
    c.p32.reserve(n);
    c.q32.reserve(n);
  }
  const int64_t nparts = std::max<int64_t>(div_up(c.N, kRowWaves), vec_grid(n)) * 2 + 16;
  c.partials.reserve(nparts);
}

int solve(Ctx& c, const sfem_solve_opts& o, sfem_solve_info& info) {
  const int64_t n = c.n_dof();
  const bool f32 = o.mode == SFEM_MODE_F32_IR;
  ensure_work(c, f32);
  const int check_every = o.check_every > 0 ? o.check_every : 50;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 100000;
  SFEM_HIP(hipEventRecord(c.ev0, c.stream));

  // ||f||: the residual of u = 0
  k_zero<<<div_up(n, 256), 256, 0, c.stream>>>(n, c.x.get());
  SFEM_HIP(hipGetLastError());
  (void)true_residual(c, c.x.get());
  const double fnorm = std::sqrt(c.sc_host->ff);
  info = sfem_solve_info{};
  if (fnorm == 0.0) {
    info.converged = 1;
    info.outer_steps = 0;
    SFEM_HIP(hipEventRecord(c.ev1, c.stream));
    SFEM_HIP(hipEventSynchronize(c.ev1));
    float ms = 0;
    SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    info.ms_solve = ms;
    return SFEM_OK;
  }

  int status = SFEM_OK;
  if (!f32) {
    CgBuffers B{c.val.get(), c.dinv.get(), c.f_bc.get(), c.x.get(), c.r.get(), c.z.get(),
                c.p.get(), c.q.get()};
    bool met = false, brk = false;
    info.iters = pcg<double, double>(c, B, c.f_bc.get(), 1.0, o.rtol * fnorm, max_iter,
                                     check_every, met, brk);
    info.outer_steps = 1;
    info.true_relres = true_residual(c, c.x.get());
    info.converged = info.true_relres <= o.rtol;
  } else {
    SFEM_REQUIRE(c.have_f32, SFEM_ESTATE,
                 "SFEM_MODE_F32_IR needs sfem_assemble(..., SFEM_ASM_F32_COPY)");
    const double inner = o.inner_rtol > 0 ? o.inner_rtol : 1e-3;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 30;
    double* u = c.x.get();
    k_zero<<<div_up(n, 256), 256, 0, c.stream>>>(n, u);
    CgBuffers B{c.val32.get(), c.dinv32.get(), c.q32.get(), nullptr, c.r32.get(), c.z32.get(),
                c.p32.get(), nullptr};
    // inner vectors: x32 is the correction d, q reused as float storage
    B.x = c.x32.get();
    float* qf = reinterpret_cast<float*>(c.q.get());
    B.q = qf;
    double relres = 1.0;
    int iters = 0, outer = 0;
    double* r64 = c.w.get();
    while (outer < max_outer && iters < max_iter) {
      // FP64 outer residual into r64
      k_resid64<<<div_up(c.N, kRowWaves), kRowWaves * kWave, 0, c.stream>>>(
          c.N, c.topo.bptr.get(), c.topo.bcol.get(), c.val.get(), c.f_bc.get(), u, r64,
          c.sc.get(), c.partials.get());
      SFEM_HIP(hipGetLastError());
      read_scalars(c);
      const double rnorm = std::sqrt(c.sc_host->rr_true);
      relres = rnorm / fnorm;
      if (relres <= o.rtol) break;
      // inner FP32 solve of K d = r64 / scale (scale keeps values O(1))
      const double scale = rnorm / std::sqrt(double(n));
      bool met = false, brk = false;
      const double tol = inner * std::sqrt(double(n));  // ||r/scale|| = sqrt(n)
      iters += pcg<float, float>(c, B, r64, 1.0 / scale, tol, max_iter - iters, check_every, met,
                                 brk);
      k_axpy_f32<<<div_up(n, 256), 256, 0, c.stream>>>(n, scale, c.x32.get(), u);
      SFEM_HIP(hipGetLastError());
      ++outer;
      if (brk) {
        status = SFEM_ENOCONV;
        break;
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
  if (!info.converged && status == SFEM_OK) status = SFEM_ENOCONV;
  return status;
}

}  // namespace sfem
