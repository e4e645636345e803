// extern "C" entry points of include/sfem.h.  Every call catches the
// library's internal errors and turns them into an sfem_status plus a
// message kept on the context.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "handles.h"

using sfem::Ctx;
using sfem::Error;

namespace {

template <typename F>
int guarded(sfem_ctx* h, F&& fn) {
  if (!h) return SFEM_EINVAL;
  h->c.err.clear();
  try {
    SFEM_HIP(hipSetDevice(h->c.device));
    return fn(h->c);
  } catch (const Error& e) {
    h->c.err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    h->c.err = e.what();
    return SFEM_EINVAL;
  }
}

template <typename F>
int gnn_guarded(sfem_gnn* h, F&& fn) {
  if (!h) return SFEM_EINVAL;
  h->g.err.clear();
  try {
    SFEM_HIP(hipSetDevice(h->g.device));
    return fn(h->g);
  } catch (const Error& e) {
    h->g.err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    h->g.err = e.what();
    return SFEM_EINVAL;
  }
}

// Copy n elements from a caller buffer into a device buffer.
template <typename T>
void upload(Ctx& c, T* dst, const T* src, int64_t n, int ptr_kind) {
  SFEM_REQUIRE(src != nullptr || n == 0, SFEM_EINVAL, "null input pointer");
  SFEM_REQUIRE(ptr_kind == SFEM_PTR_HOST || ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL,
               "ptr_kind must be SFEM_PTR_HOST or SFEM_PTR_DEVICE");
  if (n == 0) return;
  SFEM_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n,
                          ptr_kind == SFEM_PTR_HOST ? hipMemcpyHostToDevice
                                                    : hipMemcpyDeviceToDevice,
                          c.stream));
  if (ptr_kind == SFEM_PTR_HOST) SFEM_HIP(hipStreamSynchronize(c.stream));
}

template <typename T>
void download(Ctx& c, T* dst, const T* src, int64_t n, int ptr_kind) {
  SFEM_REQUIRE(ptr_kind == SFEM_PTR_HOST || ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL,
               "ptr_kind must be SFEM_PTR_HOST or SFEM_PTR_DEVICE");
  if (!dst || n == 0) return;
  SFEM_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n,
                          ptr_kind == SFEM_PTR_HOST ? hipMemcpyDeviceToHost
                                                    : hipMemcpyDeviceToDevice,
                          c.stream));
  if (ptr_kind == SFEM_PTR_HOST) SFEM_HIP(hipStreamSynchronize(c.stream));
}

__global__ void k_check_index(const int32_t* idx, int64_t n, int64_t lim, int32_t* err) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && (idx[i] < 0 || idx[i] >= lim)) atomicOr(err, 1);
}

bool indices_ok(Ctx& c, const int32_t* dev_idx, int64_t n, int64_t lim) {
  if (n == 0) return true;
  sfem::TmpBuf<int32_t> err(1, c.stream);
  SFEM_HIP(hipMemsetAsync(err.get(), 0, sizeof(int32_t), c.stream));
  k_check_index<<<sfem::div_up(n, 256), 256, 0, c.stream>>>(dev_idx, n, lim, err.get());
  SFEM_HIP(hipGetLastError());
  int32_t h = 0;
  SFEM_HIP(hipMemcpyAsync(&h, err.get(), sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  SFEM_HIP(hipStreamSynchronize(c.stream));
  return h == 0;
}

__global__ void k_lame(int64_t T, const double* E, const double* nu, double* lam, double* mu,
                       int32_t* err) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double e = E[t], v = nu[t];
  if (!(e > 0.0) || !(v > -1.0 && v < 0.5)) atomicOr(err, 1);
  lam[t] = e * v / ((1.0 + v) * (1.0 - 2.0 * v));
  mu[t] = e / (2.0 * (1.0 + v));
}

__global__ void k_set_fixed(int64_t n, const int32_t* dof, const double* value, uint8_t* fixed,
                            double* ubar, int32_t* flags) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = dof[i];
  const double v = value ? value[i] : 0.0;
  fixed[d] = 1;
  ubar[d] = v;
  if (v != 0.0) atomicOr(flags, 1);
}

void reset_problem(Ctx& c) {
  c.have_learned = false;
  c.nb4 = 0;
  c.lds_tables = 0;
  c.mapply_kernel = 0;
  c.mapply_tuned = c.mgrp_ok = false;
  c.mapply_us[0] = c.mapply_us[1] = c.mapply_us[2] = 0.0;
  c.gnn.reset();
  c.have_material = false;
  c.per_tet = false;
  c.any_fixed = c.any_nonzero_bc = false;
  c.bc_row_valid = false;
  c.penalty = 0.0;
  c.assembled = false;
  c.val_has_bc = false;
  c.have_f32 = false;
  const int64_t n = c.n_dof();
  c.fixed.reserve(n);
  c.ubar.reserve(n);
  c.f_user.reserve(n);
  SFEM_HIP(hipMemsetAsync(c.fixed.get(), 0, n, c.stream));
  SFEM_HIP(hipMemsetAsync(c.ubar.get(), 0, n * sizeof(double), c.stream));
  SFEM_HIP(hipMemsetAsync(c.f_user.get(), 0, n * sizeof(double), c.stream));
}

}  // namespace

extern "C" {

int sfem_create(sfem_ctx** out, int device, void* hip_stream) {
  if (!out) return SFEM_EINVAL;
  *out = nullptr;
  sfem_ctx* h = new (std::nothrow) sfem_ctx;
  if (!h) return SFEM_ENOMEM;
  h->c.device = device;
  int st = guarded(h, [&](Ctx& c) {
    int count = 0;
    SFEM_HIP(hipGetDeviceCount(&count));
    SFEM_REQUIRE(device >= 0 && device < count, SFEM_EINVAL, "bad device ordinal");
    if (hip_stream) {
      c.stream = static_cast<hipStream_t>(hip_stream);
    } else {
      SFEM_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
      c.own_stream = true;
    }
    SFEM_HIP(hipEventCreate(&c.ev0));
    SFEM_HIP(hipEventCreate(&c.ev1));
    SFEM_HIP(hipEventCreate(&c.tev0));
    SFEM_HIP(hipEventCreate(&c.tev1));
    SFEM_HIP(hipHostMalloc((void**)&c.sc_host, sizeof(sfem::CgScalars), hipHostMallocDefault));
    // this device's scratch address for the allocation-free entry point
    sfem::scratch_init(device);
    c.sc.reserve(1);
    SFEM_HIP(hipMemsetAsync(c.sc.get(), 0, sizeof(sfem::CgScalars), c.stream));
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
  if (st != SFEM_OK) {
    sfem_destroy(h);
    return st;
  }
  *out = h;
  return SFEM_OK;
}

void sfem_destroy(sfem_ctx* h) {
  if (!h) return;
  Ctx& c = h->c;
  (void)hipSetDevice(c.device);
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (c.ev0) (void)hipEventDestroy(c.ev0);
  if (c.ev1) (void)hipEventDestroy(c.ev1);
  if (c.tev0) (void)hipEventDestroy(c.tev0);
  if (c.tev1) (void)hipEventDestroy(c.tev1);
  for (hipEvent_t e : c.prof_ev) (void)hipEventDestroy(e);
  c.drop_cg_graph();
  if (c.sc_host) (void)hipHostFree(c.sc_host);
  if (c.own_stream && c.stream) (void)hipStreamDestroy(c.stream);
  delete h;
}

const char* sfem_last_error(const sfem_ctx* h) { return h ? h->c.err.c_str() : "null context"; }

int sfem_set_stream(sfem_ctx* h, void* hip_stream) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(hip_stream != nullptr, SFEM_EINVAL, "null stream");
    SFEM_HIP(hipStreamSynchronize(c.stream));
    if (c.own_stream) SFEM_HIP(hipStreamDestroy(c.stream));
    c.own_stream = false;
    c.stream = static_cast<hipStream_t>(hip_stream);
    return SFEM_OK;
  });
}

int sfem_set_graph_replay(sfem_ctx* h, int enabled) {
  return guarded(h, [&](Ctx& c) {
    c.graph_replay = enabled != 0;
    if (!c.graph_replay) {
      SFEM_HIP(hipStreamSynchronize(c.stream));
      c.drop_cg_graph();
    }
    return SFEM_OK;
  });
}

int sfem_set_mesh(sfem_ctx* h, int64_t n_nodes, const double* xyz, int64_t n_tets,
                  const int32_t* tets, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(n_nodes > 0 && n_tets > 0 && xyz && tets, SFEM_EINVAL, "empty or null mesh");
    SFEM_REQUIRE(n_nodes < (int64_t(1) << 29), SFEM_EINVAL, "n_nodes must be < 2^29");
    c.topo.valid = false;
    c.N = n_nodes;
    c.T = n_tets;
    c.xyz.reserve(3 * n_nodes);
    c.tets.reserve(4 * n_tets);
    upload(c, c.xyz.get(), xyz, 3 * n_nodes, ptr_kind);
    upload(c, c.tets.get(), tets, 4 * n_tets, ptr_kind);
    if (!indices_ok(c, c.tets.get(), 4 * n_tets, n_nodes)) {
      c.N = c.T = 0;
      throw Error{SFEM_EINVAL, "tet node index out of range"};
    }
    reset_problem(c);
    SFEM_HIP(hipEventRecord(c.ev0, c.stream));
    try {
      sfem::build_topology(c);
    } catch (...) {
      c.N = c.T = 0;
      throw;
    }
    SFEM_HIP(hipEventRecord(c.ev1, c.stream));
    SFEM_HIP(hipEventSynchronize(c.ev1));
    float ms = 0;
    SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    c.ms_topology = ms;
    return SFEM_OK;
  });
}

int sfem_set_smoothing_domain(sfem_ctx* h, int domain) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(domain == SFEM_DOMAIN_FACE || domain == SFEM_DOMAIN_EDGE, SFEM_EINVAL,
                 "domain must be SFEM_DOMAIN_FACE or SFEM_DOMAIN_EDGE");
    if (domain == c.domain) return SFEM_OK;
    c.domain = domain;
    if (c.N > 0 && c.T > 0) {
      c.topo.valid = false;
      reset_problem(c);
      try {
        sfem::build_topology(c);
      } catch (...) {
        c.N = c.T = 0;
        throw;
      }
    }
    return SFEM_OK;
  });
}

int sfem_set_material(sfem_ctx* h, double E, double nu) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(E > 0.0 && nu > -1.0 && nu < 0.5, SFEM_EINVAL, "need E > 0 and -1 < nu < 0.5");
    c.lam0 = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    c.mu0 = E / (2.0 * (1.0 + nu));
    c.per_tet = false;
    c.have_material = true;
    c.assembled = false;
    return SFEM_OK;
  });
}

int sfem_set_material_per_tet(sfem_ctx* h, const double* E, const double* nu, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    sfem::TmpBuf<double> dE(c.T, c.stream), dn(c.T, c.stream);
    sfem::TmpBuf<int32_t> err(1, c.stream);
    SFEM_HIP(hipMemsetAsync(err.get(), 0, sizeof(int32_t), c.stream));
    c.lam_t.reserve(c.T);
    c.mu_t.reserve(c.T);
    upload(c, dE.get(), E, c.T, ptr_kind);
    upload(c, dn.get(), nu, c.T, ptr_kind);
    k_lame<<<sfem::div_up(c.T, 256), 256, 0, c.stream>>>(c.T, dE.get(), dn.get(), c.lam_t.get(),
                                                          c.mu_t.get(), err.get());
    SFEM_HIP(hipGetLastError());
    int32_t he = 0;
    SFEM_HIP(hipMemcpyAsync(&he, err.get(), sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    SFEM_HIP(hipStreamSynchronize(c.stream));
    SFEM_REQUIRE(he == 0, SFEM_EINVAL, "need E > 0 and -1 < nu < 0.5 for every tet");
    c.per_tet = true;
    c.have_material = true;
    c.assembled = false;
    return SFEM_OK;
  });
}

int sfem_set_dirichlet(sfem_ctx* h, int64_t n, const int32_t* dof, const double* value,
                       int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(n >= 0, SFEM_EINVAL, "negative count");
    sfem::TmpBuf<int32_t> ddof(n, c.stream), flags(4, c.stream);
    sfem::TmpBuf<double> dval(n, c.stream);
    SFEM_HIP(hipMemsetAsync(flags.get(), 0, sizeof(int32_t) * 4, c.stream));
    upload(c, ddof.get(), dof, n, ptr_kind);
    if (value) upload(c, dval.get(), value, n, ptr_kind);
    const bool ok = indices_ok(c, ddof.get(), n, c.n_dof());
    if (ok) {
      SFEM_HIP(hipMemsetAsync(c.fixed.get(), 0, c.n_dof(), c.stream));
      SFEM_HIP(hipMemsetAsync(c.ubar.get(), 0, c.n_dof() * sizeof(double), c.stream));
      if (n)
        k_set_fixed<<<sfem::div_up(n, 256), 256, 0, c.stream>>>(
            n, ddof.get(), value ? dval.get() : nullptr, c.fixed.get(), c.ubar.get(), flags.get());
      SFEM_HIP(hipGetLastError());
    }
    int32_t hf[4] = {0, 0, 0, 0};
    SFEM_HIP(hipMemcpyAsync(hf, flags.get(), sizeof(hf), hipMemcpyDeviceToHost, c.stream));
    SFEM_HIP(hipStreamSynchronize(c.stream));
    SFEM_REQUIRE(ok, SFEM_EINVAL, "Dirichlet DOF index out of range");
    c.any_fixed = n > 0;
    c.bc_row_valid = false;
    if (c.any_fixed) sfem::bc_rows(c);  // with the BCs, not in the assembly
    c.any_nonzero_bc = hf[0] != 0;
    c.assembled = false;
    return SFEM_OK;
  });
}

int sfem_set_bc_penalty(sfem_ctx* h, double alpha) {
  return guarded(h, [&](Ctx& c) {
    c.penalty = alpha > 0.0 ? alpha : 0.0;
    c.assembled = false;
    return SFEM_OK;
  });
}

int sfem_set_nodal_load(sfem_ctx* h, const double* f, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    upload(c, c.f_user.get(), f, c.n_dof(), ptr_kind);
    c.assembled = false;
    return SFEM_OK;
  });
}

int sfem_add_traction(sfem_ctx* h, int64_t n_tri, const int32_t* tri, const double t[3],
                      int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(n_tri >= 0 && t && (tri || n_tri == 0), SFEM_EINVAL, "bad traction arguments");
    if (n_tri == 0) return SFEM_OK;
    sfem::TmpBuf<int32_t> dtri(3 * n_tri, c.stream);
    upload(c, dtri.get(), tri, 3 * n_tri, ptr_kind);
    sfem::traction_load(c, n_tri, dtri.get(), t);
    c.assembled = false;
    return SFEM_OK;
  });
}

int sfem_assemble(sfem_ctx* h, int flags) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(c.have_material, SFEM_ESTATE, "set a material first");
    // a new matrix invalidates the learned preconditioner, its features and
    // the training pairs (r = K e) of the old one
    c.have_learned = false;
    c.gnn.reset();
    c.packed64 = c.packed32 = false;
    c.have_rsum = c.have_rcorr = false;
    const int64_t nnz = 9 * c.topo.nb;
    c.val.reserve(nnz);
    SFEM_REQUIRE((flags & ~(SFEM_ASM_F32_COPY | SFEM_ASM_F32_ARITH)) == 0, SFEM_EINVAL,
                 "unknown assembly flag");
    const bool f32_arith = (flags & SFEM_ASM_F32_ARITH) != 0;
    const bool f32 = (flags & SFEM_ASM_F32_COPY) != 0 || f32_arith;
    if (f32) c.val32.reserve(nnz);
    c.have_f32 = f32;
    c.w.reserve(c.n_dof());
    c.q.reserve(c.n_dof());
    const bool two_step = c.any_fixed && c.any_nonzero_bc && c.penalty <= 0.0;
    // the packed tables (once per mesh; a host read) before the timed region
    if (!two_step && c.domain == SFEM_DOMAIN_FACE) sfem::pack_pattern(c);
    SFEM_HIP(hipEventRecord(c.ev0, c.stream));
    // the solver's packed copy is written by the same pass, except when the
    // BCs are applied afterwards (it is then packed from the masked values)
    // face domains without two-step BCs: only the packed copy the solver
    // reads is written (the CSR order is made on demand)
    const bool packed_only = !two_step && c.domain == SFEM_DOMAIN_FACE;
    sfem::assemble_values(c, packed_only ? nullptr : c.val.get(), f32 ? c.val32.get() : nullptr,
                          !two_step, !two_step, f32_arith);
    SFEM_HIP(hipEventRecord(c.ev1, c.stream));
    sfem::rhs_with_bc(c);
    if (two_step) {
      sfem::bc_mask_values(c);
      // a packed copy made from the unconstrained values (rhs_with_bc's
      // product under a packed schedule) is stale now
      c.packed64 = c.packed32 = false;
    }
    sfem::extract_dinv(c);
    SFEM_HIP(hipEventSynchronize(c.ev1));
    float ms = 0;
    SFEM_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    c.ms_assemble = ms;
    SFEM_HIP(hipStreamSynchronize(c.stream));
    c.assembled = true;
    c.val_has_bc = c.any_fixed;
    return SFEM_OK;
  });
}

int sfem_get_sizes(sfem_ctx* h, int64_t* n_faces, int64_t* n_exterior, int64_t* n_rows,
                   int64_t* nnz, int64_t* n_blocks) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    if (n_faces) *n_faces = c.topo.nf;
    if (n_exterior) *n_exterior = c.topo.ne;
    if (n_rows) *n_rows = c.n_dof();
    if (nnz) *nnz = 9 * c.topo.nb;
    if (n_blocks) *n_blocks = c.topo.nb;
    return SFEM_OK;
  });
}

int sfem_get_faces(sfem_ctx* h, int32_t* table, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(table != nullptr, SFEM_EINVAL, "null output");
    sfem::DBuf<int32_t> tmp;
    tmp.reserve(7 * c.topo.nf);
    sfem::face_table_public(c, tmp.get());
    download(c, table, tmp.get(), 7 * c.topo.nf, ptr_kind);
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

namespace {
__global__ void k_widen(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = double(a[i]);
}
}  // namespace

int sfem_get_csr(sfem_ctx* h, int32_t* row_ptr, int32_t* col_idx, double* val, int which,
                 int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(which == SFEM_K_UNCONSTRAINED || which == SFEM_K_WITH_BC ||
                     which == SFEM_K_F32,
                 SFEM_EINVAL, "bad `which`");
    const int64_t nnz = 9 * c.topo.nb, n = c.n_dof();
    if (row_ptr || col_idx) {
      sfem::DBuf<int32_t> rp, ci;
      if (row_ptr) rp.reserve(n + 1);
      if (col_idx) ci.reserve(nnz);
      sfem::scalar_csr_pattern(c, rp.get(), ci.get());
      download(c, row_ptr, rp.get(), n + 1, ptr_kind);
      download(c, col_idx, ci.get(), nnz, ptr_kind);
      SFEM_HIP(hipStreamSynchronize(c.stream));
    }
    if (val) {
      SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
      if (which == SFEM_K_F32) {
        SFEM_REQUIRE(c.have_f32, SFEM_ESTATE, "no FP32 copy: assemble with SFEM_ASM_F32_*");
        sfem::DBuf<double> tmp;
        tmp.reserve(nnz);
        k_widen<<<sfem::div_up(nnz, 256), 256, 0, c.stream>>>(nnz, c.val32.get(), tmp.get());
        SFEM_HIP(hipGetLastError());
        download(c, val, tmp.get(), nnz, ptr_kind);
      } else if (which == SFEM_K_WITH_BC || !c.val_has_bc) {
        sfem::ensure_csr64(c);
        download(c, val, c.val.get(), nnz, ptr_kind);
      } else {
        sfem::DBuf<double> tmp;
        tmp.reserve(nnz);
        sfem::assemble_values(c, tmp.get(), nullptr, false);
        download(c, val, tmp.get(), nnz, ptr_kind);
      }
      SFEM_HIP(hipStreamSynchronize(c.stream));
    }
    return SFEM_OK;
  });
}

int sfem_get_rhs(sfem_ctx* h, double* f, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
    download(c, f, c.f_bc.get(), c.n_dof(), ptr_kind);
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

int sfem_spmv(sfem_ctx* h, const double* x, double* y, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
    SFEM_REQUIRE(x && y, SFEM_EINVAL, "null vector");
    const int64_t n = c.n_dof();
    if (ptr_kind == SFEM_PTR_DEVICE) {
      sfem::spmv_f64(c, c.val.get(), x, y, c.stream);
      SFEM_HIP(hipStreamSynchronize(c.stream));
    } else {
      sfem::DBuf<double> dx, dy;
      dx.reserve(n);
      dy.reserve(n);
      upload(c, dx.get(), x, n, ptr_kind);
      sfem::spmv_f64(c, c.val.get(), dx.get(), dy.get(), c.stream);
      download(c, y, dy.get(), n, ptr_kind);
    }
    return SFEM_OK;
  });
}

int sfem_solve(sfem_ctx* h, const sfem_solve_opts* opts, double* u, int ptr_kind,
               sfem_solve_info* info) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
    SFEM_REQUIRE(opts && u, SFEM_EINVAL, "null opts or u");
    SFEM_REQUIRE(opts->rtol > 0.0, SFEM_EINVAL, "rtol must be > 0");
    sfem_solve_info tmp{};
    int st = sfem::solve(c, *opts, tmp);
    download(c, u, c.x.get(), c.n_dof(), ptr_kind);
    SFEM_HIP(hipStreamSynchronize(c.stream));
    if (info) *info = tmp;
    return st;
  });
}

int sfem_rcm_permutation(sfem_ctx* h, int64_t n_nodes, int64_t n_tets, const int32_t* tets,
                         int ptr_kind, int32_t* perm, int perm_ptr_kind, double* ms) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(n_nodes > 0 && n_tets > 0 && tets && perm, SFEM_EINVAL, "empty or null mesh");
    SFEM_REQUIRE(n_nodes < (int64_t(1) << 29) && n_tets < (int64_t(1) << 29), SFEM_EINVAL,
                 "mesh too large");
    SFEM_REQUIRE(perm_ptr_kind == SFEM_PTR_HOST || perm_ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL,
                 "bad ptr_kind");
    sfem::DBuf<int32_t> dt, dp;
    const int32_t* td = tets;
    if (ptr_kind == SFEM_PTR_HOST) {
      upload(c, dt.reserve(4 * n_tets), tets, 4 * n_tets, ptr_kind);
      td = dt.get();
    } else {
      SFEM_REQUIRE(ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL, "bad ptr_kind");
    }
    SFEM_REQUIRE(indices_ok(c, td, 4 * n_tets, n_nodes), SFEM_EINVAL,
                 "tet node index out of range");
    int32_t* pd = perm_ptr_kind == SFEM_PTR_DEVICE ? perm : dp.reserve(n_nodes);
    SFEM_HIP(hipEventRecord(c.tev0, c.stream));
    sfem::rcm_order(c.stream, n_nodes, n_tets, td, pd);
    SFEM_HIP(hipEventRecord(c.tev1, c.stream));
    SFEM_HIP(hipEventSynchronize(c.tev1));
    if (ms) {
      float t = 0;
      SFEM_HIP(hipEventElapsedTime(&t, c.tev0, c.tev1));
      *ms = t;
    }
    if (perm_ptr_kind == SFEM_PTR_HOST) download(c, perm, pd, n_nodes, SFEM_PTR_HOST);
    return SFEM_OK;
  });
}

int sfem_permute_mesh(sfem_ctx* h, int64_t n_nodes, int64_t n_tets, const int32_t* perm,
                      const double* xyz, const int32_t* tets, double* xyz_out, int32_t* tets_out,
                      int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(n_nodes > 0 && n_tets >= 0 && perm, SFEM_EINVAL, "empty or null input");
    SFEM_REQUIRE((xyz == nullptr) == (xyz_out == nullptr) &&
                     (tets == nullptr) == (tets_out == nullptr),
                 SFEM_EINVAL, "give both an input and an output array, or neither");
    SFEM_REQUIRE(ptr_kind == SFEM_PTR_HOST || ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL,
                 "bad ptr_kind");
    const bool host = ptr_kind == SFEM_PTR_HOST;
    sfem::DBuf<int32_t> dp, dt, dto;
    sfem::DBuf<double> dx, dxo;
    const int32_t* pd = perm;
    const double* xd = xyz;
    const int32_t* td = tets;
    double* xo = xyz_out;
    int32_t* to = tets_out;
    if (host) {
      upload(c, dp.reserve(n_nodes), perm, n_nodes, ptr_kind);
      pd = dp.get();
      if (xyz) {
        upload(c, dx.reserve(3 * n_nodes), xyz, 3 * n_nodes, ptr_kind);
        xd = dx.get();
        xo = dxo.reserve(3 * n_nodes);
      }
      if (tets && n_tets > 0) {
        upload(c, dt.reserve(4 * n_tets), tets, 4 * n_tets, ptr_kind);
        td = dt.get();
        to = dto.reserve(4 * n_tets);
      }
    }
    SFEM_REQUIRE(sfem::is_permutation(c.stream, n_nodes, pd), SFEM_EINVAL,
                 "perm is not a permutation of 0..n_nodes-1");
    if (tets && n_tets > 0)
      SFEM_REQUIRE(indices_ok(c, td, 4 * n_tets, n_nodes), SFEM_EINVAL,
                   "tet node index out of range");
    sfem::permute_mesh(c.stream, n_nodes, n_tets, pd, xd, n_tets > 0 ? td : nullptr, xo,
                       n_tets > 0 ? to : nullptr);
    if (host) {
      if (xyz) download(c, xyz_out, xo, 3 * n_nodes, ptr_kind);
      if (tets && n_tets > 0) download(c, tets_out, to, 4 * n_tets, ptr_kind);
    }
    return SFEM_OK;
  });
}

int sfem_face_stress(sfem_ctx* h, const double* u, double* strain, double* stress,
                     int ptr_kind, double* ms) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(c.have_material, SFEM_ESTATE, "set a material first");
    SFEM_REQUIRE(c.domain == SFEM_DOMAIN_FACE, SFEM_ESTATE,
                 "stress recovery is implemented for face smoothing domains");
    SFEM_REQUIRE(u, SFEM_EINVAL, "null displacement vector");
    const int64_t n = c.n_dof(), m = 6 * c.topo.nf;
    sfem::DBuf<double> du, de, ds;
    const double* ud = u;
    double *ed = strain, *sd = stress;
    if (ptr_kind == SFEM_PTR_HOST) {
      du.reserve(n);
      upload(c, du.get(), u, n, ptr_kind);
      ud = du.get();
      ed = strain ? de.reserve(m) : nullptr;
      sd = stress ? ds.reserve(m) : nullptr;
    } else {
      SFEM_REQUIRE(ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL, "bad ptr_kind");
    }
    SFEM_HIP(hipEventRecord(c.tev0, c.stream));
    sfem::face_stress(c, ud, ed, sd);
    SFEM_HIP(hipEventRecord(c.tev1, c.stream));
    SFEM_HIP(hipEventSynchronize(c.tev1));
    if (ms) {
      float t = 0;
      SFEM_HIP(hipEventElapsedTime(&t, c.tev0, c.tev1));
      *ms = t;
    }
    if (ptr_kind == SFEM_PTR_HOST) {
      download(c, strain, ed, m, ptr_kind);
      download(c, stress, sd, m, ptr_kind);
    }
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

int sfem_get_timings(sfem_ctx* h, double* ms_topology, double* ms_assemble) {
  return guarded(h, [&](Ctx& c) {
    if (ms_topology) *ms_topology = c.ms_topology;
    if (ms_assemble) *ms_assemble = c.ms_assemble;
    return SFEM_OK;
  });
}

int sfem_set_schedule(sfem_ctx* h, int precision, int variant, int grid_cap) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(variant >= 0 && variant < sfem::kNumSched && grid_cap >= 8, SFEM_EINVAL,
                 "bad schedule");
    if (variant == sfem::kNumSched - 1) {
      SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first (schedule 17 needs its tables)");
      SFEM_REQUIRE(sfem::ensure_lds_tables(c), SFEM_EINVAL,
                   "schedule 17 unavailable: a chunk's x window exceeds 1,024 nodes");
    }
    const sfem::RowSched rs{variant, grid_cap};
    if (precision == SFEM_ASM_F32_COPY) c.sched32 = rs;
    else c.sched64 = rs;
    return SFEM_OK;
  });
}

int sfem_get_schedule(sfem_ctx* h, int precision, int* variant, int* grid_cap) {
  return guarded(h, [&](Ctx& c) {
    const sfem::RowSched rs = precision == SFEM_ASM_F32_COPY ? c.sched32 : c.sched64;
    if (variant) *variant = rs.variant;
    if (grid_cap) *grid_cap = rs.grid_cap;
    return SFEM_OK;
  });
}

int sfem_autotune(sfem_ctx* h, int reps, double* best_us_f64, double* best_us_f32) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
    sfem::autotune_rows(c, reps > 0 ? reps : 10, best_us_f64, best_us_f32);
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

int sfem_timer_start(sfem_ctx* h) {
  return guarded(h, [&](Ctx& c) {
    SFEM_HIP(hipEventRecord(c.tev0, c.stream));
    return SFEM_OK;
  });
}

int sfem_timer_stop(sfem_ctx* h, double* ms) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(ms != nullptr, SFEM_EINVAL, "null output");
    SFEM_HIP(hipEventRecord(c.tev1, c.stream));
    SFEM_HIP(hipEventSynchronize(c.tev1));
    float t = 0;
    SFEM_HIP(hipEventElapsedTime(&t, c.tev0, c.tev1));
    *ms = t;
    return SFEM_OK;
  });
}

int sfem_synchronize(sfem_ctx* h) {
  return guarded(h, [&](Ctx& c) {
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

// ------------------------------------------------- learned preconditioner
int64_t sfem_gnn_num_params(void) { return sfem::param_layout().total; }

int sfem_gnn_create(sfem_gnn** out, int device, uint64_t seed) {
  if (!out) return SFEM_EINVAL;
  *out = nullptr;
  sfem_gnn* h = new (std::nothrow) sfem_gnn;
  if (!h) return SFEM_ENOMEM;
  h->g.device = device;
  const int st = gnn_guarded(h, [&](sfem::Gnn& g) {
    int count = 0;
    SFEM_HIP(hipGetDeviceCount(&count));
    SFEM_REQUIRE(device >= 0 && device < count, SFEM_EINVAL, "bad device ordinal");
    const int64_t n = sfem::param_layout().total;
    g.params.reserve(n);
    g.grad.reserve(n);
    g.adam_m.reserve(n);
    g.adam_v.reserve(n);
    g.params_bf16.reserve(n);
    sfem::gnn_init_params(g, seed);
    return SFEM_OK;
  });
  if (st != SFEM_OK) {
    sfem_gnn_destroy(h);
    return st;
  }
  *out = h;
  return SFEM_OK;
}

void sfem_gnn_destroy(sfem_gnn* h) {
  if (!h) return;
  (void)hipSetDevice(h->g.device);
  (void)hipDeviceSynchronize();
  delete h;
}

const char* sfem_gnn_last_error(const sfem_gnn* h) { return h ? h->g.err.c_str() : "null network"; }

int sfem_gnn_get_params(sfem_gnn* h, float* params, int64_t n) {
  return gnn_guarded(h, [&](sfem::Gnn& g) {
    SFEM_REQUIRE(params && n == sfem::param_layout().total, SFEM_EINVAL,
                 "params must hold sfem_gnn_num_params() floats");
    SFEM_HIP(hipDeviceSynchronize());
    SFEM_HIP(hipMemcpy(params, g.params.get(), sizeof(float) * n, hipMemcpyDeviceToHost));
    return SFEM_OK;
  });
}

int sfem_gnn_set_params(sfem_gnn* h, const float* params, int64_t n) {
  return gnn_guarded(h, [&](sfem::Gnn& g) {
    SFEM_REQUIRE(params && n == sfem::param_layout().total, SFEM_EINVAL,
                 "params must hold sfem_gnn_num_params() floats");
    SFEM_HIP(hipDeviceSynchronize());
    const std::vector<float> zero(n, 0.f);
    SFEM_HIP(hipMemcpy(g.params.get(), params, sizeof(float) * n, hipMemcpyHostToDevice));
    SFEM_HIP(hipMemcpy(g.adam_m.get(), zero.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    SFEM_HIP(hipMemcpy(g.adam_v.get(), zero.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    g.adam_t = 0;
    return SFEM_OK;
  });
}

// Weights file: eight little-endian uint32 header words (magic "SFGN",
// format version, width, layers, node features, edge features, parameter
// count, 0), then the parameters as float32 in the order of
// sfem_gnn_get_params.
namespace {
constexpr uint32_t kWeightsMagic = 0x4e474653u;  // bytes 'S' 'F' 'G' 'N'
constexpr uint32_t kWeightsVersion = 1;

void weights_header(uint32_t (&h)[8]) {
  const uint32_t n = uint32_t(sfem::param_layout().total);
  const uint32_t v[8] = {kWeightsMagic, kWeightsVersion, uint32_t(sfem::kH),
                         uint32_t(sfem::kLayers), uint32_t(sfem::kFNode),
                         uint32_t(sfem::kFEdge), n, 0u};
  for (int i = 0; i < 8; ++i) h[i] = v[i];
}
}  // namespace

int sfem_precond_save(sfem_gnn* h, const char* path) {
  return gnn_guarded(h, [&](sfem::Gnn& g) {
    SFEM_REQUIRE(path != nullptr, SFEM_EINVAL, "null path");
    const int64_t n = sfem::param_layout().total;
    std::vector<float> host(n);
    SFEM_HIP(hipDeviceSynchronize());
    SFEM_HIP(hipMemcpy(host.data(), g.params.get(), sizeof(float) * n, hipMemcpyDeviceToHost));
    uint32_t hdr[8];
    weights_header(hdr);
    FILE* f = std::fopen(path, "wb");
    SFEM_REQUIRE(f != nullptr, SFEM_EINVAL, std::string("cannot open for writing: ") + path);
    const bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
                    std::fwrite(host.data(), sizeof(float), size_t(n), f) == size_t(n);
    const bool closed = std::fclose(f) == 0;
    SFEM_REQUIRE(ok && closed, SFEM_EINVAL, std::string("write failed: ") + path);
    return SFEM_OK;
  });
}

int sfem_precond_load(sfem_gnn* h, const char* path) {
  return gnn_guarded(h, [&](sfem::Gnn& g) {
    SFEM_REQUIRE(path != nullptr, SFEM_EINVAL, "null path");
    FILE* f = std::fopen(path, "rb");
    SFEM_REQUIRE(f != nullptr, SFEM_EINVAL, std::string("cannot open: ") + path);
    const int64_t n = sfem::param_layout().total;
    uint32_t hdr[8], want[8];
    weights_header(want);
    std::vector<float> host(n);
    const bool got_hdr = std::fread(hdr, sizeof(hdr), 1, f) == 1;
    bool same = got_hdr;
    for (int i = 0; same && i < 8; ++i) same = hdr[i] == want[i];
    const bool got = same && std::fread(host.data(), sizeof(float), size_t(n), f) == size_t(n);
    const bool at_end = got && std::fgetc(f) == EOF;
    std::fclose(f);
    SFEM_REQUIRE(got_hdr && hdr[0] == kWeightsMagic, SFEM_EINVAL,
                 std::string("not a weights file: ") + path);
    SFEM_REQUIRE(same, SFEM_EINVAL,
                 std::string("weights file of another format version or network shape: ") + path);
    SFEM_REQUIRE(got && at_end, SFEM_EINVAL, std::string("truncated or oversized weights file: ") + path);
    for (int64_t i = 0; i < n; ++i)
      SFEM_REQUIRE(std::isfinite(host[i]), SFEM_EINVAL,
                   std::string("non-finite parameter in weights file: ") + path);
    SFEM_HIP(hipDeviceSynchronize());
    const std::vector<float> zero(n, 0.f);
    SFEM_HIP(hipMemcpy(g.params.get(), host.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    SFEM_HIP(hipMemcpy(g.adam_m.get(), zero.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    SFEM_HIP(hipMemcpy(g.adam_v.get(), zero.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    g.adam_t = 0;
    return SFEM_OK;
  });
}

int sfem_gnn_set_pairs(sfem_ctx* h, int64_t n_pairs, const float* r, const float* e,
                       int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.topo.valid, SFEM_ESTATE, "set a mesh first");
    SFEM_REQUIRE(n_pairs >= 1 && r && e, SFEM_EINVAL, "need n_pairs >= 1 and non-null r, e");
    SFEM_REQUIRE(ptr_kind == SFEM_PTR_HOST || ptr_kind == SFEM_PTR_DEVICE, SFEM_EINVAL,
                 "ptr_kind must be SFEM_PTR_HOST or SFEM_PTR_DEVICE");
    sfem::gnn_set_pairs(c, n_pairs, r, e);
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

int sfem_gnn_generate_pairs(sfem_ctx* h, int n_rhs, int snaps_per_rhs, uint64_t seed,
                            int64_t* n_pairs) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
    const int64_t k = sfem::gnn_generate_pairs(c, n_rhs, snaps_per_rhs, seed);
    if (n_pairs) *n_pairs = k;
    return SFEM_OK;
  });
}

int sfem_gnn_loss_grad(sfem_gnn* gh, sfem_ctx* h, const int32_t* pair_ids, int n_ids,
                       double* loss, float* grad) {
  if (!gh) return SFEM_EINVAL;
  return guarded(h, [&](Ctx& c) {
    sfem::Gnn& g = gh->g;
    SFEM_REQUIRE(g.device == c.device, SFEM_EINVAL, "network and context on different devices");
    SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
    SFEM_REQUIRE(pair_ids && n_ids >= 1, SFEM_EINVAL, "need pair ids");
    const double L = sfem::gnn_loss_grad(c, g, pair_ids, n_ids, grad != nullptr);
    if (grad) {
      SFEM_HIP(hipStreamSynchronize(c.stream));
      SFEM_HIP(hipMemcpy(grad, g.grad.get(), sizeof(float) * sfem::param_layout().total,
                         hipMemcpyDeviceToHost));
    }
    SFEM_HIP(hipStreamSynchronize(c.stream));
    if (loss) *loss = L;
    return SFEM_OK;
  });
}

int sfem_gnn_train(sfem_gnn* gh, sfem_ctx* const* ctxs, int n_ctx, int steps, int batch,
                   double lr, uint64_t seed, float* losses) {
  if (!gh || !ctxs || n_ctx < 1) return SFEM_EINVAL;
  for (int i = 0; i < n_ctx; ++i)
    if (!ctxs[i]) return SFEM_EINVAL;
  return guarded(ctxs[0], [&](Ctx&) {
    sfem::Gnn& g = gh->g;
    SFEM_REQUIRE(steps >= 0 && batch >= 1 && batch <= 64 && lr > 0.0, SFEM_EINVAL,
                 "need steps >= 0, 1 <= batch <= 64, lr > 0");
    for (int i = 0; i < n_ctx; ++i) {
      Ctx& c = ctxs[i]->c;
      SFEM_REQUIRE(c.device == g.device, SFEM_EINVAL, "network and context on different devices");
      SFEM_REQUIRE(c.assembled && c.gnn && c.gnn->n_pairs > 0, SFEM_ESTATE,
                   "every context needs sfem_assemble and training pairs");
    }
    uint64_t st = seed;
    auto next = [&]() {  // splitmix64
      st += 0x9e3779b97f4a7c15ull;
      uint64_t z = st;
      z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
      z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
      return z ^ (z >> 31);
    };
    std::vector<int32_t> ids(batch);
    for (int k = 0; k < steps; ++k) {
      Ctx& c = ctxs[k % n_ctx]->c;
      const uint64_t np = uint64_t(c.gnn->n_pairs);
      for (int p = 0; p < batch; ++p) ids[p] = int32_t(next() % np);
      const double L = sfem::gnn_loss_grad(c, g, ids.data(), batch, true);
      sfem::gnn_adam(g, c.stream, lr, 0.9, 0.999, 1e-8);
      // the next step may run on another context's stream
      SFEM_HIP(hipStreamSynchronize(c.stream));
      if (losses) losses[k] = float(L);
    }
    return SFEM_OK;
  });
}

int sfem_gnn_apply(sfem_gnn* gh, sfem_ctx* h, double* ms) {
  if (!gh) return SFEM_EINVAL;
  return guarded(h, [&](Ctx& c) {
    sfem::Gnn& g = gh->g;
    SFEM_REQUIRE(g.device == c.device, SFEM_EINVAL, "network and context on different devices");
    SFEM_REQUIRE(c.assembled, SFEM_ESTATE, "call sfem_assemble first");
    SFEM_HIP(hipEventRecord(c.ev0, c.stream));
    sfem::gnn_precondition(c, g);
    SFEM_HIP(hipEventRecord(c.ev1, c.stream));
    SFEM_HIP(hipEventSynchronize(c.ev1));
    float t = 0;
    SFEM_HIP(hipEventElapsedTime(&t, c.ev0, c.ev1));
    if (ms) *ms = t;
    // the M apply kernel, once per mesh (outside the timed inference)
    if (!c.mapply_tuned) {
      sfem::tune_mapply(c);
      c.mapply_tuned = true;
    }
    return SFEM_OK;
  });
}

int sfem_get_precond(sfem_ctx* h, float* correction, double* dinv_sqrt, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "call sfem_gnn_apply first");
    download(c, correction, c.mval.get(), 9 * c.topo.nb, ptr_kind);
    download(c, dinv_sqrt, c.msqrt.get(), c.n_dof(), ptr_kind);
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

int sfem_get_precond_info(sfem_ctx* h, double* theta, double* lambda_min, double* lambda_max) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "call sfem_gnn_apply first");
    if (theta) *theta = c.m_theta;
    if (lambda_min) *lambda_min = c.m_lmin;
    if (lambda_max) *lambda_max = c.m_lmax;
    return SFEM_OK;
  });
}

int sfem_set_precond_kernel(sfem_ctx* h, int variant) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "call sfem_gnn_apply first");
    sfem::tune_mapply(c, variant);
    c.mapply_tuned = true;
    return SFEM_OK;
  });
}

int sfem_get_precond_kernel(sfem_ctx* h, int* variant, double* us_rows, double* us_lds,
                            double* us_grouped) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "call sfem_gnn_apply first");
    if (variant) *variant = c.mapply_kernel;
    if (us_rows) *us_rows = c.mapply_us[0];
    if (us_lds) *us_lds = c.mapply_us[1];
    if (us_grouped) *us_grouped = c.mapply_us[2];
    return SFEM_OK;
  });
}

int sfem_precond_apply(sfem_ctx* h, const double* r, double* z, int ptr_kind) {
  return guarded(h, [&](Ctx& c) {
    SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "call sfem_gnn_apply first");
    SFEM_REQUIRE(r && z, SFEM_EINVAL, "null vector");
    const int64_t n = c.n_dof();
    sfem::DBuf<double> dr, dz;
    dr.reserve(n);
    dz.reserve(n);
    upload(c, dr.get(), r, n, ptr_kind);
    sfem::learned_apply(c, dr.get(), dz.get());
    download(c, z, dz.get(), n, ptr_kind);
    SFEM_HIP(hipStreamSynchronize(c.stream));
    return SFEM_OK;
  });
}

int sfem_precond_apply_noalloc(sfem_ctx* h, const double* r, double* z) {
  return guarded(h, [&](Ctx& c) {
    sfem::precond_apply_noalloc(c, r, z);
    return SFEM_OK;
  });
}

}  // extern "C"
