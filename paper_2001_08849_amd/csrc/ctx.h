// The library context: every device buffer of one mesh / problem.
#pragma once
#include <memory>

#include "common.h"

namespace sfem {

// Numeric-assembly tile: a run of consecutive node rows whose 3x3 blocks
// (and their FP64 values) fit in LDS.  kTileBlocks is the block capacity.
constexpr int kTileBlocks = 320;
// Largest node degree (3x3 blocks in a row) the slot map can encode.
constexpr int kMaxDeg = 64;

// Face record in HBM: support nodes (a, b, c, o1, o2), tets (t1, t2), and
// the face's assembly bound max(V_i G_i) as FP32 bits (32 bytes).  o2 = t2 =
// -1 for an exterior face.
constexpr int kFaceStride = 8;

struct Topology {
  int64_t N = 0, T = 0;
  int64_t nf = 0, ne = 0;        // faces, exterior faces
  int64_t n_inc = 0;             // node-face incidences (sum of support sizes)
  int64_t nb = 0;                // 3x3 blocks of the pattern
  int maxdeg = 0;                // most blocks in one node row
  int max_inc = 0;               // most incident faces of one node
  int n_tiles = 0;
  int64_t key_w = 0;             // face-key base: largest tet vertex-id spread + 1
  DBuf<int32_t> face;            // [nf][kFaceStride]
  DBuf<int32_t> inc_ptr;         // [N+2] (bucket N collects exterior padding)
  DBuf<int32_t> inc;             // face ids per node, ascending
  DBuf<uint32_t> slot;           // per incidence: block slots of the face's support
  DBuf<int32_t> bptr;            // [N+1] block-row offsets
  DBuf<int32_t> bcol;            // [nb] block column (node) ids, ascending per row
  DBuf<int32_t> tile_first;      // [n_tiles+1] first node of each tile
  DBuf<uint16_t> irow;           // per incidence: its row's index within the row's tile
  DBuf<float> row_vg;            // [N] largest face bound max(V_i G_i) of each row
  bool valid = false;
};

// Edge-based smoothing domains (ES-FEM): one domain per mesh edge, made of
// a sixth of every tet around the edge; its support is all nodes of those
// tets.
constexpr int kEdgeSup = 16;   // support nodes of an edge domain, at most
constexpr int kEdgeTets = 12;  // tets around one edge, at most
constexpr int kEdgeRec = 4 + 3 * kEdgeSup;  // V_k, lam, mu, (unused), b[kEdgeSup][3]

struct EdgeTopo {
  int64_t ne = 0;                // edges
  int64_t n_inc = 0;             // (node, edge) incidences: sum of support sizes
  int max_inc = 0;               // most edge domains holding one node
  int max_sup = 0;               // largest support of an edge domain
  DBuf<int32_t> etab;            // [ne][4]: a < b, first entry, tet count
  DBuf<uint64_t> ent;            // tet entries (b << 32 | tet), grouped by edge
  DBuf<int32_t> esup;            // [ne][kEdgeSup] support nodes ascending, -1 padded
  DBuf<int32_t> inc_ptr, inc;    // node -> edges whose support holds it (ascending)
  DBuf<uint8_t> slot;            // [n_inc][kEdgeSup] block slot of each support node
  DBuf<double> rec;              // [ne][kEdgeRec], per assembly
  DBuf<double> ebound;           // [ne] bound of one contribution of each edge, per assembly
  DBuf<int16_t> rexp;            // [N] per-row fixed-point unit exponent (per-tet materials)
  DBuf<float> row_eg;            // [N] per-row geometric bound factor, with the topology
};

// Row-kernel schedule: variant index (lanes per row, rows per group step)
// and a cap on the grid size.
constexpr int kNumSched = 18;
// LDS-staged product (schedule 17): node rows in chunks of kChunkRows; the
// x entries a chunk gathers (at most kWindow nodes) are staged in LDS once
// per chunk.
constexpr int kChunkRows = 128;
constexpr int kWindow = 1024;
struct RowSched {
  int variant;
  int grid_cap;
};

struct GnnWork;

struct CgScalars {
  double rz, rz_new, pq, alpha, beta, rr, rr_true, ff;
  double aux[8];
  int converged;
  int pad;
  unsigned int counter[8];
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  // mesh
  int64_t N = 0, T = 0;
  DBuf<double> xyz;
  DBuf<int32_t> tets;
  Topology topo;
  int domain = SFEM_DOMAIN_FACE;  // smoothing domains of the assembly
  EdgeTopo et;                    // SFEM_DOMAIN_EDGE only

  // material
  bool have_material = false;
  bool per_tet = false;
  double lam0 = 0, mu0 = 0;
  DBuf<double> lam_t, mu_t;

  // BCs and loads
  DBuf<uint8_t> fixed;           // [3N] 1 if the DOF is prescribed
  // [N] 1 if node row I or one of its block columns has a prescribed DOF
  // (only those rows can need the BC rule when K is written); remade after
  // the BCs or the pattern change
  DBuf<uint8_t> bc_row;
  bool bc_row_valid = false;
  DBuf<double> ubar;             // [3N] prescribed values (0 where free)
  bool any_fixed = false, any_nonzero_bc = false;
  double penalty = 0.0;          // > 0: penalty form instead of elimination
  DBuf<double> f_user;           // [3N] loads as given
  DBuf<double> f_bc;             // [3N] right-hand side after BCs

  // assembled matrix (values in the scalar CSR order of the block pattern)
  bool assembled = false;
  bool val_has_bc = false;
  bool have_f32 = false;
  DBuf<double> val;
  DBuf<float> val32;
  // Packed layout of the block pattern (for the packed row schedules and
  // the learned M): node row I holds a [9][d4] array (component q = 3a + c
  // major, blocks minor; d4 = deg rounded up to 4, zero padding) at
  // 9 * ptr4[I]; col4 lists its block columns padded with I.
  DBuf<int32_t> ptr4, col4;
  int64_t nb4 = 0;
  // Window tables of the LDS-staged schedule (once per mesh): per chunk its
  // window's node ids ascending (wcol [chunks][kWindow]) and count (wcnt),
  // and per packed block column its index in the chunk's window (lcol4).
  // lds_tables: 0 not built, 1 built, -1 a chunk's window does not fit.
  DBuf<int32_t> wcol, wcnt;
  DBuf<uint16_t> lcol4;
  int lds_tables = 0;
  DBuf<double> valp;             // K_bc packed (valid while packed64)
  DBuf<float> valp32;            // FP32 copy packed (valid while packed32)
  bool packed64 = false, packed32 = false;
  // val holds the current K_bc (the face assembly writes only the packed
  // copy; the CSR order is made from it when a caller needs it)
  bool csr64 = false;
  DBuf<double> dinv;             // Jacobi: 1 / diag(K_bc)
  DBuf<float> dinv32;
  // [N][9] block row sums of K_bc: R_I[a][c] = sum_J K_bc[3I+a][3J+c] (the
  // row's response to a unit translation along c), each compensated-summed
  // and rounded once; they let products run in the translation form
  // (valid while have_rsum, remade after every assembly)
  DBuf<double> rsum;
  bool have_rsum = false;
  // [N][9] C_I = sum_J (K_bc_IJ - K32_IJ), the block row sums of the FP32
  // copy's rounding (valid while have_rcorr, remade after every assembly):
  // sum_J K32_IJ x_J + C_I x_I is the translation form's value with plain
  // FP32 rows
  DBuf<double> rcorr;
  bool have_rcorr = false;

  // learned preconditioner M = diag(msqrt) (I + S') diag(msqrt), S' in the
  // scalar-CSR value layout of K
  bool have_learned = false;
  double m_theta = 1.0, m_lmin = 0.0, m_lmax = 0.0;  // S' = theta S; Lanczos range of S
  DBuf<float> mval;
  DBuf<__bf16> mvalp;            // the same values, BF16, in the packed layout
  DBuf<double> msqrt;
  // S' also in the grouped layout: per node row, one 80-byte group per 4
  // packed blocks, the 36 BF16 values [q][t] then the 4 int16 column
  // offsets J - I (mgrp_ok: every offset fits; remade with each M)
  DBuf<uint4> mgrp;
  bool mgrp_ok = false;
  // M apply kernel: 0 rows (k_mapply), 1 rh staged in LDS per chunk of rows
  // (k_mapply_lds, needs the window tables), 2 the grouped layout
  // (k_mapply_grp, needs mgrp_ok); chosen by timing each after the first M
  // of a mesh is built (mapply_us: their times, 0 if not timed)
  int mapply_kernel = 0;
  bool mapply_tuned = false;
  double mapply_us[3] = {0.0, 0.0, 0.0};
  DBuf<float> msqrt32;
  std::shared_ptr<GnnWork> gnn;  // features, activations and training pairs

  // solver work vectors
  DBuf<double> x, r, z, p, p2, q, w, xs, rh;
  DBuf<float> x32, r32, z32, p32, p32b, q32, b32, rh32;
  DBuf<double> partials;
  DBuf<CgScalars> sc;
  CgScalars* sc_host = nullptr;  // pinned mirror

  // one full check period of CG iterations captured as a hipGraph, with the
  // addresses, sizes and schedule it was captured for
  bool graph_replay = true;
  hipGraph_t cg_graph = nullptr;
  hipGraphExec_t cg_exec = nullptr;
  std::vector<const void*> cg_key;
  void drop_cg_graph() {
    if (cg_exec) (void)hipGraphExecDestroy(cg_exec);
    if (cg_graph) (void)hipGraphDestroy(cg_graph);
    cg_exec = nullptr;
    cg_graph = nullptr;
    cg_key.clear();
  }

  // row-kernel schedules (FP64 and FP32 matrices), set by the autotuner
  RowSched sched64{2, 4096};
  RowSched sched32{2, 4096};

  // timings
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t tev0 = nullptr, tev1 = nullptr;  // sfem_timer_*
  std::vector<hipEvent_t> prof_ev;             // per-launch SpMV timing
  bool profile = false;
  double prof_ms = 0, prof_mms = 0;  // summed SpMV / learned-M launch times
  int prof_n = 0, prof_mn = 0;
  double ms_topology = 0, ms_assemble = 0;

  int64_t n_dof() const { return 3 * N; }
};

// topology.hip
void build_topology(Ctx& c);
void face_bounds(Ctx& c);  // fills the face records' assembly bound
// Reverse Cuthill-McKee: perm[new] = old (device arrays, synchronous).
void rcm_order(hipStream_t s, int64_t N, int64_t T, const int32_t* tets, int32_t* perm);
bool is_permutation(hipStream_t s, int64_t N, const int32_t* perm);
void permute_mesh(hipStream_t s, int64_t N, int64_t T, const int32_t* perm, const double* xyz,
                  const int32_t* tets, double* xyz_out, int32_t* tets_out);
// Block pattern + assembly tiles of smoothing domains (rows of STRIDE ints,
// PER support nodes or -1 each); returns the most domains holding a node.
template <int STRIDE, int PER>
int build_pattern(Ctx& c, const int32_t* inc_ptr, const int32_t* inc, const int32_t* rows);
// esfem.hip: edge topology (replaces the face pattern) and edge assembly
void build_edge_topology(Ctx& c);
void assemble_edge_values(Ctx& c, double* val_out, float* val32_out, bool apply_mask);
// assemble.hip
void assemble_values(Ctx& c, double* val_out, float* val32_out, bool apply_mask,
                     bool packed = false, bool f32_arith = false);
void bc_mask_values(Ctx& c);
const uint8_t* bc_rows(Ctx& c);  // c.bc_row, remade if stale
void traction_load(Ctx& c, int64_t n_tri, const int32_t* tri_dev, const double t[3]);
void face_stress(Ctx& c, const double* u, double* eps, double* sig);
void scalar_csr_pattern(Ctx& c, int32_t* row_ptr, int32_t* col_idx);
void face_table_public(Ctx& c, int32_t* out);
void extract_dinv(Ctx& c);
void rhs_with_bc(Ctx& c);
// spmv.hip
void spmv_f64(Ctx& c, const double* val, const double* x, double* y, hipStream_t s);
void spmv_f32(Ctx& c, const float* val, const float* x, float* y, hipStream_t s);
void spmv_f32val(Ctx& c, const float* val, const double* x, double* y, hipStream_t s);
// Packed layout: pattern tables (once per mesh) and a value repack.
void pack_pattern(Ctx& c);
void pack_values64(Ctx& c);  // packed copy of the FP64 K (once per assembly)
void ensure_csr64(Ctx& c);   // CSR-order FP64 K from the packed copy, if stale
bool ensure_lds_tables(Ctx& c);  // window tables of schedule 17; false: unavailable
// Times the available M apply kernels on the current M and keeps the
// fastest (or the one forced: variant 0 rows, 1 LDS-staged, 2 grouped; -1
// time them all).
void tune_mapply(Ctx& c, int variant = -1);
void build_mgroups(Ctx& c);  // S' in the grouped layout, after each new packed M
void ensure_rowsum(Ctx& c);      // block row sums R of K_bc (once per assembly)
void ensure_rowcorr(Ctx& c);     // C = R - R32 of the FP32 copy (once per assembly)
// diag(K_bc) from whichever copy of K is current
void matrix_diagonal(Ctx& c, double* diag);
void pack_values_f32(Ctx& c, const float* csr, float* packed);
void pack_values_bf16(Ctx& c, const float* csr, __bf16* packed);
// solve.hip
int solve(Ctx& c, const sfem_solve_opts& o, sfem_solve_info& info);
int64_t learned_apply_partials(Ctx& c);
void learned_apply_into(Ctx& c, const double* r, double* z, double* rh, double* partials);
// noalloc.hip: the static device scratch of the allocation-free entry point
void scratch_init(int device);
void precond_apply_noalloc(Ctx& c, const double* r, double* z);
double true_residual(Ctx& c, const double* u);
void autotune_rows(Ctx& c, int reps, double* best_us64, double* best_us32);

}  // namespace sfem
