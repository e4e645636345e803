/*
 * sfem.h -- C ABI of the MI355X (gfx950) face-based smoothed FEM library.
 *
 * What it computes (juSFEM, arXiv 2001.08849):
 *   - the FS-FEM stiffness of a mesh of four-noded tetrahedra: one smoothing
 *     domain per face (Sec. 2.1 STEP 2, Fig. 1), smoothed gradients b_Ih of
 *     Eq. 7 with the Table-1 Gauss values, K_k = V_k B_k^T c B_k (Eq. 9),
 *     summed over faces into one global matrix (Eq. 8, Eq. 12, STEP 5 of
 *     Sec. 3.3: COO triplets summed into a compressed matrix);
 *   - essential boundary conditions (STEP 5 of Sec. 2.1) and nodal loads;
 *   - the displacements solving K u = f, by preconditioned conjugate
 *     gradients (the paper's direct solver is replaced; see sfem_solve).
 *
 * Conventions (all calls):
 *   - indices are 0-based; node n has the DOFs 3n, 3n+1, 3n+2 (x, y, z);
 *   - every matrix is returned in CSR with int32 row_ptr/col_idx, column
 *     indices ascending within a row; the pattern is STRUCTURAL: the union
 *     of the face supports (Eq. 12's triplet positions), entries that sum to
 *     exactly zero are kept;
 *   - `ptr_kind` says where a caller buffer lives: SFEM_PTR_HOST or
 *     SFEM_PTR_DEVICE (device memory of the context's GPU);
 *   - the caller owns every buffer it passes; the library copies inputs and
 *     never keeps a caller pointer after a call returns;
 *   - all device work is ordered on the context's HIP stream; a call that
 *     writes host memory synchronises that stream before returning;
 *   - every call returns an sfem_status; on failure sfem_last_error() gives
 *     a message.  A failed call leaves previously set inputs unchanged.
 */
#ifndef SFEM_H
#define SFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfem_ctx sfem_ctx;

typedef enum {
  SFEM_OK = 0,
  SFEM_EINVAL = -1,   /* bad argument (null pointer, size, index out of range) */
  SFEM_EMESH = -2,    /* degenerate tet, or a face shared by more than 2 tets */
  SFEM_ENOMEM = -3,   /* device allocation failed */
  SFEM_EHIP = -4,     /* HIP runtime error */
  SFEM_ENOCONV = -5,  /* solve stopped before rtol; u and info still written */
  SFEM_ESTATE = -6    /* call out of order (e.g. solve before a mesh is set) */
} sfem_status;

enum { SFEM_PTR_HOST = 0, SFEM_PTR_DEVICE = 1 };

/* Which matrix sfem_get_csr returns (SFEM_K_F32: the FP32 copy of the
 * BC-applied K, its values widened to float64; needs an FP32 assembly). */
enum { SFEM_K_UNCONSTRAINED = 0, SFEM_K_WITH_BC = 1, SFEM_K_F32 = 2 };

/* sfem_assemble flags. */
enum {
  SFEM_ASM_F64 = 0,       /* FP64 values only */
  SFEM_ASM_F32_COPY = 1,  /* also keep an FP32 copy (the FP64 values rounded;
                             used by the FP32 solve modes) */
  SFEM_ASM_F32_ARITH = 2  /* an FP32 copy assembled with FP32 face arithmetic:
                             FP64 only for tet volumes and inverse Jacobians;
                             the smoothed gradients, V_k, the Lame constants
                             and the 3x3 blocks in FP32, each contribution
                             rounded once to the row's fixed-point unit and
                             summed exactly (a second pass after the FP64
                             one; face-based domains only) */
};

/* Solver choices (sfem_solve_opts). */
enum { SFEM_PRECOND_JACOBI = 0, SFEM_PRECOND_LEARNED = 1 };
enum { SFEM_MODE_F64 = 0, SFEM_MODE_F32_IR = 1, SFEM_MODE_F32_RR = 2, SFEM_MODE_F32_TF = 3 };

/* ----------------------------------------------------------------------------
 * Context.  `device` is a HIP device ordinal; `hip_stream` is a hipStream_t
 * (NULL: the library creates and owns one).  A caller-provided stream must
 * outlive the context.  Not thread-safe: one thread per context at a time.
 */
int sfem_create(sfem_ctx** out, int device, void* hip_stream);
void sfem_destroy(sfem_ctx* ctx);
const char* sfem_last_error(const sfem_ctx* ctx);   /* valid until the next call */
int sfem_set_stream(sfem_ctx* ctx, void* hip_stream);
/* Graph replay of PCG check periods (default on): after the first period
 * of a solve, each full period of check_every iterations is captured once
 * as a hipGraph on the context stream and replayed while the buffers, sizes
 * and row schedule stay the same.  enabled = 0 launches every kernel one by
 * one instead (same results bit for bit), for tools that cannot follow
 * graph launches; the captured graph is released.  Applies to sfem_solve
 * and the training-pair solves of sfem_gnn_generate_pairs (the batched
 * solve always runs as one graph). */
int sfem_set_graph_replay(sfem_ctx* ctx, int enabled);

/* ----------------------------------------------------------------------------
 * Mesh (Sec. 3.2: the matrices Node [N][3] and Element [T][4]).
 * xyz: float64 [n_nodes][3] row-major; tets: int32 [n_tets][4].
 * Vertex order within a tet is free (orientation is not required).
 * Copies both arrays, checks every index is in [0, n_nodes), and builds the
 * topology on the device: the face table (Alg. 1, by device sort of face
 * keys), the node-to-face incidence and the CSR pattern.  Errors:
 * SFEM_EINVAL (bad index / sizes; n_nodes must be < 2^29, the matrix's
 * 9 x (3x3 blocks) < 2^31, and (largest vertex-id spread of a tet + 1)^2 *
 * 4 n_tets < 2^63: renumber arbitrary numberings with sfem_rcm_permutation),
 * SFEM_EMESH (a face in more than two tets, a tet of zero volume, a node in
 * no tet, a node with more than 64 neighbours).  Resets material, BCs and
 * loads.
 */
int sfem_set_mesh(sfem_ctx* ctx, int64_t n_nodes, const double* xyz,
                  int64_t n_tets, const int32_t* tets, int ptr_kind);

/* Smoothing domains of the assembly.  SFEM_DOMAIN_FACE (default): the
 * paper's face-based domains (FS-FEM, Sec. 2.1).  SFEM_DOMAIN_EDGE: the
 * edge-based member of the S-FEM family (ES-FEM), built the same way: the
 * domain of edge (a, b) is, in every tet around the edge, the two sub-tets
 * (a, b, face centroid, tet centroid) of the faces through the edge (a
 * sixth of the tet); V_k = sum V_e / 6; b_I = sum (V_e / 6) grad N_I^e /
 * V_k (the boundary integral of n N_I over the domain); the support is
 * every node of those tets; K_k = V_k B^T c B with volume-weighted c.
 * Limits of the edge domains: at most 12 tets around an edge and 64 block
 * columns per node row (SFEM_EMESH otherwise).  Takes effect at the next
 * sfem_set_mesh; called after a mesh was set, it rebuilds the topology and,
 * as sfem_set_mesh does, resets material, BCs and loads.  Stress recovery
 * (sfem_face_stress) is for face domains only (SFEM_ESTATE otherwise). */
enum { SFEM_DOMAIN_FACE = 0, SFEM_DOMAIN_EDGE = 1 };
int sfem_set_smoothing_domain(sfem_ctx* ctx, int domain);

/* Homogeneous isotropic material (the c of Eq. 9): E > 0, -1 < nu < 0.5. */
int sfem_set_material(sfem_ctx* ctx, double E, double nu);

/* Per-tet material: float64 E[n_tets], nu[n_tets].  A smoothing domain
 * uses the quarter-volume-weighted means of its tets' Lame constants (the
 * exact integral of a piecewise-constant c over the domain). */
int sfem_set_material_per_tet(sfem_ctx* ctx, const double* E, const double* nu,
                              int ptr_kind);

/* Essential BCs (STEP 5 of Sec. 2.1): n DOF indices with prescribed values
 * (value == NULL: all zero).  Replaces any previous set.  They are imposed
 * by elimination: row and column of each fixed DOF zeroed except the
 * diagonal, the column's contribution moved to the right-hand side, and
 * f_i = K_ii * value (sfem_set_bc_penalty picks the penalty form instead).
 * Indices must be in [0, 3 n_nodes) and distinct. */
int sfem_set_dirichlet(sfem_ctx* ctx, int64_t n, const int32_t* dof,
                       const double* value, int ptr_kind);

/* The paper's penalty form of STEP 5 (Sec. 3.3): alpha > 0 makes the next
 * assembly add alpha to K_ii of each fixed DOF and set f_i = alpha * value,
 * leaving rows and columns in place; alpha <= 0 restores elimination (the
 * default).  The paper gives no alpha, so the caller must. */
int sfem_set_bc_penalty(sfem_ctx* ctx, double alpha);

/* Nodal load vector f: float64 [3 n_nodes], replaces the current load. */
int sfem_set_nodal_load(sfem_ctx* ctx, const double* f, int ptr_kind);

/* Adds the consistent load of a uniform traction t[3] (host, N/m^2) on n_tri
 * boundary triangles tri: int32 [n_tri][3]: each vertex receives t*A/3 with
 * A the triangle area (Eq. 11). */
int sfem_add_traction(sfem_ctx* ctx, int64_t n_tri, const int32_t* tri,
                      const double t[3], int ptr_kind);

/* ----------------------------------------------------------------------------
 * Numeric assembly of K (Eq. 9 summed over all faces, Eq. 12) into the CSR
 * values, with the essential BCs of sfem_set_dirichlet eliminated in the same
 * pass.  Needs mesh + material.  flags: SFEM_ASM_*. */
int sfem_assemble(sfem_ctx* ctx, int flags);

/* Sizes of the topology: faces (all / exterior), CSR rows and nonzeros,
 * 3x3 node blocks.  Any pointer may be NULL. */
int sfem_get_sizes(sfem_ctx* ctx, int64_t* n_faces, int64_t* n_exterior,
                   int64_t* n_rows, int64_t* nnz, int64_t* n_blocks);

/* Face table, int32 [n_faces][7] = (a, b, c, t1, t2, o1, o2): a < b < c the
 * face's node ids, t1 < t2 its tets (t2 = -1 for an exterior face), o_i the
 * vertex of t_i opposite the face (o2 = -1 if exterior); rows in ascending
 * (a, b, c) order.  Sec. 3.2's Face_in / Face_out are its two row subsets. */
int sfem_get_faces(sfem_ctx* ctx, int32_t* table, int ptr_kind);

/* CSR of K: row_ptr int32 [n_rows+1], col_idx int32 [nnz], val float64
 * [nnz] (any may be NULL to skip).  which: SFEM_K_UNCONSTRAINED or
 * SFEM_K_WITH_BC.  Needs sfem_assemble. */
int sfem_get_csr(sfem_ctx* ctx, int32_t* row_ptr, int32_t* col_idx, double* val,
                 int which, int ptr_kind);

/* Right-hand side after BCs, float64 [3 n_nodes]. */
int sfem_get_rhs(sfem_ctx* ctx, double* f, int ptr_kind);

/* y = K_bc x (FP64), x and y float64 [3 n_nodes]. */
int sfem_spmv(sfem_ctx* ctx, const double* x, double* y, int ptr_kind);

/* ----------------------------------------------------------------------------
 * Solve K u = f.  The FP64 true relative residual ||f - K u||_2 / ||f||_2,
 * recomputed from u with the FP64 matrix, is the stopping test and is
 * reported in info->true_relres.
 *   SFEM_MODE_F64    : Jacobi (or learned) PCG in FP64, true residual every
 *                      check_every iterations and at every candidate stop,
 *                      with residual replacement.
 * precond: SFEM_PRECOND_JACOBI (z = D^-1 r) or SFEM_PRECOND_LEARNED (z = M r
 * with the M of the last sfem_gnn_apply on this context; flexible CG with
 * the Polak-Ribiere beta, in every mode).  M is symmetric but not forced
 * positive definite: if r.M r <= 0 or the solve stops short of rtol, the
 * solve continues with Jacobi PCG from the current u (info->fell_back = 1);
 * the FP64 true residual remains the only stopping test.
 *   SFEM_MODE_F32_IR : iterative refinement: FP64 residual r = f - K u, an
 *                      FP32-matrix PCG solve of K d = r whose recursive
 *                      residual falls by inner_rtol (dot products in FP64),
 *                      u += d.  Needs SFEM_ASM_F32_COPY.
 *   SFEM_MODE_F32_TF : PCG with FP64 vectors, dots and residual replacement
 *                      (every check_every iterations, the convergence test)
 *                      and FP32-matrix products in the translation form:
 *                      q_I = sum_J K32_IJ (p_J - p_I) + R_I p_I, R_I =
 *                      sum_J K_IJ the FP64 block row sums.  K maps rigid
 *                      translations to (nearly) zero, so the FP32 rounding
 *                      of the values only meets neighbour differences of p
 *                      and perturbs the smooth, slowly converging modes far
 *                      less than a plain FP32 product; the recurrence runs
 *                      to rtol without a restart.  The kernels compute the
 *                      same value as sum_J K32_IJ p_J + C_I p_I with C_I =
 *                      sum_J (K_IJ - K32_IJ) (FP64, made once per
 *                      assembly), so the rows are plain FP32 products.
 *                      With f32_from the first part of the solve uses FP64
 *                      products.  Needs SFEM_ASM_F32_COPY.
 *   SFEM_MODE_F32_RR : PCG with FP64 vectors and dots and FP32-matrix
 *                      products, the residual replaced every check_every
 *                      iterations by the FP64 residual f - K u, until the
 *                      FP64 true relative residual reaches f32_until (0:
 *                      1e-3) or stagnates; then FP64 PCG on the correction
 *                      K d = f - K u from the current u.  K u is a small
 *                      difference of large entries (K annihilates rigid
 *                      motions, u is smooth), so an FP32 product's error is
 *                      large relative to ||f||: FP32 products only pay at
 *                      loose accuracy.  Needs SFEM_ASM_F32_COPY.
 * u: float64 [3 n_nodes] output (x0 = 0).  Returns SFEM_ENOCONV if rtol was
 * not reached within max_iter (u and info are still written).
 */
typedef struct {
  int precond;        /* SFEM_PRECOND_* */
  int mode;           /* SFEM_MODE_* */
  double rtol;        /* on the FP64 true relative residual */
  int max_iter;       /* cap on inner iterations (all outer steps) */
  int check_every;    /* true-residual period in iterations (0: 100 in
                         SFEM_MODE_F64, 50 in the FP32 modes) */
  double inner_rtol;  /* F32_IR inner tolerance (0: 1e-2) */
  int max_outer;      /* F32_IR outer-step cap (0: 30) */
  int profile;        /* nonzero: time every SpMV launch with HIP events */
  double f32_until;   /* F32_RR: FP32 products down to this relres (0: 1e-3) */
  double f32_from;    /* F32_TF: FP64 products until the FP64 true relres
                         reaches this level, then FP32 translation-form
                         products continuing the same recurrence (0, or
                         >= 1: FP32 from the first iteration) */
} sfem_solve_opts;

typedef struct {
  int iters;          /* inner CG iterations, all outer steps */
  int outer_steps;    /* refinement steps (1 in SFEM_MODE_F64) */
  int fell_back;      /* 1 if the learned preconditioner was abandoned */
  int converged;      /* 1 if true_relres <= rtol */
  double true_relres; /* FP64 ||f - K u|| / ||f|| at return */
  double ms_solve;    /* device time of the solve (HIP events) */
  double ms_spmv_avg; /* mean device time of one CG SpMV launch (profile) */
  int n_spmv;         /* SpMV launches timed (profile) */
  double ms_mapply_avg; /* mean device time of one learned-M launch (profile) */
  int n_mapply;       /* learned-M launches timed (profile) */
} sfem_solve_info;

int sfem_solve(sfem_ctx* ctx, const sfem_solve_opts* opts, double* u, int ptr_kind,
               sfem_solve_info* info);

/* Post-processing (Sec. 3.4): smoothed strain and stress of every smoothing
 * domain for displacements u (float64 [3 n_nodes]).  strain = B_k d_k (the B
 * of Eq. 4 with the smoothed gradients of Eq. 7 and the displacements of
 * the domain's support nodes), stress = c_k strain (the domain's isotropic
 * c of Eq. 9, volume-weighted Lame constants as in the stiffness); each
 * float64 [n_faces][6] in the order of sfem_get_faces, Voigt xx, yy, zz,
 * yz, xz, xy with engineering shear strains.  Either output may be NULL.
 * Needs a mesh and a material (not an assembly).  ms (may be NULL): device
 * time of the kernel. */
int sfem_face_stress(sfem_ctx* ctx, const double* u, double* strain, double* stress,
                     int ptr_kind, double* ms);

/* Device time in milliseconds of the most recent topology build and the
 * most recent numeric assembly (HIP events on the context stream). */
int sfem_get_timings(sfem_ctx* ctx, double* ms_topology, double* ms_assemble);

/* Row-kernel schedules (SpMV, residual and CG product kernels; the learned
 * M's apply has its own three kernels, see sfem_set_precond_kernel):
 * `variant` in [0, SFEM_NUM_SCHEDULES) picks lanes per node row and a loop
 * shape:
 *   0-3   8/16/32/64 lanes, one row per lane group and step;
 *   4-7   8/16/32/64 lanes, two rows per step (loads of both in flight);
 *   8-9   16/32 lanes, one row, column loop unrolled by 3;
 *   10-12 16/32/64 lanes, unrolled, nontemporal matrix-value loads;
 *   13    32 lanes, two rows, nontemporal matrix-value loads;
 *   14-16 4/8/16 lanes, packed layout: a copy of the values made once per
 *         assembly in which each node row is a [9][deg rounded up to 4]
 *         array, read 4 blocks per lane with 16-byte loads;
 *   17    8 lanes, packed layout, x staged in LDS: a workgroup takes 128
 *         consecutive node rows, loads the x entries they gather (a window
 *         of at most 1,024 nodes, tables made once per mesh) into LDS, then
 *         runs its rows against it (the CG product; the other row kernels
 *         run schedule 15 for it).  Unavailable (SFEM_EINVAL from
 *         sfem_set_schedule, skipped by the autotuner) when a chunk's
 *         window exceeds 1,024 nodes, e.g. under an arbitrary numbering.
 * `grid_cap` caps the workgroups launched.  precision: SFEM_ASM_F64 or
 * SFEM_ASM_F32_COPY (the schedule of the FP32 products of the
 * SFEM_MODE_F32_* solves).  All schedules compute the same products up to
 * floating-point summation order. */
enum { SFEM_NUM_SCHEDULES = 18 };
int sfem_set_schedule(sfem_ctx* ctx, int precision, int variant, int grid_cap);
int sfem_get_schedule(sfem_ctx* ctx, int precision, int* variant, int* grid_cap);

/* Autotuner: times every schedule (variant x grid cap in {1024, 2048, 4096,
 * 8192}) on the context's assembled matrix and keeps the fastest.  FP64:
 * `reps` (0: 10) Jacobi-PCG iterations from b = 1 per candidate, i.e. the
 * product inside the CG loop; *best_us_f64 is the time per iteration.  FP32
 * copy (if any): the same iterations with its values in the translation
 * form (SFEM_MODE_F32_TF's product), over the packed schedules 14-17;
 * *best_us_f32 per iteration.
 * Pointers may be NULL.  Needs sfem_assemble; leaves the solver's work
 * vectors overwritten. */
int sfem_autotune(sfem_ctx* ctx, int reps, double* best_us_f64, double* best_us_f32);

/* Wall-clock device timer on the context stream: start records an event,
 * stop records a second one, waits for it and returns the elapsed ms. */
int sfem_timer_start(sfem_ctx* ctx);
int sfem_timer_stop(sfem_ctx* ctx, double* ms);

/* Waits until all work queued on the context stream has finished. */
int sfem_synchronize(sfem_ctx* ctx);

/* ----------------------------------------------------------------------------
 * Learned preconditioner (an extension: the paper solves directly).
 *
 * Graph: nodes = mesh nodes, edges = the 3x3 blocks (I, J) of K's pattern
 * (self edges included).  With d = diag(K_bc) and A = D^-1/2 K_bc D^-1/2:
 *   node features (8): A_II[0,1], A_II[0,2], A_II[1,2], log(d_3I+a / dbar)
 *                      (a = 0..2; dbar = mean d over free DOFs), fixed(I), 1
 *   edge features (12): A_IJ row-major, (p_J - p_I) / hbar (hbar = mean
 *                      length of the off-diagonal edges)
 * Network (width 64, 4 layers, ReLU):
 *   h = relu(Wn x + bn), e = relu(We y + be)
 *   per layer l: z = W_l [h_I; h_J; e_IJ] + b_l,  e += relu(z),
 *                a_I = mean_J relu(z_IJ),  h += relu(U_l [h_I; a_I] + c_l)
 *   R_IJ = Wo e_IJ (3x3),  S_IJ = (R_IJ + R_JI^T) / 2, zero in the rows and
 *   columns of fixed DOFs;  M = D^-1/2 (I + theta S) D^-1/2 with
 *   theta = min(1, 0.9 / (1.05 |lambda_min(S)|)) if lambda_min(S) < 0, else
 *   1: I + theta S is then positive definite (lambda_min >= 0.1, allowing a
 *   5% underestimate of |lambda_min| by the 40-step Lanczos run that
 *   estimates it on the device).  Training uses the unscaled S.
 * Loss over pairs (r, e) with K e = r:  mean (M r - e).K(M r - e) / e.K e.
 * Parameters: one flat float32 vector, in this order, matrices row-major
 * [fan_out][fan_in]: Wn[64][8] bn[64] We[64][12] be[64], then per layer
 * W[64][192] b[64] U[64][128] c[64], then Wo[9][64]
 * (sfem_gnn_num_params() floats).  Dense layers run in BF16 on the matrix
 * cores with FP32 accumulation; the master copy and Adam state are FP32.
 * A network lives on one device; every context it is used with must be on
 * that device.  Re-assembling a context drops its M, features and pairs.
 * Calls that take a context report errors through sfem_last_error(ctx)
 * (sfem_gnn_train: the first context); the others through
 * sfem_gnn_last_error.
 */
typedef struct sfem_gnn sfem_gnn;

int64_t sfem_gnn_num_params(void);
/* Glorot-uniform weights from `seed`, zero biases, zero decoder (so the
 * untrained M equals Jacobi). */
int sfem_gnn_create(sfem_gnn** out, int device, uint64_t seed);
void sfem_gnn_destroy(sfem_gnn* g);
const char* sfem_gnn_last_error(const sfem_gnn* g);
/* Host float32 copies of the parameters (n must equal num_params).
 * set_params also resets the Adam state. */
int sfem_gnn_get_params(sfem_gnn* g, float* params, int64_t n);
int sfem_gnn_set_params(sfem_gnn* g, const float* params, int64_t n);

/* Weights file of a network (so that a trained network is not retrained).
 * Layout: eight little-endian uint32 header words -- magic 0x4e474653 (the
 * bytes "SFGN"), format version 1, width 64, layers 4, node features 8,
 * edge features 12, parameter count (sfem_gnn_num_params()), 0 -- then the
 * parameters as little-endian float32 in the order of sfem_gnn_get_params.
 * save writes the FP32 master copy; load checks every header word, the
 * length and that each value is finite, then sets the parameters and resets
 * the Adam state (as sfem_gnn_set_params).  Errors (SFEM_EINVAL, message in
 * sfem_gnn_last_error): unopenable file, short write, wrong magic, another
 * version or network shape, truncated or oversized file, non-finite value.
 * A failed load leaves the network unchanged. */
int sfem_precond_save(sfem_gnn* g, const char* path);
int sfem_precond_load(sfem_gnn* g, const char* path);

/* Training pairs of a context: r, e float32 [n_pairs][3 n_nodes] (ptr_kind),
 * copied; r should be K_bc e.  Replaces earlier pairs. */
int sfem_gnn_set_pairs(sfem_ctx* ctx, int64_t n_pairs, const float* r, const float* e,
                       int ptr_kind);
/* Pairs from the plain solver: n_rhs Jacobi-PCG solves K_bc x = b to 1e-10
 * (b_0 = the load vector; b_k = K_bc D^-1/2 u_k for k > 0, u_k seeded
 * uniform in [-1, 1) and zero on fixed DOFs), each giving up to
 * snaps_per_rhs pairs e = x* - x_j, r = K_bc e for the iterates x_j at
 * iterations its (j / snaps_per_rhs)^2 (x_0 = 0 included).  Replaces earlier
 * pairs; *n_pairs gets the count kept.  Needs sfem_assemble. */
int sfem_gnn_generate_pairs(sfem_ctx* ctx, int n_rhs, int snaps_per_rhs, uint64_t seed,
                            int64_t* n_pairs);
/* Loss of the pairs pair_ids[0..n_ids) (host, 1 <= n_ids <= 64) and, if grad
 * is not NULL, its gradient (host float32 [num_params]).  Leaves the
 * forward's M on the context. */
int sfem_gnn_loss_grad(sfem_gnn* g, sfem_ctx* ctx, const int32_t* pair_ids, int n_ids,
                       double* loss, float* grad);
/* Adam training: step k uses context ctxs[k % n_ctx] and `batch` pair
 * indices drawn uniformly (seeded); lr is the Adam step size (betas 0.9,
 * 0.999, eps 1e-8).  losses (host, may be NULL) receives each step's
 * minibatch loss. */
int sfem_gnn_train(sfem_gnn* g, sfem_ctx* const* ctxs, int n_ctx, int steps, int batch,
                   double lr, uint64_t seed, float* losses);
/* Inference: computes M for the context (features, forward, Lanczos and
 * theta) and enables SFEM_PRECOND_LEARNED there.  ms (may be NULL): device
 * time including the host round trips of the Lanczos run. */
int sfem_gnn_apply(sfem_gnn* g, sfem_ctx* ctx, double* ms);
/* theta and the Lanczos estimates of the extreme eigenvalues of S from the
 * last sfem_gnn_apply (pointers may be NULL). */
int sfem_get_precond_info(sfem_ctx* ctx, double* theta, double* lambda_min, double* lambda_max);
/* The kernel that applies M = D^-1/2 (I + theta S) D^-1/2 (Sec. 3.3's
 * preconditioned solve; the network only fills S): variant 0 walks node rows
 * of the packed BF16 copy of theta S gathering r_hat = D^-1/2 r from HBM; 1
 * stages r_hat in LDS per chunk of 128 rows (the window tables of row
 * schedule 17; unavailable when a chunk gathers more than 1,024 nodes); 2
 * walks node rows of a grouped copy in which each 4 blocks of a row are one
 * 80-byte record (36 BF16 values, then the 4 column offsets J - I as int16;
 * made with every M, unavailable when some |J - I| > 32767).
 * The first sfem_gnn_apply on a mesh times each available one (10 applies
 * each, after its own timed inference) and keeps the fastest.
 * set: variant 0, 1 or 2 forces one (times it), -1 times them again;
 * errors SFEM_EINVAL (unknown variant, or one unavailable), SFEM_ESTATE (no
 * M).  get: the variant in use and the three times in microseconds (0: not
 * timed); pointers may be NULL.
 * All give the same z = M r bit for bit; the dot products of the learned
 * solve are grouped per workgroup differently under variant 1. */
int sfem_set_precond_kernel(sfem_ctx* ctx, int variant);
int sfem_get_precond_kernel(sfem_ctx* ctx, int* variant, double* us_rows, double* us_lds,
                            double* us_grouped);

/* The learned preconditioner of a context: the correction theta S (float32
 * [nnz], in the order of sfem_get_csr's values; the solver applies these
 * values rounded to BF16) and d^-1/2 (float64 [3 n_nodes]); either pointer
 * may be NULL. */
int sfem_get_precond(sfem_ctx* ctx, float* correction, double* dinv_sqrt, int ptr_kind);
/* z = M r (float64 [3 n_nodes]) with the learned preconditioner. */
int sfem_precond_apply(sfem_ctx* ctx, const double* r, double* z, int ptr_kind);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): z = M r as
 * sfem_precond_apply, but r and z must be device memory of the context's
 * GPU, the work is only enqueued on the context stream (no synchronisation),
 * and nothing is allocated or freed: the work memory (3 n_nodes + up to
 * 3 x 4096 doubles) is a static 8 MiB device array of the library, one per
 * GPU, held until the process ends.  Limit: n_nodes <= 345,429.  All calls
 * on one GPU share that array, so calls that overlap in time on one GPU
 * (other streams, threads or contexts) race; calls ordered on one stream do
 * not.  The results equal sfem_precond_apply's bit for bit.  Errors, in this
 * order: SFEM_EINVAL (mesh beyond the limit), SFEM_ESTATE (no
 * sfem_gnn_apply on this context), SFEM_EINVAL (null, host or other-GPU
 * pointer). */
int sfem_precond_apply_noalloc(sfem_ctx* ctx, const double* r, double* z);

/* ----------------------------------------------------------------------------
 * Batched solves: many meshes, up to four load cases each, in one solve
 * (an extension; the paper solves one mesh).  The meshes are concatenated
 * into one block-diagonal system built by the single-mesh pipeline; the four
 * load cases of a mesh share K and are multiplied together.  Every (mesh,
 * load case) pair is its own CG system with its own scalars, Jacobi
 * preconditioner and FP64 true-residual stopping test (every check_every
 * iterations, with residual replacement); a system that meets rtol, breaks
 * down (p.K p <= 0) or stagnates for 40 checks stops iterating while the
 * others continue.  With use_graph, one check period (check_every
 * iterations + the residual check) is captured in a hipGraph once and
 * replayed.  Inputs are host arrays, copied; errors through
 * sfem_batch_last_error.
 */
typedef struct sfem_batch sfem_batch;

int sfem_batch_create(sfem_batch** out, int device);
void sfem_batch_destroy(sfem_batch* b);
const char* sfem_batch_last_error(const sfem_batch* b);
/* Adds a mesh (0-based local node ids): xyz float64 [n_nodes][3], tets int32
 * [n_tets][4], homogeneous E, nu, and the local DOFs fixed to zero.
 * *mesh_index (may be NULL) gets its index. */
int sfem_batch_add_mesh(sfem_batch* b, int64_t n_nodes, const double* xyz, int64_t n_tets,
                        const int32_t* tets, double E, double nu, int64_t n_fixed,
                        const int32_t* fixed_dofs, int* mesh_index);
/* Uniform traction t (force per area) on triangles (local node ids, int32
 * [n_tri][3]) of a mesh, for load case rhs in [0, 4).  Load cases without
 * any traction are zero and count as solved. */
int sfem_batch_add_traction(sfem_batch* b, int mesh, int rhs, int64_t n_tri,
                            const int32_t* tri, const double t[3]);
/* Topology, assembly, loads and BCs of all meshes (flags: SFEM_ASM_F64 or
 * SFEM_ASM_F32_COPY, needed by SFEM_MODE_F32_RR). */
int sfem_batch_build(sfem_batch* b, int flags);
int sfem_batch_sizes(sfem_batch* b, int* n_meshes, int64_t* n_nodes, int64_t* n_tets,
                     int64_t* n_faces, int64_t* nnz);
/* Autotuner.  Meshes fall into size buckets by node count: 0 (< 8192),
 * 1 (< 32768), 2 (larger).  For each non-empty bucket every schedule of the
 * 4-right-hand-side product is timed over `reps` launches (0: 5) of that
 * bucket alone: (lanes per node row in {8, 16, 32} on the CSR-order values,
 * or in {4, 8} on the packed layout, FP64 only) x (node rows per workgroup
 * in {16, 64, 256}, at least 256 / lanes so that no lane group idles).
 * A candidate's cost is its time with every system active plus its time
 * with only the bucket's largest mesh active (late in a solve most meshes
 * have finished); the solver's own compacted work lists are used for both.
 * The cheapest is kept and cached for the process under
 * the bucket's shape (bucket, log2 of its node rows, mean block degree).
 * With use_cache, a cached shape is reused without timing.  precision:
 * SFEM_ASM_F64 or SFEM_ASM_F32_COPY (CSR-order candidates only; an FP32
 * product under a packed schedule uses 16 lanes on the CSR order).
 * *us: the tuned product's time.  get_schedule reports a bucket's choice;
 * *packed = 1 for the packed layout. */
int sfem_batch_autotune(sfem_batch* b, int reps, int use_cache, int precision, double* us);
int sfem_batch_get_schedule(sfem_batch* b, int bucket, int* lanes_per_row, int* rows_per_wg,
                            int* n_meshes, int* from_cache, int* packed);
/* Sets a bucket's schedule by hand (one of the tuner's candidates; tests and
 * tools).  Errors: SFEM_EINVAL (not a candidate), SFEM_ESTATE (not built). */
int sfem_batch_set_schedule(sfem_batch* b, int bucket, int lanes_per_row, int rows_per_wg,
                            int packed);

typedef struct {
  int mode;           /* SFEM_MODE_F64 or SFEM_MODE_F32_RR (FP32 products, FP64 rest) */
  double rtol;        /* per system, on the FP64 true relative residual */
  int max_iter;       /* cap on iterations (0: 100000) */
  int check_every;    /* iterations per check period (0: 50) */
  int use_graph;      /* nonzero: replay a captured hipGraph per period */
} sfem_batch_opts;

typedef struct {
  double ms_solve;    /* device time of the whole batched solve */
  int periods;        /* check periods run */
  int all_converged;
  int max_iters;      /* most iterations of any system */
  double worst_relres;
  int fp64_from_period; /* SFEM_MODE_F32_RR: the check period after which the
                           batch continued with FP64 products because a
                           system stagnated with FP32 ones (0: never) */
} sfem_batch_info;

/* Solves all systems by CG with Jacobi preconditioning, every system from
 * x = 0, in check periods: each period runs check_every iterations of the
 * 4-right-hand-side product and the per-system updates, then the FP64
 * residual replacement and the convergence test.  A mesh whose 4 systems
 * have all finished (converged, broken down or stagnated) drops out of the
 * work lists remade at the start of the next period.  In SFEM_MODE_F32_RR a
 * system past relres 1e-3 whose residual makes no new minimum for 10 checks
 * (FP32 products too coarse for its conditioning) makes the whole batch
 * continue with FP64 products, every active system restarting CG from its
 * current x.
 * SFEM_ENOCONV if any system did not converge. */
int sfem_batch_solve(sfem_batch* b, const sfem_batch_opts* opts, sfem_batch_info* info);
/* Displacements of (mesh, load case): float64 [3 n_nodes(mesh)]. */
int sfem_batch_get_solution(sfem_batch* b, int mesh, int rhs, double* u, int ptr_kind);
/* Per system s = 4 mesh + rhs (host arrays of 4 n_meshes, NULL to skip). */
int sfem_batch_get_system_info(sfem_batch* b, int32_t* iters, int32_t* converged,
                               double* relres, int32_t* breakdown);

/* ----------------------------------------------------------------------------
 * Mesh files and node renumbering (the step before the path).
 *
 * TetGen output (Sec. 3.2 reads the Node / Element / Face matrices from
 * TetGen's .node, .ele and .face files).  sfem_tetgen_read parses
 * <stem>.node and <stem>.ele, and <stem>.face when present, on the host:
 * '#' comments, point attributes and markers are skipped, the first point's
 * index (0 or 1) is the base of all node references, and every reference is
 * range-checked.  Only 4-node tets are accepted.  *out is always set (free
 * it with sfem_tetgen_free, also after an error: sfem_tetgen_last_error
 * holds the message).  Errors: SFEM_EINVAL (missing file, malformed line,
 * index out of range, not 4-node tets), SFEM_ENOMEM.
 */
typedef struct sfem_tetgen sfem_tetgen;
int sfem_tetgen_read(sfem_tetgen** out, const char* stem);
const char* sfem_tetgen_last_error(const sfem_tetgen* m);
/* n_faces = -1 when there is no .face file; has_markers: the .face file has
 * a boundary-marker column. */
int sfem_tetgen_sizes(const sfem_tetgen* m, int64_t* n_nodes, int64_t* n_tets, int64_t* n_faces,
                      int* has_markers, int* index_base);
/* Host copies, 0-based: xyz float64 [n_nodes][3], tets int32 [n_tets][4],
 * faces int32 [n_faces][3], markers int32 [n_faces]; any may be NULL. */
int sfem_tetgen_get(const sfem_tetgen* m, double* xyz, int32_t* tets, int32_t* faces,
                    int32_t* markers);
void sfem_tetgen_free(sfem_tetgen* m);

/* Reverse Cuthill-McKee numbering of the nodes, computed on ctx's device
 * and stream (ctx's own mesh and problem are not touched).  Graph: nodes
 * sharing a tet.  Start of each connected component: George & Liu's
 * pseudo-peripheral node, beginning from the least (degree, id) node still
 * to be numbered.  Cuthill & McKee: each node numbers its unnumbered
 * neighbours by increasing (degree, id); components follow one another;
 * the order is then reversed.  The result depends only on the mesh.
 * perm int32 [n_nodes] gets perm[new] = old.  tets: int32 [n_tets][4]
 * (ptr_kind), perm: perm_ptr_kind; ms (may be NULL) gets the device time.
 * Errors: SFEM_EINVAL (sizes, index out of range). */
int sfem_rcm_permutation(sfem_ctx* ctx, int64_t n_nodes, int64_t n_tets, const int32_t* tets,
                         int ptr_kind, int32_t* perm, int perm_ptr_kind, double* ms);

/* Applies perm[new] = old on the device: xyz_out[new] = xyz[perm[new]] and
 * tets_out = old -> new ids of tets.  All arrays of one ptr_kind; xyz /
 * xyz_out or tets / tets_out may be NULL.  Errors: SFEM_EINVAL (perm is not
 * a permutation of 0..n_nodes-1, sizes, indices). */
int sfem_permute_mesh(sfem_ctx* ctx, int64_t n_nodes, int64_t n_tets, const int32_t* perm,
                      const double* xyz, const int32_t* tets, double* xyz_out,
                      int32_t* tets_out, int ptr_kind);

#ifdef __cplusplus
}
#endif
#endif /* SFEM_H */
