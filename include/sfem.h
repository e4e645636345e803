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

/* Which matrix sfem_get_csr returns. */
enum { SFEM_K_UNCONSTRAINED = 0, SFEM_K_WITH_BC = 1 };

/* sfem_assemble flags. */
enum {
  SFEM_ASM_F64 = 0,       /* FP64 values only */
  SFEM_ASM_F32_COPY = 1   /* also keep an FP32 copy (used by SFEM_MODE_F32_IR) */
};

/* Solver choices (sfem_solve_opts). */
enum { SFEM_PRECOND_JACOBI = 0, SFEM_PRECOND_LEARNED = 1 };
enum { SFEM_MODE_F64 = 0, SFEM_MODE_F32_IR = 1, SFEM_MODE_F32_RR = 2 };

/* ----------------------------------------------------------------------------
 * Context.  `device` is a HIP device ordinal; `hip_stream` is a hipStream_t
 * (NULL: the library creates and owns one).  A caller-provided stream must
 * outlive the context.  Not thread-safe: one thread per context at a time.
 */
int sfem_create(sfem_ctx** out, int device, void* hip_stream);
void sfem_destroy(sfem_ctx* ctx);
const char* sfem_last_error(const sfem_ctx* ctx);   /* valid until the next call */
int sfem_set_stream(sfem_ctx* ctx, void* hip_stream);

/* ----------------------------------------------------------------------------
 * Mesh (Sec. 3.2: the matrices Node [N][3] and Element [T][4]).
 * xyz: float64 [n_nodes][3] row-major; tets: int32 [n_tets][4].
 * Vertex order within a tet is free (orientation is not required).
 * Copies both arrays, checks every index is in [0, n_nodes), and builds the
 * topology on the device: the face table (Alg. 1, by device sort of face
 * keys), the node-to-face incidence and the CSR pattern.  Errors:
 * SFEM_EINVAL (bad index / sizes; n_nodes must be < 2^21 and
 * n_nodes^2 * 4 n_tets < 2^63), SFEM_EMESH (a face in more than two tets,
 * or a tet of zero volume).  Resets material, BCs and loads.
 */
int sfem_set_mesh(sfem_ctx* ctx, int64_t n_nodes, const double* xyz,
                  int64_t n_tets, const int32_t* tets, int ptr_kind);

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
 *   SFEM_MODE_F32_IR : iterative refinement: FP64 residual r = f - K u, an
 *                      FP32-matrix PCG solve of K d = r whose recursive
 *                      residual falls by inner_rtol (dot products in FP64),
 *                      u += d.  Needs SFEM_ASM_F32_COPY.
 *   SFEM_MODE_F32_RR : one PCG run whose products use the FP32 matrix and
 *                      whose vectors and dots are FP64; every check_every
 *                      iterations the residual is replaced by the FP64
 *                      residual f - K u (a refinement step that keeps the
 *                      Krylov recurrences).  Needs SFEM_ASM_F32_COPY.
 * u: float64 [3 n_nodes] output (x0 = 0).  Returns SFEM_ENOCONV if rtol was
 * not reached within max_iter (u and info are still written).
 */
typedef struct {
  int precond;        /* SFEM_PRECOND_* */
  int mode;           /* SFEM_MODE_* */
  double rtol;        /* on the FP64 true relative residual */
  int max_iter;       /* cap on inner iterations (all outer steps) */
  int check_every;    /* true-residual period in iterations (0: 50) */
  double inner_rtol;  /* F32_IR inner tolerance (0: 1e-2) */
  int max_outer;      /* F32_IR outer-step cap (0: 30) */
  int profile;        /* nonzero: time every SpMV launch with HIP events */
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
} sfem_solve_info;

int sfem_solve(sfem_ctx* ctx, const sfem_solve_opts* opts, double* u, int ptr_kind,
               sfem_solve_info* info);

/* Device time in milliseconds of the most recent topology build and the
 * most recent numeric assembly (HIP events on the context stream). */
int sfem_get_timings(sfem_ctx* ctx, double* ms_topology, double* ms_assemble);

/* Row-kernel schedules (SpMV, residual and CG product kernels): `variant`
 * in [0, 8) picks the lanes per node row {8,16,32,64} (variant % 4) and one
 * or two rows per lane group per step (variant / 4); `grid_cap` caps the
 * workgroups launched.  precision: SFEM_ASM_F64 or SFEM_ASM_F32_COPY (the
 * schedule of the FP32 matrix).  All schedules compute the same products up
 * to floating-point summation order. */
int sfem_set_schedule(sfem_ctx* ctx, int precision, int variant, int grid_cap);
int sfem_get_schedule(sfem_ctx* ctx, int precision, int* variant, int* grid_cap);

/* Autotuner: times every schedule (variant x grid cap in {1024, 2048, 4096,
 * 8192}) on the context's assembled matrix, `reps` launches each (0: 10),
 * with HIP events, and keeps the fastest for FP64 and, if an FP32 copy
 * exists, for FP32.  Returns the best microseconds per SpMV (pointers may
 * be NULL).  Needs sfem_assemble. */
int sfem_autotune(sfem_ctx* ctx, int reps, double* best_us_f64, double* best_us_f32);

/* Wall-clock device timer on the context stream: start records an event,
 * stop records a second one, waits for it and returns the elapsed ms. */
int sfem_timer_start(sfem_ctx* ctx);
int sfem_timer_stop(sfem_ctx* ctx, double* ms);

/* Waits until all work queued on the context stream has finished. */
int sfem_synchronize(sfem_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SFEM_H */
