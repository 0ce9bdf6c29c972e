/*
 * hhg.h -- C ABI of the MI355X (gfx950) hierarchical-hybrid-grid full-multigrid library.
 *
 * The library solves the P1 finite-element diffusion problem  -div(kappa grad u) = f  with
 * Dirichlet data g on a hierarchical hybrid grid: a coarse simplicial macro mesh T_0
 * (triangles in 2D, tetrahedra in 3D) refined uniformly L times (Section 2 of the kl-refinement
 * paper).  It runs the full multigrid of Algorithm 4 (procedure FMG) matrix-free on the GPU
 * and computes the FMG-difference error estimate of Section 4 (procedure ErrorEstimate of
 * Algorithm 4), plus an adjoint gradient of a goal functional.
 *
 * Conventions shared by every entry point
 *   - Status codes: every call returns HHG_OK (0) or a negative hhg_status; nothing aborts,
 *     throws across the ABI or prints.  hhg_last_error() gives a message for the last failure
 *     on that context (thread-local for calls that had no context).
 *   - Ownership: the caller owns every buffer it passes; the library copies host mesh arrays
 *     during hhg_setup and never frees caller memory.  The device workspace is allocated by
 *     the caller (for example by PyTorch) and must outlive the context.
 *   - Memory spaces: arguments documented "device" are HIP device pointers on the device that
 *     was current at hhg_bind_workspace; "host" are ordinary host pointers.
 *   - Vectors: float64, one entry per degree of freedom (DoF) of a level, in the library's
 *     canonical DoF order: coarse-vertex DoFs by vertex id, then DoFs interior to coarse
 *     edges, then (3D) interior to coarse faces, then interior to macro elements.  Edges and
 *     faces are numbered by their sorted global vertex tuples; within a primitive DoFs are
 *     ordered lexicographically by their integer coordinates along the primitive's vertices
 *     (sorted by global id), last coordinate most significant; inside a macro element, by the
 *     coordinates along the element's own vertex order.  hhg_dof_coords exports this order.
 *   - Streams: all device work is enqueued on the stream given to hhg_bind_workspace.  Calls
 *     that return host values synchronise that stream first.
 *   - Calls on one context must not overlap (they share the workspace).
 */
#ifndef HHG_H
#define HHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hhg_ctx_s* hhg_ctx;

typedef enum {
  HHG_OK = 0,
  HHG_EINVAL = -1,    /* bad argument or option                                           */
  HHG_EMESH = -2,     /* invalid macro mesh (degenerate or inverted cell, non-manifold face)  */
  HHG_ENOMEM = -3,    /* workspace too small                                                */
  HHG_EHIP = -4,      /* a HIP runtime call failed                                         */
  HHG_ENOTCONV = -5,  /* iteration stagnated or produced NaN                                */
  HHG_ESTATE = -6     /* call made in the wrong state (no workspace, no preceding solve)    */
} hhg_status;

enum { HHG_KAPPA_MACRO = 0, HHG_KAPPA_P1 = 1 };
enum { HHG_GS_REDBLACK = 0, HHG_GS_MULTICOLOR = 1, HHG_JACOBI = 2 };
enum { HHG_FP64 = 0, HHG_FP32_REFINED = 1 };
enum { HHG_OP_STIFFNESS = 0, HHG_OP_MASS = 1 };
/* Norm of the error estimate (remark on the choice of norm, Section 4.4): the consistent mass
 * matrix M_L (L2, the paper's choice), the stiffness matrix A_L with the context's per-macro
 * coefficients (energy), or the row-sum lumped mass matrix. */
enum { HHG_NORM_L2 = 0, HHG_NORM_ENERGY = 1, HHG_NORM_LUMPED = 2 };
/* Local indicator (Section 4.3): ||e~_{L-1}||_T for every j (what the paper implements for
 * P1), the unscaled eta'_{j,T} = ||e~_{L-j}||_T, or the scaled eta_{j,T} =
 * theta~_{L-j,T}^j ||e~_{L-j}||_T with the per-macro factor
 * theta~_{L-j,T} = ||e~_{L-j}||_T / ||e~_{L-j-1}||_T. */
enum { HHG_LOCAL_L1 = 0, HHG_LOCAL_UNSCALED = 1, HHG_LOCAL_SCALED = 2 };

/* Coarse macro mesh T_0.  All arrays are host memory and are copied by hhg_setup. */
typedef struct {
  int dim;                    /* 2 (triangles) or 3 (tetrahedra)                               */
  int64_t n_vertices;
  const double* coords;       /* n_vertices * dim, row-major                                   */
  int64_t n_cells;
  const int32_t* cells;       /* n_cells * (dim+1) vertex ids; vertex 0 is the local origin    */
  const uint8_t* dirichlet;   /* per vertex: 1 = Dirichlet.  A boundary vertex, edge or face is
                                 Dirichlet when all its vertices are flagged.  NULL = the whole
                                 boundary is Dirichlet.                                       */
  const double* kappa_cell;   /* per macro coefficient; NULL = 1                               */
} hhg_mesh;

typedef struct {
  int coefficient;            /* HHG_KAPPA_MACRO: kappa constant per macro element;
                                 HHG_KAPPA_P1: nodal coefficient set by hhg_set_kappa_nodal,
                                 averaged over the vertices of every micro element.  The
                                 nodal-coefficient path is switched off in this build:
                                 hhg_setup returns HHG_EINVAL for HHG_KAPPA_P1.               */
  int smoother;               /* HHG_GS_REDBLACK | HHG_GS_MULTICOLOR | HHG_JACOBI              */
  double jacobi_omega;        /* damping of the Jacobi smoother (0 selects 2/3)                */
  int flags;                  /* HHG_FLAG_NO_FUSED: sweep macro interiors one colour class per
                                 launch instead of all classes in one launch (same result up to
                                 rounding; for checking the fused kernels).
                                 HHG_FLAG_NO_LANE_IFACE: update interface DoFs one thread per
                                 DoF instead of one lane per (DoF, macro) pair (same result up
                                 to rounding; for checking the lane-parallel kernels).
                                 HHG_FLAG_NO_GRAPH: launch every kernel of a solve directly
                                 instead of replaying recorded HIP graphs (same result).
                                 HHG_FLAG_NO_PRELOAD: in the single-workgroup interface sweep,
                                 load every row in its own class instead of loading the
                                 sweep-invariant part of all rows first (same result).
                                 HHG_FLAG_ROWS3D: use the 3D kernels that take one wavefront
                                 per lattice row (operator application; class-by-class
                                 interior sweep) on every level, not only from n = 128 on
                                 (same result; for checking them on small levels).
                                 HHG_FLAG_STREAM3D: with the red-black smoother and a per-macro
                                 coefficient, use the plane-streaming 3D interior sweep on every
                                 level with n >= 4, not only from n = 256 on (same result; for
                                 checking it on small levels).
                                 HHG_FLAG_GENERIC_EST: compute the 2D L2 estimate with the
                                 one-thread-per-node kernel instead of the row kernel (same
                                 result up to rounding; for checking the row kernel).
                                 HHG_FLAG_CLASSWISE_IFACE: sweep the 2D interface classes one
                                 launch per class (or per run of small classes) instead of
                                 all of a sweep in one launch (identical result; for checking
                                 the one-launch form).
                                 HHG_FLAG_NO_PLANES3D: with the red-black smoother and a
                                 per-macro coefficient, sweep the 3D levels with n = 64 with
                                 the kernels used without the whole-plane sweep (same result;
                                 for checking and timing it).
                                 HHG_FLAG_PLANES3D: use the whole-plane 3D sweep on every
                                 level with 16 <= n <= 64, not only on n = 64 (same result;
                                 for checking it on small levels).
                                 HHG_FLAG_TWO_LAUNCH_IFACE: sweep the 2D edge classes and the
                                 vertex classes in two launches (the vertex classes reading the
                                 new edge values from memory) instead of one launch in which
                                 they recompute them (identical result; for checking and
                                 timing the one-launch form).
                                 HHG_FLAG_NO_DENSE_COARSE: run the cycle on every coarse level
                                 kernel by kernel instead of applying the dense map of the
                                 coarse cycle (same result up to rounding; for checking and
                                 timing the map).
                                 HHG_FLAG_DENSE_COARSE: build the dense map on the largest
                                 level that fits, up to L - 1, instead of only when the finest
                                 level lies at least three levels above it (for checking it on
                                 small problems).
                                 HHG_FLAG_NO_FUSED_PROLONG: in 2D, run the cycle's
                                 prolongation as a launch of its own instead of inside the
                                 first post-smoothing sweep, and clear a zero correction
                                 before the first pre-smoothing sweep instead of starting
                                 that sweep from zero (identical result; for checking and
                                 timing the fused forms)                                        */
} hhg_options;

enum {
  HHG_FLAG_NO_FUSED = 1,
  HHG_FLAG_NO_LANE_IFACE = 2,
  HHG_FLAG_NO_GRAPH = 4,
  HHG_FLAG_NO_PRELOAD = 8,
  HHG_FLAG_ROWS3D = 16,
  HHG_FLAG_STREAM3D = 32,
  HHG_FLAG_GENERIC_EST = 64,
  HHG_FLAG_CLASSWISE_IFACE = 128,
  HHG_FLAG_NO_PLANES3D = 256,
  HHG_FLAG_PLANES3D = 512,
  HHG_FLAG_TWO_LAUNCH_IFACE = 1024,
  HHG_FLAG_NO_DENSE_COARSE = 2048,
  HHG_FLAG_DENSE_COARSE = 4096,
  HHG_FLAG_NO_FUSED_PROLONG = 8192
};

typedef struct {
  int nu;                     /* V-cycles per FMG level (Algorithm 4's nu)                     */
  int pre, post;              /* V(pre, post) smoothing sweeps                                 */
  int precision;              /* HHG_FP64, or HHG_FP32_REFINED: float32 V-cycles on the
                                 correction inside float64 residual/update steps              */
  double rtol;                /* extra cycles on level L until ||r|| <= rtol * ||r_0||, where
                                 r_0 is the residual of u = g on the boundary and 0 inside.
                                 rtol = 0 with max_iter > 0: exactly max_iter extra cycles and
                                 no residual norm at all (no host synchronisation inside the
                                 solve; final_rel_residual is then -1)                        */
  int max_iter;               /* cap on those extra cycles (0 = FMG only)                      */
} hhg_solve_params;

typedef struct {
  int vcycles;                /* V-cycles on all FMG levels plus extra cycles                  */
  int ir_steps;               /* extra cycles on level L                                       */
  double final_rel_residual;  /* ||r|| / ||r_0|| after the solve (computed only if max_iter > 0
                                 and rtol > 0; else -1)                                       */
  double ms_total;            /* device time of the solve (HIP events), milliseconds          */
  int dense_level;            /* coarse level k whose cycle from a zero iterate (levels k..0)
                                 ran as one product with its dense map, built on first use for
                                 the precision and sweep counts; -1 if none.  The map is the
                                 same linear map as those launches, so results agree up to
                                 rounding.  Level k is the largest with at most 8192 inner
                                 DoFs and at most 512 MiB for its float32 and float64 maps
                                 together, k <= L - 3 (L - 1 with HHG_FLAG_DENSE_COARSE),
                                 k >= 1                                                        */
} hhg_solve_stats;

/* Validate the macro mesh, build primitives, per-macro stencils and colourings for levels
 * 0..L (Section 2 hierarchy), and plan the workspace.  L >= 1.  On failure *out is NULL. */
hhg_status hhg_setup(const hhg_mesh* coarse, int L, const hhg_options* opt, hhg_ctx* out);

/* Bytes of device workspace the context needs. */
hhg_status hhg_workspace_bytes(hhg_ctx ctx, size_t* bytes);

/* Bind caller-allocated device memory (>= hhg_workspace_bytes, 256-byte aligned) and a HIP
 * stream (NULL = default stream); uploads tables.  Must precede every device call. */
hhg_status hhg_bind_workspace(hhg_ctx ctx, void* device_ptr, size_t bytes, void* hip_stream);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): bind the library's own static workspace instead of caller memory, a variant of
 * hhg_bind_workspace that allocates nothing (no hipMalloc, no HIP events, no graphs).  The
 * workspace is one file-scope device array of HHG_STATIC_WORKSPACE_BYTES per device, held
 * until the process ends; its address on the current device is looked up once.  A context
 * needing more (hhg_workspace_bytes) gets HHG_ENOMEM.  The part the context uses is cleared
 * by a fill kernel on the given stream (NULL = default stream) and the tables are uploaded
 * from host memory (hipMemcpyAsync); the call synchronises the stream.
 * One context per device holds the array: binding another context to it leaves the previous
 * one unbound (its calls return HHG_ESTATE until it is bound again), and the caller must let
 * the previous owner's work finish first; calls of several threads or streams that overlap on
 * one device race.  Contexts bound this way run every launch eagerly (no recorded graphs) and
 * report ms_total = 0 in hhg_solve_stats.  Binding with hhg_bind_workspace releases the array. */
#define HHG_STATIC_WORKSPACE_BYTES (64u << 20)
hhg_status hhg_bind_static_workspace(hhg_ctx ctx, void* hip_stream);

/* Number of DoFs (including Dirichlet ones) on a level, 0 <= level <= L. */
hhg_status hhg_num_dofs(hhg_ctx ctx, int level, int64_t* n);

/* Coordinates of the DoFs of a level in canonical order: device, num_dofs * dim doubles. */
hhg_status hhg_dof_coords(hhg_ctx ctx, int level, double* device_xyz);

/* Replace the per-macro coefficients (host, n_cells values > 0); refactors level 0. */
hhg_status hhg_set_kappa_cell(hhg_ctx ctx, const double* host_kappa);

/* Nodal coefficient on level L (device, canonical order, values > 0); HHG_KAPPA_P1 only
 * (switched off in this build: no context with HHG_KAPPA_P1 can be set up, so every call
 * returns HHG_ESTATE).  Coarser levels use its values at their nodes. */
hhg_status hhg_set_kappa_nodal(hhg_ctx ctx, const double* device_kappa);

/* Full multigrid solve of A_L u = b_L (equation of the per-level linear system, Section 4.4)
 * with b_l = M_l f_l on every level l (f_l = nodal values of f) and u = g on Dirichlet DoFs,
 * following procedure FMG of Algorithm 4, then optional extra cycles.  f_nodal, g_nodal and
 * u_out are device vectors on level L.  The prolongated level solutions w_l are kept for
 * hhg_estimate.  stats may be NULL. */
hhg_status hhg_fmg_solve(hhg_ctx ctx, const double* f_nodal, const double* g_nodal, double* u_out,
                         const hhg_solve_params* params, hhg_solve_stats* stats);

/* V-cycles on level L for the system of hhg_fmg_solve, started from the iterate u_inout
 * (device, canonical order of level L; its Dirichlet values are replaced by g) instead of the
 * FMG pass: cycles of V(pre, post) until the residual norm is at most params->rtol times that
 * of the zero iterate (g on Dirichlet DoFs, 0 elsewhere), at most params->max_iter >= 1 cycles
 * (params->nu is not used).  A warm start, e.g. from hhg_transfer after a k-step.  The result
 * overwrites u_inout.  Afterwards hhg_macro_norms may use u_L; hhg_estimate, which needs the
 * FMG level solutions, returns HHG_ESTATE.  Stagnation gives HHG_ENOTCONV (u_inout still
 * holds the last iterate). */
hhg_status hhg_cycle_solve(hhg_ctx ctx, const double* f_nodal, const double* g_nodal, double* u_inout,
                           const hhg_solve_params* params, hhg_solve_stats* stats);

/* Transfer of a level-L vector between two contexts on the same domain: the solution
 * transfer from the fine level of one macro mesh to that of the next one in a kl-loop, which
 * the conclusion (Section 6) lists as missing.  u_new[i] is the P1 function with nodal values
 * u_old (device, canonical order of ctx_old's level L) evaluated at the coordinates of DoF i of
 * ctx_new's level L (device, canonical order).  Both contexts are bound on one device; the
 * work runs on ctx_new's stream and uses scratch vectors of both contexts (the state of their
 * last solves is kept); ctx_old must not be in use meanwhile.  A DoF outside every macro of
 * ctx_old gets NaN.  Triangle or tetrahedral meshes, both of the same dimension (HHG_EINVAL
 * otherwise).  Synchronises the stream. */
hhg_status hhg_transfer(hhg_ctx ctx_new, hhg_ctx ctx_old, const double* u_old, double* u_new);

/* Error estimate of procedure ErrorEstimate (Algorithm 4) from the last hhg_fmg_solve, for
 * 0 < j < L: eta_cell_host[T] = ||u_L - w_{L-1}||_{L2(T)} for every macro T (host, n_cells),
 * *eta_j = theta^j ||e~_{L-j}||, *theta_est = ||e~_{L-j}|| / ||e~_{L-j-1}||,
 * *norm_e = ||e~_{L-j}||.  Any output pointer may be NULL.  Synchronises the stream. */
hhg_status hhg_estimate(hhg_ctx ctx, int j, double* eta_cell_host, double* eta_j, double* theta_est,
                        double* norm_e);

/* hhg_estimate with a choice of norm (HHG_NORM_*) and of local indicator (HHG_LOCAL_*):
 * every norm below is the chosen one.  eta_cell_host[T] receives the chosen local indicator;
 * a scaled indicator whose ||e~_{L-j-1}||_T is zero is reported as 0.  *eta_j, *theta_est and
 * *norm_e are as for hhg_estimate (equations of the global estimate eta_j and of theta~).
 * HHG_NORM_ENERGY needs HHG_KAPPA_MACRO (HHG_EINVAL otherwise); unknown norm or indicator
 * values give HHG_EINVAL.  hhg_estimate(ctx, j, ...) equals
 * hhg_estimate_ex(ctx, j, HHG_NORM_L2, HHG_LOCAL_L1, ...).  Synchronises the stream. */
hhg_status hhg_estimate_ex(hhg_ctx ctx, int j, int norm, int local, double* eta_cell_host, double* eta_j,
                           double* theta_est, double* norm_e);

/* Per-macro squared norms on level L (norm = HHG_NORM_*; the local norms of Section 4.3):
 * sq_host[T] = ||d||_T^2 over the fine elements of macro T, T = 0..n_cells-1 (host array),
 * where, with x a device vector on level L in canonical order (NULL: u_L of the last solve),
 *   level = -1:          d = x                  (x must not be NULL),
 *   0 <= level < L:      d = x - I_{level+1}^L w_level   (w_level: the stored prolongation
 *                                                         of the FMG solution of that level),
 *   level = L:           d = x - u_L.
 * With x the nodal interpolant of an exact solution this gives the local errors of u_L
 * (level = L) or of a coarser FMG solution (level < L), the criterion of the convergence
 * studies of Section 5; with x = NULL and level = L-j it gives ||e~_{L-j}||_T.  level >= 0 or
 * x = NULL needs a preceding hhg_fmg_solve (HHG_ESTATE).  HHG_NORM_ENERGY needs
 * HHG_KAPPA_MACRO.  Leaves the state of the last solve intact.  Synchronises the stream. */
hhg_status hhg_macro_norms(hhg_ctx ctx, const double* x, int level, int norm, double* sq_host);

/* y = A x or y = M x on a level with the full (unconstrained) assembled matrix; x, y device
 * vectors in canonical order (op = HHG_OP_STIFFNESS | HHG_OP_MASS).  Leaves the state of the
 * last hhg_fmg_solve intact (hhg_estimate may still follow). */
hhg_status hhg_apply(hhg_ctx ctx, int level, int op, const double* x, double* y);

/* y = M_L x with the consistent mass matrix M_L of level L (the matrix of the L2 norm the
 * estimate is taken in, Section 4.4: entries |t|/((d+1)(d+2)) (1 + delta_ij) summed over the
 * micro elements t), full rows including Dirichlet DoFs; x, y device vectors in canonical
 * order of level L (length hhg_num_dofs(L)), owned by the caller.  HHG_EINVAL for NULL
 * vectors, HHG_ESTATE without a workspace.  Used for L2 goal functionals and norms. */
hhg_status hhg_mass_apply(hhg_ctx ctx, const double* x, double* y);

/* Smoother sweeps on one level: u (device, in/out) <- `sweeps` sweeps for A u = b with the
 * context's smoother; b (device) is the assembled right-hand side; Dirichlet DoFs are kept. */
hhg_status hhg_smooth(hhg_ctx ctx, int level, double* u, const double* b, int sweeps);

/* r_c = P^T r_f restricted from level (level) to level-1, zero on coarse Dirichlet DoFs;
 * e_f = P e_c prolongated from level-1 to level.  Device vectors in canonical order. */
hhg_status hhg_restrict(hhg_ctx ctx, int level, const double* r_fine, double* r_coarse);
hhg_status hhg_prolongate(hhg_ctx ctx, int level, const double* e_coarse, double* e_fine);

/* Gradient of J(u(f, kappa)) for the converged discrete solution: solves the adjoint system
 * A lambda = dJdu (lambda = 0 on Dirichlet DoFs) by FMG + extra cycles after recomputing u,
 * then dJdf = M_L lambda (device, level L) and dJdkappa_host[e] = -lambda^T A_e u (host,
 * n_cells; A_e = unit-coefficient stiffness of macro e).  Either output may be NULL. */
hhg_status hhg_adjoint(hhg_ctx ctx, const double* f_nodal, const double* g_nodal, const double* dJdu,
                       double* dJdf, double* dJdkappa_host, const hhg_solve_params* params);

/* Time `sweeps` smoother sweeps on level L on internal vectors (precision HHG_FP64, or
 * HHG_FP32_REFINED = float32 sweeps).  *ms: device time of all sweeps (HIP events);
 * *bytes: algorithmic bytes they move (24 B per DoF-update in float64, 12 B in float32, plus
 * 8 B for a nodal coefficient).  If launch_ms / launch_bytes are not NULL, every launch of the
 * macro-interior smoother kernel is bracketed by events: *launch_ms is its average duration
 * and *launch_bytes the algorithmic bytes of one such launch.  Outputs may be NULL. */
hhg_status hhg_bench_smoother(hhg_ctx ctx, int precision, int sweeps, double* ms, double* bytes, double* launch_ms,
                              double* launch_bytes);

/* Relative residuals ||r|| / ||r_0|| after each extra cycle of the last solve on this context
 * (host array of `capacity` doubles); *count receives the number recorded. */
hhg_status hhg_residual_history(hhg_ctx ctx, double* out, int capacity, int* count);

const char* hhg_status_string(hhg_status s);
const char* hhg_last_error(hhg_ctx ctx);
void hhg_destroy(hhg_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* HHG_H */
