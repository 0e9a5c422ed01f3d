/*
 * fbto.h -- C ABI of the MI355X matrix-free SIMP hot path.
 *
 * Method: first-order bilevel topology optimization (arXiv 2204.06204).
 * The design problem (Sec. 3, Eq. opt) is
 *     min_{x in X}  c(x) = f^T K(rho(x))^{-1} f,
 *     K(rho) = sum_e (rho_min + (1 - rho_min) rho_e^p) P_e^T KE P_e,
 *     X = { lo <= x <= hi, 1^T x <= vmax },
 * with rho = C(x) a linear density filter (Remark on modifiers, Sec. 3).
 * Alg. 1 alternates an inexact low-level refinement of u (here: a few
 * Jacobi-PCG steps) with one projected gradient step on x (Alg. 4 is the
 * projection).  The grid is a structured nx*ny*nz voxel grid of unit-cube
 * trilinear hex8 elements (the paper's regular-grid case, Sec. 4.3).
 *
 * Numbering (shared with every caller):
 *   node n = i + (nx+1)*(j + (ny+1)*k)      (0 <= i <= nx, ...)
 *   DOF 3*n + c                               (c = 0, 1, 2 for x, y, z)
 *   element e = ex + nx*(ey + ny*ez)
 *   multi-RHS vectors are [nrhs][3N], contiguous.
 *
 * Precision: `prec` selects the element type of every `void*` float array
 * of a call: double for FBTO_F64, float for FBTO_F32.  Reductions (dot
 * products, norms, sums of the projection) are always FP64, and every
 * `double*` output is FP64.
 *
 * Ownership: every data pointer is a caller-owned HIP *device* pointer
 * unless marked "host".  The library never frees or retains them beyond
 * the call.  The library owns the grid handle and its workspace (created
 * by fbto_setup_grid, released by fbto_destroy_grid).
 *
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Calls are
 * stream-ordered and asynchronous unless stated otherwise; results in
 * device memory are valid once the stream reaches them.  One grid handle
 * must not be used on two streams at once (its workspace is shared).
 *
 * Errors: each call returns FBTO_OK or an error code and never throws.
 * Argument errors are detected on the host before any launch; the message
 * is available from fbto_last_error() (thread-local).  Conditions found on
 * the device (CG breakdown, non-finite values) are reported in the FP64
 * status slot of the caller's info buffer (see fbto_inner_solve).
 */
#ifndef FBTO_H
#define FBTO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fbto_grid_s* fbto_grid_t;

typedef enum fbto_status {
  FBTO_OK = 0,
  FBTO_ERR_ARG = 1,          /* invalid argument (host check)             */
  FBTO_ERR_ALLOC = 2,        /* device allocation failed                  */
  FBTO_ERR_HIP = 3,          /* HIP runtime error                         */
  FBTO_ERR_INFEASIBLE = 4,   /* vmax < lo * E: X is empty                 */
  FBTO_ERR_BREAKDOWN = 5,    /* device: p^T K p <= 0 in CG                 */
  FBTO_ERR_NONFINITE = 6,    /* device: NaN / Inf met                     */
  FBTO_ERR_UNSUPPORTED = 7,  /* valid request the library does not handle */
  FBTO_INEXACT = 8           /* device: the volume projection used up its   */
                             /* pass budget; x is feasible (sum x <= vmax)  */
                             /* but not the exact projection               */
} fbto_status_t;

typedef enum fbto_prec { FBTO_F64 = 0, FBTO_F32 = 1 } fbto_prec_t;

/* Low-level update of Alg. 1 / 3 (Sec. 4).  PCG_JACOBI: conjugate
 * gradients preconditioned by diag(K), restarted at every call and
 * warm-started from u.  RICHARDSON: Alg. 1's u <- u - beta (K u - f).
 * DAMPED_JACOBI: u <- u - omega diag(K)^{-1} (K u - f). */
typedef enum fbto_method {
  FBTO_PCG_JACOBI = 0,
  FBTO_RICHARDSON = 1,
  FBTO_DAMPED_JACOBI = 2,
  FBTO_KRYLOV = 3
} fbto_method_t;

typedef struct fbto_grid_desc {
  int32_t nx, ny, nz;        /* elements per axis, each >= 1              */
  int32_t max_rhs;           /* right-hand sides per call, 1..4            */
  double young, poisson;     /* E > 0, -1 < nu < 0.5                       */
  double penal;              /* SIMP exponent p >= 1 (p = 3 by products;   */
                             /* other p: FP64 pow(), FP32 2^(p log2 rho)   */
                             /* from the hardware, a few ulp)              */
  double rho_min;            /* 0 <= rho_min < 1 (stiffness floor)          */
  double filter_radius;      /* cone-filter radius r in element widths;    */
                             /* r <= 1 makes the filter the identity       */
} fbto_grid_desc_t;

/* Plane grid (the paper's own 2D setting): nx * ny unit-square bilinear
 * quadrilaterals (Q4), plane stress, with the separable Gaussian density
 * filter of the paper's experiments (Sec. 5: a 7 x 7 window, filter_half =
 * 3).  1D weights g(d) = exp(-d^2 / (2 sigma^2)), |d| <= filter_half; the
 * 2D weight H_ej = g(dx) g(dy) over element centres, truncated at the grid
 * boundary and normalised by its row sum.  Numbering:
 *   node n = i + (nx+1)*j, DOF 2*n + c (c = 0, 1 for x, y),
 *   element e = ex + nx*ey, vectors [nrhs][2N]. */
typedef struct fbto_grid2d_desc {
  int32_t nx, ny;            /* elements per axis, each >= 1              */
  int32_t max_rhs;           /* right-hand sides per call, 1..4            */
  int32_t filter_half;       /* Gaussian window half-width, 0..8 (0: none) */
  double young, poisson;     /* E > 0, -1 < nu < 0.5                       */
  double penal;              /* SIMP exponent p >= 1                        */
  double rho_min;            /* 0 <= rho_min < 1 (the paper's law: 0, with  */
                             /* the box's lower bound lo > 0)               */
  double filter_sigma;       /* sigma > 0 in element widths                 */
} fbto_grid2d_desc_t;

/* Slots of the FP64 info record written by fbto_inner_solve (per RHS,
 * FBTO_SOLVE_INFO doubles each) and by fbto_outer_step. */
enum {
  FBTO_SI_RNORM2 = 0,        /* ||r||_2 of the recursive residual          */
  FBTO_SI_RNORMI = 1,        /* ||r||_inf                                  */
  FBTO_SI_FNORM2 = 2,        /* ||f||_2                                    */
  FBTO_SI_STEPS = 3,         /* steps taken                                */
  FBTO_SI_STATUS = 4,        /* 0 or an fbto_status_t value                */
  FBTO_SOLVE_INFO = 8
};
enum {
  FBTO_OI_COMPLIANCE = 0,    /* c = sum_r f_r^T u_r after the inner solve   */
  FBTO_OI_DX_INF = 1,        /* ||x_{k+1} - x_k||_inf                       */
  FBTO_OI_R_INF = 2,         /* max_r ||r_r||_inf after the inner solve     */
  FBTO_OI_LAMBDA = 3,        /* multiplier of the volume constraint         */
  FBTO_OI_VOLUME = 4,        /* sum(x_{k+1})                                */
  FBTO_OI_RREL = 5,          /* max_r ||r_r||_2 / ||f_r||_2                  */
  FBTO_OI_STATUS = 6,        /* 0 or an fbto_status_t value                 */
  FBTO_OI_GRAD_MEAN = 7,     /* mean of the filtered gradient (before the   */
                             /* mean projection)                            */
  FBTO_OUTER_INFO = 8
};

/* Create a grid handle.  Defines the operator of Sec. 3 on the voxel grid
 * of Sec. 4.3: supports and springs are fixed here, densities are passed
 * per call.
 *   fixed_dof_mask  host, [3N] bytes, nonzero = DOF fixed.  A fixed DOF gets
 *                   an identity row and column in K (y_i = u_i); callers
 *                   keep f_i = 0 and u_i = 0 there.  May be NULL (none).
 *   spring_dof/k    host, n_springs entries: K_ii += k on free DOF i
 *                   (ignored on fixed DOFs).  May be NULL if n_springs = 0.
 *   out             receives the handle.
 * Allocates device workspace (FP32 and FP64 vectors for max_rhs RHS are
 * allocated on first use of each precision).  Limits: every axis <= 65534
 * elements, fewer than 2^29 nodes, and a node plane (nx+1)(ny+1) of at most
 * 22,369,621 nodes (the K u kernels address a few planes with 32-bit byte
 * offsets).  Errors: FBTO_ERR_ARG, FBTO_ERR_UNSUPPORTED (plane too large),
 * FBTO_ERR_ALLOC, FBTO_ERR_HIP. */
fbto_status_t fbto_setup_grid(const fbto_grid_desc_t* desc,
                              const uint8_t* fixed_dof_mask,
                              int32_t n_springs, const int64_t* spring_dof,
                              const double* spring_k, fbto_grid_t* out);

/* Create a plane-grid handle (fbto_grid2d_desc_t).  The handle serves the
 * same calls as a voxel grid's -- fbto_apply_K, fbto_inner_solve (every
 * method), fbto_solve_refined, fbto_sensitivity, fbto_filter, the
 * projections and the three outer steps -- on [nrhs][2N] vectors; the CG
 * steps run unfused in both precisions.
 *   fixed_dof_mask  host, [2N] bytes, nonzero = DOF fixed (identity row and
 *                   column, as on voxel grids).  May be NULL.  Plane grids
 *                   take no springs.
 * Errors: FBTO_ERR_ARG, FBTO_ERR_ALLOC, FBTO_ERR_HIP. */
fbto_status_t fbto_setup_grid_2d(const fbto_grid2d_desc_t* desc, const uint8_t* fixed_dof_mask,
                                 fbto_grid_t* out);

/* Release the handle and its workspace (synchronises the device). */
fbto_status_t fbto_destroy_grid(fbto_grid_t g);

/* Sizes of a grid: elements, nodes, DOFs (host pointers, any may be NULL). */
fbto_status_t fbto_grid_sizes(fbto_grid_t g, int64_t* n_elem, int64_t* n_node,
                              int64_t* n_dof);

/* y = K(rho_phys) u for nrhs vectors (Sec. 3, K(v) = sum_e A_e K_e; the
 * regular-grid matrix-free product of Sec. 4.3).  rho_phys: [E] physical
 * (filtered) densities; u, y: [nrhs][3N]; 1 <= nrhs <= max_rhs.  u and y
 * must not overlap.  Fixed DOFs: y_i = u_i; free rows ignore u at fixed
 * DOFs. */
fbto_status_t fbto_apply_K(fbto_grid_t g, fbto_prec_t prec, const void* rho_phys,
                           const void* u, void* y, int32_t nrhs, void* stream);

/* Low-level refinement of u towards K(rho_phys) u = f (Alg. 1 / 3 low-level
 * line), `steps` steps of `method` from the warm start in u, per RHS.
 * PCG_JACOBI runs the textbook preconditioned CG recurrence rearranged as in
 * Chronopoulos and Gear (one reduction phase per step; same iterates in
 * exact arithmetic).
 * KRYLOV is ONE low-level step of Alg. 3 with the Krylov preconditioner of
 * Eq. LSP (Sec. 4.1), of degree D = `steps` (0 .. 1000):
 *   u <- u - omega M^-1 (K u - f),  M^-1 b = sum_{i<=D} c_i K^i b,
 *   c = argmin || b - sum_{i=1}^{D+1} c_{i-1} K^i b ||,
 * computed by the MINRES recurrence (D + 1 products; the same minimiser as
 * the paper's QR of the monomial basis, by a stable route).  The RHS are
 * processed one after another.
 *   omega   step of RICHARDSON (beta), DAMPED_JACOBI (omega) or KRYLOV
 *           (Alg. 3's beta_k; 1 is the paper's choice); unused by PCG.
 *   rtol    0: run exactly `steps` steps, asynchronously.  rtol > 0 (PCG
 *           only): stop once ||r||_2 <= rtol ||f||_2 or after `steps`
 *           steps; this mode synchronises the stream every 64 steps.
 *   info    device, FP64 [nrhs][FBTO_SOLVE_INFO], may be NULL.
 * Device-detected breakdown/non-finite values go to FBTO_SI_STATUS. */
fbto_status_t fbto_inner_solve(fbto_grid_t g, fbto_prec_t prec, const void* rho_phys,
                               const void* f, void* u, int32_t nrhs,
                               fbto_method_t method, int32_t steps, double omega,
                               double rtol, double* info, void* stream);

/* Mixed-precision solve with FP64 iterative refinement:
 *   repeat: r = f - K64 u (FP64 operator);  stop if ||r||_2 <= rtol ||f||_2;
 *           d = PCG in `inner_prec` on K d = r from d = 0, at most
 *               `inner_steps` steps, stopping once its own residual has
 *               dropped by inner_rtol (0: always inner_steps steps);  u += d
 * rho_phys, f, u are FP64 ([E], [nrhs][3N], [nrhs][3N]).  Synchronises the
 * stream after each refinement step.  info: device FP64
 * [nrhs][FBTO_SOLVE_INFO] (STEPS counts inner steps), may be NULL.
 * *refinements (host, may be NULL) receives the number of refinements. */
fbto_status_t fbto_solve_refined(fbto_grid_t g, fbto_prec_t inner_prec,
                                 const double* rho_phys, const double* f, double* u,
                                 int32_t nrhs, double rtol, int32_t max_refine,
                                 int32_t inner_steps, double inner_rtol, double* info,
                                 int32_t* refinements, void* stream);

/* Sensitivity of Sec. 3 / Alg. 1, summed over the nrhs load cases:
 *   dobj[e] = -ds_e sum_r lam_{r,e}^T KE u_{r,e},
 *   ds_e = p (1 - rho_min) rho_e^(p-1),
 * with lam = u when lam == NULL (then dobj = dc/drho for c = sum_r f_r.u_r).
 * For a linear objective L = t^T u pass the adjoint lam = K^{-1} t.
 * Element strains are recomputed from the nodal vectors (nothing stored).
 *   rho_phys [E]; u, lam, f [nrhs][3N]; dobj [E].
 *   f, obj  if both non-NULL, obj (device FP64 scalar) receives
 *           sum_r f_r . u_r (the compliance). */
fbto_status_t fbto_sensitivity(fbto_grid_t g, fbto_prec_t prec, const void* rho_phys,
                               const void* u, const void* lam, const void* f,
                               int32_t nrhs, void* dobj, double* obj, void* stream);

/* Linear cone filter (Remark on modifiers, Sec. 3):
 *   transpose = 0:  out = (H in) / Hs          (x -> rho)
 *   transpose = 1:  out = H^T (in / Hs)        (d/drho -> d/dx)
 * H_ej = max(0, r - |c_e - c_j|), Hs_e = sum_j H_ej, boundary-truncated.
 * in, out: [E], must not overlap. */
fbto_status_t fbto_filter(fbto_grid_t g, fbto_prec_t prec, int32_t transpose,
                          const void* in, void* out, void* stream);

/* Euclidean projection onto X = {lo <= x <= hi, sum x <= vmax} (Sec. 4.2,
 * Eq. piecewiseLinearEQ; Alg. 4 computes the same point by sorting).
 * x = clamp(y - lambda, lo, hi) with lambda = 0 if clamp(y) is feasible,
 * else the root of sum clamp(y - lambda, lo, hi) = vmax found on the device
 * in FP64 by passes over y: each pass evaluates the sum and the linear
 * piece on either side of the current lambda; the next pass solves that
 * piece exactly, which ends the search when the root lies on it, and
 * otherwise takes a Newton step safeguarded by bisection of the bracket.
 *   max_passes  pass budget, 1 .. 64; 0 selects 8.  Each pass is one launch
 *               that streams y once; passes after the search has ended
 *               return at once.  Seeded U[0.2, 0.4] densities after a
 *               gradient step need 3-4 passes; values spread over many
 *               decades (lognormal, Pareto), or spread far wider than
 *               hi - lo, can need 20-45.
 *   lambda      device FP64 scalar, may be NULL: the multiplier.
 *   status      device FP64 scalar, may be NULL: 0; FBTO_INEXACT when the
 *               budget ran out before the root's piece was found (x is then
 *               clamp(y - b, lo, hi) for the feasible end b of the last
 *               bracket: sum x <= vmax, but not the projection;
 *               fbto_project_volume_sorted is exact for any input); or
 *               FBTO_ERR_NONFINITE for non-finite y.
 * y, x: [E] (may alias).  Asynchronous (no host synchronisation).
 * Errors: FBTO_ERR_INFEASIBLE if vmax < lo * E; FBTO_ERR_ARG for a budget
 * outside 0 .. 64. */
fbto_status_t fbto_project_volume(fbto_grid_t g, fbto_prec_t prec, const void* y,
                                  void* x, double lo, double hi, double vmax,
                                  int32_t max_passes, double* lambda, double* status,
                                  void* stream);

/* The same projection computed the way Alg. 4 does it, in its GPU form
 * (Sec. 4.3: a radix sort and parallel scans), as a cross-check of
 * fbto_project_volume:
 *   - y is sorted once (LSD radix sort, 8-bit digits: 4 passes in FP32, 8 in
 *     FP64).  The nodes y_e - lo and y_e - hi of Eq. piecewiseLinearEQ are
 *     this order shifted by a constant.
 *   - FP64 prefix sums of the sorted values give the sum of
 *     clamp(y - t, lo, hi) at any t in closed form (the running RHS of
 *     Alg. 4).  It is evaluated at all 2E nodes in parallel.
 *   - The nodes on either side of vmax bound one linear piece, and lambda
 *     solves it.  lambda = 0 when clamp(y, lo, hi) is feasible.
 * Arguments, aliasing, lambda and the errors are those of
 * fbto_project_volume.  Where the root is not unique (a flat piece at
 * vmax), x is the same for every root; lambda may differ.
 * A non-finite y gives lambda = NaN and x = NaN.
 * The first call on a grid allocates the workspace: 24 bytes per element
 * (two key buffers and the prefix sums) + 1 KiB of digit counts per 2048
 * elements.  Errors: as
 * fbto_project_volume; FBTO_ERR_ARG if E >= 2^31. */
fbto_status_t fbto_project_volume_sorted(fbto_grid_t g, fbto_prec_t prec, const void* y,
                                         void* x, double lo, double hi, double vmax,
                                         double* lambda, void* stream);

/* One outer iteration k (1-based) of the first-order bilevel method
 * (Alg. 1 with the Jacobi-PCG low-level step):
 *   rho = C(x); u <- inner_steps PCG steps on K(rho) u = f from u;
 *   g = C^T(dc/drho); g <- g - mean(g) if mean_project (Sec. 4.2);
 *   x <- Proj_X(x - alpha_k g / 2),  alpha_k = alpha0 k^(-3/4) (Sec. 5).
 * x: [E] in/out, u: [nrhs][3N] in/out, f: [nrhs][3N].  hi = 1.
 * info: device FP64 [FBTO_OUTER_INFO] (may be NULL). */
fbto_status_t fbto_outer_step(fbto_grid_t g, fbto_prec_t prec, void* x, void* u,
                              const void* f, int32_t nrhs, int32_t k, double alpha0,
                              int32_t inner_steps, int32_t mean_project, double lo,
                              double vmax, double* info, void* stream);

/* Outer iterations k .. k + n_steps - 1 of Alg. 1 in one call: the same
 * results as n_steps calls of fbto_outer_step, bitwise.  Since x changes
 * only inside the call, the final projection pass of an iteration also
 * filters the new x for the next one (voxel grids with a filter radius of at
 * most 2), one pass over the elements fewer per iteration.
 * info: device FP64 [n_steps][FBTO_OUTER_INFO], one record per iteration
 * (may be NULL).  Errors: as fbto_outer_step; FBTO_ERR_ARG if n_steps < 1;
 * an error stops the call after the iteration it occurred in. */
fbto_status_t fbto_outer_steps(fbto_grid_t g, fbto_prec_t prec, void* x, void* u,
                               const void* f, int32_t nrhs, int32_t k, int32_t n_steps,
                               double alpha0, int32_t inner_steps, int32_t mean_project,
                               double lo, double vmax, double* info, void* stream);

/* One step of projected gradient descent with an exact low-level solve,
 * the baseline the paper compares against (Sec. 5): as fbto_outer_step,
 * but u is refined by Jacobi-PCG until ||f - K u||_2 <= rtol ||f||_2 (or
 * max_steps steps), so the gradient is that of the true objective and
 * info's compliance is the true objective f^T K^-1 f (to rtol).  The
 * stream is synchronised every 64 PCG steps.  rtol: (0, 1). */
fbto_status_t fbto_outer_step_exact(fbto_grid_t g, fbto_prec_t prec, void* x, void* u,
                                    const void* f, int32_t nrhs, int32_t k, double alpha0,
                                    double rtol, int32_t max_steps, int32_t mean_project,
                                    double lo, double vmax, double* info, void* stream);

/* One outer iteration k of Alg. 3 (CPFBTO): as fbto_outer_step, with the
 * low-level update replaced by one step with the Krylov preconditioner of
 * degree `degree` (Eq. LSP, fbto_inner_solve's FBTO_KRYLOV):
 *   u <- u - beta M^-1 (K(rho) u - f),  beta > 0 (the paper uses 1).
 * info's R_INF is the true residual after that step.  degree: 0 .. 1000. */
fbto_status_t fbto_outer_step_krylov(fbto_grid_t g, fbto_prec_t prec, void* x, void* u,
                                     const void* f, int32_t nrhs, int32_t k, double alpha0,
                                     int32_t degree, double beta, int32_t mean_project,
                                     double lo, double vmax, double* info, void* stream);

/* Optimality metrics of a design, the error measures of Thm. 1 (Sec. 4)
 * that Sec. 5 plots along a run:
 *   l(x)    = 1/2 sum_r f_r^T K(rho(x))^-1 f_r        the true objective
 *   Delta^v = |Proj_X(x - alpha grad l(x)) - x|^2 / alpha^2   high-level error
 *   Delta   = sum_r |u_r - K^-1 f_r|^2                  low-level (tracking) error
 * K^-1 f is computed by Jacobi-PCG in `prec` to ||f - K u*|| <= rtol ||f||
 * (at most max_steps steps, warm-started from u) into library workspace;
 * x and u are not modified.  grad l = 1/2 C^T(-ds_e u*_e^T KE u*_e) (the
 * exact gradient; no mean projection).  The projection is the one of
 * fbto_project_volume (hi = 1), run cold with its own search state, so the
 * warm start of the outer steps is kept.  alpha: the step size at which
 * Delta^v is measured (the paper's alpha_k), > 0.
 *   out  device FP64 [5]: l, Delta^v, Delta, max_r ||f_r - K u*_r|| / ||f_r||,
 *        status (0, FBTO_ERR_BREAKDOWN / _NONFINITE of the solve, or the
 *        projection's FBTO_INEXACT).
 * Synchronises the stream every 64 PCG steps.  The first call allocates the
 * workspace (max_rhs x N DOF values).  Errors: FBTO_ERR_ARG,
 * FBTO_ERR_INFEASIBLE, FBTO_ERR_ALLOC, FBTO_ERR_HIP. */
fbto_status_t fbto_optimality(fbto_grid_t g, fbto_prec_t prec, const void* x, const void* u,
                              const void* f, int32_t nrhs, double alpha, double lo, double vmax,
                              double rtol, int32_t max_steps, double* out, void* stream);

/* The projection of fbto_project_volume for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  No grid handle: n_elem is the length
 * of y and x.  It calls no hipMalloc, hipFree or allocating routine.
 * Its workspace -- the per-block FP64 partials of the passes and the search
 * state, 222,016 bytes -- is a static device array that each GPU the
 * library runs on holds until the process ends; the first call on a device
 * looks up its address there.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, or two threads) race
 * and give wrong results; calls ordered on one stream do not interfere.
 * Each call starts cold (no warm start from an earlier multiplier), so the
 * result equals fbto_project_volume's for the same y, bit for bit.
 *   n_elem  1 .. FBTO_NOALLOC_MAX_ELEMS; larger values are rejected with
 *           FBTO_ERR_ARG.
 * y, x, lo, hi, vmax, max_passes, lambda, status, stream, the errors and
 * the asynchrony are those of fbto_project_volume. */
#define FBTO_NOALLOC_MAX_ELEMS 2147483647LL
fbto_status_t fbto_project_volume_noalloc(fbto_prec_t prec, int64_t n_elem, const void* y,
                                          void* x, double lo, double hi, double vmax,
                                          int32_t max_passes, double* lambda, double* status,
                                          void* stream);

/* Tuning options of a grid handle (fbto_set_option).  They change how the
 * work is laid out or how long a search may run, not what is computed.
 *   FBTO_OPT_PROJ_PASSES  pass budget of the volume projection inside
 *                         fbto_outer_step / _krylov / _exact, 1 .. 64
 *                         (default 2).  These projections start from the
 *                         previous multiplier: the gradient-step kernel
 *                         already evaluates the volume there, and one pass
 *                         sufficed on every iteration of the workloads
 *                         measured; FBTO_INEXACT in the info record's
 *                         status says the budget ran out.
 *   FBTO_OPT_APPLY_TILE   tile of the z-marching K(rho)u kernels (apply,
 *   FBTO_OPT_CGF_TILE     residual and CG products; the fused CG step):
 *                         bx | by << 8 | dz << 16 | cap << 24 (element
 *                         columns per tile row and column, 8 <= bx <= 64,
 *                         4 <= by <= 64; the fused CG step has a thread
 *                         per node column: 128 <= (bx + 1) (by + 1) <= 256;
 *                         FBTO_OPT_APPLY_TILE also sets kernels with a
 *                         thread per element column: bx by >= 128 and
 *                         (bx + 1) (by + 1) <= 256; slab depth
 *                         dz 1 .. 64; a zero field is chosen by the cost
 *                         model; cap 2 .. 15 limits the blocks resident on
 *                         a CU by the LDS each block requests, 0 leaves
 *                         them to the registers and LDS the kernel needs),
 *                         or 0 for the built-in choice.  A shape the kernel
 *                         cannot run makes the next launch fail
 *                         (FBTO_ERR_HIP).
 * Errors: FBTO_ERR_ARG for an unknown option or a value out of range. */
typedef enum fbto_option {
  FBTO_OPT_PROJ_PASSES = 0,
  FBTO_OPT_APPLY_TILE = 1,
  FBTO_OPT_CGF_TILE = 2
} fbto_option_t;
fbto_status_t fbto_set_option(fbto_grid_t g, fbto_option_t option, int64_t value);

/* Message of the last error on this thread ("" if none). */
const char* fbto_last_error(void);

/* Library version string. */
const char* fbto_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FBTO_H */
