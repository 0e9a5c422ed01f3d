// Internal declarations shared by the kernels (kernels.hip) and the C ABI
// layer (api.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fbto.h"

namespace fbto {

// Grid geometry, passed to every kernel by value.
struct Geo {
  int nx, ny, nz;      // elements per axis
  int nxn, nyn, nzn;   // nodes per axis (n + 1)
  int64_t N, E;        // nodes, elements
  int64_t ndof;        // 3N
  double rnx, rny, rnxn, rnyn;  // reciprocals for 32-bit index division
};

// Element stiffness in the sum/difference ("modal") basis.  Per axis the
// two nodal values (u0, u1) map to (u0 + u1, u1 - u0); on the unit cube the
// 24x24 KE becomes a 45-entry sparse matrix:
//   diagonal  dg[q_i][number of the other two bits of q that are set]
//             (component i, mode q; by the cube's symmetry six values)
//   coupling  component i, mode q  <-  component j, mode q ^ (1<<i) ^ (1<<j)
//             whenever bits i and j of q differ, with weight
//             lam4[bit k of q] if bit i of q is set, else mu4[bit k of q]
// (k the third axis).  Mode q has bit b set when it is the difference mode
// along axis b.  Derived from the 1D integrals of the basis {1/2, t - 1/2}.
template <typename T>
struct Modal {
  T dg[2][3];
  T lam4[2];
  T mu4[2];
};

// Element stiffness of the unit-square Q4 (plane stress), local DOF 2a + c.
template <typename T>
struct Q4 {
  T k[8][8];
};

// 1D weights of the separable Gaussian filter of a plane grid: w[d + half]
// for d = -half .. half.
constexpr int kGaussMaxHalf = 8;
template <typename T>
struct GaussW {
  T w[2 * kGaussMaxHalf + 1];
  int half;
};

struct Simp {
  double penal;
  double rho_min;
  int cubic;           // penal == 3 exactly: rho^3 by multiplication
};

// Device-resident scalars of one grid handle (FP64).  Indexed per RHS
// where marked [4].
struct Scalars {
  double rz[4];        // r . z of the current CG iterate
  double pq[4];
  double alpha[4];
  double beta[4];
  double rnorm2[4];    // ||r||_2
  double rinf[4];      // ||r||_inf
  double fnorm2[4];
  double tol[4];       // convergence threshold on ||r||_2 (0: none)
  double steps[4];
  double done[4];      // 1 once converged
  double status[4];    // fbto_status_t of the RHS
  double dot[4];       // scratch dot results
  double cg_gamma[2][4];  // r.z of the previous CG step (by step parity)
  double cg_alpha[2][4];  // alpha of the previous CG step
  // projection search state, double-buffered across passes: pass t reads
  // ps[t & 1] and writes ps[(t + 1) & 1] = {lambda, a, b, done}, where the
  // bracket satisfies f(a) > vmax >= f(b)
  double ps[2][4];
  double lam;          // multiplier of the last projection
  double lam_prev;     // warm start of the next projection
  double proj_status;
  double sum0;         // sum clamp(y)
  double ymax, ymin;
  double gsum;         // sum of the filtered gradient
  double gmean;
  double work[8];
  // Krylov step (MINRES recurrence), carried from one vector pass to the
  // next: beta (||current Lanczos vector||), alpha of the last iteration,
  // and the Givens state dbar, epsln, phibar, cs, sn.  Pass t writes
  // kr[t & 1] while its blocks read kr[(t + 1) & 1].
  double kr[2][8];
};

// Per-block FP64 partial results.  A producing kernel writes one value per
// block (and per RHS); the consuming kernel reduces them in a fixed order in
// every block (no atomics, no inter-block fences, bitwise reproducible).
enum PartSlot {
  // CG-mode apply of step k (and the fused step that produces step k's
  // apply) writes the set of parity k & 1: r.z, w.z, r.r, max|r|
  P_RZ0, P_RZ1,
  P_PQ0, P_PQ1,
  P_RN0, P_RN1,
  P_RI0, P_RI1,
  P_RNF, P_RIF,        // final residual norms (residual apply, last CG vector step)
  P_FN,                // ||f||_2^2
  P_DOT,               // sum_r f_r . u_r
  P_GSUM,              // sum of the filtered gradient
  P_S0, P_YMAX, P_NACT,  // projection seed: sum clamp(y), max y, #interior
  P_E0,                // projection pass: two sets of 11 slots, P_E0 + 11 q .. P_E0 + 11 q + 10;
                       // pass t reads set t & 1 (written by pass t - 1) and writes set (t + 1) & 1
  P_VOL = P_E0 + 22,   // sum x_new
  P_DX,                // max |x_new - x_old|
  P_KRN0, P_KRN1,      // Krylov step: ||y||^2 of the new Lanczos vector, by iteration parity
  P_MET0, P_MET1,      // optimality metrics: squared distances (low-level, high-level)
  P_COUNT
};
constexpr int kMaxVecBlocks = 1024;
constexpr int kProjMaxPasses = 64;   // pass budget limit of the volume projection

// Workspace vectors of one precision.  The CG vectors come in two sets:
// the fused CG step reads one and writes the other (x of the second set is
// `x1`; the caller's vector is x of the first).
struct Vecs {
  void* r[2] = {nullptr, nullptr};   // [max_rhs][3N] residual
  void* p[2] = {nullptr, nullptr};   // search direction
  void* s[2] = {nullptr, nullptr};   // s = K p (by recurrence)
  void* w[2] = {nullptr, nullptr};   // w = K z
  void* x1 = nullptr;                // iterate, second set
  void* q = nullptr;                 // z = D^-1 r (unfused steps)
  void* invD = nullptr;   // [3N]
  void* rho = nullptr;    // [E]  filtered density
  void* ge = nullptr;     // [E]  element gradient
  void* gx = nullptr;     // [E]  design gradient
  void* y = nullptr;      // [E]  step / projection input
  void* Hs = nullptr;     // [E]  inverse filter normalisation 1 / Hs
  bool ready = false;
};

// One set of CG vectors (pointers into Vecs or the caller's x).
template <typename T>
struct CgSet {
  T* x;
  T* r;
  T* p;
  T* s;
  T* w;
};

// Tile shape and slab depth of one apply variant (chosen once per grid).
struct TileChoice {
  int bx, by, dz, tiles_x, tiles_y, slabs, nblocks;
  int cap;  // resident blocks per CU at most (0: as the registers and LDS allow)
};

constexpr size_t kApplyMaxLds = 64 * 1024;  // LDS of one z-march block at most

// LDS a block requests so that at most `cap` blocks fit on a CU with
// lds_per_cu bytes (allocation granule 512 bytes).
constexpr int lds_for_block_cap(int lds_per_cu, int cap) { return (lds_per_cu / (cap + 1) / 512 + 1) * 512; }

struct StencilPt {
  int dx, dy, dz;
  double w;
};

}  // namespace fbto

namespace fbto {
constexpr int kSortBracketBlocks = 2048;
// Workspace of the sort-based projection (one allocation, carved by
// sort_ws_layout; allocated on the first call).
struct SortWs {
  void* base = nullptr;
  void* keys[2] = {nullptr, nullptr};  // [E] sort keys, 8 bytes per entry (FP32 keys use 4)
  double* S = nullptr;                 // [E + 1] exclusive prefix sums of the sorted values
  uint32_t* hist = nullptr;            // [256][tiles] digit counts per tile, then their offsets
  uint32_t* tot = nullptr;             // [256] digit totals
  double* part = nullptr;              // [tiles] tile sums of the prefix scan, then their offsets
  double* brk = nullptr;               // [2][kSortBracketBlocks] per-block bracket of the root
  double* lam = nullptr;               // the multiplier
};
}  // namespace fbto

struct fbto_grid_s {
  fbto_grid_desc_t desc;
  int dim = 3;               // 3: hex8 voxels; 2: Q4 plane grid (nz = 1 in geo, 2 DOFs per node)
  fbto::Q4<double> q4_64;    // plane grids: element stiffness and filter weights
  fbto::Q4<float> q4_32;
  fbto::GaussW<double> gauss64;
  fbto::GaussW<float> gauss32;
  fbto::Geo geo;
  fbto::Modal<double> km64;
  fbto::Modal<float> km32;
  fbto::Simp simp;
  double ke_diag;            // every diagonal entry of KE: (lambda + 4 mu) / 9
  uint8_t* mask = nullptr;   // [N] bit c < 3: DOF c of the node fixed; bit 3: a spring at the node
  int n_springs = 0;
  int64_t* spring_dof = nullptr;
  double* spring_k64 = nullptr;
  float* spring_k32 = nullptr;
  int n_stencil = 0;
  int* stencil_off = nullptr;      // [n_stencil][3]
  double* stencil_w64 = nullptr;
  float* stencil_w32 = nullptr;
  fbto::Scalars* sc = nullptr;     // device
  double* partials = nullptr;      // device [P_COUNT][4][max_partials]
  int max_partials = 0;
  fbto::Vecs v64, v32;
  int device = 0;
  int n_cu = 256;
  int lds_per_cu = 160 * 1024;
  int n_gsum = 0;                        // blocks of the last filter launch that left a sum
  fbto::TileChoice tiles[2][2][6] = {};  // apply tiling by [FP64][NR - 1][mode], chosen on first use
  int tile_override[2] = {0, 0};         // FBTO_OPT_APPLY_TILE, FBTO_OPT_CGF_TILE (0: cost model)
  int proj_passes_warm = 2;              // FBTO_OPT_PROJ_PASSES: projection passes of the outer steps
  fbto::SortWs sort;                     // sort-based projection
};

namespace fbto {

// ---- launchers (kernels.hip) ----------------------------------------------
// All return hipSuccess or the launch error; none synchronises.  Kernels that
// leave per-block partials report how many blocks wrote them (nb_out), which
// the consumer is told.
int vec_blocks(int64_t n);
int apply_max_blocks(const Geo& G, int n_cu);
template <typename T>
hipError_t launch_apply(fbto_grid_s* g, const T* rho, const T* u, T* y, int nrhs, hipStream_t st);
template <typename T>
hipError_t launch_resid(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, const T* invD,
                        T* z, int nrhs, hipStream_t st, int* nb_out);
// Residual apply that also forms the Jacobi diagonal (stored to invD_out)
// from the densities it reads, instead of a separate diagonal kernel.
template <typename T>
hipError_t launch_resid_diag(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, T* invD_out, T* z,
                             int nrhs, hipStream_t st, int* nb_out);
template <typename T>
hipError_t launch_apply_cg(fbto_grid_s* g, const T* rho, const T* z, const T* r, T* w, int nrhs, int step,
                           hipStream_t st, int* nb_out);
// One fused CG step k (FP32 only): vector update of step k from `in`, stored
// into `out`, and out.w = K z of step k + 1 with its partials.
template <typename T>
hipError_t launch_cg_fused(fbto_grid_s* g, const T* rho, const CgSet<T>& in, const CgSet<T>& out,
                           const T* invD, int nrhs, int step, int n_apply, int n_fn, double rtol,
                           hipStream_t st, int* nb_out);
template <typename T>
hipError_t launch_diag(fbto_grid_s* g, const T* rho, T* invD, hipStream_t st);
// The last CG step k (one RHS) fused with the sensitivity: x = x_in + alpha p
// into `x`, final residual norms and f . x into the partial slots, and
// dobj_e = -ds_e x_e^T KE x_e (times Hsi_e when given).
template <typename T>
hipError_t launch_cg_sens(fbto_grid_s* g, const T* rho, const CgSet<T>& in, T* x, const T* invD, const T* f,
                          T* dobj, const T* Hsi, int step, int n_apply, int n_fn, double rtol, hipStream_t st,
                          int* nb_out);
// Vector update of CG step k: x = x_in + alpha p, r, p, s in place; z from
// z_in or D^-1 r; z_out optional (the next unfused product's input).
template <typename T>
hipError_t launch_cg_step(fbto_grid_s* g, const T* x_in, T* x, T* r, const T* z_in, T* z_out, const T* w,
                          T* p, T* s, const T* invD, const T* f, int nrhs, int n_apply, int n_fn,
                          int step, double rtol, hipStream_t st, int* nb_out);
hipError_t launch_pcg_finish(fbto_grid_s* g, int nrhs, int n_r, int n_fn, double* info, int n_dot,
                             int n_e, int n_gsum, hipStream_t st);
template <typename T>
hipError_t launch_relax_update(fbto_grid_s* g, T* u, const T* r, const T* invD, int nrhs,
                               double omega, int use_diag, hipStream_t st);
template <typename T>
hipError_t launch_sens(fbto_grid_s* g, const T* rho, const T* u, const T* lam, int nrhs,
                       T* dobj, const T* Hsi, hipStream_t st);
template <typename T>
hipError_t launch_dot(fbto_grid_s* g, const T* a, const T* b, int nrhs, hipStream_t st);
hipError_t launch_dot_store(fbto_grid_s* g, double* out, hipStream_t st);
template <typename T>
hipError_t launch_filter(fbto_grid_s* g, int kind, const T* in, T* out, int want_sum,
                         hipStream_t st);
template <typename T>
hipError_t launch_step(fbto_grid_s* g, const T* x, const T* gx, T* y, double half_alpha,
                       int mean_project, double lo, double hi, hipStream_t st);
// The plain-sum filter of the element gradient ge fused with the design
// step y = x - half_alpha (H ge - mean), leaving the projection's seed
// partials (their count in *nb_seed).  The mean comes from nb_sum partials
// in slot GSUM.  hipErrorNotSupported where the filter is not a z-march
// (plane grids, stencils wider than 3): the caller then filters and steps
// apart.
template <typename T>
hipError_t launch_filter_step(fbto_grid_s* g, const T* ge, const T* x, T* y, double half_alpha,
                              int mean_project, int nb_sum, double lo, double hi, hipStream_t st,
                              int* nb_seed);
template <typename T>
hipError_t launch_hs(fbto_grid_s* g, T* Hs, hipStream_t st);
// Sort-based projection (project_sort.hip).  sort_ws_layout returns the
// workspace bytes for E elements and, when W->base is set, points W's arrays
// into it.
size_t sort_ws_layout(int64_t E, SortWs* W);
template <typename T>
hipError_t launch_project_sorted(fbto_grid_s* g, const T* y, T* x, double lo, double hi, double vmax,
                                 double* lam_out, hipStream_t st);
// Workspace of the volume projection: kProjSlots arrays of maxp per-block
// FP64 partials (array i at base + i * stride) and the search state in a
// Scalars record.  On a grid handle the arrays are the partial slots
// P_S0 .. P_DX (stride 4 maxp); a caller-free workspace packs them.
enum ProjSlot {
  L_S0, L_YMAX, L_NACT,   // seed: sum clamp(y), max y, #interior
  L_E0,                   // evaluation sets: L_E0 + 11 q .. L_E0 + 11 q + 10, q = 0, 1
  L_VOL = L_E0 + 22,      // sum x_new
  L_DX,                   // max |x_new - x_old|
  kProjSlots
};
static_assert(P_YMAX == P_S0 + L_YMAX && P_NACT == P_S0 + L_NACT && P_E0 == P_S0 + L_E0 &&
                  P_VOL == P_S0 + L_VOL && P_DX == P_S0 + L_DX,
              "the projection's slots are consecutive grid partial slots");
struct ProjWs {
  double* base;
  int64_t stride;
  int maxp;
  Scalars* sc;
};
// Projection of y onto {lo <= x <= hi, sum x <= vmax} with `passes` search
// passes.  seeded: the seed partials (P_S0, P_YMAX, P_NACT and evaluation
// set 0) were left by the step, nb_seed of each (0: as many as the passes
// write), and the search starts from the multiplier of the previous
// projection; otherwise the seed pass runs and the search starts cold.
// lam_out, status_out: device FP64 scalars, may be NULL.
// skip_final: launch the search passes only (the caller runs the final
// pass, fused with the next forward filter: launch_proj_final_filter).
template <typename T>
hipError_t launch_project(const ProjWs& W, int64_t E, const T* y, T* x, double lo, double hi, double vmax,
                          int seeded, int passes, const T* x_old, double* lam_out, double* status_out,
                          hipStream_t st, int nb_seed = 0, int skip_final = 0);
bool zmarch_filter(const fbto_grid_s* g);
// The final pass (x updated in place, x_old = x) fused with the forward
// filter of the new design into rho, after launch_project(.., skip_final),
// where zmarch_filter(g) holds (else hipErrorNotSupported).  *nb_final: the
// count of the volume partials (slots VOL, DX).
template <typename T>
hipError_t launch_proj_final_filter(fbto_grid_s* g, const ProjWs& W, const T* y, T* x, T* rho, double lo,
                                    double hi, double vmax, int passes, hipStream_t st, int* nb_final);
template <typename T>
hipError_t launch_convert(const void* in, void* out, int64_t n, int to_double, hipStream_t st);
hipError_t launch_axpy64(double* u, const double* d, int64_t n, hipStream_t st);
hipError_t launch_ir_scale(fbto_grid_s* g, const double* r64, float* r32, int nrhs,
                           hipStream_t st);
hipError_t launch_ir_accum(fbto_grid_s* g, double* u64, const float* d32, int nrhs,
                           hipStream_t st);
hipError_t launch_solve_info(fbto_grid_s* g, double* info, int nrhs, double steps_override,
                             hipStream_t st);
// Partials of sum_i (a_i - b_i)^2 over n entries into slot `slot`; returns the block count.
template <typename T>
hipError_t launch_sqdist(fbto_grid_s* g, const T* a, const T* b, int64_t n, int slot, hipStream_t st, int* nb_out);
// Optimality record out[0..4] = l, Delta^v, Delta, max_r ||r_r|| / ||f_r||, status from the
// partials of f . u* (DOT), the two squared distances (MET0: low-level, MET1:
// high-level, the latter divided by alpha^2) and the solve's and projection's states.
hipError_t launch_opt_finish(fbto_grid_s* g, int nrhs, int nb_dot, int nb_lo, int nb_hi, double alpha,
                             const Scalars* sc_proj, double* out, hipStream_t st);

// ---- plane grids (plane.hip); the launchers above dispatch to these ----
template <typename T>
hipError_t plane_apply(fbto_grid_s* g, const T* rho, const T* u, T* y, int nrhs, hipStream_t st);
template <typename T>
hipError_t plane_resid(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, const T* invD, T* invD_out,
                       T* z, int nrhs, hipStream_t st, int* nb_out);
template <typename T>
hipError_t plane_apply_cg(fbto_grid_s* g, const T* rho, const T* z, const T* r, T* w, int nrhs, int step,
                          hipStream_t st, int* nb_out);
template <typename T>
hipError_t plane_diag(fbto_grid_s* g, const T* rho, T* invD, hipStream_t st);
template <typename T>
hipError_t plane_sens(fbto_grid_s* g, const T* rho, const T* u, const T* lam, int nrhs, T* dobj, const T* Hsi,
                      hipStream_t st);
template <typename T>
hipError_t plane_filter(fbto_grid_s* g, int kind, const T* in, T* out, T* tmp, const T* Hsi, int want_sum,
                        hipStream_t st);
template <typename T>
hipError_t plane_hs(fbto_grid_s* g, T* Hsi, hipStream_t st);
// One vector pass of the Krylov step (MINRES recurrence), iteration `itn`
// of 0 .. last (see k_minres); returns the block count of its partials.
template <typename T>
hipError_t launch_minres(fbto_grid_s* g, int itn, int last, const T* Y, T* R1, const T* R2, T* W2, const T* W,
                         T* x, int n_apply, int n_prev, double damp, hipStream_t st, int* nb_out);
// FP32: the vector pass of iteration itn (1 .. D) fused with iteration
// itn + 1's product (k_apply's MRF mode): y -> R3, K y -> Ynext.
template <typename T>
hipError_t launch_minres_fused(fbto_grid_s* g, const T* rho, int itn, const T* Y, const T* R1, const T* R2, T* R3,
                               const T* W, T* W2, T* x, T* Ynext, int n_apply, int n_kr, double damp,
                               hipStream_t st, int* nb_out);

}  // namespace fbto
