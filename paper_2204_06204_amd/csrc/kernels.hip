// HIP kernels of the matrix-free SIMP hot path for gfx950 (MI355X).
//
// K(rho) u = sum_e s_e P_e^T KE P_e u on a structured hex8 grid
// (Sec. 3 and the regular-grid product of Sec. 4.3), the Jacobi-PCG low-level
// refinement (Alg. 1 / 3 low-level line with a Jacobi preconditioner,
// Sec. 4.1), the sensitivity of Sec. 3, the linear density filter (Remark on
// modifiers, Sec. 3) and the projection onto the volume-constrained box
// (Sec. 4.2, Eq. piecewiseLinearEQ).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <type_traits>

#include "device.h"
#include "internal.h"

namespace fbto {

namespace {

constexpr int kVecBlock = 256;


template <typename T> const Modal<T>& modal_of(fbto_grid_s* g);
template <> const Modal<double>& modal_of<double>(fbto_grid_s* g) { return g->km64; }
template <> const Modal<float>& modal_of<float>(fbto_grid_s* g) { return g->km32; }
template <typename T> const T* spring_k_of(fbto_grid_s* g);
template <> const double* spring_k_of<double>(fbto_grid_s* g) { return g->spring_k64; }
template <> const float* spring_k_of<float>(fbto_grid_s* g) { return g->spring_k32; }
template <typename T> const T* stencil_w_of(fbto_grid_s* g);
template <> const double* stencil_w_of<double>(fbto_grid_s* g) { return g->stencil_w64; }
template <> const float* stencil_w_of<float>(fbto_grid_s* g) { return g->stencil_w32; }
template <typename T> Vecs& vecs_of(fbto_grid_s* g);
template <> Vecs& vecs_of<double>(fbto_grid_s* g) { return g->v64; }
template <> Vecs& vecs_of<float>(fbto_grid_s* g) { return g->v32; }

}  // namespace

// Grid of the vector kernels: at least 4 entries per thread, at most
// kMaxVecBlocks blocks (the number of partials a consumer reduces).
int vec_blocks(int64_t n) {
  int64_t b = (n + 4 * kVecBlock - 1) / (4 * kVecBlock);
  if (b > kMaxVecBlocks) b = kMaxVecBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

__device__ __forceinline__ const double* pslot(const double* P, int slot, int r, int maxp) {
  return P + ((int64_t)slot * 4 + r) * maxp;
}
__device__ __forceinline__ double* pslot(double* P, int slot, int r, int maxp) {
  return P + ((int64_t)slot * 4 + r) * maxp;
}

// Grid for element / node kernels without partials: one entry per thread.
static int flat_grid(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kVecBlock - 1) / kVecBlock, 1 << 20));
}

// ===========================================================================
// apply_K: z-marching tiles in the sum/difference basis.
//
// A block owns a BX x BY tile of element columns (a runtime shape fitted to
// the grid) and a slab of node planes.  Thread (tx, ty) owns element column
// (ex, ey) = (x0 + tx, y0 + ty), x0 = bx (BX - 1) - 1, y0 = by (BY - 1) - 1,
// and writes node (ex, ey) of every plane of the slab when tx, ty >= 1:
// column and row 0 are the halo shared with the neighbouring tiles.
//
// Per element layer ez:
//   - every node of plane ez + 2 is read from HBM once per tile (the own
//     node, plus the far column and row of the tile by the first BX + BY + 1
//     threads), masked and staged in LDS one layer ahead of its use;
//   - the thread turns the upper face of its element into face modes
//     (x, then y butterflies); the lower face's modes are the upper face's
//     of the layer below, kept in registers;
//   - z butterflies give 8 modes x 3 components; the modal KE (45 entries)
//     times s_e; inverse z butterflies split the result into a lower-face
//     and an upper-face part.  The upper part is carried to the next layer in
//     modal form and added to that layer's lower part before the inverse x/y
//     butterflies, so each face is transformed once in each direction;
//   - the four corner values of plane ez are summed over the four element
//     columns around each node through LDS, in a fixed order.
// Node and corner buffers are double-buffered: one barrier per layer.
// Tiles overlap by one element column / row and slabs by one element layer,
// so there are no atomics and the result is bitwise reproducible.
//
// Modes:
//   APPLY  y = K u
//   RESID  y = r = f - K u; if invD is given, also z = D^-1 r and the
//          partials of r.r, max|r|, f.f (the start of a CG solve)
//   CG     y = w = K z with the partials of r.z, w.z, r.r, max|r| (one
//          reduction phase per step of the Chronopoulos-Gear recurrence)
//   CGF    one fused Chronopoulos-Gear step: the vector update of step k is
//          done where each node is staged (z = D^-1 r, p = z + beta p,
//          s = w + beta s, x += alpha p, r -= alpha s, z' = D^-1 r'), the
//          owner of the node stores x', r', p', s' into the output set, and
//          the product is w' = K z' (step k + 1's apply) with its partials.
//          Input and output sets are distinct buffers: halo nodes of a tile
//          are read by its neighbours while their owner writes the update.
// ===========================================================================
//   MRF    the fused MINRES step of the Krylov low-level step (one RHS):
//          the vector pass of iteration t (see k_minres) done where each
//          node is staged, and iteration t + 1's product K y of the new
//          Lanczos vector y in the same pass.  Y, R1, R2 are read at halo
//          nodes too, so y goes to a third buffer R3 and the product to the
//          other Y buffer.
enum { MODE_APPLY = 0, MODE_RESID = 1, MODE_CG = 2, MODE_CGF = 3, MODE_SENSF = 4, MODE_MRF = 5 };
constexpr int kApplyMaxThreads = 512;
constexpr int kApplyMaxBlocks = 8192;
constexpr double kTinyNorm = 1e-30;  // Krylov step: a norm below this is zero (FP32 reciprocals stay finite)

// Bits 3 R + 1 for R < nr: the |r|_inf entries (max-reduced) of the
// per-RHS triples (sum of squares, |r|_inf, another sum) that the residual
// and finishing reductions lay out.
constexpr unsigned rinf_mask(int nr) {
  unsigned m = 0u;
  for (int R = 0; R < nr; ++R) m |= 1u << (3 * R + 1);
  return m;
}

template <typename T>
struct ApplyArgs {
  Geo g;
  const T* rho;
  const T* u;          // input vector
  T* y;
  const T* f;          // RESID
  const T* invD;       // RESID (optional): start of a CG solve
  T* invD_out;         // RESID (optional): the Jacobi diagonal is formed here and stored
  double ke_diag;      // diagonal entry of KE (with invD_out)
  T* z;                // RESID: z = D^-1 r
  const T* r;          // CG: current residual (for r.z, r.r)
  const uint8_t* mask; // bits 0-2: fixed DOFs of the node; bit 3: the node has a spring
  Modal<T> km;
  Simp sp;
  int nspring;
  const int64_t* sdof;
  const T* sk;
  int bx, by;          // tile of bx * by element columns (threads = (bx + 1) * (by + 1), one per node column)
  int tiles_x, tiles_y, slabs, dz, nblocks, per_xcd;
  double* P;           // partial slots
  int maxp;
  const Scalars* sc;
  int step;            // CG, CGF: step k; CG writes, CGF reads the partial set of parity k & 1
  // CGF only
  const T *xi, *ri, *pi, *si, *wi;   // step k's x, r, p, s, w (p, s unread on the first step)
  T *xo, *ro, *po, *so;              // step k + 1's x, r, p, s (w goes to y)
  int n_apply, n_fn;                 // partial counts of step k's product and of f.f
  double rtol;
  // SENSF only (last CG step fused with the sensitivity)
  T* dobj;                           // [E] -ds_e x_e^T KE x_e (times Hsi_e)
  const T* Hsi;                      // [E] 1/Hs_e, or NULL
  const T* fvec;                     // loads, for f . x (NULL: not formed)
  // MRF only (fused MINRES step; `step` is the iteration t, A.y the product)
  const T *mY, *mR1, *mR2, *mW;      // K R2 of iteration t, Lanczos vectors t - 1 and t, direction t - 2
  T *mR3, *mW2, *mx;                 // new Lanczos vector; direction t - 3 in, t - 1 out; iterate
  int n_kr;                          // partial count of ||R2||^2
  double damp;                       // step size of the low-level step
};

// Step coefficients of the Chronopoulos-Gear recurrence for one RHS from
// gamma = r.z, delta = w.z, r.r and f.f of step k (identical in every
// block):  beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma /
// alpha_prev); beta = 0, alpha = gamma / delta on the first step.  A solved,
// converged or broken-down RHS gets alpha = beta = 0.  The lead thread
// records gamma and alpha in the step-parity slot k & 1 (this kernel reads
// the other one), the flags and the step count.
__device__ __forceinline__ void cg_coefficients(double gam, double del, double rr, double ff, int R,
                                                int step, double rtol, Scalars* sc, bool lead,
                                                double& alpha, double& beta) {
  const bool first = step == 0;
  const int rd = (step + 1) & 1, wr = step & 1;
  const double rn = sqrt(rr), fn = sqrt(ff);
  bool done = sc->done[R] != 0.0 || (rtol > 0.0 && rn <= rtol * fn);
  double status = 0.0;
  alpha = 0.0;
  beta = 0.0;
  if (!done) {
    double denom = del;
    if (!first) {
      beta = gam / sc->cg_gamma[rd][R];
      denom = del - beta * gam / sc->cg_alpha[rd][R];
    }
    if (denom > 0.0 && isfinite(denom) && isfinite(gam)) {
      alpha = gam / denom;
    } else if (gam == 0.0) {
      done = true;
      beta = 0.0;
    } else {
      status = isfinite(denom) && isfinite(gam) ? (double)FBTO_ERR_BREAKDOWN : (double)FBTO_ERR_NONFINITE;
      done = true;
      beta = 0.0;
    }
  }
  if (lead) {
    sc->cg_gamma[wr][R] = gam;
    sc->cg_alpha[wr][R] = alpha;
    if (done) sc->done[R] = 1.0;
    if (status != 0.0) sc->status[R] = status;
    if (alpha != 0.0) sc->steps[R] += 1.0;
    sc->alpha[R] = alpha;
    sc->beta[R] = beta;
  }
}

// Face modes of one face: u[a][c] at local node a = ax + 2 ay -> F[q][c],
// bit 0 / 1 of q set for the difference mode along x / y.
template <typename T>
__device__ __forceinline__ void face_modes(const T (&u)[4][3], T (&F)[4][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T s0 = u[0][c] + u[1][c], d0 = u[1][c] - u[0][c];
    const T s1 = u[2][c] + u[3][c], d1 = u[3][c] - u[2][c];
    F[0][c] = s0 + s1;
    F[1][c] = d0 + d1;
    F[2][c] = s1 - s0;
    F[3][c] = d1 - d0;
  }
}
// Transpose of face_modes.
template <typename T>
__device__ __forceinline__ void face_values(const T (&F)[4][3], T (&u)[4][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T v0 = F[0][c] - F[1][c], v1 = F[0][c] + F[1][c];
    const T v2 = F[2][c] - F[3][c], v3 = F[2][c] + F[3][c];
    u[0][c] = v0 - v2;
    u[2][c] = v0 + v2;
    u[1][c] = v1 - v3;
    u[3][c] = v1 + v3;
  }
}

// One element (one RHS): face modes of its lower and upper face, scale s.
// `carry` holds the modal upper-face result of the element below on entry
// and this element's on exit; `out` receives the values at the 4 nodes of
// the lower face (both elements' contributions).
template <typename T>
__device__ __forceinline__ void layer_product(const T (&Flo)[4][3], const T (&Fup)[4][3], T s,
                                              const Modal<T>& km, T (&carry)[4][3],
                                              T (&out)[4][3]) {
  T c[3][8], z[3][8];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c[i][0] = (T)0;  // the all-sum mode (translation) carries no energy
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q) c[i][q] = s * (Flo[q][i] + Fup[q][i]);
      c[i][q + 4] = s * (Fup[q][i] - Flo[q][i]);
    }
  }
  modal_ke(c, km, z);
  T lo[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lo[q][i] = (z[i][q] - z[i][q + 4]) + carry[q][i];
      carry[q][i] = z[i][q] + z[i][q + 4];
    }
  face_values(lo, out);
}

template <typename T, int NR>
struct ApplyStage {
  T v[2][NR][3];
  unsigned m[2];
};

// Loads of one node plane for the fused CG step (one RHS).
template <typename T>
struct FusedStage {
  T x[3], p[3];                           // owned node only
  T r[2][3], s[2][3], w[2][3], d[2][3];
  unsigned m[2];
};

// Loads of one node plane for the fused MINRES step.
template <typename T>
struct MinresStage {
  T w[3], w2[3], x[3];                    // owned node only
  T y[2][3], r1[2][3], r2[2][3];
  unsigned m[2];
};

// Buffer access of the z-march kernels.  A resource spans 2^31 - 1 bytes
// from its base; kOOR, and kOOR plus the 8 and 16 bytes of an FP64 triple's
// later values, lie beyond it, so an access there loads 0 or is dropped
// without a cache request.
constexpr uint32_t kOOR = 0x80000000u;
// Thread layout of a z-march variant.  Node layout: one thread per node
// column of the tile ((bx + 1) (by + 1) threads), each staging one node per
// plane; the fused steps take it (fewer memory instructions per node; their
// staging does the CG or MINRES vector update too).  Element layout: one
// thread per element column (bx by threads), the tile's far column and row
// staged by a second slot of threads 0 .. bx + by; the plain product, the
// residual and the step-0 product take it (fewer threads for the same
// elements, measured faster for them).
template <int MODE>
constexpr bool node_layout() { return MODE == MODE_CGF || MODE == MODE_MRF || MODE == MODE_SENSF; }
// threads of a z-march block for a tile of bx x by element columns
template <int MODE>
constexpr int zmarch_threads(int bx, int by) {
  return ((node_layout<MODE>() ? (bx + 1) * (by + 1) : bx * by) + 63) / 64 * 64;
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t zrsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7FFFFFFF, 0x00020000);
}
typedef float zf3 __attribute__((ext_vector_type(3)));
typedef unsigned zu3 __attribute__((ext_vector_type(3)));
typedef unsigned zu2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ void zload3(__amdgpu_buffer_rsrc_t rs, uint32_t off, T (&v)[3]) {
  if constexpr (sizeof(T) == 4) {
    const zf3 t = __builtin_bit_cast(zf3, __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0));
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off + 8u * c, 0, 0));
  }
}
template <typename T>
__device__ __forceinline__ void zstore3(__amdgpu_buffer_rsrc_t rs, uint32_t off, const T (&v)[3]) {
  if constexpr (sizeof(T) == 4) {
    zu3 t;
    t.x = __builtin_bit_cast(unsigned, v[0]);
    t.y = __builtin_bit_cast(unsigned, v[1]);
    t.z = __builtin_bit_cast(unsigned, v[2]);
    __builtin_amdgcn_raw_buffer_store_b96(t, rs, off, 0, 0);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(zu2, v[c]), rs, off + 8u * c, 0, 0);
  }
}
template <typename T>
__device__ __forceinline__ T zload1(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void zstore1(__amdgpu_buffer_rsrc_t rs, uint32_t off, T v) {
  if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, off, 0, 0);
  else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(zu2, v), rs, off, 0, 0);
}

// A value that is the same in every lane of the wave, kept in a scalar
// register (FP32; FP64 values stay in vector registers).
// Wave priority around the plane loads of a z-march layer (FP32 only): the
// loads then go out ahead of the element products of the other waves on the
// SIMD.  Measured: FP32 fused steps 1.5-2.5% and the FP32 apply up to 2%
// faster; the FP64 fused CG step at 256x128x128 ran 14% slower with it, so
// FP64 keeps the default priority.
template <typename T>
__device__ __forceinline__ void loads_priority(bool raise) {
  if constexpr (sizeof(T) == 4) {
    if (raise) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(0);
  }
}

template <typename T>
__device__ __forceinline__ T wave_uniform(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
  else return v;
}

// Waves per SIMD the register allocation of a z-march variant must allow:
// three for the single-RHS FP32 fused steps (at most 168 VGPRs), which run
// many blocks per CU on large grids; the others are left to the compiler.
template <typename T, int NR, int MODE>
constexpr int apply_min_waves() {
  return (sizeof(T) == 4 && NR == 1 && (MODE == MODE_CGF || MODE == MODE_MRF)) ? 3 : 1;
}

// RR (fused CG step): form r.r for the tolerance test; solves of a fixed
// step count (rtol = 0) read no r.r and run the variant without it.
template <typename T, int NR, int MODE, bool RR = true>
__global__ void __launch_bounds__(kApplyMaxThreads) __attribute__((amdgpu_waves_per_eu(apply_min_waves<T, NR, MODE>())))
    k_apply(ApplyArgs<T> A, int rhs0) {
  extern __shared__ __align__(16) unsigned char apply_smem[];
  const int b = blockIdx.x;
  const int lb = (b & 7) * A.per_xcd + (b >> 3);  // XCD-aware: neighbours share an L2
  if (lb >= A.nblocks) return;                    // whole block
  const Geo G = A.g;
  const int BX = A.bx, BY = A.by;
  constexpr bool NL = node_layout<MODE>();
  constexpr int kSlots = NL ? 1 : 2;  // node columns a thread stages per plane
  const int NW = BX + 1;          // LDS node row
  const int NS = NW * (BY + 1);   // LDS nodes per plane
  const int TW = NL ? NW : BX;    // threads per tile row
  const int TS = NL ? NS : BX * BY;  // threads with a node (node layout) or an element (element layout)
  T* nodes = reinterpret_cast<T*>(apply_smem);   // [2][NR][3][NS]
  T* corners = nodes + 2 * NR * 3 * NS;         // [2][NR][9][TS]
  T* dcorn = corners + 2 * NR * 9 * TS;          // [2][TS] density sums of the diagonal

  // Thread (tx, ty) of the tile computes element column (x0 + tx, y0 + ty)
  // for tx < BX, ty < BY and stages node (x0 + tx, y0 + ty).  In the node
  // layout the threads of the tile's far column and row (tx = BX or
  // ty = BY) stage those nodes and run the element code on neighbouring LDS
  // values; nothing reads what they produce.  In the element layout
  // threads 0 .. BX + BY stage them in a second slot.  The block is padded
  // to whole waves (the DPP reductions read every lane of a wave); padding
  // threads mirror thread 0 and store nothing.
  const int tid = threadIdx.x;
  const bool live = tid < TS;
  const int tl = live ? tid : 0;
  const int ty = tl / TW, tx = tl - ty * TW;
  const int bxi = lb % A.tiles_x;
  const int t2 = lb / A.tiles_x;
  const int byi = t2 % A.tiles_y;
  const int bz = t2 / A.tiles_y;
  const int x0 = bxi * (BX - 1) - 1, y0 = byi * (BY - 1) - 1;
  const int ex = x0 + tx, ey = y0 + ty;
  const int k0 = bz * A.dz;
  const int kend = min(k0 + A.dz, G.nz + 1);  // emitted planes [k0, kend)
  const int ez0 = k0 == 0 ? 0 : k0 - 1;        // first element layer (a halo layer if k0 > 0)
  const int plane = G.nxn * G.nyn;
  const bool elem_t = live && tx < BX && ty < BY;  // a thread with an element column
  const bool col_elem = elem_t && ex >= 0 && ex < G.nx && ey >= 0 && ey < G.ny;
  // nodes whose four element columns are all in the tile: their outputs
  const bool writer = live && tx >= 1 && ty >= 1 && tx < BX && ty < BY && ex <= G.nx && ey <= G.ny;

  // Node columns staged by this thread: slot 0 its own (ex, ey); in the
  // element layout slot 1 one node of the tile's far column / row (threads
  // 0 .. BX + BY).  Padding threads stage thread 0's node again (the same
  // value into the same LDS slot).
  // Every memory operation of the z-march is issued unconditionally (loads
  // and stores a thread does not need go out of range, see below).  With no
  // branch around them the compiler can
  // count the loads in flight and wait only for the ones it consumes, so
  // the planes prefetched for the next layers stay in flight.
  const bool has_extra = !NL && tid <= BX + BY;
  int li[2], gcol[2];
  li[0] = tx + NW * ty;
  gcol[0] = (ex >= 0 && ex <= G.nx && ey >= 0 && ey <= G.ny) ? ex + G.nxn * ey : -1;
  {
    const int lx = tid <= BY ? BX : tid - BY - 1;
    const int ly = tid <= BY ? tid : BY;
    const int i1 = x0 + lx, j1 = y0 + ly;
    li[1] = has_extra ? lx + NW * ly : li[0];  // the own node again: the same value, same thread
    gcol[1] = has_extra ? ((i1 >= 0 && i1 <= G.nx && j1 >= 0 && j1 <= G.ny) ? i1 + G.nxn * j1 : -1) : gcol[0];
  }

  // Memory access of the z-march.  Every array is addressed through a buffer
  // resource based at the block's first plane ez0, with 32-bit byte offsets
  // relative to it (the host keeps 3 b plane (dz + 3) < 2^31, b the value
  // size).  A lane whose node is not needed -- the far-node slot of a thread
  // without a far node, planes past the slab, values only the owner of a
  // node uses, outputs of a thread that owns none -- passes an out-of-range
  // offset: its load returns 0 and its store is dropped, without a cache
  // request, while every memory instruction is still issued unconditionally.
  const int64_t pbase = (int64_t)ez0 * plane;               // first node of plane ez0
  const int64_t vbase = (int64_t)rhs0 * G.ndof + 3 * pbase;  // its first value in RHS rhs0
  auto rsrc = [](const void* p) { return zrsrc(p); };
  auto vres = [&](const T* v, int r = 0) { return rsrc(v ? v + vbase + (int64_t)r * G.ndof : v); };  // [nrhs][3N]
  auto dres = [&](const T* v) { return rsrc(v ? v + 3 * pbase : v); };  // [3N], one set
  // byte offset of the first value of node column `col` in plane k (k >= ez0)
  auto voff = [&](int col, int k) -> uint32_t {
    return (uint32_t)(3 * sizeof(T)) * (uint32_t)(col + (k - ez0) * plane);
  };
  const __amdgpu_buffer_rsrc_t rs_m = rsrc(A.mask + pbase);
  auto bload3 = [](__amdgpu_buffer_rsrc_t rs, uint32_t off, T (&v)[3]) { zload3<T>(rs, off, v); };
  auto bstore3 = [](__amdgpu_buffer_rsrc_t rs, uint32_t off, const T (&v)[3]) { zstore3<T>(rs, off, v); };
  // the mask byte of a node (kOOR: 0)
  auto bmask = [&](int col, int k, bool ok) -> unsigned {
    return __builtin_amdgcn_raw_buffer_load_b8(rs_m, ok ? (uint32_t)(col + (k - ez0) * plane) : kOOR, 0, 0);
  };

  // Planes past the slab's last one (kend) are staged but never read; their
  // loads are out of range.
  __amdgpu_buffer_rsrc_t rs_u[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) rs_u[r] = vres(A.u, r);
  auto issue = [&](int k, ApplyStage<T, NR>& S) {
    const bool kv = k >= 0 && k <= kend && k <= G.nz;  // planes the block reads
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const bool ok = kv && gcol[sl] >= 0 && (sl == 0 || has_extra);
      const uint32_t ob = ok ? voff(gcol[sl], k) : kOOR;
      const unsigned mv = bmask(gcol[sl], k, ok);
      S.m[sl] = ok ? mv : 7u;
#pragma unroll
      for (int r = 0; r < NR; ++r) bload3(rs_u[r], ob, S.v[sl][r]);
    }
  };
  auto stage = [&](const ApplyStage<T, NR>& S, int buf) {
    T* nb = nodes + buf * (NR * 3 * NS);
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      if (sl == 1 && !has_extra) continue;  // no far node: nothing staged
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          nb[(r * 3 + c) * NS + li[sl]] = ((S.m[sl] >> c) & 1u) ? (T)0 : S.v[sl][r][c];
    }
  };
  // the lower-left node of the thread's element (node 0's for threads
  // without an element, whose face values nothing reads: their reads stay
  // inside the plane)
  const int lf = elem_t ? li[0] : 0;
  auto read_face = [&](int buf, T (&F)[NR][4][3], T (&own)[NR][3]) {
    const T* nb = nodes + buf * (NR * 3 * NS);
    const int o4[4] = {0, 1, NW, NW + 1};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T u4[4][3];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) u4[a][c] = nb[(r * 3 + c) * NS + lf + o4[a]];
#pragma unroll
      for (int c = 0; c < 3; ++c) own[r][c] = u4[0][c];
      face_modes(u4, F[r]);
    }
  };
  // The density of the next layer is loaded raw and turned into s_e only
  // when it is used: consuming a load right after it was issued would make
  // the wave wait for every load issued before it (the counter is in order),
  // including the node planes prefetched for the next layers.
  const __amdgpu_buffer_rsrc_t rs_rho = rsrc(A.rho + (int64_t)G.nx * G.ny * ez0);
  auto load_rho = [&](int ez) -> T {
    const bool el = col_elem && ez >= 0 && ez < G.nz && ez < kend;  // element layers of this block
    const uint32_t off = el ? (uint32_t)sizeof(T) * (uint32_t)(ex + G.nx * (ey + G.ny * (ez - ez0))) : kOOR;
    return zload1<T>(rs_rho, off);
  };
  auto scale_of = [&](int ez, T rv) -> T {
    const bool el = col_elem && ez >= 0 && ez < G.nz;
    return el ? simp_s<T>(rv, A.sp) : (T)0;
  };

  static_assert(MODE != MODE_CGF || NR == 1, "the fused CG step handles one RHS per launch");
  static_assert(MODE != MODE_MRF || NR == 1, "the fused MINRES step handles one RHS per launch");
  constexpr int NP = MODE == MODE_APPLY ? 1 : 4 * NR;  // partial values per block
  double part[NP];
  // The thread's own sums of non-negative terms (r.r, r.z = sum r^2 / d,
  // f.f) and max|r| over its owned nodes, at most 3 (dz + 1) terms per RHS,
  // accumulate in T and join the FP64 partials before the block reduction;
  // sums with terms of either sign (w.z) stay FP64 throughout.
  //   RESID: r.r, max|r|, f.f   CG, CGF: r.z, r.r (the step's coefficients
  //   need no max|r|; the final residual's comes from the last step)
  T tpart[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r) tpart[r][0] = tpart[r][1] = tpart[r][2] = (T)0;
#pragma unroll
  for (int i = 0; i < NP; ++i) part[i] = 0.0;

  // fused CG step: coefficients of step k from its partials (every block;
  // called in the prologue, after the first planes' loads are issued, so
  // the two latencies overlap)
  T al = (T)0, be = (T)0;
  const bool first = A.step == 0;
  auto cg_prologue = [&]() {
    const int par = A.step & 1;
    double pre[4];
    const double* src[4] = {pslot(A.P, P_RZ0 + par, rhs0, A.maxp), pslot(A.P, P_PQ0 + par, rhs0, A.maxp),
                            pslot(A.P, P_RN0 + par, rhs0, A.maxp), pslot(A.P, P_FN, rhs0, A.maxp)};
    const int cnt[4] = {A.n_apply, A.n_apply, A.n_apply, A.n_fn};
    reduce_parts<4, 0u>(pre, src, cnt);
    double alpha, beta;
    cg_coefficients(pre[0], pre[1], pre[2], pre[3], rhs0, A.step, A.rtol, const_cast<Scalars*>(A.sc),
                    lb == 0 && tid == 0, alpha, beta);
    // the same value in every lane: kept in scalar registers
    al = wave_uniform((T)alpha);
    be = wave_uniform((T)beta);
  };
  // fused CG step: loads of one plane, and the update at staging time.
  const __amdgpu_buffer_rsrc_t rs_r = vres(A.ri), rs_w = vres(A.wi), rs_s = vres(A.si), rs_x = vres(A.xi),
                               rs_p = vres(A.pi), rs_d = dres(A.invD);
  const __amdgpu_buffer_rsrc_t rs_xo = vres(A.xo), rs_ro = vres(A.ro), rs_po = vres(A.po), rs_so = vres(A.so);
  auto issue_f = [&](int k, FusedStage<T>& S) {
    const bool kv = k >= 0 && k <= kend && k <= G.nz;  // planes the block reads
    const bool own_plane = k >= k0 && k < kend;
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const bool ok = kv && gcol[sl] >= 0 && (sl == 0 || has_extra);
      const uint32_t ob = ok ? voff(gcol[sl], k) : kOOR;
      const unsigned mv = bmask(gcol[sl], k, ok);
      S.m[sl] = ok ? mv : 7u;
      bload3(rs_r, ob, S.r[sl]);
      bload3(rs_w, ob, S.w[sl]);
      bload3(rs_d, ob, S.d[sl]);
      bload3(rs_s, first ? kOOR : ob, S.s[sl]);  // zero on the first step (not read)
      if (sl == 0) {  // p and x are used by the owner only
        const uint32_t oo = (own_plane && writer && ok) ? ob : kOOR;
        bload3(rs_x, oo, S.x);
        bload3(rs_p, first ? kOOR : oo, S.p);
      }
    }
  };
  auto stage_f = [&](const FusedStage<T>& S, int buf, int k, T (&zq)[3]) {
    T* nb = nodes + buf * (3 * NS);
    const bool own_plane = k >= k0 && k < kend;
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const bool owner = sl == 0 && writer && own_plane;  // the owner's node index is valid
      // the owner's byte offset; other threads store out of range (dropped)
      const uint32_t ob = owner ? voff(gcol[0], k) : kOOR;
      T xn[3], rn[3], pn[3], sn[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sn[c] = S.w[sl][c] + be * S.s[sl][c];
        rn[c] = S.r[sl][c] - al * sn[c];
        const T zn = S.d[sl][c] * rn[c];
        if (sl == 0 || has_extra) nb[c * NS + li[sl]] = ((S.m[sl] >> c) & 1u) ? (T)0 : zn;
        if (sl == 0) {
          zq[c] = zn;  // unmasked: the output of a fixed DOF
          pn[c] = S.d[sl][c] * S.r[sl][c] + be * S.p[c];
          xn[c] = S.x[c] + al * pn[c];
          if (owner) {
            tpart[0][0] += rn[c] * zn;     // r.z
            if constexpr (RR) tpart[0][1] += rn[c] * rn[c];  // r.r
          }
        }
      }
      if (sl == 0) {
        bstore3(rs_xo, ob, xn);
        bstore3(rs_ro, ob, rn);
        bstore3(rs_po, ob, pn);
        bstore3(rs_so, ob, sn);
      }
    }
  };

  // fused MINRES step: the scalar recurrence of iteration t (every block,
  // same order; block 0 keeps the state), as in k_minres
  T ms = (T)0, mc1 = (T)0, mas = (T)0, minvb = (T)0, mwc1 = (T)0, mwc2 = (T)0, minvg = (T)0, mstep = (T)0;
  auto uniform = [](T v) -> T { return wave_uniform(v); };
  auto mrf_prologue = [&]() {
    const int itn = A.step;
    double v[3];
    const double* src[3] = {pslot(A.P, P_KRN0 + ((itn - 1) & 1), 0, A.maxp), pslot(A.P, P_RZ0 + (itn & 1), 0, A.maxp),
                            pslot(A.P, P_PQ0 + (itn & 1), 0, A.maxp)};
    const int cnt[3] = {A.n_kr, A.n_apply, A.n_apply};
    reduce_parts<3, 0u>(v, src, cnt);
    const double beta = sqrt(fmax(v[0], 0.0)), r12 = v[1], yr2 = v[2];
    double oldb = 0.0, alfa_prev = 0.0, dbar = 0.0, epsln = 0.0, phibar = beta, cs = -1.0, sn = 0.0;
    Scalars* sc = const_cast<Scalars*>(A.sc);
    if (itn >= 2) {
      const double* k = sc->kr[(itn + 1) & 1];
      oldb = k[0];
      alfa_prev = k[1];
      dbar = k[2];
      epsln = k[3];
      phibar = k[4];
      cs = k[5];
      sn = k[6];
    }
    double oldeps = 0.0, delta = 0.0, gamma = 1.0, phi = 0.0;
    if (itn >= 2) {
      oldeps = epsln;
      delta = cs * dbar + sn * alfa_prev;
      const double gbar = sn * dbar - cs * alfa_prev;
      epsln = sn * beta;
      dbar = -cs * beta;
      gamma = fmax(sqrt(gbar * gbar + beta * beta), 1e-300);
      cs = gbar / gamma;
      sn = beta / gamma;
      phi = cs * phibar;
      phibar = sn * phibar;
    }
    const double sv = beta > kTinyNorm ? 1.0 / beta : 0.0;  // as in k_minres
    const double c1 = (itn >= 2 && oldb > kTinyNorm) ? beta / oldb : 0.0;
    const double alfa = sv * (sv * yr2 - c1 * r12);
    if (lb == 0 && tid == 0) {
      double* k = sc->kr[itn & 1];
      k[0] = beta;
      k[1] = alfa;
      k[2] = dbar;
      k[3] = epsln;
      k[4] = phibar;
      k[5] = cs;
      k[6] = sn;
    }
    ms = uniform((T)sv);
    mc1 = uniform((T)c1);
    mas = uniform((T)(alfa * sv));
    minvb = uniform((T)(oldb > kTinyNorm ? 1.0 / oldb : 0.0));
    mwc1 = uniform((T)oldeps);
    mwc2 = uniform((T)delta);
    minvg = uniform((T)(gamma > kTinyNorm ? 1.0 / gamma : 0.0));
    mstep = uniform((T)(A.damp * phi));
  };
  // fused MINRES step (single vectors, rhs0 = 0): the memory access of the fused CG step
  const __amdgpu_buffer_rsrc_t rs_mY = vres(A.mY), rs_mR1 = vres(A.mR1), rs_mR2 = vres(A.mR2), rs_mW = vres(A.mW),
                               rs_mW2 = vres(A.mW2), rs_mx = vres(A.mx), rs_mR3 = vres(A.mR3);
  auto issue_m = [&](int k, MinresStage<T>& S) {
    const bool kv = k >= 0 && k <= kend && k <= G.nz;  // planes the block reads
    const bool own_plane = k >= k0 && k < kend;
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const bool ok = kv && gcol[sl] >= 0 && (sl == 0 || has_extra);
      const uint32_t ob = ok ? voff(gcol[sl], k) : kOOR;
      const unsigned mv = bmask(gcol[sl], k, ok);
      S.m[sl] = ok ? mv : 7u;
      bload3(rs_mY, ob, S.y[sl]);
      bload3(rs_mR1, ob, S.r1[sl]);
      bload3(rs_mR2, ob, S.r2[sl]);
      if (sl == 0) {  // the iterate and the directions: owner only
        const uint32_t oo = (own_plane && writer && ok) ? ob : kOOR;
        bload3(rs_mW, oo, S.w);
        bload3(rs_mW2, oo, S.w2);
        bload3(rs_mx, oo, S.x);
      }
    }
  };
  auto stage_m = [&](const MinresStage<T>& S, int buf, int k, T (&zq)[3]) {
    T* nb = nodes + buf * (3 * NS);
    const bool own_plane = k >= k0 && k < kend;
    const int itn = A.step;
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      T yn[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T r1m = itn >= 2 ? S.r1[sl][c] : (T)0;  // R1 holds no vector yet on the first iteration
        yn[c] = ms * S.y[sl][c] - mc1 * r1m - mas * S.r2[sl][c];
        if (sl == 0 || has_extra) nb[c * NS + li[sl]] = ((S.m[sl] >> c) & 1u) ? (T)0 : yn[c];
      }
      if (sl == 0) {
        const bool owner = writer && own_plane;
        const uint32_t ob = owner ? voff(gcol[0], k) : kOOR;
        T wn[3], xn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          zq[c] = yn[c];  // unmasked: the output of a fixed DOF
          const T wm = itn >= 3 ? S.w[c] : (T)0, w2m = itn >= 4 ? S.w2[c] : (T)0;
          wn[c] = (S.r1[0][c] * minvb - mwc1 * w2m - mwc2 * wm) * minvg;
          xn[c] = S.x[c] + mstep * wn[c];
          if constexpr (NP >= 3) {
            if (owner) {
              part[0] += (double)yn[c] * (double)yn[c];        // ||y||^2
              part[2] += (double)S.r2[0][c] * (double)yn[c];   // <R2, y>: R1.R2 of iteration t + 1
            }
          }
        }
        bstore3(rs_mR3, ob, yn);
        if (itn >= 2) {  // finishes iteration t - 1 (uniform)
          bstore3(rs_mW2, ob, wn);
          bstore3(rs_mx, ob, xn);
        }
      }
    }
  };

  // The element stiffness constants.  The FP32 fused steps keep them in
  // vector registers (copied once, here): in scalar registers they pushed
  // the kernel past the scalar register file, and the spilled values came
  // back by v_readlane in every layer.
  Modal<T> km = A.km;
  if constexpr (sizeof(T) == 4 && (MODE == MODE_CGF || MODE == MODE_MRF)) {
    float* q = reinterpret_cast<float*>(&km);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Modal<T>) / sizeof(float)); ++i) {
      float v;
      asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(q[i]));
      q[i] = v;
    }
  }
  ApplyStage<T, NR> S[2];
  FusedStage<T> SF;
  MinresStage<T> SM;
  T F[2][NR][4][3];
  T own[2][NR][3];
  T carry[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[r][q][c] = (T)0;

  // prologue: planes ez0, ez0 + 1 staged (and, unfused, plane ez0 + 2 in flight)
  unsigned mq;     // masks of the own node, plane ez in byte 0, ez + 1 in byte 1, ..
  T rq[3][NR][3];  // unmasked input value of the own node, planes ez, ez + 1, ez + 2
  T rho_next;
  // residual and CG modes: values of the own node read only at its output
  // (RESID: f and D^-1 (or f again); CG: r), loaded one layer ahead.  FP64
  // loads them at the output instead: the queue would not fit its registers.
  constexpr bool kOwnQ = sizeof(T) == 4 && (MODE == MODE_RESID || MODE == MODE_CG);
  T oq[2][NR][2][3];
  __amdgpu_buffer_rsrc_t rs_f[NR], rs_cr[NR], rs_y[NR], rs_z[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    rs_f[r] = vres(A.f, r);
    rs_cr[r] = vres(A.r, r);
    rs_y[r] = vres(A.y, r);
    rs_z[r] = vres(A.z, r);
  }
  const __amdgpu_buffer_rsrc_t rs_do = dres(A.invD_out);
  auto load_own = [&](int k, T (&q)[NR][2][3]) {
    const bool ok = gcol[0] >= 0 && k < kend;  // planes this block outputs
    const uint32_t ob = ok ? voff(gcol[0], k) : kOOR;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if constexpr (MODE == MODE_RESID) {
        bload3(rs_f[r], ob, q[r][0]);
        bload3(rs_d, A.invD ? ob : kOOR, q[r][1]);
      } else {
        bload3(rs_cr[r], ob, q[r][0]);
      }
    }
  };
  if constexpr (MODE == MODE_CGF) {
    FusedStage<T> SF1;
    issue_f(ez0, SF);
    rho_next = load_rho(ez0);
    issue_f(ez0 + 1, SF1);
    cg_prologue();
    stage_f(SF, ez0 & 1, ez0, rq[0][0]);
    mq = SF.m[0] & 0xffu;
    stage_f(SF1, (ez0 + 1) & 1, ez0 + 1, rq[1][0]);
    mq |= (SF1.m[0] & 0xffu) << 8;
  } else if constexpr (MODE == MODE_MRF) {
    MinresStage<T> SM1;
    issue_m(ez0, SM);
    rho_next = load_rho(ez0);
    issue_m(ez0 + 1, SM1);
    mrf_prologue();
    stage_m(SM, ez0 & 1, ez0, rq[0][0]);
    mq = SM.m[0] & 0xffu;
    stage_m(SM1, (ez0 + 1) & 1, ez0 + 1, rq[1][0]);
    mq |= (SM1.m[0] & 0xffu) << 8;
  } else {
    issue(ez0, S[0]);
    issue(ez0 + 1, S[1]);
    stage(S[0], ez0 & 1);
    stage(S[1], (ez0 + 1) & 1);
    mq = (S[0].m[0] & 0xffu) | ((S[1].m[0] & 0xffu) << 8);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        rq[0][r][c] = S[0].v[0][r][c];
        rq[1][r][c] = S[1].v[0][r][c];
      }
    // the density first, then the next plane: as in every layer, so that
    // the wait for the density leaves the plane's loads in flight
    rho_next = load_rho(ez0);
    if constexpr (kOwnQ) load_own(ez0, oq[0]);
    issue(ez0 + 2, S[0]);
  }
  T s_below = (T)0;  // s of the element below (diagonal of the residual mode)
  __syncthreads();
  read_face(ez0 & 1, F[0], own[0]);
  __syncthreads();  // the first layer restages the buffer of plane ez0

  auto layer = [&](auto parity, int ez) {
    constexpr int P = decltype(parity)::value;
    const T s = scale_of(ez, rho_next);
    rho_next = load_rho(ez + 1);
    if constexpr (kOwnQ) load_own(ez + 1, oq[P ^ 1]);
    loads_priority<T>(true);
    if constexpr (MODE == MODE_CGF) {
      issue_f(ez + 2, SF);
    } else if constexpr (MODE == MODE_MRF) {
      issue_m(ez + 2, SM);
    } else {
      issue(ez + 3, S[P ^ 1]);
    }
    loads_priority<T>(false);
    const T dcol = s_below + s;  // this column's share of the lower-face nodes' diagonal
    s_below = s;
    read_face((ez + 1) & 1, F[P ^ 1], own[P ^ 1]);
    const bool emit = ez >= k0;  // uniform over the block
    T out[NR][4][3];
#pragma unroll
    for (int r = 0; r < NR; ++r) layer_product(F[P][r], F[P ^ 1][r], s, km, carry[r], out[r]);
    const int cb = ez & 1;
    if (emit && live) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int a = 1; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            corners[((cb * NR + r) * 9 + (a - 1) * 3 + c) * TS + tid] = out[r][a][c];
      if constexpr (MODE == MODE_RESID) {
        if (A.invD_out) dcorn[cb * TS + tid] = dcol;
      }
    }
    if constexpr (MODE == MODE_CGF) {
      stage_f(SF, ez & 1, ez + 2, rq[2][0]);
      mq |= (SF.m[0] & 0xffu) << 16;
    } else if constexpr (MODE == MODE_MRF) {
      stage_m(SM, ez & 1, ez + 2, rq[2][0]);
      mq |= (SM.m[0] & 0xffu) << 16;
    } else {
      stage(S[P], ez & 1);
      mq |= (S[P].m[0] & 0xffu) << 16;
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) rq[2][r][c] = S[P].v[0][r][c];
    }
    __syncthreads();
    {
      // every thread runs the output code; a thread that owns no output node
      // reads its own LDS slots, loads and stores out of range
      const bool wr = emit && writer;
      const int n = wr ? gcol[0] + ez * plane : 0;
      const uint32_t ob = wr ? voff(gcol[0], ez) : kOOR;
      const unsigned m = wr ? (mq & 0xffu) : 0u;
      const int tl1 = wr ? tid - 1 : tl, tlb = wr ? tid - TW : tl, tlbb = wr ? tid - TW - 1 : tl;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const T* cr = corners + (cb * NR + r) * 9 * TS;
        T acc[3], pv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc[c] = ((out[r][0][c] + cr[(0 + c) * TS + tl1]) + cr[(3 + c) * TS + tlb]) + cr[(6 + c) * TS + tlbb];
          pv[c] = own[P][r][c];  // masked input value at this node
        }
        if (m) {  // springs, then identity rows of fixed DOFs (rare nodes)
          if (m & 8u) {
            for (int sI = 0; sI < A.nspring; ++sI) {
              const int64_t d = A.sdof[sI] - (int64_t)3 * n;
#pragma unroll
              for (int c = 0; c < 3; ++c)
                if (d == c) acc[c] += A.sk[sI] * pv[c];
            }
          }
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if ((m >> c) & 1u) {  // the unmasked input value, as staged
              pv[c] = rq[0][r][c];
              acc[c] = pv[c];
            }
        }
        // partial sums count owned nodes only (a select: values of a thread
        // without an owned node may be anything, NaN included)
        auto own_only = [wr](double v) { return wr ? v : 0.0; };
        auto own_t = [wr](T v) { return wr ? v : (T)0; };
        if constexpr (MODE == MODE_RESID) {
          const bool zout = A.invD || A.invD_out;
          T fv[3], rv[3], dv[3], dl[3], zv[3];
          if constexpr (kOwnQ) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              fv[c] = oq[P][r][0][c];
              dl[c] = oq[P][r][1][c];
            }
          } else {
            bload3(rs_f[r], ob, fv);
            bload3(rs_d, A.invD ? ob : kOOR, dl);
          }
          const T D = ((dcol + dcorn[cb * TS + tl1]) + dcorn[cb * TS + tlb]) + dcorn[cb * TS + tlbb];
          // Jacobi diagonal: ke_diag * sum of s over the node's 8 elements,
          // one value (and one division) for the node's three DOFs; springs
          // and fixed DOFs (nodes with m != 0, rare) set single entries
          const T d0 = (T)A.ke_diag * D;
          T dinv0 = (T)0;
          if (A.invD_out) dinv0 = d0 > (T)0 ? (T)1 / d0 : (T)0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            rv[c] = fv[c] - acc[c];
            if (A.invD_out) {
              T di = dinv0;
              if (m) {
                T d = d0;
                if (m & 8u)
                  for (int sI = 0; sI < A.nspring; ++sI)
                    if (A.sdof[sI] == (int64_t)(3 * n + c)) d += A.sk[sI];
                if ((m >> c) & 1u) d = (T)1;
                di = d > (T)0 ? (T)1 / d : (T)0;
              }
              dv[c] = di;
            } else {
              dv[c] = dl[c];
            }
            zv[c] = dv[c] * rv[c];
          }
          bstore3(rs_y[r], ob, rv);
          bstore3(rs_z[r], zout ? ob : kOOR, zv);
          if (A.invD_out) bstore3(rs_do, ob, dv);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            tpart[r][0] += own_t(rv[c] * rv[c]);
            tpart[r][1] = fmax(tpart[r][1], own_t(fabs(rv[c])));
            tpart[r][2] += own_t(fv[c] * fv[c]);
          }
        } else {
          bstore3(rs_y[r], ob, acc);
          if constexpr (MODE == MODE_CG) {
            T rv3[3];
            if constexpr (kOwnQ) {
#pragma unroll
              for (int c = 0; c < 3; ++c) rv3[c] = oq[P][r][0][c];
            } else {
              bload3(rs_cr[r], ob, rv3);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const T rv = rv3[c];
              tpart[r][0] += own_t(rv * pv[c]);                             // r.z
              part[4 * r + 1] += own_only((double)acc[c] * (double)pv[c]);  // w.z
              tpart[r][1] += own_t(rv * rv);                                // r.r
            }
          }
          if constexpr (MODE == MODE_CGF || MODE == MODE_MRF) {
#pragma unroll
            for (int c = 0; c < 3; ++c) part[1] += own_only((double)acc[c] * (double)pv[c]);  // w'.z' / <K y, y>
          }
        }
      }
    }
    mq >>= 8;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        rq[0][r][c] = rq[1][r][c];
        rq[1][r][c] = rq[2][r][c];
      }
  };
  for (int ez = ez0; ez < kend; ez += 2) {
    layer(std::integral_constant<int, 0>{}, ez);
    if (ez + 1 >= kend) break;
    layer(std::integral_constant<int, 1>{}, ez + 1);
  }

  if constexpr (MODE == MODE_CG || MODE == MODE_CGF) {
    // CG: step k's product -> set k & 1; CGF: step k + 1's -> set (k + 1) & 1
    const int par = (MODE == MODE_CG ? A.step : A.step + 1) & 1;
    constexpr int NV = RR ? 3 : 2;  // r.z, w.z (, r.r)
    double* dst[NV * NR];
    double v[NV * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      dst[NV * r + 0] = pslot(A.P, P_RZ0 + par, rhs0 + r, A.maxp);
      dst[NV * r + 1] = pslot(A.P, P_PQ0 + par, rhs0 + r, A.maxp);
      v[NV * r + 0] = (double)tpart[r][0];
      v[NV * r + 1] = part[4 * r + 1];
      if constexpr (RR) {
        dst[NV * r + 2] = pslot(A.P, P_RN0 + par, rhs0 + r, A.maxp);
        v[NV * r + 2] = (double)tpart[r][1];
      }
    }
    write_parts<NV * NR, 0u>(v, dst, lb);
  }
  if constexpr (MODE == MODE_MRF) {
    // ||y||^2 -> the norm slot of iteration t; <K y, y> and <R2, y> -> the
    // product partials of iteration t + 1
    const int itn = A.step;
    double v[3] = {part[0], part[1], part[2]};
    double* dst[3] = {pslot(A.P, P_KRN0 + (itn & 1), 0, A.maxp), pslot(A.P, P_PQ0 + ((itn + 1) & 1), 0, A.maxp),
                      pslot(A.P, P_RZ0 + ((itn + 1) & 1), 0, A.maxp)};
    write_parts<3, 0u>(v, dst, lb);
  }
  if constexpr (MODE == MODE_RESID) {
    if (A.invD == nullptr && A.invD_out == nullptr) return;
    if (lb == 0 && tid == 0) {   // a new solve starts from this residual
      Scalars* sc = const_cast<Scalars*>(A.sc);
      for (int r = 0; r < NR; ++r) {
        sc->done[rhs0 + r] = 0.0;
        sc->status[rhs0 + r] = 0.0;
        sc->steps[rhs0 + r] = 0.0;
      }
    }
    double v[3 * NR];
    double* dst[3 * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      v[3 * r + 0] = (double)tpart[r][0];
      v[3 * r + 1] = (double)tpart[r][1];
      v[3 * r + 2] = (double)tpart[r][2];
      dst[3 * r + 0] = pslot(A.P, P_RNF, rhs0 + r, A.maxp);
      dst[3 * r + 1] = pslot(A.P, P_RIF, rhs0 + r, A.maxp);
      dst[3 * r + 2] = pslot(A.P, P_FN, rhs0 + r, A.maxp);
    }
    write_parts<3 * NR, rinf_mask(NR)>(v, dst, lb);
  }
}

// ===========================================================================
// The last Chronopoulos-Gear step of a solve fused with the sensitivity of
// Sec. 3 (one RHS).  On the tiling of k_apply, every staged node gets
// x' = x + alpha (D^-1 r + beta p); the owner of the node stores x', and
// forms r' = r - alpha (w + beta s) for the final residual norms and f . x'.
// Each element owned by the block gets
//   dobj_e = -ds_e x'_e^T KE x'_e  (times 1/Hs_e when given)
// from the face modes of its two faces.  Nothing is scattered back to the
// nodes, so there is no corner exchange; one barrier per layer guards the
// double-buffered node planes.
// ===========================================================================
template <typename T>
struct SensStage {
  T x[2][3], r[2][3], p[2][3], d[2][3];  // every staged node
  T w[3], s[3], f[3];                    // owned node only
  unsigned m[2];
};

template <typename T>
__global__ void __launch_bounds__(kApplyMaxThreads)
    k_cg_sens(ApplyArgs<T> A) {
  extern __shared__ __align__(16) unsigned char apply_smem[];
  const int b = blockIdx.x;
  const int lb = (b & 7) * A.per_xcd + (b >> 3);
  if (lb >= A.nblocks) return;
  const Geo G = A.g;
  const int BX = A.bx, BY = A.by;
  const int NW = BX + 1;
  const int NS = NW * (BY + 1);
  T* nodes = reinterpret_cast<T*>(apply_smem);  // [2][3][NS]
  // one thread per node column of the tile (the node layout of k_apply)
  constexpr int kSlots = 1;
  const int tid = threadIdx.x;
  const bool live = tid < NS;
  const int tl = live ? tid : 0;
  const int ty = tl / NW, tx = tl - ty * NW;
  const int bxi = lb % A.tiles_x;
  const int t2 = lb / A.tiles_x;
  const int byi = t2 % A.tiles_y;
  const int bz = t2 / A.tiles_y;
  const int x0 = bxi * (BX - 1) - 1, y0 = byi * (BY - 1) - 1;
  const int ex = x0 + tx, ey = y0 + ty;
  const int k0 = bz * A.dz;
  const int kend = min(k0 + A.dz, G.nz + 1);
  const int ez0 = k0 == 0 ? 0 : k0 - 1;
  const int elem_end = min(k0 + A.dz, G.nz);   // element layers [k0, elem_end) belong to this slab
  const int plane = G.nxn * G.nyn;
  const bool writer = live && tx >= 1 && ty >= 1 && tx < BX && ty < BY && ex <= G.nx && ey <= G.ny;
  const bool elem_owner = writer && ex < G.nx && ey < G.ny;
  // As in k_apply, the vectors are addressed through buffer resources based
  // at the block's first plane ez0: a plane past the slab or a thread that
  // owns no node gets an out-of-range offset, so its loads return 0 and its
  // stores are dropped, with no branch around them.
  constexpr bool has_extra = false;
  int li[2], gcol[2];
  li[0] = tl;  // padding threads stage thread 0's node again (the same value into the same slot)
  gcol[0] = (ex >= 0 && ex <= G.nx && ey >= 0 && ey <= G.ny) ? ex + G.nxn * ey : -1;
  li[1] = li[0];
  gcol[1] = gcol[0];
  const int64_t pbase = (int64_t)ez0 * plane;  // first node of plane ez0
  auto vres = [&](const T* v) { return zrsrc(v ? v + 3 * pbase : v); };
  auto voff = [&](int col, int k) -> uint32_t {
    return (uint32_t)(3 * sizeof(T)) * (uint32_t)(col + (k - ez0) * plane);
  };
  const __amdgpu_buffer_rsrc_t rs_m = zrsrc(A.mask + pbase), rs_x = vres(A.xi), rs_r = vres(A.ri),
                               rs_d = vres(A.invD), rs_p = vres(A.pi), rs_w = vres(A.wi), rs_s = vres(A.si),
                               rs_f = vres(A.fvec), rs_xo = vres(A.xo);
  const int64_t ebase = (int64_t)ez0 * G.nx * G.ny;  // first element of layer ez0
  const __amdgpu_buffer_rsrc_t rs_rho = zrsrc(A.rho + ebase), rs_hs = zrsrc(A.Hsi ? A.Hsi + ebase : A.Hsi),
                               rs_do = zrsrc(A.dobj + ebase);

  // step coefficients (every block, same order; called after the first
  // planes' loads are issued, so the two latencies overlap)
  const bool first = A.step == 0;
  T al = (T)0, be = (T)0;
  auto coefficients = [&]() {
    const int par = A.step & 1;
    double pre[4];
    const double* src[4] = {pslot(A.P, P_RZ0 + par, 0, A.maxp), pslot(A.P, P_PQ0 + par, 0, A.maxp),
                            pslot(A.P, P_RN0 + par, 0, A.maxp), pslot(A.P, P_FN, 0, A.maxp)};
    const int cnt[4] = {A.n_apply, A.n_apply, A.n_apply, A.n_fn};
    reduce_parts<4, 0u>(pre, src, cnt);
    double alpha, beta;
    cg_coefficients(pre[0], pre[1], pre[2], pre[3], 0, A.step, A.rtol, const_cast<Scalars*>(A.sc),
                    lb == 0 && tid == 0, alpha, beta);
    al = wave_uniform((T)alpha);
    be = wave_uniform((T)beta);
  };
  // r'.r', max|r'|, f.x', and the sum of the block's element sensitivities
  double part[4] = {0.0, 0.0, 0.0, 0.0};

  auto owns = [&](int k) { return k >= 0 && k <= G.nz && writer && k >= k0 && k < kend; };
  auto issue = [&](int k, SensStage<T>& S) {
    const bool kv = k >= 0 && k <= kend && k <= G.nz;  // planes past kend are never read
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const bool ok = kv && gcol[sl] >= 0 && (sl == 0 || has_extra);
      const uint32_t off = ok ? voff(gcol[sl], k) : kOOR;
      const unsigned mv = __builtin_amdgcn_raw_buffer_load_b8(rs_m, ok ? (uint32_t)(gcol[sl] + (k - ez0) * plane) : kOOR, 0, 0);
      S.m[sl] = ok ? mv : 7u;
      zload3<T>(rs_x, off, S.x[sl]);
      zload3<T>(rs_r, off, S.r[sl]);
      zload3<T>(rs_d, off, S.d[sl]);
      zload3<T>(rs_p, first ? kOOR : off, S.p[sl]);  // allocated on the first step too, its contents unused
      if (sl == 0) {  // used by the owner only
        const uint32_t oo = owns(k) ? off : kOOR;
        zload3<T>(rs_w, oo, S.w);
        zload3<T>(rs_s, first ? kOOR : oo, S.s);
        zload3<T>(rs_f, A.fvec ? oo : kOOR, S.f);
      }
    }
  };
  auto stage = [&](const SensStage<T>& S, int buf, int k) {
    T* nb = nodes + buf * (3 * NS);
    const bool own = owns(k);
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      T xn[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T pn = S.d[sl][c] * S.r[sl][c] + be * S.p[sl][c];
        xn[c] = S.x[sl][c] + al * pn;
        if (sl == 0 || has_extra) nb[c * NS + li[sl]] = ((S.m[sl] >> c) & 1u) ? (T)0 : xn[c];
      }
      if (sl == 0) {
        zstore3<T>(rs_xo, own ? voff(gcol[0], k) : kOOR, xn);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T rn = S.r[0][c] - al * (S.w[c] + be * S.s[c]);
          part[0] += own ? (double)rn * (double)rn : 0.0;
          part[1] = fmax(part[1], own ? fabs((double)rn) : 0.0);
          part[2] += own ? (double)S.f[c] * (double)xn[c] : 0.0;
        }
      }
    }
  };
  // the lower-left node of the thread's element (node 0's for threads
  // without an element: their reads stay inside the plane)
  const int lf = (live && tx < BX && ty < BY) ? li[0] : 0;
  auto read_face = [&](int buf, T (&F)[4][3]) {
    const T* nb = nodes + buf * (3 * NS);
    const int o4[4] = {0, 1, NW, NW + 1};
    T u4[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) u4[a][c] = nb[c * NS + lf + o4[a]];
    face_modes(u4, F);
  };
  // byte offset of the element of layer ez in this thread's column (kOOR if
  // the element is not this block's)
  auto eoff = [&](int ez) -> uint32_t {
    const bool el = elem_owner && ez >= k0 && ez < elem_end;
    return el ? (uint32_t)sizeof(T) * (uint32_t)(ex + G.nx * (ey + G.ny * (ez - ez0))) : kOOR;
  };
  // density and 1/Hs of the element of a layer, loaded a layer ahead
  auto load_elem = [&](int ez, T (&v)[2]) {
    const uint32_t off = eoff(ez);
    v[0] = zload1<T>(rs_rho, off);
    const T hv = zload1<T>(rs_hs, A.Hsi ? off : kOOR);
    v[1] = A.Hsi ? hv : (T)1;
  };

  SensStage<T> S;
  T F[2][4][3];
  T ev[2][2];
  {
    SensStage<T> S1;
    issue(ez0, S);
    issue(ez0 + 1, S1);
    coefficients();
    stage(S, ez0 & 1, ez0);
    stage(S1, (ez0 + 1) & 1, ez0 + 1);
  }
  load_elem(ez0, ev[0]);
  __syncthreads();
  read_face(ez0 & 1, F[0]);
  __syncthreads();

  auto layer = [&](auto parity, int ez) {
    constexpr int P = decltype(parity)::value;
    load_elem(ez + 1, ev[P ^ 1]);
    loads_priority<T>(true);
    issue(ez + 2, S);
    loads_priority<T>(false);
    read_face((ez + 1) & 1, F[P ^ 1]);
    {
      T c[3][8], z[3][8];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        c[i][0] = (T)0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q) c[i][q] = F[P][q][i] + F[P ^ 1][q][i];
          c[i][q + 4] = F[P ^ 1][q][i] - F[P][q][i];
        }
      }
      modal_ke(c, A.km, z);
      double en = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int q = 1; q < 8; ++q) en += (double)c[i][q] * (double)z[i][q];
      const double dc = -(double)simp_ds<T>(ev[P][0], A.sp) * en;  // d objective / d rho_e
      zstore1<T>(rs_do, eoff(ez), (T)(dc * (double)ev[P][1]));
      // The filter weights are symmetric, so the filtered gradient
      // H^T (dc / Hs) sums to sum_e dc_e: its mean for the step, formed here.
      part[3] += (elem_owner && ez >= k0 && ez < elem_end) ? dc : 0.0;
    }
    stage(S, ez & 1, ez + 2);
    __syncthreads();
  };
  for (int ez = ez0; ez < kend; ez += 2) {
    layer(std::integral_constant<int, 0>{}, ez);
    if (ez + 1 >= kend) break;
    layer(std::integral_constant<int, 1>{}, ez + 1);
  }
  double* dst[4] = {pslot(A.P, P_RNF, 0, A.maxp), pslot(A.P, P_RIF, 0, A.maxp), pslot(A.P, P_DOT, 0, A.maxp),
                     pslot(A.P, P_GSUM, 0, A.maxp)};
  write_parts<4, 0x2u>(part, dst, lb);
}

template <typename T>
static size_t sens_lds_bytes(int bx, int by) {
  return sizeof(T) * (size_t)(2 * 3 * (bx + 1) * (by + 1));
}

template <typename T, int NR, int MODE>
static size_t apply_lds_bytes(int bx, int by) {
  const size_t ns = (size_t)(bx + 1) * (by + 1);                      // nodes per plane
  const size_t ts = node_layout<MODE>() ? ns : (size_t)bx * by;      // corner slots
  return sizeof(T) * (2 * NR * 3 * ns + 2 * NR * 9 * ts + 2 * ts);
}

// The z-march addresses each vector from the block's first plane with
// 32-bit byte offsets: its planes (dz + 3 at most: the slab, the halo layer
// below, the prefetched plane above) must span less than 2 GiB.
bool apply_offsets_fit(const Geo& G, int dz, size_t value_bytes) {
  return (int64_t)(3 * value_bytes) * G.nxn * G.nyn * (dz + 3) < ((int64_t)1 << 31);
}

// Tile shape and slab depth for one apply variant.  The cost is the work of
// the busiest CU in wave-layers (each block: its waves x (layers + 1 for the
// prologue)), with a floor of kMinWaves resident waves per round below which
// latency, not issue, sets the time.
template <typename T, int NR, int MODE>
static TileChoice choose_tile(const Geo& G, int n_cu, int lds_per_cu, int override_shape) {
  // fixed fields of a caller's override (FBTO_OPT_APPLY_TILE / _CGF_TILE)
  const int want_bx = override_shape & 0xff, want_by = (override_shape >> 8) & 0xff,
            want_dz = (override_shape >> 16) & 0xff;
  constexpr double kMinWaves = 8.0;
  TileChoice best{};
  double best_cost = 1e300;
  // The fused steps on large grids (2^22 elements and more): 27 x 8 element
  // columns (28 x 9 = 252 threads, rows of 28 nodes) in slabs of 33 layers.
  // Long rows keep the L1 path, which bounds these steps there, on few
  // partial cache lines.  The CG step runs at most two blocks per CU (the
  // L1 path then serves fewer waves) unless three per CU (as many as its
  // registers allow) finish the grid in fewer rounds: a round of three
  // measured 1.31 times as long as a round of two.  Measured (FP32 CG step):
  // 155 us at 256x128x128 (one round of three) and 497 us at 384x192x192
  // (two per CU), against 167 and 527 us for the cost model's choice.
  if constexpr (MODE == MODE_CGF || MODE == MODE_MRF) {
    if (override_shape == 0 && G.E >= ((int64_t)1 << 22)) {
      const int bx = 27, by = 8, dz = std::min(33, G.nzn);
      const int threads = zmarch_threads<MODE>(bx, by);
      const int tiles_x = (G.nxn + bx - 2) / (bx - 1), tiles_y = (G.nyn + by - 2) / (by - 1);
      const int slabs = (G.nzn + dz - 1) / dz;
      const int64_t nb = (int64_t)tiles_x * tiles_y * slabs;
      int cap = 0;
      if constexpr (MODE == MODE_CGF) {
        const int64_t r2 = (nb + 2 * n_cu - 1) / (2 * n_cu), r3 = (nb + 3 * n_cu - 1) / (3 * n_cu);
        cap = 1.31 * (double)r3 < (double)r2 ? 0 : 2;
      }
      const size_t lds = std::max(apply_lds_bytes<T, NR, MODE>(bx, by), cap ? (size_t)lds_for_block_cap(lds_per_cu, cap) : 0);
      int occ = 0;
      const hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_apply<T, NR, MODE>, threads, lds);
      if (oe == hipSuccess && occ >= 1 && lds <= kApplyMaxLds && nb <= kApplyMaxBlocks &&
          apply_offsets_fit(G, dz, sizeof(T)))
        return TileChoice{bx, by, dz, tiles_x, tiles_y, slabs, (int)nb, cap};
    }
  }
  for (int bx = 8; bx <= 64; ++bx) {
    if (want_bx && bx != want_bx) continue;
    for (int by = 4; by <= 64; ++by) {
      if (want_by && by != want_by) continue;
      const int ts = node_layout<MODE>() ? (bx + 1) * (by + 1) : bx * by;  // threads
      // at most four waves: every layer ends at a block-wide barrier, and
      // blocks of up to one wave per SIMD measured fastest
      if (ts < 128 || ts > 256) continue;
      const size_t lds = MODE == MODE_SENSF ? sens_lds_bytes<T>(bx, by) : apply_lds_bytes<T, NR, MODE>(bx, by);
      if (lds > kApplyMaxLds) continue;
      const int waves = (ts + 63) / 64;
      int occ = 0;
      hipError_t oe;
      if constexpr (MODE == MODE_SENSF)
        oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_cg_sens<T>, 64 * waves, lds);
      else
        oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_apply<T, NR, MODE>, 64 * waves, lds);
      if (oe != hipSuccess || occ < 1) continue;
      const int tiles_x = (G.nxn + bx - 2) / (bx - 1);
      const int tiles_y = (G.nyn + by - 2) / (by - 1);
      for (int dz = 1; dz <= std::min(G.nzn, 64); ++dz) {
        if (want_dz && dz != want_dz) continue;
        // the planes a block reads, addressed by 32-bit byte offsets
        if (!apply_offsets_fit(G, dz, sizeof(T))) continue;
        const int slabs = (G.nzn + dz - 1) / dz;
        const int64_t nb = (int64_t)tiles_x * tiles_y * slabs;
        if (nb > kApplyMaxBlocks) continue;
        const int64_t per_cu = (nb + n_cu - 1) / n_cu;
        const int64_t full = per_cu / occ, rem = per_cu % occ;
        const double layers = dz + 2.0;
        // a block's waves go to the CU's four SIMDs; a count that does not
        // spread evenly (3, 5, 6, 7) leaves one SIMD with more work, as if
        // the block had the next multiple of four
        const double w = (waves == 1 || waves == 2 || waves == 4 || waves == 8) ? waves : (waves + 3) / 4 * 4;
        const double cost = full * std::max((double)occ * w, kMinWaves) * layers +
                            (rem ? std::max((double)rem * w, kMinWaves) * layers : 0.0);
        if (cost < best_cost) {
          best_cost = cost;
          best = TileChoice{bx, by, dz, tiles_x, tiles_y, slabs, (int)nb, (override_shape >> 24) & 0xf};
        }
      }
    }
  }
  return best;
}

template <typename T, int NR, int MODE, bool RR = true>
static hipError_t launch_apply_t(fbto_grid_s* g, const ApplyArgs<T>& A0, int rhs0, hipStream_t st,
                                 int* nb_out) {
  TileChoice& t = g->tiles[sizeof(T) == 8 ? 1 : 0][NR - 1][MODE];
  if (t.nblocks == 0) {
    t = choose_tile<T, NR, MODE>(g->geo, g->n_cu, g->lds_per_cu, g->tile_override[MODE == MODE_CGF ? 1 : 0]);
    if (t.nblocks == 0) return hipErrorInvalidConfiguration;
  }
  if (t.nblocks > g->max_partials) return hipErrorInvalidValue;
  if (nb_out) *nb_out = t.nblocks;
  ApplyArgs<T> A = A0;
  A.bx = t.bx;
  A.by = t.by;
  A.tiles_x = t.tiles_x;
  A.tiles_y = t.tiles_y;
  A.slabs = t.slabs;
  A.dz = t.dz;
  A.nblocks = t.nblocks;
  A.per_xcd = (t.nblocks + 7) / 8;
  const int grid = A.per_xcd * 8;
  size_t lds = apply_lds_bytes<T, NR, MODE>(t.bx, t.by);
  if (t.cap) lds = std::max(lds, (size_t)lds_for_block_cap(g->lds_per_cu, t.cap));
  const int threads = zmarch_threads<MODE>(t.bx, t.by);  // whole waves
  hipLaunchKernelGGL((k_apply<T, NR, MODE, RR>), dim3(grid), dim3(threads), lds, st, A, rhs0);
  return hipGetLastError();
}

template <typename T, int MODE, bool RR = true>
static hipError_t launch_apply_mode(fbto_grid_s* g, ApplyArgs<T> A, int nrhs, hipStream_t st, int* nb_out) {
  A.g = g->geo;
  A.mask = g->mask;
  A.km = modal_of<T>(g);
  A.sp = g->simp;
  A.nspring = g->n_springs;
  A.sdof = g->spring_dof;
  A.sk = spring_k_of<T>(g);
  A.P = g->partials;
  A.maxp = g->max_partials;
  A.sc = g->sc;
  // one RHS per launch: the per-RHS state of the z-march (two face-mode
  // sets, the modal carry, staged loads) fills the register file at NR = 1
  hipError_t e = hipSuccess;
  for (int r0 = 0; r0 < nrhs && e == hipSuccess; ++r0) e = launch_apply_t<T, 1, MODE, RR>(g, A, r0, st, nb_out);
  return e;
}

int apply_max_blocks(const Geo&, int) { return kApplyMaxBlocks; }

template <typename T>
hipError_t launch_apply(fbto_grid_s* g, const T* rho, const T* u, T* y, int nrhs, hipStream_t st) {
  if (g->dim == 2) return plane_apply<T>(g, rho, u, y, nrhs, st);
  ApplyArgs<T> A{};
  A.rho = rho;
  A.u = u;
  A.y = y;
  return launch_apply_mode<T, MODE_APPLY>(g, A, nrhs, st, nullptr);
}

template <typename T>
hipError_t launch_resid(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, const T* invD, T* z,
                        int nrhs, hipStream_t st, int* nb_out) {
  if (g->dim == 2) return plane_resid<T>(g, rho, u, f, r, invD, nullptr, z, nrhs, st, nb_out);
  ApplyArgs<T> A{};
  A.rho = rho;
  A.u = u;
  A.y = r;
  A.f = f;
  A.invD = invD;
  A.z = z;
  return launch_apply_mode<T, MODE_RESID>(g, A, nrhs, st, nb_out);
}

template <typename T>
hipError_t launch_resid_diag(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, T* invD_out, T* z,
                             int nrhs, hipStream_t st, int* nb_out) {
  if (g->dim == 2) return plane_resid<T>(g, rho, u, f, r, nullptr, invD_out, z, nrhs, st, nb_out);
  ApplyArgs<T> A{};
  A.rho = rho;
  A.u = u;
  A.y = r;
  A.f = f;
  A.invD_out = invD_out;
  A.ke_diag = g->ke_diag;
  A.z = z;
  return launch_apply_mode<T, MODE_RESID>(g, A, nrhs, st, nb_out);
}

template <typename T>
hipError_t launch_apply_cg(fbto_grid_s* g, const T* rho, const T* z, const T* r, T* w, int nrhs, int step,
                           hipStream_t st, int* nb_out) {
  if (g->dim == 2) return plane_apply_cg<T>(g, rho, z, r, w, nrhs, step, st, nb_out);
  ApplyArgs<T> A{};
  A.rho = rho;
  A.u = z;
  A.r = r;
  A.y = w;
  A.step = step;
  return launch_apply_mode<T, MODE_CG>(g, A, nrhs, st, nb_out);
}

template <typename T>
hipError_t launch_cg_sens(fbto_grid_s* g, const T* rho, const CgSet<T>& in, T* x, const T* invD, const T* f,
                          T* dobj, const T* Hsi, int step, int n_apply, int n_fn, double rtol, hipStream_t st,
                          int* nb_out) {
  TileChoice& t = g->tiles[sizeof(T) == 8 ? 1 : 0][0][MODE_SENSF];
  if (t.nblocks == 0) {
    t = choose_tile<T, 1, MODE_SENSF>(g->geo, g->n_cu, g->lds_per_cu, g->tile_override[0]);
    if (t.nblocks == 0) return hipErrorInvalidConfiguration;
  }
  if (t.nblocks > g->max_partials) return hipErrorInvalidValue;
  if (nb_out) *nb_out = t.nblocks;
  ApplyArgs<T> A{};
  A.g = g->geo;
  A.mask = g->mask;
  A.km = modal_of<T>(g);
  A.sp = g->simp;
  A.P = g->partials;
  A.maxp = g->max_partials;
  A.sc = g->sc;
  A.rho = rho;
  A.invD = invD;
  A.xi = in.x; A.ri = in.r; A.pi = in.p; A.si = in.s; A.wi = in.w;
  A.xo = x;
  A.dobj = dobj;
  A.Hsi = Hsi;
  A.fvec = f;
  A.step = step;
  A.n_apply = n_apply;
  A.n_fn = n_fn;
  A.rtol = rtol;
  A.bx = t.bx;
  A.by = t.by;
  A.tiles_x = t.tiles_x;
  A.tiles_y = t.tiles_y;
  A.slabs = t.slabs;
  A.dz = t.dz;
  A.nblocks = t.nblocks;
  A.per_xcd = (t.nblocks + 7) / 8;
  const int grid = A.per_xcd * 8;
  const int threads = zmarch_threads<MODE_SENSF>(t.bx, t.by);
  size_t lds = sens_lds_bytes<T>(t.bx, t.by);
  if (t.cap) lds = std::max(lds, (size_t)lds_for_block_cap(g->lds_per_cu, t.cap));
  hipLaunchKernelGGL((k_cg_sens<T>), dim3(grid), dim3(threads), lds, st, A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_fused(fbto_grid_s* g, const T* rho, const CgSet<T>& in, const CgSet<T>& out,
                           const T* invD, int nrhs, int step, int n_apply, int n_fn, double rtol,
                           hipStream_t st, int* nb_out) {
  ApplyArgs<T> A{};
  A.rho = rho;
  A.y = out.w;
  A.invD = invD;
  A.step = step;
  A.xi = in.x; A.ri = in.r; A.pi = in.p; A.si = in.s; A.wi = in.w;
  A.xo = out.x; A.ro = out.r; A.po = out.p; A.so = out.s;
  A.n_apply = n_apply;
  A.n_fn = n_fn;
  A.rtol = rtol;
  // r.r only for the tolerance test
  return rtol > 0.0 ? launch_apply_mode<T, MODE_CGF, true>(g, A, nrhs, st, nb_out)
                    : launch_apply_mode<T, MODE_CGF, false>(g, A, nrhs, st, nb_out);
}

template <typename T>
hipError_t launch_minres_fused(fbto_grid_s* g, const T* rho, int itn, const T* Y, const T* R1, const T* R2, T* R3,
                               const T* W, T* W2, T* x, T* Ynext, int n_apply, int n_kr, double damp,
                               hipStream_t st, int* nb_out) {
  ApplyArgs<T> A{};
  A.rho = rho;
  A.y = Ynext;
  A.step = itn;
  A.mY = Y; A.mR1 = R1; A.mR2 = R2; A.mW = W;
  A.mR3 = R3; A.mW2 = W2; A.mx = x;
  A.n_apply = n_apply;
  A.n_kr = n_kr;
  A.damp = damp;
  return launch_apply_mode<T, MODE_MRF>(g, A, 1, st, nb_out);
}

// ===========================================================================
// Jacobi diagonal: D = ke_diag * sum_{e at node} s_e (+ springs), 1 on fixed
// DOFs; stores its inverse per DOF.  Every diagonal entry of the unit-cube
// hex8 KE is the same number, so one sum per node serves all 3 DOFs.
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_diag(Geo G, const T* rho, T* invD, const uint8_t* mask, Simp sp, double ke_diag, int nspring,
           const int64_t* sdof, const T* sk) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (int)G.N) return;
  const int row = fdiv(n, G.nxn, G.rnxn);
  const int i = n - row * G.nxn;
  const int k = fdiv(row, G.nyn, G.rnyn);
  const int j = row - k * G.nyn;
  T acc = (T)0;
#pragma unroll
  for (int dz = -1; dz <= 0; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 0; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 0; ++dx) {
        const int ex = i + dx, ey = j + dy, ez = k + dz;
        const bool ok = ex >= 0 && ex < G.nx && ey >= 0 && ey < G.ny && ez >= 0 && ez < G.nz;
        const T rv = rho[ok ? ex + G.nx * (ey + G.ny * ez) : 0];
        acc += ok ? simp_s<T>(rv, sp) : (T)0;
      }
  const unsigned m = mask[n];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T d = (T)ke_diag * acc;
    for (int s = 0; s < nspring; ++s)
      if (sdof[s] == 3 * (int64_t)n + c) d += sk[s];
    if ((m >> c) & 1u) d = (T)1;
    invD[3 * n + c] = d > (T)0 ? (T)1 / d : (T)0;
  }
}

template <typename T>
hipError_t launch_diag(fbto_grid_s* g, const T* rho, T* invD, hipStream_t st) {
  if (g->dim == 2) return plane_diag<T>(g, rho, invD, st);
  hipLaunchKernelGGL((k_diag<T>), dim3(flat_grid(g->geo.N)), dim3(kVecBlock), 0, st, g->geo, rho, invD,
                     g->mask, g->simp, g->ke_diag, g->n_springs, g->spring_dof, spring_k_of<T>(g));
  return hipGetLastError();
}

// ===========================================================================
// Jacobi-PCG in the Chronopoulos-Gear arrangement: one reduction phase per
// step.  With z = D^-1 r and w = K z (from the CG-mode apply, which also
// leaves the partials of gamma = r.z, delta = w.z, r.r, max|r|):
//   beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev)
//   p = z + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,  z = D^-1 r
// (beta = 0, alpha = gamma / delta on the first step).  In exact arithmetic
// the iterates are those of the textbook recurrence.  The scalars are
// reduced from the partials in every block's prologue; gamma and alpha of
// the previous step are kept in the scalars, double-buffered by step parity
// (block 0 writes the slot no block of this kernel reads).  Convergence and
// breakdown are decided identically in every block.
// ===========================================================================
constexpr int kU = 8;

struct CgCnt {
  int apply;   // partials of the last apply (gamma, delta, r.r, max|r|)
  int fn;      // partials of f.f (the residual apply)
};

template <typename T, int NR>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_step(int64_t ndof, const T* x_in, T* x, T* r, const T* z_in, T* z_out, const T* w, T* p, T* s,
              const T* invD, const T* f, double* P, int maxp, CgCnt cn, int step, double rtol, Scalars* sc) {
  // first chunk of this thread's vector entries is loaded before the prologue
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i_first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool first = step == 0;
  // entries per thread and chunk: fewer with more load cases, so that the
  // chunk stays in registers
  constexpr int kU = NR <= 2 ? 8 : 4;
  T zv[kU][NR], wv[kU][NR], pv[kU][NR], sv[kU][NR], xv[kU][NR], rv[kU][NR], dv[kU];
  bool ok[kU];
  auto load_chunk = [&](int64_t i0) {
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int64_t i = i0 + k * stride;
      ok[k] = i < ndof;
      const int64_t ii = ok[k] ? i : 0;
      dv[k] = invD[ii];
#pragma unroll
      for (int R = 0; R < NR; ++R) {
        const int64_t o = R * ndof + ii;
        rv[k][R] = r[o];
        zv[k][R] = z_in ? z_in[o] : dv[k] * rv[k][R];
        wv[k][R] = w[o];
        xv[k][R] = x_in[o];
        pv[k][R] = first ? (T)0 : p[o];
        sv[k][R] = first ? (T)0 : s[o];
      }
    }
  };
  if (i_first < ndof) load_chunk(i_first);

  double pre[4 * NR];
  {
    const int par = step & 1;
    const double* src[4 * NR];
    int cnt[4 * NR];
#pragma unroll
    for (int R = 0; R < NR; ++R) {
      src[4 * R + 0] = pslot(P, P_RZ0 + par, R, maxp);
      src[4 * R + 1] = pslot(P, P_PQ0 + par, R, maxp);
      src[4 * R + 2] = pslot(P, P_RN0 + par, R, maxp);
      src[4 * R + 3] = pslot(P, P_FN, R, maxp);
      cnt[4 * R + 0] = cn.apply;
      cnt[4 * R + 1] = cn.apply;
      cnt[4 * R + 2] = cn.apply;
      cnt[4 * R + 3] = cn.fn;
    }
    reduce_parts<4 * NR, 0u, kVecBlock>(pre, src, cnt);
  }
  T al[NR], be[NR];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
#pragma unroll
  for (int R = 0; R < NR; ++R) {
    double alpha, beta;
    cg_coefficients(pre[4 * R], pre[4 * R + 1], pre[4 * R + 2], pre[4 * R + 3], R, step, rtol, sc, lead, alpha,
                    beta);
    al[R] = (T)alpha;
    be[R] = (T)beta;
  }

  double v[2 * NR + 1];
#pragma unroll
  for (int i = 0; i < 2 * NR + 1; ++i) v[i] = 0.0;
  for (int64_t i0 = i_first; i0 < ndof; i0 += kU * stride) {
    if (i0 != i_first) load_chunk(i0);
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      if (!ok[k]) continue;
      const int64_t i = i0 + k * stride;
#pragma unroll
      for (int R = 0; R < NR; ++R) {
        const int64_t o = R * ndof + i;
        const T pn = zv[k][R] + be[R] * pv[k][R];
        const T sn = wv[k][R] + be[R] * sv[k][R];
        const T xn = xv[k][R] + al[R] * pn;
        const T rn = rv[k][R] - al[R] * sn;
        p[o] = pn;
        s[o] = sn;
        x[o] = xn;
        r[o] = rn;
        if (z_out) z_out[o] = dv[k] * rn;
        v[2 * R] += (double)rn * (double)rn;
        v[2 * R + 1] = fmax(v[2 * R + 1], fabs((double)rn));
        if (f) v[2 * NR] += (double)f[o] * (double)xn;
      }
    }
  }
  double* dst[2 * NR + 1];
#pragma unroll
  for (int R = 0; R < NR; ++R) {
    dst[2 * R] = pslot(P, P_RNF, R, maxp);
    dst[2 * R + 1] = pslot(P, P_RIF, R, maxp);
  }
  dst[2 * NR] = pslot(P, P_DOT, 0, maxp);
  write_parts<2 * NR + 1, 0xAAAu, kVecBlock>(v, dst, blockIdx.x);
}

// Threads of the one-block finishing kernels: a block of 256 measured twice
// as fast as one of 1024 for the few thousand partials they reduce (fewer
// waves meet at each barrier).
constexpr int kFinishThreads = 256;

// Reduce the final residual norms into the scalars (slots RN1, RI1 with n_r
// partials, f.f from FN); with `info`, also write the outer-iteration record
// (compliance from DOT, projection results, gradient mean).
template <int NR>
__global__ void __launch_bounds__(kFinishThreads)
    k_pcg_finish(const double* P, int maxp, int n_r, int n_fn, Scalars* sc, double* info, int n_dot, int n_e,
                 int n_gsum, int64_t E) {
  double v[3 * NR + 4];
  const double* src[3 * NR + 4];
  int cnt[3 * NR + 4];
#pragma unroll
  for (int R = 0; R < NR; ++R) {
    src[3 * R + 0] = pslot(P, P_RNF, R, maxp);
    src[3 * R + 1] = pslot(P, P_RIF, R, maxp);
    src[3 * R + 2] = pslot(P, P_FN, R, maxp);
    cnt[3 * R + 0] = n_r;
    cnt[3 * R + 1] = n_r;
    cnt[3 * R + 2] = n_fn;
  }
  src[3 * NR + 0] = pslot(P, P_DOT, 0, maxp);
  src[3 * NR + 1] = pslot(P, P_VOL, 0, maxp);
  src[3 * NR + 2] = pslot(P, P_DX, 0, maxp);
  src[3 * NR + 3] = pslot(P, P_GSUM, 0, maxp);
  cnt[3 * NR + 0] = info ? n_dot : 0;
  cnt[3 * NR + 1] = info ? n_e : 0;
  cnt[3 * NR + 2] = info ? n_e : 0;
  cnt[3 * NR + 3] = info ? n_gsum : 0;
  // the scalars read by the lead thread are loaded before the reduction,
  // so their latency overlaps it
  double st_in[NR], proj_status = 0.0, lam = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int R = 0; R < NR; ++R) st_in[R] = sc->status[R];
    proj_status = sc->proj_status;
    lam = sc->lam;
  }
  // max-reduced entries: |r|_inf of each RHS (3 R + 1, R < NR) and
  // |dx|_inf (3 NR + 2); the rest are sums
  constexpr unsigned MM = rinf_mask(NR) | (1u << (3 * NR + 2));
  reduce_parts<3 * NR + 4, MM, kFinishThreads>(v, src, cnt);
  if (threadIdx.x == 0) {
    double rinf = 0.0, rrel = 0.0, status = 0.0;
#pragma unroll
    for (int R = 0; R < NR; ++R) {
      const double rn = sqrt(v[3 * R]), fnrm = sqrt(v[3 * R + 2]);
      sc->rnorm2[R] = rn;
      sc->rinf[R] = v[3 * R + 1];
      sc->fnorm2[R] = fnrm;
      double stR = st_in[R];
      if (!isfinite(v[3 * R]) && stR == 0.0) {
        stR = (double)FBTO_ERR_NONFINITE;
        sc->status[R] = stR;
      }
      rinf = fmax(rinf, v[3 * R + 1]);
      rrel = fmax(rrel, fnrm > 0.0 ? rn / fnrm : rn);
      if (stR != 0.0) status = stR;
    }
    if (info) {
      // the projection's status: non-finite values take precedence, an
      // inexact projection (FBTO_INEXACT) only reports when the solve had none
      if (proj_status > 0.0 && (status == 0.0 || proj_status == (double)FBTO_ERR_NONFINITE)) status = proj_status;
      sc->dot[0] = v[3 * NR];
      info[FBTO_OI_COMPLIANCE] = v[3 * NR];
      info[FBTO_OI_DX_INF] = v[3 * NR + 2];
      info[FBTO_OI_R_INF] = rinf;
      info[FBTO_OI_LAMBDA] = lam;
      info[FBTO_OI_VOLUME] = v[3 * NR + 1];
      info[FBTO_OI_RREL] = rrel;
      info[FBTO_OI_STATUS] = status;
      info[FBTO_OI_GRAD_MEAN] = v[3 * NR + 3] / (double)E;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_relax_update(int64_t ndof, int nrhs, T* u, const T* r, const T* invD, T omega, int use_diag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ndof;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T w = use_diag ? omega * invD[i] : omega;
    for (int R = 0; R < nrhs; ++R) u[R * ndof + i] += w * r[R * ndof + i];
  }
}

#define FBTO_NR_DISPATCH(nrhs, CALL) \
  switch (nrhs) {                    \
    case 1: { constexpr int NR = 1; CALL; break; } \
    case 2: { constexpr int NR = 2; CALL; break; } \
    case 3: { constexpr int NR = 3; CALL; break; } \
    default: { constexpr int NR = 4; CALL; break; } \
  }

template <typename T>
hipError_t launch_cg_step(fbto_grid_s* g, const T* x_in, T* x, T* r, const T* z_in, T* z_out, const T* w, T* p,
                          T* s, const T* invD, const T* f, int nrhs, int n_apply, int n_fn, int step,
                          double rtol, hipStream_t st, int* nb_out) {
  const int nb = vec_blocks(g->geo.ndof);
  if (nb_out) *nb_out = nb;
  const CgCnt cn{n_apply, n_fn};
  FBTO_NR_DISPATCH(nrhs, hipLaunchKernelGGL((k_cg_step<T, NR>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof,
                                            x_in, x, r, z_in, z_out, w, p, s, invD, f, g->partials,
                                            g->max_partials, cn, step, rtol, g->sc));
  return hipGetLastError();
}
hipError_t launch_pcg_finish(fbto_grid_s* g, int nrhs, int n_r, int n_fn, double* info, int n_dot, int n_e,
                             int n_gsum, hipStream_t st) {
  FBTO_NR_DISPATCH(nrhs, hipLaunchKernelGGL((k_pcg_finish<NR>), dim3(1), dim3(kFinishThreads), 0, st,
                                            (const double*)g->partials, g->max_partials, n_r, n_fn, g->sc, info,
                                            n_dot, n_e, n_gsum, g->geo.E));
  return hipGetLastError();
}
template <typename T>
hipError_t launch_relax_update(fbto_grid_s* g, T* u, const T* r, const T* invD, int nrhs,
                               double omega, int use_diag, hipStream_t st) {
  const int nb = vec_blocks(g->geo.ndof);
  hipLaunchKernelGGL((k_relax_update<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, nrhs, u, r,
                     invD, (T)omega, use_diag);
  return hipGetLastError();
}

// ===========================================================================
// Krylov step of Alg. 3 (Eq. LSP, beta = 1): the new iterate minimises the
// residual over u + span{r, K r, ..., K^D r}.  It is computed by the MINRES
// recurrence (Lanczos vectors and Givens rotations, as in Paige and
// Saunders), D + 1 iterations from u.  Iteration itn (1 .. D + 1) is one
// CG-mode apply Y = K R2 (partials <R1, R2>, <Y, R2>) and one pass of this
// kernel, which
//   - reduces beta = ||R2|| (the previous pass's partials) and, from the
//     apply's partials, alpha = <v, K v - (beta/oldb) R1> with v = R2/beta;
//   - finishes iteration itn - 1: its Givens rotation needs beta, then
//     w = (v' - oldeps w'' - delta w') / gamma, x += damp * phi * w, where
//     v' = R1 / oldb is that iteration's Lanczos vector;
//   - forms the next Lanczos vector y = K v - (beta/oldb) R1 - (alpha/beta) R2
//     into R1's buffer and leaves ||y||^2 as partials.
// Pass 0 only leaves ||R2||^2 (R2 = f - K u); pass D + 2 only finishes
// iteration D + 1.  Every block runs the scalar recurrence on the same
// reduced values in the same order; block 0 keeps its state for the next
// pass.  The caller rotates the buffers: R1 <- R2, R2 <- the buffer y went
// to, W <- the buffer w went to (W2), W2 <- W.  `damp` scales the step
// (Alg. 3's beta_k).
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_minres(int64_t n, int itn, int last, const T* Y, T* R1, const T* R2, T* W2, const T* W, T* x,
             double* P, int maxp, int n_apply, int n_prev, Scalars* sc, double damp) {
  double beta = 0.0;
  if (itn >= 1) {
    double v[1];
    const double* src[1] = {pslot(P, P_KRN0 + ((itn - 1) & 1), 0, maxp)};
    const int cnt[1] = {n_prev};
    reduce_parts<1, 0u>(v, src, cnt);
    beta = sqrt(fmax(v[0], 0.0));
  }
  const bool lanczos = itn >= 1 && itn < last;
  const bool finish = itn >= 2;
  double yr2 = 0.0, r12 = 0.0;
  if (lanczos) {
    double v[2];
    const double* src[2] = {pslot(P, P_RZ0 + (itn & 1), 0, maxp), pslot(P, P_PQ0 + (itn & 1), 0, maxp)};
    const int cnt[2] = {n_apply, n_apply};
    reduce_parts<2, 0u>(v, src, cnt);
    r12 = v[0];
    yr2 = v[1];
  }
  // state carried from the previous pass
  double oldb = 0.0, alfa_prev = 0.0, dbar = 0.0, epsln = 0.0, phibar = beta, cs = -1.0, sn = 0.0;
  if (itn >= 2) {
    const double* k = sc->kr[(itn + 1) & 1];  // written by pass itn - 1
    oldb = k[0];
    alfa_prev = k[1];
    dbar = k[2];
    epsln = k[3];
    phibar = k[4];
    cs = k[5];
    sn = k[6];
  }
  // Givens rotation of iteration itn - 1
  double oldeps = 0.0, delta = 0.0, gamma = 1.0, phi = 0.0;
  if (finish) {
    oldeps = epsln;
    delta = cs * dbar + sn * alfa_prev;
    const double gbar = sn * dbar - cs * alfa_prev;
    epsln = sn * beta;
    dbar = -cs * beta;
    gamma = fmax(sqrt(gbar * gbar + beta * beta), 1e-300);
    cs = gbar / gamma;
    sn = beta / gamma;
    phi = cs * phibar;
    phibar = sn * phibar;
  }
  // Lanczos step of iteration itn.  Norms below kTinyNorm mean the Krylov
  // space is exhausted (the residual is zero to rounding): the
  // reciprocals are then taken as 0, so every further vector and update is
  // 0 rather than 0 * inf in FP32.
  const double s = beta > kTinyNorm ? 1.0 / beta : 0.0;
  const double c1 = (itn >= 2 && oldb > kTinyNorm) ? beta / oldb : 0.0;
  const double alfa = lanczos ? s * (s * yr2 - c1 * r12) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && itn >= 1) {
    double* k = sc->kr[itn & 1];
    k[0] = beta;
    k[1] = alfa;
    k[2] = dbar;
    k[3] = epsln;
    k[4] = phibar;
    k[5] = cs;
    k[6] = sn;
  }
  const int j = itn - 1;  // the iteration finished here
  const T inv_oldb = (T)(oldb > kTinyNorm ? 1.0 / oldb : 0.0);
  const T wc1 = (T)oldeps, wc2 = (T)delta, inv_gamma = (T)(gamma > kTinyNorm ? 1.0 / gamma : 0.0);
  const T step = (T)(damp * phi);
  const T ts = (T)s, tc1 = (T)c1, ta = (T)(alfa * s);
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T r1 = R1[i];
    if (finish) {
      const T w1v = W[i], w2v = W2[i];  // w of iterations j - 1 and j - 2 (zero before the first)
      const T wp = j >= 2 ? w1v : (T)0, wpp = j >= 3 ? w2v : (T)0;
      const T wn = (r1 * inv_oldb - wc1 * wpp - wc2 * wp) * inv_gamma;
      W2[i] = wn;
      x[i] += step * wn;
    }
    if (itn == 0) {
      const T r2 = R2[i];
      acc += (double)r2 * (double)r2;
    } else if (lanczos) {
      const T r1m = itn >= 2 ? r1 : (T)0;  // R1 holds no vector yet on the first iteration
      const T yn = ts * Y[i] - tc1 * r1m - ta * R2[i];
      R1[i] = yn;
      acc += (double)yn * (double)yn;
    }
  }
  if (itn == 0 || lanczos) {
    double v[1] = {acc};
    double* dst[1] = {pslot(P, P_KRN0 + (itn & 1), 0, maxp)};
    write_parts<1, 0u>(v, dst, blockIdx.x);
  }
}

template <typename T>
hipError_t launch_minres(fbto_grid_s* g, int itn, int last, const T* Y, T* R1, const T* R2, T* W2, const T* W,
                         T* x, int n_apply, int n_prev, double damp, hipStream_t st, int* nb_out) {
  const int nb = vec_blocks(g->geo.ndof);
  if (nb > g->max_partials || n_apply > g->max_partials) return hipErrorInvalidValue;
  if (nb_out) *nb_out = nb;
  hipLaunchKernelGGL((k_minres<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, itn, last, Y, R1, R2, W2, W,
                     x, g->partials, g->max_partials, n_apply, n_prev, g->sc, damp);
  return hipGetLastError();
}

// ===========================================================================
// Sensitivity: dobj_e = -ds_e sum_r lam_{r,e}^T KE u_{r,e} (times 1/Hs_e when
// Hsi is given, which turns the filter transpose into a plain weighted sum),
// element strains recomputed from the nodal vectors (one element per thread).
// ===========================================================================
template <typename T>
__device__ __forceinline__ void gather_elem(const Geo& G, const T* v, const uint8_t* mask, int ex,
                                            int ey, int ez, T (&ue)[8][3]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int n = (ex + (a & 1)) + G.nxn * ((ey + ((a >> 1) & 1)) + G.nyn * (ez + (a >> 2)));
    const unsigned m = mask[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T x = v[3 * n + c];
      ue[a][c] = ((m >> c) & 1u) ? (T)0 : x;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_sens(Geo G, const T* rho, const T* u, const T* lam, int nrhs, T* dobj, const uint8_t* mask,
           Modal<T> km, Simp sp, const T* Hsi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int)G.E) return;
  const int row = fdiv(e, G.nx, G.rnx);
  const int ex = e - row * G.nx;
  const int ez = fdiv(row, G.ny, G.rny);
  const int ey = row - ez * G.ny;
  double acc = 0.0;
  for (int R = 0; R < nrhs; ++R) {
    T ue[8][3];
    gather_elem<T>(G, u + R * G.ndof, mask, ex, ey, ez, ue);
    if (lam) {
      T le[8][3];
      gather_elem<T>(G, lam + R * G.ndof, mask, ex, ey, ez, le);
      acc += elem_bilinear<T>(le, ue, km);
    } else {
      acc += elem_bilinear<T>(ue, ue, km);
    }
  }
  double val = -(double)simp_ds<T>(rho[e], sp) * acc;
  if (Hsi) val *= (double)Hsi[e];
  dobj[e] = (T)val;
}

template <typename T>
hipError_t launch_sens(fbto_grid_s* g, const T* rho, const T* u, const T* lam, int nrhs, T* dobj,
                       const T* Hsi, hipStream_t st) {
  if (g->dim == 2) return plane_sens<T>(g, rho, u, lam, nrhs, dobj, Hsi, st);
  hipLaunchKernelGGL((k_sens<T>), dim3(flat_grid(g->geo.E)), dim3(kVecBlock), 0, st, g->geo, rho, u, lam, nrhs,
                     dobj, g->mask, modal_of<T>(g), g->simp, Hsi);
  return hipGetLastError();
}

// partials of sum_r a_r . b_r (vectors of length ndof) into slot DOT
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_dot(int64_t n, int nrhs, const T* a, const T* b, double* P, int maxp) {
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int R = 0; R < nrhs; ++R) v[0] += (double)a[R * n + i] * (double)b[R * n + i];
  }
  double* dst[1] = {pslot(P, P_DOT, 0, maxp)};
  write_parts<1, 0u>(v, dst, blockIdx.x);
}

__global__ void __launch_bounds__(kVecBlock) k_dot_store(const double* P, int maxp, int nb, double* out) {
  double v[1];
  const double* src[1] = {pslot(P, P_DOT, 0, maxp)};
  const int cnt[1] = {nb};
  reduce_parts<1, 0u>(v, src, cnt);
  if (threadIdx.x == 0) out[0] = v[0];
}

template <typename T>
hipError_t launch_dot(fbto_grid_s* g, const T* a, const T* b, int nrhs, hipStream_t st) {
  const int nb = vec_blocks(g->geo.ndof);
  hipLaunchKernelGGL((k_dot<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, nrhs, a, b, g->partials,
                     g->max_partials);
  return hipGetLastError();
}
hipError_t launch_dot_store(fbto_grid_s* g, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_store, dim3(1), dim3(kVecBlock), 0, st, (const double*)g->partials,
                     g->max_partials, vec_blocks(g->geo.ndof), out);
  return hipGetLastError();
}

// ===========================================================================
// Linear cone filter: gather over the stencil (offsets with r - |d| > 0).
//   FWD:    out_e = sum_o w_o in_{e+o} / Hs_e
//   TRANS:  out_j = sum_o w_o in_{j+o} / Hs_{j+o}
//   SUM:    out_j = sum_o w_o in_{j+o}      (input already divided by Hs)
// One element per thread; want_sum: partials of sum(out) into slot GSUM.
// ===========================================================================
enum { FILT_FWD = 0, FILT_TRANS = 1, FILT_SUM = 2 };

template <typename T, int R>
struct StencilW {
  T w[(2 * R + 1) * (2 * R + 1) * (2 * R + 1)];   // weight of offset (dx, dy, dz), x fastest
};

template <typename T, int R>
__global__ void __launch_bounds__(kVecBlock)
    k_filter(Geo G, int kind, const T* in, T* out, const T* Hsi, StencilW<T, R> W, int want_sum,
             double* P, int maxp) {
  constexpr int D = 2 * R + 1;
  double v[1] = {0.0};
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (int)G.E; e += gridDim.x * blockDim.x) {
    const int row = fdiv(e, G.nx, G.rnx);
    const int ex = e - row * G.nx;
    const int ez = fdiv(row, G.ny, G.rny);
    const int ey = row - ez * G.ny;
    T acc = (T)0;
#pragma unroll
    for (int dz = -R; dz <= R; ++dz)
#pragma unroll
      for (int dy = -R; dy <= R; ++dy)
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
          const int jx = ex + dx, jy = ey + dy, jz = ez + dz;
          const bool ok = jx >= 0 && jx < G.nx && jy >= 0 && jy < G.ny && jz >= 0 && jz < G.nz;
          const int j = ok ? e + dx + G.nx * (dy + G.ny * dz) : e;
          const T wv = ok ? W.w[(dx + R) + D * ((dy + R) + D * (dz + R))] : (T)0;
          const T x = kind == FILT_TRANS ? in[j] * Hsi[j] : in[j];
          acc += wv * x;
        }
    const T res = kind == FILT_FWD ? acc * Hsi[e] : acc;
    out[e] = res;
    v[0] += (double)res;
  }
  if (want_sum) {
    double* dst[1] = {pslot(P, P_GSUM, 0, maxp)};
    write_parts<1, 0u>(v, dst, blockIdx.x);
  }
}

// Density filter for R <= 1 by z-march: a thread owns element column
// (ex, ey) of a z-slab and keeps the 2R+1 planes of its (2R+1)^2
// neighbourhood in registers, so a slab of dz layers reads each input
// (2R+1)^2 (dz + 2R) / dz times instead of (2R+1)^3.  Out-of-grid
// neighbours load as 0 (the stencil is truncated at the boundary).
// The evaluation of one search pass at lam for one entry: f(lam) and the
// classification of the entry just right (+) and just left (-) of lam, plus
// the nearest breakpoints on either side (slots of proj_decide).
// (Written with selects only: branches here let the compiler pick v[9] or
// v[10] by a dynamic index, which puts the array in scratch memory.)
__device__ __forceinline__ void proj_eval(double (&v)[11], double yd, double lam, double lo, double hi) {
  const double t = yd - lam;
  v[0] += fmin(fmax(t, lo), hi);
  const bool rU = t > hi, rL = !rU && t <= lo, rA = !rU && !rL;   // just right of lambda
  v[3] += rU ? 1.0 : 0.0;
  v[4] += rL ? 1.0 : 0.0;
  v[1] += rA ? 1.0 : 0.0;
  v[2] += rA ? yd : 0.0;
  const bool lU = t >= hi, lL = !lU && t < lo, lA = !lU && !lL;   // just left of lambda
  v[7] += lU ? 1.0 : 0.0;
  v[8] += lL ? 1.0 : 0.0;
  v[5] += lA ? 1.0 : 0.0;
  v[6] += lA ? yd : 0.0;
  const double b1 = yd - lo, b2 = yd - hi;
  v[9] = fmax(v[9], fmax(b1 < lam ? b1 : -INFINITY, b2 < lam ? b2 : -INFINITY));
  v[10] = fmax(v[10], fmax(b1 > lam ? -b1 : -INFINITY, b2 > lam ? -b2 : -INFINITY));
}
__device__ __forceinline__ void proj_eval_init(double (&v)[11]) {
#pragma unroll
  for (int i = 0; i < 11; ++i) v[i] = 0.0;
  v[9] = -INFINITY;
  v[10] = -INFINITY;
}

// The step's partials of one block in one reduction: the projection's seed
// (sum clamp(y), max y, #interior: slots S0, YMAX, NACT) and the evaluation
// at the warm-start multiplier (evaluation set 0, the next 11 slots).
static_assert(P_YMAX == P_S0 + 1 && P_NACT == P_S0 + 2 && P_E0 == P_S0 + 3, "seed and set 0 are consecutive slots");
template <int NTHR>
__device__ __forceinline__ void step_parts(double (&v3)[3], double (&ev)[11], double* P, int maxp) {
  double w[14];
  double* dst[14];
#pragma unroll
  for (int i = 0; i < 14; ++i) {
    w[i] = i < 3 ? v3[i] : ev[i - 3];
    dst[i] = pslot(P, P_S0 + i, 0, maxp);
  }
  // max-reduced: max y (1) and the nearest breakpoints (3 + 9, 3 + 10)
  write_parts<14, 0x3002u, NTHR>(w, dst, blockIdx.x);
}

constexpr int kFiltBX = 64, kFiltBY = 4, kFiltDZ = 4;

// The gradient step fused into the plain-sum filter (the transposed filter
// after the 1/Hs fold): each filtered value g_e gives y_e = x_e -
// half_alpha (g_e - mean), with the projection's seed and its evaluation at
// the warm-start multiplier, as k_step forms them.  The mean comes from the
// partials in slot GSUM (the sensitivity kernel's sum of the unfiltered
// gradient, equal to the filtered one's since the weights are symmetric).
template <typename T>
struct FiltStep {
  const T* x;
  T* y;
  double half_alpha;
  int mean_project, nb_sum;
  double lo, hi;
  const Scalars* sc;
};

// Thread geometry of the z-march filter: tile b of 64 x 4 element columns
// and kFiltDZ layers; the thread's column (ex, ey) and output layers
// [z0, z1).
struct FiltPos {
  int ex, ey, z0, z1;
  bool col;  // the column lies in the grid
};
__device__ __forceinline__ FiltPos filt_pos(const Geo& G, int tiles_x, int tiles_y) {
  FiltPos q;
  const int tx = threadIdx.x % kFiltBX, ty = threadIdx.x / kFiltBX;
  const int b = blockIdx.x;
  const int bx = b % tiles_x, t2 = b / tiles_x, by = t2 % tiles_y, bz = t2 / tiles_y;
  q.ex = bx * kFiltBX + tx;
  q.ey = by * kFiltBY + ty;
  q.z0 = bz * kFiltDZ;
  q.z1 = min(q.z0 + kFiltDZ, G.nz);
  q.col = q.ex < G.nx && q.ey < G.ny;
  return q;
}

// Every value the thread's outputs read (its kFiltDZ layers and R halo
// planes on each side, (2R + 1)^2 columns), loaded up front: one memory
// latency per block.  Values outside the grid are 0.  trans: each value
// times Hsi.  proj: each value v becomes the design value clamp(v - lam,
// lo, hi) (in FP64, rounded to T, as the projection's final pass writes it).
template <typename T, int R>
__device__ __forceinline__ void filt_window(const Geo& G, const FiltPos& q, const T* in, const T* Hsi, bool trans,
                                            T (&win)[kFiltDZ + 2 * R][2 * R + 1][2 * R + 1], bool proj = false,
                                            double lam = 0.0, double lo = 0.0, double hi = 0.0) {
  constexpr int D = 2 * R + 1;
  const int plane = G.nx * G.ny;
  bool okxy[D][D];
  int offxy[D][D];
#pragma unroll
  for (int dy = 0; dy < D; ++dy)
#pragma unroll
    for (int dx = 0; dx < D; ++dx) {
      const int jx = q.ex + dx - R, jy = q.ey + dy - R;
      okxy[dy][dx] = q.col && jx >= 0 && jx < G.nx && jy >= 0 && jy < G.ny;
      offxy[dy][dx] = okxy[dy][dx] ? jx + G.nx * jy : 0;
    }
#pragma unroll
  for (int p = 0; p < kFiltDZ + 2 * R; ++p) {
    const int jz = q.z0 - R + p;
    const bool zok = jz >= 0 && jz < G.nz;
#pragma unroll
    for (int dy = 0; dy < D; ++dy)
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        const bool ok = okxy[dy][dx] && zok;
        const int j = ok ? offxy[dy][dx] + jz * plane : 0;
        T v = in[j];
        if (trans) v *= Hsi[j];
        if (proj) v = (T)fmin(fmax((double)v - lam, lo), hi);
        win[p][dy][dx] = ok ? v : (T)0;
      }
  }
}

// The stencil sum of output layer l of the window.
template <typename T, int R>
__device__ __forceinline__ T filt_sum(const StencilW<T, R>& W, const T (&win)[kFiltDZ + 2 * R][2 * R + 1][2 * R + 1],
                                      int l) {
  constexpr int D = 2 * R + 1;
  T acc = (T)0;
#pragma unroll
  for (int dz = 0; dz < D; ++dz)
#pragma unroll
    for (int dy = 0; dy < D; ++dy)
#pragma unroll
      for (int dx = 0; dx < D; ++dx) acc += W.w[dx + D * (dy + D * dz)] * win[l + dz][dy][dx];
  return acc;
}

template <typename T, int R, bool STEP>
__global__ void __launch_bounds__(kFiltBX * kFiltBY)
    k_filter_z(Geo G, int kind, const T* in, T* out, const T* Hsi, StencilW<T, R> W, int want_sum,
               double* P, int maxp, int tiles_x, int tiles_y, FiltStep<T> S) {
  const FiltPos q = filt_pos(G, tiles_x, tiles_y);
  T win[kFiltDZ + 2 * R][2 * R + 1][2 * R + 1];  // [plane][dy][dx]
  filt_window<T, R>(G, q, in, Hsi, kind == FILT_TRANS, win);
  // step: the design values of the slab's outputs, and the mean of g
  T xv[kFiltDZ];
  double mean = 0.0, lam_w = 0.0;
  if constexpr (STEP) {
#pragma unroll
    for (int l = 0; l < kFiltDZ; ++l) {
      const int ez = q.z0 + l;
      xv[l] = S.x[(q.col && ez < q.z1) ? q.ex + G.nx * (q.ey + G.ny * ez) : 0];
    }
    lam_w = S.sc->lam_prev;
    if (S.mean_project) {
      double v[1];
      const double* src[1] = {pslot(P, P_GSUM, 0, maxp)};
      const int cnt[1] = {S.nb_sum};
      reduce_parts<1, 0u, kFiltBX * kFiltBY>(v, src, cnt);
      mean = v[0] / (double)G.E;
    }
  }
  double vs[1] = {0.0};
  double v3[3] = {0.0, -INFINITY, 0.0};  // step: sum clamp(y), max y, #interior
  double ev[11];                         // step: evaluation at lam_w
  proj_eval_init(ev);
#pragma unroll
  for (int l = 0; l < kFiltDZ; ++l) {
    const int ez = q.z0 + l;
    const T acc = filt_sum<T, R>(W, win, l);
    if (q.col && ez < q.z1) {
      const int e = q.ex + G.nx * (q.ey + G.ny * ez);
      const T res = kind == FILT_FWD ? acc * Hsi[e] : acc;
      if constexpr (STEP) {
        const T ye = (T)((double)xv[l] - S.half_alpha * ((double)res - mean));
        S.y[e] = ye;
        const double yd = (double)ye;
        v3[0] += fmin(fmax(yd, S.lo), S.hi);
        v3[1] = fmax(v3[1], yd);
        v3[2] += (yd > S.lo && yd < S.hi) ? 1.0 : 0.0;
        proj_eval(ev, yd, lam_w, S.lo, S.hi);
      } else {
        out[e] = res;
        vs[0] += (double)res;
      }
    }
  }
  if constexpr (STEP) {
    step_parts<kFiltBX * kFiltBY>(v3, ev, P, maxp);
  } else if (want_sum) {
    double* dst[1] = {pslot(P, P_GSUM, 0, maxp)};
    write_parts<1, 0u>(vs, dst, blockIdx.x);
  }
}

// Generic gather for wide stencils (R > 2): offsets and weights from memory.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_filter_wide(Geo G, int kind, const T* in, T* out, const T* Hsi, int nst, const int* off,
                  const T* w, int want_sum, double* P, int maxp) {
  double v[1] = {0.0};
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (int)G.E; e += gridDim.x * blockDim.x) {
    const int row = fdiv(e, G.nx, G.rnx);
    const int ex = e - row * G.nx;
    const int ez = fdiv(row, G.ny, G.rny);
    const int ey = row - ez * G.ny;
    T acc = (T)0;
    for (int o = 0; o < nst; ++o) {
      const int jx = ex + off[3 * o], jy = ey + off[3 * o + 1], jz = ez + off[3 * o + 2];
      if (jx < 0 || jx >= G.nx || jy < 0 || jy >= G.ny || jz < 0 || jz >= G.nz) continue;
      const int j = jx + G.nx * (jy + G.ny * jz);
      acc += w[o] * (kind == FILT_TRANS ? in[j] * Hsi[j] : in[j]);
    }
    const T res = kind == FILT_FWD ? acc * Hsi[e] : acc;
    out[e] = res;
    v[0] += (double)res;
  }
  if (want_sum) {
    double* dst[1] = {pslot(P, P_GSUM, 0, maxp)};
    write_parts<1, 0u>(v, dst, blockIdx.x);
  }
}

template <typename T>
__global__ void k_hs(Geo G, T* Hsi, int nst, const int* off, const T* w) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (int)G.E; e += gridDim.x * blockDim.x) {
    const int row = fdiv(e, G.nx, G.rnx);
    const int ex = e - row * G.nx;
    const int ez = fdiv(row, G.ny, G.rny);
    const int ey = row - ez * G.ny;
    double acc = 0.0;
    for (int o = 0; o < nst; ++o) {
      const int jx = ex + off[3 * o], jy = ey + off[3 * o + 1], jz = ez + off[3 * o + 2];
      if (jx < 0 || jx >= G.nx || jy < 0 || jy >= G.ny || jz < 0 || jz >= G.nz) continue;
      acc += (double)w[o];
    }
    Hsi[e] = (T)(1.0 / acc);
  }
}

template <typename T, int R>
static StencilW<T, R> stencil_weights(double r) {
  StencilW<T, R> W{};
  constexpr int D = 2 * R + 1;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        double w = r - std::sqrt((double)(dx * dx + dy * dy + dz * dz));
        if (r <= 1.0) w = (dx == 0 && dy == 0 && dz == 0) ? 1.0 : 0.0;
        W.w[(dx + R) + D * ((dy + R) + D * (dz + R))] = (T)(w > 0.0 ? w : 0.0);
      }
  return W;
}

template <typename T>
hipError_t launch_filter(fbto_grid_s* g, int kind, const T* in, T* out, int want_sum, hipStream_t st) {
  Vecs& V = vecs_of<T>(g);
  if (g->dim == 2)  // separable Gaussian: two passes through the step buffer y (unused while filtering)
    return plane_filter<T>(g, kind, in, out, (T*)V.y, (const T*)V.Hs, want_sum, st);
  // with a sum, the grid is capped so that its partials stay few
  const int nb = want_sum ? vec_blocks(g->geo.E) : flat_grid(g->geo.E);
  const double r = g->desc.filter_radius;
  const int R = r > 1.0 ? (int)std::ceil(r) - 1 : 0;
  const T* Hsi = (const T*)V.Hs;
  const Geo& G = g->geo;
  const int tiles_x = (G.nx + kFiltBX - 1) / kFiltBX, tiles_y = (G.ny + kFiltBY - 1) / kFiltBY;
  const int64_t nbz = (int64_t)tiles_x * tiles_y * ((G.nz + kFiltDZ - 1) / kFiltDZ);
  if (R <= 1 && nbz <= g->max_partials) {
    if (want_sum) g->n_gsum = (int)nbz;
    if (R == 0)
      hipLaunchKernelGGL((k_filter_z<T, 0, false>), dim3(nbz), dim3(kFiltBX * kFiltBY), 0, st, G, kind, in, out,
                         Hsi, stencil_weights<T, 0>(r), want_sum, g->partials, g->max_partials, tiles_x, tiles_y,
                         FiltStep<T>{});
    else
      hipLaunchKernelGGL((k_filter_z<T, 1, false>), dim3(nbz), dim3(kFiltBX * kFiltBY), 0, st, G, kind, in, out,
                         Hsi, stencil_weights<T, 1>(r), want_sum, g->partials, g->max_partials, tiles_x, tiles_y,
                         FiltStep<T>{});
    return hipGetLastError();
  }
  if (want_sum) g->n_gsum = nb;
  if (R <= 1)
    hipLaunchKernelGGL((k_filter<T, 1>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, kind, in, out, Hsi,
                       stencil_weights<T, 1>(r), want_sum, g->partials, g->max_partials);
  else if (R == 2)
    hipLaunchKernelGGL((k_filter<T, 2>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, kind, in, out, Hsi,
                       stencil_weights<T, 2>(r), want_sum, g->partials, g->max_partials);
  else
    hipLaunchKernelGGL((k_filter_wide<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, kind, in, out, Hsi,
                       g->n_stencil, (const int*)g->stencil_off, stencil_w_of<T>(g), want_sum, g->partials,
                       g->max_partials);
  return hipGetLastError();
}

// Whether the grid's filter runs as the z-march filter (voxel grid, stencil
// of radius R <= 1, its tiles within the partial slots): the variants fused
// with the step and with the final projection pass need it.
bool zmarch_filter(const fbto_grid_s* g) {
  if (g->dim == 2) return false;
  const double r = g->desc.filter_radius;
  const int R = r > 1.0 ? (int)std::ceil(r) - 1 : 0;
  const Geo& G = g->geo;
  const int64_t tiles_x = (G.nx + kFiltBX - 1) / kFiltBX, tiles_y = (G.ny + kFiltBY - 1) / kFiltBY;
  const int64_t nbz = tiles_x * tiles_y * ((G.nz + kFiltDZ - 1) / kFiltDZ);
  return R <= 1 && nbz <= g->max_partials;
}

template <typename T>
hipError_t launch_filter_step(fbto_grid_s* g, const T* ge, const T* x, T* y, double half_alpha,
                              int mean_project, int nb_sum, double lo, double hi, hipStream_t st,
                              int* nb_seed) {
  if (!zmarch_filter(g)) return hipErrorNotSupported;
  const double r = g->desc.filter_radius;
  const int R = r > 1.0 ? (int)std::ceil(r) - 1 : 0;
  const Geo& G = g->geo;
  const int tiles_x = (G.nx + kFiltBX - 1) / kFiltBX, tiles_y = (G.ny + kFiltBY - 1) / kFiltBY;
  const int64_t nbz = (int64_t)tiles_x * tiles_y * ((G.nz + kFiltDZ - 1) / kFiltDZ);
  if (mean_project && (nb_sum < 1 || nb_sum > g->max_partials)) return hipErrorInvalidValue;
  const FiltStep<T> S{x, y, half_alpha, mean_project, nb_sum, lo, hi, (const Scalars*)g->sc};
  const T* Hsi = (const T*)vecs_of<T>(g).Hs;  // not read by the plain sum
  if (R == 0)
    hipLaunchKernelGGL((k_filter_z<T, 0, true>), dim3(nbz), dim3(kFiltBX * kFiltBY), 0, st, G, (int)FILT_SUM, ge,
                       (T*)nullptr, Hsi, stencil_weights<T, 0>(r), 0, g->partials, g->max_partials, tiles_x,
                       tiles_y, S);
  else
    hipLaunchKernelGGL((k_filter_z<T, 1, true>), dim3(nbz), dim3(kFiltBX * kFiltBY), 0, st, G, (int)FILT_SUM, ge,
                       (T*)nullptr, Hsi, stencil_weights<T, 1>(r), 0, g->partials, g->max_partials, tiles_x,
                       tiles_y, S);
  *nb_seed = (int)nbz;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hs(fbto_grid_s* g, T* Hs, hipStream_t st) {
  if (g->dim == 2) return plane_hs<T>(g, Hs, st);
  hipLaunchKernelGGL((k_hs<T>), dim3(flat_grid(g->geo.E)), dim3(kVecBlock), 0, st, g->geo, Hs, g->n_stencil,
                     (const int*)g->stencil_off, stencil_w_of<T>(g));
  return hipGetLastError();
}
template hipError_t launch_hs<double>(fbto_grid_s*, double*, hipStream_t);
template hipError_t launch_hs<float>(fbto_grid_s*, float*, hipStream_t);
// ===========================================================================
// Design step and projection onto {lo <= x <= hi, sum x <= vmax}.
//
// f(l) = sum_e clamp(y_e - l, lo, hi) is continuous, non-increasing and
// linear between the breakpoints y_e - lo, y_e - hi (Eq. piecewiseLinearEQ).
// Each search pass evaluates, at the current l, f and the classification of
// every entry just right (+) and just left (-) of l, which fixes the linear
// piece on either side:  f(l') = hi nU + lo nL + sum_A y - l' nA.  The next
// pass solves that piece exactly; if the solution leaves the piece (beyond
// the nearest breakpoint) it becomes a Newton step safeguarded by the
// bracket [a, b] with f(a) > vmax >= f(b), else bisection.
// The gradient step y = x - alpha/2 (g - mean g), with the seed of the
// projection (sum clamp(y), max y, #interior) and its first evaluation, at
// the multiplier of the previous projection (the warm start), into
// evaluation set 0: the first search pass decides from it directly.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_step(int64_t E, const T* x, const T* gx, T* y, double half_alpha, int mean_project, double lo,
           double hi, double* P, int maxp, int nb_sum, const Scalars* sc) {
  const double lam_w = sc->lam_prev;
  double mean = 0.0;
  if (mean_project) {
    double v[1];
    const double* src[1] = {pslot(P, P_GSUM, 0, maxp)};
    const int cnt[1] = {nb_sum};
    reduce_parts<1, 0u>(v, src, cnt);
    mean = v[0] / (double)E;
  }
  double v[3] = {0.0, -INFINITY, 0.0};
  double ev[11];
  proj_eval_init(ev);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const T ye = (T)((double)x[e] - half_alpha * ((double)gx[e] - mean));
    y[e] = ye;
    const double yd = (double)ye;
    v[0] += fmin(fmax(yd, lo), hi);
    v[1] = fmax(v[1], yd);
    v[2] += (yd > lo && yd < hi) ? 1.0 : 0.0;
    proj_eval(ev, yd, lam_w, lo, hi);
  }
  step_parts<kVecBlock>(v, ev, P, maxp);
}

__device__ __forceinline__ double* lslot(const ProjWs& W, int i) { return W.base + i * W.stride; }

// Seed of a cold projection: sum clamp(y), max y and the interior count;
// the warm start of the search is cleared.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_init(int64_t E, const T* y, double lo, double hi, ProjWs W) {
  if (blockIdx.x == 0 && threadIdx.x == 0) W.sc->lam_prev = 0.0;
  double v[3] = {0.0, -INFINITY, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double yd = (double)y[e];
    v[0] += fmin(fmax(yd, lo), hi);
    v[1] = fmax(v[1], yd);
    v[2] += (yd > lo && yd < hi) ? 1.0 : 0.0;
  }
  double* dst[3] = {lslot(W, L_S0), lslot(W, L_YMAX), lslot(W, L_NACT)};
  write_parts<3, 0x2u, kVecBlock>(v, dst, blockIdx.x);
}

struct ProjDecision {
  double lam, a, b;
  bool done;
  bool bad;
};

// First slot of the evaluation set q of the projection passes.
__host__ __device__ constexpr int proj_set(int q) { return L_E0 + 11 * (q & 1); }
// pass t reads set t and writes set t + 1: two disjoint runs of 11 slots
static_assert(proj_set(0) + 11 <= proj_set(1) && proj_set(1) + 11 <= L_VOL, "projection slot sets overlap");

// Decision from the evaluation at lam left in evaluation set `set`, with the
// bracket [a, b] of the root.
__device__ ProjDecision proj_decide_eval(const ProjWs& W, int nb, int set, double lo, double hi, double vmax,
                                         double lam, double a, double b) {
  ProjDecision d{};
  double v[11];
  const double* src[11];
  int cnt[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) {
    src[i] = lslot(W, proj_set(set) + i);
    cnt[i] = nb;
  }
  reduce_parts<11, 0x600u, kVecBlock>(v, src, cnt);
  const double F = v[0];
  const double lb = v[9], ub = -v[10];
  double next;
  bool done = false;
  d.bad = !isfinite(F);
  if (d.bad) {
    d.done = true;
    d.lam = b;
    d.a = a;
    d.b = b;
    return d;
  }
  if (F > vmax) {
    a = lam;
    const double nA = v[1];
    if (nA > 0.0) {
      const double ls = (hi * v[3] + lo * v[4] + v[2] - vmax) / nA;
      if (ls <= ub) { next = fmax(ls, lam); done = true; }
      else next = (ls > a && ls < b) ? ls : 0.5 * (a + b);
    } else {
      next = 0.5 * (a + b);
    }
  } else if (F < vmax) {
    b = lam;
    const double nA = v[5];
    if (nA > 0.0) {
      const double ls = (hi * v[7] + lo * v[8] + v[6] - vmax) / nA;
      if (ls >= lb) { next = fmin(ls, lam); done = true; }
      else next = (ls > a && ls < b) ? ls : 0.5 * (a + b);
    } else {
      next = 0.5 * (a + b);
    }
  } else {
    next = lam;
    done = true;
  }
  if (!done && (!(b > a) || next <= a || next >= b)) {  // bracket exhausted: b is feasible
    done = true;
    next = b;
  }
  d.lam = next;
  d.a = a;
  d.b = b;
  d.done = done;
  return d;
}

// The search state after a pass (identical in every block).  `first`: from
// the seed (sum clamp(y), max y, #interior), and -- warm_eval -- from the
// evaluation at the warm start lam_prev in set 0 when lam_prev lies in the
// bracket; otherwise from the evaluation at `lam` left in set `set`.
__device__ ProjDecision proj_decide(const ProjWs& W, int nb, bool first, int set, double lo, double hi,
                                    double vmax, double lam_prev, double lam, double a, double b,
                                    bool warm_eval = false) {
  if (!first) return proj_decide_eval(W, nb, set, lo, hi, vmax, lam, a, b);
  ProjDecision d{};
  double v[3];
  const double* src[3] = {lslot(W, L_S0), lslot(W, L_YMAX), lslot(W, L_NACT)};
  const int cnt[3] = {nb, nb, nb};
  reduce_parts<3, 0x2u, kVecBlock>(v, src, cnt);
  const double S0 = v[0], ymax = v[1], nact0 = v[2];
  d.bad = !isfinite(S0);
  if (S0 <= vmax || d.bad) {
    d.done = true;
    d.lam = 0.0;
    d.a = d.b = 0.0;
    return d;
  }
  d.a = 0.0;
  d.b = ymax - lo;
  if (warm_eval && lam_prev > d.a && lam_prev < d.b)
    return proj_decide_eval(W, nb, 0, lo, hi, vmax, lam_prev, d.a, d.b);
  double l0;
  if (lam_prev > d.a && lam_prev < d.b) l0 = lam_prev;
  else if (nact0 > 0.0) {
    l0 = (S0 - vmax) / nact0;
    if (!(l0 > d.a && l0 < d.b)) l0 = 0.5 * (d.a + d.b);
  } else {
    l0 = 0.5 * (d.a + d.b);
  }
  d.lam = l0;
  d.done = false;
  return d;
}

// Pass t of the search: decides from the seed (t = 0) or from pass t - 1's
// evaluation (set t & 1), then evaluates at the new multiplier into set
// (t + 1) & 1.  The two sets keep a block that starts late from reading
// partials that blocks of the same pass have already overwritten.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_pass(int64_t E, const T* y, double lo, double hi, double vmax, int pass, ProjWs W, int nb,
                int warm_eval) {
  // nb: the partials the decision reduces (on pass 0 the seed's, which the
  // step may have written with another grid)
  Scalars* sc = W.sc;
  const double* in = sc->ps[pass & 1];
  double* out = sc->ps[(pass + 1) & 1];
  if (pass > 0 && in[3] != 0.0) {            // already solved: carry the state forward
    if (blockIdx.x == 0 && threadIdx.x == 0)
      for (int i = 0; i < 4; ++i) out[i] = in[i];
    return;
  }
  const ProjDecision d =
      proj_decide(W, nb, pass == 0, pass, lo, hi, vmax, sc->lam_prev, in[0], in[1], in[2], warm_eval != 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[0] = d.lam;
    out[1] = d.a;
    out[2] = d.b;
    out[3] = d.done ? 1.0 : 0.0;
    if (d.bad) sc->proj_status = (double)FBTO_ERR_NONFINITE;
    else if (pass == 0) sc->proj_status = 0.0;
  }
  if (d.done) return;
  const double lam = d.lam;
  double v[11];
  proj_eval_init(v);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x)
    proj_eval(v, (double)y[e], lam, lo, hi);
  double* dst[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) dst[i] = lslot(W, proj_set(pass + 1) + i);
  write_parts<11, 0x600u, kVecBlock>(v, dst, blockIdx.x);
}

// x = clamp(y - lambda, lo, hi) after `passes` passes.  A search still open
// then decides once more from the last evaluation (set passes & 1); if that
// does not land on the root's piece either, x takes the feasible end of the
// bracket and the status says FBTO_INEXACT.  The lead thread records the
// status (also into *status_out) and lambda.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_final(int64_t E, const T* y, T* x, double lo, double hi, double vmax, const T* x_old, ProjWs W, int nb,
                 int passes, double* lam_out, double* status_out) {
  Scalars* sc = W.sc;
  const double* in = sc->ps[passes & 1];
  double lam = in[0];
  bool bad = false, unfinished = false;
  if (in[3] == 0.0) {  // pass budget spent: decide from the last evaluation
    const ProjDecision d =
        proj_decide(W, nb, false, passes, lo, hi, vmax, sc->lam_prev, in[0], in[1], in[2]);
    lam = d.done ? d.lam : d.b;
    bad = d.bad;
    unfinished = !d.done;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double status = sc->proj_status;  // 0, or FBTO_ERR_NONFINITE from a pass
    if (bad) status = (double)FBTO_ERR_NONFINITE;
    else if (unfinished && status == 0.0) status = (double)FBTO_INEXACT;
    sc->proj_status = status;
    sc->lam = lam;
    sc->lam_prev = lam;   // warm start of the next projection (no block here reads it)
    if (lam_out) *lam_out = lam;
    if (status_out) *status_out = status;
  }
  double v[2] = {0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const T xe = (T)fmin(fmax((double)y[e] - lam, lo), hi);
    if (x_old) v[1] = fmax(v[1], fabs((double)xe - (double)x_old[e]));
    x[e] = xe;
    v[0] += (double)xe;
  }
  double* dst[2] = {lslot(W, L_VOL), lslot(W, L_DX)};
  write_parts<2, 0x2u, kVecBlock>(v, dst, blockIdx.x);
}

// The final pass fused with the forward filter of the next outer iteration:
// both need only y and the multiplier.  Each thread writes x = clamp(y -
// lam, lo, hi) at its own elements, as k_proj_final does, and rho = (H x) /
// Hs there from the same values in the window around them, recomputed from
// y, so that no block waits for another's x.  The multiplier, the status
// and the partials (sum x, max |x - x_old|, x updated in place) are those of
// k_proj_final; rho equals the forward filter of the new x bitwise.
template <typename T, int R>
__global__ void __launch_bounds__(kFiltBX * kFiltBY)
    k_proj_final_filter(Geo G, const T* y, T* x, T* rho, const T* Hsi, StencilW<T, R> Wf, double lo, double hi,
                        double vmax, ProjWs W, int nb, int passes, int tiles_x, int tiles_y) {
  constexpr int D = 2 * R + 1;
  const FiltPos q = filt_pos(G, tiles_x, tiles_y);
  T xo[kFiltDZ];  // the design before the step at the own elements (only their owner reads them)
#pragma unroll
  for (int l = 0; l < kFiltDZ; ++l) {
    const int ez = q.z0 + l;
    xo[l] = x[(q.col && ez < q.z1) ? q.ex + G.nx * (q.ey + G.ny * ez) : 0];
  }
  Scalars* sc = W.sc;
  const double* in = sc->ps[passes & 1];
  double lam = in[0];
  bool bad = false, unfinished = false;
  if (in[3] == 0.0) {  // pass budget spent: decide from the last evaluation
    const ProjDecision d =
        proj_decide(W, nb, false, passes, lo, hi, vmax, sc->lam_prev, in[0], in[1], in[2]);
    lam = d.done ? d.lam : d.b;
    bad = d.bad;
    unfinished = !d.done;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double status = sc->proj_status;  // 0, or FBTO_ERR_NONFINITE from a pass
    if (bad) status = (double)FBTO_ERR_NONFINITE;
    else if (unfinished && status == 0.0) status = (double)FBTO_INEXACT;
    sc->proj_status = status;
    sc->lam = lam;
    sc->lam_prev = lam;
  }
  // the window of new design values, from y and the multiplier
  T win[kFiltDZ + 2 * R][D][D];
  filt_window<T, R>(G, q, y, nullptr, false, win, true, lam, lo, hi);
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int l = 0; l < kFiltDZ; ++l) {
    const int ez = q.z0 + l;
    const T acc = filt_sum<T, R>(Wf, win, l);
    if (q.col && ez < q.z1) {
      const int e = q.ex + G.nx * (q.ey + G.ny * ez);
      const T xe = win[l + R][R][R];
      v[1] = fmax(v[1], fabs((double)xe - (double)xo[l]));
      x[e] = xe;
      v[0] += (double)xe;
      rho[e] = acc * Hsi[e];
    }
  }
  double* dst[2] = {lslot(W, L_VOL), lslot(W, L_DX)};
  write_parts<2, 0x2u, kFiltBX * kFiltBY>(v, dst, blockIdx.x);
}

template <typename T>
hipError_t launch_proj_final_filter(fbto_grid_s* g, const ProjWs& W, const T* y, T* x, T* rho, double lo,
                                    double hi, double vmax, int passes, hipStream_t st, int* nb_final) {
  if (!zmarch_filter(g)) return hipErrorNotSupported;
  const double r = g->desc.filter_radius;
  const int R = r > 1.0 ? (int)std::ceil(r) - 1 : 0;
  const Geo& G = g->geo;
  const int tiles_x = (G.nx + kFiltBX - 1) / kFiltBX, tiles_y = (G.ny + kFiltBY - 1) / kFiltBY;
  const int64_t nbz = (int64_t)tiles_x * tiles_y * ((G.nz + kFiltDZ - 1) / kFiltDZ);
  if (nbz > W.maxp) return hipErrorInvalidValue;
  const int nb = vec_blocks(G.E);  // the passes' partials
  const T* Hsi = (const T*)vecs_of<T>(g).Hs;
  if (R == 0)
    hipLaunchKernelGGL((k_proj_final_filter<T, 0>), dim3(nbz), dim3(kFiltBX * kFiltBY), 0, st, G, y, x, rho, Hsi,
                       stencil_weights<T, 0>(r), lo, hi, vmax, W, nb, passes, tiles_x, tiles_y);
  else
    hipLaunchKernelGGL((k_proj_final_filter<T, 1>), dim3(nbz), dim3(kFiltBX * kFiltBY), 0, st, G, y, x, rho, Hsi,
                       stencil_weights<T, 1>(r), lo, hi, vmax, W, nb, passes, tiles_x, tiles_y);
  *nb_final = (int)nbz;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step(fbto_grid_s* g, const T* x, const T* gx, T* y, double half_alpha,
                       int mean_project, double lo, double hi, hipStream_t st) {
  const int nb = vec_blocks(g->geo.E);
  hipLaunchKernelGGL((k_step<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.E, x, gx, y, half_alpha,
                     mean_project, lo, hi, g->partials, g->max_partials, g->n_gsum, (const Scalars*)g->sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_project(const ProjWs& W, int64_t E, const T* y, T* x, double lo, double hi, double vmax,
                          int seeded, int passes, const T* x_old, double* lam_out, double* status_out,
                          hipStream_t st, int nb_seed, int skip_final) {
  const int nb = vec_blocks(E);
  if (nb > W.maxp || nb_seed > W.maxp) return hipErrorInvalidValue;
  if (!seeded || nb_seed < 1) nb_seed = nb;
  if (!seeded) {
    hipLaunchKernelGGL((k_proj_init<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, lo, hi, W);
  }
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_proj_pass<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, lo, hi, vmax, p, W,
                       p == 0 ? nb_seed : nb, seeded);
  }
  if (skip_final) return hipGetLastError();
  hipLaunchKernelGGL((k_proj_final<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, x, lo, hi, vmax, x_old, W, nb,
                     passes, lam_out, status_out);
  return hipGetLastError();
}

// ===========================================================================
// Conversions and iterative-refinement helpers.
// ===========================================================================
__global__ void k_f64_to_f32(const double* in, float* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void k_f32_to_f64(const float* in, double* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}
__global__ void k_axpy64(double* u, const double* d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    u[i] += d[i];
}
__global__ void k_accum_f32(double* u, const float* d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    u[i] += (double)d[i];
}

static int flat_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

template <typename T>
hipError_t launch_convert(const void* in, void* out, int64_t n, int to_double, hipStream_t st) {
  if (to_double)
    hipLaunchKernelGGL(k_f32_to_f64, dim3(flat_blocks(n)), dim3(256), 0, st, (const float*)in, (double*)out, n);
  else
    hipLaunchKernelGGL(k_f64_to_f32, dim3(flat_blocks(n)), dim3(256), 0, st, (const double*)in, (float*)out, n);
  return hipGetLastError();
}
template hipError_t launch_convert<float>(const void*, void*, int64_t, int, hipStream_t);

hipError_t launch_axpy64(double* u, const double* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy64, dim3(flat_blocks(n)), dim3(256), 0, st, u, d, n);
  return hipGetLastError();
}
hipError_t launch_ir_scale(fbto_grid_s* g, const double* r64, float* r32, int nrhs, hipStream_t st) {
  return launch_convert<float>(r64, r32, g->geo.ndof * nrhs, 0, st);
}
hipError_t launch_ir_accum(fbto_grid_s* g, double* u64, const float* d32, int nrhs, hipStream_t st) {
  const int64_t n = g->geo.ndof * nrhs;
  hipLaunchKernelGGL(k_accum_f32, dim3(flat_blocks(n)), dim3(256), 0, st, u64, d32, n);
  return hipGetLastError();
}

__global__ void k_solve_info(Scalars* sc, double* info, int nrhs, double steps_override) {
  for (int R = 0; R < nrhs; ++R) {
    double* o = info + R * FBTO_SOLVE_INFO;
    o[FBTO_SI_RNORM2] = sc->rnorm2[R];
    o[FBTO_SI_RNORMI] = sc->rinf[R];
    o[FBTO_SI_FNORM2] = sc->fnorm2[R];
    o[FBTO_SI_STEPS] = steps_override >= 0.0 ? steps_override : sc->steps[R];
    o[FBTO_SI_STATUS] = sc->status[R];
    for (int k = 5; k < FBTO_SOLVE_INFO; ++k) o[k] = 0.0;
  }
}
hipError_t launch_solve_info(fbto_grid_s* g, double* info, int nrhs, double steps_override, hipStream_t st) {
  hipLaunchKernelGGL(k_solve_info, dim3(1), dim3(1), 0, st, g->sc, info, nrhs, steps_override);
  return hipGetLastError();
}

// ===========================================================================
// Optimality metrics of a design (Sec. 4, the error metrics of Thm. 1).
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_sqdist(int64_t n, const T* a, const T* b, double* P, int maxp, int slot) {
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)a[i] - (double)b[i];
    v[0] += d * d;
  }
  double* dst[1] = {pslot(P, slot, 0, maxp)};
  write_parts<1, 0u>(v, dst, blockIdx.x);
}

template <typename T>
hipError_t launch_sqdist(fbto_grid_s* g, const T* a, const T* b, int64_t n, int slot, hipStream_t st, int* nb_out) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL((k_sqdist<T>), dim3(nb), dim3(kVecBlock), 0, st, n, a, b, g->partials, g->max_partials, slot);
  if (nb_out) *nb_out = nb;
  return hipGetLastError();
}

__global__ void __launch_bounds__(kVecBlock)
    k_opt_finish(const double* P, int maxp, int nrhs, int nb_dot, int nb_lo, int nb_hi, double alpha,
                 const Scalars* sc, const Scalars* sc_proj, double* out) {
  double v[3];
  const double* src[3] = {pslot(P, P_DOT, 0, maxp), pslot(P, P_MET0, 0, maxp), pslot(P, P_MET1, 0, maxp)};
  const int cnt[3] = {nb_dot, nb_lo, nb_hi};
  reduce_parts<3, 0u, kVecBlock>(v, src, cnt);
  if (threadIdx.x == 0) {
    double rrel = 0.0, status = 0.0;
    for (int R = 0; R < nrhs; ++R) {
      const double fn = sc->fnorm2[R];
      rrel = fmax(rrel, fn > 0.0 ? sc->rnorm2[R] / fn : sc->rnorm2[R]);
      if (sc->status[R] != 0.0) status = sc->status[R];
    }
    const double ps = sc_proj->proj_status;
    if (ps > 0.0 && (status == 0.0 || ps == (double)FBTO_ERR_NONFINITE)) status = ps;
    out[0] = 0.5 * v[0];
    out[1] = v[2] / (alpha * alpha);
    out[2] = v[1];
    out[3] = rrel;
    out[4] = status;
  }
}

hipError_t launch_opt_finish(fbto_grid_s* g, int nrhs, int nb_dot, int nb_lo, int nb_hi, double alpha,
                             const Scalars* sc_proj, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_opt_finish, dim3(1), dim3(kVecBlock), 0, st, (const double*)g->partials, g->max_partials,
                     nrhs, nb_dot, nb_lo, nb_hi, alpha, (const Scalars*)g->sc, sc_proj, out);
  return hipGetLastError();
}

// ---- explicit instantiations ----------------------------------------------
#define FBTO_INST(T)                                                                                   \
  template hipError_t launch_apply<T>(fbto_grid_s*, const T*, const T*, T*, int, hipStream_t);         \
  template hipError_t launch_resid<T>(fbto_grid_s*, const T*, const T*, const T*, T*, const T*, T*, int, \
                                      hipStream_t, int*);                                              \
  template hipError_t launch_resid_diag<T>(fbto_grid_s*, const T*, const T*, const T*, T*, T*, T*, int,  \
                                           hipStream_t, int*);                                         \
  template hipError_t launch_apply_cg<T>(fbto_grid_s*, const T*, const T*, const T*, T*, int, int,     \
                                         hipStream_t, int*);                                           \
  template hipError_t launch_cg_step<T>(fbto_grid_s*, const T*, T*, T*, const T*, T*, const T*, T*, T*, \
                                        const T*, const T*, int, int, int, int, double, hipStream_t,   \
                                        int*);                                                         \
  template hipError_t launch_cg_sens<T>(fbto_grid_s*, const T*, const CgSet<T>&, T*, const T*, const T*, \
                                        T*, const T*, int, int, int, double, hipStream_t, int*);       \
  template hipError_t launch_cg_fused<T>(fbto_grid_s*, const T*, const CgSet<T>&, const CgSet<T>&,      \
                                         const T*, int, int, int, int, double, hipStream_t, int*);      \
  template hipError_t launch_diag<T>(fbto_grid_s*, const T*, T*, hipStream_t);                         \
  template hipError_t launch_relax_update<T>(fbto_grid_s*, T*, const T*, const T*, int, double, int,    \
                                             hipStream_t);                                             \
  template hipError_t launch_minres<T>(fbto_grid_s*, int, int, const T*, T*, const T*, T*, const T*, T*, \
                                       int, int, double, hipStream_t, int*);                          \
  template hipError_t launch_minres_fused<T>(fbto_grid_s*, const T*, int, const T*, const T*, const T*, T*,  \
                                             const T*, T*, T*, T*, int, int, double, hipStream_t, int*);  \
  template hipError_t launch_sens<T>(fbto_grid_s*, const T*, const T*, const T*, int, T*, const T*,    \
                                     hipStream_t);                                                     \
  template hipError_t launch_dot<T>(fbto_grid_s*, const T*, const T*, int, hipStream_t);               \
  template hipError_t launch_filter<T>(fbto_grid_s*, int, const T*, T*, int, hipStream_t);             \
  template hipError_t launch_sqdist<T>(fbto_grid_s*, const T*, const T*, int64_t, int, hipStream_t, int*); \
  template hipError_t launch_step<T>(fbto_grid_s*, const T*, const T*, T*, double, int, double,       \
                                     double, hipStream_t);                                             \
  template hipError_t launch_project<T>(const ProjWs&, int64_t, const T*, T*, double, double, double, int, \
                                        int, const T*, double*, double*, hipStream_t, int, int);          \
  template hipError_t launch_proj_final_filter<T>(fbto_grid_s*, const ProjWs&, const T*, T*, T*, double, \
                                                  double, double, int, hipStream_t, int*);               \
  template hipError_t launch_filter_step<T>(fbto_grid_s*, const T*, const T*, T*, double, int, int, double, \
                                            double, hipStream_t, int*);

FBTO_INST(double)
FBTO_INST(float)

}  // namespace fbto
