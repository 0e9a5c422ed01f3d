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
// apply_K: z-marching tiles, one element column per thread.
//
// Block = BX x BY threads; thread (tx, ty) owns element column
// (ex, ey) = (bx (BX-1) - 1 + tx, by (BY-1) - 1 + ty) and marches the element
// layers of one z-slab.  Per layer it uses the four nodes of the element's
// upper face (loaded one layer ahead; the lower face is carried from the
// previous layer), computes the full 24-entry element product in the
// sum/difference basis, adds the lower-face half to the upper-face half
// carried from the layer below (this completes the z-sum of every node of
// the plane), and exchanges the four xy-corners through LDS so that each
// interior thread sums the four element columns around its node in a fixed
// order.  Neighbouring tiles overlap by one element column / row / layer, so
// no atomics are needed and the result is bitwise reproducible.
//
// Modes:
//   APPLY  y = K u
//   RESID  y = r = f - K u; if invD is given, also z = D^-1 r and the
//          partials of r.r, max|r|, f.f (the start of a CG solve)
//   CG     y = w = K z with the partials of r.z, w.z, r.r, max|r| (one
//          reduction phase per step of the Chronopoulos-Gear recurrence)
// ===========================================================================
enum { MODE_APPLY = 0, MODE_RESID = 1, MODE_CG = 2 };

template <typename T>
struct ApplyArgs {
  Geo g;
  const T* rho;
  const T* u;          // input vector
  T* y;
  const T* f;          // RESID
  const T* invD;       // RESID (optional): start of a CG solve
  T* z;                // RESID: z = D^-1 r
  const T* r;          // CG: current residual (for r.z, r.r)
  const uint8_t* mask;
  Modal<T> km;
  Simp sp;
  int nspring;
  const int64_t* sdof;
  const T* sk;
  int tiles_x, tiles_y, slabs, dz, nblocks, per_xcd;
  double* P;           // partial slots
  int maxp;
  const Scalars* sc;
};

template <typename T, int BX, int BY, int NR, int MODE>
__global__ void __launch_bounds__(BX* BY)
    k_apply(ApplyArgs<T> A, int rhs0) {
  __shared__ T lds[NR][3][3][BY][BX];  // [rhs][corner 0..2][comp][ty][tx]
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int b = blockIdx.x;
  const int lb = (b & 7) * A.per_xcd + (b >> 3);  // XCD-aware: neighbours share an L2
  if (lb >= A.nblocks) return;
  const Geo G = A.g;

  const int bx = lb % A.tiles_x;
  const int t2 = lb / A.tiles_x;
  const int by = t2 % A.tiles_y;
  const int bz = t2 / A.tiles_y;
  const int ex = bx * (BX - 1) - 1 + tx;
  const int ey = by * (BY - 1) - 1 + ty;
  const int k0 = bz * A.dz;
  const int kend = min(k0 + A.dz, G.nz + 1);
  const bool xy_elem = ex >= 0 && ex < G.nx && ey >= 0 && ey < G.ny;
  const bool out_xy = tx < BX - 1 && ty < BY - 1 && ex + 1 <= G.nx && ey + 1 <= G.ny;
  const int plane = G.nxn * G.nyn;

  bool vxy[4];
  int nb0[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = ex + (a & 1), j = ey + (a >> 1);
    vxy[a] = i >= 0 && i <= G.nx && j >= 0 && j <= G.ny;
    nb0[a] = vxy[a] ? i + G.nxn * j : 0;
  }
  const T* ub[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) ub[r] = A.u + (int64_t)(rhs0 + r) * G.ndof;

  // raw loads of a face, issued one layer ahead of their use
  T raw[NR][4][3];
  unsigned rmask[4];
  auto issue_face = [&](int k) {
    const bool kv = k >= 0 && k <= G.nz;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const bool ok = vxy[a] && kv;
      const int n = ok ? nb0[a] + k * plane : 0;
      rmask[a] = ok ? (unsigned)A.mask[n] : 7u;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) raw[r][a][c] = ub[r][3 * n + c];
    }
  };
  auto take_face = [&](T(&dst)[NR][4][3]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          dst[r][a][c] = ((rmask[a] >> c) & 1u) ? (T)0 : raw[r][a][c];
        }
  };
  auto load_rho = [&](int ez) -> T {
    const bool el = xy_elem && ez >= 0 && ez < G.nz;
    const T rv = A.rho[el ? ex + G.nx * (ey + G.ny * ez) : 0];
    return el ? simp_s<T>(rv, A.sp) : (T)0;
  };

  constexpr int NP = MODE == MODE_APPLY ? 1 : 4 * NR;  // partial values per block
  double part[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) part[i] = 0.0;

  T ul[NR][4][3], uu[NR][4][3], carry[NR][4][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[r][a][c] = (T)0;

  issue_face(k0 - 1);
  take_face(ul);
  issue_face(k0);
  T s_next = load_rho(k0 - 1);
  for (int ez = k0 - 1; ez < kend; ++ez) {
    take_face(uu);
    const T s = s_next;
    if (ez + 1 < kend) {  // prefetch the next layer (uniform over the block)
      issue_face(ez + 2);
      s_next = load_rho(ez + 1);
    }
    const bool emit = ez >= k0;  // uniform over the block
    T own[NR][3];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T ue[8][3], ye[8][3];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ue[a][c] = ul[r][a][c];
          ue[a + 4][c] = uu[r][a][c];
        }
      elem_apply<T>(ue, s, A.km, ye);
      if (emit) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
          for (int a = 0; a < 3; ++a) lds[r][a][c][ty][tx] = carry[r][a][c] + ye[a][c];
          own[r][c] = carry[r][3][c] + ye[3][c];
        }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) carry[r][a][c] = ye[a + 4][c];
    }
    if (emit) {
      __syncthreads();
      if (out_xy) {
        const int n = (ex + 1) + G.nxn * (ey + 1) + ez * plane;
        const unsigned m = A.mask[n];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int64_t o = (int64_t)(rhs0 + r) * G.ndof + 3 * n;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            T acc = ((own[r][c] + lds[r][2][c][ty][tx + 1]) + lds[r][1][c][ty + 1][tx]) +
                    lds[r][0][c][ty + 1][tx + 1];
            T pv = ul[r][3][c];  // masked input value at this node
            for (int sI = 0; sI < A.nspring; ++sI)
              if (A.sdof[sI] == (int64_t)(3 * n + c)) acc += A.sk[sI] * pv;
            const bool fixed = (m >> c) & 1u;
            if (fixed) pv = A.u[o + c];
            if (fixed) acc = pv;
            if constexpr (MODE == MODE_RESID) {
              const T fv = A.f[o + c];
              const T rv = fv - acc;
              A.y[o + c] = rv;
              if (A.invD) {
                A.z[o + c] = A.invD[3 * n + c] * rv;
                part[4 * r + 0] += (double)rv * (double)rv;
                part[4 * r + 1] = fmax(part[4 * r + 1], fabs((double)rv));
                part[4 * r + 2] += (double)fv * (double)fv;
              }
            } else {
              A.y[o + c] = acc;
              if constexpr (MODE == MODE_CG) {
                const T rv = A.r[o + c];
                part[4 * r + 0] += (double)rv * (double)pv;     // r.z
                part[4 * r + 1] += (double)acc * (double)pv;    // w.z
                part[4 * r + 2] += (double)rv * (double)rv;     // r.r
                part[4 * r + 3] = fmax(part[4 * r + 3], fabs((double)rv));
              }
            }
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) ul[r][a][c] = uu[r][a][c];
  }

  if constexpr (MODE == MODE_CG) {
    double* dst[4 * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      dst[4 * r + 0] = A.P + ((int64_t)P_RZ0 * 4 + rhs0 + r) * A.maxp;
      dst[4 * r + 1] = A.P + ((int64_t)P_PQ * 4 + rhs0 + r) * A.maxp;
      dst[4 * r + 2] = A.P + ((int64_t)P_RN0 * 4 + rhs0 + r) * A.maxp;
      dst[4 * r + 3] = A.P + ((int64_t)P_RI0 * 4 + rhs0 + r) * A.maxp;
    }
    write_parts<4 * NR, 0x8888u>(part, dst, lb);
  }
  if constexpr (MODE == MODE_RESID) {
    if (A.invD == nullptr) return;
    if (lb == 0 && tx == 0 && ty == 0) {   // a new solve starts from this residual
      Scalars* sc = const_cast<Scalars*>(A.sc);
      for (int r = 0; r < NR; ++r) {
        sc->done[rhs0 + r] = 0.0;
        sc->status[rhs0 + r] = 0.0;
        sc->steps[rhs0 + r] = 0.0;
      }
    }
    double* dst[4 * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      dst[4 * r + 0] = A.P + ((int64_t)P_RN1 * 4 + rhs0 + r) * A.maxp;
      dst[4 * r + 1] = A.P + ((int64_t)P_RI1 * 4 + rhs0 + r) * A.maxp;
      dst[4 * r + 2] = A.P + ((int64_t)P_FN * 4 + rhs0 + r) * A.maxp;
      dst[4 * r + 3] = A.P + ((int64_t)P_RZ1 * 4 + rhs0 + r) * A.maxp;
    }
    write_parts<4 * NR, 0x2222u>(part, dst, lb);
  }
}

struct TileChoice {
  int bx, by, dz, tiles_x, tiles_y, slabs, nblocks;
};

static TileChoice choose_tile(const Geo& G, int n_cu, int nr, bool fp64) {
  const char* env = getenv("FBTO_APPLY_TILE");
  int want_bx = 0, want_by = 0, want_dz = 0;
  if (env) sscanf(env, "%dx%dx%d", &want_bx, &want_by, &want_dz);
  const int opts[2][2] = {{16, 16}, {32, 8}};
  const int dzs[] = {2, 3, 4, 5, 6, 8, 10, 12, 16, 24, 32, 48, 64};
  TileChoice best{};
  double best_cost = 1e300;
  for (auto& o : opts) {
    if (want_bx && (o[0] != want_bx || o[1] != want_by)) continue;
    for (int dz : dzs) {
      if (want_dz && dz != want_dz) continue;
      TileChoice t;
      t.bx = o[0];
      t.by = o[1];
      t.dz = dz;
      t.tiles_x = (G.nxn + t.bx - 2) / (t.bx - 1);
      t.tiles_y = (G.nyn + t.by - 2) / (t.by - 1);
      t.slabs = (G.nzn + dz - 1) / dz;
      const int64_t nb = (int64_t)t.tiles_x * t.tiles_y * t.slabs;
      if (nb > (1 << 30)) continue;
      t.nblocks = (int)nb;
      // element-steps of work, inflated when the chip is under-filled or
      // the last wave of blocks is ragged
      const double work = (double)nb * t.bx * t.by * (dz + 1);
      const double slots = 2.0 * n_cu;  // resident 256-thread blocks
      const double waves = std::ceil(nb / slots);
      const double fill = nb / (waves * slots);
      const double cost = work / fill;
      if (cost < best_cost) {
        best_cost = cost;
        best = t;
      }
    }
  }
  (void)nr;
  (void)fp64;
  return best;
}


int apply_max_blocks(const Geo& G, int n_cu) {
  int m = 0;
  for (int nr : {1, 2, 4})
    for (bool fp64 : {false, true}) m = std::max(m, choose_tile(G, n_cu, nr, fp64).nblocks);
  return m;
}

template <typename T, int BX, int BY, int NR, int MODE>
static hipError_t launch_apply_t(const ApplyArgs<T>& A0, const TileChoice& t, int rhs0, hipStream_t st) {
  ApplyArgs<T> A = A0;
  A.tiles_x = t.tiles_x;
  A.tiles_y = t.tiles_y;
  A.slabs = t.slabs;
  A.dz = t.dz;
  A.nblocks = t.nblocks;
  A.per_xcd = (t.nblocks + 7) / 8;
  const int grid = A.per_xcd * 8;
  hipLaunchKernelGGL((k_apply<T, BX, BY, NR, MODE>), dim3(grid), dim3(BX, BY), 0, st, A, rhs0);
  return hipGetLastError();
}

template <typename T, int MODE>
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
  constexpr bool fp64 = sizeof(T) == 8;
  const int maxnr = fp64 ? 2 : 4;
  int r0 = 0;
  hipError_t e = hipSuccess;
  while (r0 < nrhs && e == hipSuccess) {
    int nr = std::min(nrhs - r0, maxnr);
    if (nr == 3) nr = 2;
    const TileChoice t = choose_tile(g->geo, g->n_cu, nr, fp64);
    if (t.nblocks > g->max_partials) return hipErrorInvalidValue;
    if (nb_out) *nb_out = t.nblocks;
    if (nr == 1) {
      e = t.bx == 32 ? launch_apply_t<T, 32, 8, 1, MODE>(A, t, r0, st) : launch_apply_t<T, 16, 16, 1, MODE>(A, t, r0, st);
    } else if (nr == 2) {
      e = t.bx == 32 ? launch_apply_t<T, 32, 8, 2, MODE>(A, t, r0, st) : launch_apply_t<T, 16, 16, 2, MODE>(A, t, r0, st);
    } else {
      if constexpr (!fp64) {
        e = t.bx == 32 ? launch_apply_t<T, 32, 8, 4, MODE>(A, t, r0, st) : launch_apply_t<T, 16, 16, 4, MODE>(A, t, r0, st);
      }
    }
    r0 += nr;
  }
  return e;
}

template <typename T>
hipError_t launch_apply(fbto_grid_s* g, const T* rho, const T* u, T* y, int nrhs, hipStream_t st) {
  ApplyArgs<T> A{};
  A.rho = rho;
  A.u = u;
  A.y = y;
  return launch_apply_mode<T, MODE_APPLY>(g, A, nrhs, st, nullptr);
}

template <typename T>
hipError_t launch_resid(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, const T* invD, T* z,
                        int nrhs, hipStream_t st, int* nb_out) {
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
hipError_t launch_apply_cg(fbto_grid_s* g, const T* rho, const T* z, const T* r, T* w, int nrhs, hipStream_t st,
                           int* nb_out) {
  ApplyArgs<T> A{};
  A.rho = rho;
  A.u = z;
  A.r = r;
  A.y = w;
  return launch_apply_mode<T, MODE_CG>(g, A, nrhs, st, nb_out);
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
constexpr int kU = 4;

struct CgCnt {
  int apply;   // partials of the last apply (gamma, delta, r.r, max|r|)
  int fn;      // partials of f.f (the residual apply)
};

template <typename T, int NR>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_step(int64_t ndof, T* x, T* r, T* z, const T* w, T* p, T* s, const T* invD, const T* f, double* P,
              int maxp, CgCnt cn, int step, double rtol, Scalars* sc) {
  // first chunk of this thread's vector entries is loaded before the prologue
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i_first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool first = step == 0;
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
        zv[k][R] = z[o];
        wv[k][R] = w[o];
        xv[k][R] = x[o];
        rv[k][R] = r[o];
        pv[k][R] = first ? (T)0 : p[o];
        sv[k][R] = first ? (T)0 : s[o];
      }
    }
  };
  if (i_first < ndof) load_chunk(i_first);

  double pre[4 * NR];
  {
    const double* src[4 * NR];
    int cnt[4 * NR];
#pragma unroll
    for (int R = 0; R < NR; ++R) {
      src[4 * R + 0] = pslot(P, P_RZ0, R, maxp);
      src[4 * R + 1] = pslot(P, P_PQ, R, maxp);
      src[4 * R + 2] = pslot(P, P_RN0, R, maxp);
      src[4 * R + 3] = pslot(P, P_FN, R, maxp);
      cnt[4 * R + 0] = cn.apply;
      cnt[4 * R + 1] = cn.apply;
      cnt[4 * R + 2] = cn.apply;
      cnt[4 * R + 3] = cn.fn;
    }
    reduce_parts<4 * NR, 0u>(pre, src, cnt);
  }
  T al[NR], be[NR];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  const int rd = (step + 1) & 1, wr = step & 1;
#pragma unroll
  for (int R = 0; R < NR; ++R) {
    const double gam = pre[4 * R], del = pre[4 * R + 1], rn = sqrt(pre[4 * R + 2]), fn = sqrt(pre[4 * R + 3]);
    bool done = sc->done[R] != 0.0 || (rtol > 0.0 && rn <= rtol * fn);
    double alpha = 0.0, beta = 0.0, status = 0.0;
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
    al[R] = (T)alpha;
    be[R] = (T)beta;
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
        z[o] = dv[k] * rn;
        v[2 * R] += (double)rn * (double)rn;
        v[2 * R + 1] = fmax(v[2 * R + 1], fabs((double)rn));
        if (f) v[2 * NR] += (double)f[o] * (double)xn;
      }
    }
  }
  double* dst[2 * NR + 1];
#pragma unroll
  for (int R = 0; R < NR; ++R) {
    dst[2 * R] = pslot(P, P_RN1, R, maxp);
    dst[2 * R + 1] = pslot(P, P_RI1, R, maxp);
  }
  dst[2 * NR] = pslot(P, P_DOT, 0, maxp);
  write_parts<2 * NR + 1, 0xAAAu>(v, dst, blockIdx.x);
}

// Reduce the final residual norms into the scalars (slots RN1, RI1 with n_r
// partials, f.f from FN); with `info`, also write the outer-iteration record
// (compliance from DOT, projection results, gradient mean).
template <int NR>
__global__ void __launch_bounds__(kVecBlock)
    k_pcg_finish(const double* P, int maxp, int n_r, int n_fn, Scalars* sc, double* info, int n_dot, int n_e,
                 int n_gsum, int64_t E) {
  double v[3 * NR + 4];
  const double* src[3 * NR + 4];
  int cnt[3 * NR + 4];
#pragma unroll
  for (int R = 0; R < NR; ++R) {
    src[3 * R + 0] = pslot(P, P_RN1, R, maxp);
    src[3 * R + 1] = pslot(P, P_RI1, R, maxp);
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
  constexpr unsigned MM = 0x492u | (1u << (3 * NR + 2));
  reduce_parts<3 * NR + 4, MM>(v, src, cnt);
  if (threadIdx.x == 0) {
    double rinf = 0.0, rrel = 0.0, status = 0.0;
    for (int R = 0; R < NR; ++R) {
      sc->rnorm2[R] = sqrt(v[3 * R]);
      sc->rinf[R] = v[3 * R + 1];
      sc->fnorm2[R] = sqrt(v[3 * R + 2]);
      if (!isfinite(v[3 * R]) && sc->status[R] == 0.0) sc->status[R] = (double)FBTO_ERR_NONFINITE;
      rinf = fmax(rinf, sc->rinf[R]);
      rrel = fmax(rrel, sc->fnorm2[R] > 0.0 ? sc->rnorm2[R] / sc->fnorm2[R] : sc->rnorm2[R]);
      if (sc->status[R] != 0.0) status = sc->status[R];
    }
    if (info) {
      if (sc->proj_status > 0.0) status = sc->proj_status;
      sc->dot[0] = v[3 * NR];
      info[FBTO_OI_COMPLIANCE] = v[3 * NR];
      info[FBTO_OI_DX_INF] = v[3 * NR + 2];
      info[FBTO_OI_R_INF] = rinf;
      info[FBTO_OI_LAMBDA] = sc->lam;
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
hipError_t launch_cg_step(fbto_grid_s* g, T* x, T* r, T* z, const T* w, T* p, T* s, const T* invD, const T* f,
                          int nrhs, int n_apply, int n_fn, int step, double rtol, hipStream_t st, int* nb_out) {
  const int nb = vec_blocks(g->geo.ndof);
  if (nb_out) *nb_out = nb;
  const CgCnt cn{n_apply, n_fn};
  FBTO_NR_DISPATCH(nrhs, hipLaunchKernelGGL((k_cg_step<T, NR>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof,
                                            x, r, z, w, p, s, invD, f, g->partials, g->max_partials, cn, step,
                                            rtol, g->sc));
  return hipGetLastError();
}
hipError_t launch_pcg_finish(fbto_grid_s* g, int nrhs, int n_r, int n_fn, double* info, int n_dot, int n_e,
                             int n_gsum, hipStream_t st) {
  FBTO_NR_DISPATCH(nrhs, hipLaunchKernelGGL((k_pcg_finish<NR>), dim3(1), dim3(kVecBlock), 0, st,
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
  // with a sum, the grid is capped so that its partials stay few
  const int nb = want_sum ? vec_blocks(g->geo.E) : flat_grid(g->geo.E);
  const double r = g->desc.filter_radius;
  const int R = r > 1.0 ? (int)std::ceil(r) - 1 : 0;
  const T* Hsi = (const T*)V.Hs;
  if (R == 0)
    hipLaunchKernelGGL((k_filter<T, 0>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, kind, in, out, Hsi,
                       stencil_weights<T, 0>(r), want_sum, g->partials, g->max_partials);
  else if (R == 1)
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

template <typename T>
hipError_t launch_hs(fbto_grid_s* g, T* Hs, hipStream_t st) {
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
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_step(int64_t E, const T* x, const T* gx, T* y, double half_alpha, int mean_project, double lo,
           double hi, double* P, int maxp, int nb_sum) {
  double mean = 0.0;
  if (mean_project) {
    double v[1];
    const double* src[1] = {pslot(P, P_GSUM, 0, maxp)};
    const int cnt[1] = {nb_sum};
    reduce_parts<1, 0u>(v, src, cnt);
    mean = v[0] / (double)E;
  }
  double v[3] = {0.0, -INFINITY, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const T ye = (T)((double)x[e] - half_alpha * ((double)gx[e] - mean));
    y[e] = ye;
    const double yd = (double)ye;
    v[0] += fmin(fmax(yd, lo), hi);
    v[1] = fmax(v[1], yd);
    v[2] += (yd > lo && yd < hi) ? 1.0 : 0.0;
  }
  double* dst[3] = {pslot(P, P_S0, 0, maxp), pslot(P, P_YMAX, 0, maxp), pslot(P, P_NACT, 0, maxp)};
  write_parts<3, 0x2u>(v, dst, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_init(int64_t E, const T* y, double lo, double hi, double* P, int maxp) {
  double v[3] = {0.0, -INFINITY, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double yd = (double)y[e];
    v[0] += fmin(fmax(yd, lo), hi);
    v[1] = fmax(v[1], yd);
    v[2] += (yd > lo && yd < hi) ? 1.0 : 0.0;
  }
  double* dst[3] = {pslot(P, P_S0, 0, maxp), pslot(P, P_YMAX, 0, maxp), pslot(P, P_NACT, 0, maxp)};
  write_parts<3, 0x2u>(v, dst, blockIdx.x);
}

struct ProjDecision {
  double lam, a, b;
  bool done;
  bool bad;
};

// The search state after a pass (identical in every block).  `first`: the
// partials are the seed (sum clamp(y), max y, #interior); otherwise the
// evaluation at sc->lam.
__device__ ProjDecision proj_decide(const double* P, int maxp, int nb, bool first, double lo, double hi,
                                    double vmax, double lam_prev, double lam, double a, double b) {
  ProjDecision d{};
  if (first) {
    double v[3];
    const double* src[3] = {pslot(P, P_S0, 0, maxp), pslot(P, P_YMAX, 0, maxp), pslot(P, P_NACT, 0, maxp)};
    const int cnt[3] = {nb, nb, nb};
    reduce_parts<3, 0x2u>(v, src, cnt);
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
  double v[11];
  const double* src[11];
  int cnt[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) {
    src[i] = pslot(P, P_E0 + i, 0, maxp);
    cnt[i] = nb;
  }
  reduce_parts<11, 0x600u>(v, src, cnt);
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

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_pass(int64_t E, const T* y, double lo, double hi, double vmax, int pass, double* P, int maxp,
                int nb, Scalars* sc) {
  const double* in = sc->ps[pass & 1];
  double* out = sc->ps[(pass + 1) & 1];
  if (pass > 0 && in[3] != 0.0) {            // already solved: carry the state forward
    if (blockIdx.x == 0 && threadIdx.x == 0)
      for (int i = 0; i < 4; ++i) out[i] = in[i];
    return;
  }
  const ProjDecision d = proj_decide(P, maxp, nb, pass == 0, lo, hi, vmax, sc->lam_prev, in[0], in[1], in[2]);
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
#pragma unroll
  for (int i = 0; i < 11; ++i) v[i] = 0.0;
  v[9] = -INFINITY;
  v[10] = -INFINITY;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double yd = (double)y[e];
    const double t = yd - lam;
    v[0] += fmin(fmax(t, lo), hi);
    if (t > hi) v[3] += 1.0;            // just right of lambda
    else if (t <= lo) v[4] += 1.0;
    else { v[1] += 1.0; v[2] += yd; }
    if (t >= hi) v[7] += 1.0;           // just left of lambda
    else if (t < lo) v[8] += 1.0;
    else { v[5] += 1.0; v[6] += yd; }
    const double b1 = yd - lo, b2 = yd - hi;
    if (b1 < lam) v[9] = fmax(v[9], b1); else if (b1 > lam) v[10] = fmax(v[10], -b1);
    if (b2 < lam) v[9] = fmax(v[9], b2); else if (b2 > lam) v[10] = fmax(v[10], -b2);
  }
  double* dst[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) dst[i] = pslot(P, P_E0 + i, 0, maxp);
  write_parts<11, 0x600u>(v, dst, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_final(int64_t E, const T* y, T* x, double lo, double hi, double vmax, const T* x_old, double* P,
                 int maxp, int nb, int passes, Scalars* sc, double* lam_out) {
  const double* in = sc->ps[passes & 1];
  double lam = in[0];
  bool bad = false, unfinished = false;
  if (in[3] == 0.0) {  // pass budget spent: decide from the last evaluation
    const ProjDecision d = proj_decide(P, maxp, nb, false, lo, hi, vmax, sc->lam_prev, in[0], in[1], in[2]);
    lam = d.done ? d.lam : d.b;
    bad = d.bad;
    unfinished = !d.done;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (unfinished) sc->proj_status = -1.0;   // finished on the feasible end of the bracket
    if (bad) sc->proj_status = (double)FBTO_ERR_NONFINITE;
    sc->lam = lam;
    sc->lam_prev = lam;   // warm start of the next projection (no block here reads it)
    if (lam_out) *lam_out = lam;
  }
  double v[2] = {0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const T xe = (T)fmin(fmax((double)y[e] - lam, lo), hi);
    if (x_old) v[1] = fmax(v[1], fabs((double)xe - (double)x_old[e]));
    x[e] = xe;
    v[0] += (double)xe;
  }
  double* dst[2] = {pslot(P, P_VOL, 0, maxp), pslot(P, P_DX, 0, maxp)};
  write_parts<2, 0x2u>(v, dst, blockIdx.x);
}

static int proj_passes() {
  const char* env = getenv("FBTO_PROJ_PASSES");
  int p = env ? atoi(env) : 8;
  return p < 1 ? 1 : (p > 64 ? 64 : p);
}

template <typename T>
hipError_t launch_step(fbto_grid_s* g, const T* x, const T* gx, T* y, double half_alpha,
                       int mean_project, double lo, double hi, hipStream_t st) {
  const int nb = vec_blocks(g->geo.E);
  hipLaunchKernelGGL((k_step<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.E, x, gx, y, half_alpha,
                     mean_project, lo, hi, g->partials, g->max_partials, nb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_project(fbto_grid_s* g, const T* y, T* x, double lo, double hi, double vmax,
                          int seeded, const T* x_old, double* lam_out, hipStream_t st) {
  const int64_t E = g->geo.E;
  const int nb = vec_blocks(E);
  if (!seeded) {
    hipLaunchKernelGGL((k_proj_init<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, lo, hi, g->partials,
                       g->max_partials);
  }
  const int passes = proj_passes();
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_proj_pass<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, lo, hi, vmax, p,
                       g->partials, g->max_partials, nb, g->sc);
  }
  hipLaunchKernelGGL((k_proj_final<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, x, lo, hi, vmax, x_old,
                     g->partials, g->max_partials, nb, passes, g->sc, lam_out);
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

// ---- explicit instantiations ----------------------------------------------
#define FBTO_INST(T)                                                                                   \
  template hipError_t launch_apply<T>(fbto_grid_s*, const T*, const T*, T*, int, hipStream_t);         \
  template hipError_t launch_resid<T>(fbto_grid_s*, const T*, const T*, const T*, T*, const T*, T*, int, \
                                      hipStream_t, int*);                                              \
  template hipError_t launch_apply_cg<T>(fbto_grid_s*, const T*, const T*, const T*, T*, int, hipStream_t, \
                                         int*);                                                        \
  template hipError_t launch_cg_step<T>(fbto_grid_s*, T*, T*, T*, const T*, T*, T*, const T*, const T*,  \
                                        int, int, int, int, double, hipStream_t, int*);                \
  template hipError_t launch_diag<T>(fbto_grid_s*, const T*, T*, hipStream_t);                         \
  template hipError_t launch_relax_update<T>(fbto_grid_s*, T*, const T*, const T*, int, double, int,    \
                                             hipStream_t);                                             \
  template hipError_t launch_sens<T>(fbto_grid_s*, const T*, const T*, const T*, int, T*, const T*,    \
                                     hipStream_t);                                                     \
  template hipError_t launch_dot<T>(fbto_grid_s*, const T*, const T*, int, hipStream_t);               \
  template hipError_t launch_filter<T>(fbto_grid_s*, int, const T*, T*, int, hipStream_t);             \
  template hipError_t launch_step<T>(fbto_grid_s*, const T*, const T*, T*, double, int, double,       \
                                     double, hipStream_t);                                             \
  template hipError_t launch_project<T>(fbto_grid_s*, const T*, T*, double, double, double, int,       \
                                        const T*, double*, hipStream_t);

FBTO_INST(double)
FBTO_INST(float)

}  // namespace fbto
