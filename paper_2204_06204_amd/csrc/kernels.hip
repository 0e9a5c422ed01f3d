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

inline int vec_blocks(int64_t n, int n_cu) {
  int64_t b = (n + kVecBlock - 1) / kVecBlock;
  int64_t cap = (int64_t)n_cu * 8;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

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

// ===========================================================================
// apply_K: z-marching tiles, one element column per thread.
//
// Block = BX x BY threads; thread (tx, ty) owns element column
// (ex, ey) = (bx (BX-1) - 1 + tx, by (BY-1) - 1 + ty) and marches the element
// layers of one z-slab.  Per layer it loads the four nodes of the element's
// upper face (the lower face is carried from the previous layer), computes
// the full 24-entry element product in the sum/difference basis, adds the
// lower-face half to the upper-face half carried from the layer below (this
// completes the z-sum of every node of the plane), and exchanges the four
// xy-corners through LDS so that each interior thread sums the four element
// columns around its node in a fixed order.  Neighbouring tiles overlap by
// one element column / row / layer, so no atomics are needed and the result
// is bitwise reproducible.
// ===========================================================================
template <typename T>
struct ApplyArgs {
  Geo g;
  const T* rho;
  const T* u;
  T* y;
  const T* f;
  const uint8_t* mask;
  Modal<T> km;
  Simp sp;
  int nspring;
  const int64_t* sdof;
  const T* sk;
  int tiles_x, tiles_y, slabs, dz, nblocks, per_xcd;
  double* partials;
  unsigned* counter;
  Scalars* sc;
};

template <typename T, int BX, int BY, int NR>
__global__ void __launch_bounds__(BX* BY)
    k_apply(ApplyArgs<T> A, int mode, int rhs0) {
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
  const int64_t ndof = G.ndof;

  T ul[NR][4][3], uu[NR][4][3], carry[NR][4][3];
  double dotacc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    dotacc[r] = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[r][a][c] = (T)0;
  }

  auto load_face = [&](int k, T(&dst)[NR][4][3]) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = ex + (a & 1), j = ey + (a >> 1);
      const bool ok = i >= 0 && i <= G.nx && j >= 0 && j <= G.ny && k >= 0 && k <= G.nz;
      int64_t n = 0;
      unsigned m = 7u;
      if (ok) {
        n = (int64_t)i + (int64_t)G.nxn * ((int64_t)j + (int64_t)G.nyn * k);
        m = A.mask[n];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          dst[r][a][c] = ((m >> c) & 1u) ? (T)0 : A.u[(int64_t)(rhs0 + r) * ndof + 3 * n + c];
    }
  };

  load_face(k0 - 1, ul);
  for (int ez = k0 - 1; ez < kend; ++ez) {
    load_face(ez + 1, uu);
    const bool el = xy_elem && ez >= 0 && ez < G.nz;
    T s = (T)0;
    if (el) s = simp_s<T>(A.rho[(int64_t)ex + (int64_t)G.nx * ((int64_t)ey + (int64_t)G.ny * ez)], A.sp);
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
        const int64_t n = (int64_t)(ex + 1) + (int64_t)G.nxn * ((int64_t)(ey + 1) + (int64_t)G.nyn * ez);
        const unsigned m = A.mask[n];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int64_t base = (int64_t)(rhs0 + r) * ndof + 3 * n;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            T acc = ((own[r][c] + lds[r][2][c][ty][tx + 1]) + lds[r][1][c][ty + 1][tx]) +
                    lds[r][0][c][ty + 1][tx + 1];
            T pv = ul[r][3][c];  // masked value of u at this node
            for (int sI = 0; sI < A.nspring; ++sI) {
              const int64_t d = A.sdof[sI];
              if (d == 3 * n + c) acc += A.sk[sI] * pv;
            }
            if ((m >> c) & 1u) {
              pv = A.u[base + c];
              acc = pv;
            }
            T outv = acc;
            if (mode == 1) outv = A.f[base + c] - acc;
            if (mode == 2) dotacc[r] += (double)pv * (double)acc;
            A.y[base + c] = outv;
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

  if (mode == 2) {
    if (grid_reduce<NR, 0u>(dotacc, lb, A.nblocks, A.partials, A.counter)) {
      if (tx == 0 && ty == 0) {
        Scalars* sc = A.sc;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int R = rhs0 + r;
          const double pq = dotacc[r], rz = sc->rz[R];
          sc->pq[R] = pq;
          double alpha = 0.0;
          if (sc->done[R] == 0.0) {
            if (pq > 0.0 && isfinite(pq)) {
              alpha = rz / pq;
            } else if (rz == 0.0) {
              sc->done[R] = 1.0;
            } else {
              sc->status[R] = isfinite(pq) ? (double)FBTO_ERR_BREAKDOWN : (double)FBTO_ERR_NONFINITE;
              sc->done[R] = 1.0;
            }
          }
          sc->alpha[R] = alpha;
        }
      }
    }
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

template <typename T, int BX, int BY, int NR>
static hipError_t launch_apply_t(const ApplyArgs<T>& A0, const TileChoice& t, int mode, int rhs0,
                                 hipStream_t st) {
  ApplyArgs<T> A = A0;
  A.tiles_x = t.tiles_x;
  A.tiles_y = t.tiles_y;
  A.slabs = t.slabs;
  A.dz = t.dz;
  A.nblocks = t.nblocks;
  A.per_xcd = (t.nblocks + 7) / 8;
  const int grid = A.per_xcd * 8;
  hipLaunchKernelGGL((k_apply<T, BX, BY, NR>), dim3(grid), dim3(BX, BY), 0, st, A, mode, rhs0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply(fbto_grid_s* g, const T* rho, const T* u, T* y, const T* f, int nrhs,
                        int mode, hipStream_t st) {
  ApplyArgs<T> A{};
  A.g = g->geo;
  A.rho = rho;
  A.u = u;
  A.y = y;
  A.f = f;
  A.mask = g->mask;
  A.km = modal_of<T>(g);
  A.sp = g->simp;
  A.nspring = g->n_springs;
  A.sdof = g->spring_dof;
  A.sk = spring_k_of<T>(g);
  A.partials = g->partials;
  A.counter = g->counters + CNT_APPLY;
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
    const bool wide = t.bx == 32;
    if (nr == 1) {
      e = wide ? launch_apply_t<T, 32, 8, 1>(A, t, mode, r0, st) : launch_apply_t<T, 16, 16, 1>(A, t, mode, r0, st);
    } else if (nr == 2) {
      e = wide ? launch_apply_t<T, 32, 8, 2>(A, t, mode, r0, st) : launch_apply_t<T, 16, 16, 2>(A, t, mode, r0, st);
    } else {
      if constexpr (!fp64) {
        e = wide ? launch_apply_t<T, 32, 8, 4>(A, t, mode, r0, st) : launch_apply_t<T, 16, 16, 4>(A, t, mode, r0, st);
      }
    }
    r0 += nr;
  }
  return e;
}

// ===========================================================================
// Jacobi diagonal: D = ke_diag * sum_{e at node} s_e (+ springs), 1 on fixed
// DOFs; stores its inverse per DOF.  Every diagonal entry of the unit-cube
// hex8 KE is the same number, so one sum per node serves all 3 DOFs.
// ===========================================================================
template <typename T>
__global__ void k_diag(Geo G, const T* rho, T* invD, const uint8_t* mask, Simp sp, double ke_diag,
                       int nspring, const int64_t* sdof, const T* sk) {
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < G.N;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % G.nxn);
    const int j = (int)((n / G.nxn) % G.nyn);
    const int k = (int)(n / ((int64_t)G.nxn * G.nyn));
    T acc = (T)0;
#pragma unroll
    for (int dz = -1; dz <= 0; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 0; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 0; ++dx) {
          const int ex = i + dx, ey = j + dy, ez = k + dz;
          if (ex >= 0 && ex < G.nx && ey >= 0 && ey < G.ny && ez >= 0 && ez < G.nz)
            acc += simp_s<T>(rho[(int64_t)ex + (int64_t)G.nx * ((int64_t)ey + (int64_t)G.ny * ez)], sp);
        }
    const unsigned m = mask[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T d = (T)ke_diag * acc;
      for (int s = 0; s < nspring; ++s)
        if (sdof[s] == 3 * n + c) d += sk[s];
      if ((m >> c) & 1u) d = (T)1;
      invD[3 * n + c] = d > (T)0 ? (T)1 / d : (T)0;
    }
  }
}

template <typename T>
hipError_t launch_diag(fbto_grid_s* g, const T* rho, T* invD, hipStream_t st) {
  const int nb = vec_blocks(g->geo.N, g->n_cu);
  hipLaunchKernelGGL((k_diag<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, rho, invD, g->mask,
                     g->simp, g->ke_diag, g->n_springs, g->spring_dof, spring_k_of<T>(g));
  return hipGetLastError();
}

// ===========================================================================
// PCG vector kernels (FP64 dot products with a fixed summation order).
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_pcg_init(int64_t ndof, int nrhs, const T* r, T* p, const T* invD, const T* f, double rtol,
               Scalars* sc, double* partials, unsigned* counter) {
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ndof;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T di = invD[i];
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if (R >= nrhs) break;
      const T ri = r[R * ndof + i];
      const T zi = di * ri;
      p[R * ndof + i] = zi;
      const T fi = f[R * ndof + i];
      v[4 * R + 0] += (double)ri * (double)zi;
      v[4 * R + 1] += (double)fi * (double)fi;
      v[4 * R + 2] += (double)ri * (double)ri;
      v[4 * R + 3] = fmax(v[4 * R + 3], fabs((double)ri));
    }
  }
  if (grid_reduce<16, 0x8888u>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) {
      for (int R = 0; R < nrhs; ++R) {
        sc->rz[R] = v[4 * R + 0];
        sc->fnorm2[R] = sqrt(v[4 * R + 1]);
        sc->rnorm2[R] = sqrt(v[4 * R + 2]);
        sc->rinf[R] = v[4 * R + 3];
        sc->tol[R] = rtol * sc->fnorm2[R];
        sc->steps[R] = 0.0;
        sc->status[R] = isfinite(v[4 * R + 0]) ? 0.0 : (double)FBTO_ERR_NONFINITE;
        sc->done[R] = (rtol > 0.0 && sc->rnorm2[R] <= sc->tol[R]) || sc->status[R] != 0.0 ? 1.0 : 0.0;
        sc->alpha[R] = 0.0;
        sc->beta[R] = 0.0;
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_pcg_update(int64_t ndof, int nrhs, T* u, T* r, const T* p, const T* q, const T* invD,
                 Scalars* sc, double* partials, unsigned* counter) {
  double v[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) v[i] = 0.0;
  T al[4];
#pragma unroll
  for (int R = 0; R < 4; ++R) al[R] = R < nrhs ? (T)sc->alpha[R] : (T)0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ndof;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T di = invD[i];
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if (R >= nrhs) break;
      const int64_t o = R * ndof + i;
      const T pi = p[o];
      u[o] = u[o] + al[R] * pi;
      const T ri = r[o] - al[R] * q[o];
      r[o] = ri;
      const T zi = di * ri;
      v[3 * R + 0] += (double)ri * (double)zi;
      v[3 * R + 1] += (double)ri * (double)ri;
      v[3 * R + 2] = fmax(v[3 * R + 2], fabs((double)ri));
    }
  }
  if (grid_reduce<12, 0x924u>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) {
      for (int R = 0; R < nrhs; ++R) {
        if (sc->done[R] != 0.0) {
          sc->beta[R] = 0.0;
          continue;
        }
        const double rz_new = v[3 * R + 0];
        const double rz = sc->rz[R];
        sc->beta[R] = rz != 0.0 ? rz_new / rz : 0.0;
        sc->rz[R] = rz_new;
        sc->rnorm2[R] = sqrt(v[3 * R + 1]);
        sc->rinf[R] = v[3 * R + 2];
        sc->steps[R] += 1.0;
        if (!isfinite(rz_new)) {
          sc->status[R] = (double)FBTO_ERR_NONFINITE;
          sc->done[R] = 1.0;
        } else if (sc->tol[R] > 0.0 && sc->rnorm2[R] <= sc->tol[R]) {
          sc->done[R] = 1.0;
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_pcg_pupdate(int64_t ndof, int nrhs, const T* r, T* p, const T* invD, const Scalars* sc) {
  T be[4];
#pragma unroll
  for (int R = 0; R < 4; ++R) be[R] = R < nrhs ? (T)sc->beta[R] : (T)0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ndof;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T di = invD[i];
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if (R >= nrhs) break;
      const int64_t o = R * ndof + i;
      p[o] = di * r[o] + be[R] * p[o];
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

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_norms(int64_t ndof, int nrhs, const T* r, Scalars* sc, double* partials, unsigned* counter) {
  double v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ndof;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if (R >= nrhs) break;
      const double ri = (double)r[R * ndof + i];
      v[2 * R] += ri * ri;
      v[2 * R + 1] = fmax(v[2 * R + 1], fabs(ri));
    }
  }
  if (grid_reduce<8, 0xAAu>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) {
      for (int R = 0; R < nrhs; ++R) {
        sc->rnorm2[R] = sqrt(v[2 * R]);
        sc->rinf[R] = v[2 * R + 1];
        if (!isfinite(v[2 * R])) sc->status[R] = (double)FBTO_ERR_NONFINITE;
      }
    }
  }
}

template <typename T>
hipError_t launch_pcg_init(fbto_grid_s* g, const T* r, T* p, const T* invD, int nrhs, const T* f,
                           double rtol, hipStream_t st) {
  const int nb = vec_blocks(g->geo.ndof, g->n_cu);
  hipLaunchKernelGGL((k_pcg_init<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, nrhs, r, p, invD,
                     f, rtol, g->sc, g->partials, g->counters + CNT_INIT);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_pcg_update(fbto_grid_s* g, T* u, T* r, const T* p, const T* q, const T* invD,
                             int nrhs, hipStream_t st) {
  const int nb = vec_blocks(g->geo.ndof, g->n_cu);
  hipLaunchKernelGGL((k_pcg_update<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, nrhs, u, r, p,
                     q, invD, g->sc, g->partials, g->counters + CNT_UPDATE);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_pcg_pupdate(fbto_grid_s* g, const T* r, T* p, const T* invD, int nrhs,
                              hipStream_t st) {
  const int nb = vec_blocks(g->geo.ndof, g->n_cu);
  hipLaunchKernelGGL((k_pcg_pupdate<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, nrhs, r, p,
                     invD, (const Scalars*)g->sc);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_relax_update(fbto_grid_s* g, T* u, const T* r, const T* invD, int nrhs,
                               double omega, int use_diag, hipStream_t st) {
  const int nb = vec_blocks(g->geo.ndof, g->n_cu);
  hipLaunchKernelGGL((k_relax_update<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, nrhs, u, r,
                     invD, (T)omega, use_diag);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_norms(fbto_grid_s* g, const T* r, int nrhs, hipStream_t st) {
  const int nb = vec_blocks(g->geo.ndof, g->n_cu);
  hipLaunchKernelGGL((k_norms<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.ndof, nrhs, r, g->sc,
                     g->partials, g->counters + CNT_MISC);
  return hipGetLastError();
}

// ===========================================================================
// Sensitivity: dobj_e = -ds_e sum_r lam_{r,e}^T KE u_{r,e}, element strains
// recomputed from the nodal vectors (one element per thread).
// ===========================================================================
template <typename T>
__device__ __forceinline__ void gather_elem(const Geo& G, const T* v, const uint8_t* mask, int ex,
                                            int ey, int ez, T (&ue)[8][3]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int64_t n = (int64_t)(ex + (a & 1)) +
                      (int64_t)G.nxn * ((int64_t)(ey + ((a >> 1) & 1)) + (int64_t)G.nyn * (ez + (a >> 2)));
    const unsigned m = mask[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) ue[a][c] = ((m >> c) & 1u) ? (T)0 : v[3 * n + c];
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_sens(Geo G, const T* rho, const T* u, const T* lam, int nrhs, T* dobj, const uint8_t* mask,
           Modal<T> km, Simp sp) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < G.E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int ex = (int)(e % G.nx);
    const int ey = (int)((e / G.nx) % G.ny);
    const int ez = (int)(e / ((int64_t)G.nx * G.ny));
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
    dobj[e] = (T)(-(double)simp_ds<T>(rho[e], sp) * acc);
  }
}

template <typename T>
hipError_t launch_sens(fbto_grid_s* g, const T* rho, const T* u, const T* lam, int nrhs, T* dobj,
                       hipStream_t st) {
  const int nb = vec_blocks(g->geo.E, g->n_cu);
  hipLaunchKernelGGL((k_sens<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, rho, u, lam, nrhs, dobj,
                     g->mask, modal_of<T>(g), g->simp);
  return hipGetLastError();
}

// sum_r a_r . b_r for nrhs vectors of length n (stride n) -> out[r]
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_dot(int64_t n, int nrhs, const T* a, const T* b, double* out, double* partials, unsigned* counter) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if (R >= nrhs) break;
      v[R] += (double)a[R * n + i] * (double)b[R * n + i];
    }
  }
  if (grid_reduce<4, 0u>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int R = 0; R < nrhs; ++R) tot += v[R];
      out[0] = tot;
    }
  }
}

template <typename T>
hipError_t launch_dot(fbto_grid_s* g, const T* a, const T* b, int64_t n, int nrhs, double* out,
                      hipStream_t st) {
  const int nb = vec_blocks(n, g->n_cu);
  hipLaunchKernelGGL((k_dot<T>), dim3(nb), dim3(kVecBlock), 0, st, n, nrhs, a, b, out, g->partials,
                     g->counters + CNT_DOT);
  return hipGetLastError();
}

// ===========================================================================
// Linear cone filter: gather over the stencil (offsets with r - |d| > 0).
//   forward:   out_e = sum_o w_o in_{e+o} / Hs_e
//   transpose: out_j = sum_o w_o in_{j+o} / Hs_{j+o}
// want_sum: also reduce sum(out) into sc->gsum / gmean.
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_filter(Geo G, int transpose, const T* in, T* out, const T* Hs, int nst, const int* off,
             const T* w, int want_sum, Scalars* sc, double* partials, unsigned* counter) {
  double v[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < G.E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int ex = (int)(e % G.nx);
    const int ey = (int)((e / G.nx) % G.ny);
    const int ez = (int)(e / ((int64_t)G.nx * G.ny));
    T acc = (T)0;
    for (int o = 0; o < nst; ++o) {
      const int jx = ex + off[3 * o], jy = ey + off[3 * o + 1], jz = ez + off[3 * o + 2];
      if (jx < 0 || jx >= G.nx || jy < 0 || jy >= G.ny || jz < 0 || jz >= G.nz) continue;
      const int64_t j = (int64_t)jx + (int64_t)G.nx * ((int64_t)jy + (int64_t)G.ny * jz);
      acc += transpose ? w[o] * (in[j] / Hs[j]) : w[o] * in[j];
    }
    const T res = transpose ? acc : acc / Hs[e];
    out[e] = res;
    v[0] += (double)res;
  }
  if (want_sum) {
    if (grid_reduce<1, 0u>(v, blockIdx.x, gridDim.x, partials, counter)) {
      if (threadIdx.x == 0) {
        sc->gsum = v[0];
        sc->gmean = v[0] / (double)G.E;
      }
    }
  }
}

template <typename T>
__global__ void k_hs(Geo G, T* Hs, int nst, const int* off, const T* w) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < G.E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int ex = (int)(e % G.nx);
    const int ey = (int)((e / G.nx) % G.ny);
    const int ez = (int)(e / ((int64_t)G.nx * G.ny));
    T acc = (T)0;
    for (int o = 0; o < nst; ++o) {
      const int jx = ex + off[3 * o], jy = ey + off[3 * o + 1], jz = ez + off[3 * o + 2];
      if (jx < 0 || jx >= G.nx || jy < 0 || jy >= G.ny || jz < 0 || jz >= G.nz) continue;
      acc += w[o];
    }
    Hs[e] = acc;
  }
}

template <typename T>
hipError_t launch_filter(fbto_grid_s* g, int transpose, const T* in, T* out, int want_sum,
                         hipStream_t st) {
  Vecs& V = vecs_of<T>(g);
  const int nb = vec_blocks(g->geo.E, g->n_cu);
  hipLaunchKernelGGL((k_filter<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, transpose, in, out,
                     (const T*)V.Hs, g->n_stencil, (const int*)g->stencil_off, stencil_w_of<T>(g),
                     want_sum, g->sc, g->partials, g->counters + CNT_FILT);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hs(fbto_grid_s* g, T* Hs, hipStream_t st) {
  const int nb = vec_blocks(g->geo.E, g->n_cu);
  hipLaunchKernelGGL((k_hs<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo, Hs, g->n_stencil,
                     (const int*)g->stencil_off, stencil_w_of<T>(g));
  return hipGetLastError();
}
template hipError_t launch_hs<double>(fbto_grid_s*, double*, hipStream_t);
template hipError_t launch_hs<float>(fbto_grid_s*, float*, hipStream_t);

// ===========================================================================
// Design step and projection onto {lo <= x <= hi, sum x <= vmax}.
// ===========================================================================
// Shared by the step kernel and the stand-alone projection: after the
// reduction of S0 = sum clamp(y), ymax and the count of strictly interior
// entries, decide whether the box clamp is feasible and seed the search.
__device__ void proj_seed(Scalars* sc, double S0, double ymax, double nact0, double lo, double hi,
                          double vmax) {
  sc->sum0 = S0;
  sc->ymax = ymax;
  sc->proj_status = 0.0;
  if (S0 <= vmax) {
    sc->proj_done = 1.0;
    sc->lam = 0.0;
    return;
  }
  sc->proj_done = 0.0;
  const double a = 0.0, b = ymax - lo;  // f(0) = S0 > vmax, f(b) = E lo <= vmax
  sc->br_a = a;
  sc->br_b = b;
  double lam;
  const double prev = sc->lam_prev;
  if (prev > a && prev < b) {
    lam = prev;
  } else if (nact0 > 0.0) {
    lam = (S0 - vmax) / nact0;
    if (!(lam > a && lam < b)) lam = 0.5 * (a + b);
  } else {
    lam = 0.5 * (a + b);
  }
  sc->lam = lam;
  (void)hi;
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_step(int64_t E, const T* x, const T* gx, T* y, double half_alpha, int mean_project, double lo,
           double hi, double vmax, Scalars* sc, double* partials, unsigned* counter) {
  const double mean = mean_project ? sc->gmean : 0.0;
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
  if (grid_reduce<3, 0x2u>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) proj_seed(sc, v[0], v[1], v[2], lo, hi, vmax);
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_init(int64_t E, const T* y, double lo, double hi, double vmax, Scalars* sc,
                double* partials, unsigned* counter) {
  double v[3] = {0.0, -INFINITY, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double yd = (double)y[e];
    v[0] += fmin(fmax(yd, lo), hi);
    v[1] = fmax(v[1], yd);
    v[2] += (yd > lo && yd < hi) ? 1.0 : 0.0;
  }
  if (grid_reduce<3, 0x2u>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) proj_seed(sc, v[0], v[1], v[2], lo, hi, vmax);
  }
}

// One search pass at the current lambda.  f(lambda) = sum clamp(y - lambda)
// is continuous, non-increasing and linear between the breakpoints y - lo,
// y - hi.  The pass classifies every entry both just right (+) and just left
// (-) of lambda, which fixes the linear piece on each side:
//   f(l') = hi nU + lo nL + sum_A y - l' nA   on that piece,
// so the root on the piece towards vmax is solved exactly; if it lies
// beyond the neighbouring breakpoint the pass becomes a safeguarded Newton
// (or bisection) step on the bracket [a, b].
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_pass(int64_t E, const T* y, double lo, double hi, double vmax, Scalars* sc,
                double* partials, unsigned* counter) {
  if (sc->proj_done != 0.0) return;
  const double lam = sc->lam;
  // 0 f, 1 nA+, 2 sA+, 3 nU+, 4 nL+, 5 nA-, 6 sA-, 7 nU-, 8 nL-, 9 lb (max), 10 -ub (max)
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
    // right of lambda: U if t > hi, L if t <= lo, else active
    if (t > hi) v[3] += 1.0;
    else if (t <= lo) v[4] += 1.0;
    else { v[1] += 1.0; v[2] += yd; }
    // left of lambda: U if t >= hi, L if t < lo, else active
    if (t >= hi) v[7] += 1.0;
    else if (t < lo) v[8] += 1.0;
    else { v[5] += 1.0; v[6] += yd; }
    const double b1 = yd - lo, b2 = yd - hi;
    if (b1 < lam) v[9] = fmax(v[9], b1); else if (b1 > lam) v[10] = fmax(v[10], -b1);
    if (b2 < lam) v[9] = fmax(v[9], b2); else if (b2 > lam) v[10] = fmax(v[10], -b2);
  }
  if (grid_reduce<11, 0x600u>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) {
      const double F = v[0];
      double a = sc->br_a, b = sc->br_b;
      const double lb = v[9], ub = -v[10];
      double next;
      bool done = false;
      if (!isfinite(F)) {
        sc->proj_status = (double)FBTO_ERR_NONFINITE;
        sc->proj_done = 1.0;
        return;
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
      sc->br_a = a;
      sc->br_b = b;
      sc->lam = next;
      if (done || !(b > a) || next == a || next == b) {
        sc->proj_done = 1.0;
        if (!done) sc->lam = b;  // bracket collapsed: b is feasible
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_proj_final(int64_t E, const T* y, T* x, double lo, double hi, const T* x_old, Scalars* sc,
                 double* info, double* lam_out, double* partials, unsigned* counter) {
  double lam = sc->lam;
  if (sc->proj_done == 0.0) lam = sc->br_b;  // search not finished: feasible end
  double v[2] = {0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (int64_t)gridDim.x * blockDim.x) {
    const T xe = (T)fmin(fmax((double)y[e] - lam, lo), hi);
    if (x_old) v[1] = fmax(v[1], fabs((double)xe - (double)x_old[e]));
    x[e] = xe;
    v[0] += (double)xe;
  }
  if (grid_reduce<2, 0x2u>(v, blockIdx.x, gridDim.x, partials, counter)) {
    if (threadIdx.x == 0) {
      if (sc->proj_done == 0.0) sc->proj_status = -1.0;  // not converged in the pass budget
      sc->lam_prev = lam;
      sc->work[0] = v[0];
      sc->work[1] = v[1];
      sc->work[2] = lam;
      if (lam_out) *lam_out = lam;
      if (info) {
        info[FBTO_OI_LAMBDA] = lam;
        info[FBTO_OI_VOLUME] = v[0];
        info[FBTO_OI_DX_INF] = v[1];
      }
    }
  }
}

static int proj_passes() {
  const char* env = getenv("FBTO_PROJ_PASSES");
  int p = env ? atoi(env) : 12;
  return p < 1 ? 1 : (p > 64 ? 64 : p);
}

template <typename T>
hipError_t launch_step_v(fbto_grid_s* g, const T* x, const T* gx, T* y, double half_alpha,
                         int mean_project, double lo, double hi, double vmax, hipStream_t st) {
  const int nb = vec_blocks(g->geo.E, g->n_cu);
  hipLaunchKernelGGL((k_step<T>), dim3(nb), dim3(kVecBlock), 0, st, g->geo.E, x, gx, y, half_alpha,
                     mean_project, lo, hi, vmax, g->sc, g->partials, g->counters + CNT_STEP);
  return hipGetLastError();
}
template hipError_t launch_step_v<double>(fbto_grid_s*, const double*, const double*, double*, double,
                                          int, double, double, double, hipStream_t);
template hipError_t launch_step_v<float>(fbto_grid_s*, const float*, const float*, float*, double, int,
                                         double, double, double, hipStream_t);

template <typename T>
hipError_t launch_project(fbto_grid_s* g, const T* y, T* x, double lo, double hi, double vmax,
                          int have_seed, const T* x_old, double* lam_out, double* info,
                          hipStream_t st) {
  const int64_t E = g->geo.E;
  const int nb = vec_blocks(E, g->n_cu);
  if (!have_seed) {
    hipLaunchKernelGGL((k_proj_init<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, lo, hi, vmax, g->sc,
                       g->partials, g->counters + CNT_PROJ);
  }
  const int passes = proj_passes();
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_proj_pass<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, lo, hi, vmax, g->sc,
                       g->partials, g->counters + CNT_PROJ);
  }
  hipLaunchKernelGGL((k_proj_final<T>), dim3(nb), dim3(kVecBlock), 0, st, E, y, x, lo, hi, x_old,
                     g->sc, info, lam_out, g->partials, g->counters + CNT_PROJF);
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

template <typename T>
hipError_t launch_convert(const void* in, void* out, int64_t n, int to_double, hipStream_t st) {
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (to_double)
    hipLaunchKernelGGL(k_f32_to_f64, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, (const float*)in,
                       (double*)out, n);
  else
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, (const double*)in,
                       (float*)out, n);
  return hipGetLastError();
}
template hipError_t launch_convert<float>(const void*, void*, int64_t, int, hipStream_t);

hipError_t launch_axpy64(double* u, const double* d, int64_t n, hipStream_t st) {
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_axpy64, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, u, d, n);
  return hipGetLastError();
}
hipError_t launch_ir_scale(fbto_grid_s* g, const double* r64, float* r32, int nrhs, hipStream_t st) {
  return launch_convert<float>(r64, r32, g->geo.ndof * nrhs, 0, st);
}
hipError_t launch_ir_accum(fbto_grid_s* g, double* u64, const float* d32, int nrhs, hipStream_t st) {
  const int64_t n = g->geo.ndof * nrhs;
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_accum_f32, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, u64, d32, n);
  return hipGetLastError();
}

// ===========================================================================
// Info records and scalar resets (single-thread bookkeeping kernels).
// ===========================================================================
__global__ void k_outer_info(Scalars* sc, double* info, int nrhs) {
  double rinf = 0.0, rrel = 0.0, status = 0.0;
  for (int R = 0; R < nrhs; ++R) {
    rinf = fmax(rinf, sc->rinf[R]);
    const double rel = sc->fnorm2[R] > 0.0 ? sc->rnorm2[R] / sc->fnorm2[R] : sc->rnorm2[R];
    rrel = fmax(rrel, rel);
    if (sc->status[R] != 0.0) status = sc->status[R];
  }
  if (sc->proj_status > 0.0) status = sc->proj_status;
  info[FBTO_OI_COMPLIANCE] = sc->dot[0];
  info[FBTO_OI_R_INF] = rinf;
  info[FBTO_OI_RREL] = rrel;
  info[FBTO_OI_STATUS] = status;
  info[FBTO_OI_GRAD_MEAN] = sc->gmean;
}
__global__ void k_solve_info(Scalars* sc, double* info, int nrhs) {
  for (int R = 0; R < nrhs; ++R) {
    double* o = info + R * FBTO_SOLVE_INFO;
    o[FBTO_SI_RNORM2] = sc->rnorm2[R];
    o[FBTO_SI_RNORMI] = sc->rinf[R];
    o[FBTO_SI_FNORM2] = sc->fnorm2[R];
    o[FBTO_SI_STEPS] = sc->steps[R];
    o[FBTO_SI_STATUS] = sc->status[R];
    for (int k = 5; k < FBTO_SOLVE_INFO; ++k) o[k] = 0.0;
  }
}
__global__ void k_scalar_reset(Scalars* sc, int nrhs) {
  for (int R = 0; R < 4; ++R) {
    sc->status[R] = 0.0;
    sc->done[R] = 0.0;
    sc->steps[R] = 0.0;
  }
  (void)nrhs;
}

hipError_t launch_outer_info(fbto_grid_s* g, double* info, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_outer_info, dim3(1), dim3(1), 0, st, g->sc, info, nrhs);
  return hipGetLastError();
}
hipError_t launch_solve_info(fbto_grid_s* g, double* info, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_solve_info, dim3(1), dim3(1), 0, st, g->sc, info, nrhs);
  return hipGetLastError();
}
hipError_t launch_scalar_reset(fbto_grid_s* g, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_reset, dim3(1), dim3(1), 0, st, g->sc, nrhs);
  return hipGetLastError();
}

// ---- explicit instantiations ----------------------------------------------
#define FBTO_INST(T)                                                                                 \
  template hipError_t launch_apply<T>(fbto_grid_s*, const T*, const T*, T*, const T*, int, int,     \
                                      hipStream_t);                                                  \
  template hipError_t launch_diag<T>(fbto_grid_s*, const T*, T*, hipStream_t);                       \
  template hipError_t launch_pcg_init<T>(fbto_grid_s*, const T*, T*, const T*, int, const T*, double, \
                                         hipStream_t);                                               \
  template hipError_t launch_pcg_update<T>(fbto_grid_s*, T*, T*, const T*, const T*, const T*, int,   \
                                           hipStream_t);                                             \
  template hipError_t launch_pcg_pupdate<T>(fbto_grid_s*, const T*, T*, const T*, int, hipStream_t);  \
  template hipError_t launch_relax_update<T>(fbto_grid_s*, T*, const T*, const T*, int, double, int,  \
                                             hipStream_t);                                           \
  template hipError_t launch_norms<T>(fbto_grid_s*, const T*, int, hipStream_t);                     \
  template hipError_t launch_sens<T>(fbto_grid_s*, const T*, const T*, const T*, int, T*,            \
                                     hipStream_t);                                                   \
  template hipError_t launch_dot<T>(fbto_grid_s*, const T*, const T*, int64_t, int, double*,         \
                                    hipStream_t);                                                    \
  template hipError_t launch_filter<T>(fbto_grid_s*, int, const T*, T*, int, hipStream_t);           \
  template hipError_t launch_project<T>(fbto_grid_s*, const T*, T*, double, double, double, int,     \
                                        const T*, double*, double*, hipStream_t);

FBTO_INST(double)
FBTO_INST(float)

}  // namespace fbto
