// Plane (2D) variant of the hot path: the unit-square bilinear quadrilateral
// (Q4, plane stress) on a regular nx x ny grid -- the paper's own setting
// (Sec. 4.3 regular-grid discretisation, Sec. 5 experiments) -- and the
// separable Gaussian density filter of its experiments (Sec. 5, filter
// paragraph; Remark on modifiers, Sec. 3).
//
// Layout: node n = i + (nx + 1) j, DOF 2 n + c, element e = ex + nx ey,
// element-local node a = ax + 2 ay.  Multi-RHS vectors are [nrhs][2N].
//
// The plane grids of the paper (at most 192 x 576 elements, 0.9 MB per FP32
// vector) sit in the L2 and Infinity caches, so these kernels gather
// directly from global memory: one node (apply) or element (sensitivity)
// per thread, its 3 x 3 node neighbourhood read through L1/L2.  The
// reductions use the per-block partial slots of the 3D path, with the same
// meaning, so the CG, MINRES, projection and finishing kernels serve both.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "internal.h"

namespace fbto {

namespace {
constexpr int kPlaneBlock = 256;

enum { PL_APPLY = 0, PL_RESID = 1, PL_CG = 2 };

template <typename T>
struct PlaneArgs {
  int nx, ny;
  int64_t N, ndof;
  const T* rho;
  const T* u;          // input vector
  T* y;                // output: K u, r = f - K u, or w = K z
  const T* f;          // RESID
  const T* invD;       // RESID (optional): z = D^-1 r from this diagonal
  T* invD_out;         // RESID (optional): form the Jacobi diagonal, store it, z from it
  T* z;                // RESID
  const T* r;          // CG: the residual paired with the product's partials
  const uint8_t* mask; // bit c: DOF c of the node fixed
  Q4<T> ke;
  double ke_diag;
  Simp sp;
  double* P;
  int maxp;
  Scalars* sc;
  int step;            // CG: the partials go to the set of parity step & 1
};

// the |r|_inf entries (max-reduced) of the per-RHS triples |r|^2, |r|_inf, |f|^2
constexpr unsigned resid_max_mask(int nr) {
  unsigned m = 0u;
  for (int r = 0; r < nr; ++r) m |= 1u << (3 * r + 1);
  return m;
}

__device__ __forceinline__ double* pslot2(double* P, int slot, int r, int maxp) {
  return P + ((int64_t)slot * 4 + r) * maxp;
}

// y = K u at node (i, j) for NR vectors, gathered from the four elements
// around the node; fixed DOFs of the neighbours enter as zero.
template <typename T, int NR, int MODE>
__global__ void __launch_bounds__(kPlaneBlock) k_plane_apply(PlaneArgs<T> A, int rhs0) {
  constexpr int NP = MODE == PL_APPLY ? 1 : 4 * NR;
  double part[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) part[i] = 0.0;
  const int nxn = A.nx + 1;
  for (int64_t nn = (int64_t)blockIdx.x * kPlaneBlock + threadIdx.x; nn < A.N;
       nn += (int64_t)gridDim.x * kPlaneBlock) {
    const int n = (int)nn;
    const int j = n / nxn, i = n - j * nxn;
    // masked values of the 3 x 3 node neighbourhood, [dy][dx][c]
    T un[NR][3][3][2];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int ii = i + dx - 1, jj = j + dy - 1;
        const bool ok = ii >= 0 && ii <= A.nx && jj >= 0 && jj <= A.ny;
        const int m = ok ? ii + nxn * jj : n;
        const unsigned mv = ok ? A.mask[m] : 3u;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const T v = A.u[(int64_t)(rhs0 + r) * A.ndof + 2 * m + c];
            un[r][dy][dx][c] = ((mv >> c) & 1u) ? (T)0 : v;
          }
      }
    // the four elements: (i - ax, j - ay), node local index a = ax + 2 ay
    T acc[NR][2];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r][0] = acc[r][1] = (T)0;
    T ssum = (T)0;
#pragma unroll
    for (int ay = 0; ay < 2; ++ay)
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) {
        const int ex = i - ax, ey = j - ay;
        const bool ok = ex >= 0 && ex < A.nx && ey >= 0 && ey < A.ny;
        const T rv = A.rho[ok ? ex + A.nx * ey : 0];
        const T s = ok ? simp_s<T>(rv, A.sp) : (T)0;
        ssum += s;
        const int a = ax + 2 * ay;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            T t = (T)0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const int bx = b & 1, by = b >> 1;
              // element node b is neighbourhood node (bx - ax + 1, by - ay + 1)
#pragma unroll
              for (int d = 0; d < 2; ++d) t += A.ke.k[2 * a + c][2 * b + d] * un[r][by - ay + 1][bx - ax + 1][d];
            }
            acc[r][c] += s * t;
          }
      }
    const unsigned m = A.mask[n];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t o = (int64_t)(rhs0 + r) * A.ndof + 2 * (int64_t)n;
      T pv[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        pv[c] = A.u[o + c];  // the own value, unmasked
        if ((m >> c) & 1u) acc[r][c] = pv[c];  // identity row of a fixed DOF
      }
      if constexpr (MODE == PL_APPLY) {
#pragma unroll
        for (int c = 0; c < 2; ++c) A.y[o + c] = acc[r][c];
      } else if constexpr (MODE == PL_RESID) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const T fv = A.f[o + c];
          const T rv = fv - acc[r][c];
          A.y[o + c] = rv;
          if (A.invD_out || A.invD) {
            T dl;
            if (A.invD_out) {
              T d = (T)A.ke_diag * ssum;
              if ((m >> c) & 1u) d = (T)1;
              dl = d > (T)0 ? (T)1 / d : (T)0;
              if (r == 0) A.invD_out[2 * (int64_t)n + c] = dl;
            } else {
              dl = A.invD[2 * (int64_t)n + c];
            }
            A.z[o + c] = dl * rv;
          }
          part[4 * r + 0] += (double)rv * (double)rv;
          part[4 * r + 1] = fmax(part[4 * r + 1], fabs((double)rv));
          part[4 * r + 2] += (double)fv * (double)fv;
        }
      } else {  // PL_CG
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          A.y[o + c] = acc[r][c];
          const T rv = A.r[o + c];
          part[4 * r + 0] += (double)rv * (double)pv[c];          // r.z
          part[4 * r + 1] += (double)acc[r][c] * (double)pv[c];   // w.z
          part[4 * r + 2] += (double)rv * (double)rv;             // r.r
          part[4 * r + 3] = fmax(part[4 * r + 3], fabs((double)rv));
        }
      }
    }
  }
  if constexpr (MODE == PL_CG) {
    const int par = A.step & 1;
    double* dst[4 * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      dst[4 * r + 0] = pslot2(A.P, P_RZ0 + par, rhs0 + r, A.maxp);
      dst[4 * r + 1] = pslot2(A.P, P_PQ0 + par, rhs0 + r, A.maxp);
      dst[4 * r + 2] = pslot2(A.P, P_RN0 + par, rhs0 + r, A.maxp);
      dst[4 * r + 3] = pslot2(A.P, P_RI0 + par, rhs0 + r, A.maxp);
    }
    write_parts<4 * NR, 0x8888u>(part, dst, blockIdx.x);
  }
  if constexpr (MODE == PL_RESID) {
    if (A.invD == nullptr && A.invD_out == nullptr) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // a new solve starts from this residual
      for (int r = 0; r < NR; ++r) {
        A.sc->done[rhs0 + r] = 0.0;
        A.sc->status[rhs0 + r] = 0.0;
        A.sc->steps[rhs0 + r] = 0.0;
      }
    }
    double v[3 * NR];
    double* dst[3 * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      v[3 * r + 0] = part[4 * r + 0];
      v[3 * r + 1] = part[4 * r + 1];
      v[3 * r + 2] = part[4 * r + 2];
      dst[3 * r + 0] = pslot2(A.P, P_RNF, rhs0 + r, A.maxp);
      dst[3 * r + 1] = pslot2(A.P, P_RIF, rhs0 + r, A.maxp);
      dst[3 * r + 2] = pslot2(A.P, P_FN, rhs0 + r, A.maxp);
    }
    write_parts<3 * NR, resid_max_mask(NR)>(v, dst, blockIdx.x);
  }
}

// Jacobi diagonal: ke_diag * (sum of s over the node's elements), 1 at fixed DOFs.
template <typename T>
__global__ void __launch_bounds__(kPlaneBlock)
    k_plane_diag(int nx, int ny, int64_t N, const T* rho, T* invD, const uint8_t* mask, Simp sp, double ke_diag) {
  const int nxn = nx + 1;
  for (int64_t nn = (int64_t)blockIdx.x * kPlaneBlock + threadIdx.x; nn < N; nn += (int64_t)gridDim.x * kPlaneBlock) {
    const int n = (int)nn;
    const int j = n / nxn, i = n - j * nxn;
    T acc = (T)0;
#pragma unroll
    for (int dy = -1; dy <= 0; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 0; ++dx) {
        const int ex = i + dx, ey = j + dy;
        const bool ok = ex >= 0 && ex < nx && ey >= 0 && ey < ny;
        const T rv = rho[ok ? ex + nx * ey : 0];
        acc += ok ? simp_s<T>(rv, sp) : (T)0;
      }
    const unsigned m = mask[n];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      T d = (T)ke_diag * acc;
      if ((m >> c) & 1u) d = (T)1;
      invD[2 * nn + c] = d > (T)0 ? (T)1 / d : (T)0;
    }
  }
}

// dobj_e = -ds_e sum_r lam_{r,e}^T KE u_{r,e} (times Hsi_e when given).
template <typename T>
__global__ void __launch_bounds__(kPlaneBlock)
    k_plane_sens(int nx, int ny, int64_t ndof, const T* rho, const T* u, const T* lam, int nrhs, T* dobj,
                 const uint8_t* mask, Q4<T> ke, Simp sp, const T* Hsi) {
  const int64_t E = (int64_t)nx * ny;
  const int nxn = nx + 1;
  for (int64_t ee = (int64_t)blockIdx.x * kPlaneBlock + threadIdx.x; ee < E; ee += (int64_t)gridDim.x * kPlaneBlock) {
    const int e = (int)ee;
    const int ey = e / nx, ex = e - ey * nx;
    double acc = 0.0;
    for (int R = 0; R < nrhs; ++R) {
      T ue[8], le[8];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int n = (ex + (a & 1)) + nxn * (ey + (a >> 1));
        const unsigned m = mask[n];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const T uv = u[R * ndof + 2 * n + c];
          const T lv = lam ? lam[R * ndof + 2 * n + c] : uv;
          ue[2 * a + c] = ((m >> c) & 1u) ? (T)0 : uv;
          le[2 * a + c] = ((m >> c) & 1u) ? (T)0 : lv;
        }
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        T t = (T)0;
#pragma unroll
        for (int q = 0; q < 8; ++q) t += ke.k[p][q] * ue[q];
        acc += (double)le[p] * (double)t;
      }
    }
    double val = -(double)simp_ds<T>(rho[e], sp) * acc;
    if (Hsi) val *= (double)Hsi[e];
    dobj[e] = (T)val;
  }
}

// One 1D pass of the separable Gaussian along `axis` (0: x, 1: y):
//   out_e = sum_{|d| <= half, e + d inside} g(d) pre_{e+d} in_{e+d}  (/ h_e if normalise)
// h_e = sum of g(d) over the offsets inside the grid.  pre: optional
// per-element factor (1/Hs of the transpose).  want_sum: per-block partial
// sums of out into slot GSUM.
template <typename T>
__global__ void __launch_bounds__(kPlaneBlock)
    k_plane_gauss(int nx, int ny, int axis, const T* in, T* out, const T* pre, int normalise, GaussW<T> gw,
                  int want_sum, double* P, int maxp) {
  const int64_t E = (int64_t)nx * ny;
  double v[1] = {0.0};
  for (int64_t ee = (int64_t)blockIdx.x * kPlaneBlock + threadIdx.x; ee < E; ee += (int64_t)gridDim.x * kPlaneBlock) {
    const int e = (int)ee;
    const int ey = e / nx, ex = e - ey * nx;
    const int pos = axis == 0 ? ex : ey, len = axis == 0 ? nx : ny, stride = axis == 0 ? 1 : nx;
    T acc = (T)0, h = (T)0;
    for (int d = -gw.half; d <= gw.half; ++d) {
      const int q = pos + d;
      if (q < 0 || q >= len) continue;
      const int k = e + d * stride;
      const T w = gw.w[d + gw.half];
      const T x = pre ? in[k] * pre[k] : in[k];
      acc += w * x;
      h += w;
    }
    const T o = normalise ? acc / h : acc;
    out[e] = o;
    v[0] += (double)o;
  }
  if (want_sum) {
    double* dst[1] = {pslot2(P, P_GSUM, 0, maxp)};
    write_parts<1, 0u>(v, dst, blockIdx.x);
  }
}

// 1 / Hs_e = 1 / (h_x(ex) h_y(ey)): the 2D row sum of a separable window
// truncated at the grid's edges factors over the axes.
template <typename T>
__global__ void __launch_bounds__(kPlaneBlock) k_plane_hs(int nx, int ny, T* Hsi, GaussW<T> gw) {
  const int64_t E = (int64_t)nx * ny;
  for (int64_t ee = (int64_t)blockIdx.x * kPlaneBlock + threadIdx.x; ee < E; ee += (int64_t)gridDim.x * kPlaneBlock) {
    const int e = (int)ee;
    const int ey = e / nx, ex = e - ey * nx;
    double hx = 0.0, hy = 0.0;
    for (int d = -gw.half; d <= gw.half; ++d) {
      if (ex + d >= 0 && ex + d < nx) hx += (double)gw.w[d + gw.half];
      if (ey + d >= 0 && ey + d < ny) hy += (double)gw.w[d + gw.half];
    }
    Hsi[e] = (T)(1.0 / (hx * hy));
  }
}

int plane_blocks(int64_t n) {
  int64_t b = (n + kPlaneBlock - 1) / kPlaneBlock;
  if (b > kMaxVecBlocks) b = kMaxVecBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T> const Q4<T>& q4_of(fbto_grid_s* g);
template <> const Q4<double>& q4_of<double>(fbto_grid_s* g) { return g->q4_64; }
template <> const Q4<float>& q4_of<float>(fbto_grid_s* g) { return g->q4_32; }
template <typename T> GaussW<T> gauss_of(fbto_grid_s* g);
template <> GaussW<double> gauss_of<double>(fbto_grid_s* g) { return g->gauss64; }
template <> GaussW<float> gauss_of<float>(fbto_grid_s* g) { return g->gauss32; }

template <typename T>
PlaneArgs<T> plane_args(fbto_grid_s* g) {
  PlaneArgs<T> A{};
  A.nx = g->geo.nx;
  A.ny = g->geo.ny;
  A.N = g->geo.N;
  A.ndof = g->geo.ndof;
  A.mask = g->mask;
  A.ke = q4_of<T>(g);
  A.ke_diag = g->ke_diag;
  A.sp = g->simp;
  A.P = g->partials;
  A.maxp = g->max_partials;
  A.sc = g->sc;
  return A;
}

template <typename T, int MODE>
hipError_t plane_launch(fbto_grid_s* g, const PlaneArgs<T>& A, int nrhs, hipStream_t st, int* nb_out) {
  const int nb = plane_blocks(g->geo.N);
  if (nb > g->max_partials) return hipErrorInvalidValue;
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    if (left >= 2 && MODE != PL_APPLY) {
      hipLaunchKernelGGL((k_plane_apply<T, 2, MODE>), dim3(nb), dim3(kPlaneBlock), 0, st, A, r0);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_plane_apply<T, 1, MODE>), dim3(nb), dim3(kPlaneBlock), 0, st, A, r0);
      r0 += 1;
    }
  }
  if (nb_out) *nb_out = nb;
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t plane_apply(fbto_grid_s* g, const T* rho, const T* u, T* y, int nrhs, hipStream_t st) {
  PlaneArgs<T> A = plane_args<T>(g);
  A.rho = rho;
  A.u = u;
  A.y = y;
  return plane_launch<T, PL_APPLY>(g, A, nrhs, st, nullptr);
}

template <typename T>
hipError_t plane_resid(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, const T* invD, T* invD_out,
                       T* z, int nrhs, hipStream_t st, int* nb_out) {
  PlaneArgs<T> A = plane_args<T>(g);
  A.rho = rho;
  A.u = u;
  A.y = r;
  A.f = f;
  A.invD = invD;
  A.invD_out = invD_out;
  A.z = z;
  return plane_launch<T, PL_RESID>(g, A, nrhs, st, nb_out);
}

template <typename T>
hipError_t plane_apply_cg(fbto_grid_s* g, const T* rho, const T* z, const T* r, T* w, int nrhs, int step,
                          hipStream_t st, int* nb_out) {
  PlaneArgs<T> A = plane_args<T>(g);
  A.rho = rho;
  A.u = z;
  A.r = r;
  A.y = w;
  A.step = step;
  return plane_launch<T, PL_CG>(g, A, nrhs, st, nb_out);
}

template <typename T>
hipError_t plane_diag(fbto_grid_s* g, const T* rho, T* invD, hipStream_t st) {
  hipLaunchKernelGGL((k_plane_diag<T>), dim3(plane_blocks(g->geo.N)), dim3(kPlaneBlock), 0, st, g->geo.nx,
                     g->geo.ny, g->geo.N, rho, invD, g->mask, g->simp, g->ke_diag);
  return hipGetLastError();
}

template <typename T>
hipError_t plane_sens(fbto_grid_s* g, const T* rho, const T* u, const T* lam, int nrhs, T* dobj, const T* Hsi,
                      hipStream_t st) {
  hipLaunchKernelGGL((k_plane_sens<T>), dim3(plane_blocks(g->geo.E)), dim3(kPlaneBlock), 0, st, g->geo.nx,
                     g->geo.ny, g->geo.ndof, rho, u, lam, nrhs, dobj, g->mask, q4_of<T>(g), g->simp, Hsi);
  return hipGetLastError();
}

// kind 0: out = (H in) / Hs (x pass, then y pass, each normalised);
// kind 1: out = H^T (in / Hs);  kind 2: out = H^T in (input already / Hs).
// `tmp` holds the intermediate pass (E values, distinct from in and out).
template <typename T>
hipError_t plane_filter(fbto_grid_s* g, int kind, const T* in, T* out, T* tmp, const T* Hsi, int want_sum,
                        hipStream_t st) {
  const int nb = plane_blocks(g->geo.E);
  const int nx = g->geo.nx, ny = g->geo.ny;
  const GaussW<T> gw = gauss_of<T>(g);
  if (want_sum) g->n_gsum = nb;
  if (kind == 0) {
    hipLaunchKernelGGL((k_plane_gauss<T>), dim3(nb), dim3(kPlaneBlock), 0, st, nx, ny, 0, in, tmp, (const T*)nullptr,
                       1, gw, 0, g->partials, g->max_partials);
    hipLaunchKernelGGL((k_plane_gauss<T>), dim3(nb), dim3(kPlaneBlock), 0, st, nx, ny, 1, (const T*)tmp, out,
                       (const T*)nullptr, 1, gw, want_sum, g->partials, g->max_partials);
  } else {
    hipLaunchKernelGGL((k_plane_gauss<T>), dim3(nb), dim3(kPlaneBlock), 0, st, nx, ny, 1, in, tmp,
                       kind == 1 ? Hsi : (const T*)nullptr, 0, gw, 0, g->partials, g->max_partials);
    hipLaunchKernelGGL((k_plane_gauss<T>), dim3(nb), dim3(kPlaneBlock), 0, st, nx, ny, 0, (const T*)tmp, out,
                       (const T*)nullptr, 0, gw, want_sum, g->partials, g->max_partials);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t plane_hs(fbto_grid_s* g, T* Hsi, hipStream_t st) {
  hipLaunchKernelGGL((k_plane_hs<T>), dim3(plane_blocks(g->geo.E)), dim3(kPlaneBlock), 0, st, g->geo.nx, g->geo.ny,
                     Hsi, gauss_of<T>(g));
  return hipGetLastError();
}

#define FBTO_PLANE_INST(T)                                                                                   \
  template hipError_t plane_apply<T>(fbto_grid_s*, const T*, const T*, T*, int, hipStream_t);                \
  template hipError_t plane_resid<T>(fbto_grid_s*, const T*, const T*, const T*, T*, const T*, T*, T*, int,  \
                                     hipStream_t, int*);                                                     \
  template hipError_t plane_apply_cg<T>(fbto_grid_s*, const T*, const T*, const T*, T*, int, int, hipStream_t, \
                                        int*);                                                               \
  template hipError_t plane_diag<T>(fbto_grid_s*, const T*, T*, hipStream_t);                                \
  template hipError_t plane_sens<T>(fbto_grid_s*, const T*, const T*, const T*, int, T*, const T*,           \
                                    hipStream_t);                                                            \
  template hipError_t plane_filter<T>(fbto_grid_s*, int, const T*, T*, T*, const T*, int, hipStream_t);      \
  template hipError_t plane_hs<T>(fbto_grid_s*, T*, hipStream_t);

FBTO_PLANE_INST(double)
FBTO_PLANE_INST(float)

}  // namespace fbto
