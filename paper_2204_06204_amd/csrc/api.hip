// C ABI of the MI355X matrix-free SIMP hot path: argument checks, workspace,
// and the order of kernel launches of each call (no arithmetic here beyond
// the element-matrix constants and the filter stencil, both set up once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fbto.h"
#include "internal.h"

using namespace fbto;


namespace {

thread_local std::string g_last_error;

fbto_status_t fail(fbto_status_t s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

fbto_status_t ok() {
  g_last_error.clear();
  return FBTO_OK;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(_e == hipErrorOutOfMemory ? FBTO_ERR_ALLOC : FBTO_ERR_HIP, "%s: %s", #expr, \
                  hipGetErrorString(_e));                                                   \
  } while (0)

template <typename T>
Vecs& vecs(fbto_grid_s* g);
template <>
Vecs& vecs<double>(fbto_grid_s* g) { return g->v64; }
template <>
Vecs& vecs<float>(fbto_grid_s* g) { return g->v32; }

// Element stiffness of the unit-cube hex8 in the sum/difference basis.
// Per axis the basis of the pair (u0 + u1, u1 - u0) is {1/2, t - 1/2}, whose
// 1D integrals are M(m,m) = 1/4, M(d,d) = 1/12, G(d,d) = 1 and
// int psi_d' psi_m = 1/2.  The isotropic bilinear form
//   int lambda div u div v + mu (grad u : grad v + grad u : grad v^T)
// then has, for component i and mode q (bit b set = difference mode along b),
//   diagonal  (lambda + mu) [q_i] W_i(q) + mu sum_l [q_l] W_l(q),
//             W_l(q) = prod_{k != l} M(q_k),
//   coupling  to component j, mode q ^ (1<<i) ^ (1<<j) when q_i != q_j:
//             lambda/4 M(q_k) if q_i = d, else mu/4 M(q_k).
// The diagonal depends on q only through q_i and how many of the other two
// bits are set (W_l is a product over the other axes), so it is stored as
// dg[q_i][count] and computed for component 0 at a representative mode.
void modal_coefficients(double young, double poisson, Modal<double>& km, double& ke_diag) {
  const double lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson));
  const double mu = young / (2.0 * (1.0 + poisson));
  const double M[2] = {0.25, 1.0 / 12.0};
  for (int qi = 0; qi < 2; ++qi) {
    for (int cnt = 0; cnt < 3; ++cnt) {
      const int q = qi | (cnt >= 1 ? 2 : 0) | (cnt >= 2 ? 4 : 0);
      double W[3];
      for (int l = 0; l < 3; ++l) {
        W[l] = 1.0;
        for (int k = 0; k < 3; ++k)
          if (k != l) W[l] *= M[(q >> k) & 1];
      }
      double d = qi ? (lam + mu) * W[0] : 0.0;
      for (int l = 0; l < 3; ++l)
        if ((q >> l) & 1) d += mu * W[l];
      km.dg[qi][cnt] = d;
    }
  }
  // dg[0][0] is mode 0 (rigid translation): no energy, computed as 0
  for (int b = 0; b < 2; ++b) {
    km.lam4[b] = 0.25 * lam * M[b];
    km.mu4[b] = 0.25 * mu * M[b];
  }
  ke_diag = (lam + 4.0 * mu) / 9.0;
}

// Element stiffness of the unit-square Q4 in plane stress, by 2 x 2 Gauss
// quadrature of B^T D B (exact for the bilinear element):
//   D = E / (1 - nu^2) [[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]],
// strains (u_x,x, u_y,y, u_x,y + u_y,x); local DOF 2a + c, a = ax + 2 ay.
void q4_plane_stress(double young, double poisson, Q4<double>& ke, double& ke_diag) {
  const double f = young / (1.0 - poisson * poisson);
  const double D[3][3] = {{f, f * poisson, 0.0}, {f * poisson, f, 0.0}, {0.0, 0.0, f * 0.5 * (1.0 - poisson)}};
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int p = 0; p < 8; ++p)
    for (int q = 0; q < 8; ++q) ke.k[p][q] = 0.0;
  for (int ix = 0; ix < 2; ++ix)
    for (int iy = 0; iy < 2; ++iy) {
      const double x = gp[ix], y = gp[iy];
      double B[3][8] = {};
      for (int a = 0; a < 4; ++a) {
        const int ax = a & 1, ay = a >> 1;
        const double nx = ax ? x : 1.0 - x, ny = ay ? y : 1.0 - y;
        const double dnx = (ax ? 1.0 : -1.0) * ny, dny = nx * (ay ? 1.0 : -1.0);
        B[0][2 * a] = dnx;
        B[1][2 * a + 1] = dny;
        B[2][2 * a] = dny;
        B[2][2 * a + 1] = dnx;
      }
      for (int p = 0; p < 8; ++p)
        for (int q = 0; q < 8; ++q) {
          double acc = 0.0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc += B[i][p] * D[i][j] * B[j][q];
          ke.k[p][q] += 0.25 * acc;
        }
    }
  ke_diag = ke.k[0][0];  // the eight diagonal entries are equal on the square
}

// The projection's partial arrays are the grid's slots P_S0 .. P_DX.
ProjWs proj_ws(fbto_grid_s* g) {
  return ProjWs{g->partials + (size_t)P_S0 * 4 * g->max_partials, (int64_t)4 * g->max_partials, g->max_partials,
                g->sc};
}

fbto_status_t check_grid(fbto_grid_t g) {
  if (!g) return fail(FBTO_ERR_ARG, "grid handle is NULL");
  return FBTO_OK;
}
fbto_status_t check_prec(fbto_prec_t p) {
  if (p != FBTO_F64 && p != FBTO_F32) return fail(FBTO_ERR_ARG, "unknown precision %d", (int)p);
  return FBTO_OK;
}
fbto_status_t check_nrhs(fbto_grid_t g, int nrhs) {
  if (nrhs < 1 || nrhs > g->desc.max_rhs)
    return fail(FBTO_ERR_ARG, "nrhs = %d outside [1, %d]", nrhs, g->desc.max_rhs);
  return FBTO_OK;
}

template <typename T>
fbto_status_t ensure_vecs(fbto_grid_s* g) {
  Vecs& V = vecs<T>(g);
  if (V.ready) return FBTO_OK;
  const int64_t nd = g->geo.ndof * g->desc.max_rhs, E = g->geo.E;
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(hipMalloc(&V.r[b], nd * sizeof(T)));
    HIP_TRY(hipMalloc(&V.p[b], nd * sizeof(T)));
    HIP_TRY(hipMalloc(&V.s[b], nd * sizeof(T)));
    HIP_TRY(hipMalloc(&V.w[b], nd * sizeof(T)));
  }
  HIP_TRY(hipMalloc(&V.x1, nd * sizeof(T)));
  HIP_TRY(hipMalloc(&V.q, nd * sizeof(T)));
  HIP_TRY(hipMalloc(&V.invD, g->geo.ndof * sizeof(T)));
  HIP_TRY(hipMalloc(&V.rho, E * sizeof(T)));
  HIP_TRY(hipMalloc(&V.ge, E * sizeof(T)));
  HIP_TRY(hipMalloc(&V.gx, E * sizeof(T)));
  HIP_TRY(hipMalloc(&V.y, E * sizeof(T)));
  HIP_TRY(hipMalloc(&V.Hs, E * sizeof(T)));
  HIP_TRY(launch_hs<T>(g, (T*)V.Hs, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  V.ready = true;
  return FBTO_OK;
}

fbto_status_t ensure_sort(fbto_grid_s* g) {
  SortWs& W = g->sort;
  if (W.base) return FBTO_OK;
  HIP_TRY(hipMalloc(&W.base, sort_ws_layout(g->geo.E, nullptr)));
  (void)sort_ws_layout(g->geo.E, &W);
  return FBTO_OK;
}

void free_vecs(Vecs& V) {
  void* ps[] = {V.r[0], V.r[1], V.p[0], V.p[1], V.s[0], V.s[1], V.w[0], V.w[1], V.x1, V.q,
                V.invD, V.rho, V.ge, V.gx, V.y, V.Hs};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  V = Vecs{};
}

// Per-grid buffers of the mixed-precision refinement (allocated on demand).
struct IrBufs {
  void* f = nullptr;   // inner right-hand side
  void* d = nullptr;   // inner correction
  double* r64 = nullptr;
};
struct GridExtra {
  IrBufs ir32, ir64;
  void* ustar32 = nullptr;     // optimality metrics: K^-1 f, [max_rhs][ndof]
  void* ustar64 = nullptr;
  Scalars* sc_metrics = nullptr;  // search state of the metrics' projection
};
std::vector<std::pair<fbto_grid_s*, GridExtra*>>& extras() {
  static std::vector<std::pair<fbto_grid_s*, GridExtra*>> v;
  return v;
}
GridExtra* extra_of(fbto_grid_s* g) {
  for (auto& p : extras())
    if (p.first == g) return p.second;
  auto* e = new GridExtra();
  extras().push_back({g, e});
  return e;
}
void drop_extra(fbto_grid_s* g) {
  auto& v = extras();
  for (size_t i = 0; i < v.size(); ++i) {
    if (v[i].first == g) {
      GridExtra* e = v[i].second;
      for (IrBufs* b : {&e->ir32, &e->ir64}) {
        if (b->f) (void)hipFree(b->f);
        if (b->d) (void)hipFree(b->d);
        if (b->r64) (void)hipFree(b->r64);
      }
      for (void* q : {e->ustar32, e->ustar64, (void*)e->sc_metrics})
        if (q) (void)hipFree(q);
      delete e;
      v.erase(v.begin() + i);
      return;
    }
  }
}

// Jacobi-PCG on K(rho) x = f from the warm start x, `steps` steps in the
// Chronopoulos-Gear arrangement (one apply and one vector kernel per step,
// one reduction phase).  rtol > 0 stops early (checked on the host every 32
// steps).  f_dot: also leave the f.x partials (slot DOT) after the last
// step.  Returns the partial counts the finish kernel needs.
struct CgCounts {
  int r, fn;
  int dot;  // partials of f . x (final vector step, or the dot kernel)
};

template <typename T>
fbto_status_t pcg_run(fbto_grid_s* g, const T* rho, const T* f, T* x, int nrhs, int steps,
                      double rtol, hipStream_t st, bool f_dot, CgCounts* cn_out, T* sens = nullptr,
                      const T* sens_hsi = nullptr, bool* sens_done = nullptr) {
  Vecs& V = vecs<T>(g);
  T* invD = (T*)V.invD;
  T* z = (T*)V.q;
  CgSet<T> set[2] = {{x, (T*)V.r[0], (T*)V.p[0], (T*)V.s[0], (T*)V.w[0]},
                     {(T*)V.x1, (T*)V.r[1], (T*)V.p[1], (T*)V.s[1], (T*)V.w[1]}};
  int nb_a = 0, nb_v = 0;
  HIP_TRY(launch_resid_diag<T>(g, rho, x, f, set[0].r, invD, z, nrhs, st, &nb_a));
  CgCounts cn{nb_a, nb_a, vec_blocks(g->geo.ndof)};
  if (steps == 0) {
    if (f_dot) HIP_TRY(launch_dot<T>(g, f, x, nrhs, st));
    *cn_out = cn;
    return FBTO_OK;
  }
  auto all_done = [&](bool& done) -> fbto_status_t {
    Scalars host;
    HIP_TRY(hipMemcpyAsync(&host, g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    done = true;
    for (int R = 0; R < nrhs; ++R) done = done && host.done[R] != 0.0;
    return FBTO_OK;
  };
  // step 0's product w = K z from the residual's z
  HIP_TRY(launch_apply_cg<T>(g, rho, z, set[0].r, set[0].w, nrhs, 0, st, &nb_a));
  int k = 0;
  // voxel grids: fused steps (both precisions); plane grids: unfused
  const bool fused = g->dim == 3;
  if (fused) {
    // fused steps: the update of step k and the product of step k + 1 in one pass
    for (; k + 1 < steps; ++k) {
      HIP_TRY(launch_cg_fused<T>(g, rho, set[k & 1], set[(k + 1) & 1], invD, nrhs, k, nb_a, cn.fn, rtol, st,
                                 &nb_a));
      if (rtol > 0.0 && (k + 2) % 64 == 0 && k + 2 < steps) {
        bool done = false;
        if (fbto_status_t e = all_done(done)) return e;
        if (done) {
          ++k;
          break;
        }
      }
    }
  } else {
    // unfused steps (plane grids): vector update, then the next product
    for (; k + 1 < steps; ++k) {
      HIP_TRY(launch_cg_step<T>(g, x, x, set[0].r, z, z, set[0].w, set[0].p, set[0].s, invD, nullptr, nrhs, nb_a,
                                cn.fn, k, rtol, st, &nb_v));
      HIP_TRY(launch_apply_cg<T>(g, rho, z, set[0].r, set[0].w, nrhs, k + 1, st, &nb_a));
      if (rtol > 0.0 && (k + 2) % 64 == 0 && k + 2 < steps) {
        bool done = false;
        if (fbto_status_t e = all_done(done)) return e;
        if (done) {
          ++k;
          break;
        }
      }
    }
  }
  // last vector update of step k, into the caller's x; with one RHS and a
  // sensitivity wanted, fused with it
  const CgSet<T>& cur = set[fused ? (k & 1) : 0];
  // The fused kernel reads x at halo nodes while their owners store x', so it
  // may only run when its input and output are different buffers: after an
  // odd number of fused steps, when the input is the second set.
  if (sens && nrhs == 1 && cur.x != x) {
    HIP_TRY(launch_cg_sens<T>(g, rho, cur, x, invD, f_dot ? f : nullptr, sens, sens_hsi, k, nb_a, cn.fn, rtol, st,
                              &nb_v));
    if (sens_done) *sens_done = true;
  } else {
    HIP_TRY(launch_cg_step<T>(g, cur.x, x, cur.r, nullptr, nullptr, cur.w, cur.p, cur.s, invD,
                              f_dot ? f : nullptr, nrhs, nb_a, cn.fn, k, rtol, st, &nb_v));
  }
  cn.r = nb_v;
  cn.dot = nb_v;
  *cn_out = cn;
  return FBTO_OK;
}

template <typename T>
fbto_status_t pcg_solve(fbto_grid_s* g, const T* rho, const T* f, T* u, int nrhs, int steps, double rtol,
                        hipStream_t st) {
  CgCounts cn{};
  fbto_status_t s = pcg_run<T>(g, rho, f, u, nrhs, steps, rtol, st, false, &cn);
  if (s) return s;
  HIP_TRY(launch_pcg_finish(g, nrhs, cn.r, cn.fn, nullptr, 0, 0, 0, st));
  return FBTO_OK;
}

// r = f - K u with its norms (into the scalars)
template <typename T>
fbto_status_t residual_norms(fbto_grid_s* g, const T* rho, const T* u, const T* f, T* r, const T* invD, int nrhs,
                             hipStream_t st) {
  int nb = 0;
  HIP_TRY(launch_resid<T>(g, rho, u, f, r, invD, (T*)vecs<T>(g).q, nrhs, st, &nb));
  HIP_TRY(launch_pcg_finish(g, nrhs, nb, nb, nullptr, 0, 0, 0, st));
  return FBTO_OK;
}

template <typename T>
fbto_status_t relax_run(fbto_grid_s* g, const T* rho, const T* f, T* u, int nrhs, int steps,
                        double omega, int use_diag, hipStream_t st) {
  Vecs& V = vecs<T>(g);
  T* r = (T*)V.r[0];
  T* invD = (T*)V.invD;
  HIP_TRY(launch_diag<T>(g, rho, invD, st));
  for (int s = 0; s < steps; ++s) {
    HIP_TRY(launch_resid<T>(g, rho, u, f, r, (const T*)nullptr, (T*)nullptr, nrhs, st, nullptr));
    HIP_TRY(launch_relax_update<T>(g, u, r, invD, nrhs, omega, use_diag, st));
  }
  return residual_norms<T>(g, rho, u, f, r, invD, nrhs, st);
}

// One low-level step of Alg. 3 with the Krylov preconditioner of degree D
// (Eq. LSP), per RHS: u <- u + damp * (u_D - u), where u_D minimises the
// residual over u + span{r, ..., K^D r} (MINRES, D + 1 iterations; see
// k_minres).  Workspace: w[0] (products), r[0..1] (Lanczos vectors), p[0..1]
// (MINRES directions).
template <typename T>
fbto_status_t krylov_run(fbto_grid_s* g, const T* rho, const T* f, T* u, int nrhs, int D, double damp,
                         hipStream_t st, CgCounts* cn_out = nullptr) {
  Vecs& V = vecs<T>(g);
  const int64_t nd = g->geo.ndof;
  T* Y = (T*)V.w[0];
  const int last = D + 2;
  for (int R = 0; R < nrhs; ++R) {
    T* x = u + R * nd;
    const T* fr = f + R * nd;
    T* R1 = (T*)V.r[1];
    T* R2 = (T*)V.r[0];
    T* Wc = (T*)V.p[0];
    T* W2 = (T*)V.p[1];
    HIP_TRY(launch_resid<T>(g, rho, x, fr, R2, (const T*)nullptr, (T*)nullptr, 1, st, nullptr));  // R2 = f - K u
    int nb_v = 0, nb_a = 0;
    HIP_TRY(launch_minres<T>(g, 0, last, Y, R1, R2, W2, Wc, x, 0, 0, damp, st, &nb_v));
    int itn0 = 1;
    if (g->dim == 3) {
      // voxel grids: iterations 1 .. D fused (vector pass t with the product of
      // t + 1); products alternate between two buffers, the Lanczos
      // vectors rotate through three (halo nodes read them while their
      // owners write the next one)
      T* Yb[2] = {(T*)V.w[0], (T*)V.w[1]};
      T* R3 = (T*)V.s[0];
      HIP_TRY(launch_apply_cg<T>(g, rho, R2, R2, Yb[1], 1, 1, st, &nb_a));
      for (int itn = 1; itn <= D; ++itn) {
        int nb = 0;
        HIP_TRY(launch_minres_fused<T>(g, rho, itn, Yb[itn & 1], R1, R2, R3, Wc, W2, x, Yb[(itn + 1) & 1], nb_a,
                                       nb_v, damp, st, &nb));
        nb_a = nb_v = nb;
        T* t = R1;
        R1 = R2;
        R2 = R3;
        R3 = t;
        if (itn >= 2) std::swap(Wc, W2);
      }
      // iteration D + 1: the unfused vector pass on the last product
      int nb = 0;
      HIP_TRY(launch_minres<T>(g, D + 1, last, Yb[(D + 1) & 1], R1, R2, W2, Wc, x, nb_a, nb_v, damp, st, &nb));
      nb_v = nb;
      std::swap(R1, R2);
      if (D + 1 >= 2) std::swap(Wc, W2);
      itn0 = D + 2;
    }
    for (int itn = itn0; itn <= D + 1; ++itn) {
      // Y = K R2 with <A.r, R2> and <Y, R2>; A.r = R1 (R2 on the first iteration, where R1 is unused)
      HIP_TRY(launch_apply_cg<T>(g, rho, R2, itn == 1 ? R2 : R1, Y, 1, itn, st, &nb_a));
      int nb = 0;
      HIP_TRY(launch_minres<T>(g, itn, last, Y, R1, R2, W2, Wc, x, nb_a, nb_v, damp, st, &nb));
      nb_v = nb;
      std::swap(R1, R2);                 // R1 <- R2, R2 <- the new Lanczos vector
      if (itn >= 2) std::swap(Wc, W2);   // W <- the new direction, W2 <- W
    }
    HIP_TRY(launch_minres<T>(g, last, last, Y, R1, R2, W2, Wc, x, 0, nb_v, damp, st, nullptr));
  }
  // the final residual and its norms; the residual kernel forms the Jacobi
  // diagonal on the way (its partials are written when it forms or reads one)
  int nb = 0;
  HIP_TRY(launch_resid_diag<T>(g, rho, u, f, (T*)V.r[0], (T*)V.invD, (T*)V.q, nrhs, st, &nb));
  if (!cn_out) {
    HIP_TRY(launch_pcg_finish(g, nrhs, nb, nb, nullptr, 0, 0, 0, st));
    return FBTO_OK;
  }
  // inside an outer step: leave the residual norms and f . u as partials
  // for the step's final reduction
  HIP_TRY(launch_dot<T>(g, f, u, nrhs, st));
  *cn_out = CgCounts{nb, nb, vec_blocks(g->geo.ndof)};
  return FBTO_OK;
}

// One outer iteration: Alg. 1 with `inner_steps` Jacobi-PCG steps, or
// (krylov_degree >= 0) Alg. 3 with one Krylov-preconditioned step of that
// degree and step beta.
//
// rho_ready (several iterations in one call): on entry, whether the filtered
// density of x is already in V.rho (left by the previous iteration); on
// return, whether this iteration left the next one's there.  fuse_next: the
// final projection pass also filters the new design (another iteration
// follows in the same call, so x does not change in between).
template <typename T>
fbto_status_t outer_run(fbto_grid_s* g, T* x, T* u, const T* f, int nrhs, int k, double alpha0,
                        int inner_steps, int mean_project, double lo, double vmax, double* info,
                        hipStream_t st, int krylov_degree = -1, double beta = 1.0, double inner_rtol = 0.0,
                        bool* rho_ready = nullptr, bool fuse_next = false) {
  Vecs& V = vecs<T>(g);
  T* rho = (T*)V.rho;
  if (!(rho_ready && *rho_ready)) HIP_TRY(launch_filter<T>(g, 0, x, rho, 0, st));
  if (rho_ready) *rho_ready = false;
  CgCounts cn{};
  bool sens_done = false;
  fbto_status_t s = krylov_degree >= 0
                        ? krylov_run<T>(g, rho, f, u, nrhs, krylov_degree, beta, st, &cn)
                        : pcg_run<T>(g, rho, f, u, nrhs, inner_steps, inner_rtol, st, true, &cn, (T*)V.ge,
                                     (const T*)V.Hs, &sens_done);
  if (s != FBTO_OK) return s;
  // element gradient already divided by Hs, so the filter transpose is a plain sum
  if (!sens_done) HIP_TRY(launch_sens<T>(g, rho, u, nullptr, nrhs, (T*)V.ge, (const T*)V.Hs, st));
  const double alpha_k = alpha0 * std::pow((double)k, -0.75);
  int nb_seed = 0;
  hipError_t fe = hipErrorNotSupported;
  if (sens_done) {
    // the last CG step left the gradient's sum (slot GSUM, cn.dot partials):
    // the filter and the step run as one pass
    g->n_gsum = cn.dot;
    fe = launch_filter_step<T>(g, (const T*)V.ge, x, (T*)V.y, 0.5 * alpha_k, mean_project, cn.dot, lo, 1.0, st,
                               &nb_seed);
    if (fe != hipSuccess && fe != hipErrorNotSupported) HIP_TRY(fe);
  }
  if (fe == hipErrorNotSupported) {
    HIP_TRY(launch_filter<T>(g, 2, (const T*)V.ge, (T*)V.gx, 1, st));
    HIP_TRY(launch_step<T>(g, x, (const T*)V.gx, (T*)V.y, 0.5 * alpha_k, mean_project, lo, 1.0, st));
    nb_seed = 0;
  }
  int nbE = vec_blocks(g->geo.E);  // the final pass's volume partials
  if (fuse_next && zmarch_filter(g)) {
    // the search passes, then the final pass fused with the next iteration's
    // forward filter
    HIP_TRY(launch_project<T>(proj_ws(g), g->geo.E, (const T*)V.y, x, lo, 1.0, vmax, 1, g->proj_passes_warm, x,
                              nullptr, nullptr, st, nb_seed, 1));
    HIP_TRY(launch_proj_final_filter<T>(g, proj_ws(g), (const T*)V.y, x, rho, lo, 1.0, vmax, g->proj_passes_warm,
                                        st, &nbE));
    if (rho_ready) *rho_ready = true;
  } else {
    HIP_TRY(launch_project<T>(proj_ws(g), g->geo.E, (const T*)V.y, x, lo, 1.0, vmax, 1, g->proj_passes_warm, x,
                              nullptr, nullptr, st, nb_seed));
  }
  HIP_TRY(launch_pcg_finish(g, nrhs, cn.r, cn.fn, info, cn.dot, nbE, g->n_gsum, st));
  return FBTO_OK;
}

// Optimality metrics of a design x with the caller's displacement u (the
// error metrics of Thm. 1): u* = K(rho(x))^-1 f by Jacobi-PCG to rtol,
// warm-started from u, in a workspace; then
//   l = 1/2 sum_r f_r . u*_r,  grad l = 1/2 C^T(-ds_e u*_e^T KE u*_e),
//   z = Proj_X(x - alpha grad l),  Delta^v = |z - x|^2 / alpha^2,
//   Delta = sum_r |u_r - u*_r|^2.
// The projection runs cold with its own search state, so the warm start of
// the outer steps is left as it was.
template <typename T>
fbto_status_t optimality_run(fbto_grid_s* g, const T* x, const T* u, const T* f, int nrhs, double alpha, double lo,
                             double vmax, double rtol, int max_steps, double* out, hipStream_t st) {
  Vecs& V = vecs<T>(g);
  GridExtra* ex = extra_of(g);
  void*& us_buf = sizeof(T) == 8 ? ex->ustar64 : ex->ustar32;
  const int64_t nd = g->geo.ndof, E = g->geo.E;
  if (!us_buf) HIP_TRY(hipMalloc(&us_buf, (size_t)g->desc.max_rhs * nd * sizeof(T)));
  if (!ex->sc_metrics) {
    HIP_TRY(hipMalloc(&ex->sc_metrics, sizeof(Scalars)));
    HIP_TRY(hipMemsetAsync(ex->sc_metrics, 0, sizeof(Scalars), st));
  }
  T* us = (T*)us_buf;
  T* rho = (T*)V.rho;
  HIP_TRY(launch_filter<T>(g, 0, x, rho, 0, st));
  HIP_TRY(hipMemcpyAsync(us, u, (size_t)nrhs * nd * sizeof(T), hipMemcpyDeviceToDevice, st));
  if (fbto_status_t s = pcg_solve<T>(g, rho, f, us, nrhs, max_steps, rtol, st)) return s;
  int nb_lo = 0, nb_hi = 0;
  HIP_TRY(launch_sqdist<T>(g, u, us, (int64_t)nrhs * nd, P_MET0, st, &nb_lo));
  HIP_TRY(launch_dot<T>(g, f, us, nrhs, st));
  HIP_TRY(launch_sens<T>(g, rho, us, nullptr, nrhs, (T*)V.ge, (const T*)V.Hs, st));
  HIP_TRY(launch_filter<T>(g, 2, (const T*)V.ge, (T*)V.gx, 0, st));
  // y = x - alpha grad l = x - (alpha / 2) C^T(dc/drho)
  HIP_TRY(launch_step<T>(g, x, (const T*)V.gx, (T*)V.y, 0.5 * alpha, 0, lo, 1.0, st));
  ProjWs W = proj_ws(g);
  W.sc = ex->sc_metrics;
  HIP_TRY(launch_project<T>(W, E, (const T*)V.y, (T*)V.ge, lo, 1.0, vmax, 0, kProjMaxPasses, nullptr, nullptr,
                            nullptr, st));
  HIP_TRY(launch_sqdist<T>(g, (const T*)V.ge, x, E, P_MET1, st, &nb_hi));
  HIP_TRY(launch_opt_finish(g, nrhs, vec_blocks(nd), nb_lo, nb_hi, alpha, ex->sc_metrics, out, st));
  return FBTO_OK;
}

// ---- allocation-free projection --------------------------------------------
// fbto_project_volume_noalloc keeps the projection's per-block partials
// (kProjSlots arrays of kMaxVecBlocks FP64 values) and its search state (one
// Scalars record) in this array.  Each device holds its own copy until the
// process ends; its address there is looked up once per device, and host
// code uses only that address (the array's name is a host-side stand-in).
constexpr size_t kNoAllocPartDoubles = (size_t)kProjSlots * kMaxVecBlocks;
constexpr size_t kNoAllocDoubles = kNoAllocPartDoubles + (sizeof(Scalars) + sizeof(double) - 1) / sizeof(double);
constexpr int kNoAllocMaxDevices = 64;
static_assert(sizeof(Scalars) % sizeof(double) == 0, "the search state is a record of doubles");

static __device__ __align__(256) double scratch[kNoAllocDoubles];

std::mutex g_scratch_mu;
double* g_scratch_dev[kNoAllocMaxDevices] = {};

// The scratch address on the current device (looked up on its first use).
fbto_status_t scratch_on_current_device(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(FBTO_ERR_UNSUPPORTED, "device %d: the scratch table holds devices 0 .. %d", dev,
                kNoAllocMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    double* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(FBTO_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return FBTO_OK;
}

}  // namespace

extern "C" {

const char* fbto_last_error(void) { return g_last_error.c_str(); }

const char* fbto_version(void) { return "fbto-mi355x 0.1 (gfx950)"; }

fbto_status_t fbto_setup_grid(const fbto_grid_desc_t* d, const uint8_t* fixed_dof_mask,
                              int32_t n_springs, const int64_t* spring_dof, const double* spring_k,
                              fbto_grid_t* out) {
  if (!d || !out) return fail(FBTO_ERR_ARG, "desc and out must be non-NULL");
  *out = nullptr;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1)
    return fail(FBTO_ERR_ARG, "grid %d x %d x %d: every axis needs >= 1 element", d->nx, d->ny, d->nz);
  if (d->nx > 65534 || d->ny > 65534 || d->nz > 65534)
    return fail(FBTO_ERR_ARG, "grid axis longer than 65534 elements");
  const int64_t N = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
  if (N >= ((int64_t)1 << 29))
    return fail(FBTO_ERR_ARG, "grid has %lld nodes (limit 2^29, so that DOF indices fit 32 bits)",
                (long long)N);
  if (d->max_rhs < 1 || d->max_rhs > 4) return fail(FBTO_ERR_ARG, "max_rhs = %d outside [1, 4]", d->max_rhs);
  {
    // the K u kernels address four node planes of FP64 values with 32-bit byte offsets
    const int64_t plane = (int64_t)(d->nx + 1) * (d->ny + 1);
    if (24 * plane * 4 >= ((int64_t)1 << 31))
      return fail(FBTO_ERR_UNSUPPORTED, "a node plane of %lld nodes exceeds the %lld the K u kernels address",
                  (long long)plane, (long long)(((int64_t)1 << 31) / 96));
  }
  if (!(d->young > 0.0) || !std::isfinite(d->young)) return fail(FBTO_ERR_ARG, "young must be > 0");
  if (!(d->poisson > -1.0 && d->poisson < 0.5)) return fail(FBTO_ERR_ARG, "poisson must be in (-1, 0.5)");
  if (!(d->penal >= 1.0) || !std::isfinite(d->penal)) return fail(FBTO_ERR_ARG, "penal must be >= 1");
  if (!(d->rho_min >= 0.0 && d->rho_min < 1.0)) return fail(FBTO_ERR_ARG, "rho_min must be in [0, 1)");
  if (!(d->filter_radius >= 0.0) || !(d->filter_radius <= 16.0))
    return fail(FBTO_ERR_ARG, "filter_radius must be in [0, 16]");
  if (n_springs < 0 || (n_springs > 0 && (!spring_dof || !spring_k)))
    return fail(FBTO_ERR_ARG, "n_springs = %d with NULL spring arrays", n_springs);
  if (n_springs > 4096) return fail(FBTO_ERR_ARG, "at most 4096 springs");
  for (int s = 0; s < n_springs; ++s) {
    if (spring_dof[s] < 0 || spring_dof[s] >= 3 * N)
      return fail(FBTO_ERR_ARG, "spring %d: DOF %lld out of range", s, (long long)spring_dof[s]);
    if (!(spring_k[s] >= 0.0) || !std::isfinite(spring_k[s]))
      return fail(FBTO_ERR_ARG, "spring %d: stiffness must be finite and >= 0", s);
  }

  fbto_grid_s* g = new (std::nothrow) fbto_grid_s();
  if (!g) return fail(FBTO_ERR_ALLOC, "host allocation failed");
  g->desc = *d;
  Geo& G = g->geo;
  G.nx = d->nx;
  G.ny = d->ny;
  G.nz = d->nz;
  G.nxn = d->nx + 1;
  G.nyn = d->ny + 1;
  G.nzn = d->nz + 1;
  G.N = N;
  G.E = (int64_t)d->nx * d->ny * d->nz;
  G.ndof = 3 * N;
  G.rnx = 1.0 / G.nx;
  G.rny = 1.0 / G.ny;
  G.rnxn = 1.0 / G.nxn;
  G.rnyn = 1.0 / G.nyn;
  modal_coefficients(d->young, d->poisson, g->km64, g->ke_diag);
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 3; ++c) g->km32.dg[a][c] = (float)g->km64.dg[a][c];
  for (int b = 0; b < 2; ++b) {
    g->km32.lam4[b] = (float)g->km64.lam4[b];
    g->km32.mu4[b] = (float)g->km64.mu4[b];
  }
  g->simp.penal = d->penal;
  g->simp.rho_min = d->rho_min;
  g->simp.cubic = d->penal == 3.0 ? 1 : 0;

  // cone-filter stencil: offsets with r - |d| > 0
  std::vector<int> off;
  std::vector<double> w64;
  const double r = d->filter_radius;
  const int R = r > 1.0 ? (int)std::ceil(r) - 1 : 0;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const double dist = std::sqrt((double)(dx * dx + dy * dy + dz * dz));
        double w = r - dist;
        if (r <= 1.0) w = (dx == 0 && dy == 0 && dz == 0) ? 1.0 : 0.0;
        if (w > 0.0) {
          off.push_back(dx);
          off.push_back(dy);
          off.push_back(dz);
          w64.push_back(w);
        }
      }
  std::vector<float> w32(w64.begin(), w64.end());
  g->n_stencil = (int)w64.size();

  std::vector<uint8_t> nm(N, 0);
  if (fixed_dof_mask)
    for (int64_t n = 0; n < N; ++n)
      nm[n] = (uint8_t)((fixed_dof_mask[3 * n] ? 1 : 0) | (fixed_dof_mask[3 * n + 1] ? 2 : 0) |
                        (fixed_dof_mask[3 * n + 2] ? 4 : 0));
  for (int s = 0; s < n_springs; ++s) nm[spring_dof[s] / 3] |= 8;

  auto cleanup_fail = [&](fbto_status_t s) {
    fbto_destroy_grid(g);
    return s;
  };
#define SETUP_TRY(expr)                                                                      \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return cleanup_fail(fail(_e == hipErrorOutOfMemory ? FBTO_ERR_ALLOC : FBTO_ERR_HIP,     \
                               "%s: %s", #expr, hipGetErrorString(_e)));                     \
  } while (0)

  SETUP_TRY(hipGetDevice(&g->device));
  int ncu = 0;
  SETUP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, g->device));
  g->n_cu = ncu > 0 ? ncu : 256;
  int lds_cu = 0;
  SETUP_TRY(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, g->device));
  g->lds_per_cu = lds_cu > 0 ? lds_cu : 160 * 1024;
  SETUP_TRY(hipMalloc(&g->mask, N));
  SETUP_TRY(hipMemcpy(g->mask, nm.data(), N, hipMemcpyHostToDevice));
  g->n_springs = n_springs;
  if (n_springs > 0) {
    std::vector<float> k32(spring_k, spring_k + n_springs);
    SETUP_TRY(hipMalloc(&g->spring_dof, n_springs * sizeof(int64_t)));
    SETUP_TRY(hipMalloc(&g->spring_k64, n_springs * sizeof(double)));
    SETUP_TRY(hipMalloc(&g->spring_k32, n_springs * sizeof(float)));
    SETUP_TRY(hipMemcpy(g->spring_dof, spring_dof, n_springs * sizeof(int64_t), hipMemcpyHostToDevice));
    SETUP_TRY(hipMemcpy(g->spring_k64, spring_k, n_springs * sizeof(double), hipMemcpyHostToDevice));
    SETUP_TRY(hipMemcpy(g->spring_k32, k32.data(), n_springs * sizeof(float), hipMemcpyHostToDevice));
  }
  SETUP_TRY(hipMalloc(&g->stencil_off, off.size() * sizeof(int)));
  SETUP_TRY(hipMalloc(&g->stencil_w64, w64.size() * sizeof(double)));
  SETUP_TRY(hipMalloc(&g->stencil_w32, w32.size() * sizeof(float)));
  SETUP_TRY(hipMemcpy(g->stencil_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
  SETUP_TRY(hipMemcpy(g->stencil_w64, w64.data(), w64.size() * sizeof(double), hipMemcpyHostToDevice));
  SETUP_TRY(hipMemcpy(g->stencil_w32, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice));
  SETUP_TRY(hipMalloc(&g->sc, sizeof(Scalars)));
  SETUP_TRY(hipMemset(g->sc, 0, sizeof(Scalars)));
  g->max_partials = std::max(apply_max_blocks(G, g->n_cu), kMaxVecBlocks);
  SETUP_TRY(hipMalloc(&g->partials, (size_t)P_COUNT * 4 * g->max_partials * sizeof(double)));
  SETUP_TRY(hipMemset(g->partials, 0, (size_t)P_COUNT * 4 * g->max_partials * sizeof(double)));
  SETUP_TRY(hipDeviceSynchronize());
#undef SETUP_TRY
  *out = g;
  return ok();
}

fbto_status_t fbto_setup_grid_2d(const fbto_grid2d_desc_t* d, const uint8_t* fixed_dof_mask, fbto_grid_t* out) {
  if (!d || !out) return fail(FBTO_ERR_ARG, "desc and out must be non-NULL");
  *out = nullptr;
  if (d->nx < 1 || d->ny < 1) return fail(FBTO_ERR_ARG, "grid %d x %d: every axis needs >= 1 element", d->nx, d->ny);
  if (d->nx > 65534 || d->ny > 65534) return fail(FBTO_ERR_ARG, "grid axis longer than 65534 elements");
  const int64_t N = (int64_t)(d->nx + 1) * (d->ny + 1);
  if (N >= ((int64_t)1 << 29))
    return fail(FBTO_ERR_ARG, "grid has %lld nodes (limit 2^29, so that DOF indices fit 32 bits)", (long long)N);
  if (d->max_rhs < 1 || d->max_rhs > 4) return fail(FBTO_ERR_ARG, "max_rhs = %d outside [1, 4]", d->max_rhs);
  if (!(d->young > 0.0) || !std::isfinite(d->young)) return fail(FBTO_ERR_ARG, "young must be > 0");
  if (!(d->poisson > -1.0 && d->poisson < 0.5)) return fail(FBTO_ERR_ARG, "poisson must be in (-1, 0.5)");
  if (!(d->penal >= 1.0) || !std::isfinite(d->penal)) return fail(FBTO_ERR_ARG, "penal must be >= 1");
  if (!(d->rho_min >= 0.0 && d->rho_min < 1.0)) return fail(FBTO_ERR_ARG, "rho_min must be in [0, 1)");
  if (d->filter_half < 0 || d->filter_half > kGaussMaxHalf)
    return fail(FBTO_ERR_ARG, "filter_half = %d outside [0, %d]", d->filter_half, kGaussMaxHalf);
  if (!(d->filter_sigma > 0.0) || !std::isfinite(d->filter_sigma))
    return fail(FBTO_ERR_ARG, "filter_sigma must be finite and > 0");

  fbto_grid_s* g = new (std::nothrow) fbto_grid_s();
  if (!g) return fail(FBTO_ERR_ALLOC, "host allocation failed");
  g->dim = 2;
  g->desc = fbto_grid_desc_t{d->nx, d->ny, 1, d->max_rhs, d->young, d->poisson, d->penal, d->rho_min, 0.0};
  Geo& G = g->geo;
  G.nx = d->nx;
  G.ny = d->ny;
  G.nz = 1;
  G.nxn = d->nx + 1;
  G.nyn = d->ny + 1;
  G.nzn = 1;
  G.N = N;
  G.E = (int64_t)d->nx * d->ny;
  G.ndof = 2 * N;
  G.rnx = 1.0 / G.nx;
  G.rny = 1.0 / G.ny;
  G.rnxn = 1.0 / G.nxn;
  G.rnyn = 1.0 / G.nyn;
  q4_plane_stress(d->young, d->poisson, g->q4_64, g->ke_diag);
  for (int p = 0; p < 8; ++p)
    for (int q = 0; q < 8; ++q) g->q4_32.k[p][q] = (float)g->q4_64.k[p][q];
  g->gauss64 = GaussW<double>{};
  g->gauss32 = GaussW<float>{};
  g->gauss64.half = g->gauss32.half = d->filter_half;
  for (int k = -d->filter_half; k <= d->filter_half; ++k) {
    const double w = std::exp(-(double)(k * k) / (2.0 * d->filter_sigma * d->filter_sigma));
    g->gauss64.w[k + d->filter_half] = w;
    g->gauss32.w[k + d->filter_half] = (float)w;
  }
  g->simp.penal = d->penal;
  g->simp.rho_min = d->rho_min;
  g->simp.cubic = d->penal == 3.0 ? 1 : 0;

  std::vector<uint8_t> nm(N, 0);
  if (fixed_dof_mask)
    for (int64_t n = 0; n < N; ++n)
      nm[n] = (uint8_t)((fixed_dof_mask[2 * n] ? 1 : 0) | (fixed_dof_mask[2 * n + 1] ? 2 : 0));

  auto cleanup_fail = [&](fbto_status_t s) {
    fbto_destroy_grid(g);
    return s;
  };
#define SETUP_TRY(expr)                                                                      \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return cleanup_fail(fail(_e == hipErrorOutOfMemory ? FBTO_ERR_ALLOC : FBTO_ERR_HIP,     \
                               "%s: %s", #expr, hipGetErrorString(_e)));                     \
  } while (0)
  SETUP_TRY(hipGetDevice(&g->device));
  int ncu = 0;
  SETUP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, g->device));
  g->n_cu = ncu > 0 ? ncu : 256;
  int lds_cu = 0;
  SETUP_TRY(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, g->device));
  g->lds_per_cu = lds_cu > 0 ? lds_cu : 160 * 1024;
  SETUP_TRY(hipMalloc(&g->mask, N));
  SETUP_TRY(hipMemcpy(g->mask, nm.data(), N, hipMemcpyHostToDevice));
  SETUP_TRY(hipMalloc(&g->sc, sizeof(Scalars)));
  SETUP_TRY(hipMemset(g->sc, 0, sizeof(Scalars)));
  g->max_partials = kMaxVecBlocks;
  SETUP_TRY(hipMalloc(&g->partials, (size_t)P_COUNT * 4 * g->max_partials * sizeof(double)));
  SETUP_TRY(hipMemset(g->partials, 0, (size_t)P_COUNT * 4 * g->max_partials * sizeof(double)));
  SETUP_TRY(hipDeviceSynchronize());
#undef SETUP_TRY
  *out = g;
  return ok();
}

fbto_status_t fbto_destroy_grid(fbto_grid_t g) {
  if (!g) return fail(FBTO_ERR_ARG, "grid handle is NULL");
  (void)hipDeviceSynchronize();
  void* ps[] = {g->mask, g->spring_dof, g->spring_k64, g->spring_k32, g->stencil_off,
                g->stencil_w64, g->stencil_w32, g->sc, g->partials, g->sort.base};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  free_vecs(g->v64);
  free_vecs(g->v32);
  drop_extra(g);
  delete g;
  return ok();
}

fbto_status_t fbto_set_option(fbto_grid_t g, fbto_option_t option, int64_t value) {
  if (check_grid(g)) return FBTO_ERR_ARG;
  switch (option) {
    case FBTO_OPT_PROJ_PASSES:
      if (value < 1 || value > kProjMaxPasses)
        return fail(FBTO_ERR_ARG, "projection passes %lld outside [1, %d]", (long long)value, kProjMaxPasses);
      g->proj_passes_warm = (int)value;
      return ok();
    case FBTO_OPT_APPLY_TILE:
    case FBTO_OPT_CGF_TILE: {
      if (value < 0 || value >= ((int64_t)1 << 28)) return fail(FBTO_ERR_ARG, "tile value %lld out of range", (long long)value);
      const int bx = (int)(value & 0xff), by = (int)((value >> 8) & 0xff), dz = (int)((value >> 16) & 0xff);
      const int cap = (int)((value >> 24) & 0xf);
      // the fused CG step has a thread per node column, (bx + 1) (by + 1);
      // the other z-march kernels take the shape in both layouts
      const int lo_t = option == FBTO_OPT_CGF_TILE ? (bx + 1) * (by + 1) : bx * by;
      if ((bx && (bx < 8 || bx > 64)) || (by && (by < 4 || by > 64)) || dz > 64 ||
          (bx && by && (lo_t < 128 || (bx + 1) * (by + 1) > 256)))
        return fail(FBTO_ERR_ARG, "tile %d x %d x %d outside the kernel's limits", bx, by, dz);
      if (cap && (cap < 2 || lds_for_block_cap(g->lds_per_cu, cap) > (int)kApplyMaxLds))
        return fail(FBTO_ERR_ARG, "blocks per CU %d: not 2 or more, or needs more than %d bytes of LDS per block", cap,
                    (int)kApplyMaxLds);
      g->tile_override[option == FBTO_OPT_CGF_TILE ? 1 : 0] = (int)value;
      for (auto& a : g->tiles)  // chosen again on the next launch
        for (auto& b : a)
          for (auto& t : b) t = TileChoice{};
      return ok();
    }
  }
  return fail(FBTO_ERR_ARG, "unknown option %d", (int)option);
}

fbto_status_t fbto_grid_sizes(fbto_grid_t g, int64_t* n_elem, int64_t* n_node, int64_t* n_dof) {
  if (check_grid(g)) return FBTO_ERR_ARG;
  if (n_elem) *n_elem = g->geo.E;
  if (n_node) *n_node = g->geo.N;
  if (n_dof) *n_dof = g->geo.ndof;
  return ok();
}

fbto_status_t fbto_apply_K(fbto_grid_t g, fbto_prec_t prec, const void* rho_phys, const void* u,
                           void* y, int32_t nrhs, void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!rho_phys || !u || !y) return fail(FBTO_ERR_ARG, "rho_phys, u and y must be non-NULL");
  if (u == y) return fail(FBTO_ERR_ARG, "u and y must not overlap");
  hipStream_t st = (hipStream_t)stream;
  if (prec == FBTO_F64)
    HIP_TRY(launch_apply<double>(g, (const double*)rho_phys, (const double*)u, (double*)y, nrhs, st));
  else
    HIP_TRY(launch_apply<float>(g, (const float*)rho_phys, (const float*)u, (float*)y, nrhs, st));
  return ok();
}

fbto_status_t fbto_inner_solve(fbto_grid_t g, fbto_prec_t prec, const void* rho_phys, const void* f,
                               void* u, int32_t nrhs, fbto_method_t method, int32_t steps,
                               double omega, double rtol, double* info, void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!rho_phys || !f || !u) return fail(FBTO_ERR_ARG, "rho_phys, f and u must be non-NULL");
  if (steps < 0) return fail(FBTO_ERR_ARG, "steps must be >= 0");
  if (!(rtol >= 0.0)) return fail(FBTO_ERR_ARG, "rtol must be >= 0");
  if (method != FBTO_PCG_JACOBI && method != FBTO_RICHARDSON && method != FBTO_DAMPED_JACOBI &&
      method != FBTO_KRYLOV)
    return fail(FBTO_ERR_ARG, "unknown method %d", (int)method);
  if (method != FBTO_PCG_JACOBI && rtol > 0.0)
    return fail(FBTO_ERR_UNSUPPORTED, "rtol > 0 is supported for PCG only");
  if (method != FBTO_PCG_JACOBI && !(std::isfinite(omega) && omega > 0.0))
    return fail(FBTO_ERR_ARG, "omega must be finite and > 0");
  if (method == FBTO_KRYLOV && steps > 1000) return fail(FBTO_ERR_ARG, "Krylov degree %d > 1000", (int)steps);
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s;
  if (prec == FBTO_F64) {
    if ((s = ensure_vecs<double>(g))) return s;
    if (method == FBTO_PCG_JACOBI)
      s = pcg_solve<double>(g, (const double*)rho_phys, (const double*)f, (double*)u, nrhs, steps, rtol, st);
    else if (method == FBTO_KRYLOV)
      s = krylov_run<double>(g, (const double*)rho_phys, (const double*)f, (double*)u, nrhs, steps, omega, st);
    else
      s = relax_run<double>(g, (const double*)rho_phys, (const double*)f, (double*)u, nrhs, steps, omega,
                            method == FBTO_DAMPED_JACOBI, st);
  } else {
    if ((s = ensure_vecs<float>(g))) return s;
    if (method == FBTO_PCG_JACOBI)
      s = pcg_solve<float>(g, (const float*)rho_phys, (const float*)f, (float*)u, nrhs, steps, rtol, st);
    else if (method == FBTO_KRYLOV)
      s = krylov_run<float>(g, (const float*)rho_phys, (const float*)f, (float*)u, nrhs, steps, omega, st);
    else
      s = relax_run<float>(g, (const float*)rho_phys, (const float*)f, (float*)u, nrhs, steps, omega,
                           method == FBTO_DAMPED_JACOBI, st);
  }
  if (s) return s;
  const double steps_done = method == FBTO_PCG_JACOBI ? -1.0 : (method == FBTO_KRYLOV ? steps + 1.0 : steps);
  if (info) HIP_TRY(launch_solve_info(g, info, nrhs, steps_done, st));
  return ok();
}

fbto_status_t fbto_solve_refined(fbto_grid_t g, fbto_prec_t inner_prec, const double* rho_phys,
                                 const double* f, double* u, int32_t nrhs, double rtol,
                                 int32_t max_refine, int32_t inner_steps, double inner_rtol,
                                 double* info, int32_t* refinements, void* stream) {
  if (check_grid(g) || check_prec(inner_prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!rho_phys || !f || !u) return fail(FBTO_ERR_ARG, "rho_phys, f and u must be non-NULL");
  if (!(rtol > 0.0)) return fail(FBTO_ERR_ARG, "rtol must be > 0");
  if (max_refine < 1 || inner_steps < 1) return fail(FBTO_ERR_ARG, "max_refine and inner_steps must be >= 1");
  if (!(inner_rtol >= 0.0 && inner_rtol < 1.0)) return fail(FBTO_ERR_ARG, "inner_rtol must be in [0, 1)");
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s;
  if ((s = ensure_vecs<double>(g))) return s;
  if (inner_prec == FBTO_F32 && (s = ensure_vecs<float>(g))) return s;
  GridExtra* ex = extra_of(g);
  IrBufs& B = inner_prec == FBTO_F32 ? ex->ir32 : ex->ir64;
  const size_t es = inner_prec == FBTO_F32 ? sizeof(float) : sizeof(double);
  const int64_t nd = g->geo.ndof * g->desc.max_rhs;
  if (!B.f) HIP_TRY(hipMalloc(&B.f, nd * es));
  if (!B.d) HIP_TRY(hipMalloc(&B.d, nd * es));
  if (!B.r64) HIP_TRY(hipMalloc(&B.r64, nd * sizeof(double)));
  const int64_t n = g->geo.ndof * nrhs;
  float* rho32 = (float*)g->v32.rho;
  if (inner_prec == FBTO_F32) HIP_TRY(launch_convert<float>(rho_phys, rho32, g->geo.E, 0, st));
  HIP_TRY(launch_diag<double>(g, rho_phys, (double*)g->v64.invD, st));
  int it = 0;
  double total_inner = 0.0;
  std::vector<double> fn(nrhs, 0.0);
  for (;;) {
    // FP64 residual r = f - K64 u and its norms
    if ((s = residual_norms<double>(g, rho_phys, u, f, B.r64, (const double*)g->v64.invD, nrhs, st))) return s;
    Scalars h;
    HIP_TRY(hipMemcpyAsync(&h, g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool conv = true;
    for (int R = 0; R < nrhs; ++R) {
      fn[R] = h.fnorm2[R];
      if (!std::isfinite(h.rnorm2[R])) return fail(FBTO_ERR_NONFINITE, "non-finite refinement residual");
      conv = conv && h.rnorm2[R] <= rtol * h.fnorm2[R];
    }
    if (conv || it >= max_refine) break;
    ++it;
    if (inner_prec == FBTO_F32) {
      HIP_TRY(launch_ir_scale(g, B.r64, (float*)B.f, nrhs, st));
      HIP_TRY(hipMemsetAsync(B.d, 0, n * sizeof(float), st));
      if ((s = pcg_solve<float>(g, rho32, (const float*)B.f, (float*)B.d, nrhs, inner_steps, inner_rtol, st))) return s;
      HIP_TRY(launch_ir_accum(g, u, (const float*)B.d, nrhs, st));
    } else {
      HIP_TRY(hipMemcpyAsync(B.f, B.r64, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemsetAsync(B.d, 0, n * sizeof(double), st));
      if ((s = pcg_solve<double>(g, rho_phys, (const double*)B.f, (double*)B.d, nrhs, inner_steps, inner_rtol, st))) return s;
      HIP_TRY(launch_axpy64(u, (const double*)B.d, n, st));
    }
    // inner steps taken (the largest over the RHS), read back with the
    // refinement loop's own synchronisation budget: one copy per refinement
    double steps_h[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(steps_h, g->sc->steps, sizeof(steps_h), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double mx = 0.0;
    for (int R = 0; R < nrhs; ++R) mx = std::max(mx, steps_h[R]);
    total_inner += mx;
  }
  // final norms are in the scalars (from the last FP64 residual)
  if (info) HIP_TRY(launch_solve_info(g, info, nrhs, total_inner, st));
  if (refinements) *refinements = it;
  return ok();
}

fbto_status_t fbto_sensitivity(fbto_grid_t g, fbto_prec_t prec, const void* rho_phys, const void* u,
                               const void* lam, const void* f, int32_t nrhs, void* dobj, double* obj,
                               void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!rho_phys || !u || !dobj) return fail(FBTO_ERR_ARG, "rho_phys, u and dobj must be non-NULL");
  hipStream_t st = (hipStream_t)stream;
  if (prec == FBTO_F64) {
    HIP_TRY(launch_sens<double>(g, (const double*)rho_phys, (const double*)u, (const double*)lam, nrhs,
                                (double*)dobj, (const double*)nullptr, st));
    if (f && obj) {
      HIP_TRY(launch_dot<double>(g, (const double*)f, (const double*)u, nrhs, st));
      HIP_TRY(launch_dot_store(g, obj, st));
    }
  } else {
    HIP_TRY(launch_sens<float>(g, (const float*)rho_phys, (const float*)u, (const float*)lam, nrhs,
                               (float*)dobj, (const float*)nullptr, st));
    if (f && obj) {
      HIP_TRY(launch_dot<float>(g, (const float*)f, (const float*)u, nrhs, st));
      HIP_TRY(launch_dot_store(g, obj, st));
    }
  }
  return ok();
}

fbto_status_t fbto_filter(fbto_grid_t g, fbto_prec_t prec, int32_t transpose, const void* in, void* out,
                          void* stream) {
  if (check_grid(g) || check_prec(prec)) return FBTO_ERR_ARG;
  if (!in || !out) return fail(FBTO_ERR_ARG, "in and out must be non-NULL");
  if (in == out) return fail(FBTO_ERR_ARG, "in and out must not overlap");
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s;
  if (prec == FBTO_F64) {
    if ((s = ensure_vecs<double>(g))) return s;
    HIP_TRY(launch_filter<double>(g, transpose ? 1 : 0, (const double*)in, (double*)out, 0, st));
  } else {
    if ((s = ensure_vecs<float>(g))) return s;
    HIP_TRY(launch_filter<float>(g, transpose ? 1 : 0, (const float*)in, (float*)out, 0, st));
  }
  return ok();
}

fbto_status_t fbto_project_volume(fbto_grid_t g, fbto_prec_t prec, const void* y, void* x, double lo,
                                  double hi, double vmax, int32_t max_passes, double* lambda, double* status,
                                  void* stream) {
  if (check_grid(g) || check_prec(prec)) return FBTO_ERR_ARG;
  if (!y || !x) return fail(FBTO_ERR_ARG, "y and x must be non-NULL");
  if (!(std::isfinite(lo) && std::isfinite(hi) && lo <= hi)) return fail(FBTO_ERR_ARG, "need finite lo <= hi");
  if (!std::isfinite(vmax)) return fail(FBTO_ERR_ARG, "vmax must be finite");
  if (max_passes < 0 || max_passes > kProjMaxPasses)
    return fail(FBTO_ERR_ARG, "max_passes = %d outside [0, %d]", (int)max_passes, kProjMaxPasses);
  if (vmax < lo * (double)g->geo.E)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g: the feasible set is empty", vmax,
                lo * (double)g->geo.E);
  const int passes = max_passes == 0 ? 8 : max_passes;
  hipStream_t st = (hipStream_t)stream;
  if (prec == FBTO_F64)
    HIP_TRY(launch_project<double>(proj_ws(g), g->geo.E, (const double*)y, (double*)x, lo, hi, vmax, 0, passes,
                                   nullptr, lambda, status, st));
  else
    HIP_TRY(launch_project<float>(proj_ws(g), g->geo.E, (const float*)y, (float*)x, lo, hi, vmax, 0, passes,
                                  nullptr, lambda, status, st));
  return ok();
}

fbto_status_t fbto_project_volume_sorted(fbto_grid_t g, fbto_prec_t prec, const void* y, void* x, double lo,
                                         double hi, double vmax, double* lambda, void* stream) {
  if (check_grid(g) || check_prec(prec)) return FBTO_ERR_ARG;
  if (!y || !x) return fail(FBTO_ERR_ARG, "y and x must be non-NULL");
  if (!(std::isfinite(lo) && std::isfinite(hi) && lo <= hi)) return fail(FBTO_ERR_ARG, "need finite lo <= hi");
  if (!std::isfinite(vmax)) return fail(FBTO_ERR_ARG, "vmax must be finite");
  if (g->geo.E > (int64_t)INT32_MAX) return fail(FBTO_ERR_ARG, "the sort ranks keys in 32 bits: E must be < 2^31");
  if (vmax < lo * (double)g->geo.E)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g: the feasible set is empty", vmax,
                lo * (double)g->geo.E);
  fbto_status_t s;
  if ((s = ensure_sort(g))) return s;
  hipStream_t st = (hipStream_t)stream;
  if (prec == FBTO_F64)
    HIP_TRY(launch_project_sorted<double>(g, (const double*)y, (double*)x, lo, hi, vmax, lambda, st));
  else
    HIP_TRY(launch_project_sorted<float>(g, (const float*)y, (float*)x, lo, hi, vmax, lambda, st));
  return ok();
}

fbto_status_t fbto_outer_step(fbto_grid_t g, fbto_prec_t prec, void* x, void* u, const void* f,
                              int32_t nrhs, int32_t k, double alpha0, int32_t inner_steps,
                              int32_t mean_project, double lo, double vmax, double* info,
                              void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!x || !u || !f) return fail(FBTO_ERR_ARG, "x, u and f must be non-NULL");
  if (k < 1) return fail(FBTO_ERR_ARG, "k is 1-based");
  if (inner_steps < 0) return fail(FBTO_ERR_ARG, "inner_steps must be >= 0");
  if (!(std::isfinite(alpha0) && alpha0 >= 0.0)) return fail(FBTO_ERR_ARG, "alpha0 must be finite and >= 0");
  if (!(std::isfinite(lo) && lo <= 1.0)) return fail(FBTO_ERR_ARG, "need lo <= 1");
  if (vmax < lo * (double)g->geo.E)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g", vmax, lo * (double)g->geo.E);
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s;
  if (prec == FBTO_F64) {
    if ((s = ensure_vecs<double>(g))) return s;
    s = outer_run<double>(g, (double*)x, (double*)u, (const double*)f, nrhs, k, alpha0, inner_steps,
                          mean_project, lo, vmax, info, st);
  } else {
    if ((s = ensure_vecs<float>(g))) return s;
    s = outer_run<float>(g, (float*)x, (float*)u, (const float*)f, nrhs, k, alpha0, inner_steps,
                         mean_project, lo, vmax, info, st);
  }
  if (s) return s;
  return ok();
}

fbto_status_t fbto_outer_steps(fbto_grid_t g, fbto_prec_t prec, void* x, void* u, const void* f,
                               int32_t nrhs, int32_t k, int32_t n_steps, double alpha0, int32_t inner_steps,
                               int32_t mean_project, double lo, double vmax, double* info, void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!x || !u || !f) return fail(FBTO_ERR_ARG, "x, u and f must be non-NULL");
  if (k < 1) return fail(FBTO_ERR_ARG, "k is 1-based");
  if (n_steps < 1) return fail(FBTO_ERR_ARG, "n_steps = %d: need at least one iteration", (int)n_steps);
  if (n_steps > INT32_MAX - k) return fail(FBTO_ERR_ARG, "k + n_steps overflows");
  if (inner_steps < 0) return fail(FBTO_ERR_ARG, "inner_steps must be >= 0");
  if (!(std::isfinite(alpha0) && alpha0 >= 0.0)) return fail(FBTO_ERR_ARG, "alpha0 must be finite and >= 0");
  if (!(std::isfinite(lo) && lo <= 1.0)) return fail(FBTO_ERR_ARG, "need lo <= 1");
  if (vmax < lo * (double)g->geo.E)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g", vmax, lo * (double)g->geo.E);
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s = prec == FBTO_F64 ? ensure_vecs<double>(g) : ensure_vecs<float>(g);
  if (s) return s;
  bool rho_ready = false;  // the first iteration filters the caller's x
  for (int32_t i = 0; i < n_steps; ++i) {
    double* inf = info ? info + (int64_t)i * FBTO_OUTER_INFO : nullptr;
    const bool fuse_next = i + 1 < n_steps;
    if (prec == FBTO_F64)
      s = outer_run<double>(g, (double*)x, (double*)u, (const double*)f, nrhs, k + i, alpha0, inner_steps,
                            mean_project, lo, vmax, inf, st, -1, 1.0, 0.0, &rho_ready, fuse_next);
    else
      s = outer_run<float>(g, (float*)x, (float*)u, (const float*)f, nrhs, k + i, alpha0, inner_steps,
                           mean_project, lo, vmax, inf, st, -1, 1.0, 0.0, &rho_ready, fuse_next);
    if (s) return s;
  }
  return ok();
}

fbto_status_t fbto_outer_step_exact(fbto_grid_t g, fbto_prec_t prec, void* x, void* u, const void* f,
                                    int32_t nrhs, int32_t k, double alpha0, double rtol, int32_t max_steps,
                                    int32_t mean_project, double lo, double vmax, double* info, void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!x || !u || !f) return fail(FBTO_ERR_ARG, "x, u and f must be non-NULL");
  if (k < 1) return fail(FBTO_ERR_ARG, "k is 1-based");
  if (!(rtol > 0.0 && rtol < 1.0)) return fail(FBTO_ERR_ARG, "rtol must be in (0, 1)");
  if (max_steps < 1) return fail(FBTO_ERR_ARG, "max_steps must be >= 1");
  if (!(std::isfinite(alpha0) && alpha0 >= 0.0)) return fail(FBTO_ERR_ARG, "alpha0 must be finite and >= 0");
  if (!(std::isfinite(lo) && lo <= 1.0)) return fail(FBTO_ERR_ARG, "need lo <= 1");
  if (vmax < lo * (double)g->geo.E)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g", vmax, lo * (double)g->geo.E);
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s;
  if (prec == FBTO_F64) {
    if ((s = ensure_vecs<double>(g))) return s;
    s = outer_run<double>(g, (double*)x, (double*)u, (const double*)f, nrhs, k, alpha0, max_steps, mean_project,
                          lo, vmax, info, st, -1, 1.0, rtol);
  } else {
    if ((s = ensure_vecs<float>(g))) return s;
    s = outer_run<float>(g, (float*)x, (float*)u, (const float*)f, nrhs, k, alpha0, max_steps, mean_project, lo,
                         vmax, info, st, -1, 1.0, rtol);
  }
  if (s) return s;
  return ok();
}

fbto_status_t fbto_outer_step_krylov(fbto_grid_t g, fbto_prec_t prec, void* x, void* u, const void* f,
                                     int32_t nrhs, int32_t k, double alpha0, int32_t degree, double beta,
                                     int32_t mean_project, double lo, double vmax, double* info,
                                     void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!x || !u || !f) return fail(FBTO_ERR_ARG, "x, u and f must be non-NULL");
  if (k < 1) return fail(FBTO_ERR_ARG, "k is 1-based");
  if (degree < 0 || degree > 1000) return fail(FBTO_ERR_ARG, "Krylov degree must be in [0, 1000]");
  if (!(std::isfinite(beta) && beta > 0.0)) return fail(FBTO_ERR_ARG, "beta must be finite and > 0");
  if (!(std::isfinite(alpha0) && alpha0 >= 0.0)) return fail(FBTO_ERR_ARG, "alpha0 must be finite and >= 0");
  if (!(std::isfinite(lo) && lo <= 1.0)) return fail(FBTO_ERR_ARG, "need lo <= 1");
  if (vmax < lo * (double)g->geo.E)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g", vmax, lo * (double)g->geo.E);
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s;
  if (prec == FBTO_F64) {
    if ((s = ensure_vecs<double>(g))) return s;
    s = outer_run<double>(g, (double*)x, (double*)u, (const double*)f, nrhs, k, alpha0, 0, mean_project, lo,
                          vmax, info, st, degree, beta);
  } else {
    if ((s = ensure_vecs<float>(g))) return s;
    s = outer_run<float>(g, (float*)x, (float*)u, (const float*)f, nrhs, k, alpha0, 0, mean_project, lo, vmax,
                         info, st, degree, beta);
  }
  if (s) return s;
  return ok();
}

fbto_status_t fbto_optimality(fbto_grid_t g, fbto_prec_t prec, const void* x, const void* u, const void* f,
                              int32_t nrhs, double alpha, double lo, double vmax, double rtol, int32_t max_steps,
                              double* out, void* stream) {
  if (check_grid(g) || check_prec(prec) || check_nrhs(g, nrhs)) return FBTO_ERR_ARG;
  if (!x || !u || !f || !out) return fail(FBTO_ERR_ARG, "x, u, f and out must be non-NULL");
  if (!(std::isfinite(alpha) && alpha > 0.0)) return fail(FBTO_ERR_ARG, "alpha must be finite and > 0");
  if (!(rtol > 0.0 && rtol < 1.0)) return fail(FBTO_ERR_ARG, "rtol must be in (0, 1)");
  if (max_steps < 1) return fail(FBTO_ERR_ARG, "max_steps must be >= 1");
  if (!(std::isfinite(lo) && lo <= 1.0)) return fail(FBTO_ERR_ARG, "need lo <= 1");
  if (vmax < lo * (double)g->geo.E)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g", vmax, lo * (double)g->geo.E);
  hipStream_t st = (hipStream_t)stream;
  fbto_status_t s;
  if (prec == FBTO_F64) {
    if ((s = ensure_vecs<double>(g))) return s;
    s = optimality_run<double>(g, (const double*)x, (const double*)u, (const double*)f, nrhs, alpha, lo, vmax,
                               rtol, max_steps, out, st);
  } else {
    if ((s = ensure_vecs<float>(g))) return s;
    s = optimality_run<float>(g, (const float*)x, (const float*)u, (const float*)f, nrhs, alpha, lo, vmax, rtol,
                              max_steps, out, st);
  }
  if (s) return s;
  return ok();
}

fbto_status_t fbto_project_volume_noalloc(fbto_prec_t prec, int64_t n_elem, const void* y, void* x, double lo,
                                          double hi, double vmax, int32_t max_passes, double* lambda,
                                          double* status, void* stream) {
  if (check_prec(prec)) return FBTO_ERR_ARG;
  if (n_elem < 1 || n_elem > FBTO_NOALLOC_MAX_ELEMS)
    return fail(FBTO_ERR_ARG, "n_elem = %lld outside [1, %lld]: the allocation-free projection serves at most "
                "%lld elements", (long long)n_elem, (long long)FBTO_NOALLOC_MAX_ELEMS,
                (long long)FBTO_NOALLOC_MAX_ELEMS);
  if (!y || !x) return fail(FBTO_ERR_ARG, "y and x must be non-NULL");
  if (!(std::isfinite(lo) && std::isfinite(hi) && lo <= hi)) return fail(FBTO_ERR_ARG, "need finite lo <= hi");
  if (!std::isfinite(vmax)) return fail(FBTO_ERR_ARG, "vmax must be finite");
  if (max_passes < 0 || max_passes > kProjMaxPasses)
    return fail(FBTO_ERR_ARG, "max_passes = %d outside [0, %d]", (int)max_passes, kProjMaxPasses);
  if (vmax < lo * (double)n_elem)
    return fail(FBTO_ERR_INFEASIBLE, "vmax = %g < lo * E = %g: the feasible set is empty", vmax,
                lo * (double)n_elem);
  const int nb = vec_blocks(n_elem);
  if (nb > kMaxVecBlocks)
    return fail(FBTO_ERR_ARG, "%d partial blocks exceed the scratch's %d", nb, kMaxVecBlocks);
  double* base = nullptr;
  if (fbto_status_t s = scratch_on_current_device(&base)) return s;
  const ProjWs W{base, (int64_t)kMaxVecBlocks, kMaxVecBlocks, reinterpret_cast<Scalars*>(base + kNoAllocPartDoubles)};
  const int passes = max_passes == 0 ? 8 : max_passes;
  hipStream_t st = (hipStream_t)stream;
  // cold start: k_proj_init writes the seed partials and clears the warm
  // start; every later slot is written before it is read
  if (prec == FBTO_F64)
    HIP_TRY(launch_project<double>(W, n_elem, (const double*)y, (double*)x, lo, hi, vmax, 0, passes, nullptr,
                                   lambda, status, st));
  else
    HIP_TRY(launch_project<float>(W, n_elem, (const float*)y, (float*)x, lo, hi, vmax, 0, passes, nullptr, lambda,
                                  status, st));
  return ok();
}

}  // extern "C"
