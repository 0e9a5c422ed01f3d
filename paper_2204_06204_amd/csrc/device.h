// Device helpers: deterministic FP64 reductions, SIMP scaling, node loads
// and the element product in the sum/difference basis.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace fbto {

// --------------------------------------------------------------------------
// FP64 reductions with a fixed summation order (deterministic run to run).
// --------------------------------------------------------------------------
// Wave-wide sum / max of a double with DPP lane moves (no LDS traffic):
// xor-1 and xor-2 within quads, mirrors within 8 and 16 lanes, then the
// row broadcasts fold the four 16-lane rows into lane 63, which is read
// back as a wave-uniform value.  The order of operations is fixed.
// DPP and readlane read all 64 lanes whatever the execution mask, so every
// kernel that reduces this way is launched with whole waves (a partial last
// wave would mix in the stale registers of its missing lanes).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int rlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(rhi, rlo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_move<0x140, 0xf>(v);   // row_mirror: every lane holds its row's sum
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<0xB1, 0xf>(v));
  v = fmax(v, dpp_move<0x4E, 0xf>(v));
  v = fmax(v, dpp_move<0x141, 0xf>(v));
  v = fmax(v, dpp_move<0x140, 0xf>(v));
  // rows not written by a broadcast receive 0 from dpp_move; max with a
  // non-negative or -inf identity needs the real value, so fold explicitly
  const double b15 = dpp_move<0x142, 0xa>(v);
  v = ((__lane_id() >> 4) & 1) ? fmax(v, b15) : v;
  const double b31 = dpp_move<0x143, 0xc>(v);
  v = (__lane_id() >= 32) ? fmax(v, b31) : v;
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Reduce NV values over the block: entry i is a sum, or a max when bit i of
// MAXMASK is set.  The result is returned to every thread.
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void block_reduce(double (&v)[NV]) {
  __shared__ double sh[NV][16];
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int lane = tid & 63, w = tid >> 6, nw = (nthr + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double x = ((MAXMASK >> i) & 1u) ? wave_max(v[i]) : wave_sum(v[i]);
    if (lane == 0) sh[i][w] = x;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double acc = sh[i][0];
    for (int k = 1; k < nw; ++k) acc = ((MAXMASK >> i) & 1u) ? fmax(acc, sh[i][k]) : acc + sh[i][k];
    v[i] = acc;
  }
  __syncthreads();
}

// The same for a block of NTHR threads (a multiple of 64) through LDS: the
// values are stored, then 16 lanes per value fold a strided sixteenth of the
// block's entries each and a row-wise DPP butterfly joins the 16 lanes.
// Every thread does about NV + NTHR / 16 operations, against some 20 per
// value and wave for the DPP reduction of every value above.  The order of
// operations is fixed.
template <int NV, unsigned MAXMASK, int NTHR>
__device__ __forceinline__ void block_reduce_lds(double (&v)[NV]) {
  static_assert(NTHR % 64 == 0 && NTHR <= 1024, "whole waves");
  constexpr int SEG = NTHR / 16;
  __shared__ double sh[NV][NTHR];
  __shared__ double res[NV];
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NV; ++i) sh[i][tid] = v[i];
  __syncthreads();
  for (int t = tid; t < NV * 16; t += NTHR) {  // rows of 16 lanes: one value each
    const int i = t >> 4, l = t & 15;
    const bool is_max = (MAXMASK >> i) & 1u;
    double acc = sh[i][l];
#pragma unroll
    for (int j = 1; j < SEG; ++j) {
      const double x = sh[i][l + 16 * j];
      acc = is_max ? fmax(acc, x) : acc + x;
    }
    const double a1 = dpp_move<0xB1, 0xf>(acc);   // quad_perm [1,0,3,2]
    acc = is_max ? fmax(acc, a1) : acc + a1;
    const double a2 = dpp_move<0x4E, 0xf>(acc);   // quad_perm [2,3,0,1]
    acc = is_max ? fmax(acc, a2) : acc + a2;
    const double a3 = dpp_move<0x141, 0xf>(acc);  // row_half_mirror
    acc = is_max ? fmax(acc, a3) : acc + a3;
    const double a4 = dpp_move<0x140, 0xf>(acc);  // row_mirror: every lane holds the row's result
    acc = is_max ? fmax(acc, a4) : acc + a4;
    if (l == 0) res[i] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = res[i];
}

// Reduce NV arrays of per-block partials (entry i: n[i] values at src[i];
// sum, or max where bit i of MAXMASK is set).  Every block computes the same
// result in the same order; the producing kernel has finished, so plain
// loads see its stores.  Each round loads two entries per thread of every
// array before folding any, so that the arrays cost one memory latency per
// round, not one each.
template <int NV, unsigned MAXMASK, int NTHR = 0>
__device__ __forceinline__ void reduce_parts(double (&v)[NV], const double* const (&src)[NV],
                                             const int (&n)[NV]) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  int nmax = 0;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    nmax = n[i] > nmax ? n[i] : nmax;
    v[i] = ((MAXMASK >> i) & 1u) ? -INFINITY : 0.0;
  }
  for (int k = tid; k - tid < nmax; k += 2 * nthr) {
    double x[NV][2];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double id = ((MAXMASK >> i) & 1u) ? -INFINITY : 0.0;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int kk = k + u * nthr;
        x[i][u] = kk < n[i] ? src[i][kk] : id;
      }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int u = 0; u < 2; ++u) v[i] = ((MAXMASK >> i) & 1u) ? fmax(v[i], x[i][u]) : v[i] + x[i][u];
  }
  if constexpr (NTHR > 0) block_reduce_lds<NV, MAXMASK, NTHR>(v);
  else block_reduce<NV, MAXMASK>(v);
}

// Block-reduce NV values and let thread 0 store them as this block's
// partials: entry i goes to dst[i][block].  NTHR > 0: the block has NTHR
// threads, reduced through LDS.
template <int NV, unsigned MAXMASK, int NTHR = 0>
__device__ __forceinline__ void write_parts(double (&v)[NV], double* const (&dst)[NV], int block) {
  if constexpr (NTHR > 0) block_reduce_lds<NV, MAXMASK, NTHR>(v);
  else block_reduce<NV, MAXMASK>(v);
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) dst[i][block] = v[i];
  }
}

// q = n / d for 0 <= n < 2^31 with rd = 1.0 / d: the FP64 product is within
// 2^-21 of n / d, so one correction step makes the quotient exact.
__device__ __forceinline__ int fdiv(int n, int d, double rd) {
  int q = (int)((double)n * rd);
  const int r = n - q * d;
  q += (r >= d) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return q;
}

// --------------------------------------------------------------------------
// SIMP scaling s = rho_min + (1 - rho_min) rho^p and ds/drho.
// --------------------------------------------------------------------------
// General exponents: FP64 goes through pow() in a separate function, so that
// the cubic case (the common SIMP exponent) keeps the hot loops free of its
// code; FP32 takes rho^e = 2^(e log2 rho) from the hardware's base-2
// exponential and logarithm (a few ulp, no call: a call inside the z-march
// makes the compiler keep its live scalar registers in vector lanes).
__device__ __noinline__ double simp_pow(double rho, double e) { return pow(rho, e); }

template <typename T>
__device__ __forceinline__ T simp_pow_t(T rho, double e) {
  if constexpr (sizeof(T) == 4) {
    if (!(rho > 0.0f)) return rho == 0.0f ? (e == 0.0 ? 1.0f : 0.0f) : __builtin_nanf("");
    return __builtin_amdgcn_exp2f((float)e * __builtin_amdgcn_logf(rho));
  } else {
    return simp_pow(rho, e);
  }
}

template <typename T>
__device__ __forceinline__ T simp_s(T rho, const Simp& sp) {
  const T rm = (T)sp.rho_min;
  T pw;
  if (sp.cubic) pw = rho * rho * rho;
  else pw = simp_pow_t<T>(rho, sp.penal);
  return rm + ((T)1 - rm) * pw;
}
template <typename T>
__device__ __forceinline__ T simp_ds(T rho, const Simp& sp) {
  const T rm = (T)sp.rho_min;
  T pw;
  if (sp.cubic) pw = rho * rho;
  else pw = simp_pow_t<T>(rho, sp.penal - 1.0);
  return (T)sp.penal * ((T)1 - rm) * pw;
}

// --------------------------------------------------------------------------
// Element product in the sum/difference basis (45 nonzeros instead of the
// dense 24 x 24): analysis butterflies, sparse modal KE, synthesis.
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void analysis8(T (&v)[8]) {
#pragma unroll
  for (int bit = 1; bit < 8; bit <<= 1) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i & bit) continue;
      const T lo = v[i], hi = v[i | bit];
      v[i] = lo + hi;
      v[i | bit] = hi - lo;
    }
  }
}
template <typename T>
__device__ __forceinline__ void synthesis8(T (&v)[8]) {
#pragma unroll
  for (int bit = 1; bit < 8; bit <<= 1) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i & bit) continue;
      const T lo = v[i], hi = v[i | bit];
      v[i] = lo - hi;
      v[i | bit] = lo + hi;
    }
  }
}

// z = KE_modal c  (component-major c[3][8], z[3][8]; mode 0 carries no energy)
template <typename T>
__device__ __forceinline__ void modal_ke(const T (&c)[3][8], const Modal<T>& km, T (&z)[3][8]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    z[i][0] = (T)0;
#pragma unroll
    for (int q = 1; q < 8; ++q) z[i][q] = km.dg[(q >> i) & 1][__builtin_popcount((unsigned)q & ~(1u << i))] * c[i][q];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (i == j) continue;
      const int k = 3 - i - j;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int qi = (q >> i) & 1, qj = (q >> j) & 1;
        if (qi == qj) continue;
        const int qp = q ^ (1 << i) ^ (1 << j);
        const T w = qi ? km.lam4[(q >> k) & 1] : km.mu4[(q >> k) & 1];
        z[i][q] += w * c[j][qp];
      }
    }
  }
}

// ye = s * KE ue   (ue, ye: [local node a][component])
template <typename T>
__device__ __forceinline__ void elem_apply(const T (&ue)[8][3], T s, const Modal<T>& km,
                                           T (&ye)[8][3]) {
  T c[3][8], z[3][8];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int a = 0; a < 8; ++a) c[i][a] = ue[a][i];
    analysis8(c[i]);
#pragma unroll
    for (int q = 1; q < 8; ++q) c[i][q] *= s;
  }
  modal_ke(c, km, z);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    synthesis8(z[i]);
#pragma unroll
    for (int a = 0; a < 8; ++a) ye[a][i] = z[i][a];
  }
}

// le^T KE ue  (FP64 accumulation of the final dot)
template <typename T>
__device__ __forceinline__ double elem_bilinear(const T (&le)[8][3], const T (&ue)[8][3],
                                                const Modal<T>& km) {
  T cu[3][8], cl[3][8], z[3][8];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int a = 0; a < 8; ++a) { cu[i][a] = ue[a][i]; cl[i][a] = le[a][i]; }
    analysis8(cu[i]);
    analysis8(cl[i]);
  }
  modal_ke(cu, km, z);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int q = 1; q < 8; ++q) acc += (double)cl[i][q] * (double)z[i][q];
  }
  return acc;
}

}  // namespace fbto
