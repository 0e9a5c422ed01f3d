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
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Grid-wide reduction through per-block partials and a "last block
// finishes" counter.  Every block calls it exactly once with its threads'
// values; the function returns true in all threads of the block that
// arrived last, with tot[] = reduction over all blocks in block order
// (independent of arrival order).  `nblocks` is the number of blocks that
// call it; the counter is reset for the next launch.
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ bool grid_reduce(double (&v)[NV], int block, int nblocks,
                                            double* partials, unsigned* counter) {
  __shared__ int am_last;
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  block_reduce<NV, MAXMASK>(v);
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) st_agent(&partials[(int64_t)block * NV + i], v[i]);
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    am_last = (prev == (unsigned)(nblocks - 1));
  }
  __syncthreads();
  if (!am_last) return false;
  __threadfence();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const bool is_max = (MAXMASK >> i) & 1u;
    double acc = is_max ? -INFINITY : 0.0;
    for (int b = tid; b < nblocks; b += nthr) {
      const double x = ld_agent(&partials[(int64_t)b * NV + i]);
      acc = is_max ? fmax(acc, x) : acc + x;
    }
    v[i] = acc;
  }
  block_reduce<NV, MAXMASK>(v);
  if (tid == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// --------------------------------------------------------------------------
// SIMP scaling s = rho_min + (1 - rho_min) rho^p and ds/drho.
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T simp_s(T rho, const Simp& sp) {
  const T rm = (T)sp.rho_min;
  const T pw = sp.cubic ? rho * rho * rho : (T)pow((double)rho, sp.penal);
  return rm + ((T)1 - rm) * pw;
}
template <typename T>
__device__ __forceinline__ T simp_ds(T rho, const Simp& sp) {
  const T rm = (T)sp.rho_min;
  const T pw = sp.cubic ? rho * rho : (T)pow((double)rho, sp.penal - 1.0);
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
    for (int q = 1; q < 8; ++q) z[i][q] = km.dg[i][q] * c[i][q];
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
