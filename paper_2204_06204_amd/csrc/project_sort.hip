// Projection onto X = {lo <= x <= hi, sum x <= vmax} by sorting (Sec. 4.2,
// Alg. 4 and its GPU form in Sec. 4.3: one radix sort and parallel scans).
//
// The multiplier lambda solves sum_e clamp(y_e - lambda, lo, hi) = vmax
// (Eq. piecewiseLinearEQ).  Its left-hand side phi(lambda) is piecewise
// linear with nodes y_e - lo and y_e - hi.  Both families are the values of
// y shifted by a constant, so one sort of y orders all 2E nodes.  With S
// the exclusive prefix sums of the sorted values, phi at any lambda is
//   lo * c_lo + hi * (E - c_hi) + S[c_hi] - S[c_lo] - lambda * (c_hi - c_lo),
//   c_lo = #{y_e <= lambda + lo},  c_hi = #{y_e < lambda + hi},
// which is the running RHS of Alg. 4 in closed form (the running SLOPE is
// c_lo - c_hi).  The largest node with phi >= vmax and the smallest with
// phi <= vmax bound the linear piece that holds the root, which is then
// solved exactly.  phi is monotone along each family, so a coarse pass over
// every 255th node finds the windows that hold these two nodes, and a fine
// pass evaluates the nodes of those windows.
//
// Kernels, in launch order:
//   k_radix_hist     per 2048-key tile, counts of the current 8-bit digit
//                    (on the top digit, equal digits of a wave are added
//                    up before the LDS atomic)
//                    (the first pass maps y to order-preserving unsigned
//                    keys as it reads it)
//   k_radix_scan     per digit, exclusive scan of the tile counts
//   k_radix_scatter  stable scatter of each tile (wave ballots rank the keys)
//                    (the three above run 4 times for FP32, 8 for FP64)
//   k_prefix_part    FP64 sum of each tile of sorted values
//   k_prefix_top     exclusive scan of the tile sums (one block)
//   k_prefix_down    S[i] for every i, S[E] = the total
//   k_bracket_coarse phi at every 255th node of each family, and phi(0)
//   k_bracket_lambda one block: phi at every node of the four windows that
//                    hold the crossing of vmax, then lambda
//   k_clamp          x = clamp(y - lambda, lo, hi)
#include "device.h"

namespace fbto {
namespace {

constexpr int kSortBlock = 256;  // four waves; every kernel here assumes it
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kRadix = 256;
constexpr int kScanBlock = 1024;  // the single-block scans over tile counts and tile sums
constexpr int kRadixBits = 8;
constexpr int kBracketBlocks = kSortBracketBlocks;
constexpr int kCoarseStride = 255;            // nodes between the coarse samples of a family
constexpr int kWindow = kCoarseStride + 1;     // nodes of a fine window
constexpr int kFineBlock = 4 * kWindow;        // one block: the four windows, a node per thread
static_assert(kFineBlock % 64 == 0 && kFineBlock <= 1024, "fine block");

template <typename T> struct KeyOf;
template <> struct KeyOf<float> { using type = uint32_t; };
template <> struct KeyOf<double> { using type = uint64_t; };

// IEEE values to unsigned keys whose unsigned order is the numeric order
// (negative values: all bits flipped; others: the sign bit set).
__device__ __forceinline__ uint32_t to_key(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint64_t to_key(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double from_key(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k ^ 0x80000000u) : ~k;
  return (double)__uint_as_float(u);
}
__device__ __forceinline__ double from_key(uint64_t k) {
  const uint64_t u = (k >> 63) ? (k ^ (1ull << 63)) : ~k;
  return __longlong_as_double((long long)u);
}

// Inclusive scans over the 64 lanes of a wave (shift-up steps, fixed order).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ double wave_scan_incl(double v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan over a block of NT threads (sh: NT / 64 entries); `total`
// receives the block's sum.  Every thread must call it (it synchronises
// twice).
template <int NT = kSortBlock, typename V>
__device__ __forceinline__ V block_scan_excl(V v, V* sh, V& total) {
  const int w = threadIdx.x >> 6;
  const V incl = wave_scan_incl(v);
  if (__lane_id() == 63) sh[w] = incl;
  __syncthreads();
  V off = V(0), tot = V(0);
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    if (k < w) off += sh[k];
    tot += sh[k];
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

// Key i of a pass: from y itself on the first pass (y != NULL), otherwise
// from the previous pass's output.
template <typename K, typename T>
__device__ __forceinline__ K load_key(const K* keys, const T* y, int64_t i) {
  return y ? to_key(y[i]) : keys[i];
}

// Lanes of the wave holding the same digit d as this lane (eight ballots,
// one per digit bit), among the lanes in `valid`.
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d, uint64_t valid) {
  uint64_t same = valid;
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    same &= bit ? m : ~m;
  }
  return same;
}

// Digit counts of one tile.  `aggregate` (the top digit, which takes few
// values here, so that one LDS atomic per key piles up on one bin): the
// lanes of a wave with the same digit add their count once, from the lowest
// of them.  The eight ballots this costs are slower than plain atomics on
// the other digits.
template <typename K, typename T>
__global__ void __launch_bounds__(kSortBlock)
    k_radix_hist(const K* keys, const T* y, int64_t n, int shift, int aggregate, uint32_t* hist, int ntiles) {
  __shared__ uint32_t h[kRadix];
  const int tid = threadIdx.x;
  const uint64_t earlier = (1ull << __lane_id()) - 1ull;
  h[tid] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + k * kSortBlock + tid;
    const bool valid = i < n;
    const uint32_t d = valid ? (uint32_t)(load_key(keys, y, i) >> shift) & (kRadix - 1) : 0u;
    if (aggregate) {
      const uint64_t same = same_digit_lanes(d, __ballot(valid));
      if (valid && (same & earlier) == 0ull) atomicAdd(&h[d], (uint32_t)__popcll(same));
    } else if (valid) {
      atomicAdd(&h[d], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// One block per digit: the tile counts of the digit become the number of
// keys with that digit in earlier tiles; tot[digit] the digit's total.
__global__ void __launch_bounds__(kScanBlock) k_radix_scan(uint32_t* hist, int ntiles, uint32_t* tot) {
  __shared__ uint32_t sh[kScanBlock / 64];
  uint32_t* row = hist + (int64_t)blockIdx.x * ntiles;
  uint32_t carry = 0u;
  for (int c = 0; c < ntiles; c += kScanBlock) {
    const int j = c + threadIdx.x;
    const uint32_t v = j < ntiles ? row[j] : 0u;
    uint32_t total;
    const uint32_t ex = block_scan_excl<kScanBlock>(v, sh, total);
    if (j < ntiles) row[j] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Stable scatter of one tile by the current digit.
//  1. Rank, wave by wave with no block barrier: wave w takes the kWaveKeys
//     consecutive keys from w * kWaveKeys, in kSortItems rounds of 64, so
//     wave, round and lane order are the key order.  In a round the lanes
//     holding the same digit are found with eight ballots (one per digit
//     bit).  A key's rank within its digit among its wave's keys is the
//     wave's running count of that digit plus the same-digit lanes before
//     it; the lowest of those lanes then advances the count.
//  2. Per digit, the counts of earlier waves are added (one barrier), and
//     the keys are placed in LDS in digit order (the tile's digit starts are
//     a scan of its digit counts).
//  3. LDS entry j goes to the digit's global start for this tile plus its
//     offset in the digit's run, so consecutive threads write consecutive
//     addresses within each run.
template <typename K, typename T>
__global__ void __launch_bounds__(kSortBlock)
    k_radix_scatter(const K* in, const T* y, K* out, int64_t n, int shift, const uint32_t* hist,
                    const uint32_t* tot, int ntiles) {
  constexpr int kWaves = kSortBlock / 64;
  constexpr int kWaveKeys = 64 * kSortItems;
  __shared__ K stage[kSortTile];
  __shared__ uint32_t wcnt[kWaves][kRadix];   // per-wave digit counts, then the counts of earlier waves
  __shared__ uint32_t tstart[kRadix];          // tile-local start of each digit
  __shared__ uint32_t gbase[kRadix];           // global position minus tile-local start (mod 2^32)
  __shared__ uint32_t sh[kWaves];
  const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) wcnt[q][tid] = 0u;
  __syncthreads();
  const uint64_t earlier = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * kWaveKeys + lane;
  K key[kSortItems];
  uint32_t rank[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + (int64_t)k * 64;
    const bool valid = i < n;
    key[k] = valid ? load_key(in, y, i) : (K)0;
    const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
    const uint64_t same = same_digit_lanes(d, __ballot(valid));
    const uint32_t before = (uint32_t)__popcll(same & earlier);
    const uint32_t r = wcnt[w][d] + before;
    rank[k] = r;
    // the lowest same-digit lane advances the wave's count; a wave's LDS
    // accesses complete in program order, so the next round reads it
    if (valid && before == 0u) wcnt[w][d] = r + (uint32_t)__popcll(same);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  uint32_t c = 0u;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    const uint32_t v = wcnt[q][tid];
    wcnt[q][tid] = c;  // keys of this digit in earlier waves
    c += v;
  }
  uint32_t total;
  const uint32_t ts = block_scan_excl(c, sh, total);
  const uint32_t ds = block_scan_excl(tot[tid], sh, total);
  tstart[tid] = ts;
  gbase[tid] = ds + hist[(int64_t)tid * ntiles + blockIdx.x] - ts;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    if (base + (int64_t)k * 64 < n) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
      const uint32_t j = tstart[d] + wcnt[w][d] + rank[k];
      if (j < (uint32_t)kSortTile) stage[j] = key[k];  // always true when the counts are consistent
    }
  }
  __syncthreads();
  const int64_t left = n - (int64_t)blockIdx.x * kSortTile;
  const int tile_n = left < kSortTile ? (int)left : kSortTile;
  for (int j = tid; j < tile_n; j += kSortBlock) {
    const K kk = stage[j];
    const uint32_t pos = gbase[(uint32_t)(kk >> shift) & (kRadix - 1)] + (uint32_t)j;
    if ((int64_t)pos < n) out[pos] = kk;  // always true when the counts are consistent
  }
}

// FP64 prefix sums of the sorted values, tile by tile in the striped order
// of the sort (round k of a tile: kSortBlock consecutive values).
template <typename K>
__global__ void __launch_bounds__(kSortBlock) k_prefix_part(const K* sk, int64_t n, double* part) {
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + (int64_t)k * kSortBlock + threadIdx.x;
    v[0] += i < n ? from_key(sk[i]) : 0.0;
  }
  block_reduce<1, 0u>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kScanBlock) k_prefix_top(double* part, int nb) {
  __shared__ double sh[kScanBlock / 64];
  double carry = 0.0;
  for (int c = 0; c < nb; c += kScanBlock) {
    const int j = c + threadIdx.x;
    const double v = j < nb ? part[j] : 0.0;
    double total;
    const double ex = block_scan_excl<kScanBlock>(v, sh, total);
    if (j < nb) part[j] = carry + ex;
    carry += total;
  }
}

template <typename K>
__global__ void __launch_bounds__(kSortBlock) k_prefix_down(const K* sk, int64_t n, const double* part, double* S) {
  __shared__ double sh[kSortBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  double carry = part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + (int64_t)k * kSortBlock + threadIdx.x;
    const double v = i < n ? from_key(sk[i]) : 0.0;
    double total;
    const double ex = block_scan_excl(v, sh, total);
    if (i < n) S[i] = carry + ex;
    if (i == n - 1) S[n] = carry + ex + v;
    carry += total;
  }
}

// phi(t) = sum_e clamp(y_e - t, lo, hi) from the sorted values and S.
template <typename K>
__device__ double phi_at(const K* sk, const double* S, int64_t n, double t, double lo, double hi) {
  const double a = t + lo, b = t + hi;
  int64_t l = 0, r = n;                // first index with y > a
  while (l < r) {
    const int64_t m = (l + r) >> 1;
    if (from_key(sk[m]) <= a) l = m + 1;
    else r = m;
  }
  const int64_t c_lo = l;
  r = n;                               // first index >= c_lo with y >= b
  while (l < r) {
    const int64_t m = (l + r) >> 1;
    if (from_key(sk[m]) < b) l = m + 1;
    else r = m;
  }
  const int64_t c_hi = l;
  return lo * (double)c_lo + hi * (double)(n - c_hi) + (S[c_hi] - S[c_lo]) - t * (double)(c_hi - c_lo);
}

// Node i of family f: y_i - hi (f = 0, where element i leaves hi) or
// y_i - lo (f = 1, where it reaches lo).  Along a family phi does not
// increase with i.
template <typename K>
__device__ __forceinline__ double node_t(const K* sk, int64_t i, int f, double lo, double hi) {
  const double yi = from_key(sk[i]);
  return f == 0 ? yi - hi : yi - lo;
}

// Coarse pass: phi at the samples i = j * kCoarseStride (j < ns) of both
// families.  Per block, the number of samples with phi > vmax and with
// phi >= vmax, family by family: since phi is monotone along a family,
// these counts locate the crossing to within one sample interval.  The
// thread after the last sample stores phi(0).
template <typename K>
__global__ void __launch_bounds__(kSortBlock)
    k_bracket_coarse(const K* sk, const double* S, int64_t n, double lo, double hi, double vmax, int64_t ns,
                     double* part, int nb, double* phi0) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // family 0: > and >=, family 1: > and >=
  for (int64_t g = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; g <= 2 * ns;
       g += (int64_t)gridDim.x * kSortBlock) {
    if (g == 2 * ns) {
      *phi0 = phi_at(sk, S, n, 0.0, lo, hi);
      continue;
    }
    const int f = (int)(g & 1);
    const double ph = phi_at(sk, S, n, node_t(sk, (g >> 1) * kCoarseStride, f, lo, hi), lo, hi);
    const double gt = ph > vmax ? 1.0 : 0.0, ge = ph >= vmax ? 1.0 : 0.0;
    if (f == 0) {
      v[0] += gt;
      v[1] += ge;
    } else {
      v[2] += gt;
      v[3] += ge;
    }
  }
  block_reduce<4, 0u>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) part[(int64_t)k * nb + blockIdx.x] = v[k];
  }
}

// Fine pass and lambda, in one block: four windows of kWindow nodes, a node
// per thread.  Window 2 q + f covers family f around its first sample with
// phi <= vmax (q = 0: the smallest node with phi <= vmax lies there) or its
// last sample with phi >= vmax (q = 1: the largest node with phi >= vmax).
// Over all four windows, the largest node with phi >= vmax and the
// smallest with phi <= vmax bound the linear piece of the root.  lambda is
// 0 when phi(0) <= vmax, else the root on that piece.
template <typename K>
__global__ void __launch_bounds__(kFineBlock)
    k_bracket_lambda(const K* sk, const double* S, int64_t n, double lo, double hi, double vmax,
                     const double* part, int nb, const double* phi0, double* lam_ws, double* lam_out) {
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kFineBlock) {
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] += part[(int64_t)k * nb + b];
  }
  block_reduce<4, 0u>(c);
  const int wdw = threadIdx.x / kWindow;
  const int f = wdw & 1, q = wdw >> 1;
  const int64_t cnt = (int64_t)(q == 0 ? (f == 0 ? c[0] : c[2]) : (f == 0 ? c[1] : c[3]));
  int64_t i0 = (cnt - 1) * kCoarseStride, i1 = cnt * kCoarseStride;
  if (i0 < 0) i0 = 0;
  if (i1 > n - 1) i1 = n - 1;
  const int64_t i = i0 + threadIdx.x % kWindow;
  const bool have = i <= i1;
  double t = 0.0, ph = 0.0;
  if (have) {
    t = node_t(sk, i, f, lo, hi);
    ph = phi_at(sk, S, n, t, lo, hi);
  }
  double v[2] = {have && ph >= vmax ? t : -INFINITY, have && ph <= vmax ? -t : -INFINITY};
  block_reduce<2, 0x3u>(v);
  // phi at the two extremes (equal nodes give equal phi)
  double p[2] = {have && ph >= vmax && t == v[0] ? ph : -INFINITY, have && ph <= vmax && -t == v[1] ? ph : -INFINITY};
  block_reduce<2, 0x3u>(p);
  if (threadIdx.x != 0) return;
  const double tl = v[0], fl = p[0], tu = -v[1], fu = p[1];
  double lam;
  if (!isfinite(S[n])) {
    lam = NAN;                                   // a non-finite y
  } else if (*phi0 <= vmax) {
    lam = 0.0;                                   // the clamped point is feasible
  } else if (!(tl > -INFINITY && tu < INFINITY)) {
    lam = NAN;                                   // no bracket: vmax < lo * E (checked on the host)
  } else {
    lam = fl > fu ? tl + (fl - vmax) * (tu - tl) / (fl - fu) : tl;
    lam = fmin(fmax(lam, tl), tu);
  }
  *lam_ws = lam;
  if (lam_out) *lam_out = lam;
}

// x = clamp(y - lambda, lo, hi); four independent elements per thread and
// iteration (the grid stride apart) keep more loads in flight.
template <typename T>
__global__ void __launch_bounds__(kSortBlock)
    k_clamp(const T* y, T* x, int64_t n, double lo, double hi, const double* lam_ws) {
  const double lam = *lam_ws;
  const int64_t stride = (int64_t)gridDim.x * kSortBlock;
  for (int64_t i = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; i < n; i += 4 * stride) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = i + u * stride < n ? y[i + u * stride] : (T)0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * stride < n) x[i + u * stride] = isnan(lam) ? (T)NAN : (T)fmin(fmax((double)v[u] - lam, lo), hi);
  }
}

}  // namespace

size_t sort_ws_layout(int64_t E, SortWs* W) {
  const int64_t ntiles = (E + kSortTile - 1) / kSortTile;
  const size_t sz[7] = {(size_t)E * 8, (size_t)E * 8, (size_t)(E + 1) * 8, (size_t)kRadix * ntiles * 4,
                        (size_t)kRadix * 4, (size_t)ntiles * 8, (size_t)(4 * kBracketBlocks + 16 + 2) * 8};
  size_t off[7], tot = 0;
  for (int i = 0; i < 7; ++i) {
    off[i] = tot;
    tot += (sz[i] + 255) & ~(size_t)255;
  }
  if (W && W->base) {
    char* p = (char*)W->base;
    W->keys[0] = p + off[0];
    W->keys[1] = p + off[1];
    W->S = (double*)(p + off[2]);
    W->hist = (uint32_t*)(p + off[3]);
    W->tot = (uint32_t*)(p + off[4]);
    W->part = (double*)(p + off[5]);
    W->brk = (double*)(p + off[6]);          // [4][kBracketBlocks] coarse counts, then [4][4] windows
    W->lam = W->brk + 4 * kBracketBlocks + 16;
  }
  return tot;
}

template <typename T>
hipError_t launch_project_sorted(fbto_grid_s* g, const T* y, T* x, double lo, double hi, double vmax,
                                 double* lam_out, hipStream_t st) {
  using K = typename KeyOf<T>::type;
  const SortWs& W = g->sort;
  const int64_t n = g->geo.E;
  const int ntiles = (int)((n + kSortTile - 1) / kSortTile);
  // the first pass reads y (src = NULL); later passes alternate between
  // the two key buffers
  K* src = nullptr;
  K* dst = (K*)W.keys[0];
  K* spare = (K*)W.keys[1];
  const int nv = vec_blocks(n);
  for (int shift = 0; shift < (int)(8 * sizeof(K)); shift += kRadixBits) {
    const T* yk = shift == 0 ? y : nullptr;
    const int top = shift + kRadixBits == (int)(8 * sizeof(K));
    hipLaunchKernelGGL((k_radix_hist<K, T>), dim3(ntiles), dim3(kSortBlock), 0, st, (const K*)src, yk, n, shift,
                       top, W.hist, ntiles);
    hipLaunchKernelGGL(k_radix_scan, dim3(kRadix), dim3(kScanBlock), 0, st, W.hist, ntiles, W.tot);
    hipLaunchKernelGGL((k_radix_scatter<K, T>), dim3(ntiles), dim3(kSortBlock), 0, st, (const K*)src, yk, dst, n,
                       shift, (const uint32_t*)W.hist, (const uint32_t*)W.tot, ntiles);
    K* nxt = src ? src : spare;
    src = dst;
    dst = nxt;
  }
  K* a = src;  // the sorted keys
  hipLaunchKernelGGL((k_prefix_part<K>), dim3(ntiles), dim3(kSortBlock), 0, st, (const K*)a, n, W.part);
  hipLaunchKernelGGL(k_prefix_top, dim3(1), dim3(kScanBlock), 0, st, W.part, ntiles);
  hipLaunchKernelGGL((k_prefix_down<K>), dim3(ntiles), dim3(kSortBlock), 0, st, (const K*)a, n,
                     (const double*)W.part, W.S);
  const int64_t ns = (n + kCoarseStride - 1) / kCoarseStride;  // samples per family
  const int64_t nbc64 = (2 * ns + 1 + kSortBlock - 1) / kSortBlock;
  const int nbc = (int)(nbc64 < kBracketBlocks ? nbc64 : kBracketBlocks);
  double* phi0 = W.lam + 1;
  hipLaunchKernelGGL((k_bracket_coarse<K>), dim3(nbc), dim3(kSortBlock), 0, st, (const K*)a, (const double*)W.S, n,
                     lo, hi, vmax, ns, W.brk, nbc, phi0);
  hipLaunchKernelGGL((k_bracket_lambda<K>), dim3(1), dim3(kFineBlock), 0, st, (const K*)a, (const double*)W.S, n,
                     lo, hi, vmax, (const double*)W.brk, nbc, (const double*)phi0, W.lam, lam_out);
  hipLaunchKernelGGL((k_clamp<T>), dim3(nv), dim3(kSortBlock), 0, st, y, x, n, lo, hi, (const double*)W.lam);
  return hipGetLastError();
}

template hipError_t launch_project_sorted<float>(fbto_grid_s*, const float*, float*, double, double, double,
                                                 double*, hipStream_t);
template hipError_t launch_project_sorted<double>(fbto_grid_s*, const double*, double*, double, double, double,
                                                  double*, hipStream_t);

}  // namespace fbto
