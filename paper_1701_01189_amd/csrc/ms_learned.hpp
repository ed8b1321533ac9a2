// Fit of the learned bucket identifier for range buckets (two-stage
// piecewise-linear model of the bucket as a function of the key; not in the
// paper, whose range buckets use a binary search over the splitters held in
// shared memory, Section 7.3).
//
// Root: the line that spreads the sample's key range [x_min, x_max] over the
// 256 leaves.  Leaves: least squares of the bucket centre (label + 1/2) on x
// over the samples the float root routes to the leaf; an empty leaf copies
// its nearest non-empty neighbour, left first.
//
// Every sample is read twice, whatever the number of leaves:
//   pass 1  per leaf: count, sum of x, sum of (2 label + 1);
//   pass 2  per leaf, around the leaf's rounded mean M = round(sum x / count):
//           sum of (x - M)^2 and sum of (x - M)(2 label + 1).
// x = (float)key is an integer (at most 2^32), so every sum is an exact
// integer: 64-bit where it cannot overflow for fewer than 2^32 samples, 128
// bits (two words, carry propagated by the adder) for the squares and cross
// products.  Integer addition is associative, so the result does not depend
// on the order in which workgroups and lanes add (LDS and global atomics),
// and the fit is deterministic.  The centred sums around M are the two-pass
// least-squares form: Sxx = S2 - S1^2 / n with |S1| <= n/2, so the
// subtraction loses nothing that matters.
#pragma once

#include "ms_device.hpp"

namespace ms {

constexpr int kFitThreads = 256;
constexpr int kFitBlocks = 256;      // range pass
constexpr int kFitSumBlocks = 128;   // summation passes
constexpr int kFitAccWords = 8;      // u64 words per leaf in the accumulator

// Accumulator words of one leaf.
enum FitAcc {
  kAccN = 0,      // samples routed to the leaf
  kAccSx = 1,     // sum x
  kAccSy = 2,     // sum (2 label + 1)
  kAccS2lo = 3,   // sum (x - M)^2, low word
  kAccS2hi = 4,   //                high word
  kAccT1lo = 5,   // sum (x - M)(2 label + 1), two's complement, low word
  kAccT1hi = 6,   //                                             high word
  kAccM = 7       // M, the leaf's rounded mean (written before pass 2)
};

struct FitParams {
  const uint32_t* sample;
  const uint32_t* labels;  // nullable: labels are then the upper bounds
  uint32_t ns;
  const uint32_t* splitters;
  uint32_t m;
  float* model;
  uint32_t* range;         // 2 * kFitBlocks: per-workgroup key min, max
  unsigned long long* acc; // kLeaves * kFitAccWords
};

// 128-bit add into two words (lo, hi) that other lanes add into as well:
// each adder propagates its own carry, so the pair is exact once all adds
// are done.  Works for LDS (workgroup scope) and global (agent scope)
// memory through the generic atomics.
template <int SCOPE>
__device__ __forceinline__ void add_u128(unsigned long long* lo, unsigned long long* hi,
                                         unsigned long long vlo, unsigned long long vhi) {
  const unsigned long long old = __hip_atomic_fetch_add(lo, vlo, __ATOMIC_RELAXED, SCOPE);
  const unsigned long long carry = (old + vlo < old) ? 1ull : 0ull;
  if (vhi + carry) __hip_atomic_fetch_add(hi, vhi + carry, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ void add_u64(unsigned long long* p, unsigned long long v) {
  if (v) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, SCOPE);
}

__device__ __forceinline__ uint32_t fit_label(const FitParams& p, const uint32_t* spl,
                                              uint32_t i, uint32_t k) {
  if (p.labels) return min(p.labels[i], p.m - 1);
  return lds_upper_bound<8>(spl, p.m, k);
}

// Per-workgroup minimum and maximum key (x = (float)key is non-decreasing in
// the key, so these give x_min and x_max).
__global__ void __launch_bounds__(kFitThreads) fit_range_kernel(FitParams p) {
  __shared__ uint32_t lo, hi;
  if (threadIdx.x == 0) {
    lo = 0xFFFFFFFFu;
    hi = 0u;
  }
  __syncthreads();
  uint32_t a = 0xFFFFFFFFu, b = 0u;
  for (uint32_t i = blockIdx.x * kFitThreads + threadIdx.x; i < p.ns; i += kFitBlocks * kFitThreads) {
    const uint32_t k = p.sample[i];
    a = min(a, k);
    b = max(b, k);
  }
  atomicMin(&lo, a);
  atomicMax(&hi, b);
  __syncthreads();
  if (threadIdx.x == 0) {
    p.range[2 * blockIdx.x] = lo;
    p.range[2 * blockIdx.x + 1] = hi;
  }
}

static_assert(kFitThreads == kFitBlocks, "the root kernel reads one range pair per thread");

// Root line from the range of x: x_min -> 0, x_max -> L (clamped to L-1 at
// evaluation).  Also clears the per-leaf accumulators.  One workgroup.
__global__ void __launch_bounds__(kFitThreads) fit_root_kernel(FitParams p) {
  __shared__ uint32_t lo, hi;
  if (threadIdx.x == 0) {
    lo = 0xFFFFFFFFu;
    hi = 0u;
  }
  __syncthreads();
  atomicMin(&lo, p.range[2 * threadIdx.x]);
  atomicMax(&hi, p.range[2 * threadIdx.x + 1]);
  for (uint32_t i = threadIdx.x; i < (uint32_t)(kLeaves * kFitAccWords); i += kFitThreads)
    p.acc[i] = 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double xmin = (double)(float)lo, xmax = (double)(float)hi;
    float a0 = 0.0f, b0 = 0.0f;
    if (xmax > xmin) {
      a0 = (float)((double)kLeaves / (xmax - xmin));
      b0 = (float)(-(double)a0 * xmin);
    }
    p.model[0] = a0;
    p.model[1] = b0;
  }
}

// One summation pass over the sample (PASS 1: count, sum x, sum y; PASS 2:
// centred squares and cross products).  Lanes add into per-leaf LDS
// accumulators; each workgroup then adds its non-empty leaves into the
// global ones.  The leaf comes from the float root exactly as at inference.
template <int PASS>
__global__ void __launch_bounds__(kFitThreads) fit_sum_kernel(FitParams p) {
  constexpr int SW = __HIP_MEMORY_SCOPE_WORKGROUP, SA = __HIP_MEMORY_SCOPE_AGENT;
  __shared__ uint32_t spl[kMaxBuckets];
  __shared__ unsigned long long s_acc[kLeaves * kFitAccWords];
  __shared__ unsigned long long s_mean[kLeaves];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kMaxBuckets; i += kFitThreads)
    spl[i] = (i + 1 < p.m && p.splitters) ? p.splitters[i] : 0xFFFFFFFFu;
  for (uint32_t i = threadIdx.x; i < (uint32_t)(kLeaves * kFitAccWords); i += kFitThreads)
    s_acc[i] = 0ull;
  if (PASS == 2)
    for (uint32_t l = threadIdx.x; l < (uint32_t)kLeaves; l += kFitThreads)
      s_mean[l] = p.acc[l * kFitAccWords + kAccM];
  __syncthreads();
  const float a0 = p.model[0], b0 = p.model[1];
  for (uint32_t i = blockIdx.x * kFitThreads + threadIdx.x; i < p.ns;
       i += kFitSumBlocks * kFitThreads) {
    const uint32_t k = p.sample[i];
    const float xf = (float)k;
    const uint32_t leaf = clamp_trunc(__builtin_fmaf(a0, xf, b0), (uint32_t)kLeaves);
    const unsigned long long x = (unsigned long long)xf;  // integer, <= 2^32
    const unsigned long long y = 2ull * fit_label(p, spl, i, k) + 1ull;
    unsigned long long* a = s_acc + leaf * kFitAccWords;
    if (PASS == 1) {
      add_u64<SW>(a + kAccN, 1ull);
      add_u64<SW>(a + kAccSx, x);
      add_u64<SW>(a + kAccSy, y);
    } else {
      const long long d = (long long)x - (long long)s_mean[leaf];  // |d| <= 2^32
      const unsigned __int128 sq = (unsigned __int128)((__int128)d * d);
      add_u128<SW>(a + kAccS2lo, a + kAccS2hi, (unsigned long long)sq,
                   (unsigned long long)(sq >> 64));
      const long long t = d * (long long)y;  // |t| < 2^42
      add_u128<SW>(a + kAccT1lo, a + kAccT1hi, (unsigned long long)t,
                   t < 0 ? ~0ull : 0ull);
    }
  }
  __syncthreads();
  for (uint32_t l = threadIdx.x; l < (uint32_t)kLeaves; l += kFitThreads) {
    const unsigned long long* a = s_acc + l * kFitAccWords;
    unsigned long long* g = p.acc + l * kFitAccWords;
    if (PASS == 1) {
      add_u64<SA>(g + kAccN, a[kAccN]);
      add_u64<SA>(g + kAccSx, a[kAccSx]);
      add_u64<SA>(g + kAccSy, a[kAccSy]);
    } else {
      add_u128<SA>(g + kAccS2lo, g + kAccS2hi, a[kAccS2lo], a[kAccS2hi]);
      add_u128<SA>(g + kAccT1lo, g + kAccT1hi, a[kAccT1lo], a[kAccT1hi]);
    }
  }
}

// Between the passes: every leaf's rounded mean M = floor((sum x + n/2) / n).
__global__ void __launch_bounds__(kFitThreads) fit_mean_kernel(FitParams p) {
  for (uint32_t l = threadIdx.x; l < (uint32_t)kLeaves; l += kFitThreads) {
    unsigned long long* g = p.acc + l * kFitAccWords;
    const unsigned long long n = g[kAccN];
    // sum x < 2^64 and n < 2^32: the rounding term cannot overflow in 128 bits
    g[kAccM] = n ? (unsigned long long)(((unsigned __int128)g[kAccSx] + n / 2) / n) : 0ull;
  }
}

// Leaf lines from the exact sums, then empty leaves copy their nearest
// non-empty neighbour (left first).  One workgroup, one thread per leaf.
__global__ void __launch_bounds__(kFitThreads) fit_finish_kernel(FitParams p) {
  __shared__ int have[kLeaves];
  __shared__ float ab[2 * kLeaves];
  for (uint32_t l = threadIdx.x; l < (uint32_t)kLeaves; l += kFitThreads) {
    const unsigned long long* g = p.acc + l * kFitAccWords;
    const unsigned long long n = g[kAccN];
    float a = 0.0f, b = 0.0f;
    if (n) {
      const unsigned long long M = g[kAccM];
      // S1 = sum (x - M) = sum x - n M, exactly (|S1| <= n/2)
      const __int128 s1 = (__int128)g[kAccSx] - (__int128)n * (__int128)M;
      const unsigned __int128 s2 = ((unsigned __int128)g[kAccS2hi] << 64) | g[kAccS2lo];
      const __int128 t1 = (__int128)(((unsigned __int128)g[kAccT1hi] << 64) | g[kAccT1lo]);
      const double dn = (double)n, ds1 = (double)s1, sy = (double)g[kAccSy];
      const double sxx = (double)s2 - ds1 * ds1 / dn;
      const double sxy = 0.5 * ((double)t1 - ds1 * sy / dn);  // y = (2 label + 1) / 2
      const double mx = (double)M + ds1 / dn, my = 0.5 * sy / dn;
      double slope = 0.0, icpt = my;
      if (sxx > 0) {
        slope = sxy / sxx;
        icpt = my - slope * mx;
      }
      a = (float)slope;
      b = (float)icpt;
    }
    have[l] = n ? 1 : 0;
    ab[2 * l] = a;
    ab[2 * l + 1] = b;
  }
  __syncthreads();
  for (uint32_t l = threadIdx.x; l < (uint32_t)kLeaves; l += kFitThreads) {
    int src = have[l] ? (int)l : -1;
    for (int j = (int)l - 1; src < 0 && j >= 0; --j)
      if (have[j]) src = j;
    for (int j = (int)l + 1; src < 0 && j < kLeaves; ++j)
      if (have[j]) src = j;
    p.model[2 + 2 * l] = src >= 0 ? ab[2 * src] : 0.0f;
    p.model[3 + 2 * l] = src >= 0 ? ab[2 * src + 1] : 0.0f;
  }
}

}  // namespace ms
