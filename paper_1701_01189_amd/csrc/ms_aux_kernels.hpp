// Kernels that are not templates (scan of H, fill, copy); included by the
// host translation unit only.
#pragma once

#include "ms_kernels.hpp"

namespace ms {

// ---------------------------------------------------------------------------
// Scan: exclusive prefix sum of every row of H in place (the second term of
// Eq. 2), and the row totals (bucket sizes).  The scan of the m totals (the
// first term of Eq. 2) is done by every post-scan workgroup on its own; the
// two together are the exclusive scan of the row-vectorised H (Section 4.3).
// One workgroup per bucket row.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;

__global__ void __launch_bounds__(kScanThreads)
scan_rows_kernel(uint32_t* __restrict__ H, uint32_t L0, uint32_t* __restrict__ totals) {
  constexpr int E = 8;
  __shared__ uint32_t tmp[kScanThreads / kWave];
  uint32_t* row = H + (size_t)blockIdx.x * L0;
  const uint32_t lane = lane_id(), wg = threadIdx.x / kWave;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < L0; base += kScanThreads * E) {
    uint32_t v[E], s = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      uint32_t i = base + threadIdx.x * E + e;
      v[e] = i < L0 ? row[i] : 0u;
      s += v[e];
    }
    uint32_t total;
    uint32_t pre = group_exclusive_scan<kScanThreads / kWave>(s, tmp, wg, lane, &total) + carry;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      uint32_t i = base + threadIdx.x * E + e;
      if (i < L0) row[i] = pre;
      pre += v[e];
    }
    carry += total;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Bucket starts of a bucket-ordered array: offsets[j] = first index whose
// bucket is >= j (n if none), for j in [0, m].  One lane per boundary runs a
// lower-bound binary search over the whole array: m + 1 searches of
// ceil(log2(n + 1)) probes each instead of a pass over all n elements, and
// the first probes of every search hit the same few lines, which stay in L2.
// Used after the two passes of a multisplit into more than 256 buckets.
template <int Kind>
__global__ void __launch_bounds__(256)
bucket_starts_kernel(const uint32_t* __restrict__ out, uint32_t n, uint32_t m, BucketParams bp,
                     uint32_t* __restrict__ offsets) {
  Bucket<Kind, 8> f(bp, nullptr);
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > m) return;
  // Invariant: every index below lo has a bucket < j, every index at or past
  // lo + len has a bucket >= j, and lo + len <= n, so each probe is in range.
  uint32_t lo = 0, len = n;
  while (len > 0) {
    const uint32_t half = len >> 1;
    if (f(out[lo + half]) < j) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  offsets[j] = lo;
}

// Fill n words with a value (used for empty inputs: offsets of zero).
__global__ void fill_u32_kernel(uint32_t* p, uint32_t n, uint32_t v) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Streaming copy, 16 bytes per lane where aligned.
__global__ void __launch_bounds__(256) copy_u32_kernel(uint32_t* __restrict__ dst,
                                                       const uint32_t* __restrict__ src,
                                                       size_t n) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  size_t n4 = n / 4;
  const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
  u32x4* d4 = reinterpret_cast<u32x4*>(dst);
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(s4 + i), d4 + i);
  for (size_t i = n4 * 4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace ms
