// Device building blocks for the gfx950 multisplit kernels: 64-lane ballots,
// the ballot-based histogram and local-offset solves, the bucket identifiers
// and small workgroup scans.
//
// Paper: Ashkiani et al., "GPU Multisplit: an extended study of a parallel
// algorithm".  Section 5.4 (ballot-based voting), Section 5.5.1 / Algorithm 2
// (warp histogram), Section 5.5.2 / Algorithm 3 (warp local offsets),
// Section 5.7 (more buckets than lanes), Section 6 (bucket identifiers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ms {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxBuckets = 256;   // m <= 256
constexpr int kLeaves = 256;       // learned model leaves
constexpr int kModelFloats = 2 + 2 * kLeaves;

enum BucketKind { kShiftMask = 0, kDiv = 1, kSplitters = 2, kLearned = 3 };

// ---------------------------------------------------------------------------
// wavefront primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` at lanes strictly below this lane.  This is
// the "mask away higher lanes, then population count" step of Algorithm 3,
// done by the hardware's masked bit count.
__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t x) {
  return (uint32_t)__builtin_popcountll(x);
}

// ~(b ^ sel): b where sel is all ones, ~b where sel is zero.
__device__ __forceinline__ uint64_t pick(uint64_t b, uint64_t sel) { return ~(b ^ sel); }

// Lanes whose (valid) element has the same bucket as this lane's element.
// Section 5.4: the vote of every lane is published one bit at a time with
// BITS = ceil(log2 m) ballots; Algorithm 3 keeps, per lane, the lanes whose
// vote agrees with its own vote on every bit.
template <int BITS>
__device__ __forceinline__ uint64_t match_bucket(uint32_t b, bool valid, uint64_t valid_mask) {
  uint64_t m = valid_mask;
#pragma unroll
  for (int k = 0; k < BITS; ++k) {
    uint32_t bit = (b >> k) & 1u;
    uint64_t bal = ballot(valid && bit);
    m &= pick(bal, (uint64_t)0 - (uint64_t)bit);
  }
  return m;
}

// Buckets owned per lane by the histogram solve: ceil(2^BITS / 64).
template <int BITS>
struct Owned {
  static constexpr int value = BITS <= 6 ? 1 : (1 << (BITS - 6));
};

// Algorithm 2 generalised to wave64 and m <= 256 (Section 5.7): lane l owns
// buckets l + 64 t, t < ceil(m/64).  For vote bits k < 6 the lane compares
// the ballot with its own lane bit (lane-dependent); for k >= 6 the owned
// bucket's bit is bit (k-6) of t, the same for all lanes, so that part of the
// mask is a uniform (scalar) value per t.  cnt[t] += count of bucket l+64t.
template <int BITS>
__device__ __forceinline__ void window_histogram(uint32_t b, bool valid, uint64_t valid_mask,
                                                 uint32_t lane,
                                                 uint32_t (&cnt)[Owned<BITS>::value]) {
  constexpr int MB = Owned<BITS>::value;
  uint64_t bal[BITS > 0 ? BITS : 1];
#pragma unroll
  for (int k = 0; k < BITS; ++k) bal[k] = ballot(valid && ((b >> k) & 1u));
  uint64_t low = valid_mask;
#pragma unroll
  for (int k = 0; k < (BITS < 6 ? BITS : 6); ++k)
    low &= pick(bal[k], (uint64_t)0 - (uint64_t)((lane >> k) & 1u));
#pragma unroll
  for (int t = 0; t < MB; ++t) {
    uint64_t s = ~0ull;
#pragma unroll
    for (int k = 6; k < BITS; ++k) s &= ((t >> (k - 6)) & 1) ? bal[k] : ~bal[k];
    cnt[t] += popc64(low & s);
  }
}

// ---------------------------------------------------------------------------
// scans
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, uint32_t lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= (uint32_t)d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_broadcast(uint32_t v, int src) {
  return __shfl(v, src, kWave);
}

// ---------------------------------------------------------------------------
// bucket identifiers (Section 6, "Bucket identification")
// ---------------------------------------------------------------------------
struct BucketParams {
  uint32_t m;
  uint32_t shift;     // SHIFT_MASK
  uint32_t mask;      // SHIFT_MASK
  uint32_t magic;     // DIV: Granlund-Montgomery multiplier
  uint32_t sh1, sh2;  // DIV: post shifts
  const uint32_t* splitters;
  const float* model;
  unsigned long long* mispredicts;
};

// Range-bucket lookup tables staged in LDS: splitters padded to a power of
// two with 0xFFFFFFFF, and the learned model.
struct BucketLds {
  uint32_t spl[kMaxBuckets];
  float model[kModelFloats];
};

template <int Kind, int BITS>
struct Bucket;

template <int BITS>
struct Bucket<kShiftMask, BITS> {
  uint32_t shift, mask;
  __device__ Bucket(const BucketParams& p, const BucketLds*) : shift(p.shift), mask(p.mask) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const { return (k >> shift) & mask; }
  __device__ __forceinline__ uint32_t misses() const { return 0; }
};

// floor(k / d) by a multiply-high and two shifts (Granlund and Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994, the
// unsigned N-bit algorithm): t = mulhi(magic, k); q = (t + ((k - t) >> sh1)) >> sh2.
template <int BITS>
struct Bucket<kDiv, BITS> {
  uint32_t magic, sh1, sh2;
  __device__ Bucket(const BucketParams& p, const BucketLds*) : magic(p.magic), sh1(p.sh1), sh2(p.sh2) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const {
    uint32_t t = __umulhi(magic, k);
    return (t + ((k - t) >> sh1)) >> sh2;
  }
  __device__ __forceinline__ uint32_t misses() const { return 0; }
};

// Upper bound over the splitters in LDS: the number of splitters <= k.  The
// table is padded to 2^STEPS - 1 entries with 0xFFFFFFFF (2^STEPS >= m), so a
// branch-free search of STEPS probes finds the count; only k = 0xFFFFFFFF can
// count padding, and the clamp to m - 1 removes it.
template <int STEPS>
__device__ __forceinline__ uint32_t lds_upper_bound(const uint32_t* spl, uint32_t m, uint32_t k) {
  uint32_t pos = 0;
#pragma unroll
  for (int s = STEPS - 1; s >= 0; --s) {
    const uint32_t step = 1u << s;
    pos += (spl[pos + step - 1] <= k) ? step : 0u;
  }
  return pos < m - 1 ? pos : m - 1;
}

template <int BITS>
struct Bucket<kSplitters, BITS> {
  const uint32_t* spl;
  uint32_t m;
  __device__ Bucket(const BucketParams& p, const BucketLds* l) : spl(l->spl), m(p.m) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const {
    return lds_upper_bound<BITS>(spl, m, k);
  }
  __device__ __forceinline__ uint32_t misses() const { return 0; }
};

// Learned identifier: x = (float)k; leaf = clamp(trunc(fma(a0, x, b0)));
// guess = clamp(trunc(fma(a_leaf, x, b_leaf)), 0, m-1); then an exact check
// s[guess-1] <= k < s[guess] (open ends at 0 and m-1), one step down or up,
// else the binary search.  The returned id always equals the upper bound.
__device__ __forceinline__ uint32_t clamp_trunc(float v, uint32_t hi) {
  if (v < 0.0f) return 0;
  if (v >= (float)hi) return hi - 1;
  return (uint32_t)v;
}

template <int BITS>
struct Bucket<kLearned, BITS> {
  const uint32_t* spl;
  const float* model;
  uint32_t m;
  mutable uint32_t miss;
  __device__ Bucket(const BucketParams& p, const BucketLds* l)
      : spl(l->spl), model(l->model), m(p.m), miss(0) {}
  __device__ __forceinline__ bool in_bucket(uint32_t g, uint32_t k) const {
    bool lo = (g == 0) || (spl[g - 1] <= k);
    bool hi = (g + 1 >= m) || (k < spl[g]);
    return lo && hi;
  }
  __device__ __forceinline__ uint32_t predict(uint32_t k) const {
    float x = (float)k;
    uint32_t leaf = clamp_trunc(__builtin_fmaf(model[0], x, model[1]), (uint32_t)kLeaves);
    return clamp_trunc(__builtin_fmaf(model[2 + 2 * leaf], x, model[3 + 2 * leaf]), m);
  }
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const {
    uint32_t g = predict(k);
    if (in_bucket(g, k)) return g;
    miss += 1;
    if (g > 0 && in_bucket(g - 1, k)) return g - 1;
    if (g + 1 < m && in_bucket(g + 1, k)) return g + 1;
    return lds_upper_bound<BITS>(spl, m, k);
  }
  __device__ __forceinline__ uint32_t misses() const { return miss; }
};

// Stage splitters (padded) and the learned model into LDS.
template <int Kind>
__device__ __forceinline__ void stage_bucket_tables(const BucketParams& p, BucketLds* l) {
  if (Kind == kSplitters || Kind == kLearned) {
    for (uint32_t i = threadIdx.x; i < (uint32_t)kMaxBuckets; i += blockDim.x)
      l->spl[i] = (i + 1 < p.m) ? p.splitters[i] : 0xFFFFFFFFu;
  }
  if (Kind == kLearned) {
    for (uint32_t i = threadIdx.x; i < (uint32_t)kModelFloats; i += blockDim.x)
      l->model[i] = p.model[i];
  }
}

// XCD-aware placement: workgroups are dispatched round-robin over the 8
// accelerator dies, each with its own L2.  Map workgroup i to a chunk so that
// the workgroups of one die get consecutive chunks; neighbouring chunks then
// share the cache lines at their output boundaries inside one L2.
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t bid, uint32_t grid) {
  const uint32_t X = 8;
  uint32_t x = bid % X, r = bid / X;
  uint32_t q = grid / X, rem = grid % X;
  return x * q + (x < rem ? x : rem) + r;
}

}  // namespace ms
