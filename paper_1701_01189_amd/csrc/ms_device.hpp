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

enum BucketKind { kShiftMask = 0, kDiv = 1, kSplitters = 2, kLearned = 3, kKeptIds = 4 };

// ---------------------------------------------------------------------------
// wavefront primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

// Index of this wavefront in its workgroup, as a wavefront-uniform value.
__device__ __forceinline__ uint32_t wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` at lanes strictly below this lane: Algorithm
// 3's count of same-bucket lanes below this one, done by the hardware's
// masked bit count.
__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t x) {
  return (uint32_t)__builtin_popcountll(x);
}

// m & ~(b ^ sel) in one gfx950 three-input bitwise op: keeps the bits of m
// where the ballot b agrees with the selector (sel all ones: b; zero: ~b).
// Truth table over (S0, S1, S2) = (0xF0, 0xCC, 0xAA): 0xF0 & ~(0xCC ^ 0xAA).
__device__ __forceinline__ uint32_t and_agree(uint32_t m, uint32_t b, uint32_t sel) {
  return __builtin_amdgcn_bitop3_b32(m, b, sel, 0x90);
}

// Bit k of b spread over a word: 0 or 0xFFFFFFFF (a signed bit-field extract).
__device__ __forceinline__ uint32_t bit_spread(uint32_t b, int k) {
  return (uint32_t)(((int32_t)(b << (31 - k))) >> 31);
}

// Lanes whose element has the same bucket as this lane's element, among the
// lanes of valid_mask.  Section 5.4: every lane publishes its vote one bit
// at a time with BITS = ceil(log2 m) ballots; Algorithm 3 keeps, per lane,
// the lanes that agree with its own vote on every bit.  Invalid lanes must
// carry bucket 0 (they then vote 0 on every bit and are removed by
// valid_mask).
template <int BITS>
__device__ __forceinline__ uint64_t match_bucket(uint32_t b, uint64_t valid_mask) {
  uint32_t lo = (uint32_t)valid_mask, hi = (uint32_t)(valid_mask >> 32);
#pragma unroll
  for (int k = 0; k < BITS; ++k) {
    uint32_t sel = bit_spread(b, k);
    // Opaque to the optimiser, so the ballot compares `sel` itself instead
    // of re-deriving the bit with an extra shift.
    asm("" : "+v"(sel));
    const uint64_t bal = ballot(sel != 0u);
    lo = and_agree(lo, (uint32_t)bal, sel);
    hi = and_agree(hi, (uint32_t)(bal >> 32), sel);
  }
  return ((uint64_t)hi << 32) | lo;
}

// Buckets owned per lane by the histogram solve: ceil(2^BITS / 64).
template <int BITS>
struct Owned {
  static constexpr int value = BITS <= 6 ? 1 : (1 << (BITS - 6));
};

// Per-lane selectors of Algorithm 2: bit k of the lane index, spread.
struct LaneSel {
  uint32_t s[6];
  __device__ explicit LaneSel(uint32_t lane) {
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = bit_spread(lane, k);
  }
};

// Algorithm 2 generalised to wave64 and m <= 256 (Section 5.7): lane l owns
// buckets l + 64 t, t < ceil(m/64).  For vote bits k < 6 the lane compares
// the ballot with its own lane bit (lane-dependent); for k >= 6 the owned
// bucket's bit is bit (k-6) of t, the same for all lanes, so that part of the
// mask is a uniform (scalar) value per t.  cnt[t] += count of bucket l+64t.
// Invalid lanes must carry bucket 0.
template <int BITS>
__device__ __forceinline__ void window_histogram(uint32_t b, uint64_t valid_mask,
                                                 const LaneSel& ls,
                                                 uint32_t (&cnt)[Owned<BITS>::value]) {
  constexpr int MB = Owned<BITS>::value;
  uint64_t bal[BITS > 0 ? BITS : 1];
#pragma unroll
  for (int k = 0; k < BITS; ++k) bal[k] = ballot(bit_spread(b, k) != 0u);
  uint32_t lo = (uint32_t)valid_mask, hi = (uint32_t)(valid_mask >> 32);
#pragma unroll
  for (int k = 0; k < (BITS < 6 ? BITS : 6); ++k) {
    lo = and_agree(lo, (uint32_t)bal[k], ls.s[k]);
    hi = and_agree(hi, (uint32_t)(bal[k] >> 32), ls.s[k]);
  }
#pragma unroll
  for (int t = 0; t < MB; ++t) {
    uint64_t s = ~0ull;
#pragma unroll
    for (int k = 6; k < BITS; ++k) s &= ((t >> (k - 6)) & 1) ? bal[k] : ~bal[k];
    cnt[t] += __builtin_popcount(lo & (uint32_t)s) + __builtin_popcount(hi & (uint32_t)(s >> 32));
  }
}

// LDS words shared by the lanes of one wavefront between ballot windows.
// Relaxed wavefront-scope atomics compile to plain ds_read/ds_write (a
// wavefront's LDS operations complete in order) while keeping the compiler
// from caching or forwarding values that another lane wrote.
__device__ __forceinline__ uint32_t lds_get(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void lds_put(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void wave_order() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// ---------------------------------------------------------------------------
// scans
// ---------------------------------------------------------------------------
// Inclusive scan over the 64 lanes with data-parallel primitives (DPP): four
// row shifts (1, 2, 4, 8) scan each row of 16 lanes; broadcasting lane 15
// into rows 1 and 3 and then lane 31 into rows 2 and 3 carries the row
// totals across.  A lane whose DPP source is outside its row, or whose row
// is masked off, receives the `old` operand, 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v) {
  return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, uint32_t /*lane*/) {
  v = dpp_add<0x111, 0xF>(v);  // row_shr:1
  v = dpp_add<0x112, 0xF>(v);  // row_shr:2
  v = dpp_add<0x114, 0xF>(v);  // row_shr:4
  v = dpp_add<0x118, 0xF>(v);  // row_shr:8
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
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

// Range-bucket lookup tables staged in LDS.  spl[] holds two zero words
// (splitter indices -2 and -1: every key is >= them), the m-1 splitters from
// index 2 on, then 0xFFFFFFFF padding up to a power of two; model[] is the
// learned model (2 root floats, then slope and intercept of each leaf).
constexpr int kSplPad = 2;
struct BucketLds {
  uint32_t spl[kSplPad + kMaxBuckets + 2];
  float model[kModelFloats];
};

template <int Kind, int BITS>
struct Bucket;

template <int BITS>
struct Bucket<kShiftMask, BITS> {
  static constexpr bool kCheap = true;  // recomputed from the key instead of stored
  uint32_t shift, mask;
  __device__ Bucket(const BucketParams& p, const BucketLds*) : shift(p.shift), mask(p.mask) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const { return (k >> shift) & mask; }
  __device__ __forceinline__ uint32_t misses() const { return 0; }
};

// floor(k / d) by a multiply-high and two shifts (Granlund and Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994, the
// unsigned N-bit algorithm): t = mulhi(magic, k); q = (t + ((k - t) >> sh1)) >> sh2.
// `mask` keeps the low digit of the quotient when more than 256 buckets are
// split in two passes (all ones otherwise).
template <int BITS>
struct Bucket<kDiv, BITS> {
  static constexpr bool kCheap = true;
  uint32_t magic, sh1, sh2, mask;
  __device__ Bucket(const BucketParams& p, const BucketLds*)
      : magic(p.magic), sh1(p.sh1), sh2(p.sh2), mask(p.mask) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const {
    uint32_t t = __umulhi(magic, k);
    return ((t + ((k - t) >> sh1)) >> sh2) & mask;
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
  static constexpr bool kCheap = false;  // an LDS search: computed once, then stored
  const uint32_t* spl;
  uint32_t m;
  __device__ Bucket(const BucketParams& p, const BucketLds* l) : spl(l->spl + kSplPad), m(p.m) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const {
    return lds_upper_bound<BITS>(spl, m, k);
  }
  __device__ __forceinline__ uint32_t misses() const { return 0; }
};

// Learned identifier (not in the paper; binary search is the paper's way):
//   x = (float)k;  leaf = trunc(clamp(fma(a0, x, b0), 0, 255));
//   g = trunc(clamp(fma(a_leaf, x, b_leaf), 0, m-1))
// then one branch-free step: down if k < s[g-1], up if k >= s[g] (s[-1] =
// -inf, s[m-1] = +inf).  The stepped bucket is checked against its other
// neighbouring splitter; only if that fails (the model was off by more than
// one bucket) does the lane fall back to the binary search.  The result is
// always the upper bound.  clamp-then-truncate equals the oracle's
// "< 0 -> 0, >= hi -> hi-1, else truncate" for finite values.
__device__ __forceinline__ uint32_t clamp_trunc(float v, uint32_t hi) {
  return (uint32_t)__builtin_amdgcn_fmed3f(v, 0.0f, (float)(hi - 1));
}

template <int BITS>
struct Bucket<kLearned, BITS> {
  static constexpr bool kCheap = false;
  const uint32_t* tbl;  // spl with the two zero words in front
  const float* model;
  uint32_t m;
  mutable uint32_t miss;
  __device__ Bucket(const BucketParams& p, const BucketLds* l)
      : tbl(l->spl), model(l->model), m(p.m), miss(0) {}
  __device__ __forceinline__ uint32_t predict(uint32_t k) const {
    const float x = (float)k;
    const uint32_t leaf = clamp_trunc(__builtin_fmaf(model[0], x, model[1]), (uint32_t)kLeaves);
    const float2 ab = reinterpret_cast<const float2*>(model + 2)[leaf];
    return clamp_trunc(__builtin_fmaf(ab.x, x, ab.y), m);
  }
  __device__ __forceinline__ uint32_t operator()(uint32_t k) const {
    const uint32_t g = predict(k);
    const uint32_t sm2 = tbl[g], sm1 = tbl[g + 1], s0 = tbl[g + 2], sp1 = tbl[g + 3];
    const bool down = k < sm1;                 // s[g-1] > k
    const bool up = (g + 1 < m) && k >= s0;    // s[g] <= k
    uint32_t c = g - (down ? 1u : 0u) + (up ? 1u : 0u);
    const bool bad = (down && k < sm2) || (up && g + 2 < m && k >= sp1);
    if (bad) c = lds_upper_bound<BITS>(tbl + kSplPad, m, k);
    miss += (c != g) ? 1u : 0u;
    return c;
  }
  __device__ __forceinline__ uint32_t misses() const { return miss; }
};

// Post-scan of table-search buckets whose ids the pre-scan kept: every id
// comes from the kept bytes, so the post-scan carries no table, model or
// search (fewer registers, no LDS tables).  The key is never looked at.
template <int BITS>
struct Bucket<kKeptIds, BITS> {
  static constexpr bool kCheap = false;
  __device__ Bucket(const BucketParams&, const BucketLds*) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t) const { return 0u; }
  __device__ __forceinline__ uint32_t misses() const { return 0; }
};

// Stage splitters (padded) and the learned model into LDS.
template <int Kind>
__device__ __forceinline__ void stage_bucket_tables(const BucketParams& p, BucketLds* l) {
  if (Kind == kSplitters || Kind == kLearned) {
    for (uint32_t i = threadIdx.x; i < (uint32_t)(kSplPad + kMaxBuckets + 2); i += blockDim.x) {
      uint32_t v;
      if (i < (uint32_t)kSplPad) v = 0u;
      else v = (i - kSplPad + 1 < p.m) ? p.splitters[i - kSplPad] : 0xFFFFFFFFu;
      l->spl[i] = v;
    }
  }
  if (Kind == kLearned) {
    for (uint32_t i = threadIdx.x; i < (uint32_t)kModelFloats; i += blockDim.x)
      l->model[i] = p.model[i];
  }
}

}  // namespace ms
