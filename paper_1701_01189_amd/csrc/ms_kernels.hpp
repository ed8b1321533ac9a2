// gfx950 kernels of the three-stage multisplit (Section 4.6: pre-scan, scan,
// post-scan) with wavefront-level (WMS), block-level (BMS) or no (DMS)
// reordering (Sections 5.3 and 5.6).
//
// Vocabulary (Section 5.3): a *window* is 64 consecutive elements ranked by
// one wavefront with ballots; a *tile* is the set of windows reordered
// together in LDS (one wavefront's NW windows for WMS, all wavefronts' for
// BMS); a *chunk* is a run of consecutive tiles owned by one group (a
// wavefront for WMS/DMS, a workgroup for BMS) -- one column of H.
#pragma once

#include <type_traits>

#include "ms_device.hpp"

namespace ms {

enum Mode { kBlock = 1, kWaveMode = 2, kDirect = 3 };

struct Plan {
  uint32_t n;         // elements
  uint32_t m;         // buckets
  uint32_t L0;        // chunks = columns of H
  uint32_t chunk;     // elements per chunk (multiple of the tile size)
  uint32_t tile;      // elements per tile
};

// ---------------------------------------------------------------------------
// group barriers: a whole workgroup (BMS) or a single wavefront (WMS/DMS)
// ---------------------------------------------------------------------------
template <int WPG>
__device__ __forceinline__ void group_sync() {
  if (WPG > 1) {
    __syncthreads();
  } else {
    // one wavefront: its LDS operations complete in order; only the
    // compiler has to be kept from moving accesses across this point.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Exclusive scan of one value per thread over a group of WPG wavefronts.
// `tmp` holds WPG words of LDS private to the group.  Returns the exclusive
// prefix; *total receives the group total.
template <int WPG>
__device__ __forceinline__ uint32_t group_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t wg,
                                                         uint32_t lane, uint32_t* total) {
  uint32_t inc = wave_inclusive_scan(v, lane);
  if (WPG == 1) {
    *total = wave_broadcast(inc, kWave - 1);
    return inc - v;
  }
  if (lane == kWave - 1) tmp[wg] = inc;
  group_sync<WPG>();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < WPG; ++w) {
    uint32_t t = tmp[w];
    before += (w < (int)wg) ? t : 0u;
    all += t;
  }
  group_sync<WPG>();  // tmp may be reused right after
  *total = all;
  return before + inc - v;
}

// ---------------------------------------------------------------------------
// Pre-scan: one column of H per chunk (Algorithm 1's pre-scan).  WPG
// wavefronts share a chunk; a workgroup of WPB wavefronts serves WPB / WPG
// chunks.  Order inside a chunk does not matter for a histogram, so
// wavefronts stride over its windows.  H is bucket-major: H[b * L0 + c].
//
// Two ways to count, same result:
//  kHistBallot  the window histogram of Algorithm 2 (ballots, counts in
//               registers; about 4 VALU per vote bit per window);
//  kHistLanes   one LDS counter per (bucket, lane) shared by the workgroup's
//               wavefronts: every element adds 1 to its lane's counter of its
//               bucket with an LDS atomic.  The 64 lanes of an instruction
//               always hit 64 distinct counters in 64 distinct banks, so
//               neither skew nor m changes its cost (one address VALU per
//               window besides the bucket id).
//               Workgroup-shared chunks only (WPG > 1).
// ---------------------------------------------------------------------------
enum Hist { kHistBallot = 0, kHistLanes = 1 };

template <int Kind, int BITS, int WPB, int WPG, int HIST>
__global__ void __launch_bounds__(WPB* kWave)
prescan_kernel(const uint32_t* __restrict__ keys, Plan plan, BucketParams bp,
               uint32_t* __restrict__ H) {
  static_assert(HIST == kHistBallot || WPG > 1, "lane counters need a shared chunk");
  constexpr int GPB = WPB / WPG;
  constexpr int MB = Owned<BITS>::value;
  constexpr int U = 16;  // windows in flight per wavefront
  constexpr bool LANES = (HIST == kHistLanes);
  constexpr int NB = 1 << BITS;  // counter rows of kHistLanes
  __shared__ BucketLds tables;
  __shared__ uint32_t s_hist[(WPG > 1 && !LANES) ? WPB * kMaxBuckets : 1];
  __shared__ uint32_t s_lane[LANES ? NB * kWave : 1];  // [bucket][lane]
  if (LANES)
    for (uint32_t i = threadIdx.x; i < NB * kWave; i += WPB * kWave) s_lane[i] = 0u;
  stage_bucket_tables<Kind>(bp, &tables);
  __syncthreads();
  auto lane_count = [&](uint32_t b, uint32_t lane) {
    __hip_atomic_fetch_add(&s_lane[b * kWave + lane], 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  Bucket<Kind, BITS> bf(bp, &tables);

  const uint32_t lane = lane_id();
  const LaneSel ls(lane);
  const uint32_t w = wave_id();
  const uint32_t g = w / WPG, wg = w % WPG;
  const uint32_t c = blockIdx.x * GPB + g;
  // The chunk's count of bucket b goes to its column of H.
  auto emit = [&](uint32_t b, uint32_t v) { H[b * plan.L0 + c] = v; };
  uint32_t cnt[MB];
#pragma unroll
  for (int t = 0; t < MB; ++t) cnt[t] = 0;

  if (c < plan.L0) {
    const uint32_t c0 = c * plan.chunk;
    const uint32_t len = min(plan.chunk, plan.n - c0);
    constexpr uint32_t BATCH = U * kWave;
    const uint32_t full = len / BATCH;       // complete batches of U windows
    const uint32_t* base = keys + c0 + lane;
    // Complete batches, software pipelined: the bucket ids of a batch are
    // computed first (their table lookups overlap), then the next batch's
    // loads are issued into the freed registers while the histogram solve
    // of this batch runs.
    uint32_t gi = wg;
    uint32_t k[U];
    if (gi < full) {
#pragma unroll
      for (int u = 0; u < U; ++u) k[u] = base[gi * BATCH + u * kWave];
    }
    while (gi < full) {
      uint32_t b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) b[u] = bf(k[u]);
      const uint32_t next = gi + WPG;
      if (next < full) {
#pragma unroll
        for (int u = 0; u < U; ++u) k[u] = base[next * BATCH + u * kWave];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (LANES) {
          lane_count(b[u], lane);
        } else {
          window_histogram<BITS>(b[u], ~0ull, ls, cnt);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      gi = next;
    }
    // The incomplete last batch, if any, belongs to one wavefront.
    const uint32_t rem = len - full * BATCH;
    if (rem > 0 && wg == full % WPG) {
      const uint32_t* p = base + full * BATCH;
      for (int u = 0; u < U; ++u) {
        const bool valid = (uint32_t)(u * kWave) + lane < rem;
        const uint32_t b = valid ? bf(p[u * kWave]) : 0u;
        if (LANES) {
          if (valid) lane_count(b, lane);
        } else {
          window_histogram<BITS>(b, ballot(valid), ls, cnt);
        }
      }
    }
  }
  if (WPG == 1) {
    if (c < plan.L0) {
#pragma unroll
      for (int t = 0; t < MB; ++t) {
        uint32_t b = lane + kWave * t;
        if (b < plan.m) emit(b, cnt[t]);
      }
    }
  } else if (LANES) {
    // column total of bucket b = sum of its 64 lane counters
    __syncthreads();
    if (c < plan.L0) {
      for (uint32_t b = w; b < plan.m; b += WPB) {
        const uint32_t s = wave_inclusive_scan(s_lane[b * kWave + lane], lane);
        if (lane == kWave - 1) emit(b, s);
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < MB; ++t) {
      uint32_t b = lane + kWave * t;
      if (b < plan.m) s_hist[w * kMaxBuckets + b] = cnt[t];
    }
    __syncthreads();
    if (c < plan.L0) {
      for (uint32_t b = threadIdx.x; b < plan.m; b += WPB * kWave) {
        uint32_t s = 0;
#pragma unroll
        for (int ww = 0; ww < WPB; ++ww) s += s_hist[ww * kMaxBuckets + b];
        emit(b, s);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// One tile of the post-scan (steps 2-5 below) for a group of WPG wavefronts
// whose keys (and values) are already in registers k, v: element (wave wg,
// window j, lane) of the tile is k[j] of that lane.  run[b] holds the output
// position of the tile's first bucket-b element and is advanced past the
// tile's bucket-b elements.  `after_stage` runs once k, v are no longer
// needed (used to issue the next tile's loads early).
// ---------------------------------------------------------------------------
template <bool KV>
struct TileCtx {
  uint32_t* s_k;       // LDS reorder buffer: keys
  uint32_t* s_v;       // LDS reorder buffer: values
  uint8_t* s_b;        // LDS reorder buffer: bucket ids
  uint32_t* my_cnt;    // this wavefront's counters [bucket]
  uint32_t* grp_cnt;   // the group's counters [wave][bucket], stride CNT_STRIDE
  uint32_t* run;       // [bucket] output position of the next element
  uint32_t* delta;     // [bucket] scratch: output position minus LDS slot
  uint32_t* tmp;       // WPG words for the group scan
  uint32_t* keys_out;
  uint32_t* vals_out;
  uint32_t m, tcount, wg, lane, tid_g;
};

constexpr int kCntStride = kMaxBuckets + 1;

// The post-scan visits a chunk's tiles last to first.  The pre-scan swept
// every chunk first to last, so the last lines it read -- the ends of the
// chunks -- are the ones still in the memory-side cache when the post-scan
// starts; beginning there re-reads them from the cache instead of HBM.
// Each tile then takes its bucket runs from the top of what is left of the
// chunk's bucket ranges, which places every element exactly where the
// forward order would (the tile's local order is unchanged).
constexpr bool kReverseTiles = true;

template <int BITS, bool KV, int WPG, int NW, bool FULL, class BF, class AfterStage,
          bool REV = false>
__device__ __forceinline__ void tile_rank_reorder_write(const BF& bf, uint32_t (&k)[NW],
                                                        uint32_t (&v)[NW], const TileCtx<KV>& c,
                                                        AfterStage after_stage) {
  const uint32_t m = c.m, tcount = c.tcount, lane = c.lane, wg = c.wg, tid_g = c.tid_g;
  const uint32_t wbase = wg * NW * kWave;
  for (uint32_t b = lane; b < m; b += kWave) lds_put(c.my_cnt + b, 0u);
  uint32_t bk[NW], lr[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const bool valid = FULL || wbase + (uint32_t)(j * kWave) + lane < tcount;
    bk[j] = valid ? bf(k[j]) : 0u;
  }
  wave_order();
  // ranking: Algorithm 3 per window + per-wavefront running counts.  The
  // next window's count is read right after this window's store (a
  // wavefront's LDS operations complete in order), so the read's latency
  // overlaps the next window's ballots instead of stalling after them.
  uint32_t before = lds_get(c.my_cnt + bk[0]);
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const bool valid = FULL || wbase + (uint32_t)(j * kWave) + lane < tcount;
    const uint64_t mm = match_bucket<BITS>(bk[j], FULL ? ~0ull : ballot(valid));
    const uint32_t r = count_below(mm), cnt = popc64(mm);
    lr[j] = before + r;
    // With values (more registers live), materialise the rank now: otherwise
    // the compiler sinks it past the barriers and keeps both halves of every
    // window's match mask alive instead (measured: 2^25 pairs, m = 32,
    // post-scan 120 -> 110 us; key-only runs faster without it).
    if (KV) asm("" : "+v"(lr[j]));
    // Every lane of a bucket read the same `before` and holds the same
    // count, so all of them store the same new value (no branch).  An
    // invalid lane carries bucket 0 and counts the valid bucket-0 lanes, so
    // it stores that same value too.
    lds_put(c.my_cnt + bk[j], before + cnt);
    wave_order();
    if (j + 1 < NW) before = lds_get(c.my_cnt + bk[j + 1]);
  }
  group_sync<WPG>();
  // exclusive scan of the bucket-major table: entry e = b*WPG + wave
  {
    const uint32_t E = m * WPG;
    const uint32_t ept = (E + WPG * kWave - 1) / (WPG * kWave);
    const uint32_t e0 = tid_g * ept;
    uint32_t vals[4];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t e = e0 + i;
      vals[i] = ((uint32_t)i < ept && e < E) ? c.grp_cnt[(e % WPG) * kCntStride + e / WPG] : 0u;
      s += vals[i];
    }
    uint32_t total;
    uint32_t pre = group_exclusive_scan<WPG>(s, c.tmp, wg, lane, &total);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t e = e0 + i;
      if ((uint32_t)i < ept && e < E) c.grp_cnt[(e % WPG) * kCntStride + e / WPG] = pre;
      pre += vals[i];
    }
  }
  group_sync<WPG>();
  // tile bucket starts -> output delta; advance the running bases
  for (uint32_t b = tid_g; b < m; b += WPG * kWave) {
    const uint32_t st = c.grp_cnt[b];
    const uint32_t nx = (b + 1 < m) ? c.grp_cnt[b + 1] : tcount;
    if (REV) {  // tiles visited last to first: run[b] is the end of what is left
      c.run[b] -= nx - st;
      c.delta[b] = c.run[b] - st;
    } else {
      c.delta[b] = c.run[b] - st;
      c.run[b] += nx - st;
    }
  }
  // local reorder: slot = tile base of (bucket, wavefront) + rank
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const bool valid = FULL || wbase + (uint32_t)(j * kWave) + lane < tcount;
    if (valid) {
      const uint32_t slot = c.my_cnt[bk[j]] + lr[j];
      c.s_k[slot] = k[j];
      if (KV) c.s_v[slot] = v[j];
      c.s_b[slot] = (uint8_t)bk[j];
    }
  }
  group_sync<WPG>();
  after_stage();
  // coalesced write-back: consecutive slots of a bucket are consecutive
  // output positions
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const uint32_t q = j * (WPG * kWave) + tid_g;
    if (FULL || q < tcount) {
      const uint32_t b = c.s_b[q];
      const uint32_t o = c.delta[b] + q;
      c.keys_out[o] = c.s_k[q];
      if (KV) c.vals_out[o] = c.s_v[q];
    }
  }
  group_sync<WPG>();
}

// ---------------------------------------------------------------------------
// Post-scan (Algorithm 1's post-scan, Sections 5.5.3-5.6).
//
// For every tile of the group's chunk:
//  1. each wavefront loads NW windows, element (wave wg, window j, lane l) at
//     tile_base + (wg*NW + j)*64 + l -- so (wg, j, l) is input order;
//  2. per window: match mask of the lane's bucket (Algorithm 3), rank among
//     lower lanes, and a per-wavefront running count per bucket kept in LDS
//     (every lane of a bucket stores the same new count): the first and
//     second terms of Eq. (4);
//  3. one exclusive scan over the bucket-major table [bucket][wavefront] of
//     those counts gives, for wavefront wg and bucket b, the number of tile
//     elements in buckets < b plus those of bucket b in earlier wavefronts --
//     the tile-local destination base (third term of Eq. 4 plus the tile
//     histogram scan of Section 5.6.2);
//  4. write the element into its slot of the reorder buffer (a stable local
//     multisplit of the tile, Section 4.7);
//  5. read the buffer linearly; slot q of bucket b goes to
//     G[b][chunk] + (elements of b in earlier tiles) + (q - tile start of b).
// Mode kDirect skips 3-5 and writes from registers (DMS).
// ---------------------------------------------------------------------------
template <int Kind, int BITS, bool KV, int WPB, int NW, int MODE>
__global__ void __launch_bounds__(WPB* kWave)
postscan_kernel(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
                uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                const uint32_t* __restrict__ G, const uint32_t* __restrict__ totals,
                uint32_t* __restrict__ offsets, Plan plan, BucketParams bp) {
  constexpr int WPG = (MODE == kBlock) ? WPB : 1;
  constexpr int GPB = WPB / WPG;
  constexpr int T = WPG * NW * kWave;
  constexpr bool REORDER = (MODE != kDirect);
  constexpr int CNT_STRIDE = kCntStride;

  __shared__ BucketLds tables;
  __shared__ uint32_t s_cnt[WPB * CNT_STRIDE];           // per wavefront counts
  __shared__ uint32_t s_run[GPB * kMaxBuckets];          // running output base
  __shared__ uint32_t s_delta[REORDER ? GPB * kMaxBuckets : 1];
  __shared__ uint32_t s_keys[REORDER ? GPB * T : 1];
  __shared__ uint32_t s_vals[(REORDER && KV) ? GPB * T : 1];
  __shared__ uint8_t s_bk[REORDER ? GPB * T : 1];
  __shared__ uint32_t s_tmp[WPB];

  const uint32_t lane = lane_id();
  const uint32_t w = wave_id();
  const uint32_t g = w / WPG, wg = w % WPG;
  const uint32_t tid_g = wg * kWave + lane;
  const uint32_t m = plan.m;

  stage_bucket_tables<Kind>(bp, &tables);

  // Bucket bases: exclusive scan of the bucket totals (first term of Eq. 2),
  // computed by every workgroup.  m <= 256 <= threads per workgroup.
  {
    uint32_t v = threadIdx.x < m ? totals[threadIdx.x] : 0u;
    uint32_t total;
    uint32_t pre = group_exclusive_scan<WPB>(v, s_tmp, w, lane, &total);
    __syncthreads();
    if (threadIdx.x < m) {
      s_cnt[threadIdx.x] = pre;  // staged bucket base
      if (blockIdx.x == 0) offsets[threadIdx.x] = pre;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[m] = plan.n;
    __syncthreads();
    // Running output position of each bucket in the group's chunk: its
    // start, or with tiles visited last to first its end (the next chunk's
    // start, or the bucket's end for the last chunk).
    for (uint32_t i = threadIdx.x; i < GPB * m; i += WPB * kWave) {
      uint32_t gg = i / m, b = i % m;
      uint32_t cc = blockIdx.x * GPB + gg;
      uint32_t r = 0;
      if (cc < plan.L0) {
        if (!kReverseTiles || MODE == kDirect)
          r = s_cnt[b] + G[b * plan.L0 + cc];
        else
          r = s_cnt[b] + (cc + 1 < plan.L0 ? G[b * plan.L0 + cc + 1] : totals[b]);
      }
      s_run[gg * kMaxBuckets + b] = r;
    }
    __syncthreads();
  }

  Bucket<Kind, BITS> bf(bp, &tables);
  const uint32_t c = blockIdx.x * GPB + g;
  if (c >= plan.L0) return;  // only whole idle groups leave (never a BMS group)
  const uint32_t c0 = c * plan.chunk;
  const uint32_t len = min(plan.chunk, plan.n - c0);
  uint32_t* my_cnt = s_cnt + w * CNT_STRIDE;
  uint32_t* run = s_run + g * kMaxBuckets;

  if (MODE == kDirect) {
    // DMS: counters are the running output positions of this wavefront.
    for (uint32_t b = lane; b < m; b += kWave) lds_put(my_cnt + b, run[b]);
    wave_order();
    const uint32_t steps = (uint32_t)(((uint64_t)len + NW * kWave - 1) / (NW * kWave));
    for (uint32_t si = 0; si < steps; ++si) {
      const uint32_t rem = len - si * (NW * kWave);
      // invalid lanes read the step's first element, which always exists
      const uint32_t* bk0 = keys_in + c0 + si * (NW * kWave);
      const uint32_t* bv0 = vals_in + c0 + si * (NW * kWave);
      uint32_t k[NW], v[NW];
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const bool valid = (uint32_t)(j * kWave) + lane < rem;
        const uint32_t o = valid ? (uint32_t)(j * kWave) + lane : 0u;
        k[j] = bk0[o];
        if (KV) v[j] = bv0[o];
      }
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const bool valid = (uint32_t)(j * kWave) + lane < rem;
        const uint32_t b = valid ? bf(k[j]) : 0u;
        const uint64_t mm = match_bucket<BITS>(b, ballot(valid));
        const uint32_t r = count_below(mm), cnt = popc64(mm);
        const uint32_t pos = lds_get(my_cnt + b);
        lds_put(my_cnt + b, pos + cnt);  // same value from every lane of b
        wave_order();
        const uint32_t o = pos + r;
        if (valid && o < plan.n) {
          keys_out[o] = k[j];
          if (KV) vals_out[o] = v[j];
        }
      }
    }
  } else {
    uint32_t* s_k = s_keys + g * T;
    uint32_t* s_v = s_vals + (KV ? g * T : 0);
    uint8_t* s_b = s_bk + g * T;
    uint32_t* delta = s_delta + g * kMaxBuckets;
    uint32_t* grp_cnt = s_cnt + (g * WPG) * CNT_STRIDE;
    const uint32_t ntiles = (uint32_t)(((uint64_t)len + T - 1) / T);
    const uint32_t wbase = wg * NW * kWave;
    uint32_t k[NW], v[NW];

    // Loads of tile ti into k, v (element (wg, j, lane) of the tile).  In a
    // partial tile, lanes past the end read the tile's first element, which
    // always exists, and are masked out later.
    auto load = [&](uint32_t ti, auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const uint32_t tb = c0 + ti * T;
      const uint32_t tcount = FULL ? (uint32_t)T : min((uint32_t)T, len - ti * T);
      const uint32_t* pk = keys_in + tb + wbase + lane;
      const uint32_t* pv = vals_in + tb + wbase + lane;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        if (FULL) {
          k[j] = __builtin_nontemporal_load(pk + j * kWave);
          if (KV) v[j] = __builtin_nontemporal_load(pv + j * kWave);
        } else {
          const bool valid = wbase + (uint32_t)(j * kWave) + lane < tcount;
          k[j] = __builtin_nontemporal_load(valid ? pk + j * kWave : keys_in + tb);
          if (KV) v[j] = __builtin_nontemporal_load(valid ? pv + j * kWave : vals_in + tb);
        }
      }
    };
    auto load_tile = [&](uint32_t ti) {
      if (len - ti * T >= (uint32_t)T)
        load(ti, std::true_type{});
      else
        load(ti, std::false_type{});
    };

    auto tile = [&](uint32_t ti, auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const uint32_t tcount = FULL ? (uint32_t)T : min((uint32_t)T, len - ti * T);
      TileCtx<KV> ctx{s_k, s_v, s_b, my_cnt, grp_cnt, run, delta, s_tmp + g * WPG,
                      keys_out, vals_out, m, tcount, wg, lane, tid_g};
      auto next = [&] {
        if (kReverseTiles) {
          if (ti > 0) load_tile(ti - 1);
        } else if (ti + 1 < ntiles) {
          load_tile(ti + 1);
        }
      };
      tile_rank_reorder_write<BITS, KV, WPG, NW, FULL, decltype(bf), decltype(next),
                              kReverseTiles>(bf, k, v, ctx, next);
    };

    if (ntiles > 0) load_tile(kReverseTiles ? ntiles - 1 : 0);
    for (uint32_t it = 0; it < ntiles; ++it) {
      const uint32_t ti = kReverseTiles ? ntiles - 1 - it : it;
      if (len - ti * T >= (uint32_t)T)
        tile(ti, std::true_type{});
      else
        tile(ti, std::false_type{});
    }
  }
  if (Kind == kLearned && bp.mispredicts) {
    uint32_t miss = bf.misses();
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) miss += __shfl_xor(miss, d, kWave);
    if (lane == 0 && miss) atomicAdd(bp.mispredicts, (unsigned long long)miss);
  }
}

}  // namespace ms
