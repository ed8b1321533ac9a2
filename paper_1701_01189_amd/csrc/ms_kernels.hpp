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

#include "ms_tile.hpp"

namespace ms {

enum Mode { kBlock = 1, kWaveMode = 2, kDirect = 3 };

struct Plan {
  uint32_t n;         // elements
  uint32_t m;         // buckets
  uint32_t L0;        // chunks = columns of H
  uint32_t chunk;     // elements per chunk (multiple of the tile size)
  uint32_t tile;      // elements per tile
  uint32_t h_raw;     // 1: H is not scanned; every post-scan workgroup reads it
                      // whole (block-level reordering, at most 64 buckets)
  uint32_t nt_lines;  // 1: whole output lines are stored nontemporally
};

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
               uint32_t* __restrict__ H, uint8_t* __restrict__ ids) {
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
  // (one group per workgroup: its LDS offsets are then constants)
  const uint32_t g = GPB == 1 ? 0u : w / WPG, wg = GPB == 1 ? w : w % WPG;
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
    constexpr bool TABLES = (Kind == kSplitters || Kind == kLearned);
    while (gi < full) {
      uint32_t b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) b[u] = bf(k[u]);
      if (TABLES && ids) {  // kept for the post-scan
#pragma unroll
        for (int u = 0; u < U; ++u) ids[c0 + gi * BATCH + u * kWave + lane] = (uint8_t)b[u];
      }
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
        if (TABLES && ids && valid) ids[c0 + full * BATCH + u * kWave + lane] = (uint8_t)b;
        if (LANES) {
          if (valid) lane_count(b, lane);
        } else {
          window_histogram<BITS>(b, ballot(valid), ls, cnt);
        }
      }
    }
  }
  if (Kind == kLearned && ids && bp.mispredicts) {
    // the post-scan reads the kept ids: the raw predictions are counted here
    uint32_t miss = bf.misses();
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) miss += __shfl_xor(miss, d, kWave);
    if (lane == 0 && miss) atomicAdd(bp.mispredicts, (unsigned long long)miss);
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

// The post-scan visits a chunk's tiles last to first.  The pre-scan swept
// every chunk first to last, so the last lines it read -- the ends of the
// chunks -- are the ones still in the memory-side cache when the post-scan
// starts; beginning there re-reads them from the cache instead of HBM.
// Each tile then takes its bucket runs from the top of what is left of the
// chunk's bucket ranges, which places every element exactly where the
// forward order would (the tile's local order is unchanged).
constexpr bool kReverseTiles = true;

// ---------------------------------------------------------------------------
// Post-scan (Algorithm 1's post-scan, Sections 5.5.3-5.6).
//
// Each group (a workgroup for BMS, a wavefront for WMS/DMS) owns one chunk
// and visits its tiles; a tile's loads are issued while the previous tile
// is being written back.  The per-tile work (rank, bases, local reorder,
// coalesced write-back) is tile_small / tile_large.  The output position of
// bucket b's elements of chunk c starts at the bucket's base (exclusive scan
// of the bucket totals, first term of Eq. 2) plus G[b][c] (second term).
// Mode kDirect ranks the same way but writes from registers (DMS).
// ---------------------------------------------------------------------------
// Static LDS bytes of a post-scan instantiation (the arrays declared in
// postscan_kernel, same rounding), for shapes that do not fit a CU.
template <int Kind, int BITS, bool KV, int WPB, int NW, int MODE>
constexpr size_t postscan_lds_bytes() {
  constexpr int WPG = (MODE == kBlock) ? WPB : 1;
  constexpr size_t GPB = WPB / WPG, T = (size_t)WPG * NW * kWave;
  constexpr bool REORDER = MODE != kDirect, SMALL = BITS <= 6;
  constexpr bool TABLES = (Kind == kSplitters || Kind == kLearned);
  constexpr size_t SLOT = reorder_bytes_per_slot<SMALL, Bucket<Kind, BITS>::kCheap>();
  return (TABLES ? (sizeof(BucketLds) + 3) / 4 * 4 : 4) +
         (size_t)WPB * (SMALL ? kWave : kCntStride) * 4 + (SMALL ? 4 : GPB * kMaxBuckets * 4) +
         ((REORDER && !SMALL) ? GPB * kMaxBuckets * (KV ? 8 : 4) : 8) +
         (REORDER ? (GPB * T * SLOT + 7) / 8 * 8 : 8) + ((REORDER && KV) ? GPB * T * 4 : 4) +
         (size_t)WPB * 4;
}
constexpr size_t kLdsLimit = 160 * 1024;

template <int Kind, int BITS, bool KV, int WPB, int NW, int MODE>
__global__ void __launch_bounds__(WPB* kWave)
postscan_kernel(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
                uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                const uint32_t* __restrict__ G, const uint32_t* __restrict__ totals,
                uint32_t* __restrict__ offsets, Plan plan, BucketParams bp,
                const uint8_t* __restrict__ ids) {
  constexpr int WPG = (MODE == kBlock) ? WPB : 1;
  constexpr int GPB = WPB / WPG;
  constexpr int T = WPG * NW * kWave;
  constexpr bool REORDER = (MODE != kDirect);
  constexpr bool SMALL = BITS <= 6;  // one bucket per lane
  constexpr bool TABLES = (Kind == kSplitters || Kind == kLearned);
  constexpr bool KEPT = Kind == kKeptIds;  // ids always come from the pre-scan's bytes
  constexpr int S = SMALL ? kWave : kCntStride;  // counter row stride
  constexpr bool REV = kReverseTiles && REORDER;
  static_assert(SMALL || WPB * kWave >= kMaxBuckets, "one thread per bucket base");

  __shared__ uint32_t s_tables[TABLES ? (sizeof(BucketLds) + 3) / 4 : 1];
  __shared__ uint32_t s_cnt[WPB * S];
  __shared__ uint32_t s_run[SMALL ? 1 : GPB * kMaxBuckets];
  __shared__ __align__(8) uint32_t s_delta[(REORDER && !SMALL) ? GPB * (KV ? 2 : 1) * kMaxBuckets : 2];
  constexpr int SLOT = reorder_bytes_per_slot<SMALL, Bucket<Kind, BITS>::kCheap>();
  __shared__ uint64_t s_reorder[REORDER ? (GPB * T * SLOT + 7) / 8 : 1];
  __shared__ uint32_t s_vals[(REORDER && KV) ? GPB * T : 1];
  __shared__ uint32_t s_tmp[WPB];
  BucketLds* tables = reinterpret_cast<BucketLds*>(s_tables);

  const uint32_t lane = lane_id();
  const uint32_t w = wave_id();
  // (one group per workgroup: its LDS offsets are then constants)
  const uint32_t g = GPB == 1 ? 0u : w / WPG, wg = GPB == 1 ? w : w % WPG;
  const uint32_t m = plan.m;
  const uint32_t c = blockIdx.x * GPB + g;

  if (TABLES) stage_bucket_tables<Kind>(bp, tables);

  // Running output position of each bucket in the group's chunk: the
  // bucket's base plus G[b][c], or with tiles visited last to first the
  // chunk's end (the next chunk's start, or the bucket's end for the last
  // chunk).  Up to 64 buckets every wavefront scans the totals itself and
  // keeps bucket b's position in lane b.
  uint32_t run = 0;
  if (SMALL) {
    uint32_t tot, gpos = 0;  // gpos: G[b][c] (or G[b][c + 1] for reversed tiles)
    if (GPB == 1 && plan.h_raw) {
      // Small H (the scan kernel is not launched): every workgroup sums it
      // itself.  Wavefront w takes buckets w, w + WPB, ...: its lanes stride
      // over the bucket's row, and the row total and the sum of the columns
      // before the group's position go to LDS (s_cnt is free until the
      // tiles start).
      const uint32_t cend = REV ? c + 1 : c;  // columns summed into gpos
      for (uint32_t b = w; b < m; b += WPB) {
        uint32_t all = 0, before = 0;
        for (uint32_t cc = lane; cc < plan.L0; cc += kWave) {
          const uint32_t h = G[b * plan.L0 + cc];
          all += h;
          before += cc < cend ? h : 0u;
        }
        all = wave_inclusive_scan(all, lane);
        before = wave_inclusive_scan(before, lane);
        if (lane == kWave - 1) {
          s_cnt[b] = all;
          s_cnt[kWave + b] = before;
        }
      }
      __syncthreads();
      tot = lane < m ? s_cnt[lane] : 0u;
      gpos = lane < m ? s_cnt[kWave + lane] : 0u;
      __syncthreads();  // s_cnt is reused by the tiles
    } else {
      tot = lane < m ? totals[lane] : 0u;
    }
    const uint32_t bb = wave_inclusive_scan(tot, lane) - tot;
    if (blockIdx.x == 0 && w == 0) {
      if (lane < m) offsets[lane] = bb;
      if (lane == 0) offsets[m] = plan.n;
    }
    if (c < plan.L0 && lane < m) {
      if (GPB == 1 && plan.h_raw)
        run = bb + gpos;
      else if (REV)
        run = bb + (c + 1 < plan.L0 ? G[lane * plan.L0 + c + 1] : tot);
      else
        run = bb + G[lane * plan.L0 + c];
    }
    if (TABLES) __syncthreads();
  } else {
    uint32_t v = threadIdx.x < m ? totals[threadIdx.x] : 0u;
    uint32_t total;
    uint32_t pre = group_exclusive_scan<WPB>(v, s_tmp, w, lane, &total);
    if (threadIdx.x < m) {
      s_cnt[threadIdx.x] = pre;  // staged bucket base
      if (blockIdx.x == 0) offsets[threadIdx.x] = pre;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[m] = plan.n;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < GPB * m; i += WPB * kWave) {
      const uint32_t gg = i / m, b = i % m;
      const uint32_t cc = blockIdx.x * GPB + gg;
      uint32_t r = 0;
      if (cc < plan.L0) {
        if (REV)
          r = s_cnt[b] + (cc + 1 < plan.L0 ? G[b * plan.L0 + cc + 1] : totals[b]);
        else
          r = s_cnt[b] + G[b * plan.L0 + cc];
      }
      s_run[gg * kMaxBuckets + b] = r;
    }
    __syncthreads();
  }

  Bucket<Kind, BITS> bf(bp, tables);
  if (c >= plan.L0) return;  // only whole idle groups leave (never a BMS group)
  const uint32_t c0 = c * plan.chunk;
  const uint32_t len = min(plan.chunk, plan.n - c0);
  uint32_t* my_cnt = s_cnt + w * S;
  uint32_t* grun = s_run + (SMALL ? 0 : g * kMaxBuckets);

  if (MODE == kDirect) {
    // DMS: counters are the running output positions of this wavefront.
    if (SMALL) {
      lds_put(my_cnt + lane, run);
    } else {
      for (uint32_t b = lane; b < m; b += kWave) lds_put(my_cnt + b, grun[b]);
    }
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
        uint32_t b = 0;
        if (valid)
          b = (KEPT || (TABLES && ids)) ? (uint32_t)ids[c0 + si * (NW * kWave) + j * kWave + lane]
                                        : bf(k[j]);
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
    const TileBufs<KV> tb{reinterpret_cast<char*>(s_reorder) + (size_t)g * T * SLOT,
                          s_vals + (KV ? g * T : 0),
                          s_cnt + (g * WPG) * S,
                          grun,
                          s_delta + (SMALL ? 0 : g * (KV ? 2 : 1) * kMaxBuckets),
                          s_tmp + g * WPG,
                          keys_out,
                          vals_out,
                          plan.n <= (1u << 30) ? 2u : 0u,
                          plan.nt_lines};
    const uint32_t ntiles = (uint32_t)(((uint64_t)len + T - 1) / T);
    const uint32_t wbase = wg * NW * kWave;
    uint32_t k[NW], v[NW], idv[NW];
    const bool use_ids = KEPT || (TABLES && ids != nullptr);

    // Loads of tile ti into k, v (and the kept bucket ids into idv) --
    // element (wg, j, lane) of the tile.  In a partial tile, lanes past the
    // end read the tile's first element, which always exists, and are
    // masked out later.
    // A lane's address is a uniform base (scalar registers) plus its 32-bit
    // byte offset, and in a whole tile the window's distance is the
    // instruction's immediate offset.  The lane offset passes through an
    // empty volatile asm so that it is not hoisted out of the tile loop as
    // eight 64-bit addresses.
    auto load = [&](uint32_t ti, auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const uint32_t tb0 = c0 + ti * T;
      const uint32_t tcount = FULL ? (uint32_t)T : min((uint32_t)T, len - ti * T);
      if (FULL) {
        const char* kb = reinterpret_cast<const char*>(keys_in + tb0 + wbase);
        const char* vb = reinterpret_cast<const char*>(vals_in + tb0 + wbase);
        uint32_t lo = lane * 4u;
        asm volatile("" : "+v"(lo));
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const size_t off = (size_t)lo + (size_t)(j * kWave * 4);
          k[j] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(kb + off));
          if (KV) v[j] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(vb + off));
        }
      } else {
        const char* kb = reinterpret_cast<const char*>(keys_in + tb0);
        const char* vb = reinterpret_cast<const char*>(vals_in + tb0);
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const uint32_t e = wbase + (uint32_t)(j * kWave) + lane;  // element of the tile
          const size_t off = e < tcount ? (size_t)e * 4u : 0u;
          k[j] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(kb + off));
          if (KV) v[j] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(vb + off));
        }
      }
      if ((TABLES || KEPT) && use_ids) {
        const uint8_t* pi = ids + tb0 + wbase + lane;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const bool valid = FULL || wbase + (uint32_t)(j * kWave) + lane < tcount;
          idv[j] = __builtin_nontemporal_load(valid ? pi + j * kWave : ids + tb0);
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
      auto next = [&] {
        if (REV) {
          // only a chunk's last tile can be partial
          if (ti > 0) load(ti - 1, std::true_type{});
        } else if (ti + 1 < ntiles) {
          load_tile(ti + 1);
        }
      };
      if constexpr (SMALL)
        tile_small<BITS, KV, WPG, NW, FULL, REV>(bf, k, v, idv, use_ids, tb, tcount, wg, lane, run,
                                                 next);
      else
        tile_large<BITS, KV, WPG, NW, FULL, REV>(bf, k, v, idv, use_ids, tb, m, tcount, wg, lane,
                                                 next);
    };

    if (ntiles > 0) load_tile(REV ? ntiles - 1 : 0);
    for (uint32_t it = 0; it < ntiles; ++it) {
      const uint32_t ti = REV ? ntiles - 1 - it : it;
      if (len - ti * T >= (uint32_t)T)
        tile(ti, std::true_type{});
      else
        tile(ti, std::false_type{});
    }
  }
  if (Kind == kLearned && bp.mispredicts && !ids) {
    uint32_t miss = bf.misses();
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) miss += __shfl_xor(miss, d, kWave);
    if (lane == 0 && miss) atomicAdd(bp.mispredicts, (unsigned long long)miss);
  }
}

}  // namespace ms
