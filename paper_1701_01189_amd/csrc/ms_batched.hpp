// Batched stable multisplit: many independent instances (segments of one
// concatenated array) in one persistent launch.  Not in the paper; it uses
// the paper's per-tile machinery (pre-scan histogram, scan of the
// row-vectorised H of Eq. 2, post-scan rank/reorder/scatter) with one
// subproblem per tile.
//
// Work items, handed out by one atomic queue counter in this order:
//   [0, P)      pre-scan of tile t (all tiles of all instances, P in total);
//   [P, 2P)     post-scan of tile t - P.
// The last pre-scan tile of an instance to finish (a per-instance atomic
// counter) scans that instance's H and raises its ready flag; a post-scan
// tile waits for its instance's flag.  Every pre-scan item is dequeued before
// any post-scan item, by a workgroup that is already running and never
// waits, so each awaited flag is eventually raised whatever the residency.
// The wait is bounded all the same (spin_limit polls); on expiry the tile is
// skipped and the status word records MS_ERR_TIMEOUT.  A workgroup takes
// `claim` consecutive items per queue access and loads the next item's keys
// (and values) while it works on the current one: inputs are ready from the
// start, only the bucket bases of a post-scan item wait for its instance.
#pragma once

#include "ms_kernels.hpp"

namespace ms {

struct BatchedArgs {
  const uint32_t* keys_in;
  const uint32_t* vals_in;
  uint32_t* keys_out;
  uint32_t* vals_out;
  const uint64_t* seg;   // num + 1 segment starts
  uint32_t num;
  uint32_t m;
  uint32_t* offsets;     // num * (m+1)
  uint32_t* tile_start;  // num + 1: first global tile of each instance
  uint4* tile_info;      // per global tile: first key, key count, instance, tile index
  uint32_t* H;           // m * P words; instance i at m * tile_start[i]
  uint32_t* done;        // num: finished pre-scan tiles
  uint32_t* ready;       // num: 1 once G of the instance is published
  uint32_t* ctl;         // [0] queue counter, [1] status
  uint32_t tile;         // elements per tile
  uint32_t claim;        // work items per queue claim
  uint32_t spin_limit;   // polls before a wait gives up
  uint32_t never_ready;  // test hook: never raise ready flags (forces timeouts)
  uint32_t osh;          // 2: total <= 2^30, output positions as byte offsets
  uint32_t ntl;          // 1: whole output lines stored nontemporally
  BucketParams bp;
};

constexpr int kSetupThreads = 1024;
constexpr int kMaxClaim = 64;  // work items per queue claim, at most

// (Internal linkage: every translation unit that launches it has a copy.)
// Tiles per instance, their exclusive prefix (tile_start), counters and
// flags cleared, offsets of empty instances written.  One workgroup.
static __global__ void __launch_bounds__(kSetupThreads) batched_setup_kernel(BatchedArgs a) {
  __shared__ uint32_t tmp[kSetupThreads / kWave];
  const uint32_t lane = lane_id(), w = wave_id();
  const uint32_t per = (a.num + kSetupThreads - 1) / kSetupThreads;
  const uint32_t i0 = threadIdx.x * per;
  uint32_t sum = 0;
  for (uint32_t e = 0; e < per; ++e) {
    const uint32_t i = i0 + e;
    if (i < a.num) {
      const uint64_t n = a.seg[i + 1] - a.seg[i];
      sum += n == 0 ? 0u : ((uint32_t)n - 1u) / a.tile + 1u;  // no overflow near 2^32
    }
  }
  uint32_t total;
  uint32_t pre = group_exclusive_scan<kSetupThreads / kWave>(sum, tmp, w, lane, &total);
  for (uint32_t e = 0; e < per; ++e) {
    const uint32_t i = i0 + e;
    if (i < a.num) {
      const uint64_t n = a.seg[i + 1] - a.seg[i];
      a.tile_start[i] = pre;
      pre += n == 0 ? 0u : ((uint32_t)n - 1u) / a.tile + 1u;
      a.done[i] = 0;
      a.ready[i] = 0;
      if (n == 0)
        for (uint32_t b = 0; b <= a.m; ++b) a.offsets[(uint64_t)i * (a.m + 1) + b] = 0;
    }
  }
  if (threadIdx.x == 0) {
    a.tile_start[a.num] = total;
    a.ctl[0] = 0;
    a.ctl[1] = 0;
  }
  // Per-tile records, written once here so that a work item finds its keys
  // with one read instead of a chain of dependent ones (the workgroup's own
  // tile_start writes are visible after the barrier).  Each wavefront takes
  // 64 consecutive instances, reads their tile ranges and segment starts
  // with coalesced loads and walks them with lane broadcasts; the records of
  // one instance are stored by consecutive lanes.
  __syncthreads();
  for (uint32_t base = w * kWave; base < a.num; base += kSetupThreads) {
    const uint32_t i = base + lane;
    const uint32_t t0 = i < a.num ? a.tile_start[i] : 0u;
    const uint32_t t1 = i < a.num ? a.tile_start[i + 1] : 0u;
    const uint32_t k0 = i < a.num ? (uint32_t)a.seg[i] : 0u;
    const uint32_t k1 = i < a.num ? (uint32_t)a.seg[i + 1] : 0u;
    const uint32_t cnt = min((uint32_t)kWave, a.num - base);
    for (uint32_t j = 0; j < cnt; ++j) {
      const uint32_t s0 = __builtin_amdgcn_readlane(t0, j);
      const uint32_t s1 = __builtin_amdgcn_readlane(t1, j);
      const uint32_t f0 = __builtin_amdgcn_readlane(k0, j);
      const uint32_t f1 = __builtin_amdgcn_readlane(k1, j);
      for (uint32_t t = s0 + lane; t < s1; t += kWave) {
        const uint32_t first = f0 + (t - s0) * a.tile;
        a.tile_info[t] = make_uint4(first, min(a.tile, f1 - first), base + j, t - s0);
      }
    }
  }
}

// Exclusive scan in place of E words by one workgroup.
template <int WPB>
__device__ void block_scan_inplace(uint32_t* data, uint32_t E, uint32_t* tmp) {
  constexpr int PER = 4;
  const uint32_t lane = lane_id(), w = wave_id();
  uint32_t carry = 0;
  for (uint32_t base = 0; base < E; base += WPB * kWave * PER) {
    uint32_t v[PER], s = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const uint32_t i = base + threadIdx.x * PER + e;
      v[e] = i < E ? data[i] : 0u;
      s += v[e];
    }
    uint32_t total;
    uint32_t pre = group_exclusive_scan<WPB>(s, tmp, w, lane, &total) + carry;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const uint32_t i = base + threadIdx.x * PER + e;
      if (i < E) data[i] = pre;
      pre += v[e];
    }
    carry += total;
  }
}

template <int Kind, int BITS, bool KV, int WPB, int NW>
__global__ void __launch_bounds__(WPB* kWave) batched_kernel(BatchedArgs a) {
  constexpr int T = WPB * NW * kWave;
  constexpr int MB = Owned<BITS>::value;
  constexpr bool TABLES = (Kind == kSplitters || Kind == kLearned);
  __shared__ uint32_t s_tables[TABLES ? (sizeof(BucketLds) + 3) / 4 : 1];
  // counter rows of the pre-scan's histogram and of the post-scan tiles
  __shared__ uint32_t s_cnt[WPB * kCntStride];
  __shared__ uint32_t s_run[kMaxBuckets];
  __shared__ __align__(8) uint32_t s_delta[2 * kMaxBuckets];
  constexpr int SLOT = reorder_bytes_per_slot<(BITS <= 6), !TABLES>();
  __shared__ uint64_t s_reorder[(T * SLOT + 7) / 8];
  __shared__ uint32_t s_vals[KV ? T : 1];
  __shared__ uint32_t s_tmp[WPB];
  __shared__ uint32_t s_next, s_flag;
  __shared__ uint4 s_info[kMaxClaim];   // records of the claim's items
  __shared__ uint32_t s_tiles[kMaxClaim];  // H row length of each item's instance
  // pre-scan up to 64 buckets: one counter per (bucket, lane), shared by the
  // workgroup's wavefronts (as the multisplit pre-scan's lane counters);
  // zero between tiles
  constexpr bool LANES = BITS <= 6;
  __shared__ uint32_t s_lane[LANES ? kWave * kWave : 1];
  if (LANES)
    for (uint32_t i = threadIdx.x; i < kWave * kWave; i += WPB * kWave) s_lane[i] = 0u;

  BucketLds* tables = reinterpret_cast<BucketLds*>(s_tables);
  if (TABLES) stage_bucket_tables<Kind>(a.bp, tables);
  __syncthreads();
  Bucket<Kind, BITS> bf_pre(a.bp, tables);
  Bucket<Kind, BITS> bf_post(a.bp, tables);
  const uint32_t lane = lane_id(), w = wave_id();
  const uint32_t tid = threadIdx.x;
  const LaneSel ls(lane);
  const uint32_t m = a.m;
  const uint32_t P = a.tile_start[a.num];
  const uint32_t items = 2 * P;
  const uint32_t wbase = w * NW * kWave;

  // The next claim is taken from the queue while the current one is worked
  // on, so the atomic's latency is hidden.
  if (tid == 0)
    s_next = __hip_atomic_fetch_add(a.ctl, a.claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    __syncthreads();
    const uint32_t first = s_next;
    __syncthreads();
    if (first >= items) break;
    if (tid == 0)
      s_next = __hip_atomic_fetch_add(a.ctl, a.claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t last = min(items, first + a.claim);
    // the claim's tile records and H row lengths, one lane per item
    if (tid < last - first) {
      const uint32_t it = first + tid;
      const uint32_t tg = it < P ? it : it - P;
      const uint4 r = a.tile_info[tg];
      s_info[tid] = r;
      s_tiles[tid] = a.tile_start[r.z + 1] - (tg - r.w);
    }
    __syncthreads();

    // Keys of work item `it` (a global tile index below P for a pre-scan
    // item, P + tile for a post-scan item).  Lanes past the tile's end read
    // the tile's first element, which exists, and are masked out later.
    uint32_t k[NW], v[NW];
    auto load_item = [&](uint32_t it, auto vals_tag) {
      constexpr bool with_vals = decltype(vals_tag)::value;
      const uint4 r = s_info[it - first];
      const uint32_t tcount = r.y;
      const uint32_t tb = r.x;
      const uint32_t* pk = a.keys_in + tb + wbase + lane;
      const uint32_t* pv = a.vals_in + tb + wbase + lane;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const bool valid = wbase + (uint32_t)(j * kWave) + lane < tcount;
        k[j] = __builtin_nontemporal_load(valid ? pk + j * kWave : a.keys_in + tb);
        if (KV && with_vals) v[j] = __builtin_nontemporal_load(valid ? pv + j * kWave : a.vals_in + tb);
      }
    };
    // ---- pre-scan items of this claim: one column of H per tile; the
    // columns of one instance are published together (one release) ----
    const uint32_t pre_end = min(last, P);
    uint32_t pub_inst = 0xFFFFFFFFu, pub_count = 0;
    auto publish = [&]() {
      __syncthreads();
      if (tid == 0) {
        const uint32_t tiles = a.tile_start[pub_inst + 1] - a.tile_start[pub_inst];
        const uint32_t prev = __hip_atomic_fetch_add(a.done + pub_inst, pub_count, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        s_flag = (prev + pub_count == tiles) ? 1u : 0u;
      }
      __syncthreads();
      if (s_flag) {
        // the instance's last columns: scan its H into G and publish G
        const uint32_t i = pub_inst;
        const uint32_t tiles = a.tile_start[i + 1] - a.tile_start[i];
        uint32_t* Hi = a.H + (size_t)m * a.tile_start[i];
        block_scan_inplace<WPB>(Hi, m * tiles, s_tmp);
        __syncthreads();
        for (uint32_t b = tid; b < m; b += WPB * kWave)
          a.offsets[(size_t)i * (m + 1) + b] = Hi[b * tiles];
        if (tid == 0) a.offsets[(size_t)i * (m + 1) + m] = (uint32_t)(a.seg[i + 1] - a.seg[i]);
        __syncthreads();
        if (tid == 0 && !a.never_ready)
          __hip_atomic_store(a.ready + i, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
    };
    // ---- pre-scan items: keys only, two items ahead ----
    uint32_t k2[NW];
    auto load_keys = [&](uint32_t it, uint32_t (&dst)[NW]) {
      const uint4 r = s_info[it - first];
      const uint32_t* pk = a.keys_in + r.x + wbase + lane;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const bool valid = wbase + (uint32_t)(j * kWave) + lane < r.y;
        dst[j] = __builtin_nontemporal_load(valid ? pk + j * kWave : a.keys_in + r.x);
      }
    };
    auto pre_item = [&](uint32_t it, uint32_t (&kc)[NW]) {
      const uint4 r = s_info[it - first];
      const uint32_t i = r.z;
      if (i != pub_inst) {
        if (pub_count) publish();
        pub_inst = i;
        pub_count = 0;
      }
      const uint32_t t = r.w;
      const uint32_t tiles = s_tiles[it - first];
      const uint32_t tcount = r.y;
      uint32_t* Hi = a.H + (size_t)m * (it - t);
      uint32_t cnt[MB];
#pragma unroll
      for (int q = 0; q < MB; ++q) cnt[q] = 0;
      // bucket ids of this tile, then the keys of the item after the next are
      // requested while the histogram is solved: two items' loads in flight
      // (one workgroup of these shapes fills a compute unit)
      uint32_t bk[NW];
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const bool valid = wbase + (uint32_t)(j * kWave) + lane < tcount;
        bk[j] = valid ? bf_pre(kc[j]) : 0u;
      }
      // (only items of this claim: their records are the ones staged)
      if (it + 2 < pre_end) load_keys(it + 2, kc);
      if constexpr (LANES) {
        // every element adds 1 to its lane's counter of its bucket: the 64
        // lanes of an instruction hit 64 distinct counters
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const bool valid = wbase + (uint32_t)(j * kWave) + lane < tcount;
          if (valid)
            __hip_atomic_fetch_add(&s_lane[bk[j] * kWave + lane], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        // bucket b's count is the sum of its 64 lane counters, which are
        // cleared for the next tile on the way
        for (uint32_t b = w; b < m; b += WPB) {
          const uint32_t c = s_lane[b * kWave + lane];
          s_lane[b * kWave + lane] = 0u;
          const uint32_t sum = wave_inclusive_scan(c, lane);
          if (lane == kWave - 1) Hi[b * tiles + t] = sum;
        }
      } else {
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const bool valid = wbase + (uint32_t)(j * kWave) + lane < tcount;
          window_histogram<BITS>(bk[j], ballot(valid), ls, cnt);
        }
#pragma unroll
        for (int q = 0; q < MB; ++q) {
          const uint32_t b = lane + kWave * q;
          if (b < m) s_cnt[w * kCntStride + b] = cnt[q];
        }
        __syncthreads();
        for (uint32_t b = tid; b < m; b += WPB * kWave) {
          uint32_t s = 0;
#pragma unroll
          for (int ww = 0; ww < WPB; ++ww) s += s_cnt[ww * kCntStride + b];
          Hi[b * tiles + t] = s;
        }
      }
      __syncthreads();
      ++pub_count;
    };
    if (first < pre_end) load_keys(first, k);
    if (first + 1 < pre_end) load_keys(first + 1, k2);
    for (uint32_t it = first; it < pre_end; it += 2) {
      pre_item(it, k);
      if (it + 1 < pre_end) pre_item(it + 1, k2);
    }
    if (pub_count) publish();

    // ---- post-scan items of this claim; the wait (an acquire) is done
    // once per instance ----
    uint32_t seen = 0xFFFFFFFFu;
    const uint32_t post_first = first > P ? first : P;
    if (post_first < last) load_item(post_first, std::true_type{});
    for (uint32_t it = post_first; it < last; ++it) {
      const uint32_t tg = it - P;
      const uint4 r = s_info[it - first];
      const uint32_t i = r.z;
      if (i != seen) {
        if (tid == 0) {
          uint32_t ok = 1, polls = 0;
          while (__hip_atomic_load(a.ready + i, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            if (++polls > a.spin_limit) {
              ok = 0;
              __hip_atomic_fetch_or(a.ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
          s_flag = ok;
        }
        __syncthreads();
        seen = s_flag ? i : 0xFFFFFFFFu;
        if (!s_flag) {
          __syncthreads();
          if (it + 1 < last) load_item(it + 1, std::true_type{});
          continue;  // instance not published in time: tile skipped, status set
        }
      }
      const uint32_t t = r.w;
      const uint32_t tiles = s_tiles[it - first];
      const uint32_t s0 = r.x - t * (uint32_t)T;  // the instance's first key
      const uint32_t tcount = r.y;
      const uint32_t* Hi = a.H + (size_t)m * (tg - t);
      const TileBufs<KV> tb{s_reorder, s_vals, s_cnt, s_run, s_delta, s_tmp, a.keys_out,
                            a.vals_out, a.osh, a.ntl};
      const uint32_t idv[NW] = {};  // (bucket ids are computed here)
      // the next item's loads go out once this tile sits in LDS
      auto next = [&] { if (it + 1 < last) load_item(it + 1, std::true_type{}); };
      if constexpr (BITS <= 6) {
        // lane b of every wavefront holds bucket b's output position
        uint32_t run = lane < m ? s0 + Hi[lane * tiles + t] : 0u;
        if (tcount == (uint32_t)T)
          tile_small<BITS, KV, WPB, NW, true, false>(bf_post, k, v, idv, false, tb, tcount, w, lane,
                                                     run, next);
        else
          tile_small<BITS, KV, WPB, NW, false, false>(bf_post, k, v, idv, false, tb, tcount, w, lane,
                                                      run, next);
      } else {
        for (uint32_t b = tid; b < m; b += WPB * kWave) s_run[b] = s0 + Hi[b * tiles + t];
        __syncthreads();
        if (tcount == (uint32_t)T)
          tile_large<BITS, KV, WPB, NW, true, false>(bf_post, k, v, idv, false, tb, m, tcount, w,
                                                     lane, next);
        else
          tile_large<BITS, KV, WPB, NW, false, false>(bf_post, k, v, idv, false, tb, m, tcount, w,
                                                      lane, next);
      }
      // No closing barrier (as between the tiles of a multisplit chunk): the
      // next item's tile writes LDS only after its own first barrier; the
      // running positions above 64 buckets (s_run), written before it, are
      // read only before this tile's second barrier, which every wavefront
      // has passed; s_flag is next written by a wavefront past both.
    }
  }
  if (Kind == kLearned && a.bp.mispredicts) {
    uint32_t miss = bf_post.misses();
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) miss += __shfl_xor(miss, d, kWave);
    if (lane == 0 && miss) atomicAdd(a.bp.mispredicts, (unsigned long long)miss);
  }
}

}  // namespace ms
