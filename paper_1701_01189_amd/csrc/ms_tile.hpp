// One tile of the post-scan: rank, local reorder and coalesced write-back
// (Algorithm 1's post-scan; Sections 5.5.2, 5.6 and 5.7), shared by the
// multisplit post-scan and the batched kernel.
//
// A group of WPG wavefronts (the whole workgroup for block-level reordering,
// one wavefront for wavefront-level reordering) holds a tile of
// T = WPG * NW * 64 elements in registers: element (wave wg, window j, lane)
// of the tile is k[j] of that lane, so (wg, j, lane) is input order.
//
//  1. rank: per window, the lanes of the same bucket (Algorithm 3) give the
//     rank among lower lanes; a per-wavefront running count per bucket in
//     LDS gives the rank among the wavefront's earlier windows (first and
//     second terms of Eq. 4);
//  2. bases: an exclusive scan of the bucket-major table [bucket][wavefront]
//     of those counts gives the tile slot where wavefront wg's bucket-b
//     elements start (third term of Eq. 4 plus the tile histogram scan of
//     Section 5.6.2), and each bucket's output offset for this tile;
//  3. reorder: every element is written to its slot of the LDS buffer (a
//     stable local multisplit of the tile, Section 4.7);
//  4. write-back: the buffer is read linearly and slot q goes to its output
//     position (the bucket's position for this tile plus the slot's offset
//     in the bucket's run), so consecutive lanes of a bucket store to
//     consecutive addresses.
//
// Between the barriers only the keys (and values) and one packed rank word
// per window stay in registers.  Bucket ids that are cheap to compute (a
// shift and mask, a multiply-high) are recomputed from the key when needed
// again; ids that come from a table search are computed once and carried in
// the rank word (and stored next to the key in LDS above 64 buckets).
//
// Up to 64 buckets (BITS <= 6) lane b of every wavefront holds bucket b's
// counts, bases and running output position in registers: step 2 is a
// wavefront scan done by each wavefront for itself, and step 3 fetches a
// bucket's values from its lane with ds_bpermute and stores each key with
// its output position, so that step 4 only copies.  A tile then needs two
// group barriers.  Above 64 buckets the group scans the table together and
// keeps the per-bucket values in LDS (four barriers); the reorder buffer
// holds keys only (half the LDS: two workgroups per compute unit), and
// step 4 looks up the bucket's output offset.
#pragma once

#include <type_traits>

#include "ms_device.hpp"

namespace ms {

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

// The value that lane b of this wavefront holds (b < 64), for every lane at
// once: a backward permute through the LDS crossbar, no bank conflicts.
// Every lane of the wavefront must be active.
__device__ __forceinline__ uint32_t from_lane(uint32_t v, uint32_t b) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(b << 2), (int)v);
}

constexpr int kCntStride = kMaxBuckets + 1;  // counter rows above 64 buckets

// A cheap bucket id computed again from the key.  The key passes through an
// empty volatile asm first, so the compiler cannot reuse the id computed in
// step 1 (which would keep one more register per window alive across the
// barrier).
template <class BF>
__device__ __forceinline__ uint32_t recompute(const BF& bf, uint32_t& key) {
  asm volatile("" : "+v"(key));
  return bf(key);
}

// LDS of one group's reorder buffer: up to 64 buckets a (key, output
// position) pair per slot; above, the key alone (plus its bucket id for
// table-search kinds), the position being looked up in step 4.
template <bool SMALL, bool CHEAP>
constexpr int reorder_bytes_per_slot() {
  return SMALL ? 8 : (4 + (CHEAP ? 0 : 1));
}

template <bool KV>
struct TileBufs {
  void* buf;          // reorder buffer, T slots (layout: reorder_bytes_per_slot)
  uint32_t* s_v;      // reorder buffer [T]: values
  uint32_t* cnt;      // the group's counters, wavefront wg's row at wg * stride
  uint32_t* run;      // above 64 buckets: [m] running output position
  uint32_t* delta;    // above 64 buckets: [m] output position minus slot (key-value
                      // tiles: pairs of it and the whole-line slots, first | count << 16)
  uint32_t* tmp;      // above 64 buckets: WPG words
  uint32_t* keys_out;
  uint32_t* vals_out;
  // Output positions are carried as byte offsets (shift 2) when every output
  // index is below 2^30: a 32-bit offset from the uniform output base then
  // addresses the store directly.  Shift 0: element indices.
  uint32_t osh;
  // 1: elements of whole output lines are stored nontemporally (with byte
  // offsets only; see tile_small)
  uint32_t ntl;
};

// Step 1 for the group's tile: fills lr[j] with the element's rank among
// its bucket's elements in earlier windows of this wavefront and lower
// lanes of its window (bits 0-15), plus the bucket id in bits 16-23 for
// table-search kinds.  `my` is this wavefront's counter row, already zero.
template <int BITS, int NW, bool FULL, class BF>
__device__ __forceinline__ void rank_windows(const BF& bf, const uint32_t (&k)[NW],
                                             const uint32_t (&idv)[NW], bool use_ids,
                                             uint32_t (&lr)[NW], uint32_t* my, uint32_t wbase,
                                             uint32_t lane, uint32_t tcount) {
  constexpr bool CHEAP = BF::kCheap;
  auto valid_at = [&](int j) { return FULL || wbase + (uint32_t)(j * kWave) + lane < tcount; };
  // Table-search ids are all computed first, so that their LDS probes
  // overlap (or taken from the ids the pre-scan kept); cheap ids are
  // computed one window ahead.
  uint32_t bk[CHEAP ? 1 : NW];
  if (!CHEAP) {
#pragma unroll
    for (int j = 0; j < NW; ++j)
      bk[CHEAP ? 0 : j] = valid_at(j) ? (use_ids ? idv[j] : bf(k[j])) : 0u;
  }
  auto bucket = [&](int j) -> uint32_t {
    if (CHEAP) return valid_at(j) ? bf(k[j]) : 0u;
    return bk[CHEAP ? 0 : j];
  };
  uint32_t b = bucket(0);
  // The next window's count is read right after this window's store (a
  // wavefront's LDS operations complete in order), so the read's latency
  // overlaps the next window's ballots.
  uint32_t before = lds_get(my + b);
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const uint64_t mm = match_bucket<BITS>(b, FULL ? ~0ull : ballot(valid_at(j)));
    const uint32_t r = count_below(mm), c = popc64(mm);
    lr[j] = (before + r) | (CHEAP ? 0u : (b << 16));
    // Materialised now (volatile: not movable past the barrier): one
    // register per window lives across the barriers instead of both halves
    // of the window's match mask.
    asm volatile("" : "+v"(lr[j]));
    // Every lane of a bucket read the same `before` and holds the same
    // count, so all of them store the same new value.  An invalid lane
    // carries bucket 0 and counts the valid bucket-0 lanes, so it stores
    // that same value too.
    lds_put(my + b, before + c);
    wave_order();
    if (j + 1 < NW) {
      b = bucket(j + 1);
      before = lds_get(my + b);
    }
  }
}

// Bucket id and rank of window j for step 3.
template <class BF>
__device__ __forceinline__ uint32_t bucket_of(const BF& bf, uint32_t& key, uint32_t lr) {
  if (BF::kCheap) return recompute(bf, key);
  return lr >> 16;
}
template <class BF>
__device__ __forceinline__ uint32_t rank_of(uint32_t lr) {
  return BF::kCheap ? lr : (lr & 0xFFFFu);
}

// Step 4 up to 64 buckets: the buffer holds (key, output position) per slot.
template <bool KV, int GT, int NW, bool FULL>
__device__ __forceinline__ void write_back(const TileBufs<KV>& t, uint32_t tcount,
                                           uint32_t tid_g) {
  const uint2* s_ko = static_cast<const uint2*>(t.buf);
  if (t.osh) {
    char* kb = reinterpret_cast<char*>(t.keys_out);
    char* vb = reinterpret_cast<char*>(t.vals_out);
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const uint32_t q = (uint32_t)j * GT + tid_g;
      if (FULL || q < tcount) {
        const uint2 ko = s_ko[q];
        const size_t off = ko.y & ~3u;  // bit 0: a whole line, stored nontemporally
        uint32_t* pk = reinterpret_cast<uint32_t*>(kb + off);
        uint32_t* pv = reinterpret_cast<uint32_t*>(vb + off);
        if (ko.y & 1u) {
          // (the empty asm keeps the compiler from merging the two branches'
          // stores into one ordinary store)
          asm volatile("");
          __builtin_nontemporal_store(ko.x, pk);
          if (KV) __builtin_nontemporal_store(t.s_v[q], pv);
          asm volatile("");
        } else {
          *pk = ko.x;
          if (KV) *pv = t.s_v[q];
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const uint32_t q = (uint32_t)j * GT + tid_g;
      if (FULL || q < tcount) {
        const uint2 ko = s_ko[q];
        t.keys_out[ko.y] = ko.x;
        if (KV) t.vals_out[ko.y] = t.s_v[q];
      }
    }
  }
}

// Up to 64 buckets.  `run` is this lane's bucket's (bucket = lane) running
// output position: the first position of the tile's bucket-b elements in
// forward order (advanced past them), or with tiles visited last to first
// the end of what is left of the bucket's range (moved back over them).
template <int BITS, bool KV, int WPG, int NW, bool FULL, bool REV, class BF, class After>
__device__ __forceinline__ void tile_small(const BF& bf, uint32_t (&k)[NW], uint32_t (&v)[NW],
                                           const uint32_t (&idv)[NW], bool use_ids,
                                           const TileBufs<KV>& t, uint32_t tcount, uint32_t wg,
                                           uint32_t lane, uint32_t& run, After after) {
  static_assert(BITS <= 6, "one bucket per lane");
  constexpr uint32_t S = kWave;
  const uint32_t wbase = wg * NW * kWave;
  const uint32_t tid_g = wg * kWave + lane;
  uint32_t* my = t.cnt + wg * S;
  lds_put(my + lane, 0u);  // buckets >= m stay zero
  wave_order();
  uint32_t lr[NW];
  rank_windows<BITS, NW, FULL>(bf, k, idv, use_ids, lr, my, wbase, lane, tcount);
  group_sync<WPG>();

  // step 2, lane = bucket: the group's count and this wavefront's prefix
  uint32_t tot = 0, pre = 0;
#pragma unroll
  for (int w2 = 0; w2 < WPG; ++w2) {
    const uint32_t x = t.cnt[w2 * S + lane];
    tot += x;
    pre += (w2 < (int)wg) ? x : 0u;
  }
  const uint32_t start = wave_inclusive_scan(tot, lane) - tot;  // tile slot of the bucket
  // this wavefront's first slot of the bucket, as a byte offset in the buffer
  const uint32_t base8 = (start + pre) * (uint32_t)sizeof(uint2);
  if (REV) run -= tot;
  // ... and that element's output position (scaled as t.osh says)
  const uint32_t first = (run + pre) << t.osh;
  // With byte offsets: the whole 128-byte output lines inside the tile's run
  // of the bucket ([run, run + tot) here), as [lo, lo + span) with lo taken
  // relative to this wavefront's first position, in words: low half
  // (first - lo) / 4 + 32 (at least 1), high half span / 4.  Elements there
  // are stored nontemporally: their lines are complete, and the stores do not
  // stay in the caches as dirty lines that the next pass over the input has
  // to write back.  Elements of partial lines keep ordinary stores, which
  // merge with the neighbouring tile's run in L2.
  uint32_t lines = 0;
  if (t.osh && t.ntl) {
    const uint32_t lo = ((run << 2) + 127u) & ~127u, hi = ((run + tot) << 2) & ~127u;
    const uint32_t span = hi > lo ? (hi - lo) >> 2 : 0u;
    lines = ((uint32_t)((int32_t)(first - lo) >> 2) + 32u) | (span << 16);
  }
  if (!REV) run += tot;

  // step 3: slot and output position of every element
  char* buf = static_cast<char*>(t.buf);
  char* vbuf = reinterpret_cast<char*>(t.s_v);
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const bool valid = FULL || wbase + (uint32_t)(j * kWave) + lane < tcount;
    // (an invalid lane holds the tile's first key: its id is in range)
    const uint32_t bj = bucket_of(bf, k[j], lr[j]);
    const uint32_t r = rank_of<BF>(lr[j]);
    const uint32_t a = from_lane(base8, bj) + (r << 3);
    uint32_t o = from_lane(first, bj) + (r << t.osh);
    {
      // bit 0 of a byte offset: the element's line is whole (see `lines`)
      const uint32_t x = from_lane(lines, bj);
      o |= ((x & 0xFFFFu) + r - 32u < (x >> 16)) ? 1u : 0u;
    }
    if (valid) {
      *reinterpret_cast<uint2*>(buf + a) = make_uint2(k[j], o);
      if (KV) *reinterpret_cast<uint32_t*>(vbuf + (a >> 1)) = v[j];
    }
  }
  after();  // k, v are free: the next tile's loads go out
  group_sync<WPG>();
  write_back<KV, WPG * kWave, NW, FULL>(t, tcount, tid_g);
  // No closing barrier: the next tile writes the buffer only after its own
  // first barrier, which every wavefront reaches after finishing step 4; a
  // wavefront's counter row is read by others only before the second one.
}

// 65 to 256 buckets.  t.run[b] is bucket b's running output position as in
// tile_small, shared by the group.  In step 2 each thread of the group owns
// up to BPT consecutive buckets (the whole row of counts of each), so that
// it can finish the bucket's bookkeeping itself.
template <int BITS, bool KV, int WPG, int NW, bool FULL, bool REV, class BF, class After>
__device__ __forceinline__ void tile_large(const BF& bf, uint32_t (&k)[NW], uint32_t (&v)[NW],
                                           const uint32_t (&idv)[NW], bool use_ids,
                                           const TileBufs<KV>& t, uint32_t m, uint32_t tcount,
                                           uint32_t wg, uint32_t lane, After after) {
  constexpr uint32_t S = kCntStride;
  constexpr uint32_t GT = WPG * kWave;  // threads of the group
  constexpr int BPT = (kMaxBuckets + GT - 1) / GT;
  const uint32_t wbase = wg * NW * kWave;
  const uint32_t tid_g = wg * kWave + lane;
  uint32_t* my = t.cnt + wg * S;
  for (uint32_t b = lane; b < m; b += kWave) lds_put(my + b, 0u);
  wave_order();
  uint32_t lr[NW];
  rank_windows<BITS, NW, FULL>(bf, k, idv, use_ids, lr, my, wbase, lane, tcount);
  group_sync<WPG>();

  // step 2: buckets b0 .. b0 + bpt - 1 of this thread; their totals, an
  // exclusive scan of the thread sums over the group, then per bucket the
  // wavefront bases (rewritten in place), the running position and delta
  {
    const uint32_t bpt = (m + GT - 1) / GT;
    const uint32_t b0 = tid_g * bpt;
    uint32_t tot[BPT], s = 0;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const uint32_t b = b0 + i;
      const bool own = (uint32_t)i < bpt && b < m;
      tot[i] = 0;
#pragma unroll
      for (int w2 = 0; w2 < WPG; ++w2) tot[i] += own ? t.cnt[w2 * S + b] : 0u;
      s += tot[i];
    }
    const uint32_t inc = wave_inclusive_scan(s, lane);
    uint32_t pre = inc - s;
    if (WPG > 1) {
      if (lane == kWave - 1) t.tmp[wg] = inc;
      group_sync<WPG>();
#pragma unroll
      for (int w2 = 0; w2 < WPG; ++w2) pre += (w2 < (int)wg) ? t.tmp[w2] : 0u;
    }
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const uint32_t b = b0 + i;
      if ((uint32_t)i < bpt && b < m) {
        const uint32_t st = pre;  // tile slot of the bucket's first element
        uint32_t acc = st;
#pragma unroll
        for (int w2 = 0; w2 < WPG; ++w2) {  // (read again: fewer live registers)
          const uint32_t x = t.cnt[w2 * S + b];
          t.cnt[w2 * S + b] = acc;
          acc += x;
        }
        uint32_t rb;  // the bucket's first output position in this tile
        if (REV) {
          rb = t.run[b] - tot[i];
          t.run[b] = rb;
        } else {
          rb = t.run[b];
          t.run[b] = rb + tot[i];
        }
        if (KV) {
          // The slots whose output lines (32 elements, 128 bytes) lie wholly
          // inside the tile's run [rb, rb + tot): stored nontemporally
          // (key-value tiles only: key-only ones measured slower with it).
          uint32_t wl = 0;
          if (t.osh && t.ntl) {
            const uint32_t l0 = (rb + 31u) & ~31u, l1 = (rb + tot[i]) & ~31u;
            if (l1 > l0) wl = (st + (l0 - rb)) | ((l1 - l0) << 16);
          }
          t.delta[2 * b] = (rb - st) << t.osh;
          t.delta[2 * b + 1] = wl;
        } else {
          t.delta[b] = (rb - st) << t.osh;
        }
      }
      pre += tot[i];
    }
  }
  group_sync<WPG>();

  // step 3
  constexpr bool CHEAP = BF::kCheap;
  constexpr uint32_t T = WPG * NW * kWave;
  uint32_t* s_k = static_cast<uint32_t*>(t.buf);
  uint8_t* s_b = reinterpret_cast<uint8_t*>(s_k + T);
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const bool valid = FULL || wbase + (uint32_t)(j * kWave) + lane < tcount;
    if (valid) {
      const uint32_t bj = bucket_of(bf, k[j], lr[j]);
      const uint32_t slot = my[bj] + rank_of<BF>(lr[j]);
      s_k[slot] = k[j];
      if (KV) t.s_v[slot] = v[j];
      if (!CHEAP) s_b[slot] = (uint8_t)bj;
    }
  }
  after();
  group_sync<WPG>();

  // step 4: slot q of bucket b goes to delta[b] + q (both scaled by t.osh;
  // modulo 2^32 the difference is exact)
  auto step4 = [&](auto byte_tag) {
    constexpr bool BYTES = decltype(byte_tag)::value;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const uint32_t q = (uint32_t)j * GT + tid_g;
      if (FULL || q < tcount) {
        uint32_t key = s_k[q];
        const uint32_t bq = CHEAP ? recompute(bf, key) : (uint32_t)s_b[q];
        const uint2 dw = KV ? reinterpret_cast<const uint2*>(t.delta)[bq]
                            : make_uint2(t.delta[bq], 0u);
        if (BYTES) {
          const uint32_t o = dw.x + (q << 2);
          uint32_t* pk = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(t.keys_out) + (size_t)o);
          uint32_t* pv = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(t.vals_out) + (size_t)o);
          if (KV && q - (dw.y & 0xFFFFu) < (dw.y >> 16)) {
            asm volatile("");  // (as in write_back: two stores, not one)
            __builtin_nontemporal_store(key, pk);
            if (KV) __builtin_nontemporal_store(t.s_v[q], pv);
            asm volatile("");
          } else {
            *pk = key;
            if (KV) *pv = t.s_v[q];
          }
        } else {
          const uint32_t o = dw.x + q;
          t.keys_out[o] = key;
          if (KV) t.vals_out[o] = t.s_v[q];
        }
      }
    }
  };
  if (t.osh)
    step4(std::true_type{});
  else
    step4(std::false_type{});
  // No closing barrier (as in tile_small): counters, run and delta are next
  // written after the next tile's first barrier, tmp after its first too.
}

}  // namespace ms
