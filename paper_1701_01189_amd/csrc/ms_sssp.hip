// Single-source shortest paths by delta-stepping with multisplit bucketing
// (Section 7.2, "Multisplit-SSSP": the Bucketing strategy with its radix
// sort replaced by a multisplit).
//
// The work frontier is a list of (tentative distance, vertex) pairs.  Each
// round:
//   1. a stable multisplit of the pairs (key = distance) into B range
//      buckets of width Delta above a moving base: bucket j holds distances
//      in [base + j*Delta, base + (j+1)*Delta), the last bucket everything
//      from base + (B-1)*Delta up (the splitter bucket kind of Section 6);
//   2. the lowest non-empty bucket is the near set; the buckets above it
//      stay pending, minus entries whose vertex has since been reached by a
//      shorter path (stale entries);
//   3. every out-edge of every near vertex is relaxed with an atomic
//      minimum on the distance array; each relaxation that lowers a
//      distance appends (new distance, vertex) to the pending list.
// The base moves up to the near bucket's lower edge; when only the last
// bucket holds entries, the base jumps to the least pending distance and the
// round relaxes nothing.  The loop ends when no entry is pending.  The
// result is the shortest-path distance of every vertex (unique), whatever
// Delta, B or the order of the atomic updates.
//
// Work balance: relaxation is edge parallel.  The near vertices' degrees are
// scanned (inside each 1024-entry filter workgroup, then over the workgroup
// sums) and each edge finds its vertex by binary search in the scanned
// degrees, so high-degree and low-degree vertices cost the same per edge.
//
// One host synchronisation per round reads the pending count, which sizes
// the next multisplit.  Everything else (the near bucket, the base, the
// splitters of the next round) stays on the device.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "multisplit.h"
#include "ms_device.hpp"

namespace {

using ms::count_below;
using ms::kWave;
using ms::lane_id;
using ms::popc64;

constexpr uint32_t kInf = 0xFFFFFFFFu;      // unreachable
constexpr uint32_t kDistMax = 0xFFFFFFFEu;  // longest representable path
constexpr int kThreads = 256;
constexpr int kPer = 4;
constexpr uint32_t kBlockItems = kThreads * kPer;  // entries per filter workgroup
constexpr int kEdgePer = 8;
constexpr uint32_t kChunk = kThreads * kEdgePer;   // edges per relaxation chunk
constexpr uint32_t kExpandBlocks = 1024;           // 4 workgroups per CU
constexpr uint32_t kFusedSums = 4096;  // workgroup sums the relaxation scans in LDS
constexpr size_t kAlign = 256;

// Loop state in device memory (one aligned slot of the workspace).  The
// append counter and the least pending distance are kept per round parity:
// a round's single-workgroup scan kernel clears the next round's pair, so no
// launch is spent on resetting them.
struct State {
  uint32_t count[2];     // entries appended to the pending list, by round parity
  uint32_t overflow;     // an append found the pending list full
  uint32_t bad_edge;     // an edge pointed past the last vertex
  uint32_t base;         // lower edge of bucket 0
  uint32_t edges;        // edges to relax this round
  uint32_t far_min[2];   // least valid pending distance, by round parity
  unsigned long long relaxed;  // edges relaxed, all rounds
  unsigned long long pushes;   // entries appended by relaxations, all rounds
};

// The round's near bucket, read from the multisplit's bucket starts: the
// first occupied bucket j.  When only the last (open-ended) bucket is
// occupied the round is a jump: nothing is near, everything stays pending
// and the base moves to the least pending distance.  Wavefront uniform.
struct Near {
  uint32_t j, lo, hi;  // near entries [lo, hi); pending entries above from hi
  bool jump;
};

__device__ __forceinline__ Near near_bucket(const uint32_t* offsets, uint32_t nb) {
  Near r;
  uint32_t j = 0;
  while (j + 1 < nb && offsets[j + 1] == offsets[j]) ++j;
  r.j = j;
  r.lo = offsets[j];
  r.jump = j + 1 == nb;
  r.hi = r.jump ? r.lo : offsets[j + 1];
  return r;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  const uint64_t s = (uint64_t)a + b;
  return s > kDistMax ? kDistMax : (uint32_t)s;
}

// Splitters of the next round: base + (i+1)*Delta, saturated.
__device__ __forceinline__ void write_splitters(uint32_t* spl, uint32_t nb, uint32_t base,
                                                uint32_t delta) {
  for (uint32_t i = threadIdx.x; i + 1 < nb; i += blockDim.x) {
    const uint64_t s = (uint64_t)base + (uint64_t)(i + 1) * delta;
    spl[i] = s > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)s;
  }
}

// Reserves `mine` consecutive pending-list slots for every thread of the
// workgroup with one atomic, and returns this thread's first slot (threads
// in order).  Every thread of the workgroup must call it.
__device__ __forceinline__ uint32_t group_reserve(uint32_t mine, uint32_t* counter,
                                                  unsigned long long* pushes, uint32_t* s_w,
                                                  uint32_t* s_base) {
  const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
  const uint32_t inc = ms::wave_inclusive_scan(mine, lane);
  if (lane == kWave - 1) s_w[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t total = 0;
    for (int k = 0; k < kThreads / kWave; ++k) total += s_w[k];
    uint32_t base = 0;
    if (total) {
      base = atomicAdd(counter, total);
      if (pushes) atomicAdd(pushes, (unsigned long long)total);
    }
    *s_base = base;
  }
  __syncthreads();
  uint32_t first = *s_base + inc - mine;
  for (uint32_t k = 0; k < w; ++k) first += s_w[k];
  __syncthreads();  // s_w and s_base may be reused right after
  return first;
}

// Stores one reserved entry; an entry past the list's capacity is dropped
// and flags the overflow.
__device__ __forceinline__ void put_entry(uint32_t idx, uint32_t d, uint32_t v, State* st,
                                          uint32_t* pk, uint32_t* pv, uint32_t cap) {
  if (idx < cap) {
    pk[idx] = d;
    pv[idx] = v;
  } else {
    st->overflow = 1u;
  }
}

__global__ void __launch_bounds__(kThreads)
sssp_init_kernel(uint32_t* __restrict__ dist, uint32_t nv, uint32_t src, uint32_t* pk,
                 uint32_t* pv, State* st, uint32_t* spl, uint32_t nb, uint32_t delta) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
       i += (uint64_t)gridDim.x * blockDim.x)
    dist[i] = i == src ? 0u : kInf;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      pk[0] = 0u;
      pv[0] = src;
      st->count[0] = st->count[1] = 0u;
      st->overflow = 0u;
      st->bad_edge = 0u;
      st->base = 0u;
      st->edges = 0u;
      st->far_min[0] = st->far_min[1] = kInf;
      st->relaxed = 0ull;
      st->pushes = 0ull;
    }
    write_splitters(spl, nb, 0u, delta);
  }
}

// Per workgroup of 1024 multisplit-output entries: keeps the valid pending
// entries above the near bucket (appended to the next pending list), and
// sums the degrees of the valid near entries (written per entry, and per
// workgroup into partial[]).  An entry is valid while its distance equals
// the vertex's current distance.
__global__ void __launch_bounds__(kThreads)
sssp_filter_kernel(const uint32_t* __restrict__ ok, const uint32_t* __restrict__ ov, uint32_t n,
                   const uint64_t* __restrict__ row, const uint32_t* __restrict__ dist, State* st,
                   uint32_t* pk, uint32_t* pv, uint32_t cap, uint32_t* __restrict__ deg,
                   uint32_t* __restrict__ partial, const uint32_t* __restrict__ offsets,
                   uint32_t nb, uint32_t par) {
  __shared__ uint32_t s_w[kThreads / kWave];
  __shared__ uint32_t s_base;
  __shared__ uint32_t s_deg[kBlockItems];
  const Near nr = near_bucket(offsets, nb);
  const uint32_t near_lo = nr.lo, near_hi = nr.hi, far_lo = nr.hi;
  const bool jump = nr.jump;
  const uint32_t b0 = blockIdx.x * kBlockItems;
  uint32_t d[kPer], v[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const uint32_t i = b0 + (uint32_t)e * kThreads + threadIdx.x;
    d[e] = i < n ? ok[i] : kInf;
    v[e] = i < n ? ov[i] : 0u;
  }
  uint32_t dv[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) dv[e] = dist[v[e]];  // v < nv on every lane
  uint32_t fmin = kInf, nkeep = 0;
  bool keep[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const uint32_t i = b0 + (uint32_t)e * kThreads + threadIdx.x;
    const bool valid = i < n && dv[e] == d[e];
    keep[e] = valid && i >= far_lo;
    nkeep += keep[e] ? 1u : 0u;
    if (keep[e] && d[e] < fmin) fmin = d[e];
    uint32_t g = 0;
    if (valid && i >= near_lo && i < near_hi) g = (uint32_t)(row[v[e] + 1] - row[v[e]]);
    s_deg[(uint32_t)e * kThreads + threadIdx.x] = g;
  }
  uint32_t slot = group_reserve(nkeep, &st->count[par], nullptr, s_w, &s_base);
#pragma unroll
  for (int e = 0; e < kPer; ++e)
    if (keep[e]) put_entry(slot++, d[e], v[e], st, pk, pv, cap);
  if (jump) {
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const uint32_t t = __shfl_xor(fmin, o, kWave);
      fmin = t < fmin ? t : fmin;
    }
    if (lane_id() == 0 && fmin != kInf) atomicMin(&st->far_min[par], fmin);
  }
  // Exclusive prefix of the near degrees inside the workgroup, in entry
  // order (a thread scans kPer consecutive entries), and the workgroup total.
  // An entry's first edge in the round is partial[workgroup] (scanned by the
  // scan kernel) plus this local prefix.  group_reserve's last barrier made
  // s_deg complete.
  uint32_t gl[kPer], tsum = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    gl[e] = s_deg[threadIdx.x * kPer + e];
    tsum += gl[e];
  }
  const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
  const uint32_t inc = ms::wave_inclusive_scan(tsum, lane);
  if (lane == kWave - 1) s_w[w] = inc;
  __syncthreads();
  uint32_t run = inc - tsum, total = 0;
  for (uint32_t k = 0; k < kThreads / kWave; ++k) {
    run += k < w ? s_w[k] : 0u;
    total += s_w[k];
  }
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const uint32_t i = b0 + threadIdx.x * kPer + (uint32_t)e;
    if (i < n) deg[i] = run;
    run += gl[e];
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of count per-workgroup degree sums from src into dst (dst
// may be src, or an LDS array); returns the total, this round's edge count.
// Four consecutive sums per thread per pass.  Every thread of the workgroup
// calls it.
__device__ __forceinline__ uint32_t group_scan_sums(const uint32_t* src, uint32_t count,
                                                    uint32_t* dst, uint32_t* s_w,
                                                    uint32_t* s_carry) {
  const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) *s_carry = 0;
  __syncthreads();
  for (uint32_t b = 0; b < count; b += 4 * kThreads) {
    const uint32_t i0 = b + 4 * threadIdx.x;
    uint32_t v[4], t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = i0 + k < count ? src[i0 + k] : 0u;
      t += v[k];
    }
    const uint32_t inc = ms::wave_inclusive_scan(t, lane);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t before = *s_carry + inc - t, all = 0;
    for (uint32_t k = 0; k < kThreads / kWave; ++k) {
      before += k < w ? s_w[k] : 0u;
      all += s_w[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < count) dst[i0 + k] = before;
      before += v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) *s_carry += all;
    __syncthreads();
  }
  return *s_carry;
}

// End of a round's bookkeeping (one workgroup): records the edge count,
// moves the base (up to the near bucket's lower edge, or to the least
// pending distance in a jump round), clears the next round's counters and
// writes the next round's splitters.  Every thread of the workgroup calls it.
__device__ __forceinline__ void finish_round(State* st, uint32_t edges,
                                             const uint32_t* offsets, uint32_t nb,
                                             uint32_t par, uint32_t* spl, uint32_t delta,
                                             uint32_t* s_base) {
  if (threadIdx.x == 0) {
    st->edges = edges;
    st->relaxed += edges;
    const Near nr = near_bucket(offsets, nb);
    uint32_t base = st->base;
    if (nr.jump) {
      if (st->far_min[par] != kInf) base = st->far_min[par];
    } else {
      const uint64_t b = (uint64_t)base + (uint64_t)nr.j * delta;
      base = b > kDistMax ? kDistMax : (uint32_t)b;
    }
    st->base = base;
    st->count[par ^ 1u] = 0u;  // the next round appends there
    st->far_min[par ^ 1u] = kInf;
    *s_base = base;
  }
  __syncthreads();
  write_splitters(spl, nb, *s_base, delta);
}

// The scan of the per-workgroup degree sums as a kernel of its own (one
// workgroup), for rounds with more filter workgroups than the relaxation
// kernel scans in LDS.
__global__ void __launch_bounds__(kThreads)
sssp_scan_kernel(uint32_t* __restrict__ partial, uint32_t nblocks, State* st, uint32_t* spl,
                 uint32_t nb, uint32_t delta, const uint32_t* __restrict__ offsets, uint32_t par) {
  __shared__ uint32_t s_w[kThreads / kWave];
  __shared__ uint32_t s_carry, s_base;
  const uint32_t total = group_scan_sums(partial, nblocks, partial, s_w, &s_carry);
  finish_round(st, total, offsets, nb, par, spl, delta, &s_base);
}

// First-edge index of entry i in this round: its workgroup's scanned degree
// sum plus its prefix inside the workgroup.
__device__ __forceinline__ uint32_t first_edge(const uint32_t* loc, const uint32_t* partial,
                                               uint32_t i) {
  return partial[i / kBlockItems] + loc[i];
}

// Last near entry whose first-edge index is <= e, searched in global memory
// over [lo, hi) (entry lo's first edge is <= e).
__device__ __forceinline__ uint32_t entry_of(const uint32_t* loc, const uint32_t* partial,
                                             uint32_t lo, uint32_t hi, uint32_t e) {
  uint32_t len = hi - lo;
  while (len > 0) {  // first entry whose first-edge index exceeds e
    const uint32_t half = len >> 1;
    if (first_edge(loc, partial, lo + half) <= e) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo - 1;
}

// Edge-parallel relaxation of the near bucket.  Edge e of the round belongs
// to the last near entry whose first-edge index is <= e (entries with no
// edges share their successor's index and are passed over).  A workgroup
// takes 2048 consecutive edges at a time: two global searches bound the
// entries they belong to, whose first-edge indices are staged in LDS (when
// they fit) for the per-edge searches.  A relaxation first compares with a
// plain load of the distance, which can only be larger than the current
// value (distances only decrease), so skipping the atomic when it is not
// larger loses nothing.  Improvements are appended with one atomic per
// workgroup and chunk.
template <bool FUSED>
__global__ void __launch_bounds__(kThreads)
sssp_relax_kernel(const uint32_t* __restrict__ ok, const uint32_t* __restrict__ ov,
                  const uint64_t* __restrict__ row, const uint32_t* __restrict__ col,
                  const uint32_t* __restrict__ wt, uint32_t nv, uint32_t* dist, State* st,
                  const uint32_t* __restrict__ loc, const uint32_t* __restrict__ partial,
                  uint32_t nblocks, uint32_t* pk, uint32_t* pv, uint32_t cap,
                  const uint32_t* __restrict__ offsets, uint32_t nb, uint32_t par,
                  uint32_t* spl, uint32_t delta) {
  __shared__ uint32_t s_eoff[kChunk];
  __shared__ uint32_t s_part[FUSED ? kFusedSums : 1];
  __shared__ uint32_t s_rng[2];
  __shared__ uint32_t s_w[kThreads / kWave];
  __shared__ uint32_t s_base, s_carry;
  uint64_t edges;
  if (FUSED) {
    // Every workgroup scans the (few) per-workgroup degree sums into LDS;
    // workgroup 0 also does the round's bookkeeping.
    edges = group_scan_sums(partial, nblocks, s_part, s_w, &s_carry);
    if (blockIdx.x == 0) finish_round(st, (uint32_t)edges, offsets, nb, par, spl, delta, &s_base);
  } else {
    edges = st->edges;
  }
  const uint32_t* part = FUSED ? s_part : partial;  // scanned sums
  const Near nr = near_bucket(offsets, nb);
  const uint32_t near_lo = nr.lo, near_hi = nr.hi;
  for (uint64_t c0 = (uint64_t)blockIdx.x * kChunk; c0 < edges;
       c0 += (uint64_t)gridDim.x * kChunk) {
    const uint64_t c1 = c0 + kChunk < edges ? c0 + kChunk : edges;
    if (threadIdx.x == 0) {
      s_rng[0] = entry_of(loc, part, near_lo, near_hi, (uint32_t)c0);
      s_rng[1] = entry_of(loc, part, near_lo, near_hi, (uint32_t)(c1 - 1));
    }
    __syncthreads();
    const uint32_t i0 = s_rng[0], i1 = s_rng[1];
    const uint32_t cnt = i1 - i0 + 1;
    const bool staged = cnt <= kChunk;
    if (staged)
      for (uint32_t k = threadIdx.x; k < cnt; k += kThreads)
        s_eoff[k] = first_edge(loc, part, i0 + k);
    __syncthreads();
    uint32_t nd[kEdgePer], u[kEdgePer], nput = 0;
    bool put[kEdgePer];
#pragma unroll
    for (int k = 0; k < kEdgePer; ++k) {
      const uint64_t e64 = c0 + threadIdx.x + (uint64_t)k * kThreads;
      put[k] = false;
      nd[k] = 0;
      u[k] = 0;
      if (e64 < c1) {
        const uint32_t e = (uint32_t)e64;
        uint32_t item, first;
        if (staged) {
          uint32_t lo = 0, len = cnt;  // s_eoff[0] <= e
          while (len > 0) {
            const uint32_t half = len >> 1;
            if (s_eoff[lo + half] <= e) {
              lo += half + 1;
              len -= half + 1;
            } else {
              len = half;
            }
          }
          item = i0 + lo - 1;
          first = s_eoff[lo - 1];
        } else {
          item = entry_of(loc, part, i0, i1 + 1, e);
          first = first_edge(loc, part, item);
        }
        const uint32_t v = ov[item];
        const uint64_t ge = row[v] + (e - first);
        const uint32_t t = col[ge];
        if (t < nv) {
          const uint32_t cand = sat_add(ok[item], wt[ge]);
          if (cand < dist[t]) put[k] = atomicMin(&dist[t], cand) > cand;
          nd[k] = cand;
          u[k] = t;
        } else {
          st->bad_edge = 1u;
        }
      }
      nput += put[k] ? 1u : 0u;
    }
    uint32_t slot = group_reserve(nput, &st->count[par], &st->pushes, s_w, &s_base);
#pragma unroll
    for (int k = 0; k < kEdgePer; ++k)
      if (put[k]) put_entry(slot++, nd[k], u[k], st, pk, pv, cap);
    // group_reserve ends with a barrier: s_rng and s_eoff are free again
  }
}

}  // namespace

extern "C" {

size_t ms_sssp_workspace_size(uint32_t nv, uint64_t ne, uint32_t num_buckets) {
  if (nv == 0 || num_buckets < 2 || num_buckets > 256) return 0;
  const uint64_t cap = (uint64_t)nv + ne;
  if (cap >= 0xFFFFFFFFull) return 0;
  const size_t ms_ws = ms_workspace_size(MS_OP_PAIRS, (size_t)cap, num_buckets, 0, nullptr);
  if (ms_ws == 0) return 0;
  const size_t nblk = (cap + kBlockItems - 1) / kBlockItems;
  return align_up(sizeof(State)) + align_up(256 * 4) + align_up(257 * 4) +
         5 * align_up(cap * 4) + align_up(nblk * 4) + align_up(ms_ws);
}

ms_status ms_sssp(const uint64_t* d_row, const uint32_t* d_col, const uint32_t* d_wt,
                  uint32_t nv, uint64_t ne, uint32_t source, uint32_t delta,
                  uint32_t num_buckets, uint32_t* d_dist, void* d_ws, size_t ws_bytes,
                  ms_sssp_stats* stats, void* stream) {
  if (!d_row || !d_dist || nv == 0 || source >= nv || delta == 0) return MS_ERR_INVALID_ARG;
  if (ne > 0 && (!d_col || !d_wt)) return MS_ERR_INVALID_ARG;
  if (num_buckets < 2 || num_buckets > 256) return MS_ERR_INVALID_ARG;
  const uint64_t cap64 = (uint64_t)nv + ne;
  if (cap64 >= 0xFFFFFFFFull) return MS_ERR_INVALID_ARG;
  const size_t need = ms_sssp_workspace_size(nv, ne, num_buckets);
  if (!d_ws || ws_bytes < need) return MS_ERR_WORKSPACE;
  const uint32_t cap = (uint32_t)cap64;
  const uint32_t nb = num_buckets;
  hipStream_t s = (hipStream_t)stream;

  char* p = (char*)d_ws;
  State* st = (State*)p;
  p += align_up(sizeof(State));
  uint32_t* spl = (uint32_t*)p;
  p += align_up(256 * 4);
  uint32_t* offsets = (uint32_t*)p;
  p += align_up(257 * 4);
  uint32_t* pk = (uint32_t*)p;
  p += align_up((size_t)cap * 4);
  uint32_t* pv = (uint32_t*)p;
  p += align_up((size_t)cap * 4);
  uint32_t* ok = (uint32_t*)p;
  p += align_up((size_t)cap * 4);
  uint32_t* ov = (uint32_t*)p;
  p += align_up((size_t)cap * 4);
  uint32_t* deg = (uint32_t*)p;
  p += align_up((size_t)cap * 4);
  uint32_t* partial = (uint32_t*)p;
  p += align_up(((size_t)cap + kBlockItems - 1) / kBlockItems * 4);
  void* ms_ws = p;
  const size_t ms_ws_bytes = ws_bytes - (size_t)(p - (char*)d_ws);

  const uint64_t want = ((uint64_t)nv + kThreads - 1) / kThreads;
  const uint32_t init_blocks = want < 4096 ? (uint32_t)want : 4096u;
  hipLaunchKernelGGL(sssp_init_kernel, dim3(init_blocks), dim3(kThreads), 0, s, d_dist, nv,
                     source, pk, pv, st, spl, nb, delta);
  if (hipGetLastError() != hipSuccess) return MS_ERR_HIP;

  ms_sssp_stats acc;
  memset(&acc, 0, sizeof(acc));
  const ms_bucket_fn fn = {MS_BUCKET_SPLITTERS, 0u, 0u, 0u, spl, nullptr};
  // Each round either lowers some distance, shrinks the pending list or
  // jumps the base; this bound only guards against a broken invariant.
  const uint64_t max_rounds = 4 * cap64 + 64;
  uint32_t n = 1;
  while (n > 0) {
    if (acc.rounds >= max_rounds) return MS_ERR_TIMEOUT;
    ms_status rc = ms_pairs(pk, pv, ok, ov, offsets, n, nb, &fn, ms_ws, ms_ws_bytes, nullptr, s);
    if (rc != MS_OK) return rc;
    const uint32_t nblocks = (uint32_t)(((uint64_t)n + kBlockItems - 1) / kBlockItems);
    const uint32_t par = (uint32_t)(acc.rounds & 1u);
    hipLaunchKernelGGL(sssp_filter_kernel, dim3(nblocks), dim3(kThreads), 0, s, ok, ov, n, d_row,
                       d_dist, st, pk, pv, cap, deg, partial, offsets, nb, par);
    if (nblocks <= kFusedSums) {
      hipLaunchKernelGGL(sssp_relax_kernel<true>, dim3(kExpandBlocks), dim3(kThreads), 0, s, ok,
                         ov, d_row, d_col, d_wt, nv, d_dist, st, deg, partial, nblocks, pk, pv,
                         cap, offsets, nb, par, spl, delta);
    } else {
      hipLaunchKernelGGL(sssp_scan_kernel, dim3(1), dim3(kThreads), 0, s, partial, nblocks, st,
                         spl, nb, delta, offsets, par);
      hipLaunchKernelGGL(sssp_relax_kernel<false>, dim3(kExpandBlocks), dim3(kThreads), 0, s, ok,
                         ov, d_row, d_col, d_wt, nv, d_dist, st, deg, partial, nblocks, pk, pv,
                         cap, offsets, nb, par, spl, delta);
    }
    if (hipGetLastError() != hipSuccess) return MS_ERR_HIP;
    uint32_t h[4];  // count[0], count[1], overflow, bad_edge
    if (hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return MS_ERR_HIP;
    if (h[2]) return MS_ERR_WORKSPACE;  // cannot happen: the list holds nv + ne
    if (h[3]) return MS_ERR_INVALID_ARG;  // an edge names a vertex >= nv
    acc.rounds += 1;
    acc.items_split += n;
    if (n > acc.max_pending) acc.max_pending = n;
    n = h[par];
  }
  State hs;
  if (hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return MS_ERR_HIP;
  acc.edges_relaxed = hs.relaxed;
  acc.pushes = hs.pushes;
  if (stats) *stats = acc;
  return MS_OK;
}

}  // extern "C"
