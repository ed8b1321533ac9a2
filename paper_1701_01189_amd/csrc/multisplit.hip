// Host dispatch and C ABI of the gfx950 multisplit library.
//
// Implements include/multisplit.h: argument validation (before any HIP call),
// work planning (tile and chunk sizes, the number of subproblems L0 of
// Section 4.4), workspace carving and the stream-ordered launch sequence
// pre-scan -> scan -> post-scan of Section 4.6 (Algorithm 1).
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <mutex>

#include "multisplit.h"
#include "ms_aux_kernels.hpp"
#include "ms_learned.hpp"
#include "ms_dispatch.hpp"

namespace {

using ms::BucketParams;
using ms::Plan;

constexpr uint32_t kNumCUs = 256;        // MI355X compute units
constexpr uint32_t kLdsPerCU = 160 * 1024;
constexpr size_t kWsAlign = 256;

struct Shape {
  int mode;     // ms::kBlock / kWaveMode / kDirect
  int wpb;      // wavefronts per workgroup
  int nw;       // windows per wavefront per tile
  uint32_t max_chunks;
  int hist;     // pre-scan histogram: ms::kHistBallot / kHistLanes
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Smallest b with 2^b >= m, for any 32-bit m (64-bit shifts: at m > 2^31 the
// answer is 32, which a 32-bit shift cannot represent).
uint32_t ceil_log2(uint32_t m) {
  uint32_t b = 0;
  while ((1ull << b) < (uint64_t)m) ++b;
  return b;
}

bool shape_supported(const Shape& s) { return ms::post_shape_supported(s.mode, s.wpb, s.nw); }

constexpr size_t kLdsPerWorkgroup = 160 * 1024;  // gfx950: all of a CU's LDS

// Static LDS of one post-scan workgroup (mirrors postscan_kernel's arrays).
size_t post_lds_bytes(const Shape& s, uint32_t m, int kind, bool kv) {
  const bool small = m <= 64;
  const bool tables = kind == MS_BUCKET_SPLITTERS || kind == MS_BUCKET_LEARNED;
  const bool reorder = s.mode != ms::kDirect;
  const size_t wpg = s.mode == ms::kBlock ? (size_t)s.wpb : 1;
  const size_t gpb = (size_t)s.wpb / wpg;
  const size_t T = wpg * (size_t)s.nw * ms::kWave;
  const size_t slot = small ? 8 : (4 + (tables ? 1 : 0));
  size_t b = tables ? sizeof(ms::BucketLds) : 4;
  b += (size_t)s.wpb * (small ? ms::kWave : ms::kCntStride) * 4;
  b += small ? 4 : gpb * ms::kMaxBuckets * 4;
  b += (reorder && !small) ? gpb * ms::kMaxBuckets * (kv ? 8 : 4) : 8;
  b += reorder ? (gpb * T * slot + 7) / 8 * 8 : 8;
  b += (reorder && kv) ? gpb * T * 4 : 4;
  b += (size_t)s.wpb * 4;
  return b;
}

// Default: block-level reordering (BMS).  Tile shapes measured on MI355X
// (2^28 keys and pairs, m = 2 .. 256, back-to-back calls):
//  * key-only up to 4 buckets: 4 wavefronts x 16 windows; up to 64 buckets:
//    8 x 8 (more resident wavefronts, same 4096-element tile);
//  * key-value up to 64 buckets: 16 x 8 from 2^26 pairs on (8192-element
//    tiles: longer bucket runs per tile at the scatter), 8 x 8 below (with
//    one 16-wavefront workgroup per compute unit a smaller input gives each
//    workgroup too few tiles);
//  * above 64 buckets, for bucket functions computed in registers, 16 x 16
//    from 2^26 elements on and 16 x 8 below: a bucket's run per tile is T/m
//    elements, and the partial cache lines at the ends of the runs cost
//    about 5000 us x m/T at 2^28 keys (m = 256: 906, 762 and 667 us for
//    T = 4096, 8192 and 16384); 8 x 8 for bucket functions that search LDS
//    tables (their extra registers make the larger tiles slower).
// The paper's own defaults are 8 warps x 4 windows of 32 (Section 6,
// "Parameters").  With wave-level or no reordering the default is 8 x 8
// (4 x 16 for wave level at m <= 64).
int resolve_shape(const ms_options* opt, size_t n, uint32_t m, int kind, bool kv, Shape* s) {
  const bool table_kind = kind == MS_BUCKET_SPLITTERS || kind == MS_BUCKET_LEARNED;
  s->mode = ms::kBlock;
  if (opt) {
    if (opt->reorder < 0 || opt->reorder > MS_REORDER_NONE) return MS_ERR_INVALID_ARG;
    if (opt->reorder == MS_REORDER_WAVE) s->mode = ms::kWaveMode;
    if (opt->reorder == MS_REORDER_NONE) s->mode = ms::kDirect;
  }
  if (s->mode == ms::kBlock) {
    if (m <= 64) {
      const bool big_kv = kv && n >= ((size_t)1 << 26);
      s->wpb = big_kv ? 16 : (m <= 4 && !kv ? 4 : 8);
      s->nw = big_kv ? 8 : (m <= 4 && !kv ? 16 : 8);
    } else {
      s->wpb = table_kind ? 8 : 16;
      s->nw = (!table_kind && n >= ((size_t)1 << 26)) ? 16 : 8;
    }
  } else {
    s->wpb = (s->mode == ms::kWaveMode && m <= 64) ? 4 : 8;
    s->nw = (s->mode == ms::kWaveMode && m <= 64) ? 16 : 8;
  }
  s->max_chunks = 0;
  int prescan = MS_PRESCAN_AUTO;
  if (opt) {
    if (opt->waves_per_block) s->wpb = opt->waves_per_block;
    if (opt->items_per_lane) s->nw = opt->items_per_lane;
    if (opt->max_chunks < 0) return MS_ERR_INVALID_ARG;
    s->max_chunks = (uint32_t)opt->max_chunks;
    if (opt->prescan < MS_PRESCAN_AUTO || opt->prescan > MS_PRESCAN_LANES) return MS_ERR_INVALID_ARG;
    prescan = opt->prescan;
  }
  // Lane counters need a chunk shared by a workgroup (block reordering).
  if (prescan == MS_PRESCAN_LANES && s->mode != ms::kBlock) return MS_ERR_UNSUPPORTED;
  s->hist = (prescan == MS_PRESCAN_BALLOT || s->mode != ms::kBlock) ? ms::kHistBallot
                                                                     : ms::kHistLanes;
  if (!shape_supported(*s)) return MS_ERR_UNSUPPORTED;
  // a tile whose buffers do not fit in LDS (16 x 16 key-value up to 64 buckets)
  if (post_lds_bytes(*s, m, kind, kv) > kLdsPerWorkgroup) return MS_ERR_UNSUPPORTED;
  return MS_OK;
}

// Chunks (columns of H) at most: bounds the workspace.
constexpr uint32_t kMaxChunks = 4096;
// The pre-scan runs one 8-wavefront workgroup per chunk: with at least four
// per compute unit it keeps 32 wavefronts per unit streaming.
constexpr uint32_t kMinChunks = 4 * kNumCUs;

// Subproblems: chunks of consecutive tiles (Section 4.4: few first-level
// subproblems, large local ones).  Their number is a whole multiple of the
// post-scan groups resident at once (`groups`; 0 if unknown), at least
// `min_chunks` (kMinChunks unless the caller asks for more), so that every
// round of post-scan workgroups is a full one.
Plan make_plan(size_t n, uint32_t m, const Shape& s, uint32_t groups,
               uint32_t min_chunks = kMinChunks) {
  Plan p;
  p.n = (uint32_t)n;
  p.m = m;
  int wpg = s.mode == ms::kBlock ? s.wpb : 1;
  p.tile = (uint32_t)(wpg * s.nw * ms::kWave);
  uint64_t tiles = (n + p.tile - 1) / p.tile;
  uint32_t cap = kMaxChunks;
  if (s.max_chunks) {
    cap = s.max_chunks;
  } else if (groups) {
    cap = groups * ((min_chunks + groups - 1) / groups);
  }
  if (cap > kMaxChunks) cap = kMaxChunks;
  uint64_t L0 = tiles < cap ? tiles : cap;
  if (L0 == 0) L0 = 1;
  uint64_t tpc = (tiles + L0 - 1) / L0;
  if (tpc == 0) tpc = 1;
  // A chunk's length is a 32-bit count: near n = 2^32 a forced small chunk
  // count gets one more chunk rather than a length that wraps.
  const uint64_t max_tpc = 0xFFFFFFFFull / p.tile;
  if (tpc > max_tpc) tpc = max_tpc;
  L0 = (tiles + tpc - 1) / tpc;
  if (L0 == 0) L0 = 1;
  p.L0 = (uint32_t)L0;
  p.chunk = (uint32_t)(tpc * p.tile);
  p.h_raw = 0;
  p.nt_lines = 0;
  return p;
}

// Workspace: [bucket totals (256) | spare offsets (257)] then H (m x L0).
constexpr size_t kWsHeader = ((ms::kMaxBuckets + ms::kMaxBuckets + 1) * 4 + kWsAlign - 1) / kWsAlign * kWsAlign;

size_t ms_ws_bytes(const Plan& p) {
  return kWsHeader + align_up((size_t)p.m * p.L0 * 4, kWsAlign);
}

struct Workspace {
  uint32_t* totals;
  uint32_t* H;
};

Workspace carve(void* ws, const Plan& p) {
  Workspace w;
  char* b = (char*)ws;
  w.totals = (uint32_t*)b;
  w.H = (uint32_t*)(b + kWsHeader);
  return w;
}

// Granlund-Montgomery constants for floor(k / d), 32-bit unsigned.
void div_magic(uint32_t d, uint32_t* magic, uint32_t* sh1, uint32_t* sh2) {
  uint32_t l = ceil_log2(d);
  unsigned __int128 num = ((unsigned __int128)1 << 32) * (((unsigned __int128)1 << l) - d);
  *magic = (uint32_t)(num / d + 1);
  *sh1 = l < 1 ? l : 1;
  *sh2 = l >= 1 ? l - 1 : 0;
}

int validate_fn(const ms_bucket_fn* fn, uint32_t m) {
  if (!fn) return MS_ERR_INVALID_ARG;
  switch (fn->kind) {
    case MS_BUCKET_SHIFT_MASK:
      if (fn->shift > 31) return MS_ERR_INVALID_ARG;
      if (fn->mask > m - 1) return MS_ERR_BUCKET_RANGE;
      return MS_OK;
    case MS_BUCKET_DIV:
      if (fn->divisor == 0) return MS_ERR_INVALID_ARG;
      if (0xFFFFFFFFu / fn->divisor > m - 1) return MS_ERR_BUCKET_RANGE;
      return MS_OK;
    case MS_BUCKET_SPLITTERS:
      if (m > 1 && !fn->splitters) return MS_ERR_INVALID_ARG;
      return MS_OK;
    case MS_BUCKET_LEARNED:
      if ((m > 1 && !fn->splitters) || !fn->model) return MS_ERR_INVALID_ARG;
      return MS_OK;
    default:
      return MS_ERR_INVALID_ARG;
  }
}

BucketParams make_params(const ms_bucket_fn* fn, uint32_t m, uint64_t* mispredicts,
                         uint32_t div_mask = 0xFFFFFFFFu) {
  BucketParams bp;
  memset(&bp, 0, sizeof(bp));
  bp.m = m;
  bp.shift = fn->shift;
  bp.mask = fn->mask;
  if (fn->kind == MS_BUCKET_DIV) {
    div_magic(fn->divisor, &bp.magic, &bp.sh1, &bp.sh2);
    bp.mask = div_mask;  // the quotient's kept bits (all for a plain delta bucket)
  }
  bp.splitters = fn->splitters;
  bp.model = fn->model;
  bp.mispredicts = (unsigned long long*)mispredicts;
  return bp;
}

bool overlaps(const void* a, const void* b, size_t bytes) {
  if (!a || !b) return false;
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

hipError_t pre_by_kind(int kind, const ms::PreArgs& a, int bits) {
  switch (kind) {
    case MS_BUCKET_SHIFT_MASK: return ms::pre_shift_mask(a, bits);
    case MS_BUCKET_DIV: return ms::pre_div(a, bits);
    case MS_BUCKET_SPLITTERS: return ms::pre_splitters(a, bits);
    default: return ms::pre_learned(a, bits);
  }
}

// Post-scan kind: a table-search kind whose ids the pre-scan keeps runs the
// post-scan that only reads them.
constexpr int kPostKeptIds = ms::kKeptIds;

hipError_t post_by_kind(int kind, const ms::PostArgs& a, int bits) {
  switch (kind) {
    case MS_BUCKET_SHIFT_MASK: return ms::post_shift_mask(a, bits);
    case MS_BUCKET_DIV: return ms::post_div(a, bits);
    case MS_BUCKET_SPLITTERS: return ms::post_splitters(a, bits);
    case kPostKeptIds: return ms::post_kept_ids(a, bits);
    default: return ms::post_learned(a, bits);
  }
}

hipError_t record(const ms_options* opt, int i, hipStream_t st) {
  if (opt && opt->stage_events && opt->stage_events[i])
    return hipEventRecord((hipEvent_t)opt->stage_events[i], st);
  return hipSuccess;
}

hipError_t fill(uint32_t* p, uint32_t n, uint32_t v, hipStream_t st) {
  if (!p || !n) return hipSuccess;
  hipLaunchKernelGGL(ms::fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched multisplit: shape, workspace
// ---------------------------------------------------------------------------
struct BatchShape {
  int wpb, nw;
  uint32_t tile, claim, spin_limit, never_ready;
};

int resolve_batch_shape(const ms_options* opt, BatchShape* b) {
  b->wpb = 8;
  b->nw = 8;
  b->claim = 16;
  b->spin_limit = 1u << 22;
  b->never_ready = 0;
  if (opt) {
    if (opt->waves_per_block) b->wpb = opt->waves_per_block;
    if (opt->items_per_lane) b->nw = opt->items_per_lane;
    if (opt->batch_claim) b->claim = opt->batch_claim;
    if (opt->spin_limit) b->spin_limit = opt->spin_limit;
    b->never_ready = opt->test_flags & 1u;
    if (opt->reorder != MS_REORDER_AUTO && opt->reorder != MS_REORDER_BLOCK) return MS_ERR_UNSUPPORTED;
  }
  if (b->claim > (uint32_t)ms::kMaxClaim) return MS_ERR_INVALID_ARG;
  if (!ms::batched_shape_supported(b->wpb, b->nw)) return MS_ERR_UNSUPPORTED;
  b->tile = (uint32_t)(b->wpb * b->nw * ms::kWave);
  return MS_OK;
}

struct BatchWorkspace {
  uint32_t* ctl;
  uint32_t* tile_start;
  uint4* tile_info;
  uint32_t* done;
  uint32_t* ready;
  uint32_t* offsets;
  uint32_t* H;
};

// [ctl: 2 words | tile_start: num+1 | tile_info: 4 words per tile | done: num |
//  ready: num | spare offsets: num*(m+1) | H: m x tiles words], with
// tiles = total/tile + num bounding the number of tiles.
size_t batch_layout(size_t total, uint32_t m, uint32_t num, const BatchShape& bs,
                    BatchWorkspace* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes, kWsAlign);
    return o;
  };
  size_t o_ctl = take(64);
  size_t o_ts = take(((size_t)num + 1) * 4);
  size_t tiles = (total + bs.tile - 1) / bs.tile + num;
  size_t o_ti = take(tiles * 16);
  size_t o_done = take((size_t)num * 4);
  size_t o_ready = take((size_t)num * 4);
  size_t o_off = take((size_t)num * (m + 1) * 4);
  size_t o_h = take((size_t)m * tiles * 4);
  if (w && base) {
    w->ctl = (uint32_t*)(base + o_ctl);
    w->tile_start = (uint32_t*)(base + o_ts);
    w->tile_info = (uint4*)(base + o_ti);
    w->done = (uint32_t*)(base + o_done);
    w->ready = (uint32_t*)(base + o_ready);
    w->offsets = (uint32_t*)(base + o_off);
    w->H = (uint32_t*)(base + o_h);
  }
  return off;
}

BatchWorkspace carve_batch(void* ws, size_t total, uint32_t m, uint32_t num, const BatchShape& bs) {
  BatchWorkspace w;
  batch_layout(total, m, num, bs, &w, (char*)ws);
  return w;
}

// Compute units of the current device (asked once per device).
uint32_t device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return kNumCUs;
  if (cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
      c = (int)kNumCUs;
    cus[dev] = c;
  }
  return (uint32_t)cus[dev];
}

// Post-scan groups of this shape resident at once on the device (0 if the
// runtime cannot tell: the plan then takes the upper bound).
uint32_t resident_groups(int kind, int bits, bool kv, const Shape& s) {
  int occ = 0;
  ms::PostArgs q;
  memset(&q, 0, sizeof(q));
  q.mode = s.mode;
  q.wpb = s.wpb;
  q.nw = s.nw;
  q.kv = kv;
  q.occupancy = &occ;
  if (post_by_kind(kind, q, bits) != hipSuccess || occ < 1) return 0;
  const int wpg = s.mode == ms::kBlock ? s.wpb : 1;
  return device_cus() * (uint32_t)occ * (uint32_t)(s.wpb / wpg);
}

constexpr size_t kRawH = 4096;

// Whole output lines stored nontemporally.  Measured on MI355X: such lines then do not sit dirty in
// the caches for the next pass over the input to write back (2^28 keys,
// m = 32: pre-scan 265 -> 241 us, whole call +3 %; 2^25 pairs +9 %), but
// with 16-wavefront tiles on large inputs the post-scan loses more than the
// pre-scan gains (2^28 pairs, 16 x 8: -2 to -8 %), and inputs that stay in
// the caches gain nothing.
constexpr size_t kNtMin = (size_t)1 << 22;
bool nt_lines(size_t n, uint32_t m, bool kv, const Shape& s) {
  if (n < kNtMin) return false;
  // Above 64 buckets the runs are short and only key-value tiles gain
  // (2^28 pairs, m = 256: 164.6 -> 170.5 Gpairs/s, radix sort 41.1 -> 42.5;
  // keys m = 256: 281.0 -> 276.6 Gkeys/s); key-only tiles there do not
  // carry the whole-line bounds at all.
  if (m > 64) return kv;
  return !(s.wpb > 8 && n > ((size_t)1 << 26));
}

// The three stages for one multisplit on already validated arguments.
ms_status run_multisplit(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo,
                         uint32_t* offsets, size_t n, uint32_t m, const ms_bucket_fn* fn,
                         void* ws, const Shape& s, const ms_options* opt, hipStream_t st,
                         uint32_t div_mask = 0xFFFFFFFFu) {
  const bool kv = vi != nullptr;
  if (n == 0) {
    if (fill(offsets, m + 1, 0, st) != hipSuccess) return MS_ERR_HIP;
    return MS_OK;
  }
  const int bits = (int)ceil_log2(m);
  // Bucket ids kept by the pre-scan (table-search kinds, on request): the
  // last n bytes of the workspace.
  uint8_t* ids = nullptr;
  if (opt && opt->keep_bucket_ids && m <= (uint32_t)ms::kMaxBuckets &&
      (fn->kind == MS_BUCKET_SPLITTERS || fn->kind == MS_BUCKET_LEARNED)) {
    const size_t total = ms_workspace_size(kv ? MS_OP_PAIRS : MS_OP_KEYS, n, m, 0, opt);
    ids = (uint8_t*)ws + (total - align_up(n, kWsAlign));
  }
  const int post_kind = ids ? kPostKeptIds : fn->kind;
  // Block-level tiles up to 64 buckets (key-value ones of at most 8
  // wavefronts): 4096 chunks.  A chunk's runs per bucket are then shorter
  // and the write fronts of the resident workgroups closer together in each
  // bucket's range; measured at 2^28 keys, m = 32: post-scan 476 -> 457 us,
  // whole call 359 -> 365 Gkeys/s; m = 8: 389 -> 399; 2^25 pairs, m = 32,
  // 8 x 8: 233 -> 247 Gpairs/s.  16-wavefront key-value tiles (2^28 pairs,
  // m = 32: 216 -> 211) and more buckets do not gain.
  const uint32_t min_chunks =
      (m <= 64 && s.mode == ms::kBlock && (!kv || s.wpb <= 8)) ? kMaxChunks : kMinChunks;
  Plan p = make_plan(n, m, s, resident_groups(post_kind, bits, kv, s), min_chunks);
  Workspace w = carve(ws, p);
  BucketParams bp = make_params(fn, m, opt ? opt->d_mispredicts : nullptr, div_mask);
  if (record(opt, 0, st) != hipSuccess) return MS_ERR_HIP;
  ms::PreArgs pa{ki, p, bp, w.H, s.mode, s.hist, st, ids};
  if (pre_by_kind(fn->kind, pa, bits) != hipSuccess) return MS_ERR_HIP;
  if (record(opt, 1, st) != hipSuccess) return MS_ERR_HIP;
  // A small H (at most kRawH words, block-level reordering, up to 64
  // buckets) is summed by every post-scan workgroup itself: one launch less
  // for inputs that take microseconds.
  p.h_raw = (s.mode == ms::kBlock && m <= 64 && (size_t)m * p.L0 <= kRawH) ? 1u : 0u;
  p.nt_lines = nt_lines(n, m, kv, s) ? 1u : 0u;
  if (!p.h_raw) {
    hipLaunchKernelGGL(ms::scan_rows_kernel, dim3(m), dim3(ms::kScanThreads), 0, st, w.H, p.L0,
                       w.totals);
    if (hipGetLastError() != hipSuccess) return MS_ERR_HIP;
  }
  if (record(opt, 2, st) != hipSuccess) return MS_ERR_HIP;
  // offsets are written by workgroup 0 of the post-scan; a NULL offsets
  // pointer is redirected to the spare words after the bucket totals.
  uint32_t* off = offsets ? offsets : w.totals + ms::kMaxBuckets;
  ms::PostArgs qa{ki, vi, ko, vo, w.H, w.totals, off, p, bp, s.mode, s.wpb, s.nw, kv, st, nullptr,
                  ids};
  if (post_by_kind(post_kind, qa, bits) != hipSuccess) return MS_ERR_HIP;
  if (record(opt, 3, st) != hipSuccess) return MS_ERR_HIP;
  return MS_OK;
}

ms_status check_common(const uint32_t* ki, const uint32_t* vi, const uint32_t* ko,
                       const uint32_t* vo, size_t n, uint32_t m, bool kv,
                       uint32_t m_max = ms::kMaxBuckets) {
  if (m < 1 || m > m_max) return MS_ERR_INVALID_ARG;
  if (n >= 0xFFFFFFFFull) return MS_ERR_INVALID_ARG;
  if (n > 0) {
    if (!ki || !ko) return MS_ERR_INVALID_ARG;
    if (kv && (!vi || !vo)) return MS_ERR_INVALID_ARG;
    size_t bytes = n * 4;
    if (overlaps(ki, ko, bytes)) return MS_ERR_INVALID_ARG;
    if (kv && (overlaps(vi, vo, bytes) || overlaps(ko, vo, bytes) || overlaps(ki, vo, bytes) ||
               overlaps(vi, ko, bytes)))
      return MS_ERR_INVALID_ARG;
  }
  return MS_OK;
}

// ---------------------------------------------------------------------------
// More than 256 buckets (Section 6, "Performance for more than 256 buckets":
// iterated multisplits of at most 256 buckets, as radix sort does).  For
// shift/mask and delta buckets the bucket id B = f(k) < 2^16 splits into
// digits lo = B & 255 and hi = B >> 8, each itself a shift/mask or delta
// bucket function: a stable pass on lo, then a stable pass on hi, leaves the
// elements ordered by (hi, lo) = B with input order kept inside a bucket.
// The bucket starts then come from one pass over the output.
// ---------------------------------------------------------------------------
constexpr uint32_t kMaxBucketsWide = 1u << 16;

struct WidePasses {
  ms_bucket_fn lo, hi;
  uint32_t m_lo, m_hi;
  uint32_t lo_div_mask;  // delta: the quotient's low byte
};

WidePasses wide_passes(const ms_bucket_fn* fn, uint32_t m) {
  WidePasses w;
  memset(&w, 0, sizeof(w));
  w.lo = *fn;
  w.hi = *fn;
  w.m_lo = 256;
  w.m_hi = (m - 1) / 256 + 1;
  w.lo_div_mask = 0xFFFFFFFFu;
  if (fn->kind == MS_BUCKET_SHIFT_MASK) {
    w.lo.mask = fn->mask & 255u;
    if (fn->shift + 8 < 32) {
      w.hi.shift = fn->shift + 8;
      w.hi.mask = fn->mask >> 8;
    } else {  // every id has its high byte zero
      w.hi.shift = 0;
      w.hi.mask = 0;
    }
  } else {  // delta: floor(floor(k / d) / 256) = floor(k / 256d)
    w.lo_div_mask = 255u;
    const uint64_t d2 = (uint64_t)fn->divisor * 256u;
    if (d2 <= 0xFFFFFFFFull) {
      w.hi.divisor = (uint32_t)d2;
    } else {  // k / d < 256 for every key: the high byte is zero
      w.hi.kind = MS_BUCKET_SHIFT_MASK;
      w.hi.shift = 0;
      w.hi.mask = 0;
    }
  }
  return w;
}

size_t wide_ws_bytes(size_t n, uint32_t m, bool kv, const ms_options* opt) {
  size_t data = align_up(n * 4, kWsAlign) * (kv ? 2 : 1);
  size_t best = 0;
  const uint32_t ms_[2] = {256u, (m - 1) / 256 + 1};
  const int kinds[2] = {MS_BUCKET_SHIFT_MASK, MS_BUCKET_SPLITTERS};
  for (uint32_t mm : ms_)
    for (int kd : kinds) {
      Shape s;
      if (resolve_shape(opt, n, mm, kd, kv, &s) != MS_OK) return 0;
      size_t b = ms_ws_bytes(make_plan(n, mm, s, 0));
      if (b > best) best = b;
    }
  return data + best;
}

ms_status run_wide(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo,
                   uint32_t* offsets, size_t n, uint32_t m, const ms_bucket_fn* fn, void* ws,
                   const ms_options* opt, hipStream_t st) {
  if (n == 0) return fill(offsets, m + 1, 0, st) == hipSuccess ? MS_OK : MS_ERR_HIP;
  const bool kv = vi != nullptr;
  const WidePasses w = wide_passes(fn, m);
  char* b = (char*)ws;
  uint32_t* tk = (uint32_t*)b;
  b += align_up(n * 4, kWsAlign);
  uint32_t* tv = nullptr;
  if (kv) {
    tv = (uint32_t*)b;
    b += align_up(n * 4, kWsAlign);
  }
  Shape s_lo, s_hi;
  int r = resolve_shape(opt, n, w.m_lo, w.lo.kind, kv, &s_lo);
  if (r != MS_OK) return (ms_status)r;
  r = resolve_shape(opt, n, w.m_hi, w.hi.kind, kv, &s_hi);
  if (r != MS_OK) return (ms_status)r;
  ms_options o;
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  o.stage_events = nullptr;  // stages of the second pass only
  ms_status e = run_multisplit(ki, vi, tk, tv, nullptr, n, w.m_lo, &w.lo, b, s_lo, &o, st,
                               w.lo_div_mask);
  if (e != MS_OK) return e;
  if (opt) o.stage_events = opt->stage_events;
  e = run_multisplit(tk, tv, ko, vo, nullptr, n, w.m_hi, &w.hi, b, s_hi, &o, st);
  if (e != MS_OK) return e;
  if (offsets) {
    const BucketParams bp = make_params(fn, m, nullptr);
    const uint32_t blocks = (m + 1 + 255) / 256;  // one lane per bucket start
    if (fn->kind == MS_BUCKET_SHIFT_MASK)
      hipLaunchKernelGGL(ms::bucket_starts_kernel<ms::kShiftMask>, dim3(blocks), dim3(256), 0, st,
                         ko, (uint32_t)n, m, bp, offsets);
    else
      hipLaunchKernelGGL(ms::bucket_starts_kernel<ms::kDiv>, dim3(blocks), dim3(256), 0, st, ko,
                         (uint32_t)n, m, bp, offsets);
    if (hipGetLastError() != hipSuccess) return MS_ERR_HIP;
  }
  return MS_OK;
}

// ---------------------------------------------------------------------------
// Workspace of ms_pairs_noalloc: a file-scope device array.  Up to 256
// buckets a multisplit needs the bucket totals and spare offsets (a few KiB)
// plus H, m x L0 words with L0 <= kMaxChunks: at most 4 MiB whatever n.
// Every GPU the library runs on holds its own copy until the process ends.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = kWsHeader + (size_t)ms::kMaxBuckets * kMaxChunks * 4;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per device

// The array's address on the current device, asked once per device (in host
// code `scratch` itself only stands in for the symbol).
void* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> hold(g_scratch_lock);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" {

const char* ms_status_str(int status) {
  switch (status) {
    case MS_OK: return "MS_OK";
    case MS_ERR_INVALID_ARG: return "MS_ERR_INVALID_ARG";
    case MS_ERR_WORKSPACE: return "MS_ERR_WORKSPACE";
    case MS_ERR_HIP: return "MS_ERR_HIP";
    case MS_ERR_BUCKET_RANGE: return "MS_ERR_BUCKET_RANGE";
    case MS_ERR_TIMEOUT: return "MS_ERR_TIMEOUT";
    case MS_ERR_UNSUPPORTED: return "MS_ERR_UNSUPPORTED";
    default: return "MS_ERR_UNKNOWN";
  }
}

const char* ms_version(void) { return "multisplit-gfx950 0.1"; }

size_t ms_workspace_size(int op, size_t n, uint32_t m, uint32_t num_inst, const ms_options* opt) {
  (void)num_inst;
  if ((op == MS_OP_KEYS || op == MS_OP_PAIRS) && m > (uint32_t)ms::kMaxBuckets) {
    if (m > kMaxBucketsWide || n >= 0xFFFFFFFFull) return 0;
    return wide_ws_bytes(n, m, op == MS_OP_PAIRS, opt);
  }
  const bool kv_op = op == MS_OP_PAIRS || op == MS_OP_RADIX_SORT_PAIRS;
  Shape s;  // radix passes use shift/mask buckets
  const bool multisplit_op = op != MS_OP_BATCHED && op != MS_OP_LEARNED_FIT;
  if (multisplit_op && resolve_shape(opt, n, m, MS_BUCKET_SHIFT_MASK, kv_op, &s) != MS_OK)
    return 0;
  switch (op) {
    case MS_OP_KEYS:
    case MS_OP_PAIRS:
    case MS_OP_HISTOGRAM: {
      if (m < 1 || m > (uint32_t)ms::kMaxBuckets || n >= 0xFFFFFFFFull) return 0;
      // The default shape depends on the bucket kind: size for both (a
      // shape that table-search kinds cannot run is sized for the others).
      Shape t;
      const size_t ids = (op != MS_OP_HISTOGRAM && opt && opt->keep_bucket_ids)
                             ? align_up(n, kWsAlign) : 0;  // kept bucket ids, last
      const size_t a = ms_ws_bytes(make_plan(n, m, s, 0));
      if (resolve_shape(opt, n, m, MS_BUCKET_SPLITTERS, kv_op, &t) != MS_OK) return a + ids;
      const size_t b = ms_ws_bytes(make_plan(n, m, t, 0));
      return (a > b ? a : b) + ids;
    }
    case MS_OP_RADIX_SORT:
    case MS_OP_RADIX_SORT_PAIRS: {
      // m: the digit's bucket count 2^bits_per_pass
      if (n >= 0xFFFFFFFFull || m < 2 || m > (uint32_t)ms::kMaxBuckets || (m & (m - 1))) return 0;
      bool kv = op == MS_OP_RADIX_SORT_PAIRS;
      size_t data = align_up(n * 4, kWsAlign) * (kv ? 2 : 1);
      return data + ms_ws_bytes(make_plan(n, m, s, 0));
    }
    case MS_OP_BATCHED: {
      if (m < 1 || m > (uint32_t)ms::kMaxBuckets || n >= 0xFFFFFFFFull || num_inst == 0) return 0;
      BatchShape bs;
      if (resolve_batch_shape(opt, &bs) != MS_OK) return 0;
      return batch_layout(n, m, num_inst, bs, nullptr, nullptr);
    }
    case MS_OP_LEARNED_FIT: {
      // per-workgroup key ranges, then the per-leaf integer sums
      if (n == 0 || n >= 0xFFFFFFFFull) return 0;
      return align_up(2 * ms::kFitBlocks * sizeof(uint32_t), kWsAlign) +
             align_up((size_t)ms::kLeaves * ms::kFitAccWords * 8, kWsAlign);
    }
    default:
      return 0;
  }
}

ms_status ms_keys(const uint32_t* d_keys_in, uint32_t* d_keys_out, uint32_t* d_offsets, size_t n,
                  uint32_t m, const ms_bucket_fn* fn, void* d_ws, size_t ws_bytes,
                  const ms_options* opt, void* stream) {
  return ms_pairs(d_keys_in, nullptr, d_keys_out, nullptr, d_offsets, n, m, fn, d_ws, ws_bytes,
                  opt, stream);
}

ms_status ms_pairs(const uint32_t* d_keys_in, const uint32_t* d_vals_in, uint32_t* d_keys_out,
                   uint32_t* d_vals_out, uint32_t* d_offsets, size_t n, uint32_t m,
                   const ms_bucket_fn* fn, void* d_ws, size_t ws_bytes, const ms_options* opt,
                   void* stream) {
  bool kv = d_vals_in != nullptr || d_vals_out != nullptr;
  ms_status rc = check_common(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, m, kv,
                              kMaxBucketsWide);
  if (rc != MS_OK) return rc;
  int fr = validate_fn(fn, m);
  if (fr != MS_OK) return (ms_status)fr;
  if (m > (uint32_t)ms::kMaxBuckets) {
    if (fn->kind != MS_BUCKET_SHIFT_MASK && fn->kind != MS_BUCKET_DIV) return MS_ERR_UNSUPPORTED;
    if (n > 0 && (!d_ws || ws_bytes < wide_ws_bytes(n, m, kv, opt))) return MS_ERR_WORKSPACE;
    return run_wide(d_keys_in, kv ? d_vals_in : nullptr, d_keys_out, d_vals_out, d_offsets, n, m,
                    fn, d_ws, opt, (hipStream_t)stream);
  }
  Shape s;
  int sr = resolve_shape(opt, n, m, fn->kind, kv, &s);
  if (sr != MS_OK) return (ms_status)sr;
  size_t need = ms_workspace_size(kv ? MS_OP_PAIRS : MS_OP_KEYS, n, m, 0, opt);
  if (n > 0 && (!d_ws || ws_bytes < need)) return MS_ERR_WORKSPACE;
  return run_multisplit(d_keys_in, kv ? d_vals_in : nullptr, d_keys_out, d_vals_out, d_offsets,
                        n, m, fn, d_ws, s, opt, (hipStream_t)stream);
}

ms_status ms_pairs_noalloc(const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                           uint32_t* d_keys_out, uint32_t* d_vals_out, uint32_t* d_offsets,
                           size_t n, uint32_t m, const ms_bucket_fn* fn, const ms_options* opt,
                           void* stream) {
  bool kv = d_vals_in != nullptr || d_vals_out != nullptr;
  ms_status rc = check_common(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, m, kv,
                              kMaxBucketsWide);
  if (rc != MS_OK) return rc;
  int fr = validate_fn(fn, m);
  if (fr != MS_OK) return (ms_status)fr;
  // more than 256 buckets need a copy of the data: beyond the static array
  if (m > (uint32_t)ms::kMaxBuckets) return MS_ERR_WORKSPACE;
  Shape s;
  int sr = resolve_shape(opt, n, m, fn->kind, kv, &s);
  if (sr != MS_OK) return (ms_status)sr;
  ms_options plain;
  memset(&plain, 0, sizeof(plain));
  if (opt) plain = *opt;
  plain.keep_bucket_ids = 0;
  if (ms_workspace_size(kv ? MS_OP_PAIRS : MS_OP_KEYS, n, m, 0, &plain) > kScratchBytes)
    return MS_ERR_WORKSPACE;
  void* ws = scratch_on_current_device();
  if (!ws) return MS_ERR_HIP;
  ms_options o;  // (kept bucket ids would need n bytes: not in the static array)
  memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  o.keep_bucket_ids = 0;
  return run_multisplit(d_keys_in, kv ? d_vals_in : nullptr, d_keys_out, d_vals_out, d_offsets,
                        n, m, fn, ws, s, &o, (hipStream_t)stream);
}

ms_status ms_histogram(const uint32_t* d_keys, size_t n, uint32_t m, const ms_bucket_fn* fn,
                       uint32_t* d_hist, void* d_ws, size_t ws_bytes, const ms_options* opt,
                       void* stream) {
  if (m < 1 || m > (uint32_t)ms::kMaxBuckets || n >= 0xFFFFFFFFull || !d_hist)
    return MS_ERR_INVALID_ARG;
  if (n > 0) {
    if (!d_keys) return MS_ERR_INVALID_ARG;
    const char* k = (const char*)d_keys;
    const char* h = (const char*)d_hist;
    if (k < h + (size_t)m * 4 && h < k + n * 4) return MS_ERR_INVALID_ARG;  // overlap
  }
  int fr = validate_fn(fn, m);
  if (fr != MS_OK) return (ms_status)fr;
  Shape s;
  int sr = resolve_shape(opt, n, m, fn->kind, false, &s);
  if (sr != MS_OK) return (ms_status)sr;
  const size_t need = ms_workspace_size(MS_OP_HISTOGRAM, n, m, 0, opt);
  if (n > 0 && (!d_ws || ws_bytes < need)) return MS_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) return fill(d_hist, m, 0, st) == hipSuccess ? MS_OK : MS_ERR_HIP;
  // Section 7.3 names two ways to combine the subproblems' counts: store
  // them and reduce per bucket, or add them into the output with atomics.
  // The first is used: with ~2^11 subproblems, the atomic additions to each
  // bin serialise in L2 (2^25 keys, m = 32: 245 us against 25 us).  Here the
  // reduction is the row-total output of the scan kernel.
  Plan p = make_plan(n, m, s, resident_groups(fn->kind, (int)ceil_log2(m), false, s));
  Workspace w = carve(d_ws, p);
  BucketParams bp = make_params(fn, m, nullptr);
  if (record(opt, 0, st) != hipSuccess) return MS_ERR_HIP;
  ms::PreArgs pa{d_keys, p, bp, w.H, s.mode, s.hist, st};
  if (pre_by_kind(fn->kind, pa, (int)ceil_log2(m)) != hipSuccess) return MS_ERR_HIP;
  if (record(opt, 1, st) != hipSuccess) return MS_ERR_HIP;
  hipLaunchKernelGGL(ms::scan_rows_kernel, dim3(m), dim3(ms::kScanThreads), 0, st, w.H, p.L0,
                     d_hist);
  if (hipGetLastError() != hipSuccess) return MS_ERR_HIP;
  for (int e = 2; e < 4; ++e)
    if (record(opt, e, st) != hipSuccess) return MS_ERR_HIP;
  return MS_OK;
}

ms_status ms_radix_sort(const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                        uint32_t* d_keys_out, uint32_t* d_vals_out, size_t n,
                        uint32_t bits_per_pass, void* d_ws, size_t ws_bytes,
                        const ms_options* opt, void* stream) {
  bool kv = d_vals_in != nullptr || d_vals_out != nullptr;
  if (bits_per_pass < 1 || bits_per_pass > 8) return MS_ERR_INVALID_ARG;
  const uint32_t m_digit = 1u << bits_per_pass;
  ms_status rc = check_common(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, m_digit, kv);
  if (rc != MS_OK) return rc;
  Shape s;
  int sr = resolve_shape(opt, n, m_digit, MS_BUCKET_SHIFT_MASK, kv, &s);
  if (sr != MS_OK) return (ms_status)sr;
  size_t need =
      ms_workspace_size(kv ? MS_OP_RADIX_SORT_PAIRS : MS_OP_RADIX_SORT, n, m_digit, 0, opt);
  if (n > 0 && (!d_ws || ws_bytes < need)) return MS_ERR_WORKSPACE;
  if (n == 0) return MS_OK;
  hipStream_t st = (hipStream_t)stream;
  char* b = (char*)d_ws;
  uint32_t* tk = (uint32_t*)b;
  b += align_up(n * 4, kWsAlign);
  uint32_t* tv = nullptr;
  if (kv) {
    tv = (uint32_t*)b;
    b += align_up(n * 4, kWsAlign);
  }
  void* ms_ws = b;
  const uint32_t r = bits_per_pass;
  const uint32_t passes = (32 + r - 1) / r;
  // Ping-pong so that the last pass lands in the output buffers.
  const uint32_t* src_k = d_keys_in;
  const uint32_t* src_v = d_vals_in;
  bool to_out = (passes % 2) == 1;
  for (uint32_t pass = 0; pass < passes; ++pass) {
    uint32_t shift = pass * r;
    uint32_t width = (32 - shift) < r ? (32 - shift) : r;
    uint32_t m = 1u << width;
    ms_bucket_fn fn;
    memset(&fn, 0, sizeof(fn));
    fn.kind = MS_BUCKET_SHIFT_MASK;
    fn.shift = shift;
    fn.mask = m - 1;
    uint32_t* dk = to_out ? d_keys_out : tk;
    uint32_t* dv = to_out ? d_vals_out : tv;
    ms_options o;
    memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    o.stage_events = (pass == passes - 1 && opt) ? opt->stage_events : nullptr;
    ms_status e = run_multisplit(src_k, kv ? src_v : nullptr, dk, kv ? dv : nullptr, nullptr, n, m,
                                 &fn, ms_ws, s, &o, st);
    if (e != MS_OK) return e;
    src_k = dk;
    src_v = dv;
    to_out = !to_out;
  }
  return MS_OK;
}

ms_status ms_batched(const uint32_t* d_keys_in, const uint32_t* d_vals_in, uint32_t* d_keys_out,
                     uint32_t* d_vals_out, const uint64_t* d_seg, uint32_t num_inst, size_t total,
                     uint32_t m, const ms_bucket_fn* fn, uint32_t* d_offsets, void* d_ws,
                     size_t ws_bytes, const ms_options* opt, void* stream) {
  const bool kv = d_vals_in != nullptr || d_vals_out != nullptr;
  ms_status rc = check_common(d_keys_in, d_vals_in, d_keys_out, d_vals_out, total, m, kv);
  if (rc != MS_OK) return rc;
  if (num_inst == 0) return MS_OK;
  if (!d_seg) return MS_ERR_INVALID_ARG;
  int fr = validate_fn(fn, m);
  if (fr != MS_OK) return (ms_status)fr;
  BatchShape bs;
  int sr = resolve_batch_shape(opt, &bs);
  if (sr != MS_OK) return (ms_status)sr;
  const size_t need = ms_workspace_size(MS_OP_BATCHED, total, m, num_inst, opt);
  if (!d_ws || ws_bytes < need) return MS_ERR_WORKSPACE;
  BatchWorkspace w = carve_batch(d_ws, total, m, num_inst, bs);
  ms::BatchedArgs a;
  memset(&a, 0, sizeof(a));
  a.keys_in = d_keys_in;
  a.vals_in = kv ? d_vals_in : nullptr;
  a.keys_out = d_keys_out;
  a.vals_out = kv ? d_vals_out : nullptr;
  a.seg = d_seg;
  a.num = num_inst;
  a.m = m;
  a.offsets = d_offsets ? d_offsets : w.offsets;
  a.tile_start = w.tile_start;
  a.tile_info = w.tile_info;
  a.H = w.H;
  a.done = w.done;
  a.ready = w.ready;
  a.ctl = w.ctl;
  a.tile = bs.tile;
  a.claim = bs.claim;
  a.spin_limit = bs.spin_limit;
  a.never_ready = bs.never_ready;
  a.osh = total <= ((size_t)1 << 30) ? 2u : 0u;
  a.ntl = total >= kNtMin ? 1u : 0u;
  a.bp = make_params(fn, m, opt ? opt->d_mispredicts : nullptr);
  const int bits = (int)ceil_log2(m);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  switch (fn->kind) {
    case MS_BUCKET_SHIFT_MASK: e = ms::batched_shift_mask(a, bits, kv, bs.wpb, bs.nw, st); break;
    case MS_BUCKET_DIV: e = ms::batched_div(a, bits, kv, bs.wpb, bs.nw, st); break;
    case MS_BUCKET_SPLITTERS: e = ms::batched_splitters(a, bits, kv, bs.wpb, bs.nw, st); break;
    default: e = ms::batched_learned(a, bits, kv, bs.wpb, bs.nw, st); break;
  }
  return e == hipSuccess ? MS_OK : MS_ERR_HIP;
}

ms_status ms_batched_status(const void* d_ws, void* stream) {
  if (!d_ws) return MS_ERR_INVALID_ARG;
  uint32_t ctl[2] = {0, 0};
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(ctl, d_ws, sizeof(ctl), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MS_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return MS_ERR_HIP;
  return ctl[1] ? MS_ERR_TIMEOUT : MS_OK;
}

ms_status ms_learned_fit(const uint32_t* d_sample, const uint32_t* d_labels, size_t n_sample,
                         const uint32_t* d_splitters, uint32_t m, float* d_model, void* d_ws,
                         size_t ws_bytes, void* stream) {
  if (m < 1 || m > (uint32_t)ms::kMaxBuckets) return MS_ERR_INVALID_ARG;
  if (n_sample == 0 || n_sample >= 0xFFFFFFFFull) return MS_ERR_INVALID_ARG;
  if (!d_sample || !d_model || (m > 1 && !d_splitters && !d_labels)) return MS_ERR_INVALID_ARG;
  size_t need = ms_workspace_size(MS_OP_LEARNED_FIT, n_sample, m, 0, nullptr);
  if (!d_ws || ws_bytes < need) return MS_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* b = (char*)d_ws;
  ms::FitParams p;
  p.sample = d_sample;
  p.labels = d_labels;
  p.ns = (uint32_t)n_sample;
  p.splitters = m > 1 ? d_splitters : nullptr;
  p.m = m;
  p.model = d_model;
  p.range = (uint32_t*)b;
  b += align_up(2 * ms::kFitBlocks * sizeof(uint32_t), kWsAlign);
  p.acc = (unsigned long long*)b;
  dim3 B(ms::kFitThreads);
  hipLaunchKernelGGL(ms::fit_range_kernel, dim3(ms::kFitBlocks), B, 0, st, p);
  hipLaunchKernelGGL(ms::fit_root_kernel, dim3(1), B, 0, st, p);
  hipLaunchKernelGGL(ms::fit_sum_kernel<1>, dim3(ms::kFitSumBlocks), B, 0, st, p);
  hipLaunchKernelGGL(ms::fit_mean_kernel, dim3(1), B, 0, st, p);
  hipLaunchKernelGGL(ms::fit_sum_kernel<2>, dim3(ms::kFitSumBlocks), B, 0, st, p);
  hipLaunchKernelGGL(ms::fit_finish_kernel, dim3(1), B, 0, st, p);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_ERR_HIP;
}

ms_status ms_autotune(int op, const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                      uint32_t* d_keys_out, uint32_t* d_vals_out, const uint64_t* d_seg,
                      uint32_t num_inst, size_t n, uint32_t m, const ms_bucket_fn* fn,
                      void* d_ws, size_t ws_bytes, int reps, const ms_options* base,
                      ms_options* best, float* best_ms, void* stream) {
  if (!best || reps < 1 || reps > 1000) return MS_ERR_INVALID_ARG;
  struct Cand { int reorder, wpb, nw; uint32_t claim; };
  static const Cand kMulti[] = {{MS_REORDER_BLOCK, 8, 8, 0},  {MS_REORDER_BLOCK, 8, 4, 0},
                                {MS_REORDER_BLOCK, 4, 8, 0},  {MS_REORDER_BLOCK, 4, 16, 0},
                                {MS_REORDER_BLOCK, 16, 8, 0}, {MS_REORDER_BLOCK, 16, 16, 0},
                                {MS_REORDER_WAVE, 8, 8, 0},   {MS_REORDER_WAVE, 4, 16, 0},
                                {MS_REORDER_NONE, 8, 8, 0}};
  static const Cand kBatch[] = {{MS_REORDER_BLOCK, 8, 8, 4},   {MS_REORDER_BLOCK, 8, 8, 16},
                                {MS_REORDER_BLOCK, 8, 8, 32},  {MS_REORDER_BLOCK, 8, 4, 4},
                                {MS_REORDER_BLOCK, 8, 4, 16},  {MS_REORDER_BLOCK, 8, 4, 32},
                                {MS_REORDER_BLOCK, 4, 16, 16}, {MS_REORDER_BLOCK, 4, 8, 16},
                                {MS_REORDER_BLOCK, 16, 4, 16}, {MS_REORDER_BLOCK, 16, 4, 32},
                                {MS_REORDER_BLOCK, 16, 8, 16}, {MS_REORDER_BLOCK, 16, 8, 32}};
  const bool batched = op == MS_OP_BATCHED;
  const bool radix = op == MS_OP_RADIX_SORT || op == MS_OP_RADIX_SORT_PAIRS;
  if (!batched && !radix && op != MS_OP_KEYS && op != MS_OP_PAIRS) return MS_ERR_INVALID_ARG;
  const Cand* cands = batched ? kBatch : kMulti;
  const int ncand = batched ? (int)(sizeof(kBatch) / sizeof(Cand)) : (int)(sizeof(kMulti) / sizeof(Cand));
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return MS_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return MS_ERR_HIP;
  }
  // A candidate that fails (an unsupported shape, a launch error) is skipped
  // and the search goes on; the call fails only when every candidate did,
  // with the last candidate's error.
  ms_status last_err = MS_ERR_UNSUPPORTED;
  bool have = false;
  float best_t = 0.0f;
  for (int c = 0; c < ncand; ++c) {
    ms_options o;
    memset(&o, 0, sizeof(o));
    if (base) o = *base;
    o.stage_events = nullptr;
    o.reorder = cands[c].reorder;
    o.waves_per_block = cands[c].wpb;
    o.items_per_lane = cands[c].nw;
    if (batched) o.batch_claim = cands[c].claim;
    if (o.prescan == MS_PRESCAN_LANES && o.reorder != MS_REORDER_BLOCK) o.prescan = MS_PRESCAN_AUTO;
    if (c == 0 && base && (base->test_flags & 2u)) {  // test hook: the first candidate fails
      last_err = MS_ERR_UNSUPPORTED;
      continue;
    }
    o.test_flags &= ~2u;
    int wop = batched ? MS_OP_BATCHED
                      : radix ? (d_vals_in ? MS_OP_RADIX_SORT_PAIRS : MS_OP_RADIX_SORT)
                              : (d_vals_in ? MS_OP_PAIRS : MS_OP_KEYS);
    size_t need = ms_workspace_size(wop, n, radix ? (1u << m) : m, num_inst, &o);
    if (need == 0 || need > ws_bytes) continue;
    auto run = [&]() -> ms_status {
      if (batched)
        return ms_batched(d_keys_in, d_vals_in, d_keys_out, d_vals_out, d_seg, num_inst, n, m, fn,
                          nullptr, d_ws, ws_bytes, &o, stream);
      if (radix)
        return ms_radix_sort(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, m, d_ws, ws_bytes,
                             &o, stream);
      return ms_pairs(d_keys_in, d_vals_in, d_keys_out, d_vals_out, nullptr, n, m, fn, d_ws,
                      ws_bytes, &o, stream);
    };
    ms_status rc = run();  // warm-up
    if (rc != MS_OK) {
      last_err = rc;
      continue;
    }
    if (hipEventRecord(e0, st) != hipSuccess) {
      last_err = MS_ERR_HIP;
      break;
    }
    for (int r = 0; r < reps && rc == MS_OK; ++r) rc = run();
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      last_err = MS_ERR_HIP;
      break;
    }
    if (rc != MS_OK) {
      last_err = rc;
      continue;
    }
    float t = 0.0f;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      last_err = MS_ERR_HIP;
      break;
    }
    t /= (float)reps;
    if (!have || t < best_t) {
      best_t = t;
      *best = o;
      have = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (have && best_ms) *best_ms = best_t;
  // With a winner, the outputs are rewritten with it, so that they hold its
  // result whatever candidate ran last.
  if (have) {
    ms_options o = *best;
    if (batched)
      return ms_batched(d_keys_in, d_vals_in, d_keys_out, d_vals_out, d_seg, num_inst, n, m, fn,
                        nullptr, d_ws, ws_bytes, &o, stream);
    if (radix)
      return ms_radix_sort(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, m, d_ws, ws_bytes,
                           &o, stream);
    return ms_pairs(d_keys_in, d_vals_in, d_keys_out, d_vals_out, nullptr, n, m, fn, d_ws,
                    ws_bytes, &o, stream);
  }
  return last_err;
}

ms_status ms_copy_u32(uint32_t* d_dst, const uint32_t* d_src, size_t n, void* stream) {
  if (n == 0) return MS_OK;
  if (!d_dst || !d_src || overlaps(d_dst, d_src, n * 4)) return MS_ERR_INVALID_ARG;
  if (((uintptr_t)d_dst | (uintptr_t)d_src) & 15) return MS_ERR_INVALID_ARG;
  hipLaunchKernelGGL(ms::copy_u32_kernel, dim3(kNumCUs * 8), dim3(256), 0, (hipStream_t)stream,
                     d_dst, d_src, n);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_ERR_HIP;
}

}  // extern "C"
