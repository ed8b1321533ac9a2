/*
 * multisplit.h -- C ABI of the MI355X (gfx950) stable multisplit library.
 *
 * Paper: Ashkiani, Davidson, Meyer, Owens, "GPU Multisplit: an extended study
 * of a parallel algorithm" (ACM TOPC 2017).
 *
 * Multisplit (Section 3.1): permute n keys (or key-value pairs) so that
 * all elements of bucket 0 come first, then bucket 1, ..., then bucket m-1,
 * where the bucket of a key is given by a bucket identifier f.  This library
 * is always *stable*: inside a bucket the input order is kept, so the output
 * is the unique permutation of Eq. (1) (Section 4.2):
 *     p(i) = sum_{j < f(u_i)} h_j  +  #{ r < i : f(u_r) = f(u_i) }.
 * It runs the paper's three stages (Section 4.6): a pre-scan that builds the
 * bucket-major histogram matrix H (m rows, one column per subproblem), a
 * scan of H (Eq. 2), and a post-scan that ranks every element inside its
 * tile with wavefront ballots (Algorithms 2 and 3 on 64-lane wavefronts),
 * reorders the tile in LDS (Section 5.6) and scatters it.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are DEVICE pointers (HIP device memory or managed
 *     memory visible to the current device).  They are owned by the caller;
 *     the library never allocates device memory and never frees anything.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call only enqueues work on `stream` and returns without
 *     synchronising; outputs are valid once the stream has completed.
 *   - Outputs must not overlap inputs (no in-place operation).
 *   - Arguments are validated on the host before any launch; an invalid
 *     call enqueues nothing and leaves outputs untouched.
 *   - Errors: see ms_status.  MS_ERR_HIP reports a failed HIP launch.
 *   - The workspace d_ws (ws_bytes bytes, 256-byte aligned) is scratch owned
 *     by the caller; its required size comes from ms_workspace_size().  Two
 *     calls that run at the same time must not share a workspace.
 *   - Indices and offsets are uint32: n must be below 2^32.
 *   - Keys and values are 32-bit words; values are moved, never inspected.
 */
#ifndef MULTISPLIT_H
#define MULTISPLIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MS_OK = 0,
  MS_ERR_INVALID_ARG = -1, /* bad size, null pointer, m out of range, ...        */
  MS_ERR_WORKSPACE = -2,   /* ws_bytes smaller than ms_workspace_size()      */
  MS_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed     */
  MS_ERR_BUCKET_RANGE = -4,/* bucket function can produce ids >= m           */
  MS_ERR_TIMEOUT = -5,     /* a bounded device wait expired                  */
  MS_ERR_UNSUPPORTED = -6  /* valid request the library does not implement   */
} ms_status;

/* Human-readable name of a status code (static string). */
const char* ms_status_str(int status);

/*
 * Bucket identifiers (Section 6, "Bucket identification"; Section 7.1).
 *   MS_BUCKET_SHIFT_MASK  f(k) = (k >> shift) & mask.  Identity buckets and
 *                         radix digits f_p(k) = (k >> p r) & (2^r - 1) of
 *                         Section 7.1; delta buckets of width 2^s.
 *                         Requires mask <= m - 1.
 *   MS_BUCKET_DIV         f(k) = floor(k / divisor): the paper's delta
 *                         buckets of width Delta = divisor.  Requires
 *                         (2^32 - 1) / divisor <= m - 1.
 *   MS_BUCKET_SPLITTERS   range buckets: f(k) = number of splitters <= k,
 *                         i.e. s_{j-1} <= k < s_j with open-ended first and
 *                         last buckets (an upper bound over the splitters,
 *                         Section 7.3).  `splitters` points to m-1 ascending
 *                         uint32 in device memory (duplicates allowed: they
 *                         make empty buckets).  Found by binary search.
 *   MS_BUCKET_LEARNED     the same ids as MS_BUCKET_SPLITTERS, found by a
 *                         two-stage piecewise-linear model (`model`, device
 *                         pointer to MS_MODEL_FLOATS floats written by
 *                         ms_learned_fit) whose prediction is then checked
 *                         against the neighbouring splitters and corrected
 *                         exactly (one step either way, else binary search).
 *                         Not in the paper; the output is bit-identical to
 *                         MS_BUCKET_SPLITTERS.
 */
enum {
  MS_BUCKET_SHIFT_MASK = 0,
  MS_BUCKET_DIV = 1,
  MS_BUCKET_SPLITTERS = 2,
  MS_BUCKET_LEARNED = 3
};

#define MS_MODEL_LEAVES 256
#define MS_MODEL_FLOATS (2 + 2 * MS_MODEL_LEAVES)

typedef struct {
  int32_t kind;              /* one of MS_BUCKET_*                             */
  uint32_t shift;            /* SHIFT_MASK                                     */
  uint32_t mask;             /* SHIFT_MASK                                     */
  uint32_t divisor;          /* DIV                                            */
  const uint32_t* splitters; /* SPLITTERS, LEARNED: m-1 ascending, device      */
  const float* model;        /* LEARNED: MS_MODEL_FLOATS floats, device        */
} ms_bucket_fn;

/*
 * Reordering granularity (Section 5.3 and 5.6):
 *   MS_REORDER_BLOCK  block-level multisplit (BMS): each workgroup owns a
 *                     chunk of consecutive tiles; a tile is ranked by all of
 *                     its wavefronts and reordered in LDS across them.
 *   MS_REORDER_WAVE   wave-level multisplit (WMS): each wavefront owns a
 *                     chunk and reorders its own tiles in LDS.
 *   MS_REORDER_NONE   direct multisplit (DMS): each wavefront owns a chunk;
 *                     elements are scattered straight from registers.
 * All three give the same (unique) stable result.
 */
enum {
  MS_REORDER_AUTO = 0,
  MS_REORDER_BLOCK = 1,
  MS_REORDER_WAVE = 2,
  MS_REORDER_NONE = 3
};

/*
 * Optional tuning and instrumentation; pass NULL for defaults.  Every field
 * may be 0 (= choose automatically).  Tuning never changes results.
 *   reorder          MS_REORDER_*.
 *   waves_per_block  4, 8 or 16 wavefronts of 64 lanes per workgroup.
 *   items_per_lane   windows of 64 elements each wavefront ranks per tile
 *                    (the paper's N_window): 4, 8 or 16.  Block-level shapes
 *                    (waves x windows): 8x8, 8x4, 4x8, 4x16, 16x8, 16x16
 *                    (16x16 only where its buffers fit in LDS); wave level
 *                    8x8, 4x16; no reordering 8x8.  ms_batched: 8x8, 8x4,
 *                    4x16, 4x8, 16x4, 16x8.
 *   max_chunks       upper bound on the number of subproblems L0 (columns
 *                    of H, at most 4096); 0 = a whole multiple of the
 *                    post-scan workgroups resident at once, at least 1024.
 *   stage_events     if non-NULL, four hipEvent_t (as void*) that are
 *                    recorded on `stream` before the pre-scan, before the
 *                    scan, before the post-scan and after the post-scan.
 *   d_mispredicts    LEARNED only, optional device uint64: the number of
 *                    keys whose raw model prediction was wrong is ADDED to
 *                    it (the caller zeroes it).
 *   batch_claim      ms_batched: work items taken per queue access (1..64).
 *   spin_limit       ms_batched: polls a post-scan tile makes for its
 *                    instance's ready flag before giving up (0 = 2^22).
 *   test_flags       bit 0: ms_batched never raises ready flags, so every
 *                    wait expires (exercises the timeout path; for tests).
 *                    bit 1: ms_autotune treats its first candidate as
 *                    failed (exercises the skip of failing candidates).
 *   prescan          MS_PRESCAN_*: how the pre-scan counts buckets.
 *   keep_bucket_ids  SPLITTERS and LEARNED buckets, ms_keys / ms_pairs up to
 *                    256 buckets: 1 = the pre-scan stores every key's bucket
 *                    id (one byte) in the workspace and the post-scan reads
 *                    it instead of identifying the bucket again (2 more
 *                    bytes of traffic per key, one bucket search less);
 *                    ms_workspace_size then counts n more bytes.  With
 *                    LEARNED buckets d_mispredicts is then counted by the
 *                    pre-scan.  Other kinds and operations ignore it.
 */
typedef struct {
  int32_t reorder;
  int32_t waves_per_block;
  int32_t items_per_lane;
  int32_t max_chunks;
  void* const* stage_events;
  uint64_t* d_mispredicts;
  uint32_t batch_claim;
  uint32_t spin_limit;
  uint32_t test_flags;
  int32_t prescan;
  int32_t keep_bucket_ids;
} ms_options;

/*
 * Pre-scan histogram method (both give the same H):
 *   MS_PRESCAN_BALLOT  Algorithm 2's window histogram from ballots (Section
 *                      5.5.1; Section 5.7 for m > 64).
 *   MS_PRESCAN_LANES   per-(bucket, lane) LDS counters incremented by LDS
 *                      atomics; cost independent of m and of skew.  Block
 *                      reordering only (MS_ERR_UNSUPPORTED otherwise).
 *   MS_PRESCAN_AUTO    LANES with block reordering, BALLOT otherwise.
 * ms_batched always counts with ballots.
 */
enum {
  MS_PRESCAN_AUTO = 0,
  MS_PRESCAN_BALLOT = 1,
  MS_PRESCAN_LANES = 2
};

/* Operations for ms_workspace_size(). */
enum {
  MS_OP_KEYS = 0,
  MS_OP_PAIRS = 1,
  MS_OP_BATCHED = 2,
  MS_OP_RADIX_SORT = 3,
  MS_OP_RADIX_SORT_PAIRS = 4,
  MS_OP_LEARNED_FIT = 5,
  MS_OP_HISTOGRAM = 6
};

/*
 * Bytes of workspace an operation needs.  n = elements (for MS_OP_BATCHED the
 * total over all instances, for MS_OP_LEARNED_FIT the sample size), m =
 * buckets (for the radix sort: 2^bits_per_pass), num_inst = instances
 * (MS_OP_BATCHED only), opt as passed to the call (NULL = defaults).  Returns
 * 0 only for arguments that are invalid.
 */
size_t ms_workspace_size(int op, size_t n, uint32_t m, uint32_t num_inst,
                         const ms_options* opt);

/*
 * Stable multisplit of keys (Section 3.1, Eq. 1).
 *   d_keys_in   n uint32 keys.
 *   d_keys_out  n uint32: keys in ascending bucket order, input order kept
 *               inside every bucket.
 *   d_offsets   m+1 uint32 or NULL: d_offsets[j] = first output index of
 *               bucket j, d_offsets[m] = n (the paper's optional bucket-start
 *               array, Section 3.1, plus its end).
 *   n           0 <= n < 2^32.  n = 0 writes offsets of zero.
 *   m           1 <= m <= 256 buckets, or up to 65536 for SHIFT_MASK and
 *               DIV buckets: then two stable passes of at most 256 buckets
 *               run, on the low byte of the bucket id and then on its high
 *               byte (Section 6, "Performance for more than 256 buckets"),
 *               and the bucket starts come from one pass over the output.
 *               SPLITTERS and LEARNED buckets above 256 give
 *               MS_ERR_UNSUPPORTED; the workspace then also holds one copy
 *               of the data.
 *   fn          bucket identifier (host pointer to the descriptor).
 */
ms_status ms_keys(const uint32_t* d_keys_in, uint32_t* d_keys_out,
                  uint32_t* d_offsets, size_t n, uint32_t m,
                  const ms_bucket_fn* fn, void* d_ws, size_t ws_bytes,
                  const ms_options* opt, void* stream);

/* Stable multisplit of key-value pairs: as ms_keys, and every value moves
 * with its key (d_vals_in, d_vals_out: n uint32 each). */
ms_status ms_pairs(const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                   uint32_t* d_keys_out, uint32_t* d_vals_out,
                   uint32_t* d_offsets, size_t n, uint32_t m,
                   const ms_bucket_fn* fn, void* d_ws, size_t ws_bytes,
                   const ms_options* opt, void* stream);

/*
 * ms_pairs (or ms_keys, with both value pointers NULL) for callers that
 * cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  It takes no workspace
 * and allocates nothing: its scratch words (the bucket totals and the
 * subproblem histograms H, at most 4 MiB) live in a static device array of
 * the library, one per GPU, held until the process ends.  Arguments,
 * results and errors are those of ms_pairs, plus:
 *   m above 256   MS_ERR_WORKSPACE (that path needs a copy of the data).
 * The first call on a device looks the array up (MS_ERR_HIP if that
 * fails).  Calls share the device's array, so calls that overlap on one GPU
 * (on different streams, or from different threads) race: serialise them.
 * Every word the call reads is first written by the same call.
 */
ms_status ms_pairs_noalloc(const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                           uint32_t* d_keys_out, uint32_t* d_vals_out,
                           uint32_t* d_offsets, size_t n, uint32_t m,
                           const ms_bucket_fn* fn, const ms_options* opt,
                           void* stream);

/*
 * Device-wide histogram (Section 7.3): d_hist[j] = number of the n keys with
 * fn(key) = j, for j < m.  It is the multisplit pre-scan (one count per
 * bucket and subproblem), followed by a per-bucket reduction of those counts
 * into d_hist (Section 7.3's store-and-reduce option); no key moves.  Even
 * bins are SHIFT_MASK or DIV buckets, range bins SPLITTERS or LEARNED
 * buckets.
 *   d_keys   n uint32 keys (device).  n = 0 writes m zeros.
 *   d_hist   m uint32 (device), overwritten; must not overlap d_keys.
 *   d_ws     ms_workspace_size(MS_OP_HISTOGRAM, n, m, 0, opt) bytes.
 * opt->d_mispredicts is not updated by this call.  Errors as ms_keys.
 */
ms_status ms_histogram(const uint32_t* d_keys, size_t n, uint32_t m,
                       const ms_bucket_fn* fn, uint32_t* d_hist, void* d_ws,
                       size_t ws_bytes, const ms_options* opt, void* stream);

/*
 * LSD radix sort built from multisplit passes (Section 7.1): with r =
 * bits_per_pass, pass p is a stable multisplit on f_p(k) = (k >> p r) &
 * (2^r - 1), p = 0 .. ceil(32 / r) - 1, so the result is the stable sort of
 * the keys (values follow their keys).  d_vals_in / d_vals_out may both be
 * NULL for a key-only sort.  bits_per_pass in [1, 8].  The workspace holds
 * the ping-pong copy of the data.
 */
ms_status ms_radix_sort(const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                        uint32_t* d_keys_out, uint32_t* d_vals_out, size_t n,
                        uint32_t bits_per_pass, void* d_ws, size_t ws_bytes,
                        const ms_options* opt, void* stream);

/*
 * Batched stable multisplit: num_inst independent instances in one
 * persistent launch (after a one-workgroup set-up kernel).  Instance i is
 * elements [d_seg[i], d_seg[i+1]) of the concatenated arrays (d_seg:
 * num_inst+1 ascending uint64 in device memory, d_seg[0] = 0, d_seg[num_inst]
 * = total < 2^32 - 1).  Each instance is multisplit on its own into the same
 * index range of the outputs.  d_offsets: num_inst*(m+1) uint32 or NULL,
 * instance i's bucket starts relative to its own first element (last entry =
 * its size).  d_vals_in and d_vals_out may both be NULL.  The call neither
 * synchronises nor allocates and clears its own counters with a kernel, so it
 * can be captured into a HIP graph and replayed.  Whether any internal wait
 * expired can be read afterwards with ms_batched_status().
 */
ms_status ms_batched(const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                     uint32_t* d_keys_out, uint32_t* d_vals_out,
                     const uint64_t* d_seg, uint32_t num_inst, size_t total,
                     uint32_t m, const ms_bucket_fn* fn, uint32_t* d_offsets,
                     void* d_ws, size_t ws_bytes, const ms_options* opt,
                     void* stream);

/*
 * Status of the last ms_batched call that used workspace d_ws: MS_OK, or
 * MS_ERR_TIMEOUT if a post-scan tile gave up waiting for its instance (its
 * output is then incomplete).  Waits for `stream` (not capture-safe).
 */
ms_status ms_batched_status(const void* d_ws, void* stream);

/*
 * Fit the learned bucket model for range buckets from n_sample device sample
 * keys (not in the paper; Section 7.3 finds range buckets by binary search).
 *   d_sample     n_sample uint32 keys, 1 <= n_sample < 2^32 - 1.
 *   d_labels     n_sample uint32 bucket ids, or NULL: the labels are then
 *                the exact upper bounds over the splitters (the ids that
 *                MS_BUCKET_SPLITTERS gives).  Given labels at or above m
 *                count as m - 1.
 *   d_splitters  m-1 ascending uint32 (may be NULL when d_labels is given).
 *   d_model      receives MS_MODEL_FLOATS floats.
 * Root: the line that maps the sample's key range [x_min, x_max], x =
 * (float)key, onto the leaves [0, 256): x_min to 0, x_max to 256 (clamped to
 * 255 when evaluated).  Each sample is routed to a leaf by that root
 * evaluated in float exactly as at inference.  Each leaf is the
 * least-squares line of the bucket centre (label + 1/2) on x over its
 * samples; a leaf with no samples copies its nearest non-empty neighbour
 * (left first, else right).  The sums are exact integers, so the fit is
 * deterministic.  Workspace: ms_workspace_size(MS_OP_LEARNED_FIT, n_sample,
 * m, 0, NULL) bytes (a few KiB, independent of n_sample).
 */
ms_status ms_learned_fit(const uint32_t* d_sample, const uint32_t* d_labels,
                         size_t n_sample, const uint32_t* d_splitters,
                         uint32_t m, float* d_model, void* d_ws,
                         size_t ws_bytes, void* stream);

/*
 * Autotuner: runs `op` (MS_OP_KEYS, MS_OP_PAIRS, MS_OP_BATCHED,
 * MS_OP_RADIX_SORT or MS_OP_RADIX_SORT_PAIRS) on the caller's buffers once
 * per candidate tuning (reordering mode, waves per workgroup, windows per
 * wavefront and, for MS_OP_BATCHED, the queue claim size), `reps` timed
 * times each after one warm-up, and writes the fastest candidate to *best
 * (fields other than the tuned ones are copied from `base`, which may be
 * NULL) and its mean time in milliseconds to *best_ms.  The outputs hold the
 * result of a final run with the winner.  Candidates whose workspace exceeds
 * ws_bytes, and candidates whose run fails, are skipped; the call returns
 * the last failure only if no candidate ran.  Arguments as for the operation itself (d_seg / num_inst for
 * MS_OP_BATCHED only, fn ignored for the radix sort, m = bits per pass for
 * the radix sort).  Synchronises `stream`; not capture-safe.
 */
ms_status ms_autotune(int op, const uint32_t* d_keys_in, const uint32_t* d_vals_in,
                      uint32_t* d_keys_out, uint32_t* d_vals_out, const uint64_t* d_seg,
                      uint32_t num_inst, size_t n, uint32_t m, const ms_bucket_fn* fn,
                      void* d_ws, size_t ws_bytes, int reps, const ms_options* base,
                      ms_options* best, float* best_ms, void* stream);

/*
 * Streaming copy of n uint32 (d_dst[i] = d_src[i]).  Not part of the
 * method: it measures the achievable HBM copy bandwidth that the multisplit
 * kernels are compared against.
 */
ms_status ms_copy_u32(uint32_t* d_dst, const uint32_t* d_src, size_t n,
                      void* stream);

/*
 * Single-source shortest paths by delta-stepping whose work frontier is
 * bucketed with the stable multisplit (Section 7.2, Multisplit-SSSP: the
 * Bucketing strategy with its radix sort replaced by a multisplit).
 *
 * Graph: directed, CSR on the device -- d_row[nv + 1] uint64 edge offsets
 * (d_row[0] = 0, non-decreasing, d_row[nv] = ne), d_col[ne] target vertices
 * (< nv; an edge past the last vertex makes the call return
 * MS_ERR_INVALID_ARG after it has run), d_wt[ne] non-negative integer
 * weights.  Paths are summed in 32 bits saturating at 0xFFFFFFFE, so the
 * caller keeps every shortest path below that.
 *
 * Output: d_dist[nv], the least total weight of a path from `source`
 * (0xFFFFFFFF where unreachable).  The distances do not depend on `delta`
 * (bucket width, >= 1) or `num_buckets` (B in [2, 256]: B - 1 buckets of
 * width delta above a moving base plus one open-ended bucket); they set how
 * much work a round does and how many rounds there are.
 *
 * Each round multisplits the pending (distance, vertex) pairs into the B
 * buckets (splitter buckets), relaxes every out-edge of the lowest occupied
 * bucket's vertices on the GPU and appends each improvement to the pending
 * list; see ms_sssp.hip for the steps.  The call synchronises `stream` once
 * per round (the pending count sizes the next multisplit) and returns when
 * nothing is pending; not capture-safe.  The workspace (caller owned, size
 * from ms_sssp_workspace_size, at least nv + ne pending entries) is
 * clobbered.  `stats` (host, nullable) receives the round counts.
 * Errors: MS_ERR_INVALID_ARG (null pointer, nv = 0, source >= nv, delta =
 * 0, B out of range, nv + ne >= 2^32 - 1, a bad edge), MS_ERR_WORKSPACE,
 * MS_ERR_HIP, MS_ERR_TIMEOUT (more rounds than the algorithm can need).
 */
typedef struct {
  uint64_t rounds;         /* multisplit rounds                             */
  uint64_t items_split;    /* pending entries multisplit, summed over rounds */
  uint64_t edges_relaxed;  /* out-edges relaxed, summed over rounds         */
  uint64_t pushes;         /* improvements appended to the pending list      */
  uint64_t max_pending;    /* largest pending list                           */
} ms_sssp_stats;

size_t ms_sssp_workspace_size(uint32_t nv, uint64_t ne, uint32_t num_buckets);

ms_status ms_sssp(const uint64_t* d_row, const uint32_t* d_col, const uint32_t* d_wt,
                  uint32_t nv, uint64_t ne, uint32_t source, uint32_t delta,
                  uint32_t num_buckets, uint32_t* d_dist, void* d_ws, size_t ws_bytes,
                  ms_sssp_stats* stats, void* stream);

/* Version string of the library build. */
const char* ms_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MULTISPLIT_H */
