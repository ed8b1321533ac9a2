// CPU oracle for stable multisplit -- TEST INFRASTRUCTURE ONLY.
//
// Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
// this library.  It shares no code with the GPU path: no headers, no tables,
// no helpers.  Everything here is deliberately plain, single-threaded and
// unblocked so that it can be read against the paper line by line.
//
// Paper: Ashkiani, Davidson, Meyer, Owens, "GPU Multisplit: an extended study
// of a parallel algorithm" (ACM TOPC 2017).
//
// What is computed, and where it is defined:
//   * stable multisplit -- Section 3.1 (definition) and Eq. (1) of Section 4.2:
//     p(i) = (number of keys in buckets < f(u_i))
//          + (number of earlier keys in the same bucket).
//     Written out as a counting sort (histogram, exclusive prefix sum of the
//     histogram, then an in-order placement).
//   * bucket identifiers -- Section 6 "Bucket identification": delta buckets
//     f(u) = floor(u / Delta); identity/radix-digit buckets f(u) = (u >> s) & mask
//     (Section 7.1); range buckets by splitters, s_j <= u < s_{j+1}, an upper
//     bound over the splitters (Sections 6 and 7.3).  The first and last range
//     buckets are open ended.
//   * LSD radix sort -- Section 7.1: the output equals a stable sort by key;
//     std::stable_sort is that definition.
//   * batched multisplit -- the stable multisplit applied to each segment on
//     its own; offsets are relative to the segment start.
//   * device-wide histogram -- Section 7.3: the number of keys per bucket,
//     h_j = #{i : f(u_i) = j} (the same h_j as in Eq. 1), counted in one pass.
//   * single-source shortest paths -- Section 7.2 uses multisplit to bucket
//     the work frontier of delta-stepping; whatever the bucketing, the result
//     is the shortest-path distance of every vertex, which is unique.  The
//     oracle is Dijkstra's algorithm (a binary heap with lazy deletion).
//   * learned bucket identifier -- a two-stage piecewise-linear model of the
//     bucket as a function of the key (an even split of the key range into
//     leaves, then a least-squares line per leaf) fit in double precision,
//     evaluated in single precision with fused multiply-add.  It is
//     not in the paper (the paper's range buckets use binary search); its
//     corrected output must equal the upper bound exactly, which is how it is
//     pinned.  Only the fitted parameter bits are checked to a tolerance.
//
// Readings where the paper is silent are listed with each function.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <vector>

namespace {

enum { OR_SHIFT_MASK = 0, OR_DIV = 1, OR_SPLITTERS = 2, OR_LEARNED = 3 };

// Upper bound: the number of splitters s with s <= k.  With ascending
// splitters s_0 <= ... <= s_{m-2} this is the j with s_{j-1} <= k < s_j,
// where s_{-1} = -inf and s_{m-1} = +inf (open-ended first and last bucket).
uint32_t upper_bound_count(const uint32_t* spl, uint32_t nspl, uint32_t k) {
  return (uint32_t)(std::upper_bound(spl, spl + nspl, k) - spl);
}

uint32_t bucket_of(int kind, uint32_t p0, uint32_t p1, const uint32_t* spl,
                   uint32_t m, uint32_t k) {
  switch (kind) {
    case OR_SHIFT_MASK:  // (k >> shift) & mask
      return (k >> p0) & p1;
    case OR_DIV:         // floor(k / Delta); Delta = 0 is not a bucket function
      return p0 ? k / p0 : 0xFFFFFFFFu;
    case OR_SPLITTERS:
    case OR_LEARNED:     // the learned identifier must reproduce this exactly
      return upper_bound_count(spl, m - 1, k);
    default:
      return 0xFFFFFFFFu;
  }
}

}  // namespace

extern "C" {

// Bucket id of every key.  Returns 0, or -1 if some id is >= m.
int or_bucket_ids(const uint32_t* keys, uint64_t n, uint32_t m, int kind,
                  uint32_t p0, uint32_t p1, const uint32_t* spl, uint32_t* out) {
  for (uint64_t i = 0; i < n; ++i) {
    out[i] = bucket_of(kind, p0, p1, spl, m, keys[i]);
    if (out[i] >= m) return -1;
  }
  return 0;
}

// Histogram of the bucket ids (Section 7.3): hist[j] = #{i : f(keys[i]) = j}.
// Returns 0, or -1 if a key maps outside [0, m).
int or_histogram(const uint32_t* keys, uint64_t n, uint32_t m, int kind,
                 uint32_t p0, uint32_t p1, const uint32_t* spl, uint32_t* hist) {
  for (uint32_t j = 0; j < m; ++j) hist[j] = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t b = bucket_of(kind, p0, p1, spl, m, keys[i]);
    if (b >= m) return -1;
    hist[b] += 1;
  }
  return 0;
}

// Stable multisplit of keys (and values when vals != nullptr).
// offsets: m+1 entries, offsets[j] = first output index of bucket j,
// offsets[m] = n (reading: the paper's optional size-m start array, plus n).
// Returns 0, or -1 if a key maps outside [0, m).
int or_multisplit(const uint32_t* keys, const uint32_t* vals, uint64_t n,
                  uint32_t m, int kind, uint32_t p0, uint32_t p1,
                  const uint32_t* spl, uint32_t* out_keys, uint32_t* out_vals,
                  uint32_t* offsets) {
  std::vector<uint32_t> b(n);
  std::vector<uint64_t> count(m, 0);
  // 1. bucket of every key; 2. histogram h_j.
  for (uint64_t i = 0; i < n; ++i) {
    b[i] = bucket_of(kind, p0, p1, spl, m, keys[i]);
    if (b[i] >= m) return -1;
    count[b[i]] += 1;
  }
  // 3. global offset of bucket j = sum of h_k over k < j (first term of Eq. 1).
  std::vector<uint64_t> start(m + 1, 0);
  for (uint32_t j = 0; j < m; ++j) start[j + 1] = start[j] + count[j];
  if (offsets)
    for (uint32_t j = 0; j <= m; ++j) offsets[j] = (uint32_t)start[j];
  // 4. visit keys in input order; the running cursor of bucket j adds the
  //    number of earlier keys of bucket j (second term of Eq. 1).
  std::vector<uint64_t> cursor(start.begin(), start.begin() + m);
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t p = cursor[b[i]]++;
    out_keys[p] = keys[i];
    if (vals && out_vals) out_vals[p] = vals[i];
  }
  return 0;
}

// Stable sort of (key, value) by key (Section 7.1's target result).
void or_radix_sort(const uint32_t* keys, const uint32_t* vals, uint64_t n,
                   uint32_t* out_keys, uint32_t* out_vals) {
  std::vector<uint64_t> idx(n);
  std::iota(idx.begin(), idx.end(), (uint64_t)0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](uint64_t a, uint64_t c) { return keys[a] < keys[c]; });
  for (uint64_t i = 0; i < n; ++i) {
    out_keys[i] = keys[idx[i]];
    if (vals && out_vals) out_vals[i] = vals[idx[i]];
  }
}

// Independent instances: instance i is keys[seg[i] .. seg[i+1]).
// offsets: num*(m+1) entries, relative to the instance start.
int or_batched(const uint32_t* keys, const uint32_t* vals, const uint64_t* seg,
               uint32_t num, uint32_t m, int kind, uint32_t p0, uint32_t p1,
               const uint32_t* spl, uint32_t* out_keys, uint32_t* out_vals,
               uint32_t* offsets) {
  for (uint32_t i = 0; i < num; ++i) {
    uint64_t a = seg[i], n = seg[i + 1] - seg[i];
    int rc = or_multisplit(keys + a, vals ? vals + a : nullptr, n, m, kind, p0,
                           p1, spl, out_keys + a, out_vals ? out_vals + a : nullptr,
                           offsets ? offsets + (uint64_t)i * (m + 1) : nullptr);
    if (rc) return rc;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Learned bucket identifier (range buckets given by m-1 splitters).
//
// Model layout (2 + 2*L floats, L = 256 leaves):
//   model[0], model[1]            root slope a0 and intercept b0
//   model[2 + 2l], model[3 + 2l]  slope and intercept of leaf l
//
// Evaluation, all in float with fused multiply-add:
//   x    = (float)k                       (round to nearest even)
//   v    = fmaf(a0, x, b0);   leaf = v < 0 ? 0 : v >= L ? L-1 : trunc(v)
//   w    = fmaf(a_leaf, x, b_leaf); pred = w < 0 ? 0 : w >= m ? m-1 : trunc(w)
// The root spreads the sample's key range evenly over the leaves.
// ---------------------------------------------------------------------------
static const uint32_t OR_LEAVES = 256;

static uint32_t clamp_trunc(float v, uint32_t hi) {
  if (v < 0.0f) return 0;
  if (v >= (float)hi) return hi - 1;
  return (uint32_t)v;
}

uint32_t or_learned_leaf(const float* model, uint32_t k) {
  float x = (float)k;
  return clamp_trunc(std::fmaf(model[0], x, model[1]), OR_LEAVES);
}

uint32_t or_learned_predict(const float* model, uint32_t m, uint32_t k) {
  float x = (float)k;
  uint32_t leaf = clamp_trunc(std::fmaf(model[0], x, model[1]), OR_LEAVES);
  return clamp_trunc(std::fmaf(model[2 + 2 * leaf], x, model[3 + 2 * leaf]), m);
}

// Least squares line y ~ a x + b over the given points in double precision,
// accumulated in index order.  Degenerate cases: no points -> (0, 0) and
// *ok = 0; zero x-variance -> slope 0, intercept mean(y).
static void lsq_line(const std::vector<double>& x, const std::vector<double>& y,
                     double* a, double* b, int* ok) {
  size_t n = x.size();
  if (n == 0) { *a = 0; *b = 0; *ok = 0; return; }
  double sx = 0, sy = 0;
  for (size_t i = 0; i < n; ++i) { sx += x[i]; sy += y[i]; }
  double mx = sx / (double)n, my = sy / (double)n;
  double sxx = 0, sxy = 0;
  for (size_t i = 0; i < n; ++i) {
    double dx = x[i] - mx;
    sxx += dx * dx;
    sxy += dx * (y[i] - my);
  }
  if (sxx > 0) { *a = sxy / sxx; *b = my - (*a) * mx; }
  else { *a = 0; *b = my; }
  *ok = 1;
}

// Fit the two-stage model to sample keys labelled by the exact upper bound
// (or by the given labels, clamped to m - 1, when labels is not null).
// Root: the line that maps the sample's key range [x_min, x_max] onto the
// leaves [0, L) (x_min to 0, x_max to L, clamped to L-1), so that every leaf
// covers an equal slice of the key range.  Leaves: least squares of the
// bucket centre y + 1/2 on x over the samples the float root routes there,
// so truncation of the line lands inside the bucket.  An empty leaf copies
// the nearest non-empty leaf to its left (else to its right).
void or_learned_fit(const uint32_t* sample, uint64_t ns, const uint32_t* spl,
                    uint32_t m, const uint32_t* labels, float* model) {
  std::vector<double> x(ns), y(ns);
  double xmin = 0, xmax = 0;
  for (uint64_t i = 0; i < ns; ++i) {
    x[i] = (double)(float)sample[i];
    const uint32_t lab = labels ? (labels[i] < m ? labels[i] : m - 1)
                                : upper_bound_count(spl, m - 1, sample[i]);
    y[i] = (double)lab + 0.5;
    if (i == 0 || x[i] < xmin) xmin = x[i];
    if (i == 0 || x[i] > xmax) xmax = x[i];
  }
  float a0 = 0.0f, b0 = 0.0f;
  if (xmax > xmin) {
    a0 = (float)((double)OR_LEAVES / (xmax - xmin));
    b0 = (float)(-(double)a0 * xmin);
  }
  model[0] = a0;
  model[1] = b0;
  std::vector<std::vector<double>> lx(OR_LEAVES), ly(OR_LEAVES);
  for (uint64_t i = 0; i < ns; ++i) {
    uint32_t l = or_learned_leaf(model, sample[i]);
    lx[l].push_back(x[i]);
    ly[l].push_back(y[i]);
  }
  std::vector<int> have(OR_LEAVES, 0);
  for (uint32_t l = 0; l < OR_LEAVES; ++l) {
    double a, b;
    lsq_line(lx[l], ly[l], &a, &b, &have[l]);
    model[2 + 2 * l] = (float)a;
    model[3 + 2 * l] = (float)b;
  }
  for (uint32_t l = 0; l < OR_LEAVES; ++l) {
    if (have[l]) continue;
    int src = -1;
    for (int j = (int)l - 1; j >= 0; --j) if (have[j]) { src = j; break; }
    if (src < 0)
      for (uint32_t j = l + 1; j < OR_LEAVES; ++j) if (have[j]) { src = (int)j; break; }
    if (src >= 0) {
      model[2 + 2 * l] = model[2 + 2 * src];
      model[3 + 2 * l] = model[3 + 2 * src];
    }
  }
}

// Learned bucket ids: the exact upper bound (the only correct answer), plus
// the number of keys whose raw model prediction differs from it.
void or_learned_bucket_ids(const float* model, const uint32_t* spl, uint32_t m,
                           const uint32_t* keys, uint64_t n, uint32_t* out,
                           uint64_t* mispredicts) {
  uint64_t miss = 0;
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t exact = upper_bound_count(spl, m - 1, keys[i]);
    if (or_learned_predict(model, m, keys[i]) != exact) ++miss;
    if (out) out[i] = exact;
  }
  if (mispredicts) *mispredicts = miss;
}

// Single-source shortest paths on a directed graph in CSR form (row offsets
// nv + 1, column and weight per edge): dist[v] = the least total weight of a
// path from src to v, 0xFFFFFFFF if v is unreachable.  Dijkstra's algorithm:
// pop the closest unsettled vertex, relax its out-edges.  Distances are
// accumulated in 64 bits; a graph whose shortest path reaches 0xFFFFFFFF
// returns -1.  Section 7.2 (the problem it solves; the paper's delta-stepping
// must produce the same distances).
int or_sssp(const uint64_t* row, const uint32_t* col, const uint32_t* wt, uint32_t nv,
            uint32_t src, uint32_t* dist) {
  const uint64_t kInf = ~0ull;
  std::vector<uint64_t> d(nv, kInf);
  typedef std::pair<uint64_t, uint32_t> Item;  // (distance, vertex)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  d[src] = 0;
  heap.push(Item(0, src));
  while (!heap.empty()) {
    const Item top = heap.top();
    heap.pop();
    const uint32_t u = top.second;
    if (top.first != d[u]) continue;  // a stale entry: u was settled closer
    for (uint64_t e = row[u]; e < row[u + 1]; ++e) {
      const uint64_t nd = d[u] + wt[e];
      if (nd < d[col[e]]) {
        d[col[e]] = nd;
        heap.push(Item(nd, col[e]));
      }
    }
  }
  for (uint32_t v = 0; v < nv; ++v) {
    if (d[v] != kInf && d[v] >= 0xFFFFFFFFull) return -1;
    dist[v] = d[v] == kInf ? 0xFFFFFFFFu : (uint32_t)d[v];
  }
  return 0;
}

}  // extern "C"
