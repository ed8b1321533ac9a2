// Fit of the learned bucket identifier for range buckets (two-stage
// piecewise-linear model of the bucket as a function of the key; not in the
// paper, whose range buckets use a binary search over the splitters held in
// shared memory, Section 7.3).
//
// Root: the line that spreads the sample's key range [x_min, x_max] over the
// 256 leaves.  Leaves: least squares of the bucket centre (label + 1/2) on x
// over the samples the float root routes to the leaf; an empty leaf copies
// its nearest non-empty neighbour.  Every sum is in double and reduced in a
// fixed order (each workgroup sums a fixed slice of the sample with a fixed
// thread-to-element mapping and a fixed tree; partials are then combined in
// workgroup order), so the fit is deterministic.  Least squares use the
// two-pass form: means first, then the centred sums.
#pragma once

#include "ms_device.hpp"

namespace ms {

constexpr int kFitThreads = 256;
constexpr int kFitBlocks = 256;

// Fixed-order workgroup sum of one double per thread.
__device__ __forceinline__ double block_sum(double v, double* tmp) {
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (int s = kFitThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) tmp[threadIdx.x] += tmp[threadIdx.x + s];
    __syncthreads();
  }
  double r = tmp[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ uint32_t fit_upper_bound(const uint32_t* spl, uint32_t m, uint32_t k) {
  return lds_upper_bound<8>(spl, m, k);
}

struct FitParams {
  const uint32_t* sample;
  uint32_t ns;
  const uint32_t* splitters;
  uint32_t m;
  float* model;
  uint32_t* labels;    // ns
  uint32_t* leaves;    // ns
  double* partial;     // kFitBlocks * 2 per-workgroup partials
  double* moments;     // [8 + leaf]: 1 if the leaf received samples
};

__device__ __forceinline__ double block_min(double v, double* tmp) {
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (int s = kFitThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) tmp[threadIdx.x] = fmin(tmp[threadIdx.x], tmp[threadIdx.x + s]);
    __syncthreads();
  }
  double r = tmp[0];
  __syncthreads();
  return r;
}

// Labels (exact upper bound) and per-workgroup minimum and maximum of x.
__global__ void __launch_bounds__(kFitThreads) fit_label_kernel(FitParams p) {
  __shared__ uint32_t spl[kMaxBuckets];
  __shared__ double tmp[kFitThreads];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kMaxBuckets; i += kFitThreads)
    spl[i] = (i + 1 < p.m) ? p.splitters[i] : 0xFFFFFFFFu;
  __syncthreads();
  double lo = 1e300, neg_hi = 1e300;
  for (uint32_t i = blockIdx.x * kFitThreads + threadIdx.x; i < p.ns; i += kFitBlocks * kFitThreads) {
    const uint32_t k = p.sample[i];
    p.labels[i] = fit_upper_bound(spl, p.m, k);
    const double x = (double)(float)k;
    lo = fmin(lo, x);
    neg_hi = fmin(neg_hi, -x);
  }
  lo = block_min(lo, tmp);
  neg_hi = block_min(neg_hi, tmp);
  if (threadIdx.x == 0) {
    p.partial[2 * blockIdx.x] = lo;
    p.partial[2 * blockIdx.x + 1] = neg_hi;
  }
}

// Root line from the range of x: x_min -> 0, x_max -> L (clamped to L-1 at
// evaluation).
__global__ void __launch_bounds__(kFitThreads) fit_root_kernel(FitParams p) {
  __shared__ double tmp[kFitThreads];
  const double xmin = block_min(p.partial[2 * threadIdx.x], tmp);
  const double xmax = -block_min(p.partial[2 * threadIdx.x + 1], tmp);
  if (threadIdx.x == 0) {
    float a0 = 0.0f, b0 = 0.0f;
    if (xmax > xmin) {
      a0 = (float)((double)kLeaves / (xmax - xmin));
      b0 = (float)(-(double)a0 * xmin);
    }
    p.model[0] = a0;
    p.model[1] = b0;
  }
}

// Route every sample to its leaf with the float root (the same evaluation
// as inference).
__global__ void __launch_bounds__(kFitThreads) fit_route_kernel(FitParams p) {
  const float a0 = p.model[0], b0 = p.model[1];
  for (uint32_t i = blockIdx.x * kFitThreads + threadIdx.x; i < p.ns; i += kFitBlocks * kFitThreads)
    p.leaves[i] = clamp_trunc(__builtin_fmaf(a0, (float)p.sample[i], b0), (uint32_t)kLeaves);
}

// One workgroup per leaf: count, means, centred sums, line.  Whether the
// leaf received samples is recorded in moments[8 + leaf].
__global__ void __launch_bounds__(kFitThreads) fit_leaf_kernel(FitParams p) {
  __shared__ double tmp[kFitThreads];
  const uint32_t leaf = blockIdx.x;
  double cnt = 0, sx = 0, sy = 0;
  for (uint32_t i = threadIdx.x; i < p.ns; i += kFitThreads) {
    if (p.leaves[i] == leaf) {
      cnt += 1.0;
      sx += (double)(float)p.sample[i];
      sy += (double)p.labels[i] + 0.5;
    }
  }
  cnt = block_sum(cnt, tmp);
  sx = block_sum(sx, tmp);
  sy = block_sum(sy, tmp);
  if (cnt == 0.0) {
    if (threadIdx.x == 0) {
      p.model[2 + 2 * leaf] = 0.0f;
      p.model[3 + 2 * leaf] = 0.0f;
      p.moments[8 + leaf] = 0.0;
    }
    return;
  }
  const double mx = sx / cnt, my = sy / cnt;
  double sxx = 0, sxy = 0;
  for (uint32_t i = threadIdx.x; i < p.ns; i += kFitThreads) {
    if (p.leaves[i] == leaf) {
      const double dx = (double)(float)p.sample[i] - mx;
      sxx += dx * dx;
      sxy += dx * ((double)p.labels[i] + 0.5 - my);
    }
  }
  sxx = block_sum(sxx, tmp);
  sxy = block_sum(sxy, tmp);
  if (threadIdx.x == 0) {
    double slope = 0.0, icpt = my;
    if (sxx > 0) {
      slope = sxy / sxx;
      icpt = my - slope * mx;
    }
    p.model[2 + 2 * leaf] = (float)slope;
    p.model[3 + 2 * leaf] = (float)icpt;
    p.moments[8 + leaf] = 1.0;
  }
}

// An empty leaf copies its nearest non-empty neighbour to the left, else to
// the right.
__global__ void fit_fill_empty_kernel(FitParams p) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int l = 0; l < kLeaves; ++l) {
    if (p.moments[8 + l] != 0.0) continue;
    int src = -1;
    for (int j = l - 1; j >= 0; --j)
      if (p.moments[8 + j] != 0.0) { src = j; break; }
    if (src < 0)
      for (int j = l + 1; j < kLeaves; ++j)
        if (p.moments[8 + j] != 0.0) { src = j; break; }
    if (src >= 0) {
      p.model[2 + 2 * l] = p.model[2 + 2 * src];
      p.model[3 + 2 * l] = p.model[3 + 2 * src];
    }
  }
}

}  // namespace ms
