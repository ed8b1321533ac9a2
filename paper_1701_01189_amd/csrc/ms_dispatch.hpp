// Launch-time selection of kernel instantiations: bucket kind, ballot rounds
// (BITS = ceil(log2 m)), key-only or key-value, workgroup shape and
// reordering mode are all template parameters of the kernels, so the inner
// loops carry no run-time branches.  One translation unit per bucket kind
// instantiates its share (ms_kind_*.hip).
#pragma once

#include "ms_batched.hpp"
#include "ms_kernels.hpp"

namespace ms {

struct PreArgs {
  const uint32_t* keys;
  Plan plan;
  BucketParams bp;
  uint32_t* H;
  int mode;
  int hist;  // kHistBallot / kHistLanes (block mode only)
  hipStream_t stream;
  uint8_t* ids;  // table-search kinds: each key's bucket id is stored here (or NULL)
};

struct PostArgs {
  const uint32_t* keys_in;
  const uint32_t* vals_in;
  uint32_t* keys_out;
  uint32_t* vals_out;
  const uint32_t* G;
  const uint32_t* totals;
  uint32_t* offsets;
  Plan plan;
  BucketParams bp;
  int mode, wpb, nw;
  bool kv;
  hipStream_t stream;
  int* occupancy;  // if set: store the kernel's resident workgroups per CU, launch nothing
  const uint8_t* ids;  // table-search kinds: bucket ids kept by the pre-scan (or NULL)
};

// Shapes with an instantiated post-scan: (mode, waves per block, windows).
inline bool post_shape_supported(int mode, int wpb, int nw) {
  if (mode == kBlock)
    return (wpb == 8 && (nw == 4 || nw == 8)) || (wpb == 4 && (nw == 8 || nw == 16)) ||
           (wpb == 16 && (nw == 8 || nw == 16));
  if (mode == kWaveMode) return (wpb == 8 && nw == 8) || (wpb == 4 && nw == 16);
  if (mode == kDirect) return wpb == 8 && nw == 8;
  return false;
}

// Pre-scan workgroups are always 8 wavefronts: BMS chunks are shared by the
// whole workgroup, WMS/DMS chunks belong to single wavefronts.
constexpr int kPreWaves = 8;

template <int Kind, int BITS>
hipError_t pre_launch(const PreArgs& a) {
  if (a.mode == kBlock && a.hist == kHistLanes) {
    hipLaunchKernelGGL((prescan_kernel<Kind, BITS, kPreWaves, kPreWaves, kHistLanes>),
                       dim3(a.plan.L0), dim3(kPreWaves * kWave), 0, a.stream, a.keys, a.plan,
                       a.bp, a.H, a.ids);
  } else if (a.mode == kBlock) {
    hipLaunchKernelGGL((prescan_kernel<Kind, BITS, kPreWaves, kPreWaves, kHistBallot>),
                       dim3(a.plan.L0), dim3(kPreWaves * kWave), 0, a.stream, a.keys, a.plan,
                       a.bp, a.H, a.ids);
  } else {
    hipLaunchKernelGGL((prescan_kernel<Kind, BITS, kPreWaves, 1, kHistBallot>),
                       dim3((a.plan.L0 + kPreWaves - 1) / kPreWaves), dim3(kPreWaves * kWave), 0,
                       a.stream, a.keys, a.plan, a.bp, a.H, a.ids);
  }
  return hipGetLastError();
}

template <int Kind>
hipError_t pre_dispatch(const PreArgs& a, int bits) {
  switch (bits) {
    case 0: return pre_launch<Kind, 0>(a);
    case 1: return pre_launch<Kind, 1>(a);
    case 2: return pre_launch<Kind, 2>(a);
    case 3: return pre_launch<Kind, 3>(a);
    case 4: return pre_launch<Kind, 4>(a);
    case 5: return pre_launch<Kind, 5>(a);
    case 6: return pre_launch<Kind, 6>(a);
    case 7: return pre_launch<Kind, 7>(a);
    case 8: return pre_launch<Kind, 8>(a);
    default: return hipErrorInvalidValue;
  }
}

template <int Kind, int BITS, bool KV, int WPB, int NW, int MODE>
hipError_t post_launch(const PostArgs& a) {
  constexpr int WPG = (MODE == kBlock) ? WPB : 1;
  constexpr int GPB = WPB / WPG;
  auto kern = postscan_kernel<Kind, BITS, KV, WPB, NW, MODE>;
  if (a.occupancy) {
    // The kernel's registers and LDS fix its residency; it is the same on
    // every call, so it is asked once.
    static int cached = 0;
    if (cached == 0) {
      int per_cu = 0;
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WPB * kWave, 0);
      if (e != hipSuccess) return e;
      cached = per_cu > 0 ? per_cu : 1;
    }
    *a.occupancy = cached;
    return hipSuccess;
  }
  dim3 grid((a.plan.L0 + GPB - 1) / GPB), block(WPB * kWave);
  hipLaunchKernelGGL(kern, grid, block, 0, a.stream, a.keys_in, a.vals_in, a.keys_out,
                     a.vals_out, a.G, a.totals, a.offsets, a.plan, a.bp, a.ids);
  return hipGetLastError();
}

template <int Kind, int BITS, bool KV>
hipError_t post_shape(const PostArgs& a) {
  if (a.mode == kBlock) {
    if (a.wpb == 8 && a.nw == 8) return post_launch<Kind, BITS, KV, 8, 8, kBlock>(a);
    if (a.wpb == 8 && a.nw == 4) return post_launch<Kind, BITS, KV, 8, 4, kBlock>(a);
    if (a.wpb == 16 && a.nw == 8) return post_launch<Kind, BITS, KV, 16, 8, kBlock>(a);
    if (a.wpb == 16 && a.nw == 16) {
      // (16384-element key-value tiles up to 64 buckets do not fit in LDS)
      if constexpr (postscan_lds_bytes<Kind, BITS, KV, 16, 16, kBlock>() <= kLdsLimit)
        return post_launch<Kind, BITS, KV, 16, 16, kBlock>(a);
      return hipErrorInvalidValue;
    }
    if (a.wpb == 4 && a.nw == 8) return post_launch<Kind, BITS, KV, 4, 8, kBlock>(a);
    if (a.wpb == 4 && a.nw == 16) return post_launch<Kind, BITS, KV, 4, 16, kBlock>(a);
  } else if (a.mode == kWaveMode) {
    if (a.wpb == 8 && a.nw == 8) return post_launch<Kind, BITS, KV, 8, 8, kWaveMode>(a);
    if (a.wpb == 4 && a.nw == 16) return post_launch<Kind, BITS, KV, 4, 16, kWaveMode>(a);
  } else if (a.mode == kDirect) {
    if (a.wpb == 8 && a.nw == 8) return post_launch<Kind, BITS, KV, 8, 8, kDirect>(a);
  }
  return hipErrorInvalidValue;
}

template <int Kind, int BITS>
hipError_t post_kv(const PostArgs& a) {
  return a.kv ? post_shape<Kind, BITS, true>(a) : post_shape<Kind, BITS, false>(a);
}

template <int Kind>
hipError_t post_dispatch(const PostArgs& a, int bits) {
  switch (bits) {
    case 0: return post_kv<Kind, 0>(a);
    case 1: return post_kv<Kind, 1>(a);
    case 2: return post_kv<Kind, 2>(a);
    case 3: return post_kv<Kind, 3>(a);
    case 4: return post_kv<Kind, 4>(a);
    case 5: return post_kv<Kind, 5>(a);
    case 6: return post_kv<Kind, 6>(a);
    case 7: return post_kv<Kind, 7>(a);
    case 8: return post_kv<Kind, 8>(a);
    default: return hipErrorInvalidValue;
  }
}

// Batched: shapes (waves per block, windows) with an instantiated kernel.
inline bool batched_shape_supported(int wpb, int nw) {
  return (wpb == 8 && (nw == 8 || nw == 4)) || (wpb == 4 && (nw == 16 || nw == 8)) ||
         (wpb == 16 && (nw == 4 || nw == 8));
}

template <int Kind, int BITS, bool KV, int WPB, int NW>
hipError_t batched_launch(const BatchedArgs& a, hipStream_t st) {
  auto kern = batched_kernel<Kind, BITS, KV, WPB, NW>;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WPB * kWave, 0) != hipSuccess)
    return hipErrorInvalidValue;
  if (per_cu < 1) per_cu = 1;
  hipLaunchKernelGGL(batched_setup_kernel, dim3(1), dim3(kSetupThreads), 0, st, a);
  hipLaunchKernelGGL(kern, dim3(per_cu * cus), dim3(WPB * kWave), 0, st, a);
  return hipGetLastError();
}

template <int Kind, int BITS>
hipError_t batched_shape(const BatchedArgs& a, bool kv, int wpb, int nw, hipStream_t st) {
  if (wpb == 8 && nw == 8)
    return kv ? batched_launch<Kind, BITS, true, 8, 8>(a, st) : batched_launch<Kind, BITS, false, 8, 8>(a, st);
  if (wpb == 8 && nw == 4)
    return kv ? batched_launch<Kind, BITS, true, 8, 4>(a, st) : batched_launch<Kind, BITS, false, 8, 4>(a, st);
  if (wpb == 4 && nw == 16)
    return kv ? batched_launch<Kind, BITS, true, 4, 16>(a, st) : batched_launch<Kind, BITS, false, 4, 16>(a, st);
  if (wpb == 4 && nw == 8)
    return kv ? batched_launch<Kind, BITS, true, 4, 8>(a, st) : batched_launch<Kind, BITS, false, 4, 8>(a, st);
  if (wpb == 16 && nw == 4)
    return kv ? batched_launch<Kind, BITS, true, 16, 4>(a, st) : batched_launch<Kind, BITS, false, 16, 4>(a, st);
  if (wpb == 16 && nw == 8)
    return kv ? batched_launch<Kind, BITS, true, 16, 8>(a, st) : batched_launch<Kind, BITS, false, 16, 8>(a, st);
  return hipErrorInvalidValue;
}

template <int Kind>
hipError_t batched_dispatch(const BatchedArgs& a, int bits, bool kv, int wpb, int nw,
                            hipStream_t st) {
  switch (bits) {
    case 0: return batched_shape<Kind, 0>(a, kv, wpb, nw, st);
    case 1: return batched_shape<Kind, 1>(a, kv, wpb, nw, st);
    case 2: return batched_shape<Kind, 2>(a, kv, wpb, nw, st);
    case 3: return batched_shape<Kind, 3>(a, kv, wpb, nw, st);
    case 4: return batched_shape<Kind, 4>(a, kv, wpb, nw, st);
    case 5: return batched_shape<Kind, 5>(a, kv, wpb, nw, st);
    case 6: return batched_shape<Kind, 6>(a, kv, wpb, nw, st);
    case 7: return batched_shape<Kind, 7>(a, kv, wpb, nw, st);
    case 8: return batched_shape<Kind, 8>(a, kv, wpb, nw, st);
    default: return hipErrorInvalidValue;
  }
}

// Entry points defined in the per-kind translation units.
hipError_t pre_shift_mask(const PreArgs& a, int bits);
hipError_t pre_div(const PreArgs& a, int bits);
hipError_t pre_splitters(const PreArgs& a, int bits);
hipError_t pre_learned(const PreArgs& a, int bits);
hipError_t post_shift_mask(const PostArgs& a, int bits);
hipError_t post_div(const PostArgs& a, int bits);
hipError_t post_splitters(const PostArgs& a, int bits);
hipError_t post_learned(const PostArgs& a, int bits);
hipError_t post_kept_ids(const PostArgs& a, int bits);
hipError_t batched_shift_mask(const BatchedArgs& a, int bits, bool kv, int wpb, int nw, hipStream_t st);
hipError_t batched_div(const BatchedArgs& a, int bits, bool kv, int wpb, int nw, hipStream_t st);
hipError_t batched_splitters(const BatchedArgs& a, int bits, bool kv, int wpb, int nw, hipStream_t st);
hipError_t batched_learned(const BatchedArgs& a, int bits, bool kv, int wpb, int nw, hipStream_t st);

}  // namespace ms
