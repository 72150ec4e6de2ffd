// rn_wave.h -- wave-level helpers of the one-wave-per-trajectory kernels
// (rn_hybrid.hip, rn_ros.hip): a trajectory's species sit one per lane, so
// sums over species are wave reductions and scalars move between lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rn_kernel.h"

namespace rn {
namespace wave {
namespace {

// v from another lane of the same row of 16 through DPP (both halves moved
// with the same control word).
template <int kCtrl>
__device__ __forceinline__ double dpp_double(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), kCtrl, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double lane_double(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave, the same bits on every lane.  Within each
// row of 16 lanes: partner lanes xor 1 and xor 2 (quad permutations), then the
// mirror of the half row and of the row; each level adds the same two operands
// in either order, so all 16 lanes hold the same row sum.  The four row sums
// are then added as (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum(double v) {
  v = v + dpp_double<0xB1>(v);   // quad_perm [1,0,3,2]
  v = v + dpp_double<0x4E>(v);   // quad_perm [2,3,0,1]
  v = v + dpp_double<0x141>(v);  // row_half_mirror
  v = v + dpp_double<0x140>(v);  // row_mirror
  return (lane_double(v, 0) + lane_double(v, 16)) + (lane_double(v, 32) + lane_double(v, 48));
}

// Largest value over the 64 lanes, the same on every lane (the same DPP
// pattern as wave_sum; the values must not be NaN).
__device__ __forceinline__ double wave_max(double v) {
  double o = dpp_double<0xB1>(v);
  v = o > v ? o : v;
  o = dpp_double<0x4E>(v);
  v = o > v ? o : v;
  o = dpp_double<0x141>(v);
  v = o > v ? o : v;
  o = dpp_double<0x140>(v);
  v = o > v ? o : v;
  const double a = lane_double(v, 0), b = lane_double(v, 16);
  const double c = lane_double(v, 32), d = lane_double(v, 48);
  const double ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// A rate law packed for registers: ia | ib << 8 | dimer << 16 (species < 256).
__device__ __forceinline__ int pack_law(const RateLaw& law) {
  return law.ia | (law.ib << 8) | (law.dimer ? 1 << 16 : 0);
}

}  // namespace
}  // namespace wave
}  // namespace rn
