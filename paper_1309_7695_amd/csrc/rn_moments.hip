// rn_moments.hip -- ensemble moments of a sweep's samples.
//
// A parameter sweep is followed by statistics over its trajectories (paper,
// Aims and motivation section: sweeps, sensitivity analysis and parameter
// estimation all repeat many simulations and summarize them).  For every
// (sample s, species i) row of the trajectory-minor sample array this computes
// the exact integer sums  sum_t x  (int64)  and  sum_t x^2  (unsigned 128-bit),
// from which mean and variance follow exactly.
//
// One workgroup reduces one row: its 256 lanes stream the row with 16-byte
// loads when the row is 16-byte aligned (4-byte loads otherwise), accumulate in
// registers, then reduce across the wave with cross-lane shuffles and across the
// four waves through LDS.  The pass is bound by HBM reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rn_kernel.h"

namespace rn {
namespace {

constexpr int kMomWG = 256;

struct U128 {
  uint64_t lo, hi;
};

__device__ __forceinline__ void add128(U128& a, uint64_t lo, uint64_t hi) {
  const uint64_t s = a.lo + lo;
  a.hi += hi + (s < lo ? 1u : 0u);
  a.lo = s;
}

__device__ __forceinline__ void add_value(int64_t& sx, U128& sq, int32_t x) {
  sx += x;
  const int64_t x64 = x;
  add128(sq, (uint64_t)(x64 * x64), 0u);
}

template <bool kVec4>
__global__ __launch_bounds__(kMomWG) void moments_kernel(const int32_t* __restrict__ out,
                                                         int64_t out_ld, int64_t n_traj,
                                                         int64_t* __restrict__ sum_x,
                                                         uint64_t* __restrict__ sum_x2) {
  const int64_t row = blockIdx.x;
  const int32_t* r = out + row * out_ld;
  const int tid = (int)threadIdx.x;
  int64_t sx = 0;
  U128 sq = {0u, 0u};
  if constexpr (kVec4) {
    const int4* r4 = (const int4*)r;
    const int64_t n4 = n_traj >> 2;
    for (int64_t k = tid; k < n4; k += kMomWG) {
      const int4 v = r4[k];
      add_value(sx, sq, v.x);
      add_value(sx, sq, v.y);
      add_value(sx, sq, v.z);
      add_value(sx, sq, v.w);
    }
    for (int64_t k = (n4 << 2) + tid; k < n_traj; k += kMomWG) add_value(sx, sq, r[k]);
  } else {
    for (int64_t k = tid; k < n_traj; k += kMomWG) add_value(sx, sq, r[k]);
  }
  // wave reduction
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t ox = __shfl_xor(sx, off);
    const uint64_t olo = __shfl_xor(sq.lo, off);
    const uint64_t ohi = __shfl_xor(sq.hi, off);
    sx += ox;
    add128(sq, olo, ohi);
  }
  __shared__ int64_t px[kMomWG / 64];
  __shared__ uint64_t plo[kMomWG / 64], phi[kMomWG / 64];
  const int wave = tid >> 6;
  if ((tid & 63) == 0) {
    px[wave] = sx;
    plo[wave] = sq.lo;
    phi[wave] = sq.hi;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t tx = 0;
    U128 tq = {0u, 0u};
    for (int w = 0; w < kMomWG / 64; ++w) {
      tx += px[w];
      add128(tq, plo[w], phi[w]);
    }
    sum_x[row] = tx;
    sum_x2[2 * row] = tq.lo;
    sum_x2[2 * row + 1] = tq.hi;
  }
}

// Fused statistics of a sweep: the arrays start at zero; during the sweep each
// x^2 sum is kept as the sums A and B of its low and high 32-bit words (each
// below 2^64 for fewer than 2^32 trajectories), and afterwards
// A + B * 2^32 is written back as a 128-bit (low, high) pair.
__global__ void stats_zero_kernel(uint64_t* sum_x, uint64_t* sum_x2, int64_t cells,
                                  uint32_t* hist, int64_t hcells) {
  const int64_t n = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells; k += n) {
    sum_x[k] = 0u;
    sum_x2[2 * k] = 0u;
    sum_x2[2 * k + 1] = 0u;
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < hcells; k += n)
    hist[k] = 0u;
}

__global__ void stats_finish_kernel(uint64_t* sum_x2, int64_t cells) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cells) return;
  const uint64_t a = sum_x2[2 * k], b = sum_x2[2 * k + 1];
  const uint64_t lo = a + (b << 32);
  sum_x2[2 * k] = lo;
  sum_x2[2 * k + 1] = (b >> 32) + (lo < a ? 1u : 0u);
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p,
                     n, v);
  return hipGetLastError();
}

hipError_t launch_stats_zero(const SweepParams& p, hipStream_t stream) {
  const int64_t cells = p.sum_x ? (int64_t)p.n_times * p.net.N : 0;
  const int64_t hcells = p.hist ? (int64_t)p.n_times * p.net.N * p.hist_bins : 0;
  const int64_t most = cells > hcells ? cells : hcells;
  if (most == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((most + 255) / 256, 4096);
  hipLaunchKernelGGL(stats_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p.sum_x,
                     p.sum_x2, cells, p.hist, hcells);
  return hipGetLastError();
}

hipError_t launch_stats_finish(const SweepParams& p, hipStream_t stream) {
  if (!p.sum_x2) return hipSuccess;
  const int64_t cells = (int64_t)p.n_times * p.net.N;
  hipLaunchKernelGGL(stats_finish_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0,
                     stream, p.sum_x2, cells);
  return hipGetLastError();
}

hipError_t launch_moments(const int32_t* out, int64_t out_ld, int64_t rows, int64_t n_traj,
                          int64_t* sum_x, uint64_t* sum_x2, hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  const bool vec4 = (out_ld % 4 == 0) && (((uintptr_t)out & 15u) == 0);
  if (vec4)
    hipLaunchKernelGGL(moments_kernel<true>, dim3((unsigned)rows), dim3(kMomWG), 0, stream, out,
                       out_ld, n_traj, sum_x, sum_x2);
  else
    hipLaunchKernelGGL(moments_kernel<false>, dim3((unsigned)rows), dim3(kMomWG), 0, stream, out,
                       out_ld, n_traj, sum_x, sum_x2);
  return hipGetLastError();
}

}  // namespace rn
