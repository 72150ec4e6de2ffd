// rn_device.h -- device building blocks of the sweep kernels: the counter-based
// random numbers, the uniform conversions of both precisions, the Poisson and
// Langevin samplers and the mass-action combinatorial factor.  Included by the
// generic kernels (rn_sweep_kernel.h) and by the network-compiled kernels
// (rn_net_kernel.h), which the library builds at run time with hipRTC.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "rn_kernel.h"

namespace rn {
namespace dev {
namespace {


// Philox counter layout: (trajectory id, attempt counter n, slot, stream).
constexpr uint32_t kStreamEvent = 0u;  // slot 0: words 0-1 waiting time, 2-3 reaction pick
constexpr uint32_t kStreamFirst = 1u;  // slot j/2: words 2(j%2), 2(j%2)+1 = inversion uniform of j
constexpr uint32_t kStreamPtrs = 2u;   // slot j, stream 2+r: round r of the PTRS sampler for j
constexpr int kInvMax = 100;           // inversion search cap
constexpr uint32_t kPtrsMax = 1000u;   // PTRS round cap
constexpr double kClamp = 2147483648.0;  // draws are clamped to 2^31

enum : int { kDecide = 0, kSsa = 1, kLeap = 2, kDone = 3 };

constexpr uint32_t kStAbsorbed = 1u, kStMaxSteps = 2u, kStOverflow = 4u;

struct Words {
  uint32_t w0, w1, w2, w3;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key schedule is
// wave-uniform, so it stays in scalar registers.
__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t y2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = y0;
    c2 = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// Uniform on [0,1) with 53 random bits: the top 53 bits of (hi:lo) times 2^-53.
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
  const uint64_t z = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
  return (double)z * 0x1p-53;
}

// Uniform on [0,1) with 24 random bits: the top 24 bits of hi times 2^-24.
__device__ __forceinline__ float u24(uint32_t hi) { return (float)(hi >> 8) * 0x1p-24f; }

template <typename R>
struct Real;
template <>
struct Real<double> {
  static constexpr bool kF64 = true;
  __device__ static __forceinline__ double uni(uint32_t hi, uint32_t lo) { return u53(hi, lo); }
  __device__ static __forceinline__ double log_(double x) { return log(x); }
  __device__ static __forceinline__ double exp_(double x) { return exp(x); }
  __device__ static __forceinline__ double abs_(double x) { return fabs(x); }
};
template <>
struct Real<float> {
  static constexpr bool kF64 = false;
  __device__ static __forceinline__ float uni(uint32_t hi, uint32_t) { return u24(hi); }
  __device__ static __forceinline__ float log_(float x) { return logf(x); }
  __device__ static __forceinline__ float exp_(float x) { return expf(x); }
  __device__ static __forceinline__ float abs_(float x) { return fabsf(x); }
};
template <typename R>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(16)));
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(16)));
};

// 1/k, correctly rounded, for the inversion walk (k = 1 .. kInvMax).  The
// constant evaluator divides in IEEE round-to-nearest, so each entry is the
// quotient 1.0 / k itself.
template <typename R>
struct RecipTable {
  R v[kInvMax + 2];  // one spare entry: the walk reads one step ahead
  constexpr RecipTable() : v() {
    for (int k = 1; k <= kInvMax + 1; ++k) v[k] = R(1) / R(k);
  }
};
template <typename R>
__device__ __forceinline__ R recip(int k) {
  static constexpr RecipTable<R> table{};
  return table.v[k];
}

// Poisson(lam) for 0 < lam < 10: walk the CDF from k = 0 with one uniform,
// p_k = p_{k-1} * (lam * (1/k)).  In FP32 the walk also stops once a term no
// longer changes F (the CDF has saturated below u; the mass left is below the
// 24-bit resolution of u).
template <typename R>
__device__ __forceinline__ uint32_t poisson_inversion(R lam, R u) {
  R pk = Real<R>::exp_(-lam);
  R F = pk;
  int k = 0;
  // Every lane still walking has the same k, so 1/k comes from a scalar load,
  // issued one step ahead to hide its latency.
  R rk = recip<R>(1);
  while (u > F && k < kInvMax) {
    k = k + 1;
    const R r = rk;
    rk = recip<R>(k + 1);
    pk = pk * (lam * r);
    const R Fn = F + pk;
    if constexpr (!Real<R>::kF64) {
      if (Fn == F) break;
    }
    F = Fn;
  }
  return (uint32_t)k;
}

__device__ __forceinline__ uint32_t clamp_draw(double kf) {
  return kf < kClamp ? (uint32_t)kf : 0x80000000u;
}

// log(k!) for a non-negative integer k held in a double: the host-built table
// below kLogFactTable, else Stirling's series for log Gamma(x), x = k + 1, to the
// x^-5 term (the first omitted term is below 1e-18 for x >= 1024).
__device__ __forceinline__ double log_factorial(double kf, const double* table) {
  if (kf < (double)kLogFactTable) return table[(int)kf];
  const double x = kf + 1.0;
  const double r = 1.0 / x;
  const double r2 = r * r;
  const double series = r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0)));
  return (x - 0.5) * log(x) - x + 0.91893853320467274178 + series;
}

// Poisson(lam) for lam >= 10: Hoermann's transformed rejection with squeeze
// (PTRS, Insurance: Math. & Econ. 12 (1993) 39); round r draws its (U, V) pair
// from its own Philox block.  The body is inlined where a kernel has one call
// site; the out-of-line copy below serves kernels with many.
__device__ __forceinline__ uint32_t ptrs_body(double lam, uint32_t traj, uint32_t n, uint32_t j,
                                              uint32_t k0, uint32_t k1, const double* lfact) {
  const double smu = sqrt(lam);
  const double b = 0.931 + 2.53 * smu;
  const double a = -0.059 + 0.02483 * b;
  const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  const double vr = 0.9277 - 3.6224 / (b - 2.0);
  const double loglam = log(lam);
#pragma unroll 1
  for (uint32_t r = 0; r < kPtrsMax; ++r) {
    const Words w = philox10(traj, n, j, kStreamPtrs + r, k0, k1);
    const double U = u53(w.w0, w.w1) - 0.5;
    const double V = u53(w.w2, w.w3);
    const double us = 0.5 - fabs(U);
    const double kf = floor((2.0 * a / us + b) * U + lam + 0.43);
    if (us >= 0.07 && V <= vr) return clamp_draw(kf);
    if (kf < 0.0 || (us < 0.013 && V > us)) continue;
    const double lhs = log(V * inv_alpha / (a / (us * us) + b));
    const double rhs = -lam + kf * loglam - log_factorial(kf, lfact);
    if (lhs <= rhs) return clamp_draw(kf);
  }
  return clamp_draw(floor(lam));
}

__device__ __noinline__ uint32_t poisson_ptrs(double lam, uint32_t traj, uint32_t n, uint32_t j,
                                              uint32_t k0, uint32_t k1, const double* lfact) {
  return ptrs_body(lam, traj, n, j, k0, k1, lfact);
}

// Chemical Langevin increment for mean lam: round(lam + sqrt(lam) z), z standard
// normal by Box-Muller, (u1, u2) from the reaction's first PTRS block; floored
// at 0 and clamped like every draw.
__device__ __noinline__ uint32_t cle_count(double lam, uint32_t traj, uint32_t n, uint32_t j,
                                           uint32_t k0, uint32_t k1) {
  const Words w = philox10(traj, n, j, kStreamPtrs, k0, k1);
  const double u1 = u53(w.w0, w.w1);
  const double u2 = u53(w.w2, w.w3);
  const double z = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
  double kf = floor(lam + sqrt(lam) * z + 0.5);
  if (kf < 0.0) kf = 0.0;
  return clamp_draw(kf);
}

// kInline: the PTRS body is inlined (one call site per kernel) instead of called.
template <typename R, bool kInline = false>
__device__ __forceinline__ uint32_t poisson(R lam, uint32_t hi, uint32_t lo, uint32_t traj,
                                            uint32_t n, uint32_t j, uint32_t k0, uint32_t k1,
                                            const double* lfact, double cle) {
  if (!(lam > R(0))) return 0u;
  if (lam < R(10)) return poisson_inversion<R>(lam, Real<R>::uni(hi, lo));
  const double ld = (double)lam;
  if (cle > 0.0 && ld >= cle) return cle_count(ld, traj, n, j, k0, k1);
  if constexpr (kInline) return ptrs_body(ld, traj, n, j, k0, k1, lfact);
  else return poisson_ptrs(ld, traj, n, j, k0, k1, lfact);
}

// Fused ensemble statistics of one recorded state, counts x[i * stride] for
// i < n at sample si: exact sums of x and of x^2 (as the sums of its two
// 32-bit words) and the histogram counts, by device-wide atomic additions
// (every trajectory of the sweep adds to the same cells, at its own time).
// Out of line, so that each recording site of a kernel adds one call; the
// kernel passes the fields rather than its parameter block, whose address
// would force a private copy of it.
__device__ __noinline__ void add_stats_row(uint64_t* sum_x, uint64_t* sum_x2, uint32_t* hist,
                                           const int32_t* hist_lo, const int32_t* hist_width,
                                           int32_t bins, int n, int si, const int32_t* x,
                                           int stride) {
  for (int i = 0; i < n; ++i) {
    const int32_t v = x[i * stride];
    const int64_t cell = (int64_t)si * n + i;
    if (sum_x) {
      const uint64_t q = (uint64_t)((int64_t)v * (int64_t)v);
      __hip_atomic_fetch_add(sum_x + cell, (uint64_t)(uint32_t)v, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(sum_x2 + 2 * cell, q & 0xffffffffull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      if (q >> 32)
        __hip_atomic_fetch_add(sum_x2 + 2 * cell + 1, q >> 32, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (hist) {
      const int64_t d = (int64_t)v - (int64_t)hist_lo[i];
      uint32_t b = 0u;
      if (d > 0) {
        const uint64_t q = (uint64_t)d / (uint64_t)(uint32_t)hist_width[i];
        b = q < (uint64_t)bins ? (uint32_t)q : (uint32_t)(bins - 1);
      }
      __hip_atomic_fetch_add(hist + cell * bins + b, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Mass-action combinatorial factor h = A * B (halved for a homodimer, where
// B = A - 1), each count converted to R (exactly, for double).
template <typename R>
__device__ __forceinline__ R hval(int32_t A, int32_t B, int32_t dimer) {
  const R scale = dimer ? R(0.5) : R(1);  // wave-uniform; 1 * h == h exactly
  return scale * ((R)A * (R)B);
}

}  // namespace
}  // namespace dev
}  // namespace rn
