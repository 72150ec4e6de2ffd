// rn_jit.h -- internal interface of the network-compiled sweep kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "rn_kernel.h"

namespace rn {

constexpr int kJitFP64 = 0, kJitFP32 = 1;
// Added to the precision: the exact-SSA kernel with the reaction dependency
// graph (sweep_net_ssa) instead of the general one.
constexpr int kJitSsaDep = 2;
// Networks whose counts and rates fit the compiled kernel's registers.
constexpr int kJitMaxSpecies = 63, kJitMaxReactions = 128;

// Row stride (words) of the dense stoichiometry matrix for n species: whole
// 16-byte vectors plus one more, which moves consecutive rows to other banks.
inline int jit_dense_ld(int n) { return 4 * ((n + 3) / 4) + 4; }

// LDS of one workgroup: the dense matrix [M][jit_dense_ld(N)], every lane's
// N-word leap candidate, and each wave's leap draw list (means [16][64],
// counts [16][64], attempt counters [64], items [8 * 64]).
inline size_t jit_lds_bytes(int n, int m, int wg, bool fp32) {
  const size_t wave_words = 16 * 64 * (fp32 ? 1 : 2) + 16 * 64 + 64 + 8 * 64;
  return ((size_t)m * jit_dense_ld(n) + (size_t)n * wg + (size_t)(wg / 64) * wave_words) *
         sizeof(int32_t);
}

// LDS of one workgroup of the dependency-graph SSA kernel: the compact
// stoichiometry (m + 1 offsets, nnz entries), then per lane n count words and
// the group start sums of its pick (groups as in ssa_group of the kernel).
inline size_t jit_ssa_lds_bytes(int n, int m, int nnz, int wg, bool fp32) {
  const int rw = fp32 ? 1 : 2;
  int gs = 4;
  while (gs < m && rw * ((m + gs - 1) / gs - 1) > n) gs *= 2;
  const int g = (m + gs - 1) / gs;
  const size_t off = ((size_t)(m + 1 + nnz) + 3) / 4 * 4;
  return (off + (size_t)n * wg + (size_t)(g - 1) * rw * wg) * sizeof(int32_t);
}
// The dependency-graph kernel keeps M propensities in registers: networks
// with M * (words per value) <= kJitSsaDepMaxWords.
constexpr int kJitSsaDepMaxWords = 200;

// False when the environment sets RN_JIT=0 (the generic kernels are used).
bool jit_enabled();
// The compiled kernel for a network prelude, compiled on first use; null when
// hipRTC is unavailable or the compilation fails.
hipFunction_t jit_kernel(const std::string& consts, int precision, int wg);
// The compiled kernel if it is ready now; otherwise null, after starting its
// compilation on a background thread (so a later call finds it).
hipFunction_t jit_kernel_nowait(const std::string& consts, int precision, int wg);
// Drop background compilations not yet started (their networks keep the
// generic kernels) and wait for the running ones.
void jit_drain();
hipError_t jit_launch(hipFunction_t fn, const SweepParams& p, int wg, size_t lds,
                      hipStream_t stream);

}  // namespace rn
