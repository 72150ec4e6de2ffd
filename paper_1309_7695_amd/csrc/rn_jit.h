// rn_jit.h -- internal interface of the network-compiled sweep kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "rn_kernel.h"

namespace rn {

constexpr int kJitFP64 = 0, kJitFP32 = 1;
// Networks whose counts and rates fit the compiled kernel's registers.
constexpr int kJitMaxSpecies = 63, kJitMaxReactions = 128;

// Row stride (words) of the dense stoichiometry matrix for n species: whole
// 16-byte vectors plus one more, which moves consecutive rows to other banks.
inline int jit_dense_ld(int n) { return 4 * ((n + 3) / 4) + 4; }

// LDS of one workgroup: the dense matrix [M][jit_dense_ld(N)] and every lane's
// N-word leap candidate.
inline size_t jit_lds_bytes(int n, int m, int wg) {
  return ((size_t)m * jit_dense_ld(n) + (size_t)n * wg) * sizeof(int32_t);
}

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
