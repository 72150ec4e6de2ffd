// rn_wsweep.hip -- the sweep with one wave64 per trajectory, for networks too
// large for the network-compiled kernel (up to 512 reactions).  The method is
// the same Cao-Gillespie-Petzold tau-leaping with critical reactions and SSA
// bursts as rn_sweep_kernel.h (the paper's Methods section: X(t) counts
// molecules, each firing adds the reaction's stoichiometric vector), and every
// trajectory is bit for bit the one the lane-per-trajectory kernels give.
//
// Lane l holds reactions j = l + 64k (k < K: rate constant, rate law,
// propensity in registers) and species i = l + 64m.  A step's reaction-wise
// work (propensities, critical flags, Poisson draws) and species-wise work
// (leap-condition bounds, the candidate state) is spread over the lanes; the
// results whose value depends on summation order (a0, the SSA pick, a0c and
// the critical pick) come from one walk over the reactions in index order, in
// which every lane adds the broadcast propensity of reaction j to a running sum
// and lane j % 64 keeps the partial sum for the pick.  A lane-per-trajectory
// kernel pays O(M) issue slots per step on one lane's critical path; here the
// critical path of a step is the index-order walk only, so a sweep of few
// trajectories finishes in a fraction of the time.
//
// LDS, per wave: counts x[N + 1] (x[N] == 1 for lower-order rate laws), the
// propensities a[M] for the species-wise sums, the leap draws k[M], and the
// critical bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rn_device.h"
#include "rn_kernel.h"

namespace rn {
namespace {
using namespace dev;

typedef const int32_t __attribute__((address_space(4)))* const_i32_ptr;
__device__ __forceinline__ int32_t sld(const void* base, int64_t i) {
  return ((const_i32_ptr)base)[i];
}

// Value of v on lane l (l wave-uniform), on every lane.
__device__ __forceinline__ double bcast(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float bcast(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Smallest value over the wave (no NaN): min is exact and order-free, so a
// butterfly gives every lane the same result.
template <typename R>
__device__ __forceinline__ R wave_min(R v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const R o = __shfl_xor(v, m, 64);
    v = o < v ? o : v;
  }
  return v;
}

// Index-order walk: sum = ((v_0 + v_1) + v_2) + ... over reactions j < m, where
// v_j sits on lane j % 64 in v[j / 64]; cend[k] receives the running sum after
// the last reaction of chunk k.  Every lane returns the full sum.  Eight
// broadcasts are issued ahead of their additions, so that only the chain of
// additions is serial.
template <int K, typename S>
__device__ __forceinline__ S ordered_sum(const S (&v)[K], S (&cend)[K], int m) {
  S sum = S(0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int n = min(64, m - 64 * k);
    int l = 0;
    for (; l + 8 <= n; l += 8) {
      S b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = bcast(v[k], l + u);
#pragma unroll
      for (int u = 0; u < 8; ++u) sum = sum + b[u];
    }
    for (; l < n; ++l) sum = sum + bcast(v[k], l);
    cend[k] = sum;
  }
  return sum;
}

// The first reaction j < m whose running sum (the walk above) exceeds r, or -1.
// The running sums never decrease (the values are non-negative), so j lies in
// the first chunk whose end sum exceeds r; only that chunk is walked again,
// from the sum the walk had on entering it, each lane keeping the partial sum
// through its own reaction.
template <int K, typename S>
__device__ __forceinline__ int ordered_pick(const S (&v)[K], const S (&cend)[K], S r, int m,
                                            int lane) {
  int pick = -1;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (pick >= 0 || 64 * k >= m || !(r < cend[k])) continue;
    S acc = k > 0 ? cend[k - 1] : S(0);
    S pre = S(0);
    const int n = min(64, m - 64 * k);
    for (int l = 0; l < n; ++l) {
      acc = acc + bcast(v[k], l);
      pre = lane == l ? acc : pre;
    }
    const uint64_t hit = __ballot(lane < n && r < pre);
    pick = 64 * k + __builtin_ctzll(hit);  // hit != 0: lane n - 1 holds cend[k] > r
  }
  return pick;
}

// The last reaction (in index order) whose lane flag is set, or -1.
template <int K>
__device__ __forceinline__ int last_set(const bool (&f)[K]) {
  int r = -1;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t b = __ballot(f[k]);
    if (b) r = 64 * k + 63 - __builtin_clzll(b);
  }
  return r;
}

// One trajectory per 64-lane workgroup.  K: reaction registers per lane
// (M_real <= 64 K).
template <int K, typename R, int kWaves>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWaves)))
void wsweep_kernel(const SweepParams p) {
  extern __shared__ int32_t lds[];
  const DevNet& g = p.net;
  const int N = g.N, M = g.M_real;
  const int lane = (int)threadIdx.x;
  const int64_t tl = blockIdx.x;
  if (tl >= p.n_traj) return;
  const uint32_t traj = p.traj_offset + (uint32_t)tl;
  const uint32_t k0 = p.key0, k1 = p.key1;
  const int S = p.n_times;
  const double* __restrict__ times = p.times;

  const int xw = (N + 2) & ~1;  // words of x, even so that a[] is 8-byte aligned
  int32_t* const x = lds;
  R* const a_l = (R*)(lds + xw);
  uint32_t* const kd = (uint32_t*)(a_l + M);
  uint32_t* const critw = kd + M;

  // the lane's reactions: rate constant and packed rate law
  // (ia | ib << 15 | dimer << 30; the homodimer law has db == -1)
  R c[K];
  int32_t law[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = lane + 64 * k;
    c[k] = R(0);
    law[k] = N | (N << 15);
    if (j < M) {
      c[k] = (R)p.rates[(int64_t)j * p.rates_ld + tl];
      const int ia = g.law[j].ia, ib = g.law[j].ib, dm = g.law[j].dimer;
      law[k] = ia | (ib << 15) | (dm ? 1 << 30 : 0);
    }
  }
  auto prop = [&](int k) -> R {
    const int L = law[k];
    const int ia = L & 0x7fff, ib = (L >> 15) & 0x7fff, dm = (L >> 30) & 1;
    return c[k] * hval<R>(x[ia], x[ib] - dm, dm);
  };

  for (int i = lane; i < N; i += 64)
    x[i] = p.x0_ld ? p.x0[(int64_t)i * p.x0_ld + tl] : p.x0[i];
  if (lane == 0) x[N] = 1;
  __syncthreads();

  double t = 0.0, tau_p = 0.0, a0 = 0.0;
  double t_next = S > 0 ? times[0] : 0.0;
  uint32_t n = 0, burst_left = 0, status = 0;
  uint64_t leaps = 0, ssa = 0, rej = 0;
  int s = 0;
  int mode = p.method == 1 ? kSsa : kDecide;
  const bool ssa_only = p.method == 1;

  auto record = [&](int si) {
    if (p.out) {
      if (p.out_traj_major) {
        int32_t* o = p.out + tl * p.out_ld + (int64_t)si * N;
        for (int i = lane; i < N; i += 64) o[i] = x[i];
      } else {
        int32_t* o = p.out + (int64_t)si * N * p.out_ld + tl;
        for (int i = lane; i < N; i += 64) o[(int64_t)i * p.out_ld] = x[i];
      }
    }
    if (p.sum_x || p.hist) {
      for (int i = lane; i < N; i += 64) {
        const int32_t v = x[i];
        const int64_t cell = (int64_t)si * N + i;
        if (p.sum_x) {
          const uint64_t q = (uint64_t)((int64_t)v * (int64_t)v);
          __hip_atomic_fetch_add(p.sum_x + cell, (uint64_t)(uint32_t)v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_add(p.sum_x2 + 2 * cell, q & 0xffffffffull, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          if (q >> 32)
            __hip_atomic_fetch_add(p.sum_x2 + 2 * cell + 1, q >> 32, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (p.hist) {
          const int64_t d = (int64_t)v - (int64_t)p.hist_lo[i];
          uint32_t b = 0u;
          if (d > 0) {
            const uint64_t q = (uint64_t)d / (uint64_t)(uint32_t)p.hist_width[i];
            b = q < (uint64_t)p.hist_bins ? (uint32_t)q : (uint32_t)(p.hist_bins - 1);
          }
          __hip_atomic_fetch_add(p.hist + cell * p.hist_bins + b, 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  };
  auto record_next = [&]() {
    record(s);
    s = s + 1;
    if (s < S) t_next = times[s];
  };
  auto finish = [&](uint32_t why) {
    status |= why;
    while (s < S) record(s++);
    mode = kDone;
  };
  auto steps = [&]() -> uint64_t { return leaps + ssa + rej; };

  while (s < S && t_next <= t) record_next();
  if (s == S) mode = kDone;

  R a[K];
  while (mode != kDone) {
    if (steps() >= p.max_steps) {
      finish(kStMaxSteps);
      break;
    }

    // ---------------- one exact SSA event ----------------
    if (mode == kSsa) {
#pragma unroll
      for (int k = 0; k < K; ++k) a[k] = prop(k);
      R cend[K];
      const R sum = ordered_sum<K, R>(a, cend, M);
      if (sum == R(0)) {
        finish(kStAbsorbed);
        break;
      }
      const Words w = philox10(traj, n, 0u, kStreamEvent, k0, k1);
      const R tau = -Real<R>::log_(R(1) - Real<R>::uni(w.w0, w.w1)) / sum;
      const double tn = t + (double)tau;
      while (s < S && t_next < tn) record_next();
      if (s == S) {
        mode = kDone;
        break;
      }
      const R r = Real<R>::uni(w.w2, w.w3) * sum;
      int pick = ordered_pick<K, R>(a, cend, r, M, lane);
      if (pick < 0) {
        bool pos[K];
#pragma unroll
        for (int k = 0; k < K; ++k) pos[k] = lane + 64 * k < M && a[k] > R(0);
        pick = last_set<K>(pos);
      }
      if (pick < 0) {
        finish(kStAbsorbed);
        break;
      }
      // the fired reaction's net changes, one species per lane (all distinct)
      const int e0 = sld(g.nu_ptr, pick), e1 = sld(g.nu_ptr, pick + 1);
      bool bad = false;
      for (int e = e0 + lane; e < e1; e += 64) {
        const int2 en = g.nu_ent[e];
        const int64_t y = (int64_t)x[en.x] + en.y;
        bad = bad || y > INT32_MAX || y < 0;
      }
      if (__any(bad)) {
        finish(kStOverflow);
        break;
      }
      for (int e = e0 + lane; e < e1; e += 64) {
        const int2 en = g.nu_ent[e];
        x[en.x] += en.y;
      }
      __syncthreads();
      t = tn;
      n = n + 1;
      ssa = ssa + 1;
      while (s < S && t_next <= t) record_next();
      if (s == S) {
        mode = kDone;
        break;
      }
      if (!ssa_only && --burst_left == 0) mode = kDecide;
      continue;
    }

    // ---------------- decide: propensities, critical set, tau' ----------------
    if (mode == kDecide) {
      double ad[K];
      bool cr[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = lane + 64 * k;
        a[k] = prop(k);
        ad[k] = (double)a[k];
        cr[k] = false;
        if (j < M) {
          a_l[j] = a[k];
          if (a[k] > R(0)) {
            const int c1 = g.cons_ptr[j + 1];
            for (int q = g.cons_ptr[j]; q < c1; ++q) {
              const int2 ce = g.cons_ent[q];
              if ((int64_t)x[ce.x] < (int64_t)p.n_c * ce.y) cr[k] = true;
            }
          }
        }
      }
      double cend[K];
      const double sum = ordered_sum<K, double>(ad, cend, M);
      // critical bits as words of 32 reactions
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint64_t b = __ballot(cr[k]);
        if (lane == 0 && 64 * k < M) critw[2 * k] = (uint32_t)b;
        if (lane == 0 && 64 * k + 32 < M) critw[2 * k + 1] = (uint32_t)(b >> 32);
      }
      __syncthreads();
      a0 = sum;
      if (sum == 0.0) {
        finish(kStAbsorbed);
        break;
      }
      R tp = (R)__builtin_inf();
      const R eps = (R)p.eps;
      for (int r = lane; r < g.n_rs; r += 64) {
        const TauSpecies ts = g.rs[r];
        R mu = R(0), sig = R(0);
        for (int q = ts.begin; q < ts.end; ++q) {
          const int2 en = g.rs_ent[q];
          if ((critw[en.x >> 5] >> (en.x & 31)) & 1u) continue;
          const R av = a_l[en.x];
          mu = mu + (R)en.y * av;
          sig = sig + (R)(en.y * en.y) * av;
        }
        const int32_t xi = x[ts.species];
        R bnd = R(1);
        if (xi > 1) {
          const R gi = ts.gkind == 1 ? R(1) : ts.gkind == 2 ? R(2) : R(2) + R(1) / (R)(xi - 1);
          bnd = eps * (R)xi / gi;
          if (bnd < R(1)) bnd = R(1);
        }
        if (mu != R(0)) {
          const R q = bnd / Real<R>::abs_(mu);
          if (q < tp) tp = q;
        }
        if (sig != R(0)) {
          const R q = (bnd * bnd) / sig;
          if (q < tp) tp = q;
        }
      }
      tau_p = (double)wave_min<R>(tp);
      mode = kLeap;
      continue;
    }

    // ---------------- one leap attempt ----------------
    if (tau_p < p.ssa_factor / a0) {
      mode = kSsa;
      burst_left = (uint32_t)p.ssa_burst;
      continue;
    }
    bool crk[K];
    double vc[K];
    uint64_t cmask[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = lane + 64 * k;
      a[k] = prop(k);
      crk[k] = j < M && ((critw[j >> 5] >> (j & 31)) & 1u);
      vc[k] = (double)a[k];
      cmask[k] = __ballot(crk[k]);
    }
    // a0c: the critical reactions' propensities added in index order (the
    // others contribute nothing), one broadcast per critical reaction
    double a0c = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      for (uint64_t b = cmask[k]; b; b &= b - 1) a0c = a0c + bcast(vc[k], __builtin_ctzll(b));
    }
    Words ev = {0u, 0u, 0u, 0u};
    double tau_c = __builtin_inf();
    if (a0c > 0.0) {
      ev = philox10(traj, n, 0u, kStreamEvent, k0, k1);
      tau_c = -log(1.0 - u53(ev.w0, ev.w1)) / a0c;
    }
    const double delta = t_next - t;
    const bool fire = (tau_c <= tau_p) && (tau_c <= delta);
    const double tau = fire ? tau_c : (tau_p < delta ? tau_p : delta);

    // Poisson firings of the non-critical reactions over tau
    const R taur = (R)tau;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = lane + 64 * k;
      if (j >= M) continue;
      const R lam = crk[k] ? R(0) : a[k] * taur;
      Words w = {0u, 0u, 0u, 0u};
      if (lam > R(0) && lam < R(10))
        w = philox10(traj, n, (uint32_t)(j >> 1), kStreamFirst, k0, k1);
      const uint32_t hi = (j & 1) ? w.w2 : w.w0;
      const uint32_t lo = (j & 1) ? w.w3 : w.w1;
      kd[j] = poisson<R>(lam, hi, lo, traj, n, (uint32_t)j, k0, k1, g.log_fact,
                         p.cle_threshold);
    }
    if (fire) {
      // the first critical reaction whose running sum exceeds r, walking the
      // same additions again; else the last one with a positive propensity
      const double r = u53(ev.w2, ev.w3) * a0c;
      int jc = -1, last = -1;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        for (uint64_t b = cmask[k]; b && jc < 0; b &= b - 1) {
          const int l = __builtin_ctzll(b);
          const double av = bcast(vc[k], l);
          acc = acc + av;
          if (av > 0.0) last = 64 * k + l;
          if (r < acc) jc = 64 * k + l;
        }
      }
      if (jc < 0) jc = last;
      if (jc < 0) {
        finish(kStAbsorbed);
        break;
      }
      if (lane == (jc & 63)) kd[jc] = 1u;
    }
    __syncthreads();
    // the candidate state, exact in 64 bits (lane l: species l + 64m)
    int32_t nx[kWsweepMaxSpecies / 64];
    bool neg = false, big = false;
#pragma unroll
    for (int m = 0; m < kWsweepMaxSpecies / 64; ++m) {
      const int i = lane + 64 * m;
      if (i >= N) break;
      int64_t acc = x[i];
      const int q1 = g.col_ptr[i + 1];
      for (int q = g.col_ptr[i]; q < q1; ++q) {
        const int2 en = g.col_ent[q];
        acc += (int64_t)kd[en.x] * en.y;
      }
      if (acc < 0) neg = true;
      else if (acc > INT32_MAX) big = true;
      nx[m] = (int32_t)acc;
    }
    if (__any(neg)) {
      tau_p = tau_p * 0.5;
      n = n + 1;
      rej = rej + 1;
      __syncthreads();  // every lane has read kd before the next attempt rewrites it
      continue;         // stays in leap mode
    }
    if (__any(big)) {
      finish(kStOverflow);
      break;
    }
    // accepted: each lane rewrites its own species once every lane's reads are done
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kWsweepMaxSpecies / 64; ++m) {
      const int i = lane + 64 * m;
      if (i >= N) break;
      x[i] = nx[m];
    }
    __syncthreads();
    if (tau == delta) t = t_next;
    else t = t + tau;
    n = n + 1;
    leaps = leaps + 1;
    while (s < S && t_next <= t) record_next();
    if (s == S) {
      mode = kDone;
      break;
    }
    mode = kDecide;
  }

  if (lane == 0) {
    uint64_t* st = p.stats + tl * 4;
    st[0] = leaps;
    st[1] = ssa;
    st[2] = rej;
    st[3] = status;
  }
}

// Occupancy forms, for sweeps with more trajectories than the chip has SIMDs:
//  * K = 8 needs 275-302 registers, one wave per SIMD; the two-wave form caps it
//    at 256 (16-53 registers spill to scratch) and is 1.5-1.65x faster on
//    sweeps of 1,900-15,000 trajectories of 300-450 reactions (6% slower on
//    285 trajectories, where the chip has SIMDs to spare anyway);
//  * K = 1 runs three waves per SIMD (167-168 registers, at most 15 spilled):
//    1.12-1.45x on 2,100-3,100 trajectories of 20-55 reactions.  For K = 2 and
//    4 three waves measured no faster, or slower.
template <int K, typename R>
hipError_t launch_k(const SweepParams& p, size_t lds, bool many, hipStream_t stream) {
  const dim3 grid((unsigned)p.n_traj), block(64);
  if (K == 8 && many)
    hipLaunchKernelGGL((wsweep_kernel<K, R, 2>), grid, block, lds, stream, p);
  else if (K == 1 && many)
    hipLaunchKernelGGL((wsweep_kernel<K, R, 3>), grid, block, lds, stream, p);
  else
    hipLaunchKernelGGL((wsweep_kernel<K, R, 1>), grid, block, lds, stream, p);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_prec(const SweepParams& p, size_t lds, bool many, hipStream_t stream) {
  const int m = p.net.M_real;
  if (m <= 64) return launch_k<1, R>(p, lds, many, stream);
  if (m <= 128) return launch_k<2, R>(p, lds, many, stream);
  if (m <= 256) return launch_k<4, R>(p, lds, many, stream);
  if (m <= 512) return launch_k<8, R>(p, lds, many, stream);
  return hipErrorInvalidValue;
}

}  // namespace

bool wsweep_fits(int n_species, int m_real) {
  return n_species >= 1 && n_species <= kWsweepMaxSpecies && m_real <= kWsweepMaxReactions;
}

size_t wsweep_lds_bytes(int n_species, int m_real, bool fp32) {
  const size_t xw = (size_t)((n_species + 2) & ~1);
  return xw * 4 + (size_t)m_real * (fp32 ? 4 : 8) + (size_t)m_real * 4 +
         (size_t)((m_real + 63) / 64) * 8;
}

hipError_t launch_wsweep(const SweepParams& p, bool fp32, int n_simd, hipStream_t stream) {
  if (p.n_traj <= 0) return hipSuccess;
  const size_t lds = wsweep_lds_bytes(p.net.N, p.net.M_real, fp32);
  const bool many = p.n_traj > (int64_t)n_simd;
  return fp32 ? launch_prec<float>(p, lds, many, stream) : launch_prec<double>(p, lds, many, stream);
}

}  // namespace rn
