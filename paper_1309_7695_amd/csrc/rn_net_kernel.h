// rn_net_kernel.h -- the sweep kernel compiled for one network.
//
// The library builds this source at run time with hipRTC, after a generated
// prelude that defines the loaded network as compile-time constants in
// namespace rnnet (N species, M reactions, rate laws, stoichiometry, consumed
// reactants, reactant species with their g rule, species-major changes; see
// rn_jit.cpp).  Every loop over reactions or species is expanded at compile
// time, so each species count x_i, rate constant c_j and critical bit sits in
// a fixed register and a propensity is a few register operations: no table
// reads, no LDS round trips.  The method, the random-number layout and the
// floating-point operations, in their order, are those of the generic kernel
// (rn_sweep_kernel.h): both give identical trajectories.
//
// Two steps pick a reaction that differs between lanes (an SSA event and a
// critical firing); they add that reaction's row of the dense stoichiometry
// matrix, which the workgroup keeps in LDS.  Leap draws run in a rolled loop
// over each block of 16 reactions (the samplers are long) and are applied,
// reaction by reaction, to candidate counts in lane-private LDS words.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "rn_device.h"
#include "rn_kernel.h"

namespace rn {
namespace netk {
namespace {
using namespace dev;

// Compile-time loops: f(Ix<i>{}) for i = B .. E-1.
template <typename T, T... I>
struct ISeq {};
template <int V>
struct Ix {
  static constexpr int value = V;
};
template <int B, typename F, int... I>
__device__ __forceinline__ void sfor_(F& f, ISeq<int, I...>*) {
  (f(Ix<B + I>{}), ...);
}
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (E > B) sfor_<B>(f, (__make_integer_seq<ISeq, int, E - B>*)nullptr);
}

// An empty asm that claims to change v (and emits nothing).
__device__ __forceinline__ void opaque(int32_t& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void opaque(uint32_t& v) { asm volatile("" : "+v"(v)); }
template <typename T, int... I>
__device__ __forceinline__ void opaque_all_(T* x, ISeq<int, I...>*) {
  (opaque(x[I]), ...);
}

// The lane's rate constants in accumulation registers (AGPRs): written once,
// read with v_accvgpr_read at each use, so the architectural VGPRs are left to
// the counts and the working values of each phase.
template <typename R, int M>
struct RateRegs;
template <int M>
struct RateRegs<double, M> {
  uint32_t lo[M], hi[M];
  __device__ __forceinline__ void put(int j, double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    asm volatile("v_accvgpr_write_b32 %0, %1" : "=a"(lo[j]) : "v"((uint32_t)u));
    asm volatile("v_accvgpr_write_b32 %0, %1" : "=a"(hi[j]) : "v"((uint32_t)(u >> 32)));
  }
  __device__ __forceinline__ double get(int j) const {
    uint32_t l, h;
    asm("v_accvgpr_read_b32 %0, %1" : "=v"(l) : "a"(lo[j]));
    asm("v_accvgpr_read_b32 %0, %1" : "=v"(h) : "a"(hi[j]));
    return __builtin_bit_cast(double, ((uint64_t)h << 32) | l);
  }
};
template <int M>
struct RateRegs<float, M> {
  uint32_t w[M];
  __device__ __forceinline__ void put(int j, float v) {
    asm volatile("v_accvgpr_write_b32 %0, %1" : "=a"(w[j]) : "v"(__builtin_bit_cast(uint32_t, v)));
  }
  __device__ __forceinline__ float get(int j) const {
    uint32_t u;
    asm("v_accvgpr_read_b32 %0, %1" : "=v"(u) : "a"(w[j]));
    return __builtin_bit_cast(float, u);
  }
};

// One Poisson draw of reaction j for mean lam, with its inversion uniform
// (the exact 64-bit path, which is rare, calls it once per stoichiometry
// entry; keeping it out of line keeps that path small).
template <typename R>
__device__ __noinline__ uint32_t draw_one(R lam, uint32_t traj, uint32_t n, uint32_t j,
                                          uint32_t k0, uint32_t k1, const double* lfact,
                                          double cle) {
  Words w = {0u, 0u, 0u, 0u};
  if (lam > R(0) && lam < R(10)) w = philox10(traj, n, j >> 1, kStreamFirst, k0, k1);
  const uint32_t hi = (j & 1) ? w.w2 : w.w0;
  const uint32_t lo = (j & 1) ? w.w3 : w.w1;
  return poisson<R>(lam, hi, lo, traj, n, j, k0, k1, lfact, cle);
}

// Words of one wave's leap draw list: means [16][64] of type R, counts
// [16][64], attempt counters [64], items [8 * 64].
template <typename R>
constexpr int kLeapWaveWords = 16 * 64 * (int)(sizeof(R) / 4) + 16 * 64 + 64 + 8 * 64;

// Group size of the SSA pick: the smallest power of two from 4 whose group
// start sums (G - 1 values of type R) fit in the lane's N candidate words.
template <typename R>
constexpr int ssa_group(int n, int m) {
  int gs = 4;
  while (gs < m && (int)(sizeof(R) / 4) * ((m + gs - 1) / gs - 1) > n) gs *= 2;
  return gs;
}

template <int WG, typename R>
__device__ __forceinline__ void sweep_net(const SweepParams& p) {
  constexpr int N = rnnet::N, M = rnnet::M, CW = (M + 31) / 32, DLD = rnnet::DLD;
  // LDS: the dense stoichiometry matrix [M][DLD], then each lane's leap
  // candidate counts (N words, lane-minor).
  extern __shared__ int32_t lds[];
  const int tid = (int)threadIdx.x;
  const int64_t tl = (int64_t)blockIdx.x * WG + tid;
  const bool valid = tl < p.n_traj;
  const uint32_t traj = p.traj_offset + (uint32_t)tl;
  uint32_t k0, k1;
  asm volatile("v_mov_b32 %0, %1" : "=v"(k0) : "s"(p.key0));
  asm volatile("v_mov_b32 %0, %1" : "=v"(k1) : "s"(p.key1));
  const int S = p.n_times;
  const double* __restrict__ times = p.times;
  typedef typename Vec16<R>::type V16;
  typedef int32_t I16 __attribute__((ext_vector_type(16)));

  for (int k = tid; k < M * DLD; k += WG) lds[k] = p.net.nu_dense[k];
  __syncthreads();
  int32_t* const xn = lds + M * DLD + tid;  // xn[i * WG]
  // Per wave, after every lane's candidate words: the leap draw list of the
  // wave (means [16][64] of type R, counts [16][64], the lanes' attempt
  // counters [64], items [8 * 64]); see the leap attempt.
  int32_t* const wbase = lds + M * DLD + N * WG + (tid >> 6) * kLeapWaveWords<R>;
  R* const lamw = (R*)wbase;
  int32_t* const kres = wbase + 16 * 64 * (int)(sizeof(R) / 4);
  int32_t* const nl = kres + 16 * 64;
  int32_t* const items = nl + 64;
  // The same lane-private words hold, during an SSA event, the running sums of
  // a0 at the group starts g = 1 .. G-1, each in the lane's words
  // (g - 1) * RW .. (g - 1) * RW + RW - 1 (RW words per value): groups of GS
  // reactions, GS the smallest power of two from 4 whose G - 1 sums fit in N
  // words.  Only the lane's own words: other lanes, and other waves of the
  // workgroup, may be in a leap with their candidates in theirs.
  constexpr int GS = ssa_group<R>(N, M), G = (M + GS - 1) / GS;
  constexpr int RW = (int)(sizeof(R) / 4);
  auto ps_put = [&](auto gc, R v) {
    constexpr int g = decltype(gc)::value;
    if constexpr (RW == 2) {
      const uint64_t u = __builtin_bit_cast(uint64_t, v);
      xn[(2 * (g - 1)) * WG] = (int32_t)(uint32_t)u;
      xn[(2 * (g - 1) + 1) * WG] = (int32_t)(uint32_t)(u >> 32);
    } else {
      xn[(g - 1) * WG] = __builtin_bit_cast(int32_t, v);
    }
  };
  auto ps_get = [&](auto gc) -> R {
    constexpr int g = decltype(gc)::value;
    if constexpr (RW == 2) {
      const uint64_t u = (uint64_t)(uint32_t)xn[(2 * (g - 1)) * WG] |
                         ((uint64_t)(uint32_t)xn[(2 * (g - 1) + 1) * WG] << 32);
      return __builtin_bit_cast(R, u);
    } else {
      return __builtin_bit_cast(R, xn[(g - 1) * WG]);
    }
  };

  const double* const crate = p.rates + (valid ? tl : 0);
  const int64_t rld = p.rates_ld;
  RateRegs<R, M> c;
  sfor<0, M>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    c.put(j, valid ? (R)crate[(int64_t)j * rld] : R(0));
  });
  int32_t x[N + 1];  // x[N] == 1: the constant factor of lower-order rate laws
  sfor<0, N>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    int32_t v = 0;
    if (valid) v = p.x0_ld ? p.x0[(int64_t)i * p.x0_ld + tl] : p.x0[i];
    x[i] = v;
  });
  x[N] = 1;
  uint32_t crit[CW];
  sfor<0, CW>([&](auto wc) { crit[decltype(wc)::value] = 0u; });

  // h_j(x) as the generic kernel forms it (scale * (A * B), written out per
  // order: 1 * (1 * 1) = 1 and 1 * (A * 1) = A exactly).
  auto hj = [&](auto jc) -> R {
    constexpr int j = decltype(jc)::value;
    constexpr int ia = rnnet::LAW[j][0], ib = rnnet::LAW[j][1];
    constexpr int db = rnnet::LAW[j][2], dimer = rnnet::LAW[j][3];
    if constexpr (ia == N) return R(1);
    else if constexpr (ib == N) return (R)x[ia];
    else if constexpr (dimer != 0) return R(0.5) * ((R)x[ia] * (R)(x[ib] + db));
    else return (R)x[ia] * (R)x[ib];
  };
  auto aj = [&](auto jc) -> R { return c.get(decltype(jc)::value) * hj(jc); };
  // An empty asm that claims to change every count and critical-bit word:
  // placed at the start of each phase, it keeps the compiler from carrying
  // propensities or per-reaction critical tests from one phase into the next
  // (or computing a whole leap's means at once), which would hold hundreds of
  // values in registers and spill them.
  auto fence = [&]() {
    opaque_all_(x, (__make_integer_seq<ISeq, int, N>*)nullptr);
    opaque_all_(crit, (__make_integer_seq<ISeq, int, CW>*)nullptr);
  };
  auto critbit = [&](auto jc) -> bool {
    constexpr int j = decltype(jc)::value;
    return (crit[j >> 5] >> (j & 31)) & 1u;
  };

  double t = 0.0, tau_p = 0.0, a0 = 0.0;
  double t_next = (valid && S > 0) ? times[0] : 0.0;
  uint32_t n = 0, burst_left = 0, status = 0;
  uint64_t leaps = 0, ssa = 0, rej = 0;
  int s = 0;
  int mode = valid ? (p.method == 1 ? kSsa : kDecide) : kDone;
  const bool ssa_only = p.method == 1;

  const bool want_out = p.out != nullptr;
  const bool want_stats = p.sum_x != nullptr || p.hist != nullptr;
  auto record = [&](int si) {
    if (!valid) return;
    if (want_out) {
      // a fresh copy of the row stride per call keeps the N row offsets from
      // being hoisted out of the main loop (they would pin 2N scalar registers)
      int64_t ld = p.out_ld;
      asm volatile("" : "+s"(ld));
      if (p.out_traj_major) {
        int32_t* o = p.out + tl * ld + (int64_t)si * N;
        sfor<0, N>([&](auto ic) { o[decltype(ic)::value] = x[decltype(ic)::value]; });
      } else {
        int32_t* o = p.out + (int64_t)si * N * ld + tl;
        sfor<0, N>([&](auto ic) {
          o[0] = x[decltype(ic)::value];
          o += ld;
        });
      }
    }
    if (want_stats) {
      // the lane's candidate words are free whenever a state is recorded:
      // stage the counts there for the out-of-line statistics pass
      sfor<0, N>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        xn[i * WG] = x[i];
      });
      add_stats_row(p.sum_x, p.sum_x2, p.hist, p.hist_lo, p.hist_width, p.hist_bins, N, si,
                    xn, WG);
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
  // Add row j (per lane) of the dense stoichiometry matrix to counts y, in
  // wrapping 32-bit arithmetic; returns the OR of the results (the sign bit
  // marks a count outside [0, 2^31) when y started non-negative).
  // `stride` is 1 for the register counts x and WG for the LDS candidate xn.
  auto add_row = [&](int32_t* y, int stride, int j, bool sub) -> int32_t {
    const int32_t* row = lds + j * DLD;
    int32_t acc = 0;
    sfor<0, (N + 3) / 4>([&](auto qc) {
      constexpr int q = 4 * decltype(qc)::value;
      const int4 d = *(const int4*)(row + q);
      const int32_t dv[4] = {d.x, d.y, d.z, d.w};
      sfor<0, 4>([&](auto ec) {
        constexpr int i = q + decltype(ec)::value;
        if constexpr (i < N) {
          const uint32_t u = (uint32_t)dv[decltype(ec)::value];
          int32_t& yi = y[i * stride];
          yi = (int32_t)(sub ? (uint32_t)yi - u : (uint32_t)yi + u);
          acc |= yi;
        }
      });
    });
    return acc;
  };

  if (valid) {
    while (s < S && t_next <= t) record_next();
    if (s == S) mode = kDone;
  }

#ifdef RN_NET_TIMERS
  // shader-clock cycles per phase for this wave: SSA, decide, leap, total
  uint64_t tph[4] = {0, 0, 0, 0}, tmark = 0;
  const uint64_t tstart = clock64();
#define RN_TB() (tmark = clock64())
#define RN_TE(k) (tph[k] += clock64() - tmark)
#else
#define RN_TB() ((void)0)
#define RN_TE(k) ((void)0)
#endif

  for (;;) {
    const uint64_t act = __ballot(mode != kDone);
    if (act == 0) break;
    const uint64_t in_ssa = __ballot(mode == kSsa);
    const uint64_t waiting = act & ~in_ssa;
    const bool leap_turn = in_ssa == 0 ||
                           (waiting != 0 && (float)__popcll(waiting) >=
                                                p.theta * (float)__popcll(act));

    // ---------------- one exact SSA event ----------------
    const bool ph_ssa = in_ssa != 0;
    if (ph_ssa) RN_TB();
    if (mode == kSsa) {
      do {
        if (steps() >= p.max_steps) { finish(kStMaxSteps); break; }
        fence();
        // a0 in index order; the running sum at the start of every group of
        // GS reactions is kept in the lane's LDS words for the pick below
        R sum = R(0);
        sfor<0, M>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          if constexpr (j > 0 && j % GS == 0) ps_put(Ix<j / GS>{}, sum);
          sum = sum + aj(jc);
        });
        if (sum == R(0)) { finish(kStAbsorbed); break; }
        const Words w = philox10(traj, n, 0u, kStreamEvent, k0, k1);
        const R tau = -Real<R>::log_(R(1) - Real<R>::uni(w.w0, w.w1)) / sum;
        const double tn = t + (double)tau;
        // The reaction: the first j whose running sum exceeds r.  The sums do
        // not decrease, so it lies in the group gp with S_gp <= r < S_gp+1
        // (S_g the kept sum at group g's start, S_0 = 0, S_G = a0); r >= a0
        // leaves none (gp = G) and takes the last reaction with a_j > 0.  A
        // group is evaluated, from its kept start, only when some lane picks
        // in it; the sums inside it are those of the loop above.
        const R r = Real<R>::uni(w.w2, w.w3) * sum;
        int gp = 0;
        sfor<1, G>([&](auto gc) {
          constexpr int g = decltype(gc)::value;
          gp += (ps_get(gc) <= r) ? 1 : 0;
        });
        if (!(r < sum)) gp = G;
        fence();
        int pick = -1;
        sfor<0, G>([&](auto gc) {
          constexpr int g = decltype(gc)::value;
          if (__any(gp == g)) {
            R acc = R(0);
            if constexpr (g > 0) acc = ps_get(gc);
            sfor<g * GS, ((g + 1) * GS < M ? (g + 1) * GS : M)>([&](auto jc) {
              constexpr int j = decltype(jc)::value;
              acc = acc + aj(jc);
              // a select, not a branch: a lane that has picked keeps its pick
              pick = (gp == g && pick < 0 && r < acc) ? j : pick;
            });
          }
        });
        if (__any(gp == G)) {
          int last = -1;
          sfor<0, M>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            last = (gp == G && aj(jc) > R(0)) ? j : last;
          });
          if (gp == G) pick = last;
        }
        // samples before the event take the pre-event state
        while (s < S && t_next < tn) record_next();
        if (s == S) { mode = kDone; break; }
        if (pick < 0) { finish(kStAbsorbed); break; }
        if (add_row(x, 1, pick, false) < 0) {  // a count left the int32 range
          add_row(x, 1, pick, true);
          finish(kStOverflow);
          break;
        }
        t = tn;
        n = n + 1;
        ssa = ssa + 1;
        while (s < S && t_next <= t) record_next();
        if (s == S) { mode = kDone; break; }
        if (!ssa_only && --burst_left == 0) mode = kDecide;
      } while (false);
    }
    if (ph_ssa) RN_TE(0);

    if (!leap_turn) continue;

    // ---------------- decide: propensities, critical set, tau' ----------------
    const bool ph_dec = __any(mode == kDecide);
    if (ph_dec) RN_TB();
    if (mode == kDecide) {
      do {
        if (steps() >= p.max_steps) { finish(kStMaxSteps); break; }
        fence();
        double sum = 0.0;  // FP64 in both precisions: it feeds the SSA-switch test
        sfor<0, CW>([&](auto wc) { crit[decltype(wc)::value] = 0u; });
        sfor<0, M>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const R a = aj(jc);
          sum = sum + (double)a;
          bool cr = false;
          sfor<rnnet::CONS_PTR[j], rnnet::CONS_PTR[j + 1]>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            cr = cr | ((int64_t)x[rnnet::CONS_ENT[e][0]] < (int64_t)p.n_c * rnnet::CONS_ENT[e][1]);
          });
          crit[j >> 5] |= (uint32_t)(cr & (a > R(0))) << (j & 31);
        });
        a0 = sum;
        if (sum == 0.0) { finish(kStAbsorbed); break; }
        R tp = (R)__builtin_inf();
        const R eps = (R)p.eps;
        fence();
        sfor<0, rnnet::NRS>([&](auto rc) {
          constexpr int r = decltype(rc)::value;
          constexpr int sp = rnnet::RS[r][0], gk = rnnet::RS[r][1];
          fence();  // recompute each species' propensities rather than hold all M
          R mu = R(0), sig = R(0);
          sfor<rnnet::RS[r][2], rnnet::RS[r][3]>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            constexpr int j = rnnet::RS_ENT[e][0], v = rnnet::RS_ENT[e][1];
            // a critical reaction's term is skipped: select a zero propensity,
            // whose product is +-0 and leaves the (never -0) sums unchanged
            const R a = aj(Ix<j>{});
            const R am = critbit(Ix<j>{}) ? R(0) : a;
            mu = mu + (R)v * am;
            sig = sig + (R)(v * v) * am;
          });
          const int32_t xi = x[sp];
          R bnd = R(1);
          if (xi > 1) {
            const R gi = gk == 1 ? R(1) : gk == 2 ? R(2) : R(2) + R(1) / (R)(xi - 1);
            bnd = eps * (R)xi / gi;
            if (bnd < R(1)) bnd = R(1);
          }
          if (mu != R(0)) { const R q = bnd / Real<R>::abs_(mu); if (q < tp) tp = q; }
          if (sig != R(0)) { const R q = (bnd * bnd) / sig; if (q < tp) tp = q; }
        });
        tau_p = (double)tp;
        mode = kLeap;
      } while (false);
    }
    if (ph_dec) RN_TE(1);

    // ---------------- one leap attempt ----------------
    const bool ph_leap = __any(mode == kLeap);
    if (ph_leap) {
      RN_TB();
      // Lanes in leap mode: the switch test, the critical race and the leap
      // length; `go` marks the lanes that go on to draw.
      bool go = false, fire = false;
      Words ev = {0u, 0u, 0u, 0u};
      double a0c = 0.0, tau = 0.0, delta = 0.0;
      int32_t xmax = 0;
      if (mode == kLeap) {
        do {
          if (steps() >= p.max_steps) { finish(kStMaxSteps); break; }
          if (tau_p < p.ssa_factor / a0) {
            mode = kSsa;
            burst_left = (uint32_t)p.ssa_burst;
            break;
          }
          uint32_t any_crit = 0;
          sfor<0, CW>([&](auto wc) { any_crit |= crit[decltype(wc)::value]; });
          fence();
          if (__any(any_crit != 0u)) {
            sfor<0, M>([&](auto jc) {
              const double a = (double)aj(jc);
              a0c = critbit(jc) ? a0c + a : a0c;
            });
          }
          double tau_c = __builtin_inf();
          if (a0c > 0.0) {
            ev = philox10(traj, n, 0u, kStreamEvent, k0, k1);
            tau_c = -log(1.0 - u53(ev.w0, ev.w1)) / a0c;
          }
          delta = t_next - t;
          fire = (tau_c <= tau_p) && (tau_c <= delta);
          tau = fire ? tau_c : (tau_p < delta ? tau_p : delta);
          // Candidate counts xn; the additions wrap instead of overflowing,
          // and a candidate whose sums could leave the int32 range is never
          // used (the exact path below decides).
          sfor<0, N>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            xn[i * WG] = x[i];
            xmax = max(xmax, x[i]);
          });
          go = true;
        } while (false);
      }
      uint64_t kabs = 0;
      const R taur = (R)tau;
      // Poisson firings of the non-critical reactions over tau, 16 reactions
      // at a time.  The means go into one register vector.  The inversion
      // draws (means in (0, 10), the two reactions of a pair sharing one
      // Philox block of the first-uniform stream) are spread over the whole
      // wave: every (lane, pair) that needs a block becomes an item of a
      // wave-private LDS list, each lane of the wave draws items in turn, and
      // the counts go back to their lanes through LDS.  Each draw is the
      // owner's own arithmetic on the owner's counters, so the results do not
      // depend on which lane computes them.  Means of 10 and more (PTRS,
      // Langevin) are drawn by their own lanes.
      const int wl = tid & 63;
      const uint32_t traj0 = traj - (uint32_t)wl;  // the wave's first trajectory
      nl[wl] = (int32_t)n;
      sfor<0, (M + 15) / 16>([&](auto bc) {
        constexpr int base = 16 * decltype(bc)::value;
        fence();
        const uint32_t cw = crit[base >> 5] >> (base & 31);
        V16 lam;
        sfor<0, 16>([&](auto ec) {
          constexpr int e = decltype(ec)::value;
          if constexpr (base + e < M) {
            const R lv = aj(Ix<base + e>{}) * taur;
            lam[e] = (go && !((cw >> e) & 1u)) ? lv : R(0);
          } else {
            lam[e] = R(0);
          }
        });
        uint32_t need = 0u;
        sfor<0, 8>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          const R l0 = lam[2 * q], l1 = lam[2 * q + 1];
          const bool nq = (l0 > R(0) && l0 < R(10)) || (l1 > R(0) && l1 < R(10));
          need |= (nq ? 1u : 0u) << q;
          lamw[(2 * q) * 64 + wl] = l0;
          lamw[(2 * q + 1) * 64 + wl] = l1;
        });
        int total = 0;
        sfor<0, 8>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          const bool nq = (need >> q) & 1u;
          const uint64_t m = __ballot(nq);
          const int below = (int)__builtin_amdgcn_mbcnt_hi(
              (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if (nq) items[total + below] = (wl << 3) | q;
          total += (int)__popcll(m);
        });
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll 1
        for (int b0 = 0; b0 < total; b0 += 64) {
          const int it = b0 + wl;
          if (it < total) {
            const int code = items[it];
            const int o = code >> 3, q = code & 7;
            const R l0 = lamw[(2 * q) * 64 + o], l1 = lamw[(2 * q + 1) * 64 + o];
            const Words w = philox10(traj0 + (uint32_t)o, (uint32_t)nl[o],
                                     (uint32_t)((base >> 1) + q), kStreamFirst, k0, k1);
            uint32_t ka = 0u, kb = 0u;
            if (l0 > R(0) && l0 < R(10)) ka = poisson_inversion<R>(l0, Real<R>::uni(w.w0, w.w1));
            if (l1 > R(0) && l1 < R(10)) kb = poisson_inversion<R>(l1, Real<R>::uni(w.w2, w.w3));
            kres[(2 * q) * 64 + o] = (int32_t)ka;
            kres[(2 * q + 1) * 64 + o] = (int32_t)kb;
          }
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (go) {
          I16 kv;
          // the lane's own counts back from the list, or its large-mean draws
#pragma unroll 1
          for (int e = 0; e < 16; ++e) {
            const int je = base + e;
            if (je >= M) break;
            const R le = lam[e];
            int32_t k = 0;
            if (le >= R(10))
              k = (int32_t)poisson<R, true>(le, 0u, 0u, traj, n, (uint32_t)je, k0, k1,
                                            p.net.log_fact, p.cle_threshold);
            else if (le > R(0))
              k = kres[e * 64 + wl];
            kv[e] = k;
          }
          sfor<0, 16>([&](auto ec) {
            constexpr int e = decltype(ec)::value, j = base + e;
            if constexpr (j < M) {
              const uint32_t k = (uint32_t)kv[e];
              kabs += (uint64_t)k * rnnet::NU_ABS[j];
              if (__any(k != 0u)) {
                sfor<rnnet::NU_PTR[j], rnnet::NU_PTR[j + 1]>([&](auto qc) {
                  constexpr int q = decltype(qc)::value;
                  constexpr int sp = rnnet::NU_ENT[q][0], v = rnnet::NU_ENT[q][1];
                  xn[sp * WG] = (int32_t)((uint32_t)xn[sp * WG] + k * (uint32_t)v);
                });
              }
            }
          });
        }
      });
      // Lanes that drew: the critical firing, the exact check, accept or reject.
      if (go) {
        do {
          int jc = -1;
          if (fire) {
            fence();
            const double r = u53(ev.w2, ev.w3) * a0c;
            double acc = 0.0;
            int last = -1;
            sfor<0, (M + 3) / 4>([&](auto gc) {
              constexpr int g4 = 4 * decltype(gc)::value;
              if (__any(jc < 0)) {
                sfor<g4, (g4 + 4 < M ? g4 + 4 : M)>([&](auto jj) {
                  constexpr int j = decltype(jj)::value;
                  const bool open = jc < 0 && critbit(jj);
                  const double a = (double)aj(jj);
                  const double acc2 = acc + a;
                  acc = open ? acc2 : acc;
                  last = (open && a > 0.0) ? j : last;
                  jc = (open && r < acc2) ? j : jc;
                });
              }
            });
            if (jc < 0) jc = last;
            if (jc < 0) { finish(kStAbsorbed); break; }
            add_row(xn, WG, jc, false);  // jc differs between lanes
            kabs += p.net.nu_abs[jc];
          }

          bool neg = false, big = false;
          if ((uint64_t)xmax + kabs <= (uint64_t)INT32_MAX) {
            // no partial sum can leave the int32 range: the candidate is exact
            int32_t sg = 0;
            sfor<0, N>([&](auto ic) { sg |= xn[decltype(ic)::value * WG]; });
            neg = sg < 0;
          } else {
            // exact 64-bit evaluation, species by species, redrawing each k_j
            sfor<0, N>([&](auto ic) {
              constexpr int i = decltype(ic)::value;
              fence();
              int64_t acc = x[i];
              sfor<rnnet::COL_PTR[i], rnnet::COL_PTR[i + 1]>([&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr int j = rnnet::COL_ENT[e][0], v = rnnet::COL_ENT[e][1];
                int64_t kj;
                if (critbit(Ix<j>{})) {
                  kj = (fire && j == jc) ? 1 : 0;
                } else {
                  kj = draw_one<R>(aj(Ix<j>{}) * taur, traj, n, (uint32_t)j, k0, k1,
                                   p.net.log_fact, p.cle_threshold);
                }
                acc += kj * (int64_t)v;
              });
              if (acc < 0) neg = true;
              else if (acc > INT32_MAX) big = true;
            });
          }
          if (neg) {
            tau_p = tau_p * 0.5;
            n = n + 1;
            rej = rej + 1;
            break;  // stays in leap mode
          }
          if (big) { finish(kStOverflow); break; }
          sfor<0, N>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            x[i] = xn[i * WG];
          });
          if (tau == delta) t = t_next;
          else t = t + tau;
          n = n + 1;
          leaps = leaps + 1;
          while (s < S && t_next <= t) record_next();
          if (s == S) { mode = kDone; break; }
          mode = kDecide;
        } while (false);
      }
      RN_TE(2);
    }
  }
#ifdef RN_NET_TIMERS
  tph[3] = clock64() - tstart;
  if (p.phase_cycles && (tid & 63) == 0) {
    uint64_t* o = p.phase_cycles + (tl >> 6) * 4;
    for (int k = 0; k < 4; ++k) o[k] = tph[k];
  }
#endif
#undef RN_TB
#undef RN_TE

  if (valid) {
    uint64_t* st = p.stats + tl * 4;
    st[0] = leaps;
    st[1] = ssa;
    st[2] = rej;
    st[3] = status;
  }
}

// Exact SSA only (the direct method, RN_METHOD_SSA) with a reaction
// dependency graph: every propensity a_k is kept in a register and, after an
// event, only the reactions whose reactants the event changed are recomputed
// (Gibson and Bruck, J. Phys. Chem. A 104, 1876 (2000), use the same graph).
// a0 is still summed over the kept propensities in index order, and the pick
// uses the running sums of that order, so events are bit for bit those of the
// general kernel and of the oracle.  Counts live in lane-private LDS words
// (the registers hold the propensities and, in accumulation registers, the
// rates); the fired reaction's entries come from a compact list in LDS.  A
// wave recomputes a reaction when any of its lanes needs it, so the saving
// depends on how far the lanes' dependent sets overlap.
template <int WG, typename R>
__device__ __forceinline__ void sweep_net_ssa(const SweepParams& p) {
  constexpr int N = rnnet::N, M = rnnet::M;
  constexpr int NNZ = rnnet::NU_PTR[M];
  constexpr int GS = ssa_group<R>(N, M), G = (M + GS - 1) / GS;
  // LDS: the compact stoichiometry (NU_PTR[M + 1], then NU_ENT as
  // species | nu << 8), then per lane the counts xs[i * WG] and the group
  // start sums ps[(g - 1) * WG].
  extern __shared__ int32_t lds[];
  const int tid = (int)threadIdx.x;
  const int64_t tl = (int64_t)blockIdx.x * WG + tid;
  const bool valid = tl < p.n_traj;
  const uint32_t traj = p.traj_offset + (uint32_t)tl;
  uint32_t k0, k1;
  asm volatile("v_mov_b32 %0, %1" : "=v"(k0) : "s"(p.key0));
  asm volatile("v_mov_b32 %0, %1" : "=v"(k1) : "s"(p.key1));
  const int S = p.n_times;
  const double* __restrict__ times = p.times;

  int32_t* const nptr = lds;
  int32_t* const nent = lds + (M + 1);
  for (int k = tid; k <= M; k += WG) nptr[k] = rnnet::NU_PTR[k];
  for (int k = tid; k < NNZ; k += WG)
    nent[k] = rnnet::NU_ENT[k][0] | (int32_t)((uint32_t)rnnet::NU_ENT[k][1] << 8);
  __syncthreads();
  constexpr int kOff = ((M + 1 + NNZ) + 3) / 4 * 4;
  int32_t* const xs = lds + kOff + tid;                // xs[i * WG]
  R* const ps = (R*)(lds + kOff + N * WG) + tid;        // ps[(g - 1) * WG]

  const double* const crate = p.rates + (valid ? tl : 0);
  const int64_t rld = p.rates_ld;
  RateRegs<R, M> c;
  sfor<0, M>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    c.put(j, valid ? (R)crate[(int64_t)j * rld] : R(0));
  });
  sfor<0, N>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    int32_t v = 0;
    if (valid) v = p.x0_ld ? p.x0[(int64_t)i * p.x0_ld + tl] : p.x0[i];
    xs[i * WG] = v;
  });
  // h_j at the LDS counts, formed as the general kernel forms it
  auto hj = [&](auto jc) -> R {
    constexpr int j = decltype(jc)::value;
    constexpr int ia = rnnet::LAW[j][0], ib = rnnet::LAW[j][1];
    constexpr int db = rnnet::LAW[j][2], dimer = rnnet::LAW[j][3];
    if constexpr (ia == N) return R(1);
    else if constexpr (ib == N) return (R)xs[ia * WG];
    else if constexpr (dimer != 0) {
      const int32_t xa = xs[ia * WG];
      return R(0.5) * ((R)xa * (R)(xa + db));
    } else return (R)xs[ia * WG] * (R)xs[ib * WG];
  };
  R a[M];
  sfor<0, M>([&](auto jc) { a[decltype(jc)::value] = c.get(decltype(jc)::value) * hj(jc); });

  double t = 0.0;
  double t_next = (valid && S > 0) ? times[0] : 0.0;
  uint32_t n = 0, status = 0;
  uint64_t ssa = 0;
  int s = 0;
  bool live = valid;
  auto record = [&](int si) {
    if (!valid) return;
    if (p.out) {
      if (p.out_traj_major) {
        int32_t* o = p.out + tl * p.out_ld + (int64_t)si * N;
        sfor<0, N>([&](auto ic) { o[decltype(ic)::value] = xs[decltype(ic)::value * WG]; });
      } else {
        int32_t* o = p.out + (int64_t)si * N * p.out_ld + tl;
        sfor<0, N>([&](auto ic) {
          o[(int64_t)decltype(ic)::value * p.out_ld] = xs[decltype(ic)::value * WG];
        });
      }
    }
    if (p.sum_x || p.hist)
      add_stats_row(p.sum_x, p.sum_x2, p.hist, p.hist_lo, p.hist_width, p.hist_bins, N, si,
                    xs, WG);
  };
  auto record_next = [&]() {
    record(s);
    s = s + 1;
    if (s < S) t_next = times[s];
  };
  auto finish = [&](uint32_t why) {
    status |= why;
    while (s < S) record(s++);
    live = false;
  };
  if (valid) {
    while (s < S && t_next <= t) record_next();
    if (s == S) live = false;
  }

  while (__any(live)) {
    if (!live) continue;
    do {
      if (ssa >= p.max_steps) { finish(kStMaxSteps); break; }
      R sum = R(0);
      sfor<0, M>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j > 0 && j % GS == 0) ps[(j / GS - 1) * WG] = sum;
        sum = sum + a[j];
      });
      if (sum == R(0)) { finish(kStAbsorbed); break; }
      const Words w = philox10(traj, n, 0u, kStreamEvent, k0, k1);
      const R tau = -Real<R>::log_(R(1) - Real<R>::uni(w.w0, w.w1)) / sum;
      const double tn = t + (double)tau;
      // the pick, as in the general kernel: the group of the first running
      // sum above r, then the running sums inside it
      const R r = Real<R>::uni(w.w2, w.w3) * sum;
      int gp = 0;
      sfor<1, G>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        gp += (ps[(g - 1) * WG] <= r) ? 1 : 0;
      });
      if (!(r < sum)) gp = G;
      int pick = -1;
      sfor<0, G>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (__any(gp == g)) {
          R acc = R(0);
          if constexpr (g > 0) acc = ps[(g - 1) * WG];
          sfor<g * GS, ((g + 1) * GS < M ? (g + 1) * GS : M)>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            acc = acc + a[j];
            pick = (gp == g && pick < 0 && r < acc) ? j : pick;
          });
        }
      });
      if (__any(gp == G)) {
        int last = -1;
        sfor<0, M>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          last = (gp == G && a[j] > R(0)) ? j : last;
        });
        if (gp == G) pick = last;
      }
      while (s < S && t_next < tn) record_next();
      if (s == S) { live = false; break; }
      if (pick < 0) { finish(kStAbsorbed); break; }
      // apply the event to the counts; the species it changes mark the
      // reactions to recompute
      uint32_t chg0 = 0u, chg1 = 0u;
      int32_t neg = 0;
      const int e1 = nptr[pick + 1];
      for (int e = nptr[pick]; e < e1; ++e) {
        const int32_t ent = nent[e];
        const int sp = ent & 0xff;
        const int32_t v = ent >> 8;
        int32_t& xv = xs[sp * WG];
        xv = (int32_t)((uint32_t)xv + (uint32_t)v);
        neg |= xv;
        if (sp < 32) chg0 |= 1u << sp;
        else chg1 |= 1u << (sp - 32);
      }
      if (neg < 0) {  // a count left the int32 range: undo the event
        for (int e = nptr[pick]; e < e1; ++e) {
          const int32_t ent = nent[e];
          int32_t& xv = xs[(ent & 0xff) * WG];
          xv = (int32_t)((uint32_t)xv - (uint32_t)(ent >> 8));
        }
        finish(kStOverflow);
        break;
      }
      t = tn;
      n = n + 1;
      ssa = ssa + 1;
      sfor<0, M>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int ia = rnnet::LAW[j][0], ib = rnnet::LAW[j][1];
        if constexpr (ia < N) {
          constexpr uint64_t mk = (1ull << ia) | (ib < N ? (1ull << ib) : 0ull);
          const bool dirty = ((chg0 & (uint32_t)mk) | (chg1 & (uint32_t)(mk >> 32))) != 0u;
          if (__any(dirty)) {
            const R an = c.get(j) * hj(jc);
            a[j] = dirty ? an : a[j];
          }
        }
      });
      while (s < S && t_next <= t) record_next();
      if (s == S) { live = false; break; }
    } while (false);
  }
  if (valid) {
    uint64_t* st = p.stats + tl * 4;
    st[0] = 0u;
    st[1] = ssa;
    st[2] = 0u;
    st[3] = status;
  }
}

}  // namespace
}  // namespace netk
}  // namespace rn
