// rn_sweep_kernel.h -- gfx950 kernels: one wave64 lane per trajectory of a
// parameter sweep, each advanced by Cao-Gillespie-Petzold tau-leaping (J. Chem.
// Phys. 124, 044109, 2006) with critical reactions (J. Chem. Phys. 123, 054104,
// 2005) and bursts of exact SSA events (Gillespie's direct method, 1977).  The
// model is the paper's (Methods section): X(t) counts molecules per species and
// every firing adds the reaction's stoichiometric vector.
//
// The kernel template is instantiated once per arithmetic precision R, each in
// its own translation unit (rn_sweep_f64.hip, rn_sweep_f32.hip):
//  * R = double: every step in FP64.
//  * R = float: propensities, the SSA event (sum, waiting time, selection), the
//    leap-condition bound tau', the Poisson means and the inversion sampler in
//    FP32 with 24-bit uniforms; FP64 for the time t, the sample times, a0 of the
//    SSA-switch test, the critical race (a0c, tau'', its selection) and the
//    leap length tau, and for the PTRS and Langevin samplers (their acceptance
//    test and increment subtract terms of size lam log lam that FP32 cannot
//    resolve once lam exceeds about 1e4).  Each FP32 uniform is the top 24 bits
//    of the word pair the FP64 path uses for the same draw, so the two modes
//    follow the same random path until an FP32 rounding changes a decision.
//
// Layout
//  * Counts: LDS, lane-minor.  Each lane owns two buffers of N+1 words (current
//    state and leap candidate; word N is the constant 1 used by the rate laws)
//    plus ceil(M/32) critical-reaction bit words.  Lanes never share LDS words,
//    so the kernel has no barriers.
//  * Network tables: read-only global memory, always at wave-uniform indices
//    (scalar loads).
//  * Rates [M][T] and samples [S][N][T]: trajectory-minor global arrays, so a
//    wave's 64 lanes touch 64 consecutive words.
//
// Per-lane control is a small state machine (decide / SSA event / leap attempt).
// Each loop iteration runs every phase that some lane of the wave needs, masked
// to those lanes.  Counter-based random numbers make each trajectory's result
// independent of how its steps interleave with other lanes'.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rn_device.h"
#include "rn_kernel.h"

namespace rn {
namespace {
using namespace dev;

// Network tables are read-only for the whole kernel and indexed wave-uniformly;
// reading them through the constant address space lets the compiler use scalar
// loads (a divergent index still falls back to a vector load).
typedef const int32_t __attribute__((address_space(4)))* const_i32_ptr;
__device__ __forceinline__ int32_t cld(const void* base, int64_t i) {
  return ((const_i32_ptr)base)[i];
}
__device__ __forceinline__ int2 cld2(const int2* base, int64_t i) {
  return make_int2(cld(base, 2 * i), cld(base, 2 * i + 1));
}
__device__ __forceinline__ RateLaw law_at(const RateLaw* base, int j) {
  return {cld(base, 4 * j), cld(base, 4 * j + 1), cld(base, 4 * j + 2), cld(base, 4 * j + 3)};
}
__device__ __forceinline__ TauSpecies rs_at(const TauSpecies* base, int r) {
  return {cld(base, 4 * r), cld(base, 4 * r + 1), cld(base, 4 * r + 2), cld(base, 4 * r + 3)};
}

// Element j (wave-uniform, LO <= j < HI) of a register array, by binary search
// over compile-time indices, so the array never needs a dynamic register index.
template <int LO, int HI, int NS, typename R>
struct PickReg {
  __device__ static __forceinline__ R get(const R (&v)[NS], int j) {
    if constexpr (HI - LO == 1) {
      return v[LO];
    } else {
      constexpr int MID = (LO + HI) / 2;
      if (j < MID) return PickReg<LO, MID, NS, R>::get(v, j);
      return PickReg<MID, HI, NS, R>::get(v, j);
    }
  }
};

// WG lanes per workgroup.  NSEG > 0: the lane's rate constants are held in
// 16 * NSEG registers (M <= 16 * NSEG); NSEG == 0: they are read from the rates
// array.
// The trajectories [tl0, tl0 + WG) of one sweep, one per lane of the workgroup.
template <int WG, int NSEG, typename R>
__device__ __forceinline__ void sweep_block(const SweepParams& p, int64_t tl0) {
  extern __shared__ int32_t lds[];
  const DevNet& g = p.net;
  const int N = g.N, M = g.M, NP1 = N + 1;
  const int tid = (int)threadIdx.x;
  const int64_t tl = tl0 + tid;
  const bool valid = tl < p.n_traj;
  const uint32_t traj = p.traj_offset + (uint32_t)tl;
  // The Philox key is wave-uniform, but its ten round keys would crowd the
  // scalar register file; keeping the key in vector registers turns the key
  // schedule into two vector adds per round.
  uint32_t k0, k1;
  asm volatile("v_mov_b32 %0, %1" : "=v"(k0) : "s"(p.key0));
  asm volatile("v_mov_b32 %0, %1" : "=v"(k1) : "s"(p.key1));
  const int S = p.n_times;
  const double* __restrict__ times = p.times;

  int32_t* const lane = lds + tid;
  int32_t* xc = lane;                 // current counts
  int32_t* xn = lane + NP1 * WG;      // leap candidate
  int32_t* const crit = lane + 2 * NP1 * WG;
  const double* const crate = p.rates + (valid ? tl : 0);
  const int64_t rld = p.rates_ld;

  // Rate constants: RMAX = 16 * NSEG doubles indexed only by compile-time
  // constants (every pass over them is unrolled), so each is an ordinary
  // register; random access goes through a compare tree (rate_at).
  constexpr int RMAX = NSEG > 0 ? 16 * NSEG : 1;
  typedef typename Vec16<R>::type V16;
  R c[RMAX];
#pragma unroll
  for (int j = 0; j < RMAX; ++j)
    c[j] = (NSEG > 0 && valid && j < g.M_real) ? (R)crate[(int64_t)j * rld] : R(0);
  // c_j of the rates array, for the NSEG == 0 form; the null reactions that
  // pad M to whole rate vectors have no row there and rate 0, as in the
  // register form.
  // The row index is clamped rather than branched on, so that many of these
  // loads can be in flight at once.
  const int m_real = g.M_real;
  auto mrate = [&](int j) -> R {
    const R v = (R)crate[(int64_t)min(j, m_real - 1) * rld];
    return j < m_real ? v : R(0);
  };

  // Mass-action propensity a_j = c_j * h_j(x), h_j = s_j * (x[ia] * (x[ib] + db)).
  auto prop = [&](int j, R cj) -> R {
    const RateLaw L = law_at(g.law, j);
    return cj * hval<R>(xc[L.ia * WG], xc[L.ib * WG] + L.db, L.dimer);
  };
  // f(j, c_j, a_j) for j = 0..M-1 in order, a_j being the current propensity.
  // more() is a wave-uniform "keep going" vote polled every four reactions (f
  // must ignore reactions it no longer needs).  Each group of four reads its
  // rate laws and counts before any arithmetic so that the loads overlap; with
  // register rates the walk is fully unrolled (M is a multiple of 16: null
  // reactions pad the last group).
  auto each_rate = [&](auto&& f, auto&& more) {
    auto group = [&](int j0, R q0, R q1, R q2, R q3) {
      // The table is invariant; hiding the base pointer's value keeps the
      // compiler from hoisting every group's rate laws out of the loops (which
      // would pin hundreds of scalar registers).
      const RateLaw* lawp = g.law;
      asm volatile("" : "+s"(lawp));
      const RateLaw L0 = law_at(lawp, j0), L1 = law_at(lawp, j0 + 1);
      const RateLaw L2 = law_at(lawp, j0 + 2), L3 = law_at(lawp, j0 + 3);
      const int32_t A0 = xc[L0.ia * WG], B0 = xc[L0.ib * WG];
      const int32_t A1 = xc[L1.ia * WG], B1 = xc[L1.ib * WG];
      const int32_t A2 = xc[L2.ia * WG], B2 = xc[L2.ib * WG];
      const int32_t A3 = xc[L3.ia * WG], B3 = xc[L3.ib * WG];
      f(j0, q0, q0 * hval<R>(A0, B0 + L0.db, L0.dimer));
      f(j0 + 1, q1, q1 * hval<R>(A1, B1 + L1.db, L1.dimer));
      f(j0 + 2, q2, q2 * hval<R>(A2, B2 + L2.db, L2.dimer));
      f(j0 + 3, q3, q3 * hval<R>(A3, B3 + L3.db, L3.dimer));
    };
    if constexpr (NSEG == 0) {
      // Rates from memory in chunks of 16: the next chunk's loads are issued
      // before the current chunk is used, so their latency overlaps the
      // arithmetic instead of stalling every group of four.
      int j = 0;
      R q[16], nq[16];
      if (M >= 16) {
#pragma unroll
        for (int e = 0; e < 16; ++e) q[e] = mrate(e);
      }
      for (; j + 16 <= M; j += 16) {
        if (j + 32 <= M) {
#pragma unroll
          for (int e = 0; e < 16; ++e) nq[e] = mrate(j + 16 + e);
        }
        group(j, q[0], q[1], q[2], q[3]);
        if (!more()) return;
        group(j + 4, q[4], q[5], q[6], q[7]);
        if (!more()) return;
        group(j + 8, q[8], q[9], q[10], q[11]);
        if (!more()) return;
        group(j + 12, q[12], q[13], q[14], q[15]);
        if (!more()) return;
#pragma unroll
        for (int e = 0; e < 16; ++e) q[e] = nq[e];
      }
      for (; j + 4 <= M; j += 4) {
        group(j, mrate(j), mrate(j + 1), mrate(j + 2), mrate(j + 3));
        if (!more()) return;
      }
      for (; j < M; ++j) f(j, mrate(j), prop(j, mrate(j)));
    } else {
#pragma unroll
      for (int j = 0; j < RMAX; j += 4) {
        group(j, c[j], c[j + 1], c[j + 2], c[j + 3]);
        if (!more()) return;
      }
    }
  };
  auto always = []() { return true; };
  // c_j for one wave-uniform j.
  auto rate_at = [&](int j) -> R {
    if constexpr (NSEG == 0) return mrate(j);
    else return PickReg<0, RMAX, RMAX, R>::get(c, j);
  };

  for (int i = 0; i < N; ++i) {
    int32_t v = 0;
    if (valid) v = p.x0_ld ? p.x0[(int64_t)i * p.x0_ld + tl] : p.x0[i];
    xc[i * WG] = v;
  }
  xc[N * WG] = 1;
  xn[N * WG] = 1;

  double t = 0.0, tau_p = 0.0, a0 = 0.0;
  double t_next = (valid && S > 0) ? times[0] : 0.0;  // the sample time at index s
  uint32_t n = 0, burst_left = 0, status = 0;
  uint64_t leaps = 0, ssa = 0, rej = 0;
  int s = 0;
  int mode = valid ? (p.method == 1 ? kSsa : kDecide) : kDone;
  const bool ssa_only = p.method == 1;

  auto critbit = [&](int j) -> bool {
    return ((uint32_t)crit[(j >> 5) * WG] >> (j & 31)) & 1u;
  };
  // Only lanes that own a trajectory ever write: padding lanes of the last
  // workgroup (tl >= n_traj) would alias other trajectories' columns.
  auto record = [&](int si) {
    if (!valid) return;
    if (p.out) {
      if (p.out_traj_major) {
        int32_t* o = p.out + tl * p.out_ld + (int64_t)si * N;
        for (int i = 0; i < N; ++i) o[i] = xc[i * WG];
      } else {
        int32_t* o = p.out + (int64_t)si * N * p.out_ld + tl;
        for (int i = 0; i < N; ++i) o[(int64_t)i * p.out_ld] = xc[i * WG];
      }
    }
    if (p.sum_x || p.hist)
      add_stats_row(p.sum_x, p.sum_x2, p.hist, p.hist_lo, p.hist_width, p.hist_bins, N, si, xc,
                    WG);
  };
  // Record the current state at sample s and move to the next sample time.
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
  // Net change of reaction j applied k times to buffer x.
  auto apply = [&](int32_t* x, int j, int32_t k) {
    const int e1 = cld(g.nu_ptr, j + 1);
    for (int e = cld(g.nu_ptr, j); e < e1; ++e) {
      const int2 en = cld2(g.nu_ent, e);
      x[en.x * WG] += k * en.y;
    }
  };

  if (valid) {
    while (s < S && t_next <= t) record_next();
    if (s == S) mode = kDone;
  }

  for (;;) {
    const uint64_t act = __ballot(mode != kDone);
    if (act == 0) break;
    const uint64_t in_ssa = __ballot(mode == kSsa);
    // Leap-side phases run for the whole wave at once: when no lane is in an SSA
    // burst, or when enough lanes wait for them (the rest of the time waiting
    // lanes idle while the bursting lanes advance).
    const uint64_t waiting = act & ~in_ssa;
    const bool leap_turn = in_ssa == 0 ||
                           (waiting != 0 && (float)__popcll(waiting) >=
                                                p.theta * (float)__popcll(act));

    // ---------------- one exact SSA event ----------------
    if (mode == kSsa) {
      do {
        if (steps() >= p.max_steps) { finish(kStMaxSteps); break; }
        R sum = R(0);
        each_rate([&](int, R, R a) { sum = sum + a; }, always);
        if (sum == R(0)) { finish(kStAbsorbed); break; }
        const Words w = philox10(traj, n, 0u, kStreamEvent, k0, k1);
        const R tau = -Real<R>::log_(R(1) - Real<R>::uni(w.w0, w.w1)) / sum;
        const double tn = t + (double)tau;
        while (s < S && t_next < tn) record_next();
        if (s == S) { mode = kDone; break; }
        const R r = Real<R>::uni(w.w2, w.w3) * sum;
        R acc = R(0);
        int pick = -1, last = -1;
        each_rate(
            [&](int j, R, R a) {
              if (pick < 0) {
                acc = acc + a;
                if (a > R(0)) last = j;
                if (r < acc) pick = j;
              }
            },
            [&]() { return __any(pick < 0); });
        if (pick < 0) pick = last;
        if (pick < 0) { finish(kStAbsorbed); break; }
        bool bad = false;
        for (int e = g.nu_ptr[pick]; e < g.nu_ptr[pick + 1]; ++e) {
          const int2 en = g.nu_ent[e];
          const int64_t y = (int64_t)xc[en.x * WG] + en.y;
          if (y > INT32_MAX || y < 0) bad = true;
        }
        if (bad) { finish(kStOverflow); break; }
        for (int e = g.nu_ptr[pick]; e < g.nu_ptr[pick + 1]; ++e) {
          const int2 en = g.nu_ent[e];
          xc[en.x * WG] += en.y;
        }
        t = tn;
        n = n + 1;
        ssa = ssa + 1;
        while (s < S && t_next <= t) record_next();
        if (s == S) { mode = kDone; break; }
        if (!ssa_only && --burst_left == 0) mode = kDecide;
      } while (false);
    }

    if (!leap_turn) continue;

    // ---------------- decide: propensities, critical set, tau' ----------------
    if (mode == kDecide) {
      do {
        if (steps() >= p.max_steps) { finish(kStMaxSteps); break; }
        double sum = 0.0;  // FP64 in both precisions: it feeds the SSA-switch test
        uint32_t bits = 0;
        each_rate([&](int j, R, R a) {
          sum = sum + (double)a;
          if (a > R(0)) {
            bool cr = false;
            const int e1 = cld(g.cons_ptr, j + 1);
            for (int e = cld(g.cons_ptr, j); e < e1; ++e) {
              const int2 ce = cld2(g.cons_ent, e);
              if ((int64_t)xc[ce.x * WG] < (int64_t)p.n_c * ce.y) cr = true;
            }
            if (cr) bits |= 1u << (j & 31);
          }
          if ((j & 31) == 31 || j == M - 1) {
            crit[(j >> 5) * WG] = (int32_t)bits;
            bits = 0;
          }
        }, always);
        a0 = sum;
        if (sum == 0.0) { finish(kStAbsorbed); break; }
        R tp = (R)__builtin_inf();
        const R eps = (R)p.eps;
        for (int r = 0; r < g.n_rs; ++r) {
          const TauSpecies ts = rs_at(g.rs, r);
          R mu = R(0), sig = R(0);
          // four entries at a time: their table, rate and count loads are all
          // issued before the first sum; the sums keep the entries' order
          int e = ts.begin;
          for (; e + 4 <= ts.end; e += 4) {
            int2 en[4];
            R a[4];
            bool skip[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) en[u] = cld2(g.rs_ent, e + u);
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = rate_at(en[u].x);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              skip[u] = critbit(en[u].x);
              a[u] = prop(en[u].x, a[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (skip[u]) continue;
              mu = mu + (R)en[u].y * a[u];
              sig = sig + (R)(en[u].y * en[u].y) * a[u];
            }
          }
          for (; e < ts.end; ++e) {
            const int2 en = cld2(g.rs_ent, e);
            if (critbit(en.x)) continue;
            const R a = prop(en.x, rate_at(en.x));
            mu = mu + (R)en.y * a;
            sig = sig + (R)(en.y * en.y) * a;
          }
          const int32_t xi = xc[ts.species * WG];
          R bnd = R(1);
          if (xi > 1) {
            const R gi = ts.gkind == 1 ? R(1)
                         : ts.gkind == 2 ? R(2)
                                         : R(2) + R(1) / (R)(xi - 1);
            bnd = eps * (R)xi / gi;
            if (bnd < R(1)) bnd = R(1);
          }
          if (mu != R(0)) { const R q = bnd / Real<R>::abs_(mu); if (q < tp) tp = q; }
          if (sig != R(0)) { const R q = (bnd * bnd) / sig; if (q < tp) tp = q; }
        }
        tau_p = (double)tp;
        mode = kLeap;
      } while (false);
    }

    // ---------------- one leap attempt ----------------
    if (mode == kLeap) {
      do {
        if (steps() >= p.max_steps) { finish(kStMaxSteps); break; }
        if (tau_p < p.ssa_factor / a0) {
          mode = kSsa;
          burst_left = (uint32_t)p.ssa_burst;
          break;
        }
        uint32_t any_crit = 0;
        for (int w = 0; w < g.crit_words; ++w) any_crit |= (uint32_t)crit[w * WG];
        double a0c = 0.0;
        if (__any(any_crit != 0u)) {
          uint32_t cw = 0;
#pragma unroll 1
          for (int j = 0; j < M; ++j) {
            if ((j & 31) == 0) cw = (uint32_t)crit[(j >> 5) * WG];
            if ((cw >> (j & 31)) & 1u) a0c = a0c + (double)prop(j, rate_at(j));
          }
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

        int32_t xmax = 0;
        for (int i = 0; i < N; ++i) {
          const int32_t v = xc[i * WG];
          xn[i * WG] = v;
          xmax = max(xmax, v);
        }
        uint64_t kabs = 0;
        // Poisson firings of the non-critical reactions over tau, 16 reactions at
        // a time: their means go into one fresh register vector, then a rolled
        // loop draws them in pairs, the two reactions of a pair sharing one
        // Philox block of the first-uniform stream.
        const R taur = (R)tau;
        auto draw_block = [&](int base, V16 lam) {
#pragma unroll 1
          for (int e = 0; e < 16; e += 2) {
            const int je = base + e;
            if (je >= M) break;
            const bool two = je + 1 < M;
            const R le = lam[e], lo = lam[e + 1];
            Words w = {0u, 0u, 0u, 0u};
            if ((le > R(0) && le < R(10)) || (lo > R(0) && lo < R(10)))
              w = philox10(traj, n, (uint32_t)(je >> 1), kStreamFirst, k0, k1);
            const uint32_t d0 = poisson<R>(le, w.w0, w.w1, traj, n, (uint32_t)je, k0, k1,
                                           g.log_fact, p.cle_threshold);
            const uint32_t d1 = poisson<R>(lo, w.w2, w.w3, traj, n, (uint32_t)(je + 1), k0, k1,
                                           g.log_fact, p.cle_threshold);
            if (__any(d0 != 0u)) apply(xn, je, (int32_t)d0);
            kabs += (uint64_t)d0 * (uint32_t)cld(g.nu_abs, je);
            if (two) {
              if (__any(d1 != 0u)) apply(xn, je + 1, (int32_t)d1);
              kabs += (uint64_t)d1 * (uint32_t)cld(g.nu_abs, je + 1);
            }
          }
        };
        if constexpr (NSEG > 0) {
#pragma unroll
          for (int base = 0; base < RMAX; base += 16) {
            const uint32_t cw = (uint32_t)crit[(base >> 5) * WG] >> (base & 31);
            V16 lam;
#pragma unroll
            for (int e = 0; e < 16; e += 4) {
              const int j0 = base + e;
              const RateLaw* lawp = g.law;
              asm volatile("" : "+s"(lawp));
              const RateLaw L0 = law_at(lawp, j0), L1 = law_at(lawp, j0 + 1);
              const RateLaw L2 = law_at(lawp, j0 + 2), L3 = law_at(lawp, j0 + 3);
              const int32_t A0 = xc[L0.ia * WG], B0 = xc[L0.ib * WG];
              const int32_t A1 = xc[L1.ia * WG], B1 = xc[L1.ib * WG];
              const int32_t A2 = xc[L2.ia * WG], B2 = xc[L2.ib * WG];
              const int32_t A3 = xc[L3.ia * WG], B3 = xc[L3.ib * WG];
              lam[e] = ((cw >> e) & 1u) ? R(0) : c[j0] * hval<R>(A0, B0 + L0.db, L0.dimer) * taur;
              lam[e + 1] = ((cw >> (e + 1)) & 1u)
                               ? R(0)
                               : c[j0 + 1] * hval<R>(A1, B1 + L1.db, L1.dimer) * taur;
              lam[e + 2] = ((cw >> (e + 2)) & 1u)
                               ? R(0)
                               : c[j0 + 2] * hval<R>(A2, B2 + L2.db, L2.dimer) * taur;
              lam[e + 3] = ((cw >> (e + 3)) & 1u)
                               ? R(0)
                               : c[j0 + 3] * hval<R>(A3, B3 + L3.db, L3.dimer) * taur;
            }
            draw_block(base, lam);
          }
        } else {
          for (int base = 0; base < M; base += 16) {
            V16 lam;
            R q[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) q[e] = mrate(base + e);  // 0 past the last row
#pragma unroll
            for (int e = 0; e < 16; ++e) {
              const int j = base + e;
              lam[e] = (j < M && !critbit(j)) ? prop(j, q[e]) * taur : R(0);
            }
            draw_block(base, lam);
          }
        }
        int jc = -1;
        if (fire) {
          const double r = u53(ev.w2, ev.w3) * a0c;
          double acc = 0.0;
          int last = -1;
          uint32_t cw2 = 0;
#pragma unroll 1
          for (int j = 0; j < M && __any(jc < 0); ++j) {
            if ((j & 31) == 0) cw2 = (uint32_t)crit[(j >> 5) * WG];
            if (jc < 0 && ((cw2 >> (j & 31)) & 1u)) {
              const double a = (double)prop(j, rate_at(j));
              acc = acc + a;
              if (a > 0.0) last = j;
              if (r < acc) jc = j;
            }
          }
          if (jc < 0) jc = last;
          if (jc < 0) { finish(kStAbsorbed); break; }
          apply(xn, jc, 1);
          kabs += (uint32_t)cld(g.nu_abs, jc);
        }

        bool neg = false, big = false;
        if ((uint64_t)xmax + kabs <= (uint64_t)INT32_MAX) {
          // no partial sum can leave the int32 range: the candidate is exact
          for (int i = 0; i < N; ++i) neg = neg || (xn[i * WG] < 0);
        } else {
          // exact 64-bit evaluation, species by species, redrawing each k_j
          for (int i = 0; i < N; ++i) {
            int64_t acc = xc[i * WG];
            for (int e = cld(g.col_ptr, i); e < cld(g.col_ptr, i + 1); ++e) {
              const int2 en = cld2(g.col_ent, e);
              const int j = en.x;
              int64_t kj;
              if (critbit(j)) {
                kj = (fire && j == jc) ? 1 : 0;
              } else {
                const R lam = prop(j, rate_at(j)) * taur;
                Words w = {0u, 0u, 0u, 0u};
                if (lam > R(0) && lam < R(10))
                  w = philox10(traj, n, (uint32_t)(j >> 1), kStreamFirst, k0, k1);
                const uint32_t hi = (j & 1) ? w.w2 : w.w0;
                const uint32_t lo = (j & 1) ? w.w3 : w.w1;
                kj = poisson<R>(lam, hi, lo, traj, n, (uint32_t)j, k0, k1, g.log_fact,
                                p.cle_threshold);
              }
              acc += kj * (int64_t)en.y;
            }
            if (acc < 0) neg = true;
            else if (acc > INT32_MAX) big = true;
          }
        }
        if (neg) {
          tau_p = tau_p * 0.5;
          n = n + 1;
          rej = rej + 1;
          break;  // stays in leap mode
        }
        if (big) { finish(kStOverflow); break; }
        int32_t* tmp = xc;
        xc = xn;
        xn = tmp;
        if (tau == delta) t = t_next;
        else t = t + tau;
        n = n + 1;
        leaps = leaps + 1;
        while (s < S && t_next <= t) record_next();
        if (s == S) { mode = kDone; break; }
        mode = kDecide;
      } while (false);
    }
  }

  if (valid) {
    uint64_t* st = p.stats + tl * 4;
    st[0] = leaps;
    st[1] = ssa;
    st[2] = rej;
    st[3] = status;
  }
}

template <int WG, int NSEG, typename R>
__global__ __launch_bounds__(WG, 1) void sweep_kernel(const SweepParams p) {
  sweep_block<WG, NSEG, R>(p, (int64_t)blockIdx.x * WG);
}

// Persistent form for batches: each workgroup takes (job, block) items from a
// device queue until it is empty, and runs block `block` of job `job` exactly
// as sweep_kernel's workgroup `block` would.  Job parameters are read through
// the constant address space, so they land in scalar registers as a kernel
// argument does.
typedef const uint32_t __attribute__((address_space(4)))* const_u32_ptr;

template <int WG, int NSEG, typename R>
__global__ __launch_bounds__(WG, 1) void sweep_persistent(const BatchQueue q) {
  __shared__ int32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(q.next, 1u);
    __syncthreads();
    const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // every lane has read the item before it is replaced
    if (it >= q.n_items) return;
    const int32_t job = __builtin_amdgcn_readfirstlane(q.items[2 * it]);
    const int32_t blk = __builtin_amdgcn_readfirstlane(q.items[2 * it + 1]);
    SweepParams p;
    static_assert(sizeof(SweepParams) % 4 == 0, "parameter block of whole words");
    const const_u32_ptr src = (const_u32_ptr)(q.jobs + job);
    uint32_t* const dst = (uint32_t*)&p;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(SweepParams) / 4); ++k) dst[k] = src[k];
    sweep_block<WG, NSEG, R>(p, (int64_t)blk * WG);
  }
}

template <int WG, int NSEG, typename R>
hipError_t launch_one(const SweepParams& p, size_t lds, hipStream_t stream, int64_t blocks) {
  hipLaunchKernelGGL((sweep_kernel<WG, NSEG, R>), dim3((unsigned)blocks), dim3(WG), lds, stream,
                     p);
  return hipGetLastError();
}

template <int WG, typename R>
hipError_t launch_wg(const SweepParams& p, const LaunchCfg& cfg, hipStream_t stream,
                     int64_t blocks) {
  switch (cfg.rate_segs) {
    case 1: return launch_one<WG, 1, R>(p, cfg.lds_bytes, stream, blocks);
    case 2: return launch_one<WG, 2, R>(p, cfg.lds_bytes, stream, blocks);
    case 3: return launch_one<WG, 3, R>(p, cfg.lds_bytes, stream, blocks);
    case 4: return launch_one<WG, 4, R>(p, cfg.lds_bytes, stream, blocks);
    case 5: return launch_one<WG, 5, R>(p, cfg.lds_bytes, stream, blocks);
    case 6: return launch_one<WG, 6, R>(p, cfg.lds_bytes, stream, blocks);
    case 7: return launch_one<WG, 7, R>(p, cfg.lds_bytes, stream, blocks);
    case 8: return launch_one<WG, 8, R>(p, cfg.lds_bytes, stream, blocks);
    case 0: return launch_one<WG, 0, R>(p, cfg.lds_bytes, stream, blocks);
    default: return hipErrorInvalidValue;
  }
}

template <int WG, typename R>
hipError_t launch_persistent_wg(const BatchQueue& q, const LaunchCfg& cfg, hipStream_t stream,
                                int64_t groups) {
#define RN_PERSIST(K)                                                                      \
  case K:                                                                                  \
    hipLaunchKernelGGL((sweep_persistent<WG, K, R>), dim3((unsigned)groups), dim3(WG),     \
                       cfg.lds_bytes, stream, q);                                          \
    return hipGetLastError();
  switch (cfg.rate_segs) {
    RN_PERSIST(0)
    RN_PERSIST(1)
    RN_PERSIST(2)
    RN_PERSIST(3)
    RN_PERSIST(4)
    RN_PERSIST(5)
    RN_PERSIST(6)
    RN_PERSIST(7)
    RN_PERSIST(8)
    default: return hipErrorInvalidValue;
  }
#undef RN_PERSIST
}

template <typename R>
hipError_t launch_persistent_prec(const BatchQueue& q, const LaunchCfg& cfg, hipStream_t stream,
                                  int64_t groups) {
  if (groups <= 0) return hipSuccess;
  switch (cfg.wg) {
    case 64: return launch_persistent_wg<64, R>(q, cfg, stream, groups);
    case 256: return launch_persistent_wg<256, R>(q, cfg, stream, groups);
    default: return hipErrorInvalidValue;
  }
}

template <typename R>
hipError_t launch_sweep_prec(const SweepParams& p, const LaunchCfg& cfg, hipStream_t stream) {
  const int64_t blocks = (p.n_traj + cfg.wg - 1) / cfg.wg;
  if (blocks <= 0) return hipSuccess;
  switch (cfg.wg) {
    case 64: return launch_wg<64, R>(p, cfg, stream, blocks);
    case 256: return launch_wg<256, R>(p, cfg, stream, blocks);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace rn
