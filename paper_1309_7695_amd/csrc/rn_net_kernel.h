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

  auto record = [&](int si) {
    if (!valid) return;
    // a fresh copy of the row stride per call keeps the N row offsets from
    // being hoisted out of the main loop (they would pin 2N scalar registers)
    int64_t ld = p.out_ld;
    asm volatile("" : "+s"(ld));
    int32_t* o = p.out + (int64_t)si * N * ld + tl;
    sfor<0, N>([&](auto ic) {
      o[0] = x[decltype(ic)::value];
      o += ld;
    });
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
        R sum = R(0);
        sfor<0, M>([&](auto jc) { sum = sum + aj(jc); });
        if (sum == R(0)) { finish(kStAbsorbed); break; }
        const Words w = philox10(traj, n, 0u, kStreamEvent, k0, k1);
        const R tau = -Real<R>::log_(R(1) - Real<R>::uni(w.w0, w.w1)) / sum;
        const double tn = t + (double)tau;
        while (s < S && t_next < tn) record_next();
        if (s == S) { mode = kDone; break; }
        fence();
        const R r = Real<R>::uni(w.w2, w.w3) * sum;
        R acc = R(0);
        int pick = -1, last = -1;
        sfor<0, (M + 3) / 4>([&](auto gc) {
          constexpr int g4 = 4 * decltype(gc)::value;
          if (__any(pick < 0)) {
            sfor<g4, (g4 + 4 < M ? g4 + 4 : M)>([&](auto jc) {
              constexpr int j = decltype(jc)::value;
              // selects, not branches: a lane that has picked keeps its state
              const bool open = pick < 0;
              const R a = aj(jc);
              const R acc2 = acc + a;
              acc = open ? acc2 : acc;
              last = (open && a > R(0)) ? j : last;
              pick = (open && r < acc2) ? j : pick;
            });
          }
        });
        if (pick < 0) pick = last;
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
    if (ph_leap) RN_TB();
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
        double a0c = 0.0;
        fence();
        if (__any(any_crit != 0u)) {
          sfor<0, M>([&](auto jc) {
            const double a = (double)aj(jc);
            a0c = critbit(jc) ? a0c + a : a0c;
          });
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

        // Candidate counts xn; the additions wrap instead of overflowing, and a
        // candidate whose sums could leave the int32 range is never used (the
        // exact path below decides).
        int32_t xmax = 0;
        sfor<0, N>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          xn[i * WG] = x[i];
          xmax = max(xmax, x[i]);
        });
        uint64_t kabs = 0;
        const R taur = (R)tau;
        // Poisson firings of the non-critical reactions over tau, 16 reactions
        // at a time: their means go into one fresh register vector, a rolled
        // loop draws them in pairs (the two reactions of a pair share one
        // Philox block of the first-uniform stream), then each reaction's
        // draw is added to the candidate.
        sfor<0, (M + 15) / 16>([&](auto bc) {
          constexpr int base = 16 * decltype(bc)::value;
          fence();
          const uint32_t cw = crit[base >> 5] >> (base & 31);
          V16 lam;
          sfor<0, 16>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            if constexpr (base + e < M) {
              const R lv = aj(Ix<base + e>{}) * taur;
              lam[e] = ((cw >> e) & 1u) ? R(0) : lv;
            } else {
              lam[e] = R(0);
            }
          });
          I16 kv;
          // one reaction per iteration, so the samplers (PTRS inlined) have a
          // single copy per block; the pair's Philox block is made at even e
          Words w = {0u, 0u, 0u, 0u};
#pragma unroll 1
          for (int e = 0; e < 16; ++e) {
            const int je = base + e;
            if (je >= M) break;
            const R le = lam[e];
            if ((e & 1) == 0) {
              const R lo = lam[e + 1];
              w = {0u, 0u, 0u, 0u};
              if ((le > R(0) && le < R(10)) || (lo > R(0) && lo < R(10)))
                w = philox10(traj, n, (uint32_t)(je >> 1), kStreamFirst, k0, k1);
            }
            const uint32_t hi = (e & 1) ? w.w2 : w.w0;
            const uint32_t lw = (e & 1) ? w.w3 : w.w1;
            kv[e] = (int32_t)poisson<R, true>(le, hi, lw, traj, n, (uint32_t)je, k0, k1,
                                              p.net.log_fact, p.cle_threshold);
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
        });
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
    if (ph_leap) RN_TE(2);
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

}  // namespace
}  // namespace netk
}  // namespace rn
