// rn_hybrid.hip -- hybrid stochastic/deterministic sweep, one lane per
// parameterization (paper, Methods section: abundant species follow the
// mean-field equations while low-amount species keep their fluctuations; the
// process is piecewise-deterministic, Davis 1984).
//
// The caller marks each reaction continuous or discrete.  Between jumps the
// state follows dy/dt = sum over continuous j of nu_j c_j h_j(y) (rate-equation
// h), integrated by the Dormand-Prince 5(4) pair with the controller of the
// rate-equation sweep.  The integral L of the discrete intensity
// a0_D(y) = sum over discrete j of max(0, c_j h_j(y)) (stochastic h, with
// y(y-1)/2 for a homodimer) rides the same step as one more component.  A jump
// comes when L reaches an Exp(1) draw xi (the integrated-intensity construction
// of Salis and Kaznessis, J. Chem. Phys. 122, 054103 (2005)); an accepted step
// that carries L past xi has its length searched from the same start by the
// Illinois variant of regula falsi until |L - xi| <= 1e-12 (1 + xi) or 30
// trials, and the reaction that jumps is the first discrete j with
// u * a0_D < a_1 + ... + a_j.  Jump k of trajectory tr draws (xi, u) from the
// Philox block (tr, k, 0, 2^31).
//
// Two kernels compute this.
//  - Networks of at most 64 species: one wave per trajectory, one lane per
//    species.  The lane keeps its species' entries of the twelve state vectors
//    in registers; a stage argument goes through LDS so that every lane can
//    form its own right-hand side f_i over the reactions that change species
//    i, and sums over species (error norm, discrete intensity) are wave
//    reductions.  The rates of the trajectory sit in LDS.  Reductions add in a
//    butterfly order, not in index order, so results differ from the oracle by
//    rounding; the jumping reaction is still chosen from index-ordered sums,
//    as the oracle does.
//  - Larger networks: one lane per trajectory, its twelve state vectors in a
//    caller workspace, trajectory-minor (work[(v * N + i) * work_ld + t]), so
//    every access of a wave covers 64 consecutive doubles; tables and the
//    partition are read at wave-uniform indices through the scalar cache.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rn_device.h"
#include "rn_dopri.h"
#include "rn_kernel.h"
#include "rn_wave.h"

namespace rn {
namespace {

using namespace dopri;
using namespace wave;

typedef const int32_t __attribute__((address_space(4)))* const_i32_ptr;
__device__ __forceinline__ int32_t hword(const void* base, int64_t i) {
  return ((const_i32_ptr)base)[i];
}

constexpr uint32_t kStreamHybrid = 0x80000000u;
constexpr uint32_t kHybMaxSteps = 2u;  // status bit, as the other sweeps
constexpr int kHybWG = 128;
constexpr int kLocateMax = 30;
constexpr double kLocateTol = 1e-12;

// Workspace slots: state, candidate, seven stage derivatives, stage argument,
// and the candidate and last derivative of a jump-search trial.
enum : int { kY = 0, kYN, kK1, kK2, kK3, kK4, kK5, kK6, kK7, kS, kYE, kKE };

__global__ __launch_bounds__(kHybWG) void hybrid_lane_kernel(const HybridParams p) {
  const DevNet& g = p.net;
  const int N = g.N, M = g.M_real;
  const int64_t tl = (int64_t)blockIdx.x * kHybWG + threadIdx.x;
  if (tl >= p.n_traj) return;  // lanes are independent: no barrier follows
  const int64_t ld = p.work_ld;
  double* const w = p.work + tl;
  auto V = [&](int slot, int i) -> double& { return w[((int64_t)slot * N + i) * ld]; };
  const double* const crate = p.rates + tl;
  const double* __restrict__ times = p.times;
  const int S = p.n_times;
  const uint32_t traj = p.traj_offset + (uint32_t)tl;

  auto yv = [&](int slot, int32_t i) -> double { return i < N ? V(slot, i) : 1.0; };
  // Discrete intensity of reaction j at `slot` (stochastic form, floored at 0).
  auto intensity = [&](int j, int slot) -> double {
    const int32_t ia = hword(g.law, 4 * j), ib = hword(g.law, 4 * j + 1);
    const double ya = yv(slot, ia);
    double h;
    if (hword(g.law, 4 * j + 3)) h = 0.5 * (ya * (ya - 1.0));
    else h = ya * yv(slot, ib);
    const double a = crate[(int64_t)j * p.rates_ld] * h;
    return a > 0.0 ? a : 0.0;
  };
  // Flow at slot `in` into slot `outv` (each f_i over its continuous reactions
  // in increasing j); returns a0_D (discrete reactions in increasing j).
  auto rhs = [&](int in, int outv) -> double {
    for (int i = 0; i < N; ++i) {
      double f = 0.0;
      const int e1 = hword(g.col_ptr, i + 1);
      for (int e = hword(g.col_ptr, i); e < e1; ++e) {
        const int j = hword(g.col_ent, 2 * e);
        if (!hword(p.cont, j)) continue;
        const int v = hword(g.col_ent, 2 * e + 1);
        const int32_t ia = hword(g.law, 4 * j), ib = hword(g.law, 4 * j + 1);
        const double ya = yv(in, ia);
        double h;
        if (hword(g.law, 4 * j + 3)) h = 0.5 * (ya * ya);
        else h = ya * yv(in, ib);
        const double a = crate[(int64_t)j * p.rates_ld] * h;
        f = f + (double)v * a;
      }
      V(outv, i) = f;
    }
    double a0 = 0.0;
    for (int j = 0; j < M; ++j)
      if (!hword(p.cont, j)) a0 = a0 + intensity(j, in);
    return a0;
  };
  // One Dormand-Prince step of length hu from (slot y, L) with k1 and kl[0]:
  // candidate into slot yo, its derivative into slot ko, L' into *Lo; returns
  // the error norm.
  auto step = [&](double hu, int y, double L, int k1, int yo, int ko, double* kl,
                  double* Lo) -> double {
    for (int i = 0; i < N; ++i) V(kS, i) = V(y, i) + hu * (A21 * V(k1, i));
    kl[1] = rhs(kS, kK2);
    for (int i = 0; i < N; ++i) V(kS, i) = V(y, i) + hu * (A31 * V(k1, i) + A32 * V(kK2, i));
    kl[2] = rhs(kS, kK3);
    for (int i = 0; i < N; ++i)
      V(kS, i) = V(y, i) + hu * (A41 * V(k1, i) + A42 * V(kK2, i) + A43 * V(kK3, i));
    kl[3] = rhs(kS, kK4);
    for (int i = 0; i < N; ++i)
      V(kS, i) = V(y, i) + hu * (A51 * V(k1, i) + A52 * V(kK2, i) + A53 * V(kK3, i) +
                                 A54 * V(kK4, i));
    kl[4] = rhs(kS, kK5);
    for (int i = 0; i < N; ++i)
      V(kS, i) = V(y, i) + hu * (A61 * V(k1, i) + A62 * V(kK2, i) + A63 * V(kK3, i) +
                                 A64 * V(kK4, i) + A65 * V(kK5, i));
    kl[5] = rhs(kS, kK6);
    for (int i = 0; i < N; ++i)
      V(yo, i) = V(y, i) + hu * (B1 * V(k1, i) + B3 * V(kK3, i) + B4 * V(kK4, i) +
                                 B5 * V(kK5, i) + B6 * V(kK6, i));
    kl[6] = rhs(yo, ko);
    *Lo = L + hu * (B1 * kl[0] + B3 * kl[2] + B4 * kl[3] + B5 * kl[4] + B6 * kl[5]);
    double e2 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double e = hu * (E1 * V(k1, i) + E3 * V(kK3, i) + E4 * V(kK4, i) + E5 * V(kK5, i) +
                             E6 * V(kK6, i) + E7 * V(ko, i));
      const double ay = fabs(V(y, i)), an = fabs(V(yo, i));
      const double sc = p.atol + p.rtol * (ay > an ? ay : an);
      e2 = e2 + (e / sc) * (e / sc);
    }
    const double en = sqrt(e2 / N);
    const double el =
        hu * (E1 * kl[0] + E3 * kl[2] + E4 * kl[3] + E5 * kl[4] + E6 * kl[5] + E7 * kl[6]);
    const double al = fabs(L), anl = fabs(*Lo);
    const double ll = fabs(el) / (p.atol + p.rtol * (al > anl ? al : anl));
    return ll > en ? ll : en;
  };
  auto record = [&](int yslot, int si) {
    double* o = p.out + (int64_t)si * N * p.out_ld + tl;
    for (int i = 0; i < N; ++i) o[(int64_t)i * p.out_ld] = V(yslot, i);
  };
  auto draw = [&](uint32_t k, double* xi, double* u) {
    const dev::Words r = dev::philox10(traj, k, 0u, kStreamHybrid, p.key0, p.key1);
    *xi = -log(1.0 - dev::u53(r.w0, r.w1));
    *u = dev::u53(r.w2, r.w3);
  };

  int ys = kY, yn = kYN, k1 = kK1, k7 = kK7;
  for (int i = 0; i < N; ++i)
    V(ys, i) = (double)(p.x0_ld ? p.x0[(int64_t)i * p.x0_ld + tl] : p.x0[i]);
  double t = 0.0, L = 0.0, xi, u;
  uint32_t njump = 0;
  draw(0u, &xi, &u);
  int s = 0;
  uint64_t acc = 0, rej = 0;
  uint32_t status = 0;
  while (s < S && times[s] <= t) record(ys, s++);
  double kl[7];
  kl[0] = rhs(ys, k1);
  double d0 = 0.0, d1 = 0.0;
  for (int i = 0; i < N; ++i) {
    const double y = V(ys, i);
    const double sc = p.atol + p.rtol * fabs(y);
    const double f = V(k1, i);
    d0 = d0 + (y / sc) * (y / sc);
    d1 = d1 + (f / sc) * (f / sc);
  }
  d0 = sqrt(d0 / N);
  d1 = sqrt(d1 / N);
  double h = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  bool last_rejected = false;
  while (s < S) {
    if (acc + rej >= p.max_steps) {
      status |= kHybMaxSteps;
      break;
    }
    const double delta = times[s] - t;
    const bool clip = !(h < delta);
    const double hu = clip ? delta : h;
    double Ln;
    const double en = step(hu, ys, L, k1, yn, k7, kl, &Ln);
    if (!(en <= 1.0)) {
      double fac = 0.9 * pow(en, -0.2);
      if (fac < 0.2) fac = 0.2;
      h = hu * fac;
      rej = rej + 1;
      last_rejected = true;
      continue;
    }
    double fac = en == 0.0 ? 5.0 : 0.9 * pow(en, -0.2);
    if (fac > 5.0) fac = 5.0;
    if (fac < 0.2) fac = 0.2;
    if (last_rejected && fac > 1.0) fac = 1.0;
    last_rejected = false;
    acc = acc + 1;
    if (Ln < xi) {  // no jump inside the step
      int tmp = ys;
      ys = yn;
      yn = tmp;
      tmp = k1;
      k1 = k7;
      k7 = tmp;
      kl[0] = kl[6];
      L = Ln;
      if (clip) t = times[s];
      else t = t + hu;
      h = hu * fac;
      while (s < S && times[s] <= t) record(ys, s++);
      continue;
    }
    // The jump lies in (0, hu]: search the step length (Illinois regula falsi
    // on g = L - xi over [0, hu]), each trial a full step from the same start.
    double he = 0.0;
    int ye = ys;  // a zero-length search leaves the state as it is
    if (xi - L > 0.0) {
      double hl = 0.0, gl = L - xi, hr = hu, gr = Ln - xi;
      int side = 0;
      for (int r = 0; r < kLocateMax; ++r) {
        he = hl - gl * ((hr - hl) / (gr - gl));
        double kle[7], Le;
        kle[0] = kl[0];
        (void)step(he, ys, L, k1, kYE, kKE, kle, &Le);
        ye = kYE;
        rej = rej + 1;
        const double ge = Le - xi;
        if (fabs(ge) <= kLocateTol * (1.0 + xi)) break;
        if (ge < 0.0) {
          hl = he;
          gl = ge;
          if (side < 0) gr = 0.5 * gr;
          side = -1;
        } else {
          hr = he;
          gr = ge;
          if (side > 0) gl = 0.5 * gl;
          side = 1;
        }
      }
    }
    if (ye != ys)
      for (int i = 0; i < N; ++i) V(ys, i) = V(ye, i);
    t = t + he;
    h = hu * fac;
    while (s < S && times[s] <= t) record(ys, s++);  // samples take the pre-jump state
    double a0 = 0.0;
    for (int j = 0; j < M; ++j)
      if (!hword(p.cont, j)) a0 = a0 + intensity(j, ys);
    if (a0 > 0.0) {
      const double rr = u * a0;
      double cum = 0.0;
      int pick = -1, last = -1;
      for (int j = 0; j < M && pick < 0; ++j) {
        if (hword(p.cont, j)) continue;
        const double a = intensity(j, ys);
        cum = cum + a;
        if (a > 0.0) last = j;
        if (rr < cum) pick = j;
      }
      if (pick < 0) pick = last;
      const int n1 = hword(g.nu_ptr, pick + 1);
      for (int e = hword(g.nu_ptr, pick); e < n1; ++e) {
        const int sp = hword(g.nu_ent, 2 * e);
        V(ys, sp) = V(ys, sp) + (double)hword(g.nu_ent, 2 * e + 1);
      }
    }
    njump = njump + 1;
    draw(njump, &xi, &u);
    L = 0.0;
    kl[0] = rhs(ys, k1);
  }
  while (s < S) record(ys, s++);
  uint64_t* st = p.stats + tl * 4;
  st[0] = acc;
  st[1] = rej;
  st[2] = njump;
  st[3] = status;
}

constexpr int kWaveWG = 64;
constexpr int kLaneEntries = 8;  // continuous reactions of a species held in registers
constexpr int kLaneSlots = 2;     // reactions of a lane (j = lane + 64 d) held in registers
constexpr int kZ = 66;            // LDS words of the stage argument (z[N] = 1)


// kOde: every reaction continuous and p.cont unused, i.e. the reaction-rate
// equations of rn_ode_sweep (no draws, no jumps).
template <bool kOde>
__global__ __launch_bounds__(kWaveWG) __attribute__((amdgpu_waves_per_eu(3, 8)))
void hybrid_wave_kernel(const HybridParams p) {
  const DevNet& g = p.net;
  const int N = g.N, M = g.M_real;
  const int64_t tl = blockIdx.x;  // one trajectory per wave
  const int lane = (int)threadIdx.x;
  const bool own = lane < N;     // the lane carries species `lane`
  const uint32_t traj = p.traj_offset + (uint32_t)tl;
  auto is_cont = [&](int j) -> bool { return kOde || p.cont[j] != 0; };
  // LDS: stage argument z[kZ] (z[N] = 1, the pseudo-species of lower-order
  // laws), this trajectory's rates c[M], intensities av[M] at a jump, the
  // continuous reactions' rates ac[M] at the stage argument, and the discrete
  // reactions in increasing index dj[nd].
  extern __shared__ double sh[];
  double* const z = sh;
  double* const c = sh + kZ;
  double* const av = c + M;
  double* const ac = av + M;
  int* const dj = (int*)(ac + M);
  for (int j = lane; j < M; j += kWaveWG) c[j] = p.rates[(int64_t)j * p.rates_ld + tl];
  if (lane == 0) z[N] = 1.0;
  int nd = 0;  // every lane counts; lane 0 writes the list
  for (int j = 0; j < M; ++j) {
    if (is_cont(j)) continue;
    if (lane == 0) dj[nd] = j;
    ++nd;
  }
  const double* __restrict__ times = p.times;
  const int S = p.n_times;
  // Reaction slots of this lane: j = lane + 64 d for d < kLaneSlots, with
  // their packed law and rate in registers (law < 0: past M); continuous ones
  // publish a_j to LDS, discrete ones add to the lane's share of a0_D.
  double sc_[kLaneSlots];
  int sl[kLaneSlots];
  bool scont[kLaneSlots];
#pragma unroll
  for (int d = 0; d < kLaneSlots; ++d) {
    const int j = lane + kWaveWG * d;
    const bool in = j < M;
    sc_[d] = in ? p.rates[(int64_t)j * p.rates_ld + tl] : 0.0;
    sl[d] = in ? pack_law(g.law[j]) : -1;
    scont[d] = in && is_cont(j);
  }
  // This lane's species column (reactions that change it, ascending j): the
  // first kLaneEntries continuous ones as (j, nu) in registers, the rest read
  // from the tables from index `ovf` on.
  const int cb = own ? g.col_ptr[lane] : 0, ce = own ? g.col_ptr[lane + 1] : 0;
  int ej[kLaneEntries], ev[kLaneEntries];
  int cnt = 0, ovf = ce;
  for (int e = cb; e < ce; ++e) {
    const int2 ent = g.col_ent[e];
    if (!is_cont(ent.x)) continue;
    if (cnt == kLaneEntries) {
      ovf = e;
      break;
    }
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k)
      if (k == cnt) {
        ej[k] = ent.x;
        ev[k] = ent.y;
      }
    ++cnt;
  }

  auto h_stoch = [&](int pl) -> double {  // stochastic mass-action factor at z
    const double ya = z[pl & 0xff];
    return (pl >> 16) ? 0.5 * (ya * (ya - 1.0)) : ya * z[(pl >> 8) & 0xff];
  };
  auto h_det = [&](int pl) -> double {  // rate-equation factor at z
    const double ya = z[pl & 0xff];
    return (pl >> 16) ? 0.5 * (ya * ya) : ya * z[(pl >> 8) & 0xff];
  };
  auto intensity = [&](int j) -> double {  // from z and the tables, floored at 0
    const double a = c[j] * h_stoch(pack_law(g.law[j]));
    return a > 0.0 ? a : 0.0;
  };
  // Publish v as the stage argument and return (f_lane, a0_D) at it: every
  // reaction's rate is formed once (continuous ones through LDS, ac[j]), then
  // each species lane sums nu_ij a_j over its column in increasing j.
  auto rhs = [&](double v, double* a0) -> double {
    __syncthreads();
    if (own) z[lane] = v;
    __syncthreads();
    double part = 0.0;
#pragma unroll
    for (int d = 0; d < kLaneSlots; ++d) {
      if (sl[d] >= 0) {
        if (scont[d]) {
          ac[lane + kWaveWG * d] = sc_[d] * h_det(sl[d]);
        } else {
          const double a = sc_[d] * h_stoch(sl[d]);
          part = part + (a > 0.0 ? a : 0.0);
        }
      }
    }
    for (int j = lane + kWaveWG * kLaneSlots; j < M; j += kWaveWG) {
      if (is_cont(j)) ac[j] = c[j] * h_det(pack_law(g.law[j]));
      else part = part + intensity(j);
    }
    __syncthreads();
    double f = 0.0;
#pragma unroll
    for (int k = 0; k < kLaneEntries; ++k)
      if (k < cnt) f = f + (double)ev[k] * ac[ej[k]];
    for (int e = ovf; e < ce; ++e) {
      const int2 ent = g.col_ent[e];
      if (is_cont(ent.x)) f = f + (double)ent.y * ac[ent.x];
    }
    *a0 = kOde ? 0.0 : wave_sum(part);  // no discrete reactions in the ODE form
    return f;
  };
  struct Stage {
    double k2, k3, k4, k5, k6;
  };
  // One Dormand-Prince step of length hu from (y, L) with k1, kl[0]: this
  // lane's candidate and last derivative, L', the error norm.
  auto step = [&](double hu, double y, double L, double k1, double* kl, Stage& q, double* yo,
                  double* ko, double* Lo) -> double {
    q.k2 = rhs(y + hu * (A21 * k1), &kl[1]);
    q.k3 = rhs(y + hu * (A31 * k1 + A32 * q.k2), &kl[2]);
    q.k4 = rhs(y + hu * (A41 * k1 + A42 * q.k2 + A43 * q.k3), &kl[3]);
    q.k5 = rhs(y + hu * (A51 * k1 + A52 * q.k2 + A53 * q.k3 + A54 * q.k4), &kl[4]);
    q.k6 = rhs(y + hu * (A61 * k1 + A62 * q.k2 + A63 * q.k3 + A64 * q.k4 + A65 * q.k5), &kl[5]);
    *yo = y + hu * (B1 * k1 + B3 * q.k3 + B4 * q.k4 + B5 * q.k5 + B6 * q.k6);
    *ko = rhs(*yo, &kl[6]);
    *Lo = L + hu * (B1 * kl[0] + B3 * kl[2] + B4 * kl[3] + B5 * kl[4] + B6 * kl[5]);
    double t2 = 0.0;
    if (own) {
      const double e = hu * (E1 * k1 + E3 * q.k3 + E4 * q.k4 + E5 * q.k5 + E6 * q.k6 + E7 * *ko);
      const double ay = fabs(y), an = fabs(*yo);
      const double sc = p.atol + p.rtol * (ay > an ? ay : an);
      t2 = (e / sc) * (e / sc);
    }
    const double en = sqrt(wave_sum(t2) / N);
    const double el =
        hu * (E1 * kl[0] + E3 * kl[2] + E4 * kl[3] + E5 * kl[4] + E6 * kl[5] + E7 * kl[6]);
    const double al = fabs(L), anl = fabs(*Lo);
    const double ll = fabs(el) / (p.atol + p.rtol * (al > anl ? al : anl));
    return ll > en ? ll : en;
  };
  auto record = [&](double y, int si) {
    if (own) p.out[((int64_t)si * N + lane) * p.out_ld + tl] = y;
  };
  auto draw = [&](uint32_t k, double* xi, double* u) {
    const dev::Words r = dev::philox10(traj, k, 0u, kStreamHybrid, p.key0, p.key1);
    *xi = -log(1.0 - dev::u53(r.w0, r.w1));
    *u = dev::u53(r.w2, r.w3);
  };

  double y = own ? (double)(p.x0_ld ? p.x0[(int64_t)lane * p.x0_ld + tl] : p.x0[lane]) : 0.0;
  double t = 0.0, L = 0.0, xi, u;
  uint32_t njump = 0;
  if (kOde) {
    xi = __builtin_huge_val();  // no discrete reactions: L stays 0
    u = 0.0;
  } else {
    draw(0u, &xi, &u);
  }
  int s = 0;
  uint64_t acc = 0, rej = 0;
  uint32_t status = 0;
  while (s < S && times[s] <= t) record(y, s++);
  double kl[7];
  double k1 = rhs(y, &kl[0]);
  double d0 = 0.0, d1 = 0.0;
  if (own) {
    const double sc = p.atol + p.rtol * fabs(y);
    d0 = (y / sc) * (y / sc);
    d1 = (k1 / sc) * (k1 / sc);
  }
  d0 = sqrt(wave_sum(d0) / N);
  d1 = sqrt(wave_sum(d1) / N);
  double h = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  bool last_rejected = false;
  Stage q;
  // One step evaluation per iteration: an ordinary step, or a trial of the
  // jump search (Illinois regula falsi on the length of the step that carried
  // L past xi, from that step's start), so the step is inlined once.
  bool searching = false;
  double hl = 0.0, gl = 0.0, hr = 0.0, gr = 0.0, hnext = 0.0;
  int side = 0, trials = 0;
  while (s < S) {
    double hu = 0.0;
    bool clip = false;
    if (!searching) {
      if (acc + rej >= p.max_steps) {
        status |= kHybMaxSteps;
        break;
      }
      const double delta = times[s] - t;
      clip = !(h < delta);
      hu = clip ? delta : h;
    } else {
      hu = hl - gl * ((hr - hl) / (gr - gl));
    }
    double yn, k7, Ln;
    const double en = step(hu, y, L, k1, kl, q, &yn, &k7, &Ln);
    double he = 0.0, ye = y;
    if (!searching) {
      if (!(en <= 1.0)) {
        double fac = 0.9 * pow(en, -0.2);
        if (fac < 0.2) fac = 0.2;
        h = hu * fac;
        rej = rej + 1;
        last_rejected = true;
        continue;
      }
      double fac = en == 0.0 ? 5.0 : 0.9 * pow(en, -0.2);
      if (fac > 5.0) fac = 5.0;
      if (fac < 0.2) fac = 0.2;
      if (last_rejected && fac > 1.0) fac = 1.0;
      last_rejected = false;
      acc = acc + 1;
      if (Ln < xi) {  // no jump inside the step
        y = yn;
        k1 = k7;
        kl[0] = kl[6];
        L = Ln;
        if (clip) t = times[s];
        else t = t + hu;
        h = hu * fac;
        while (s < S && times[s] <= t) record(y, s++);
        continue;
      }
      hnext = hu * fac;
      if (xi - L > 0.0) {  // the jump lies in (0, hu]: search its length
        searching = true;
        hl = 0.0;
        gl = L - xi;
        hr = hu;
        gr = Ln - xi;
        side = 0;
        trials = 0;
        continue;
      }
      // xi - L <= 0: the jump is at the start of the step
    } else {
      rej = rej + 1;
      trials = trials + 1;
      const double ge = Ln - xi;
      if (!(fabs(ge) <= kLocateTol * (1.0 + xi)) && trials < kLocateMax) {
        if (ge < 0.0) {
          hl = hu;
          gl = ge;
          if (side < 0) gr = 0.5 * gr;
          side = -1;
        } else {
          hr = hu;
          gr = ge;
          if (side > 0) gl = 0.5 * gl;
          side = 1;
        }
        continue;
      }
      searching = false;
      he = hu;
      ye = yn;
    }
    y = ye;
    t = t + he;
    h = hnext;
    while (s < S && times[s] <= t) record(y, s++);  // samples take the pre-jump state
    // the jumping reaction, from intensities summed in index order
    __syncthreads();
    if (own) z[lane] = y;
    __syncthreads();
    for (int j = lane; j < M; j += kWaveWG) av[j] = is_cont(j) ? 0.0 : intensity(j);
    __syncthreads();
    double a0 = 0.0;
    for (int q = 0; q < nd; ++q) a0 = a0 + av[dj[q]];
    if (a0 > 0.0) {
      const double rr = u * a0;
      double cum = 0.0;
      int pick = -1, last = -1;
      for (int q = 0; q < nd && pick < 0; ++q) {
        const int j = dj[q];
        const double a = av[j];
        cum = cum + a;
        if (a > 0.0) last = j;
        if (rr < cum) pick = j;
      }
      if (pick < 0) pick = last;
      const int n1 = g.nu_ptr[pick + 1];
      for (int e = g.nu_ptr[pick]; e < n1; ++e) {
        const int2 ent = g.nu_ent[e];
        if (ent.x == lane) y = y + (double)ent.y;
      }
    }
    njump = njump + 1;
    draw(njump, &xi, &u);
    L = 0.0;
    k1 = rhs(y, &kl[0]);
  }
  while (s < S) record(y, s++);
  if (lane == 0) {
    uint64_t* st = p.stats + tl * 4;
    st[0] = acc;
    st[1] = rej;
    st[2] = njump;
    st[3] = status;
  }
}

// Dynamic LDS of the wave kernel: z, c, av, ac (doubles) and dj (ints).
size_t wave_lds_bytes(int64_t m) {
  return (size_t)(kZ + 3 * m) * sizeof(double) + (size_t)m * sizeof(int);
}

// Launches cover at most kLaunchChunk trajectories each (the wave kernel has
// 64 work-items per trajectory, and a dispatch holds fewer than 2^32): a
// larger sweep is enqueued as consecutive ranges, each with its pointers and
// trajectory offset moved to the range's first trajectory.
constexpr int64_t kLaunchChunk = (int64_t)1 << 24;

HybridParams sub_range(const HybridParams& p, int64_t off, int64_t n) {
  HybridParams q = p;
  q.n_traj = n;
  q.traj_offset = p.traj_offset + (uint32_t)off;
  q.rates = p.rates + off;
  if (p.x0_ld != 0) q.x0 = p.x0 + off;
  q.out = p.out + off;
  q.stats = p.stats + 4 * off;
  if (p.work) q.work = p.work + off;
  return q;
}

}  // namespace

hipError_t launch_hybrid(const HybridParams& p, hipStream_t stream) {
  const size_t lds = wave_lds_bytes(p.net.M_real);
  const bool wave = p.net.N <= kWaveWG && lds <= 65536;
  for (int64_t off = 0; off < p.n_traj; off += kLaunchChunk) {
    const HybridParams q = sub_range(p, off, std::min(kLaunchChunk, p.n_traj - off));
    if (wave) {
      hipLaunchKernelGGL(hybrid_wave_kernel<false>, dim3((unsigned)q.n_traj), dim3(kWaveWG), lds,
                         stream, q);
    } else {
      const int64_t blocks = (q.n_traj + kHybWG - 1) / kHybWG;
      hipLaunchKernelGGL(hybrid_lane_kernel, dim3((unsigned)blocks), dim3(kHybWG), 0, stream, q);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The rate-equation sweep on the wave-per-trajectory kernel (every reaction
// continuous); false when the network does not fit it (more than 64 species or
// too many reactions for its LDS), and nothing is launched.
bool ode_wave_fits(int n_species, int m_real) {
  return n_species <= kWaveWG && wave_lds_bytes(m_real) <= 65536;
}

bool launch_ode_wave(const HybridParams& p, hipStream_t stream, hipError_t* err) {
  const size_t lds = wave_lds_bytes(p.net.M_real);
  if (!ode_wave_fits(p.net.N, p.net.M_real)) return false;
  *err = hipSuccess;
  for (int64_t off = 0; off < p.n_traj; off += kLaunchChunk) {
    const HybridParams q = sub_range(p, off, std::min(kLaunchChunk, p.n_traj - off));
    hipLaunchKernelGGL(hybrid_wave_kernel<true>, dim3((unsigned)q.n_traj), dim3(kWaveWG), lds,
                       stream, q);
    *err = hipGetLastError();
    if (*err != hipSuccess) break;
  }
  return true;
}

}  // namespace rn
