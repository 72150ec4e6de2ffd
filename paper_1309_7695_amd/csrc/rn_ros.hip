// rn_ros.hip -- the reaction-rate equations of stiff networks by a linearly
// implicit Rosenbrock method, one wave per parameterization.
//
// The deterministic sweep follows dy/dt = f(y) = sum_j nu_j c_j h_j(y) (paper,
// Methods section: mean-field equations for abundant species).  Rate constants
// that span many decades make f stiff, and an explicit pair then needs steps
// of the order of the fastest time scale.  This kernel takes the Rosenbrock
// 4(3) method with gamma = 1/2 of L. F. Shampine (ACM Trans. Math. Softw. 8
// (1982) 93), in the transformed form of Hairer and Wanner (Solving ODEs II,
// Sec. IV.7): with J the exact Jacobian of f at y and W = I/(gamma h) - J,
//   W u1 = f(y)
//   W u2 = f(y + a21 u1)           + c21 u1 / h
//   W u3 = f(y + a31 u1 + a32 u2)  + (c31 u1 + c32 u2) / h
//   W u4 = f(y + a31 u1 + a32 u2)  + (c41 u1 + c42 u2 + c43 u3) / h
//   y'   = y + m1 u1 + m2 u2 + m3 u3 + m4 u4,   error = e1 u1 + e2 u2 + e3 u3 + e4 u4,
// W factored once per step by Gaussian elimination with partial pivoting.
// Error norm, step-size rule (exponent -1/4) and sample clipping are those of
// the Dormand-Prince sweep.
//
// Layout: lane i carries species i (networks of up to 64 species).  The stage
// argument goes through LDS so that each lane forms its f_i over the reactions
// that change species i, in increasing j.  W sits in LDS, one row per species;
// lane i accumulates row i of J over its column of reactions (increasing j),
// so every entry sums the same terms in the same order as a row-by-row serial
// evaluation.  Elimination keeps logical row i in the physical row held in
// lane i's `prow` (a row exchange swaps two lanes' values, i.e. whole rows
// with their stored multipliers); for column k the pivot is the first row of
// largest magnitude, each lower row's lane forms its multiplier and updates its
// own row.  Forward and back substitution run column by column: the finished
// component is broadcast and each lane subtracts its term, so each component
// takes its subtractions in the serial order.  Only the sums over species (error
// norm, first-step estimate) add in a butterfly order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rn_kernel.h"
#include "rn_wave.h"

namespace rn {
namespace {

using namespace wave;

// Shampine's Rosenbrock 4(3) coefficients, transformed form.
constexpr double kGam = 0.5;
constexpr double kA21 = 2.0, kA31 = 48.0 / 25.0, kA32 = 6.0 / 25.0;
constexpr double kC21 = -8.0, kC31 = 372.0 / 25.0, kC32 = 12.0 / 5.0;
constexpr double kC41 = -112.0 / 125.0, kC42 = -54.0 / 125.0, kC43 = -2.0 / 5.0;
constexpr double kM1 = 19.0 / 9.0, kM2 = 1.0 / 2.0, kM3 = 25.0 / 108.0, kM4 = 125.0 / 108.0;
constexpr double kE1 = 17.0 / 54.0, kE2 = 7.0 / 36.0, kE3 = 0.0, kE4 = 125.0 / 108.0;

constexpr uint32_t kRosMaxSteps = 2u;
constexpr int kRosWG = 64;
constexpr int kRosEntries = 8;  // reactions of a species column held in registers
constexpr int kRosSlots = 2;     // reactions of a lane (j = lane + 64 d) held in registers
constexpr int kRosZ = 66;        // LDS words of the stage argument (z[N] = 1)

// Row stride of W in doubles: odd, so that the rows of consecutive lanes start
// in different LDS banks.
__host__ __device__ constexpr int ros_stride(int n) { return n | 1; }

__global__ __launch_bounds__(kRosWG) __attribute__((amdgpu_waves_per_eu(2, 8)))
void ros_wave_kernel(const OdeParams p) {
  const DevNet& g = p.net;
  const int N = g.N, M = g.M_real, NS = ros_stride(N);
  const int64_t tl = blockIdx.x;  // one trajectory per wave
  const int lane = (int)threadIdx.x;
  const bool own = lane < N;
  // LDS: stage argument z (z[N] = 1), rates c[M], rates at the stage
  // argument ac[M], then W [N][NS].
  extern __shared__ double sh[];
  double* const z = sh;
  double* const c = sh + kRosZ;
  double* const ac = c + M;
  double* const W = ac + M;
  for (int j = lane; j < M; j += kRosWG) c[j] = p.rates[(int64_t)j * p.rates_ld + tl];
  if (lane == 0) z[N] = 1.0;
  const double* __restrict__ times = p.times;
  const int S = p.n_times;

  double sc_[kRosSlots];
  int sl[kRosSlots];
#pragma unroll
  for (int d = 0; d < kRosSlots; ++d) {
    const int j = lane + kRosWG * d;
    const bool in = j < M;
    sc_[d] = in ? p.rates[(int64_t)j * p.rates_ld + tl] : 0.0;
    sl[d] = in ? pack_law(g.law[j]) : -1;
  }
  // This lane's species column (reactions that change it, ascending j): the
  // first kRosEntries as (j, nu, packed law) in registers, the rest from the
  // tables from index `ovf` on.
  const int cb = own ? g.col_ptr[lane] : 0, ce = own ? g.col_ptr[lane + 1] : 0;
  int ej[kRosEntries], ev[kRosEntries], el[kRosEntries];
  const int cnt = std::min(ce - cb, kRosEntries), ovf = cb + cnt;
#pragma unroll
  for (int k = 0; k < kRosEntries; ++k) {
    const int2 ent = k < cnt ? g.col_ent[cb + k] : make_int2(0, 0);
    ej[k] = ent.x;
    ev[k] = ent.y;
    el[k] = k < cnt ? pack_law(g.law[ent.x]) : 0;
  }

  auto h_det = [&](int pl) -> double {  // rate-equation factor at z
    const double ya = z[pl & 0xff];
    return (pl >> 16) ? 0.5 * (ya * ya) : ya * z[(pl >> 8) & 0xff];
  };
  auto publish = [&](double v) {
    __syncthreads();
    if (own) z[lane] = v;
    __syncthreads();
  };
  // f_lane at v: every reaction's rate formed once into ac[], then each
  // species lane sums nu_ij a_j over its column in increasing j.
  auto rhs = [&](double v) -> double {
    publish(v);
#pragma unroll
    for (int d = 0; d < kRosSlots; ++d)
      if (sl[d] >= 0) ac[lane + kRosWG * d] = sc_[d] * h_det(sl[d]);
    for (int j = lane + kRosWG * kRosSlots; j < M; j += kRosWG)
      ac[j] = c[j] * h_det(pack_law(g.law[j]));
    __syncthreads();
    double f = 0.0;
#pragma unroll
    for (int k = 0; k < kRosEntries; ++k)
      if (k < cnt) f = f + (double)ev[k] * ac[ej[k]];
    for (int e = ovf; e < ce; ++e) {
      const int2 ent = g.col_ent[e];
      f = f + (double)ent.y * ac[ent.x];
    }
    return f;
  };
  // Row `lane` of W = I/(gamma h) - J at y (gd = 1/(gamma h)): J's row summed
  // over the lane's column in increasing j, d(c y_a)/dy_a = c,
  // d(c y_a y_b)/dy_a = c y_b, d(c y_a y_b)/dy_b = c y_a, d(c y_a^2/2)/dy_a = c y_a.
  auto jac_row = [&](double y, double gd) {
    publish(y);
    if (own) {
      double* const row = W + lane * NS;
      for (int k = 0; k < N; ++k) row[k] = 0.0;
      auto add = [&](int j, int v, int pl) {
        const int ia = pl & 0xff, ib = (pl >> 8) & 0xff;
        if (ia == N) return;  // a source: no dependence on y
        const double cj = c[j];
        if (ib == N) {
          row[ia] = row[ia] + (double)v * cj;
        } else if (pl >> 16) {
          row[ia] = row[ia] + (double)v * (cj * z[ia]);
        } else {
          row[ia] = row[ia] + (double)v * (cj * z[ib]);
          row[ib] = row[ib] + (double)v * (cj * z[ia]);
        }
      };
#pragma unroll
      for (int k = 0; k < kRosEntries; ++k)
        if (k < cnt) add(ej[k], ev[k], el[k]);
      for (int e = ovf; e < ce; ++e) {
        const int2 ent = g.col_ent[e];
        add(ent.x, ent.y, pack_law(g.law[ent.x]));
      }
      for (int k = 0; k < N; ++k) row[k] = (k == lane ? gd : 0.0) - row[k];
    }
    __syncthreads();
  };
  // LU factorization of W with partial pivoting: afterwards logical row i is
  // physical row prow (of lane i), and lane k holds the row exchanged with k
  // at step k in `piv`.
  int prow = lane, piv = lane;
  auto factor = [&]() {
    prow = lane;
    for (int k = 0; k < N; ++k) {
      // pivot: the first logical row r >= k of largest |a[r][k]| (a NaN never
      // wins, and a NaN diagonal keeps row k)
      const double v = (own && lane >= k) ? fabs(W[(own ? prow : 0) * NS + k]) : -1.0;
      const double vk = lane_double(v, k);
      int r = k;
      if (!(vk != vk)) {
        const double m = wave_max(v == v ? v : -1.0);
        const uint64_t hit = __ballot(own && lane >= k && v == m);
        r = (int)__builtin_ctzll(hit);
      }
      if (lane == k) piv = r;
      const int pk = __builtin_amdgcn_readlane(prow, k);
      const int pr = __builtin_amdgcn_readlane(prow, r);
      if (lane == k) prow = pr;
      if (lane == r) prow = pk;
      const double* const prow_k = W + pr * NS;  // physical row now at position k
      if (own && lane > k) {
        double* const row = W + prow * NS;
        const double l = row[k] / prow_k[k];
        row[k] = l;
        // four entries per pass, loads first, so their LDS latencies overlap
        int j = k + 1;
        for (; j + 3 < N; j += 4) {
          const double p0 = prow_k[j], p1 = prow_k[j + 1], p2 = prow_k[j + 2], p3 = prow_k[j + 3];
          const double r0 = row[j], r1 = row[j + 1], r2 = row[j + 2], r3 = row[j + 3];
          row[j] = r0 - l * p0;
          row[j + 1] = r1 - l * p1;
          row[j + 2] = r2 - l * p2;
          row[j + 3] = r3 - l * p3;
        }
        for (; j < N; ++j) row[j] = row[j] - l * prow_k[j];
      }
      __syncthreads();
    }
  };
  // Solve (LU) x = P b for this lane's component b: the row exchanges in
  // factorization order, then forward substitution with unit L, then back
  // substitution, column by column.
  auto solve = [&](double b) -> double {
    for (int k = 0; k < N; ++k) {
      const int r = __builtin_amdgcn_readlane(piv, k);
      if (r != k) {
        const double bk = lane_double(b, k), br = lane_double(b, r);
        if (lane == k) b = br;
        if (lane == r) b = bk;
      }
    }
    const double* const row = W + (own ? prow : 0) * NS;
    // the lane's row entries are read four at a time ahead of their use
    int k = 0;
    for (; k + 3 < N; k += 4) {
      const double w0 = row[k], w1 = row[k + 1], w2 = row[k + 2], w3 = row[k + 3];
      double bk = lane_double(b, k);
      if (own && lane > k) b = b - w0 * bk;
      bk = lane_double(b, k + 1);
      if (own && lane > k + 1) b = b - w1 * bk;
      bk = lane_double(b, k + 2);
      if (own && lane > k + 2) b = b - w2 * bk;
      bk = lane_double(b, k + 3);
      if (own && lane > k + 3) b = b - w3 * bk;
    }
    for (; k < N; ++k) {
      const double bk = lane_double(b, k);
      if (own && lane > k) b = b - row[k] * bk;
    }
    k = N - 1;
    for (; k >= 3; k -= 4) {
      const double w0 = row[k], w1 = row[k - 1], w2 = row[k - 2], w3 = row[k - 3];
      if (lane == k) b = b / w0;
      double bk = lane_double(b, k);
      if (lane < k) b = b - w0 * bk;
      if (lane == k - 1) b = b / w1;
      bk = lane_double(b, k - 1);
      if (lane < k - 1) b = b - w1 * bk;
      if (lane == k - 2) b = b / w2;
      bk = lane_double(b, k - 2);
      if (lane < k - 2) b = b - w2 * bk;
      if (lane == k - 3) b = b / w3;
      bk = lane_double(b, k - 3);
      if (lane < k - 3) b = b - w3 * bk;
    }
    for (; k >= 0; --k) {
      if (lane == k) b = b / row[k];
      const double bk = lane_double(b, k);
      if (lane < k) b = b - row[k] * bk;
    }
    return own ? b : 0.0;
  };
  auto record = [&](double y, int si) {
    if (own) p.out[((int64_t)si * N + lane) * p.out_ld + tl] = y;
  };

  double y = own ? (double)(p.x0_ld ? p.x0[(int64_t)lane * p.x0_ld + tl] : p.x0[lane]) : 0.0;
  double t = 0.0;
  int s = 0;
  uint64_t acc = 0, rej = 0;
  uint32_t status = 0;
  while (s < S && times[s] <= t) record(y, s++);
  double f0 = rhs(y);
  double d0 = 0.0, d1 = 0.0;
  if (own) {
    const double sc = p.atol + p.rtol * fabs(y);
    d0 = (y / sc) * (y / sc);
    d1 = (f0 / sc) * (f0 / sc);
  }
  d0 = sqrt(wave_sum(d0) / N);
  d1 = sqrt(wave_sum(d1) / N);
  double h = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  bool last_rejected = false;
  while (s < S) {
    if (acc + rej >= p.max_steps) {
      status |= kRosMaxSteps;
      break;
    }
    const double delta = times[s] - t;
    const bool clip = !(h < delta);
    const double hu = clip ? delta : h;
    const double ih = 1.0 / hu;
    const double gd = 1.0 / (kGam * hu);
    jac_row(y, gd);
    factor();
    const double u1 = solve(f0);
    const double fs2 = rhs(y + kA21 * u1);
    const double u2 = solve(fs2 + (kC21 * u1) * ih);
    const double fs3 = rhs(y + (kA31 * u1 + kA32 * u2));
    const double u3 = solve(fs3 + (kC31 * u1 + kC32 * u2) * ih);
    const double u4 = solve(fs3 + (kC41 * u1 + kC42 * u2 + kC43 * u3) * ih);
    const double yn = y + (kM1 * u1 + kM2 * u2 + kM3 * u3 + kM4 * u4);
    double t2 = 0.0;
    if (own) {
      const double e = kE1 * u1 + kE2 * u2 + kE3 * u3 + kE4 * u4;
      const double ay = fabs(y), an = fabs(yn);
      const double sc = p.atol + p.rtol * (ay > an ? ay : an);
      t2 = (e / sc) * (e / sc);
    }
    const double en = sqrt(wave_sum(t2) / N);
    if (en <= 1.0) {
      double fac = en == 0.0 ? 5.0 : 0.9 * pow(en, -0.25);
      if (fac > 5.0) fac = 5.0;
      if (fac < 0.2) fac = 0.2;
      if (last_rejected && fac > 1.0) fac = 1.0;
      y = yn;
      f0 = rhs(y);
      if (clip) t = times[s];
      else t = t + hu;
      h = hu * fac;
      acc = acc + 1;
      last_rejected = false;
      while (s < S && times[s] <= t) record(y, s++);
    } else {
      // a NaN norm (a singular W, an overflow) is a rejection at the smallest factor
      double fac = 0.9 * pow(en, -0.25);
      if (!(fac >= 0.2)) fac = 0.2;
      h = hu * fac;
      rej = rej + 1;
      last_rejected = true;
    }
  }
  while (s < S) record(y, s++);
  if (lane == 0) {
    uint64_t* st = p.stats + tl * 4;
    st[0] = acc;
    st[1] = rej;
    st[2] = 0;
    st[3] = status;
  }
}

size_t ros_lds_bytes(int n, int m) {
  return (size_t)(kRosZ + 2 * (size_t)m + (size_t)n * ros_stride(n)) * sizeof(double);
}

}  // namespace

bool ros_fits(int n_species, int m_real) {
  return n_species <= kRosWG && ros_lds_bytes(n_species, m_real) <= 65536;
}

// One wave per trajectory, at most 2^24 trajectories per dispatch (a dispatch
// holds fewer than 2^32 work-items).
hipError_t launch_ros(const OdeParams& p, hipStream_t stream) {
  const size_t lds = ros_lds_bytes(p.net.N, p.net.M_real);
  constexpr int64_t kChunk = (int64_t)1 << 24;
  for (int64_t off = 0; off < p.n_traj; off += kChunk) {
    OdeParams q = p;
    q.n_traj = std::min(kChunk, p.n_traj - off);
    q.rates = p.rates + off;
    if (p.x0_ld != 0) q.x0 = p.x0 + off;
    q.out = p.out + off;
    q.stats = p.stats + 4 * off;
    hipLaunchKernelGGL(ros_wave_kernel, dim3((unsigned)q.n_traj), dim3(kRosWG), lds, stream, q);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rn
