// rn_ode.hip -- deterministic counterpart of the sweep: the reaction-rate
// equations dy/dt = sum_j nu_j c_j h_j(y), h_j = 1, y_a, y_a*y_b or y_a^2/2
// (paper, Methods section: abundant species follow the mean-field equations,
// which agree with the stochastic model in the thermodynamic limit), one lane
// per parameterization, integrated by the Dormand-Prince 5(4) pair
// (J. Comput. Appl. Math. 6 (1980) 19) with an error-per-step controller and
// steps clipped to the sample times.
//
// Every lane runs the same stage sequence, so the only divergence is in the
// accept/reject decision.  The ten state vectors of a lane (y, the candidate,
// the stage argument and seven stage derivatives) live in a caller-provided
// workspace laid out trajectory-minor, work[(v * N + i) * work_ld + t], so a
// wave touches 64 consecutive doubles per access; the pass is bound by those
// reads and writes.  Tables are read at wave-uniform indices through the
// scalar cache.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "rn_dopri.h"
#include "rn_kernel.h"

namespace rn {
namespace {

typedef const int32_t __attribute__((address_space(4)))* const_i32_ptr;
__device__ __forceinline__ int32_t cword(const void* base, int64_t i) {
  return ((const_i32_ptr)base)[i];
}

using namespace dopri;

constexpr uint32_t kStMaxSteps = 2u;
constexpr int kOdeWG = 128;

// Workspace slots.
enum : int { kY0 = 0, kY1 = 1, kK1 = 2, kK2 = 3, kK3 = 4, kK4 = 5, kK5 = 6, kK6 = 7, kK7 = 8, kYS = 9 };

__global__ __launch_bounds__(kOdeWG) void ode_kernel(const OdeParams p) {
  const DevNet& g = p.net;
  const int N = g.N;
  const int64_t tl = (int64_t)blockIdx.x * kOdeWG + threadIdx.x;
  if (tl >= p.n_traj) return;  // lanes are independent: no barrier follows
  const int64_t ld = p.work_ld;
  double* const w = p.work + tl;
  auto V = [&](int slot, int i) -> double& { return w[((int64_t)slot * N + i) * ld]; };
  const double* const crate = p.rates + tl;
  const double* __restrict__ times = p.times;
  const int S = p.n_times;

  // f = dy/dt at slot `in`, into slot `outv`: species-major, each f_i summed
  // over its reactions in increasing j.
  auto rhs = [&](int in, int outv) {
    for (int i = 0; i < N; ++i) {
      double f = 0.0;
      const int e1 = cword(g.col_ptr, i + 1);
      for (int e = cword(g.col_ptr, i); e < e1; ++e) {
        const int j = cword(g.col_ent, 2 * e);
        const int v = cword(g.col_ent, 2 * e + 1);
        const int32_t ia = cword(g.law, 4 * j), ib = cword(g.law, 4 * j + 1);
        const int32_t dimer = cword(g.law, 4 * j + 3);
        const double ya = ia < N ? V(in, ia) : 1.0;
        double h;
        if (dimer) h = 0.5 * (ya * ya);
        else h = ya * (ib < N ? V(in, ib) : 1.0);
        const double a = crate[(int64_t)j * p.rates_ld] * h;
        f = f + (double)v * a;
      }
      V(outv, i) = f;
    }
  };
  auto record = [&](int yslot, int si) {
    double* o = p.out + (int64_t)si * N * p.out_ld + tl;
    for (int i = 0; i < N; ++i) o[(int64_t)i * p.out_ld] = V(yslot, i);
  };

  int ys = kY0, yn = kY1, k1 = kK1, k7 = kK7;
  for (int i = 0; i < N; ++i)
    V(ys, i) = (double)(p.x0_ld ? p.x0[(int64_t)i * p.x0_ld + tl] : p.x0[i]);
  double t = 0.0;
  int s = 0;
  uint64_t acc = 0, rej = 0;
  uint32_t status = 0;
  while (s < S && times[s] <= t) record(ys, s++);
  rhs(ys, k1);
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
      status |= kStMaxSteps;
      break;
    }
    const double delta = times[s] - t;
    const bool clip = !(h < delta);
    const double hu = clip ? delta : h;
    for (int i = 0; i < N; ++i) V(kYS, i) = V(ys, i) + hu * (A21 * V(k1, i));
    rhs(kYS, kK2);
    for (int i = 0; i < N; ++i) V(kYS, i) = V(ys, i) + hu * (A31 * V(k1, i) + A32 * V(kK2, i));
    rhs(kYS, kK3);
    for (int i = 0; i < N; ++i)
      V(kYS, i) = V(ys, i) + hu * (A41 * V(k1, i) + A42 * V(kK2, i) + A43 * V(kK3, i));
    rhs(kYS, kK4);
    for (int i = 0; i < N; ++i)
      V(kYS, i) = V(ys, i) + hu * (A51 * V(k1, i) + A52 * V(kK2, i) + A53 * V(kK3, i) +
                                   A54 * V(kK4, i));
    rhs(kYS, kK5);
    for (int i = 0; i < N; ++i)
      V(kYS, i) = V(ys, i) + hu * (A61 * V(k1, i) + A62 * V(kK2, i) + A63 * V(kK3, i) +
                                   A64 * V(kK4, i) + A65 * V(kK5, i));
    rhs(kYS, kK6);
    for (int i = 0; i < N; ++i)
      V(yn, i) = V(ys, i) + hu * (B1 * V(k1, i) + B3 * V(kK3, i) + B4 * V(kK4, i) +
                                  B5 * V(kK5, i) + B6 * V(kK6, i));
    rhs(yn, k7);
    double e2 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double e = hu * (E1 * V(k1, i) + E3 * V(kK3, i) + E4 * V(kK4, i) + E5 * V(kK5, i) +
                             E6 * V(kK6, i) + E7 * V(k7, i));
      const double ay = fabs(V(ys, i)), an = fabs(V(yn, i));
      const double sc = p.atol + p.rtol * (ay > an ? ay : an);
      e2 = e2 + (e / sc) * (e / sc);
    }
    const double en = sqrt(e2 / N);
    if (en <= 1.0) {
      double fac = en == 0.0 ? 5.0 : 0.9 * pow(en, -0.2);
      if (fac > 5.0) fac = 5.0;
      if (fac < 0.2) fac = 0.2;
      if (last_rejected && fac > 1.0) fac = 1.0;
      int tmp = ys;
      ys = yn;
      yn = tmp;
      tmp = k1;
      k1 = k7;
      k7 = tmp;
      if (clip) t = times[s];
      else t = t + hu;
      h = hu * fac;
      acc = acc + 1;
      last_rejected = false;
      while (s < S && times[s] <= t) record(ys, s++);
    } else {
      double fac = 0.9 * pow(en, -0.2);
      if (fac < 0.2) fac = 0.2;
      h = hu * fac;
      rej = rej + 1;
      last_rejected = true;
    }
  }
  while (s < S) record(ys, s++);
  uint64_t* st = p.stats + tl * 4;
  st[0] = acc;
  st[1] = rej;
  st[2] = 0;
  st[3] = status;
}

}  // namespace

// The allocation-free form of the sweep keeps the lane kernel's workspace in
// this file-scope array (one copy per device, held until the process ends).
// Host code never passes the array's name to a kernel: it resolves the
// device address once per device with hipGetSymbolAddress and passes that.
__device__ __align__(256) double scratch[kOdeScratchDoubles];

hipError_t ode_scratch(double** ptr) {
  static std::mutex mu;
  static double* dev_ptr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!dev_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    dev_ptr[dev] = (double*)p;
  }
  *ptr = dev_ptr[dev];
  return hipSuccess;
}

// At most 2^24 trajectories per dispatch (a dispatch holds fewer than 2^32
// work-items); a larger sweep is enqueued as consecutive ranges.
hipError_t launch_ode(const OdeParams& p, hipStream_t stream) {
  constexpr int64_t kChunk = (int64_t)1 << 24;
  for (int64_t off = 0; off < p.n_traj; off += kChunk) {
    OdeParams q = p;
    q.n_traj = p.n_traj - off < kChunk ? p.n_traj - off : kChunk;
    q.rates = p.rates + off;
    if (p.x0_ld != 0) q.x0 = p.x0 + off;
    q.out = p.out + off;
    q.stats = p.stats + 4 * off;
    q.work = p.work + off;
    const int64_t blocks = (q.n_traj + kOdeWG - 1) / kOdeWG;
    hipLaunchKernelGGL(ode_kernel, dim3((unsigned)blocks), dim3(kOdeWG), 0, stream, q);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rn
