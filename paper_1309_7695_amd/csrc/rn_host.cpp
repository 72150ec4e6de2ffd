// rn_host.cpp -- C ABI of the sweep library: argument validation, network
// preprocessing into packed device tables, and kernel launch selection.
//
// Preprocessing follows the method's needs (CGP 2006): rate laws of order <= 2,
// net stoichiometric changes nu_ij = products - reactants, the consumed-reactant
// lists that define critical reactions, and for every reactant species the
// highest reaction order and homodimer flag that fix its g_i factor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rn.h"
#include "rn_jit.h"
#include "rn_kernel.h"
#include "rn_plan.h"

struct rn_network {
  int32_t N = 0, M = 0;
  int device = 0;
  void* dbuf = nullptr;
  size_t bytes = 0;
  rn::DevNet dev{};
  std::string jit_consts;  // compile-time prelude of the network-compiled kernel, or empty
  int32_t nnz = 0;         // nonzero net changes (entries of the compact stoichiometry)
  // The device tables are filled by the first launch that uses them, on that
  // launch's stream, from a pinned copy of the table image (see stage_network).
  void* himg = nullptr;
  hipEvent_t staged = nullptr;  // recorded after the copy
  mutable std::mutex mu;
  mutable int stage = 0;        // 0 not copied, 1 copy enqueued, 2 copy complete
  mutable hipStream_t stage_stream = nullptr;
};

namespace {

thread_local int g_last_hip = 0;

int device_error(hipError_t e) {
  g_last_hip = (int)e;
  return RN_E_DEVICE;
}

constexpr int32_t kMaxCoeff = 1 << 20;

// A library stream of the current device (one per device, created on first
// use and kept for the process).
hipError_t library_stream(int dev, hipStream_t* out) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  std::lock_guard<std::mutex> lock(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipStream_t st = nullptr;
  const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  streams.emplace(dev, st);
  *out = st;
  return hipSuccess;
}

// Wave scheduling knob (fraction of lanes that must wait before the leap-side
// phases run).  RN_SCHED_THETA overrides it for tuning; results never depend on it.
float sched_theta() {
  static const float theta = [] {
    const char* s = std::getenv("RN_SCHED_THETA");
    if (!s) return 0.5f;
    const float v = std::strtof(s, nullptr);
    return (v >= 0.0f && v <= 1.0f) ? v : 0.5f;
  }();
  return theta;
}

// Host image of the tables before upload.
struct HostTables {
  std::vector<rn::RateLaw> law;
  std::vector<int32_t> nu_ptr, cons_ptr, col_ptr;
  std::vector<int2> nu_ent, cons_ent, rs_ent, col_ent;
  std::vector<uint32_t> nu_abs;
  std::vector<rn::TauSpecies> rs;
  std::vector<double> log_fact;
  std::vector<int32_t> nu_dense;  // [M][jit_dense_ld(N)] for network-compiled kernels
  int32_t crit_words = 0;
};

// Number of reactions the kernels see: networks held in register rate vectors
// are padded with null reactions to a multiple of 16.
int32_t padded_reactions(int32_t M) {
  return M <= 16 * rn::kMaxRateSegs ? (M + 15) / 16 * 16 : M;
}

int build_tables(const rn_network_desc* d, HostTables& T) {
  const int32_t N = d->n_species, M = d->n_reactions;
  const int32_t Mp = padded_reactions(M);
  if (!d->react_ptr || !d->prod_ptr) return RN_E_INVALID_ARG;
  if (d->react_ptr[0] != 0 || d->prod_ptr[0] != 0) return RN_E_INVALID_ARG;
  for (int32_t j = 0; j < M; ++j)
    if (d->react_ptr[j + 1] < d->react_ptr[j] || d->prod_ptr[j + 1] < d->prod_ptr[j])
      return RN_E_INVALID_ARG;
  if ((d->react_ptr[M] > 0 && (!d->react_species || !d->react_coeff)) ||
      (d->prod_ptr[M] > 0 && (!d->prod_species || !d->prod_coeff)))
    return RN_E_INVALID_ARG;

  std::vector<int32_t> hor(N, 0), dimer(N, 0);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> nu(M);  // per reaction (species, nu)
  T.law.assign(Mp, rn::RateLaw{N, N, 0, 0});
  T.nu_abs.assign(Mp, 0u);
  for (int32_t j = 0; j < M; ++j) {
    std::map<int32_t, int64_t> r, net;
    int64_t order = 0;
    for (int32_t e = d->react_ptr[j]; e < d->react_ptr[j + 1]; ++e) {
      const int32_t s = d->react_species[e], c = d->react_coeff[e];
      if (s < 0 || s >= N || c < 1 || c > kMaxCoeff) return RN_E_INVALID_NETWORK;
      r[s] += c;
      order += c;
    }
    for (int32_t e = d->prod_ptr[j]; e < d->prod_ptr[j + 1]; ++e) {
      const int32_t s = d->prod_species[e], c = d->prod_coeff[e];
      if (s < 0 || s >= N || c < 1 || c > kMaxCoeff) return RN_E_INVALID_NETWORK;
      net[s] += c;
    }
    if (order > 2) return RN_E_UNSUPPORTED;
    for (auto& kv : r) net[kv.first] -= kv.second;
    rn::RateLaw L{N, N, 0, 0};
    if (order == 1) {
      L.ia = r.begin()->first;
    } else if (order == 2) {
      if (r.size() == 2) {
        L.ia = r.begin()->first;
        L.ib = std::next(r.begin())->first;
      } else {
        L.ia = L.ib = r.begin()->first;
        L.db = -1;
        L.dimer = 1;
      }
    }
    T.law[j] = L;
    for (auto& kv : r) {
      hor[kv.first] = std::max<int32_t>(hor[kv.first], (int32_t)order);
      if (kv.second == 2) dimer[kv.first] = 1;
    }
    int64_t sum_abs = 0;
    for (auto& kv : net) {
      if (kv.second == 0) continue;
      if (kv.second > INT32_MAX || kv.second < -INT32_MAX) return RN_E_INVALID_NETWORK;
      nu[j].push_back({kv.first, (int32_t)kv.second});
      sum_abs += kv.second < 0 ? -kv.second : kv.second;
    }
    if (sum_abs > INT32_MAX) return RN_E_INVALID_NETWORK;
    T.nu_abs[j] = (uint32_t)sum_abs;
  }

  T.nu_ptr.assign(1, 0);
  T.cons_ptr.assign(1, 0);
  std::vector<std::vector<int2>> col(N);
  for (int32_t j = 0; j < M; ++j) {
    for (auto& sv : nu[j]) {
      T.nu_ent.push_back(make_int2(sv.first, sv.second));
      if (sv.second < 0) T.cons_ent.push_back(make_int2(sv.first, -sv.second));
      col[sv.first].push_back(make_int2(j, sv.second));  // ascending j
    }
    T.nu_ptr.push_back((int32_t)T.nu_ent.size());
    T.cons_ptr.push_back((int32_t)T.cons_ent.size());
  }
  for (int32_t j = M; j < Mp; ++j) {  // null reactions
    T.nu_ptr.push_back((int32_t)T.nu_ent.size());
    T.cons_ptr.push_back((int32_t)T.cons_ent.size());
  }
  T.col_ptr.assign(1, 0);
  for (int32_t i = 0; i < N; ++i) {
    for (auto& e : col[i]) T.col_ent.push_back(e);
    T.col_ptr.push_back((int32_t)T.col_ent.size());
  }
  for (int32_t i = 0; i < N; ++i) {
    if (hor[i] == 0) continue;
    rn::TauSpecies ts;
    ts.species = i;
    ts.gkind = hor[i] == 1 ? 1 : (dimer[i] ? 3 : 2);
    ts.begin = (int32_t)T.rs_ent.size();
    for (auto& e : col[i]) T.rs_ent.push_back(e);
    ts.end = (int32_t)T.rs_ent.size();
    T.rs.push_back(ts);
  }
  T.crit_words = (Mp + 31) / 32;
  if (N <= rn::kJitMaxSpecies && M <= rn::kJitMaxReactions) {
    const int ld = rn::jit_dense_ld(N);
    T.nu_dense.assign((size_t)M * ld, 0);
    for (int32_t j = 0; j < M; ++j)
      for (auto& sv : nu[j]) T.nu_dense[(size_t)j * ld + sv.first] = sv.second;
  }
  T.log_fact.resize(rn::kLogFactTable);
  for (int k = 0; k < rn::kLogFactTable; ++k) T.log_fact[k] = std::lgamma((double)k + 1.0);
  return RN_OK;
}

// The network as compile-time constants for rn_net_kernel.h (namespace rnnet).
std::string jit_constants(const HostTables& T, int32_t N, int32_t M) {
  std::string s = "namespace rnnet {\n";
  auto num = [](long long v) { return std::to_string(v); };
  s += "constexpr int N = " + num(N) + ";\nconstexpr int M = " + num(M) + ";\n";
  s += "constexpr int DLD = " + num(rn::jit_dense_ld(N)) + ";\n";
  auto list1 = [&](const char* type, const char* name, const std::vector<long long>& v) {
    s += std::string("constexpr ") + type + " " + name + "[] = {";
    if (v.empty()) s += "0";
    for (size_t k = 0; k < v.size(); ++k) s += (k ? "," : "") + num(v[k]);
    s += "};\n";
  };
  auto list2 = [&](const char* name, const std::vector<int2>& v, size_t n) {
    s += std::string("constexpr int ") + name + "[][2] = {";
    if (n == 0) s += "{0,0}";
    for (size_t k = 0; k < n; ++k) s += (k ? ",{" : "{") + num(v[k].x) + "," + num(v[k].y) + "}";
    s += "};\n";
  };
  s += "constexpr int LAW[][4] = {";
  for (int32_t j = 0; j < M; ++j) {
    const rn::RateLaw& L = T.law[j];
    s += (j ? ",{" : "{") + num(L.ia) + "," + num(L.ib) + "," + num(L.db) + "," + num(L.dimer) + "}";
  }
  s += "};\n";
  std::vector<long long> v;
  v.assign(T.nu_ptr.begin(), T.nu_ptr.begin() + M + 1);
  list1("int", "NU_PTR", v);
  list2("NU_ENT", T.nu_ent, (size_t)T.nu_ptr[M]);
  v.assign(T.nu_abs.begin(), T.nu_abs.begin() + M);
  list1("unsigned", "NU_ABS", v);
  v.assign(T.cons_ptr.begin(), T.cons_ptr.begin() + M + 1);
  list1("int", "CONS_PTR", v);
  list2("CONS_ENT", T.cons_ent, (size_t)T.cons_ptr[M]);
  s += "constexpr int NRS = " + num((long long)T.rs.size()) + ";\n";
  s += "constexpr int RS[][4] = {";
  if (T.rs.empty()) s += "{0,0,0,0}";
  for (size_t r = 0; r < T.rs.size(); ++r) {
    const rn::TauSpecies& ts = T.rs[r];
    s += (r ? ",{" : "{") + num(ts.species) + "," + num(ts.gkind) + "," + num(ts.begin) + "," +
         num(ts.end) + "}";
  }
  s += "};\n";
  list2("RS_ENT", T.rs_ent, T.rs_ent.size());
  v.assign(T.col_ptr.begin(), T.col_ptr.end());
  list1("int", "COL_PTR", v);
  list2("COL_ENT", T.col_ent, T.col_ent.size());
  s += "}  // namespace rnnet\n";
  return s;
}

// Appends a host array to a packed image, 16-byte aligned; returns its offset.
template <class V>
size_t pack(std::vector<unsigned char>& img, const V& v) {
  size_t off = (img.size() + 15) & ~(size_t)15;
  const size_t nb = v.size() * sizeof(typename V::value_type);
  img.resize(off + std::max<size_t>(nb, 16), 0);
  if (nb) std::memcpy(img.data() + off, v.data(), nb);
  return off;
}

}  // namespace

extern "C" {

const char* rn_strerror(int code) {
  switch (code) {
    case RN_OK: return "ok";
    case RN_E_INVALID_ARG: return "invalid argument";
    case RN_E_INVALID_NETWORK: return "invalid network description";
    case RN_E_UNSUPPORTED: return "unsupported network (reaction order above 2, or too large)";
    case RN_E_NOMEM: return "out of memory";
    case RN_E_DEVICE: return "HIP device error";
    case RN_E_SCRATCH: return "input too large for the fixed scratch of an allocation-free call";
    default: return "unknown error";
  }
}

int rn_last_device_error(void) { return g_last_hip; }

int rn_sample_times(double t_end, int32_t n_points, double* out) {
  if (!out || n_points < 1 || !std::isfinite(t_end) || t_end < 0.0) return RN_E_INVALID_ARG;
  if (n_points == 1) {
    out[0] = t_end;
    return RN_OK;
  }
  const double den = (double)(n_points - 1);
  for (int32_t s = 0; s < n_points - 1; ++s) out[s] = ((double)s * t_end) / den;
  out[n_points - 1] = t_end;
  return RN_OK;
}

void rn_sweep_args_init(rn_sweep_args* a) {
  if (!a) return;
  std::memset(a, 0, sizeof(*a));
  a->eps = 0.03;
  a->n_c = 10;
  a->ssa_factor = 10.0;
  a->ssa_burst = 100;
  a->max_steps = 100000000ull;
  a->method = RN_METHOD_TAULEAP;
  a->precision = RN_FP64;
}

int32_t rn_network_species(const rn_network* net) { return net ? net->N : -1; }
int32_t rn_network_reactions(const rn_network* net) { return net ? net->M : -1; }

int rn_load_network(const rn_network_desc* desc, rn_network** out) {
  if (!desc || !out) return RN_E_INVALID_ARG;
  if (desc->n_species <= 0 || desc->n_reactions <= 0) return RN_E_INVALID_ARG;
  if (desc->n_species > (1 << 20) || desc->n_reactions > (1 << 20)) return RN_E_UNSUPPORTED;
  HostTables T;
  int rc;
  try {
    rc = build_tables(desc, T);
  } catch (const std::bad_alloc&) {
    return RN_E_NOMEM;
  }
  if (rc != RN_OK) return rc;

  std::vector<unsigned char> img;
  const size_t o_law = pack(img, T.law), o_nu_ptr = pack(img, T.nu_ptr),
               o_nu_ent = pack(img, T.nu_ent), o_cons_ptr = pack(img, T.cons_ptr),
               o_cons_ent = pack(img, T.cons_ent), o_nu_abs = pack(img, T.nu_abs),
               o_rs = pack(img, T.rs), o_rs_ent = pack(img, T.rs_ent),
               o_col_ptr = pack(img, T.col_ptr), o_col_ent = pack(img, T.col_ent),
               o_log_fact = pack(img, T.log_fact), o_nu_dense = pack(img, T.nu_dense);

  rn_network* net = new (std::nothrow) rn_network;
  if (!net) return RN_E_NOMEM;
  net->N = desc->n_species;
  net->M = desc->n_reactions;
  hipError_t e = hipGetDevice(&net->device);
  if (e != hipSuccess) { delete net; return device_error(e); }
  // No copy here: a copy on any stream of its own can wait behind sweeps
  // already running on the device; the first launch that uses the network
  // copies the tables on its own stream instead.
  e = hipMalloc(&net->dbuf, img.size());
  if (e == hipSuccess) e = hipHostMalloc(&net->himg, img.size(), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&net->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    rn_free_network(net);
    return e == hipErrorOutOfMemory ? RN_E_NOMEM : device_error(e);
  }
  std::memcpy(net->himg, img.data(), img.size());
  net->bytes = img.size();
  unsigned char* b = (unsigned char*)net->dbuf;
  rn::DevNet& D = net->dev;
  D.N = net->N;
  D.M = padded_reactions(net->M);
  D.M_real = net->M;
  D.n_rs = (int32_t)T.rs.size();
  D.crit_words = T.crit_words;
  D.law = (const rn::RateLaw*)(b + o_law);
  D.nu_ptr = (const int32_t*)(b + o_nu_ptr);
  D.nu_ent = (const int2*)(b + o_nu_ent);
  D.cons_ptr = (const int32_t*)(b + o_cons_ptr);
  D.cons_ent = (const int2*)(b + o_cons_ent);
  D.nu_abs = (const uint32_t*)(b + o_nu_abs);
  D.rs = (const rn::TauSpecies*)(b + o_rs);
  D.rs_ent = (const int2*)(b + o_rs_ent);
  D.col_ptr = (const int32_t*)(b + o_col_ptr);
  D.col_ent = (const int2*)(b + o_col_ent);
  D.log_fact = (const double*)(b + o_log_fact);
  D.nu_dense = T.nu_dense.empty() ? nullptr : (const int32_t*)(b + o_nu_dense);
  net->nnz = T.nu_ptr[net->M];
  if (!T.nu_dense.empty()) {
    try {
      net->jit_consts = jit_constants(T, net->N, net->M);
    } catch (const std::bad_alloc&) {
      net->jit_consts.clear();
    }
  }
  *out = net;
  return RN_OK;
}

void rn_free_network(rn_network* net) {
  if (!net) return;
  if (net->dbuf) (void)hipFree(net->dbuf);
  if (net->himg) (void)hipHostFree(net->himg);
  if (net->staged) (void)hipEventDestroy(net->staged);
  delete net;
}

}  // extern "C"

// The network-compiled kernel for this handle, precision and workgroup size
// (compiled on first use), or null when the generic kernels run.
// wait = false: use it only if already compiled (else start compiling it in the
// background and run the generic kernel this time).
static hipFunction_t network_kernel(const rn_network* net, int32_t precision, int wg,
                                    bool wait = true, bool ssa_dep = false) {
  if (net->jit_consts.empty() || !rn::jit_enabled()) return nullptr;
  const int prec = (precision == RN_FP32 ? rn::kJitFP32 : rn::kJitFP64) |
                   (ssa_dep ? rn::kJitSsaDep : 0);
  return wait ? rn::jit_kernel(net->jit_consts, prec, wg)
              : rn::jit_kernel_nowait(net->jit_consts, prec, wg);
}

namespace rn {
// rn_hybrid.hip: the rate-equation sweep on the wave-per-trajectory kernel;
// false (nothing launched) when the network does not fit it.
bool launch_ode_wave(const HybridParams& p, hipStream_t stream, hipError_t* err);
bool ode_wave_fits(int n_species, int m_real);
}  // namespace rn

namespace rn_internal {

// Make the network's device tables valid for work enqueued next on `stream`.
// The first launch copies them on its own stream (ordered before its kernel)
// and records an event; a launch on another stream while that copy may still
// run waits for the event; once it has completed, nothing is enqueued.  Under
// stream capture the copy becomes part of the graph (replays rewrite the same
// bytes) and the handle stays unstaged for launches outside the graph.
hipError_t stage_network(const rn_network* net, hipStream_t stream) {
  std::lock_guard<std::mutex> lock(net->mu);
  if (net->stage == 2) return hipSuccess;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(stream, &cs);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusNone) {
    if (net->stage == 1) {
      // the copy was enqueued outside the graph: wait for it before capturing
      e = hipEventSynchronize(net->staged);
      if (e == hipSuccess) net->stage = 2;
      return e;
    }
    return hipMemcpyAsync(net->dbuf, net->himg, net->bytes, hipMemcpyHostToDevice, stream);
  }
  if (net->stage == 0) {
    e = hipMemcpyAsync(net->dbuf, net->himg, net->bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(net->staged, stream);
    if (e != hipSuccess) return e;
    net->stage = 1;
    net->stage_stream = stream;
    return hipSuccess;
  }
  e = hipEventQuery(net->staged);
  if (e == hipSuccess) {
    net->stage = 2;
    return hipSuccess;
  }
  if (e != hipErrorNotReady) return e;
  return stream == net->stage_stream ? hipSuccess : hipStreamWaitEvent(stream, net->staged, 0);
}

// Stage the network now on the library stream and wait for the copy.
hipError_t stage_network_now(const rn_network* net) {
  hipStream_t st = nullptr;
  hipError_t e = library_stream(net->device, &st);
  if (e == hipSuccess) e = stage_network(net, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lock(net->mu);
    if (net->stage == 1 && hipEventQuery(net->staged) == hipSuccess) net->stage = 2;
  }
  return e;
}

// The one-wave-per-trajectory kernel: RN_WSWEEP=0 never, =1 whenever the
// network fits it.  By default (measured on MI355X):
//  * networks too large for a compiled kernel: always (1.3-3x faster than one
//    lane per trajectory on 170-450 reactions, from 300 to 64k trajectories);
//  * networks with a compiled kernel: sweeps of at most kWsweepAutoTrajJit
//    trajectories per CU (the wave form wins there for 50-120 reactions); at
//    most kWsweepAutoTraj while the compiled kernel is not available yet.
constexpr int64_t kWsweepAutoTraj = 64, kWsweepAutoTrajJit = 16;
enum : int { kNoJit = 0, kJitReady = 1, kJitPending = 2 };

bool use_wsweep(const rn_network* net, int64_t n_traj, int n_cu, int jit) {
  if (!rn::wsweep_fits(net->N, net->dev.M_real)) return false;
  const char* e = std::getenv("RN_WSWEEP");
  if (e && e[0] == '0') return false;
  if (e && e[0] == '1') return true;
  if (jit == kNoJit) return true;
  return n_traj <= (jit == kJitReady ? kWsweepAutoTrajJit : kWsweepAutoTraj) * n_cu;
}

// Whether the network has (or can compile) a network-compiled kernel.
bool has_network_kernel(const rn_network* net) {
  return !net->jit_consts.empty() && rn::jit_enabled();
}

int plan_sweep(const rn_network* net, const rn_sweep_args* a, SweepPlan& plan,
               bool wait_compile) {
  if (!net || !a) return RN_E_INVALID_ARG;
  if (a->n_traj < 0 || a->traj_offset < 0 || a->traj_offset + a->n_traj > (int64_t)1 << 32)
    return RN_E_INVALID_ARG;
  if (a->n_times < 1) return RN_E_INVALID_ARG;
  if (!(a->eps > 0.0) || !std::isfinite(a->eps)) return RN_E_INVALID_ARG;
  if (a->n_c < 0 || a->n_c > (1 << 20)) return RN_E_INVALID_ARG;
  if (!(a->ssa_factor >= 0.0)) return RN_E_INVALID_ARG;
  if (a->ssa_burst < 1 || a->max_steps < 1) return RN_E_INVALID_ARG;
  if (a->method != RN_METHOD_TAULEAP && a->method != RN_METHOD_SSA) return RN_E_INVALID_ARG;
  if (a->precision != RN_FP64 && a->precision != RN_FP32) return RN_E_INVALID_ARG;
  if (!(a->cle_threshold == 0.0 || (a->cle_threshold >= 10.0 && a->cle_threshold <= 1e300)))
    return RN_E_INVALID_ARG;
  plan = SweepPlan{};
  plan.precision = a->precision;
  if (a->n_traj == 0) {
    plan.empty = true;
    return RN_OK;
  }
  // fused statistics: sums given together; a histogram needs its bins
  if ((a->sum_x == nullptr) != (a->sum_x2 == nullptr)) return RN_E_INVALID_ARG;
  if (a->hist && (!a->hist_lo || !a->hist_width || a->hist_bins < 1 ||
                  (int64_t)a->n_times * net->N * a->hist_bins >= ((int64_t)1 << 31)))
    return RN_E_INVALID_ARG;
  if (!a->rates || !a->x0 || !a->times || !a->stats) return RN_E_INVALID_ARG;
  if (!a->out && !a->sum_x && !a->hist) return RN_E_INVALID_ARG;
  if (a->out_layout != RN_OUT_SAMPLE_MAJOR && a->out_layout != RN_OUT_TRAJ_MAJOR)
    return RN_E_INVALID_ARG;
  const int64_t out_min = a->out_layout == RN_OUT_TRAJ_MAJOR ? (int64_t)a->n_times * net->N
                                                             : a->n_traj;
  if (a->rates_ld < a->n_traj || (a->out && a->out_ld < out_min)) return RN_E_INVALID_ARG;
  if (a->x0_ld != 0 && a->x0_ld < a->n_traj) return RN_E_INVALID_ARG;

  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e);
  if (dev != net->device) return RN_E_INVALID_ARG;
  int max_lds = 0, n_cu = 0;
  e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return device_error(e);
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return device_error(e);

  const size_t per_lane =
      rn::lds_words_per_lane(net->N, padded_reactions(net->M)) * sizeof(int32_t);
  rn::LaunchCfg& cfg = plan.cfg;
  cfg.rate_segs = net->M <= 16 * rn::kMaxRateSegs ? padded_reactions(net->M) / 16 : 0;
  // 256 lanes per workgroup (one wave per SIMD of a CU) when the sweep fills the
  // chip; otherwise single-wave workgroups spread over more CUs.
  if (a->n_traj >= (int64_t)256 * n_cu && per_lane * 256 <= (size_t)max_lds) cfg.wg = 256;
  else cfg.wg = 64;
  cfg.lds_bytes = per_lane * cfg.wg;
  if (cfg.lds_bytes > (size_t)max_lds) return RN_E_UNSUPPORTED;
  plan.lane_lds = per_lane;
  plan.max_segs = cfg.rate_segs;
  plan.n_species = net->N;
  plan.n_reactions = net->M;
  plan.n_simd = 4 * n_cu;
  plan.nnz = net->nnz;

  plan.net = net;
  rn::SweepParams& p = plan.p;
  p.net = net->dev;
  p.rates = a->rates;
  p.rates_ld = a->rates_ld;
  p.x0 = a->x0;
  p.x0_ld = a->x0_ld;
  p.times = a->times;
  p.n_times = a->n_times;
  p.out = a->out;
  p.out_ld = a->out_ld;
  p.stats = a->stats;
  p.n_traj = a->n_traj;
  p.traj_offset = (uint32_t)a->traj_offset;
  p.key0 = (uint32_t)a->seed;
  p.key1 = (uint32_t)(a->seed >> 32);
  p.eps = a->eps;
  p.n_c = a->n_c;
  p.ssa_factor = a->ssa_factor;
  p.ssa_burst = a->ssa_burst;
  p.max_steps = a->max_steps;
  p.method = a->method;
  p.cle_threshold = a->cle_threshold;
  p.theta = sched_theta();
  p.phase_cycles = a->phase_cycles;
  p.sum_x = a->sum_x;
  p.sum_x2 = a->sum_x2;
  p.hist = a->hist;
  p.hist_lo = a->hist_lo;
  p.hist_width = a->hist_width;
  p.hist_bins = a->hist ? a->hist_bins : 0;
  p.out_traj_major = a->out_layout == RN_OUT_TRAJ_MAJOR ? 1 : 0;
  plan.wg = a->n_traj >= (int64_t)256 * n_cu ? 256 : 64;
  // exact SSA: the dependency-graph kernel only when the environment sets
  // RN_SSA_KERNEL=dep (and its propensities fit the registers); the general
  // kernel measured faster (a wave recomputes nearly every reaction anyway)
  const bool fp32 = a->precision == RN_FP32;
  const char* sk = std::getenv("RN_SSA_KERNEL");
  const bool ssa_dep = a->method == RN_METHOD_SSA && sk && std::strcmp(sk, "dep") == 0 &&
                       net->M * (fp32 ? 1 : 2) <= rn::kJitSsaDepMaxWords;
  plan.wave = !ssa_dep &&
              use_wsweep(net, a->n_traj, n_cu, has_network_kernel(net) ? kJitReady : kNoJit);
  if (!plan.wave) plan.fn = network_kernel(net, a->precision, plan.wg, wait_compile, ssa_dep);
  if (plan.fn) {
    plan.lds = ssa_dep ? rn::jit_ssa_lds_bytes(net->N, net->M, net->nnz, plan.wg, fp32)
                       : rn::jit_lds_bytes(net->N, net->M, plan.wg, fp32);
    if (plan.lds > (size_t)max_lds) plan.fn = nullptr;
  }
  plan.ssa_dep = plan.fn && ssa_dep;
  // a network whose compiled kernel is missing (compile failed or still in
  // flight) takes the generic kernels' rule
  if (!plan.fn && !plan.wave && !ssa_dep)
    plan.wave = use_wsweep(net, a->n_traj, n_cu, has_network_kernel(net) ? kJitPending : kNoJit);
  return RN_OK;
}

// The sweep parameters of trajectories [off, off + n) of a plan: pointers and
// the trajectory offset moved to the range's first trajectory.
static rn::SweepParams sub_range(const rn::SweepParams& p, int64_t off, int64_t n) {
  rn::SweepParams q = p;
  q.n_traj = n;
  q.traj_offset = p.traj_offset + (uint32_t)off;
  q.rates = p.rates + off;
  if (p.x0_ld != 0) q.x0 = p.x0 + off;
  if (p.out) q.out = p.out + (p.out_traj_major ? off * p.out_ld : off);
  q.stats = p.stats + 4 * off;
  if (p.phase_cycles) q.phase_cycles = p.phase_cycles + 4 * (off / 64);
  return q;  // the fused statistics add up over the ranges
}

// At most 2^24 trajectories per dispatch (a dispatch holds fewer than 2^32
// work-items); a larger sweep is enqueued as consecutive ranges, which the
// global trajectory ids make identical to one launch.
constexpr int64_t kLaunchChunk = (int64_t)1 << 24;

hipError_t launch_plan(const SweepPlan& plan, hipStream_t stream) {
  if (plan.empty) return hipSuccess;
  const bool stats = plan.p.sum_x || plan.p.hist;
  hipError_t e = stage_network(plan.net, stream);
  if (e == hipSuccess && stats) e = rn::launch_stats_zero(plan.p, stream);
  for (int64_t off = 0; e == hipSuccess && off < plan.p.n_traj; off += kLaunchChunk) {
    const rn::SweepParams q =
        sub_range(plan.p, off, std::min(kLaunchChunk, plan.p.n_traj - off));
    if (plan.fn) e = rn::jit_launch(plan.fn, q, plan.wg, plan.lds, stream);
    else if (plan.wave) e = rn::launch_wsweep(q, plan.precision == RN_FP32, plan.n_simd, stream);
    else if (plan.precision == RN_FP32) e = rn::launch_sweep_f32(q, plan.cfg, stream);
    else e = rn::launch_sweep_f64(q, plan.cfg, stream);
  }
  if (e == hipSuccess && stats) e = rn::launch_stats_finish(plan.p, stream);
  return e;
}

int device_status(hipError_t e) { return e == hipSuccess ? RN_OK : device_error(e); }

void prefetch_kernel(const rn_network* net, int32_t precision, int64_t n_traj) {
  int dev = -1, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != net->device) return;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return;
  // a sweep that runs one wave per trajectory even once the kernel exists
  // leaves the compile workers to jobs that need them
  if (use_wsweep(net, n_traj, n_cu, has_network_kernel(net) ? kJitReady : kNoJit)) return;
  (void)network_kernel(net, precision, n_traj >= (int64_t)256 * n_cu ? 256 : 64, false);
}

}  // namespace rn_internal

extern "C" {

int rn_sweep(const rn_network* net, const rn_sweep_args* a, void* hip_stream) {
  rn_internal::SweepPlan plan;
  const int rc = rn_internal::plan_sweep(net, a, plan);
  if (rc != RN_OK) return rc;
  return rn_internal::device_status(rn_internal::launch_plan(plan, (hipStream_t)hip_stream));
}

int rn_sweep_kernel_kind(const rn_network* net, int32_t precision, int64_t n_traj) {
  if (!net || n_traj < 0 || (precision != RN_FP64 && precision != RN_FP32))
    return RN_E_INVALID_ARG;
  int dev = -1, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e);
  if (dev != net->device) return RN_E_INVALID_ARG;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return device_error(e);
  const int jwg = n_traj >= (int64_t)256 * n_cu ? 256 : 64;
  const bool jit = rn_internal::has_network_kernel(net);
  if (rn_internal::use_wsweep(net, n_traj, n_cu,
                              jit ? rn_internal::kJitReady : rn_internal::kNoJit))
    return 2;
  if (network_kernel(net, precision, jwg)) return 1;
  return rn_internal::use_wsweep(net, n_traj, n_cu,
                                 jit ? rn_internal::kJitPending : rn_internal::kNoJit) ? 2 : 0;
}

void rn_compile_drain(void) { rn::jit_drain(); }

void rn_ode_args_init(rn_ode_args* a) {
  if (!a) return;
  std::memset(a, 0, sizeof(*a));
  a->rtol = 1e-6;
  a->atol = 1e-6;
  a->max_steps = 10000000ull;
}

int64_t rn_ode_work_doubles(const rn_network* net, int64_t n_traj) {
  if (!net || n_traj < 0) return -1;
  return (int64_t)rn::kOdeSlots * net->N * n_traj;
}

}  // extern "C"

namespace rn_internal {

// rn_ode_sweep and rn_ode_sweep_noalloc: validate, then run the wave kernel
// (networks of up to 64 species, no workspace) or the lane kernel on `work`
// (work == null: the library's fixed scratch, RN_E_SCRATCH if it is too small).
static int ode_enqueue(const rn_network* net, const rn_ode_args* a, double* work,
                       int64_t work_ld, hipStream_t stream) {
  if (!net || !a) return RN_E_INVALID_ARG;
  if (a->n_traj < 0 || a->n_traj > ((int64_t)1 << 32) || a->n_times < 1) return RN_E_INVALID_ARG;
  if (!(a->rtol > 0.0) || !std::isfinite(a->rtol) || !(a->atol > 0.0) || !std::isfinite(a->atol))
    return RN_E_INVALID_ARG;
  if (a->max_steps < 1) return RN_E_INVALID_ARG;
  if (a->method != RN_ODE_DOPRI5 && a->method != RN_ODE_ROS4) return RN_E_INVALID_ARG;
  if (a->method == RN_ODE_ROS4 && !rn::ros_fits(net->N, net->dev.M_real)) return RN_E_UNSUPPORTED;
  if (a->n_traj == 0) return RN_OK;
  if (!a->rates || !a->x0 || !a->times || !a->out || !a->stats) return RN_E_INVALID_ARG;
  if (a->rates_ld < a->n_traj || a->out_ld < a->n_traj) return RN_E_INVALID_ARG;
  if (work && work_ld < a->n_traj) return RN_E_INVALID_ARG;
  if (a->x0_ld != 0 && a->x0_ld < a->n_traj) return RN_E_INVALID_ARG;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e);
  if (dev != net->device) return RN_E_INVALID_ARG;
  const bool wave = a->method == RN_ODE_ROS4 || rn::ode_wave_fits(net->N, net->dev.M_real);
  if (!wave && !work && (int64_t)rn::kOdeSlots * net->N * a->n_traj > rn::kOdeScratchDoubles)
    return RN_E_SCRATCH;
  rn::OdeParams p{};
  p.net = net->dev;
  p.rates = a->rates;
  p.rates_ld = a->rates_ld;
  p.x0 = a->x0;
  p.x0_ld = a->x0_ld;
  p.times = a->times;
  p.n_times = a->n_times;
  p.out = a->out;
  p.out_ld = a->out_ld;
  p.stats = a->stats;
  p.work = work;
  p.work_ld = work_ld;
  p.n_traj = a->n_traj;
  p.rtol = a->rtol;
  p.atol = a->atol;
  p.max_steps = a->max_steps;
  e = stage_network(net, stream);
  if (e != hipSuccess) return device_error(e);
  if (a->method == RN_ODE_ROS4) {
    e = rn::launch_ros(p, stream);
    if (e != hipSuccess) return device_error(e);
    return RN_OK;
  }
  // networks of up to 64 species: one wave per trajectory, state in registers
  rn::HybridParams hp{};
  hp.net = p.net;
  hp.rates = p.rates;
  hp.rates_ld = p.rates_ld;
  hp.x0 = p.x0;
  hp.x0_ld = p.x0_ld;
  hp.times = p.times;
  hp.n_times = p.n_times;
  hp.out = p.out;
  hp.out_ld = p.out_ld;
  hp.stats = p.stats;
  hp.n_traj = p.n_traj;
  hp.rtol = p.rtol;
  hp.atol = p.atol;
  hp.max_steps = p.max_steps;
  if (rn::launch_ode_wave(hp, stream, &e)) {
    if (e != hipSuccess) return device_error(e);
    return RN_OK;
  }
  if (!p.work) {
    e = rn::ode_scratch(&p.work);
    if (e != hipSuccess) return device_error(e);
    p.work_ld = p.n_traj;
  }
  e = rn::launch_ode(p, stream);
  if (e != hipSuccess) return device_error(e);
  return RN_OK;
}

}  // namespace rn_internal

extern "C" {

int rn_ode_sweep(const rn_network* net, const rn_ode_args* a, void* hip_stream) {
  if (!a || (a->n_traj != 0 && !a->work)) return RN_E_INVALID_ARG;
  return rn_internal::ode_enqueue(net, a, a->work, a->work_ld, (hipStream_t)hip_stream);
}

int rn_ode_sweep_noalloc(const rn_network* net, const rn_ode_args* a, void* hip_stream) {
  return rn_internal::ode_enqueue(net, a, nullptr, 0, (hipStream_t)hip_stream);
}

int64_t rn_ode_noalloc_max_traj(const rn_network* net) {
  if (!net) return -1;
  if (rn::ode_wave_fits(net->N, net->dev.M_real)) return (int64_t)1 << 32;
  return rn::kOdeScratchDoubles / ((int64_t)rn::kOdeSlots * net->N);
}

void rn_hybrid_args_init(rn_hybrid_args* a) {
  if (!a) return;
  std::memset(a, 0, sizeof(*a));
  a->rtol = 1e-6;
  a->atol = 1e-6;
  a->max_steps = 10000000ull;
}

int64_t rn_hybrid_work_doubles(const rn_network* net, int64_t n_traj) {
  if (!net || n_traj < 0) return -1;
  return (int64_t)rn::kHybridSlots * net->N * n_traj;
}

int rn_hybrid_sweep(const rn_network* net, const rn_hybrid_args* a, void* hip_stream) {
  if (!net || !a) return RN_E_INVALID_ARG;
  if (a->n_traj < 0 || a->traj_offset < 0 || a->n_times < 1) return RN_E_INVALID_ARG;
  if (a->traj_offset + a->n_traj > ((int64_t)1 << 32)) return RN_E_INVALID_ARG;
  if (!(a->rtol > 0.0) || !std::isfinite(a->rtol) || !(a->atol > 0.0) || !std::isfinite(a->atol))
    return RN_E_INVALID_ARG;
  if (a->max_steps < 1) return RN_E_INVALID_ARG;
  if (a->n_traj == 0) return RN_OK;
  if (!a->continuous || !a->rates || !a->x0 || !a->times || !a->out || !a->stats || !a->work)
    return RN_E_INVALID_ARG;
  if (a->rates_ld < a->n_traj || a->out_ld < a->n_traj || a->work_ld < a->n_traj)
    return RN_E_INVALID_ARG;
  if (a->x0_ld != 0 && a->x0_ld < a->n_traj) return RN_E_INVALID_ARG;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e);
  if (dev != net->device) return RN_E_INVALID_ARG;
  rn::HybridParams p{};
  p.net = net->dev;
  p.cont = a->continuous;
  p.rates = a->rates;
  p.rates_ld = a->rates_ld;
  p.x0 = a->x0;
  p.x0_ld = a->x0_ld;
  p.times = a->times;
  p.n_times = a->n_times;
  p.out = a->out;
  p.out_ld = a->out_ld;
  p.stats = a->stats;
  p.work = a->work;
  p.work_ld = a->work_ld;
  p.n_traj = a->n_traj;
  p.traj_offset = (uint32_t)a->traj_offset;
  p.key0 = (uint32_t)a->seed;
  p.key1 = (uint32_t)(a->seed >> 32);
  p.rtol = a->rtol;
  p.atol = a->atol;
  p.max_steps = a->max_steps;
  e = rn_internal::stage_network(net, (hipStream_t)hip_stream);
  if (e == hipSuccess) e = rn::launch_hybrid(p, (hipStream_t)hip_stream);
  if (e != hipSuccess) return device_error(e);
  return RN_OK;
}

int rn_moments(const int32_t* out, int64_t out_ld, int32_t n_times, int32_t n_species,
               int64_t n_traj, int64_t* sum_x, uint64_t* sum_x2, void* hip_stream) {
  if (!out || !sum_x || !sum_x2) return RN_E_INVALID_ARG;
  if (n_times < 1 || n_species < 1 || n_traj < 1 || out_ld < n_traj) return RN_E_INVALID_ARG;
  const int64_t rows = (int64_t)n_times * n_species;
  if (rows >= ((int64_t)1 << 31)) return RN_E_INVALID_ARG;
  const hipError_t e =
      rn::launch_moments(out, out_ld, rows, n_traj, sum_x, sum_x2, (hipStream_t)hip_stream);
  if (e != hipSuccess) return device_error(e);
  return RN_OK;
}

}  // extern "C"
