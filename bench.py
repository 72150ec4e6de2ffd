"""Throughput benchmark: trajectory-steps/s of one FP64 parameter sweep of the
50-species, 100-reaction synthetic network over 65,536 trajectories (t_end 50,
200 samples, eps 0.03, n_c 10), one MI355X.

A bench step is one complete sweep (``rn_sweep``: every trajectory from t = 0 to
t_end) with rates, initial counts and sample times already resident in HBM.
``value`` is the sweep's accepted leaps + SSA events divided by its wall time.

Prints one JSON line.  Also reports the dominant kernel's roofline position and
the CPU oracle's single-core rate on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trajectory-steps/sec at 65,536 sims (1 GPU); p50/p99 sweep-job latency"

# Peak VALU issue of an MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# full-rate VALU lane operation per lane per cycle (FP64 add/mul/FMA are full
# rate on CDNA4: 78.6 TFLOP/s counts an FMA as two flops).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "rn_net_sweep_synthetic_50x100_fp64_traffic.json")


def measured_traffic(kind, layout="traj"):
    """HBM bytes per launch of the FP64 sweep kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record (each counter scaled by what it
    reads for a copy of known size), or None when the record is for the other
    kernel kind or sample layout, or the kernel sources changed since the
    counters were taken."""
    import hashlib

    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    if rec.get("kind") != kind or rec.get("out_layout", "sample") != layout:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_1309_7695_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["kernel_sources_sha256"] else None


def rate_segments(m):
    """Rate-register segments of 16 the library picks for m reactions."""
    return (m + 15) // 16 if m <= 128 else 0

# Algorithmic cost of each primitive the oracle counts, in full-rate VALU lane
# operations on gfx950: the VALU instructions the compiler emits for that
# primitive in isolation (quarter-rate ones -- 32x32->64 multiplies, f64
# reciprocal/sqrt seeds -- weighted 4).  Measured from the ISA of one-primitive
# kernels: Philox4x32-10 block 140, f64 exp 45, f64 log 117, f64 divide 15,
# sqrt 31, 53-bit uniform 14.
OP_COST = {
    "prop_evals": 8,        # 2 int->f64 converts, 3 f64 multiplies, 1 add, 2 address adds
    "crit_tests": 2,        # one integer product and compare
    "tau_terms": 6,         # critical-bit test, convert, 2 multiplies, 2 adds
    "tau_species": 40,      # g_i, b_i, 2 f64 divides, 2 mins
    "philox_blocks": 140,   # 10 rounds, 20 quarter-rate multiplies
    "inv_draws": 60,        # 53-bit uniform + f64 exp + compare
    "inv_iters": 20,        # f64 divide 1/k + 2 multiplies + add + compare
    "ptrs_draws": 185,      # sqrt, log, 2 divides of the set-up
    "ptrs_iters": 60,       # 2 uniforms, divide, floor, compares
    "ptrs_log_tests": 260,  # 2 logs, a divide, the log-factorial
    "exp_draws": 146,       # 53-bit uniform + f64 log + divide
    "select_terms": 2,      # running sum and compare
    "update_terms": 2,      # integer multiply-add and range check
}


def host_cores():
    """Host cores this process may run on, at most 16 (one GPU's share of a box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-traj", type=int, default=65536)
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="trajectories of the workload the oracle runs for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="fp64: the plain FP64 sweep (the headline form); fp32: RN_FP32")
    ap.add_argument("--workload",
                    choices=("synthetic", "batch", "serve", "phases", "copy", "hybrid", "ode",
                             "ode_stiff", "moments", "stiff", "ssa"),
                    default="synthetic",
                    help="synthetic: the 50x100 sweep of 65,536 trajectories (the headline); "
                         "batch: the uneven batch of 64 networks, batched vs one sweep at a "
                         "time; serve: a Poisson stream of sweep jobs through rn_server; "
                         "phases: per-phase cycle profile of the 50x100 sweep; copy: three 1 GiB "
                         "device copies (calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE); "
                         "hybrid: the hybrid (PDMP) sweep of the 50x100 network with low counts; "
                         "ode: the rate-equation sweep of the 50x100 workload; ode_stiff: the "
                         "stiff 30x80 rate equations by the Rosenbrock method beside the "
                         "explicit pair; ssa: exact-SSA events/s of the dependency-graph and "
                         "general kernels; moments: the "
                         "ensemble-moment reduction of a 50x100 sample array; stiff: the stiff "
                         "30x80 sweep in FP64 and FP32 with per-species moment errors")
    ap.add_argument("--hybrid-cpu-sample", type=int, default=32,
                    help="trajectories the oracle runs for the hybrid cpu_baseline")
    ap.add_argument("--ode-cpu-sample", type=int, default=8,
                    help="trajectories the oracle runs for the rate-equation cpu_baseline")
    ap.add_argument("--out-layout", choices=("traj", "sample"), default="traj",
                    help="synthetic: layout of the sample array (trajectory-major by default)")
    ap.add_argument("--batch-networks", type=int, default=64)
    ap.add_argument("--batch-persistent", action="store_true",
                    help="batch: time the graph, persistent and tuned forms")
    ap.add_argument("--batch-no-sequential", action="store_true",
                    help="batch: skip the one-sweep-at-a-time timing")
    ap.add_argument("--batch-forms", default="graph",
                    help="batch: comma list of graph, persistent, tuned (the first gives value)")
    ap.add_argument("--batch-seq-precision", choices=("fp64", "fp32"), default=None,
                    help="batch: precision of the one-at-a-time timing (default --precision)")
    ap.add_argument("--serve-jobs", type=int, default=1050)
    ap.add_argument("--serve-rate", type=float, default=50.0, help="arrivals per second")
    ap.add_argument("--serve-warmup", type=int, default=50, help="jobs left out of latencies")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="scale of trajectories and t_end per job (1 = the stated stream)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-streams", type=int, default=12)
    return ap.parse_args()


def serve_main(args, torch, gen, rn):
    """Serving stream: jobs arrive as a Poisson process (--serve-rate per second),
    each a seeded network of 20-300 reactions with 1,024-65,536 trajectories and
    t_end logU[10, 500] (both times --serve-scale), 101 samples; they go through
    rn_server with a fixed HBM budget and a few stream slots.  Latency = time
    from arrival to results on the host; the first --serve-warmup jobs are left
    out.  value = trajectory-steps of the measured jobs / their wall span."""
    arrivals, specs = gen.serve_specs(n_jobs=args.serve_jobs, rate=args.serve_rate,
                                      t_scale=args.serve_scale, t_end_scale=args.serve_scale)
    ws = specs  # one entry per job; workloads are built at submission
    nets = {}
    srv = rn.Server(int(args.serve_budget_gib * 2**30), max_running=args.serve_streams)
    kw = dict(precision=args.precision)
    done_at, steps, start = {}, {}, None
    next_job, ids = 0, {}
    host = {"build_job": 0.0, "load_network": 0.0, "submit": 0.0, "poll": 0.0, "fetch": 0.0}
    t0 = time.perf_counter()
    last_print = t0
    while len(done_at) < len(ws):
        now = time.perf_counter() - t0
        while next_job < len(ws) and arrivals[next_job] <= now:
            ta = time.perf_counter()
            w = gen.serve_job(specs[next_job])
            tb = time.perf_counter()
            nets[next_job] = rn.Network(w.net)
            tc = time.perf_counter()
            ids[srv.submit(nets[next_job], w.rates, w.x0, w.times, seed=w.seed, **kw)] = next_job
            td = time.perf_counter()
            host["build_job"] += tb - ta
            host["load_network"] += tc - tb
            host["submit"] += td - tc
            next_job += 1
        ta = time.perf_counter()
        finished = srv.poll()
        host["poll"] += time.perf_counter() - ta
        for jid in finished:
            k = ids.pop(jid)
            ta = time.perf_counter()
            _, st = srv.fetch(jid)
            host["fetch"] += time.perf_counter() - ta
            done_at[k] = time.perf_counter() - t0
            steps[k] = int(st[:, 0].sum() + st[:, 1].sum())
        if time.perf_counter() - last_print > 10:
            last_print = time.perf_counter()
            print(f"[bench] serve t={now:.0f}s submitted {next_job} done {len(done_at)} "
                  f"{srv.status()}", file=sys.stderr, flush=True)
        if next_job < len(ws) and not ids:
            time.sleep(max(0.0, min(arrivals[next_job] - now, 0.01)))
        else:
            time.sleep(0.0005)
    srv.close()
    # network handles are freed only now: hipFree waits for the whole device
    nets.clear()
    meas = range(min(args.serve_warmup, len(ws) - 1), len(ws))
    lat = np.array([done_at[k] - arrivals[k] for k in meas])
    span = max(done_at[k] for k in meas) - min(arrivals[k] for k in meas)
    tot = sum(steps[k] for k in meas)
    offered = args.serve_rate
    achieved = len(meas) / span
    # steady state: jobs completed while arrivals were still coming in, over
    # that window (the span above also holds the drain of the last, heaviest jobs)
    last_arrival = float(arrivals[len(ws) - 1])
    first = float(arrivals[meas[0]])
    in_window = sum(1 for k in meas if done_at[k] <= last_arrival)
    window_rate = in_window / max(last_arrival - first, 1e-9)
    result = {
        "metric": "serving: trajectory-steps/sec and p50/p99 sweep-job latency (1 GPU)",
        "value": tot / span, "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": len(meas), "warmup": len(ws) - len(meas), "ms_per_step": 1e3 * span / len(meas),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": "Poisson stream of sweep jobs", "jobs": len(ws),
                   "rate_per_s": offered, "scale": args.serve_scale,
                   "budget_gib": args.serve_budget_gib, "streams": args.serve_streams,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "latency_ms": {"p50": float(np.percentile(lat, 50)) * 1e3,
                       "p99": float(np.percentile(lat, 99)) * 1e3},
        "jobs_per_s": {"offered": offered, "completed": achieved,
                       "completed_while_arriving": window_rate},
        "drain_s": max(done_at[k] for k in meas) - last_arrival,
        "overloaded": bool(achieved < 0.95 * offered),
        "host_s": host,
    }
    print(json.dumps(result), flush=True)


HYBRID_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "rn_hybrid_hybrid_50x100_traffic.json")


def hybrid_main(args, torch, gen, rn):
    """Hybrid (piecewise-deterministic) sweep: the 50x100 network with a fifth
    of its species below 10 molecules; reactions touching only species that
    start at >= 100 molecules are continuous, the others jump.  --n-traj
    trajectories, t_end 0.5, 11 samples, rtol = atol = 1e-6.  value = Dormand-
    Prince step evaluations (accepted, rejected and jump-search trials) per
    second of the timed sweeps."""
    import hashlib

    dev = torch.device("cuda:0")
    w = gen.hybrid_workload(n_traj=args.n_traj)
    cont = gen.abundance_partition(w.net, w.x0)
    T, M, N, S = w.n_traj, w.net.n_reactions, w.net.n_species, len(w.times)
    net = rn.Network(w.net)
    cont_d = torch.from_numpy(cont.astype(np.int32)).to(dev)
    r = torch.from_numpy(w.rates).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o = torch.empty((S, N, T), dtype=torch.float64, device=dev)
    st = torch.empty((T, 4), dtype=torch.int64, device=dev)
    work = torch.empty(rn.lib().rn_hybrid_work_doubles(net.handle, T), dtype=torch.float64,
                       device=dev)
    kw = dict(seed=w.seed, rtol=1e-6, atol=1e-6)
    print(f"[bench] hybrid {w.name}: T={T} N={N} M={M} S={S}, {int(cont.sum())} continuous "
          f"reactions", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        rn.hybrid_sweep(net, cont_d, r, x, tm, o, st, work, **kw)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        rn.hybrid_sweep(net, cont_d, r, x, tm, o, st, work, **kw)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    print(f"[bench] timed {args.steps} hybrid sweeps: wall {wall:.3f}s, kernel ms "
          f"{kern_ms.round(1)}", file=sys.stderr, flush=True)
    s2 = st.cpu().numpy().view(np.uint64)
    steps = int(s2[:, 0].sum() + s2[:, 1].sum())
    jumps = int(s2[:, 2].sum())
    kern_s = float(np.mean(kern_ms)) / 1000.0
    result = {
        "metric": "hybrid (PDMP) sweep: Dormand-Prince step evaluations/sec (1 GPU)",
        "value": steps * args.steps / wall, "unit": "step-evaluations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name} hybrid, low counts", "n_traj": T, "n_species": N,
                   "n_reactions": M, "continuous_reactions": int(cont.sum()),
                   "t_end": float(w.times[-1]), "n_samples": S, "rtol": 1e-6, "atol": 1e-6,
                   "seed": w.seed, "step_evaluations": steps, "accepted": int(s2[:, 0].sum()),
                   "jumps": jumps, "status_nonzero": int(np.count_nonzero(s2[:, 3]))},
        "latency_ms": {"p50": float(np.percentile(kern_ms, 50)),
                       "p99": float(np.percentile(kern_ms, 99))},
    }
    # Networks of up to 64 species run one wave per trajectory with the state in
    # registers, so the kernel is bound by FP64 arithmetic, not HBM.  Algorithmic
    # FP64 operations of one step evaluation of one trajectory: per species, the
    # five stage arguments and the candidate (2 per coefficient: 30 + 10) and the
    # error term (19); per right-hand side (7 per step), 4 for each continuous
    # (reaction, changed species) entry and 4 for each discrete intensity.
    nnz_c = 0
    for j in range(M):
        if cont[j]:
            d = {}
            for s_, k in w.net.products[j]:
                d[s_] = d.get(s_, 0) + k
            for s_, k in w.net.reactants[j]:
                d[s_] = d.get(s_, 0) - k
            nnz_c += sum(1 for v in d.values() if v != 0)
    m_d = int(M - cont.sum())
    flops_per_step = 59 * N + 7 * 4 * (nnz_c + m_d)
    achieved = flops_per_step * steps / kern_s
    traffic = None
    try:
        rec = json.load(open(HYBRID_TRAFFIC_RECORD))
        h = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, "paper_1309_7695_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() == rec["kernel_sources_sha256"] and rec.get("n_traj") == T:
            traffic = rec["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        traffic = None
    result["kernel"] = ("hybrid_wave_kernel (rn_hybrid.hip, one wave per trajectory)" if N <= 64
                        else "hybrid_lane_kernel (rn_hybrid.hip, one lane per trajectory)")
    result["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": 78.6,
                          "unit": "TFLOP/s", "frac": achieved / 78.6e12, "traffic": traffic,
                          "flops_per_step": flops_per_step, "kernel_ms": kern_s * 1e3}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        n = min(args.hybrid_cpu_sample, T)
        t1 = time.perf_counter()
        _, ost = oracle.hybrid_run(w.net, cont, w.rates, w.x0, w.times, traj_range=(0, n),
                                   threads=1, **kw)
        dt = time.perf_counter() - t1
        csteps = int(ost[:, 0].sum() + ost[:, 1].sum())
        cpu = {"value": csteps / dt, "unit": "step-evaluations/s", "cores": 1, "kind": "oracle",
               "sample": f"trajectories 0..{n - 1} of the same sweep, full horizon, "
                         f"{csteps} step evaluations in {dt:.1f} s, one thread"}
    result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def _timed(torch, dev, args, launch, label):
    for i in range(args.warmup):
        launch()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        launch()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    print(f"[bench] timed {args.steps} {label}: wall {wall:.3f}s, kernel ms {kern_ms.round(2)}",
          file=sys.stderr, flush=True)
    return wall, kern_ms


def ode_main(args, torch, gen, rn):
    """Rate-equation (ODE) sweep of the headline workload: the 50x100 network,
    --n-traj trajectories with their own rates, t_end 50, 200 samples,
    rtol = atol = 1e-6.  value = Dormand-Prince step evaluations (accepted and
    rejected) per second."""
    dev = torch.device("cuda:0")
    w = gen.synthetic_workload(n_traj=args.n_traj)
    T, M, N, S = w.n_traj, w.net.n_reactions, w.net.n_species, len(w.times)
    net = rn.Network(w.net)
    r = torch.from_numpy(w.rates).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o = torch.empty((S, N, T), dtype=torch.float64, device=dev)
    st = torch.empty((T, 4), dtype=torch.int64, device=dev)
    work = torch.empty(rn.lib().rn_ode_work_doubles(net.handle, T), dtype=torch.float64,
                       device=dev)
    print(f"[bench] ode {w.name}: T={T} N={N} M={M} S={S}", file=sys.stderr, flush=True)
    wall, kern_ms = _timed(torch, dev, args,
                           lambda: rn.ode_sweep(net, r, x, tm, o, st, work), "ode sweeps")
    s2 = st.cpu().numpy().view(np.uint64)
    steps = int(s2[:, 0].sum() + s2[:, 1].sum())
    kern_s = float(np.mean(kern_ms)) / 1000.0
    # Algorithmic FP64 operations of one step evaluation of one trajectory (the
    # count of the hybrid sweep with every reaction continuous): 59 per species
    # and 4 per (reaction, changed species) entry for each of the 7 right-hand
    # sides.
    nnz = 0
    for j in range(M):
        d = {}
        for s_, k in w.net.products[j]:
            d[s_] = d.get(s_, 0) + k
        for s_, k in w.net.reactants[j]:
            d[s_] = d.get(s_, 0) - k
        nnz += sum(1 for v in d.values() if v != 0)
    flops_per_step = 59 * N + 7 * 4 * nnz
    achieved = flops_per_step * steps / kern_s
    result = {
        "metric": "rate-equation sweep: Dormand-Prince step evaluations/sec (1 GPU)",
        "value": steps * args.steps / wall, "unit": "step-evaluations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name} rate equations", "n_traj": T, "n_species": N,
                   "n_reactions": M, "t_end": float(w.times[-1]), "n_samples": S,
                   "rtol": 1e-6, "atol": 1e-6, "step_evaluations": steps,
                   "accepted": int(s2[:, 0].sum()),
                   "status_nonzero": int(np.count_nonzero(s2[:, 3]))},
        "kernel": ("hybrid_wave_kernel<ode> (rn_hybrid.hip, one wave per trajectory)" if N <= 64
                   else "ode_kernel (rn_ode.hip, one lane per trajectory)"),
        "latency_ms": {"p50": float(np.percentile(kern_ms, 50)),
                       "p99": float(np.percentile(kern_ms, 99))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": achieved / 78.6e12, "traffic": None,
                     "flops_per_step": flops_per_step, "kernel_ms": kern_s * 1e3},
    }
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        n = min(args.ode_cpu_sample, T)
        t1 = time.perf_counter()
        _, ost = oracle.ode_run(w.net, w.rates, w.x0, w.times, traj_range=(0, n), threads=1)
        dt = time.perf_counter() - t1
        csteps = int(ost[:, 0].sum() + ost[:, 1].sum())
        cpu = {"value": csteps / dt, "unit": "step-evaluations/s", "cores": 1, "kind": "oracle",
               "sample": f"trajectories 0..{n - 1} of the same sweep, full horizon, "
                         f"{csteps} step evaluations in {dt:.1f} s, one thread"}
    result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def ssa_main(args, torch, gen, rn):
    """Exact SSA (RN_METHOD_SSA): events/s of the dependency-graph kernel and of
    the general network-compiled kernel (RN_SSA_KERNEL=full) on the enzyme
    workload (1,024 trajectories to t = 100) and the 50x100 network (--n-traj
    trajectories to t = 0.5).  value = the dependency-graph kernel's events/s on
    the 50x100 network."""
    dev = torch.device("cuda:0")
    cases = [("enzyme_4x3", gen.enzyme_workload()),
             ("synthetic_50x100", gen.synthetic_workload(n_traj=args.n_traj, t_end=0.5,
                                                         n_samples=11))]
    res = {}
    for name, w in cases:
        T, N, S = w.n_traj, w.net.n_species, len(w.times)
        net = rn.Network(w.net)
        r = torch.from_numpy(w.rates).to(dev)
        x = torch.from_numpy(w.x0).to(dev)
        tm = torch.from_numpy(w.times).to(dev)
        o = torch.empty((S, N, T), dtype=torch.int32, device=dev)
        st = torch.empty((T, 4), dtype=torch.int64, device=dev)
        for kern in ("dep", "full"):
            os.environ["RN_SSA_KERNEL"] = kern
            wall, kern_ms = _timed(torch, dev, args,
                                   lambda: rn.sweep(net, r, x, tm, o, st, seed=w.seed,
                                                    method=rn.METHOD_SSA),
                                   f"ssa {kern} {name}")
            ev = int(st.cpu().numpy()[:, 1].sum())
            res[f"{name}_{kern}"] = {"events_per_sweep": ev,
                                     "kernel_ms": float(np.mean(kern_ms)),
                                     "events_per_s": ev / (float(np.mean(kern_ms)) / 1e3)}
            print(f"[bench] ssa {kern} {name}: {res[f'{name}_{kern}']}", file=sys.stderr,
                  flush=True)
    os.environ.pop("RN_SSA_KERNEL", None)
    main = res["synthetic_50x100_dep"]
    result = {
        "metric": "exact SSA events/sec (1 GPU)", "value": main["events_per_s"],
        "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main["kernel_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "exact SSA, enzyme 4x3 and synthetic 50x100",
                   "n_traj_50x100": args.n_traj, "t_end_50x100": 0.5},
        "kernels": res, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def ros4_flops_per_step(net):
    """Algorithmic FP64 operations of one Rosenbrock 4(3) step of one
    trajectory: the Jacobian (3 per derivative term, N^2 for W), the pivoted LU
    factorization (a division per multiplier, a multiply and a subtract per
    updated entry), four triangular solves (2 per off-diagonal entry, N
    divisions), three right-hand sides (2 per reaction rate, 2 per (reaction,
    changed species) entry) and 45 per species for the stage arguments,
    solution, error and norm."""
    N, M = net.n_species, net.n_reactions
    nnz = 0
    dterms = 0
    for j in range(M):
        d = {}
        for s_, k in net.products[j]:
            d[s_] = d.get(s_, 0) + k
        for s_, k in net.reactants[j]:
            d[s_] = d.get(s_, 0) - k
        changed = sum(1 for v in d.values() if v != 0)
        nnz += changed
        dterms += changed * len(net.reactants[j])
    lu = sum((N - k - 1) + 2 * (N - k - 1) ** 2 for k in range(N))
    solves = 4 * (2 * N * (N - 1) + N)
    return 3 * dterms + N * N + lu + solves + 3 * (2 * M + 2 * nnz) + 45 * N


def ode_stiff_main(args, torch, gen, rn):
    """Stiff rate equations: the 30x80 network with rates over eight decades,
    --n-traj trajectories to t_end 10 (101 samples), rtol = atol = 1e-6, by the
    Rosenbrock 4(3) method (timed); one sweep of the same inputs by the
    Dormand-Prince pair gives its step counts and time for comparison.
    value = Rosenbrock steps (accepted and rejected) per second."""
    dev = torch.device("cuda:0")
    w = gen.stiff_workload(n_traj=args.n_traj)
    T, M, N, S = w.n_traj, w.net.n_reactions, w.net.n_species, len(w.times)
    net = rn.Network(w.net)
    r = torch.from_numpy(w.rates).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o = torch.empty((S, N, T), dtype=torch.float64, device=dev)
    st = torch.empty((T, 4), dtype=torch.int64, device=dev)
    work = torch.empty(rn.lib().rn_ode_work_doubles(net.handle, T), dtype=torch.float64,
                       device=dev)
    print(f"[bench] stiff ode {w.name}: T={T} N={N} M={M} S={S}", file=sys.stderr, flush=True)
    wall, kern_ms = _timed(torch, dev, args,
                           lambda: rn.ode_sweep(net, r, x, tm, o, st, work, method="ros4"),
                           "ros4 sweeps")
    s2 = st.cpu().numpy().view(np.uint64)
    steps = int(s2[:, 0].sum() + s2[:, 1].sum())
    ros_out = o.cpu().numpy()
    kern_s = float(np.mean(kern_ms)) / 1000.0
    fps = ros4_flops_per_step(w.net)
    achieved = fps * steps / kern_s
    # the explicit pair on the same inputs, once
    o2 = torch.empty_like(o)
    st2 = torch.empty_like(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rn.ode_sweep(net, r, x, tm, o2, st2, work, method="dopri5")
    torch.cuda.synchronize()
    dp_s = time.perf_counter() - t0
    d2 = st2.cpu().numpy().view(np.uint64)
    dp_out = o2.cpu().numpy()
    diff = float((np.abs(ros_out - dp_out) / (1.0 + np.abs(dp_out))).max())
    print(f"[bench] dopri5 once: {dp_s:.2f} s, accepted mean {d2[:, 0].mean():.0f}",
          file=sys.stderr, flush=True)
    result = {
        "metric": "stiff rate-equation sweep: Rosenbrock step evaluations/sec (1 GPU)",
        "value": steps * args.steps / wall, "unit": "step-evaluations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name} stiff rate equations (Rosenbrock 4(3))", "n_traj": T,
                   "n_species": N, "n_reactions": M, "t_end": float(w.times[-1]),
                   "n_samples": S, "rtol": 1e-6, "atol": 1e-6, "step_evaluations": steps,
                   "accepted_mean": float(s2[:, 0].mean()), "accepted_max": int(s2[:, 0].max()),
                   "rejected_mean": float(s2[:, 1].mean()),
                   "status_nonzero": int(np.count_nonzero(s2[:, 3]))},
        "dopri5_same_inputs": {"sweep_s": dp_s, "accepted_mean": float(d2[:, 0].mean()),
                               "accepted_max": int(d2[:, 0].max()),
                               "rejected_mean": float(d2[:, 1].mean()),
                               "status_nonzero": int(np.count_nonzero(d2[:, 3])),
                               "max_rel_sample_diff_vs_ros4": diff},
        "kernel": "ros_wave_kernel (rn_ros.hip, one wave per trajectory)",
        "latency_ms": {"p50": float(np.percentile(kern_ms, 50)),
                       "p99": float(np.percentile(kern_ms, 99))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": achieved / 78.6e12, "traffic": None,
                     "flops_per_step": fps, "kernel_ms": kern_s * 1e3},
    }
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        n = min(args.ode_cpu_sample * 16, T)
        t1 = time.perf_counter()
        _, ost = oracle.ode_run(w.net, w.rates, w.x0, w.times, traj_range=(0, n), threads=1,
                                method="ros4")
        dt = time.perf_counter() - t1
        csteps = int(ost[:, 0].sum() + ost[:, 1].sum())
        cpu = {"value": csteps / dt, "unit": "step-evaluations/s", "cores": 1, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"trajectories 0..{n - 1} of the same sweep, full horizon, "
                         f"{csteps} Rosenbrock steps in {dt:.1f} s, one thread"}
    result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def stiff_main(args, torch, gen, rn):
    """Stiff multiscale sweep: 30 species, 80 reactions, rates logU[1e-6, 1e2],
    a fifth of the species below 10 molecules, --n-traj trajectories to
    t_end 10 (101 samples).  Times the FP64 and the FP32 sweep with the same
    seed and reports, per species, the relative error of the FP32 ensemble mean
    against the FP64 one at every sample (max over samples) and its paired z."""
    dev = torch.device("cuda:0")
    w = gen.stiff_workload(n_traj=args.n_traj)
    T, M, N, S = w.n_traj, w.net.n_reactions, w.net.n_species, len(w.times)
    net = rn.Network(w.net)
    r = torch.from_numpy(w.rates).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    res = {}
    for prec in ("fp64", "fp32"):
        kind = rn.sweep_kernel_kind(net, T, prec)
        o = torch.empty((S, N, T), dtype=torch.int32, device=dev)
        st = torch.empty((T, 4), dtype=torch.int64, device=dev)
        kw = dict(seed=w.seed, eps=w.eps, n_c=w.n_c, precision=prec)
        wall, kern_ms = _timed(torch, dev, args, lambda: rn.sweep(net, r, x, tm, o, st, **kw),
                               f"{prec} stiff sweeps")
        s2 = st.cpu().numpy().view(np.uint64)
        steps = int(s2[:, 0].sum() + s2[:, 1].sum())
        res[prec] = dict(out=o.cpu().numpy().astype(np.float64), steps=steps, kind=kind,
                         wall=wall, kern_ms=float(np.mean(kern_ms)))
    a, b = res["fp64"]["out"], res["fp32"]["out"]
    m64, m32 = a.mean(axis=2), b.mean(axis=2)                    # [S][N]
    rel = np.abs(m32 - m64) / np.maximum(np.abs(m64), 1.0)
    d = b - a                                                    # paired differences
    se = d.std(axis=2, ddof=1) / np.sqrt(T)
    z = np.where(se > 0, np.abs(d.mean(axis=2)) / np.where(se > 0, se, 1.0), 0.0)
    per_species = [{"species": i, "max_rel_mean_error": float(rel[:, i].max()),
                    "max_paired_z": float(z[:, i].max())} for i in range(N)]
    v64 = res["fp64"]["steps"] / (res["fp64"]["kern_ms"] / 1e3)
    v32 = res["fp32"]["steps"] / (res["fp32"]["kern_ms"] / 1e3)
    result = {
        "metric": "stiff 30x80 sweep: trajectory-steps/sec FP64 and FP32 (1 GPU)",
        "value": v32, "unit": "trajectory-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["fp32"]["kern_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name} stiff, FP32 vs FP64", "n_traj": T, "n_species": N,
                   "n_reactions": M, "t_end": float(w.times[-1]), "n_samples": S,
                   "seed": w.seed},
        "fp64": {"value": v64, "ms": res["fp64"]["kern_ms"], "steps": res["fp64"]["steps"],
                 "kernel": res["fp64"]["kind"]},
        "fp32": {"value": v32, "ms": res["fp32"]["kern_ms"], "steps": res["fp32"]["steps"],
                 "kernel": res["fp32"]["kind"]},
        "fp32_speedup": v32 / v64,
        "moment_error": {"max_rel_mean_error": float(rel.max()),
                         "median_rel_mean_error": float(np.median(rel)),
                         "max_paired_z": float(z.max()), "per_species": per_species},
        "cpu_baseline": None, "roofline": None,
    }
    print(json.dumps(result), flush=True)


def moments_main(args, torch, gen, rn):
    """Ensemble moments (rn_moments) of a sample array of the headline shape:
    200 samples x 50 species x --n-traj trajectories of int32 counts in
    [0, 1000].  HBM-bound: value = bytes of samples read per second."""
    dev = torch.device("cuda:0")
    S, N, T = 200, 50, args.n_traj
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    out = torch.randint(0, 1001, (S, N, T), dtype=torch.int32, device=dev, generator=g)
    sx = torch.empty((S, N), dtype=torch.int64, device=dev)
    sx2 = torch.empty((S, N, 2), dtype=torch.int64, device=dev)
    wall, kern_ms = _timed(torch, dev, args,
                           lambda: rn.moments(out, sum_x=sx, sum_x2=sx2), "moment reductions")
    ref = out.to(torch.int64).sum(dim=2)
    assert torch.equal(ref, sx), "moment sums differ from torch's"
    kern_s = float(np.mean(kern_ms)) / 1000.0
    nbytes = S * N * T * 4 + S * N * 24
    result = {
        "metric": "ensemble-moment reduction: sample bytes/sec (1 GPU)",
        "value": nbytes * args.steps / wall, "unit": "B/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32/int64/u128", "data": "synthetic",
        "config": {"workload": "moments of [200][50][T] int32 samples", "n_traj": T},
        "kernel": "moments_kernel (rn_moments.hip)",
        "latency_ms": {"p50": float(np.percentile(kern_ms, 50)),
                       "p99": float(np.percentile(kern_ms, 99))},
        "roofline": {"bound": "hbm", "achieved": nbytes / kern_s / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": nbytes / kern_s / 8e12, "traffic": None,
                     "kernel_ms": kern_s * 1e3},
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def copy_main(args, torch):
    """Three device copies of 1 GiB (torch's copy kernel): the reference the
    FETCH_SIZE and WRITE_SIZE counters are scaled by."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 3
    print(json.dumps({"workload": "device copy", "bytes": 4 * n, "copies": 3,
                      "ms_per_copy": dt * 1e3, "GB_per_s": 2 * 4 * n / dt / 1e9}), flush=True)


def phases_main(args, torch, gen, rn):
    """Per-wave shader-clock cycles of the 50x100 sweep in SSA events, the decide
    phase and leap attempts (network-compiled kernel built with phase timers)."""
    os.environ["RN_PHASE_TIMERS"] = "1"  # read when the kernel is compiled
    dev = torch.device("cuda:0")
    w = gen.synthetic_workload(n_traj=args.n_traj)
    T = w.n_traj
    net = rn.Network(w.net)
    kind = rn.sweep_kernel_kind(net, T, args.precision)
    r = torch.from_numpy(w.rates).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o = torch.empty((len(w.times), w.net.n_species, T), dtype=torch.int32, device=dev)
    st = torch.empty((T, 4), dtype=torch.int64, device=dev)
    ph = torch.zeros(((T + 63) // 64) * 4, dtype=torch.int64, device=dev)
    rn.sweep(net, r, x, tm, o, st, seed=w.seed, precision=args.precision, phase_cycles=ph)
    torch.cuda.synchronize()
    d = ph.cpu().numpy().reshape(-1, 4).astype(float)
    s = st.cpu().numpy()
    tot = d[:, 3].sum()
    waves_ssa = s[:, 1].reshape(-1, 64).max(axis=1).sum() if T % 64 == 0 else None
    waves_leap = s[:, 0].reshape(-1, 64).max(axis=1).sum() if T % 64 == 0 else None
    print(json.dumps({
        "workload": f"{w.name} {args.precision.upper()}", "kernel": kind,
        "cycles_per_wave": {"mean": d[:, 3].mean(), "max": d[:, 3].max()},
        "share": {"ssa": d[:, 0].sum() / tot, "decide": d[:, 1].sum() / tot,
                  "leap": d[:, 2].sum() / tot},
        "cycles_per_ssa_pass": d[:, 0].sum() / waves_ssa if waves_ssa else None,
        "cycles_per_decide_and_leap": (d[:, 1].sum() + d[:, 2].sum()) / waves_leap
        if waves_leap else None}), flush=True)


def batch_main(args, torch, gen, rn):
    """Uneven batch: 64 seeded networks of 10-500 reactions (species = reactions/2)
    with 256-16,384 trajectories each, t_end 50, 200 samples.  Times the whole
    batch in the forms --batch-forms names (graph: one rn_batch graph of
    per-job kernels; persistent: the work-queue kernels in default shapes;
    tuned: the same after rn_batch_tune) and as one rn_sweep per network in turn
    (in --batch-seq-precision, default the batch's own); value = trajectory-steps
    of the batch / wall time of the first form's launch."""
    dev = torch.device("cuda:0")
    forms = [f for f in args.batch_forms.split(",") if f]
    if args.batch_persistent:
        forms = ["graph", "persistent", "tuned"]
    if not forms or any(f not in ("graph", "persistent", "tuned") for f in forms):
        raise SystemExit("--batch-forms: a comma list of graph, persistent, tuned")
    seq_prec = args.batch_seq_precision or args.precision
    ws = gen.batch_workloads(n_networks=args.batch_networks)
    jobs = []
    for k, w in enumerate(ws):
        S, N, T = len(w.times), w.net.n_species, w.n_traj
        jobs.append(dict(net=rn.Network(w.net), seed=w.seed, T=T,
                         rates=torch.from_numpy(w.rates).to(dev),
                         x0=torch.from_numpy(w.x0).to(dev),
                         times=torch.from_numpy(w.times).to(dev),
                         out=torch.empty((S, N, T), dtype=torch.int32, device=dev),
                         stats=torch.empty((T, 4), dtype=torch.int64, device=dev)))
    t0 = time.perf_counter()
    from concurrent.futures import ThreadPoolExecutor, as_completed
    precs = [args.precision] + ([seq_prec] if seq_prec != args.precision else [])
    tasks = [(k, pr) for pr in precs for k in range(len(jobs))]
    kinds = {}
    with ThreadPoolExecutor(max_workers=16) as ex:
        futs = {ex.submit(rn.sweep_kernel_kind, jobs[k]["net"], jobs[k]["T"], pr): (k, pr)
                for k, pr in tasks}
        for n_done, f in enumerate(as_completed(futs), 1):
            kinds[futs[f]] = f.result()
            print(f"[bench] kernels ready {n_done}/{len(tasks)} "
                  f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    setup_s = time.perf_counter() - t0
    kind_list = [kinds[(k, args.precision)] for k in range(len(jobs))]
    print(f"[bench] batch of {len(jobs)}: {kind_list.count('network')} network-compiled, "
          f"{kind_list.count('wave')} wave-per-trajectory, {kind_list.count('generic')} "
          f"lane generic kernels; setup {setup_s:.1f} s",
          file=sys.stderr, flush=True)
    kw = dict(precision=args.precision)

    def sequential(report=False):
        for k, j in enumerate(jobs):
            rn.sweep(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"],
                     seed=j["seed"], precision=seq_prec)
            if report:
                torch.cuda.synchronize()
                print(f"[bench] job {k + 1}/{len(jobs)} done (M={j['net'].n_reactions}, "
                      f"T={j['T']})", file=sys.stderr, flush=True)

    def count_steps():
        return sum(int(st[:, 0].sum() + st[:, 1].sum()) for st in
                   (j["stats"].cpu().numpy().view(np.uint64) for j in jobs))

    # one at a time (also the warm-up of every job's kernel), FIFO
    seq_s = seq_steps = None
    if not args.batch_no_sequential:
        t = time.perf_counter()
        sequential(report=True)
        torch.cuda.synchronize()
        seq_s = time.perf_counter() - t
        seq_steps = count_steps()
        print(f"[bench] one at a time ({seq_prec}): {seq_s * 1e3:.1f} ms", file=sys.stderr,
              flush=True)

    # every form's results must be those of rn_sweep one at a time (when that ran
    # in the batch's precision), else those of the first form
    ref = None
    if seq_s and seq_prec == args.precision:
        ref = [(j["out"].cpu().numpy(), j["stats"].cpu().numpy()) for j in jobs]

    def timed(b, label):
        nonlocal ref
        t = time.perf_counter()
        b.launch()  # records the graph; untimed
        torch.cuda.synchronize()
        print(f"[bench] {label} first launch (untimed): {(time.perf_counter() - t) * 1e3:.0f} ms",
              file=sys.stderr, flush=True)
        now = [(j["out"].cpu().numpy(), j["stats"].cpu().numpy()) for j in jobs]
        if ref is None:
            ref = now
        same = all(np.array_equal(a[0], r[0]) and np.array_equal(a[1], r[1])
                   for a, r in zip(now, ref))
        ts = []
        for i in range(args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            b.launch()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            print(f"[bench] {label} launch {i + 1}/{args.steps}: {ts[-1] * 1e3:.0f} ms",
                  file=sys.stderr, flush=True)
        return float(np.mean(ts)), same

    results = {}
    steps = None
    for form in forms:
        b = rn.Batch(persistent=form != "graph")
        for j in jobs:
            b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"],
                  seed=j["seed"], **kw)
        tune_s = 0.0
        if form == "tuned":
            os.environ.setdefault("RN_TUNE_LOG", "1")  # a line per bucket: progress
            t = time.perf_counter()
            b.tune()
            torch.cuda.synchronize()
            tune_s = time.perf_counter() - t
            print(f"[bench] persistent form tuned in {tune_s:.1f} s", file=sys.stderr,
                  flush=True)
        sec, same = timed(b, form)
        b.close()
        if steps is None:
            steps = count_steps()
        results[form] = {"value": steps / sec, "ms_per_step": sec * 1e3,
                         "identical_to_reference": bool(same)}
        if form == "tuned":
            results[form]["tune_s"] = tune_s
        if seq_s:
            results[form]["speedup_vs_one_at_a_time"] = seq_s / sec
    first = results[forms[0]]
    result = {
        "metric": "trajectory-steps/sec, uneven batch of 64 networks (1 GPU)",
        "value": first["value"], "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": first["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"uneven batch of {len(jobs)} synthetic networks, "
                               f"{args.precision.upper()}, {forms[0]} form",
                   "n_networks": len(jobs),
                   "n_traj_total": int(sum(j["T"] for j in jobs)),
                   "reactions": [int(j["net"].n_reactions) for j in jobs],
                   "steps_per_batch": steps},
        "kernels": {k: kind_list.count(k) for k in ("network", "wave", "generic")},
        "setup_s": {"kernel_compile": setup_s},
        "forms": results,
        "one_at_a_time": ({"precision": seq_prec, "value": seq_steps / seq_s,
                           "ms_per_step": seq_s * 1e3} if seq_s else None),
    }
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: each sweep runs on a single MI355X "
              "(trajectories shard across GPUs with no exchange, so more GPUs add "
              "throughput by splitting the trajectory range).  Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        # one hardware queue per server stream, plus the null, copy and table
        # streams (HIP reads this when it initializes; its default is 4, and
        # streams beyond the queues share them and wait for each other's work)
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, args.serve_streams + 4))
    if args.workload == "batch":
        # graph branches (the graph's launch spreads them over the process's
        # hardware queues; 16 branches on HIP's default 4 queues ran the batch
        # in 84 s, 12 branches on 16 queues in 105 s)
        os.environ.setdefault("RN_BATCH_BRANCHES", "16")
    import torch

    from paper_1309_7695_amd import gen, rn

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "batch":
        batch_main(args, torch, gen, rn)
        return
    if args.workload == "serve":
        serve_main(args, torch, gen, rn)
        return
    if args.workload == "phases":
        phases_main(args, torch, gen, rn)
        return
    if args.workload == "copy":
        copy_main(args, torch)
        return
    if args.workload == "hybrid":
        hybrid_main(args, torch, gen, rn)
        return
    if args.workload == "ode":
        ode_main(args, torch, gen, rn)
        return
    if args.workload == "ode_stiff":
        ode_stiff_main(args, torch, gen, rn)
        return
    if args.workload == "ssa":
        ssa_main(args, torch, gen, rn)
        return
    if args.workload == "moments":
        moments_main(args, torch, gen, rn)
        return
    if args.workload == "stiff":
        stiff_main(args, torch, gen, rn)
        return
    dev = torch.device("cuda:0")
    w = gen.synthetic_workload(n_traj=args.n_traj)
    T, M, N, S = w.n_traj, w.net.n_reactions, w.net.n_species, len(w.times)
    net = rn.Network(w.net)
    rates = torch.from_numpy(w.rates).to(dev)
    x0 = torch.from_numpy(w.x0).to(dev)
    times = torch.from_numpy(w.times).to(dev)
    # trajectory-major samples: each trajectory writes its own contiguous rows
    # (lanes reach the sample times at different moments, so sample-major rows
    # are written a few values per store)
    if args.out_layout == "traj":
        out = torch.empty((T, S, N), dtype=torch.int32, device=dev)
    else:
        out = torch.empty((S, N, T), dtype=torch.int32, device=dev)
    stats = torch.empty((T, 4), dtype=torch.int64, device=dev)
    kw = dict(seed=w.seed, eps=w.eps, n_c=w.n_c, precision=args.precision,
              out_layout=args.out_layout)
    print(f"[bench] workload {w.name}: T={T} N={N} M={M} S={S}", file=sys.stderr, flush=True)
    # Setup, outside every timed step: the library compiles the kernel for this
    # network on first use (hipRTC); do it here and report its cost apart.
    t0 = time.perf_counter()
    kind = rn.sweep_kernel_kind(net, T, args.precision)
    setup_s = time.perf_counter() - t0
    real = "double" if args.precision == "fp64" else "float"
    wg = 256 if T >= 256 * torch.cuda.get_device_properties(dev).multi_processor_count else 64
    kernel = (f"rn_net_sweep<{wg}, {real}> (compiled for the network)" if kind == "network"
              else f"sweep_kernel<{wg}, {rate_segments(M)}, {real}>")
    print(f"[bench] kernel {kernel}; setup {setup_s:.1f} s", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        rn.sweep(net, rates, x0, times, out, stats, **kw)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    warm_steps = None
    if args.warmup > 0:
        st = stats.cpu().numpy().view(np.uint64)
        warm_steps = int(st[:, 0].sum() + st[:, 1].sum())

    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        rn.sweep(net, rates, x0, times, out, stats, **kw)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    print(f"[bench] timed {args.steps} sweeps: wall {wall:.3f}s, kernel ms {kern_ms.round(2)}",
          file=sys.stderr, flush=True)
    st2 = stats.cpu().numpy().view(np.uint64)
    steps_per_sweep = int(st2[:, 0].sum() + st2[:, 1].sum())
    # every sweep of the same inputs and seed takes the same steps
    assert warm_steps is None or warm_steps == steps_per_sweep
    assert int(out.min().item()) >= 0
    ms_per_step = wall * 1000.0 / args.steps
    value = steps_per_sweep * args.steps / wall

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name} {args.precision.upper()} plain sweep", "n_traj": T, "n_species": N,
                   "n_reactions": M, "t_end": float(w.times[-1]), "n_samples": S,
                   "out_layout": ("trajectory-major [T][S][N]" if args.out_layout == "traj"
                                  else "sample-major [S][N][T]"),
                   "eps": w.eps, "n_c": w.n_c, "seed": w.seed,
                   "steps_per_sweep": steps_per_sweep,
                   "leaps": int(st2[:, 0].sum()), "ssa_events": int(st2[:, 1].sum()),
                   "rejections": int(st2[:, 2].sum())},
        "kernel": kernel,
        "setup_s": {"kernel_compile": setup_s},
        "latency_ms": {"p50": float(np.percentile(kern_ms, 50)),
                       "p99": float(np.percentile(kern_ms, 99))},
    }

    cpu = None
    ops_per_step = None
    if not args.no_cpu_baseline:
        import oracle

        # one thread on a prefix of the sweep (the single-core reference of the
        # speed-up), then every host core available to this process on a longer
        # prefix (one thread per core, contiguous trajectory chunks)
        n = min(args.cpu_sample, T)
        t0 = time.perf_counter()
        _, ost, ops = oracle.run(w.net, w.rates, w.x0, w.times, seed=w.seed,
                                 traj_range=(0, n), threads=1, counters=True)
        dt = time.perf_counter() - t0
        csteps = int(ost[:, 0].sum() + ost[:, 1].sum())
        one = {"value": csteps / dt, "cores": 1,
               "sample": f"trajectories 0..{n - 1} of the same sweep, full horizon, "
                         f"{csteps} steps in {dt:.1f} s, one thread"}
        print(f"[bench] cpu oracle, 1 thread: {one['value']:.4g} steps/s on {n} trajectories",
              file=sys.stderr, flush=True)
        cores = host_cores()
        na = min(n * cores, T)
        t0 = time.perf_counter()
        _, ast, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=w.seed,
                               traj_range=(0, na), threads=cores)
        dta = time.perf_counter() - t0
        asteps = int(ast[:, 0].sum() + ast[:, 1].sum())
        cpu = {"value": asteps / dta, "unit": "trajectory-steps/s", "cores": cores,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"trajectories 0..{na - 1} of the same sweep, full horizon, "
                         f"{asteps} steps in {dta:.1f} s, {cores} threads",
               "single_core": one}
        print(f"[bench] cpu oracle, {cores} threads: {cpu['value']:.4g} steps/s on {na} "
              f"trajectories ({cpu['cpu_model']})", file=sys.stderr, flush=True)
        work = sum(OP_COST[k] * ops[k] for k in OP_COST)
        ops_per_step = work / max(csteps, 1)
    result["cpu_baseline"] = cpu

    kern_s = float(np.mean(kern_ms)) / 1000.0
    if ops_per_step is not None and args.precision == "fp64":
        achieved = ops_per_step * steps_per_sweep / kern_s
        result["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                              "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                              "frac": achieved / PEAK_LANE_OPS,
                              "traffic": (measured_traffic(kind, args.out_layout) if T == 65536
                                          else None),
                              "kernel": kernel,
                              "ops_per_step": ops_per_step,
                              "kernel_ms": float(np.mean(kern_ms))}
    else:
        result["roofline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
