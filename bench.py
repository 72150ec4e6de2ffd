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


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "sweep_kernel_synthetic_50x100_fp64_traffic.json")


def measured_traffic():
    """HBM bytes per launch of the FP64 sweep kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record (each counter scaled by what it
    reads for a copy of known size), or None when the kernel sources changed
    since the counters were taken."""
    import hashlib

    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
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
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs each sweep on a single "
              "MI355X (trajectories shard with zero exchange; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1309_7695_amd import gen, rn

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    w = gen.synthetic_workload(n_traj=args.n_traj)
    T, M, N, S = w.n_traj, w.net.n_reactions, w.net.n_species, len(w.times)
    net = rn.Network(w.net)
    rates = torch.from_numpy(w.rates).to(dev)
    x0 = torch.from_numpy(w.x0).to(dev)
    times = torch.from_numpy(w.times).to(dev)
    out = torch.empty((S, N, T), dtype=torch.int32, device=dev)
    stats = torch.empty((T, 4), dtype=torch.int64, device=dev)
    kw = dict(seed=w.seed, eps=w.eps, n_c=w.n_c, precision=args.precision)
    print(f"[bench] workload {w.name}: T={T} N={N} M={M} S={S}", file=sys.stderr, flush=True)

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
                   "eps": w.eps, "n_c": w.n_c, "seed": w.seed,
                   "steps_per_sweep": steps_per_sweep,
                   "leaps": int(st2[:, 0].sum()), "ssa_events": int(st2[:, 1].sum()),
                   "rejections": int(st2[:, 2].sum())},
        "latency_ms": {"p50": float(np.percentile(kern_ms, 50)),
                       "p99": float(np.percentile(kern_ms, 99))},
    }

    cpu = None
    ops_per_step = None
    if not args.no_cpu_baseline:
        import oracle

        n = min(args.cpu_sample, T)
        t0 = time.perf_counter()
        _, ost, ops = oracle.run(w.net, w.rates, w.x0, w.times, seed=w.seed,
                                 traj_range=(0, n), threads=1, counters=True)
        dt = time.perf_counter() - t0
        csteps = int(ost[:, 0].sum() + ost[:, 1].sum())
        cpu = {"value": csteps / dt, "unit": "trajectory-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"trajectories 0..{n - 1} of the same sweep, full horizon, "
                         f"{csteps} steps in {dt:.1f} s, one thread"}
        work = sum(OP_COST[k] * ops[k] for k in OP_COST)
        ops_per_step = work / max(csteps, 1)
        print(f"[bench] cpu oracle: {cpu['value']:.4g} steps/s on {n} trajectories",
              file=sys.stderr, flush=True)
    result["cpu_baseline"] = cpu

    kern_s = float(np.mean(kern_ms)) / 1000.0
    if ops_per_step is not None and args.precision == "fp64":
        achieved = ops_per_step * steps_per_sweep / kern_s
        result["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                              "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                              "frac": achieved / PEAK_LANE_OPS,
                              "traffic": measured_traffic() if T == 65536 else None,
                              "kernel": f"sweep_kernel<256, {rate_segments(M)}, double>",
                              "ops_per_step": ops_per_step,
                              "kernel_ms": float(np.mean(kern_ms))}
    else:
        result["roofline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
