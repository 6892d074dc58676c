"""Benchmark: random-batch SOE Ewald2D long-range step at N = 1e6 on one MI355X.

Workload (configuration 3 of workloads.py): 1e6 charges +-1 in a 600 x 600 x 10
slab with a 10% surface excess of +1 near z = 0 and -1 near z = 10, alpha = 0.1,
P = 100 importance-sampled Fourier modes per step, SOE with M = 16 terms.
One step = one q2d_rbm_step call: mode sampling, z-sort, the k != 0 scans,
the FP64 k = 0 term and the reductions, with inputs resident in HBM and a
different (seed, step) -- hence different modes -- every step.

Prints one JSON line:
  value        particle-force evaluations per second (N / step time), FP32 path
  roofline     the hot kernel (k != 0 sweep): algorithmic FLOP per launch over its
               average launch time from HIP events recorded on the plan's stream
               during the timed steps, against the MI355X FP32 vector peak
  cpu_baseline the FP64 O(N) recursion of the oracle on one host core, on all
               1e6 particles but a subset of the modes, scaled to P = 100
Extra fields: the FP64 path on the same GPU and the FP32/FP64 speedup, and the
relative RMS difference of FP32 and FP64 forces for identical modes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-force evals/s at N=1e6 (SOE-RBM FP32 vs FP64 SOE) @ force err ≤1e-4"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published)
P_MODES = 100
M_SOE = 16


def flops_per_mode_particle(M):
    """Algorithmic FLOP per (mode, particle): per exponent beta (M SOE terms and
    beta = k) a forward and a backward complex recurrence step and the two
    complex combines (4 complex FMA = 32 FLOP), plus ~20 FLOP of phase and
    force assembly per mode."""
    return 32 * (M + 1) + 20


def soe_table(M):
    from oracle import soe  # the table is an input of the method; both sides read it
    return soe.load_table(os.path.join(ROOT, "tests", "golden", "soe_talbot_M%d.txt" % M))


def run_gpu(prec, c, w, s, steps, warmup, timing):
    import torch
    import paper_2403_01521_amd as q2d
    dt = torch.float32 if prec == "fp32" else torch.float64
    pos = torch.tensor(c["pos"], dtype=dt, device="cuda")
    q = torch.tensor(c["q"], dtype=dt, device="cuda")
    N = len(c["q"])
    plan = q2d.Plan(c["box"], c["alpha"], w, s, precision=prec, n_max=N, p_max=P_MODES)
    for i in range(warmup):
        plan.rbm_step(pos, q, P_MODES, seed=1, step=1000000 + i)
    torch.cuda.synchronize()
    if timing:
        plan.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        plan.rbm_step(pos, q, P_MODES, seed=1, step=i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timers = {}
    if timing:
        for name, idx in (("sweep", q2d.TIMER_SWEEP), ("agg", q2d.TIMER_AGG),
                          ("sort", q2d.TIMER_SORT), ("k0", q2d.TIMER_K0), ("call", q2d.TIMER_CALL)):
            ms, cnt = plan.timing_read(idx)
            timers[name] = (ms, cnt)
        plan.timing_enable(False)
    # one reference step for the FP32/FP64 comparison
    phi, F, E, modes = plan.rbm_step(pos, q, P_MODES, seed=1, step=0)
    torch.cuda.synchronize()
    out = dict(ms_per_step=(t1 - t0) * 1e3 / steps, timers=timers,
               F=F.double().cpu().numpy(), modes=modes.cpu().numpy())
    plan.close()
    return out


def cpu_baseline(c, w, s, modes):
    """The oracle's O(N) recursion (plain C, FP64), one thread, all particles,
    the first P_s of the step's modes; scaled to the full batch."""
    from oracle import lattice, soewald2d
    from oracle import recursion as o3
    o3.build()
    box, alpha = c["box"], c["alpha"]
    H = lattice.H_direct(box[0], box[1], alpha)
    Ps = 10
    wt = soewald2d.rb_weights(P_MODES, H, box[0], box[1])[:Ps]
    pos = c["pos"].astype(np.float64)
    q = c["q"].astype(np.float64)
    t0 = time.perf_counter()
    o3.long_range(pos, q, box, alpha, w, s, modes[:Ps], wt, include_self_pair=False, diag=0.0,
                  nthreads=1)
    t = time.perf_counter() - t0
    t_full = t * P_MODES / Ps
    return dict(value=len(q) / t_full, unit="particle-force evals/s", cores=1, kind="oracle",
                sample="O3 FP64 recursion over all %d particles for %d of the %d modes "
                       "(%.1f s), scaled by %d/%d" % (len(q), Ps, P_MODES, t, P_MODES, Ps),
                host_cpu=_cpu_model(), host_threads=os.cpu_count())


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def traffic_from_profile(scan_src):
    """HBM bytes per sweep launch from committed rocprofv3 counters, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha256") != hashlib.sha256(open(scan_src, "rb").read()).hexdigest():
        return None
    return d.get("bytes_per_launch")


def calibrate_copy():
    """A plain device-to-device copy of 256 MiB, repeated 4 times: the known
    traffic (256 MiB read + 256 MiB written per launch) calibrates the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 256 * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import workloads as wl
    w, s = soe_table(M_SOE)
    c32 = wl.make_config(3, dtype=np.float32)
    N = len(c32["q"])
    r32 = run_gpu("fp32", c32, w, s, args.steps, args.warmup, timing=True)
    ms = r32["ms_per_step"]
    fl = flops_per_mode_particle(M_SOE) * P_MODES * N
    # the sweep runs as several launches per step (whole 64-mode groups, then
    # power-of-two bands of the remaining modes): FLOP of all of them over
    # their summed time, i.e. average FLOP per launch over average duration
    sw_ms, sw_cnt = r32["timers"]["sweep"]
    per_step = max(sw_cnt, 1) / args.steps
    sweep_ms = sw_ms / max(sw_cnt, 1)
    achieved = fl / (sw_ms / args.steps * 1e-3) / 1e12
    scan_src = os.path.join(ROOT, "paper_2403_01521_amd", "csrc", "q2d_scan.hip")
    res = {
        "metric": METRIC,
        "value": N / (ms * 1e-3),
        "unit": "particle-force evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rbm_step N=1e6 slab 600x600x10 surface-excess, alpha=0.1, "
                               "P=100, M=16, FP32 scans (FP64 k=0, carries, energy)",
                   "N": N, "P": P_MODES, "M": M_SOE, "alpha": 0.1, "box": [600, 600, 10]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic_from_profile(scan_src),
                     "kernel": "k_sweep<float,8>", "flop_per_launch": fl / per_step,
                     "launch_ms": sweep_ms, "launches_per_step": per_step},
        "step_breakdown_ms": {k: v[0] / args.steps for k, v in r32["timers"].items()},
        "step_flop_frac": fl / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
    }
    if not args.no_fp64:
        c64 = dict(c32)
        c64["pos"] = c32["pos"].astype(np.float64)
        c64["q"] = c32["q"].astype(np.float64)
        r64 = run_gpu("fp64", c64, w, s, max(3, args.steps // 4), 2, timing=False)
        res["fp64_ms_per_step"] = r64["ms_per_step"]
        res["fp64_value"] = N / (r64["ms_per_step"] * 1e-3)
        res["fp32_over_fp64_speedup"] = r64["ms_per_step"] / ms
        assert np.array_equal(r64["modes"], r32["modes"])
        d = r32["F"] - r64["F"]
        res["fp32_vs_fp64_force_rel_rms"] = float(np.linalg.norm(d) / np.linalg.norm(r64["F"]))
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(c32, w, s, r32["modes"])
    print(json.dumps(res))


if __name__ == "__main__":
    main()
