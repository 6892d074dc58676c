"""Benchmark: random-batch SOE Ewald2D long-range step at N = 1e6 on one MI355X.

Workload (configuration 3 of workloads.py): 1e6 charges +-1 in a 600 x 600 x 10
slab with a 10% surface excess of +1 near z = 0 and -1 near z = 10, alpha = 0.1,
P = 100 importance-sampled Fourier modes per step, SOE with M = 16 terms.
One step = one q2d_rbm_step call: mode sampling, z-sort, the k != 0 scans,
the FP64 k = 0 term and the reductions, with inputs resident in HBM and a
different (seed, step) -- hence different modes -- every step.

Prints one JSON line:
  value        particle-force evaluations per second (N / step time), FP32 path,
               W untimed + K timed steps (default 10 + 100)
  roofline     the hot kernel (k != 0 sweep): algorithmic FLOP per launch over its
               average launch time from HIP events recorded on the plan's stream
               during the timed steps (the only events recorded there), against
               the MI355X FP32 vector peak
  cpu_baseline the FP64 O(N) recursion of the oracle on one host core, on all
               1e6 particles but a subset of the modes, scaled to P = 100
Extra fields: a per-kernel-family breakdown (separate pass with all timers),
the FP64 path on the same GPU and the FP32/FP64 speedup, the relative RMS
difference of FP32 and FP64 forces for identical modes, the FP64 exact-k SOE
sum over all 42,184 modes with e^{-k^2/4 alpha^2} >= 1e-16 (time, and as the
reference of the random-batch force error per draw and of the running mean over
the K draws), the oracle on all host cores, and the 256-replica batch of
configuration 5 (aggregate and per-replica evaluations/s, eager and replayed
as a hipGraph, against one single-system call per replica).

Also: the same workload with the model-reduced M = 10 SOE table (about the
sup error the Talbot rule needs M = 16 for): its step time and sweep roofline,
FP32 against FP64 on that table, and its FP64 forces against the M = 16 ones.

And a whole force evaluation in the O(N) regime of Sec. 4.1: alpha from
eq. 59, r_c = 4/alpha, the random-batch long range plus the cell-list real
space on the same slab.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64]
                       [--no-exact] [--no-reduced] [--no-short] [--no-replicas]
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
SEED = 1


def flops_per_mode_particle(M):
    """Algorithmic FLOP per (mode, particle): per exponent beta (M SOE terms and
    beta = k) a forward and a backward complex recurrence step and the two
    complex combines (4 complex FMA = 32 FLOP), plus ~20 FLOP of phase and
    force assembly per mode."""
    return 32 * (M + 1) + 20


def soe_table(M, reduced=False):
    """The SOE table of the run from the library's own host fit: the Talbot
    rule (the configuration's M = 16 table) or the model-reduced fit."""
    import paper_2403_01521_amd as q2d
    w, s, err = q2d.soe_fit_reduced(M) if reduced else q2d.soe_fit(M)
    return w, s, err


def exact_modes(Lx, Ly, alpha, kc):
    """Every reciprocal vector 0 < |k| <= k_c (full lattice) with its weight
    (pi/A) e^{-k^2/4 alpha^2}: the exact-k reference list."""
    mx_max, my_max = int(kc * Lx / (2 * np.pi)), int(kc * Ly / (2 * np.pi))
    mx, my = np.meshgrid(np.arange(-mx_max, mx_max + 1), np.arange(-my_max, my_max + 1),
                         indexing="ij")
    kx, ky = 2 * np.pi * mx / Lx, 2 * np.pi * my / Ly
    k2 = kx * kx + ky * ky
    keep = (k2 > 0) & (k2 <= kc * kc)
    m = np.stack([mx[keep], my[keep]], axis=1).astype(np.int32)
    return m, np.pi / (Lx * Ly) * np.exp(-k2[keep] / (4 * alpha * alpha))


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def rel(a, b):
    import torch
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def time_steps(plan, pos, q, steps, warmup, mask, stride=1):
    """Wall time per step over `steps` calls (steps 0..steps-1), after `warmup`
    untimed calls with other step numbers; timers of `mask` recorded on every
    `stride`-th call (each recorded event can delay the next launch)."""
    import torch
    for i in range(warmup):
        plan.rbm_step(pos, q, P_MODES, seed=SEED, step=1000000 + i)
    torch.cuda.synchronize()
    plan.timing_enable(mask)
    plan.timing_stride(stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        plan.rbm_step(pos, q, P_MODES, seed=SEED, step=i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps


def read_timers(plan):
    import paper_2403_01521_amd as q2d
    out = {}
    for name, idx in (("sweep", q2d.TIMER_SWEEP), ("agg", q2d.TIMER_AGG),
                      ("sort", q2d.TIMER_SORT), ("k0", q2d.TIMER_K0), ("call", q2d.TIMER_CALL)):
        out[name] = plan.timing_read(idx)
    plan.timing_enable(0)
    return out


def half_lattice(m, wt):
    """k and -k give equal contributions: keep one of each pair, doubled weight."""
    keep = (m[:, 0] > 0) | ((m[:, 0] == 0) & (m[:, 1] > 0))
    return m[keep], 2.0 * wt[keep]


def cpu_baseline(c, w, s, modes):
    """The oracle's O(N) recursion (plain C, FP64), one thread, all particles,
    the first P_s of the step's modes; scaled to the full batch.  Also on all
    host threads, and the direct pair sums (O2) on a few targets, scaled to
    N targets (the plain O(N^2)-per-mode cost)."""
    from oracle import lattice, soewald2d
    from oracle import recursion as o3
    o3.build()
    box, alpha = c["box"], c["alpha"]
    H = lattice.H_direct(box[0], box[1], alpha)
    wt = soewald2d.rb_weights(P_MODES, H, box[0], box[1])
    pos = c["pos"].astype(np.float64)
    q = c["q"].astype(np.float64)
    N = len(q)
    Ps = 10
    t0 = time.perf_counter()
    o3.long_range(pos, q, box, alpha, w, s, modes[:Ps], wt[:Ps], include_self_pair=False,
                  diag=0.0, nthreads=1)
    t1 = time.perf_counter() - t0
    nthr = effective_cores()
    Pa = 40
    t0 = time.perf_counter()
    o3.long_range(pos, q, box, alpha, w, s, modes[:Pa], wt[:Pa], include_self_pair=False,
                  diag=0.0, nthreads=nthr)
    ta = time.perf_counter() - t0
    tg, Po = 2, 5
    t0 = time.perf_counter()
    soewald2d.long_range(pos, q, box, alpha, w, s, modes[:Po], wt[:Po],
                         targets=np.arange(tg), include_self_pair=False, diag=0.0)
    to = time.perf_counter() - t0
    return dict(value=N / (t1 * P_MODES / Ps), unit="particle-force evals/s", cores=1,
                kind="oracle",
                sample="O3 FP64 recursion over all %d particles for %d of the %d modes "
                       "(%.1f s), scaled by %d/%d" % (N, Ps, P_MODES, t1, P_MODES, Ps),
                all_threads=dict(value=N / (ta * P_MODES / Pa), threads=nthr,
                                 sample="O3, OpenMP over modes, %d of %d modes (%.1f s)"
                                        % (Pa, P_MODES, ta)),
                direct_pairs_o2=dict(value=N / (to * (N / tg) * (P_MODES / Po)), threads=1,
                                     sample="O2 direct pair sums (numpy) for %d targets x %d "
                                            "modes (%.1f s), scaled to %d targets x %d modes"
                                            % (tg, Po, to, N, P_MODES)),
                host_cpu=_cpu_model(), host_threads=nthr,
                host_cores_note="threads = cores this process may run on: the CPU affinity "
                                "mask, capped by the cgroup CPU quota (os.cpu_count() = %s)"
                                % os.cpu_count())


def replicas_report(w, s, steps):
    """Configuration 5: 256 replicas of uneven N (log-uniform 1e3..2e4), P = 64,
    FP32, one batch step per call; eager calls and graph replays, against the
    same work done by one single-system call per replica."""
    import torch
    import paper_2403_01521_amd as q2d
    import workloads as wl
    c = wl.make_replicas(dtype=np.float32)
    P = c["P"]
    counts, boxes = c["counts"], c["boxes"]
    pos = torch.tensor(c["pos"], device="cuda")
    q = torch.tensor(c["q"], device="cuda")
    b = q2d.Batch(boxes, counts, c["alpha"], w, s, precision="fp32", p_max=P)
    t0 = time.perf_counter()
    S = b.tune(pos, q, P, seed=SEED)
    tune_s = time.perf_counter() - t0
    cfg = b.config()
    for i in range(3):
        b.rbm_step(pos, q, P, SEED, 1000 + i)
    torch.cuda.synchronize()
    # host time to enqueue the steps (the call returns before the GPU is done)
    # and wall time until they have run
    t0 = time.perf_counter()
    for i in range(steps):
        b.rbm_step(pos, q, P, SEED, i)
    t1 = time.perf_counter()
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / steps
    host_eager = (t1 - t0) * 1e3 / steps
    b.capture(pos, q, P, SEED, 0)
    b.replay(3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.replay(steps)
    t1 = time.perf_counter()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    host_graph = (t1 - t0) * 1e3 / steps
    b.close()
    # the same replicas one call each
    off = np.concatenate([[0], np.cumsum(counts)])
    plans = [q2d.Plan(boxes[r], c["alpha"], w, s, precision="fp32", n_max=int(counts[r]), p_max=P)
             for r in range(len(counts))]
    views = [(pos[off[r]:off[r + 1]], q[off[r]:off[r + 1]]) for r in range(len(counts))]
    for r, pl in enumerate(plans):
        pl.rbm_step(views[r][0], views[r][1], P, q2d.replica_seed(SEED, r), 0)
    torch.cuda.synchronize()
    ns = max(2, steps // 10)
    t0 = time.perf_counter()
    for i in range(ns):
        for r, pl in enumerate(plans):
            pl.rbm_step(views[r][0], views[r][1], P, q2d.replica_seed(SEED, r), i)
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3 / ns
    for pl in plans:
        pl.close()
    Ntot = int(counts.sum())
    best = min(ms_eager, ms_graph)
    per = counts / (best * 1e-3)
    return {"workload": "256 replicas, N log-uniform [1e3, 2e4] (total %d), Lx=Ly=clamp(sqrt(N/0.3),"
                        "30,150), Lz=6, alpha=0.3, P=64, M=16, FP32" % Ntot,
            "tuned_config": cfg, "tune_s": tune_s,
            "segment": S, "ms_per_step_eager": ms_eager, "ms_per_step_graph": ms_graph,
            "host_enqueue_ms_per_step_eager": host_eager,
            "host_enqueue_ms_per_step_graph": host_graph,
            "aggregate_evals_per_s": Ntot / (best * 1e-3),
            "per_replica_evals_per_s": {"min": float(per.min()), "median": float(np.median(per)),
                                        "max": float(per.max())},
            "sequential_single_plans_ms": ms_seq,
            "batch_speedup_vs_sequential": ms_seq / best}


def reduced_report(args, box, alpha, N, pos32, q32, sweep_stride, F32_m16):
    """The same workload and protocol with the model-reduced M = 10 SOE table
    (q2d_soe_fit_reduced: about the sup error the Talbot rule reaches with
    M = 16): step time, sweep roofline, FP32 against FP64 on that table, and
    the FP64 forces of the two tables against each other."""
    import torch
    import paper_2403_01521_amd as q2d
    M = 10
    log("model-reduced SOE, M = %d" % M)
    w, s, err = soe_table(M, reduced=True)
    plan = q2d.Plan(box, alpha, w, s, precision="fp32", n_max=N, p_max=P_MODES)
    ms = time_steps(plan, pos32, q32, args.steps, args.warmup, 1 << q2d.TIMER_SWEEP,
                    stride=sweep_stride)
    sw_ms, sw_cnt = read_timers(plan)["sweep"]
    _, F32, _, m = plan.rbm_step(pos32, q32, P_MODES, seed=SEED, step=0)
    torch.cuda.synchronize()
    plan.close()
    n_sampled = max(args.steps // sweep_stride, 1)
    per_step = max(sw_cnt, 1) / n_sampled
    sweep_ms = sw_ms / max(sw_cnt, 1)
    fl = flops_per_mode_particle(M) * P_MODES * N
    achieved = (fl / per_step) / (sweep_ms * 1e-3) / 1e12
    out = {"M": M, "soe": "model reduction (q2d_soe_fit_reduced), sup error %.2e" % err,
           "ms_per_step": ms, "value": N / (ms * 1e-3),
           "sweep_ms": sweep_ms, "sweep_frac": achieved / PEAK_FP32_TFLOPS}
    if not args.no_fp64:
        w16, s16, _ = soe_table(M_SOE)
        pos64, q64 = pos32.double(), q32.double()
        p64 = q2d.Plan(box, alpha, w, s, precision="fp64", n_max=N, p_max=P_MODES)
        _, F64, _, m64 = p64.rbm_step(pos64, q64, P_MODES, seed=SEED, step=0)
        p64.close()
        p16 = q2d.Plan(box, alpha, w16, s16, precision="fp64", n_max=N, p_max=P_MODES)
        _, F64_16, _, _ = p16.rbm_step(pos64, q64, P_MODES, seed=SEED, step=0)
        p16.close()
        torch.cuda.synchronize()
        assert np.array_equal(m64.cpu().numpy(), m.cpu().numpy())
        out["fp32_vs_fp64_force_rel_rms"] = rel(F32.double(), F64)
        out["fp64_vs_fp64_m16_force_rel_rms"] = rel(F64, F64_16)
    return out


def slab_ball_volume(r, Lz, n=201):
    """Mean volume of a ball of radius r centred in a slab of height Lz and cut
    by its walls (centre uniform over the height)."""
    zs = np.linspace(0.0, Lz, n)
    vol = []
    for z in zs:
        a, b = max(0.0, z - r) - z, min(Lz, z + r) - z
        vol.append(np.pi * (r * r * (b - a) - (b ** 3 - a ** 3) / 3.0))
    return float(np.mean(vol))


def full_step_report(box, N, pos32, q32, steps):
    """A whole force evaluation in the O(N) regime of Sec. 4.1: alpha from
    eq. 59, alpha = (N/V)^{1/3}, r_c = s/alpha with s = 4 (eq. rckc), on the
    bench slab; q2d_rbm_step (P = 100, M = 16) plus q2d_short_range (cell
    list), FP32.  Also the real-space sum at the configuration's own
    alpha = 0.1 (r_c = 40: thousands of neighbours per particle), for scale."""
    import torch
    import paper_2403_01521_amd as q2d
    log("long + short range at the alpha of eq. 59")
    w, s, _ = soe_table(M_SOE)
    V = box[0] * box[1] * box[2]
    rho = N / V
    alpha = rho ** (1.0 / 3.0)
    rc = 4.0 / alpha
    plan = q2d.Plan(box, alpha, w, s, rc=rc, precision="fp32", n_max=N, p_max=P_MODES)

    def timed(fn, n):
        for i in range(3):
            fn(1000 + i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            fn(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    ms_short = timed(lambda i: plan.short_range(pos32, q32), steps)
    ms_long = timed(lambda i: plan.rbm_step(pos32, q32, P_MODES, seed=SEED, step=i), steps)
    ms_step = timed(lambda i: (plan.rbm_step(pos32, q32, P_MODES, seed=SEED, step=i),
                               plan.short_range(pos32, q32)), steps)
    plan.close()
    rc1 = 40.0
    plan1 = q2d.Plan(box, 0.1, w, s, rc=rc1, precision="fp32", n_max=N, p_max=1)
    ms_short1 = timed(lambda i: plan1.short_range(pos32, q32), 3)
    plan1.close()
    return {"alpha": alpha, "r_c": rc, "s": 4.0,
            "neighbours_per_particle": rho * slab_ball_volume(rc, box[2]),
            "short_ms": ms_short, "long_rbm_ms": ms_long, "step_ms": ms_step,
            "step_evals_per_s": N / (ms_step * 1e-3),
            "short_ms_at_alpha_0.1_rc_40": ms_short1,
            "note": "alpha = (N/V)^(1/3) (eq. 59), r_c = 4/alpha (eq. rckc); FP32; "
                    "step = q2d_rbm_step (P=100, M=16) + q2d_short_range"}


def effective_cores():
    """Cores this process may use: its affinity mask, capped by a cgroup v2/v1
    CPU quota when one is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max":
            n = min(n, max(1, int(int(quota) // int(period))))
    except (OSError, ValueError):
        try:
            quota = int(open("/sys/fs/cgroup/cpu/cpu.cfs_quota_us").read())
            period = int(open("/sys/fs/cgroup/cpu/cpu.cfs_period_us").read())
            if quota > 0:
                n = min(n, max(1, quota // period))
        except (OSError, ValueError):
            pass
    return max(1, n)


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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the FP64 exact-k reference (time and random-batch error)")
    ap.add_argument("--no-reduced", action="store_true",
                    help="skip the same step with the model-reduced M = 10 SOE")
    ap.add_argument("--no-short", action="store_true",
                    help="skip the long + short range step at the alpha of eq. 59")
    ap.add_argument("--no-replicas", action="store_true",
                    help="skip the 256-replica batch (configuration 5) report")
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
    import paper_2403_01521_amd as q2d
    import workloads as wl
    w, s, soe_err = soe_table(M_SOE)
    c32 = wl.make_config(3, dtype=np.float32)
    box, alpha = c32["box"], c32["alpha"]
    N = len(c32["q"])
    pos32 = torch.tensor(c32["pos"], device="cuda")
    q32 = torch.tensor(c32["q"], device="cuda")
    plan32 = q2d.Plan(box, alpha, w, s, precision="fp32", n_max=N, p_max=P_MODES)

    # timed steps: only the sweep's events
    log("FP32 random-batch steps: %d warm-up + %d timed" % (args.warmup, args.steps))
    # the sweep's events on every 4th timed step: its launch time is averaged
    # over those, and the other steps carry no events
    sweep_stride = 4 if args.steps >= 8 else 1
    ms = time_steps(plan32, pos32, q32, args.steps, args.warmup, 1 << q2d.TIMER_SWEEP,
                    stride=sweep_stride)
    sw_ms, sw_cnt = read_timers(plan32)["sweep"]
    # breakdown: a separate pass with every timer
    nb = min(args.steps, 20)
    time_steps(plan32, pos32, q32, nb, 0, q2d.TIMING_ALL)
    brk = read_timers(plan32)

    fl = flops_per_mode_particle(M_SOE) * P_MODES * N
    # the sweep runs as one launch per step covering all modes (a 64-mode group
    # and power-of-two bands of the rest): average FLOP per launch over average
    # duration
    # (sampled calls: the plan counts calls from 1, so every stride-th one)
    n_sampled = max(args.steps // sweep_stride, 1)
    per_step = max(sw_cnt, 1) / n_sampled
    sweep_ms = sw_ms / max(sw_cnt, 1)
    achieved = (fl / per_step) / (sweep_ms * 1e-3) / 1e12
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
                               "P=100, M=16; FP32 sweeps, segment aggregates on the fp16 "
                               "matrix cores with split (hi+lo) operands, FP64 k=0 term, "
                               "carries and energy",
                   "N": N, "P": P_MODES, "M": M_SOE, "alpha": alpha, "box": list(box),
                   "soe": "Talbot rule (q2d_soe_fit), sup error %.2e" % soe_err},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic_from_profile(scan_src),
                     "kernel": "k_sweep<float,8>", "flop_per_launch": fl / per_step,
                     "launch_ms": sweep_ms, "launches_per_step": per_step},
        "step_breakdown_ms": {k: v[0] / nb for k, v in brk.items()},
        "step_flop_frac": fl / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
    }

    # random-batch force error against the full k-sum (FP64 exact-k SOE over
    # every mode with e^{-k^2/4 alpha^2} >= 1e-16), per draw and running mean,
    # for the K timed draws (same seeds)
    if not args.no_exact:
        log("FP64 exact-k reference and random-batch error over %d draws" % args.steps)
        kc = 2 * alpha * np.sqrt(np.log(1e16))
        pos64 = pos32.double()
        q64 = q32.double()
        plan_ex = q2d.Plan(box, alpha, w, s, kc=kc, precision="fp64", n_max=N)
        n_modes = plan_ex.info()["n_modes_exact"]
        plan_ex.long_range(pos64, q64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, F_ref, E_ref = plan_ex.long_range(pos64, q64)
        torch.cuda.synchronize()
        t_ex = time.perf_counter() - t0
        # the k != 0 part of the reference force (the j = i constant carries none)
        m_all, wt_all = exact_modes(box[0], box[1], alpha, kc)
        mh, wh = half_lattice(m_all, wt_all)
        _, F_ref_k, _ = plan_ex.modes_eval(pos64, q64,
                                           torch.tensor(mh, dtype=torch.int32, device="cuda"),
                                           torch.tensor(wh, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        plan_ex.close()
        per_draw = []
        run = torch.zeros_like(F_ref)
        run_err = {}
        for i in range(args.steps):
            _, F, _, _ = plan32.rbm_step(pos32, q32, P_MODES, seed=SEED, step=i)
            Fd = F.double()
            per_draw.append(rel(Fd, F_ref))
            run += Fd
            n = i + 1
            if n in (1, 10, 100, args.steps):
                run_err[str(n)] = rel(run / n, F_ref)
        nrm = float(torch.linalg.norm(F_ref))
        nrm_k = float(torch.linalg.norm(F_ref_k))
        res["exact_k_fp64"] = {
            "modes": len(m_all), "half_lattice_modes_computed": int(n_modes),
            "ms": t_ex * 1e3, "evals_per_s": N / t_ex,
            "note": "all k with e^{-k^2/4a^2} >= 1e-16 (k_c = %.4f), FP64, same GPU" % kc}
        res["rb_force_error_vs_full_k"] = {
            "per_draw_rel_rms_mean": float(np.mean(per_draw)),
            "per_draw_rel_rms_max": float(np.max(per_draw)),
            "running_mean_rel_rms": run_err,
            "k_nonzero_part_share": nrm_k / nrm,
            "per_draw_rel_to_k_nonzero_part": float(np.mean(per_draw)) * nrm / nrm_k,
            "draws": args.steps,
            "note": "relative RMS over all particles of F_RB(FP32) - F_exact(FP64); the "
                    "k = 0 part is exact in both, so the error is the k != 0 sampling "
                    "error (also given relative to the k != 0 part's norm)"}

    _, F32, _, m32 = plan32.rbm_step(pos32, q32, P_MODES, seed=SEED, step=0)
    torch.cuda.synchronize()
    r32_modes = m32.cpu().numpy()
    plan32.close()
    if not args.no_reduced:
        res["soe_reduced"] = reduced_report(args, box, alpha, N, pos32, q32, sweep_stride, F32)
    if not args.no_short:
        res["long_plus_short_eq59"] = full_step_report(box, N, pos32, q32,
                                                       max(10, args.steps // 5))
    if not args.no_fp64:
        log("FP64 random-batch steps")
        pos64 = pos32.double()
        q64 = q32.double()
        plan64 = q2d.Plan(box, alpha, w, s, precision="fp64", n_max=N, p_max=P_MODES)
        ms64 = time_steps(plan64, pos64, q64, max(10, args.steps // 4), 3, 0)
        _, F64, _, m64 = plan64.rbm_step(pos64, q64, P_MODES, seed=SEED, step=0)
        torch.cuda.synchronize()
        plan64.close()
        assert np.array_equal(m64.cpu().numpy(), r32_modes)
        res["fp64_ms_per_step"] = ms64
        res["fp64_value"] = N / (ms64 * 1e-3)
        res["fp32_over_fp64_speedup"] = ms64 / ms
        res["fp32_vs_fp64_force_rel_rms"] = rel(F32.double(), F64)
    if not args.no_replicas:
        log("256-replica batch (configuration 5)")
        res["replicas"] = replicas_report(w, s, max(10, args.steps // 5))
    if not args.no_cpu:
        log("oracle timing on the host")
        res["cpu_baseline"] = cpu_baseline(c32, w, s, r32_modes)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
