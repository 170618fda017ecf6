#!/usr/bin/env python3
"""Benchmark of the SPH neighbour loops on one MI355X.

Workload: the clustered 128^3 set -- 2,097,152 particles drawn from a
lognormal density field (sigma_ln = 1.5, Gaussian-smoothed white noise on a
64^3 grid) in a periodic unit box, u ~ U(0.5, 1.5), v ~ N(0, 0.1), float32.
A step is one pass of the whole hot path on resident device data: binning
(counting sort + task lists), density with Newton iteration on h, gradient,
force.  Timed with HIP events on the library's stream (torch's current
stream), whole steps between synchronisations.

Metric: pair interactions per second of the density and force loops
(useful pairs: r < H_i for density, r < max(H_i, H_j) for force) over the
whole step time.  Reported alongside: per-loop rates, the fraction of the
FP32 vector peak reached by the arithmetic of the useful pairs, the same
step with one kernel launch per tile task (the per-task offload baseline),
the roofline entry of the dominant kernel and the FP64 oracle on the host
cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FLOPs per useful pair, counted on the arithmetic each loop performs for a
# pair inside the support (FMA = 2, add/mul/min/max = 1, sqrt/rsqrt/rcp = 1).
F_DENS = 59.0     # full density sums (n, dn/dh, d2n/dlogh2, rho, drho/dh, div v, curl v)
F_NEWTON = 29.0   # each additional Newton sweep (n and its first two log-h derivatives)
F_GRAD = 33.0     # the gradient loop on its own
F_FORCE = 67.0
F_GRAD_JOINT = 17.0  # a gradient pair inside the joint gradient/force body
                     # (distance, 1/r, v.r and the signal speed shared with force)
PEAK_FP32 = 157.3e12   # MI355X published FP32 vector peak (packed FMA)
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_clustered_128cubed.json")


def sources_digest():
    """sha256 over the library's kernel sources (csrc/*.hip, *.h), sorted by name."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_14538_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy), or None
    when the kernel sources changed since those counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_dispatch")


def cpu_baseline(parts):
    """The FP64 oracle on the host cores: density (Newton) for every
    particle, force for a random sample; pairs per second of both."""
    from oracle import oracle as O
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    prm = O.Params(ncell=128)
    t0 = time.time()
    d = O.density(parts, prm)
    t_d = time.time() - t0
    P_d = float(np.sum(d["nngb"]))
    rng = np.random.default_rng(5)
    ns = 200000
    idx = np.sort(rng.choice(parts.n, ns, replace=False))
    t0 = time.time()
    f = O.force(parts, d, prm, idx=idx)
    t_f = time.time() - t0
    P_f = float(np.sum(f["nint"][idx]))
    rate = (P_d + P_f) / (t_d + t_f)
    return {"value": rate, "unit": "pair interactions/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, cell-list mode: density with Newton on all %d particles "
                      "(%.1f s) + force on %d random particles (%.1f s)" % (parts.n, t_d, ns, t_f)}


def per_task_step(S, dp, n_tiles, tuning):
    """One step with one kernel launch per tile task (the same tile bodies
    and the same work as the batched step: bin, density, and one joint
    gradient + force pass): the per-task offload baseline."""
    import torch
    log("per-task launch step (%d gradient/force tasks)" % n_tiles)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pt = S.Plan(flags=S.PER_TASK_LAUNCH, **tuning)
    torch.cuda.synchronize()
    ev0.record()
    pt.step(dp)
    ev1.record()
    torch.cuda.synchronize()
    log("  per-task step done")
    return ev0.elapsed_time(ev1) / 1e3


def copy_probe(nbytes):
    """A plain device copy of nbytes, five times: the reference for scaling
    the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy probe: 5 copies of %d bytes" % nbytes)


def run(args):
    import torch
    from paper_2505_14538_amd import swsph as S
    from paper_2505_14538_amd import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    log("generating clustered workload")
    parts = W.clustered()
    dp = S.to_device(parts)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # the batched path: the whole step captured in a HIP graph by the library
    # (bin + three persistent loop launches), replayed each step.  The plan's
    # default options (tile sizes, LDS capacities, task order, search leaf
    # size) are the library autotuner's choice on this workload; --autotune
    # runs the autotuner first (untimed, like a warm-up)
    plan = S.Plan()
    defaults = plan.tuning()
    tuning = {}
    if args.autotune:
        tuning = plan.autotune(dp)
        log("autotuned: %s" % tuning)
    for _ in range(args.warmup):
        d, g, f = plan.step(dp)
    torch.cuda.synchronize()
    log("warm-up done")
    ev0.record()
    for _ in range(args.steps):
        d, g, f = plan.step(dp)
    ev1.record()
    torch.cuda.synchronize()
    t_step = ev0.elapsed_time(ev1) / 1e3 / args.steps
    st = plan.stats()
    if st["code"] != 0:
        raise SystemExit("device status %s" % st)
    nngb = d["nngb"].to(torch.int64).sum().item()
    nint = f["nint"].to(torch.int64).sum().item()
    P_d, P_f, P_g = float(nngb), float(nint), float(nngb)
    sweeps = st["newton_sweeps"] / max(1, st["n_tiles_dens"])   # counters cover the last step
    value = (P_d + P_f) / t_step
    flops = P_d * (F_DENS + max(0.0, sweeps - 1) * F_NEWTON) + P_g * F_GRAD_JOINT + P_f * F_FORCE
    frac_peak = flops / t_step / PEAK_FP32
    log("step %.3f ms  P_d %.3e P_f %.3e  sweeps/tile %.2f" % (t_step * 1e3, P_d, P_f, sweeps))

    # per-launch duration of the loop kernels: the same step run eagerly with
    # HIP events recorded by the library on this stream around every launch
    tp = S.Plan(flags=S.TIMING, **tuning)
    tp.step(dp)
    torch.cuda.synchronize()
    tp.reset_timers()
    for _ in range(args.steps):
        tp.step(dp)
    kt = tp.kernel_times()
    log("kernel ms per launch: " + ", ".join("%s %.3f (%d)" % (k, v["ms"], v["launches"])
                                             for k, v in kt.items()))

    t_pt = value_pt = None
    if not args.no_per_task:
        t_pt = per_task_step(S, dp, st["n_tiles"], tuning)
        value_pt = (P_d + P_f) / t_pt
        log("per-task launch step %.1f ms" % (t_pt * 1e3))


    # roofline of the dominant kernel (largest share of the step); the
    # density kernel runs once plus its fix-up passes per step, so its
    # algorithmic FLOPs per launch are the step's density FLOPs divided by
    # the launches per step
    dom = max(kt, key=lambda k: kt[k]["ms"] * kt[k]["launches"])
    k_ms = kt[dom]["ms"]
    per_step = kt[dom]["launches"] / args.steps
    per_launch_flops = {"density": P_d * (F_DENS + max(0.0, sweeps - 1) * F_NEWTON),
                        "gradient+force": P_g * F_GRAD_JOINT + P_f * F_FORCE}[dom] / per_step
    achieved = per_launch_flops / (k_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / (PEAK_FP32 / 1e12),
                # counters were taken with the default options
                "traffic": measured_traffic({"density": "k_loop<0",
                                             "gradient+force": "k_loop<2"}[dom])
                           if not tuning or tuning == defaults else None,
                "kernel": "k_loop<%s> (loop kernel of the %s loop)" % (dom, dom),
                "kernel_ms": k_ms}
    res = {
        "metric": "pair interactions/s (density+force), % FP32 peak; batched vs per-task launch",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "clustered 128^3: 2,097,152 particles, lognormal field "
                               "sigma_ln=1.5 on 64^3 grid, periodic unit box, FP32",
                   "n": parts.n, "loops": "bin+density(Newton)+gradient+force",
                   "tuning": tuning or "defaults"},
        "pairs": {"density": P_d, "gradient": P_g, "force": P_f},
        # per loop: useful pairs over the loop kernels' time per step (the
        # density loop runs its kernel once plus its fix-up passes)
        # (the gradient and force loops run in one kernel: their pairs together)
        "rates": {k: {"pairs_per_s": {"density": P_d, "gradient+force": P_g + P_f}[k] /
                      (kt[k]["ms"] * kt[k]["launches"] / args.steps * 1e-3),
                      "kernel_ms_per_launch": kt[k]["ms"],
                      "launches_per_step": kt[k]["launches"] / args.steps}
                  for k in kt if k in ("density", "gradient+force")},
        "frac_fp32_peak": frac_peak,
        "newton_sweeps_per_tile": sweeps,
        "per_task_launch": None if args.no_per_task else {
            "value": value_pt, "ms_per_step": t_pt * 1e3, "batched_speedup": t_pt / t_step},
        "roofline": roofline,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(parts)
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner on the workload before timing")
    ap.add_argument("--no-per-task", action="store_true",
                    help="skip the per-task launch baseline (for profiler runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        raise SystemExit("bench.py runs on one GPU only: --gpus must be 1 (sharding the loops "
                         "over several GPUs is not implemented)")
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    run(args)


if __name__ == "__main__":
    main()
