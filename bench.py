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
whole step time.  Reported alongside: per-loop rates and fractions of the
FP32 vector peak reached by the arithmetic of the useful pairs, the same
step with a flat launch (static schedule) and with one kernel launch per
tile task (the per-task offload baseline), a warm-started step (the previous
h as the guess), the autotuner's choice, the roofline entry of the dominant
kernel (with FP32 VALU counter figures and HBM traffic from the committed
rocprofv3 summaries while the kernel sources match them), the many-boxes set
(256 boxes in one launch per loop, and all three loops of every box in one
launch), the differentiation set (forward and
adjoint), the Gresho-Chan vortex integrated with the switch loops, and the
FP64 oracle on the host cores.
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
F_LIGHT = 36.0    # one Halley sweep over a particle's list: n, dn/dlogh, sum q^2 w''
F_FULL = 66.0     # the final full density sums (n, dn/dh, rho, drho/dh, div v, curl v)
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
    """sha256 over the library's kernel sources (the digest the committed
    counter summaries carry)."""
    from paper_2505_14538_amd.profsum import sources_digest as digest
    return digest()


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
    ns = 1000000
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


COUNTERS_FILE = os.path.join(ROOT, "profiles", "valu_clustered_128cubed.json")


def measured_counters(kernel):
    """FP32 VALU counter figures per dispatch of `kernel` from the committed
    rocprofv3 summary (SQ_INSTS_VALU_FLOPS_FP32 and the instruction counts),
    or None when the kernel sources changed since they were taken."""
    try:
        with open(COUNTERS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_digest():
        return None
    return t.get("kernels", {}).get(kernel)


def timed_steps(plan, dp, steps, warmup):
    """Mean ms of `steps` graph-replayed steps after `warmup` untimed ones."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = None
    for _ in range(warmup):
        out = plan.step(dp)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        out = plan.step(dp)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, out


def step_flops(P_d, P_f, sweeps):
    """Useful-pair FLOPs of one step per loop: density (Halley sweeps over the
    lists plus the final full sums) and the joint gradient/force loop."""
    return {"density": P_d * (F_FULL + sweeps * F_LIGHT),
            "gradient+force": P_d * F_GRAD_JOINT + P_f * F_FORCE}


def pairs_of(d, f):
    import torch
    return (float(d["nngb"].to(torch.int64).sum().item()),
            float(f["nint"].to(torch.int64).sum().item()))


def many_boxes_leg(S, W, args):
    """The many-boxes set (256 independent periodic boxes, ~4.7M particles):
    one graph-replayed step of all boxes, every loop one persistent launch
    over the tiles of all boxes; then the single-launch step (the density,
    gradient and force loops of every box in one launch)."""
    log("many-boxes workload")
    parts = W.many_boxes()
    dp = S.to_device(parts)
    plan = S.Plan()
    ms, (d, g, f) = timed_steps(plan, dp, args.steps, args.warmup)
    st = plan.stats()
    if st["code"] != 0:
        raise SystemExit("many boxes: device status %s" % st)
    P_d, P_f = pairs_of(d, f)
    sweeps = st["newton_sweeps"] / max(1, st["n_tiles_dens"])
    fl = step_flops(P_d, P_f, sweeps)
    log("many boxes: %.3f ms per step" % ms)
    # the same step with all three loops of every box in one launch
    single = S.Plan(flags=S.SINGLE_LAUNCH)
    ms1, (d1, g1, f1) = timed_steps(single, dp, args.steps, args.warmup)
    st1 = single.stats()
    if st1["code"] != 0:
        raise SystemExit("many boxes, single launch: device status %s" % st1)
    Q_d, Q_f = pairs_of(d1, f1)
    log("many boxes, single launch: %.3f ms per step (%d of %d gradient/force tiles redone)"
        % (ms1, st1["single_redo"], st1["n_tiles"]))
    return {"workload": "256 periodic unit boxes, N_b log-uniform in [2048, 65536] rounded to "
                        "cubes, jittered lattices, FP32", "n": parts.n, "n_box": parts.n_box,
            "ms_per_step": ms, "value": (P_d + P_f) / (ms * 1e-3),
            "unit": "pair interactions/s",
            "frac_fp32_peak": sum(fl.values()) / (ms * 1e-3) / PEAK_FP32,
            "newton_sweeps_per_tile": sweeps,
            "single_launch": {"ms_per_step": ms1, "value": (Q_d + Q_f) / (ms1 * 1e-3),
                              "redone_tiles": st1["single_redo"], "tiles": st1["n_tiles"],
                              "vs_separate_launches": ms / ms1}}


def diff_leg(S, W, args):
    """The differentiation set (64^3 jittered lattice): the FP32 forward
    (bin, density with Newton, force) and the hand-written adjoint."""
    import torch
    log("differentiation workload")
    parts, w, c = W.diff()
    dp = S.to_device(parts)
    plan = S.Plan()
    gw = torch.as_tensor(w, device="cuda")
    gc = torch.as_tensor(c, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd, bwd = [], []
    for rep in range(args.warmup + args.steps):
        ev[0].record()
        plan.bin(dp)
        d = plan.density(dp)
        f = plan.force(dp, d)
        ev[1].record()
        plan.bin(dp)
        plan.force_backward(dp, d, gw[:, 0].contiguous(), gw[:, 1].contiguous(),
                            gw[:, 2].contiguous(), gc)
        ev[2].record()
        torch.cuda.synchronize()
        if rep >= args.warmup:
            fwd.append(ev[0].elapsed_time(ev[1]))
            bwd.append(ev[1].elapsed_time(ev[2]))
    st = plan.stats()
    if st["code"] != 0:
        raise SystemExit("differentiation: device status %s" % st)
    log("diff: forward %.3f ms, adjoint %.3f ms" % (np.median(fwd), np.median(bwd)))
    return {"workload": "64^3 jittered lattice, v ~ N(0, 0.1), u ~ U(0.5, 1.5), FP32; "
                        "loss sum w.a + c du/dt", "n": parts.n,
            "forward_ms": float(np.median(fwd)), "adjoint_ms": float(np.median(bwd))}


def gresho_leg(args):
    """The Gresho-Chan vortex (Sec. 3.1, Eq. 27-28) at the resolution of the
    paper's Fig. 6, 128^3 particles, integrated to t = 0.1 with the switch
    loops: time per leapfrog step and the error of the binned profiles."""
    import torch
    from paper_2505_14538_amd import gresho as G
    from paper_2505_14538_amd import workloads as W
    log("gresho 128^3 to t = 0.1")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    marks = {}

    def on_step(k, t):
        if k == 1:
            ev[0].record()
        marks["last"] = k

    out = G.run(nside=128, t_end=0.1, on_step=on_step)
    ev[1].record()
    torch.cuda.synchronize()
    steps = out["steps"]
    ms = ev[0].elapsed_time(ev[1]) / max(1, steps - 1)
    pr = G.profile(out["x"], out["y"], out["vx"], out["vy"], out["P"])
    va, Pa = W.gresho_profiles(pr["r"])
    inner = pr["r"] < 0.45
    log("gresho: %d steps, %.3f ms per step" % (steps, ms))
    return {"workload": "Gresho-Chan vortex, 128^3 lattice, switches on, leapfrog to t = 0.1",
            "n": out["n"], "steps": steps, "dt": out["dt"], "ms_per_step": ms,
            "v_phi_mean_abs_err": float(np.mean(np.abs(pr["v"] - va)[inner])),
            "pressure_mean_abs_err": float(np.mean(np.abs(pr["P"] - Pa)[inner])),
            "energy_drift": (out["energy"] - out["energy0"]) / out["energy0"]}


def run(args):
    import torch
    from paper_2505_14538_amd import swsph as S
    from paper_2505_14538_amd import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    log("generating clustered workload")
    parts = W.clustered()
    dp = S.to_device(parts)

    # the batched path: the whole step captured in a HIP graph by the library
    # (bin + persistent loop launches), replayed each step, with the plan's
    # default options (tile sizes, LDS capacities, task order, search leaf
    # size); the autotune leg below reports the autotuner's own choice
    plan = S.Plan()
    defaults = plan.tuning()
    ms, (d, g, f) = timed_steps(plan, dp, args.steps, args.warmup)
    t_step = ms * 1e-3
    log("warm-up and timed steps done")
    st = plan.stats()
    if st["code"] != 0:
        raise SystemExit("device status %s" % st)
    P_d, P_f = pairs_of(d, f)
    P_g = P_d
    sweeps = st["newton_sweeps"] / max(1, st["n_tiles_dens"])   # counters cover the last step
    value = (P_d + P_f) / t_step
    fl = step_flops(P_d, P_f, sweeps)
    frac_peak = sum(fl.values()) / t_step / PEAK_FP32
    log("step %.3f ms  P_d %.3e P_f %.3e  sweeps/tile %.2f" % (t_step * 1e3, P_d, P_f, sweeps))

    # per-launch duration of the loop kernels: the same step run eagerly with
    # HIP events recorded by the library on this stream around every launch
    tp = S.Plan(flags=S.TIMING)
    tp.step(dp)
    torch.cuda.synchronize()
    tp.reset_timers()
    for _ in range(args.steps):
        tp.step(dp)
    kt = tp.kernel_times()
    log("kernel ms per launch: " + ", ".join("%s %.3f (%d)" % (k, v["ms"], v["launches"])
                                             for k, v in kt.items()))
    loop_pairs = {"density": P_d, "gradient+force": P_g + P_f}
    loop = {}
    for k in ("density", "gradient+force"):
        if k not in kt:
            continue
        per_step_ms = kt[k]["ms"] * kt[k]["launches"] / args.steps
        loop[k] = {"pairs_per_s": loop_pairs[k] / (per_step_ms * 1e-3),
                   "kernel_ms_per_step": per_step_ms,
                   "kernel_ms_per_launch": kt[k]["ms"],
                   "launches_per_step": kt[k]["launches"] / args.steps,
                   "flops_per_step": fl[k],
                   "frac_fp32_peak": fl[k] / (per_step_ms * 1e-3) / PEAK_FP32}
    tests = {"density": st["pairs_tested"][0] / max(1, st["pairs_inside"][0]),
             "gradient+force": st["pairs_tested"][2] / max(1, st["pairs_inside"][2])}
    for k in loop:
        loop[k]["candidate_tests_per_useful_pair"] = tests[k]

    legs = not args.only_step
    flat_ms = warm_ms = warm_sweeps = tuned = tuned_ms = None
    if legs:
        # the same step with a flat launch (one launch per loop, tasks dealt
        # round-robin: a static schedule, no queue)
        flat_ms, _ = timed_steps(S.Plan(flags=S.FLAT_LAUNCH), dp, args.steps, 1)
        log("flat launch step %.3f ms" % flat_ms)

        # warm start: the converged h of the previous step as the guess
        hprev = d["h"].clone()
        dpw = S.to_device(parts)
        dpw.h = hprev
        pw = S.Plan()
        warm_ms, _ = timed_steps(pw, dpw, args.steps, args.warmup)
        stw = pw.stats()
        warm_sweeps = stw["newton_sweeps"] / max(1, stw["n_tiles_dens"])
        log("warm-start step %.3f ms, sweeps/tile %.2f" % (warm_ms, warm_sweeps))

        # the library's autotuner on this workload (untimed search), then the
        # step with its choice
        pa = S.Plan()
        tuned = pa.autotune(dp)
        tuned_ms, _ = timed_steps(pa, dp, args.steps, 1)
        log("autotuned %s: %.3f ms" % (tuned, tuned_ms))

    t_pt = value_pt = None
    if legs and not args.no_per_task:
        t_pt = per_task_step(S, dp, st["n_tiles"], {})
        value_pt = (P_d + P_f) / t_pt
        log("per-task launch step %.1f ms" % (t_pt * 1e3))

    # roofline of the dominant kernel (largest share of the step); the
    # density kernel runs once plus its fix-up passes per step, so its
    # algorithmic FLOPs per launch are the step's density FLOPs divided by
    # the launches per step
    dom = max(loop, key=lambda k: loop[k]["kernel_ms_per_step"])
    k_ms = loop[dom]["kernel_ms_per_launch"]
    per_launch_flops = fl[dom] / loop[dom]["launches_per_step"]
    achieved = per_launch_flops / (k_ms * 1e-3) / 1e12
    kname = {"density": "k_loop<0", "gradient+force": "k_loop<2"}[dom]
    cnt = measured_counters(kname)
    counters = None
    if cnt is not None:
        counters = {"valu_fp32_flops_per_launch": cnt["valu_flops_fp32"],
                    "valu_fp32_tflops": cnt["valu_flops_fp32"] / (k_ms * 1e-3) / 1e12,
                    "useful_share": per_launch_flops / cnt["valu_flops_fp32"],
                    "valu_insts_per_useful_pair":
                        cnt["valu_insts"] * loop[dom]["launches_per_step"] / loop_pairs[dom],
                    "source": os.path.relpath(COUNTERS_FILE, ROOT)}
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / (PEAK_FP32 / 1e12),
                "traffic": measured_traffic(kname),
                "kernel": "k_loop<%s> (loop kernel of the %s loop)" % (dom, dom),
                "kernel_ms": k_ms, "counters": counters}
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
                   "tuning": defaults},
        "pairs": {"density": P_d, "gradient": P_g, "force": P_f},
        "frac_fp32_peak": frac_peak,
        "newton_sweeps_per_tile": sweeps,
        "loops": loop,
        "flat_launch": None if not legs else {
            "ms_per_step": flat_ms, "value": (P_d + P_f) / (flat_ms * 1e-3),
            "batched_speedup": flat_ms * 1e-3 / t_step},
        "per_task_launch": None if t_pt is None else {
            "value": value_pt, "ms_per_step": t_pt * 1e3, "batched_speedup": t_pt / t_step},
        "warm_start": None if not legs else {
            "ms_per_step": warm_ms, "value": (P_d + P_f) / (warm_ms * 1e-3),
            "newton_sweeps_per_tile": warm_sweeps},
        "autotune": None if not legs else {
            "choice": tuned, "matches_defaults": tuned == defaults, "ms_per_step": tuned_ms},
        "roofline": roofline,
    }
    if legs and not args.no_extra:
        res["many_boxes"] = many_boxes_leg(S, W, args)
        res["differentiation"] = diff_leg(S, W, args)
        res["gresho"] = gresho_leg(args)
    if legs and not args.no_cpu:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(parts)
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the many-boxes, differentiation and Gresho legs")
    ap.add_argument("--only-step", action="store_true",
                    help="only the batched and the timed eager step (profiler runs)")
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
