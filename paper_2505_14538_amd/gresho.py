"""Gresho-Chan vortex end to end on the GPU (Sec. 3.1, Eq. 27-28, Fig. 6).

The paper checks its GPU loops on this steady vortex: particles start with
the azimuthal velocity and pressure of Eq. 27-28, are integrated in time
with the density, gradient and force loops (the SPHENIX switches on), and
at t = 0.1 their velocity and pressure against radius still follow the
analytic profiles.  This driver does the same with the library's calls
only (argument marshalling in Python, every step in HIP kernels):

    kick (dt/2) + drift (dt)   swsph_kick_drift
    bin, density               swsph_bin, swsph_density (h of the last step as guess)
    switches, gradient, force  swsph_gradient_force_sw
    kick (dt/2)                swsph_kick_drift

The time step is fixed at cfl * min_i(H_i / v_sig,i) of the initial state.
"""
from __future__ import annotations

import numpy as np

from . import swsph as S
from . import workloads as W


def profile(x, y, vx, vy, P, nbins: int = 25, rmax: float = 0.5):
    """Mean azimuthal velocity and pressure in radial bins about the axis
    (1/2, 1/2), and their standard deviations."""
    dx, dy = x - 0.5, y - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    vphi = (-dy * vx + dx * vy) / np.maximum(r, 1e-30)
    edges = np.linspace(0.0, rmax, nbins + 1)
    k = np.digitize(r, edges) - 1
    rc, vm, vs, pm, ps = [], [], [], [], []
    for b in range(nbins):
        sel = k == b
        if sel.sum() < 2:
            continue
        rc.append(0.5 * (edges[b] + edges[b + 1]))
        vm.append(vphi[sel].mean())
        vs.append(vphi[sel].std())
        pm.append(P[sel].mean())
        ps.append(P[sel].std())
    return {k: np.array(v) for k, v in
            (("r", rc), ("v", vm), ("v_std", vs), ("P", pm), ("P_std", ps))}


def run(nside: int = 64, t_end: float = 0.1, cfl: float = 0.2, dtype: str = "f32",
        max_steps: int = 100000, on_step=None):
    """Integrate the vortex to t_end; returns a dict with the final host
    arrays (x, y, vx, vy, u, rho, P), the step count, dt, the kinetic plus
    internal energy at start and end, and the momentum at the end."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    parts = W.gresho(nside)
    dp = S.to_device(parts, dtype=tdt)
    plan = S.Plan(dtype=dtype)
    n = parts.n
    gamma = 5.0 / 3.0

    def energy(d):
        m = dp.m.double()
        v2 = dp.vx.double() ** 2 + dp.vy.double() ** 2 + dp.vz.double() ** 2
        return float((m * (0.5 * v2 + dp.u.double())).sum().item())

    plan.bin(dp)
    d = plan.density(dp)
    g0 = plan.gradient(dp, d)
    state = {"alpha_v": torch.zeros(n, dtype=tdt, device="cuda"),
             "alpha_c": torch.zeros(n, dtype=tdt, device="cuda"),
             "div_v_prev": d["div_v"].clone(), "v_sig_prev": g0["v_sig"].clone()}
    H = 2.0 * d["h"].double()
    dt = cfl * float((H / g0["v_sig"].double()).min().item())
    # initial forces (a copy of the state: the switches start at t = 0)
    g, f, _ = plan.gradient_force_sw(dp, d, dt, {k: v.clone() for k, v in state.items()})
    e0 = energy(d)
    t, steps = 0.0, 0
    while t < t_end * (1 - 1e-12) and steps < max_steps:
        h = min(dt, t_end - t)
        plan.kick_drift(dp, f, 0.5 * h, h)
        dp.h = d["h"]
        plan.bin(dp)
        d = plan.density(dp)
        g, f, _ = plan.gradient_force_sw(dp, d, h, state)
        plan.kick_drift(dp, f, 0.5 * h, 0.0)
        state["div_v_prev"] = d["div_v"].clone()
        state["v_sig_prev"] = g["v_sig"].clone()
        t += h
        steps += 1
        if on_step is not None:
            on_step(steps, t)
    torch.cuda.synchronize()
    st = plan.stats()
    rho = d["rho"].double()
    out = {k: getattr(dp, k).double().cpu().numpy() for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
    out["rho"] = rho.cpu().numpy()
    out["P"] = (gamma - 1.0) * out["rho"] * out["u"]
    out["alpha_v"] = state["alpha_v"].double().cpu().numpy()
    out["alpha_c"] = state["alpha_c"].double().cpu().numpy()
    m = parts.m.astype(np.float64)
    out.update({"t": t, "steps": steps, "dt": dt, "energy0": e0, "energy": energy(d),
                "momentum": [float(np.sum(m * out[k])) for k in ("vx", "vy", "vz")],
                "status": st["code"], "n": n})
    return out
