"""Python front end of the FP64 CPU oracle (``swsph_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark load this module; the library and its Python
binding never do.  Nothing here shares code with the HIP path.

Every function takes float32 (or float64) particle arrays, widens them to
float64 exactly, and returns float64 results in the caller's particle order.
Independent periodic boxes are handled one at a time (they do not interact).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swsph_oracle.c")
_LIB = os.path.join(_HERE, "libswsph_oracle.so")

GCC_FLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("eps", ctypes.c_double),
                ("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("visc", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("ncell", ctypes.c_int32)]


@dataclass
class Params:
    """Scheme constants.  eta and eps fix the neighbour number
    (4 pi / 3)(eps eta)^3 ~ 63 for eta = 1.2348, eps = 2; gamma = 5/3 as in
    the paper's tests (Sec. 3.1); alpha = 1, beta = 3 (Monaghan viscosity,
    constant coefficients)."""

    eta: float = 1.2348
    eps: float = 2.0
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    beta: float = 3.0
    tol: float = 1e-13
    max_iter: int = 200
    visc: bool = True
    mode: str = "cells"   # or "brute"
    ncell: int = 0

    def c(self) -> OrcParams:
        return OrcParams(self.eta, self.eps, self.gamma, self.alpha, self.beta,
                         self.tol, int(self.max_iter), int(bool(self.visc)),
                         0 if self.mode == "brute" else 1, int(self.ncell))


class OrcSwitchParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("dt", "av_max", "av_min", "ell", "beta_c", "ac_min", "ac_max", "bal_eps")]


@dataclass
class SwitchParams:
    """Constants of the time-dependent switches (Sec. 2.1.3-2.1.4): the decay
    length l = 0.05 is the paper's; alpha_V,max = 2, alpha_V,min = 0,
    beta_c = 1, alpha_c in [0, 1] and the Balsara softening 1e-4 c/H are
    conventions (the paper gives no values)."""

    dt: float = 1e-3
    av_max: float = 2.0
    av_min: float = 0.0
    ell: float = 0.05
    beta_c: float = 1.0
    ac_min: float = 0.0
    ac_max: float = 1.0
    bal_eps: float = 1e-4

    def c(self) -> OrcSwitchParams:
        return OrcSwitchParams(self.dt, self.av_max, self.av_min, self.ell, self.beta_c,
                               self.ac_min, self.ac_max, self.bal_eps)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, f64p, i64p, i32p = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
        pp = ctypes.POINTER(OrcParams)
        L.orc_version.restype = ctypes.c_int
        L.orc_kernel_eval.argtypes = [ctypes.c_int, i64, f64p, ctypes.c_double,
                                      ctypes.c_double, f64p]
        L.orc_kernel_eval.restype = None
        L.orc_density.argtypes = [i64] + [f64p] * 7 + [ctypes.c_double, pp, f64p, f64p,
                                                       i64, i64p] + [f64p] * 10 + [i32p, i32p]
        L.orc_density.restype = i64
        L.orc_gradient.argtypes = [i64] + [f64p] * 8 + [ctypes.c_double, pp, f64p, f64p,
                                                        i64, i64p, f64p, f64p]
        L.orc_gradient.restype = i64
        L.orc_force.argtypes = [i64] + [f64p] * 8 + [ctypes.c_double, pp, f64p, f64p, f64p,
                                                     i64, i64p, f64p, f64p, f64p, f64p, i32p]
        L.orc_force.restype = i64
        L.orc_neighbour_sets.argtypes = [i64, f64p, f64p, f64p, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, f64p, f64p, i64,
                                         i64p, i64, i64p, i64p]
        L.orc_neighbour_sets.restype = i64
        L.orc_count_f32.argtypes = [i64, f64p, f64p, f64p, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_void_p, i64,
                                    i64p, i32p, i32p]
        L.orc_count_f32.restype = i64
        L.orc_count_f32_sym.argtypes = [i64, f64p, f64p, f64p, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_void_p, i32p,
                                        i32p]
        L.orc_count_f32_sym.restype = i64
        L.orc_loss_subset.argtypes = [i64] + [f64p] * 8 + [ctypes.c_double, pp, f64p,
                                                           ctypes.c_double, i64, i64p,
                                                           f64p, f64p, f64p, f64p, f64p]
        L.orc_loss_subset.restype = i64
        sp = ctypes.POINTER(OrcSwitchParams)
        L.orc_switch_visc.argtypes = [i64, pp, sp] + [f64p] * 11
        L.orc_switch_visc.restype = None
        L.orc_alpha_ngb.argtypes = [i64, f64p, f64p, f64p, ctypes.c_double, pp, f64p, f64p,
                                    f64p]
        L.orc_alpha_ngb.restype = i64
        L.orc_switch_cond.argtypes = [i64, pp, sp] + [f64p] * 7
        L.orc_switch_cond.restype = None
        L.orc_force_sw.argtypes = [i64] + [f64p] * 8 + [ctypes.c_double, pp] + [f64p] * 6 + \
            [i64, i64p, f64p, f64p, f64p, f64p, i32p]
        L.orc_force_sw.restype = i64
        _lib = L
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def kernel_eval(which: str, a, b: float = 1.0, eps: float = 2.0) -> np.ndarray:
    """which in {'w', 'dw', 'd2w'} (argument q) or {'W', 'dWdr', 'dWdh'}
    (argument r, smoothing length b)."""
    code = {"w": 0, "dw": 1, "d2w": 2, "W": 3, "dWdr": 4, "dWdh": 5}[which]
    a = _d(np.atleast_1d(a))
    out = np.empty_like(a)
    lib().orc_kernel_eval(code, a.size, _ptr(a), float(b), float(eps), _ptr(out))
    return out


def _boxes(p, idx):
    """Yield (box index array, local output positions, local idx or None, L)."""
    sel_all = idx is None
    for b, ib in p.box_slices():
        L = float(p.box_size[b])
        if sel_all:
            yield ib, None, None, L
        else:
            pos_in_box = {int(g): k for k, g in enumerate(ib)}
            loc = [(k, pos_in_box[int(g)]) for k, g in enumerate(idx) if int(g) in pos_in_box]
            if not loc:
                continue
            out_pos = np.array([a for a, _ in loc], dtype=np.int64)
            lidx = np.array([c for _, c in loc], dtype=np.int64)
            yield ib, out_pos, lidx, L


def density(p, params: Params = Params(), h_fixed=None, h_guess=None, idx=None):
    """Density loop with Newton on h (or at fixed h).  Returns a dict of
    float64 arrays over all particles (entries outside idx are NaN) plus
    'nngb' (int32) and 'iters' (int32, negative when not converged) and
    'n_bad' (number of particles without a converged h)."""
    n = p.n
    keys = ["h", "rho", "rho_dh", "wcount", "wcount_dh", "div_v", "curl_x",
            "curl_y", "curl_z", "f"]
    out = {k: np.full(n, np.nan) for k in keys}
    out["nngb"] = np.full(n, -1, dtype=np.int32)
    out["iters"] = np.zeros(n, dtype=np.int32)
    bad = 0
    idx = None if idx is None else np.asarray(idx, dtype=np.int64)
    for ib, out_pos, lidx, L in _boxes(p, idx):
        nb = ib.size
        arr = [_d(a[ib]) for a in (p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m)]
        hf = None if h_fixed is None else _d(np.asarray(h_fixed)[ib])
        hg = None if h_guess is None else _d(np.asarray(h_guess)[ib])
        loc = {k: np.full(nb, np.nan) for k in keys}
        nng = np.full(nb, -1, dtype=np.int32)
        its = np.zeros(nb, dtype=np.int32)
        li = None if lidx is None else np.ascontiguousarray(lidx)
        r = lib().orc_density(nb, *[_ptr(a) for a in arr], L, ctypes.byref(params.c()),
                              _ptr(hf), _ptr(hg), 0 if li is None else li.size, _ptr(li),
                              *[_ptr(loc[k]) for k in keys], _ptr(nng), _ptr(its))
        if r < 0:
            raise MemoryError("oracle density failed")
        bad += int(r)
        for k in keys:
            out[k][ib] = loc[k]
        out["nngb"][ib] = nng
        out["iters"][ib] = its
    out["n_bad"] = bad
    return out


def gradient(p, dens, params: Params = Params(), idx=None):
    """Gradient loop at the given density results (dict with 'h', 'rho')."""
    n = p.n
    vsig = np.full(n, np.nan)
    lapu = np.full(n, np.nan)
    idx = None if idx is None else np.asarray(idx, dtype=np.int64)
    for ib, out_pos, lidx, L in _boxes(p, idx):
        nb = ib.size
        arr = [_d(a[ib]) for a in (p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, p.m)]
        h = _d(np.asarray(dens["h"])[ib])
        rho = _d(np.asarray(dens["rho"])[ib])
        vs = np.full(nb, np.nan)
        lp = np.full(nb, np.nan)
        li = None if lidx is None else np.ascontiguousarray(lidx)
        lib().orc_gradient(nb, *[_ptr(a) for a in arr], L, ctypes.byref(params.c()),
                           _ptr(h), _ptr(rho), 0 if li is None else li.size, _ptr(li),
                           _ptr(vs), _ptr(lp))
        vsig[ib] = vs
        lapu[ib] = lp
    return {"v_sig": vsig, "lap_u": lapu}


def force(p, dens, params: Params = Params(), idx=None):
    """Force loop at the given density results (dict with 'h', 'rho', 'f').
    Returns ax, ay, az, dudt (float64) and nint (pairs per particle)."""
    n = p.n
    res = {k: np.full(n, np.nan) for k in ("ax", "ay", "az", "dudt")}
    res["nint"] = np.full(n, -1, dtype=np.int32)
    idx = None if idx is None else np.asarray(idx, dtype=np.int64)
    for ib, out_pos, lidx, L in _boxes(p, idx):
        nb = ib.size
        arr = [_d(a[ib]) for a in (p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, p.m)]
        h = _d(np.asarray(dens["h"])[ib])
        rho = _d(np.asarray(dens["rho"])[ib])
        f = _d(np.asarray(dens["f"])[ib])
        loc = {k: np.full(nb, np.nan) for k in ("ax", "ay", "az", "dudt")}
        ni = np.full(nb, -1, dtype=np.int32)
        li = None if lidx is None else np.ascontiguousarray(lidx)
        lib().orc_force(nb, *[_ptr(a) for a in arr], L, ctypes.byref(params.c()),
                        _ptr(h), _ptr(rho), _ptr(f), 0 if li is None else li.size, _ptr(li),
                        _ptr(loc["ax"]), _ptr(loc["ay"]), _ptr(loc["az"]), _ptr(loc["dudt"]),
                        _ptr(ni))
        for k in loc:
            res[k][ib] = loc[k]
        res["nint"][ib] = ni
    return res


def count_f32(p, h32, eps: float = 2.0, idx=None, mode: str = "cells", ncell: int = 0,
              symmetric: bool = True):
    """Binary32 neighbour counts at float32 smoothing lengths h32: returns
    (count_density, count_force) per particle (int32)."""
    n = p.n
    c1 = np.full(n, -1, dtype=np.int32)
    c2 = np.full(n, -1, dtype=np.int32)
    h32 = np.ascontiguousarray(np.asarray(h32, dtype=np.float32))
    idx_all = np.arange(n, dtype=np.int64) if idx is None else np.asarray(idx, dtype=np.int64)
    for ib, out_pos, lidx, L in _boxes(p, None if idx is None else idx_all):
        nb = ib.size
        arr = [_d(a[ib]) for a in (p.x, p.y, p.z)]
        hb = np.ascontiguousarray(h32[ib])
        li = np.arange(nb, dtype=np.int64) if lidx is None else np.ascontiguousarray(lidx)
        a = np.empty(li.size, dtype=np.int32)
        b = np.empty(li.size, dtype=np.int32)
        lib().orc_count_f32(nb, *[_ptr(x) for x in arr], L, 0 if mode == "brute" else 1,
                            int(ncell), float(eps), hb.ctypes.data, li.size, _ptr(li),
                            _ptr(a), _ptr(b) if symmetric else None)
        c1[ib[li]] = a
        if symmetric:
            c2[ib[li]] = b
    return c1, c2


def count_f32_sym(p, h32, eps: float = 2.0, mode: str = "cells", ncell: int = 0):
    """The counts of count_f32 for every particle, the force predicate
    enumerated from both sides of each pair (each particle searches only its
    own support): suited to sets whose supports span orders of magnitude."""
    n = p.n
    c1 = np.full(n, -1, dtype=np.int32)
    c2 = np.full(n, -1, dtype=np.int32)
    h32 = np.ascontiguousarray(np.asarray(h32, dtype=np.float32))
    for ib, _, _, L in _boxes(p, None):
        arr = [_d(a[ib]) for a in (p.x, p.y, p.z)]
        hb = np.ascontiguousarray(h32[ib])
        a = np.empty(ib.size, dtype=np.int32)
        b = np.empty(ib.size, dtype=np.int32)
        r = lib().orc_count_f32_sym(ib.size, *[_ptr(x) for x in arr], L,
                                    0 if mode == "brute" else 1, int(ncell), float(eps),
                                    hb.ctypes.data, _ptr(a), _ptr(b))
        if r < 0:
            raise MemoryError("oracle count failed")
        c1[ib] = a
        c2[ib] = b
    return c1, c2


def neighbour_sets(x, y, z, L, R, Hj=None, idx=None, mode="brute", ncell=0, cap=512):
    """Sorted neighbour index sets {j != i : r_ij < max(R_i, Hj_j)} (FP64)."""
    x, y, z = _d(x), _d(y), _d(z)
    n = x.size
    R = _d(np.broadcast_to(np.asarray(R, dtype=np.float64), (n,)))
    Hj = None if Hj is None else _d(Hj)
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    cnt = np.zeros(idx.size, dtype=np.int64)
    lst = np.full((idx.size, cap), -1, dtype=np.int64)
    lib().orc_neighbour_sets(n, _ptr(x), _ptr(y), _ptr(z), float(L),
                             0 if mode == "brute" else 1, int(ncell), _ptr(R), _ptr(Hj),
                             idx.size, _ptr(idx), cap, _ptr(cnt), _ptr(lst))
    return [lst[k, :min(cnt[k], cap)].copy() for k in range(idx.size)], cnt


def loss_subset(x, y, z, vx, vy, vz, u, m, L, params: Params, S, wx, wy, wz, c,
                Rbig, h_guess=None):
    """sum_{i in S} w_i . a_i + c_i du_i/dt with everything recomputed from
    scratch in FP64 (finite-difference checks).  All inputs float64."""
    arr = [_d(a) for a in (x, y, z, vx, vy, vz, u, m)]
    n = arr[0].size
    S = np.ascontiguousarray(S, dtype=np.int64)
    ws = [_d(a) for a in (wx, wy, wz, c)]
    hg = None if h_guess is None else _d(h_guess)
    out = ctypes.c_double(0.0)
    bad = lib().orc_loss_subset(n, *[_ptr(a) for a in arr], float(L), ctypes.byref(params.c()),
                                _ptr(hg), float(Rbig), S.size, _ptr(S),
                                *[_ptr(a) for a in ws], ctypes.byref(out))
    if bad != 0:
        raise RuntimeError("oracle: %d particles did not converge" % bad)
    return out.value


def derived(p, dens, params: Params = Params()):
    """Per-particle EOS quantities: P = (gamma-1) rho u, c = sqrt(gamma(gamma-1)u),
    A = f P / rho^2."""
    u = np.asarray(p.u, dtype=np.float64)
    rho = dens["rho"]
    P = (params.gamma - 1.0) * rho * u
    c = np.sqrt(params.gamma * (params.gamma - 1.0) * u)
    A = dens["f"] * P / rho ** 2
    return {"P": P, "c": c, "A": A}


def switch_visc(p, dens, sw: SwitchParams, div_prev, vsig_prev, av_in,
                params: Params = Params()):
    """Viscosity switch after the density loop (Eq. 12-16): returns
    {'alpha_v': alpha_V(t + dt), 'balsara': B} per particle."""
    n = p.n
    h, u = _d(dens["h"]), _d(p.u)
    args = [_d(dens[k]) for k in ("div_v",)] + [_d(div_prev)] + \
        [_d(dens[k]) for k in ("curl_x", "curl_y", "curl_z")] + [_d(vsig_prev), _d(av_in)]
    av = np.empty(n)
    B = np.empty(n)
    lib().orc_switch_visc(n, ctypes.byref(params.c()), ctypes.byref(sw.c()), _ptr(h),
                          _ptr(u), *[_ptr(a) for a in args], _ptr(av), _ptr(B))
    return {"alpha_v": av, "balsara": B}


def alpha_ngb(p, dens, av, params: Params = Params()):
    """Largest alpha_V over each particle's support r < H_i (own included)."""
    out = np.full(p.n, np.nan)
    av = _d(av)
    for ib, _, _, L in _boxes(p, None):
        arr = [_d(a[ib]) for a in (p.x, p.y, p.z)]
        h = _d(np.asarray(dens["h"])[ib])
        o = np.empty(ib.size)
        a = np.ascontiguousarray(av[ib])
        if lib().orc_alpha_ngb(ib.size, *[_ptr(x) for x in arr], L,
                               ctypes.byref(params.c()), _ptr(h), _ptr(a), _ptr(o)) < 0:
            raise MemoryError("oracle alpha_ngb failed")
        out[ib] = o
    return out


def switch_cond(p, dens, grad, sw: SwitchParams, av_ngb, ac_in, params: Params = Params()):
    """Conduction switch after the gradient loop (Eq. 21, 23-24): alpha_c(t+dt)."""
    n = p.n
    ac = np.empty(n)
    args = [_d(dens["h"]), _d(p.u), _d(grad["v_sig"]), _d(grad["lap_u"]), _d(av_ngb),
            _d(ac_in)]
    lib().orc_switch_cond(n, ctypes.byref(params.c()), ctypes.byref(sw.c()),
                          *[_ptr(a) for a in args], _ptr(ac))
    return ac


def force_sw(p, dens, av, B, ac, params: Params = Params(), idx=None):
    """Force loop with the switches: alpha_ij = (av_i + av_j)/2 (B_i + B_j)/2
    in the viscosity and artificial conduction in du/dt (Eq. 16, 19-20, 22)."""
    n = p.n
    res = {k: np.full(n, np.nan) for k in ("ax", "ay", "az", "dudt")}
    res["nint"] = np.full(n, -1, dtype=np.int32)
    idx = None if idx is None else np.asarray(idx, dtype=np.int64)
    av, B, ac = _d(av), _d(B), _d(ac)
    for ib, out_pos, lidx, L in _boxes(p, idx):
        nb = ib.size
        arr = [_d(a[ib]) for a in (p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, p.m)]
        per = [_d(np.asarray(dens[k])[ib]) for k in ("h", "rho", "f")] + \
            [np.ascontiguousarray(a[ib]) for a in (av, B, ac)]
        loc = {k: np.full(nb, np.nan) for k in ("ax", "ay", "az", "dudt")}
        ni = np.full(nb, -1, dtype=np.int32)
        li = None if lidx is None else np.ascontiguousarray(lidx)
        r = lib().orc_force_sw(nb, *[_ptr(a) for a in arr], L, ctypes.byref(params.c()),
                               *[_ptr(a) for a in per], 0 if li is None else li.size,
                               _ptr(li), _ptr(loc["ax"]), _ptr(loc["ay"]), _ptr(loc["az"]),
                               _ptr(loc["dudt"]), _ptr(ni))
        if r < 0:
            raise MemoryError("oracle force_sw failed")
        for k in loc:
            res[k][ib] = loc[k]
        res["nint"][ib] = ni
    return res


def kdk_step(p, f0, dt, state, sw: SwitchParams, params: Params = Params()):
    """One leapfrog (kick-drift-kick) step of the particles p (float64 arrays,
    one periodic box) with the switch loops: v and u kicked by the forces f0
    over dt/2, positions drifted by dt with the kicked v (wrapped into the
    box), density, gradient loop, switch updates and force loop at the new
    state, then the second half kick.  state: dict alpha_v, alpha_c,
    div_v_prev, v_sig_prev (time t).  Returns (particles, density, gradient,
    force, new state)."""
    L = float(p.box_size[0])
    q = p.subset(np.arange(p.n))
    h2 = 0.5 * dt
    vx = q.vx + f0["ax"] * h2
    vy = q.vy + f0["ay"] * h2
    vz = q.vz + f0["az"] * h2
    u = q.u + f0["dudt"] * h2
    q.x = np.mod(q.x + vx * dt, L)
    q.y = np.mod(q.y + vy * dt, L)
    q.z = np.mod(q.z + vz * dt, L)
    q.vx, q.vy, q.vz, q.u = vx, vy, vz, u
    sw = SwitchParams(**{**sw.__dict__, "dt": dt})
    dens = density(q, params)
    grad = gradient(q, dens, params)
    sv = switch_visc(q, dens, sw, state["div_v_prev"], state["v_sig_prev"], state["alpha_v"],
                     params)
    ngb = alpha_ngb(q, dens, sv["alpha_v"], params)
    ac = switch_cond(q, dens, grad, sw, ngb, state["alpha_c"], params)
    f1 = force_sw(q, dens, sv["alpha_v"], sv["balsara"], ac, params)
    q.vx = q.vx + f1["ax"] * h2
    q.vy = q.vy + f1["ay"] * h2
    q.vz = q.vz + f1["az"] * h2
    q.u = q.u + f1["dudt"] * h2
    new_state = {"alpha_v": sv["alpha_v"], "alpha_c": ac, "div_v_prev": dens["div_v"],
                 "v_sig_prev": grad["v_sig"], "balsara": sv["balsara"], "alpha_v_ngb": ngb}
    return q, dens, grad, f1, new_state
