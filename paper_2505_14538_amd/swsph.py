"""Thin Python binding of libswsph.so (the C ABI in include/swsph.h).

Argument marshalling only: torch supplies device memory and the current
stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback -- importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswsph.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libswsph.so is not built: run `python -c 'import __graft_entry__ as g; "
                      "g.build()'` (or python paper_2505_14538_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ C types

SWSPH_F32, SWSPH_F64 = 0, 1
FIXED_H = 0x1
NO_VISC = 0x2
PER_TASK_LAUNCH = 0x4
FLAT_LAUNCH = 0x8
TIMING = 0x10
SINGLE_LAUNCH = 0x20

ST_CAPACITY, ST_REACH, ST_NEWTON, ST_DOMAIN = 0x1, 0x2, 0x4, 0x8

STATUS = {0: "OK", -1: "E_ARG", -2: "E_HIP", -3: "E_STATE", -4: "E_CAPACITY",
          -5: "E_REACH", -6: "E_NEWTON", -7: "E_DOMAIN"}


class Config(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("eps", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("h_tol", ctypes.c_double),
                ("h_max_iter", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tile", ctypes.c_int32),
                ("lds_cap", ctypes.c_int32), ("order", ctypes.c_int32),
                ("leaf_max", ctypes.c_int32), ("tile_dens", ctypes.c_int32),
                ("lds_cap_dens", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in
                ("tile", "tile_dens", "lds_cap", "lds_cap_dens", "order", "leaf_max")]


class ParticlesC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("vx", ctypes.c_void_p), ("vy", ctypes.c_void_p), ("vz", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("box_id", ctypes.c_void_p), ("n_box", ctypes.c_int32),
                ("box_size", ctypes.POINTER(ctypes.c_double)),
                ("box_count", ctypes.POINTER(ctypes.c_int64)),
                ("h", ctypes.c_void_p)]


class DensityOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in
                ("h", "rho", "rho_dh", "wcount", "wcount_dh", "div_v", "curl_x", "curl_y",
                 "curl_z", "f", "nngb", "iters")]


class GradientOut(ctypes.Structure):
    _fields_ = [("v_sig", ctypes.c_void_p), ("lap_u", ctypes.c_void_p)]


class ForceOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("ax", "ay", "az", "dudt", "nint")]


class ForceGrad(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("gax", "gay", "gaz", "gdudt")]


class InputGrad(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("gx", "gy", "gz", "gvx", "gvy", "gvz", "gu", "gm")]


class SwitchParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("dt", "av_max", "av_min", "ell", "beta_c", "ac_min", "ac_max", "bal_eps")]


# switch constants: the decay length l = 0.05 is the paper's (Sec. 2.1.3);
# the others are conventions the paper does not fix
SWITCH_DEFAULTS = {"av_max": 2.0, "av_min": 0.0, "ell": 0.05, "beta_c": 1.0, "ac_min": 0.0,
                   "ac_max": 1.0, "bal_eps": 1e-4}


class SwitchState(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in
                ("alpha_v", "alpha_c", "div_v_prev", "v_sig_prev", "balsara", "alpha_v_ngb")]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_uint32), ("n_tiles", ctypes.c_uint32),
                ("pairs_tested", ctypes.c_uint64 * 4), ("pairs_inside", ctypes.c_uint64 * 4),
                ("newton_sweeps", ctypes.c_uint64), ("newton_max", ctypes.c_uint32),
                ("newton_failed", ctypes.c_uint32), ("listed", ctypes.c_uint64),
                ("restages", ctypes.c_uint64), ("n_tiles_dens", ctypes.c_uint64),
                ("dens_listed", ctypes.c_uint64), ("single_redo", ctypes.c_uint64),
                ("reserved", ctypes.c_uint64 * 3)]

    def as_dict(self) -> Dict:
        return {"status": self.status, "n_tiles": self.n_tiles,
                "pairs_tested": list(self.pairs_tested), "pairs_inside": list(self.pairs_inside),
                "newton_sweeps": self.newton_sweeps, "newton_max": self.newton_max,
                "newton_failed": self.newton_failed, "listed": self.listed,
                "restages": self.restages, "n_tiles_dens": self.n_tiles_dens,
                "dens_listed": self.dens_listed, "single_redo": self.single_redo}


_vp = ctypes.c_void_p
_P = ctypes.POINTER
_lib.swsph_version.restype = ctypes.c_int
_lib.swsph_last_error.restype = ctypes.c_char_p
_lib.swsph_config_default.argtypes = [_P(Config)]
_lib.swsph_config_default.restype = None
_lib.swsph_plan_create.argtypes = [_P(_vp), _P(Config)]
_lib.swsph_plan_destroy.argtypes = [_vp]
_lib.swsph_workspace_bytes.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, _P(ctypes.c_int64),
                                       _P(ctypes.c_double), _P(ctypes.c_uint64)]
_lib.swsph_bin.argtypes = [_vp, _P(ParticlesC), _vp, _vp]
_lib.swsph_density.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _vp, _vp]
_lib.swsph_gradient.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _P(GradientOut), _vp, _vp]
_lib.swsph_force.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _P(ForceOut), _vp, _vp]
_lib.swsph_gradient_force.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _P(GradientOut),
                                      _P(ForceOut), _vp, _vp]
_lib.swsph_force_backward.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _P(ForceGrad),
                                      _P(InputGrad), _vp, _vp]
_lib.swsph_step.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _P(GradientOut), _P(ForceOut),
                            _vp, _vp]
_lib.swsph_gradient_force_sw.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _P(SwitchParams),
                                         _P(SwitchState), _P(GradientOut), _P(ForceOut), _vp,
                                         _vp]
_lib.swsph_kick_drift.argtypes = [_vp, ctypes.c_int64] + [_vp] * 11 + \
    [ctypes.c_double, ctypes.c_double, _vp, ctypes.c_int32, _P(ctypes.c_double), _vp]
_lib.swsph_step_static.argtypes = [_vp, _P(ParticlesC), _P(DensityOut), _P(GradientOut),
                                   _P(ForceOut), _vp]
_lib.swsph_read_stats.argtypes = [_vp, _vp, _P(Stats), _vp]
_lib.swsph_autotune.argtypes = [_vp, _P(ParticlesC), _vp, _vp, ctypes.c_char_p]
_lib.swsph_plan_get_tuning.argtypes = [_vp, _P(Tuning)]
_lib.swsph_kernel_times.argtypes = [_vp, _P(ctypes.c_double), _P(ctypes.c_uint64), _vp]
_lib.swsph_reset_timers.argtypes = [_vp]

EXPORTS = ["swsph_version", "swsph_last_error", "swsph_config_default", "swsph_plan_create",
           "swsph_plan_destroy", "swsph_workspace_bytes", "swsph_bin", "swsph_density",
           "swsph_gradient", "swsph_force", "swsph_gradient_force", "swsph_force_backward",
           "swsph_step",
           "swsph_step_static", "swsph_gradient_force_sw", "swsph_kick_drift",
           "swsph_read_stats", "swsph_autotune", "swsph_plan_get_tuning",
           "swsph_kernel_times", "swsph_reset_timers"]


class SwsphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


def _check(code: int) -> None:
    if code != 0:
        raise SwsphError(code, _lib.swsph_last_error().decode())


def version() -> int:
    return _lib.swsph_version()


def default_config(**kw) -> Config:
    c = Config()
    _lib.swsph_config_default(ctypes.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


# ------------------------------------------------------------ torch helpers

def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class DeviceParticles:
    """Particle arrays on the GPU (torch tensors, one dtype) + host box data."""

    x: object
    y: object
    z: object
    vx: object
    vy: object
    vz: object
    u: object
    m: object
    box_size: np.ndarray
    box_count: np.ndarray
    box_id: object = None
    h: object = None
    _c: ParticlesC = field(default=None, repr=False)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def c(self) -> ParticlesC:
        self._bs = np.ascontiguousarray(self.box_size, dtype=np.float64)
        self._bc = np.ascontiguousarray(self.box_count, dtype=np.int64)
        p = ParticlesC()
        p.n = self.n
        p.x, p.y, p.z = _ptr(self.x), _ptr(self.y), _ptr(self.z)
        p.vx, p.vy, p.vz = _ptr(self.vx), _ptr(self.vy), _ptr(self.vz)
        p.u, p.m = _ptr(self.u), _ptr(self.m)
        p.box_id = _ptr(self.box_id)
        p.n_box = int(self._bs.shape[0])
        p.box_size = self._bs.ctypes.data_as(_P(ctypes.c_double))
        p.box_count = self._bc.ctypes.data_as(_P(ctypes.c_int64))
        p.h = _ptr(self.h)
        self._c = p
        return p


def to_device(parts, dtype=None, device="cuda", h=None) -> DeviceParticles:
    """Copy a workloads.Particles set to the GPU (float32 unless dtype)."""
    torch = _torch()
    dt = torch.float32 if dtype is None else dtype
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    bc = np.array([parts.n], dtype=np.int64) if parts.box_id is None else \
        np.bincount(parts.box_id, minlength=parts.n_box).astype(np.int64)
    bid = None if parts.box_id is None else torch.as_tensor(parts.box_id.astype(np.int32)).to(device)
    hh = None if h is None else f(h)
    return DeviceParticles(f(parts.x), f(parts.y), f(parts.z), f(parts.vx), f(parts.vy),
                           f(parts.vz), f(parts.u), f(parts.m), np.asarray(parts.box_size),
                           bc, bid, hh)


class Plan:
    """A library plan plus its workspace (a torch uint8 tensor)."""

    def __init__(self, dtype: str = "f32", flags: int = 0, **kw):
        self.cfg = default_config(dtype=SWSPH_F64 if dtype == "f64" else SWSPH_F32,
                                  flags=flags, **kw)
        h = ctypes.c_void_p()
        _check(_lib.swsph_plan_create(ctypes.byref(h), ctypes.byref(self.cfg)))
        self.h = h
        self.ws = None
        self.dtype = dtype

    def close(self):
        if self.h:
            _lib.swsph_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tdtype(self):
        torch = _torch()
        return torch.float64 if self.dtype == "f64" else torch.float32

    def workspace_bytes(self, p: DeviceParticles) -> int:
        pc = p.c()
        out = ctypes.c_uint64()
        _check(_lib.swsph_workspace_bytes(self.h, pc.n, pc.n_box, pc.box_count, pc.box_size,
                                          ctypes.byref(out)))
        return int(out.value)

    def ensure_workspace(self, p: DeviceParticles):
        torch = _torch()
        nb = self.workspace_bytes(p)
        if self.ws is None or self.ws.numel() < nb:
            self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=p.x.device)
        return self.ws

    def _ws_ptr(self):
        base = int(self.ws.data_ptr())
        return ctypes.c_void_p((base + 255) & ~255)

    # --------------------------------------------------------------- calls
    def bin(self, p: DeviceParticles):
        self.ensure_workspace(p)
        self._pc = p.c()
        _check(_lib.swsph_bin(self.h, ctypes.byref(self._pc), self._ws_ptr(), _stream()))

    def _alloc(self, n, dtype=None):
        torch = _torch()
        return torch.empty(n, dtype=self.tdtype() if dtype is None else dtype, device="cuda")

    def density(self, p: DeviceParticles) -> Dict[str, object]:
        torch = _torch()
        n = p.n
        o = {k: self._alloc(n) for k in ("h", "rho", "rho_dh", "wcount", "wcount_dh", "div_v",
                                          "curl_x", "curl_y", "curl_z", "f")}
        o["nngb"] = self._alloc(n, torch.int32)
        o["iters"] = self._alloc(n, torch.int32)
        d = DensityOut(**{k: _ptr(v) for k, v in o.items()})
        pc = p.c()
        _check(_lib.swsph_density(self.h, ctypes.byref(pc), ctypes.byref(d), self._ws_ptr(),
                                  _stream()))
        return o

    @staticmethod
    def _dens_c(d: Dict[str, object]) -> DensityOut:
        return DensityOut(**{k: _ptr(d.get(k)) for k in
                             ("h", "rho", "rho_dh", "wcount", "wcount_dh", "div_v", "curl_x",
                              "curl_y", "curl_z", "f", "nngb", "iters")})

    def gradient(self, p: DeviceParticles, dens) -> Dict[str, object]:
        n = p.n
        o = {"v_sig": self._alloc(n), "lap_u": self._alloc(n)}
        g = GradientOut(_ptr(o["v_sig"]), _ptr(o["lap_u"]))
        pc = p.c()
        dc = self._dens_c(dens)
        _check(_lib.swsph_gradient(self.h, ctypes.byref(pc), ctypes.byref(dc), ctypes.byref(g),
                                   self._ws_ptr(), _stream()))
        return o

    def force(self, p: DeviceParticles, dens) -> Dict[str, object]:
        torch = _torch()
        n = p.n
        o = {k: self._alloc(n) for k in ("ax", "ay", "az", "dudt")}
        o["nint"] = self._alloc(n, torch.int32)
        fo = ForceOut(**{k: _ptr(v) for k, v in o.items()})
        pc = p.c()
        dc = self._dens_c(dens)
        _check(_lib.swsph_force(self.h, ctypes.byref(pc), ctypes.byref(dc), ctypes.byref(fo),
                                self._ws_ptr(), _stream()))
        return o

    def gradient_force(self, p: DeviceParticles, dens):
        """Gradient and force outputs from one pass of the joint kernel
        (swsph_gradient_force); returns (gradient outputs, force outputs)."""
        torch = _torch()
        n = p.n
        g = {"v_sig": self._alloc(n), "lap_u": self._alloc(n)}
        f = {k: self._alloc(n) for k in ("ax", "ay", "az", "dudt")}
        f["nint"] = self._alloc(n, torch.int32)
        go = GradientOut(_ptr(g["v_sig"]), _ptr(g["lap_u"]))
        fo = ForceOut(**{k: _ptr(v) for k, v in f.items()})
        pc = p.c()
        dc = self._dens_c(dens)
        _check(_lib.swsph_gradient_force(self.h, ctypes.byref(pc), ctypes.byref(dc),
                                         ctypes.byref(go), ctypes.byref(fo), self._ws_ptr(),
                                         _stream()))
        return g, f

    def gradient_force_sw(self, p: DeviceParticles, dens, dt: float, state, **params):
        """Gradient and force loops with the time-dependent switches
        (swsph_gradient_force_sw).  state: dict of device tensors alpha_v and
        alpha_c (read at t, overwritten with t + dt), div_v_prev, v_sig_prev;
        returns (gradient outputs incl. alpha_v_ngb, force outputs, balsara)."""
        torch = _torch()
        n = p.n
        prm = dict(SWITCH_DEFAULTS)
        prm.update(params)
        sp = SwitchParams(dt=dt, **prm)
        g = {"v_sig": self._alloc(n), "lap_u": self._alloc(n), "alpha_v_ngb": self._alloc(n)}
        f = {k: self._alloc(n) for k in ("ax", "ay", "az", "dudt")}
        f["nint"] = self._alloc(n, torch.int32)
        bal = self._alloc(n)
        st = SwitchState(_ptr(state["alpha_v"]), _ptr(state["alpha_c"]),
                         _ptr(state["div_v_prev"]), _ptr(state["v_sig_prev"]), _ptr(bal),
                         _ptr(g["alpha_v_ngb"]))
        go = GradientOut(_ptr(g["v_sig"]), _ptr(g["lap_u"]))
        fo = ForceOut(**{k: _ptr(v) for k, v in f.items()})
        pc = p.c()
        dc = self._dens_c(dens)
        _check(_lib.swsph_gradient_force_sw(self.h, ctypes.byref(pc), ctypes.byref(dc),
                                            ctypes.byref(sp), ctypes.byref(st), ctypes.byref(go),
                                            ctypes.byref(fo), self._ws_ptr(), _stream()))
        return g, f, bal

    def kick_drift(self, p: DeviceParticles, f, dt_kick: float, dt_drift: float):
        """Leapfrog update of p in place (swsph_kick_drift): v += a dt_kick,
        u += du/dt dt_kick with the force outputs f (dict; may be None when
        dt_kick == 0), then x += v dt_drift wrapped into the box."""
        pc = p.c()
        a = (None, None, None, None) if f is None else \
            (_ptr(f["ax"]), _ptr(f["ay"]), _ptr(f["az"]), _ptr(f["dudt"]))
        _check(_lib.swsph_kick_drift(self.h, p.n, _ptr(p.x), _ptr(p.y), _ptr(p.z), _ptr(p.vx),
                                     _ptr(p.vy), _ptr(p.vz), _ptr(p.u), *a, float(dt_kick),
                                     float(dt_drift), _ptr(p.box_id), pc.n_box, pc.box_size,
                                     _stream()))

    def step(self, p: DeviceParticles, gradient: bool = True, force: bool = True, out=None):
        """bin + density + gradient + force in one call.  The library captures
        the whole step in a HIP graph and replays it while the particle and
        output buffers stay the same, so by default the outputs are buffers
        the plan keeps and overwrites at the next step (copy what must
        survive); `out` = (d, g, f) dicts of caller tensors instead."""
        torch = _torch()
        self.ensure_workspace(p)
        n = p.n
        if out is None:
            key = (n, bool(gradient), bool(force), self.dtype)
            if getattr(self, "_step_key", None) != key:
                d = {k: self._alloc(n) for k in ("h", "rho", "rho_dh", "wcount", "wcount_dh",
                                                  "div_v", "curl_x", "curl_y", "curl_z", "f")}
                d["nngb"] = self._alloc(n, torch.int32)
                d["iters"] = self._alloc(n, torch.int32)
                g = {"v_sig": self._alloc(n), "lap_u": self._alloc(n)} if gradient else None
                f = None
                if force:
                    f = {k: self._alloc(n) for k in ("ax", "ay", "az", "dudt")}
                    f["nint"] = self._alloc(n, torch.int32)
                self._step_out = (d, g, f)
                self._step_key = key
            d, g, f = self._step_out
        else:
            d, g, f = out
        dc = self._dens_c(d)
        gc = GradientOut(_ptr(g["v_sig"]), _ptr(g["lap_u"])) if g else None
        fc = ForceOut(**{k: _ptr(v) for k, v in f.items()}) if f else None
        self._pc = p.c()
        _check(_lib.swsph_step(self.h, ctypes.byref(self._pc), ctypes.byref(dc),
                               ctypes.byref(gc) if gc else None, ctypes.byref(fc) if fc else None,
                               self._ws_ptr(), _stream()))
        return d, g, f

    def step_static(self, p: DeviceParticles, out=None):
        """bin + density + gradient + force with the library's static device
        scratch (swsph_step_static: no workspace, nothing allocated by the
        library).  Outputs are fresh tensors unless `out` = (d, g, f) dicts of
        caller tensors.  Stats afterwards: stats(static=True)."""
        torch = _torch()
        n = p.n
        if out is None:
            d = {k: self._alloc(n) for k in ("h", "rho", "rho_dh", "wcount", "wcount_dh",
                                              "div_v", "curl_x", "curl_y", "curl_z", "f")}
            d["nngb"] = self._alloc(n, torch.int32)
            d["iters"] = self._alloc(n, torch.int32)
            g = {"v_sig": self._alloc(n), "lap_u": self._alloc(n)}
            f = {k: self._alloc(n) for k in ("ax", "ay", "az", "dudt")}
            f["nint"] = self._alloc(n, torch.int32)
        else:
            d, g, f = out
        dc = self._dens_c(d)
        gc = GradientOut(_ptr(g["v_sig"]), _ptr(g["lap_u"])) if g else None
        fc = ForceOut(**{k: _ptr(v) for k, v in f.items()}) if f else None
        self._pc = p.c()
        _check(_lib.swsph_step_static(self.h, ctypes.byref(self._pc), ctypes.byref(dc),
                                      ctypes.byref(gc) if gc else None,
                                      ctypes.byref(fc) if fc else None, _stream()))
        return d, g, f

    def force_backward(self, p: DeviceParticles, dens, gax, gay, gaz, gdudt):
        n = p.n
        o = {k: self._alloc(n) for k in ("gx", "gy", "gz", "gvx", "gvy", "gvz", "gu", "gm")}
        gi = InputGrad(**{k: _ptr(v) for k, v in o.items()})
        g = ForceGrad(_ptr(gax), _ptr(gay), _ptr(gaz), _ptr(gdudt))
        pc = p.c()
        dc = self._dens_c(dens)
        _check(_lib.swsph_force_backward(self.h, ctypes.byref(pc), ctypes.byref(dc),
                                         ctypes.byref(g), ctypes.byref(gi), self._ws_ptr(),
                                         _stream()))
        return o

    def stats(self, check: bool = False, static: bool = False) -> Dict:
        """Device statistics of the plan's last bin (static=True: of the last
        step_static, whose scratch the library owns)."""
        s = Stats()
        ws = None if static else self._ws_ptr()
        r = _lib.swsph_read_stats(self.h, ws, ctypes.byref(s), _stream())
        if check:
            _check(r)
        d = s.as_dict()
        d["code"] = r
        return d

    def kernel_times(self) -> Dict[str, Dict[str, float]]:
        """Mean ms per launch of each loop kernel (plan created with TIMING);
        the gradient and force loops share one kernel ("gradient+force")."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_uint64 * 4)()
        _check(_lib.swsph_kernel_times(self.h, ms, n, _stream()))
        names = ("density", "gradient", "gradient+force", "backward")
        return {names[k]: {"ms": ms[k], "launches": int(n[k])} for k in range(4) if n[k] > 0}

    def reset_timers(self):
        _check(_lib.swsph_reset_timers(self.h))

    def autotune(self, p: DeviceParticles, cache_path: Optional[str] = None):
        self.ensure_workspace(p)
        pc = p.c()
        _check(_lib.swsph_autotune(self.h, ctypes.byref(pc), self._ws_ptr(), _stream(),
                                   None if cache_path is None else cache_path.encode()))
        return self.tuning()

    def tuning(self):
        t = Tuning()
        _check(_lib.swsph_plan_get_tuning(self.h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}


def host(d: Dict[str, object]) -> Dict[str, np.ndarray]:
    """Copy a dict of device tensors to numpy."""
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()}


# ------------------------------------------------------------------ autograd

class _SPHForce:
    """torch.autograd.Function wrapper (built lazily so importing this module
    does not require torch)."""

    fn = None

    @classmethod
    def get(cls):
        if cls.fn is None:
            import torch

            class SPHForce(torch.autograd.Function):
                """(x, y, z, vx, vy, vz, u, m) -> (ax, ay, az, du/dt): bin, density
                (Newton on h) and force in the forward pass; the hand-written adjoint
                (swsph_force_backward) in the backward pass.  Only per-particle
                density results are saved."""

                @staticmethod
                def forward(ctx, plan, box_size, box_count, box_id, x, y, z, vx, vy, vz, u, m):
                    dp = DeviceParticles(x.detach(), y.detach(), z.detach(), vx.detach(),
                                         vy.detach(), vz.detach(), u.detach(), m.detach(),
                                         np.asarray(box_size), np.asarray(box_count), box_id)
                    plan.bin(dp)
                    d = plan.density(dp)
                    f = plan.force(dp, d)
                    ctx.plan = plan
                    ctx.dp = dp
                    ctx.d = {k: d[k] for k in ("h", "rho", "f", "rho_dh", "wcount", "wcount_dh")}
                    return f["ax"], f["ay"], f["az"], f["dudt"]

                @staticmethod
                def backward(ctx, gax, gay, gaz, gdu):
                    zeros = lambda g: torch.zeros_like(ctx.dp.x) if g is None else g.contiguous()
                    plan, dp = ctx.plan, ctx.dp
                    plan.bin(dp)
                    gi = plan.force_backward(dp, ctx.d, zeros(gax), zeros(gay), zeros(gaz),
                                             zeros(gdu))
                    return (None, None, None, None, gi["gx"], gi["gy"], gi["gz"], gi["gvx"],
                            gi["gvy"], gi["gvz"], gi["gu"], gi["gm"])

            cls.fn = SPHForce
        return cls.fn


def sph_force(plan: Plan, x, y, z, vx, vy, vz, u, m, box_size=(1.0,), box_count=None,
              box_id=None):
    """Differentiable accelerations and du/dt of particles in periodic boxes."""
    bc = np.array([x.shape[0]], dtype=np.int64) if box_count is None else np.asarray(box_count)
    return _SPHForce.get().apply(plan, np.asarray(box_size, dtype=np.float64), bc, box_id,
                                 x, y, z, vx, vy, vz, u, m)
