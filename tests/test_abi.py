"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/swsph.h, and rejects bad arguments on the host before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "swsph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(swsph_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def S():
    from paper_2505_14538_amd import swsph
    return swsph


def test_exports_every_declared_symbol(S):
    names = declared_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(S._lib, nm), nm
    assert set(S.EXPORTS) == set(names)


def test_version_and_defaults(S):
    assert S.version() == 1
    c = S.default_config()
    assert c.eta == pytest.approx(1.2348) and c.eps == 2.0
    assert c.gamma == pytest.approx(5.0 / 3.0) and c.alpha == 1.0 and c.beta == 3.0
    assert c.h_max_iter == 40 and c.dtype == 0


@pytest.mark.parametrize("field,val", [("eta", 0.0), ("eps", -1.0), ("gamma", 1.0),
                                       ("alpha", -0.5), ("h_tol", 0.0), ("h_max_iter", 0),
                                       ("dtype", 7), ("tile", 24), ("lds_cap", 100),
                                       ("order", 3), ("flags", 0x4 | 0x8), ("tile_dens", 12),
                                       ("lds_cap_dens", 64)])
def test_plan_rejects_bad_config(S, field, val):
    c = S.default_config()
    setattr(c, field, val)
    h = ctypes.c_void_p()
    r = S._lib.swsph_plan_create(ctypes.byref(h), ctypes.byref(c))
    assert r == -1
    assert len(S._lib.swsph_last_error()) > 0


def test_workspace_bytes_and_bad_boxes(S):
    p = S.Plan()
    out = ctypes.c_uint64()
    bs = (ctypes.c_double * 1)(1.0)
    assert S._lib.swsph_workspace_bytes(p.h, 4096, 1, None, bs, ctypes.byref(out)) == 0
    small = out.value
    assert S._lib.swsph_workspace_bytes(p.h, 1 << 20, 1, None, bs, ctypes.byref(out)) == 0
    assert out.value > small
    # counts must add up to n
    bc = (ctypes.c_int64 * 2)(10, 20)
    bs2 = (ctypes.c_double * 2)(1.0, 2.0)
    assert S._lib.swsph_workspace_bytes(p.h, 31, 2, bc, bs2, ctypes.byref(out)) == -1
    assert S._lib.swsph_workspace_bytes(p.h, 30, 2, bc, bs2, ctypes.byref(out)) == 0
    bs2[1] = -1.0
    assert S._lib.swsph_workspace_bytes(p.h, 30, 2, bc, bs2, ctypes.byref(out)) == -1
    assert S._lib.swsph_workspace_bytes(p.h, -5, 1, None, bs, ctypes.byref(out)) == -1


def test_calls_reject_bad_particles_on_host(S):
    """Null arrays, missing box ids, unbound workspace: rejected before any
    HIP call (this runs on a machine without a GPU)."""
    p = S.Plan()
    pc = S.ParticlesC()
    pc.n = 100
    pc.n_box = 1
    bs = np.array([1.0])
    pc.box_size = bs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ws = ctypes.c_void_p(256)
    assert S._lib.swsph_bin(p.h, ctypes.byref(pc), ws, None) == -1      # null positions
    pc.x = pc.y = pc.z = pc.vx = pc.vy = pc.vz = pc.m = 1024
    pc.n_box = 2
    assert S._lib.swsph_bin(p.h, ctypes.byref(pc), ws, None) == -1      # box ids missing
    pc.n_box = 1
    assert S._lib.swsph_bin(p.h, ctypes.byref(pc), ctypes.c_void_p(260), None) == -1  # alignment
    d = S.DensityOut()
    assert S._lib.swsph_density(p.h, ctypes.byref(pc), ctypes.byref(d), ws, None) == -1
    d.h = d.rho = d.f = 4096
    assert S._lib.swsph_density(p.h, ctypes.byref(pc), ctypes.byref(d), ws, None) == -3  # no bin
    fo = S.ForceOut()
    assert S._lib.swsph_force(p.h, ctypes.byref(pc), ctypes.byref(d), ctypes.byref(fo), ws,
                              None) == -1                                  # u missing
    assert S._lib.swsph_gradient_force(p.h, ctypes.byref(pc), ctypes.byref(d), None,
                                       ctypes.byref(fo), ws, None) == -1   # gradient output
    st = S.Stats()
    assert S._lib.swsph_read_stats(p.h, ws, ctypes.byref(st), None) == -3
    # FIXED_H needs h
    q = S.Plan(flags=S.FIXED_H)
    assert S._lib.swsph_bin(q.h, ctypes.byref(pc), ws, None) == -1



def test_static_step_rejects_oversized_set_on_host(S):
    """swsph_step_static refuses a set whose workspace exceeds its static
    scratch before any HIP call (this runs on a machine without a GPU)."""
    p = S.Plan()
    pc = S.ParticlesC()
    pc.n = 1 << 20
    pc.n_box = 1
    bs = np.array([1.0])
    pc.box_size = bs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pc.x = pc.y = pc.z = pc.vx = pc.vy = pc.vz = pc.m = pc.u = 1024
    d = S.DensityOut()
    assert S._lib.swsph_step_static(p.h, ctypes.byref(pc), ctypes.byref(d), None, None,
                                    None) == -1
    assert b"static scratch" in S._lib.swsph_last_error()
    assert S._lib.swsph_step_static(p.h, ctypes.byref(pc), None, None, None, None) == -1


def test_switch_call_rejects_bad_arguments_on_host(S):
    """swsph_gradient_force_sw checks its parameters and state on the host."""
    p = S.Plan()
    pc = S.ParticlesC()
    pc.n = 100
    pc.n_box = 1
    bs = np.array([1.0])
    pc.box_size = bs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pc.x = pc.y = pc.z = pc.vx = pc.vy = pc.vz = pc.m = pc.u = 1024
    d = S.DensityOut()
    d.h = d.rho = d.f = 4096
    sp = S.SwitchParams(dt=1e-3, **S.SWITCH_DEFAULTS)
    st = S.SwitchState(1024, 1024, 1024, 1024, None, None)
    go = S.GradientOut(1024, 1024)
    fo = S.ForceOut(1024, 1024, 1024, 1024, None)
    ws = ctypes.c_void_p(256)
    call = lambda: S._lib.swsph_gradient_force_sw(p.h, ctypes.byref(pc), ctypes.byref(d),
                                                  ctypes.byref(sp), ctypes.byref(st),
                                                  ctypes.byref(go), ctypes.byref(fo), ws, None)
    assert call() == -1                              # density lacks div v / curl v
    d.div_v = d.curl_x = d.curl_y = d.curl_z = 4096
    assert call() == -3                              # no bin on this plan
    sp.dt = 0.0
    assert call() == -1
    sp.dt = 1e-3
    sp.ac_max = -1.0
    assert call() == -1
    sp.ac_max = 1.0
    st.alpha_c = None
    assert call() == -1


def test_kick_drift_rejects_bad_arguments_on_host(S):
    p = S.Plan()
    bs = np.array([1.0])
    bsp = bs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    a = [1024] * 11
    kd = S._lib.swsph_kick_drift
    assert kd(p.h, 10, *a, 0.1, 0.1, None, 2, bsp, None) == -1        # box ids missing
    assert kd(p.h, 10, *a, 0.1, 0.1, None, 65, bsp, None) == -1       # too many boxes
    assert kd(p.h, 10, *a, float("nan"), 0.1, None, 1, bsp, None) == -1
    b = list(a)
    b[7] = None                                                        # ax missing
    assert kd(p.h, 10, *b, 0.1, 0.0, None, 1, bsp, None) == -1
    bs[0] = -1.0
    assert kd(p.h, 10, *a, 0.1, 0.1, None, 1, bsp, None) == -1
