"""GPU adjoint of density -> force against finite differences of the FP64
oracle and against autograd of an independent dense FP64 re-expression.

Bar: FP64 adjoint within 1e-6 of max|g| per input kind against central
differences (the FD step is small enough that its own error is far below).
"""
import os
import sys

import numpy as np
import pytest

from paper_2505_14538_amd import workloads as W

pytestmark = pytest.mark.gpu
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

KINDS = {"x": "gx", "y": "gy", "z": "gz", "vx": "gvx", "vy": "gvy", "vz": "gvz",
         "u": "gu", "m": "gm"}


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2505_14538_amd import swsph
    return swsph


def as64(p):
    q = p.subset(np.arange(p.n))
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m"):
        setattr(q, k, getattr(p, k).astype(np.float64))
    return q


def gpu_adjoint(S, p, w, c, dtype="f64", flags=0):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plan = S.Plan(dtype=dtype, flags=flags, h_tol=1e-14 if dtype == "f64" else 2e-6,
                  h_max_iter=100)
    dp = S.to_device(p, dtype=tdt)
    plan.bin(dp)
    d = plan.density(dp)
    wt = torch.as_tensor(np.asarray(w), dtype=tdt, device="cuda")
    ct = torch.as_tensor(np.asarray(c), dtype=tdt, device="cuda")
    gi = plan.force_backward(dp, d, wt[:, 0].contiguous(), wt[:, 1].contiguous(),
                             wt[:, 2].contiguous(), ct)
    torch.cuda.synchronize()
    st = plan.stats()
    assert st["code"] == 0, st
    return S.host(gi), S.host(d)


def fd_check(O, p, w, c, gi, comps, Rbig, visc=True, S_of=None):
    """Central differences of the oracle loss for the listed (kind, index)."""
    prm = O.Params(tol=1e-15, max_iter=300, visc=visc)
    base = {k: getattr(p, k).astype(np.float64).copy() for k in KINDS}
    wx, wy, wz = (np.ascontiguousarray(w[:, k], dtype=np.float64) for k in range(3))
    cc = np.ascontiguousarray(c, dtype=np.float64)
    out = {}
    for kind, idx in comps:
        delta = {"u": 1e-5 * base["u"][idx], "m": 1e-5 * base["m"][idx]}.get(
            kind, 1e-6 if kind in ("x", "y", "z") else 1e-5)
        Sset = np.arange(p.n) if S_of is None else S_of(idx)
        vals = []
        for sgn in (1, -1):
            a = {k: v.copy() for k, v in base.items()}
            a[kind][idx] += sgn * delta
            vals.append(O.loss_subset(a["x"], a["y"], a["z"], a["vx"], a["vy"], a["vz"], a["u"],
                                      a["m"], 1.0, prm, Sset, wx, wy, wz, cc, Rbig=Rbig))
        out.setdefault(kind, []).append(((vals[0] - vals[1]) / (2 * delta), gi[KINDS[kind]][idx]))
    return {k: np.array(v) for k, v in out.items()}


@pytest.mark.parametrize("visc", [True, False])
def test_adjoint_fd_small_box(S, oracle_mod, visc):
    """FP64 adjoint vs oracle central differences, 8^3 jittered box."""
    O = oracle_mod
    p, w, c = W.diff(nside=8)
    p = as64(p)
    gi, _ = gpu_adjoint(S, p, w, c, flags=0 if visc else S.NO_VISC)
    rng = np.random.default_rng(1)
    comps = [(k, int(i)) for k in KINDS for i in rng.choice(p.n, 5, replace=False)]
    res = fd_check(O, p, w, c, gi, comps, Rbig=0.499, visc=visc)
    for kind, arr in res.items():
        scale = np.abs(gi[KINDS[kind]]).max()
        err = np.abs(arr[:, 0] - arr[:, 1]).max() / scale
        assert err < 1e-6, (kind, err)


def test_adjoint_fd_odd_count(S, oracle_mod):
    """An odd particle count (7^3): the adjoint's per-particle scratch arrays
    are padded so every 4-vector view stays aligned; FP64 adjoint vs oracle
    central differences."""
    O = oracle_mod
    p, w, c = W.diff(nside=7)
    p = as64(p)
    assert p.n % 2 == 1
    gi, _ = gpu_adjoint(S, p, w, c)
    rng = np.random.default_rng(4)
    comps = [(k, int(i)) for k in KINDS for i in rng.choice(p.n, 3, replace=False)]
    res = fd_check(O, p, w, c, gi, comps, Rbig=0.499)
    for kind, arr in res.items():
        scale = np.abs(gi[KINDS[kind]]).max()
        err = np.abs(arr[:, 0] - arr[:, 1]).max() / scale
        assert err < 1e-6, (kind, err)


@pytest.mark.parametrize("nside", [8, 7])
def test_adjoint_matches_dense_autograd(S, nside):
    """FP64 adjoint vs torch.autograd of the dense re-expression (N = 512
    and the odd N = 343)."""
    import torch
    import dense_reference as DR
    p, w, c = W.diff(nside=nside)
    p = as64(p)
    gi, _ = gpu_adjoint(S, p, w, c)
    x = torch.tensor(np.stack([p.x, p.y, p.z], 1), dtype=torch.float64, requires_grad=True)
    v = torch.tensor(np.stack([p.vx, p.vy, p.vz], 1), dtype=torch.float64, requires_grad=True)
    u = torch.tensor(p.u, dtype=torch.float64, requires_grad=True)
    m = torch.tensor(p.m, dtype=torch.float64, requires_grad=True)
    a, du = DR.forward(x, v, u, m)
    Lss = (a * torch.tensor(w, dtype=torch.float64)).sum() + (du * torch.tensor(c, dtype=torch.float64)).sum()
    gx, gv, gu, gm = (t.numpy() for t in torch.autograd.grad(Lss, [x, v, u, m]))
    ref = {"gx": gx[:, 0], "gy": gx[:, 1], "gz": gx[:, 2], "gvx": gv[:, 0], "gvy": gv[:, 1],
           "gvz": gv[:, 2], "gu": gu, "gm": gm}
    for k, r in ref.items():
        err = np.abs(gi[k] - r).max() / np.abs(r).max()
        assert err < 1e-9, (k, err)


def test_adjoint_fd_diff_config_subblock(S, oracle_mod):
    """Differentiation workload: 64^3 jittered box, v ~ N(0, 0.1),
    u ~ U(0.5, 1.5); FP64 adjoint vs oracle central differences on sampled
    components of the 16^3 sub-block k in [24, 40)^3."""
    O = oracle_mod
    nside = 64
    p, w, c = W.diff(nside=nside)
    p = as64(p)
    gi, d = gpu_adjoint(S, p, w, c)
    k = np.arange(p.n)
    ix, iy, iz = k // (nside * nside), (k // nside) % nside, k % nside
    sub = k[(ix >= 24) & (ix < 40) & (iy >= 24) & (iy < 40) & (iz >= 24) & (iz < 40)]
    Hmax = 2.0 * float(np.max(d["h"]))
    Rbig = 1.05 * Hmax
    rng = np.random.default_rng(2)
    comps = [(kk, int(i)) for kk in KINDS for i in rng.choice(sub, 3, replace=False)]

    def S_of(idx):
        lst, _ = O.neighbour_sets(p.x, p.y, p.z, 1.0, np.full(p.n, 2.2 * Rbig), idx=[idx],
                                  mode="cells", cap=8192)
        return np.concatenate([lst[0], [idx]])

    res = fd_check(O, p, w, c, gi, comps, Rbig=Rbig, S_of=S_of)
    for kind, arr in res.items():
        scale = np.abs(gi[KINDS[kind]][sub]).max()
        err = np.abs(arr[:, 0] - arr[:, 1]).max() / scale
        assert err < 1e-6, (kind, err)


def test_adjoint_fp32_close_to_fp64(S):
    p, w, c = W.diff(nside=16)
    g64, _ = gpu_adjoint(S, as64(p), w, c, dtype="f64")
    g32, _ = gpu_adjoint(S, p, w, c, dtype="f32")
    for k in KINDS.values():
        err = np.abs(g32[k].astype(np.float64) - g64[k]).max() / np.abs(g64[k]).max()
        assert err < 2e-3, (k, err)


def test_autograd_function(S):
    """sph_force through torch.autograd gives the library's adjoint."""
    import torch
    p, w, c = W.diff(nside=8)
    p = as64(p)
    plan = S.Plan(dtype="f64", h_tol=1e-14, h_max_iter=100)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda",
                               requires_grad=True)
    ins = [t(p.x), t(p.y), t(p.z), t(p.vx), t(p.vy), t(p.vz), t(p.u), t(p.m)]
    ax, ay, az, du = S.sph_force(plan, *ins)
    wt = torch.tensor(w, dtype=torch.float64, device="cuda")
    ct = torch.tensor(c, dtype=torch.float64, device="cuda")
    Lss = (ax * wt[:, 0]).sum() + (ay * wt[:, 1]).sum() + (az * wt[:, 2]).sum() + (du * ct).sum()
    grads = torch.autograd.grad(Lss, ins)
    gi, _ = gpu_adjoint(S, p, w, c)
    for gk, gt in zip(KINDS.values(), grads):
        assert np.allclose(gt.cpu().numpy(), gi[gk], rtol=1e-12, atol=1e-12 * np.abs(gi[gk]).max())
