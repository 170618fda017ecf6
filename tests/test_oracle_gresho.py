"""Pins of the Gresho-Chan initial conditions (Sec. 3.1, Eq. 27-28) and of
the oracle's leapfrog step, against facts that fix them: the vortex is in
hydrostatic balance (dP/dr = rho v^2 / r, rho = 1) with continuous
profiles; the generated particles carry exactly that flow; and a uniform
translation of a lattice feels no force, so one step moves every particle by
v dt and changes nothing else.  None needs a GPU."""
import numpy as np
import pytest

from paper_2505_14538_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def as64(p):
    q = p.subset(np.arange(p.n))
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m"):
        setattr(q, k, getattr(p, k).astype(np.float64))
    return q


def test_gresho_profiles_hydrostatic_balance():
    """Eq. 28's pressure balances the centrifugal force of Eq. 27's flow:
    dP/dr = v^2 / r away from the kinks, and both profiles are continuous at
    r = 0.2 and 0.4 (which pins the constants of the middle piece)."""
    r = np.concatenate([np.linspace(0.01, 0.19, 40), np.linspace(0.21, 0.39, 40),
                        np.linspace(0.41, 0.7, 20)])
    d = 1e-6
    _, Pp = W.gresho_profiles(r + d)
    _, Pm = W.gresho_profiles(r - d)
    v, _ = W.gresho_profiles(r)
    assert np.allclose((Pp - Pm) / (2 * d), v * v / r, rtol=1e-7, atol=1e-8)
    for rk in (0.2, 0.4):
        va, Pa = W.gresho_profiles([rk - 1e-12])
        vb, Pb = W.gresho_profiles([rk + 1e-12])
        assert abs(va[0] - vb[0]) < 1e-9 and abs(Pa[0] - Pb[0]) < 1e-9
    v0, P0 = W.gresho_profiles([0.0])
    assert v0[0] == 0.0 and P0[0] == 5.0


def test_gresho_initial_conditions():
    """Particles on the lattice, azimuthal velocity of Eq. 27 (no radial or
    vertical component), u = P / (gamma - 1) with rho = 1, m = 1/N."""
    p = W.gresho(16)
    n = p.n
    assert n == 16 ** 3
    dx, dy = p.x.astype(np.float64) - 0.5, p.y.astype(np.float64) - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    v, P = W.gresho_profiles(r)
    vr = (dx * p.vx + dy * p.vy) / r
    vphi = (-dy * p.vx + dx * p.vy) / r
    assert np.abs(vr).max() < 1e-6 and np.all(p.vz == 0)
    assert np.abs(vphi - v).max() < 1e-6
    assert np.allclose(p.u, P / (2.0 / 3.0), rtol=1e-6)
    assert np.allclose(p.m, 1.0 / n)


def test_kdk_step_uniform_translation(oracle_mod):
    """A lattice moving as a whole with uniform u: a = 0 and du/dt = 0 by
    symmetry, so one leapfrog step moves every particle by v dt (mod 1) and
    leaves v, u and the switch state's alpha values as they are."""
    O = oracle_mod
    nside = 16  # exact in float32: a perfect lattice, forces cancel to roundoff
    lat = W.lattice(nside)
    n = lat.shape[0]
    vel = np.tile([0.3, -0.2, 0.15], (n, 1))
    p = as64(W._pack(lat, vel, np.full(n, 2.0), np.full(n, 1.0 / n), 1.0, "lat", 0))
    d = O.density(p)
    g = O.gradient(p, d)
    zero = {k: np.zeros(n) for k in ("ax", "ay", "az", "dudt")}
    st = {"alpha_v": np.zeros(n), "alpha_c": np.zeros(n), "div_v_prev": d["div_v"],
          "v_sig_prev": g["v_sig"]}
    dt = 0.01
    q, d1, g1, f1, s1 = O.kdk_step(p, zero, dt, st, O.SwitchParams(dt=dt))
    for k in ("ax", "ay", "az", "dudt"):
        assert np.abs(f1[k]).max() < 1e-9
    for k, vk in (("x", "vx"), ("y", "vy"), ("z", "vz")):
        expect = np.mod(getattr(p, k) + getattr(p, vk) * dt, 1.0)
        diff = np.abs(getattr(q, k) - expect)
        assert np.minimum(diff, 1.0 - diff).max() < 1e-12
    assert np.abs(q.vx - p.vx).max() < 1e-10 and np.abs(q.u - p.u).max() < 1e-10
    assert np.abs(s1["alpha_v"]).max() < 1e-12 and np.abs(s1["alpha_c"]).max() < 1e-12
