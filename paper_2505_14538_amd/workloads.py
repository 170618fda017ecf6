"""Seeded synthetic particle sets for the SPH neighbour loops.

This module only draws numbers: positions, velocities, internal energies,
masses and loss weights.  It holds none of the method's arithmetic (no
kernel, no density, no force), so both the FP64 oracle and the HIP library
can be fed from it without sharing any of the computation.

Every workload lives in periodic cubic boxes of side ``L = 1`` and is fully
determined by its seed (``numpy.random.default_rng``).  Positions are
float32 and lie in ``[0, L)``.

Workloads (sizes and distributions follow the setups that the paper's
offloaded loops were measured on: a unit periodic box, uniformly spaced
particles, gamma = 5/3 -- Section 3.1 -- scaled here to the particle counts
the benchmarks use):

* ``tiny``        16^3 jittered lattice, u = 1, v ~ N(0, 0.01)
* ``sedov``       64^3 jittered lattice, v = 0, u = 1e-6 except u = 1 on the
                  32 particles nearest the box centre
* ``clustered``   2^21 particles drawn from a lognormal density field on a
                  64^3 grid (Gaussian-smoothed white noise), u ~ U(0.5, 1.5),
                  v ~ N(0, 0.1)
* ``many_boxes``  256 independent boxes with log-uniform particle counts in
                  [2048, 65536] (rounded to cubes), jittered lattices
* ``diff``        64^3 jittered lattice, v ~ N(0, 0.1), u ~ U(0.5, 1.5),
                  plus loss weights w ~ N(0, 1)^3, c ~ N(0, 1)
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

GAMMA = 5.0 / 3.0
BASE_SEED = 14538


@dataclasses.dataclass
class Particles:
    """Host-side particle set in original (generator) order, float32 SoA."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    u: np.ndarray
    m: np.ndarray
    box_size: np.ndarray          # float64 [n_box]
    box_id: Optional[np.ndarray]  # int32 [n] or None for a single box
    name: str = ""
    seed: int = 0
    h_guess: Optional[np.ndarray] = None  # float32 [n] or None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_box(self) -> int:
        return int(self.box_size.shape[0])

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def vel(self) -> np.ndarray:
        return np.stack([self.vx, self.vy, self.vz], axis=1)

    def box_slices(self):
        """Yield (b, index array) for each box."""
        if self.box_id is None:
            yield 0, np.arange(self.n)
            return
        order = np.argsort(self.box_id, kind="stable")
        counts = np.bincount(self.box_id, minlength=self.n_box)
        start = 0
        for b in range(self.n_box):
            yield b, order[start:start + counts[b]]
            start += counts[b]

    def subset(self, idx: np.ndarray) -> "Particles":
        bid = None if self.box_id is None else self.box_id[idx]
        hg = None if self.h_guess is None else self.h_guess[idx]
        return Particles(self.x[idx], self.y[idx], self.z[idx], self.vx[idx],
                         self.vy[idx], self.vz[idx], self.u[idx], self.m[idx],
                         self.box_size.copy(), bid, self.name, self.seed, hg)


def _f32_in_box(a: np.ndarray, L: float) -> np.ndarray:
    """Wrap float64 coordinates into [0, L) and round to float32 < L."""
    a = np.mod(a, L)
    f = a.astype(np.float32)
    top = np.nextafter(np.float32(L), np.float32(0))
    f = np.where(f >= np.float32(L), top, f)
    f = np.where(f < 0, np.float32(0), f)
    return f.astype(np.float32)


def jittered_lattice(nside: int, rng: np.random.Generator, L: float = 1.0,
                     jitter: float = 0.1) -> np.ndarray:
    """(k + 1/2) * dx + U(-jitter, jitter) * dx per component, raster order."""
    dx = L / nside
    k = np.arange(nside, dtype=np.float64)
    gx, gy, gz = np.meshgrid(k, k, k, indexing="ij")
    p = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    p = (p + 0.5) * dx
    if jitter > 0:
        p = p + rng.uniform(-jitter, jitter, size=p.shape) * dx
    return p


def lattice(nside: int, L: float = 1.0) -> np.ndarray:
    """Unjittered lattice (k + 1/2) * dx (exact in float32 for nside = 2^k)."""
    return jittered_lattice(nside, np.random.default_rng(0), L, jitter=0.0)


def _pack(pos, vel, u, m, L, name, seed, box_id=None, box_size=None):
    if box_size is None:
        box_size = np.array([L], dtype=np.float64)
    return Particles(
        x=_f32_in_box(pos[:, 0], L) if box_id is None else pos[:, 0].astype(np.float32),
        y=_f32_in_box(pos[:, 1], L) if box_id is None else pos[:, 1].astype(np.float32),
        z=_f32_in_box(pos[:, 2], L) if box_id is None else pos[:, 2].astype(np.float32),
        vx=vel[:, 0].astype(np.float32), vy=vel[:, 1].astype(np.float32),
        vz=vel[:, 2].astype(np.float32), u=u.astype(np.float32),
        m=m.astype(np.float32), box_size=np.asarray(box_size, dtype=np.float64),
        box_id=box_id, name=name, seed=seed)


def tiny(nside: int = 16, seed: Optional[int] = None) -> Particles:
    """Plain method, tiny: 16^3 jittered lattice, u = 1, v ~ N(0, 0.01)."""
    seed = BASE_SEED + 0 if seed is None else seed
    rng = np.random.default_rng(seed)
    n = nside ** 3
    pos = jittered_lattice(nside, rng)
    vel = rng.normal(0.0, 0.01, size=(n, 3))
    return _pack(pos, vel, np.ones(n), np.full(n, 1.0 / n), 1.0, "tiny", seed)


def sedov(nside: int = 64, seed: Optional[int] = None, n_hot: int = 32) -> Particles:
    """Plain method, medium: jittered lattice, v = 0, u = 1e-6 except u = 1
    on the ``n_hot`` particles nearest the centre (minimum-image distance in
    float64 on the float32 positions, ties broken by lower index)."""
    seed = BASE_SEED + 1 if seed is None else seed
    rng = np.random.default_rng(seed)
    n = nside ** 3
    pos = jittered_lattice(nside, rng)
    p32 = pos.astype(np.float32).astype(np.float64)
    d = p32 - 0.5
    d -= np.round(d)
    r2 = np.einsum("ij,ij->i", d, d)
    hot = np.lexsort((np.arange(n), r2))[:n_hot]
    u = np.full(n, 1e-6)
    u[hot] = 1.0
    return _pack(pos, np.zeros((n, 3)), u, np.full(n, 1.0 / n), 1.0, "sedov", seed)


def _smoothed_noise(ngrid: int, sigma_cells: float, rng: np.random.Generator) -> np.ndarray:
    noise = rng.standard_normal((ngrid, ngrid, ngrid))
    k = np.fft.fftfreq(ngrid) * ngrid  # integer wavenumbers
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    # Gaussian of width sigma_cells in real space -> exp(-k^2 s^2 (2 pi / n)^2 / 2)
    s = sigma_cells * 2.0 * np.pi / ngrid
    filt = np.exp(-0.5 * (kx ** 2 + ky ** 2 + kz ** 2) * s * s)
    g = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    g = (g - g.mean()) / g.std()
    return g


def clustered(n: int = 2 ** 21, ngrid: int = 64, sigma_ln: float = 1.5,
              sigma_smooth: float = 2.0, seed: Optional[int] = None) -> Particles:
    """Batched, clustered: lognormal density field sampled by a multinomial
    draw of exactly ``n`` particles over a periodic ``ngrid``^3 grid.

    delta = sigma_ln * g - sigma_ln^2 / 2 with g the standardised
    Gaussian-smoothed white noise; expected count per grid cell is
    proportional to exp(delta).  Positions are uniform inside each grid cell;
    particles come out grouped by grid cell in raster order.
    """
    seed = BASE_SEED + 2 if seed is None else seed
    rng = np.random.default_rng(seed)
    g = _smoothed_noise(ngrid, sigma_smooth, rng)
    delta = sigma_ln * g - 0.5 * sigma_ln ** 2
    p = np.exp(delta).ravel()
    p /= p.sum()
    counts = rng.multinomial(n, p)
    cell = np.repeat(np.arange(ngrid ** 3), counts)
    ci = np.stack(np.unravel_index(cell, (ngrid, ngrid, ngrid)), axis=1).astype(np.float64)
    pos = (ci + rng.uniform(0.0, 1.0, size=(n, 3))) / ngrid
    vel = rng.normal(0.0, 0.1, size=(n, 3))
    u = rng.uniform(0.5, 1.5, size=n)
    return _pack(pos, vel, u, np.full(n, 1.0 / n), 1.0, "clustered", seed)


def many_boxes(n_box: int = 256, nmin: int = 2048, nmax: int = 65536,
               seed: Optional[int] = None) -> Particles:
    """Batched, many boxes: independent unit periodic boxes; per box
    N_b = round(exp(U(ln nmin, ln nmax))), side n_b = round(N_b^(1/3)),
    N_b := n_b^3 (a lattice needs a cube); jittered lattice, v ~ N(0, 0.05),
    u = 1, m = 1 / N_b.  Particles are grouped by box."""
    seed = BASE_SEED + 3 if seed is None else seed
    rng = np.random.default_rng(seed)
    nb = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=n_box))).astype(np.int64)
    side = np.rint(np.cbrt(nb)).astype(np.int64)
    pos_l, vel_l, m_l, id_l = [], [], [], []
    for b in range(n_box):
        p = jittered_lattice(int(side[b]), rng)
        p = np.stack([_f32_in_box(p[:, d], 1.0) for d in range(3)], axis=1)
        nbb = p.shape[0]
        pos_l.append(p)
        vel_l.append(rng.normal(0.0, 0.05, size=(nbb, 3)))
        m_l.append(np.full(nbb, 1.0 / nbb))
        id_l.append(np.full(nbb, b, dtype=np.int32))
    pos = np.concatenate(pos_l)
    vel = np.concatenate(vel_l)
    m = np.concatenate(m_l)
    box_id = np.concatenate(id_l)
    return _pack(pos, vel, np.ones(pos.shape[0]), m, 1.0, "many_boxes", seed,
                 box_id=box_id, box_size=np.ones(n_box))


def diff(nside: int = 64, seed: Optional[int] = None):
    """Differentiation: jittered lattice, v ~ N(0, 0.1), u ~ U(0.5, 1.5).
    Returns (particles, w [n,3] float32, c [n] float32) for the loss
    L = sum_i w_i . a_i + c_i du_i/dt."""
    seed = BASE_SEED + 4 if seed is None else seed
    rng = np.random.default_rng(seed)
    n = nside ** 3
    pos = jittered_lattice(nside, rng)
    vel = rng.normal(0.0, 0.1, size=(n, 3))
    u = rng.uniform(0.5, 1.5, size=n)
    p = _pack(pos, vel, u, np.full(n, 1.0 / n), 1.0, "diff", seed)
    w = rng.normal(0.0, 1.0, size=(n, 3)).astype(np.float32)
    c = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    return p, w, c


def gresho_profiles(r):
    """Azimuthal velocity and pressure of the Gresho-Chan vortex (Sec. 3.1,
    Eq. 27-28) at cylindrical radius r (rho = 1): v = 5r, 2 - 5r, 0 and
    P = 5 + 12.5 r^2, 9 - 4 ln 0.2 + 12.5 r^2 - 20 r + 4 ln r, 3 + 4 ln 2 on
    [0, 0.2), [0.2, 0.4), [0.4, inf)."""
    r = np.asarray(r, dtype=np.float64)
    v = np.where(r < 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))
    rr = np.maximum(r, 1e-300)
    P = np.where(r < 0.2, 5.0 + 12.5 * r * r,
                 np.where(r < 0.4,
                          9.0 - 4.0 * np.log(0.2) + 12.5 * r * r - 20.0 * r + 4.0 * np.log(rr),
                          3.0 + 4.0 * np.log(2.0)))
    return v, P


def gresho(nside: int = 64, gamma: float = 5.0 / 3.0) -> Particles:
    """Gresho-Chan vortex initial conditions (Sec. 3.1): nside^3 particles on
    a cubic lattice in the periodic unit box, density 1 (m = 1/N), the
    vortex axis parallel to z through (1/2, 1/2), azimuthal velocity and
    pressure of Eq. 27-28, u = P / ((gamma - 1) rho)."""
    pos = lattice(nside)
    n = pos.shape[0]
    dx, dy = pos[:, 0] - 0.5, pos[:, 1] - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    v, P = gresho_profiles(r)
    vel = np.stack([-v * dy / r, v * dx / r, np.zeros(n)], axis=1)
    return _pack(pos, vel, P / (gamma - 1.0), np.full(n, 1.0 / n), 1.0, "gresho", 0)


def shuffled(p: Particles, seed: int = 7) -> Particles:
    """Same particles in a random order (tests that results do not depend on
    input order)."""
    perm = np.random.default_rng(seed).permutation(p.n)
    return p.subset(perm)


WORKLOADS = {
    "tiny": tiny,
    "sedov": sedov,
    "clustered": clustered,
    "many_boxes": many_boxes,
}
