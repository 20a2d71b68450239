"""Seeded synthetic inputs for the shear-flow fiber workloads.

This module holds only input generation (poses, placements, lattice sizes,
random perturbations); none of the method's arithmetic lives here.  The GPU
library, the oracle and the benchmark all take their inputs from it, so the
two implementations see identical poses.  All randomness comes from numpy's
PCG64 seeded per workload.

Units are lattice units.  Cell centres sit at integer coordinates; the
walls of a shear cell lie half-way below z = 0 and above z = nz - 1 and move
at -U (bottom) and +U (top) along x, so the shear rate is 2U/nz.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def axis_uniform_on_sphere(g):
    """Unit vector uniform on the sphere: z ~ U[-1, 1], phi ~ U[0, 2 pi)."""
    z = g.uniform(-1.0, 1.0)
    phi = g.uniform(0.0, 2.0 * np.pi)
    s = np.sqrt(max(0.0, 1.0 - z * z))
    return np.array([s * np.cos(phi), s * np.sin(phi), z])


def quat_from_axis(t):
    """Unit quaternion (w, x, y, z) of the shortest rotation taking e_x to t."""
    t = np.asarray(t, dtype=np.float64)
    t = t / np.linalg.norm(t)
    q = np.array([1.0 + t[0], 0.0, -t[2], t[1]])
    n = np.linalg.norm(q)
    if n < 1e-12:                      # t = -e_x: half turn about z
        return np.array([0.0, 0.0, 0.0, 1.0])
    return q / n


@dataclass
class Fiber:
    X: np.ndarray          # centre (3)
    q: np.ndarray          # orientation quaternion (4), axis = R(q) e_x
    length: float
    radius: float
    density_ratio: float = 1.0
    V: np.ndarray = field(default_factory=lambda: np.zeros(3))
    W: np.ndarray = field(default_factory=lambda: np.zeros(3))


@dataclass
class Scenario:
    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    wall_u: float
    fibers: List[Fiber]
    steps: int
    magic: float = 3.0 / 16.0
    rho0: float = 1.0
    init_couette: bool = True

    @property
    def shear_rate(self):
        return 2.0 * self.wall_u / self.nz

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz


def couette_velocity(z, wall_u, nz):
    """Linear shear profile between the half-way walls."""
    return wall_u * (2.0 * (np.asarray(z, dtype=np.float64) + 0.5) / nz - 1.0)


def _initial_motion(X, wall_u, nz):
    """Fiber starts with the local fluid velocity and half the vorticity."""
    gd = 2.0 * wall_u / nz
    V = np.array([couette_velocity(X[2], wall_u, nz), 0.0, 0.0])
    W = np.array([0.0, 0.5 * gd, 0.0])
    return V, W


# ------------------------------------------------------------------ single fiber
def single_fiber(seed=0, n=32, tau=0.8, wall_u=0.005, length=16.0, diameter=4.0,
                 density_ratio=1.0, steps=3000, reject_ty=0.95):
    """One centred cylinder in an n^3 shear cell, orientation uniform on the
    sphere from the seed (log-rolling draws with |t_y| > reject_ty redrawn)."""
    g = rng(seed)
    while True:
        t = axis_uniform_on_sphere(g)
        if abs(t[1]) <= reject_ty:
            break
    X = np.array([(n - 1) / 2.0] * 3)
    V, W = _initial_motion(X, wall_u, n)
    f = Fiber(X, quat_from_axis(t), length, diameter / 2.0, density_ratio, V, W)
    return Scenario("single_fiber_%d" % n, n, n, n, tau, wall_u, [f], steps)


# ------------------------------------------------------------------ placement
def segment_distance(p1, d1, p2, d2):
    """Minimum distance between segments p1 + s d1 and p2 + t d2, s,t in [0,1]."""
    r = p1 - p2
    a, e, f = d1 @ d1, d2 @ d2, d2 @ r
    c, b = d1 @ r, d1 @ d2
    den = a * e - b * b
    s = np.clip((b * f - c * e) / den, 0.0, 1.0) if den > 1e-14 else 0.0
    t = (b * s + f) / e
    if t < 0.0:
        t, s = 0.0, np.clip(-c / a, 0.0, 1.0)
    elif t > 1.0:
        t, s = 1.0, np.clip((b - c) / a, 0.0, 1.0)
    return float(np.linalg.norm(p1 + s * d1 - (p2 + t * d2)))


def _capsule_gap(Xa, ta, La, ra, Xb, tb, Lb, rb, box):
    """Surface gap of two capsules (cylinders bounded by their capsules),
    minimum image in x and y."""
    d = Xb - Xa
    for k in (0, 1):
        d[k] -= box[k] * np.round(d[k] / box[k])
    pa = -0.5 * La * ta
    pb = d - 0.5 * Lb * tb
    return segment_distance(pa, La * ta, pb, Lb * tb) - ra - rb


def place_fibers(g, n_fibers, box, lengths, radii, min_gap=2.0, z_clear=2.0,
                 max_tries=200000):
    """Uniform non-overlapping placement by rejection sampling: capsule gap
    >= min_gap, and every fiber keeps |t_z| L/2 + r + z_clear from the walls."""
    nx, ny, nz = box
    placed = []
    tries = 0
    for i in range(n_fibers):
        L, r = lengths[i], radii[i]
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("placement failed after %d tries" % max_tries)
            t = axis_uniform_on_sphere(g)
            hz = 0.5 * L * abs(t[2]) + r + z_clear
            if 2 * hz >= nz - 1:
                continue
            X = np.array([g.uniform(0, nx), g.uniform(0, ny), g.uniform(hz, nz - 1 - hz)])
            ok = all(_capsule_gap(X, t, L, r, Y, s, M, rr, box) >= min_gap
                     for (Y, s, M, rr) in placed)
            if ok:
                placed.append((X, t, L, r))
                break
    return placed


def many_fibers(seed=0, n=256, n_fibers=64, tau=0.8, wall_u=0.01, length=(24.0, 40.0),
                diameter=(4.0, 6.0), density_ratio=1.0, steps=5000, nz=None):
    """Large shear cell: lengths and diameters uniform in the given ranges,
    positions uniform and non-overlapping, orientations uniform on the sphere."""
    g = rng(seed)
    nz = nz or n
    lengths = g.uniform(*length, size=n_fibers)
    radii = 0.5 * g.uniform(*diameter, size=n_fibers)
    placed = place_fibers(g, n_fibers, (n, n, nz), lengths, radii)
    fibers = []
    for X, t, L, r in placed:
        V, W = _initial_motion(X, wall_u, nz)
        fibers.append(Fiber(X, quat_from_axis(t), float(L), float(r), density_ratio, V, W))
    return Scenario("many_fibers_%d" % n, n, n, nz, tau, wall_u, fibers, steps)


# ------------------------------------------------------------------ batched cases
def batched_cases(seed=0, n_cases=512, edge=(24, 64), ar=(2.0, 10.0), diameter=4.0,
                  shear=(1e-4, 5e-4), tau=(0.6, 1.0), steps=4000, margin=8.0):
    """Independent shear cells of uneven size, one centred cylinder each.
    Aspect ratios are redrawn until L <= min(edge) - margin so that the
    fiber fits between the walls and does not meet its own periodic image."""
    g = rng(seed)
    cases = []
    for _ in range(n_cases):
        nx, ny, nz = (int(v) for v in g.integers(edge[0], edge[1] + 1, size=3))
        while True:
            a = g.uniform(*ar)
            L = a * diameter
            if L <= min(nx, ny, nz) - margin:
                break
        gd = g.uniform(*shear)
        tu = g.uniform(*tau)
        t = axis_uniform_on_sphere(g)
        U = gd * nz / 2.0
        X = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
        V, W = _initial_motion(X, U, nz)
        f = Fiber(X, quat_from_axis(t), float(L), diameter / 2.0, 1.0, V, W)
        cases.append(Scenario("case", nx, ny, nz, float(tu), float(U), [f], steps))
    return cases


def learned_coarse(seed=0, n=128, n_fibers=200, ar=(4.0, 12.0), diameter=2.0, wall_u=0.01, tau=0.8,
                   steps=5000):
    """Coarse shear cell of the learned form: under-resolved cylinders of
    diameter 2, aspect ratio uniform in `ar`, placed as in many_fibers."""
    g = rng(seed)
    lengths = g.uniform(*ar, size=n_fibers) * diameter
    radii = np.full(n_fibers, diameter / 2.0)
    fibers = []
    for X, t, L, r in place_fibers(g, n_fibers, (n, n, n), lengths, radii):
        V, W = _initial_motion(X, wall_u, n)
        fibers.append(Fiber(X, quat_from_axis(t), float(L), float(r), 1.0, V, W))
    return Scenario("learned_coarse_%d" % n, n, n, n, tau, wall_u, fibers, steps)


# ------------------------------------------------------------------ parity inputs
def random_populations(seed, shape, weights, amplitude=1e-3, velocity=0.02):
    """Near-equilibrium random populations [19][nz][ny][nx] around rest
    weights: w_q (1 + 3 c.u) with a smooth random u plus white noise.  The
    caller supplies the weights and velocities table it uses."""
    g = rng(seed)
    nx, ny, nz = shape
    w, c = weights
    u = velocity * g.standard_normal((3, nz, ny, nx))
    cu = np.einsum("qa,azyx->qzyx", c.astype(np.float64), u)
    f = w[:, None, None, None] * (1.0 + 3.0 * cu)
    f += amplitude * w[:, None, None, None] * g.standard_normal(f.shape)
    return f


# ------------------------------------------------------------------ slender-body workloads
@dataclass
class SbfScenario:
    name: str
    length: float
    eps: float
    X: np.ndarray          # [m][3] centres
    p: np.ndarray          # [m][3] unit directions
    F: np.ndarray          # [m][3] external forces
    M: np.ndarray          # [m][3] external torques
    mu: float = 1.0


def sbf_cloud(seed=0, m=1024, length=48.0, eps=1.0 / 12.0, spacing=2.0, force=(0.0, 0.0, 1.0)):
    """m fibers of length L (in units of the fiber radius times 1/eps, the
    paper's r = 4 dx fibers of 1/eps = 12 by default) in a cubic cloud of
    mean volume (spacing L)^3 per fiber, centres uniform with a minimum
    centre distance of L/4, orientations uniform on the sphere, the same
    force (gravity) on every fiber, no torque: a sedimenting suspension in
    free space."""
    g = rng(seed)
    side = spacing * length * m ** (1.0 / 3.0)
    X = np.zeros((m, 3))
    k = 0
    while k < m:
        c = g.uniform(0.0, side, 3)
        if k == 0 or np.min(np.linalg.norm(X[:k] - c, axis=1)) >= 0.25 * length:
            X[k] = c
            k += 1
    p = np.array([axis_uniform_on_sphere(g) for _ in range(m)])
    F = np.tile(np.asarray(force, dtype=np.float64), (m, 1))
    return SbfScenario("sbf_cloud_%d" % m, length, eps, X, p, F, np.zeros((m, 3)))


def sbf_pair(dist=15.1, aspect=12.0, radius=4.0, tilt=0.0, force=1.0):
    """The paper's tumbling start for the slender-body model: two fibers of
    radius r and aspect ratio 1/eps = L/r aligned with gravity (z), centres
    dist apart along x; tilt rotates both axes about y (opposite senses)."""
    length = radius * aspect
    X = np.array([[-0.5 * dist, 0.0, 0.0], [0.5 * dist, 0.0, 0.0]])
    p = np.array([[np.sin(tilt), 0.0, np.cos(tilt)], [-np.sin(tilt), 0.0, np.cos(tilt)]])
    F = np.array([[0.0, 0.0, force], [0.0, 0.0, force]])
    return SbfScenario("sbf_pair", length, 1.0 / aspect, X, p, F, np.zeros((2, 3)))
