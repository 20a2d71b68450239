"""Test helpers: population-order permutation between the library and the
oracle (matched by velocity vector), norms and scenario setup for both."""
import numpy as np

from oracle import pyoracle as O
from paper_1503_06869_amd import lbm


def perm_lib_to_oracle():
    """perm[q_lib] = q_oracle with c_lib[q] == c_oracle[perm[q]]."""
    cl, _ = lbm.lattice()
    co, _, _ = O.lattice()
    perm = np.zeros(19, int)
    for q in range(19):
        perm[q] = int(np.nonzero((co == cl[q]).all(1))[0][0])
    return perm


def to_oracle_order(f_lib):
    perm = perm_lib_to_oracle()
    out = np.empty_like(f_lib)
    out[perm] = f_lib
    return out


def to_lib_order(f_or):
    return f_or[perm_lib_to_oracle()]


def rel_l2(a, b, mask=None):
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_pair(sc, storage="f32", coupling="implicit", stream=None, history=4096, **kw):
    """GPU context and oracle sim for a scenario, fibers added to both."""
    g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u,
                    init_couette=sc.init_couette, storage=storage, coupling=coupling,
                    stream=stream, history_capacity=history, **kw)
    o = O.Sim(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u,
              init_couette=sc.init_couette, coupling=coupling,
              z_periodic=kw.get("z_periodic", False))
    for f in sc.fibers:
        g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
        o.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    return g, o


def ft_error(hg, ho, lengths):
    """Force and torque errors, max over steps and fibers, each relative to
    the fiber's hydrodynamic load over the run: F errors to
    max(max_t |F_or|, max_t |M_or| / L), M errors to max(max_t |M_or|,
    L max_t |F_or|).  (A fiber centred in the shear cell has zero net force
    by symmetry, so |F_or| alone is no scale.)  hg, ho: [steps][fibers][19]."""
    L = np.asarray(lengths, dtype=np.float64)
    dF = np.linalg.norm(hg[:, :, 0:3] - ho[:, :, 0:3], axis=2).max(0)
    dM = np.linalg.norm(hg[:, :, 3:6] - ho[:, :, 3:6], axis=2).max(0)
    nF = np.linalg.norm(ho[:, :, 0:3], axis=2).max(0)
    nM = np.linalg.norm(ho[:, :, 3:6], axis=2).max(0)
    refF = np.maximum(nF, nM / L)
    refM = np.maximum(nM, nF * L)
    return float((dF / refF).max()), float((dM / refM).max())
