"""Momentum stabilization on the GPU, through the C ABI (Sec. 4.1: the mean
fluid velocity is subtracted in every equilibrium, for periodic boxes whose
particles carry a constant force).

The device keeps the mean by bookkeeping (workgroup sums of the sweep, the
collision's uniform change, the cells the remap changes) instead of a pass
over the lattice; the oracle takes the plain mean of its state before every
step.  Checked here: populations, histories and the mean against the oracle
(FP32 at the usual tolerances, FP64 storage near rounding), the bookkept mean
against the mean of the decoded velocity field (every storage, with walls
too), and that a forced particle reaches a terminal velocity instead of
accelerating without bound."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_1503_06869_amd import lbm, scenarios

from helpers import ft_error, rel_l2, to_lib_order, to_oracle_order

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lbm.load()
    yield


def _random_state(shape, seed, amp=0.05, drift=(0.02, -0.012, 0.007)):
    """Populations (oracle order) near equilibrium at a uniform drift plus noise."""
    nx, ny, nz = shape
    c, w, _ = O.lattice()
    rng = np.random.default_rng(seed)
    cu = np.einsum("qa,a->q", c.astype(np.float64), drift)
    feq = w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * np.dot(drift, drift))
    return feq[:, None, None, None] * (1.0 + amp * rng.standard_normal((19, nz, ny, nx)))


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_stabilized_periodic_fluid_matches_oracle(storage, tol):
    """Fully periodic 20 x 18 x 16 box from a drifting random state, tau = 6
    (omega_o = 1.87, where a mean lagging one step would diverge): after 40
    steps populations and mean velocity agree with the oracle, and the total
    momentum has decayed by (1 - omega_o)^40."""
    nx, ny, nz, tau, steps = 20, 18, 16, 6.0, 40
    f0 = _random_state((nx, ny, nz), 7)
    g = lbm.Context(nx, ny, nz, tau=tau, z_periodic=True, storage=storage, stabilize=True)
    o = O.Sim(nx, ny, nz, tau=tau, z_periodic=True, stabilize=True)
    g.set_populations(to_lib_order(f0))
    o.set_populations(f0)
    ug0, n0 = g.mean_velocity()
    uo0, m0 = o.mean_velocity()
    assert n0 == m0 == nx * ny * nz
    np.testing.assert_allclose(ug0, uo0, rtol=tol, atol=0)
    g.step(steps)
    o.step(steps)
    fg = to_oracle_order(g.populations())
    fo = o.populations()
    e = rel_l2(fg - O.lattice()[1][:, None, None, None], fo - O.lattice()[1][:, None, None, None])
    ug, _ = g.mean_velocity()
    uo, _ = o.mean_velocity()
    print("%s: populations rel L2 %.3g, mean %s vs %s" % (storage, e, ug, uo), flush=True)
    assert e < tol
    oo = 8.0 * (2.0 - 1.0 / tau) / (8.0 - 1.0 / tau)
    np.testing.assert_allclose(uo, (1.0 - oo) ** steps * uo0, rtol=1e-9)
    np.testing.assert_allclose(ug, uo, rtol=100 * tol, atol=1e-9 * np.abs(uo0).max())
    g.close()


FIBERS = [  # centre, axis, L, r, shape, external force
    ((13.3, 15.1, 12.6), (0.7, 0.3, 0.65), 12.0, 2.4, "spherocylinder", (4.5e-2, -1.5e-2, 6e-2)),
    ((27.6, 20.4, 19.3), (0.2, 0.9, -0.4), 11.0, 2.0, "cylinder", (-3e-2, 2.4e-2, 4.5e-2)),
]


def _forced_pair(storage, steps_done=0):
    nx, ny, nz = 40, 36, 32
    g = lbm.Context(nx, ny, nz, tau=0.8, z_periodic=True, storage=storage, stabilize=True)
    o = O.Sim(nx, ny, nz, tau=0.8, z_periodic=True, stabilize=True)
    for X, t, L, r, shape, F in FIBERS:
        q = scenarios.quat_from_axis(np.asarray(t) / np.linalg.norm(t))
        g.add_fiber(X, q, L, r, 1.0, shape=shape, force=F)
        o.add_fiber(X, q, L, r, 1.0, shape=shape, force=F)
    return g, o


@pytest.mark.parametrize("storage,tol_u,tol_ft,tol_m", [("f32", 1e-5, 1e-4, 1e-5), ("f64", 1e-11, 1e-10, 1e-10)])
def test_stabilized_forced_particles_match_oracle(storage, tol_u, tol_ft, tol_m):
    """Two forced fibers (one spherocylinder) in a fully periodic 40 x 36 x 32
    box, 240 steps: they move by most of a cell, so cells change owner
    every few steps; maps bit-exact, histories, velocity field and the mean
    velocity the next step subtracts agree with the oracle."""
    steps = 240
    g, o = _forced_pair(storage)
    pid0 = g.fields()[3]
    g.step(steps)
    o.step(steps)
    hg, ho = g.history(0, steps), o.history()
    eF, eM = ft_error(hg, ho, [f[2] for f in FIBERS])
    _, ug, flg, pidg = g.fields()
    _, uo, flo, pido = o.fields()
    assert np.array_equal(pidg, pido) and np.array_equal(flg, flo)
    e = rel_l2(ug.astype(np.float64), uo, flo == 0)
    moved = np.abs(ho[-1, :, 6:9] - ho[0, :, 6:9]).max()
    mg, ng = g.mean_velocity()
    mo, no = o.mean_velocity()
    em = np.abs(mg - mo).max() / np.abs(uo[:, flo == 0]).max()
    print("%s: velocity rel L2 %.3g, F %.3g, M %.3g, moved %.2f cells, mean %s vs %s (%.3g)"
          % (storage, e, eF, eM, moved, mg, mo, em), flush=True)
    changed = int((pidg != pid0).sum())
    print("cells with a new owner: %d" % changed, flush=True)
    assert ng == no
    assert moved > 0.5 and changed > 100
    assert e < tol_u and eF < tol_ft and eM < tol_ft
    assert em < tol_m
    g.close()


@pytest.mark.parametrize("storage,z_periodic,tol,walls", [("f32", True, 2e-6, None), ("f16", True, 5e-6, None),
                                                          ("bf16", True, 3e-5, None), ("f32", False, 2e-6, None),
                                                          ("f32", True, 2e-6, "free-slip"),
                                                          ("f32", False, 2e-6, "free-slip z")])
def test_bookkept_mean_equals_decoded_field_mean(storage, z_periodic, tol, walls):
    """The mean the device keeps without a pass over the lattice equals the
    mean of the decoded velocity over the fluid cells, after steps with
    moving fibers (and, without z periodicity, moving-wall bounce-back;
    with free-slip walls, reflections that reverse one component), and
    again after a state change from the host (recomputed by a full pass)."""
    nx, ny, nz = 40, 36, 32
    kw = {}
    if walls == "free-slip":
        kw = dict(x_walls="free-slip", y_walls="free-slip")
    elif walls == "free-slip z":
        kw = dict(x_walls="free-slip", z_free_slip=True)
    g = lbm.Context(nx, ny, nz, tau=0.8, z_periodic=z_periodic,
                    wall_u=0.0 if (z_periodic or walls) else 0.02,
                    init_couette=not z_periodic and not walls, storage=storage, stabilize=True, **kw)
    for X, t, L, r, shape, F in FIBERS:
        q = scenarios.quat_from_axis(np.asarray(t) / np.linalg.norm(t))
        g.add_fiber(X, q, L, r, 1.0, shape=shape, force=F)
    for n in (1, 37, 200):
        g.step(n)
        ub, nf = g.mean_velocity()
        _, u, _, pid = g.fields()
        fl = pid < 0
        um = u[:, fl].astype(np.float64).mean(axis=1)
        scale = np.abs(u[:, fl]).max()
        print("%s zper=%d step+%d: bookkept %s, field %s, scale %.3g" % (storage, z_periodic, n, ub, um, scale),
              flush=True)
        assert nf == int(fl.sum())
        np.testing.assert_allclose(ub, um, rtol=0, atol=tol * scale)
    X, q, V, W = g.fiber_state()
    g.set_fiber_state(0, X[0], q[0], V[0], W[0])
    ub2, nf2 = g.mean_velocity()
    _, u, _, pid = g.fields()
    fl = pid < 0
    assert nf2 == int(fl.sum())
    np.testing.assert_allclose(ub2, u[:, fl].astype(np.float64).mean(axis=1), rtol=0,
                               atol=tol * np.abs(u[:, fl]).max())
    g.close()


def test_stabilization_gives_a_terminal_velocity():
    """A spherocylinder under a constant force F in a fully periodic box of N
    cells: with the stabilization its velocity settles (the fluid's mean
    momentum is held at zero); without it fluid and particle together gain
    F per step, so once the relative motion has settled the particle's
    velocity still grows by about F / (N rho0) per step."""
    n, F = 40, (0.0, 0.0, 2e-2)
    q = scenarios.quat_from_axis(np.array([1.0, 0.0, 0.0]))
    vz = {}
    for stab in (True, False):
        g = lbm.Context(n, n, n, tau=0.8, z_periodic=True, stabilize=stab)
        g.add_fiber((19.5, 19.5, 19.5), q, 16.0, 3.0, 1.5, shape="spherocylinder", force=F)
        g.step(2000)
        v1 = g.fiber_state()[2][0, 2]
        g.step(2000)
        v2 = g.fiber_state()[2][0, 2]
        vz[stab] = (v1, v2)
        g.close()
    print("V_z after 2000 / 4000 steps: stabilized %s, free %s" % (vz[True], vz[False]), flush=True)
    s1, s2 = vz[True]
    f1, f2 = vz[False]
    drift = 2000 * F[2] / n ** 3
    assert s1 > 0 and abs(s2 / s1 - 1.0) < 0.02
    assert f2 - f1 > 0.5 * drift and abs(s2 - s1) < 0.1 * (f2 - f1)
