"""Resting no-slip walls on the x and y faces on the GPU, through the C ABI
(Eq. BBBC, walls half-way outside the faces; with the z walls the box is
closed on all six faces, as in the paper's rotational validation)."""
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


@pytest.mark.parametrize("storage,tol", [("f32", 2e-7), ("f64", 1e-14)])
def test_closed_box_random_state_matches_oracle(storage, tol):
    """A random state in a 20 x 18 x 16 box with walls on all six faces
    (the z walls moving), after 1, 2 and 41 steps (both AA parities)."""
    nx, ny, nz = 20, 18, 16
    c, w, _ = O.lattice()
    rng = np.random.default_rng(9)
    f0 = w[:, None, None, None] * (1.0 + 0.05 * rng.standard_normal((19, nz, ny, nx)))
    g = lbm.Context(nx, ny, nz, tau=0.7, wall_u=0.01, storage=storage, x_walls=True, y_walls=True)
    o = O.Sim(nx, ny, nz, tau=0.7, wall_u=0.01, x_walls=True, y_walls=True)
    g.set_populations(to_lib_order(f0))
    o.set_populations(f0)
    done = 0
    for n in (1, 2, 41):
        g.step(n - done)
        o.step(n - done)
        done = n
        d = np.abs(to_oracle_order(g.populations()) - o.populations()).max()
        print("%s step %d: max |df| %.3g" % (storage, n, d), flush=True)
        assert d < tol
    g.close()


@pytest.mark.parametrize("axis", ["x", "y"])
def test_poiseuille_across_side_walls(axis):
    """Body-force channel flow across x (y) walls: the exact parabola of the
    TRT magic value, to FP32 rounding."""
    n, gz, tau = 24, 1e-5, 0.8
    nu = (tau - 0.5) / 3
    if axis == "x":
        g = lbm.Context(n, 4, 4, tau=tau, z_periodic=True, x_walls=True, body_force=(0, 0, gz))
    else:
        g = lbm.Context(4, n, 4, tau=tau, z_periodic=True, y_walls=True, body_force=(gz, 0, 0))
    g.step(20000)
    _, u, _, _ = g.fields()
    prof = (u[2, 0, 0, :] if axis == "x" else u[0, 0, :, 0]).astype(np.float64)
    s = np.arange(n)
    exact = gz * (s + 0.5) * (n - s - 0.5) / (2 * nu)
    err = np.abs(prof - exact).max() / exact.max()
    print("%s walls: max rel error %.3g" % (axis, err), flush=True)
    assert err < 2e-5
    g.close()


def test_rotating_spherocylinder_in_closed_box_matches_oracle():
    """A spherocylinder under a constant torque in a 36 x 34 x 32 box closed
    on all six faces: 300 steps, maps, histories and velocity field against
    the oracle."""
    nx, ny, nz, n = 36, 34, 32, 300
    q = scenarios.quat_from_axis(np.array([0.0, 1.0, 0.0]))
    g = lbm.Context(nx, ny, nz, tau=0.8, x_walls=True, y_walls=True)
    o = O.Sim(nx, ny, nz, tau=0.8, x_walls=True, y_walls=True)
    for s in (g, o):
        s.add_fiber((17.5, 16.5, 15.5), q, 16.0, 3.0, 1.2, shape="spherocylinder", torque=(2.0, 0.0, 0.0))
    g.step(n)
    o.step(n)
    hg, ho = g.history(0, n), o.history()
    eF, eM = ft_error(hg, ho, [16.0])
    _, ug, flg, pidg = g.fields()
    _, uo, flo, pido = o.fields()
    e = rel_l2(ug.astype(np.float64), uo, flo == 0)
    print("closed box: velocity rel L2 %.3g, F %.3g, M %.3g, W_x %.4g" % (e, eF, eM, ho[-1, 0, 16]), flush=True)
    assert np.array_equal(pidg, pido)
    assert e < 1e-5 and eF < 1e-4 and eM < 1e-4
    g.close()


def test_fiber_next_to_a_side_wall_is_rejected():
    q = scenarios.quat_from_axis(np.array([1.0, 0.0, 0.0]))
    g = lbm.Context(40, 40, 40, tau=0.8, x_walls=True)
    with pytest.raises(lbm.LBMError):
        g.add_fiber((8.5, 20.0, 20.0), q, 16.0, 2.0, 1.0)    # reaches x = 0.5
    g.add_fiber((12.0, 20.0, 20.0), q, 16.0, 2.0, 1.0)
    g.close()


def test_fiber_driven_into_a_side_wall_is_reported():
    """A fiber pushed towards an x wall by a constant force: the step kernel
    flags it once it comes within one cell, and the next sync reports
    LBM_E_STATE (every kernel still completes normally; the error stays
    set for the context)."""
    q = scenarios.quat_from_axis(np.array([0.0, 0.0, 1.0]))
    g = lbm.Context(32, 32, 40, tau=0.8, x_walls=True, y_walls=True)
    g.add_fiber((8.0, 16.0, 20.0), q, 12.0, 2.0, 1.0, force=(-0.1, 0.0, 0.0))
    done = 0
    with pytest.raises(lbm.LBMError) as ei:
        for _ in range(400):
            g.step(10)
            done += 10
            g.sync()
    assert ei.value.code == lbm.LBM_E_STATE and "wall" in str(ei.value)
    print("reported after %d steps" % done, flush=True)
    assert done >= 300   # it had to travel about 5 cells first (about 0.005 per step)
    g.close()


def test_closure_is_refused_with_side_walls():
    g = lbm.Context(24, 24, 24, tau=0.8, x_walls=True)
    m = lbm.Mlp()
    with pytest.raises(lbm.LBMError):
        g.set_closure(m)
    g.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_non_finite_population_is_reported_at_sync(storage):
    """A NaN written into one cell's populations spreads through the
    collisions; the next sync reports LBM_E_UNSTABLE (no fibers: the
    force/torque check cannot see it)."""
    g = lbm.Context(20, 18, 16, tau=0.8, storage=storage)
    g.step(2)
    g.sync()
    f = g.populations()
    f[3, 8, 9, 10] = np.nan
    g.set_populations(f)
    g.step(3)
    with pytest.raises(lbm.LBMError) as ei:
        g.sync()
    assert ei.value.code == lbm.LBM_E_UNSTABLE and "population" in str(ei.value)
    g.close()
