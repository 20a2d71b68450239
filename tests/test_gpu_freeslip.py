"""Free-slip walls on the GPU (Sec. 4.1, Eq. FreeSlipBC: specular
reflection), through the C ABI, against the oracle: random states with
free-slip walls on every combination of faces (edges and corners where a
link crosses two or three walls, walls of both kinds meeting), at both AA
parities, and a spherocylinder sedimenting in a box closed by free-slip
walls on all six faces (the paper's sedimentation setup, small)."""
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


CASES = {
    "x": dict(x_walls="free-slip", z_periodic=True),
    "y": dict(y_walls="free-slip", z_periodic=True),
    "z": dict(z_free_slip=True),
    "xy_edges": dict(x_walls="free-slip", y_walls="free-slip", z_periodic=True),
    "xyz_corners": dict(x_walls="free-slip", y_walls="free-slip", z_free_slip=True),
    "x_free_y_noslip": dict(x_walls="free-slip", y_walls="no-slip", z_periodic=True),
    "x_noslip_z_free": dict(x_walls="no-slip", z_free_slip=True),
    "y_free_z_moving": dict(y_walls="free-slip", wall_u=0.02),
}


@pytest.mark.parametrize("collision", ["trt", "srt"])
@pytest.mark.parametrize("storage,tol", [("f32", 2e-7), ("f64", 1e-14)])
@pytest.mark.parametrize("case", list(CASES))
def test_free_slip_random_state_matches_oracle(case, storage, tol, collision):
    """A random state in a 20 x 18 x 16 box after 1, 2 and 41 steps (the
    populations read back in the swapped layout after odd counts), with the
    two-relaxation-time and the single-relaxation-time collision."""
    nx, ny, nz = 20, 18, 16
    kw = CASES[case]
    _, w, _ = O.lattice()
    rng = np.random.default_rng(len(case))
    f0 = w[:, None, None, None] * (1.0 + 0.05 * rng.standard_normal((19, nz, ny, nx)))
    g = lbm.Context(nx, ny, nz, tau=0.7, storage=storage, collision=collision, **kw)
    o = O.Sim(nx, ny, nz, tau=0.7, srt=(collision == "srt"), **kw)
    g.set_populations(to_lib_order(f0))
    o.set_populations(f0)
    done = 0
    for n in (1, 2, 41):
        g.step(n - done)
        o.step(n - done)
        done = n
        d = np.abs(to_oracle_order(g.populations()) - o.populations()).max()
        print("%s %s %s step %d: max |df| %.3g" % (case, storage, collision, n, d), flush=True)
        assert d < tol
    g.close()


def _box(lib_or_oracle, n, **kw):
    walls = dict(x_walls="free-slip", y_walls="free-slip", z_free_slip=True)
    if lib_or_oracle == "lib":
        return lbm.Context(*n, tau=0.8, **walls, **kw)
    return O.Sim(*n, tau=0.8, **walls)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_sedimenting_spherocylinder_in_free_slip_box_matches_oracle(storage):
    """A spherocylinder (L 16, r 3, tilted) under a constant force along z in
    a 34 x 32 x 48 box with free-slip walls on all six faces: 300 steps,
    cell maps bit-exact, force/torque histories and velocity field."""
    n, steps = (34, 32, 48), 300
    q = scenarios.quat_from_axis(np.array([0.3, 0.1, 1.0]))
    g = _box("lib", n, storage=storage)
    o = _box("oracle", n)
    for s in (g, o):
        s.add_fiber((16.5, 15.5, 14.0), q, 16.0, 3.0, 1.2, shape="spherocylinder", force=(0.0, 0.0, 0.05))
    g.step(steps)
    o.step(steps)
    hg, ho = g.history(0, steps), o.history()
    eF, eM = ft_error(hg, ho, [16.0])
    _, ug, flg, pidg = g.fields()
    _, uo, flo, pido = o.fields()
    e = rel_l2(ug.astype(np.float64), uo, flo == 0)
    print("free-slip box %s: velocity rel L2 %.3g, F %.3g, M %.3g, V_z %.4g" % (
        storage, e, eF, eM, ho[-1, 0, 15]), flush=True)
    assert np.array_equal(pidg, pido)
    tol = {"f32": (1e-5, 1e-4), "f16": (2e-3, 2e-2)}[storage]
    assert e < tol[0] and eF < tol[1] and eM < tol[1]
    g.close()


def test_fiber_near_a_free_slip_z_wall_is_rejected_and_reported():
    """Fibers keep more than one cell from free-slip z walls: rejected at
    insertion, and reported at the next sync when driven into one."""
    q = scenarios.quat_from_axis(np.array([1.0, 0.0, 0.0]))
    g = _box("lib", (32, 32, 40))
    with pytest.raises(lbm.LBMError):
        g.add_fiber((16.0, 16.0, 1.5), q, 12.0, 2.0, 1.0)
    g.add_fiber((16.0, 16.0, 6.0), q, 12.0, 2.0, 1.0, force=(0.0, 0.0, -0.1))
    done = 0
    with pytest.raises(lbm.LBMError) as ei:
        for _ in range(400):
            g.step(10)
            done += 10
            g.sync()
    assert ei.value.code == lbm.LBM_E_STATE and "wall" in str(ei.value)
    print("reported after %d steps" % done, flush=True)
    g.close()
