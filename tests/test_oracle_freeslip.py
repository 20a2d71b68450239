"""Pins of the oracle's free-slip walls (Sec. 4.1, Eq. FreeSlipBC: specular
reflection of the populations that leave the lattice through a wall).

A free-slip wall half-way outside a face is a mirror plane: the flow in a
box with such walls is the flow of the periodic box of twice the size whose
second half holds the mirror image of the first (populations with the
normal component reversed).  The periodic streaming is pinned on its own
(closed forms of the other pin files), so these tests check the reflection
-- the reversed component, the tangential landing cell, edges and corners
where a link crosses two or three walls, and the rule that a no-slip wall
wins where a link crosses walls of both kinds -- against an independent
construction.  Plus conservation and the exact solutions that a free-slip
wall allows (uniform flow along it, uniform acceleration by a body force
along it)."""
import numpy as np
import pytest

from oracle import pyoracle as O

C, W, _ = O.lattice()


def mirror_perm(axis):
    """Direction index with the `axis` component of c reversed."""
    out = np.zeros(19, np.int64)
    for q in range(19):
        e = C[q].copy()
        e[axis] = -e[axis]
        out[q] = int(np.nonzero((C == e).all(axis=1))[0][0])
    return out


def doubled(f, axes):
    """The state of the periodic box of twice the size along each of `axes`
    (0 = x, 1 = y, 2 = z) whose added halves are mirror images."""
    for a in axes:
        arr_axis = 3 - a                      # populations are [q][z][y][x]
        img = np.flip(f[mirror_perm(a)], axis=arr_axis)
        f = np.concatenate([f, img], axis=arr_axis)
    return f


def random_state(shape, seed, amp=0.05, u=(0.0, 0.0, 0.0)):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    base = np.array([O.feq(1.0, 1.0, u)[q] for q in range(19)])
    return base[:, None, None, None] * (1.0 + amp * rng.standard_normal((19, nz, ny, nx)))


CASES = {
    # name: (free-slip axes, keyword arguments of the walled box, of the doubled box)
    "x": ((0,), dict(x_walls="free-slip", z_periodic=True), dict(z_periodic=True)),
    "y": ((1,), dict(y_walls="free-slip", z_periodic=True), dict(z_periodic=True)),
    "z": ((2,), dict(z_free_slip=True), dict(z_periodic=True)),
    "xy_edges": ((0, 1), dict(x_walls="free-slip", y_walls="free-slip", z_periodic=True),
                 dict(z_periodic=True)),
    "xyz_corners": ((0, 1, 2), dict(x_walls="free-slip", y_walls="free-slip", z_free_slip=True),
                    dict(z_periodic=True)),
    # a link through a free-slip x wall and a no-slip y wall bounces back
    "x_free_y_noslip": ((0,), dict(x_walls="free-slip", y_walls="no-slip", z_periodic=True),
                        dict(y_walls="no-slip", z_periodic=True)),
    # free-slip y walls beside the moving no-slip z walls of the shear cell
    "y_free_z_moving": ((1,), dict(y_walls="free-slip", wall_u=0.02), dict(wall_u=0.02)),
}


@pytest.mark.parametrize("srt", [False, True], ids=["trt", "srt"])
@pytest.mark.parametrize("case", list(CASES))
def test_free_slip_box_is_half_of_the_mirrored_periodic_box(case, srt):
    axes, kw, kw2 = CASES[case]
    nx, ny, nz = 7, 6, 5
    tau = 0.7
    f0 = random_state((nx, ny, nz), seed=len(case) + 10 * srt)
    a = O.Sim(nx, ny, nz, tau=tau, srt=srt, **kw)
    n2 = [2 * n if k in axes else n for k, n in enumerate((nx, ny, nz))]
    b = O.Sim(*n2, tau=tau, srt=srt, **kw2)
    a.set_populations(f0)
    b.set_populations(doubled(f0, axes))
    a.step(60)
    b.step(60)
    fa, fb = a.populations(), b.populations()
    np.testing.assert_allclose(fa, fb[:, :nz, :ny, :nx], rtol=0, atol=1e-13)
    # and the doubled box stayed mirror symmetric
    np.testing.assert_allclose(doubled(fa, axes), fb, rtol=0, atol=1e-13)


def test_free_slip_box_conserves_mass_and_keeps_tangential_flow():
    """All six walls free-slip: mass is conserved to rounding, the normal
    momentum of a random state decays to zero; a uniform flow along x between
    free-slip y and z walls (periodic x) is an exact steady state."""
    n = 8
    sim = O.Sim(n, n, n, tau=0.8, x_walls="free-slip", y_walls="free-slip", z_free_slip=True)
    f = random_state((n, n, n), seed=3)
    sim.set_populations(f)
    m0 = f.sum()
    sim.step(2000)
    f1 = sim.populations()
    assert abs(f1.sum() - m0) < 1e-12 * m0
    assert np.abs(np.einsum("qa,qzyx->a", C.astype(np.float64), f1)).max() < 1e-9

    U = 0.03
    sim = O.Sim(n, n, n, tau=0.6, y_walls="free-slip", z_free_slip=True)
    f = random_state((n, n, n), seed=0, amp=0.0, u=(U, 0.0, 0.0))
    sim.set_populations(f)
    sim.step(200)
    _, u, _, _ = sim.fields()
    assert np.abs(u[0] - U).max() < 1e-14
    assert np.abs(u[1:]).max() < 1e-15


def test_body_force_along_free_slip_walls_accelerates_uniformly():
    """A body force g along z between free-slip x walls (no-slip walls would
    give the Poiseuille parabola): no wall drag, so every cell's velocity
    grows by g per step, uniformly across the channel."""
    n, g, steps = 12, 1e-5, 300
    sim = O.Sim(n, 4, 4, tau=0.8, z_periodic=True, x_walls="free-slip", g=(0, 0, g))
    sim.step(steps)
    _, u, _, _ = sim.fields()
    uz = u[2]
    assert np.abs(uz - uz.mean()).max() < 1e-15
    # the reported velocity is the half-step average (j + g/2)/rho0 with j grown
    # by g per step; rounding: populations near 1/3 (half an ulp 2^-54), about
    # 19 roundings per step into the momentum
    assert abs(uz.mean() - g * (steps + 0.5)) < steps * 19 * 2.0 ** -54
    assert np.abs(u[:2]).max() < 1e-16


def _quat_from_axis(t):
    """A unit quaternion (w, x, y, z) turning e_x into the unit vector t
    (test-local; only the axis matters for an axisymmetric fiber)."""
    t = np.asarray(t, dtype=np.float64) / np.linalg.norm(t)
    q = np.array([1.0 + t[0], 0.0, -t[2], t[1]])
    return q / np.linalg.norm(q)


@pytest.mark.parametrize("coupling", ["implicit", "explicit"])
def test_particle_beside_a_free_slip_wall_equals_its_mirrored_pair(coupling):
    """A forced spherocylinder two cells from a free-slip x wall moves
    exactly like one of a mirror-symmetric pair in the periodic box of twice
    the width: same populations in the first half, mirrored position and
    velocity, angular velocity mirrored as a pseudovector (W_x kept, W_y and
    W_z reversed), mirrored force and torque histories.  Pins the reflection
    together with the particle coupling next to the wall (cell maps,
    bounce-back, momentum exchange and rigid update near it)."""
    nx, ny, nz, steps = 12, 14, 14, 60
    X = np.array([4.25, 7.3, 6.7])
    t = np.array([0.3, 0.8, 0.5])
    F = np.array([2e-2, 1e-2, -1.5e-2])
    L, r = 8.0, 2.0
    mir = np.array([-1.0, 1.0, 1.0])
    Xm = np.array([2 * nx - 1 - X[0], X[1], X[2]])
    kw = dict(tau=0.8, z_periodic=True, coupling=coupling)
    a = O.Sim(nx, ny, nz, x_walls="free-slip", **kw)
    a.add_fiber(X, _quat_from_axis(t), L, r, 1.5, shape="spherocylinder", force=F)
    b = O.Sim(2 * nx, ny, nz, **kw)
    b.add_fiber(X, _quat_from_axis(t), L, r, 1.5, shape="spherocylinder", force=F)
    b.add_fiber(Xm, _quat_from_axis(mir * t), L, r, 1.5, shape="spherocylinder", force=mir * F)
    a.step(steps)
    b.step(steps)
    np.testing.assert_allclose(a.populations(), b.populations()[:, :, :, :nx], rtol=0, atol=1e-13)
    ha, hb = a.history(), b.history()
    np.testing.assert_allclose(ha[:, 0, :], hb[:, 0, :], rtol=0, atol=1e-12)
    pv = np.array([1.0, -1.0, -1.0])               # pseudovector under the mirror x -> -x
    np.testing.assert_allclose(hb[:, 1, 0:3], mir * hb[:, 0, 0:3], rtol=0, atol=1e-12)   # force
    np.testing.assert_allclose(hb[:, 1, 3:6], pv * hb[:, 0, 3:6], rtol=0, atol=1e-12)    # torque
    np.testing.assert_allclose(hb[:, 1, 13:16], mir * hb[:, 0, 13:16], rtol=0, atol=1e-13)  # V
    np.testing.assert_allclose(hb[:, 1, 16:19], pv * hb[:, 0, 16:19], rtol=0, atol=1e-13)  # W
    np.testing.assert_allclose(hb[:, 1, 6], 2 * nx - 1 - hb[:, 0, 6], rtol=0, atol=1e-12)  # x
    assert np.abs(ha[-1, 0, 13:16]).max() > 1e-4      # the particle moves
