"""Host-side data preparation of the learned closure (numpy, CPU): the body
rotation R(q), the fine-to-coarse coordinate map and trajectory scaling of
the diffusively scaled pairs (coarse spacing 2: velocities x 2, angular
velocities x 4), the constant-spin trajectories that prescribe part of the
training data, the normalisation envelope and the error measure, each
against a closed form; and the training pairs against their stated
recipe."""
import numpy as np
import pytest

from paper_1503_06869_amd import closure, scenarios


def _hamilton(a, b):
    a0, av, b0, bv = a[0], np.asarray(a[1:]), b[0], np.asarray(b[1:])
    return np.r_[a0 * b0 - av @ bv, a0 * bv + b0 * av + np.cross(av, bv)]


def _rodrigues(axis, angle):
    k = np.asarray(axis, dtype=np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


def _unit_quats(n, seed):
    q = np.random.default_rng(seed).standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def test_rotation_is_proper_orthogonal_and_a_homomorphism():
    qs = _unit_quats(20, 0)
    for a, b in zip(qs[:10], qs[10:]):
        Ra = closure.rotation(a)
        np.testing.assert_allclose(Ra.T @ Ra, np.eye(3), atol=1e-15)
        assert abs(np.linalg.det(Ra) - 1.0) < 1e-14
        np.testing.assert_allclose(closure.rotation(_hamilton(a, b)), Ra @ closure.rotation(b), atol=1e-14)
        np.testing.assert_allclose(closure.rotation(-a), Ra, atol=0)


@pytest.mark.parametrize("theta", [0.3, 1.7, -2.9])
def test_rotation_about_a_coordinate_axis(theta):
    c, s = np.cos(theta), np.sin(theta)
    q = np.array([np.cos(theta / 2), 0.0, 0.0, np.sin(theta / 2)])
    np.testing.assert_allclose(closure.rotation(q), [[c, -s, 0], [s, c, 0], [0, 0, 1]], atol=1e-15)
    q = np.array([np.cos(theta / 2), np.sin(theta / 2), 0.0, 0.0])
    np.testing.assert_allclose(closure.rotation(q), [[1, 0, 0], [0, c, -s], [0, s, c]], atol=1e-15)


def test_the_first_body_axis_is_the_fiber_axis():
    g = scenarios.rng(3)
    for _ in range(10):
        t = scenarios.axis_uniform_on_sphere(g)
        np.testing.assert_allclose(closure.rotation(scenarios.quat_from_axis(t))[:, 0], t, atol=1e-14)


def test_two_fine_cells_straddle_their_coarse_cell_centre():
    """With coarse spacing 2, fine cells 2c and 2c + 1 lie in coarse cell c,
    a quarter of a coarse cell either side of its centre."""
    for c in range(6):
        lo, hi = closure.coarse_of(2 * c), closure.coarse_of(2 * c + 1)
        assert lo == c - 0.25 and hi == c + 0.25
    x = np.array([[10.0, 3.5, 0.5]])
    np.testing.assert_array_equal(closure.coarse_of(x), [[4.75, 1.5, 0.0]])


@pytest.mark.parametrize("W", [(0.0, 0.0, 0.01), (0.003, -0.004, 0.002), (0.0, 0.0, 0.0)])
def test_constant_spin_trajectory_is_a_rotation_by_k_omega(W):
    W = np.array(W)
    q0 = _unit_quats(1, 5)[0]
    X = np.array([3.0, 4.0, 5.0])
    rows = closure.rotation_traj(X, q0, W, 400)
    assert rows.shape == (400, 13)
    np.testing.assert_array_equal(rows[:, 0:3], np.broadcast_to(X, (400, 3)))
    np.testing.assert_array_equal(rows[:, 7:10], 0.0)
    np.testing.assert_array_equal(rows[:, 10:13], np.broadcast_to(W, (400, 3)))
    w = np.linalg.norm(W)
    for k in (1, 37, 400):
        R = closure.rotation(rows[k - 1, 3:7])
        Rk = _rodrigues(W, k * w) if w > 0 else np.eye(3)
        np.testing.assert_allclose(R, Rk @ closure.rotation(q0), atol=1e-13)


def test_fine_history_maps_to_coarse_prescribed_rows():
    """The state after fine step 4j + 3 is the state after coarse step j:
    positions through the coordinate map, orientation unchanged, velocity
    x 2 and angular velocity x 4."""
    T = 5
    rng = np.random.default_rng(7)
    h = rng.standard_normal((4 * T, 19))
    rows = closure.fine_to_coarse_traj(h)
    assert rows.shape == (T, 13)
    for j in range(T):
        s = h[4 * j + 3]
        np.testing.assert_array_equal(rows[j, 0:3], (s[6:9] - 0.5) / 2.0)
        np.testing.assert_array_equal(rows[j, 3:7], s[9:13])
        np.testing.assert_array_equal(rows[j, 7:10], 2.0 * s[13:16])
        np.testing.assert_array_equal(rows[j, 10:13], 4.0 * s[16:19])


def test_normalisation_and_envelope():
    rng = np.random.default_rng(11)
    X = rng.uniform(-1.0, 2.0, (500, 4))
    X[:, 3] = 0.0                                   # a feature that is always zero
    Y = rng.standard_normal((500, 6)) * np.array([1, 2, 3, 4, 5, 6])
    n = closure.make_norm(X, Y, envelope_margin=0.1, envelope_floor=0.05)
    np.testing.assert_allclose(n.in_mean, X.mean(0), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(n.in_inv_std[:3], 1.0 / X.std(0)[:3], rtol=1e-6)
    assert n.in_inv_std[3] == np.float32(1e6)      # the zero feature keeps a finite scale
    np.testing.assert_allclose(n.out_scale, Y.std(0), rtol=1e-6)
    assert closure.in_envelope(n, X).all()
    span = X.max(0) - X.min(0)
    assert np.allclose(n.env_max - X.max(0), 0.1 * span + 0.05, atol=1e-6)
    assert np.allclose(X.min(0) - n.env_min, 0.1 * span + 0.05, atol=1e-6)
    out = X[:3].copy()
    out[0, 0] = X[:, 0].max() + 0.1 * span[0] + 0.06   # just past the widened range
    out[1, 3] = 0.06                                    # past the zero feature's band
    assert list(closure.in_envelope(n, out)) == [False, False, True]


def test_error_measure_is_the_mean_norm_of_the_miss():
    Y = np.zeros((4, 6))
    Y[:, 0] = [3.0, 0.0, 0.0, 1.0]
    Y[:, 1] = [4.0, 0.0, 2.0, 0.0]
    Y[:, 5] = [1.0, 1.0, 1.0, 1.0]
    eF, eM = closure.relative_errors(Y, 0 * Y)
    assert eF == (5.0 + 0.0 + 2.0 + 1.0) / 4 and eM == 1.0
    assert closure.relative_errors(Y, Y) == (0.0, 0.0)


def test_training_pairs_follow_the_stated_recipe():
    """Fine 64^3 / coarse 32^3 twins, diameters 4 / 2, aspect ratio in
    [2, 12] with the coarse length fitting 8 cells inside the cell, coarse
    shear rate in [5e-4, 1.5e-3], the coarse fiber at the fine centre under
    the coordinate map with velocities x 2 and angular velocities x 4, and
    about half of the fine fibers turning at a prescribed rate."""
    pairs = closure.training_pairs(seed=0, n=40, steps=50)
    assert len(pairs) == 40
    prescribed = 0
    for pr in pairs:
        f, c = pr.fine.fibers[0], pr.coarse.fibers[0]
        assert (pr.fine.nx, pr.coarse.nx) == (64, 32)
        assert (2 * f.radius, 2 * c.radius) == (4.0, 2.0)
        assert 2.0 <= c.length / 2.0 <= 12.0 and c.length <= 32 - 8.0
        assert f.length == 2 * c.length
        assert 5e-4 <= pr.coarse.shear_rate <= 1.5e-3 + 1e-15
        np.testing.assert_allclose(pr.fine.shear_rate, pr.coarse.shear_rate / 4.0, rtol=1e-14)
        np.testing.assert_array_equal(c.X, closure.coarse_of(f.X))
        np.testing.assert_allclose(c.V, 2.0 * f.V, rtol=0, atol=0)
        np.testing.assert_allclose(c.W, 4.0 * f.W, rtol=0, atol=0)
        if pr.fine_traj is not None:
            prescribed += 1
            assert pr.fine_traj.shape == (4 * 50, 13)
            gf = 2.0 * pr.fine.wall_u / 64
            assert np.all(np.abs(f.W) <= gf) and not f.V.any()
            np.testing.assert_array_equal(pr.fine_traj[:, 10:13], np.broadcast_to(f.W, (200, 3)))
    assert 10 <= prescribed <= 30
