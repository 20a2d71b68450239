"""The seeded input generators produce the workloads the design notes state:
counts, size ranges, non-overlapping placement, clearance from the walls,
the batched cases' cell total, the slender-body cloud's spacing, and the
same inputs for the same seed."""
import numpy as np

from oracle import pyoracle as O
from paper_1503_06869_amd import scenarios as S


def _axis(q):
    w, x, y, z = q
    return np.array([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)])


def _segment_gap_brute(Xa, ta, ha, Xb, tb, hb, n=401):
    s = np.linspace(-ha, ha, n)[:, None] * ta + Xa
    u = np.linspace(-hb, hb, n)[:, None] * tb + Xb
    return np.sqrt(((s[:, None, :] - u[None, :, :]) ** 2).sum(-1)).min()


def _min_image(d, box):
    return d - np.round(d / box) * box


def test_benchmark_shear_cell():
    sc = S.many_fibers(seed=0)
    assert (sc.nx, sc.ny, sc.nz, len(sc.fibers)) == (256, 256, 256, 64)
    assert sc.tau == 0.8 and sc.wall_u == 0.01 and sc.magic == 3.0 / 16.0
    L = np.array([f.length for f in sc.fibers])
    d = np.array([2 * f.radius for f in sc.fibers])
    assert L.min() >= 24 and L.max() <= 40 and d.min() >= 4 and d.max() <= 6
    box = np.array([256.0, 256.0, 1e30])        # periodic in x and y
    for f in sc.fibers:
        t = _axis(f.q)
        assert abs(np.linalg.norm(t) - 1) < 1e-12
        hz = 0.5 * f.length * abs(t[2]) + f.radius
        assert hz + 2 <= f.X[2] <= 255 - hz - 2 + 1e-9          # clear of the walls
    # pairwise: axis segments (cylinder half-length L/2) at least 2 cells
    # apart beyond the radii, by brute force on close pairs
    X = np.array([f.X for f in sc.fibers])
    for i in range(64):
        for j in range(i + 1, 64):
            dij = _min_image(X[j] - X[i], box)
            fi, fj = sc.fibers[i], sc.fibers[j]
            if np.linalg.norm(dij) > 0.5 * (fi.length + fj.length) + fi.radius + fj.radius + 3:
                continue
            gap = _segment_gap_brute(np.zeros(3), _axis(fi.q), 0.5 * fi.length,
                                     dij, _axis(fj.q), 0.5 * fj.length) - fi.radius - fj.radius
            assert gap >= 2.0 - 0.05, (i, j, gap)
    # and no cell is claimed twice on the lattice
    pid, ov = O.map_fibers((256, 256, 256), X, np.concatenate([f.q for f in sc.fibers]),
                           L, d / 2, z_periodic=False)
    assert ov == 0 and len(np.unique(pid[pid >= 0])) == 64


def test_batched_cases():
    cases = S.batched_cases(seed=0)
    assert len(cases) == 512
    cells = np.array([c.ncell for c in cases])
    assert cells.sum() == 42861936
    assert 15000 <= cells.min() and cells.max() <= 235000
    for c in cases:
        assert all(24 <= n <= 64 for n in (c.nx, c.ny, c.nz))
        f = c.fibers[0]
        assert f.radius == 2.0 and 2 * 2.0 * 2 <= f.length <= min(c.nx, c.ny, c.nz) - 8
        np.testing.assert_array_equal(f.X, [(c.nx - 1) / 2, (c.ny - 1) / 2, (c.nz - 1) / 2])
        assert 0.6 <= c.tau <= 1.0 and 1e-4 <= c.shear_rate <= 5e-4 + 1e-12


def test_learned_coarse_cell():
    sc = S.learned_coarse(seed=0)
    assert (sc.nx, len(sc.fibers)) == (128, 200)
    ar = np.array([f.length / (2 * f.radius) for f in sc.fibers])
    assert np.all([f.radius == 1.0 for f in sc.fibers]) and ar.min() >= 4 and ar.max() <= 12


def test_slender_body_cloud():
    sc = S.sbf_cloud(seed=0)
    m, L = 1024, 48.0
    assert sc.X.shape == (m, 3) and sc.length == L and abs(sc.eps - 1 / 12) < 1e-15
    side = 2.0 * L * m ** (1 / 3)
    assert sc.X.min() >= 0 and sc.X.max() <= side
    D = np.sqrt(((sc.X[:, None] - sc.X[None]) ** 2).sum(-1)) + np.eye(m) * 1e9
    assert D.min() >= 0.25 * L
    np.testing.assert_allclose(np.linalg.norm(sc.p, axis=1), 1.0, atol=1e-14)
    assert abs(sc.p[:, 2].mean()) < 0.1                       # orientations spread over the sphere
    np.testing.assert_array_equal(sc.F, np.tile([0.0, 0.0, 1.0], (m, 1)))
    assert not sc.M.any()


def test_single_fiber_cell():
    sc = S.single_fiber(seed=0)
    f = sc.fibers[0]
    assert (sc.nx, sc.ny, sc.nz, sc.tau, sc.wall_u) == (32, 32, 32, 0.8, 0.005)
    assert (f.length, 2 * f.radius, f.density_ratio) == (16.0, 4.0, 1.0)


def test_same_seed_same_inputs_other_seed_other_inputs():
    a, b, c = S.many_fibers(seed=3, n=96, n_fibers=8), S.many_fibers(seed=3, n=96, n_fibers=8), \
        S.many_fibers(seed=4, n=96, n_fibers=8)
    for fa, fb in zip(a.fibers, b.fibers):
        np.testing.assert_array_equal(fa.X, fb.X)
        np.testing.assert_array_equal(fa.q, fb.q)
    assert not np.allclose(a.fibers[0].X, c.fibers[0].X)
