"""Pins of the FP64 reference of the learned closure (oracle/closure_ref.py):
closed-form GELU values, central finite differences of the gradient, exact
BF16 rounding cases, the first Adam step's closed form, and features of
linear velocity fields (reproduced exactly by trilinear interpolation)."""
import math

import numpy as np

from oracle import closure_ref as R


def test_gelu_closed_form_values():
    phi1 = 0.5 * (1 + math.erf(1 / math.sqrt(2)))      # standard normal CDF at 1
    assert R.gelu(np.array([0.0]))[0] == 0.0
    assert abs(R.gelu(np.array([1.0]))[0] - phi1) < 1e-15
    assert abs(R.gelu(np.array([-1.0]))[0] + (1 - phi1)) < 1e-15
    assert abs(R.gelu(np.array([12.0]))[0] - 12.0) < 1e-12
    assert abs(R.gelu_d(np.array([0.0]))[0] - 0.5) < 1e-15
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (R.gelu(z + h) - R.gelu(z - h)) / (2 * h)
    assert np.abs(fd - R.gelu_d(z)).max() < 1e-9


def test_gradient_matches_central_differences():
    g = np.random.default_rng(7)
    w = g.normal(0, 0.2, R.NPARAM)
    x = g.normal(0, 1, (5, R.NI))
    t = g.normal(0, 1, (5, R.NO))
    _, grad = R.loss_grad(w, x, t)
    idx = np.concatenate([g.choice(R.NPARAM, 300, replace=False), np.arange(R.NPARAM - 6, R.NPARAM)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (R.loss_grad(wp, x, t)[0] - R.loss_grad(wm, x, t)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), (i, fd, grad[i])
    # forward and loss agree
    y = R.forward(w, x)
    assert abs(np.mean((y - t) ** 2) - R.loss_grad(w, x, t)[0]) < 1e-14


def test_bf16_round_to_nearest_even():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 0.0], dtype=np.float32)
    r = R.bf16_round(v)
    assert list(r) == [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 0.0]


def test_first_adam_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 2e-3, -7.0], dtype=np.float32)
    w0 = np.zeros(4, np.float32)
    w, m, v = R.adam(w0, np.zeros(4), np.zeros(4), g, 1, lr=1e-2)
    assert np.allclose(w, -1e-2 * np.sign(g), rtol=1e-5)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_of_linear_fields_are_exact():
    nx, ny, nz = 24, 20, 22
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.stack([x, y, z]).astype(np.float64)            # u(p) = p
    X = np.array([11.3, 9.6, 10.4])
    q = np.array([0.9, 0.1, -0.3, 0.2])
    q /= np.linalg.norm(q)
    L, gamma = 6.0, 0.01
    f = R.features(u, X, q, np.zeros(3), np.zeros(3), L, gamma)
    Rm = R.rotation(q)
    # body axes: first column is the fiber axis R(q) e_x
    t = np.array([1 - 2 * (q[2] ** 2 + q[3] ** 2), 2 * (q[1] * q[2] + q[0] * q[3]), 2 * (q[1] * q[3] - q[0] * q[2])])
    assert np.allclose(Rm[:, 0], t) and np.allclose(Rm.T @ Rm, np.eye(3))
    for pt, side in enumerate((0.0, 3.0, -3.0)):
        for m in range(27):
            ob = 2.0 * np.array([m % 3 - 1, (m // 3) % 3 - 1, m // 9 - 1])
            p = X + side * t + Rm @ ob
            k = pt * 27 + m
            assert np.allclose(f[3 * k:3 * k + 3], Rm.T @ p / (gamma * L), atol=1e-12)
    assert np.allclose(f[243:], q)
    # a rigid motion of the field is removed exactly; q and -q are the same pose
    V, W = np.array([0.01, -0.02, 0.005]), np.array([1e-3, 2e-3, -1e-3])
    ur = V[:, None, None, None] + np.cross(W, (np.stack([x, y, z]) - X[:, None, None, None]), axis=0)
    f2 = R.features(ur, X, -q, V, W, L, gamma)
    assert np.abs(f2[:243]).max() < 1e-12 and np.allclose(f2[243:], q)
    # a uniform flow a gives R^T (a - V) at every point when W = 0
    a = np.array([0.02, 0.01, -0.03])
    ua = np.broadcast_to(a[:, None, None, None], u.shape).copy()
    f3 = R.features(ua, X, q, V, np.zeros(3), L, gamma)
    assert np.allclose(f3[:243].reshape(81, 3), (Rm.T @ (a - V)) / (gamma * L), atol=1e-14)
