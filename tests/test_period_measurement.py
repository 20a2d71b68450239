"""The tumbling-period measurement used by the tests and the benchmark
(post-processing of the fiber's orientation history), on the CPU: the axis
of a quaternion, sign changes located by linear interpolation, and the
period of an exact Jeffery orbit.

On a Jeffery orbit of a spheroid of aspect ratio r in simple shear of rate
gamma, the angle phi from the gradient direction in the flow-gradient plane
obeys tan(phi) = r tan(omega t) with omega = gamma / (r + 1/r): the flow
component of the axis, sin(phi), vanishes exactly when omega t is a
multiple of pi, twice per period T = 2 pi / omega."""
import numpy as np
import pytest

from paper_1503_06869_amd import closure, jeffery, scenarios


def test_axis_of_a_quaternion_is_its_first_body_axis():
    q = np.random.default_rng(0).standard_normal((16, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    ax = jeffery.axis_from_quat(q)
    for k in range(16):
        np.testing.assert_allclose(ax[k], closure.rotation(q[k])[:, 0], atol=1e-15)
    g = scenarios.rng(1)
    t = scenarios.axis_uniform_on_sphere(g)
    np.testing.assert_allclose(jeffery.axis_from_quat(scenarios.quat_from_axis(t)), t, atol=1e-14)


def test_linear_sign_changes_are_located_exactly():
    # tx = (c - t) on samples t = step0, step0 + 1, ...: one crossing at c
    for c in (3.25, 10.5, 17.875):
        t = np.arange(1, 30, dtype=np.float64)
        got = jeffery.crossings(c - t, step0=1)
        assert got.shape == (1,) and abs(got[0] - c) < 1e-13
    # a sampled zero is not a sign change between neighbours of opposite sign
    assert jeffery.crossings([1.0, 0.0, 1.0]).size == 0


@pytest.mark.parametrize("r,gamma", [(4.0, 3.125e-4), (8.0, 6.25e-4), (2.0, 1.0e-3)])
def test_period_of_an_exact_jeffery_orbit(r, gamma):
    T = jeffery.jeffery_period(r, gamma)
    omega = 2 * np.pi / T
    assert abs(omega - gamma / (r + 1 / r)) < 1e-18
    t = np.arange(1, int(2.6 * T), dtype=np.float64) + 0.37 * T / 4   # start off a crossing
    phi = np.arctan2(r * np.sin(omega * t), np.cos(omega * t))
    tx = np.sin(phi)
    Tm, c = jeffery.period(tx, step0=1)
    assert len(c) >= 4
    # crossing k = 1, 2, ... sits at omega t = k pi; step numbers lag t by the shift
    shift = 0.37 * T / 4
    np.testing.assert_allclose(c[:4] + shift, (np.arange(4) + 1) * np.pi / omega, rtol=0, atol=0.05)
    assert abs(Tm / T - 1) < 1e-5


def test_too_few_crossings_give_no_period():
    T, c = jeffery.period(np.sin(np.linspace(0.1, 2 * np.pi - 0.1, 400)))
    assert np.isnan(T) and len(c) == 1
