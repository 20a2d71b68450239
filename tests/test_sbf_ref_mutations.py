"""Each pin of the slender-body reference can fail: a plausible mistake
planted in one of its functions (for the duration of one test, through
monkeypatch, on the CPU) makes the named pins fail."""
import numpy as np
import pytest

from oracle import sbf_ref as S

import test_sbf_ref as T

_green, _kbar, _legendre, _theta = S.green, S.kbar_eigenvalues, S.legendre, S.theta_pair


def green_doublet_sign(R, r):
    """The doublet with I + 3 Rh Rh^T."""
    n = np.linalg.norm(R, axis=-1)
    Rh = R / n[..., None]
    RR = Rh[..., :, None] * Rh[..., None, :]
    I = np.eye(3)
    return (I + RR) / n[..., None, None] + 0.5 * r * r * (I + 3.0 * RR) / (n ** 3)[..., None, None]


def green_stokeslet_sign(R, r):
    """The Stokeslet with I - Rh Rh^T."""
    n = np.linalg.norm(R, axis=-1)
    Rh = R / n[..., None]
    RR = Rh[..., :, None] * Rh[..., None, :]
    I = np.eye(3)
    return (I - RR) / n[..., None, None] + 0.5 * r * r * (I - 3.0 * RR) / (n ** 3)[..., None, None]


def kbar_off_by_one(N):
    """L_n summed to n - 1."""
    return np.array([0.0] + [-2.0 * sum(1.0 / i for i in range(1, n)) for n in range(1, N + 1)])


def quadrature_two_point(nq):
    g, w = np.polynomial.legendre.leggauss(2)
    h = 2.0 / nq
    return (np.concatenate([-1.0 + h * (i + 0.5) + 0.5 * h * g for i in range(nq)]),
            np.concatenate([0.5 * h * w for _ in range(nq)]))


def legendre_wrong_recurrence(N, x):
    """(2n + 1) x P_n - n P_{n-1} divided by n instead of n + 1."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((N + 1,) + x.shape)
    P[0] = 1.0
    if N >= 1:
        P[1] = x
    for n in range(1, N):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / n
    return P


def theta_transposed(xm, pm, xn, pn, l, r, N, nq):
    """Theta^{k,n} in place of Theta^{n,k}."""
    return np.swapaxes(_theta(xm, pm, xn, pn, l, r, N, nq), 0, 1)


MUTATIONS = {
    "doublet sign": ("green", green_doublet_sign, [T.test_green_function_solves_the_stokes_equations]),
    "Stokeslet sign": ("green", green_stokeslet_sign, [T.test_green_function_solves_the_stokes_equations]),
    "Kbar eigenvalues off by one": ("kbar_eigenvalues", kbar_off_by_one,
                                    [lambda: T.test_kbar_eigenvalues_by_direct_quadrature(3)]),
    "two-point Gauss rule": ("quadrature", quadrature_two_point,
                             [T.test_quadrature_is_exact_for_quintics_on_each_sub_interval]),
    "Legendre recurrence": ("legendre", legendre_wrong_recurrence,
                            [T.test_legendre_recurrence_matches_the_power_series]),
    "moments transposed": ("theta_pair", theta_transposed, [T.test_solution_satisfies_the_integral_equation]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_sbf_pins_fail_on_planted_mistakes(name, monkeypatch):
    attr, wrong, pins = MUTATIONS[name]
    monkeypatch.setattr(S, attr, wrong)
    for pin in pins:
        with pytest.raises(AssertionError):
            pin()
