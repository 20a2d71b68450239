"""Each pin of the closure reference can fail: a plausible mistake planted
in one of its functions (for one test, through monkeypatch, on the CPU)
makes the named pin fail."""
import numpy as np
import pytest
from scipy.special import erf

from oracle import closure_ref as R

import test_closure_ref as T

_rotation = R.rotation


def gelu_d_first_term_only(z):
    """Phi(z) without z phi(z)."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0)))


def adam_without_bias_correction(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    f = np.float32
    w, m, v, g = (np.asarray(a, dtype=f) for a in (w, m, v, g))
    m = f(b1) * m + f(1 - b1) * g
    v = f(b2) * v + f(1 - b2) * g * g
    return w - f(lr) * m / (np.sqrt(v) + f(eps)), m, v


def bf16_truncate(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32)
    return (u & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)


def rotation_transposed(q):
    return _rotation(q).T


MUTATIONS = {
    "GELU derivative without z phi(z)": ("gelu_d", gelu_d_first_term_only,
                                         [T.test_gelu_closed_form_values, T.test_gradient_matches_central_differences]),
    "Adam without bias correction": ("adam", adam_without_bias_correction, [T.test_first_adam_step_is_lr_times_sign]),
    "BF16 by truncation": ("bf16_round", bf16_truncate, [T.test_bf16_round_to_nearest_even]),
    "body frame transposed": ("rotation", rotation_transposed, [T.test_features_of_linear_fields_are_exact]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_closure_pins_fail_on_planted_mistakes(name, monkeypatch):
    attr, wrong, pins = MUTATIONS[name]
    monkeypatch.setattr(R, attr, wrong)
    for pin in pins:
        with pytest.raises(AssertionError):
            pin()
