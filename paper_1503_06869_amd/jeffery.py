"""Tumbling-period measurement shared by the golden-value script, the GPU
tests and the benchmark (post-processing only; no simulation arithmetic).

The period of a Jeffery orbit is measured from the fiber axis history: the
x component of the axis changes sign each time the fiber passes through the
gradient direction, twice per period.  Crossing times are located by linear
interpolation; the first crossing is discarded (start-up transient) and the
period is twice the mean interval between the following crossings, up to the
fourth crossing.  (The coarse staircase fibers used here eventually settle
next to the flow direction after a few turns: a fiber of diameter 4 cells
is held where its end cells change; which turn that happens on depends on
rounding, so only the regular turns before it are used.)"""
import numpy as np


def axis_from_quat(q):
    """Rotated e_x for quaternions q[..., 4] = (w, x, y, z)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], -1)


def crossings(tx, step0=1):
    tx = np.asarray(tx, dtype=np.float64)
    s = np.sign(tx)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    t = []
    for i in idx:
        a, b = tx[i], tx[i + 1]
        t.append(step0 + i + a / (a - b))
    return np.array(t)


def period(tx, step0=1, min_crossings=3, max_crossings=4):
    """Returns (period, crossing times) or (nan, crossings) if too few."""
    c = crossings(tx, step0)
    if len(c) < min_crossings:
        return float("nan"), c
    return 2.0 * float(np.mean(np.diff(c[1:max_crossings]))), c


def jeffery_period(aspect_ratio, shear_rate):
    """Closed form T = 2 pi (r + 1/r) / shear rate for a spheroid of aspect
    ratio r in unbounded Stokes shear flow."""
    r = aspect_ratio
    return 2 * np.pi * (r + 1.0 / r) / shear_rate
