"""Tumbling period of a fiber in the 32^3 shear cell on the GPU against the
FP64 oracle's period (tests/golden/jeffery_single_fiber.json, written by
tests/golden/make_jeffery_golden.py which runs only the oracle).

The configuration is the single-fiber cell (L = 16, d = 4, tau = 0.8,
density ratio 1, Lambda = 3/16) at its wall speed U = 0.005 (shear rate
3.125e-4, particle Reynolds number 0.05: oracle period 78,581 steps, the
third measured crossing at about 119.4k steps), and at U = 0.02 (period
19,721 steps).

FP32 storage must reproduce the oracle period within 0.5 %, FP16 deviation
storage within 1 %.  BF16 keeps 8 significant bits (unit roundoff 2^-9 of
each stored deviation); this rounding is re-applied every step and no
closed bound on how it accumulates into the period is available, so the
BF16 period error is measured and printed, not asserted: the test only
requires that the fiber tumbles with a period inside the +-15 % band of
Jeffery's closed form that the oracle itself is held to."""
import json
import os

import numpy as np
import pytest

from paper_1503_06869_amd import jeffery, lbm, scenarios

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "jeffery_single_fiber.json")

# steps run on the GPU: the oracle's third crossing plus 5 % of a period
STEPS = {"U0.005/seed0": 124000, "U0.02/seed0": 62000}


def _gold(key):
    d = json.load(open(GOLD))
    if key not in d:
        pytest.skip("golden period %s not generated" % key)
    return d[key]


@pytest.mark.parametrize("key", ["U0.005/seed0", "U0.02/seed0"])
@pytest.mark.parametrize("storage,tol", [("f32", 0.005), ("f16", 0.01), ("bf16", None)])
def test_tumbling_period_matches_oracle(storage, tol, key):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gold = _gold(key)
    steps = STEPS[key]
    assert gold["crossings"][3] < steps
    sc = scenarios.single_fiber(seed=0, wall_u=gold["wall_u"])
    f = sc.fibers[0]
    g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True,
                    storage=storage, history_capacity=steps)
    g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    g.step(steps)
    h = g.history(0, steps)
    g.close()
    tx = jeffery.axis_from_quat(h[:, 0, 9:13])[:, 0]
    T, cr = jeffery.period(tx)
    rel = T / gold["period"] - 1
    print("%s %s: period %.1f (oracle %.1f), rel %+.3e, crossings %s" % (
        key, storage, T, gold["period"], rel, np.round(cr).tolist()), flush=True)
    if tol is None:
        TJ = jeffery.jeffery_period(f.length / (2 * f.radius), sc.shear_rate)
        assert np.isfinite(T) and abs(T / TJ - 1) < 0.15
    else:
        assert abs(rel) < tol
