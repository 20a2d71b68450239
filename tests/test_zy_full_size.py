"""The 256^3 shear cell with 64 fibers (the benchmark workload, same launch
path: captured graph) against the oracle over the first steps: cell maps
bit-exact, velocity and force/torque within the FP32 tolerances."""
import numpy as np
import pytest

from paper_1503_06869_amd import lbm, scenarios

from helpers import make_pair, rel_l2, ft_error

pytestmark = pytest.mark.gpu


def test_full_size_first_steps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = scenarios.many_fibers(seed=0)
    g, o = make_pair(sc, stream=torch.cuda.current_stream().cuda_stream)
    n = 4
    g.step(n)
    o.step(n)
    _, ug, flg, pidg = g.fields()
    _, uo, flo, pido = o.fields()
    assert np.array_equal(pidg, pido)
    fl = flo == 0
    e = rel_l2(ug.astype(np.float64), uo, fl)
    eF, eM = ft_error(g.history(0, n), o.history(), [f.length for f in sc.fibers])
    print("256^3: velocity %.3g F %.3g M %.3g" % (e, eF, eM), flush=True)
    assert e < 1e-5 and eF < 1e-4 and eM < 1e-4
