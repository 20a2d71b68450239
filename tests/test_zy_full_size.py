"""The 256^3 shear cell with 64 fibers (the benchmark workload, same launch
path: captured graph) against the oracle over its first 100 steps, through
remap events: cell maps bit-exact, velocity and force/torque within the FP32
tolerances."""
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
    _, _, _, pid0 = g.fields()
    n = 100
    g.step(n)
    o.step(n)
    _, ug, flg, pidg = g.fields()
    _, uo, flo, pido = o.fields()
    changed = int((pido != pid0).sum())
    assert np.array_equal(pidg, pido)
    fl = flo == 0
    e = rel_l2(ug.astype(np.float64), uo, fl)
    eF, eM = ft_error(g.history(0, n), o.history(), [f.length for f in sc.fibers])
    Xg, _, _, _ = g.fiber_state()
    Xo, _, _, _ = o.fiber_state()
    print("256^3 after %d steps: %d cells changed owner; velocity %.3g F %.3g M %.3g |dX| %.3g"
          % (n, changed, e, eF, eM, np.abs(Xg - Xo).max()), flush=True)
    assert changed > 100
    assert e < 1e-5 and eF < 1e-4 and eM < 1e-4


def test_batched_full_workload_first_steps():
    """512 uneven cases (edges 24..64, one fiber each) in one persistent
    launch: the largest and the smallest case equal their single-context
    runs bit for bit; no device error over the batch."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cases = scenarios.batched_cases(seed=0)
    b = lbm.Batch(cases)
    n = 6
    b.step(n)
    b.sync()
    info = b.info()
    print("batch: %d cases, %d cells, %d bins x %d threads" %
          (info["ncases"], info["cells"], info["bins"], info["threads"]), flush=True)
    assert info["ncases"] == 512 and info["steps_done"] == n
    sizes = [c.ncell for c in cases]
    for c in (int(np.argmax(sizes)), int(np.argmin(sizes))):
        sc = cases[c]
        g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u,
                        init_couette=True)
        f = sc.fibers[0]
        g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
        g.step(n)
        assert np.array_equal(b.history(c, 0, n), g.history(0, n)[:, 0, :]), c
        assert np.array_equal(b.populations(c), g.populations()), c
        g.close()
    F, M = b.force_torque()
    assert np.isfinite(F).all() and np.isfinite(M).all()
    b.close()
