"""The 256^3 shear cell with 64 fibers (the benchmark workload, same launch
path: captured graph) against the oracle over its first 100 steps, through
remap events: cell maps bit-exact, velocity and force/torque within the FP32
tolerances; the FP16/BF16 storage forms of the same workload within their
storage bounds; and the 512-case batched workload."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_1503_06869_amd import lbm, scenarios

from helpers import rel_l2, ft_error

pytestmark = pytest.mark.gpu


_ORACLE = {}
STEPS = 100


def _oracle(sc):
    """The oracle's run of the workload, once per module: fields before and
    after STEPS steps, the history and the final fiber state."""
    if not _ORACLE:
        o = O.Sim(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u,
                  init_couette=sc.init_couette)
        for f in sc.fibers:
            o.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
        _ORACLE["pid0"] = o.fields()[3]
        o.step(STEPS)
        _ORACLE["fields"] = o.fields()
        _ORACLE["history"] = o.history()
        _ORACLE["X"] = o.fiber_state()[0]
    return _ORACLE


def _gpu_run(sc, storage, torch):
    g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u,
                    init_couette=sc.init_couette, storage=storage,
                    stream=torch.cuda.current_stream().cuda_stream)
    for f in sc.fibers:
        g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    g.step(STEPS)
    out = g.fields(), g.history(0, STEPS), g.fiber_state()[0]
    g.close()
    return out


def test_full_size_first_steps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = scenarios.many_fibers(seed=0)
    ref = _oracle(sc)
    (_, ug, flg, pidg), hg, Xg = _gpu_run(sc, "f32", torch)
    _, uo, flo, pido = ref["fields"]
    changed = int((pido != ref["pid0"]).sum())
    assert np.array_equal(pidg, pido)
    fl = flo == 0
    e = rel_l2(ug.astype(np.float64), uo, fl)
    eF, eM = ft_error(hg, ref["history"], [f.length for f in sc.fibers])
    print("256^3 after %d steps: %d cells changed owner; velocity %.3g F %.3g M %.3g |dX| %.3g"
          % (STEPS, changed, e, eF, eM, np.abs(Xg - ref["X"]).max()), flush=True)
    assert changed > 100
    assert e < 1e-5 and eF < 1e-4 and eM < 1e-4


@pytest.mark.parametrize("storage,tol", [("f16", 3e-3), ("bf16", 3e-2)])
def test_full_size_sixteen_bit_storage(storage, tol):
    """The precision form at the benchmark size: FP16 / BF16 deviation
    storage of the 256^3 workload against the FP64 oracle after 100 steps.
    The velocity error is held to the same storage-resolution bounds as on
    the 32^3 cell; the force and torque errors are stated.  Poses differ
    from the oracle's by the storage error, so a cell whose centre lies
    that close to a fiber surface may change owner a step apart: the maps
    are compared by count."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = scenarios.many_fibers(seed=0)
    ref = _oracle(sc)
    (_, ug, flg, pidg), hg, Xg = _gpu_run(sc, storage, torch)
    _, uo, flo, pido = ref["fields"]
    fl = (flo == 0) & (flg == 0)
    e = rel_l2(ug.astype(np.float64), uo, fl)
    eF, eM = ft_error(hg, ref["history"], [f.length for f in sc.fibers])
    diff = int((pidg != pido).sum())
    print("256^3 %s after %d steps: velocity %.3g F %.3g M %.3g |dX| %.3g, %d cells with another owner"
          % (storage, STEPS, e, eF, eM, np.abs(Xg - ref["X"]).max(), diff), flush=True)
    assert e < tol
    assert diff <= 200


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
