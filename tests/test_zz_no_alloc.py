"""The allocation-free field readback (lbm_get_fields_static) against
lbm_get_fields on the same state: identical bytes, on two calls in a row,
the second on a smaller lattice, and on a lattice larger than one chunk of
the fixed staging array."""
import numpy as np
import pytest

from paper_1503_06869_amd import lbm, scenarios

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lbm.load()
    yield


def _ctx(n, steps, storage):
    sc = scenarios.many_fibers(seed=3, n=n, n_fibers=2, length=(10.0, 14.0), diameter=(3.0, 4.0),
                               wall_u=0.01)
    g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True,
                    storage=storage)
    for f in sc.fibers:
        g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    g.step(steps)
    return g


def _same(g):
    a = g.fields()
    b = g.fields_static()
    for x, y in zip(a, b):
        assert x.dtype == y.dtype and np.array_equal(x, y)
    return a


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_static_fields_equal_allocating_fields(storage):
    # 1.05M cells: more than one chunk of the 16 MiB array (1M FP32 cells, 512k FP64)
    big = _ctx(102, 3, storage)
    a = _same(big)
    assert (a[2] == 1).sum() > 0
    big.close()
    small = _ctx(40, 5, storage)     # second call: smaller lattice, odd parity
    _same(small)
    small.step(1)
    _same(small)                     # even parity
    small.close()
