"""Checkpoint and resume through the C ABI: k steps, lbm_save, lbm_load,
n - k more steps give bit-identical histories, populations, fiber states
and stabilization mean to n steps run straight."""
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


CASES = {
    # storage, context options, fibers (centre, axis, L, r, shape, force), steps before the save
    "f32_periodic_stabilized": ("f32", dict(z_periodic=True, stabilize=True, contact_k=1.0, contact_range=2.0),
                                [((13.3, 15.1, 12.6), (0.7, 0.3, 0.65), 12.0, 2.4, "spherocylinder", (0.03, 0.0, 0.04)),
                                 ((27.6, 20.4, 19.3), (0.2, 0.9, -0.4), 11.0, 2.0, "cylinder", (-0.02, 0.01, 0.03))], 31),
    "f16_closed_box": ("f16", dict(wall_u=0.0, x_walls=True, y_walls=True),
                       [((20.0, 18.0, 16.0), (1.0, 0.2, 0.1), 14.0, 2.5, "spherocylinder", (0.0, 0.0, 0.0))], 30),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_resume_is_bit_identical(name, tmp_path):
    storage, opts, fibers, k = CASES[name]
    n = k + 25

    def make():
        g = lbm.Context(40, 36, 32, tau=0.8, storage=storage, **opts)
        for X, t, L, r, shape, F in fibers:
            q = scenarios.quat_from_axis(np.asarray(t) / np.linalg.norm(t))
            g.add_fiber(X, q, L, r, 1.0, shape=shape, force=F, W=(0.0, 0.004, 0.0))
        return g

    a = make()
    a.step(k)
    path = tmp_path / "state.ckpt"
    a.save(path)
    a.step(n - k)
    b = lbm.Context.load_checkpoint(path)
    assert b.shape == a.shape and b.nfibers == a.nfibers and b.info()["steps_done"] == k
    b.step(n - k)
    ha, hb = a.history(0, n), b.history(0, n)
    assert np.array_equal(ha, hb), np.abs(ha - hb).max()
    assert np.array_equal(a.populations(), b.populations())
    for x, y in zip(a.fiber_state(), b.fiber_state()):
        assert np.array_equal(x, y)
    fa, fb = a.fields(), b.fields()
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    if opts.get("stabilize"):
        assert np.array_equal(a.mean_velocity()[0], b.mean_velocity()[0])
    moved = np.abs(ha[-1, :, 6:9] - ha[0, :, 6:9]).max()
    print("%s: resumed after %d of %d steps, bit-identical (fibers moved %.3f)" % (name, k, n, moved), flush=True)
    a.close()
    b.close()
