"""Learned closure on the GPU through the C ABI (include/lbm_mlp.h), against
the FP64 reference (oracle/closure_ref.py) and the FP64 oracle:

  * network forward with the same BF16-rounded weights (rel <= 1e-5) and
    gradient (rel <= 1e-3 in norm), one Adam step, BF16 copy = RNE(master);
  * training: deterministic and reduces the loss of a teacher problem;
  * features of a fiber after some steps against the oracle's (FP32 state
    vs FP64 state: <= 2e-4 absolute on O(1) features);
  * a step with the closure attached against the oracle stepping with the
    correction computed from its own state (force/torque <= 1e-4); a
    network that outputs zero leaves the run bit-identical; the envelope
    fallback removes the correction and is counted."""
import numpy as np
import pytest

from oracle import closure_ref as R
from oracle import pyoracle as O
from paper_1503_06869_amd import lbm, scenarios

from helpers import ft_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    lbm.load()
    return t


def random_params(seed, scale=0.15):
    g = np.random.default_rng(seed)
    return (g.normal(0, scale, R.NPARAM)).astype(np.float32)


def test_forward_and_gradient_match_reference(torch):
    w = random_params(1)
    g = np.random.default_rng(2)
    n = 77                                        # three tiles, the last ragged
    x = g.normal(0.3, 2.0, (n, R.NI)).astype(np.float32)
    t = g.normal(0, 1, (n, R.NO)).astype(np.float32)
    mean = g.normal(0.3, 0.1, R.NI).astype(np.float32)
    inv = (1.0 / g.uniform(1.5, 2.5, R.NI)).astype(np.float32)
    osc = g.uniform(0.5, 2.0, R.NO).astype(np.float32)
    m = lbm.Mlp(seed=3)
    m.set_params(w)
    m.set_norm(mean, inv, osc)
    wm, wb = m.params()
    assert np.array_equal(wm, w)
    wr = R.bf16_round(w)
    assert np.array_equal((wb.astype(np.uint32) << 16).view(np.float32).astype(np.float64), wr)
    xd = torch.tensor(x, device="cuda")
    td = torch.tensor(t, device="cuda")
    yd = torch.zeros((n, R.NO), device="cuda")
    m.forward(xd.data_ptr(), n, yd.data_ptr())
    xn = (x.astype(np.float64) - mean) * inv
    yr = R.forward(wr, xn) * osc
    e = np.abs(yd.cpu().numpy() - yr).max() / np.abs(yr).max()
    print("forward rel err %.2e" % e, flush=True)
    assert e < 1e-5
    loss, grad = m.loss_grad(xd.data_ptr(), td.data_ptr(), n)
    lr_, gr = R.loss_grad(wr, xn, t.astype(np.float64))
    eg = np.linalg.norm(grad - gr) / np.linalg.norm(gr)
    print("loss %.6g vs %.6g, gradient rel err %.2e" % (loss, lr_, eg), flush=True)
    assert abs(loss / lr_ - 1) < 1e-5 and eg < 1e-3
    # one Adam step from the zero state: w - lr * g / (|g| + eps) elementwise
    m.adam(1e-3)
    w1, wb1 = m.params()
    w_ref, _, _ = R.adam(w, np.zeros_like(w), np.zeros_like(w), gr.astype(np.float32), 1, 1e-3)
    close = np.abs(w1 - w_ref) <= 1e-6
    print("Adam: %.4f of the parameters within 1e-6" % close.mean(), flush=True)
    assert close.mean() > 0.99
    assert np.array_equal(wb1, (R.bf16_round(w1).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16))
    m.close()


def test_training_is_deterministic_and_learns_a_teacher(torch):
    g = np.random.default_rng(5)
    n = 2048
    x = g.normal(0, 1, (n, R.NI)).astype(np.float32)
    teacher = random_params(6, 0.1).astype(np.float64)
    t = R.forward(teacher, x.astype(np.float64)).astype(np.float32)
    t /= t.std(0)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    runs = []
    for _ in range(2):
        m = lbm.Mlp(seed=11)
        losses = m.train(xd.data_ptr(), td.data_ptr(), n, epochs=25, batch=128, lr=2e-3, shuffle_seed=9)
        runs.append((losses, m.params()[0]))
        m.close()
    print("loss per epoch:", np.array2string(runs[0][0][[0, 5, 10, 24]], precision=4), flush=True)
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    assert runs[0][0][-1] < 0.1 * runs[0][0][0]


def _shear_pair(steps):
    sc = scenarios.single_fiber(seed=0, wall_u=0.02)
    f = sc.fibers[0]
    g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True)
    g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    o = O.Sim(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True)
    o.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    return sc, g, o


def _oracle_features(sc, o):
    _, u, _, _ = o.fields()
    X, q, V, W = o.fiber_state()
    gamma = 2 * sc.wall_u / sc.nz
    return R.features(u, X[0], q[0], V[0], W[0], sc.fibers[0].length, gamma)


def test_features_match_oracle(torch):
    sc, g, o = _shear_pair(0)
    for n in (0, 37):
        g.step(n)
        o.step(n)
        fg = g.features()[0]
        fo = _oracle_features(sc, o)
        e = np.abs(fg - fo).max()
        print("after %d steps: max |df| %.2e (|f| max %.2f)" % (n, e, np.abs(fo).max()), flush=True)
        assert e < 2e-4
    g.close()


def test_closure_step_matches_oracle_with_the_same_correction(torch):
    sc, g, o = _shear_pair(0)
    L, gamma, nu = sc.fibers[0].length, 2 * sc.wall_u / sc.nz, (sc.tau - 0.5) / 3
    m = lbm.Mlp(seed=4)
    w = random_params(8, 0.05)
    m.set_params(w)
    osc = np.full(R.NO, 0.5, np.float32)
    m.set_norm(np.zeros(R.NI), np.full(R.NI, 0.5), osc)
    g.set_closure(m)
    wr = R.bf16_round(w)
    steps = 12
    for _ in range(steps):
        feat = _oracle_features(sc, o)
        y = R.forward(wr, (feat * 0.5)[None, :])[0] * 0.5
        sF = 1.0 * nu * gamma * L * L
        Rq = R.rotation(feat[243:])           # body-frame output to the lab frame
        o.set_correction(0, Rq @ y[:3] * sF, Rq @ y[3:] * sF * L)
        o.step(1)
    g.step(steps)
    hg, ho = g.history(0, steps), o.history(0, steps)
    eF, eM = ft_error(hg, ho, [L])
    print("closure run: F %.2e M %.2e" % (eF, eM), flush=True)
    assert eF < 1e-4 and eM < 1e-4
    applied, fallbacks = g.closure_stats()
    assert (applied, fallbacks) == (steps, 0)
    g.close()
    m.close()


def test_zero_network_is_bit_identical_and_fallback_counts(torch):
    sc = scenarios.single_fiber(seed=0, wall_u=0.02)
    f = sc.fibers[0]
    runs = []
    for mode in ("none", "zero", "fallback"):
        g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True)
        g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
        m = None
        if mode != "none":
            m = lbm.Mlp(seed=1)
            w = random_params(9)
            if mode == "zero":
                w[-(R.NO * R.NH + R.NO):] = 0.0        # W3 = 0, b3 = 0: zero output
            m.set_params(w)
            if mode == "fallback":
                m.set_norm(env_min=np.full(R.NI, -1e-9), env_max=np.full(R.NI, 1e-9))
            g.set_closure(m)
        g.step(20)
        runs.append(g.history(0, 20))
        if mode == "fallback":
            assert g.closure_stats() == (0, 20)
        g.close()
        if m is not None:
            m.close()
    assert np.array_equal(runs[0], runs[1]) and np.array_equal(runs[0], runs[2])
