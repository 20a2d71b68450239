"""Pins of the oracle's particle coupling: the implicit (Nguyen-Ladd type)
solve and its two-step mean of the velocity-free sums.

The paper couples the momentum exchange of Sec. 4.2 (Eqs. LBMMovWall,
TransferredMomentum, LBMhydrodynForce) to the rigid-body engine of Sec. 4.3
without fixing how the force enters the time integration; it cites the
solid-particle scheme of Nguyen and Ladd, in which the part of the exchange
that is linear in the surface velocity u_s = V + W x r is taken at the new
velocities.  With the link sums

    F0 = sum 2 f~_q c_q,   M0 = sum r x 2 f~_q c_q,
    A = sum 6 w_q rho0 c c^T,  B = sum 6 w_q rho0 c (r x c)^T,
    C = sum 6 w_q rho0 (r x c)(r x c)^T

the direct sums of Eq. LBMhydrodynForce at the old velocities are
F = F0 - A V - B W and M = M0 - B^T V - C W; the implicit update solves

    (m + A) V' + B W'        = m V + F0 + Fe
    B^T V' + (I(q) + C) W'   = Lang + M0 + Me

and the default coupling takes F0, M0 as the mean of this step's and the
previous step's values.  Each pin below checks that reading against
something other than itself: linear algebra with a solution chosen first,
the direct link sum, the fluid's momentum taken from the populations, and
the steady state every coupling must share.  The last test plants a
mistake in each part of the oracle and shows that a named pin fails.
"""
import numpy as np
import pytest

from oracle import pyoracle as O


def _quat_to(t):
    """A unit quaternion whose rotation maps e_x to the unit vector t."""
    t = np.asarray(t, float) / np.linalg.norm(t)
    ax = np.cross([1.0, 0.0, 0.0], t)
    s = np.linalg.norm(ax)
    if s < 1e-12:
        return np.array([1.0, 0, 0, 0]) if t[0] > 0 else np.array([0.0, 0, 0, 1])
    ang = np.arctan2(s, t[0])
    return np.r_[np.cos(ang / 2), np.sin(ang / 2) * ax / s]


def _world_inertia(q, i_par, i_perp):
    t = O.fiber_axis(q)
    return i_perp * np.eye(3) + (i_par - i_perp) * np.outer(t, t)


def _state(rng):
    st = np.zeros(16)
    st[0:3] = rng.uniform(5, 15, 3)
    q = rng.standard_normal(4)
    st[3:7] = q / np.linalg.norm(q)
    st[7:10] = 1e-3 * rng.standard_normal(3)
    st[10:13] = 1e-4 * rng.standard_normal(3)
    st[13:16] = 50.0 * rng.standard_normal(3)
    return st


def _spd(rng, scale):
    a = rng.standard_normal((3, 3))
    return scale * (a @ a.T + 3 * np.eye(3)) / 3


# ------------------------------------------------------------ the 6x6 solve
def test_implicit_step_without_linear_part_is_the_explicit_step():
    """A = B = C = 0: the system reduces to V' = V + F0/m and
    I(q) W' = Lang + M0, the explicit semi-implicit Euler step."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        st = _state(rng)
        m, ip, it = rng.uniform(50, 500), rng.uniform(10, 100), rng.uniform(100, 2000)
        F0, M0 = 0.1 * rng.standard_normal(3), rng.standard_normal(3)
        z = np.zeros(9)
        out, Fa, Ma = O.rigid_step_implicit(st, m, ip, it, F0, M0, z, z, z)
        ref = O.rigid_step(st, m, ip, it, F0, M0)
        np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(Fa, F0, rtol=0, atol=0)
        np.testing.assert_allclose(Ma, M0, rtol=0, atol=0)


def test_implicit_step_isotropic_added_mass_closed_form():
    """A = a 1, B = 0, C = c 1: V' = (m V + F0)/(m + a), and W' splits along
    the axis t into (Lang + M0).t / (I_par + c) and the rest over
    (I_perp + c); the applied force is F0 - a V' and the torque M0 - c W'."""
    rng = np.random.default_rng(12)
    for _ in range(20):
        st = _state(rng)
        m, ip, it = rng.uniform(50, 500), rng.uniform(10, 100), rng.uniform(100, 2000)
        a, c = rng.uniform(10, 200), rng.uniform(50, 3000)
        F0, M0 = 0.1 * rng.standard_normal(3), rng.standard_normal(3)
        out, Fa, Ma = O.rigid_step_implicit(st, m, ip, it, F0, M0, (a * np.eye(3)).ravel(),
                                            np.zeros(9), (c * np.eye(3)).ravel())
        V = (m * st[7:10] + F0) / (m + a)
        t = O.fiber_axis(st[3:7])
        rhs = st[13:16] + M0
        W = (rhs @ t) * t / (ip + c) + (rhs - (rhs @ t) * t) / (it + c)
        np.testing.assert_allclose(out[7:10], V, rtol=1e-13, atol=1e-18)
        np.testing.assert_allclose(out[10:13], W, rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(Fa, F0 - a * V, rtol=1e-12, atol=1e-16)
        np.testing.assert_allclose(Ma, M0 - c * W, rtol=1e-11, atol=1e-15)


def test_implicit_step_solves_the_coupled_system():
    """Choose V', W' first, with a non-symmetric B, and build F0, M0 from
    the two momentum balances; the solve must return V', W'.  The applied
    force then equals m (V' - V) and the new angular momentum equals
    I(q) W' (the torque row uses B^T: a B in its place, a sign of C or a
    dropped term moves W' far beyond the tolerance)."""
    rng = np.random.default_rng(13)
    for _ in range(30):
        st = _state(rng)
        m, ip, it = rng.uniform(50, 500), rng.uniform(10, 100), rng.uniform(100, 2000)
        A, C = _spd(rng, 100.0), _spd(rng, 1000.0)
        B = 10.0 * rng.standard_normal((3, 3))
        assert np.abs(B - B.T).max() > 1.0
        Vn, Wn = 1e-3 * rng.standard_normal(3), 1e-4 * rng.standard_normal(3)
        I = _world_inertia(st[3:7], ip, it)
        F0 = (m * np.eye(3) + A) @ Vn + B @ Wn - m * st[7:10]
        M0 = B.T @ Vn + (I + C) @ Wn - st[13:16]
        out, Fa, Ma = O.rigid_step_implicit(st, m, ip, it, F0, M0, A.ravel(), B.ravel(), C.ravel())
        np.testing.assert_allclose(out[7:10], Vn, rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(out[10:13], Wn, rtol=1e-9, atol=1e-16)
        np.testing.assert_allclose(Fa, m * (Vn - st[7:10]), rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(out[13:16], I @ Wn, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(out[0:3], st[0:3] + Vn, rtol=0, atol=1e-13)


# ------------------------------------------------------------ the link sums
def test_exchange_split_reproduces_the_direct_sums():
    """For a moving, rotating fiber off the lattice symmetry in a random
    fluid state, the split sums at the old velocities give back the direct
    sums of Eq. LBMhydrodynForce and its torque: F0 - A V - B W = F and
    M0 - B^T V - C W = M.  A and C are symmetric positive semi-definite
    (sums of outer products), B is not symmetric, so a transposed or
    sign-flipped matrix shows at the size of (B - B^T) V."""
    n = 20
    sim = O.Sim(n, n, n, tau=0.8, z_periodic=True, coupling="implicit")
    c, w, _ = O.lattice()
    rng = np.random.default_rng(1)
    V = np.array([0.01, -0.02, 0.015])
    W = np.array([0.003, -0.002, 0.004])
    sim.add_fiber([9.3, 10.6, 9.8], _quat_to([0.4, 0.7, 0.59]), 10.0, 2.3, 1.0, V=V, W=W)
    sim.set_populations(w[:, None, None, None] * (1 + 0.05 * rng.standard_normal((19, n, n, n))))
    _, _, V0, W0 = sim.fiber_state()
    sim.step(1)
    s = sim.exchange_sums()
    A, B, Cm = s["A"][0], s["B"][0], s["C"][0]
    Fs = s["F0"][0] - A @ V0[0] - B @ W0[0]
    Ms = s["M0"][0] - B.T @ V0[0] - Cm @ W0[0]
    scale = np.abs(s["F"][0]).max()
    np.testing.assert_allclose(Fs, s["F"][0], rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(Ms, s["M"][0], rtol=0, atol=1e-13 * np.abs(s["M"][0]).max())
    # a transposed B would move the torque by (B - B^T) V, far above the tolerance
    assert np.abs((B - B.T) @ V0[0]).max() > 1e-7 * np.abs(s["M"][0]).max()
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Cm, Cm.T, rtol=0, atol=1e-10)
    assert np.linalg.eigvalsh(A).min() > 0 and np.linalg.eigvalsh(Cm).min() > 0
    # A = sum over links of 6 w rho0 c c^T: its trace is 6 rho0 sum w |c|^2
    # = 6/18 per axis link and 12/36 per diagonal link, i.e. 1/3 per link
    # (every D3Q19 link has w |c|^2 = 1/18), so tr A = (number of links)/3
    nlinks = _count_links(sim, n)
    np.testing.assert_allclose(np.trace(A), nlinks / 3.0, rtol=1e-13)


def _count_links(sim, n):
    """Fluid-to-fiber links of the current map, counted from the cell map."""
    c = O.lattice()[0]
    _, _, flags, _ = sim.fields()
    solid = flags.astype(bool)
    cnt = 0
    for q in range(1, 19):
        nb = np.roll(solid, shift=(-c[q][2], -c[q][1], -c[q][0]), axis=(0, 1, 2))
        cnt += int((~solid & nb).sum())
    return cnt


# ------------------------------------------------------------ momentum budget
def _forced_fiber_box(coupling):
    n = 20
    sim = O.Sim(n, n, n, tau=0.8, z_periodic=True, coupling=coupling)
    Fe = np.array([1e-3, -5e-4, 7e-4])
    L, r = 9.0, 2.0
    sim.add_fiber([10.1, 9.7, 10.3], _quat_to([0.2, 0.9, 0.39]), L, r, 1.0,
                  shape="spherocylinder", force=Fe)
    mass = O.body_inertia("spherocylinder", L, r, 1.0)[0]
    return sim, Fe, mass


@pytest.mark.parametrize("coupling", ["implicit", "implicit_plain"])
def test_implicit_coupling_momentum_budget(coupling):
    """Fully periodic box, one fiber under a constant force Fe, no cell
    changing owner.  The fluid loses the direct sum F0 - A V - B W of the
    old velocities each step; the particle gains the applied force plus Fe.
    Summed over n steps (A fixed while the map is fixed, B drifting only
    with the lever arms), the total momentum P = fluid + m V obeys

      P(n) - P(0) - n Fe = -A (V(n) - V(0)) - sum_k B(k) (W(k+1) - W(k))
                           + 1/2 (F0(first step) - F0(last step))

    for the two-step mean (without the mean the last term is absent): the
    defect stays bounded by the velocities instead of growing with n.  A
    mean weighted other than 1/2, 1/2 leaves a term growing like n F0."""
    sim, Fe, mass = _forced_fiber_box(coupling)
    c = O.lattice()[0].astype(np.float64)

    def total():
        f = sim.populations()
        _, _, _, pid = sim.fields()
        _, _, V, W = sim.fiber_state()
        return np.einsum("qa,qzyx->a", c, f * (pid < 0)[None]) + mass * V[0], pid, V[0], W[0]

    p0, pid0, V0, W0 = total()
    F0first = None
    bsum = np.zeros(3)
    Wprev = W0
    for k in range(1, 101):
        sim.step(1)
        s = sim.exchange_sums()
        if F0first is None:
            F0first = s["F0"][0].copy()
        _, _, _, Wk = sim.fiber_state()
        bsum += s["B"][0] @ (Wk[0] - Wprev)
        Wprev = Wk[0]
    p, pid, V, W = total()
    assert np.array_equal(pid, pid0)
    defect = p - p0 - 100 * Fe
    expect = -s["A"][0] @ (V - V0) - bsum
    if coupling == "implicit":
        expect = expect + 0.5 * (F0first - s["F0"][0])
    np.testing.assert_allclose(defect, expect, rtol=0, atol=1e-7 * np.linalg.norm(100 * Fe))
    assert np.linalg.norm(defect) > 1e-3 * np.linalg.norm(100 * Fe)


# ------------------------------------------------------------ shared steady state
def _terminal(coupling, kind):
    if kind == "rotation":
        # rotation about the own axis under a constant torque: the cell map
        # never changes (the predicate depends on the distance to the axis)
        n = 16
        sim = O.Sim(n, n, n, tau=0.8, z_periodic=True, coupling=coupling)
        sim.add_fiber([7.5, 7.5, 7.5], [1.0, 0, 0, 0], 8.0, 2.5, 4.0, torque=[0.02, 0, 0])
        steps = 3000
    else:
        # translation along the own axis between resting walls, centred in
        # y and z, under a constant force: the ends stay between cell centres
        sim = O.Sim(16, 12, 12, tau=0.8, z_periodic=False, coupling=coupling)
        sim.add_fiber([7.3, 5.5, 5.5], [1.0, 0, 0, 0], 6.0, 1.6, 4.0, force=[2e-4, 0, 0])
        steps = 6000
    _, _, _, pid0 = sim.fields()
    sim.step(steps - 200)
    _, _, Va, Wa = sim.fiber_state()
    sim.step(200)
    _, _, V, W = sim.fiber_state()
    _, _, _, pid = sim.fields()
    assert np.array_equal(pid, pid0)
    return np.r_[V[0], W[0]], np.r_[Va[0], Wa[0]]


@pytest.mark.parametrize("kind", ["rotation", "translation"])
def test_couplings_share_the_terminal_state(kind):
    """At a fixed point V' = V, W' = W and F0 stops changing, so the
    explicit step, the implicit solve and the implicit solve with the
    two-step mean all reduce to the same balance F0 - A V - B W + Fe = 0,
    M0 - B^T V - C W + Me = 0 with the same fluid.  At density ratio 4,
    where the explicit coupling is stable, the three must reach the same
    terminal velocity (closed-form Stokes drag is not available for the
    staircase body; the shared fixed point is)."""
    res = {}
    for cp in ("explicit", "implicit", "implicit_plain"):
        x, xa = _terminal(cp, kind)
        # steady: no change over the last 200 steps
        np.testing.assert_allclose(x, xa, rtol=0, atol=1e-9 * np.abs(x).max())
        res[cp] = x
    big = np.abs(res["explicit"]).max()
    assert big > 1e-5
    for cp in ("implicit", "implicit_plain"):
        np.testing.assert_allclose(res[cp], res["explicit"], rtol=0, atol=1e-7 * big)


# ------------------------------------------------------------ each pin can fail
MUTATIONS = {
    1: [test_implicit_step_solves_the_coupled_system],
    2: [test_implicit_step_isotropic_added_mass_closed_form,
        test_implicit_step_solves_the_coupled_system],
    3: [test_exchange_split_reproduces_the_direct_sums],
    4: [lambda: test_implicit_coupling_momentum_budget("implicit"),
        lambda: test_couplings_share_the_terminal_state("rotation")],
}


@pytest.mark.parametrize("code", sorted(MUTATIONS))
def test_pins_fail_on_planted_mistakes(code):
    """Plant each mistake in the oracle (1: B in place of B^T in the torque
    row of the solve; 2: -C in place of C; 3: B summed transposed; 4: the
    two-step mean without its 1/2) and check that the named pins fail."""
    try:
        O.set_mutation(code)
        for pin in MUTATIONS[code]:
            with pytest.raises(AssertionError):
                pin()
    finally:
        O.set_mutation(0)
