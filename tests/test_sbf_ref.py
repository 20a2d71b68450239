"""Pins of the FP64 slender-body reference (oracle/sbf_ref.py, paper Sec. 3)
against what the paper and the mathematics fix: the single-fiber closed
forms of Sec. 5 (Eqs. SBF_Onefib_vel, SB_ForceParallPerpend, SB_Torque),
the Legendre eigenvalues of the finite-part operator of Eq. Kbar checked by
direct quadrature, the Stokes equations satisfied by the Green's function
of Eq. Gnonper, the Stokeslet far field of a distant fiber (which also fixes
the normalisation of the interaction term in the translational velocity),
mirror symmetry and convergence in the number of Legendre modes."""
import numpy as np
import pytest
from scipy import integrate

from oracle import sbf_ref as S


def test_legendre_recurrence_matches_the_power_series():
    x = np.linspace(-1, 1, 41)
    P = S.legendre(7, x)
    for n in range(8):
        c = np.zeros(n + 1)
        c[n] = 1.0
        np.testing.assert_allclose(P[n], np.polynomial.legendre.legval(x, c), rtol=0, atol=1e-14)


def test_quadrature_is_exact_for_quintics_on_each_sub_interval():
    t, w = S.quadrature(7)
    assert abs(w.sum() - 2.0) < 1e-14
    for deg in range(6):
        exact = (1 - (-1) ** (deg + 1)) / (deg + 1)
        assert abs(np.sum(w * t ** deg) - exact) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_kbar_eigenvalues_by_direct_quadrature(n):
    """Kbar[P_n](s) = int_{-1}^{1} (P_n(s') - P_n(s)) / |s' - s| ds' = L_n P_n(s)
    with L_n = -2 sum_{i<=n} 1/i (the diagonalisation the method relies on)."""
    Ln = S.kbar_eigenvalues(n)[n]
    c = np.zeros(n + 1)
    c[n] = 1.0
    P = lambda x: np.polynomial.legendre.legval(x, c)
    for s in (-0.83, -0.31, 0.0, 0.47, 0.91):
        f = lambda sp: (P(sp) - P(s)) / abs(sp - s)
        val = integrate.quad(f, -1.0, s, limit=200)[0] + integrate.quad(f, s, 1.0, limit=200)[0]
        assert abs(val - Ln * P(s)) < 1e-9, (n, s, val, Ln * P(s))


def test_green_function_solves_the_stokes_equations():
    """u(x) = G(x) F: the Stokeslet S and the doublet D are divergence free
    away from the origin, and D = (1/2) lap S, so G = S + (r^2/2) D =
    (1 + (r^2/4) lap) S: checked by central differences at random points."""
    rng = np.random.default_rng(3)
    F = rng.standard_normal(3)
    h = 1e-3
    for _ in range(5):
        x = rng.standard_normal(3) * 2.0
        x *= 1.5 / np.linalg.norm(x) if np.linalg.norm(x) < 1.5 else 1.0
        uS = lambda y: S.green(y, 0.0) @ F
        uD = lambda y: (S.green(y, np.sqrt(2.0)) - S.green(y, 0.0)) @ F   # = D F
        for u in (uS, uD):
            div = sum((u(x + h * e)[k] - u(x - h * e)[k]) / (2 * h) for k, e in enumerate(np.eye(3)))
            assert abs(div) < 1e-5 * np.linalg.norm(u(x)) / np.linalg.norm(x)
        lapS = sum((uS(x + h * e) - 2 * uS(x) + uS(x - h * e)) / h ** 2 for e in np.eye(3))
        np.testing.assert_allclose(0.5 * lapS, uD(x), rtol=1e-4, atol=1e-6 * np.linalg.norm(uD(x)))


@pytest.mark.parametrize("eps", [1 / 10.0, 1 / 14.0, 1 / 40.0])
def test_single_fiber_closed_forms(eps):
    """One fiber in free space: U_par = 2 d F/(8 pi mu L), U_perp = (d + 2) F/(8 pi mu L),
    omega = 3 d M/(2 pi mu L^3) for a torque perpendicular to the axis."""
    L, mu = 40.0, 0.7
    sb = S.SBF(L, eps, mu=mu, N=5, nq=8)
    d = S.geometry_parameter(eps)
    p = np.array([0.3, -0.5, 0.81])
    p /= np.linalg.norm(p)
    e1 = np.cross(p, [1.0, 0, 0])
    e1 /= np.linalg.norm(e1)
    for F, expect in ((2.0 * p, 2 * d * 2.0 / (8 * np.pi * mu * L) * p),
                      (1.5 * e1, (d + 2) * 1.5 / (8 * np.pi * mu * L) * e1)):
        _, V, W = sb.solve([[1.0, 2.0, 3.0]], [p], [F], [[0, 0, 0]])
        np.testing.assert_allclose(V[0], expect, rtol=1e-14, atol=1e-17)
        np.testing.assert_allclose(W[0], 0.0, atol=1e-17)
    Mt = 0.9 * e1
    _, V, W = sb.solve([[0, 0, 0]], [p], [[0, 0, 0]], [Mt])
    omega = np.cross(p, W[0])
    np.testing.assert_allclose(omega, 3 * d * Mt / (2 * np.pi * mu * L ** 3), rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(V[0], 0.0, atol=1e-18)


def test_distant_fiber_sees_the_stokeslet_of_the_other():
    """Two fibers far apart (distance 400 L): fiber 2 (no force of its own)
    moves with the Stokeslet velocity S(R) F_1/(8 pi mu) of fiber 1's force,
    to relative order (L/R)^2; this fixes the normalisation of the
    interaction term, [Lambda F + int U ds]/(8 pi mu L)."""
    L, mu, eps = 30.0, 1.3, 1 / 12.0
    sb = S.SBF(L, eps, mu=mu, N=4, nq=8)
    Rv = np.array([0.6, -0.48, 0.64]) * 400 * L
    X = [[0, 0, 0], Rv]
    p = [[1.0, 0, 0], [0, 0.6, 0.8]]
    F1 = np.array([0.2, 1.0, -0.4])
    _, V, _ = sb.solve(X, p, [F1, [0, 0, 0]], [[0, 0, 0], [0, 0, 0]])
    u = S.green(-Rv, 0.0) @ F1 / (8 * np.pi * mu)
    np.testing.assert_allclose(V[1], u, rtol=1e-5, atol=0)


def test_mirror_symmetric_pair():
    """Two fibers mirror images of each other in the plane x = 0, forces
    mirrored: velocities mirrored, rotation rates mirrored."""
    sb = S.SBF(40.0, 1 / 12.0, N=5, nq=8)
    Xa = np.array([-7.5, 0.3, 0.0])
    pa = np.array([0.2, 0.1, 0.97])
    pa /= np.linalg.norm(pa)
    Fa = np.array([0.1, 0.0, 1.0])
    mir = np.diag([-1.0, 1.0, 1.0])
    _, V, W = sb.solve([Xa, mir @ Xa], [pa, -(mir @ pa)], [Fa, mir @ Fa], [[0, 0, 0], [0, 0, 0]])
    np.testing.assert_allclose(V[1], mir @ V[0], rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(W[1], -(mir @ W[0]), rtol=1e-12, atol=1e-16)
    assert abs(V[0][0]) > 1e-6 * abs(V[0][2])     # the pair interacts


def test_close_pair_converges_in_the_legendre_modes():
    """A sedimenting side-by-side pair 15 fiber radii apart (the paper's
    tumbling start, 1/eps = 12): velocities from N = 5 agree with N = 8."""
    L, eps = 48.0, 1 / 12.0
    X = [[-7.5, 0, 0], [7.5, 0, 0]]
    p = [[0.05, 0, 1.0], [-0.05, 0, 1.0]]
    F = [[0, 0, 1.0], [0, 0, 1.0]]
    Mt = [[0, 0, 0], [0, 0, 0]]
    res = [S.SBF(L, eps, N=N, nq=16).solve(X, p, F, Mt) for N in (5, 8)]
    np.testing.assert_allclose(res[0][1], res[1][1], rtol=2e-3, atol=1e-3 * np.abs(res[1][1]).max())
    np.testing.assert_allclose(res[0][2], res[1][2], rtol=0, atol=2e-2 * np.abs(res[1][2]).max())


def test_solution_satisfies_the_integral_equation():
    """The solved force densities and velocities satisfy Eq. sev_fils
    projected on P_0 .. P_N, with every term evaluated independently of the
    solver's shortcuts: Kbar[f] by direct finite-part quadrature, the
    interaction U by a fine Gauss rule (300 points) instead of the solver's
    48-point composite rule, the projections by a 200-point rule."""
    L, eps, mu, N = 48.0, 1 / 12.0, 1.0, 5
    sb = S.SBF(L, eps, mu=mu, N=N, nq=16)
    l = 0.5 * L
    X = np.array([[-7.5, 0.4, 0.0], [7.5, -0.2, 3.0]])
    p = np.array([[0.15, 0.05, 1.0], [-0.1, 0.2, 1.0]])
    p /= np.linalg.norm(p, axis=1)[:, None]
    F = np.array([[0.1, 0.0, 1.0], [0.0, 0.05, 1.0]])
    Mt = np.array([np.cross(p[0], [0.0, 0.3, 0.0]), np.cross(p[1], [0.2, 0.0, 0.0])])
    a, V, W = sb.solve(X, p, F, Mt)
    d = S.geometry_parameter(eps)
    Ln = S.kbar_eigenvalues(N)

    def f(m, s):              # force per unit length at arc length s (array)
        P = S.legendre(N, np.asarray(s) / l)
        return F[m][None, :] / (2 * l) + np.einsum("ns,na->sa", P[1:], a[m])

    tu, wu = np.polynomial.legendre.leggauss(300)
    su, wsu = l * tu, l * wu
    tp, wp = np.polynomial.legendre.leggauss(200)
    sp, wsp = l * tp, l * wp
    for m in range(2):
        o = 1 - m
        I = np.eye(3)
        pp = np.outer(p[m], p[m])
        lam = d * (I + pp) + 2 * (I - pp)
        K = I + pp
        # Kbar f at the projection nodes, directly: f is a polynomial in s,
        # so (f(s') - f(s))/|s' - s| is integrated by adaptive quadrature
        kb = np.zeros((len(sp), 3))
        for i, s in enumerate(sp):
            for c in range(3):
                g = lambda x: (f(m, [x])[0, c] - f(m, [s])[0, c]) / abs(x - s)
                kb[i, c] = (integrate.quad(g, -l, s, limit=200)[0] + integrate.quad(g, s, l, limit=200)[0])
        R = X[m][None, None, :] + sp[:, None, None] * p[m][None, None, :] - X[o][None, None, :] \
            - su[None, :, None] * p[o][None, None, :]
        U = np.einsum("ijab,jb,j->ia", S.green(R, sb.r), f(o, su), wsu)
        lhs = 8 * np.pi * mu * (V[m][None, :] + sp[:, None] * W[m][None, :])
        res = lhs - (f(m, sp) @ lam.T) - (kb @ K.T) - U
        Pn = S.legendre(N, sp / l)
        for n in range(N + 1):
            proj = (res * (Pn[n] * wsp)[:, None]).sum(0) * (2 * n + 1) / (2 * l)
            scale = np.abs(lhs).max()
            assert np.abs(proj).max() < 2e-5 * scale, (m, n, proj, scale)


def test_time_stepping_is_second_order_against_the_exact_rotation():
    """One fiber under a constant torque M perpendicular to its axis turns
    about M at the constant rate 3 d |M| / (2 pi mu L^3) (Eq. SB_Torque; p
    stays perpendicular to M).  The Adams-Bashforth-2 trajectory of `run`
    (Euler start, p renormalised) converges to that exact rotation at second
    order in dt (an Euler or a mis-weighted scheme gives first order)."""
    L, eps, mu = 30.0, 1 / 10.0, 1.3
    sb = S.SBF(L, eps, mu=mu, N=3, nq=4)
    d = S.geometry_parameter(eps)
    p0 = np.array([1.0, 0.0, 0.0])
    M = np.array([0.0, 0.0, 2.0e3])
    F = np.array([0.0, 0.5, 0.0])
    rate = 3 * d * np.linalg.norm(M) / (2 * np.pi * mu * L ** 3)
    T = 0.6 / rate                                   # a turn of 0.6 rad
    errs = []
    for n in (40, 80, 160):
        Xs, ps = sb.run([[0, 0, 0]], [p0], [F], [M], T / n, n)
        ang = rate * T
        exact = np.array([np.cos(ang), np.sin(ang), 0.0])       # p turns about +z (M x p)
        errs.append(np.linalg.norm(ps[-1, 0] - exact))
        # force and axis stay in the plane z = 0, and so does the centre
        assert abs(Xs[-1, 0, 2]) < 1e-12
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    print("AB2 errors", errs, "ratios", r1, r2)
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5
