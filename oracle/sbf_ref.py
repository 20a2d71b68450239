"""FP64 reference of the paper's slender-body formulation (SBF), Sec. 3.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline may call this module; the library never does.

Model (Sec. 3.1, Eqs. sev_fils, SBFGeomParam, Kbar, Ucontr_def, Gnonper,
extra_cond, force_exp, xadot, padot).  M straight fibers of length L = 2l
and radius r (slenderness eps = r/L, d = -ln(eps^2 e)) in free space, fiber
m with centre x_m and unit direction p_m, external force F_m and torque M_m
(perpendicular to p_m).  The force per unit length on fiber m is expanded
in Legendre polynomials of the dimensionless arc length s/l:

    f_m(s) = F_m / (2 l) + sum_{n=1..N} a_m^n P_n(s / l),   s in [-l, l].

With Lambda = d (I + p p^T) + 2 (I - p p^T), K = I + p p^T and the
eigenvalues L_n = -2 sum_{i=1..n} 1/i of the finite-part operator Kbar on
P_n, projecting Eq. sev_fils on P_n with weight (2n + 1)/(2l) gives, for
every fiber,

    n >= 2:  (Lambda + L_n K) a^n + c_n I_n = 0,          c_n = (2n + 1)/(2l),
    n  = 1:  (I - p p^T) a^1 = 3/(2 l^2) M x p               (torque, Eq. extra_cond),
             p . [(Lambda + L_1 K) a^1 + c_1 I_1] = 0         (p . dp/dt = 0),

where I_n = int U_m(s) P_n(s/l) ds and U_m is the velocity induced by the
other fibers (Eq. Ucontr_def, Green's function of Eq. Gnonper).  The
velocities follow from the n = 0 and n = 1 projections:

    dx/dt = [Lambda F + I_0] / (8 pi mu L),
    dp/dt = 3/(2 pi mu L^3) [d M x p + (I - p p^T) l I_1].

All integrals over a pair of fibers are the moments

    Theta^{n,k}_{mm'} = int int G(R(s, s')) P_k(s'/l) P_n(s/l) ds' ds,
    R = x_m + s p_m - x_m' - s' p_m',

evaluated with composite three-point Gauss rules on nq sub-intervals of
each fiber (the paper integrates the inner integral analytically with
formulas it does not print; both integrals are taken by the same rule
here).  The linear system is solved directly (numpy), the library uses
GMRES as the paper does.  Time integration: the paper names only an
explicit method of second order with constant dt; this reference uses
Adams-Bashforth of order two with one Euler step to start, and renormalises
p.

Parity unpinned: geometry_parameter.  d = -ln(eps^2 e) is Eq. SBFGeomParam
written out; the single-fiber closed forms of Sec. 5 that pin the rest are
expressed in the same d, and the paper prints no slender-body value for a
free-space configuration that would check it independently.
"""
import numpy as np


def geometry_parameter(eps):
    """d = -ln(eps^2 e) (Eq. SBFGeomParam)."""
    return -np.log(eps * eps * np.e)


def kbar_eigenvalues(N):
    """L_n for n = 0..N: Kbar[P_n] = L_n P_n with L_0 = 0 and
    L_n = -2 sum_{i=1..n} 1/i."""
    return np.array([0.0] + [-2.0 * sum(1.0 / i for i in range(1, n + 1)) for n in range(1, N + 1)])


def legendre(N, x):
    """P_0..P_N at the points x (three-term recurrence); shape [N+1][len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((N + 1,) + x.shape)
    P[0] = 1.0
    if N >= 1:
        P[1] = x
    for n in range(1, N):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
    return P


def quadrature(nq):
    """Composite three-point Gauss-Legendre rule on [-1, 1] with nq equal
    sub-intervals: nodes and weights."""
    g, w = np.polynomial.legendre.leggauss(3)
    h = 2.0 / nq
    nodes = np.concatenate([-1.0 + h * (i + 0.5) + 0.5 * h * g for i in range(nq)])
    weights = np.concatenate([0.5 * h * w for _ in range(nq)])
    return nodes, weights


def green(R, r):
    """G(R) = S(R) + (r^2/2) D(R), S = (I + Rh Rh^T)/|R|, D = (I - 3 Rh Rh^T)/|R|^3
    (Eq. Gnonper, fibers m' != m); R [..., 3] -> [..., 3, 3]."""
    R = np.asarray(R, dtype=np.float64)
    n = np.linalg.norm(R, axis=-1)
    Rh = R / n[..., None]
    I = np.eye(3)
    RR = Rh[..., :, None] * Rh[..., None, :]
    S = (I + RR) / n[..., None, None]
    D = (I - 3.0 * RR) / (n ** 3)[..., None, None]
    return S + 0.5 * r * r * D


def theta_pair(xm, pm, xn, pn, l, r, N, nq):
    """Theta^{n,k} (n, k = 0..N) of fiber m (test) against fiber m' (trial):
    array [N+1][N+1][3][3]."""
    t, w = quadrature(nq)
    P = legendre(N, t)
    s = l * t
    # R[i][j] = x_m + s_i p_m - x_m' - s_j p_m'
    R = (xm[None, None, :] + s[:, None, None] * pm[None, None, :]
         - xn[None, None, :] - s[None, :, None] * pn[None, None, :])
    G = green(R, r)                                    # [Q][Q][3][3]
    ws = l * w                                         # ds = l dt
    return np.einsum("ni,kj,i,j,ijab->nkab", P, P, ws, ws, G)


class SBF:
    """M fibers of length L, slenderness eps, in a fluid of viscosity mu."""

    def __init__(self, L, eps, mu=1.0, N=5, nq=16):
        self.L, self.l, self.eps, self.mu, self.N, self.nq = float(L), 0.5 * L, float(eps), float(mu), N, nq
        self.r = eps * L
        self.d = geometry_parameter(eps)
        self.Ln = kbar_eigenvalues(N)

    def _blocks(self, p):
        I = np.eye(3)
        pp = np.outer(p, p)
        lam = self.d * (I + pp) + 2.0 * (I - pp)
        return lam, I + pp, pp

    def solve(self, X, p, F, Mt):
        """Legendre coefficients a [M][N][3] (n = 1..N) and the velocities
        dx/dt [M][3], dp/dt [M][3] of the configuration."""
        X, p, F, Mt = (np.asarray(v, dtype=np.float64).reshape(-1, 3) for v in (X, p, F, Mt))
        M, N, l = X.shape[0], self.N, self.l
        th = np.zeros((M, M, N + 1, N + 1, 3, 3))
        for m in range(M):
            for k in range(M):
                if k != m:
                    th[m, k] = theta_pair(X[m], p[m], X[k], p[k], l, self.r, N, self.nq)
        c = (2.0 * np.arange(N + 1) + 1.0) / (2.0 * l)
        nu = 3 * M * N
        A = np.zeros((nu, nu))
        b = np.zeros(nu)

        def row(m, n):       # n = 1..N
            return 3 * (m * N + n - 1)

        for m in range(M):
            lam, K, pp = self._blocks(p[m])
            P = np.eye(3) - pp
            for n in range(1, N + 1):
                i = row(m, n)
                # interaction terms c_n sum_m' sum_k Theta^{n,k} a^k, known part from F
                coup = np.zeros((3, 3 * M * N))
                known = np.zeros(3)
                for k2 in range(M):
                    if k2 == m:
                        continue
                    known += th[m, k2, n, 0] @ F[k2] / (2.0 * l)
                    for kk in range(1, N + 1):
                        coup[:, row(k2, kk):row(k2, kk) + 3] += th[m, k2, n, kk]
                if n >= 2:
                    A[i:i + 3, i:i + 3] += lam + self.Ln[n] * K
                    A[i:i + 3, :] += c[n] * coup
                    b[i:i + 3] = -c[n] * known
                else:
                    A[i:i + 3, i:i + 3] += P + pp @ (lam + self.Ln[1] * K)
                    A[i:i + 3, :] += c[1] * pp @ coup
                    b[i:i + 3] = 3.0 / (2.0 * l * l) * np.cross(Mt[m], p[m]) - c[1] * pp @ known
        a = np.linalg.solve(A, b).reshape(M, N, 3) if nu else np.zeros((M, N, 3))
        # velocities from the n = 0 and n = 1 moments of U
        V = np.zeros((M, 3))
        W = np.zeros((M, 3))
        for m in range(M):
            lam, K, pp = self._blocks(p[m])
            I0 = np.zeros(3)
            I1 = np.zeros(3)
            for k2 in range(M):
                if k2 == m:
                    continue
                I0 += th[m, k2, 0, 0] @ F[k2] / (2.0 * l)
                I1 += th[m, k2, 1, 0] @ F[k2] / (2.0 * l)
                for kk in range(1, N + 1):
                    I0 += th[m, k2, 0, kk] @ a[k2, kk - 1]
                    I1 += th[m, k2, 1, kk] @ a[k2, kk - 1]
            V[m] = (lam @ F[m] + I0) / (8.0 * np.pi * self.mu * self.L)
            W[m] = 3.0 / (2.0 * np.pi * self.mu * self.L ** 3) * (
                self.d * np.cross(Mt[m], p[m]) + (np.eye(3) - pp) @ (l * I1))
        return a, V, W

    def run(self, X, p, F, Mt, dt, nsteps):
        """Adams-Bashforth 2 (Euler first step), p renormalised each step;
        returns the trajectory X [nsteps+1][M][3], p [nsteps+1][M][3]."""
        X = np.array(X, dtype=np.float64).reshape(-1, 3)
        p = np.array(p, dtype=np.float64).reshape(-1, 3)
        p /= np.linalg.norm(p, axis=1)[:, None]
        Xs, ps = [X.copy()], [p.copy()]
        prev = None
        for _ in range(nsteps):
            _, V, W = self.solve(X, p, F, Mt)
            if prev is None:
                X = X + dt * V
                p = p + dt * W
            else:
                X = X + dt * (1.5 * V - 0.5 * prev[0])
                p = p + dt * (1.5 * W - 0.5 * prev[1])
            p /= np.linalg.norm(p, axis=1)[:, None]
            prev = (V, W)
            Xs.append(X.copy())
            ps.append(p.copy())
        return np.array(Xs), np.array(ps)
