/*
 * lbm_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see the
 * header for what may load it).  Written for clarity, not speed: every step
 * follows the paper's equations in the paper's order and notation.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include "lbm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define HIST 19 /* doubles per fiber per recorded step: F3 M3 X3 q4 V3 W3 */

/* ------------------------------------------------------------------------ */
/* D3Q19 lattice (Sec. 4.1, Eq. SpeedOfSound and the weights after it).     */
/* The paper fixes only the weights: 1/3 for the rest velocity, 1/18 for    */
/* the six axis velocities, 1/36 for the twelve diagonals.  The order below */
/* (rest, +-x, +-y, +-z, then the xy, xz, yz diagonals, opposites adjacent) */
/* is this oracle's own choice; it only affects rounding order.             */
/* ------------------------------------------------------------------------ */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};
static const double W0 = 1.0 / 3.0, W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;

static double weight(int q) { return q == 0 ? W0 : (q <= 6 ? W1 : W2); }

/* Planted mistakes for the tests that show each pin can fail (0: none).   */
/* Every site computes the correct expression unchanged when the code is 0. */
static int g_mutation = 0;
void or_set_mutation(int code) { g_mutation = code; }

/* opposite direction: c_opp(q) = -c_q, found by search (no index tricks) */
static int opposite(int q)
{
    for (int p = 0; p < Q; ++p)
        if (CV[p][0] == -CV[q][0] && CV[p][1] == -CV[q][1] && CV[p][2] == -CV[q][2]) return p;
    return -1;
}

/* the direction with velocity e, found by search */
static int direction_of(const int e[3])
{
    for (int p = 0; p < Q; ++p)
        if (CV[p][0] == e[0] && CV[p][1] == e[1] && CV[p][2] == e[2]) return p;
    return -1;
}

void or_lattice(int32_t *c, double *w, int32_t *opp)
{
    for (int q = 0; q < Q; ++q) {
        for (int k = 0; k < 3; ++k) c[3 * q + k] = CV[q][k];
        w[q] = weight(q);
        opp[q] = opposite(q);
    }
}

/* He-Luo incompressible equilibrium (Eq. fequ_Incompr) with c_s^2 = 1/3:   */
/* f_eq = w [rho + rho0 (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)]                    */
void or_feq(double rho, double rho0, const double u[3], double *feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < Q; ++q) {
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        feq[q] = weight(q) * (rho + rho0 * (3.0 * cu + (g_mutation == 6 ? 3.0 : 4.5) * cu * cu - 1.5 * uu));
    }
}

/* odd relaxation rate from the TRT parameter Lambda:                        */
/* Lambda = (1/omega_e - 1/2)(1/omega_o - 1/2)  (Sec. 4.1; Lambda = 3/16 is   */
/* the value for which lambda_o = -8(2-omega)/(8-omega), i.e. walls exactly  */
/* half-way).  SRT uses omega_o = omega_e.                                   */
double or_omega_odd(double tau, double magic, int srt)
{
    if (srt) return 1.0 / tau;
    return 1.0 / (0.5 + magic / (tau - 0.5));
}

/* TRT collision of one cell (Eqs. TRTOp, EqPDF_TRT, LBMCollide).            */
/* lambda_e = -omega_e, lambda_o = -omega_o.  With a body force g the        */
/* velocity carries the half-force shift and the odd part receives           */
/* (1 - omega_o/2) 3 w rho0 c.g; the paper writes no forcing term, this is   */
/* the reading used for the Poiseuille and drag pins only.  ubar is the      */
/* momentum stabilization's shift (Sec. 4.1): the equilibrium is evaluated   */
/* at u - ubar; it is zero without stabilization.                            */
void or_collide_cell_shift(const double *f, double rho0, double omega_e, double omega_o,
                           const double g[3], const double ubar[3], double *fpost)
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < Q; ++q) {
        rho += f[q];
        for (int k = 0; k < 3; ++k) j[k] += CV[q][k] * f[q];
    }
    double u[3];
    for (int k = 0; k < 3; ++k)
        u[k] = g_mutation == 14 ? j[k] / rho0 + 0.5 * g[k] + ubar[k] : j[k] / rho0 + 0.5 * g[k] - ubar[k];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < Q; ++q) {
        int qb = opposite(q);
        double w = weight(q);
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        double cg = CV[q][0] * g[0] + CV[q][1] * g[1] + CV[q][2] * g[2];
        double feq_e = w * (rho - 1.5 * rho0 * uu + (g_mutation == 7 ? 0.0 : 4.5) * rho0 * cu * cu);
        double feq_o = w * 3.0 * rho0 * cu;
        double fe = 0.5 * (f[q] + f[qb]);
        double fo = 0.5 * (f[q] - f[qb]);
        fpost[q] = f[q] - omega_e * (fe - feq_e) - (g_mutation == 5 ? omega_e : omega_o) * (fo - feq_o)
                 + (1.0 - 0.5 * omega_o) * 3.0 * w * rho0 * cg;
    }
}

void or_collide_cell(const double *f, double rho0, double omega_e, double omega_o,
                     const double g[3], double *fpost)
{
    const double zero[3] = {0.0, 0.0, 0.0};
    or_collide_cell_shift(f, rho0, omega_e, omega_o, g, zero, fpost);
}

/* ------------------------------------------------------------------------ */
/* Geometry: fibers are circular cylinders of length L and radius r.  The   */
/* axis is t = R(q) e_x for the unit quaternion q = (w, x, y, z).  A cell   */
/* belongs to a particle when its centre lies inside it (Sec. 4.2).         */
/* All expressions are written so that no fused multiply-add is formed.     */
/* ------------------------------------------------------------------------ */
void or_fiber_axis(const double q[4], double t[3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    t[0] = 1.0 - 2.0 * (y * y + z * z);
    if (g_mutation == 17) {     /* the axis of the conjugate rotation */
        t[1] = 2.0 * (x * y - w * z);
        t[2] = 2.0 * (x * z + w * y);
        return;
    }
    t[1] = 2.0 * (x * y + w * z);
    t[2] = 2.0 * (x * z - w * y);
}

/* minimum-image component of a periodic difference */
static double min_image(double d, int n, int periodic)
{
    if (!periodic || g_mutation == 24) return d;
    double h = 0.5 * n;
    if (d > h) return d - n;
    if (d < -h) return d + n;
    return d;
}

/* Sec. 4.2: a cell belongs to the particle when its centre lies inside it.
   Cylinder of length L and radius r: the axial coordinate a = d.t obeys
   |a| <= L/2 and the squared distance from the axis q = |d|^2 - a^2 <= r^2.
   Spherocylinder (Sec. 2: L includes the hemispherical caps): the set of
   points within r of the axis segment of half-length L/2 - r; with
   e = |a| - (L/2 - r) the distance past the segment's end, q <= r^2 where
   e <= 0, else q + e^2 <= r^2 (squared distance to the cap centre). */
int or_cell_inside_shape(const double c[3], const double X[3], const double t[3], double length,
                         double radius, int shape, int nx, int ny, int nz, int zper)
{
    double dx = min_image(c[0] - X[0], nx, 1);
    double dy = min_image(c[1] - X[1], ny, 1);
    double dz = min_image(c[2] - X[2], nz, zper);
    double a = dx * t[0] + dy * t[1] + dz * t[2];
    double dd = dx * dx + dy * dy + dz * dz;
    double hl = 0.5 * length;
    double q = dd - a * a, r2 = radius * radius;
    if (shape == 1) {
        double e = fabs(a) - (g_mutation == 19 ? hl : hl - radius);
        if (e <= 0.0) return q <= r2;
        return q + e * e <= r2;
    }
    double hb = g_mutation == 16 ? length : hl;
    return (a * a <= hb * hb) && (q <= r2);
}

int or_cell_inside(const double c[3], const double X[3], const double t[3],
                   double length, double radius, int nx, int ny, int nz, int zper)
{
    return or_cell_inside_shape(c, X, t, length, radius, 0, nx, ny, nz, zper);
}

static int wrapi(int i, int n) { return ((i % n) + n) % n; }

/* map np particles onto a lattice: pid = lowest covering id, -1 = fluid.    */
/* Only cells within L/2 + r of the centre in each axis are tested; any     */
/* cell inside the cylinder satisfies |d|^2 <= (L/2)^2 + r^2 <= (L/2 + r)^2. */
void or_map(int nx, int ny, int nz, int zper, int np, const double *X, const double *q,
            const double *length, const double *radius, int32_t *pid, int64_t *overlaps)
{
    or_map_shapes(nx, ny, nz, zper, np, X, q, length, radius, NULL, pid, overlaps);
}

/* shape: per-particle shape codes (NULL: all cylinders).  The search box     */
/* L/2 + r around the centre contains both shapes.                           */
void or_map_shapes(int nx, int ny, int nz, int zper, int np, const double *X, const double *q,
                   const double *length, const double *radius, const int32_t *shape, int32_t *pid,
                   int64_t *overlaps)
{
    int64_t ncell = (int64_t)nx * ny * nz, ov = 0;
    for (int64_t i = 0; i < ncell; ++i) pid[i] = -1;
    for (int p = 0; p < np; ++p) {
        double t[3];
        or_fiber_axis(q + 4 * p, t);
        double ext = 0.5 * length[p] + radius[p];
        int lo[3], hi[3], n[3] = {nx, ny, nz};
        for (int k = 0; k < 3; ++k) {
            const double a = X[3 * p + k] - ext, b = X[3 * p + k] + ext;
            if (!(a > -1e6 && b < 1e6)) {
                /* a centre that is not finite or lies far off the lattice (a run
                   that has diverged): no integer box; scan the whole axis and let
                   the predicate decide */
                lo[k] = 0;
                hi[k] = n[k] - 1;
                continue;
            }
            lo[k] = (int)floor(a) - 1;
            hi[k] = (int)ceil(b) + 1;
            if (hi[k] - lo[k] + 1 > n[k]) { lo[k] = 0; hi[k] = n[k] - 1; }
        }
        int zp = zper;
        for (int kz = lo[2]; kz <= hi[2]; ++kz) {
            if (!zp && (kz < 0 || kz >= nz)) continue;
            int z = zp ? wrapi(kz, nz) : kz;
            for (int ky = lo[1]; ky <= hi[1]; ++ky) {
                int y = wrapi(ky, ny);
                for (int kx = lo[0]; kx <= hi[0]; ++kx) {
                    int x = wrapi(kx, nx);
                    double c[3] = {(double)x, (double)y, (double)z};
                    if (!or_cell_inside_shape(c, X + 3 * p, t, length[p], radius[p], shape ? shape[p] : 0,
                                              nx, ny, nz, zper))
                        continue;
                    int64_t idx = ((int64_t)z * ny + y) * nx + x;
                    if (pid[idx] < 0) pid[idx] = p;
                    else if (pid[idx] != p) {     /* claimed twice: lowest id keeps it */
                        ++ov;
                        if (g_mutation == 18) pid[idx] = p;
                    }
                }
            }
        }
    }
    if (overlaps) *overlaps = ov;
}

/* ------------------------------------------------------------------------ */
/* Rigid-body update (Sec. 4.3).  The paper does not state the integrator;  */
/* this oracle uses semi-implicit Euler with dt = 1:                        */
/*   V' = V + F/m,  X' = X + V' (periodic wrap),                            */
/*   Lang' = Lang + M (world-frame angular momentum),                       */
/*   W' = I(q)^-1 Lang'  with I(q)^-1 = 1/I_perp + (1/I_par - 1/I_perp) t t^T */
/*   q' = normalize(exp(W'/2) (x) q).                                       */
/* ------------------------------------------------------------------------ */
/* Planted mistakes for the tests that show each pin can fail (0: none).     */
/* Only the pins' own tests set this; every other caller leaves it at 0.    */

static void quat_mul(const double a[4], const double b[4], double out[4])
{
    double r[4];
    r[0] = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
    r[1] = a[0] * b[1] + b[0] * a[1] + (a[2] * b[3] - a[3] * b[2]);
    r[2] = a[0] * b[2] + b[0] * a[2] + (a[3] * b[1] - a[1] * b[3]);
    r[3] = a[0] * b[3] + b[0] * a[3] + (a[1] * b[2] - a[2] * b[1]);
    memcpy(out, r, sizeof r);
}

static double wrap_pos(double x, int n, int periodic)
{
    if (!periodic) return x;
    if (x >= n) return x - n;
    if (x < 0.0) return x + n;
    return x;
}

void or_rigid_step(const double *s, double mass, double i_par, double i_perp,
                   const double F[3], const double M[3], int nx, int ny, int nz, int zper,
                   double *out)
{
    const double *X = s, *q = s + 3, *V = s + 7, *La = s + 13;
    double t[3];
    or_fiber_axis(q, t);
    double Vn[3], Xn[3], Ln[3], Wn[3];
    int n[3] = {nx, ny, nz}, per[3] = {1, 1, zper};
    for (int k = 0; k < 3; ++k) {
        Vn[k] = V[k] + F[k] / mass;
        Xn[k] = wrap_pos(X[k] + (g_mutation == 20 ? V[k] : Vn[k]), n[k], per[k]);
        Ln[k] = La[k] + M[k];
    }
    double tl = t[0] * Ln[0] + t[1] * Ln[1] + t[2] * Ln[2];
    const double ia = g_mutation == 21 ? i_perp : i_par, ie = g_mutation == 21 ? i_par : i_perp;
    for (int k = 0; k < 3; ++k) Wn[k] = Ln[k] / ie + (1.0 / ia - 1.0 / ie) * tl * t[k];
    double ang = sqrt(Wn[0] * Wn[0] + Wn[1] * Wn[1] + Wn[2] * Wn[2]);
    double dq[4] = {1.0, 0.0, 0.0, 0.0};
    if (ang > 0.0) {
        double sh = sin(0.5 * ang) / ang;
        dq[0] = cos(0.5 * ang);
        dq[1] = sh * Wn[0];
        dq[2] = sh * Wn[1];
        dq[3] = sh * Wn[2];
    }
    double qn[4];
    quat_mul(dq, q, qn);
    double nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int k = 0; k < 4; ++k) qn[k] /= nrm;
    memcpy(out, Xn, sizeof Xn);
    memcpy(out + 3, qn, sizeof qn);
    memcpy(out + 7, Vn, sizeof Vn);
    memcpy(out + 10, Wn, sizeof Wn);
    memcpy(out + 13, Ln, sizeof Ln);
}

/* Solve the 6x6 system K x = b by Gaussian elimination with partial pivoting. */
static void solve6(double K[6][6], double b[6], double x[6])
{
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        for (int r = col + 1; r < 6; ++r)
            if (fabs(K[r][col]) > fabs(K[piv][col])) piv = r;
        if (piv != col) {
            for (int c = 0; c < 6; ++c) { double t = K[col][c]; K[col][c] = K[piv][c]; K[piv][c] = t; }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < 6; ++r) {
            double fct = K[r][col] / K[col][col];
            for (int c = col; c < 6; ++c) K[r][c] -= fct * K[col][c];
            b[r] -= fct * b[col];
        }
    }
    for (int r = 5; r >= 0; --r) {
        double acc = b[r];
        for (int c = r + 1; c < 6; ++c) acc -= K[r][c] * x[c];
        x[r] = acc / K[r][r];
    }
}

/* Implicit velocity update: the part of the momentum-exchange force that is  */
/* linear in the surface velocity u_s = V + W x r is evaluated at the new     */
/* velocities, giving the linear system                                      */
/*   (m I + A) V' + B W'           = m V + F0                                */
/*   B^T V'       + (I(q) + C) W'  = Lang + M0                               */
/* after which X, Lang and q advance as in the explicit step.                */
/* With a constant external load Fe, Me (Eq. ForceDensDiff for the weight):  */
/* it joins the right-hand side, m V + F0 + Fe and Lang + M0 + Me, and the    */
/* angular momentum update, Lang' = Lang + M + Me; Fap, Map stay the          */
/* hydrodynamic force and torque.                                             */
static void rigid_implicit(const double *s, double mass, double i_par, double i_perp,
                           const double F0[3], const double M0[3], const double *A,
                           const double *B, const double *Cm, const double Fe[3],
                           const double Me[3], int nx, int ny, int nz, int zper, double *out,
                           double *Fap, double *Map);

void or_rigid_step_implicit(const double *s, double mass, double i_par, double i_perp,
                            const double F0[3], const double M0[3], const double *A,
                            const double *B, const double *Cm, int nx, int ny, int nz,
                            int zper, double *out, double *Fap, double *Map)
{
    const double zero[3] = {0.0, 0.0, 0.0};
    rigid_implicit(s, mass, i_par, i_perp, F0, M0, A, B, Cm, zero, zero, nx, ny, nz, zper, out, Fap,
                   Map);
}

static void rigid_implicit(const double *s, double mass, double i_par, double i_perp,
                           const double F0[3], const double M0[3], const double *A,
                           const double *B, const double *Cm, const double Fe[3],
                           const double Me[3], int nx, int ny, int nz, int zper, double *out,
                           double *Fap, double *Map)
{
    const double *X = s, *q = s + 3, *V = s + 7, *La = s + 13;
    double t[3];
    or_fiber_axis(q, t);
    double K[6][6], b[6], x[6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double Iw = (i == j ? i_perp : 0.0) + (i_par - i_perp) * t[i] * t[j];
            K[i][j] = (i == j ? mass : 0.0) + A[3 * i + j];
            K[i][3 + j] = B[3 * i + j];
            K[3 + i][j] = g_mutation == 1 ? B[3 * i + j] : B[3 * j + i];
            K[3 + i][3 + j] = Iw + (g_mutation == 2 ? -Cm[3 * i + j] : Cm[3 * i + j]);
        }
    for (int i = 0; i < 3; ++i) {
        b[i] = mass * V[i] + F0[i] + Fe[i];
        b[3 + i] = La[i] + M0[i] + Me[i];
    }
    solve6(K, b, x);
    double Vn[3] = {x[0], x[1], x[2]}, Wn[3] = {x[3], x[4], x[5]};
    for (int i = 0; i < 3; ++i) {
        double fa = F0[i], ma = M0[i];
        for (int j = 0; j < 3; ++j) {
            fa -= A[3 * i + j] * Vn[j] + B[3 * i + j] * Wn[j];
            ma -= B[3 * j + i] * Vn[j] + Cm[3 * i + j] * Wn[j];
        }
        Fap[i] = fa;
        Map[i] = ma;
    }
    int n[3] = {nx, ny, nz}, per[3] = {1, 1, zper};
    double Xn[3], Ln[3];
    for (int k = 0; k < 3; ++k) {
        Xn[k] = wrap_pos(X[k] + Vn[k], n[k], per[k]);
        Ln[k] = La[k] + Map[k] + Me[k];
    }
    double ang = sqrt(Wn[0] * Wn[0] + Wn[1] * Wn[1] + Wn[2] * Wn[2]);
    double dq[4] = {1.0, 0.0, 0.0, 0.0};
    if (ang > 0.0) {
        double sh = sin(0.5 * ang) / ang;
        dq[0] = cos(0.5 * ang);
        dq[1] = sh * Wn[0];
        dq[2] = sh * Wn[1];
        dq[3] = sh * Wn[2];
    }
    double qn[4];
    quat_mul(dq, q, qn);
    double nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int k = 0; k < 4; ++k) qn[k] /= nrm;
    memcpy(out, Xn, sizeof Xn);
    memcpy(out + 3, qn, sizeof qn);
    memcpy(out + 7, Vn, sizeof Vn);
    memcpy(out + 10, Wn, sizeof Wn);
    memcpy(out + 13, Ln, sizeof Ln);
}

/* ------------------------------------------------------------------------ */
/* Contact between fibers.  The paper's rigid-body engine resolves          */
/* frictional collisions of the particles (Sec. 4.4); this oracle uses a    */
/* short-range repulsion instead (this project's reading): each fiber is a  */
/* segment of its axis swept by its radius (rounded ends), and when the gap */
/* between two such bodies falls below the range xi, a force               */
/* K ((xi - gap)/xi)^2 pushes them apart along the line of their closest    */
/* axis points, applied at the middle of the gap.                           */
/* ------------------------------------------------------------------------ */
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

double or_segment_closest(const double Xp[3], const double tp[3], double hp, const double Xq[3],
                          const double tq[3], double hq, double *s_out, double *u_out)
{
    /* minimise |d + u tq - s tp|^2, d = Xq - Xp, over the two intervals */
    double d[3] = {Xq[0] - Xp[0], Xq[1] - Xp[1], Xq[2] - Xp[2]};
    double b = tp[0] * tq[0] + tp[1] * tq[1] + tp[2] * tq[2];
    double e = d[0] * tp[0] + d[1] * tp[1] + d[2] * tp[2];
    double f = d[0] * tq[0] + d[1] * tq[1] + d[2] * tq[2];
    double den = 1.0 - b * b, s;
    if (den > 1e-12) {
        s = clampd((e - b * f) / den, -hp, hp);   /* free minimiser in s, clamped */
    } else {
        /* parallel: middle of the overlap of the second segment's projection */
        double lo = e - hq, hi = e + hq;
        if (lo < -hp) lo = -hp;
        if (hi > hp) hi = hp;
        s = lo <= hi ? 0.5 * (lo + hi) : clampd(e, -hp, hp);
    }
    double u = clampd(s * b - f, -hq, hq);
    s = clampd(e + u * b, -hp, hp);
    double w[3];
    for (int k = 0; k < 3; ++k) w[k] = d[k] + u * tq[k] - s * tp[k];
    *s_out = s;
    *u_out = u;
    return sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
}

double or_contact_pair(const double tp[3], double hp, double rp,
                       const double dpq[3], const double tq[3], double hq, double rq, double k,
                       double range, double Fp[3], double Mp[3], double Fq[3], double Mq[3])
{
    const double zero[3] = {0.0, 0.0, 0.0};
    double s, u;
    double dist = or_segment_closest(zero, tp, hp, dpq, tq, hq, &s, &u);
    double gap = dist - rp - rq;
    for (int i = 0; i < 3; ++i) Fp[i] = Mp[i] = Fq[i] = Mq[i] = 0.0;
    if (!(k > 0.0) || gap >= range || dist <= 0.0) return gap;
    double P[3], Qp[3], n[3];   /* closest axis points relative to X_p; n from p to q */
    for (int i = 0; i < 3; ++i) {
        P[i] = s * tp[i];
        Qp[i] = dpq[i] + u * tq[i];
        n[i] = (Qp[i] - P[i]) / dist;
    }
    double x = (range - gap) / range;
    double mag = k * x * x;
    double C[3];                 /* middle of the gap, relative to X_p */
    for (int i = 0; i < 3; ++i) {
        C[i] = P[i] + (rp + 0.5 * gap) * n[i];
        Fp[i] = g_mutation == 22 ? mag * n[i] : -mag * n[i];
        Fq[i] = g_mutation == 22 ? -mag * n[i] : mag * n[i];
    }
    double Cq[3] = {C[0] - dpq[0], C[1] - dpq[1], C[2] - dpq[2]};   /* relative to X_q */
    if (g_mutation == 23)
        for (int i = 0; i < 3; ++i) Cq[i] = C[i];  /* q's lever measured from X_p */
    Mp[0] = C[1] * Fp[2] - C[2] * Fp[1];
    Mp[1] = C[2] * Fp[0] - C[0] * Fp[2];
    Mp[2] = C[0] * Fp[1] - C[1] * Fp[0];
    Mq[0] = Cq[1] * Fq[2] - Cq[2] * Fq[1];
    Mq[1] = Cq[2] * Fq[0] - Cq[0] * Fq[2];
    Mq[2] = Cq[0] * Fq[1] - Cq[1] * Fq[0];
    return gap;
}

/* ------------------------------------------------------------------------ */
/* The coupled simulation                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double st[16];          /* X3 q4 V3 W3 Lang3 */
    double length, radius, mass, i_par, i_perp;
    int shape;              /* 0 cylinder, 1 spherocylinder */
    double fext[3], mext[3];/* constant external force and torque */
    double F[3], M[3];
    double F0p[3], M0p[3];  /* velocity-free sums of the previous step */
    int have_prev;
    double sums[39];        /* last step's momentum-exchange sums (see or_get_exchange_sums) */
    double corr[6];         /* closure correction dF, dM for the next step */
    int has_corr;
    double *traj;           /* prescribed kinematics, 13 per step, or NULL */
    int64_t traj_n, traj_pos;
} fiber;

struct or_sim {
    or_params p;
    double omega_e, omega_o;
    int64_t ncell;
    double *fa, *fb, *ft;   /* A, B, post-collision */
    uint8_t *flag;          /* 0 fluid, 1 particle */
    int32_t *pid;
    int nf, capf;
    fiber *fib;
    int64_t steps, overlaps;
    double *hist;           /* [steps][nf][HIST] */
    int64_t hist_cap;
};

static int64_t cidx(const or_sim *s, int x, int y, int z)
{
    return ((int64_t)z * s->p.ny + y) * s->p.nx + x;
}

static double *slot(double *f, const or_sim *s, int q, int64_t c) { return f + (int64_t)q * s->ncell + c; }

or_sim *or_create(const or_params *p)
{
    or_sim *s = (or_sim *)calloc(1, sizeof *s);
    if (!s) return NULL;
    s->p = *p;
    s->omega_e = 1.0 / p->tau;
    s->omega_o = or_omega_odd(p->tau, p->magic, p->srt);
    s->ncell = (int64_t)p->nx * p->ny * p->nz;
    size_t nf = (size_t)Q * s->ncell;
    s->fa = (double *)malloc(nf * sizeof(double));
    s->fb = (double *)malloc(nf * sizeof(double));
    s->ft = (double *)malloc(nf * sizeof(double));
    s->flag = (uint8_t *)calloc(s->ncell, 1);
    s->pid = (int32_t *)malloc(s->ncell * sizeof(int32_t));
    if (!s->fa || !s->fb || !s->ft || !s->flag || !s->pid) { or_destroy(s); return NULL; }
    for (int64_t i = 0; i < s->ncell; ++i) s->pid[i] = -1;
    /* initial state: f = f_eq(rho0, u0(z)) everywhere */
    for (int z = 0; z < p->nz; ++z) {
        double u[3] = {0.0, 0.0, 0.0}, feq[Q];
        if (p->init_couette && !p->z_periodic) u[0] = p->wall_u * (2.0 * (z + 0.5) / p->nz - 1.0);
        or_feq(p->rho0, p->rho0, u, feq);
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int q = 0; q < Q; ++q) *slot(s->fa, s, q, cidx(s, x, y, z)) = feq[q];
    }
    memcpy(s->fb, s->fa, nf * sizeof(double));
    return s;
}

void or_destroy(or_sim *s)
{
    if (!s) return;
    free(s->fa); free(s->fb); free(s->ft); free(s->flag); free(s->pid);
    for (int i = 0; i < s->nf; ++i) free(s->fib[i].traj);
    free(s->fib); free(s->hist);
    free(s);
}

/* remap all fibers with their current poses; returns overlaps counted */
static int64_t remap(or_sim *s, int32_t *pid_out)
{
    int np = s->nf;
    double *X = (double *)malloc((size_t)(3 * np + 4 * np + 2 * np + 1) * sizeof(double));
    double *q = X + 3 * np, *L = q + 4 * np, *r = L + np;
    int32_t *shape = (int32_t *)malloc((size_t)(np + 1) * sizeof(int32_t));
    for (int i = 0; i < np; ++i) {
        memcpy(X + 3 * i, s->fib[i].st, 3 * sizeof(double));
        memcpy(q + 4 * i, s->fib[i].st + 3, 4 * sizeof(double));
        L[i] = s->fib[i].length;
        r[i] = s->fib[i].radius;
        shape[i] = s->fib[i].shape;
    }
    int64_t ov = 0;
    or_map_shapes(s->p.nx, s->p.ny, s->p.nz, s->p.z_periodic, np, X, q, L, r, shape, pid_out, &ov);
    free(shape);
    free(X);
    return ov;
}

/* velocity of particle p's rigid motion at a cell centre c: V + W x d(c, X) */
static void surface_velocity(const or_sim *s, const double *st, int x, int y, int z, double us[3])
{
    const double *X = st, *V = st + 7, *W = st + 10;
    double d[3];
    d[0] = min_image(x - X[0], s->p.nx, 1);
    d[1] = min_image(y - X[1], s->p.ny, 1);
    d[2] = min_image(z - X[2], s->p.nz, s->p.z_periodic);
    us[0] = V[0] + (W[1] * d[2] - W[2] * d[1]);
    us[1] = V[1] + (W[2] * d[0] - W[0] * d[2]);
    us[2] = V[2] + (W[0] * d[1] - W[1] * d[0]);
}

/* Mass and principal moments of inertia (about the axis, and about a      */
/* transverse axis through the centre) of a homogeneous body of density rho. */
void or_body_inertia(int shape, double length, double radius, double rho, double out[3])
{
    if (shape == 1) {
        /* spherocylinder: a cylinder of length h = L - 2r and two hemispheres */
        /* (one sphere of mass ms).  Axial moment: mc r^2/2 + 2 ms r^2/5.      */
        /* Transverse: the cylinder's mc (3r^2 + h^2)/12; each hemisphere of  */
        /* mass ms/2 has (2/5)(ms/2) r^2 about a transverse axis through its  */
        /* flat face, its centroid 3r/8 from that face, which is h/2 from     */
        /* the centre: by the parallel-axis theorem the pair adds             */
        /* ms (2r^2/5 - 9r^2/64 + (h/2 + 3r/8)^2) = ms (2r^2/5 + h^2/4 + 3hr/8). */
        double h = length - 2.0 * radius;
        double mc = rho * M_PI * radius * radius * h;
        double ms = rho * (4.0 / 3.0) * M_PI * radius * radius * radius;
        out[0] = mc + ms;
        out[1] = mc * radius * radius / 2.0 + 2.0 * ms * radius * radius / 5.0;
        out[2] = g_mutation == 26 ? mc * (3.0 * radius * radius + h * h) / 12.0 + ms * (2.0 * radius * radius / 5.0)
                                  : mc * (3.0 * radius * radius + h * h) / 12.0 +
                                    ms * (2.0 * radius * radius / 5.0 + h * h / 4.0 + 3.0 * h * radius / 8.0);
    } else {
        double m = rho * M_PI * radius * radius * length;
        out[0] = m;
        out[1] = 0.5 * m * radius * radius;
        out[2] = m * (3.0 * radius * radius + length * length) / 12.0;
    }
}

int or_add_fiber(or_sim *s, const double X[3], const double q[4], double length, double radius,
                 double density_ratio, const double V[3], const double W[3])
{
    const double zero[3] = {0.0, 0.0, 0.0};
    return or_add_fiber_ex(s, X, q, length, radius, density_ratio, V, W, 0, zero, zero);
}

int or_add_fiber_ex(or_sim *s, const double X[3], const double q[4], double length, double radius,
                    double density_ratio, const double V[3], const double W[3], int shape,
                    const double Fext[3], const double Mext[3])
{
    if (shape != 0 && shape != 1) return -1;
    if (shape == 1 && !(length >= 2.0 * radius)) return -1;
    if (s->steps != 0) return -1;
    if (s->nf == s->capf) {
        int nc = s->capf ? 2 * s->capf : 8;
        fiber *nfib = (fiber *)realloc(s->fib, nc * sizeof(fiber));
        if (!nfib) return -1;
        s->fib = nfib;
        s->capf = nc;
    }
    fiber *f = &s->fib[s->nf];
    memset(f, 0, sizeof *f);
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 3; ++k) f->st[k] = X[k];
    for (int k = 0; k < 4; ++k) f->st[3 + k] = q[k] / qn;
    for (int k = 0; k < 3; ++k) f->st[7 + k] = V[k];
    for (int k = 0; k < 3; ++k) f->st[10 + k] = W[k];
    f->length = length;
    f->radius = radius;
    f->shape = shape;
    for (int k = 0; k < 3; ++k) {
        f->fext[k] = Fext[k];
        f->mext[k] = Mext[k];
    }
    /* mass and inertia from the geometric body, not the cell count */
    double mi[3];
    or_body_inertia(shape, length, radius, density_ratio * s->p.rho0, mi);
    f->mass = mi[0];
    f->i_par = mi[1];
    f->i_perp = mi[2];
    double t[3];
    or_fiber_axis(f->st + 3, t);
    double tw = t[0] * W[0] + t[1] * W[1] + t[2] * W[2];
    for (int k = 0; k < 3; ++k) f->st[13 + k] = f->i_perp * W[k] + (f->i_par - f->i_perp) * tw * t[k];
    s->nf++;
    int64_t ov = remap(s, s->pid);
    if (ov > 0) { /* reject a fiber that overlaps another one */
        s->nf--;
        remap(s, s->pid);
    }
    for (int64_t i = 0; i < s->ncell; ++i) s->flag[i] = s->pid[i] >= 0;
    return (ov > 0) ? -2 : s->nf - 1;
}

int or_set_correction(or_sim *s, int id, const double dF[3], const double dM[3])
{
    if (id < 0 || id >= s->nf) return -1;
    fiber *f = &s->fib[id];
    for (int k = 0; k < 3; ++k) {
        f->corr[k] = dF[k];
        f->corr[3 + k] = dM[k];
    }
    f->has_corr = 1;
    return 0;
}

int or_set_kinematics(or_sim *s, int id, const double *traj, int64_t nsteps)
{
    if (id < 0 || id >= s->nf || nsteps < 0) return -1;
    fiber *f = &s->fib[id];
    free(f->traj);
    f->traj = NULL;
    f->traj_n = f->traj_pos = 0;
    if (nsteps == 0) return 0;
    f->traj = (double *)malloc((size_t)nsteps * 13 * sizeof(double));
    memcpy(f->traj, traj, (size_t)nsteps * 13 * sizeof(double));
    f->traj_n = nsteps;
    return 0;
}

static void record(or_sim *s)
{
    int64_t need = (s->steps + 1) * s->nf * HIST;
    if (need > s->hist_cap) {
        int64_t nc = s->hist_cap ? 2 * s->hist_cap : 1024 * HIST;
        while (nc < need) nc *= 2;
        s->hist = (double *)realloc(s->hist, (size_t)nc * sizeof(double));
        s->hist_cap = nc;
    }
    double *h = s->hist + s->steps * s->nf * HIST;
    for (int i = 0; i < s->nf; ++i) {
        fiber *f = &s->fib[i];
        double *r = h + i * HIST;
        memcpy(r, f->F, 3 * sizeof(double));
        memcpy(r + 3, f->M, 3 * sizeof(double));
        memcpy(r + 6, f->st, 13 * sizeof(double)); /* X q V W */
    }
}

int64_t or_mean_velocity(const or_sim *s, double ubar[3])
{
    const or_params *p = &s->p;
    const int ny = p->ny, nz = p->nz;
    /* per-plane partial sums, then added over z in order (thread-count independent) */
    double *part = (double *)calloc((size_t)nz * 4, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t c = cidx(s, x, y, z);
                if (s->flag[c]) {
                    if (g_mutation == 25) part[4 * z + 3] += 1.0;   /* solid cells counted */
                    continue;
                }
                double *a = part + 4 * z;
                for (int q = 0; q < Q; ++q) {
                    double fq = *slot(s->fa, s, q, c);
                    for (int k = 0; k < 3; ++k) a[k] += CV[q][k] * fq;
                }
                a[3] += 1.0;
            }
    double j[3] = {0.0, 0.0, 0.0}, n = 0.0;
    for (int z = 0; z < nz; ++z) {
        for (int k = 0; k < 3; ++k) j[k] += part[4 * z + k];
        n += part[4 * z + 3];
    }
    free(part);
    for (int k = 0; k < 3; ++k) ubar[k] = n > 0.0 ? j[k] / (n * p->rho0) + 0.5 * p->g[k] : 0.0;
    return (int64_t)n;
}

static void one_step(or_sim *s)
{
    const or_params *p = &s->p;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const double rho0 = p->rho0;

    /* 0. momentum stabilization (Sec. 4.1): the mean fluid velocity of the */
    /*    current state, subtracted in every cell's equilibrium below.      */
    double ubar[3] = {0.0, 0.0, 0.0};
    if (p->stabilize) or_mean_velocity(s, ubar);

    /* 1. collide every fluid cell: fa -> ft */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < s->ncell; ++c) {
        if (s->flag[c]) continue;
        double f[Q], fp[Q];
        for (int q = 0; q < Q; ++q) f[q] = *slot(s->fa, s, q, c);
        or_collide_cell_shift(f, rho0, s->omega_e, s->omega_o, p->g, ubar, fp);
        for (int q = 0; q < Q; ++q) *slot(s->ft, s, q, c) = fp[q];
    }

    /* 2. stream ft -> fb with bounce-back at walls and particle surfaces     */
    /*    (Eqs. LBMStream, BBBC, LBMMovWall); every slot of fb is written by  */
    /*    exactly one fluid cell, so the z-loop can run in parallel.          */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t c = cidx(s, x, y, z);
                if (s->flag[c]) continue;
                *slot(s->fb, s, 0, c) = *slot(s->ft, s, 0, c);
                for (int q = 1; q < Q; ++q) {
                    int qb = opposite(q);
                    double w = weight(q);
                    double ft = *slot(s->ft, s, q, c);
                    int yx = wrapi(x + CV[q][0], nx), yy = wrapi(y + CV[q][1], ny);
                    int yz = z + CV[q][2];
                    /* walls the link crosses */
                    int wx = p->x_walls && (x + CV[q][0] < 0 || x + CV[q][0] >= nx);
                    int wy = p->y_walls && (y + CV[q][1] < 0 || y + CV[q][1] >= ny);
                    int wz = !p->z_periodic && (yz < 0 || yz >= nz);
                    if (wz && !p->z_free_slip) {
                        /* moving wall, half-way: bottom -U, top +U along x */
                        double uw = (yz < 0) ? -p->wall_u : p->wall_u;
                        double mw = 6.0 * w * rho0 * (CV[q][0] * uw);
                        *slot(s->fb, s, qb, c) = g_mutation == 8 ? ft + mw : ft - mw;
                        continue;
                    }
                    if ((wx && p->x_walls == 1) || (wy && p->y_walls == 1)) {
                        /* resting no-slip wall in x or y, half-way (Eq. BBBC) */
                        *slot(s->fb, s, g_mutation == 15 ? q : qb, c) = ft;
                        continue;
                    }
                    if (wx || wy || wz) {
                        /* free-slip walls only (Eq. FreeSlipBC): the normal components
                           of the crossed walls reverse, the population lands on the
                           neighbour along the remaining components */
                        int e[3] = {wx ? -CV[q][0] : CV[q][0], wy ? -CV[q][1] : CV[q][1],
                                    wz ? -CV[q][2] : CV[q][2]};
                        int qr = g_mutation == 12 ? qb : direction_of(e);
                        int dx = wx ? x : yx, dy = wy ? y : yy, dz = wz ? z : wrapi(yz, nz);
                        *slot(s->fb, s, qr, cidx(s, dx, dy, dz)) = ft;
                        continue;
                    }
                    yz = wrapi(yz, nz);
                    int64_t cy = cidx(s, yx, yy, yz);
                    if (s->flag[cy]) {
                        double us[3];
                        surface_velocity(s, s->fib[s->pid[cy]].st, yx, yy, yz, us);
                        double cu = CV[q][0] * us[0] + CV[q][1] * us[1] + CV[q][2] * us[2];
                        *slot(s->fb, s, qb, c) = g_mutation == 9 ? ft : ft - 6.0 * w * rho0 * cu;
                    } else {
                        *slot(s->fb, s, q, cy) = ft;
                    }
                }
            }

    /* 2b. momentum exchange (Eq. LBMhydrodynForce).  Partial sums per      */
    /*     z-plane, then added over z in order, so the result does not       */
    /*     depend on the thread count.  Lever arm from the centre of mass to */
    /*     the solid cell centre x_s; the torque is (x_s - x_C) x dF (the    */
    /*     cross product written with the other operand order has the        */
    /*     opposite sign).                                                   */
    int nfb = s->nf;
    /* per (z, fiber): F3 M3 (direct), F0 3, M0 3, A 9, B 9, C 9 */
    double *part = (double *)calloc((size_t)nz * (nfb ? nfb : 1) * 39, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t c = cidx(s, x, y, z);
                if (s->flag[c] || nfb == 0) continue;
                for (int q = 1; q < Q; ++q) {
                    int yz = z + CV[q][2];
                    if (!p->z_periodic && (yz < 0 || yz >= nz)) continue;
                    if ((p->x_walls && (x + CV[q][0] < 0 || x + CV[q][0] >= nx)) ||
                        (p->y_walls && (y + CV[q][1] < 0 || y + CV[q][1] >= ny)))
                        continue;
                    int yx = wrapi(x + CV[q][0], nx), yy = wrapi(y + CV[q][1], ny);
                    yz = wrapi(yz, nz);
                    int64_t cy = cidx(s, yx, yy, yz);
                    if (!s->flag[cy]) continue;
                    int ip = s->pid[cy];
                    const fiber *f = &s->fib[ip];
                    double us[3];
                    surface_velocity(s, f->st, yx, yy, yz, us);
                    double cu = CV[q][0] * us[0] + CV[q][1] * us[1] + CV[q][2] * us[2];
                    double ftq = *slot(s->ft, s, q, c);
                    double mag = (g_mutation == 10 ? 1.0 : 2.0) * ftq - 6.0 * weight(q) * rho0 * cu;
                    double dF[3] = {mag * CV[q][0], mag * CV[q][1], mag * CV[q][2]};
                    double r[3];
                    r[0] = min_image(yx - f->st[0], nx, 1);
                    r[1] = min_image(yy - f->st[1], ny, 1);
                    r[2] = min_image(yz - f->st[2], nz, p->z_periodic);
                    double *acc = part + ((size_t)z * nfb + ip) * 39;
                    /* direct formula, every term at the old velocity */
                    for (int k = 0; k < 3; ++k) acc[k] += dF[k];
                    if (g_mutation == 11) {
                        acc[3] += dF[1] * r[2] - dF[2] * r[1];
                        acc[4] += dF[2] * r[0] - dF[0] * r[2];
                        acc[5] += dF[0] * r[1] - dF[1] * r[0];
                    } else {
                        acc[3] += r[1] * dF[2] - r[2] * dF[1];
                        acc[4] += r[2] * dF[0] - r[0] * dF[2];
                        acc[5] += r[0] * dF[1] - r[1] * dF[0];
                    }
                    /* split for the implicit update: velocity-free part and the  */
                    /* matrices of the part linear in u_s = V + W x r            */
                    double m0 = 2.0 * ftq;
                    double cq[3] = {(double)CV[q][0], (double)CV[q][1], (double)CV[q][2]};
                    double rc[3] = {r[1] * cq[2] - r[2] * cq[1], r[2] * cq[0] - r[0] * cq[2],
                                    r[0] * cq[1] - r[1] * cq[0]};
                    double k6 = 6.0 * weight(q) * rho0;
                    for (int k = 0; k < 3; ++k) {
                        acc[6 + k] += m0 * cq[k];
                        acc[9 + k] += m0 * rc[k];
                    }
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) {
                            acc[12 + 3 * i + j] += k6 * cq[i] * cq[j];
                            acc[21 + 3 * i + j] += g_mutation == 3 ? k6 * rc[i] * cq[j]
                                                                   : k6 * cq[i] * rc[j];
                            acc[30 + 3 * i + j] += k6 * rc[i] * rc[j];
                        }
                }
            }
    double *red = (double *)calloc((size_t)(nfb ? nfb : 1) * 39, sizeof(double));
    for (int i = 0; i < nfb; ++i)
        for (int z = 0; z < nz; ++z) {
            const double *acc = part + ((size_t)z * nfb + i) * 39;
            for (int k = 0; k < 39; ++k) red[39 * i + k] += acc[k];
        }
    free(part);

    /* 3. rigid-body update; keep the old states for the refill.  With      */
    /*    coupling 0 the velocity-free sums F0, M0 enter as the mean of this   */
    /*    step's and the previous step's values: the plain sums let the        */
    /*    torque build a growing oscillation of period two steps at density    */
    /*    ratio 1 and small tau, which the mean removes.                       */
    /* 2c. contact loads of every pair at the current poses (zero when the */
    /*     repulsion is off), added to the external load of this step      */
    double *cl = (double *)calloc((size_t)(s->nf ? s->nf : 1) * 6, sizeof(double));
    if (p->contact_k > 0.0)
        for (int i = 0; i < s->nf; ++i)
            for (int j = i + 1; j < s->nf; ++j) {
                const fiber *a = &s->fib[i], *b = &s->fib[j];
                double ta[3], tb[3], d[3], Fa[3], Ma[3], Fb[3], Mb[3];
                or_fiber_axis(a->st + 3, ta);
                or_fiber_axis(b->st + 3, tb);
                d[0] = min_image(b->st[0] - a->st[0], nx, 1);
                d[1] = min_image(b->st[1] - a->st[1], ny, 1);
                d[2] = min_image(b->st[2] - a->st[2], nz, p->z_periodic);
                double ha = 0.5 * a->length - a->radius, hb = 0.5 * b->length - b->radius;
                or_contact_pair(ta, ha > 0.0 ? ha : 0.0, a->radius, d, tb, hb > 0.0 ? hb : 0.0,
                                b->radius, p->contact_k, p->contact_range, Fa, Ma, Fb, Mb);
                for (int k = 0; k < 3; ++k) {
                    cl[6 * i + k] += Fa[k];
                    cl[6 * i + 3 + k] += Ma[k];
                    cl[6 * j + k] += Fb[k];
                    cl[6 * j + 3 + k] += Mb[k];
                }
            }

    double *old = (double *)malloc((size_t)(s->nf ? s->nf : 1) * 16 * sizeof(double));
    for (int i = 0; i < s->nf; ++i) {
        fiber *f = &s->fib[i];
        const double *rd = red + 39 * i;
        double fe[3], me[3];   /* external plus contact load */
        for (int k = 0; k < 3; ++k) {
            fe[k] = (g_mutation == 27 ? 0.0 : f->fext[k]) + cl[6 * i + k];
            me[k] = (g_mutation == 28 ? 0.0 : f->mext[k]) + cl[6 * i + 3 + k];
        }
        memcpy(old + 16 * i, f->st, 16 * sizeof(double));
        memcpy(f->sums, rd, 39 * sizeof(double));
        /* closure correction of this step (zero when none was set) */
        double cF[3] = {0.0, 0.0, 0.0}, cM[3] = {0.0, 0.0, 0.0};
        if (f->has_corr)
            for (int k = 0; k < 3; ++k) {
                cF[k] = f->corr[k];
                cM[k] = f->corr[3 + k];
            }
        if (f->traj && f->traj_pos < f->traj_n) {
            /* prescribed motion: the force reported is the direct formula */
            for (int k = 0; k < 3; ++k) {
                f->F[k] = f->has_corr ? rd[k] + cF[k] : rd[k];
                f->M[k] = f->has_corr ? rd[3 + k] + cM[k] : rd[3 + k];
            }
            const double *tr = f->traj + 13 * f->traj_pos++;
            memcpy(f->st, tr, 13 * sizeof(double));
            double t[3];
            or_fiber_axis(f->st + 3, t);
            const double *Wp = f->st + 10;
            double tw = t[0] * Wp[0] + t[1] * Wp[1] + t[2] * Wp[2];
            for (int k = 0; k < 3; ++k)
                f->st[13 + k] = f->i_perp * Wp[k] + (f->i_par - f->i_perp) * tw * t[k];
        } else if (p->coupling != 1) {
            double F0u[3], M0u[3];
            for (int k = 0; k < 3; ++k) {
                const int avg = p->coupling == 0 && f->have_prev;
                const double h = g_mutation == 4 ? 1.0 : 0.5;
                F0u[k] = avg ? h * (rd[6 + k] + f->F0p[k]) : rd[6 + k];
                M0u[k] = avg ? h * (rd[9 + k] + f->M0p[k]) : rd[9 + k];
                if (f->has_corr) {
                    F0u[k] += cF[k];
                    M0u[k] += cM[k];
                }
            }
            double out[16];
            rigid_implicit(f->st, f->mass, f->i_par, f->i_perp, F0u, M0u, rd + 12, rd + 21, rd + 30,
                           fe, me, nx, ny, nz, p->z_periodic, out, f->F, f->M);
            memcpy(f->st, out, 16 * sizeof(double));
        } else {
            for (int k = 0; k < 3; ++k) {
                f->F[k] = f->has_corr ? rd[k] + cF[k] : rd[k];
                f->M[k] = f->has_corr ? rd[3 + k] + cM[k] : rd[3 + k];
            }
            double out[16], Ft[3], Mt[3];
            for (int k = 0; k < 3; ++k) {   /* with the external and contact load */
                Ft[k] = f->F[k] + fe[k];
                Mt[k] = f->M[k] + me[k];
            }
            or_rigid_step(f->st, f->mass, f->i_par, f->i_perp, Ft, Mt, nx, ny, nz, p->z_periodic,
                          out);
            memcpy(f->st, out, 16 * sizeof(double));
        }
        for (int k = 0; k < 3; ++k) {
            f->F0p[k] = rd[6 + k];
            f->M0p[k] = rd[9 + k];
        }
        f->have_prev = 1;
        f->has_corr = 0;
    }
    free(red);
    free(cl);

    /* 4. remap with the new poses; refill uncovered cells with             */
    /*    f_eq(rho0, u_s) of the old owner's previous-step motion.          */
    if (s->nf > 0) {
        int32_t *pn = (int32_t *)malloc(s->ncell * sizeof(int32_t));
        s->overlaps += remap(s, pn);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    int64_t c = cidx(s, x, y, z);
                    int po = s->pid[c];
                    if (po >= 0 && pn[c] < 0) {
                        double us[3], feq[Q];
                        surface_velocity(s, g_mutation == 13 ? s->fib[po].st : old + 16 * po, x, y, z, us);
                        or_feq(rho0, rho0, us, feq);
                        for (int q = 0; q < Q; ++q) *slot(s->fb, s, q, c) = feq[q];
                    }
                    s->pid[c] = pn[c];
                    s->flag[c] = pn[c] >= 0;
                }
        free(pn);
    }
    free(old);

    /* 5. swap lattices, record the step */
    double *tmp = s->fa;
    s->fa = s->fb;
    s->fb = tmp;
    record(s);
    s->steps++;
}

void or_step(or_sim *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) one_step(s);
}

void or_get_populations(const or_sim *s, double *f)
{
    memcpy(f, s->fa, (size_t)Q * s->ncell * sizeof(double));
}

void or_set_populations(or_sim *s, const double *f)
{
    memcpy(s->fa, f, (size_t)Q * s->ncell * sizeof(double));
}

void or_get_fields(const or_sim *s, double *rho, double *u, uint8_t *flags, int32_t *pid)
{
    const or_params *p = &s->p;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t c = cidx(s, x, y, z);
                double r = 0.0, j[3] = {0.0, 0.0, 0.0}, uc[3];
                if (s->flag[c]) {
                    r = p->rho0;
                    surface_velocity(s, s->fib[s->pid[c]].st, x, y, z, uc);
                } else {
                    for (int q = 0; q < Q; ++q) {
                        double fq = s->fa[(int64_t)q * s->ncell + c];
                        r += fq;
                        for (int k = 0; k < 3; ++k) j[k] += CV[q][k] * fq;
                    }
                    for (int k = 0; k < 3; ++k) uc[k] = j[k] / p->rho0 + 0.5 * p->g[k];
                }
                if (rho) rho[c] = r;
                if (u)
                    for (int k = 0; k < 3; ++k) u[(int64_t)k * s->ncell + c] = uc[k];
                if (flags) flags[c] = s->flag[c];
                if (pid) pid[c] = s->pid[c];
            }
}

void or_get_fiber_state(const or_sim *s, double *X, double *q, double *V, double *W)
{
    for (int i = 0; i < s->nf; ++i) {
        const double *st = s->fib[i].st;
        if (X) memcpy(X + 3 * i, st, 3 * sizeof(double));
        if (q) memcpy(q + 4 * i, st + 3, 4 * sizeof(double));
        if (V) memcpy(V + 3 * i, st + 7, 3 * sizeof(double));
        if (W) memcpy(W + 3 * i, st + 10, 3 * sizeof(double));
    }
}

void or_get_force_torque(const or_sim *s, double *F, double *M)
{
    for (int i = 0; i < s->nf; ++i) {
        if (F) memcpy(F + 3 * i, s->fib[i].F, 3 * sizeof(double));
        if (M) memcpy(M + 3 * i, s->fib[i].M, 3 * sizeof(double));
    }
}

int64_t or_get_history(const or_sim *s, int64_t first, int64_t count, double *out)
{
    if (first < 0 || first >= s->steps) return 0;
    if (first + count > s->steps) count = s->steps - first;
    memcpy(out, s->hist + first * s->nf * HIST, (size_t)(count * s->nf * HIST) * sizeof(double));
    return count;
}

int64_t or_overlaps(const or_sim *s) { return s->overlaps; }

void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }

void or_get_exchange_sums(const or_sim *s, double *out)
{
    for (int i = 0; i < s->nf; ++i) memcpy(out + 39 * i, s->fib[i].sums, 39 * sizeof(double));
}
int64_t or_steps_done(const or_sim *s) { return s->steps; }
int or_nfibers(const or_sim *s) { return s->nf; }
