// lbm_particle_dev.h -- FP64 device functions of the fibers shared by the
// single-lattice kernels (particles.hip) and the batched kernel
// (batched.hip): the cell predicate, boxes and per-plane rectangles, the
// rigid-body update and the refill store.
#pragma once
#include "lbm_dev.h"

namespace lbm {

#pragma clang fp contract(off)

__device__ __forceinline__ double mi_d(double d, uint32_t n, bool per)
{
    if (!per) return d;
    const double h = 0.5 * double(n);
    if (d > h) return d - double(n);
    if (d < -h) return d + double(n);
    return d;
}

__device__ __forceinline__ int32_t wrapi(int32_t i, int32_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// axis t = R(q) e_x
__device__ __forceinline__ void axis_of(const double q[4], double t[3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    t[0] = 1.0 - 2.0 * (y * y + z * z);
    t[1] = 2.0 * (x * y + w * z);
    t[2] = 2.0 * (x * z - w * y);
}

// Cell centre (cx, cy, cz) inside the fiber: with d the minimum-image
// vector from the centre, a = d.t and q = |d|^2 - a^2 (squared distance from
// the axis line), the cylinder requires a^2 <= (L/2)^2 and q <= r^2; the
// spherocylinder, with e = |a| - (L/2 - r) beyond the cylindrical part,
// q <= r^2 where e <= 0 and q + e^2 <= r^2 in the caps.  FP64, no
// contraction, fixed evaluation order.
__device__ __forceinline__ bool inside(const PState &s, const PConst &c, double cx, double cy,
                                       double cz, const Geo &g)
{
    const double dx = mi_d(cx - s.X[0], g.nx, true);
    const double dy = mi_d(cy - s.X[1], g.ny, true);
    const double dz = mi_d(cz - s.X[2], g.nz, g.zper != 0);
    const double a = dx * s.t[0] + dy * s.t[1] + dz * s.t[2];
    const double dd = dx * dx + dy * dy + dz * dz;
    const double hl = 0.5 * c.length;
    const double q = dd - a * a, r2 = c.radius * c.radius;
    if (c.shape == 1) {
        const double e = fabs(a) - (hl - c.radius);
        return e <= 0.0 ? q <= r2 : q + e * e <= r2;
    }
    return (a * a <= hl * hl) && (q <= r2);
}

// box (dilated AABB) of the cells a fiber can own or border
__device__ __forceinline__ void fiber_box(const PState &s, const PConst &c, const Geo &g, const double Xref[3],
                          int32_t lo[3], int32_t hi[3])
{
    const uint32_t n[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        const double tk = s.t[k];
        const double ext = c.shape == 1
                               ? (0.5 * c.length - c.radius) * fabs(tk) + c.radius
                               : 0.5 * c.length * fabs(tk) + c.radius * sqrt(fmax(0.0, 1.0 - tk * tk));
        // centre expressed in the frame of Xref (minimum image), so boxes of
        // successive poses can be merged without a wrap in between
        const bool per = k < 2 || g.zper;
        const double X = Xref[k] + mi_d(s.X[k] - Xref[k], n[k], per);
        lo[k] = int32_t(floor(X - ext)) - 2;
        hi[k] = int32_t(ceil(X + ext)) + 2;
    }
}

__device__ __forceinline__ void finish_box(int32_t lo[3], int32_t hi[3], const Geo &g, Box &b)
{
    const int32_t n[3] = {int32_t(g.nx), int32_t(g.ny), int32_t(g.nz)};
    for (int k = 0; k < 3; ++k) {
        const bool per = k < 2 || g.zper;
        if (!per) {
            lo[k] = lo[k] < 0 ? 0 : lo[k];
            hi[k] = hi[k] > n[k] - 1 ? n[k] - 1 : hi[k];
        }
        int32_t len = hi[k] - lo[k] + 1;
        if (len < 0) len = 0;
        if (per && len >= n[k]) {
            lo[k] = 0;
            len = n[k];
        }
        b.lo[k] = lo[k];
        b.len[k] = len;
    }
}

__device__ __forceinline__ bool in_box(const Box &b, int32_t x, int32_t y, int32_t z, const Geo &g)
{
    const int32_t c[3] = {x, y, z}, n[3] = {int32_t(g.nx), int32_t(g.ny), int32_t(g.nz)};
    for (int k = 0; k < 3; ++k) {
        const bool per = k < 2 || g.zper;
        int32_t d = c[k] - b.lo[k];
        if (per) d = wrapi(d, n[k]);
        if (d < 0 || d >= b.len[k]) return false;
    }
    return true;
}

__device__ __forceinline__ bool boxes_meet(const Box &a, const Box &b, const Geo &g)
{
    const int32_t n[3] = {int32_t(g.nx), int32_t(g.ny), int32_t(g.nz)};
    for (int k = 0; k < 3; ++k) {
        const bool per = k < 2 || g.zper;
        bool meet;
        if (per)
            meet = wrapi(b.lo[k] - a.lo[k], n[k]) < a.len[k] || wrapi(a.lo[k] - b.lo[k], n[k]) < b.len[k];
        else
            meet = a.lo[k] < b.lo[k] + b.len[k] && b.lo[k] < a.lo[k] + a.len[k];
        if (!meet) return false;
    }
    return true;
}

// ------------------------------------------------------------------ per-plane rectangles
// Within a box, plane z is crossed by the capsule of radius r + margin
// around the fiber axis segment only in an x/y rectangle.  Every cell that a
// fiber can own lies within r of the segment (REMAP_MARGIN leaves half a
// cell for rounding); every cell that can border it (fluid neighbours lie
// within sqrt(2) of owned cell centres) within r + sqrt(2) (NEAR_MARGIN);
// RECT_MARGIN covers both with room to spare (the batched kernel, which does
// both in one pass).  Rectangles are in the unwrapped frame of the box; for
// boxes narrower than the domain they are clipped to the box.
constexpr double RECT_MARGIN = 2.5;
constexpr double REMAP_MARGIN = 0.5;
constexpr double NEAR_MARGIN = 1.5;

struct Rect {
    int32_t x0, x1, y0, y1;   // inclusive; empty when x0 > x1
};

__device__ __forceinline__ Rect plane_rect(const PState &s, const PConst &c, int32_t z, const Box &b,
                                           const Geo &g, double margin = RECT_MARGIN)
{
    Rect r{1, 0, 1, 0};
    const double R = c.radius + margin, hl = 0.5 * c.length;
    const double dz = mi_d(double(z) - s.X[2], g.nz, g.zper != 0);
    const double tz = s.t[2];
    double slo, shi;
    if (fabs(tz) < 1e-12) {
        if (fabs(dz) > R) return r;
        slo = -hl;
        shi = hl;
    } else {
        const double a = (dz - R) / tz, bb = (dz + R) / tz;
        slo = fmax(fmin(a, bb), -hl);
        shi = fmin(fmax(a, bb), hl);
        if (slo > shi) return r;
    }
    const double mx = double(b.lo[0]) + 0.5 * double(b.len[0]);
    const double my = double(b.lo[1]) + 0.5 * double(b.len[1]);
    const double cx = mx + mi_d(s.X[0] - mx, g.nx, true), cy = my + mi_d(s.X[1] - my, g.ny, true);
    const double xa = slo * s.t[0], xb = shi * s.t[0], ya = slo * s.t[1], yb = shi * s.t[1];
    r.x0 = int32_t(floor(cx + fmin(xa, xb) - R));
    r.x1 = int32_t(ceil(cx + fmax(xa, xb) + R));
    r.y0 = int32_t(floor(cy + fmin(ya, yb) - R));
    r.y1 = int32_t(ceil(cy + fmax(ya, yb) + R));
    if (b.len[0] < int32_t(g.nx)) {
        r.x0 = max(r.x0, b.lo[0]);
        r.x1 = min(r.x1, b.lo[0] + b.len[0] - 1);
    } else if (r.x1 - r.x0 + 1 > int32_t(g.nx)) {
        r.x1 = r.x0 + int32_t(g.nx) - 1;
    }
    if (b.len[1] < int32_t(g.ny)) {
        r.y0 = max(r.y0, b.lo[1]);
        r.y1 = min(r.y1, b.lo[1] + b.len[1] - 1);
    } else if (r.y1 - r.y0 + 1 > int32_t(g.ny)) {
        r.y1 = r.y0 + int32_t(g.ny) - 1;
    }
    return r;
}

__device__ __forceinline__ Rect rect_union(Rect a, Rect b, const Geo &g)
{
    if (a.x0 > a.x1 || a.y0 > a.y1) return b;
    if (b.x0 > b.x1 || b.y0 > b.y1) return a;
    Rect r{min(a.x0, b.x0), max(a.x1, b.x1), min(a.y0, b.y0), max(a.y1, b.y1)};
    if (r.x1 - r.x0 + 1 > int32_t(g.nx)) r.x1 = r.x0 + int32_t(g.nx) - 1;
    if (r.y1 - r.y0 + 1 > int32_t(g.ny)) r.y1 = r.y0 + int32_t(g.ny) - 1;
    return r;
}

__device__ __forceinline__ bool in_rect(const Rect &r, int32_t x, int32_t y, const Geo &g)
{
    if (r.x0 > r.x1 || r.y0 > r.y1) return false;
    return wrapi(x - r.x0, g.nx) <= r.x1 - r.x0 && wrapi(y - r.y0, g.ny) <= r.y1 - r.y0;
}

// is plane z (domain coordinate) inside the z-range of box b?
__device__ __forceinline__ bool in_zrange(const Box &b, int32_t z, const Geo &g)
{
    int32_t d = z - b.lo[2];
    if (g.zper) d = wrapi(d, g.nz);
    return d >= 0 && d < b.len[2];
}

__device__ __forceinline__ int32_t wrapc(int32_t v, int32_t n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

__device__ __forceinline__ void quat_mul(const double a[4], const double b[4], double r[4])
{
    r[0] = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
    r[1] = a[0] * b[1] + b[0] * a[1] + (a[2] * b[3] - a[3] * b[2]);
    r[2] = a[0] * b[2] + b[0] * a[2] + (a[3] * b[1] - a[1] * b[3]);
    r[3] = a[0] * b[3] + b[0] * a[3] + (a[1] * b[2] - a[2] * b[1]);
}

// K x = b for a symmetric positive definite 6x6 K (Cholesky, FP64)
__device__ __forceinline__ void chol6(double K[6][6], const double b[6], double x[6])
{
    double Lm[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (j > i) continue;
            double s = K[i][j];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if (k < j) s -= Lm[i][k] * Lm[j][k];
            if (i == j) Lm[i][i] = sqrt(s);
            else Lm[i][j] = s / Lm[j][j];
        }
    double yv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (k < i) s -= Lm[i][k] * yv[k];
        yv[i] = s / Lm[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = yv[i];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (k > i) s -= Lm[k][i] * x[k];
        x[i] = s / Lm[i][i];
    }
}

__device__ __forceinline__ double wrap_pos(double x, uint32_t n, bool per)
{
    if (!per) return x;
    if (x >= double(n)) return x - double(n);
    if (x < 0.0) return x + double(n);
    return x;
}

// unpack the symmetric accumulators
__device__ __forceinline__ void unpack(const double *acc, double A[3][3], double B[3][3], double C[3][3])
{
    const int si[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int k = 0; k < 6; ++k) {
        A[si[k][0]][si[k][1]] = A[si[k][1]][si[k][0]] = acc[6 + k];
        C[si[k][0]][si[k][1]] = C[si[k][1]][si[k][0]] = acc[21 + k];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = acc[12 + 3 * i + j];
}

// Advance one fiber from state s with the momentum-exchange sums acc.
// Semi-implicit Euler, dt = 1 (the paper leaves the integrator open):
//   V' = V + (F + Fe)/m, X' = X + V', Lang' = Lang + M + Me,
//   W' = I(q)^-1 Lang', q' = normalize(exp(W'/2) (x) q),
// with the constant external load Fe, Me of the fiber (c.fext, c.mext);
// F, M (reported) are the hydrodynamic force and torque.
// coupling 1 (explicit): F, M at the old velocities.  Coupling 0 and 2
// evaluate F = F0 - A V' - B W', M = M0 - B^T V' - C W' at the new
// velocities and solve the 6x6 system for (V', W'); coupling 0 takes for
// F0, M0 the mean of this and the previous step's sums, which removes a
// growing period-two oscillation of the torque at density ratio 1 and
// small tau.  The new state carries this step's F0, M0 forward.  corr
// (dF[3], dM[3] of a closure, or null) is added to the force and torque
// (to F0, M0 for the implicit forms).
// ------------------------------------------------------------------ contact
// Short-range repulsion between fibers (in place of the collision handling
// of the paper's rigid-body engine, Sec. 4.4): a fiber is the segment of its
// axis of half-length max(L/2 - r, 0) swept by its radius.  With the closest
// axis points P (on a) and Q (on b), dist = |Q - P| and gap = dist - r_a - r_b,
// a gap below the range xi gives the force k ((xi - gap)/xi)^2 along
// n = (Q - P)/dist: -that on a, +that on b, both at the middle of the gap.

__device__ __forceinline__ double clamp_d(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Contact load (force, torque about the own centre) on fiber `me` of the pair
// (a, b), a < b, computed in this orientation for either member so that the
// two loads are exact opposites.
__device__ __forceinline__ void contact_load(const PState &sa, const PConst &ca, const PState &sb,
                                             const PConst &cb, bool me_is_a, double k, double range,
                                             const Geo &g, double out[6])
{
    const double d[3] = {mi(sb.X[0] - sa.X[0], g.nx, true), mi(sb.X[1] - sa.X[1], g.ny, true),
                         mi(sb.X[2] - sa.X[2], g.nz, g.zper != 0)};
    const double ha0 = 0.5 * ca.length - ca.radius, hb0 = 0.5 * cb.length - cb.radius;
    const double ha = ha0 > 0.0 ? ha0 : 0.0, hb = hb0 > 0.0 ? hb0 : 0.0;
    const double *ta = sa.t, *tb = sb.t;
    const double bb = ta[0] * tb[0] + ta[1] * tb[1] + ta[2] * tb[2];
    const double e = d[0] * ta[0] + d[1] * ta[1] + d[2] * ta[2];
    const double f = d[0] * tb[0] + d[1] * tb[1] + d[2] * tb[2];
    const double den = 1.0 - bb * bb;
    double s;
    if (den > 1e-12) {
        s = clamp_d((e - bb * f) / den, -ha, ha);
    } else {   // parallel axes: middle of the overlap
        const double lo = e - hb < -ha ? -ha : e - hb, hi = e + hb > ha ? ha : e + hb;
        s = lo <= hi ? 0.5 * (lo + hi) : clamp_d(e, -ha, ha);
    }
    const double u = clamp_d(s * bb - f, -hb, hb);
    s = clamp_d(e + u * bb, -ha, ha);
    double w[3];
    for (int i = 0; i < 3; ++i) w[i] = d[i] + u * tb[i] - s * ta[i];
    const double dist = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    const double gap = dist - ca.radius - cb.radius;
    for (int i = 0; i < 6; ++i) out[i] = 0.0;
    if (!(gap < range) || !(dist > 0.0)) return;
    const double x = (range - gap) / range;
    const double mag = k * x * x;
    double P[3], n[3], C[3], F[3];
    for (int i = 0; i < 3; ++i) {
        P[i] = s * ta[i];
        n[i] = ((d[i] + u * tb[i]) - P[i]) / dist;
    }
    for (int i = 0; i < 3; ++i) {
        C[i] = P[i] + (ca.radius + 0.5 * gap) * n[i];   // relative to X_a
        F[i] = me_is_a ? -mag * n[i] : mag * n[i];
        if (!me_is_a) C[i] = C[i] - d[i];               // relative to X_b
    }
    for (int i = 0; i < 3; ++i) out[i] = F[i];
    out[3] = C[1] * F[2] - C[2] * F[1];
    out[4] = C[2] * F[0] - C[0] * F[2];
    out[5] = C[0] * F[1] - C[1] * F[0];
}

// fc: contact force and torque added to the external load of this step (or null)
__device__ __forceinline__ void rigid_update(const PState &s, const PConst &c, const double *acc, int coupling,
                             const double *traj_row, const Geo &g, PState &o, double F[3], double M[3],
                             const double *corr = nullptr, const double *fc = nullptr)
{
    double A[3][3], B[3][3], C[3][3];
    unpack(acc, A, B, C);
    const double *F0 = acc, *M0 = acc + 3;
    // direct formula (all terms at the old velocity)
    for (int i = 0; i < 3; ++i) {
        double f = F0[i], m = M0[i];
        for (int j = 0; j < 3; ++j) {
            f -= A[i][j] * s.V[j] + B[i][j] * s.W[j];
            m -= B[j][i] * s.V[j] + C[i][j] * s.W[j];
        }
        F[i] = corr ? f + corr[i] : f;
        M[i] = corr ? m + corr[3 + i] : m;
    }
    const bool per[3] = {true, true, g.zper != 0};
    const uint32_t n[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        o.F0p[k] = F0[k];
        o.M0p[k] = M0[k];
    }
    o.have_prev = 1.0;
    if (traj_row) {
        for (int k = 0; k < 3; ++k) o.X[k] = traj_row[k];
        for (int k = 0; k < 4; ++k) o.q[k] = traj_row[3 + k];
        for (int k = 0; k < 3; ++k) o.V[k] = traj_row[7 + k];
        for (int k = 0; k < 3; ++k) o.W[k] = traj_row[10 + k];
        axis_of(o.q, o.t);
        const double tw = o.t[0] * o.W[0] + o.t[1] * o.W[1] + o.t[2] * o.W[2];
        for (int k = 0; k < 3; ++k) o.L[k] = c.i_perp * o.W[k] + (c.i_par - c.i_perp) * tw * o.t[k];
        return;
    }
    double Vn[3], Wn[3], Ln[3];
    if (coupling != 1) {
        const bool avg = coupling == 0 && s.have_prev != 0.0;
        double F0u[3], M0u[3];
        for (int k = 0; k < 3; ++k) {
            F0u[k] = avg ? 0.5 * (F0[k] + s.F0p[k]) : F0[k];
            M0u[k] = avg ? 0.5 * (M0[k] + s.M0p[k]) : M0[k];
            if (corr) {
                F0u[k] += corr[k];
                M0u[k] += corr[3 + k];
            }
        }
        double K[6][6], b[6], x[6];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double Iw = (i == j ? c.i_perp : 0.0) + (c.i_par - c.i_perp) * s.t[i] * s.t[j];
                K[i][j] = (i == j ? c.mass : 0.0) + A[i][j];
                K[i][3 + j] = B[i][j];
                K[3 + i][j] = B[j][i];
                K[3 + i][3 + j] = Iw + C[i][j];
            }
        double fe[3], me[3];
        for (int i = 0; i < 3; ++i) {
            fe[i] = fc ? c.fext[i] + fc[i] : c.fext[i];
            me[i] = fc ? c.mext[i] + fc[3 + i] : c.mext[i];
        }
        for (int i = 0; i < 3; ++i) {
            b[i] = c.mass * s.V[i] + F0u[i] + fe[i];
            b[3 + i] = s.L[i] + M0u[i] + me[i];
        }
        chol6(K, b, x);
        for (int i = 0; i < 3; ++i) {
            Vn[i] = x[i];
            Wn[i] = x[3 + i];
        }
        for (int i = 0; i < 3; ++i) {
            double f = F0u[i], m = M0u[i];
            for (int j = 0; j < 3; ++j) {
                f -= A[i][j] * Vn[j] + B[i][j] * Wn[j];
                m -= B[j][i] * Vn[j] + C[i][j] * Wn[j];
            }
            F[i] = f;
            M[i] = m;
        }
        for (int i = 0; i < 3; ++i) Ln[i] = s.L[i] + M[i] + me[i];
    } else {
        for (int i = 0; i < 3; ++i) {
            const double fe = fc ? c.fext[i] + fc[i] : c.fext[i];
            const double me = fc ? c.mext[i] + fc[3 + i] : c.mext[i];
            Vn[i] = s.V[i] + (F[i] + fe) / c.mass;
            Ln[i] = s.L[i] + (M[i] + me);
        }
        const double tl = s.t[0] * Ln[0] + s.t[1] * Ln[1] + s.t[2] * Ln[2];
        for (int i = 0; i < 3; ++i)
            Wn[i] = Ln[i] / c.i_perp + (1.0 / c.i_par - 1.0 / c.i_perp) * tl * s.t[i];
    }
    for (int k = 0; k < 3; ++k) {
        o.X[k] = wrap_pos(s.X[k] + Vn[k], n[k], per[k]);
        o.V[k] = Vn[k];
        o.W[k] = Wn[k];
        o.L[k] = Ln[k];
    }
    const double ang = sqrt(Wn[0] * Wn[0] + Wn[1] * Wn[1] + Wn[2] * Wn[2]);
    double dq[4] = {1.0, 0.0, 0.0, 0.0};
    if (ang > 0.0) {
        const double sh = sin(0.5 * ang) / ang;
        dq[0] = cos(0.5 * ang);
        dq[1] = sh * Wn[0];
        dq[2] = sh * Wn[1];
        dq[3] = sh * Wn[2];
    }
    double qn[4];
    quat_mul(dq, s.q, qn);
    const double nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int k = 0; k < 4; ++k) o.q[k] = qn[k] / nrm;
    axis_of(o.q, o.t);
}

// Boxes of the remap of one fiber: nb = box of the new pose s, ub = union of
// nb with the boxes of older poses (a box with len[0] == 0 is absent), each
// old interval moved by whole periods next to the new one where periodic.
__device__ __forceinline__ void remap_boxes(const PState &s, const PConst &c, const Box &old, const Box &older,
                                            const Geo &g, Box &ub, Box &nb)
{
    double Xref[3];
    for (int k = 0; k < 3; ++k) Xref[k] = s.X[k];
    int32_t lo[3], hi[3];
    fiber_box(s, c, g, Xref, lo, hi);
    int32_t lo2[3] = {lo[0], lo[1], lo[2]}, hi2[3] = {hi[0], hi[1], hi[2]};
    finish_box(lo2, hi2, g, nb);
    const int32_t n[3] = {int32_t(g.nx), int32_t(g.ny), int32_t(g.nz)};
    int32_t mid_new[3];
    for (int k = 0; k < 3; ++k) mid_new[k] = (lo[k] + hi[k]) / 2;
    const Box *olds[2] = {&old, &older};
    for (int j = 0; j < 2; ++j) {
        const Box &ob = *olds[j];
        if (ob.len[0] <= 0) continue;
        for (int k = 0; k < 3; ++k) {
            const bool per = k < 2 || g.zper;
            int32_t olo = ob.lo[k];
            if (per) {
                const int32_t mid_old = olo + ob.len[k] / 2;
                int32_t sh = mid_new[k] - mid_old;
                sh = int32_t(floor(double(sh) / n[k] + 0.5)) * n[k];
                olo += sh;
            }
            lo[k] = min(lo[k], olo);
            hi[k] = max(hi[k], olo + ob.len[k] - 1);
        }
    }
    finish_box(lo, hi, g, ub);
}
__device__ __forceinline__ void remap_boxes(const PState &s, const PConst &c, const Box &old, const Geo &g,
                                            Box &ub, Box &nb)
{
    remap_boxes(s, c, old, Box{{0, 0, 0}, {0, 0, 0}}, g, ub, nb);
}

// neighbour mask of cell (x, y, z): bit q set when x + c_q is a fiber cell
__device__ __forceinline__ uint32_t fiber_mask(const int32_t *pid, const Geo &g, int32_t x, int32_t y, int32_t z)
{
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    uint32_t mask = 0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        int32_t zz = z + CZ[q];
        if (g.zper) zz = wrapc(zz, nz);
        else if (zz < 0 || zz >= nz) continue;
        const int32_t xx = wrapc(x + CX[q], nx), yy = wrapc(y + CY[q], ny);
        if (pid[(uint32_t(zz) * g.ny + uint32_t(yy)) * g.nx + uint32_t(xx)] >= 0) mask |= 1u << q;
    }
    return mask;
}

// ------------------------------------------------------------------ population-free link sums
// The part of Eq. LBMhydrodynForce (and the torque after it) that is linear
// in the surface velocity u_s = V + W x r has the matrices
//   A = sum k c c^T,  B = sum k c (r x c)^T,  C = sum k (r x c)(r x c)^T
// over a fiber's links, k = 6 w_q rho0, r = y - X the lever arm of the solid
// cell y.  With the reference point Xr = floor(X), s = y - Xr (integer,
// minimum image) and delta = X - Xr, r = s - delta, so
//   A = (rho0/6) SA,  B = (rho0/6) (SB - M),  C = (rho0/6) (SC - N - N^T + P)
// with the integer sums SA = sum kappa c c^T, SB = sum kappa c (s x c)^T,
// SC = sum kappa (s x c)(s x c)^T (kappa = 36 w_q: 2 for the six axis
// links, 1 for the twelve diagonals) and
//   M_ij = eps_jab delta_a SA_ib,  N_ij = eps_jab delta_a SB_bi,
//   P_ij = eps_iab eps_jcd delta_a delta_c SA_bd.
// The sums are exact, so they do not depend on the order of the links, and
// are formed from the list once per step when it is built.

// reference point of a fiber centre: the cell corner floor(X)
__device__ __forceinline__ void fiber_ref(const double X[3], int32_t r[3])
{
    for (int k = 0; k < 3; ++k) r[k] = int32_t(floor(X[k]));
}

__device__ __forceinline__ int32_t mi_i(int32_t d, int32_t n, bool per)
{
    if (!per) return d;
    if (2 * d > n) return d - n;
    if (2 * d < -n) return d + n;
    return d;
}

// integer terms of link q to the solid cell whose offset from its fiber's
// reference point is (sx, sy, sz), added to acc[0 .. 20] = SA[6] SB[9] SC[6]
template <int q>
__device__ __forceinline__ void link_int_terms(long long *acc, int32_t sx, int32_t sy, int32_t sz)
{
    constexpr int32_t c0 = CX[q], c1 = CY[q], c2 = CZ[q];
    constexpr int32_t kap = (c0 * c0 + c1 * c1 + c2 * c2) == 1 ? 2 : 1;
    const int32_t sc0 = sy * c2 - sz * c1, sc1 = sz * c0 - sx * c2, sc2 = sx * c1 - sy * c0;
    acc[0] += kap * c0 * c0;
    acc[1] += kap * c0 * c1;
    acc[2] += kap * c0 * c2;
    acc[3] += kap * c1 * c1;
    acc[4] += kap * c1 * c2;
    acc[5] += kap * c2 * c2;
    acc[6] += kap * c0 * sc0;
    acc[7] += kap * c0 * sc1;
    acc[8] += kap * c0 * sc2;
    acc[9] += kap * c1 * sc0;
    acc[10] += kap * c1 * sc1;
    acc[11] += kap * c1 * sc2;
    acc[12] += kap * c2 * sc0;
    acc[13] += kap * c2 * sc1;
    acc[14] += kap * c2 * sc2;
    acc[15] += (long long)(kap * sc0) * sc0;
    acc[16] += (long long)(kap * sc0) * sc1;
    acc[17] += (long long)(kap * sc0) * sc2;
    acc[18] += (long long)(kap * sc1) * sc1;
    acc[19] += (long long)(kap * sc1) * sc2;
    acc[20] += (long long)(kap * sc2) * sc2;
}

// Levi-Civita symbol
__device__ __forceinline__ int32_t eps3(int i, int j, int k)
{
    return (i == j || j == k || i == k) ? 0 : (((j - i + 3) % 3) == 1 ? 1 : -1);
}

// A, B, C (packed as the momentum-exchange accumulators 6 .. 26: A[6]
// symmetric, B[9], C[6] symmetric) from the integer sums S (exact values in
// FP64) of a fiber centred at X, in place
__device__ __forceinline__ void abc_restore(double *acc, const double X[3], double rho0)
{
    const int si[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    double SA[3][3], SB[3][3], SC[3][3], d[3];
    for (int k = 0; k < 6; ++k) {
        SA[si[k][0]][si[k][1]] = SA[si[k][1]][si[k][0]] = acc[6 + k];
        SC[si[k][0]][si[k][1]] = SC[si[k][1]][si[k][0]] = acc[21 + k];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) SB[i][j] = acc[12 + 3 * i + j];
    for (int k = 0; k < 3; ++k) d[k] = X[k] - floor(X[k]);
    // (delta x c) components as linear maps of c: E[j][b] = eps_jab delta_a
    double E[3][3];
    for (int j = 0; j < 3; ++j)
        for (int b = 0; b < 3; ++b) {
            double e = 0.0;
            for (int a = 0; a < 3; ++a) e += double(eps3(j, a, b)) * d[a];
            E[j][b] = e;
        }
    const double k6 = rho0 / 6.0;
    double B[3][3], C[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double m = 0.0, nn = 0.0, nt = 0.0;
            for (int b = 0; b < 3; ++b) {
                m += E[j][b] * SA[i][b];    // M_ij
                nn += E[j][b] * SB[b][i];   // N_ij
                nt += E[i][b] * SB[b][j];   // N_ji
            }
            double pp = 0.0;                // P_ij = E[i][b] E[j][e] SA_be
            for (int b = 0; b < 3; ++b)
                for (int e = 0; e < 3; ++e) pp += E[i][b] * E[j][e] * SA[b][e];
            B[i][j] = k6 * (SB[i][j] - m);
            C[i][j] = k6 * (((SC[i][j] - nn) - nt) + pp);
        }
    for (int k = 0; k < 6; ++k) {
        acc[6 + k] = k6 * SA[si[k][0]][si[k][1]];
        acc[21 + k] = C[si[k][0]][si[k][1]];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc[12 + 3 * i + j] = B[i][j];
}

// fiber_mask with the owner of each linked cell: own[q] for the set bits
__device__ __forceinline__ uint32_t fiber_links(const int32_t *pid, const Geo &g, int32_t x, int32_t y, int32_t z,
                                                int32_t (&own)[Q])
{
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    uint32_t mask = 0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        own[q] = -1;
        int32_t zz = z + CZ[q];
        if (g.zper) zz = wrapc(zz, nz);
        else if (zz < 0 || zz >= nz) continue;
        const int32_t xx = wrapc(x + CX[q], nx), yy = wrapc(y + CY[q], ny);
        own[q] = pid[(uint32_t(zz) * g.ny + uint32_t(yy)) * g.nx + uint32_t(xx)];
        if (own[q] >= 0) mask |= 1u << q;
    }
    return mask;
}

template <typename S>
__device__ __forceinline__ void store_dev(S *f, uint64_t i, double v, double scale);
template <>
__device__ __forceinline__ void store_dev<float>(float *f, uint64_t i, double v, double) { f[i] = float(v); }
template <>
__device__ __forceinline__ void store_dev<double>(double *f, uint64_t i, double v, double) { f[i] = v; }
template <>
__device__ __forceinline__ void store_dev<_Float16>(_Float16 *f, uint64_t i, double v, double scale)
{
    f[i] = _Float16(float(v) * float(scale));
}
template <>
__device__ __forceinline__ void store_dev<uint16_t>(uint16_t *f, uint64_t i, double v, double)
{
    uint32_t u = __float_as_uint(float(v));
    u += 0x7FFFu + ((u >> 16) & 1u);
    f[i] = uint16_t(u >> 16);
}


// Refill of a cell uncovered by the remap (Sec. 4.2): f = f_eq(rho0, u_s)
// with u_s the rigid-body velocity there of the old owner's state so.  The
// values go to the slots the next sweep reads: for an odd sweep, slot
// opp(q) of x - c_q (its gather source); for an even sweep, the natural slots.
template <typename S>
__device__ __forceinline__ void refill_cell(S *f, const Geo &g, int32_t x, int32_t y, int32_t z,
                                            const PState &so, double rho0, double scale, int next_odd)
{
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    const double cx = x, cy = y, cz = z;
    const double dx = mi_d(cx - so.X[0], g.nx, true), dy = mi_d(cy - so.X[1], g.ny, true),
                 dz = mi_d(cz - so.X[2], g.nz, g.zper != 0);
    const double u0 = so.V[0] + (so.W[1] * dz - so.W[2] * dy);
    const double u1 = so.V[1] + (so.W[2] * dx - so.W[0] * dz);
    const double u2 = so.V[2] + (so.W[0] * dy - so.W[1] * dx);
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    for (int q = 0; q < Q; ++q) {
        const double cu = CX[q] * u0 + CY[q] * u1 + CZ[q] * u2;
        const double dev = wq(q) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        uint64_t slot;
        if (next_odd) {
            const int32_t sx = wrapc(x - CX[q], nx), sy = wrapc(y - CY[q], ny);
            int32_t sz = z - CZ[q];
            if (g.zper) sz = wrapc(sz, nz);
            slot = uint64_t(opp(q)) * g.qstride + (uint64_t(sz + 1) * g.ny + uint64_t(sy)) * g.nx + uint64_t(sx);
        } else {
            slot = uint64_t(q) * g.qstride + (uint64_t(z + 1) * g.ny + uint64_t(y)) * g.nx + uint64_t(x);
        }
        store_dev<S>(f, slot, dev, scale);
    }
}

}  // namespace lbm
