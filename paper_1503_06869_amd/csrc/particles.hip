// particles.hip -- per-fiber work of one time step on the device:
//   k_particles  momentum exchange (Eq. LBMhydrodynForce and the torque
//                after it, Sec. 4.2) reduced in FP64 per fiber, then the
//                rigid-body update (Sec. 4.3) and, in the last block to
//                finish, the cell boxes and neighbour lists of the remap;
//   k_remap      cell mapping with the new poses (Sec. 4.2: a cell is an
//                obstacle cell when its centre lies inside a particle) and
//                refill of uncovered cells with f_eq(rho0, u_s) of the
//                previous step's motion;
//   k_near       flags of fluid cells next to fibers and the boundary-cell
//                list consumed by the next sweep.
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

// Cell centre (cx, cy, cz) inside the cylinder: with d the minimum-image
// vector from the centre and a = d.t, require a^2 <= (L/2)^2 and
// |d|^2 - a^2 <= r^2.  FP64, no contraction, fixed evaluation order.
__device__ __forceinline__ bool inside(const PState &s, const PConst &c, double cx, double cy,
                                       double cz, const Geo &g)
{
    const double dx = mi_d(cx - s.X[0], g.nx, true);
    const double dy = mi_d(cy - s.X[1], g.ny, true);
    const double dz = mi_d(cz - s.X[2], g.nz, g.zper != 0);
    const double a = dx * s.t[0] + dy * s.t[1] + dz * s.t[2];
    const double dd = dx * dx + dy * dy + dz * dz;
    const double hl = 0.5 * c.length;
    return (a * a <= hl * hl) && (dd - a * a <= c.radius * c.radius);
}

// box (dilated AABB) of the cells a fiber can own or border
__device__ void fiber_box(const PState &s, const PConst &c, const Geo &g, const double Xref[3],
                          int32_t lo[3], int32_t hi[3])
{
    const uint32_t n[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        const double tk = s.t[k];
        const double ext = 0.5 * c.length * fabs(tk) + c.radius * sqrt(fmax(0.0, 1.0 - tk * tk));
        // centre expressed in the frame of Xref (minimum image), so boxes of
        // successive poses can be merged without a wrap in between
        const bool per = k < 2 || g.zper;
        const double X = Xref[k] + mi_d(s.X[k] - Xref[k], n[k], per);
        lo[k] = int32_t(floor(X - ext)) - 2;
        hi[k] = int32_t(ceil(X + ext)) + 2;
    }
}

__device__ void finish_box(int32_t lo[3], int32_t hi[3], const Geo &g, Box &b)
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
// Within a box, plane z is crossed by the capsule of radius r + RECT_MARGIN
// around the fiber axis segment only in an x/y rectangle; every cell that a
// fiber can own, or border (fluid neighbours lie within sqrt(2) of owned
// cell centres), is inside it.  Rectangles are in the unwrapped frame of
// the box; for boxes narrower than the domain they are clipped to the box.
constexpr double RECT_MARGIN = 2.5;

struct Rect {
    int32_t x0, x1, y0, y1;   // inclusive; empty when x0 > x1
};

__device__ __forceinline__ Rect plane_rect(const PState &s, const PConst &c, int32_t z, const Box &b,
                                           const Geo &g)
{
    Rect r{1, 0, 1, 0};
    const double R = c.radius + RECT_MARGIN, hl = 0.5 * c.length;
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

// plane rectangle of fiber o's remap region: both poses of the step
__device__ __forceinline__ Rect remap_rect(const PartData &pd, int o, int32_t z, const Geo &g)
{
    const Box b = pd.box_remap[o];
    const PConst c = pd.pc[o];
    return rect_union(plane_rect(pd.ps_cur[o], c, z, b, g), plane_rect(pd.ps_next[o], c, z, b, g), g);
}

// ------------------------------------------------------------------ boxes of the remap
// Runs in one block: union of the box of the old pose (box_cur) and the new
// pose (ps_next) per fiber, their cell-count prefix, and for every fiber the
// ascending list of other fibers whose boxes meet its box.
__device__ void build_remap_work(const PartData &pd, const Geo &g)
{
    const int np = pd.np;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const PState s = pd.ps_next[p];   // visible: acquire fence by the caller
        const PConst c = pd.pc[p];
        Box old = pd.box_cur[p];
        double Xref[3];
        for (int k = 0; k < 3; ++k) Xref[k] = s.X[k];
        int32_t lo[3], hi[3];
        fiber_box(s, c, g, Xref, lo, hi);
        Box nb;
        int32_t lo2[3] = {lo[0], lo[1], lo[2]}, hi2[3] = {hi[0], hi[1], hi[2]};
        finish_box(lo2, hi2, g, nb);
        // union with the old box, expressed around the new box where periodic
        if (old.len[0] > 0) {
            const int32_t n[3] = {int32_t(g.nx), int32_t(g.ny), int32_t(g.nz)};
            for (int k = 0; k < 3; ++k) {
                const bool per = k < 2 || g.zper;
                int32_t olo = old.lo[k];
                if (per) {
                    // move the old interval by whole periods next to the new one
                    const int32_t mid_new = (lo[k] + hi[k]) / 2;
                    const int32_t mid_old = olo + old.len[k] / 2;
                    int32_t sh = mid_new - mid_old;
                    sh = int32_t(floor(double(sh) / n[k] + 0.5)) * n[k];
                    olo += sh;
                }
                lo[k] = min(lo[k], olo);
                hi[k] = max(hi[k], olo + old.len[k] - 1);
            }
        }
        Box ub;
        finish_box(lo, hi, g, ub);
        pd.box_remap[p] = ub;
        pd.box_cur[p] = nb;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < np; p += blockDim.x) pd.seg_cnt[p] = 0u;
    // neighbour lists: the boxes are staged in LDS in chunks
    __shared__ Box sbox[512];
    for (int p0 = 0; p0 < np; p0 += blockDim.x) {
    const int p = p0 + threadIdx.x;
    const Box a = p < np ? pd.box_remap[p] : Box{};
    int cnt = 0;
    for (int o0 = 0; o0 < np; o0 += 512) {
        const int no = min(512, np - o0);
        __syncthreads();
        for (int k = threadIdx.x; k < no; k += blockDim.x) sbox[k] = pd.box_remap[o0 + k];
        __syncthreads();
        if (p >= np) continue;
        for (int oo = 0; oo < no; ++oo) {
            const int o = o0 + oo;
            if (o == p) continue;
            if (!boxes_meet(a, sbox[oo], g)) continue;
            if (cnt < NBR_CAP) pd.nbr[p * NBR_CAP + cnt] = o;
            ++cnt;
        }
    }
    if (p < np) {
        if (cnt > NBR_CAP) {
            atomicOr(&pd.ctr->err_capacity, 1u);
            cnt = NBR_CAP;
        }
        pd.nbr_n[p] = cnt;
    }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        pd.ctr->block_ticket = 0u;
    }
}

// end of a time step: advance the device step counter (last block only)
__device__ void finish_step(const PartData &pd)
{
    if (threadIdx.x == 0) pd.ctr->step += 1ull;
}

__global__ __launch_bounds__(256) void k_setup_boxes(PartData pd, Geo g)
{
    build_remap_work(pd, g);
}

// ------------------------------------------------------------------ rigid body
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
//   V' = V + F/m, X' = X + V', Lang' = Lang + M, W' = I(q)^-1 Lang',
//   q' = normalize(exp(W'/2) (x) q).
// Implicit coupling evaluates F = F0 - A V' - B W', M = M0 - B^T V' - C W'
// at the new velocities and solves the 6x6 system for (V', W').
__device__ __forceinline__ void rigid_update(const PState &s, const PConst &c, const double *acc, int implicit,
                             const double *traj_row, const Geo &g, PState &o, double F[3], double M[3])
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
        F[i] = f;
        M[i] = m;
    }
    const bool per[3] = {true, true, g.zper != 0};
    const uint32_t n[3] = {g.nx, g.ny, g.nz};
    if (traj_row) {
        for (int k = 0; k < 3; ++k) o.X[k] = traj_row[k];
        for (int k = 0; k < 4; ++k) o.q[k] = traj_row[3 + k];
        for (int k = 0; k < 3; ++k) o.V[k] = traj_row[7 + k];
        for (int k = 0; k < 3; ++k) o.W[k] = traj_row[10 + k];
        axis_of(o.q, o.t);
        const double tw = o.t[0] * o.W[0] + o.t[1] * o.W[1] + o.t[2] * o.W[2];
        for (int k = 0; k < 3; ++k) o.L[k] = c.i_perp * o.W[k] + (c.i_par - c.i_perp) * tw * o.t[k];
        o.pad = 0.0;
        return;
    }
    double Vn[3], Wn[3], Ln[3];
    if (implicit) {
        double K[6][6], b[6], x[6];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double Iw = (i == j ? c.i_perp : 0.0) + (c.i_par - c.i_perp) * s.t[i] * s.t[j];
                K[i][j] = (i == j ? c.mass : 0.0) + A[i][j];
                K[i][3 + j] = B[i][j];
                K[3 + i][j] = B[j][i];
                K[3 + i][3 + j] = Iw + C[i][j];
            }
        for (int i = 0; i < 3; ++i) {
            b[i] = c.mass * s.V[i] + F0[i];
            b[3 + i] = s.L[i] + M0[i];
        }
        chol6(K, b, x);
        for (int i = 0; i < 3; ++i) {
            Vn[i] = x[i];
            Wn[i] = x[3 + i];
        }
        for (int i = 0; i < 3; ++i) {
            double f = F0[i], m = M0[i];
            for (int j = 0; j < 3; ++j) {
                f -= A[i][j] * Vn[j] + B[i][j] * Wn[j];
                m -= B[j][i] * Vn[j] + C[i][j] * Wn[j];
            }
            F[i] = f;
            M[i] = m;
        }
        for (int i = 0; i < 3; ++i) Ln[i] = s.L[i] + M[i];
    } else {
        for (int i = 0; i < 3; ++i) {
            Vn[i] = s.V[i] + F[i] / c.mass;
            Ln[i] = s.L[i] + M[i];
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
    o.pad = 0.0;
}

// ------------------------------------------------------------------ rigid update kernel
__device__ __forceinline__ int32_t wrapc(int32_t v, int32_t n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// One block: the momentum-exchange sums of every fiber (accumulated in fixed
// point by the boundary sweep) back to FP64, the rigid-body update, outputs,
// then the boxes and neighbour lists of the remap and the list reset.
__global__ __launch_bounds__(256) void k_rigid(PartData pd, Geo g)
{
    extern __shared__ double tot[];   // [np][NACC]
    const int np = pd.np;
    for (int t = threadIdx.x; t < np * NACC; t += blockDim.x) {
        const int k = t % NACC;
        tot[t] = ldexp(double(pd.mea[t]), -fx_shift(k));
        pd.mea[t] = 0;   // cleared for the next step's boundary sweep
    }
    __syncthreads();
    const int64_t step = int64_t(pd.ctr->step);
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        double ac[NACC];
        for (int k = 0; k < NACC; ++k) ac[k] = tot[p * NACC + k];
        const PConst c = pd.pc[p];
        const PState s = pd.ps_cur[p];
        const double *row = nullptr;
        if (c.traj_off >= 0 && pd.traj_pos[p] < c.traj_n) {
            row = pd.traj + (c.traj_off + pd.traj_pos[p]) * 13;
            pd.traj_pos[p] += 1;
        }
        PState o;
        double F[3], M[3];
        rigid_update(s, c, ac, pd.implicit, row, g, o, F, M);
        bool bad = false;
        for (int k = 0; k < 3; ++k) bad |= !isfinite(F[k]) || !isfinite(M[k]);
        if (bad) atomicOr(&pd.ctr->err_unstable, 1u);
        pd.ps_next[p] = o;
        for (int k = 0; k < 3; ++k) {
            pd.ft_out[p * 6 + k] = F[k];
            pd.ft_out[p * 6 + 3 + k] = M[k];
        }
        double *h = pd.hist + ((step % pd.hist_cap) * np + p) * 19;
        for (int k = 0; k < 3; ++k) { h[k] = F[k]; h[3 + k] = M[k]; h[6 + k] = o.X[k]; }
        for (int k = 0; k < 4; ++k) h[9 + k] = o.q[k];
        for (int k = 0; k < 3; ++k) { h[13 + k] = o.V[k]; h[16 + k] = o.W[k]; }
    }
    __syncthreads();
    build_remap_work(pd, g);
    finish_step(pd);
}

// ------------------------------------------------------------------ remap and boundary list
// Grid: np * nslab blocks; block (p, s) walks the z-planes s, s + nslab, ...
// of fiber p's remap box.  A cell inside the box of a lower-indexed fiber is
// left to that fiber's blocks, so every cell is handled once.  The boxes of
// the neighbouring fibers are staged in LDS.
struct NbrStage {
    int32_t id[NBR_CAP];
    Box box[NBR_CAP];
    Rect rect[NBR_CAP];   // plane rectangle of each lower-indexed neighbour (current plane)
    uint8_t zin[NBR_CAP]; // current plane inside the neighbour's box
    int32_t n, nlow;
};

__device__ __forceinline__ void stage_nbrs(const PartData &pd, int p, NbrStage &sh)
{
    const int nn = pd.nbr_n[p];
    for (int k = threadIdx.x; k < nn; k += blockDim.x) {
        const int o = pd.nbr[p * NBR_CAP + k];
        sh.id[k] = o;
        sh.box[k] = pd.box_remap[o];
    }
    if (threadIdx.x == 0) {
        int nl = 0;
        while (nl < nn && pd.nbr[p * NBR_CAP + nl] < p) ++nl;   // ascending ids
        sh.n = nn;
        sh.nlow = nl;
    }
    __syncthreads();
}

// rectangles of the lower-indexed neighbours for plane z (block-uniform call)
__device__ __forceinline__ void stage_plane(const PartData &pd, NbrStage &sh, int32_t z, const Geo &g)
{
    __syncthreads();
    for (int k = threadIdx.x; k < sh.nlow; k += blockDim.x) {
        const int o = sh.id[k];
        sh.zin[k] = in_zrange(sh.box[k], z, g);
        if (sh.zin[k]) sh.rect[k] = remap_rect(pd, o, z, g);
    }
    __syncthreads();
}

// a cell is handled by the lowest-indexed fiber whose remap region holds it
__device__ __forceinline__ bool owned_here(const NbrStage &sh, int32_t x, int32_t y, const Geo &g)
{
    for (int k = 0; k < sh.nlow; ++k)
        if (sh.zin[k] && in_rect(sh.rect[k], x, y, g)) return false;
    return true;
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

// new owner of each cell of the remap boxes; refill of uncovered cells
template <typename S>
__global__ __launch_bounds__(256) void k_remap(S *__restrict__ f, int32_t *__restrict__ pid, PartData pd,
                                               Geo g, int next_odd, double rho0, double scale)
{
    const int ns = pd.nslab;
    const int p = blockIdx.x / ns, sl = blockIdx.x % ns;
    __shared__ NbrStage sh;
    stage_nbrs(pd, p, sh);
    const Box b = pd.box_remap[p];
    const PState sp = pd.ps_next[p];
    const PConst cp = pd.pc[p];
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    for (int iz = sl; iz < b.len[2]; iz += ns) {   // block-uniform
        int32_t z = b.lo[2] + iz;
        if (g.zper) z = wrapc(z, nz);
        else if (z < 0 || z >= nz) continue;
        stage_plane(pd, sh, z, g);
        const Rect rc = remap_rect(pd, p, z, g);
        if (rc.x0 > rc.x1 || rc.y0 > rc.y1) continue;
        const int wx = rc.x1 - rc.x0 + 1, area = wx * (rc.y1 - rc.y0 + 1);
        for (int i = threadIdx.x; i < area; i += blockDim.x) {
            const int iy = i / wx, ix = i - iy * wx;
            const int32_t x = wrapi(rc.x0 + ix, nx), y = wrapi(rc.y0 + iy, ny);
            if (!owned_here(sh, x, y, g)) continue;
            const double cx = x, cy = y, cz = z;
            int owner = -1, claims = 0;
            if (inside(sp, cp, cx, cy, cz, g)) {
                owner = p;
                claims = 1;
            }
            for (int k = sh.nlow; k < sh.n; ++k) {
                const int o = sh.id[k];
                if (!in_box(sh.box[k], x, y, z, g)) continue;
                if (inside(pd.ps_next[o], pd.pc[o], cx, cy, cz, g)) {
                    if (owner < 0) owner = o;
                    ++claims;
                }
            }
            if (claims > 1) atomicAdd(&pd.ctr->overlaps, (unsigned long long)(claims - 1));
            const uint32_t cell = (uint32_t(z) * g.ny + uint32_t(y)) * g.nx + uint32_t(x);
            const int old = pid[cell];
            if (old >= 0 && owner < 0) {
                // uncovered: f = f_eq(rho0, u_s) of the old owner's previous motion
                const PState &so = pd.ps_cur[old];
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
                        // the odd gather of this cell reads slot opp(q) of x - c_q
                        const int32_t sx = wrapc(x - CX[q], nx), sy = wrapc(y - CY[q], ny);
                        int32_t sz = z - CZ[q];
                        if (g.zper) sz = wrapc(sz, nz);
                        slot = uint64_t(opp(q)) * g.qstride +
                               (uint64_t(sz + 1) * g.ny + uint64_t(sy)) * g.nx + uint64_t(sx);
                    } else {
                        slot = uint64_t(q) * g.qstride + (uint64_t(z + 1) * g.ny + uint64_t(y)) * g.nx +
                               uint64_t(x);
                    }
                    store_dev<S>(f, slot, dev, scale);
                }
            }
            pid[cell] = owner;
        }
    }
}

// Flags of the cells in the remap regions and the boundary-cell list.  The
// list is cut into one segment per fiber; a block stages the boundary cells
// it finds in LDS and reserves a range of its fiber's segment with a single
// atomic.
constexpr int LSTAGE = 2048;

__global__ __launch_bounds__(256) void k_near(uint8_t *__restrict__ flags, const int32_t *__restrict__ pid,
                                              uint32_t *__restrict__ list_cell,
                                              uint32_t *__restrict__ list_mask, PartData pd, Geo g)
{
    const int ns = pd.nslab;
    const int p = blockIdx.x / ns, sl = blockIdx.x % ns;
    __shared__ NbrStage sh;
    __shared__ uint32_t s_cell[LSTAGE], s_mask[LSTAGE];
    __shared__ uint32_t s_n, s_base;
    stage_nbrs(pd, p, sh);
    if (threadIdx.x == 0) s_n = 0u;
    __syncthreads();
    const Box b = pd.box_remap[p];
    const uint32_t off = pd.seg_off[p], cap = pd.seg_cap[p];
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    for (int iz = sl; iz < b.len[2]; iz += ns) {   // block-uniform
        int32_t z = b.lo[2] + iz;
        if (g.zper) z = wrapc(z, nz);
        else if (z < 0 || z >= nz) continue;
        stage_plane(pd, sh, z, g);
        const Rect rc = remap_rect(pd, p, z, g);
        const int wx = rc.x1 - rc.x0 + 1;
        const int area = (rc.x0 > rc.x1 || rc.y0 > rc.y1) ? 0 : wx * (rc.y1 - rc.y0 + 1);
        for (int i = threadIdx.x; i < area; i += blockDim.x) {
            const int iy = i / wx, ix = i - iy * wx;
            const int32_t x = wrapi(rc.x0 + ix, nx), y = wrapi(rc.y0 + iy, ny);
            if (!owned_here(sh, x, y, g)) continue;
            const uint32_t cell = (uint32_t(z) * g.ny + uint32_t(y)) * g.nx + uint32_t(x);
            if (pid[cell] >= 0) {
                flags[cell] = F_SOLID;
                continue;
            }
            uint32_t mask = 0;
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                int32_t zz = z + CZ[q];
                if (g.zper) zz = wrapc(zz, nz);
                else if (zz < 0 || zz >= nz) continue;
                const int32_t xx = wrapc(x + CX[q], nx), yy = wrapc(y + CY[q], ny);
                if (pid[(uint32_t(zz) * g.ny + uint32_t(yy)) * g.nx + uint32_t(xx)] >= 0) mask |= 1u << q;
            }
            if (!mask) {
                flags[cell] = 0;
                continue;
            }
            const uint32_t k = atomicAdd(&s_n, 1u);
            if (k < LSTAGE) {
                s_cell[k] = cell;
                s_mask[k] = mask;
            } else {
                // stage full: append directly
                const uint32_t r = atomicAdd(&pd.seg_cnt[p], 1u);
                if (r < cap) {
                    const uint32_t e = off + r;
                    list_cell[e] = cell;
                    list_mask[e] = mask;
                    flags[cell] = F_NEAR;
                } else {
                    flags[cell] = 0;
                        atomicOr(&pd.ctr->err_capacity, 2u);
                }
            }
        }
        __syncthreads();
        const uint32_t n = min(s_n, uint32_t(LSTAGE));
        if (threadIdx.x == 0 && n) s_base = atomicAdd(&pd.seg_cnt[p], n);
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
            const uint32_t r = s_base + k, cell = s_cell[k];
            if (r < cap) {
                const uint32_t e = off + r;
                list_cell[e] = cell;
                list_mask[e] = s_mask[k];
                flags[cell] = F_NEAR;
            } else {
                flags[cell] = 0;
                atomicOr(&pd.ctr->err_capacity, 2u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) s_n = 0u;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_rigid(const PartData &pd, const Geo &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_rigid, dim3(1), dim3(256), size_t(pd.np) * NACC * sizeof(double), st, pd, g);
    return hipGetLastError();
}

hipError_t launch_setup_boxes(const PartData &pd, const Geo &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_setup_boxes, dim3(1), dim3(256), 0, st, pd, g);
    return hipGetLastError();
}

hipError_t launch_remap(int sk, bool next_odd, void *f, int32_t *pid, const PartData &pd, const Geo &g,
                        double rho0, double scale, hipStream_t st)
{
    const int no = next_odd ? 1 : 0;
    const dim3 gr(pd.np * pd.nslab), bl(256);
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_remap<float>, gr, bl, 0, st, (float *)f, pid, pd, g, no, rho0, scale); break;
    case S_F16: hipLaunchKernelGGL(k_remap<_Float16>, gr, bl, 0, st, (_Float16 *)f, pid, pd, g, no, rho0, scale); break;
    case S_BF16: hipLaunchKernelGGL(k_remap<uint16_t>, gr, bl, 0, st, (uint16_t *)f, pid, pd, g, no, rho0, scale); break;
    default: hipLaunchKernelGGL(k_remap<double>, gr, bl, 0, st, (double *)f, pid, pd, g, no, rho0, scale); break;
    }
    return hipGetLastError();
}

hipError_t launch_near(uint8_t *flags, const int32_t *pid, uint32_t *list_cell, uint32_t *list_mask,
                       const PartData &pd, const Geo &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_near, dim3(pd.np * pd.nslab), dim3(256), 0, st, flags, pid, list_cell, list_mask,
                       pd, g);
    return hipGetLastError();
}

}  // namespace lbm
