// lbm_sweep_dev.h -- device functions of the stream-collide update shared by
// the single-lattice kernels (sweep.hip) and the batched kernel (batched.hip):
// storage conversions, the TRT collision, the AA update of one cell with
// wall and fiber bounce-back, and the momentum-exchange terms of a link.
#pragma once
#include "lbm_dev.h"

namespace lbm {

// ------------------------------------------------------------------ storage
template <typename S>
struct St;
template <>
struct St<float> {
    using R = float;
    static __device__ __forceinline__ float ld(const float *p, uint64_t i, float) { return p[i]; }
    static __device__ __forceinline__ void st(float *p, uint64_t i, float v, float)
    {
        __builtin_nontemporal_store(v, p + i);
    }
};
template <>
struct St<double> {
    using R = double;
    static __device__ __forceinline__ double ld(const double *p, uint64_t i, double) { return p[i]; }
    static __device__ __forceinline__ void st(double *p, uint64_t i, double v, double)
    {
        __builtin_nontemporal_store(v, p + i);
    }
};
template <>
struct St<_Float16> {
    using R = float;
    static __device__ __forceinline__ float ld(const _Float16 *p, uint64_t i, float inv)
    {
        return float(p[i]) * inv;
    }
    static __device__ __forceinline__ void st(_Float16 *p, uint64_t i, float v, float scale)
    {
        __builtin_nontemporal_store(_Float16(v * scale), p + i);   // v_cvt_f16_f32: RNE
    }
};
struct bf16s {
    uint16_t b;
};
template <>
struct St<bf16s> {
    using R = float;
    static __device__ __forceinline__ float ld(const bf16s *p, uint64_t i, float)
    {
        const uint16_t *u = reinterpret_cast<const uint16_t *>(p);
        return __uint_as_float(uint32_t(u[i]) << 16);
    }
    static __device__ __forceinline__ void st(bf16s *p, uint64_t i, float v, float)
    {
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
        __builtin_nontemporal_store(uint16_t(u >> 16), reinterpret_cast<uint16_t *>(p) + i);
    }
};

// Each XCD receives every 8th block; renumber so that each XCD works on a
// contiguous range of cells (neighbouring blocks share partial cache lines).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t per = nb >> 3, rem = nb & 7u;
    const uint32_t xcd = b & 7u, k = b >> 3;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// the physical parameters in the collision type R (host side, for launches)
template <typename R>
inline Phys<R> cast_phys(const Phys<double> &p)
{
    Phys<R> o;
    o.rho0 = R(p.rho0);
    o.omega_e = R(p.omega_e);
    o.omega_o = R(p.omega_o);
    o.wall_u = R(p.wall_u);
    for (int k = 0; k < 3; ++k) o.g[k] = R(p.g[k]);
    o.has_g = p.has_g;
    o.scale = R(p.scale);
    o.inv_scale = R(p.inv_scale);
    return o;
}

// Where population q of cell (x, y, z) sits in the swapped layout (between
// the even and the odd sweep of a pair), i.e. where the odd sweep gathers
// it: slot opp(q) of x - c_q; through a no-slip x or y wall (and not a
// no-slip z wall), the cell's own slot q; through free-slip walls only,
// slot opp(refl(q)) of x - t, refl(q) the direction it had before the
// reflection and t the components of c_q along the walls it did not cross.
// Returns the plane-shifted cell index, the slot's direction in qq.
__device__ __forceinline__ uint32_t swapped_src(const Geo &g, uint32_t x, uint32_t y, uint32_t z, int q, int &qq)
{
    bool ix = g.xw && ((CX[q] > 0 && x == 0) || (CX[q] < 0 && x + 1 == g.nx));
    bool iy = g.yw && ((CY[q] > 0 && y == 0) || (CY[q] < 0 && y + 1 == g.ny));
    bool iz = !g.zper && ((CZ[q] > 0 && z == 0) || (CZ[q] < 0 && z + 1 == g.nz));
    if (iz && !g.zs) {
        ix = iy = iz = false;      // the z wall's ghost-plane mailbox
    } else if ((ix && g.xw == 1) || (iy && g.yw == 1)) {
        qq = q;
        return (z + 1) * g.nxy + y * g.nx + x;
    }
    const int m = (ix ? 1 : 0) | (iy ? 2 : 0) | (iz ? 4 : 0);
    qq = opp(refl_sel(q, m));
    const int tx = ix ? 0 : CX[q], ty = iy ? 0 : CY[q], tz = iz ? 0 : CZ[q];
    const uint32_t sx = (x + g.nx - tx) % g.nx, sy = (y + g.ny - ty) % g.ny;
    const int32_t szi = int32_t(z) - tz;
    const uint32_t szs = g.zper ? uint32_t((szi + int32_t(g.nz)) % int32_t(g.nz)) + 1 : uint32_t(szi + 1);
    return szs * g.nxy + sy * g.nx + sx;
}

// ------------------------------------------------------------------ stabilization
// Momentum stabilization (Sec. 4.1): the collisions of a step take their
// equilibrium at u - ub, ub the mean fluid velocity of the state they read.
// Each thread also sums, over the cells it updates, the momentum j before
// collision, the momentum change of its bounce-back links and the cell count;
// the per-workgroup totals give the next step's mean without a further pass
// over the lattice (the collision changes each cell's momentum by the uniform
// rho0 (g - omega_o ub), streaming in the interior conserves it).
template <typename R>
struct StabAcc {
    R ub[3];
    R j[3];
    R n;
};

template <typename R>
__device__ __forceinline__ void stab_begin(StabAcc<R> &sa, const double *stab)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        sa.ub[k] = R(stab[k]);
        sa.j[k] = R(0);
    }
    sa.n = R(0);
}

// Workgroup total (256 threads, every thread calls) of 4 doubles, written to
// out by thread 0..3: wave sums by shuffles, then the 4 waves in order.
__device__ __forceinline__ void block_sum4(const double (&v)[4], double *out)
{
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) red[wid][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// j and n of a thread's cells into the workgroup's slot
template <typename R>
__device__ __forceinline__ void stab_flush(const StabAcc<R> &sa, double *out)
{
    const double v[4] = {double(sa.j[0]), double(sa.j[1]), double(sa.j[2]), double(sa.n)};
    block_sum4(v, out);
}

// ------------------------------------------------------------------ collision
// TRT in deviation form: f' = f - w rho0, drho = sum f', j = sum c f'.
// Even/odd equilibrium parts of Eq. EqPDF_TRT minus w rho0:
//   feq_e' = w (drho - 3/2 rho0 u.u + 9/2 rho0 (c.u)^2),  feq_o = 3 w rho0 c.u
// lambda_e = -omega_e, lambda_o = -omega_o (Eq. LBMCollide).  With a body
// force the velocity carries +g/2 and the odd part gains (1 - omega_o/2) 3 w rho0 c.g.
// STAB: the equilibrium velocity is u - sa.ub, and j and the cell are counted.
template <typename R, bool STAB = false>
__device__ __forceinline__ void collide(R (&f)[Q], const Phys<R> &ph, R inv_rho0, StabAcc<R> *sa = nullptr)
{
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        drho += f[q];
        if (CX[q]) jx += CX[q] > 0 ? f[q] : -f[q];
        if (CY[q]) jy += CY[q] > 0 ? f[q] : -f[q];
        if (CZ[q]) jz += CZ[q] > 0 ? f[q] : -f[q];
    }
    R ux = jx * inv_rho0, uy = jy * inv_rho0, uz = jz * inv_rho0;
    if (ph.has_g) {
        ux += R(0.5) * ph.g[0];
        uy += R(0.5) * ph.g[1];
        uz += R(0.5) * ph.g[2];
    }
    if constexpr (STAB) {
        sa->j[0] += jx;
        sa->j[1] += jy;
        sa->j[2] += jz;
        sa->n += R(1);
        ux -= sa->ub[0];
        uy -= sa->ub[1];
        uz -= sa->ub[2];
    }
    const R r0 = ph.rho0, we = ph.omega_e, wo = ph.omega_o;
    const R base = drho - R(1.5) * r0 * (ux * ux + uy * uy + uz * uz);
    f[0] = f[0] - we * (f[0] - R(wq(0)) * base);
#pragma unroll
    for (int q = 1; q <= 9; ++q) {
        const R w = R(wq(q));
        const R cu = R(CX[q]) * ux + R(CY[q]) * uy + R(CZ[q]) * uz;
        const R eeq = w * (base + R(4.5) * r0 * cu * cu);
        const R oeq = R(3) * w * r0 * cu;
        const R e = R(0.5) * (f[q] + f[q + 9]);
        const R o = R(0.5) * (f[q] - f[q + 9]);
        const R de = we * (e - eeq);
        R dd = wo * (o - oeq);
        if (ph.has_g)
            dd -= (R(1) - R(0.5) * wo) * R(3) * w * r0 *
                  (R(CX[q]) * ph.g[0] + R(CY[q]) * ph.g[1] + R(CZ[q]) * ph.g[2]);
        f[q] = f[q] - de - dd;
        f[q + 9] = f[q + 9] - de + dd;
    }
}

// rigid-body velocity of fiber p at the centre of cell (cx, cy, cz):
// u_s = V + W x d with d the minimum-image vector from the centre of mass.
__device__ __forceinline__ double mi(double d, uint32_t n, bool per)
{
    if (!per) return d;
    const double h = 0.5 * double(n);
    return d > h ? d - double(n) : (d < -h ? d + double(n) : d);
}
__device__ __forceinline__ void surf_vel(const PState &s, double cx, double cy, double cz,
                                         const Geo &g, double us[3])
{
    const double dx = mi(cx - s.X[0], g.nx, true), dy = mi(cy - s.X[1], g.ny, true),
                 dz = mi(cz - s.X[2], g.nz, g.zper != 0);
    us[0] = s.V[0] + (s.W[1] * dz - s.W[2] * dy);
    us[1] = s.V[1] + (s.W[2] * dx - s.W[0] * dz);
    us[2] = s.V[2] + (s.W[0] * dy - s.W[1] * dx);
}

// ------------------------------------------------------------------ one cell
// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int I>
struct IntC {
    static constexpr int value = I;
};
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&fn)
{
    if constexpr (B < E) {
        fn(IntC<B>{});
        static_for<B + 1, E>(fn);
    }
}

// fixed-point term of the momentum-exchange sums (see fx_shift)
__device__ __forceinline__ long long fx(double v, int k) { return __double2ll_rn(ldexp(v, fx_shift(k))); }

// Momentum exchange of one link x -> y = x + c_q into fiber-local sums
// (Eq. LBMhydrodynForce and the torque after it): with r = y - X,
//   dF = 2 (f~_q + w_q rho0) c_q - 6 w_q rho0 (c_q.u_s) c_q,  dM = r x dF,
// split into the velocity-free part F0, M0 and the matrices of the part
// linear in u_s = V + W x r: A = k c c^T, B = k c (r x c)^T, C = k (r x c)(r x c)^T,
// k = 6 w_q rho0, so that F = F0 - A V - B W and M = M0 - B^T V - C W.
// This adds the link's F0, M0 terms to acc[0 .. 5]; A, B, C do not depend
// on the populations and are summed as integers when the list is built
// (link_int_terms).
template <int q>
__device__ __forceinline__ void link_terms(long long *acc, double ft, double rx, double ry, double rz,
                                           double r0)
{
    const double m2 = 2.0 * (ft + wq(q) * r0);
    const double c0 = CX[q], c1 = CY[q], c2 = CZ[q];
    const double rc0 = ry * c2 - rz * c1, rc1 = rz * c0 - rx * c2, rc2 = rx * c1 - ry * c0;
    const double t[6] = {m2 * c0, m2 * c1, m2 * c2, m2 * rc0, m2 * rc1, m2 * rc2};
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += fx(t[k], k);
}

// BND: a boundary cell of the list, whose fiber links add their F0, M0
// terms to acc[0 .. 5] (links to fiber `home`) or directly to the sums of
// another fiber.  NK: length of acc (6).
// STAB: momentum stabilization with the accumulator sa (see StabAcc).
// XYW: walls on the x and/or y faces (g.xw, g.yw) or free-slip z walls
// (g.zs).  A link leaving the lattice through a resting no-slip x or y wall
// bounces back (Eq. BBBC) into the cell's own slot opp(q) in both sweeps
// (the image cell across the periodic seam is live, so its slots cannot
// serve as a mailbox), and the odd sweep reads a population that arrives
// through such a wall from the cell's own slot; a link crossing a no-slip z
// wall as well keeps the z wall's ghost-plane mailbox.  A link that crosses
// free-slip walls only is reflected (Eq. FreeSlipBC): the components normal
// to the crossed walls reverse and the population lands on the neighbour
// along the other components, x + t.  The even sweep stores it in its own
// slot opp(q) like a streaming population; the odd sweep gathers it there
// from x + t and scatters its own reflected populations into the slot
// refl(q) of x + t, which no other cell touches in that sweep (the slot it
// gathered from for the reverse link), so both sweeps stay in place.  A
// link that crosses walls of both kinds bounces back.
template <typename S, bool ODD, bool BND, int NK = NACC, bool STAB = false, bool XYW = false>
__device__ __forceinline__ void update_cell(S *__restrict__ f, const Geo &g,
                                            const Phys<typename St<S>::R> &ph, uint32_t cell,
                                            uint32_t mask, int home, long long *acc, const BndData &b,
                                            StabAcc<typename St<S>::R> *sa = nullptr)
{
    using R = typename St<S>::R;
    const uint32_t z = fdiv(cell, g.dnxy);
    const uint32_t rr = cell - z * g.nxy;
    const uint32_t y = fdiv(rr, g.dnx);
    const uint32_t x = rr - y * g.nx;
    const uint32_t xo[3] = {x == 0 ? g.nx - 1 : x - 1, x, x + 1 == g.nx ? 0 : x + 1};
    const uint32_t yo[3] = {(y == 0 ? g.ny - 1 : y - 1) * g.nx, y * g.nx,
                            (y + 1 == g.ny ? 0 : y + 1) * g.nx};
    uint32_t zo[3];
    if (g.zper) {
        zo[0] = ((z == 0 ? g.nz - 1 : z - 1) + 1) * g.nxy;
        zo[1] = (z + 1) * g.nxy;
        zo[2] = ((z + 1 == g.nz ? 0 : z + 1) + 1) * g.nxy;
    } else {
        zo[0] = z * g.nxy;
        zo[1] = (z + 1) * g.nxy;
        zo[2] = (z + 2) * g.nxy;
    }
    const uint64_t qs = g.qstride;
    const R inv = ph.inv_scale, sc = ph.scale;
    const bool wall_lo = !g.zper && z == 0;
    const bool wall_hi = !g.zper && z + 1 == g.nz;
    bool wx0 = false, wx1 = false, wy0 = false, wy1 = false, zs = false;
    if constexpr (XYW) {
        wx0 = g.xw && x == 0;
        wx1 = g.xw && x + 1 == g.nx;
        wy0 = g.yw && y == 0;
        wy1 = g.yw && y + 1 == g.ny;
        zs = g.zs != 0;
    }
    const uint32_t own = zo[1] + yo[1] + xo[1];
    R fv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!ODD) {
            fv[q] = St<S>::ld(f, uint64_t(q) * qs + own, inv);
        } else {
            // walls crossed on the way in (a no-slip z wall: its mailbox, a normal read)
            bool ix = false, iy = false, iz = false, side_in = false;
            if constexpr (XYW) {
                ix = (CX[q] > 0 && wx0) || (CX[q] < 0 && wx1);
                iy = (CY[q] > 0 && wy0) || (CY[q] < 0 && wy1);
                iz = zs && ((CZ[q] > 0 && wall_lo) || (CZ[q] < 0 && wall_hi));
                const bool nsz = !zs && ((CZ[q] > 0 && wall_lo) || (CZ[q] < 0 && wall_hi));
                if (nsz) ix = iy = false;
                side_in = (ix && g.xw == 1) || (iy && g.yw == 1);
            }
            if (side_in) {
                fv[q] = St<S>::ld(f, uint64_t(q) * qs + own, inv);
            } else if (ix || iy || iz) {
                const int m = (ix ? 1 : 0) | (iy ? 2 : 0) | (iz ? 4 : 0);
                const uint32_t src = zo[1 - (iz ? 0 : CZ[q])] + yo[1 - (iy ? 0 : CY[q])] + xo[1 - (ix ? 0 : CX[q])];
                fv[q] = St<S>::ld(f, uint64_t(opp(refl_sel(q, m))) * qs + src, inv);
            } else {
                const uint32_t src = zo[1 - CZ[q]] + yo[1 - CY[q]] + xo[1 - CX[q]];
                fv[q] = St<S>::ld(f, uint64_t(opp(q)) * qs + src, inv);
            }
        }
    }
    collide<R, STAB>(fv, ph, R(1) / ph.rho0, sa);

    const R six_r0 = R(6) * ph.rho0;
    const PState *ps = nullptr;
    if (BND) ps = b.ps;
    static_for<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const uint32_t nb = zo[1 + CZ[q]] + yo[1 + CY[q]] + xo[1 + CX[q]];
        const bool oz = (CZ[q] < 0 && wall_lo) || (CZ[q] > 0 && wall_hi);
        const bool to_wall = oz && !zs;
        bool to_side = false, to_slip = false;
        int slip_m = 0;
        if constexpr (XYW) {
            const bool ox = (CX[q] < 0 && wx0) || (CX[q] > 0 && wx1);
            const bool oy = (CY[q] < 0 && wy0) || (CY[q] > 0 && wy1);
            to_side = !to_wall && ((ox && g.xw == 1) || (oy && g.yw == 1));
            to_slip = !to_wall && !to_side && (ox || oy || oz);
            slip_m = (ox ? 1 : 0) | (oy ? 2 : 0) | (oz ? 4 : 0);
        }
        bool to_part = false;
        if (BND) to_part = ((mask >> q) & 1u) && !to_slip;
        R out = fv[q];
        if (CX[q] != 0 && to_wall) {
            const R uw = CZ[q] < 0 ? -ph.wall_u : ph.wall_u;
            out -= six_r0 * R(wq(q)) * R(CX[q]) * uw;
        }
        if (BND && to_part && !to_side) {   // (to_part excludes reflected links)
            // moving-obstacle bounce-back (Eq. LBMMovWall) and the link's
            // momentum exchange, from the post-collision value in registers
            const int32_t p = b.pid[nb - g.nxy];
            const uint32_t yx = xo[1 + CX[q]], yy = (y + g.ny + CY[q]) % g.ny;
            const int32_t yzi = int32_t(z) + CZ[q];
            const uint32_t yz = g.zper ? uint32_t((yzi + int32_t(g.nz)) % int32_t(g.nz)) : uint32_t(yzi);
            const PState &sp = ps[p];
            const double rx = mi(double(yx) - sp.X[0], g.nx, true);
            const double ry = mi(double(yy) - sp.X[1], g.ny, true);
            const double rz = mi(double(yz) - sp.X[2], g.nz, g.zper != 0);
            const double us0 = sp.V[0] + (sp.W[1] * rz - sp.W[2] * ry);
            const double us1 = sp.V[1] + (sp.W[2] * rx - sp.W[0] * rz);
            const double us2 = sp.V[2] + (sp.W[0] * ry - sp.W[1] * rx);
            const double cu = double(CX[q]) * us0 + double(CY[q]) * us1 + double(CZ[q]) * us2;
            out -= R(6.0 * wq(q) * double(ph.rho0) * cu);
            if (!isfinite(double(fv[q]))) atomicOr(&b.ctr->err_unstable, 1u);
            if (p == home) {
                link_terms<q>(acc, double(fv[q]), rx, ry, rz, double(ph.rho0));
            } else {
                // link to another fiber (fibers closer than the region margin)
                long long tmp[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) tmp[k] = 0;
                link_terms<q>(tmp, double(fv[q]), rx, ry, rz, double(ph.rho0));
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    atomicAdd(reinterpret_cast<unsigned long long *>(b.mea + size_t(p) * NACC + k),
                              (unsigned long long)tmp[k]);
            }
        }
        const bool bounce = to_wall || to_side || to_part;
        if constexpr (STAB) {
            // a bounced link returns out in direction -c_q instead of
            // streaming fv[q] along c_q; a reflected one reverses the
            // components normal to the crossed walls
            if (bounce) {
                const R m = fv[q] + out;
                if (CX[q]) sa->j[0] -= CX[q] > 0 ? m : -m;
                if (CY[q]) sa->j[1] -= CY[q] > 0 ? m : -m;
                if (CZ[q]) sa->j[2] -= CZ[q] > 0 ? m : -m;
            } else if (to_slip) {
                const R m = fv[q] + fv[q];
                if (slip_m & 1) sa->j[0] -= CX[q] > 0 ? m : -m;
                if (slip_m & 2) sa->j[1] -= CY[q] > 0 ? m : -m;
                if (slip_m & 4) sa->j[2] -= CZ[q] > 0 ? m : -m;
            }
        }
        if (!ODD) {
            // mailbox for z walls and fibers; normal streaming, side walls
            // and reflections: own slot
            if (to_wall || (to_part && !to_side)) St<S>::st(f, uint64_t(q) * qs + nb, out, sc);
            else St<S>::st(f, uint64_t(opp(q)) * qs + own, out, sc);
        } else {
            if (to_slip) {
                const uint32_t dst = zo[1 + ((slip_m & 4) ? 0 : CZ[q])] + yo[1 + ((slip_m & 2) ? 0 : CY[q])] +
                                     xo[1 + ((slip_m & 1) ? 0 : CX[q])];
                St<S>::st(f, uint64_t(refl_sel(q, slip_m)) * qs + dst, out, sc);
            } else if (bounce) {
                St<S>::st(f, uint64_t(opp(q)) * qs + own, out, sc);
            } else {
                St<S>::st(f, uint64_t(q) * qs + nb, out, sc);
            }
        }
    });
    (void)six_r0;
    (void)home;
    (void)acc;
}


}  // namespace lbm
