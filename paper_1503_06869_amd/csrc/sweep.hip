// sweep.hip -- fused stream-collide sweep of the D3Q19 lattice (Sec. 4.1,
// Eqs. TRTOp, EqPDF_TRT, LBMCollide, LBMStream) with half-way bounce-back at
// the moving walls and at moving fiber surfaces (Eqs. BBBC, LBMMovWall),
// written for gfx950 as an in-place AA-pattern kernel over an SoA layout.
//
// Layout: f[q][zs][y][x] with x fastest; zs = z + 1 so that planes zs = 0 and
// zs = nz + 1 are ghost planes below and above the walls.  Stored value is
// the deviation f_q - w_q rho0 (scaled for FP16).
//
// AA pattern.  Even sweeps read a cell's own slots f[q][x] and write the
// post-collision value of direction q into the cell's own slot opp(q).  Odd
// sweeps gather f_q(x) from slot opp(q) of x - c_q, collide, and scatter into
// slot q of x + c_q.  Bounce-back towards a wall or fiber cell y = x + c_q:
//   even sweep: the bounced value goes to slot q of y ("mailbox"; y is a
//               ghost or fiber cell, so no other thread touches that slot);
//               the next odd gather of x reads exactly that slot.
//   odd sweep:  the bounced value goes to x's own slot opp(q), which is
//               what the next even sweep of x reads.
// With this, the odd gather is uniform (no flags needed) and every slot is
// read and written by exactly one thread of a sweep.
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

// ------------------------------------------------------------------ collision
// TRT in deviation form: f' = f - w rho0, drho = sum f', j = sum c f'.
// Even/odd equilibrium parts of Eq. EqPDF_TRT minus w rho0:
//   feq_e' = w (drho - 3/2 rho0 u.u + 9/2 rho0 (c.u)^2),  feq_o = 3 w rho0 c.u
// lambda_e = -omega_e, lambda_o = -omega_o (Eq. LBMCollide).  With a body
// force the velocity carries +g/2 and the odd part gains (1 - omega_o/2) 3 w rho0 c.g.
template <typename R>
__device__ __forceinline__ void collide(R (&f)[Q], const Phys<R> &ph, R inv_rho0)
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
template <int q>
__device__ __forceinline__ void link_terms(long long *acc, double ft, double rx, double ry, double rz,
                                           double r0)
{
    const double m2 = 2.0 * (ft + wq(q) * r0);
    const double c0 = CX[q], c1 = CY[q], c2 = CZ[q];
    const double rc0 = ry * c2 - rz * c1, rc1 = rz * c0 - rx * c2, rc2 = rx * c1 - ry * c0;
    const double k6 = 6.0 * wq(q) * r0;
    const double t[NACC] = {m2 * c0, m2 * c1, m2 * c2, m2 * rc0, m2 * rc1, m2 * rc2,
                            k6 * c0 * c0, k6 * c0 * c1, k6 * c0 * c2, k6 * c1 * c1, k6 * c1 * c2, k6 * c2 * c2,
                            k6 * c0 * rc0, k6 * c0 * rc1, k6 * c0 * rc2,
                            k6 * c1 * rc0, k6 * c1 * rc1, k6 * c1 * rc2,
                            k6 * c2 * rc0, k6 * c2 * rc1, k6 * c2 * rc2,
                            k6 * rc0 * rc0, k6 * rc0 * rc1, k6 * rc0 * rc2,
                            k6 * rc1 * rc1, k6 * rc1 * rc2, k6 * rc2 * rc2};
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] += fx(t[k], k);
}

template <typename S, bool ODD, bool BND>
__device__ __forceinline__ void update_cell(S *__restrict__ f, const Geo &g,
                                            const Phys<typename St<S>::R> &ph, uint32_t cell,
                                            uint32_t mask, int home, long long *acc, const BndData &b)
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
    R fv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!ODD) {
            fv[q] = St<S>::ld(f, uint64_t(q) * qs + zo[1] + yo[1] + xo[1], inv);
        } else {
            const uint32_t src = zo[1 - CZ[q]] + yo[1 - CY[q]] + xo[1 - CX[q]];
            fv[q] = St<S>::ld(f, uint64_t(opp(q)) * qs + src, inv);
        }
    }
    collide<R>(fv, ph, R(1) / ph.rho0);

    const bool wall_lo = !g.zper && z == 0;
    const bool wall_hi = !g.zper && z + 1 == g.nz;
    const uint32_t own = zo[1] + yo[1] + xo[1];
    const R six_r0 = R(6) * ph.rho0;
    const PState *ps = nullptr;
    if (BND) ps = b.ps;
    static_for<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const uint32_t nb = zo[1 + CZ[q]] + yo[1 + CY[q]] + xo[1 + CX[q]];
        const bool to_wall = (CZ[q] < 0 && wall_lo) || (CZ[q] > 0 && wall_hi);
        bool to_part = false;
        if (BND) to_part = (mask >> q) & 1u;
        R out = fv[q];
        if (CX[q] != 0 && to_wall) {
            const R uw = CZ[q] < 0 ? -ph.wall_u : ph.wall_u;
            out -= six_r0 * R(wq(q)) * R(CX[q]) * uw;
        }
        if (BND && to_part) {
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
                long long tmp[NACC];
#pragma unroll
                for (int k = 0; k < NACC; ++k) tmp[k] = 0;
                link_terms<q>(tmp, double(fv[q]), rx, ry, rz, double(ph.rho0));
#pragma unroll
                for (int k = 0; k < NACC; ++k)
                    atomicAdd(reinterpret_cast<unsigned long long *>(b.mea + size_t(p) * NACC + k),
                              (unsigned long long)tmp[k]);
            }
        }
        const bool bounce = to_wall || to_part;
        if (!ODD) {
            if (bounce) St<S>::st(f, uint64_t(q) * qs + nb, out, sc);
            else St<S>::st(f, uint64_t(opp(q)) * qs + own, out, sc);
        } else {
            if (bounce) St<S>::st(f, uint64_t(opp(q)) * qs + own, out, sc);
            else St<S>::st(f, uint64_t(q) * qs + nb, out, sc);
        }
    });
    (void)six_r0;
    (void)home;
    (void)acc;
}

// Grid-stride over 256-cell chunks: at any time the resident workgroups work
// on one compact band of the lattice, which keeps each of the 38 access
// streams (19 directions read, 19 written) within a few DRAM pages.
template <typename S, bool ODD>
__global__ __launch_bounds__(256) void k_sweep_bulk(S *__restrict__ f, const uint8_t *__restrict__ flags,
                                                    Geo g, Phys<typename St<S>::R> ph)
{
    const uint32_t nchunk = (g.ncell + 255u) >> 8;
    for (uint32_t ch = xcd_block(blockIdx.x, gridDim.x); ch < nchunk; ch += gridDim.x) {
        const uint32_t cell = (ch << 8) + threadIdx.x;
        if (cell < g.ncell && !flags[cell])   // fiber cells idle; boundary cells: k_sweep_bnd
            update_cell<S, ODD, false>(f, g, ph, cell, 0u, -1, nullptr, BndData{});
    }
}

template <typename S, bool ODD>
__global__ __launch_bounds__(256) void k_sweep_bnd(S *__restrict__ f, Geo g,
                                                   Phys<typename St<S>::R> ph, BndData b)
{
    // block (fiber p, part j) of the fiber's list segment
    const int p = blockIdx.x / b.bpf, j = blockIdx.x % b.bpf;
    const uint32_t cnt = b.seg_cnt[p], cap = b.seg_cap[p];
    const uint32_t n = cnt < cap ? cnt : cap, off = b.seg_off[p];
    long long acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0;
    for (uint32_t r = j * 256u + threadIdx.x; r < n; r += b.bpf * 256u) {
        const uint32_t e = off + r;
        update_cell<S, ODD, true>(f, g, ph, b.cell[e], b.mask[e], p, acc, b);
    }
    // integer sums: exact, so the reduction order does not matter
    __shared__ long long red[4][NACC];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        long long v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NACC) {
        const int k = threadIdx.x;
        const long long v = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        if (v) atomicAdd(reinterpret_cast<unsigned long long *>(b.mea + size_t(p) * NACC + k),
                         (unsigned long long)v);
    }
}

// ------------------------------------------------------------------ init
// f = f_eq(rho0, u0(z)) (Eq. fequ_Incompr), stored as deviation, natural slots.
template <typename S>
__global__ void k_init(S *__restrict__ f, Geo g, double rho0, double wall_u, int couette,
                       double scale)
{
    const uint64_t total = g.qstride;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t zs = uint32_t(i / g.nxy);
        const bool ghost = zs == 0 || zs == g.nz + 1;
        double ux = 0.0;
        if (couette && !g.zper && !ghost) ux = wall_u * (2.0 * (double(zs - 1) + 0.5) / g.nz - 1.0);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double cu = CX[q] * ux;
            const double dev = ghost ? 0.0 : wq(q) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);
            St<S>::st(f, uint64_t(q) * g.qstride + i, typename St<S>::R(dev), typename St<S>::R(scale));
        }
    }
}

// ------------------------------------------------------------------ decode / encode
template <typename S>
__global__ void k_decode(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                         const int32_t *__restrict__ pid, const PState *__restrict__ ps, Geo g,
                         Phys<double> ph, int swapped, typename St<S>::R *rho,
                         typename St<S>::R *u, double *fout)
{
    using R = typename St<S>::R;
    for (uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x; cell < g.ncell;
         cell += gridDim.x * blockDim.x) {
        const uint32_t z = cell / g.nxy, y = (cell % g.nxy) / g.nx, x = cell % g.nx;
        double fv[Q];
        for (int q = 0; q < Q; ++q) {
            uint32_t src = (z + 1) * g.nxy + y * g.nx + x;
            int qq = q;
            if (swapped) {
                const uint32_t sx = (x + g.nx - CX[q]) % g.nx, sy = (y + g.ny - CY[q]) % g.ny;
                const int32_t szi = int32_t(z) - CZ[q];
                const uint32_t szs = g.zper ? uint32_t((szi + int32_t(g.nz)) % int32_t(g.nz)) + 1
                                            : uint32_t(szi + 1);
                src = szs * g.nxy + sy * g.nx + sx;
                qq = opp(q);
            }
            fv[q] = double(St<S>::ld(f, uint64_t(qq) * g.qstride + src, R(ph.inv_scale)));
        }
        const bool solid = flags[cell] & F_SOLID;
        double r = ph.rho0, uu[3] = {0.0, 0.0, 0.0};
        if (solid) {
            surf_vel(ps[pid[cell]], double(x), double(y), double(z), g, uu);
        } else {
            double dr = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int q = 0; q < Q; ++q) {
                dr += fv[q];
                j[0] += CX[q] * fv[q];
                j[1] += CY[q] * fv[q];
                j[2] += CZ[q] * fv[q];
            }
            r = ph.rho0 + dr;
            for (int k = 0; k < 3; ++k) uu[k] = j[k] / ph.rho0 + 0.5 * ph.g[k];
        }
        if (rho) rho[cell] = R(r);
        if (u)
            for (int k = 0; k < 3; ++k) u[uint64_t(k) * g.ncell + cell] = R(uu[k]);
        if (fout)
            for (int q = 0; q < Q; ++q) fout[uint64_t(q) * g.ncell + cell] = fv[q] + wq(q) * ph.rho0;
    }
}

template <typename S>
__global__ void k_encode(S *__restrict__ f, Geo g, double rho0, double scale, int swapped,
                         const double *__restrict__ fin)
{
    for (uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x; cell < g.ncell;
         cell += gridDim.x * blockDim.x) {
        const uint32_t z = cell / g.nxy, y = (cell % g.nxy) / g.nx, x = cell % g.nx;
        for (int q = 0; q < Q; ++q) {
            uint32_t dst = (z + 1) * g.nxy + y * g.nx + x;
            int qq = q;
            if (swapped) {
                const uint32_t sx = (x + g.nx - CX[q]) % g.nx, sy = (y + g.ny - CY[q]) % g.ny;
                const int32_t szi = int32_t(z) - CZ[q];
                const uint32_t szs = g.zper ? uint32_t((szi + int32_t(g.nz)) % int32_t(g.nz)) + 1
                                            : uint32_t(szi + 1);
                dst = szs * g.nxy + sy * g.nx + sx;
                qq = opp(q);
            }
            const double dev = fin[uint64_t(q) * g.ncell + cell] - wq(q) * rho0;
            St<S>::st(f, uint64_t(qq) * g.qstride + dst, typename St<S>::R(dev),
                      typename St<S>::R(scale));
        }
    }
}

// ------------------------------------------------------------------ copy reference
__global__ __launch_bounds__(256) void k_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                              uint64_t n16)
{
    for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n16;
         i += uint64_t(gridDim.x) * 256)
        dst[i] = src[i];
}

// ------------------------------------------------------------------ launchers
template <typename R>
static Phys<R> cast_phys(const Phys<double> &p)
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

template <typename S>
static hipError_t sweep_t(bool odd, void *f, const uint8_t *flags, const Geo &g,
                          const Phys<double> &ph, const BndData &b, uint32_t sweep_grid,
                          uint32_t bnd_grid, hipStream_t st, hipStream_t st_bnd, hipEvent_t ev0,
                          hipEvent_t ev1)
{
    using R = typename St<S>::R;
    const Phys<R> p = cast_phys<R>(ph);
    if (sweep_grid) {
        if (ev0) hipEventRecord(ev0, st);
        if (odd)
            hipLaunchKernelGGL((k_sweep_bulk<S, true>), dim3(sweep_grid), dim3(256), 0, st, (S *)f, flags, g, p);
        else
            hipLaunchKernelGGL((k_sweep_bulk<S, false>), dim3(sweep_grid), dim3(256), 0, st, (S *)f, flags, g, p);
        if (ev1) hipEventRecord(ev1, st);
    }
    if (bnd_grid) {
        bnd_grid = uint32_t(b.np * b.bpf);
        if (odd)
            hipLaunchKernelGGL((k_sweep_bnd<S, true>), dim3(bnd_grid), dim3(256), 0, st_bnd, (S *)f, g, p, b);
        else
            hipLaunchKernelGGL((k_sweep_bnd<S, false>), dim3(bnd_grid), dim3(256), 0, st_bnd, (S *)f, g, p, b);
    }
    return hipGetLastError();
}

hipError_t launch_sweep(int sk, bool odd, void *f, const uint8_t *flags, const Geo &g,
                        const Phys<double> &ph, const BndData &b, uint32_t sweep_grid,
                        uint32_t bnd_grid, hipStream_t st, hipStream_t st_bnd, hipEvent_t ev0,
                        hipEvent_t ev1)
{
    switch (sk) {
    case S_F32: return sweep_t<float>(odd, f, flags, g, ph, b, sweep_grid, bnd_grid, st, st_bnd, ev0, ev1);
    case S_F16: return sweep_t<_Float16>(odd, f, flags, g, ph, b, sweep_grid, bnd_grid, st, st_bnd, ev0, ev1);
    case S_BF16: return sweep_t<bf16s>(odd, f, flags, g, ph, b, sweep_grid, bnd_grid, st, st_bnd, ev0, ev1);
    default: return sweep_t<double>(odd, f, flags, g, ph, b, sweep_grid, bnd_grid, st, st_bnd, ev0, ev1);
    }
}

static uint32_t grid_for(uint64_t n, uint32_t bs) { return uint32_t(n / bs + 1 < 65536 ? n / bs + 1 : 65536); }

hipError_t launch_init(int sk, void *f, const Geo &g, double rho0, double wall_u, int couette,
                       double scale, hipStream_t st)
{
    const uint32_t gr = grid_for(g.qstride, 256);
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_init<float>, dim3(gr), dim3(256), 0, st, (float *)f, g, rho0, wall_u, couette, scale); break;
    case S_F16: hipLaunchKernelGGL(k_init<_Float16>, dim3(gr), dim3(256), 0, st, (_Float16 *)f, g, rho0, wall_u, couette, scale); break;
    case S_BF16: hipLaunchKernelGGL(k_init<bf16s>, dim3(gr), dim3(256), 0, st, (bf16s *)f, g, rho0, wall_u, couette, scale); break;
    default: hipLaunchKernelGGL(k_init<double>, dim3(gr), dim3(256), 0, st, (double *)f, g, rho0, wall_u, couette, scale); break;
    }
    return hipGetLastError();
}

hipError_t launch_decode(int sk, bool swapped, const void *f, const uint8_t *flags,
                         const int32_t *pid, const PState *ps, const Geo &g, const Phys<double> &ph,
                         void *rho, void *u, double *fout, hipStream_t st)
{
    const uint32_t gr = grid_for(g.ncell, 256);
    const int sw = swapped ? 1 : 0;
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_decode<float>, dim3(gr), dim3(256), 0, st, (const float *)f, flags, pid, ps, g, ph, sw, (float *)rho, (float *)u, fout); break;
    case S_F16: hipLaunchKernelGGL(k_decode<_Float16>, dim3(gr), dim3(256), 0, st, (const _Float16 *)f, flags, pid, ps, g, ph, sw, (float *)rho, (float *)u, fout); break;
    case S_BF16: hipLaunchKernelGGL(k_decode<bf16s>, dim3(gr), dim3(256), 0, st, (const bf16s *)f, flags, pid, ps, g, ph, sw, (float *)rho, (float *)u, fout); break;
    default: hipLaunchKernelGGL(k_decode<double>, dim3(gr), dim3(256), 0, st, (const double *)f, flags, pid, ps, g, ph, sw, (double *)rho, (double *)u, fout); break;
    }
    return hipGetLastError();
}

hipError_t launch_encode(int sk, bool swapped, void *f, const Geo &g, double rho0, double scale,
                         const double *fin, hipStream_t st)
{
    const uint32_t gr = grid_for(g.ncell, 256);
    const int sw = swapped ? 1 : 0;
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_encode<float>, dim3(gr), dim3(256), 0, st, (float *)f, g, rho0, scale, sw, fin); break;
    case S_F16: hipLaunchKernelGGL(k_encode<_Float16>, dim3(gr), dim3(256), 0, st, (_Float16 *)f, g, rho0, scale, sw, fin); break;
    case S_BF16: hipLaunchKernelGGL(k_encode<bf16s>, dim3(gr), dim3(256), 0, st, (bf16s *)f, g, rho0, scale, sw, fin); break;
    default: hipLaunchKernelGGL(k_encode<double>, dim3(gr), dim3(256), 0, st, (double *)f, g, rho0, scale, sw, fin); break;
    }
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t nbytes, hipStream_t st)
{
    const uint64_t n16 = nbytes / 16;
    if (n16 == 0) return hipSuccess;
    const uint32_t gr = uint32_t(n16 / 256 + 1 < 8192 ? n16 / 256 + 1 : 8192);
    hipLaunchKernelGGL(k_copy, dim3(gr), dim3(256), 0, st, (uint4 *)dst, (const uint4 *)src, n16);
    return hipGetLastError();
}

}  // namespace lbm
