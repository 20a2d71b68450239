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
#include "lbm_sweep_dev.h"

namespace lbm {

// Grid-stride over 256-cell chunks: at any time the resident workgroups work
// on one compact band of the lattice, which keeps each of the 38 access
// streams (19 directions read, 19 written) within a few DRAM pages.
// STAB: momentum stabilization; stab[0..2] is the mean velocity the
// collisions subtract, and workgroup b writes its sums to part[4 b .. 4 b + 3].
// XYW: walls on the x and/or y faces.
template <typename S, bool ODD, bool STAB, bool XYW>
__global__ __launch_bounds__(256) void k_sweep_bulk(S *__restrict__ f, const uint8_t *__restrict__ flags,
                                                    Geo g, Phys<typename St<S>::R> ph, const double *stab,
                                                    double *part)
{
    using R = typename St<S>::R;
    StabAcc<R> sa;
    if constexpr (STAB) stab_begin(sa, stab);
    const uint32_t nchunk = (g.ncell + 255u) >> 8;
    for (uint32_t ch = xcd_block(blockIdx.x, gridDim.x); ch < nchunk; ch += gridDim.x) {
        const uint32_t cell = (ch << 8) + threadIdx.x;
        if (cell < g.ncell && !flags[cell])   // fiber cells idle; boundary cells: k_boundary
            update_cell<S, ODD, false, NACC, STAB, XYW>(f, g, ph, cell, 0u, -1, nullptr, BndData{}, &sa);
    }
    if constexpr (STAB) stab_flush(sa, part + 4 * size_t(blockIdx.x));
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
// Cells [c0, c1) of the lattice; rho and u are written at cell - c0 (u's
// components ustride apart), fout (all cells, c0 = 0) at the cell index.
template <typename S>
__global__ void k_decode(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                         const int32_t *__restrict__ pid, const PState *__restrict__ ps, Geo g,
                         Phys<double> ph, int swapped, typename St<S>::R *rho,
                         typename St<S>::R *u, double *fout, uint32_t c0, uint32_t c1,
                         uint64_t ustride)
{
    using R = typename St<S>::R;
    for (uint32_t cell = c0 + blockIdx.x * blockDim.x + threadIdx.x; cell < c1;
         cell += gridDim.x * blockDim.x) {
        const uint32_t z = cell / g.nxy, y = (cell % g.nxy) / g.nx, x = cell % g.nx;
        double fv[Q];
        for (int q = 0; q < Q; ++q) {
            uint32_t src = (z + 1) * g.nxy + y * g.nx + x;
            int qq = q;
            if (swapped) src = swapped_src(g, x, y, z, q, qq);
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
        if (rho) rho[cell - c0] = R(r);
        if (u)
            for (int k = 0; k < 3; ++k) u[uint64_t(k) * ustride + (cell - c0)] = R(uu[k]);
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
            if (swapped) dst = swapped_src(g, x, y, z, q, qq);
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
template <typename S>
static hipError_t sweep_t(bool odd, void *f, const uint8_t *flags, const Geo &g, const Phys<double> &ph,
                          uint32_t sweep_grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                          const double *stab, double *part)
{
    using R = typename St<S>::R;
    const Phys<R> p = cast_phys<R>(ph);
    if (!sweep_grid) return hipSuccess;
    if (ev0) hipEventRecord(ev0, st);
    const dim3 gr(sweep_grid), bl(256);
    const int mode = (odd ? 1 : 0) | (stab ? 2 : 0) | ((g.xw || g.yw || g.zs) ? 4 : 0);
    switch (mode) {
    case 0: hipLaunchKernelGGL((k_sweep_bulk<S, false, false, false>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    case 1: hipLaunchKernelGGL((k_sweep_bulk<S, true, false, false>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    case 2: hipLaunchKernelGGL((k_sweep_bulk<S, false, true, false>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    case 3: hipLaunchKernelGGL((k_sweep_bulk<S, true, true, false>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    case 4: hipLaunchKernelGGL((k_sweep_bulk<S, false, false, true>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    case 5: hipLaunchKernelGGL((k_sweep_bulk<S, true, false, true>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    case 6: hipLaunchKernelGGL((k_sweep_bulk<S, false, true, true>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    default: hipLaunchKernelGGL((k_sweep_bulk<S, true, true, true>), gr, bl, 0, st, (S *)f, flags, g, p, stab, part); break;
    }
    if (ev1) hipEventRecord(ev1, st);
    return hipGetLastError();
}

hipError_t launch_sweep(int sk, bool odd, void *f, const uint8_t *flags, const Geo &g, const Phys<double> &ph,
                        uint32_t sweep_grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, const double *stab,
                        double *part)
{
    switch (sk) {
    case S_F32: return sweep_t<float>(odd, f, flags, g, ph, sweep_grid, st, ev0, ev1, stab, part);
    case S_F16: return sweep_t<_Float16>(odd, f, flags, g, ph, sweep_grid, st, ev0, ev1, stab, part);
    case S_BF16: return sweep_t<bf16s>(odd, f, flags, g, ph, sweep_grid, st, ev0, ev1, stab, part);
    default: return sweep_t<double>(odd, f, flags, g, ph, sweep_grid, st, ev0, ev1, stab, part);
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

hipError_t launch_decode_range(int sk, bool swapped, const void *f, const uint8_t *flags,
                               const int32_t *pid, const PState *ps, const Geo &g,
                               const Phys<double> &ph, void *rho, void *u, double *fout,
                               uint32_t c0, uint32_t c1, uint64_t ustride, hipStream_t st)
{
    if (c1 <= c0) return hipSuccess;
    const uint32_t gr = grid_for(c1 - c0, 256);
    const int sw = swapped ? 1 : 0;
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_decode<float>, dim3(gr), dim3(256), 0, st, (const float *)f, flags, pid, ps, g, ph, sw, (float *)rho, (float *)u, fout, c0, c1, ustride); break;
    case S_F16: hipLaunchKernelGGL(k_decode<_Float16>, dim3(gr), dim3(256), 0, st, (const _Float16 *)f, flags, pid, ps, g, ph, sw, (float *)rho, (float *)u, fout, c0, c1, ustride); break;
    case S_BF16: hipLaunchKernelGGL(k_decode<bf16s>, dim3(gr), dim3(256), 0, st, (const bf16s *)f, flags, pid, ps, g, ph, sw, (float *)rho, (float *)u, fout, c0, c1, ustride); break;
    default: hipLaunchKernelGGL(k_decode<double>, dim3(gr), dim3(256), 0, st, (const double *)f, flags, pid, ps, g, ph, sw, (double *)rho, (double *)u, fout, c0, c1, ustride); break;
    }
    return hipGetLastError();
}

hipError_t launch_decode(int sk, bool swapped, const void *f, const uint8_t *flags,
                         const int32_t *pid, const PState *ps, const Geo &g, const Phys<double> &ph,
                         void *rho, void *u, double *fout, hipStream_t st)
{
    return launch_decode_range(sk, swapped, f, flags, pid, ps, g, ph, rho, u, fout, 0, g.ncell,
                               g.ncell, st);
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
