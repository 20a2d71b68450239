// boundary.hip -- the boundary-list work of one time step, in one launch:
//   blocks [0, np*bpf)        update of the boundary cells (the fused
//                             stream-collide of the bulk sweep with the
//                             moving-obstacle bounce-back, Eq. LBMMovWall)
//                             and the population-dependent momentum-exchange
//                             sums F0, M0 of their fiber links (Eq.
//                             LBMhydrodynForce and the torque after it);
//   blocks [np*bpf, 2*np*bpf) the population-free sums A, B, C of the same
//                             links at the current poses (the part of the
//                             exchange linear in the surface velocity).
// Both halves walk the same list segments (block (fiber p, part j)) and add
// into disjoint slots of the fixed-point sums, so they run side by side; one
// launch keeps them concurrent wherever the step's graph puts it.
#include "lbm_sweep_dev.h"

namespace lbm {

template <typename S, bool ODD, bool STAB, bool XYW>
__device__ __forceinline__ void bnd_block(S *__restrict__ f, const Geo &g, const Phys<typename St<S>::R> &ph,
                                          const BndData &b, int blk, const double *stab, double *part)
{
    // block (fiber p, part j) of the fiber's list segment
    const int p = blk / b.bpf, j = blk % b.bpf;
    const uint32_t cnt = b.seg_cnt[p], cap = b.seg_cap[p];
    const uint32_t n = cnt < cap ? cnt : cap, off = b.seg_off[p];
    long long acc[6] = {0, 0, 0, 0, 0, 0};
    StabAcc<typename St<S>::R> sa;
    if constexpr (STAB) stab_begin(sa, stab);
    for (uint32_t r = j * 256u + threadIdx.x; r < n; r += b.bpf * 256u) {
        const uint32_t e = off + r;
        update_cell<S, ODD, true, 6, STAB, XYW>(f, g, ph, b.cell[e], b.mask[e], p, acc, b, &sa);
    }
    if constexpr (STAB) stab_flush(sa, part + 4 * size_t(blk));
    // integer sums: exact, so the reduction order does not matter
    __shared__ long long red[4][6];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        long long v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        const long long v = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        if (v) atomicAdd(reinterpret_cast<unsigned long long *>(b.mea + size_t(p) * NACC + k),
                         (unsigned long long)v);
    }
}

}  // namespace lbm

// the particle-side arithmetic below follows the header's contraction-off
// pragma, like the rest of the per-fiber code
#include "lbm_particle_dev.h"

namespace lbm {

// Terms 6..26 of the momentum exchange (A, B, C) of every link of a boundary
// cell at the poses ps of the sweep, added to acc for links to fiber home and
// with atomics for links to another fiber.  The neighbour coordinates and
// lever arm are formed as in the sweep; the owners across all links are
// loaded together first, the home pose is passed in.
__device__ __forceinline__ void abc_links(uint32_t cell, uint32_t mask, const int32_t *pid, const PState *ps,
                                          const double hX[3], long long *mea, const Geo &g, int home, double r0,
                                          long long (&acc)[NABC])
{
    const uint32_t z = cell / g.nxy, rem = cell - z * g.nxy, y = rem / g.nx, x = rem - y * g.nx;
    // far cell of link q (periodic x, y; z periodic or walled)
    auto far = [&](auto qc, uint32_t &yx, uint32_t &yy, uint32_t &yz) {
        constexpr int q = decltype(qc)::value;
        yx = uint32_t(wrapc(int32_t(x) + CX[q], int32_t(g.nx)));
        yy = uint32_t(wrapc(int32_t(y) + CY[q], int32_t(g.ny)));
        const int32_t yzi = int32_t(z) + CZ[q];
        yz = g.zper ? uint32_t(wrapc(yzi, int32_t(g.nz))) : uint32_t(yzi);
    };
    int32_t own[Q];
    static_for<1, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        uint32_t yx, yy, yz;
        far(qc, yx, yy, yz);
        own[q] = pid[((mask >> q) & 1u) ? (yz * g.ny + yy) * g.nx + yx : cell];
    });
    static_for<1, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if ((mask >> q) & 1u) {
            uint32_t yx, yy, yz;
            far(qc, yx, yy, yz);
            const int o = own[q];
            double sX[3];
            if (o == home) {
                for (int k = 0; k < 3; ++k) sX[k] = hX[k];
            } else {
                for (int k = 0; k < 3; ++k) sX[k] = ps[o].X[k];
            }
            const double rx = mi(double(yx) - sX[0], g.nx, true);
            const double ry = mi(double(yy) - sX[1], g.ny, true);
            const double rz = mi(double(yz) - sX[2], g.nz, g.zper != 0);
            if (o == home) {
                link_terms<q, 6, NACC>(acc, 0.0, rx, ry, rz, r0);
            } else {
                long long tmp[NABC];
#pragma unroll
                for (int k = 0; k < NABC; ++k) tmp[k] = 0;
                link_terms<q, 6, NACC>(tmp, 0.0, rx, ry, rz, r0);
#pragma unroll
                for (int k = 0; k < NABC; ++k)
                    atomicAdd(reinterpret_cast<unsigned long long *>(mea + size_t(o) * NACC + 6 + k),
                              (unsigned long long)tmp[k]);
            }
        }
    });
}

// A, B, C of the current list at the current poses: block (fiber p, part j)
// of the fiber's list segment, as in the boundary update.
__device__ __forceinline__ void abc_block(const BndData &b, const Geo &g, double r0, int blk)
{
    const int p = blk / b.bpf, j = blk % b.bpf;
    const uint32_t cnt = b.seg_cnt[p], cap = b.seg_cap[p];
    const uint32_t n = cnt < cap ? cnt : cap, off = b.seg_off[p];
    long long acc[NABC];
#pragma unroll
    for (int k = 0; k < NABC; ++k) acc[k] = 0;
    const double hX[3] = {b.ps[p].X[0], b.ps[p].X[1], b.ps[p].X[2]};
    for (uint32_t r = j * 256u + threadIdx.x; r < n; r += b.bpf * 256u)
        abc_links(b.cell[off + r], b.mask[off + r], b.pid, b.ps, hX, b.mea, g, p, r0, acc);
    __shared__ long long red[4][NABC];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NABC; ++k) {
        long long v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NABC) {
        const int k = threadIdx.x;
        const long long v = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        if (v) atomicAdd(reinterpret_cast<unsigned long long *>(b.mea + size_t(p) * NACC + 6 + k),
                         (unsigned long long)v);
    }
}

// Register budget: the bulk sweep keeps 2 waves of 80 VGPRs per SIMD
// resident for its whole grid-stride run; this kernel runs beside it with
// up to 2 waves per SIMD, so it must stay within 176 VGPRs (171 for FP32),
// or bulk workgroups launched after it start late and the sweep stretches.
// STAB: momentum stabilization (mean velocity stab[0..2]; the boundary-cell
// workgroup blk writes its sums to part[4 blk .. 4 blk + 3]).  XYW: walls on
// the x and/or y faces.
template <typename S, bool ODD, bool STAB, bool XYW>
__global__ __launch_bounds__(256) void k_boundary(S *__restrict__ f, Geo g, Phys<typename St<S>::R> ph,
                                                  BndData b, double r0, const double *stab, double *part)
{
    const int nb = b.np * b.bpf;   // block-uniform split
    if (int(blockIdx.x) < nb) bnd_block<S, ODD, STAB, XYW>(f, g, ph, b, int(blockIdx.x), stab, part);
    else abc_block(b, g, r0, int(blockIdx.x) - nb);
}

template <typename S>
static hipError_t boundary_t(bool odd, void *f, const Geo &g, const Phys<double> &ph, const BndData &b,
                             double r0, hipStream_t st, const double *stab, double *part)
{
    using R = typename St<S>::R;
    const Phys<R> p = cast_phys<R>(ph);
    const dim3 grid(uint32_t(2 * b.np * b.bpf)), bl(256);
    const int mode = (odd ? 1 : 0) | (stab ? 2 : 0) | ((g.xw || g.yw) ? 4 : 0);
    switch (mode) {
    case 0: hipLaunchKernelGGL((k_boundary<S, false, false, false>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    case 1: hipLaunchKernelGGL((k_boundary<S, true, false, false>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    case 2: hipLaunchKernelGGL((k_boundary<S, false, true, false>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    case 3: hipLaunchKernelGGL((k_boundary<S, true, true, false>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    case 4: hipLaunchKernelGGL((k_boundary<S, false, false, true>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    case 5: hipLaunchKernelGGL((k_boundary<S, true, false, true>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    case 6: hipLaunchKernelGGL((k_boundary<S, false, true, true>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    default: hipLaunchKernelGGL((k_boundary<S, true, true, true>), grid, bl, 0, st, (S *)f, g, p, b, r0, stab, part); break;
    }
    return hipGetLastError();
}

hipError_t launch_boundary(int sk, bool odd, void *f, const Geo &g, const Phys<double> &ph, const BndData &b,
                           double r0, hipStream_t st, const double *stab, double *part)
{
    if (b.np <= 0 || b.bpf <= 0) return hipSuccess;
    switch (sk) {
    case S_F32: return boundary_t<float>(odd, f, g, ph, b, r0, st, stab, part);
    case S_F16: return boundary_t<_Float16>(odd, f, g, ph, b, r0, st, stab, part);
    case S_BF16: return boundary_t<bf16s>(odd, f, g, ph, b, r0, st, stab, part);
    default: return boundary_t<double>(odd, f, g, ph, b, r0, st, stab, part);
    }
}

}  // namespace lbm
