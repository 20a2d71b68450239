// boundary.hip -- the boundary-list work of one time step, in one launch:
//   blocks [0, np*bpf)        update of the boundary cells (the fused
//                             stream-collide of the bulk sweep with the
//                             moving-obstacle bounce-back, Eq. LBMMovWall)
//                             and the population-dependent momentum-exchange
//                             sums F0, M0 of their fiber links (Eq.
//                             LBMhydrodynForce and the torque after it);
//   blocks [np*bpf, 2*np*bpf) the population-free part of the exchange (A,
//                             B, C; linear in the surface velocity) of the
//                             same links as exact integer sums at the
//                             current poses (see abc_restore).
// Both halves walk the same list segments (block (fiber p, part j)) and add
// into disjoint slots of the sums, so they run side by side.
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

// integer index arithmetic of the particle side (shared with the list rebuild)
#include "lbm_particle_dev.h"

namespace lbm {

// The integer sums SA, SB, SC of every link of a list segment's part j at
// the poses ps (links to fiber p into the block's sums, links to another
// fiber with atomics into that fiber's): block (fiber p, part j).
__device__ __forceinline__ void abc_block(const BndData &b, const Geo &g, int blk)
{
    const int p = blk / b.bpf, j = blk % b.bpf;
    const uint32_t cnt = b.seg_cnt[p], cap = b.seg_cap[p];
    const uint32_t n = cnt < cap ? cnt : cap, off = b.seg_off[p];
    long long acc[NABC];
#pragma unroll
    for (int k = 0; k < NABC; ++k) acc[k] = 0;
    int32_t hr[3];
    fiber_ref(b.ps[p].X, hr);
    for (uint32_t r = j * 256u + threadIdx.x; r < n; r += b.bpf * 256u) {
        const uint32_t cell = b.cell[off + r], mask = b.mask[off + r];
        const int32_t z = int32_t(cell / g.nxy), rem = int32_t(cell - uint32_t(z) * g.nxy);
        const int32_t y = rem / int32_t(g.nx), x = rem - y * int32_t(g.nx);
        int32_t own[Q];
        fiber_links(b.pid, g, x, y, z, own);
        static_for<1, Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if ((mask >> q) & 1u) {
                const int o = own[q];
                int32_t rf[3] = {hr[0], hr[1], hr[2]};
                if (o != p) fiber_ref(b.ps[o].X, rf);
                const int32_t yx = wrapc(x + CX[q], int32_t(g.nx)), yy = wrapc(y + CY[q], int32_t(g.ny));
                const int32_t yz = g.zper ? wrapc(z + CZ[q], int32_t(g.nz)) : z + CZ[q];
                const int32_t sx = mi_i(yx - rf[0], int32_t(g.nx), true);
                const int32_t sy = mi_i(yy - rf[1], int32_t(g.ny), true);
                const int32_t sz = mi_i(yz - rf[2], int32_t(g.nz), g.zper != 0);
                if (o == p) {
                    link_int_terms<q>(acc, sx, sy, sz);
                } else {
                    // link to another fiber (fibers closer than the region margin)
                    long long tmp[NABC];
#pragma unroll
                    for (int k = 0; k < NABC; ++k) tmp[k] = 0;
                    link_int_terms<q>(tmp, sx, sy, sz);
#pragma unroll
                    for (int k = 0; k < NABC; ++k)
                        if (tmp[k])
                            atomicAdd(reinterpret_cast<unsigned long long *>(b.mea + size_t(o) * NACC + 6 + k),
                                      (unsigned long long)tmp[k]);
                }
            }
        });
    }
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
                                                  BndData b, const double *stab, double *part)
{
    const int nb = b.np * b.bpf;   // block-uniform split
    if (int(blockIdx.x) < nb) bnd_block<S, ODD, STAB, XYW>(f, g, ph, b, int(blockIdx.x), stab, part);
    else abc_block(b, g, int(blockIdx.x) - nb);
}

template <typename S>
static hipError_t boundary_t(bool odd, void *f, const Geo &g, const Phys<double> &ph, const BndData &b,
                             hipStream_t st, const double *stab, double *part)
{
    using R = typename St<S>::R;
    const Phys<R> p = cast_phys<R>(ph);
    const dim3 grid(uint32_t(2 * b.np * b.bpf)), bl(256);
    const int mode = (odd ? 1 : 0) | (stab ? 2 : 0) | ((g.xw || g.yw || g.zs) ? 4 : 0);
    switch (mode) {
    case 0: hipLaunchKernelGGL((k_boundary<S, false, false, false>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    case 1: hipLaunchKernelGGL((k_boundary<S, true, false, false>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    case 2: hipLaunchKernelGGL((k_boundary<S, false, true, false>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    case 3: hipLaunchKernelGGL((k_boundary<S, true, true, false>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    case 4: hipLaunchKernelGGL((k_boundary<S, false, false, true>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    case 5: hipLaunchKernelGGL((k_boundary<S, true, false, true>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    case 6: hipLaunchKernelGGL((k_boundary<S, false, true, true>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    default: hipLaunchKernelGGL((k_boundary<S, true, true, true>), grid, bl, 0, st, (S *)f, g, p, b, stab, part); break;
    }
    return hipGetLastError();
}

hipError_t launch_boundary(int sk, bool odd, void *f, const Geo &g, const Phys<double> &ph, const BndData &b,
                           hipStream_t st, const double *stab, double *part)
{
    if (b.np <= 0 || b.bpf <= 0) return hipSuccess;
    switch (sk) {
    case S_F32: return boundary_t<float>(odd, f, g, ph, b, st, stab, part);
    case S_F16: return boundary_t<_Float16>(odd, f, g, ph, b, st, stab, part);
    case S_BF16: return boundary_t<bf16s>(odd, f, g, ph, b, st, stab, part);
    default: return boundary_t<double>(odd, f, g, ph, b, st, stab, part);
    }
}

}  // namespace lbm
