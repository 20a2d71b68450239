// stab.hip -- momentum stabilization for fully periodic domains under a
// constant particle force (Sec. 4.1): every collision of a step takes its
// equilibrium at u - ub, ub the mean velocity of all fluid cells of the state
// the step starts from.
//
// The sweep kernels sum, per workgroup, the momentum before collision of the
// cells they update, the momentum change of their bounce-back links and the
// cell count.  After the step (both branches joined) k_stab_update adds the
// collision's uniform change N rho0 (g - omega_o ub) and the cells whose
// owner the remap changed (newly covered ones leave with the momentum of
// their populations, uncovered ones enter with that of their refill), both
// read here in the layout the next sweep reads, and writes the next step's
// mean.  So the mean costs no pass over the lattice; k_stab_scan computes it
// by such a pass only after set-up or a state change from the host.
#include "lbm_sweep_dev.h"

namespace lbm {

// momentum sum_q c_q f_q of cell as the next sweep reads it (deviations:
// the w rho0 part carries none)
template <typename S>
__device__ __forceinline__ void cell_momentum(const S *__restrict__ f, const Geo &g, uint32_t cell, int swapped,
                                              typename St<S>::R inv, double (&j)[3])
{
    const uint32_t z = cell / g.nxy, y = (cell % g.nxy) / g.nx, x = cell % g.nx;
    j[0] = j[1] = j[2] = 0.0;
    for (int q = 1; q < Q; ++q) {
        uint32_t src = (z + 1) * g.nxy + y * g.nx + x;
        int qq = q;
        if (swapped) src = swapped_src(g, x, y, z, q, qq);
        const double v = double(St<S>::ld(f, uint64_t(qq) * g.qstride + src, inv));
        j[0] += CX[q] * v;
        j[1] += CY[q] * v;
        j[2] += CZ[q] * v;
    }
}

// One workgroup.  scan = 0: from the nslot workgroup sums of the step just
// done, plus the uniform collision change and the changed cells; scan = 1:
// from the nslot sums of k_stab_scan alone.  Writes stab[0..3] and empties
// the changed-cell list.
template <typename S>
__global__ __launch_bounds__(256) void k_stab_update(const S *__restrict__ f, Geo g, Phys<double> ph, double *stab,
                                                     uint32_t nslot, uint32_t *cov, uint32_t cov_cap, int swapped,
                                                     int scan)
{
    using R = typename St<S>::R;
    const double *part = stab + STAB_HEAD;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t s = threadIdx.x; s < nslot; s += blockDim.x)
        for (int k = 0; k < 4; ++k) a[k] += part[4 * size_t(s) + k];
    // changed cells in fixed point (2^-32): exact, so the list order (set by
    // atomics) does not change the result
    long long c[4] = {0, 0, 0, 0};
    const uint32_t n = (cov && !scan) ? min(cov[0], cov_cap) : 0u;
    for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) {
        const uint32_t v = cov[1 + e];
        const long long sg = (v & COV_UNCOVERED) ? 1 : -1;
        double j[3];
        cell_momentum<S>(f, g, v & ~COV_UNCOVERED, swapped, R(ph.inv_scale), j);
        for (int k = 0; k < 3; ++k) c[k] += sg * __double2ll_rn(ldexp(j[k], 32));
        c[3] += sg;
    }
    __shared__ double tot[4];
    __shared__ long long ctot[4];
    block_sum4(a, tot);
    __shared__ long long red[4][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 4; ++k) {
        long long x = c[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) red[wid][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        ctot[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double nsw = tot[3];
        const double nf = nsw + double(ctot[3]);
        double ub[3];
        for (int k = 0; k < 3; ++k) {
            const double gk = ph.has_g ? ph.g[k] : 0.0;
            double J = tot[k];
            // each updated cell's collision adds rho0 (g - omega_o ub)
            if (!scan) J += nsw * ph.rho0 * (gk - ph.omega_o * stab[k]) + ldexp(double(ctot[k]), -32);
            ub[k] = nf > 0.0 ? J / (nf * ph.rho0) + 0.5 * gk : 0.0;
        }
        for (int k = 0; k < 3; ++k) stab[k] = ub[k];
        stab[3] = nf;
        if (cov) cov[0] = 0u;
    }
}

// Sums of the fluid cells (pid < 0) of the current state, STAB_SCAN_GRID
// workgroups of 256 threads, into the workgroup slots.
template <typename S>
__global__ __launch_bounds__(256) void k_stab_scan(const S *__restrict__ f, const int32_t *__restrict__ pid, Geo g,
                                                   Phys<double> ph, double *stab, int swapped)
{
    using R = typename St<S>::R;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x; cell < g.ncell; cell += gridDim.x * blockDim.x) {
        if (pid[cell] >= 0) continue;
        double j[3];
        cell_momentum<S>(f, g, cell, swapped, R(ph.inv_scale), j);
        for (int k = 0; k < 3; ++k) a[k] += j[k];
        a[3] += 1.0;
    }
    block_sum4(a, stab + STAB_HEAD + 4 * size_t(blockIdx.x));
}

template <typename S>
static hipError_t stab_update_t(bool swapped, const void *f, const Geo &g, const Phys<double> &ph, double *stab,
                                uint32_t nslot, uint32_t *cov, uint32_t cov_cap, int scan, hipStream_t st)
{
    hipLaunchKernelGGL(k_stab_update<S>, dim3(1), dim3(256), 0, st, (const S *)f, g, ph, stab, nslot, cov, cov_cap,
                       swapped ? 1 : 0, scan);
    return hipGetLastError();
}

hipError_t launch_stab_update(int sk, bool swapped, const void *f, const Geo &g, const Phys<double> &ph,
                              double *stab, uint32_t nslot, uint32_t *cov, uint32_t cov_cap, hipStream_t st)
{
    switch (sk) {
    case S_F32: return stab_update_t<float>(swapped, f, g, ph, stab, nslot, cov, cov_cap, 0, st);
    case S_F16: return stab_update_t<_Float16>(swapped, f, g, ph, stab, nslot, cov, cov_cap, 0, st);
    case S_BF16: return stab_update_t<bf16s>(swapped, f, g, ph, stab, nslot, cov, cov_cap, 0, st);
    default: return stab_update_t<double>(swapped, f, g, ph, stab, nslot, cov, cov_cap, 0, st);
    }
}

template <typename S>
static hipError_t stab_scan_t(bool swapped, const void *f, const int32_t *pid, const Geo &g, const Phys<double> &ph,
                              double *stab, uint32_t *cov, hipStream_t st)
{
    hipLaunchKernelGGL(k_stab_scan<S>, dim3(STAB_SCAN_GRID), dim3(256), 0, st, (const S *)f, pid, g, ph, stab,
                       swapped ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return stab_update_t<S>(swapped, f, g, ph, stab, STAB_SCAN_GRID, cov, 0u, 1, st);
}

hipError_t launch_stab_scan(int sk, bool swapped, const void *f, const int32_t *pid, const Geo &g,
                            const Phys<double> &ph, double *stab, uint32_t *cov, hipStream_t st)
{
    switch (sk) {
    case S_F32: return stab_scan_t<float>(swapped, f, pid, g, ph, stab, cov, st);
    case S_F16: return stab_scan_t<_Float16>(swapped, f, pid, g, ph, stab, cov, st);
    case S_BF16: return stab_scan_t<bf16s>(swapped, f, pid, g, ph, stab, cov, st);
    default: return stab_scan_t<double>(swapped, f, pid, g, ph, stab, cov, st);
    }
}

}  // namespace lbm
