// check.hip -- device-side health check used when the host synchronises:
// every stored population (both AA layouts, ghost planes and padding
// included, all initialised by k_init) must be finite; a non-finite value
// sets bit 1 of the instability flag, reported as LBM_E_UNSTABLE.
#include "lbm_sweep_dev.h"

namespace lbm {

template <typename S>
__global__ __launch_bounds__(256) void k_check_finite(const S *__restrict__ f, uint64_t n, DevCounters *ctr)
{
    using R = typename St<S>::R;
    bool bad = false;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        bad |= !isfinite(double(St<S>::ld(f, i, R(1))));
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&ctr->err_unstable, 2u);
}

hipError_t launch_check_finite(int sk, const void *f, uint64_t n, DevCounters *ctr, hipStream_t st)
{
    const dim3 gr(2048), bl(256);
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_check_finite<float>, gr, bl, 0, st, (const float *)f, n, ctr); break;
    case S_F16: hipLaunchKernelGGL(k_check_finite<_Float16>, gr, bl, 0, st, (const _Float16 *)f, n, ctr); break;
    case S_BF16: hipLaunchKernelGGL(k_check_finite<bf16s>, gr, bl, 0, st, (const bf16s *)f, n, ctr); break;
    default: hipLaunchKernelGGL(k_check_finite<double>, gr, bl, 0, st, (const double *)f, n, ctr); break;
    }
    return hipGetLastError();
}

}  // namespace lbm
