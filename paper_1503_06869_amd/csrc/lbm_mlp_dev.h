// lbm_mlp_dev.h -- parameter layout and activation of the closure network
// (247 -> 64 -> 64 -> 6, exact GELU, BF16 weights), shared by the network
// kernels and the fused closure kernel of the step.
#pragma once
#include "../../include/lbm_mlp.h"
#include "lbm_dev.h"

namespace lbm {

constexpr int NI = LBM_MLP_IN, NH = LBM_MLP_HIDDEN, NO = LBM_MLP_OUT, NP = LBM_MLP_NPARAM;
constexpr int OW1 = 0, OB1 = NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NO * NH;
static_assert(OB3 + NO == NP, "parameter layout");

__device__ __forceinline__ float bf(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// exact GELU: g(z) = z Phi(z)
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

}  // namespace lbm
