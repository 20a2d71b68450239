// mlp.hip -- the closure network (247 -> 64 -> 64 -> 6, GELU, BF16 weights,
// FP32 activations and accumulation): forward, loss and gradient, Adam and
// the training loop.  The per-step closure (features, one-sample forward,
// correction in one launch) is in features.hip.
//
// Work layout.  A workgroup of 256 threads takes a tile of 32 samples: the
// tile's inputs, both hidden layers and the BF16 weights sit in LDS; thread
// (j, g) owns output unit j of a layer for samples g, g+4, ... (so a wave
// reads one input value per step, broadcast from LDS).  The gradient kernel
// runs a fixed grid; workgroup b accumulates the weight gradients of its
// tiles b, b+G, ... in its own slice of a partial buffer, and a reduction
// kernel adds the slices in order b = 0..G-1, so the gradient is the same
// on every run.  These products are tiny (about 20k multiply-adds per
// sample), far from the matrix cores' break-even size, and are written as
// plain FP32 FMA loops.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_mlp_dev.h"

namespace lbm {

constexpr int TILE = 32, MB = 256, GRAD_BLOCKS = 64;

__host__ __device__ inline uint16_t to_bf16(float v)
{
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return uint16_t((u >> 16) | 0x40u);   // NaN stays NaN
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return uint16_t(u >> 16);
}

// derivative of the exact GELU: g'(z) = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_d(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct MlpTile {
    uint16_t w1[NH * NI];
    uint16_t w2[NH * NH];
    uint16_t w3[NO * NH];
    float b[NH + NH + NO];
    float x[TILE][NI];
    float z1[TILE][NH], h1[TILE][NH];
    float z2[TILE][NH], h2[TILE][NH];
    float y[TILE][NO];
    float dy[TILE][NO];
    float d2[TILE][NH];   // dL/dz2
    float d1[TILE][NH];   // dL/dz1
};

__device__ void load_weights(const uint16_t *wb, MlpTile &s)
{
    for (int i = threadIdx.x; i < NH * NI; i += MB) s.w1[i] = wb[OW1 + i];
    for (int i = threadIdx.x; i < NH * NH; i += MB) s.w2[i] = wb[OW2 + i];
    for (int i = threadIdx.x; i < NO * NH; i += MB) s.w3[i] = wb[OW3 + i];
    for (int i = threadIdx.x; i < NH; i += MB) {
        s.b[i] = bf(wb[OB1 + i]);
        s.b[NH + i] = bf(wb[OB2 + i]);
    }
    if (threadIdx.x < NO) s.b[2 * NH + threadIdx.x] = bf(wb[OB3 + threadIdx.x]);
}

// inputs of samples base .. base+cnt-1 (through idx if given), normalised
__device__ void load_inputs(const float *x, const int32_t *idx, int base, int cnt, const float *mean,
                            const float *inv_std, MlpTile &s)
{
    for (int e = threadIdx.x; e < TILE * NI; e += MB) {
        const int r = e / NI, i = e - r * NI;
        float v = 0.0f;
        if (r < cnt) {
            const int src = idx ? idx[base + r] : base + r;
            v = (x[size_t(src) * NI + i] - mean[i]) * inv_std[i];
        }
        s.x[r][i] = v;
    }
}

// forward pass of the tile (all TILE rows; rows past cnt hold zeros)
__device__ void forward_tile(MlpTile &s)
{
    __syncthreads();
    const int j = threadIdx.x & 63, g = threadIdx.x >> 6;
    {
        float acc[TILE / 4];
        for (int k = 0; k < TILE / 4; ++k) acc[k] = s.b[j];
        for (int i = 0; i < NI; ++i) {
            const float w = bf(s.w1[j * NI + i]);
#pragma unroll
            for (int k = 0; k < TILE / 4; ++k) acc[k] = fmaf(w, s.x[g + 4 * k][i], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < TILE / 4; ++k) {
            s.z1[g + 4 * k][j] = acc[k];
            s.h1[g + 4 * k][j] = gelu(acc[k]);
        }
    }
    __syncthreads();
    {
        float acc[TILE / 4];
        for (int k = 0; k < TILE / 4; ++k) acc[k] = s.b[NH + j];
        for (int i = 0; i < NH; ++i) {
            const float w = bf(s.w2[j * NH + i]);
#pragma unroll
            for (int k = 0; k < TILE / 4; ++k) acc[k] = fmaf(w, s.h1[g + 4 * k][i], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < TILE / 4; ++k) {
            s.z2[g + 4 * k][j] = acc[k];
            s.h2[g + 4 * k][j] = gelu(acc[k]);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TILE * NO; e += MB) {
        const int r = e / NO, o = e - r * NO;
        float acc = s.b[2 * NH + o];
        for (int i = 0; i < NH; ++i) acc = fmaf(bf(s.w3[o * NH + i]), s.h2[r][i], acc);
        s.y[r][o] = acc;
    }
    __syncthreads();
}

__global__ __launch_bounds__(MB) void k_mlp_forward(const uint16_t *__restrict__ wb, const float *__restrict__ x,
                                                    int n, const float *__restrict__ mean,
                                                    const float *__restrict__ inv_std,
                                                    const float *__restrict__ out_scale, float *__restrict__ y)
{
    __shared__ MlpTile s;
    const int base = blockIdx.x * TILE, cnt = min(TILE, n - base);
    load_weights(wb, s);
    load_inputs(x, nullptr, base, cnt, mean, inv_std, s);
    forward_tile(s);
    for (int e = threadIdx.x; e < cnt * NO; e += MB) {
        const int r = e / NO, o = e - r * NO;
        y[size_t(base + r) * NO + o] = s.y[r][o] * out_scale[o];
    }
}

// Squared-error sums and parameter gradients of the samples idx[first ..
// first+n-1] (or first .. first+n-1), scaled by gscale; workgroup b writes
// its partial sums to part[b][NP] and lpart[b].
__global__ __launch_bounds__(MB) void k_mlp_grad(const uint16_t *__restrict__ wb, const float *__restrict__ x,
                                                 const float *__restrict__ t, const int32_t *__restrict__ idx,
                                                 int first, int n, const float *__restrict__ mean,
                                                 const float *__restrict__ inv_std, float gscale,
                                                 float *__restrict__ part, double *__restrict__ lpart)
{
    __shared__ MlpTile s;
    __shared__ double sl[MB / 64];
    float *gp = part + size_t(blockIdx.x) * NP;
    for (int p = threadIdx.x; p < NP; p += MB) gp[p] = 0.0f;
    load_weights(wb, s);
    double lsum = 0.0;
    const int ntile = (n + TILE - 1) / TILE;
    for (int tl = blockIdx.x; tl < ntile; tl += gridDim.x) {
        const int base = tl * TILE, cnt = min(TILE, n - base);
        __syncthreads();
        load_inputs(x, idx, first + base, cnt, mean, inv_std, s);
        forward_tile(s);
        for (int e = threadIdx.x; e < TILE * NO; e += MB) {
            const int r = e / NO, o = e - r * NO;
            float d = 0.0f;
            if (r < cnt) {
                const int src = idx ? idx[first + base + r] : first + base + r;
                d = s.y[r][o] - t[size_t(src) * NO + o];
                lsum += double(d) * double(d);
            }
            s.dy[r][o] = gscale * d;
        }
        __syncthreads();
        // output layer: dW3, db3 and dL/dz2
        for (int p = threadIdx.x; p < NO * NH; p += MB) {
            const int o = p / NH, i = p - o * NH;
            float a = 0.0f;
            for (int r = 0; r < TILE; ++r) a = fmaf(s.dy[r][o], s.h2[r][i], a);
            gp[OW3 + p] += a;
        }
        if (threadIdx.x < NO) {
            float a = 0.0f;
            for (int r = 0; r < TILE; ++r) a += s.dy[r][threadIdx.x];
            gp[OB3 + threadIdx.x] += a;
        }
        for (int e = threadIdx.x; e < TILE * NH; e += MB) {
            const int r = e / NH, j = e - r * NH;
            float a = 0.0f;
            for (int o = 0; o < NO; ++o) a = fmaf(bf(s.w3[o * NH + j]), s.dy[r][o], a);
            s.d2[r][j] = a * gelu_d(s.z2[r][j]);
        }
        __syncthreads();
        // second layer: dW2, db2 and dL/dz1
        for (int p = threadIdx.x; p < NH * NH; p += MB) {
            const int j = p / NH, i = p - j * NH;
            float a = 0.0f;
            for (int r = 0; r < TILE; ++r) a = fmaf(s.d2[r][j], s.h1[r][i], a);
            gp[OW2 + p] += a;
        }
        if (threadIdx.x < NH) {
            float a = 0.0f;
            for (int r = 0; r < TILE; ++r) a += s.d2[r][threadIdx.x];
            gp[OB2 + threadIdx.x] += a;
        }
        for (int e = threadIdx.x; e < TILE * NH; e += MB) {
            const int r = e / NH, i = e - r * NH;
            float a = 0.0f;
            for (int j = 0; j < NH; ++j) a = fmaf(bf(s.w2[j * NH + i]), s.d2[r][j], a);
            s.d1[r][i] = a * gelu_d(s.z1[r][i]);
        }
        __syncthreads();
        // first layer: dW1, db1
        for (int p = threadIdx.x; p < NH * NI; p += MB) {
            const int j = p / NI, i = p - j * NI;
            float a = 0.0f;
            for (int r = 0; r < TILE; ++r) a = fmaf(s.d1[r][j], s.x[r][i], a);
            gp[OW1 + p] += a;
        }
        if (threadIdx.x < NH) {
            float a = 0.0f;
            for (int r = 0; r < TILE; ++r) a += s.d1[r][threadIdx.x];
            gp[OB1 + threadIdx.x] += a;
        }
    }
    // loss partial: waves, then workgroup
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if ((threadIdx.x & 63) == 0) sl[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < MB / 64; ++w) v += sl[w];
        lpart[blockIdx.x] = v;
    }
}

// grad[p] = sum over b of part[b][p] in order b; loss = sum of lpart
__global__ void k_mlp_reduce(const float *__restrict__ part, int nb, float *__restrict__ grad,
                             const double *__restrict__ lpart, double *__restrict__ loss, double lscale,
                             double *__restrict__ loss_acc)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) {
        float a = 0.0f;
        for (int b = 0; b < nb; ++b) a += part[size_t(b) * NP + p];
        grad[p] = a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double l = 0.0;
        for (int b = 0; b < nb; ++b) l += lpart[b];
        *loss = l * lscale;
        if (loss_acc) *loss_acc += l * lscale;
    }
}

// Adam on the FP32 master; corrected step size from the step counter t
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, uint16_t *__restrict__ wb, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) {
        const float gg = g[p];
        const float mm = b1 * m[p] + (1.0f - b1) * gg;
        const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
        m[p] = mm;
        v[p] = vv;
        const float mh = mm / c1, vh = vv / c2;
        const float nw = w[p] - lr * mh / (sqrtf(vh) + eps);
        w[p] = nw;
        wb[p] = to_bf16(nw);
    }
}

__global__ void k_bf16_copy(const float *__restrict__ w, uint16_t *__restrict__ wb)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) wb[p] = to_bf16(w[p]);
}

__global__ void k_zero_d(double *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

}  // namespace lbm

using namespace lbm;

struct lbm_mlp {
    std::string err;
    hipStream_t st = nullptr;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t *wb = nullptr;
    float *in_mean = nullptr, *in_inv_std = nullptr, *out_scale = nullptr, *env_min = nullptr,
          *env_max = nullptr;
    float *part = nullptr;
    double *lpart = nullptr, *loss = nullptr, *loss_acc = nullptr;
    int64_t t = 0;   // Adam steps taken
};

namespace lbm {
MlpDev mlp_device_view(const lbm_mlp *m)
{
    MlpDev d{};
    d.wb = m->wb;
    d.in_mean = m->in_mean;
    d.in_inv_std = m->in_inv_std;
    d.out_scale = m->out_scale;
    d.env_min = m->env_min;
    d.env_max = m->env_max;
    return d;
}

hipError_t launch_mlp_forward(const MlpDev &m, const float *x, int n, float *y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + TILE - 1) / TILE), dim3(MB), 0, st, m.wb, x, n, m.in_mean,
                       m.in_inv_std, m.out_scale, y);
    return hipGetLastError();
}

}  // namespace lbm

static lbm_status mfail(lbm_mlp *m, lbm_status s, const std::string &e)
{
    if (m) m->err = e;
    return s;
}

#define MHIP(m, call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return mfail((m), e_ == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_HIP,            \
                         std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

// splitmix64 (Steele, Lea and Flood; the constants of Vigna's reference code)
static uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double unit(uint64_t &s) { return double(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

static lbm_status upload_master(lbm_mlp *m, const float *w)
{
    MHIP(m, hipMemcpyAsync(m->w, w, NP * sizeof(float), hipMemcpyHostToDevice, m->st));
    hipLaunchKernelGGL(k_bf16_copy, dim3(80), dim3(256), 0, m->st, m->w, m->wb);
    MHIP(m, hipGetLastError());
    MHIP(m, hipMemsetAsync(m->m, 0, NP * sizeof(float), m->st));
    MHIP(m, hipMemsetAsync(m->v, 0, NP * sizeof(float), m->st));
    MHIP(m, hipStreamSynchronize(m->st));
    m->t = 0;
    return LBM_OK;
}

extern "C" {

lbm_status lbm_mlp_create(uint64_t seed, void *stream, lbm_mlp **out)
{
    if (!out) return LBM_E_ARG;
    *out = nullptr;
    lbm_mlp *m = new (std::nothrow) lbm_mlp;
    if (!m) return LBM_E_NOMEM;
    m->st = (hipStream_t)stream;
    auto bail = [&](lbm_status s) {
        lbm_mlp_destroy(m);
        return s;
    };
    if (hipMalloc(&m->w, NP * 4) != hipSuccess || hipMalloc(&m->m, NP * 4) != hipSuccess ||
        hipMalloc(&m->v, NP * 4) != hipSuccess || hipMalloc(&m->g, NP * 4) != hipSuccess ||
        hipMalloc(&m->wb, NP * 2) != hipSuccess || hipMalloc(&m->in_mean, NI * 4) != hipSuccess ||
        hipMalloc(&m->in_inv_std, NI * 4) != hipSuccess || hipMalloc(&m->out_scale, NO * 4) != hipSuccess ||
        hipMalloc(&m->env_min, NI * 4) != hipSuccess || hipMalloc(&m->env_max, NI * 4) != hipSuccess ||
        hipMalloc(&m->part, size_t(GRAD_BLOCKS) * NP * 4) != hipSuccess ||
        hipMalloc(&m->lpart, GRAD_BLOCKS * 8) != hipSuccess || hipMalloc(&m->loss, 8) != hipSuccess ||
        hipMalloc(&m->loss_acc, 8) != hipSuccess)
        return bail(LBM_E_NOMEM);
    std::vector<float> w(NP, 0.0f);
    uint64_t s = seed;
    auto fill = [&](int off, int rows, int cols, double gain) {
        const double a = gain * std::sqrt(6.0 / cols);
        for (int i = 0; i < rows * cols; ++i) w[off + i] = float((2.0 * unit(s) - 1.0) * a);
    };
    fill(OW1, NH, NI, 1.0);
    fill(OW2, NH, NH, 1.0);
    fill(OW3, NO, NH, 0.1);
    std::vector<float> zero(NI, 0.0f), one(NI, 1.0f), lo(NI, -3.0e38f), hi(NI, 3.0e38f);
    if (upload_master(m, w.data()) != LBM_OK) return bail(LBM_E_HIP);
    if (lbm_mlp_set_norm(m, zero.data(), one.data(), one.data(), lo.data(), hi.data()) != LBM_OK)
        return bail(LBM_E_HIP);
    *out = m;
    return LBM_OK;
}

lbm_status lbm_mlp_destroy(lbm_mlp *m)
{
    if (!m) return LBM_E_ARG;
    if (m->st) hipStreamSynchronize(m->st);
    else hipDeviceSynchronize();
    for (void *p : {(void *)m->w, (void *)m->m, (void *)m->v, (void *)m->g, (void *)m->wb, (void *)m->in_mean,
                    (void *)m->in_inv_std, (void *)m->out_scale, (void *)m->env_min, (void *)m->env_max,
                    (void *)m->part, (void *)m->lpart, (void *)m->loss, (void *)m->loss_acc})
        if (p) hipFree(p);
    delete m;
    return LBM_OK;
}

const char *lbm_mlp_last_error(const lbm_mlp *m) { return m ? m->err.c_str() : "null network"; }

lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *w)
{
    if (!m || !w) return mfail(m, LBM_E_ARG, "null argument");
    return upload_master(m, w);
}

lbm_status lbm_mlp_get_params(lbm_mlp *m, float *w, uint16_t *wb)
{
    if (!m) return LBM_E_ARG;
    MHIP(m, hipStreamSynchronize(m->st));
    if (w) MHIP(m, hipMemcpy(w, m->w, NP * sizeof(float), hipMemcpyDeviceToHost));
    if (wb) MHIP(m, hipMemcpy(wb, m->wb, NP * sizeof(uint16_t), hipMemcpyDeviceToHost));
    return LBM_OK;
}

lbm_status lbm_mlp_set_norm(lbm_mlp *m, const float *in_mean, const float *in_inv_std, const float *out_scale,
                            const float *env_min, const float *env_max)
{
    if (!m) return LBM_E_ARG;
    if (in_mean) MHIP(m, hipMemcpyAsync(m->in_mean, in_mean, NI * 4, hipMemcpyHostToDevice, m->st));
    if (in_inv_std) MHIP(m, hipMemcpyAsync(m->in_inv_std, in_inv_std, NI * 4, hipMemcpyHostToDevice, m->st));
    if (out_scale) MHIP(m, hipMemcpyAsync(m->out_scale, out_scale, NO * 4, hipMemcpyHostToDevice, m->st));
    if (env_min) MHIP(m, hipMemcpyAsync(m->env_min, env_min, NI * 4, hipMemcpyHostToDevice, m->st));
    if (env_max) MHIP(m, hipMemcpyAsync(m->env_max, env_max, NI * 4, hipMemcpyHostToDevice, m->st));
    MHIP(m, hipStreamSynchronize(m->st));
    return LBM_OK;
}

lbm_status lbm_mlp_forward(lbm_mlp *m, const float *x, int32_t n, float *y)
{
    if (!m || n < 0 || (n > 0 && (!x || !y))) return mfail(m, LBM_E_ARG, "bad argument");
    MHIP(m, launch_mlp_forward(mlp_device_view(m), x, n, y, m->st));
    MHIP(m, hipStreamSynchronize(m->st));
    return LBM_OK;
}

// gradient of the mean squared error over samples first .. first+n-1 of
// the order idx (or natural order), into m->g; loss into m->loss
static hipError_t grad_pass(lbm_mlp *m, const float *x, const float *t, const int32_t *idx, int first, int n,
                            bool accumulate)
{
    const int ntile = (n + TILE - 1) / TILE;
    const int nb = std::min(GRAD_BLOCKS, ntile);
    const float gscale = 2.0f / float(n * NO);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(MB), 0, m->st, m->wb, x, t, idx, first, n, m->in_mean,
                       m->in_inv_std, gscale, m->part, m->lpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3(80), dim3(256), 0, m->st, m->part, nb, m->g, m->lpart, m->loss,
                       1.0 / double(n * NO), accumulate ? m->loss_acc : nullptr);
    return hipGetLastError();
}

lbm_status lbm_mlp_loss_grad(lbm_mlp *m, const float *x, const float *t, int32_t n, double *loss, float *grad)
{
    if (!m || !x || !t || n < 1) return mfail(m, LBM_E_ARG, "bad argument");
    MHIP(m, grad_pass(m, x, t, nullptr, 0, n, false));
    if (loss) MHIP(m, hipMemcpyAsync(loss, m->loss, 8, hipMemcpyDeviceToHost, m->st));
    if (grad) MHIP(m, hipMemcpyAsync(grad, m->g, NP * 4, hipMemcpyDeviceToHost, m->st));
    MHIP(m, hipStreamSynchronize(m->st));
    return LBM_OK;
}

static hipError_t adam_pass(lbm_mlp *m, float lr, float b1, float b2, float eps)
{
    m->t += 1;
    const float c1 = float(1.0 - std::pow(double(b1), double(m->t)));
    const float c2 = float(1.0 - std::pow(double(b2), double(m->t)));
    hipLaunchKernelGGL(k_adam, dim3(80), dim3(256), 0, m->st, m->w, m->m, m->v, m->g, m->wb, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

lbm_status lbm_mlp_adam(lbm_mlp *m, float lr, float beta1, float beta2, float eps)
{
    if (!m || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return mfail(m, LBM_E_ARG, "bad Adam parameters");
    MHIP(m, adam_pass(m, lr, beta1, beta2, eps));
    MHIP(m, hipStreamSynchronize(m->st));
    return LBM_OK;
}

lbm_status lbm_mlp_train(lbm_mlp *m, const float *x, const float *t, int32_t n, int32_t epochs, int32_t batch,
                         float lr, uint64_t shuffle_seed, double *loss_per_epoch)
{
    if (!m || !x || !t || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.0f))
        return mfail(m, LBM_E_ARG, "bad argument");
    int32_t *didx = nullptr;
    MHIP(m, hipMalloc(&didx, size_t(n) * sizeof(int32_t)));
    std::vector<int32_t> idx(n);
    uint64_t s = shuffle_seed;
    const int nbatch = (n + batch - 1) / batch;
    lbm_status st = LBM_OK;
    for (int ep = 0; ep < epochs && st == LBM_OK; ++ep) {
        for (int i = 0; i < n; ++i) idx[i] = i;
        for (int i = n - 1; i > 0; --i) {   // Fisher-Yates
            const int j = int(splitmix64(s) % uint64_t(i + 1));
            std::swap(idx[i], idx[j]);
        }
        hipError_t e = hipMemcpyAsync(didx, idx.data(), size_t(n) * 4, hipMemcpyHostToDevice, m->st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, m->st, m->loss_acc, 1);
            e = hipGetLastError();
        }
        for (int b = 0; b < nbatch && e == hipSuccess; ++b) {
            const int first = b * batch, cnt = std::min(batch, n - first);
            e = grad_pass(m, x, t, didx, first, cnt, true);
            if (e == hipSuccess) e = adam_pass(m, lr, 0.9f, 0.999f, 1e-8f);
        }
        double acc = 0.0;
        if (e == hipSuccess) e = hipMemcpyAsync(&acc, m->loss_acc, 8, hipMemcpyDeviceToHost, m->st);
        if (e == hipSuccess) e = hipStreamSynchronize(m->st);
        if (e != hipSuccess) st = mfail(m, LBM_E_HIP, std::string("train: ") + hipGetErrorString(e));
        else if (loss_per_epoch) loss_per_epoch[ep] = acc / nbatch;
    }
    hipStreamSynchronize(m->st);
    hipFree(didx);
    return st;
}

}  // extern "C"
