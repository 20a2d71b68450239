// features.hip -- the learned closure's per-fiber work on the device:
//   features: velocities relative to the fiber's rigid motion on a 3 x 27
//             stencil (centre and both tips, offsets {-2,0,2}^3 cells along
//             the body axes), trilinear in the cell-centre velocities,
//             expressed in the body frame and scaled by 1 / (gamma L), and
//             the orientation;
//   k_closure_step: features, the network (one sample per workgroup) and
//             the correction dF, dM of one step, fused in one launch with one
//             workgroup per fiber.
// The network's own kernels (batches of samples, training) are in mlp.hip;
// both use the same parameter layout and BF16 weights.
#include "lbm_sweep_dev.h"
#include "lbm_mlp_dev.h"

namespace lbm {

constexpr int NPT = 81, NCORNER = 8, NITEM = NPT * NCORNER;   // stencil points x trilinear corners
constexpr int FB = 256;                                       // threads per fiber workgroup
constexpr int ITEMS_PER_THREAD = (NITEM + FB - 1) / FB;

struct FeatStage {
    double u[NPT][NCORNER][3];   // weighted corner velocities
    float x[NI];                 // raw features
};

// Velocity at the centre of cell (x, y, z): decoded from the populations at
// the current parity for a fluid cell (as the field readback does), the
// rigid-body velocity of the owner for a fiber cell.  The flag, the owner
// and all populations are loaded together; the flag then picks the result.
template <typename S>
__device__ __forceinline__ void cell_velocity(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                                              const int32_t *__restrict__ pid, const PState *__restrict__ ps,
                                              const Geo &g, const Phys<double> &ph, int swapped, uint32_t x,
                                              uint32_t y, uint32_t z, double u[3])
{
    using R = typename St<S>::R;
    const uint32_t cell = (z * g.ny + y) * g.nx + x;
    const uint8_t fl = flags[cell];
    const int32_t own = pid[cell];
    R fv[Q];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        uint32_t src = (z + 1) * g.nxy + y * g.nx + x;
        int qq = q;
        if (swapped) {
            const uint32_t sx = (x + g.nx - CX[q]) % g.nx, sy = (y + g.ny - CY[q]) % g.ny;
            const int32_t szi = int32_t(z) - CZ[q];
            const uint32_t szs = g.zper ? uint32_t((szi + int32_t(g.nz)) % int32_t(g.nz)) + 1 : uint32_t(szi + 1);
            src = szs * g.nxy + sy * g.nx + sx;
            qq = opp(q);
        }
        fv[q] = St<S>::ld(f, uint64_t(qq) * g.qstride + src, R(ph.inv_scale));
    }
    if ((fl & F_SOLID) && own >= 0) {
        surf_vel(ps[own], double(x), double(y), double(z), g, u);
        return;
    }
    double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const double v = double(fv[q]);
        j[0] += CX[q] * v;
        j[1] += CY[q] * v;
        j[2] += CZ[q] * v;
    }
    for (int k = 0; k < 3; ++k) u[k] = j[k] / ph.rho0 + 0.5 * ph.g[k];
}

// body frame of quaternion q: columns R(q) e_x (the axis), R(q) e_y, R(q) e_z
__device__ __forceinline__ void body_frame(const double q[4], double Rm[3][3])
{
    const double w = q[0], qx = q[1], qy = q[2], qz = q[3];
    Rm[0][0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    Rm[0][1] = 2.0 * (qx * qy - w * qz);
    Rm[0][2] = 2.0 * (qx * qz + w * qy);
    Rm[1][0] = 2.0 * (qx * qy + w * qz);
    Rm[1][1] = 1.0 - 2.0 * (qx * qx + qz * qz);
    Rm[1][2] = 2.0 * (qy * qz - w * qx);
    Rm[2][0] = 2.0 * (qx * qz - w * qy);
    Rm[2][1] = 2.0 * (qy * qz + w * qx);
    Rm[2][2] = 1.0 - 2.0 * (qx * qx + qy * qy);
}

// offset of stencil point k from the centre of mass (lab frame)
__device__ __forceinline__ void point_offset(int k, double L, const double Rm[3][3], double d[3])
{
    const int pt = k / 27, m = k % 27;
    const double ob[3] = {2.0 * (m % 3 - 1), 2.0 * ((m / 3) % 3 - 1), 2.0 * (m / 9 - 1)};
    const double side = pt == 0 ? 0.0 : (pt == 1 ? 0.5 * L : -0.5 * L);
    for (int e = 0; e < 3; ++e) d[e] = side * Rm[e][0] + (Rm[e][0] * ob[0] + Rm[e][1] * ob[1] + Rm[e][2] * ob[2]);
}

// The features of fiber p into sh.x (block-uniform call, FB threads).  Work
// item i = (point k, corner c): the weighted velocity of one corner cell of
// the trilinear interpolation; every thread issues the loads of all its
// items before using any.  Then thread k sums its point's corners in the
// order c = 0..7.
template <typename S>
__device__ void features_block(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                               const int32_t *__restrict__ pid, const PState *__restrict__ ps,
                               const PConst *__restrict__ pc, const Geo &g, const Phys<double> &ph, int swapped,
                               double gamma, int p, FeatStage &sh)
{
    const PState s = ps[p];
    const double L = pc[p].length;
    double Rm[3][3];
    body_frame(s.q, Rm);
#pragma unroll
    for (int r = 0; r < ITEMS_PER_THREAD; ++r) {
        const int item = int(threadIdx.x) + r * FB;
        const int it = item < NITEM ? item : NITEM - 1;   // loads for every slot; store only real items
        const int k = it / NCORNER, c = it % NCORNER;
        double d[3];
        point_offset(k, L, Rm, d);
        const double px = s.X[0] + d[0], py = s.X[1] + d[1];
        double pz = s.X[2] + d[2];
        const double zmax = double(g.nz) - 1.0;
        pz = pz < 0.0 ? 0.0 : (pz > zmax ? zmax : pz);
        const double fx0 = floor(px), fy0 = floor(py);
        int32_t z0 = int32_t(floor(pz));
        if (z0 > int32_t(g.nz) - 2) z0 = int32_t(g.nz) - 2;
        const double ax = px - fx0, ay = py - fy0, az = pz - double(z0);
        const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
        const double wt = (cx ? ax : 1.0 - ax) * (cy ? ay : 1.0 - ay) * (cz ? az : 1.0 - az);
        int32_t xx = (int32_t(fx0) + cx) % int32_t(g.nx), yy = (int32_t(fy0) + cy) % int32_t(g.ny);
        xx += xx < 0 ? int32_t(g.nx) : 0;
        yy += yy < 0 ? int32_t(g.ny) : 0;
        double uc[3];
        cell_velocity<S>(f, flags, pid, ps, g, ph, swapped, uint32_t(xx), uint32_t(yy), uint32_t(z0 + cz), uc);
        if (item < NITEM)
            for (int e = 0; e < 3; ++e) sh.u[k][c][e] = wt * uc[e];
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < NPT) {
        double u[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < NCORNER; ++c)
            for (int e = 0; e < 3; ++e) u[e] += sh.u[k][c][e];
        double d[3];
        point_offset(k, L, Rm, d);
        // velocity relative to the rigid motion, in the body frame
        const double v[3] = {u[0] - (s.V[0] + (s.W[1] * d[2] - s.W[2] * d[1])),
                             u[1] - (s.V[1] + (s.W[2] * d[0] - s.W[0] * d[2])),
                             u[2] - (s.V[2] + (s.W[0] * d[1] - s.W[1] * d[0]))};
        const double vs = 1.0 / (gamma * L);
        for (int e = 0; e < 3; ++e) sh.x[k * 3 + e] = float((Rm[0][e] * v[0] + Rm[1][e] * v[1] + Rm[2][e] * v[2]) * vs);
    } else if (k < NPT + 4) {
        const double sg = s.q[0] < 0.0 ? -1.0 : 1.0;
        sh.x[3 * NPT + (k - NPT)] = float(sg * s.q[k - NPT]);
    }
    __syncthreads();
}

template <typename S>
__global__ __launch_bounds__(FB) void k_features(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                                                 const int32_t *__restrict__ pid, const PState *__restrict__ ps,
                                                 const PConst *__restrict__ pc, Geo g, Phys<double> ph,
                                                 int swapped, double gamma, float *__restrict__ out)
{
    __shared__ FeatStage sh;
    const int p = blockIdx.x;
    features_block<S>(f, flags, pid, ps, pc, g, ph, swapped, gamma, p, sh);
    for (int i = threadIdx.x; i < NI; i += FB) out[size_t(p) * NI + i] = sh.x[i];
}

// sum over the 64 lanes of a wave; every lane ends with the same value (the
// butterfly pairs each sum with its operands swapped, and FP addition is
// commutative), so the result does not depend on the lane read
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One step's closure for fiber p: features, then the network on this one
// sample -- wave w computes units 16w .. 16w+15 of a hidden layer with the
// lanes spread over the inputs (coalesced weight rows) and a wave sum per
// unit -- then the correction: outside the envelope none (counted), else the
// body-frame outputs rotated to the lab frame and scaled by rho0 nu gamma L^2
// (force) and rho0 nu gamma L^3 (torque).
template <typename S>
__global__ __launch_bounds__(FB) void k_closure_step(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                                                     const int32_t *__restrict__ pid, const PState *__restrict__ ps,
                                                     const PConst *__restrict__ pc, Geo g, Phys<double> ph,
                                                     int swapped, double gamma, MlpDev m, double rho0, double nu,
                                                     double *__restrict__ corr,
                                                     unsigned long long *__restrict__ stats)
{
    __shared__ FeatStage sh;
    __shared__ float s_xn[NI], s_h1[NH], s_h2[NH], s_y[NO];
    __shared__ int s_out;
    const int p = blockIdx.x;
    if (threadIdx.x == 0) s_out = 0;
    features_block<S>(f, flags, pid, ps, pc, g, ph, swapped, gamma, p, sh);
    for (int i = threadIdx.x; i < NI; i += FB) {
        const float v = sh.x[i];
        if (!(v >= m.env_min[i] && v <= m.env_max[i])) atomicOr(&s_out, 1);
        s_xn[i] = (v - m.in_mean[i]) * m.in_inv_std[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint16_t *wb = m.wb;
    // layer 1: 247 inputs, lane l takes inputs l, l + 64, l + 128, l + 192
    for (int u = 0; u < 16; ++u) {
        const int j = w * 16 + u;
        float a = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = lane + 64 * r;
            if (i < NI) a = fmaf(bf(wb[OW1 + j * NI + i]), s_xn[i], a);
        }
        a = wave_sum(a);
        if (lane == 0) s_h1[j] = gelu(a + bf(wb[OB1 + j]));
    }
    __syncthreads();
    for (int u = 0; u < 16; ++u) {
        const int j = w * 16 + u;
        const float a = wave_sum(bf(wb[OW2 + j * NH + lane]) * s_h1[lane]);
        if (lane == 0) s_h2[j] = gelu(a + bf(wb[OB2 + j]));
    }
    __syncthreads();
    if (w == 0) {
        for (int o = 0; o < NO; ++o) {
            const float a = wave_sum(bf(wb[OW3 + o * NH + lane]) * s_h2[lane]);
            if (lane == 0) s_y[o] = (a + bf(wb[OB3 + o])) * m.out_scale[o];
        }
    }
    __syncthreads();
    if (threadIdx.x < NO) {
        const int o = threadIdx.x, part = o / 3, row = o % 3;
        const double qf[4] = {sh.x[243], sh.x[244], sh.x[245], sh.x[246]};
        double Rm[3][3];
        body_frame(qf, Rm);
        const double L = pc[p].length;
        const double sF = rho0 * nu * gamma * L * L, sc = part == 0 ? sF : sF * L;
        const float *yp = s_y + 3 * part;
        const double lab = Rm[row][0] * yp[0] + Rm[row][1] * yp[1] + Rm[row][2] * yp[2];
        corr[size_t(p) * NO + o] = s_out ? 0.0 : lab * sc;
    }
    if (threadIdx.x == 0) atomicAdd(&stats[s_out ? 1 : 0], 1ull);
}

hipError_t launch_sample_features(int sk, bool swapped, const void *f, const uint8_t *flags, const int32_t *pid,
                                  const PState *ps, const PConst *pc, int np, const Geo &g, const Phys<double> &ph,
                                  double gamma, float *out, hipStream_t st)
{
    if (np <= 0) return hipSuccess;
    const int sw = swapped ? 1 : 0;
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_features<float>, dim3(np), dim3(FB), 0, st, (const float *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    case S_F16: hipLaunchKernelGGL(k_features<_Float16>, dim3(np), dim3(FB), 0, st, (const _Float16 *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    case S_BF16: hipLaunchKernelGGL(k_features<bf16s>, dim3(np), dim3(FB), 0, st, (const bf16s *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    default: hipLaunchKernelGGL(k_features<double>, dim3(np), dim3(FB), 0, st, (const double *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_closure_step(int sk, bool swapped, const void *f, const uint8_t *flags, const int32_t *pid,
                               const PState *ps, const PConst *pc, int np, const Geo &g, const Phys<double> &ph,
                               double gamma, const MlpDev &m, double rho0, double nu, double *corr,
                               unsigned long long *stats, hipStream_t st)
{
    if (np <= 0) return hipSuccess;
    const int sw = swapped ? 1 : 0;
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_closure_step<float>, dim3(np), dim3(FB), 0, st, (const float *)f, flags, pid, ps, pc, g, ph, sw, gamma, m, rho0, nu, corr, stats); break;
    case S_F16: hipLaunchKernelGGL(k_closure_step<_Float16>, dim3(np), dim3(FB), 0, st, (const _Float16 *)f, flags, pid, ps, pc, g, ph, sw, gamma, m, rho0, nu, corr, stats); break;
    case S_BF16: hipLaunchKernelGGL(k_closure_step<bf16s>, dim3(np), dim3(FB), 0, st, (const bf16s *)f, flags, pid, ps, pc, g, ph, sw, gamma, m, rho0, nu, corr, stats); break;
    default: hipLaunchKernelGGL(k_closure_step<double>, dim3(np), dim3(FB), 0, st, (const double *)f, flags, pid, ps, pc, g, ph, sw, gamma, m, rho0, nu, corr, stats); break;
    }
    return hipGetLastError();
}

}  // namespace lbm
