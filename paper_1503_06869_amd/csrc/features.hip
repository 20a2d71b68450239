// features.hip -- the flow features of a fiber for the learned closure:
// velocities relative to the fiber's rigid motion on a 3 x 27 stencil
// (centre and both tips, offsets {-2,0,2}^3 cells along the body axes),
// trilinear in the cell-centre velocities, expressed in the body frame and
// scaled by 1 / (gamma L), and the orientation.  One workgroup per fiber,
// one thread per stencil point.
#include "lbm_sweep_dev.h"

namespace lbm {

constexpr int NFEAT = 247;

// velocity at the centre of cell (x, y, z): decoded from the populations at
// the current parity for a fluid cell (as the field readback does), the
// rigid-body velocity of the owner for a fiber cell
template <typename S>
__device__ void cell_velocity(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                              const int32_t *__restrict__ pid, const PState *__restrict__ ps, const Geo &g,
                              const Phys<double> &ph, int swapped, uint32_t x, uint32_t y, uint32_t z, double u[3])
{
    using R = typename St<S>::R;
    const uint32_t cell = (z * g.ny + y) * g.nx + x;
    if (flags[cell] & F_SOLID) {
        surf_vel(ps[pid[cell]], double(x), double(y), double(z), g, u);
        return;
    }
    double j[3] = {0.0, 0.0, 0.0};
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
        const double fv = double(St<S>::ld(f, uint64_t(qq) * g.qstride + src, R(ph.inv_scale)));
        j[0] += CX[q] * fv;
        j[1] += CY[q] * fv;
        j[2] += CZ[q] * fv;
    }
    for (int k = 0; k < 3; ++k) u[k] = j[k] / ph.rho0 + 0.5 * ph.g[k];
}

template <typename S>
__global__ __launch_bounds__(128) void k_features(const S *__restrict__ f, const uint8_t *__restrict__ flags,
                                                  const int32_t *__restrict__ pid, const PState *__restrict__ ps,
                                                  const PConst *__restrict__ pc, Geo g, Phys<double> ph,
                                                  int swapped, double gamma, float *__restrict__ out)
{
    const int p = blockIdx.x, k = threadIdx.x;
    const PState s = ps[p];
    const double L = pc[p].length, vs = 1.0 / (gamma * L);
    float *o = out + size_t(p) * NFEAT;
    // body frame: columns e0 = t (axis), e1 = R(q) e_y, e2 = R(q) e_z
    const double w = s.q[0], qx = s.q[1], qy = s.q[2], qz = s.q[3];
    const double Rm[3][3] = {{1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - w * qz), 2.0 * (qx * qz + w * qy)},
                             {2.0 * (qx * qy + w * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - w * qx)},
                             {2.0 * (qx * qz - w * qy), 2.0 * (qy * qz + w * qx), 1.0 - 2.0 * (qx * qx + qy * qy)}};
    if (k < 81) {
        const int pt = k / 27, m = k % 27;
        const double ob[3] = {2.0 * (m % 3 - 1), 2.0 * ((m / 3) % 3 - 1), 2.0 * (m / 9 - 1)};
        const double side = pt == 0 ? 0.0 : (pt == 1 ? 0.5 * L : -0.5 * L);
        // offset from the centre of mass (lab frame), then the sample position
        double d[3];
        for (int e = 0; e < 3; ++e) d[e] = side * Rm[e][0] + (Rm[e][0] * ob[0] + Rm[e][1] * ob[1] + Rm[e][2] * ob[2]);
        const double px = s.X[0] + d[0], py = s.X[1] + d[1];
        double pz = s.X[2] + d[2];
        const double zmax = double(g.nz) - 1.0;
        pz = pz < 0.0 ? 0.0 : (pz > zmax ? zmax : pz);
        const double fx0 = floor(px), fy0 = floor(py);
        int32_t z0 = int32_t(floor(pz));
        if (z0 > int32_t(g.nz) - 2) z0 = int32_t(g.nz) - 2;
        const double ax = px - fx0, ay = py - fy0, az = pz - double(z0);
        const int32_t x0 = int32_t(fx0), y0 = int32_t(fy0);
        double u[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 8; ++c) {
            const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
            const double wt = (cx ? ax : 1.0 - ax) * (cy ? ay : 1.0 - ay) * (cz ? az : 1.0 - az);
            int32_t xx = (x0 + cx) % int32_t(g.nx), yy = (y0 + cy) % int32_t(g.ny);
            xx += xx < 0 ? int32_t(g.nx) : 0;
            yy += yy < 0 ? int32_t(g.ny) : 0;
            double uc[3];
            cell_velocity<S>(f, flags, pid, ps, g, ph, swapped, uint32_t(xx), uint32_t(yy), uint32_t(z0 + cz), uc);
            for (int e = 0; e < 3; ++e) u[e] += wt * uc[e];
        }
        // velocity relative to the rigid motion, in the body frame
        const double v[3] = {u[0] - (s.V[0] + (s.W[1] * d[2] - s.W[2] * d[1])),
                             u[1] - (s.V[1] + (s.W[2] * d[0] - s.W[0] * d[2])),
                             u[2] - (s.V[2] + (s.W[0] * d[1] - s.W[1] * d[0]))};
        for (int e = 0; e < 3; ++e)
            o[k * 3 + e] = float((Rm[0][e] * v[0] + Rm[1][e] * v[1] + Rm[2][e] * v[2]) * vs);
    } else if (k < 85) {
        const double sg = s.q[0] < 0.0 ? -1.0 : 1.0;
        o[243 + (k - 81)] = float(sg * s.q[k - 81]);
    }
}

hipError_t launch_sample_features(int sk, bool swapped, const void *f, const uint8_t *flags, const int32_t *pid,
                                  const PState *ps, const PConst *pc, int np, const Geo &g, const Phys<double> &ph,
                                  double gamma, float *out, hipStream_t st)
{
    if (np <= 0) return hipSuccess;
    const int sw = swapped ? 1 : 0;
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_features<float>, dim3(np), dim3(128), 0, st, (const float *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    case S_F16: hipLaunchKernelGGL(k_features<_Float16>, dim3(np), dim3(128), 0, st, (const _Float16 *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    case S_BF16: hipLaunchKernelGGL(k_features<bf16s>, dim3(np), dim3(128), 0, st, (const bf16s *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    default: hipLaunchKernelGGL(k_features<double>, dim3(np), dim3(128), 0, st, (const double *)f, flags, pid, ps, pc, g, ph, sw, gamma, out); break;
    }
    return hipGetLastError();
}

}  // namespace lbm
