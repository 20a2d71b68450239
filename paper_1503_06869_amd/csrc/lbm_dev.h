// lbm_dev.h -- device-side data structures, lattice tables and the launch
// interface shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct lbm_mlp;

namespace lbm {

// ---------------------------------------------------------------------------
// D3Q19 velocity set (Sec. 4.1: weights 1/3, 1/18, 1/36).  Order used on the
// device and at the ABI: 0 = rest, 1..9 one of each opposite pair, q+9 the
// opposite of q.  Keeping opposites nine apart lets the TRT pairs and the
// AA slot swap be written as q <-> q+9.
// ---------------------------------------------------------------------------
constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
constexpr int CY[Q] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
constexpr int CZ[Q] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : (q <= 9 ? q + 9 : q - 9); }
// Specular reflection (Sec. 4.1, Eq. FreeSlipBC): the direction with the
// components of c_q selected by m (bit 0: x, 1: y, 2: z) reversed.
__host__ __device__ constexpr int refl(int q, int m)
{
    const int ex = (m & 1) ? -CX[q] : CX[q], ey = (m & 2) ? -CY[q] : CY[q], ez = (m & 4) ? -CZ[q] : CZ[q];
    int r = q;
    for (int k = 0; k < Q; ++k)
        if (CX[k] == ex && CY[k] == ey && CZ[k] == ez) r = k;
    return r;
}
// the same as a choice among the eight reflections of q, which fold to
// constants where q is known at compile time (unrolled loops over q)
__host__ __device__ __forceinline__ int refl_sel(int q, int m)
{
    return m == 0 ? q
         : m == 1 ? refl(q, 1)
         : m == 2 ? refl(q, 2)
         : m == 3 ? refl(q, 3)
         : m == 4 ? refl(q, 4)
         : m == 5 ? refl(q, 5)
         : m == 6 ? refl(q, 6)
                  : refl(q, 7);
}
__host__ __device__ constexpr double wq(int q)
{
    return q == 0 ? 1.0 / 3.0 : ((q <= 3 || (q >= 10 && q <= 12)) ? 1.0 / 18.0 : 1.0 / 36.0);
}

// cell flags
constexpr uint8_t F_SOLID = 1;   // cell centre inside a fiber
constexpr uint8_t F_NEAR = 2;    // fluid cell with at least one fiber neighbour

// uint32 division by a runtime constant (round-up multiply-shift method)
struct FastDiv {
    uint32_t m, s;
};
inline FastDiv make_fastdiv(uint32_t d)
{
    if ((d & (d - 1)) == 0) {
        uint32_t s = 0;
        while ((1u << s) < d) ++s;
        return {0u, s};
    }
    uint32_t l = 32 - __builtin_clz(d - 1);
    uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    return {uint32_t(m), l};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f)
{
    if (f.m == 0) return n >> f.s;
    uint32_t t = __umulhi(n, f.m);
    return (t + ((n - t) >> 1)) >> (f.s - 1);
}

// ---------------------------------------------------------------------------
// Particle data (FP64 throughout)
// ---------------------------------------------------------------------------
struct PState {            // one fiber, state at a time level
    double X[3];           // centre of mass
    double q[4];           // orientation (w, x, y, z)
    double V[3];           // velocity
    double W[3];           // angular velocity (world frame)
    double L[3];           // angular momentum (world frame)
    double t[3];           // axis R(q) e_x
    double have_prev;      // 1: F0p, M0p hold the previous step's sums
    double F0p[3], M0p[3]; // velocity-free momentum-exchange sums of the step that led here
};
struct PConst {
    double length, radius, mass, i_par, i_perp;
    int64_t traj_off;      // offset (rows) into the trajectory array, or -1
    int64_t traj_n;        // rows prescribed
    int32_t shape;         // 0 cylinder, 1 spherocylinder (L including the caps)
    double fext[3], mext[3];   // constant external force and torque
};
// Constants of a fiber (host side): mass and principal moments of inertia
// of the cylinder or spherocylinder of the given density, external load.
inline PConst fiber_constants(double length, double radius, double density, int shape, const double force[3],
                              const double torque[3])
{
    const double pi = 3.14159265358979323846;
    PConst pc{};
    pc.length = length;
    pc.radius = radius;
    pc.shape = shape;
    const double r2 = radius * radius;
    if (shape == 1) {
        const double h = length - 2.0 * radius;
        const double mc = density * pi * r2 * h, ms = density * 4.0 / 3.0 * pi * r2 * radius;
        pc.mass = mc + ms;
        pc.i_par = 0.5 * mc * r2 + 0.4 * ms * r2;
        pc.i_perp = mc * (3.0 * r2 + h * h) / 12.0 + ms * (0.4 * r2 + 0.25 * h * h + 0.375 * h * radius);
    } else {
        pc.mass = density * pi * radius * radius * length;
        pc.i_par = 0.5 * pc.mass * radius * radius;
        pc.i_perp = pc.mass * (3.0 * radius * radius + length * length) / 12.0;
    }
    for (int k = 0; k < 3; ++k) {
        pc.fext[k] = force ? force[k] : 0.0;
        pc.mext[k] = torque ? torque[k] : 0.0;
    }
    pc.traj_off = -1;
    pc.traj_n = 0;
    return pc;
}
struct Box {               // cells lo[k] .. lo[k]+len[k]-1 (wrapped where periodic)
    int32_t lo[3];
    int32_t len[3];
};
constexpr int NBR_CAP = 128;   // neighbours per fiber whose boxes may intersect

// Per-fiber sums of the momentum exchange: F0[3] M0[3], then the exact
// integer sums SA[6] (symmetric: xx xy xz yy yz zz) SB[9] SC[6] from which
// the matrices A, B, C of the part linear in the surface velocity are formed
// (abc_restore).  F0 and M0 are accumulated as int64 fixed point (each
// link's FP64 term scaled by 2^FX_k and rounded); SA, SB, SC are integers
// to begin with.  Either way the sums are exact and do not depend on the
// order in which links are added; FP64 is restored once per step.  Ranges:
// |F0| < 2^11, |M0| < 2^17; |SC| stays below 2^53 for fibers of a million
// links within 2^20 cells of their reference point.
constexpr int NACC = 27;
constexpr int NABC = NACC - 6;   // the population-free sums SA, SB, SC
__host__ __device__ constexpr int fx_shift(int k)
{
    return k < 3 ? 52 : (k < 6 ? 46 : 0);
}

// device-side counters and error flags
struct DevCounters {
    uint32_t list_count;       // boundary-cell list length
    uint32_t err_unstable;     // bit 0: non-finite F/M seen; bit 1: non-finite population
    uint32_t err_capacity;     // list or neighbour capacity exceeded
    unsigned long long overlaps;
    uint32_t err_wall;         // a fiber came within one cell of an x or y wall
    uint32_t pad;
    unsigned long long step;   // steps completed by the particle kernel (history index)
};

// ---------------------------------------------------------------------------
// Kernel argument bundles
// ---------------------------------------------------------------------------
struct Geo {
    uint32_t nx, ny, nz, nxy;
    uint32_t ncell;
    uint64_t qstride;          // elements per direction array: (nz+2) * nxy
    FastDiv dnx, dnxy;
    int32_t zper;
    int32_t xw, yw;            // walls half-way outside the x (y) faces: 0 none (periodic),
                               // 1 resting no-slip, 2 free-slip
    int32_t zs;                // 1: the z walls (zper = 0) are free-slip, not moving no-slip
};

template <typename R>
struct Phys {
    R rho0, omega_e, omega_o, wall_u;
    R g[3];
    int32_t has_g;
    R scale, inv_scale;        // storage scaling of the deviation
};

struct BndData {               // boundary-cell list and particle access for the sweep
    const uint32_t *cell;
    const uint32_t *mask;      // bit q (1..18) set: neighbour x + c_q is a fiber cell
    const uint32_t *seg_off;   // [np] start of each fiber's list segment
    const uint32_t *seg_cnt;   // [np] entries in each segment
    const uint32_t *seg_cap;   // [np] capacity of each segment
    int32_t np;
    int32_t bpf;               // blocks per fiber segment
    const int32_t *pid;
    const PState *ps;          // state at the time level of the sweep
    long long *mea;            // [np][NACC] fixed-point momentum-exchange sums
    DevCounters *ctr;          // error flags
};

struct PartData {
    int32_t np;
    const PConst *pc;
    PState *ps_cur, *ps_next;
    PState *ps_prev;           // pose of the previous step (saved by the rigid update)
    Box *box_cur;              // box of the current pose
    Box *box_prev;             // box of the previous pose
    Box *box_remap;            // union of the boxes of the previous, current and new poses
    const double *traj;        // prescribed rows [.][13]
    int64_t *traj_pos;         // [np] rows consumed
    double *ft_out;            // [np][6] F, M of the step
    double *hist;              // ring [cap][np][19]
    int64_t hist_cap;
    int32_t coupling;          // lbm_coupling
    double rho0;
    double rho0_link;          // rho0 as the collision type holds it (k = 6 w rho0 of the link sums)
    const double *corr;        // [np][6] closure corrections dF, dM, or null
    DevCounters *ctr;
    uint32_t list_cap;
    int32_t nslab;             // blocks per fiber (z-planes of a box dealt round robin)
    long long *mea;            // [np][NACC] fixed-point momentum-exchange sums
    const uint32_t *seg_off;   // [np] list segment of each fiber: start
    const uint32_t *seg_cap;   // [np] capacity
    uint32_t *seg_cnt;         // [np] entries
    uint32_t *cov;             // cells whose owner changed (stabilization), or null
    uint32_t cov_cap;
    double contact_k;          // > 0: repulsion between fibers of stiffness contact_k
    double contact_range;      // gap below which it acts
};

// ---------------------------------------------------------------------------
// Launch wrappers (defined in sweep.hip / particles.hip)
// ---------------------------------------------------------------------------
enum StorageKind { S_F32 = 0, S_F16 = 1, S_BF16 = 2, S_F64 = 3 };

hipError_t launch_init(int sk, void *f, const Geo &g, double rho0, double wall_u, int couette,
                       double scale, hipStream_t st);
// Momentum stabilization (stab.hip).  Device buffer stab: [0..2] the mean
// fluid velocity the collisions of the coming step subtract, [3] the fluid
// cell count, [4..7] unused, then 4 doubles per workgroup of the sweep
// kernels (bulk workgroups first, then the boundary-cell workgroups).  cov:
// [0] entries, then cells whose owner changed in the remap (bit 31: fluid
// again, else newly covered).
constexpr int STAB_HEAD = 8;
constexpr uint32_t COV_UNCOVERED = 0x80000000u;
// the next step's mean from this step's workgroup sums (nslot of them) and
// the changed cells, read in the layout of the next sweep (swapped: odd)
hipError_t launch_stab_update(int sk, bool swapped, const void *f, const Geo &g, const Phys<double> &ph,
                              double *stab, uint32_t nslot, uint32_t *cov, uint32_t cov_cap, hipStream_t st);
// the mean of the current state by a pass over all cells (after set-up)
hipError_t launch_stab_scan(int sk, bool swapped, const void *f, const int32_t *pid, const Geo &g,
                            const Phys<double> &ph, double *stab, uint32_t *cov, hipStream_t st);
constexpr uint32_t STAB_SCAN_GRID = 1024;

// bulk sweep on st (bracketed by ev0/ev1 if given); skipped when the grid is
// 0; with stab (else null) the stabilized collision writing its workgroup
// sums to part
hipError_t launch_sweep(int sk, bool odd, void *f, const uint8_t *flags, const Geo &g, const Phys<double> &ph,
                        uint32_t sweep_grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, const double *stab,
                        double *part);
// boundary cells of the list (update, F0, M0) and the integer A, B, C sums
// of their links, one launch (boundary.hip); stab and part as for the sweep
hipError_t launch_boundary(int sk, bool odd, void *f, const Geo &g, const Phys<double> &ph, const BndData &b,
                           hipStream_t st, const double *stab, double *part);
hipError_t launch_decode(int sk, bool swapped, const void *f, const uint8_t *flags,
                         const int32_t *pid, const PState *ps, const Geo &g, const Phys<double> &ph,
                         void *rho, void *u, double *fout, hipStream_t st);
// decode of the cells [c0, c1) only: rho[cell - c0], u[k * ustride + cell - c0]
hipError_t launch_decode_range(int sk, bool swapped, const void *f, const uint8_t *flags,
                               const int32_t *pid, const PState *ps, const Geo &g,
                               const Phys<double> &ph, void *rho, void *u, double *fout,
                               uint32_t c0, uint32_t c1, uint64_t ustride, hipStream_t st);
hipError_t launch_encode(int sk, bool swapped, void *f, const Geo &g, double rho0, double scale,
                         const double *fin, hipStream_t st);
hipError_t launch_rigid(const PartData &pd, const Geo &g, hipStream_t st);
hipError_t launch_setup_boxes(const PartData &pd, const Geo &g, hipStream_t st);
hipError_t launch_remap(int sk, bool next_odd, void *f, int32_t *pid, const PartData &pd, const Geo &g,
                        double rho0, double scale, hipStream_t st);
hipError_t launch_near(uint8_t *flags, const int32_t *pid, uint32_t *list_cell, uint32_t *list_mask,
                       const PartData &pd, const Geo &g, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t nbytes, hipStream_t st);
// non-finite stored populations (n elements of the population array) set
// bit 1 of ctr->err_unstable (check.hip)
hipError_t launch_check_finite(int sk, const void *f, uint64_t n, DevCounters *ctr, hipStream_t st);

// closure network (mlp.hip) and feature sampling (features.hip)
struct MlpDev {
    const uint16_t *wb;        // BF16 parameters
    const float *in_mean, *in_inv_std, *out_scale, *env_min, *env_max;
};
MlpDev mlp_device_view(const ::lbm_mlp *m);
hipError_t launch_mlp_forward(const MlpDev &m, const float *x, int n, float *y, hipStream_t st);
// one step's closure of np fibers (features, network, correction into
// corr[np][6], applied/fallback counts into stats[2]), one launch
hipError_t launch_closure_step(int sk, bool swapped, const void *f, const uint8_t *flags, const int32_t *pid,
                               const PState *ps, const PConst *pc, int np, const Geo &g, const Phys<double> &ph,
                               double gamma, const MlpDev &m, double rho0, double nu, double *corr,
                               unsigned long long *stats, hipStream_t st);
// features [np][247] of np fibers whose states are ps[k * ps_stride] (one
// lattice: the arrays of that lattice)
hipError_t launch_sample_features(int sk, bool swapped, const void *f, const uint8_t *flags, const int32_t *pid,
                                  const PState *ps, const PConst *pc, int np, const Geo &g,
                                  const Phys<double> &ph, double gamma, float *out, hipStream_t st);

}  // namespace lbm
