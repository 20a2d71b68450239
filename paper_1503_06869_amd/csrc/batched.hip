// batched.hip -- the batched form: many small independent shear cells, one
// fiber each, advanced by one persistent launch.
//
// Each case is the full coupled method (Sec. 4): the AA stream-collide sweep
// with wall and fiber bounce-back and the momentum exchange, the rigid-body
// update, the remap with refill and the boundary-list rebuild.  The cases
// are packed into bins; workgroup b runs the cases of bin b, one after the
// other, all steps of a case in a row, with __syncthreads() between the
// phases of a step.  No workgroup waits for another, so the launch cannot
// stall on residency, and there are no device-wide fences or atomics.
//
// The per-cell update, the link terms of the momentum exchange, the rigid
// update, the cell predicate, the rectangles and the refill are the same
// device functions the single-lattice kernels use, and the momentum-exchange
// sums are exact int64 fixed point, so a case reproduces the single-lattice
// run of the same parameters bit for bit.  One difference of organisation
// keeps the sweep's register use low: the population-free sums of the
// exchange (the A, B, C matrices, terms 6..26) are formed while the list is
// rebuilt, from the new pose, and the sweep accumulates only F0 and M0.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbm_batch.h"
#include "../../include/lbm_mlp.h"
#include "lbm_sweep_dev.h"
#include "lbm_particle_dev.h"   // FP contraction off from here on, as in particles.hip

namespace lbm {

constexpr int BMAXP = 512;   // planes of a case (nz <= 512)

struct CaseDev {
    Geo g;
    Phys<float> pf;
    Phys<double> pd;
    uint64_t f_off;      // first population element of the case
    uint64_t cell_off;   // first element of its cell arrays (flags, pid)
    uint32_t list_off, list_cap;
    PConst pc;
};

struct BatchDev {
    const CaseDev *cases;
    const int32_t *bin_case;   // case ids of all bins, concatenated
    const int32_t *bin_off;    // [bins + 1]
    void *f;
    uint8_t *flags;
    int32_t *pid;
    uint32_t *list_cell, *list_mask;
    uint32_t *list_n;          // [ncase] entries found by the last rebuild (may exceed the cap)
    PState *ps;                // [ncase][2]: state at even / odd time levels
    Box *box_cur;              // [ncase]
    long long *abc;            // [ncase][NABC] population-free integer sums (SA, SB, SC) for the next step
    long long *foreign;        // [NACC] sink for links to another fiber (none in a one-fiber case)
    double *ft;                // [ncase][6]
    double *hist;              // [ncase][hist_cap][19]
    int64_t hist_cap;
    int64_t *steps;            // [ncase] steps completed
    const double *traj;        // prescribed rows [.][13]
    int64_t *traj_pos;         // [ncase]
    DevCounters *ctr;
    int32_t coupling;          // lbm_coupling
};

template <int BS>
struct BShared {
    long long red[BS / 64][NACC];
    long long tot[NACC];
    PState cur, nxt;
    Box ub;
    Rect rect[BMAXP];
    int32_t zpl[BMAXP];
    uint32_t aoff[BMAXP + 1];
    uint32_t nlist;
};

// A value that every lane loads from the same address: keep it in scalar
// registers (the compiler cannot prove that memory written by the kernel is
// uniform when read back).
template <typename T>
__device__ __forceinline__ T uniform(const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    T r;
    const int *s = reinterpret_cast<const int *>(&v);
    int *d = reinterpret_cast<int *>(&r);
#pragma unroll
    for (int k = 0; k < int(sizeof(T) / 4); ++k) d[k] = __builtin_amdgcn_readfirstlane(s[k]);
    return r;
}

template <typename S>
using RefillT = typename std::conditional<std::is_same<S, bf16s>::value, uint16_t, S>::type;

template <typename R>
__device__ __forceinline__ const Phys<R> &case_phys(const CaseDev &cd);
template <>
__device__ __forceinline__ const Phys<float> &case_phys<float>(const CaseDev &cd) { return cd.pf; }
template <>
__device__ __forceinline__ const Phys<double> &case_phys<double>(const CaseDev &cd) { return cd.pd; }

// out[k] = sum over the workgroup of acc[k], k < NK (exact: integers)
template <int BS, int NK>
__device__ __forceinline__ void block_sum(const long long (&acc)[NK], BShared<BS> &sh, long long *out)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        long long v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) sh.red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NK) {
        long long v = 0;
        for (int w = 0; w < BS / 64; ++w) v += sh.red[w][threadIdx.x];
        out[threadIdx.x] = v;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ sweep of one case
template <typename S, bool ODD, int BS>
__device__ __forceinline__ void case_sweep(const BatchDev &bd, S *__restrict__ f, const uint8_t *__restrict__ flags,
                                           int c, const CaseDev &cd, int64_t s, BShared<BS> &sh)
{
    using R = typename St<S>::R;
    const Phys<R> &ph = case_phys<R>(cd);
    S *fc = f + cd.f_off;
    const uint8_t *flc = flags + cd.cell_off;
    for (uint32_t cell = threadIdx.x; cell < cd.g.ncell; cell += BS)
        if (!flc[cell]) update_cell<S, ODD, false>(fc, cd.g, ph, cell, 0u, -1, nullptr, BndData{});
    BndData b{};
    b.pid = bd.pid + cd.cell_off;
    b.ps = bd.ps + size_t(c) * 2 + size_t(s & 1);
    b.mea = bd.foreign;
    b.ctr = bd.ctr;
    const uint32_t cnt = uniform(bd.list_n[c]);
    const uint32_t n = cnt < cd.list_cap ? cnt : cd.list_cap;
    const uint32_t *lc = bd.list_cell + cd.list_off, *lm = bd.list_mask + cd.list_off;
    long long acc[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t r = threadIdx.x; r < n; r += BS)
        update_cell<S, ODD, true, 6>(fc, cd.g, ph, lc[r], lm[r], 0, acc, b);
    block_sum<BS, 6>(acc, sh, sh.tot);
}

// ------------------------------------------------------------------ particle phase of one case
// Rigid update from the sums (skipped when mapping the initial pose), boxes,
// remap with refill, flags and boundary list, and the population-free sums
// of the next sweep.  Ends with a workgroup barrier.
template <typename S, int BS>
__device__ __forceinline__ void case_particles(const BatchDev &bd, int c, const CaseDev &cd, int64_t s, BShared<BS> &sh,
                               bool setup)
{
    using R = typename St<S>::R;
    const Geo &g = cd.g;
    const int cur = int(s & 1), nxt = setup ? cur : int((s + 1) & 1);
    if (threadIdx.x == 0) {
        const PState so = bd.ps[size_t(c) * 2 + cur];
        PState o = so;
        if (!setup) {
            double ac[NACC];
            for (int k = 0; k < 6; ++k) ac[k] = ldexp(double(sh.tot[k]), -fx_shift(k));
            for (int k = 6; k < NACC; ++k) ac[k] = double(bd.abc[size_t(c) * NABC + k - 6]);
            abc_restore(ac, so.X, double(case_phys<R>(cd).rho0));
            const double *row = nullptr;
            if (cd.pc.traj_off >= 0 && bd.traj_pos[c] < cd.pc.traj_n) {
                row = bd.traj + (cd.pc.traj_off + bd.traj_pos[c]) * 13;
                bd.traj_pos[c] += 1;
            }
            double F[3], M[3];
            rigid_update(so, cd.pc, ac, bd.coupling, row, g, o, F, M);
            bool bad = false;
            for (int k = 0; k < 3; ++k) bad |= !isfinite(F[k]) || !isfinite(M[k]);
            if (bad) atomicOr(&bd.ctr->err_unstable, 1u);
            bd.ps[size_t(c) * 2 + nxt] = o;
            for (int k = 0; k < 3; ++k) {
                bd.ft[size_t(c) * 6 + k] = F[k];
                bd.ft[size_t(c) * 6 + 3 + k] = M[k];
            }
            double *h = bd.hist + (size_t(c) * bd.hist_cap + size_t(s % bd.hist_cap)) * 19;
            for (int k = 0; k < 3; ++k) { h[k] = F[k]; h[3 + k] = M[k]; h[6 + k] = o.X[k]; }
            for (int k = 0; k < 4; ++k) h[9 + k] = o.q[k];
            for (int k = 0; k < 3; ++k) { h[13 + k] = o.V[k]; h[16 + k] = o.W[k]; }
        }
        Box ub, nb;
        remap_boxes(o, cd.pc, bd.box_cur[c], g, ub, nb);
        bd.box_cur[c] = nb;
        sh.cur = so;
        sh.nxt = o;
        sh.ub = ub;
        sh.nlist = 0u;
    }
    __syncthreads();
    // plane rectangles of the remap region (both poses), then their offsets
    const Box ub = sh.ub;
    const int32_t nz = g.nz, nplane = ub.len[2] < BMAXP ? ub.len[2] : BMAXP;
    for (int k = threadIdx.x; k < nplane; k += BS) {
        int32_t z = ub.lo[2] + k;
        bool ok = true;
        if (g.zper) z = wrapc(z, nz);
        else ok = z >= 0 && z < nz;
        Rect r{1, 0, 1, 0};
        if (ok) r = rect_union(plane_rect(sh.cur, cd.pc, z, ub, g), plane_rect(sh.nxt, cd.pc, z, ub, g), g);
        sh.zpl[k] = ok ? z : -1;
        sh.rect[k] = r;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        uint32_t a[BMAXP / 64], sum = 0;
#pragma unroll
        for (int j = 0; j < BMAXP / 64; ++j) {
            const int k = l * (BMAXP / 64) + j;
            uint32_t v = 0;
            if (k < nplane && sh.zpl[k] >= 0) {
                const Rect r = sh.rect[k];
                if (r.x0 <= r.x1 && r.y0 <= r.y1) v = uint32_t(r.x1 - r.x0 + 1) * uint32_t(r.y1 - r.y0 + 1);
            }
            a[j] = v;
            sum += v;
        }
        uint32_t inc = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(inc, o, 64);
            if (l >= o) inc += v;
        }
        uint32_t run = inc - sum;
#pragma unroll
        for (int j = 0; j < BMAXP / 64; ++j) {
            const int k = l * (BMAXP / 64) + j;
            if (k < nplane) sh.aoff[k] = run;
            run += a[j];
        }
        if (l == 63) sh.aoff[nplane] = inc;
    }
    __syncthreads();
    const uint32_t total = sh.aoff[nplane];
    int32_t *pidc = bd.pid + cd.cell_off;
    uint8_t *flc = bd.flags + cd.cell_off;
    const int next_odd = setup ? int(s & 1) : int((s + 1) & 1);
    const double rho0 = cd.pd.rho0, scale = cd.pd.scale;
    RefillT<S> *fr = reinterpret_cast<RefillT<S> *>(bd.f) + cd.f_off;
    // cell (x, y, z) of the i-th cell of the region
    auto locate = [&](uint32_t i, int32_t &x, int32_t &y, int32_t &z) {
        int lo = 0, hi = nplane;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sh.aoff[mid] <= i) lo = mid;
            else hi = mid;
        }
        const Rect r = sh.rect[lo];
        const uint32_t loc = i - sh.aoff[lo], wx = uint32_t(r.x1 - r.x0 + 1);
        const uint32_t iy = loc / wx, ix = loc - iy * wx;
        x = wrapi(r.x0 + int32_t(ix), g.nx);
        y = wrapi(r.y0 + int32_t(iy), g.ny);
        z = sh.zpl[lo];
    };
    // remap: new owner of every cell of the region; refill of uncovered cells
    for (uint32_t i = threadIdx.x; i < total; i += BS) {
        int32_t x, y, z;
        locate(i, x, y, z);
        const int owner = inside(sh.nxt, cd.pc, double(x), double(y), double(z), g) ? 0 : -1;
        const uint32_t cell = (uint32_t(z) * g.ny + uint32_t(y)) * g.nx + uint32_t(x);
        const int old = pidc[cell];
        if (old >= 0 && owner < 0) refill_cell<RefillT<S>>(fr, g, x, y, z, sh.cur, rho0, scale, next_odd);
        pidc[cell] = owner;
    }
    __syncthreads();
    // flags, boundary list, and the population-free link sums at the new pose
    uint32_t *lc = bd.list_cell + cd.list_off, *lm = bd.list_mask + cd.list_off;
    long long acc[NABC];
#pragma unroll
    for (int k = 0; k < NABC; ++k) acc[k] = 0;
    int32_t xr[3];
    fiber_ref(sh.nxt.X, xr);
    for (uint32_t i = threadIdx.x; i < total; i += BS) {
        int32_t x, y, z;
        locate(i, x, y, z);
        const uint32_t cell = (uint32_t(z) * g.ny + uint32_t(y)) * g.nx + uint32_t(x);
        if (pidc[cell] >= 0) {
            flc[cell] = F_SOLID;
            continue;
        }
        const uint32_t mask = fiber_mask(pidc, g, x, y, z);
        if (!mask) {
            flc[cell] = 0;
            continue;
        }
        const uint32_t r = atomicAdd(&sh.nlist, 1u);
        if (r >= cd.list_cap) {
            flc[cell] = 0;
            atomicOr(&bd.ctr->err_capacity, 2u);
            continue;
        }
        lc[r] = cell;
        lm[r] = mask;
        flc[cell] = F_NEAR;
        static_for<1, Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if ((mask >> q) & 1u) {
                // the solid neighbour y = x + c_q, as the sweep forms it
                const uint32_t yx = uint32_t(wrapc(x + CX[q], int32_t(g.nx)));
                const uint32_t yy = (uint32_t(y) + g.ny + CY[q]) % g.ny;
                const int32_t yzi = z + CZ[q];
                const uint32_t yz = g.zper ? uint32_t((yzi + int32_t(g.nz)) % int32_t(g.nz)) : uint32_t(yzi);
                link_int_terms<q>(acc, mi_i(int32_t(yx) - xr[0], int32_t(g.nx), true),
                                  mi_i(int32_t(yy) - xr[1], int32_t(g.ny), true),
                                  mi_i(int32_t(yz) - xr[2], int32_t(g.nz), g.zper != 0));
            }
        });
    }
    block_sum<BS, NABC>(acc, sh, sh.tot + 6);
    if (threadIdx.x < NABC) bd.abc[size_t(c) * NABC + threadIdx.x] = sh.tot[6 + threadIdx.x];
    if (threadIdx.x == 0) bd.list_n[c] = sh.nlist;
    __syncthreads();
}

// ------------------------------------------------------------------ persistent kernel
// Workgroup b runs every case of bin b through nsteps steps (setup != 0:
// maps the initial poses instead).  Register budget: two waves per SIMD for
// 256- and 512-thread workgroups (256 VGPRs: the bulk loop does not spill),
// four for 1024 threads (128 VGPRs: more waves, but spills).
template <typename S, int BS>
__global__ __launch_bounds__(BS, BS == 1024 ? 4 : 2) void k_batch(BatchDev bd, S *__restrict__ f, const uint8_t *__restrict__ flags,
                                                 int32_t nsteps, int32_t setup)
{
    __shared__ BShared<BS> sh;
    const int bin = blockIdx.x;
    const int i0 = uniform(bd.bin_off[bin]), i1 = uniform(bd.bin_off[bin + 1]);
    for (int i = i0; i < i1; ++i) {
        const int c = uniform(bd.bin_case[i]);
        const CaseDev cd = uniform(bd.cases[c]);
        int64_t s = uniform(bd.steps[c]);
        if (setup) {
            case_particles<S, BS>(bd, c, cd, s, sh, true);
            continue;
        }
        for (int k = 0; k < nsteps; ++k, ++s) {
            if (s & 1) case_sweep<S, true, BS>(bd, f, flags, c, cd, s, sh);
            else case_sweep<S, false, BS>(bd, f, flags, c, cd, s, sh);
            case_particles<S, BS>(bd, c, cd, s, sh, false);
        }
        if (threadIdx.x == 0) bd.steps[c] = s;
    }
}

template <typename S>
static hipError_t launch_batch_t(const BatchDev &bd, int threads, int bins, int nsteps, int setup, hipStream_t st)
{
    S *f = reinterpret_cast<S *>(bd.f);
    switch (threads) {
    case 256: hipLaunchKernelGGL((k_batch<S, 256>), dim3(bins), dim3(256), 0, st, bd, f, bd.flags, nsteps, setup); break;
    case 1024: hipLaunchKernelGGL((k_batch<S, 1024>), dim3(bins), dim3(1024), 0, st, bd, f, bd.flags, nsteps, setup); break;
    default: hipLaunchKernelGGL((k_batch<S, 512>), dim3(bins), dim3(512), 0, st, bd, f, bd.flags, nsteps, setup); break;
    }
    return hipGetLastError();
}

static hipError_t launch_batch(int sk, const BatchDev &bd, int threads, int bins, int nsteps, int setup,
                               hipStream_t st)
{
    switch (sk) {
    case S_F32: return launch_batch_t<float>(bd, threads, bins, nsteps, setup, st);
    case S_F16: return launch_batch_t<_Float16>(bd, threads, bins, nsteps, setup, st);
    case S_BF16: return launch_batch_t<bf16s>(bd, threads, bins, nsteps, setup, st);
    default: return launch_batch_t<double>(bd, threads, bins, nsteps, setup, st);
    }
}

}  // namespace lbm

// ====================================================================== host side
using namespace lbm;

struct lbm_batch {
    lbm_batch_params p{};
    std::string err;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int sk = 0;
    size_t esz = 4;
    double scale = 1.0;
    int ncase = 0;
    int cu = 0;
    std::string arch;
    std::vector<lbm_batch_case> hc;
    std::vector<CaseDev> hcd;
    std::vector<PState> ps0;                 // initial states
    std::vector<std::vector<double>> traj_h;
    int threads = 512, bins = 1;
    CaseDev *cases = nullptr;
    int32_t *bin_case = nullptr, *bin_off = nullptr;
    void *f = nullptr;
    uint8_t *flags = nullptr;
    int32_t *pid = nullptr;
    uint32_t *list_cell = nullptr, *list_mask = nullptr, *list_n = nullptr;
    PState *ps = nullptr;
    Box *box_cur = nullptr;
    long long *abc = nullptr, *foreign = nullptr;
    double *ft = nullptr, *hist = nullptr, *traj = nullptr;
    int64_t *steps_d = nullptr, *traj_pos = nullptr;
    DevCounters *ctr = nullptr;
    uint64_t nf = 0, ncells = 0;
    uint64_t nlist = 0;
    int64_t steps = 0;
    int64_t device_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t graph_n = -1;
};

static std::string g_create_err;

static lbm_status bfail(lbm_batch *b, lbm_status s, const std::string &m)
{
    if (b) b->err = m;
    else g_create_err = m;
    return s;
}

#define BHIP(b, call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return bfail((b), e_ == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_HIP,            \
                         std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

template <typename T>
static hipError_t balloc(lbm_batch *b, T **ptr, size_t n)
{
    *ptr = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)ptr, n * sizeof(T));
    if (e == hipSuccess) b->device_bytes += int64_t(n * sizeof(T));
    return e;
}
template <typename T>
static void bfree(T *&p)
{
    if (p) hipFree((void *)p);
    p = nullptr;
}

static void drop_bgraph(lbm_batch *b)
{
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_n = -1;
}

static void host_axis_b(const double q[4], double t[3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    t[0] = 1.0 - 2.0 * (y * y + z * z);
    t[1] = 2.0 * (x * y + w * z);
    t[2] = 2.0 * (x * z - w * y);
}

// the same geometry rules as lbm_add_fiber (walls at the z ends)
static const char *check_case(const lbm_batch_case &k)
{
    if (k.nx < 3 || k.ny < 3 || k.nz < 3 || k.nx > 512 || k.ny > 512 || k.nz > 512) return "size out of range";
    if (!(k.tau > 0.5) || !(std::fabs(k.wall_u) < 0.1)) return "tau or wall_u out of range";
    const lbm_fiber &f = k.fiber;
    if (!(f.length > 0.0) || !(f.radius > 0.0) || !(f.density_ratio > 0.0)) return "bad fiber size";
    if (f.shape != LBM_SHAPE_CYLINDER && f.shape != LBM_SHAPE_SPHEROCYLINDER) return "unknown fiber shape";
    if (f.shape == LBM_SHAPE_SPHEROCYLINDER && !(f.length >= 2.0 * f.radius)) return "spherocylinder shorter than 2 r";
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(f.force[i]) || !std::isfinite(f.torque[i])) return "non-finite external load";
    const double qn = std::sqrt(f.quat[0] * f.quat[0] + f.quat[1] * f.quat[1] + f.quat[2] * f.quat[2] +
                                f.quat[3] * f.quat[3]);
    if (!(qn > 0.0)) return "zero quaternion";
    double q[4], t[3];
    for (int i = 0; i < 4; ++i) q[i] = f.quat[i] / qn;
    host_axis_b(q, t);
    const int n[3] = {k.nx, k.ny, k.nz};
    for (int i = 0; i < 3; ++i) {
        if (!(f.center[i] >= 0.0 && f.center[i] < n[i])) return "fiber centre outside the domain";
        const double ext = f.shape == LBM_SHAPE_SPHEROCYLINDER
                               ? (0.5 * f.length - f.radius) * std::fabs(t[i]) + f.radius
                               : 0.5 * f.length * std::fabs(t[i]) +
                                     f.radius * std::sqrt(std::fmax(0.0, 1.0 - t[i] * t[i]));
        if (i < 2 && !(f.length * 0.5 + f.radius < 0.5 * n[i] - 1.0)) return "fiber longer than half the periodic domain";
        if (i == 2 && (f.center[i] - ext < 1.0 || f.center[i] + ext > n[i] - 2.0)) return "fiber within one cell of a wall";
    }
    return nullptr;
}

static PState make_state_b(const lbm_fiber &f, const PConst &c)
{
    PState s{};
    const double qn = std::sqrt(f.quat[0] * f.quat[0] + f.quat[1] * f.quat[1] + f.quat[2] * f.quat[2] +
                                f.quat[3] * f.quat[3]);
    for (int k = 0; k < 3; ++k) s.X[k] = f.center[k];
    for (int k = 0; k < 4; ++k) s.q[k] = f.quat[k] / qn;
    for (int k = 0; k < 3; ++k) s.V[k] = f.vel[k];
    for (int k = 0; k < 3; ++k) s.W[k] = f.omega[k];
    host_axis_b(s.q, s.t);
    const double tw = s.t[0] * s.W[0] + s.t[1] * s.W[1] + s.t[2] * s.W[2];
    for (int k = 0; k < 3; ++k) s.L[k] = c.i_perp * s.W[k] + (c.i_par - c.i_perp) * tw * s.t[k];
    return s;
}

static BatchDev batch_dev(lbm_batch *b)
{
    BatchDev d{};
    d.cases = b->cases;
    d.bin_case = b->bin_case;
    d.bin_off = b->bin_off;
    d.f = b->f;
    d.flags = b->flags;
    d.pid = b->pid;
    d.list_cell = b->list_cell;
    d.list_mask = b->list_mask;
    d.list_n = b->list_n;
    d.ps = b->ps;
    d.box_cur = b->box_cur;
    d.abc = b->abc;
    d.foreign = b->foreign;
    d.ft = b->ft;
    d.hist = b->hist;
    d.hist_cap = b->p.history_capacity;
    d.steps = b->steps_d;
    d.traj = b->traj;
    d.traj_pos = b->traj_pos;
    d.ctr = b->ctr;
    d.coupling = b->p.coupling;
    return d;
}

// Longest-processing-time packing of the cases into nb bins: cases by
// descending cost (cells plus a per-step constant for the particle phase),
// each into the currently lightest bin.
static lbm_status set_bins(lbm_batch *b, int nb)
{
    drop_bgraph(b);
    nb = std::max(1, std::min(nb, b->ncase));
    std::vector<int> order(b->ncase);
    for (int i = 0; i < b->ncase; ++i) order[i] = i;
    auto cost = [&](int i) { return double(b->hcd[i].g.ncell) + 4096.0; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
    std::vector<std::vector<int>> bin(nb);
    std::vector<double> load(nb, 0.0);
    for (int i : order) {
        int best = 0;
        for (int k = 1; k < nb; ++k)
            if (load[k] < load[best]) best = k;
        bin[best].push_back(i);
        load[best] += cost(i);
    }
    std::vector<int32_t> bc, bo(nb + 1, 0);
    for (int k = 0; k < nb; ++k) {
        bo[k] = int32_t(bc.size());
        bc.insert(bc.end(), bin[k].begin(), bin[k].end());
    }
    bo[nb] = int32_t(bc.size());
    bfree(b->bin_case);
    bfree(b->bin_off);
    BHIP(b, hipMalloc((void **)&b->bin_case, bc.size() * sizeof(int32_t)));
    BHIP(b, hipMalloc((void **)&b->bin_off, bo.size() * sizeof(int32_t)));
    BHIP(b, hipMemcpy(b->bin_case, bc.data(), bc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->bin_off, bo.data(), bo.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    b->bins = nb;
    return LBM_OK;
}

// initial lattice, states and mapping of every case (also after autotuning trials)
static lbm_status reset_state(lbm_batch *b)
{
    drop_bgraph(b);
    for (int i = 0; i < b->ncase; ++i) {
        const CaseDev &cd = b->hcd[i];
        void *fc = static_cast<char *>(b->f) + cd.f_off * b->esz;
        BHIP(b, launch_init(b->sk, fc, cd.g, b->p.rho0, cd.pd.wall_u, b->p.init_profile == LBM_INIT_COUETTE,
                            b->scale, b->st));
    }
    BHIP(b, hipMemsetAsync(b->flags, 0, b->ncells, b->st));
    BHIP(b, hipMemsetAsync(b->pid, 0xFF, b->ncells * sizeof(int32_t), b->st));
    BHIP(b, hipMemsetAsync(b->list_n, 0, b->ncase * sizeof(uint32_t), b->st));
    BHIP(b, hipMemsetAsync(b->box_cur, 0, b->ncase * sizeof(Box), b->st));
    BHIP(b, hipMemsetAsync(b->abc, 0, size_t(b->ncase) * NABC * sizeof(long long), b->st));
    BHIP(b, hipMemsetAsync(b->foreign, 0, NACC * sizeof(long long), b->st));
    BHIP(b, hipMemsetAsync(b->ft, 0, size_t(b->ncase) * 6 * sizeof(double), b->st));
    BHIP(b, hipMemsetAsync(b->steps_d, 0, b->ncase * sizeof(int64_t), b->st));
    BHIP(b, hipMemsetAsync(b->traj_pos, 0, b->ncase * sizeof(int64_t), b->st));
    BHIP(b, hipMemsetAsync(b->ctr, 0, sizeof(DevCounters), b->st));
    std::vector<PState> ps(size_t(b->ncase) * 2);
    for (int i = 0; i < b->ncase; ++i) ps[size_t(i) * 2] = ps[size_t(i) * 2 + 1] = b->ps0[i];
    BHIP(b, hipMemcpyAsync(b->ps, ps.data(), ps.size() * sizeof(PState), hipMemcpyHostToDevice, b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    b->steps = 0;
    BHIP(b, launch_batch(b->sk, batch_dev(b), b->threads, b->bins, 0, 1, b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    return LBM_OK;
}

static lbm_status check_batch_errors(lbm_batch *b)
{
    DevCounters h{};
    BHIP(b, hipMemcpyAsync(&h, b->ctr, sizeof h, hipMemcpyDeviceToHost, b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    if (h.err_unstable) return bfail(b, LBM_E_UNSTABLE, "non-finite force or torque on the device");
    if (h.err_capacity) return bfail(b, LBM_E_STATE, "internal capacity exceeded (boundary list)");
    return LBM_OK;
}

static uint64_t fnv(uint64_t h, const void *p, size_t n)
{
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

static std::string tune_key(const lbm_batch *b)
{
    uint64_t h = 1469598103934665603ull;
    for (const auto &k : b->hc) {
        const int32_t d[3] = {k.nx, k.ny, k.nz};
        h = fnv(h, d, sizeof d);
    }
    h = fnv(h, &b->sk, sizeof b->sk);
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s-cu%d-n%d-%016llx", b->arch.c_str(), b->cu, b->ncase, (unsigned long long)h);
    return buf;
}

extern "C" {

lbm_status lbm_batch_params_default(lbm_batch_params *p)
{
    if (!p) return LBM_E_ARG;
    std::memset(p, 0, sizeof *p);
    p->collision = LBM_TRT;
    p->magic = 3.0 / 16.0;
    p->rho0 = 1.0;
    p->storage = LBM_F32;
    p->init_profile = LBM_INIT_COUETTE;
    p->coupling = LBM_COUPLING_IMPLICIT;
    p->fp16_scale_log2 = 14;
    p->history_capacity = 4096;
    return LBM_OK;
}

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_create_err.c_str(); }

lbm_status lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return LBM_E_ARG;
    if (b->st) hipStreamSynchronize(b->st);
    drop_bgraph(b);
    bfree(b->cases);
    bfree(b->bin_case);
    bfree(b->bin_off);
    bfree(b->f);
    bfree(b->flags);
    bfree(b->pid);
    bfree(b->list_cell);
    bfree(b->list_mask);
    bfree(b->list_n);
    bfree(b->ps);
    bfree(b->box_cur);
    bfree(b->abc);
    bfree(b->foreign);
    bfree(b->ft);
    bfree(b->hist);
    bfree(b->traj);
    bfree(b->steps_d);
    bfree(b->traj_pos);
    bfree(b->ctr);
    if (b->own_stream && b->st) hipStreamDestroy(b->st);
    delete b;
    return LBM_OK;
}

lbm_status lbm_batch_create(const lbm_batch_params *p, const lbm_batch_case *cases, int32_t ncases,
                            lbm_batch **out)
{
    if (!p || !cases || !out || ncases < 1) return bfail(nullptr, LBM_E_ARG, "null argument or no cases");
    *out = nullptr;
    if (p->collision != LBM_TRT && p->collision != LBM_SRT) return bfail(nullptr, LBM_E_ARG, "collision");
    if (p->collision == LBM_TRT && !(p->magic > 0.0)) return bfail(nullptr, LBM_E_ARG, "magic");
    if (!(p->rho0 > 0.0) || p->storage < 0 || p->storage > 3 || p->history_capacity < 1)
        return bfail(nullptr, LBM_E_ARG, "rho0, storage or history_capacity");
    if (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 20) return bfail(nullptr, LBM_E_ARG, "fp16_scale_log2");
    if (p->coupling < LBM_COUPLING_IMPLICIT || p->coupling > LBM_COUPLING_IMPLICIT_PLAIN)
        return bfail(nullptr, LBM_E_ARG, "coupling");
    if (p->threads != 0 && p->threads != 256 && p->threads != 512 && p->threads != 1024)
        return bfail(nullptr, LBM_E_ARG, "threads must be 0, 256, 512 or 1024");
    if (p->bins < 0) return bfail(nullptr, LBM_E_ARG, "bins");
    for (int i = 0; i < ncases; ++i) {
        const char *m = check_case(cases[i]);
        if (m) return bfail(nullptr, LBM_E_GEOM, "case " + std::to_string(i) + ": " + m);
    }
    lbm_batch *b = new (std::nothrow) lbm_batch;
    if (!b) return bfail(nullptr, LBM_E_NOMEM, "host allocation");
    b->p = *p;
    b->ncase = ncases;
    b->hc.assign(cases, cases + ncases);
    b->traj_h.resize(ncases);
    b->sk = p->storage;
    b->esz = b->sk == S_F64 ? 8 : (b->sk == S_F32 ? 4 : 2);
    b->scale = b->sk == S_F16 ? std::ldexp(1.0, p->fp16_scale_log2) : 1.0;
    auto bail = [&](lbm_status s, const std::string &m) {
        g_create_err = m + (b->err.empty() ? "" : ": " + b->err);
        lbm_batch_destroy(b);
        return s;
    };
    b->st = (hipStream_t)p->stream;
    if (!b->st) {
        if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess) return bail(LBM_E_HIP, "stream");
        b->own_stream = true;
    }
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return bail(LBM_E_HIP, "device properties");
    b->cu = prop.multiProcessorCount;
    b->arch = prop.gcnArchName;
    for (auto &ch : b->arch)
        if (ch == ' ' || ch == ':') ch = '_';
    // per-case geometry, physics and offsets
    uint64_t foff = 0, coff = 0, loff = 0;
    b->hcd.resize(ncases);
    b->ps0.resize(ncases);
    for (int i = 0; i < ncases; ++i) {
        const lbm_batch_case &k = cases[i];
        CaseDev &cd = b->hcd[i];
        Geo &g = cd.g;
        g.nx = k.nx;
        g.ny = k.ny;
        g.nz = k.nz;
        g.nxy = uint32_t(k.nx) * uint32_t(k.ny);
        g.ncell = g.nxy * uint32_t(k.nz);
        g.qstride = uint64_t(k.nz + 2) * g.nxy + 64;
        g.dnx = make_fastdiv(g.nx);
        g.dnxy = make_fastdiv(g.nxy);
        g.zper = 0;
        g.xw = g.yw = g.zs = 0;
        Phys<double> &ph = cd.pd;
        ph.rho0 = p->rho0;
        ph.omega_e = 1.0 / k.tau;
        ph.omega_o = p->collision == LBM_SRT ? 1.0 / k.tau : 1.0 / (0.5 + p->magic / (k.tau - 0.5));
        ph.wall_u = k.wall_u;
        for (int j = 0; j < 3; ++j) ph.g[j] = 0.0;
        ph.has_g = 0;
        ph.scale = b->scale;
        ph.inv_scale = 1.0 / b->scale;
        Phys<float> &pf = cd.pf;
        pf.rho0 = float(ph.rho0);
        pf.omega_e = float(ph.omega_e);
        pf.omega_o = float(ph.omega_o);
        pf.wall_u = float(ph.wall_u);
        for (int j = 0; j < 3; ++j) pf.g[j] = 0.0f;
        pf.has_g = 0;
        pf.scale = float(ph.scale);
        pf.inv_scale = float(ph.inv_scale);
        cd.f_off = foff;
        foff += (uint64_t(Q) * g.qstride + 63) / 64 * 64;
        cd.cell_off = coff;
        coff += (uint64_t(g.ncell) + 255) / 256 * 256;
        const lbm_fiber &fb = k.fiber;
        const double r = fb.radius + 2.5, L = fb.length + 5.0;
        const double cap = 1.25 * (M_PI * r * r * L + 4.0 * M_PI * r * r) + 256.0;
        cd.list_off = uint32_t(loff);
        cd.list_cap = uint32_t(cap);
        loff += cd.list_cap;
        cd.pc = fiber_constants(fb.length, fb.radius, fb.density_ratio * p->rho0, fb.shape, fb.force, fb.torque);
        const PConst &pc = cd.pc;
        b->ps0[i] = make_state_b(fb, pc);
    }
    if (loff >= 4294967295ull) return bail(LBM_E_ARG, "boundary lists too large");
    b->nf = foff;
    b->ncells = coff;
    b->nlist = loff;
    if (hipMalloc(&b->f, b->nf * b->esz) != hipSuccess) return bail(LBM_E_NOMEM, "populations");
    b->device_bytes += int64_t(b->nf * b->esz);
    if (balloc(b, &b->cases, ncases) != hipSuccess || balloc(b, &b->flags, b->ncells) != hipSuccess ||
        balloc(b, &b->pid, b->ncells) != hipSuccess || balloc(b, &b->list_cell, b->nlist) != hipSuccess ||
        balloc(b, &b->list_mask, b->nlist) != hipSuccess || balloc(b, &b->list_n, ncases) != hipSuccess ||
        balloc(b, &b->ps, size_t(ncases) * 2) != hipSuccess || balloc(b, &b->box_cur, ncases) != hipSuccess ||
        balloc(b, &b->abc, size_t(ncases) * NABC) != hipSuccess || balloc(b, &b->foreign, NACC) != hipSuccess ||
        balloc(b, &b->ft, size_t(ncases) * 6) != hipSuccess ||
        balloc(b, &b->hist, size_t(ncases) * size_t(p->history_capacity) * 19) != hipSuccess ||
        balloc(b, &b->traj, 13) != hipSuccess || balloc(b, &b->steps_d, ncases) != hipSuccess ||
        balloc(b, &b->traj_pos, ncases) != hipSuccess || balloc(b, &b->ctr, 1) != hipSuccess)
        return bail(LBM_E_NOMEM, "device buffers");
    if (hipMemcpy(b->cases, b->hcd.data(), ncases * sizeof(CaseDev), hipMemcpyHostToDevice) != hipSuccess)
        return bail(LBM_E_HIP, "case table");
    b->threads = p->threads ? p->threads : 512;
    if (set_bins(b, p->bins ? p->bins : b->cu) != LBM_OK) return bail(LBM_E_HIP, "bins");
    lbm_status s = reset_state(b);
    if (s == LBM_OK) s = check_batch_errors(b);
    if (s != LBM_OK) return bail(s, "initial mapping");
    *out = b;
    g_create_err.clear();
    return LBM_OK;
}

lbm_status lbm_batch_set_kinematics(lbm_batch *b, int32_t c, const double *traj, int64_t nsteps)
{
    if (!b || c < 0 || c >= b->ncase || nsteps < 0 || (nsteps > 0 && !traj))
        return bfail(b, LBM_E_ARG, "bad case or trajectory");
    if (b->steps != 0) return bfail(b, LBM_E_STATE, "kinematics can only be set before the first step");
    b->traj_h[c].assign(traj, traj + nsteps * 13);
    std::vector<double> all;
    for (int i = 0; i < b->ncase; ++i) {
        PConst &pc = b->hcd[i].pc;
        if (b->traj_h[i].empty()) {
            pc.traj_off = -1;
            pc.traj_n = 0;
        } else {
            pc.traj_off = int64_t(all.size() / 13);
            pc.traj_n = int64_t(b->traj_h[i].size() / 13);
            all.insert(all.end(), b->traj_h[i].begin(), b->traj_h[i].end());
        }
    }
    BHIP(b, hipStreamSynchronize(b->st));
    drop_bgraph(b);
    bfree(b->traj);
    BHIP(b, hipMalloc((void **)&b->traj, (all.size() + 13) * sizeof(double)));
    if (!all.empty())
        BHIP(b, hipMemcpy(b->traj, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->cases, b->hcd.data(), b->ncase * sizeof(CaseDev), hipMemcpyHostToDevice));
    BHIP(b, hipMemset(b->traj_pos, 0, b->ncase * sizeof(int64_t)));
    return LBM_OK;
}

lbm_status lbm_batch_set_config(lbm_batch *b, int32_t threads, int32_t bins)
{
    if (!b) return LBM_E_ARG;
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return bfail(b, LBM_E_ARG, "threads must be 256, 512 or 1024");
    if (bins < 0) return bfail(b, LBM_E_ARG, "bins");
    BHIP(b, hipStreamSynchronize(b->st));
    if (threads) {
        b->threads = threads;
        drop_bgraph(b);
    }
    if (bins) return set_bins(b, bins);
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t n)
{
    if (!b) return LBM_E_ARG;
    if (n < 0 || n > (1ll << 30)) return bfail(b, LBM_E_ARG, "step count");
    if (n == 0) return LBM_OK;
    if (!b->gexec || b->graph_n != n) {
        drop_bgraph(b);
        hipError_t e = hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return bfail(b, LBM_E_HIP, std::string("capture: ") + hipGetErrorString(e));
        hipError_t le = launch_batch(b->sk, batch_dev(b), b->threads, b->bins, int(n), 0, b->st);
        e = hipStreamEndCapture(b->st, &b->graph);
        if (le != hipSuccess || e != hipSuccess) {
            drop_bgraph(b);
            return bfail(b, LBM_E_HIP, std::string("capture failed: ") + hipGetErrorString(le != hipSuccess ? le : e));
        }
        e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_bgraph(b);
            return bfail(b, LBM_E_HIP, std::string("instantiate: ") + hipGetErrorString(e));
        }
        b->graph_n = n;
    }
    BHIP(b, hipGraphLaunch(b->gexec, b->st));
    b->steps += n;
    return LBM_OK;
}

lbm_status lbm_batch_sync(lbm_batch *b)
{
    if (!b) return LBM_E_ARG;
    BHIP(b, hipStreamSynchronize(b->st));
    return check_batch_errors(b);
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t trial_steps, const char *cache_path, lbm_batch_tuning *out)
{
    if (!b || trial_steps < 1) return bfail(b, LBM_E_ARG, "trial_steps must be >= 1");
    if (b->steps != 0) return bfail(b, LBM_E_STATE, "autotuning only before the first step");
    const std::string key = tune_key(b);
    lbm_batch_tuning t{};
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int th = 0, bn = 0;
            double ms = 0.0;
            if ((ls >> k >> th >> bn >> ms) && k == key && (th == 256 || th == 512 || th == 1024) && bn > 0) {
                t.threads = th;
                t.bins = bn;
                t.ms_per_step = ms;
                t.from_cache = 1;
            }
        }
    }
    if (!t.from_cache) {
        const double mult[4] = {0.5, 1.0, 2.0, 4.0};
        const int ths[3] = {256, 512, 1024};
        std::vector<std::pair<int, int>> cand;
        for (int th : ths)
            for (double m : mult) {
                const int bn = std::max(1, std::min(b->ncase, int(std::lround(m * b->cu))));
                if (std::find(cand.begin(), cand.end(), std::make_pair(th, bn)) == cand.end())
                    cand.emplace_back(th, bn);
            }
        hipEvent_t e0, e1;
        BHIP(b, hipEventCreate(&e0));
        BHIP(b, hipEventCreate(&e1));
        double best = 1e300;
        for (auto &cb : cand) {
            b->threads = cb.first;
            lbm_status s = set_bins(b, cb.second);
            if (s != LBM_OK) return s;
            BHIP(b, launch_batch(b->sk, batch_dev(b), b->threads, b->bins, 1, 0, b->st));   // warm-up
            BHIP(b, hipEventRecord(e0, b->st));
            BHIP(b, launch_batch(b->sk, batch_dev(b), b->threads, b->bins, trial_steps, 0, b->st));
            BHIP(b, hipEventRecord(e1, b->st));
            BHIP(b, hipEventSynchronize(e1));
            float ms = 0.f;
            BHIP(b, hipEventElapsedTime(&ms, e0, e1));
            const double per = double(ms) / trial_steps;
            ++t.trials;
            if (per < best) {
                best = per;
                t.threads = cb.first;
                t.bins = b->bins;
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        t.ms_per_step = best;
        if (cache_path) {
            std::ofstream o(cache_path, std::ios::app);
            if (o) o << key << " " << t.threads << " " << t.bins << " " << t.ms_per_step << "\n";
        }
    }
    b->threads = t.threads;
    lbm_status s = set_bins(b, t.bins);
    if (s != LBM_OK) return s;
    if (!t.from_cache) {
        s = reset_state(b);
        if (s != LBM_OK) return s;
        s = check_batch_errors(b);
        if (s != LBM_OK) return s;
    }
    if (out) *out = t;
    return LBM_OK;
}

lbm_status lbm_batch_get_force_torque(lbm_batch *b, double *F, double *M)
{
    if (!b) return LBM_E_ARG;
    lbm_status s = check_batch_errors(b);
    if (s != LBM_OK) return s;
    std::vector<double> h(size_t(b->ncase) * 6);
    BHIP(b, hipMemcpy(h.data(), b->ft, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < b->ncase; ++i)
        for (int k = 0; k < 3; ++k) {
            if (F) F[3 * i + k] = h[6 * i + k];
            if (M) M[3 * i + k] = h[6 * i + 3 + k];
        }
    return LBM_OK;
}

lbm_status lbm_batch_get_fiber_state(lbm_batch *b, double *X, double *q, double *V, double *W)
{
    if (!b) return LBM_E_ARG;
    lbm_status s = check_batch_errors(b);
    if (s != LBM_OK) return s;
    std::vector<PState> h(size_t(b->ncase) * 2);
    BHIP(b, hipMemcpy(h.data(), b->ps, h.size() * sizeof(PState), hipMemcpyDeviceToHost));
    const int cur = int(b->steps & 1);
    for (int i = 0; i < b->ncase; ++i) {
        const PState &p = h[size_t(i) * 2 + cur];
        for (int k = 0; k < 3; ++k) {
            if (X) X[3 * i + k] = p.X[k];
            if (V) V[3 * i + k] = p.V[k];
            if (W) W[3 * i + k] = p.W[k];
        }
        if (q)
            for (int k = 0; k < 4; ++k) q[4 * i + k] = p.q[k];
    }
    return LBM_OK;
}

lbm_status lbm_batch_get_history(lbm_batch *b, int32_t c, int64_t first, int64_t count, double *out)
{
    if (!b || !out || count < 0 || c < 0 || c >= b->ncase) return bfail(b, LBM_E_ARG, "bad argument");
    lbm_status s = check_batch_errors(b);
    if (s != LBM_OK) return s;
    const int64_t cap = b->p.history_capacity;
    if (first < 0 || first + count > b->steps || first < b->steps - cap)
        return bfail(b, LBM_E_ARG, "history window not available");
    const double *base = b->hist + size_t(c) * size_t(cap) * 19;
    for (int64_t i = 0; i < count;) {
        const int64_t slot = (first + i) % cap;
        const int64_t run = std::min<int64_t>(count - i, cap - slot);
        BHIP(b, hipMemcpy(out + i * 19, base + slot * 19, size_t(run) * 19 * sizeof(double), hipMemcpyDeviceToHost));
        i += run;
    }
    return LBM_OK;
}

lbm_status lbm_batch_get_fields(lbm_batch *b, int32_t c, void *rho, void *u, uint8_t *flags, int32_t *pid,
                                int32_t dst_is_device)
{
    if (!b || c < 0 || c >= b->ncase) return bfail(b, LBM_E_ARG, "bad case");
    lbm_status s = check_batch_errors(b);
    if (s != LBM_OK) return s;
    const CaseDev &cd = b->hcd[c];
    const size_t n = cd.g.ncell, rsz = b->sk == S_F64 ? 8 : 4;
    void *drho = nullptr, *du = nullptr;
    if (rho) {
        if (dst_is_device) drho = rho;
        else BHIP(b, hipMalloc(&drho, n * rsz));
    }
    if (u) {
        if (dst_is_device) du = u;
        else BHIP(b, hipMalloc(&du, 3 * n * rsz));
    }
    const void *fc = static_cast<const char *>(b->f) + cd.f_off * b->esz;
    const PState *ps = b->ps + size_t(c) * 2 + size_t(b->steps & 1);
    if (rho || u)
        BHIP(b, launch_decode(b->sk, (b->steps & 1) != 0, fc, b->flags + cd.cell_off, b->pid + cd.cell_off, ps,
                              cd.g, cd.pd, drho, du, nullptr, b->st));
    const hipMemcpyKind k = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (rho && !dst_is_device) BHIP(b, hipMemcpyAsync(rho, drho, n * rsz, k, b->st));
    if (u && !dst_is_device) BHIP(b, hipMemcpyAsync(u, du, 3 * n * rsz, k, b->st));
    if (flags) {
        std::vector<uint8_t> hf(n);
        BHIP(b, hipMemcpyAsync(hf.data(), b->flags + cd.cell_off, n, hipMemcpyDeviceToHost, b->st));
        BHIP(b, hipStreamSynchronize(b->st));
        for (auto &v : hf) v &= F_SOLID;
        BHIP(b, hipMemcpyAsync(flags, hf.data(), n, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost, b->st));
        BHIP(b, hipStreamSynchronize(b->st));
    }
    if (pid) BHIP(b, hipMemcpyAsync(pid, b->pid + cd.cell_off, n * 4, k, b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    if (rho && !dst_is_device) hipFree(drho);
    if (u && !dst_is_device) hipFree(du);
    return LBM_OK;
}

lbm_status lbm_batch_get_populations(lbm_batch *b, int32_t c, double *f)
{
    if (!b || !f || c < 0 || c >= b->ncase) return bfail(b, LBM_E_ARG, "bad argument");
    lbm_status s = check_batch_errors(b);
    if (s != LBM_OK) return s;
    const CaseDev &cd = b->hcd[c];
    double *d = nullptr;
    const size_t n = size_t(Q) * cd.g.ncell;
    BHIP(b, hipMalloc(&d, n * sizeof(double)));
    const void *fc = static_cast<const char *>(b->f) + cd.f_off * b->esz;
    const PState *ps = b->ps + size_t(c) * 2 + size_t(b->steps & 1);
    hipError_t e = launch_decode(b->sk, (b->steps & 1) != 0, fc, b->flags + cd.cell_off, b->pid + cd.cell_off,
                                 ps, cd.g, cd.pd, nullptr, nullptr, d, b->st);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, b->st);
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    hipFree(d);
    if (e != hipSuccess) return bfail(b, LBM_E_HIP, hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_batch_sample_features(lbm_batch *b, float *out, int32_t dst_is_device)
{
    if (!b || !out) return LBM_E_ARG;
    lbm_status s = check_batch_errors(b);
    if (s != LBM_OK) return s;
    for (int i = 0; i < b->ncase; ++i)
        if (b->hc[i].wall_u == 0.0) return bfail(b, LBM_E_ARG, "features need U != 0 in every case");
    const size_t n = size_t(b->ncase) * LBM_MLP_IN;
    float *d = out;
    if (!dst_is_device) BHIP(b, hipMalloc(&d, n * sizeof(float)));
    hipError_t e = hipSuccess;
    for (int i = 0; i < b->ncase && e == hipSuccess; ++i) {
        const CaseDev &cd = b->hcd[i];
        const void *fc = static_cast<const char *>(b->f) + cd.f_off * b->esz;
        const PState *ps = b->ps + size_t(i) * 2 + size_t(b->steps & 1);
        const PConst *pc = &b->cases[i].pc;
        const double gamma = 2.0 * b->hc[i].wall_u / b->hc[i].nz;
        e = launch_sample_features(b->sk, (b->steps & 1) != 0, fc, b->flags + cd.cell_off, b->pid + cd.cell_off,
                                   ps, pc, 1, cd.g, cd.pd, gamma, d + size_t(i) * LBM_MLP_IN, b->st);
    }
    if (e == hipSuccess && !dst_is_device) e = hipMemcpyAsync(out, d, n * sizeof(float), hipMemcpyDeviceToHost, b->st);
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (!dst_is_device) hipFree(d);
    if (e != hipSuccess) return bfail(b, LBM_E_HIP, hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_batch_get_info(lbm_batch *b, lbm_batch_info *info)
{
    if (!b || !info) return LBM_E_ARG;
    BHIP(b, hipStreamSynchronize(b->st));
    std::vector<uint32_t> ln(b->ncase);
    BHIP(b, hipMemcpy(ln.data(), b->list_n, ln.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t nb = 0, cells = 0;
    for (int i = 0; i < b->ncase; ++i) {
        nb += std::min<uint32_t>(ln[i], b->hcd[i].list_cap);
        cells += b->hcd[i].g.ncell;
    }
    info->steps_done = b->steps;
    info->ncases = b->ncase;
    info->bins = b->bins;
    info->threads = b->threads;
    info->cells = cells;
    info->boundary_cells = nb;
    info->device_bytes = b->device_bytes;
    info->population_bytes = int64_t(b->nf * b->esz);
    return LBM_OK;
}

}  // extern "C"
