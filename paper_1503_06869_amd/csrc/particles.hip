// particles.hip -- per-fiber work of one time step on the device:
//   k_rigid      the momentum-exchange sums of each fiber (Eq.
//                LBMhydrodynForce and the torque after it, Sec. 4.2),
//                accumulated by the boundary sweep, back to FP64; the
//                rigid-body update (Sec. 4.3); the cell boxes of the remap;
//   k_remap      cell mapping with the new poses (Sec. 4.2: a cell is an
//                obstacle cell when its centre lies inside a particle) and
//                refill of uncovered cells with f_eq(rho0, u_s) of the
//                previous step's motion;
//   k_near       flags of fluid cells next to fibers, written into the flag
//                buffer of the next step, and the boundary-cell list consumed
//                by the next step's boundary launch.
#include "lbm_sweep_dev.h"
#include "lbm_particle_dev.h"

namespace lbm {

#pragma clang fp contract(off)

// Plane rectangle of fiber o's remap region: the current and new poses
// (where cell owners can change; margin for owned cells), and with PREV, for
// the flag rebuild, also the previous pose (the flags of the next step are
// written into the buffer that held those of the previous step, so the
// rebuild covers every cell flagged then; margin for bordering cells).
template <bool PREV>
__device__ __forceinline__ Rect remap_rect(const PartData &pd, int o, int32_t z, const Geo &g)
{
    const Box b = pd.box_remap[o];
    const PConst c = pd.pc[o];
    const double m = PREV ? NEAR_MARGIN : REMAP_MARGIN;
    const Rect r = rect_union(plane_rect(pd.ps_cur[o], c, z, b, g, m), plane_rect(pd.ps_next[o], c, z, b, g, m), g);
    return PREV ? rect_union(r, plane_rect(pd.ps_prev[o], c, z, b, g, m), g) : r;
}

// ------------------------------------------------------------------ boxes of the remap
// Union of the boxes of the previous (box_prev), current (box_cur) and new
// pose s of fiber p, the new box, and the reset of the fiber's boundary-list
// segment.
__device__ __forceinline__ void fiber_remap_boxes(const PartData &pd, int p, const PState &s, const Geo &g)
{
    Box ub, nb;
    const Box bc = pd.box_cur[p];
    remap_boxes(s, pd.pc[p], bc, pd.box_prev[p], g, ub, nb);
    pd.box_remap[p] = ub;
    pd.box_prev[p] = bc;
    pd.box_cur[p] = nb;
    pd.seg_cnt[p] = 0u;
}

// end of a time step: advance the device step counter
__device__ void finish_step(const PartData &pd)
{
    if (threadIdx.x == 0) pd.ctr->step += 1ull;
}

// Set-up of the mapping from ps_cur (old poses, or the current ones) to
// ps_next: the previous pose is taken equal to the old one.
__global__ __launch_bounds__(256) void k_setup_boxes(PartData pd, Geo g)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < pd.np; p += gridDim.x * blockDim.x) {
        pd.ps_prev[p] = pd.ps_cur[p];
        pd.box_prev[p] = pd.box_cur[p];
        fiber_remap_boxes(pd, p, pd.ps_next[p], g);
    }
}

// ------------------------------------------------------------------ rigid update kernel
// One block: the momentum-exchange sums of every fiber (accumulated in fixed
// point by the boundary sweep) back to FP64, the contact loads (when on), the
// rigid-body update, outputs, the boxes of the remap and the list reset.
__global__ __launch_bounds__(256) void k_rigid(PartData pd, Geo g)
{
    extern __shared__ double tot[];   // [np][NACC]
    const int np = pd.np;
    for (int t = threadIdx.x; t < np * NACC; t += blockDim.x) {
        const int k = t % NACC;
        tot[t] = ldexp(double(pd.mea[t]), -fx_shift(k));
        pd.mea[t] = 0;   // cleared for the next step's boundary sweep
    }
    // contact loads at the current poses, each pair in the orientation (lower
    // id, higher id) and summed over partners in ascending order
    double *cl = tot + size_t(np) * NACC;   // [np][6] when contacts are on
    if (pd.contact_k > 0.0)
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            const PState sp = pd.ps_cur[p];
            const PConst cp = pd.pc[p];
            for (int q = 0; q < np; ++q) {
                if (q == p) continue;
                double l[6];
                if (p < q) contact_load(sp, cp, pd.ps_cur[q], pd.pc[q], true, pd.contact_k, pd.contact_range, g, l);
                else contact_load(pd.ps_cur[q], pd.pc[q], sp, cp, false, pd.contact_k, pd.contact_range, g, l);
                for (int k = 0; k < 6; ++k) acc[k] += l[k];
            }
            for (int k = 0; k < 6; ++k) cl[p * 6 + k] = acc[k];
        }
    __syncthreads();
    const int64_t step = int64_t(pd.ctr->step);
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        double ac[NACC];
        for (int k = 0; k < NACC; ++k) ac[k] = tot[p * NACC + k];
        const PConst c = pd.pc[p];
        const PState s = pd.ps_cur[p];
        abc_restore(ac, s.X, pd.rho0_link);
        const double *row = nullptr;
        if (c.traj_off >= 0 && pd.traj_pos[p] < c.traj_n) {
            row = pd.traj + (c.traj_off + pd.traj_pos[p]) * 13;
            pd.traj_pos[p] += 1;
        }
        PState o;
        double F[3], M[3];
        rigid_update(s, c, ac, pd.coupling, row, g, o, F, M, pd.corr ? pd.corr + size_t(p) * 6 : nullptr,
                     pd.contact_k > 0.0 ? cl + size_t(p) * 6 : nullptr);
        bool bad = false;
        for (int k = 0; k < 3; ++k) bad |= !isfinite(F[k]) || !isfinite(M[k]);
        if (bad) atomicOr(&pd.ctr->err_unstable, 1u);
        pd.ps_prev[p] = pd.ps_next[p];   // the pose of the previous step, about to be overwritten
        pd.ps_next[p] = o;
        if (g.xw || g.yw || g.zs) {
            // fibers keep more than one cell from x and y walls (the mapping
            // and momentum exchange take x and y as periodic) and from
            // free-slip z walls (a reflected population lands on a cell of
            // the wall layer, which must be fluid)
            for (int k = 0; k < 3; ++k) {
                if (!(k == 0 ? g.xw : (k == 1 ? g.yw : g.zs))) continue;
                const double ext = c.shape == 1 ? (0.5 * c.length - c.radius) * fabs(o.t[k]) + c.radius
                                                : 0.5 * c.length * fabs(o.t[k]) +
                                                      c.radius * sqrt(fmax(0.0, 1.0 - o.t[k] * o.t[k]));
                const double nk = k == 0 ? double(g.nx) : (k == 1 ? double(g.ny) : double(g.nz));
                if (o.X[k] - ext < 1.0 || o.X[k] + ext > nk - 2.0) atomicOr(&pd.ctr->err_wall, 1u);
            }
        }
        fiber_remap_boxes(pd, p, o, g);
        for (int k = 0; k < 3; ++k) {
            pd.ft_out[p * 6 + k] = F[k];
            pd.ft_out[p * 6 + 3 + k] = M[k];
        }
        double *h = pd.hist + ((step % pd.hist_cap) * np + p) * 19;
        for (int k = 0; k < 3; ++k) { h[k] = F[k]; h[3 + k] = M[k]; h[6 + k] = o.X[k]; }
        for (int k = 0; k < 4; ++k) h[9 + k] = o.q[k];
        for (int k = 0; k < 3; ++k) { h[13 + k] = o.V[k]; h[16 + k] = o.W[k]; }
    }
    __syncthreads();   // every thread has read the step counter
    finish_step(pd);
}

// ------------------------------------------------------------------ remap and boundary list
// Grid: np * nslab blocks; block (p, s) takes the z-planes s, s + nslab, ...
// of fiber p's remap box.  A cell inside the plane rectangle of a
// lower-indexed fiber is left to that fiber's blocks, so every cell is
// handled once.  The ids and boxes of the neighbouring fibers are staged in
// LDS.
struct NbrStage {
    int32_t id[NBR_CAP];
    Box box[NBR_CAP];
    int32_t n, nlow;
};

// Rectangles of a chunk of the block's planes, for one flattened pass over
// all their cells: rect[k * ne + 0] is the own fiber's rectangle in plane k
// of the chunk, rect[k * ne + j] that of the j-th lower-indexed neighbour
// (empty where the plane is outside the neighbour's box); pref holds the
// prefix of the own rectangles' cell counts.
constexpr int RT_MAXE = 512, RT_MAXP = 32;
struct RegionTable {
    Rect rect[RT_MAXE];
    int32_t z[RT_MAXP];
    int32_t pref[RT_MAXP + 1];
    int32_t npl, ne;
};

__device__ __forceinline__ void stage_nbrs(const PartData &pd, int p, NbrStage &sh, const Geo &g)
{
    __shared__ uint32_t s_wc[4], s_low;
    const Box a = pd.box_remap[p];
    if (threadIdx.x == 0) {
        sh.n = 0;
        s_low = 0u;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int o0 = 0; o0 < pd.np; o0 += blockDim.x) {   // block-uniform
        const int o = o0 + int(threadIdx.x);
        Box bo{};
        bool hit = false;
        if (o < pd.np && o != p) {
            bo = pd.box_remap[o];
            hit = boxes_meet(a, bo, g);
        }
        const unsigned long long bal = __ballot(hit);
        if (lane == 0) s_wc[wid] = uint32_t(__popcll(bal));
        __syncthreads();
        uint32_t k = uint32_t(sh.n) + uint32_t(__popcll(bal & ((1ull << lane) - 1ull)));
        for (int w = 0; w < wid; ++w) k += s_wc[w];
        const uint32_t pass = s_wc[0] + s_wc[1] + s_wc[2] + s_wc[3];   // read before the next pass writes
        if (hit) {
            if (k < uint32_t(NBR_CAP)) {
                sh.id[k] = o;
                sh.box[k] = bo;
            }
            if (o < p) atomicAdd(&s_low, 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) sh.n += int32_t(pass);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sh.n > NBR_CAP) {
            atomicOr(&pd.ctr->err_capacity, 1u);
            sh.n = NBR_CAP;
        }
        sh.nlow = min(int32_t(s_low), sh.n);
    }
    __syncthreads();
}

// Table of the planes iz0, iz0 + ns, ... of box b (as many as fit); returns
// the number of planes taken (block-uniform call).
template <bool PREV>
__device__ int build_table(const PartData &pd, const NbrStage &sh, int p, const Box &b, int iz0, int ns,
                           const Geo &g, RegionTable &t)
{
    const int ne = sh.nlow + 1;
    const int left = iz0 < b.len[2] ? (b.len[2] - iz0 + ns - 1) / ns : 0;
    const int npl = min(left, min(RT_MAXP, RT_MAXE / ne));
    __syncthreads();   // the previous chunk's pass is done with the table
    for (int e = threadIdx.x; e < npl * ne; e += blockDim.x) {
        const int k = e / ne, j = e - k * ne;
        int32_t z = b.lo[2] + iz0 + k * ns;
        bool valid = true;
        if (g.zper) z = wrapc(z, int32_t(g.nz));
        else valid = z >= 0 && z < int32_t(g.nz);
        Rect r{1, 0, 1, 0};
        if (valid) {
            if (j == 0) r = remap_rect<PREV>(pd, p, z, g);
            else if (in_zrange(sh.box[j - 1], z, g)) r = remap_rect<PREV>(pd, sh.id[j - 1], z, g);
        }
        t.rect[e] = r;
        if (j == 0) t.z[k] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int k = 0; k < npl; ++k) {
            t.pref[k] = acc;
            const Rect r = t.rect[k * ne];
            if (r.x0 <= r.x1 && r.y0 <= r.y1) acc += (r.x1 - r.x0 + 1) * (r.y1 - r.y0 + 1);
        }
        t.pref[npl] = acc;
        t.npl = npl;
        t.ne = ne;
    }
    __syncthreads();
    return npl;
}

// cell idx of the chunk's flattened index space: plane k, position (x, y)
__device__ __forceinline__ void table_cell(const RegionTable &t, int idx, const Geo &g, int &k, int32_t &x,
                                           int32_t &y)
{
    k = 0;
    while (k + 1 < t.npl && t.pref[k + 1] <= idx) ++k;
    const Rect r = t.rect[k * t.ne];
    const int wx = r.x1 - r.x0 + 1, i = idx - t.pref[k];
    const int iy = i / wx, ix = i - iy * wx;
    x = wrapi(r.x0 + ix, int32_t(g.nx));
    y = wrapi(r.y0 + iy, int32_t(g.ny));
}

// a cell is handled by the lowest-indexed fiber whose region holds it
__device__ __forceinline__ bool owned_here(const RegionTable &t, int k, int32_t x, int32_t y, const Geo &g)
{
    for (int j = 1; j < t.ne; ++j)
        if (in_rect(t.rect[k * t.ne + j], x, y, g)) return false;
    return true;
}

// new owner of each cell of the remap boxes; refill of uncovered cells
template <typename S>
__global__ __launch_bounds__(256) void k_remap(S *__restrict__ f, int32_t *__restrict__ pid, PartData pd,
                                               Geo g, int next_odd, double rho0, double scale)
{
    const int ns = pd.nslab;
    const int p = blockIdx.x / ns, sl = blockIdx.x % ns;
    __shared__ NbrStage sh;
    stage_nbrs(pd, p, sh, g);
    const Box b = pd.box_remap[p];
    const PState sp = pd.ps_next[p];
    const PConst cp = pd.pc[p];
    __shared__ RegionTable t;
    for (int iz0 = sl; iz0 < b.len[2];) {   // block-uniform: chunks of planes
        iz0 += ns * build_table<false>(pd, sh, p, b, iz0, ns, g, t);
        for (int idx = threadIdx.x; idx < t.pref[t.npl]; idx += blockDim.x) {
            int k;
            int32_t x, y;
            table_cell(t, idx, g, k, x, y);
            if (!owned_here(t, k, x, y, g)) continue;
            const int32_t z = t.z[k];
            const double cx = x, cy = y, cz = z;
            int owner = -1, claims = 0;
            if (inside(sp, cp, cx, cy, cz, g)) {
                owner = p;
                claims = 1;
            }
            for (int j = sh.nlow; j < sh.n; ++j) {
                const int o = sh.id[j];
                if (!in_box(sh.box[j], x, y, z, g)) continue;
                if (inside(pd.ps_next[o], pd.pc[o], cx, cy, cz, g)) {
                    if (owner < 0) owner = o;
                    ++claims;
                }
            }
            if (claims > 1) atomicAdd(&pd.ctr->overlaps, (unsigned long long)(claims - 1));
            const uint32_t cell = (uint32_t(z) * g.ny + uint32_t(y)) * g.nx + uint32_t(x);
            const int old = pid[cell];
            if (old >= 0 && owner < 0)   // uncovered
                refill_cell<S>(f, g, x, y, z, pd.ps_cur[old], rho0, scale, next_odd);
            if (pd.cov && (old < 0) != (owner < 0)) {
                // fluid cell count and momentum change for the stabilization
                const uint32_t k = atomicAdd(pd.cov, 1u);
                if (k < pd.cov_cap) pd.cov[1 + k] = cell | (owner < 0 ? COV_UNCOVERED : 0u);
                else atomicOr(&pd.ctr->err_capacity, 4u);
            }
            pid[cell] = owner;
        }
    }
}

// Flags of the cells in the remap regions and the boundary-cell list.  The
// list is cut into one segment per fiber; a block stages the boundary cells
// it finds in all its planes in LDS and reserves a range of its fiber's
// segment with a single atomic (cells beyond the stage are appended one by
// one).
constexpr int LSTAGE = 1024;

__global__ __launch_bounds__(256) void k_near(uint8_t *__restrict__ flags, const int32_t *__restrict__ pid,
                                              uint32_t *__restrict__ list_cell,
                                              uint32_t *__restrict__ list_mask, PartData pd, Geo g)
{
    const int ns = pd.nslab;
    const int p = blockIdx.x / ns, sl = blockIdx.x % ns;
    __shared__ NbrStage sh;
    __shared__ uint32_t s_cell[LSTAGE], s_mask[LSTAGE];
    __shared__ uint32_t s_n, s_base;
    stage_nbrs(pd, p, sh, g);
    if (threadIdx.x == 0) s_n = 0u;
    __syncthreads();
    const Box b = pd.box_remap[p];
    const uint32_t off = pd.seg_off[p], cap = pd.seg_cap[p];
    __shared__ RegionTable t;
    for (int iz0 = sl; iz0 < b.len[2];) {   // block-uniform: chunks of planes
        iz0 += ns * build_table<true>(pd, sh, p, b, iz0, ns, g, t);
        for (int idx = threadIdx.x; idx < t.pref[t.npl]; idx += blockDim.x) {
            int k;
            int32_t x, y;
            table_cell(t, idx, g, k, x, y);
            if (!owned_here(t, k, x, y, g)) continue;
            const int32_t z = t.z[k];
            const uint32_t cell = (uint32_t(z) * g.ny + uint32_t(y)) * g.nx + uint32_t(x);
            // the cell's owner and its neighbours' in one round of loads
            const int32_t own = pid[cell];
            const uint32_t mask = fiber_mask(pid, g, x, y, z);
            const bool near = (own < 0) & (mask != 0u);
            if (!near) {
                flags[cell] = own >= 0 ? F_SOLID : uint8_t(0);
                continue;
            }
            const uint32_t kk = atomicAdd(&s_n, 1u);
            if (kk < LSTAGE) {
                s_cell[kk] = cell;
                s_mask[kk] = mask;
            } else {
                // stage full: append directly
                const uint32_t r = atomicAdd(&pd.seg_cnt[p], 1u);
                if (r < cap) {
                    const uint32_t e = off + r;
                    list_cell[e] = cell;
                    list_mask[e] = mask;
                    flags[cell] = F_NEAR;
                } else {
                    flags[cell] = 0;
                    atomicOr(&pd.ctr->err_capacity, 2u);
                }
            }
        }
    }
    // one reservation for all planes of the block
    __syncthreads();
    const uint32_t n = min(s_n, uint32_t(LSTAGE));
    if (threadIdx.x == 0 && n) s_base = atomicAdd(&pd.seg_cnt[p], n);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
        const uint32_t r = s_base + k, cell = s_cell[k];
        if (r < cap) {
            const uint32_t e = off + r;
            list_cell[e] = cell;
            list_mask[e] = s_mask[k];
            flags[cell] = F_NEAR;
        } else {
            flags[cell] = 0;
            atomicOr(&pd.ctr->err_capacity, 2u);
        }
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_rigid(const PartData &pd, const Geo &g, hipStream_t st)
{
    const size_t per = NACC + (pd.contact_k > 0.0 ? 6 : 0);
    hipLaunchKernelGGL(k_rigid, dim3(1), dim3(256), size_t(pd.np) * per * sizeof(double), st, pd, g);
    return hipGetLastError();
}

hipError_t launch_setup_boxes(const PartData &pd, const Geo &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_setup_boxes, dim3((pd.np + 255) / 256), dim3(256), 0, st, pd, g);
    return hipGetLastError();
}

hipError_t launch_remap(int sk, bool next_odd, void *f, int32_t *pid, const PartData &pd, const Geo &g,
                        double rho0, double scale, hipStream_t st)
{
    const int no = next_odd ? 1 : 0;
    const dim3 gr(pd.np * pd.nslab), bl(256);
    switch (sk) {
    case S_F32: hipLaunchKernelGGL(k_remap<float>, gr, bl, 0, st, (float *)f, pid, pd, g, no, rho0, scale); break;
    case S_F16: hipLaunchKernelGGL(k_remap<_Float16>, gr, bl, 0, st, (_Float16 *)f, pid, pd, g, no, rho0, scale); break;
    case S_BF16: hipLaunchKernelGGL(k_remap<uint16_t>, gr, bl, 0, st, (uint16_t *)f, pid, pd, g, no, rho0, scale); break;
    default: hipLaunchKernelGGL(k_remap<double>, gr, bl, 0, st, (double *)f, pid, pd, g, no, rho0, scale); break;
    }
    return hipGetLastError();
}

hipError_t launch_near(uint8_t *flags, const int32_t *pid, uint32_t *list_cell, uint32_t *list_mask,
                       const PartData &pd, const Geo &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_near, dim3(pd.np * pd.nslab), dim3(256), 0, st, flags, pid, list_cell, list_mask,
                       pd, g);
    return hipGetLastError();
}

}  // namespace lbm
