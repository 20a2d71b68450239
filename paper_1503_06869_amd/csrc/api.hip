// api.hip -- host side of the library: context, device buffers, the step
// scheduler (direct launches or a captured two-step HIP graph) and the C ABI
// declared in include/lbm.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "../../include/lbm_mlp.h"
#include "lbm_dev.h"

using namespace lbm;

struct lbm_ctx {
    lbm_params p{};
    std::string err;
    int dev = 0;              // device current at creation (the stream's device)
    hipStream_t st = nullptr;
    int sk = 0;
    size_t esz = 4;
    Geo g{};
    Phys<double> ph{};
    double scale = 1.0;
    // lattice
    void *f = nullptr;
    // cell flags of the even and odd steps: step n reads flags[n & 1] and
    // writes those of step n + 1 into the other buffer
    uint8_t *flags[2] = {nullptr, nullptr};
    int32_t *pid = nullptr;
    // particles
    int np = 0;
    std::vector<lbm_fiber> fib;
    std::vector<PConst> pch;
    std::vector<std::vector<double>> traj_h;
    PState *ps[2] = {nullptr, nullptr};
    PConst *pc = nullptr;
    Box *box_cur = nullptr, *box_prev = nullptr, *box_remap = nullptr;
    PState *ps_prev = nullptr;
    long long *mea = nullptr;
    uint32_t *seg_off = nullptr, *seg_cap = nullptr, *seg_cnt = nullptr;
    int nslab = 4, bpf = 1;
    double *traj = nullptr;
    int64_t *traj_pos = nullptr;
    double *ft = nullptr, *hist = nullptr;
    uint32_t *list_cell = nullptr, *list_mask = nullptr;
    uint32_t list_cap = 0;
    DevCounters *ctr = nullptr;
    uint32_t remap_grid = 0, bnd_grid = 0, sweep_grid = 0;
    int64_t steps = 0;
    int64_t device_bytes = 0;
    // graph of one even + one odd step
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    // sweep timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    bool own_stream = false;
    // second stream: boundary sweep and the particle chain run beside the bulk sweep
    hipStream_t st2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    size_t ev_used = 0;
    int64_t timed_sweeps = 0;
    double timed_ms = 0.0;
    // momentum stabilization: mean velocity, workgroup sums, changed cells
    double *stab = nullptr;
    uint32_t *cov = nullptr;
    uint32_t cov_cap = 0;
    bool stab_stale = true;   // state changed from the host: the mean needs a full pass
    // learned closure (not owned)
    lbm_mlp *closure = nullptr;
    double *corr = nullptr;
    unsigned long long *cstats = nullptr;
};

static lbm_status fail(lbm_ctx *c, lbm_status s, const std::string &m)
{
    if (c) c->err = m;
    return s;
}

#define HIPCHK(c, call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((c), e_ == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_HIP,             \
                        std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

template <typename T>
static hipError_t dalloc(lbm_ctx *c, T **ptr, size_t n)
{
    *ptr = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)ptr, n * sizeof(T));
    if (e == hipSuccess) c->device_bytes += int64_t(n * sizeof(T));
    return e;
}
template <typename T>
static void dfree(T *&p)
{
    if (p) hipFree((void *)p);
    p = nullptr;
}

static void free_particles(lbm_ctx *c)
{
    dfree(c->ps[0]);
    dfree(c->ps[1]);
    dfree(c->pc);
    dfree(c->box_cur);
    dfree(c->box_prev);
    dfree(c->box_remap);
    dfree(c->ps_prev);
    dfree(c->mea);
    dfree(c->seg_off);
    dfree(c->seg_cap);
    dfree(c->seg_cnt);
    dfree(c->traj);
    dfree(c->traj_pos);
    dfree(c->ft);
    dfree(c->hist);
    dfree(c->list_cell);
    dfree(c->list_mask);
}

// buffers of the momentum stabilization, sized for the current sweep and
// boundary grids and boundary list
static lbm_status alloc_stab(lbm_ctx *c)
{
    if (!c->p.stabilize) return LBM_OK;
    dfree(c->stab);
    dfree(c->cov);
    const uint32_t nslot = std::max(STAB_SCAN_GRID, c->sweep_grid + c->bnd_grid);
    HIPCHK(c, dalloc(c, &c->stab, size_t(STAB_HEAD) + 4 * size_t(nslot)));
    HIPCHK(c, hipMemsetAsync(c->stab, 0, (size_t(STAB_HEAD) + 4 * size_t(nslot)) * sizeof(double), c->st));
    // cells changing owner in one remap: fewer than the boundary list holds
    c->cov_cap = std::max(4096u, c->list_cap);
    HIPCHK(c, dalloc(c, &c->cov, size_t(c->cov_cap) + 1));
    HIPCHK(c, hipMemsetAsync(c->cov, 0, (size_t(c->cov_cap) + 1) * sizeof(uint32_t), c->st));
    c->stab_stale = true;
    return LBM_OK;
}

// the mean velocity of the current state by a full pass, when the host has
// changed the state since the last step
static hipError_t refresh_stab(lbm_ctx *c)
{
    if (!c->p.stabilize || !c->stab_stale) return hipSuccess;
    c->stab_stale = false;
    return launch_stab_scan(c->sk, (c->steps & 1) != 0, c->f, c->pid, c->g, c->ph, c->stab, c->cov, c->st);
}

static void drop_graph(lbm_ctx *c)
{
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

// axis t = R(q) e_x, same expression order as the device
static void host_axis(const double q[4], double t[3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    t[0] = 1.0 - 2.0 * (y * y + z * z);
    t[1] = 2.0 * (x * y + w * z);
    t[2] = 2.0 * (x * z - w * y);
}

static PState make_state(const lbm_fiber &f, const PConst &c)
{
    PState s{};
    const double qn = std::sqrt(f.quat[0] * f.quat[0] + f.quat[1] * f.quat[1] + f.quat[2] * f.quat[2] +
                                f.quat[3] * f.quat[3]);
    for (int k = 0; k < 3; ++k) s.X[k] = f.center[k];
    for (int k = 0; k < 4; ++k) s.q[k] = f.quat[k] / qn;
    for (int k = 0; k < 3; ++k) s.V[k] = f.vel[k];
    for (int k = 0; k < 3; ++k) s.W[k] = f.omega[k];
    host_axis(s.q, s.t);
    const double tw = s.t[0] * s.W[0] + s.t[1] * s.W[1] + s.t[2] * s.W[2];
    for (int k = 0; k < 3; ++k) s.L[k] = c.i_perp * s.W[k] + (c.i_par - c.i_perp) * tw * s.t[k];
    return s;
}

static double link_rho0(const lbm_ctx *c)
{
    return c->sk == S_F64 ? c->p.rho0 : double(float(c->p.rho0));
}

static PartData part_data(lbm_ctx *c, PState *cur, PState *next)
{
    PartData pd{};
    pd.np = c->np;
    pd.pc = c->pc;
    pd.ps_cur = cur;
    pd.ps_next = next;
    pd.ps_prev = c->ps_prev;
    pd.box_cur = c->box_cur;
    pd.box_prev = c->box_prev;
    pd.box_remap = c->box_remap;
    pd.mea = c->mea;
    pd.seg_off = c->seg_off;
    pd.seg_cap = c->seg_cap;
    pd.seg_cnt = c->seg_cnt;
    pd.nslab = c->nslab;
    pd.traj = c->traj;
    pd.traj_pos = c->traj_pos;
    pd.ft_out = c->ft;
    pd.hist = c->hist;
    pd.hist_cap = c->p.history_capacity;
    pd.coupling = c->p.coupling;
    pd.rho0 = c->p.rho0;
    pd.rho0_link = link_rho0(c);
    pd.corr = c->closure ? c->corr : nullptr;
    pd.ctr = c->ctr;
    pd.list_cap = c->list_cap;
    pd.contact_k = c->p.contact_stiffness;
    pd.contact_range = c->p.contact_range;
    return pd;
}

// rho0 as the sweep's collision type holds it (float except for FP64 storage)

static uint32_t grid_cap(uint64_t work, uint32_t lo, uint32_t hi)
{
    uint64_t b = (work + 255) / 256;
    if (b < lo) b = lo;
    if (b > hi) b = hi;
    return uint32_t(b);
}

// (re)allocate the per-fiber buffers for c->np fibers and upload states
static lbm_status upload_particles(lbm_ctx *c)
{
    drop_graph(c);
    free_particles(c);
    const int np = c->np;
    if (np == 0) return LBM_OK;
    HIPCHK(c, dalloc(c, &c->ps[0], np));
    HIPCHK(c, dalloc(c, &c->ps[1], np));
    HIPCHK(c, dalloc(c, &c->pc, np));
    HIPCHK(c, dalloc(c, &c->ps_prev, np));
    HIPCHK(c, dalloc(c, &c->box_cur, np));
    HIPCHK(c, dalloc(c, &c->box_prev, np));
    HIPCHK(c, dalloc(c, &c->box_remap, np));
    // blocks per fiber of the remap and list kernels: about 1024 blocks in
    // all (measured on 64 and 200 fibers), at least 8 per fiber
    c->nslab = std::max(8, std::min(32, 1024 / np));
    HIPCHK(c, dalloc(c, &c->mea, size_t(np) * NACC));
    HIPCHK(c, hipMemsetAsync(c->mea, 0, size_t(np) * NACC * sizeof(long long), c->st));
    HIPCHK(c, dalloc(c, &c->seg_off, np));
    HIPCHK(c, dalloc(c, &c->seg_cap, np));
    HIPCHK(c, dalloc(c, &c->seg_cnt, np));
    HIPCHK(c, hipMemsetAsync(c->seg_cnt, 0, np * sizeof(uint32_t), c->st));
    HIPCHK(c, dalloc(c, &c->traj_pos, np));
    HIPCHK(c, dalloc(c, &c->ft, size_t(np) * 6));
    HIPCHK(c, dalloc(c, &c->hist, size_t(c->p.history_capacity) * np * 19));
    // boundary-list segments, one per fiber: fluid cells next to a fiber lie
    // within sqrt(2) of its cylinder; bound them by the cylinder widened by 2.5
    std::vector<uint32_t> soff(np), scap(np);
    double total = 0.0, maxsurf = 0.0;
    for (int i = 0; i < np; ++i) {
        const double r = c->fib[i].radius + 2.5, L = c->fib[i].length + 5.0;
        const double cap = 1.25 * (M_PI * r * r * L + 4.0 * M_PI * r * r) + 256.0;
        soff[i] = uint32_t(total);
        scap[i] = uint32_t(cap);
        total += double(scap[i]);
        // expected boundary cells: about one shell of the cylinder widened by 1
        const double rs = c->fib[i].radius + 1.0, ls = c->fib[i].length + 2.0;
        maxsurf = std::max(maxsurf, 2.0 * M_PI * rs * ls);
    }
    if (total >= 4294967295.0) return fail(c, LBM_E_ARG, "boundary list too large");
    c->list_cap = uint32_t(total);
    HIPCHK(c, dalloc(c, &c->list_cell, c->list_cap));
    HIPCHK(c, dalloc(c, &c->list_mask, c->list_cap));
    HIPCHK(c, hipMemcpyAsync(c->seg_off, soff.data(), np * sizeof(uint32_t), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->seg_cap, scap.data(), np * sizeof(uint32_t), hipMemcpyHostToDevice, c->st));
    // boundary launch: blocks per fiber segment, about one entry per thread
    // for the largest fiber (each pass over a segment is a chain of
    // dependent loads, so extra passes add latency, not throughput)
    c->bpf = std::max(1, std::min(16, int(std::ceil(maxsurf / 256.0))));
    c->remap_grid = uint32_t(np * c->nslab);
    c->bnd_grid = uint32_t(np * c->bpf);
    std::vector<PState> hs(np);
    int64_t off = 0;
    std::vector<double> alltraj;
    for (int i = 0; i < np; ++i) {
        PConst &pc = c->pch[i];
        if (!c->traj_h[i].empty()) {
            pc.traj_off = off;
            pc.traj_n = int64_t(c->traj_h[i].size() / 13);
            alltraj.insert(alltraj.end(), c->traj_h[i].begin(), c->traj_h[i].end());
            off += pc.traj_n;
        } else {
            pc.traj_off = -1;
            pc.traj_n = 0;
        }
        hs[i] = make_state(c->fib[i], pc);
    }
    HIPCHK(c, dalloc(c, &c->traj, alltraj.size() + 13));
    if (!alltraj.empty())
        HIPCHK(c, hipMemcpyAsync(c->traj, alltraj.data(), alltraj.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->pc, c->pch.data(), np * sizeof(PConst), hipMemcpyHostToDevice, c->st));
    const int cur = int(c->steps & 1);
    HIPCHK(c, hipMemcpyAsync(c->ps[cur], hs.data(), np * sizeof(PState), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemsetAsync(c->traj_pos, 0, np * sizeof(int64_t), c->st));
    HIPCHK(c, hipMemsetAsync(c->box_cur, 0, np * sizeof(Box), c->st));
    HIPCHK(c, hipMemsetAsync(c->ft, 0, np * 6 * sizeof(double), c->st));
    return alloc_stab(c);
}

// map all fibers from their current states (cells of the old boxes included)
static lbm_status setup_mapping(lbm_ctx *c, PState *old_states)
{
    c->stab_stale = true;
    if (c->np == 0) return LBM_OK;
    PState *cur = c->ps[c->steps & 1];
    PartData pd = part_data(c, old_states ? old_states : cur, cur);
    HIPCHK(c, launch_setup_boxes(pd, c->g, c->st));
    HIPCHK(c, launch_remap(c->sk, (c->steps & 1) != 0, c->f, c->pid, pd, c->g, c->p.rho0, c->scale,
                           c->st));
    const int s = int(c->steps & 1);
    HIPCHK(c, launch_near(c->flags[s], c->pid, c->list_cell, c->list_mask, pd, c->g, c->st));
    // the other flag buffer and pose buffer start as copies of the current
    // ones: the first step writes its successor flags over the region of
    // this pose, which then covers every flag the buffer holds
    HIPCHK(c, hipMemcpyAsync(c->flags[s ^ 1], c->flags[s], c->g.ncell, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->ps[s ^ 1], c->ps[s], size_t(c->np) * sizeof(PState), hipMemcpyDeviceToDevice,
                             c->st));
    return LBM_OK;
}

static lbm_status check_device_errors(lbm_ctx *c)
{
    DevCounters h;
    HIPCHK(c, hipMemcpyAsync(&h, c->ctr, sizeof h, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (h.err_unstable)
        return fail(c, LBM_E_UNSTABLE, (h.err_unstable & 1) ? "non-finite force or torque on the device"
                                                            : "non-finite population on the device");
    if (h.err_wall) return fail(c, LBM_E_STATE, "a fiber came within one cell of an x or y wall");
    if (h.err_capacity)
        return fail(c, LBM_E_STATE,
                    std::string("internal capacity exceeded (") +
                        ((h.err_capacity & 4) ? "changed-cell list"
                                                  : (h.err_capacity & 2) ? "boundary list" : "neighbour list") +
                        ")");
    return LBM_OK;
}

// One time step as a two-branch graph of kernels:
//   st : bulk sweep -----------------------------------------------------------+
//   st2: boundary cells (F0, M0) + A, B, C sums -> rigid -> remap -> near/list -+--> next step
// The bulk sweep touches only slots of bulk cells; the boundary update, the
// refill of the remap and the momentum exchange touch only slots and data
// of cells next to fibers, so the branches are independent; the sums A, B, C
// read only the list, the cell owners and the poses.  The bulk sweep of step
// n reads flags[n & 1]; the flag and list rebuild writes the flags of step
// n + 1 into flags[(n + 1) & 1], over the remap region of the previous,
// current and new poses, which holds every cell whose flag differs between
// steps n - 1 and n + 1, so it runs beside the bulk sweep.
static void launch_one_step(lbm_ctx *c, int64_t step_index, bool with_events, hipEvent_t e0,
                            hipEvent_t e1, hipError_t *err)
{
    const bool odd = (step_index & 1) != 0;
    PState *cur = c->ps[step_index & 1], *next = c->ps[(step_index + 1) & 1];
    BndData b{};
    b.cell = c->list_cell;
    b.mask = c->list_mask;
    b.seg_off = c->seg_off;
    b.seg_cnt = c->seg_cnt;
    b.seg_cap = c->seg_cap;
    b.np = c->np;
    b.bpf = c->bpf;
    b.pid = c->pid;
    b.ps = cur;
    b.mea = c->mea;
    b.ctr = c->ctr;
    hipError_t e = hipSuccess;
    // momentum stabilization: the sweep kernels read the mean and write their
    // sums (bulk workgroups first); after the join the next mean is formed
    const bool stab = c->p.stabilize != 0;
    const double *su = stab ? c->stab : nullptr;
    double *sp = stab ? c->stab + STAB_HEAD : nullptr;
    double *sp_b = stab ? sp + 4 * size_t(c->sweep_grid) : nullptr;
    if (!c->np) {
        e = launch_sweep(c->sk, odd, c->f, c->flags[step_index & 1], c->g, c->ph, c->sweep_grid, c->st,
                         with_events ? e0 : nullptr, with_events ? e1 : nullptr, su, sp);
        if (e == hipSuccess && stab)
            e = launch_stab_update(c->sk, !odd, c->f, c->g, c->ph, c->stab, c->sweep_grid, c->cov, c->cov_cap, c->st);
        if (e != hipSuccess && *err == hipSuccess) *err = e;
        return;
    }
    if (c->closure) {
        // learned closure: features of the state the sweep reads, network,
        // corrections for the rigid-body update of this step
        const MlpDev md = mlp_device_view(c->closure);
        const double gamma = 2.0 * c->p.wall_u / c->p.nz, nu = (c->p.tau - 0.5) / 3.0;
        e = launch_closure_step(c->sk, odd, c->f, c->flags[step_index & 1], c->pid, cur, c->pc, c->np, c->g, c->ph,
                                gamma, md, c->p.rho0, nu, c->corr, c->cstats, c->st);
    }
    if (e == hipSuccess) e = hipEventRecord(c->ev_fork, c->st);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->st2, c->ev_fork, 0);
    // Launch order of the two branches (measured): the branch expected to be
    // longer goes first.  A resident grid-stride bulk grid (up to 1024
    // workgroups, FP32/FP64) over a lattice large against the boundary list
    // (256^3 with 64 fibers) goes first, since all its workgroups must start
    // together; the boundary launch goes first when the bulk grid is large
    // (16-bit storage: it would hold the boundary workgroups off until it
    // drains) or the lattice is small against the list (128^3 with 200
    // fibers: the particle branch is the longer one).
    const bool bulk_first = c->sweep_grid <= 1024u && uint64_t(c->g.ncell) >= 32ull * c->list_cap;
    if (e == hipSuccess && !bulk_first)
        e = launch_boundary(c->sk, odd, c->f, c->g, c->ph, b, c->st2, su, sp_b);
    if (e == hipSuccess)
        e = launch_sweep(c->sk, odd, c->f, c->flags[step_index & 1], c->g, c->ph, c->sweep_grid, c->st,
                         with_events ? e0 : nullptr, with_events ? e1 : nullptr, su, sp);
    if (e == hipSuccess && bulk_first)
        e = launch_boundary(c->sk, odd, c->f, c->g, c->ph, b, c->st2, su, sp_b);
    PartData pd = part_data(c, cur, next);
    if (stab) {
        pd.cov = c->cov;
        pd.cov_cap = c->cov_cap;
    }
    if (e == hipSuccess) e = launch_rigid(pd, c->g, c->st2);
    if (e == hipSuccess) e = launch_remap(c->sk, !odd, c->f, c->pid, pd, c->g, c->p.rho0, c->scale, c->st2);
    if (e == hipSuccess)
        e = launch_near(c->flags[(step_index + 1) & 1], c->pid, c->list_cell, c->list_mask, pd, c->g, c->st2);
    if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->st2);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->st, c->ev_join, 0);
    if (e == hipSuccess && stab)
        e = launch_stab_update(c->sk, !odd, c->f, c->g, c->ph, c->stab, c->sweep_grid + c->bnd_grid, c->cov,
                               c->cov_cap, c->st);
    if (e != hipSuccess && *err == hipSuccess) *err = e;
}

static lbm_status build_graph(lbm_ctx *c)
{
    hipError_t e = hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("capture: ") + hipGetErrorString(e));
    hipError_t le = hipSuccess;
    launch_one_step(c, 0, false, nullptr, nullptr, &le);
    launch_one_step(c, 1, false, nullptr, nullptr, &le);
    e = hipStreamEndCapture(c->st, &c->graph);
    if (le != hipSuccess || e != hipSuccess) {
        drop_graph(c);
        return fail(c, LBM_E_HIP, std::string("capture failed: ") +
                                      hipGetErrorString(le != hipSuccess ? le : e));
    }
    e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(c);
        return fail(c, LBM_E_HIP, std::string("instantiate: ") + hipGetErrorString(e));
    }
    return LBM_OK;
}

// ====================================================================== ABI
extern "C" {

lbm_status lbm_params_default(lbm_params *p)
{
    if (!p) return LBM_E_ARG;
    std::memset(p, 0, sizeof *p);
    p->nx = p->ny = p->nz = 32;
    p->collision = LBM_TRT;
    p->tau = 0.8;
    p->magic = 3.0 / 16.0;
    p->rho0 = 1.0;
    p->storage = LBM_F32;
    p->init_profile = LBM_INIT_REST;
    p->coupling = LBM_COUPLING_IMPLICIT;
    p->fp16_scale_log2 = 14;
    p->history_capacity = 4096;
    p->sweep_grid = 0;
    p->q_pad = -1;
    p->contact_range = 1.0;
    return LBM_OK;
}

lbm_status lbm_lattice(int32_t *c, double *w)
{
    for (int q = 0; q < Q; ++q) {
        if (c) {
            c[3 * q] = CX[q];
            c[3 * q + 1] = CY[q];
            c[3 * q + 2] = CZ[q];
        }
        if (w) w[q] = wq(q);
    }
    return LBM_OK;
}

lbm_status lbm_create(const lbm_params *p, lbm_ctx **out)
{
    if (!p || !out) return LBM_E_ARG;
    *out = nullptr;
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return LBM_E_ARG;
    const double ncell = double(p->nx) * p->ny * p->nz;
    if ((double(p->nz) + 2.0) * p->nx * p->ny + 65536.0 >= 4294967295.0) return LBM_E_ARG;
    if (p->sweep_grid < 0 || p->q_pad > (1 << 20)) return LBM_E_ARG;
    if (!(p->tau > 0.5) || !(std::fabs(p->wall_u) < 0.1) || !(p->rho0 > 0.0)) return LBM_E_ARG;
    if (p->collision != LBM_TRT && p->collision != LBM_SRT) return LBM_E_ARG;
    if (p->collision == LBM_TRT && !(p->magic > 0.0)) return LBM_E_ARG;
    if (p->storage < 0 || p->storage > 3 || p->history_capacity < 1) return LBM_E_ARG;
    if (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 20) return LBM_E_ARG;
    if (p->coupling < LBM_COUPLING_IMPLICIT || p->coupling > LBM_COUPLING_IMPLICIT_PLAIN) return LBM_E_ARG;
    if (p->stabilize != 0 && p->stabilize != 1) return LBM_E_ARG;
    if (p->x_walls < 0 || p->x_walls > 2 || p->y_walls < 0 || p->y_walls > 2) return LBM_E_ARG;
    if (p->z_free_slip != 0 && (p->z_free_slip != 1 || p->z_periodic || p->wall_u != 0.0)) return LBM_E_ARG;
    if (!(p->contact_stiffness >= 0.0) || !std::isfinite(p->contact_stiffness)) return LBM_E_ARG;
    if (p->contact_stiffness > 0.0 && !(p->contact_range > 0.0 && std::isfinite(p->contact_range))) return LBM_E_ARG;
    // changed-cell entries keep a flag in bit 31
    if (p->stabilize && ncell >= 2147483648.0) return LBM_E_ARG;
    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return LBM_E_NOMEM;
    c->p = *p;
    if (hipGetDevice(&c->dev) != hipSuccess) {
        delete c;
        return LBM_E_HIP;
    }
    c->st = (hipStream_t)p->stream;
    if (!c->st) {
        // graph capture needs a real stream: make a private one (default priority)
        if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return LBM_E_HIP;
        }
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        lbm_destroy(c);
        return LBM_E_HIP;
    }
    c->sk = p->storage;
    // bulk sweep: a grid-stride loop over 256-cell chunks with a few
    // resident workgroups per CU keeps the 38 access streams compact
    {
        const uint32_t nchunk = uint32_t((double(p->nx) * p->ny * p->nz + 255.0) / 256.0);
        // measured on the 256^3 cell: FP32/FP64 best near 512 workgroups
        // (leaving room for the boundary branch), 16-bit storage near 4096
        const uint32_t dflt = (p->storage == LBM_F16DEV || p->storage == LBM_BF16DEV) ? 4096u : 512u;
        uint32_t gsz = p->sweep_grid > 0 ? uint32_t(p->sweep_grid) : dflt;
        c->sweep_grid = gsz < nchunk ? gsz : nchunk;
    }
    c->esz = c->sk == S_F64 ? 8 : (c->sk == S_F32 ? 4 : 2);
    c->scale = c->sk == S_F16 ? std::ldexp(1.0, p->fp16_scale_log2) : 1.0;
    Geo &g = c->g;
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = p->nz;
    g.nxy = uint32_t(p->nx) * uint32_t(p->ny);
    g.ncell = uint32_t(ncell);
    // Direction arrays are padded apart so that the 19 streams of a sweep do
    // not start at addresses that are equal modulo a large power of two.
    const uint64_t pad = p->q_pad >= 0 ? uint64_t(p->q_pad) : 1088u;
    g.qstride = uint64_t(p->nz + 2) * g.nxy + pad;
    g.dnx = make_fastdiv(g.nx);
    g.dnxy = make_fastdiv(g.nxy);
    g.zper = p->z_periodic ? 1 : 0;
    g.xw = p->x_walls;
    g.yw = p->y_walls;
    g.zs = p->z_free_slip;
    Phys<double> &ph = c->ph;
    ph.rho0 = p->rho0;
    ph.omega_e = 1.0 / p->tau;
    ph.omega_o = p->collision == LBM_SRT ? 1.0 / p->tau : 1.0 / (0.5 + p->magic / (p->tau - 0.5));
    ph.wall_u = p->z_periodic ? 0.0 : p->wall_u;
    for (int k = 0; k < 3; ++k) ph.g[k] = p->body_force[k];
    ph.has_g = (p->body_force[0] != 0.0 || p->body_force[1] != 0.0 || p->body_force[2] != 0.0);
    ph.scale = c->scale;
    ph.inv_scale = 1.0 / c->scale;
    lbm_status s = LBM_OK;
    auto bail = [&](lbm_status st, const char *m) {
        lbm_destroy(c);
        (void)m;
        return st;
    };
    if (hipMalloc(&c->f, size_t(Q) * g.qstride * c->esz) != hipSuccess) return bail(LBM_E_NOMEM, "f");
    c->device_bytes += int64_t(size_t(Q) * g.qstride * c->esz);
    if (dalloc(c, &c->flags[0], g.ncell) != hipSuccess || dalloc(c, &c->flags[1], g.ncell) != hipSuccess ||
        dalloc(c, &c->pid, g.ncell) != hipSuccess ||
        dalloc(c, &c->ctr, 1) != hipSuccess)
        return bail(LBM_E_NOMEM, "fields");
    if (hipMemsetAsync(c->flags[0], 0, g.ncell, c->st) != hipSuccess ||
        hipMemsetAsync(c->flags[1], 0, g.ncell, c->st) != hipSuccess ||
        hipMemsetAsync(c->pid, 0xFF, size_t(g.ncell) * 4, c->st) != hipSuccess ||
        hipMemsetAsync(c->ctr, 0, sizeof(DevCounters), c->st) != hipSuccess)
        return bail(LBM_E_HIP, "memset");
    if (launch_init(c->sk, c->f, g, p->rho0, ph.wall_u, p->init_profile == LBM_INIT_COUETTE, c->scale,
                    c->st) != hipSuccess)
        return bail(LBM_E_HIP, "init");
    if (alloc_stab(c) != LBM_OK) return bail(LBM_E_NOMEM, "stabilization");
    if (hipStreamSynchronize(c->st) != hipSuccess) return bail(LBM_E_HIP, "sync");
    (void)s;
    *out = c;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx *c)
{
    if (!c) return LBM_E_ARG;
    hipStreamSynchronize(c->st);
    drop_graph(c);
    for (hipEvent_t e : c->ev) hipEventDestroy(e);
    free_particles(c);
    dfree(c->stab);
    dfree(c->cov);
    dfree(c->corr);
    dfree(c->cstats);
    dfree(c->f);
    dfree(c->flags[0]);
    dfree(c->flags[1]);
    dfree(c->pid);
    dfree(c->ctr);
    if (c->st2) hipStreamDestroy(c->st2);
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_join) hipEventDestroy(c->ev_join);
    if (c->own_stream) hipStreamDestroy(c->st);
    delete c;
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : "null context"; }

lbm_status lbm_add_fiber(lbm_ctx *c, const lbm_fiber *f, int32_t *id)
{
    if (!c || !f) return fail(c, LBM_E_ARG, "null argument");
    if (c->steps != 0) return fail(c, LBM_E_STATE, "fibers can only be added before the first step");
    if (c->closure) return fail(c, LBM_E_STATE, "detach the closure before adding fibers");
    if (!(f->length > 0.0) || !(f->radius > 0.0) || !(f->density_ratio > 0.0))
        return fail(c, LBM_E_ARG, "length, radius and density_ratio must be positive");
    if (f->shape != LBM_SHAPE_CYLINDER && f->shape != LBM_SHAPE_SPHEROCYLINDER)
        return fail(c, LBM_E_ARG, "unknown fiber shape");
    if (f->shape == LBM_SHAPE_SPHEROCYLINDER && !(f->length >= 2.0 * f->radius))
        return fail(c, LBM_E_ARG, "a spherocylinder needs length >= 2 radius");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(f->force[k]) || !std::isfinite(f->torque[k]))
            return fail(c, LBM_E_ARG, "non-finite external force or torque");
    const double qn = std::sqrt(f->quat[0] * f->quat[0] + f->quat[1] * f->quat[1] +
                                f->quat[2] * f->quat[2] + f->quat[3] * f->quat[3]);
    if (!(qn > 0.0)) return fail(c, LBM_E_ARG, "zero quaternion");
    const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    double q[4], t[3];
    for (int k = 0; k < 4; ++k) q[k] = f->quat[k] / qn;
    host_axis(q, t);
    for (int k = 0; k < 3; ++k) {
        if (!(f->center[k] >= 0.0 && f->center[k] < n[k]))
            return fail(c, LBM_E_GEOM, "centre outside the domain");
        const double ext = f->shape == LBM_SHAPE_SPHEROCYLINDER
                               ? (0.5 * f->length - f->radius) * std::fabs(t[k]) + f->radius
                               : 0.5 * f->length * std::fabs(t[k]) +
                                     f->radius * std::sqrt(std::fmax(0.0, 1.0 - t[k] * t[k]));
        const bool per = (k == 0 && !c->p.x_walls) || (k == 1 && !c->p.y_walls) || (k == 2 && c->p.z_periodic);
        if (per && !(f->length * 0.5 + f->radius < 0.5 * n[k] - 1.0))
            return fail(c, LBM_E_GEOM, "fiber longer than half the periodic domain");
        if (!per && (f->center[k] - ext < 1.0 || f->center[k] + ext > n[k] - 2.0))
            return fail(c, LBM_E_GEOM, "fiber within one cell of a wall");
    }
    if ((c->np + 1) * NACC * 8 > 65536) return fail(c, LBM_E_ARG, "at most 302 fibers per context");
    if (c->p.contact_stiffness > 0.0 && (c->np + 1) * (NACC + 6) * 8 > 65536)
        return fail(c, LBM_E_ARG, "at most 248 fibers per context with contacts");
    const PConst pc = fiber_constants(f->length, f->radius, f->density_ratio * c->p.rho0, f->shape, f->force,
                                      f->torque);
    c->fib.push_back(*f);
    c->pch.push_back(pc);
    c->traj_h.emplace_back();
    c->np++;
    lbm_status s = upload_particles(c);
    if (s == LBM_OK) s = setup_mapping(c, nullptr);
    unsigned long long ov_before = 0;
    DevCounters h{};
    if (s == LBM_OK) {
        hipError_t e = hipMemcpyAsync(&h, c->ctr, sizeof h, hipMemcpyDeviceToHost, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        if (e != hipSuccess) s = fail(c, LBM_E_HIP, hipGetErrorString(e));
    }
    if (s == LBM_OK && (h.overlaps > ov_before || h.err_capacity)) {
        // reject: remove the fiber and re-map the others from scratch
        c->fib.pop_back();
        c->pch.pop_back();
        c->traj_h.pop_back();
        c->np--;
        hipError_t e = hipMemsetAsync(c->flags[0], 0, c->g.ncell, c->st);
        if (e == hipSuccess) e = hipMemsetAsync(c->flags[1], 0, c->g.ncell, c->st);
        if (e == hipSuccess) e = hipMemsetAsync(c->pid, 0xFF, size_t(c->g.ncell) * 4, c->st);
        if (e == hipSuccess) e = hipMemsetAsync(c->ctr, 0, sizeof(DevCounters), c->st);
        if (e != hipSuccess) return fail(c, LBM_E_HIP, hipGetErrorString(e));
        lbm_status s2 = upload_particles(c);
        if (s2 == LBM_OK) s2 = setup_mapping(c, nullptr);
        if (s2 != LBM_OK) return s2;
        e = hipStreamSynchronize(c->st);
        if (e != hipSuccess) return fail(c, LBM_E_HIP, hipGetErrorString(e));
        return fail(c, LBM_E_GEOM, h.err_capacity ? "internal capacity exceeded while mapping"
                                                 : "fiber overlaps another fiber");
    }
    if (s != LBM_OK) return s;
    if (id) *id = c->np - 1;
    c->err.clear();
    return LBM_OK;
}

lbm_status lbm_set_fiber_kinematics(lbm_ctx *c, int32_t id, const double *traj, int64_t nsteps)
{
    if (!c || id < 0 || id >= c->np || nsteps < 0 || (nsteps > 0 && !traj))
        return fail(c, LBM_E_ARG, "bad fiber id or trajectory");
    HIPCHK(c, hipStreamSynchronize(c->st));
    // fetch the current states so that the re-upload keeps them
    std::vector<PState> hs(c->np);
    HIPCHK(c, hipMemcpy(hs.data(), c->ps[c->steps & 1], c->np * sizeof(PState), hipMemcpyDeviceToHost));
    std::vector<int64_t> pos(c->np);
    HIPCHK(c, hipMemcpy(pos.data(), c->traj_pos, c->np * sizeof(int64_t), hipMemcpyDeviceToHost));
    // keep only the unconsumed part of the other trajectories
    for (int i = 0; i < c->np; ++i) {
        if (i == id) continue;
        auto &t = c->traj_h[i];
        const size_t used = size_t(std::min<int64_t>(pos[i], int64_t(t.size() / 13))) * 13;
        t.erase(t.begin(), t.begin() + used);
    }
    c->traj_h[id].assign(traj, traj + nsteps * 13);
    std::vector<Box> boxes(c->np);
    HIPCHK(c, hipMemcpy(boxes.data(), c->box_cur, c->np * sizeof(Box), hipMemcpyDeviceToHost));
    lbm_status s = upload_particles(c);
    if (s != LBM_OK) return s;
    HIPCHK(c, hipMemcpyAsync(c->ps[c->steps & 1], hs.data(), c->np * sizeof(PState),
                             hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->box_cur, boxes.data(), c->np * sizeof(Box), hipMemcpyHostToDevice, c->st));
    // rebuild the remap work and list for the unchanged poses
    s = setup_mapping(c, nullptr);
    if (s != LBM_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->st));
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t n)
{
    if (!c) return LBM_E_ARG;
    if (n < 0) return fail(c, LBM_E_ARG, "negative step count");
    hipError_t err = n > 0 ? refresh_stab(c) : hipSuccess;
    auto direct = [&](void) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            while (c->ev.size() < c->ev_used + 2) {
                hipEvent_t e;
                const hipError_t ce = hipEventCreate(&e);
                if (ce != hipSuccess) {   // no step without its events
                    err = ce;
                    return;
                }
                c->ev.push_back(e);
            }
            e0 = c->ev[c->ev_used];
            e1 = c->ev[c->ev_used + 1];
            c->ev_used += 2;
        }
        launch_one_step(c, c->steps, c->timing, e0, e1, &err);
        c->steps++;
    };
    int64_t left = n;
    if (!c->timing && left >= 4) {
        if (c->steps & 1) {
            direct();
            --left;
        }
        if (!c->gexec) {
            lbm_status s = build_graph(c);
            if (s != LBM_OK) return s;
        }
        while (left >= 2 && err == hipSuccess) {
            err = hipGraphLaunch(c->gexec, c->st);
            c->steps += 2;
            left -= 2;
        }
    }
    while (left > 0 && err == hipSuccess) {
        direct();
        --left;
    }
    if (err != hipSuccess) return fail(c, LBM_E_HIP, std::string("launch: ") + hipGetErrorString(err));
    return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx *c)
{
    if (!c) return LBM_E_ARG;
    HIPCHK(c, launch_check_finite(c->sk, c->f, uint64_t(Q) * c->g.qstride, c->ctr, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return check_device_errors(c);
}

lbm_status lbm_get_force_torque(lbm_ctx *c, double *F, double *M)
{
    if (!c) return LBM_E_ARG;
    lbm_status s = check_device_errors(c);
    if (s != LBM_OK) return s;
    if (c->np == 0) return LBM_OK;
    std::vector<double> h(size_t(c->np) * 6);
    HIPCHK(c, hipMemcpy(h.data(), c->ft, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < c->np; ++i)
        for (int k = 0; k < 3; ++k) {
            if (F) F[3 * i + k] = h[6 * i + k];
            if (M) M[3 * i + k] = h[6 * i + 3 + k];
        }
    return LBM_OK;
}

lbm_status lbm_get_fields(lbm_ctx *c, void *rho, void *u, uint8_t *flags, int32_t *pid,
                          int32_t dst_is_device)
{
    if (!c) return LBM_E_ARG;
    lbm_status s = check_device_errors(c);
    if (s != LBM_OK) return s;
    const size_t n = c->g.ncell, rsz = c->sk == S_F64 ? 8 : 4;
    void *drho = nullptr, *du = nullptr;
    if (rho) {
        if (dst_is_device) drho = rho;
        else HIPCHK(c, hipMalloc(&drho, n * rsz));
    }
    if (u) {
        if (dst_is_device) du = u;
        else HIPCHK(c, hipMalloc(&du, 3 * n * rsz));
    }
    PState *cur = c->np ? c->ps[c->steps & 1] : nullptr;
    if (rho || u)
        HIPCHK(c, launch_decode(c->sk, (c->steps & 1) != 0, c->f, c->flags[c->steps & 1], c->pid, cur, c->g, c->ph,
                                drho, du, nullptr, c->st));
    const hipMemcpyKind k = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (rho && !dst_is_device) HIPCHK(c, hipMemcpyAsync(rho, drho, n * rsz, k, c->st));
    if (u && !dst_is_device) HIPCHK(c, hipMemcpyAsync(u, du, 3 * n * rsz, k, c->st));
    if (flags) {
        // logical flags: 0 fluid, 1 fiber (the near-boundary bit is internal)
        std::vector<uint8_t> hf(n);
        HIPCHK(c, hipMemcpyAsync(hf.data(), c->flags[c->steps & 1], n, hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        for (auto &v : hf) v &= F_SOLID;
        HIPCHK(c, hipMemcpyAsync(flags, hf.data(), n, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    if (pid) HIPCHK(c, hipMemcpyAsync(pid, c->pid, n * 4, k, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (rho && !dst_is_device) hipFree(drho);
    if (u && !dst_is_device) hipFree(du);
    return LBM_OK;
}

// ------------------------------------------------------------------ allocation-free field readback
// The staging memory of lbm_get_fields_static: a fixed device array, one copy
// per GPU, held until the process ends.  Host code never passes the name
// `scratch` to a kernel or a copy (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns, kept
// per device in scratch_ptr.
static constexpr size_t SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static constexpr int SCRATCH_MAX_DEV = 64;
static void *scratch_ptr[SCRATCH_MAX_DEV] = {};
static std::mutex scratch_mu;

// device address of `scratch` on device dev, resolved once with dev current
static hipError_t scratch_on(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = ptr;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

lbm_status lbm_get_fields_static(lbm_ctx *c, void *rho, void *u, uint8_t *flags, int32_t *pid)
{
    if (!c) return LBM_E_ARG;
    if (c->dev < 0 || c->dev >= SCRATCH_MAX_DEV)
        return fail(c, LBM_E_ARG, "lbm_get_fields_static: device index beyond the scratch table");
    lbm_status s = check_device_errors(c);
    if (s != LBM_OK) return s;
    void *sp = nullptr;
    HIPCHK(c, scratch_on(c->dev, &sp));
    const size_t n = c->g.ncell, rsz = c->sk == S_F64 ? 8 : 4;
    // cells per chunk: rho (1 value) and u (3 values) of each cell in the scratch
    const size_t chunk = SCRATCH_BYTES / (4 * rsz);
    char *srho = (char *)sp, *su = (char *)sp + chunk * rsz;
    PState *cur = c->np ? c->ps[c->steps & 1] : nullptr;
    const bool sw = (c->steps & 1) != 0;
    for (size_t c0 = 0; (rho || u) && c0 < n; c0 += chunk) {
        const size_t m = std::min(chunk, n - c0);
        HIPCHK(c, launch_decode_range(c->sk, sw, c->f, c->flags[c->steps & 1], c->pid, cur, c->g, c->ph,
                                      rho ? (void *)srho : nullptr, u ? (void *)su : nullptr, nullptr,
                                      uint32_t(c0), uint32_t(c0 + m), chunk, c->st));
        if (rho)
            HIPCHK(c, hipMemcpyAsync((char *)rho + c0 * rsz, srho, m * rsz, hipMemcpyDeviceToHost, c->st));
        if (u)
            for (int k = 0; k < 3; ++k)
                HIPCHK(c, hipMemcpyAsync((char *)u + (k * n + c0) * rsz, su + k * chunk * rsz, m * rsz,
                                         hipMemcpyDeviceToHost, c->st));
        // the next chunk overwrites the scratch: wait for the copies out of it
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    if (flags) HIPCHK(c, hipMemcpyAsync(flags, c->flags[c->steps & 1], n, hipMemcpyDeviceToHost, c->st));
    if (pid) HIPCHK(c, hipMemcpyAsync(pid, c->pid, n * 4, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    // logical flags: 0 fluid, 1 fiber (the near-boundary bit is internal)
    if (flags)
        for (size_t i = 0; i < n; ++i) flags[i] &= F_SOLID;
    return LBM_OK;
}

lbm_status lbm_get_fiber_state(lbm_ctx *c, double *X, double *q, double *V, double *W)
{
    if (!c) return LBM_E_ARG;
    lbm_status s = check_device_errors(c);
    if (s != LBM_OK) return s;
    if (c->np == 0) return LBM_OK;
    std::vector<PState> h(c->np);
    HIPCHK(c, hipMemcpy(h.data(), c->ps[c->steps & 1], c->np * sizeof(PState), hipMemcpyDeviceToHost));
    for (int i = 0; i < c->np; ++i) {
        for (int k = 0; k < 3; ++k) {
            if (X) X[3 * i + k] = h[i].X[k];
            if (V) V[3 * i + k] = h[i].V[k];
            if (W) W[3 * i + k] = h[i].W[k];
        }
        if (q)
            for (int k = 0; k < 4; ++k) q[4 * i + k] = h[i].q[k];
    }
    return LBM_OK;
}

lbm_status lbm_set_fiber_state(lbm_ctx *c, int32_t id, const double X[3], const double q[4],
                               const double V[3], const double W[3])
{
    if (!c || id < 0 || id >= c->np || !X || !q || !V || !W) return fail(c, LBM_E_ARG, "bad argument");
    HIPCHK(c, hipStreamSynchronize(c->st));
    PState *cur = c->ps[c->steps & 1], *other = c->ps[(c->steps + 1) & 1];
    std::vector<PState> h(c->np);
    HIPCHK(c, hipMemcpy(h.data(), cur, c->np * sizeof(PState), hipMemcpyDeviceToHost));
    // keep the old states for the refill of uncovered cells
    HIPCHK(c, hipMemcpy(other, h.data(), c->np * sizeof(PState), hipMemcpyHostToDevice));
    lbm_fiber f = c->fib[id];
    for (int k = 0; k < 3; ++k) {
        f.center[k] = X[k];
        f.vel[k] = V[k];
        f.omega[k] = W[k];
    }
    for (int k = 0; k < 4; ++k) f.quat[k] = q[k];
    h[id] = make_state(f, c->pch[id]);
    HIPCHK(c, hipMemcpy(cur, h.data(), c->np * sizeof(PState), hipMemcpyHostToDevice));
    lbm_status s = setup_mapping(c, other);
    if (s != LBM_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->st));
    return check_device_errors(c);
}

lbm_status lbm_get_history(lbm_ctx *c, int64_t first, int64_t count, double *out)
{
    if (!c || !out || count < 0) return fail(c, LBM_E_ARG, "bad argument");
    lbm_status s = check_device_errors(c);
    if (s != LBM_OK) return s;
    const int64_t cap = c->p.history_capacity;
    if (first < 0 || first + count > c->steps || first < c->steps - cap)
        return fail(c, LBM_E_ARG, "history window not available");
    if (c->np == 0 || count == 0) return LBM_OK;
    const size_t rec = size_t(c->np) * 19;
    for (int64_t i = 0; i < count;) {
        const int64_t slot = (first + i) % cap;
        const int64_t run = std::min<int64_t>(count - i, cap - slot);
        HIPCHK(c, hipMemcpy(out + i * rec, c->hist + slot * rec, size_t(run) * rec * sizeof(double),
                            hipMemcpyDeviceToHost));
        i += run;
    }
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx *c, double *f)
{
    if (!c || !f) return LBM_E_ARG;
    lbm_status s = check_device_errors(c);
    if (s != LBM_OK) return s;
    double *d = nullptr;
    const size_t n = size_t(Q) * c->g.ncell;
    HIPCHK(c, hipMalloc(&d, n * sizeof(double)));
    PState *cur = c->np ? c->ps[c->steps & 1] : nullptr;
    hipError_t e = launch_decode(c->sk, (c->steps & 1) != 0, c->f, c->flags[c->steps & 1], c->pid, cur, c->g, c->ph,
                                 nullptr, nullptr, d, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(d);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx *c, const double *f)
{
    if (!c || !f) return LBM_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->st));
    double *d = nullptr;
    const size_t n = size_t(Q) * c->g.ncell;
    HIPCHK(c, hipMalloc(&d, n * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d, f, n * sizeof(double), hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) e = launch_encode(c->sk, (c->steps & 1) != 0, c->f, c->g, c->p.rho0, c->scale, d, c->st);
    c->stab_stale = true;
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(d);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_get_mean_velocity(lbm_ctx *c, double ubar[3], int64_t *nfluid)
{
    if (!c || !ubar) return fail(c, LBM_E_ARG, "null argument");
    if (!c->p.stabilize) return fail(c, LBM_E_STATE, "momentum stabilization is off");
    HIPCHK(c, refresh_stab(c));
    double h[4];
    HIPCHK(c, hipMemcpyAsync(h, c->stab, sizeof h, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (int k = 0; k < 3; ++k) ubar[k] = h[k];
    if (nfluid) *nfluid = int64_t(h[3]);
    return check_device_errors(c);
}

// ---------------------------------------------------------------- checkpoint
// Every device buffer that carries state between steps, with its size (the
// same formulas as the allocations in lbm_create, alloc_stab and
// upload_particles), in a fixed order.
struct BufRef {
    void *p;
    size_t bytes;
};
static std::vector<BufRef> state_buffers(lbm_ctx *c)
{
    std::vector<BufRef> v;
    const size_t nc = c->g.ncell;
    v.push_back({c->f, size_t(Q) * c->g.qstride * c->esz});
    v.push_back({c->flags[0], nc});
    v.push_back({c->flags[1], nc});
    v.push_back({c->pid, nc * sizeof(int32_t)});
    v.push_back({c->ctr, sizeof(DevCounters)});
    if (c->p.stabilize) {
        const uint32_t nslot = std::max(STAB_SCAN_GRID, c->sweep_grid + c->bnd_grid);
        v.push_back({c->stab, (size_t(STAB_HEAD) + 4 * size_t(nslot)) * sizeof(double)});
        v.push_back({c->cov, (size_t(c->cov_cap) + 1) * sizeof(uint32_t)});
    }
    const size_t np = size_t(c->np);
    if (np) {
        size_t ntraj = 13;
        for (const auto &t : c->traj_h) ntraj += t.size();
        v.push_back({c->ps[0], np * sizeof(PState)});
        v.push_back({c->ps[1], np * sizeof(PState)});
        v.push_back({c->pc, np * sizeof(PConst)});
        v.push_back({c->ps_prev, np * sizeof(PState)});
        v.push_back({c->box_cur, np * sizeof(Box)});
        v.push_back({c->box_prev, np * sizeof(Box)});
        v.push_back({c->box_remap, np * sizeof(Box)});
        v.push_back({c->mea, np * NACC * sizeof(long long)});
        v.push_back({c->seg_off, np * sizeof(uint32_t)});
        v.push_back({c->seg_cap, np * sizeof(uint32_t)});
        v.push_back({c->seg_cnt, np * sizeof(uint32_t)});
        v.push_back({c->traj, ntraj * sizeof(double)});
        v.push_back({c->traj_pos, np * sizeof(int64_t)});
        v.push_back({c->ft, np * 6 * sizeof(double)});
        v.push_back({c->hist, size_t(c->p.history_capacity) * np * 19 * sizeof(double)});
        v.push_back({c->list_cell, size_t(c->list_cap) * sizeof(uint32_t)});
        v.push_back({c->list_mask, size_t(c->list_cap) * sizeof(uint32_t)});
    }
    return v;
}

static const char CKPT_MAGIC[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};
static constexpr size_t CKPT_CHUNK = size_t(64) << 20;

lbm_status lbm_save(lbm_ctx *c, const char *path)
{
    if (!c || !path) return fail(c, LBM_E_ARG, "null argument");
    HIPCHK(c, hipStreamSynchronize(c->st));
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return fail(c, LBM_E_ARG, std::string("cannot write ") + path);
    bool ok = true;
    auto put = [&](const void *d, size_t n) { ok = ok && std::fwrite(d, 1, n, fp) == n; };
    lbm_params p = c->p;
    p.stream = nullptr;
    const uint64_t psz = sizeof p;
    const int64_t steps = c->steps;
    const int32_t np = c->np, stale = c->stab_stale ? 1 : 0;
    put(CKPT_MAGIC, 8);
    put(&psz, 8);
    put(&p, sizeof p);
    put(&steps, 8);
    put(&np, 4);
    put(&stale, 4);
    if (np) {
        put(c->fib.data(), size_t(np) * sizeof(lbm_fiber));
        put(c->pch.data(), size_t(np) * sizeof(PConst));
        for (const auto &t : c->traj_h) {
            const uint64_t n = t.size();
            put(&n, 8);
            if (n) put(t.data(), n * sizeof(double));
        }
    }
    const std::vector<BufRef> bufs = state_buffers(c);
    const uint64_t nb = bufs.size();
    put(&nb, 8);
    std::vector<char> h(CKPT_CHUNK);
    for (const BufRef &b : bufs) {
        const uint64_t n = b.bytes;
        put(&n, 8);
        for (size_t o = 0; ok && o < b.bytes; o += CKPT_CHUNK) {
            const size_t k = std::min(CKPT_CHUNK, b.bytes - o);
            if (hipMemcpy(h.data(), static_cast<char *>(b.p) + o, k, hipMemcpyDeviceToHost) != hipSuccess) {
                std::fclose(fp);
                return fail(c, LBM_E_HIP, "device read for the checkpoint");
            }
            put(h.data(), k);
        }
    }
    if (std::fclose(fp) != 0) ok = false;
    if (!ok) return fail(c, LBM_E_ARG, std::string("short write to ") + path);
    return LBM_OK;
}

lbm_status lbm_load(const char *path, void *stream, lbm_ctx **out)
{
    if (!path || !out) return LBM_E_ARG;
    *out = nullptr;
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return LBM_E_ARG;
    bool ok = true;
    auto get = [&](void *d, size_t n) { ok = ok && std::fread(d, 1, n, fp) == n; };
    char magic[8] = {0};
    uint64_t psz = 0;
    lbm_params p{};
    get(magic, 8);
    get(&psz, 8);
    if (!ok || std::memcmp(magic, CKPT_MAGIC, 8) != 0 || psz != sizeof p) {
        std::fclose(fp);
        return LBM_E_ARG;
    }
    int64_t steps = 0;
    int32_t np = 0, stale = 1;
    get(&p, sizeof p);
    get(&steps, 8);
    get(&np, 4);
    get(&stale, 4);
    if (!ok || steps < 0 || np < 0 || np > 302) {
        std::fclose(fp);
        return LBM_E_ARG;
    }
    p.stream = stream;
    lbm_ctx *c = nullptr;
    lbm_status s = lbm_create(&p, &c);
    if (s != LBM_OK) {
        std::fclose(fp);
        return s;
    }
    auto bail = [&](lbm_status st) {
        std::fclose(fp);
        lbm_destroy(c);
        return st;
    };
    if (np) {
        c->fib.resize(np);
        c->pch.resize(np);
        c->traj_h.assign(np, std::vector<double>());
        get(c->fib.data(), size_t(np) * sizeof(lbm_fiber));
        get(c->pch.data(), size_t(np) * sizeof(PConst));
        for (int i = 0; ok && i < np; ++i) {
            uint64_t n = 0;
            get(&n, 8);
            if (!ok || n % 13 != 0 || n > (uint64_t(1) << 32)) return bail(LBM_E_ARG);
            c->traj_h[i].resize(n);
            if (n) get(c->traj_h[i].data(), n * sizeof(double));
        }
        if (!ok) return bail(LBM_E_ARG);
        c->np = np;
        c->steps = steps;
        if (upload_particles(c) != LBM_OK) return bail(LBM_E_NOMEM);
    }
    if (hipStreamSynchronize(c->st) != hipSuccess) return bail(LBM_E_HIP);
    const std::vector<BufRef> bufs = state_buffers(c);
    uint64_t nb = 0;
    get(&nb, 8);
    if (!ok || nb != bufs.size()) return bail(LBM_E_ARG);
    std::vector<char> h(CKPT_CHUNK);
    for (const BufRef &b : bufs) {
        uint64_t n = 0;
        get(&n, 8);
        if (!ok || n != b.bytes) return bail(LBM_E_ARG);
        for (size_t o = 0; o < b.bytes; o += CKPT_CHUNK) {
            const size_t k = std::min(CKPT_CHUNK, b.bytes - o);
            get(h.data(), k);
            if (!ok) return bail(LBM_E_ARG);
            if (hipMemcpy(static_cast<char *>(b.p) + o, h.data(), k, hipMemcpyHostToDevice) != hipSuccess)
                return bail(LBM_E_HIP);
        }
    }
    std::fclose(fp);
    c->steps = steps;
    c->stab_stale = stale != 0;
    *out = c;
    return LBM_OK;
}

lbm_status lbm_get_params(lbm_ctx *c, lbm_params *out)
{
    if (!c || !out) return LBM_E_ARG;
    *out = c->p;
    return LBM_OK;
}

lbm_status lbm_get_info(lbm_ctx *c, lbm_info *info)
{
    if (!c || !info) return LBM_E_ARG;
    DevCounters h{};
    HIPCHK(c, hipMemcpyAsync(&h, c->ctr, sizeof h, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    info->steps_done = c->steps;
    info->nfibers = c->np;
    info->parity = int32_t(c->steps & 1);
    int64_t nb = 0;
    if (c->np) {
        std::vector<uint32_t> cnt(c->np);
        HIPCHK(c, hipMemcpy(cnt.data(), c->seg_cnt, c->np * sizeof(uint32_t), hipMemcpyDeviceToHost));
        for (uint32_t v : cnt) nb += v;
    }
    info->boundary_cells = nb;
    info->overlap_events = int64_t(h.overlaps);
    info->device_bytes = c->device_bytes;
    info->population_bytes = int64_t(size_t(Q) * c->g.qstride * c->esz);
    return LBM_OK;
}

lbm_status lbm_enable_sweep_timing(lbm_ctx *c, int32_t on)
{
    if (!c) return LBM_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->timing = on != 0;
    c->ev_used = 0;
    c->timed_ms = 0.0;
    c->timed_sweeps = 0;
    return LBM_OK;
}

lbm_status lbm_get_sweep_time(lbm_ctx *c, double *total_ms, int64_t *nsweeps)
{
    if (!c) return LBM_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        c->timed_ms += ms;
        c->timed_sweeps++;
    }
    c->ev_used = 0;
    if (total_ms) *total_ms = c->timed_ms;
    if (nsweeps) *nsweeps = c->timed_sweeps;
    return LBM_OK;
}

lbm_status lbm_set_closure(lbm_ctx *c, lbm_mlp *m)
{
    if (!c) return LBM_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->st));
    drop_graph(c);
    if (!m) {
        c->closure = nullptr;
        return LBM_OK;
    }
    if (c->g.xw || c->g.yw || c->g.zs)
        return fail(c, LBM_E_STATE, "the closure's features assume periodic x and y and no free-slip walls");
    if (c->p.z_periodic || c->p.wall_u == 0.0)
        return fail(c, LBM_E_ARG, "the closure needs a shear cell (moving walls, U != 0)");
    if (c->np == 0) return fail(c, LBM_E_STATE, "add the fibers before attaching the closure");
    dfree(c->corr);
    HIPCHK(c, dalloc(c, &c->corr, size_t(c->np) * LBM_MLP_OUT));
    if (!c->cstats) HIPCHK(c, dalloc(c, &c->cstats, 2));
    HIPCHK(c, hipMemsetAsync(c->corr, 0, size_t(c->np) * LBM_MLP_OUT * sizeof(double), c->st));
    HIPCHK(c, hipMemsetAsync(c->cstats, 0, 2 * sizeof(unsigned long long), c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->closure = m;
    return LBM_OK;
}

lbm_status lbm_get_closure_stats(lbm_ctx *c, int64_t *applied, int64_t *fallbacks)
{
    if (!c) return LBM_E_ARG;
    unsigned long long h[2] = {0, 0};
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (c->cstats) HIPCHK(c, hipMemcpy(h, c->cstats, sizeof h, hipMemcpyDeviceToHost));
    if (applied) *applied = int64_t(h[0]);
    if (fallbacks) *fallbacks = int64_t(h[1]);
    return LBM_OK;
}

lbm_status lbm_sample_features(lbm_ctx *c, float *out, int32_t dst_is_device)
{
    if (!c || !out) return LBM_E_ARG;
    if (c->np == 0) return LBM_OK;
    if (c->p.z_periodic || c->p.wall_u == 0.0)
        return fail(c, LBM_E_ARG, "features need a shear cell (moving walls, U != 0)");
    lbm_status s = check_device_errors(c);
    if (s != LBM_OK) return s;
    const size_t n = size_t(c->np) * LBM_MLP_IN;
    float *d = out;
    if (!dst_is_device) HIPCHK(c, hipMalloc(&d, n * sizeof(float)));
    const double gamma = 2.0 * c->p.wall_u / c->p.nz;
    hipError_t e = launch_sample_features(c->sk, (c->steps & 1) != 0, c->f, c->flags[c->steps & 1], c->pid, c->ps[c->steps & 1],
                                          c->pc, c->np, c->g, c->ph, gamma, d, c->st);
    if (e == hipSuccess && !dst_is_device) e = hipMemcpyAsync(out, d, n * sizeof(float), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (!dst_is_device) hipFree(d);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_copy_bytes(void *dst, const void *src, size_t nbytes, void *stream)
{
    if (!dst || !src || (nbytes % 16) != 0) return LBM_E_ARG;
    if (launch_copy(dst, src, nbytes, (hipStream_t)stream) != hipSuccess) return LBM_E_HIP;
    return LBM_OK;
}

}  // extern "C"
