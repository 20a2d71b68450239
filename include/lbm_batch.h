/*
 * lbm_batch.h -- C ABI of the batched form: many small, independent shear
 * cells of uneven size, each with one rigid cylinder fiber, advanced
 * together by one persistent kernel launch (captured in a HIP graph) on one
 * GPU.  Every case runs exactly the coupled method of include/lbm.h (Sec. 4
 * of Bartuschat et al., Computers & Fluids 2015: D3Q19 TRT/SRT AA sweep with
 * moving-wall and moving-obstacle bounce-back, Eqs. LBMMovWall and
 * BBBC; momentum exchange, Eq. LBMhydrodynForce and the torque after it;
 * rigid-body update, Sec. 4.3; remap with refill, Sec. 4.2), with the same
 * per-cell and per-fiber arithmetic, so a case's results equal those of an
 * lbm_ctx created with the same parameters, bit for bit.
 *
 * Work layout: the cases are packed into bins (longest-processing-time
 * order by cell count); one workgroup owns a bin and runs its cases' steps
 * with only intra-workgroup barriers between the phases of a step, so no
 * workgroup ever waits for another.  The number of bins and the workgroup
 * size are tunables, picked by lbm_batch_autotune() from timed trials.
 *
 * Conventions: as in lbm.h (lattice units, [z][y][x] arrays with x fastest,
 * lbm_status returns, lbm_batch_last_error()).  A batch is not thread-safe;
 * lbm_batch_step() only enqueues, the getters synchronise.
 */
#ifndef LBM_BATCH_H
#define LBM_BATCH_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_batch lbm_batch;

/* One case: an nx x ny x nz cell, periodic in x and y, walls at the z ends
 * moving at -/+ wall_u along x (z_periodic = 0), TRT/SRT with relaxation
 * time tau, and one fiber (lbm_fiber of lbm.h; the same geometry checks as
 * lbm_add_fiber apply).  3 <= nx, ny, nz <= 512. */
typedef struct {
    int32_t nx, ny, nz;
    double tau;
    double wall_u;
    lbm_fiber fiber;
} lbm_batch_case;

/* Parameters shared by all cases (meaning as in lbm_params). */
typedef struct {
    int32_t collision;         /* lbm_collision */
    double magic;              /* TRT Lambda */
    double rho0;
    int32_t storage;           /* lbm_storage */
    int32_t init_profile;      /* lbm_init */
    int32_t coupling;          /* lbm_coupling */
    int32_t fp16_scale_log2;
    int64_t history_capacity;  /* steps kept per case (>= 1) */
    void *stream;              /* hipStream_t; NULL: a private stream */
    int32_t threads;           /* workgroup size: 256, 512 or 1024; 0 = 512 */
    int32_t bins;              /* workgroups (bins of cases); 0 = one per compute unit */
} lbm_batch_params;

typedef struct {
    int32_t threads;           /* chosen workgroup size */
    int32_t bins;              /* chosen number of bins */
    double ms_per_step;        /* best trial time per step (all cases) */
    int32_t from_cache;        /* 1: read from the cache file, no trials run */
    int32_t trials;            /* configurations timed */
} lbm_batch_tuning;

typedef struct {
    int64_t steps_done;
    int32_t ncases;
    int32_t bins;
    int32_t threads;
    int64_t cells;             /* sum of nx*ny*nz over the cases */
    int64_t boundary_cells;    /* sum of the cases' boundary-list lengths */
    int64_t device_bytes;
    int64_t population_bytes;
} lbm_batch_info;

/* Defaults: TRT, Lambda 3/16, rho0 1, F32, Couette start, implicit
 * coupling, k = 14, history 4096, NULL stream, automatic threads and bins. */
lbm_status lbm_batch_params_default(lbm_batch_params *p);

/* Allocate ncases cases (ncases >= 1), initialise each lattice with
 * f_eq(rho0, u0(z)) (Eq. fequ_Incompr) and map its fiber (Sec. 4.2).
 * cases[] is copied.  LBM_E_GEOM names the first offending case in the
 * message of lbm_batch_last_error(NULL) and nothing is allocated. */
lbm_status lbm_batch_create(const lbm_batch_params *p, const lbm_batch_case *cases, int32_t ncases,
                            lbm_batch **out);
lbm_status lbm_batch_destroy(lbm_batch *b);
/* Last error message of b, or of the last failed lbm_batch_create when b is NULL. */
const char *lbm_batch_last_error(const lbm_batch *b);

/* Prescribe the motion of case c's fiber for its next nsteps steps, host
 * array [nsteps][13] = X q V W after each step (as lbm_set_fiber_kinematics).
 * Only before the first step. */
lbm_status lbm_batch_set_kinematics(lbm_batch *b, int32_t c, const double *traj, int64_t nsteps);

/* Time trial_steps steps of every candidate (threads in {256, 512, 1024},
 * bins in {CU/2, CU, 2 CU, 4 CU} capped at ncases) and keep the fastest.
 * The trials run on the initial state, which is then restored; only before
 * the first step.  cache_path (may be NULL): a text file of earlier choices,
 * keyed by the case sizes, storage and device; read first and appended to. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t trial_steps, const char *cache_path,
                              lbm_batch_tuning *out);

/* Choose threads and bins directly (0 keeps the current value). */
lbm_status lbm_batch_set_config(lbm_batch *b, int32_t threads, int32_t bins);

/* Enqueue n steps of every case as one persistent launch (replayed from a
 * captured HIP graph when n repeats). */
lbm_status lbm_batch_step(lbm_batch *b, int64_t n);
lbm_status lbm_batch_sync(lbm_batch *b);

/* Force and torque of the last step, FP64 host [ncases][3] (either may be NULL). */
lbm_status lbm_batch_get_force_torque(lbm_batch *b, double *F, double *M);
/* Fiber states, FP64 host [ncases][3] / [ncases][4] (any may be NULL). */
lbm_status lbm_batch_get_fiber_state(lbm_batch *b, double *X, double *q, double *V, double *W);
/* Case c's records [count][19] = F3 M3 X3 q4 V3 W3 for steps first .. first+count-1. */
lbm_status lbm_batch_get_history(lbm_batch *b, int32_t c, int64_t first, int64_t count, double *out);
/* Case c's fields as lbm_get_fields (host or device destination). */
lbm_status lbm_batch_get_fields(lbm_batch *b, int32_t c, void *rho, void *u, uint8_t *flags,
                                int32_t *pid, int32_t dst_is_device);
/* Case c's logical populations, FP64 host [19][nz][ny][nx] (order of lbm_lattice). */
lbm_status lbm_batch_get_populations(lbm_batch *b, int32_t c, double *f);
lbm_status lbm_batch_get_info(lbm_batch *b, lbm_batch_info *info);

#ifdef __cplusplus
}
#endif
#endif
