/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the coupled lattice
 * Boltzmann / rigid-fiber method of Bartuschat, Fischermeier, Gustavsson and
 * Ruede, "Two computational models for simulating the tumbling motion of
 * elongated particles in fluids" (Computers & Fluids, 2015), Sec. 4.
 *
 * One context holds one lattice: by default a periodic-in-x,y shear cell, a
 * D3Q19 lattice with TRT or SRT collision (Sec. 4.1, Eqs. discrLBE-
 * LBMStream), walls half-way below z = 0 and above z = nz-1 that move at -U
 * and +U along x (Eq. LBMMovWall applied to a wall); optionally periodic z,
 * resting no-slip or free-slip walls on the x and y faces and free-slip z
 * walls (Eqs. BBBC, FreeSlipBC; lbm_params below), and rigid cylindrical or
 * spherocylindrical fibers coupled by moving-obstacle bounce-back and
 * momentum exchange (Sec. 4.2, Eqs. LBMMovWall, TransferredMomentum,
 * LBMhydrodynForce) to a rigid-body update on the device (Sec. 4.3).
 *
 * Conventions for every call:
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3.  Cell centres sit at integer
 *     coordinates (x, y, z), 0 <= x < nx etc.  Arrays over cells are
 *     [z][y][x] with x fastest; vector fields are [3][z][y][x].
 *   - Every call returns lbm_status; LBM_OK = 0.  lbm_last_error() gives
 *     the message of the last failure on that context.  No C++ exception
 *     crosses this boundary.
 *   - A context is not thread-safe.  Work is ordered on the context's HIP
 *     stream.  lbm_step() only enqueues; the lbm_get_* calls and lbm_sync()
 *     synchronise the stream and report errors raised on the device
 *     (LBM_E_UNSTABLE for a non-finite force or torque, LBM_E_STATE for an
 *     overflowing internal list).
 *   - The context owns every device buffer it allocates; the caller owns
 *     every buffer it passes in.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_E_ARG = 1,      /* invalid argument */
    LBM_E_NOMEM = 2,    /* device allocation failed */
    LBM_E_HIP = 3,      /* a HIP runtime call failed */
    LBM_E_GEOM = 4,     /* fiber outside the domain, touching a wall, or overlapping */
    LBM_E_UNSTABLE = 5, /* non-finite force/torque detected on the device */
    LBM_E_STATE = 6     /* call not allowed now, or an internal capacity was exceeded */
} lbm_status;

typedef enum { LBM_TRT = 0, LBM_SRT = 1 } lbm_collision;

/* Population storage.  All forms store the deviation f_q - w_q rho0 and
 * collide in FP32 (FP64 for LBM_F64):
 *   LBM_F32     FP32 deviation, 4 B per population
 *   LBM_F16DEV  FP16 of 2^k (f_q - w_q rho0), k = fp16_scale_log2, RNE
 *   LBM_BF16DEV BF16 of (f_q - w_q rho0), RNE
 *   LBM_F64     FP64 deviation, collision in FP64 (debug / parity) */
typedef enum { LBM_F32 = 0, LBM_F16DEV = 1, LBM_BF16DEV = 2, LBM_F64 = 3 } lbm_storage;

typedef enum { LBM_INIT_REST = 0, LBM_INIT_COUETTE = 1 } lbm_init;

/* How the momentum-exchange force enters the rigid-body update (Sec. 4.3
 * leaves the time integration open):
 *   LBM_COUPLING_IMPLICIT        the part linear in the particle surface
 *                                velocity taken at the new velocities
 *                                (solid-particle scheme of Nguyen and Ladd,
 *                                cited in Sec. 4.2), the velocity-free part
 *                                averaged over this and the previous step;
 *                                stable at density ratio 1 down to tau 0.55
 *   LBM_COUPLING_EXPLICIT        every term at the old velocities
 *   LBM_COUPLING_IMPLICIT_PLAIN  as IMPLICIT without the two-step average
 *                                (grows a period-two torque oscillation at
 *                                density ratio 1 for tau below about 0.7) */
typedef enum {
    LBM_COUPLING_IMPLICIT = 0,
    LBM_COUPLING_EXPLICIT = 1,
    LBM_COUPLING_IMPLICIT_PLAIN = 2
} lbm_coupling;

typedef struct lbm_ctx lbm_ctx;

typedef struct {
    int32_t nx, ny, nz;        /* lattice size; x and y are periodic */
    int32_t z_periodic;        /* 0: moving walls at the z ends; 1: periodic z */
    int32_t collision;         /* lbm_collision */
    double tau;                /* even relaxation time, > 0.5; omega_e = 1/tau */
    double magic;              /* TRT Lambda = (tau - 1/2)(1/omega_o - 1/2); 3/16 puts walls half-way */
    double wall_u;             /* wall speed U: top wall +U, bottom wall -U along x; |U| < 0.1 */
    double rho0;               /* mean density (> 0) */
    double body_force[3];      /* body-force acceleration (channel tests); 0 for shear cells */
    int32_t storage;           /* lbm_storage */
    int32_t init_profile;      /* lbm_init: rest, or the linear Couette profile */
    int32_t coupling;          /* lbm_coupling */
    int32_t fp16_scale_log2;   /* k for LBM_F16DEV (0..20) */
    int64_t history_capacity;  /* steps kept in the device history ring (>= 1) */
    void *stream;              /* hipStream_t to order work on; NULL: a private stream */
    int32_t sweep_grid;        /* workgroups of the bulk sweep (grid-stride); 0 = automatic */
    int32_t q_pad;             /* extra elements between direction arrays; -1 = automatic */
    int32_t stabilize;         /* 1: momentum stabilization (see lbm_get_mean_velocity); 0: off */
    int32_t z_free_slip;       /* 1: the z walls (z_periodic = 0, wall_u = 0) are free-slip
                                  (specular reflection, Eq. FreeSlipBC) instead of no-slip; 0 */
    /* Contact between fibers (0: off).  The paper's rigid-body engine resolves
     * frictional collisions of the particles (Sec. 4.4); this library applies
     * a short-range repulsion instead: each fiber is the segment of its axis
     * of half-length max(L/2 - r, 0) swept by its radius, and when the gap
     * between two of them is below contact_range a force
     * contact_stiffness ((contact_range - gap)/contact_range)^2 pushes them
     * apart along the line of their closest axis points, applied at the
     * middle of the gap and added to the external load of the step (lattice
     * units).  With contacts at most 248 fibers per context. */
    double contact_stiffness;
    double contact_range;
    /* Walls half-way outside the x faces (below x = 0 and above x = nx - 1)
     * instead of periodicity in x: 1 resting no-slip (bounce-back, Eq.
     * BBBC), 2 free-slip (specular reflection, Eq. FreeSlipBC: a population
     * leaving through the wall returns with its normal component reversed,
     * on the neighbour along the wall); 0 periodic.  Likewise y.  With z
     * walls this closes the box on all six faces (the paper's sedimentation
     * box: free-slip everywhere).  A link that crosses walls of both kinds
     * (an edge) bounces back.  Fibers must stay more than one cell from
     * these walls and from free-slip z walls (LBM_E_GEOM at lbm_add_fiber;
     * LBM_E_STATE at the next sync if one reaches a wall during the run). */
    int32_t x_walls;
    int32_t y_walls;
} lbm_params;

/* Fiber shapes: a circular cylinder of length L, or a spherocylinder (a
 * cylinder with hemispherical caps, L including the caps, so the
 * cylindrical part is L - 2r long; the particle shape of Sec. 2). */
typedef enum { LBM_SHAPE_CYLINDER = 0, LBM_SHAPE_SPHEROCYLINDER = 1 } lbm_shape;

/* A rigid fiber.  The axis is t = R(q) e_x for the unit quaternion
 * q = (w, x, y, z).  Cells whose centre lies inside belong to the fiber
 * (Sec. 4.2).  Mass m = density_ratio * rho0 * V; for the cylinder
 * V = pi r^2 L, I_par = m r^2 / 2, I_perp = m (3 r^2 + L^2) / 12; for the
 * spherocylinder with h = L - 2r, cylinder part m_c = m pi r^2 h / V and
 * caps m_s = m (4/3) pi r^3 / V: I_par = m_c r^2 / 2 + (2/5) m_s r^2,
 * I_perp = m_c (3 r^2 + h^2) / 12 + m_s (2 r^2 / 5 + h^2 / 4 + 3 h r / 8).
 * force and torque: a constant external load added to the hydrodynamic
 * force and torque in every step, e.g. the buoyancy-corrected weight
 * (rho_p - rho_f) g V of Eq. ForceDensDiff (lattice units).  The fields
 * from shape on were appended to the original layout; zero-filled they
 * give a cylinder without external load. */
typedef struct {
    double center[3];
    double quat[4];
    double length;
    double radius;
    double density_ratio;
    double vel[3];
    double omega[3];
    int32_t shape;             /* lbm_shape */
    int32_t reserved;          /* 0 */
    double force[3];
    double torque[3];
} lbm_fiber;

typedef struct {
    int64_t steps_done;
    int32_t nfibers;
    int32_t parity;            /* 0: populations in natural slots; 1: swapped (mid AA pair) */
    int64_t boundary_cells;    /* fluid cells next to a fiber (current list length) */
    int64_t overlap_events;    /* cells claimed by two fibers, summed over all remaps */
    int64_t device_bytes;      /* device memory held by the context */
    int64_t population_bytes;  /* bytes of the population array */
} lbm_info;

/* Fill *p with defaults: 32^3, walls, TRT, tau 0.8, Lambda 3/16, U 0,
 * rho0 1, F32, rest, implicit coupling, k = 14, history 4096, NULL stream,
 * automatic sweep grid and padding, no stabilization, no contacts (range 1). */
lbm_status lbm_params_default(lbm_params *p);

/* Allocate the lattice and initialise f = f_eq(rho0, u0(z)) (Eq.
 * fequ_Incompr) with u0 = 0 or the Couette profile
 * u0_x(z) = U (2 (z + 1/2)/nz - 1).  *out receives the context. */
lbm_status lbm_create(const lbm_params *p, lbm_ctx **out);

/* Free every buffer of the context (synchronises its stream first). */
lbm_status lbm_destroy(lbm_ctx *ctx);

/* Message of the last error on ctx (never NULL; "" after success). */
const char *lbm_last_error(const lbm_ctx *ctx);

/* D3Q19 velocity set in the order used by lbm_get_populations /
 * lbm_set_populations: c[19][3] and w[19].  Either pointer may be NULL. */
lbm_status lbm_lattice(int32_t *c, double *w);

/* Add a fiber before the first step (Sec. 4.2 mapping).  *id receives its
 * index (dense from 0).  LBM_E_GEOM if the fiber leaves the domain or comes
 * within one cell of a wall, or if it shares a cell with another fiber;
 * the fiber is then not added.  LBM_E_STATE after the first step.
 * LBM_E_ARG beyond 302 fibers per context (248 with contacts): the
 * rigid-body update of all fibers runs in one workgroup that keeps their
 * momentum-exchange sums (27 doubles per fiber) in 64 KiB of LDS.  Each
 * insertion re-maps the lattice, so setting up np fibers costs O(np^2). */
lbm_status lbm_add_fiber(lbm_ctx *ctx, const lbm_fiber *f, int32_t *id);

/* Prescribe the motion of fiber id for its next nsteps steps.  traj is a
 * host array [nsteps][13] = X[3] q[4] V[3] W[3]: row j is the state after
 * the j-th following step.  The force reported for those steps is the
 * momentum exchange of Eq. LBMhydrodynForce at the old velocity.  After
 * the last row the fiber moves freely again.  nsteps = 0 clears it. */
lbm_status lbm_set_fiber_kinematics(lbm_ctx *ctx, int32_t id, const double *traj,
                                    int64_t nsteps);

/* Enqueue n coupled time steps (n >= 0): AA-pattern fused stream-collide
 * with wall and particle bounce-back, momentum exchange, rigid-body update,
 * re-mapping with refill of uncovered cells (Sec. 4.2), rebuild of the
 * boundary-cell list.  Returns after enqueueing. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Wait for all enqueued work; report device-side errors: LBM_E_UNSTABLE
 * for a non-finite force or torque seen by a step, or a non-finite stored
 * population (one read pass over the population array, on the stream,
 * before waiting); LBM_E_STATE for exceeded internal capacities or a fiber
 * that reached an x or y wall. */
lbm_status lbm_sync(lbm_ctx *ctx);

/* Hydrodynamic force and torque of the last completed step, FP64 host
 * arrays [nfibers][3] (either may be NULL).  Torque about the centre of
 * mass.  For freely moving fibers with implicit coupling this is the
 * force that was applied in the rigid-body update. */
lbm_status lbm_get_force_torque(lbm_ctx *ctx, double *F, double *M);

/* Macroscopic fields of the current state, decoded from the AA layout.
 * rho [z][y][x] and u [3][z][y][x] are float (double for LBM_F64); in
 * fiber cells rho = rho0 and u = the rigid-body velocity there.  flags
 * [z][y][x]: 0 fluid, 1 fiber.  pid [z][y][x]: owning fiber or -1.  Any
 * pointer may be NULL.  dst_is_device != 0: the pointers are device
 * memory, filled on the stream; otherwise host memory. */
lbm_status lbm_get_fields(lbm_ctx *ctx, void *rho, void *u, uint8_t *flags, int32_t *pid,
                          int32_t dst_is_device);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * monitoring loops, harnesses that forbid allocation): lbm_get_fields with
 * host destinations (dst_is_device = 0) that calls no hipMalloc, hipFree or
 * other allocating routine.  The fields are decoded in chunks of cells into
 * a fixed 16 MiB device array held by the library (one per GPU, kept until
 * the process ends) and copied out chunk by chunk, so any lattice size is
 * accepted.  Arguments, layout and values are those of lbm_get_fields; the
 * call synchronises the context's stream.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (from several host threads)
 * race and must be serialised by the caller.  Errors: LBM_E_ARG for a NULL
 * context or a device index of 64 or more, LBM_E_HIP, and the device errors
 * of lbm_sync. */
lbm_status lbm_get_fields_static(lbm_ctx *ctx, void *rho, void *u, uint8_t *flags, int32_t *pid);

/* Fiber states, FP64 host arrays [nfibers][3] / [nfibers][4]. */
lbm_status lbm_get_fiber_state(lbm_ctx *ctx, double *X, double *q, double *V, double *W);

/* Replace the pose and velocities of fiber id between steps and re-map:
 * uncovered cells are refilled with f_eq(rho0, u_s) of the old motion. */
lbm_status lbm_set_fiber_state(lbm_ctx *ctx, int32_t id, const double X[3], const double q[4],
                               const double V[3], const double W[3]);

/* Per-step records [count][nfibers][19] = F3 M3 X3 q4 V3 W3 (state after
 * the step) for steps first .. first+count-1 (0-based).  Only the last
 * history_capacity steps are kept: LBM_E_ARG outside that window. */
lbm_status lbm_get_history(lbm_ctx *ctx, int64_t first, int64_t count, double *out);

/* Logical populations f_q(x) as FP64 host array [19][z][y][x] in the order
 * of lbm_lattice(), decoded from storage and parity.  Values in fiber cells
 * are unspecified. */
lbm_status lbm_get_populations(lbm_ctx *ctx, double *f);

/* Overwrite the logical populations (host FP64 [19][z][y][x]). */
lbm_status lbm_set_populations(lbm_ctx *ctx, const double *f);

/* Momentum stabilization (Sec. 4.1; lbm_params.stabilize = 1), for fully
 * periodic domains whose particles carry a constant external force: every
 * collision takes its equilibrium at u - ubar, ubar the mean velocity
 * sum_q c_q f_q / rho0 (+ g/2 with a body force) over all fluid cells of
 * the state the step starts from.  The mean is kept up to date by the step
 * kernels (no extra pass over the lattice); after a state change from the
 * host it is recomputed by one pass before the next step.  This call
 * synchronises and returns the mean the next step will subtract and the
 * number of fluid cells it was taken over (nfluid may be NULL).
 * LBM_E_STATE when the context was created without stabilization. */
lbm_status lbm_get_mean_velocity(lbm_ctx *ctx, double ubar[3], int64_t *nfluid);

lbm_status lbm_get_info(lbm_ctx *ctx, lbm_info *info);

/* The parameters ctx was created with. */
lbm_status lbm_get_params(lbm_ctx *ctx, lbm_params *out);

/* Checkpoint and resume (not part of the paper's method).  lbm_save
 * synchronises the stream and writes, to the file at path, the parameters,
 * the fibers (with any prescribed trajectories), every device buffer that
 * carries state between steps (populations in their AA layout, both flag
 * buffers, owners, boundary list, particle states and boxes, history ring,
 * stabilization sums, counters) and the step count.  lbm_load creates a
 * context from such a file on stream (a hipStream_t, or NULL for a private
 * one); its steps are bit-identical to those the saved context would have
 * taken.  An attached closure is not saved (attach it again).  Errors:
 * LBM_E_ARG for an unreadable, foreign or truncated file (lbm_load returns
 * no context then), LBM_E_NOMEM, LBM_E_HIP. */
lbm_status lbm_save(lbm_ctx *ctx, const char *path);
lbm_status lbm_load(const char *path, void *stream, lbm_ctx **out);

/* Device-event timing of the stream-collide sweep: when enabled, every
 * subsequent lbm_step brackets each sweep launch with HIP events on the
 * context's stream.  lbm_get_sweep_time synchronises and returns the total
 * milliseconds and the number of sweeps timed since enabling. */
lbm_status lbm_enable_sweep_timing(lbm_ctx *ctx, int32_t on);
lbm_status lbm_get_sweep_time(lbm_ctx *ctx, double *total_ms, int64_t *nsweeps);

/* Plain device copy (16 B per lane, grid-stride) of nbytes from src to dst,
 * both device pointers, enqueued on stream (hipStream_t or NULL): the
 * bandwidth reference against which the sweep's traffic counters are
 * calibrated. */
lbm_status lbm_copy_bytes(void *dst, const void *src, size_t nbytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
