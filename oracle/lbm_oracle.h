/*
 * lbm_oracle.h -- plain FP64 CPU oracle for the coupled D3Q19 lattice
 * Boltzmann / momentum-exchange / rigid-fiber method of Bartuschat,
 * Fischermeier, Gustavsson and Ruede, "Two computational models for
 * simulating the tumbling motion of elongated particles in fluids" (2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists so that the GPU library can
 * be checked against an obviously correct implementation.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no source with the GPU library: its own lattice tables,
 * its own equilibrium, its own mapping predicate and its own integrator.
 *
 * Storage: two lattices A and B (double, layout f[q][z][y][x]), push
 * streaming A -> B, then swap.  Lattice units throughout (dx = dt = 1,
 * c_s^2 = 1/3).  Cell centres sit at integer coordinates.
 *
 * Step order (the paper only outlines the coupling in Sec. 4.3):
 *   1. TRT/SRT collision of every fluid cell          (Sec. 4.1, Eq. LBMCollide)
 *   2. streaming with half-way bounce-back at moving walls and at moving
 *      particle surfaces, plus the momentum-exchange force and torque
 *                                                      (Eqs. LBMStream, BBBC,
 *                                                       LBMMovWall,
 *                                                       LBMhydrodynForce)
 *   3. rigid-body update of every fiber                (Sec. 4.3)
 *   4. re-mapping of cells and refill of uncovered cells (Sec. 4.2)
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_sim or_sim;

typedef struct {
    int nx, ny, nz;
    int z_periodic;    /* 1: periodic in z; 0: moving walls half-way below z=0 and above z=nz-1 */
    int srt;           /* 1: single relaxation time (omega_o = omega_e); 0: TRT */
    double tau;        /* relaxation time of the even moments, omega_e = 1/tau */
    double magic;      /* TRT parameter Lambda = (1/omega_e - 1/2)(1/omega_o - 1/2) */
    double rho0;       /* mean density */
    double wall_u;     /* wall velocity along x: top wall +U, bottom wall -U */
    double g[3];       /* body-force acceleration (Poiseuille / drag tests only) */
    int init_couette;  /* 1: start from the linear Couette profile; 0: fluid at rest */
    int coupling;      /* how the momentum-exchange force enters the rigid-body update:
                          0: the part linear in the surface velocity at the new particle
                             velocity (solid-particle scheme of Nguyen and Ladd), the
                             velocity-free part averaged over this and the previous step;
                          1: fully explicit, every term at the old velocity;
                          2: as 0 without the two-step average */
    int stabilize;     /* 1: momentum stabilization (Sec. 4.1, periodic domains under a
                          constant particle force): the mean velocity of all fluid cells
                          is subtracted from the velocity of every cell's equilibrium */
    double contact_k;     /* > 0: short-range repulsion between fibers (contact model in place
                             of the paper's frictional collision handling); 0: off */
    double contact_range; /* surface gap below which the repulsion acts */
    int x_walls;          /* walls half-way below x = 0 and above x = nx - 1 instead of
                             periodicity in x: 1 stationary no-slip (Eq. BBBC), 2 free-slip
                             (specular reflection, Eq. FreeSlipBC); 0: periodic in x */
    int y_walls;          /* the same for y */
    int z_free_slip;      /* 1 (with z_periodic = 0 and wall_u = 0): the z walls reflect
                             specularly instead of bouncing back */
} or_params;

/* ---- building blocks (exposed so the tests can pin them one by one) ---- */
void   or_lattice(int32_t *c /*[19*3]*/, double *w /*[19]*/, int32_t *opp /*[19]*/);
void   or_feq(double rho, double rho0, const double u[3], double *feq /*[19]*/);
double or_omega_odd(double tau, double magic, int srt);
void   or_collide_cell(const double *f, double rho0, double omega_e, double omega_o,
                       const double g[3], double *fpost);
/* as or_collide_cell, with the equilibrium taken at the velocity u - ubar */
void   or_collide_cell_shift(const double *f, double rho0, double omega_e, double omega_o,
                             const double g[3], const double ubar[3], double *fpost);
void   or_fiber_axis(const double q[4], double t[3]);
int    or_cell_inside(const double c[3], const double X[3], const double t[3],
                      double length, double radius, int nx, int ny, int nz, int zper);
/* shape 0: cylinder; 1: spherocylinder (length including the caps) */
int    or_cell_inside_shape(const double c[3], const double X[3], const double t[3], double length,
                            double radius, int shape, int nx, int ny, int nz, int zper);
void   or_map(int nx, int ny, int nz, int zper, int np, const double *X, const double *q,
              const double *length, const double *radius, int32_t *pid, int64_t *overlaps);
void   or_map_shapes(int nx, int ny, int nz, int zper, int np, const double *X, const double *q,
                     const double *length, const double *radius, const int32_t *shape,
                     int32_t *pid, int64_t *overlaps);
/* mass, axial and transverse moment of inertia of a homogeneous cylinder
   (shape 0) or spherocylinder (shape 1) of density rho */
void   or_body_inertia(int shape, double length, double radius, double rho, double out[3]);
/* one semi-implicit Euler step; state = X[3] q[4] V[3] W[3] Lang[3] */
void   or_rigid_step(const double *state, double mass, double i_par, double i_perp,
                     const double F[3], const double M[3], int nx, int ny, int nz, int zper,
                     double *state_out);

/* implicit variant: F = F0 - A V' - B W', M = M0 - B^T V' - C W' with the
   new velocities V', W'; A, C symmetric 3x3 (row-major 9 each), B 3x3.
   Writes the new state and the force/torque actually applied. */
void   or_rigid_step_implicit(const double *state, double mass, double i_par, double i_perp,
                              const double F0[3], const double M0[3], const double *A,
                              const double *B, const double *Cm, int nx, int ny, int nz,
                              int zper, double *state_out, double *F_applied,
                              double *M_applied);

/* ---- the coupled simulation ---- */
or_sim *or_create(const or_params *p);
void    or_destroy(or_sim *s);
int     or_add_fiber(or_sim *s, const double X[3], const double q[4], double length,
                     double radius, double density_ratio, const double V[3], const double W[3]);
/* with a shape (0 cylinder, 1 spherocylinder) and a constant external force
   Fext and torque Mext added to the hydrodynamic ones in every step */
int     or_add_fiber_ex(or_sim *s, const double X[3], const double q[4], double length,
                        double radius, double density_ratio, const double V[3], const double W[3],
                        int shape, const double Fext[3], const double Mext[3]);
int     or_set_kinematics(or_sim *s, int id, const double *traj /*[nsteps][13]*/, int64_t nsteps);
/* add dF, dM to fiber id's momentum-exchange force and torque in the next
   step only (to the velocity-free part for the implicit couplings) */
int     or_set_correction(or_sim *s, int id, const double dF[3], const double dM[3]);
void    or_step(or_sim *s, int64_t n);
void    or_get_populations(const or_sim *s, double *f /*[19][nz][ny][nx]*/);
void    or_set_populations(or_sim *s, const double *f);
void    or_get_fields(const or_sim *s, double *rho, double *u /*[3][nz][ny][nx]*/,
                      uint8_t *flags, int32_t *pid);
void    or_get_fiber_state(const or_sim *s, double *X, double *q, double *V, double *W);
void    or_get_force_torque(const or_sim *s, double *F, double *M);
int64_t or_get_history(const or_sim *s, int64_t first, int64_t count, double *out);
int64_t or_overlaps(const or_sim *s);
/* momentum-exchange sums of the last step per fiber, [nf][39]: the direct
   force F3 and torque M3 of Eq. LBMhydrodynForce (every term at the velocity
   of the state the step started from), then the split used by the implicit
   couplings: velocity-free part F0 3, M0 3 and the row-major 3x3 matrices
   A, B, C of the part linear in u_s = V + W x r, so that the direct sums are
   F0 - A V - B W and M0 - B^T V - C W */
void    or_get_exchange_sums(const or_sim *s, double *out);
/* test hook: plant a known mistake (1: B instead of B^T in the torque row of
   the implicit solve; 2: -C instead of C there; 3: B accumulated transposed;
   4: the two-step mean without its factor 1/2; 5: the odd part relaxed with
   omega_e; 6: 3 instead of 9/2 for (c.u)^2 in f_eq; 7: the collision's even
   equilibrium without its (c.u)^2 term; 8: the moving-wall term with the
   wrong sign; 9: fiber bounce-back without the surface velocity; 10: the
   link force without its factor 2; 11: the torque as dF x r; 12: free-slip
   walls bouncing back; 13: the refill at the new pose and motion; 14: the
   stabilization shift added; 15: resting side walls returning the
   population in its own direction; 16: the cylinder's axial bound at L
   instead of L/2; 17: the axis of the conjugate quaternion; 18: the highest
   id keeping a cell claimed twice; 19: the spherocylinder's caps centred
   at the cylinder's ends; 20: the explicit rigid step moving with the old
   velocity; 21: I_par and I_perp swapped; 22: an attractive contact force;
   23: the contact torque on q taken about the centre of p; 24: no minimum
   image across periodic faces; 25: the mean velocity counting solid cells;
   26: the spherocylinder caps' inertia without the parallel-axis shift;
   27: the external force dropped; 28: the external torque dropped); 0
   restores the oracle, whose results are
   then bit-identical to a build without the hook */
void    or_set_mutation(int code);
/* OpenMP threads of the following steps (timing on one core or all), and
   the current count */
void    or_set_threads(int n);
int     or_get_threads(void);
/* closest points of two axis segments X + s t, |s| <= h (t unit): returns the distance and
   the parameters s (first segment) and u (second); parallel axes: middle of the overlap */
double or_segment_closest(const double Xp[3], const double tp[3], double hp, const double Xq[3],
                          const double tq[3], double hq, double *s, double *u);
/* contact force and torque of fibers p and q (rounded ends: axis segments of half-length
   L/2 - r, radius r), torques about their centres; dpq = minimum-image X_q - X_p;
   returns the surface gap */
double or_contact_pair(const double tp[3], double hp, double rp,
                       const double dpq[3], const double tq[3], double hq, double rq, double k,
                       double range, double Fp[3], double Mp[3], double Fq[3], double Mq[3]);
/* mean velocity u = sum_q c_q f_q / rho0 + g/2 over the fluid cells of the current state
   (the quantity the momentum stabilization subtracts); returns the fluid cell count */
int64_t or_mean_velocity(const or_sim *s, double ubar[3]);
int64_t or_steps_done(const or_sim *s);
int     or_nfibers(const or_sim *s);

#ifdef __cplusplus
}
#endif
#endif
