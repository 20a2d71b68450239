/*
 * sbf.h -- C ABI of the slender-body formulation (SBF) of Bartuschat,
 * Fischermeier, Gustavsson and Ruede, "Two computational models for
 * simulating the tumbling motion of elongated particles in fluids"
 * (Computers & Fluids, 2015), Sec. 3, on one MI355X (gfx950).
 *
 * M straight fibers of length L = 2l and slenderness eps = r/L in an
 * unbounded Stokes fluid of viscosity mu.  Fiber m has centre x_m, unit
 * direction p_m, and carries a constant external force F_m and torque M_m
 * (the torque's component along p_m has no effect on a slender body).  The
 * force per unit length is expanded in Legendre polynomials (Eq.
 * force_exp) f_m(s) = F_m/(2l) + sum_{n=1..N} a_m^n P_n(s/l); projecting
 * the non-local slender-body equation (Eq. sev_fils, with the finite-part
 * operator of Eq. Kbar and the free-space Green's function of Eq. Gnonper)
 * on P_1..P_N together with the force and torque balance (Eq. extra_cond)
 * gives a dense linear system for the 3MN coefficients, solved by GMRES;
 * the velocities follow from Eqs. xadot and padot:
 *   dx_m/dt = [Lambda_m F_m + int U_m ds] / (8 pi mu L),
 *   dp_m/dt = 3/(2 pi mu L^3) [d M_m x p_m + (I - p_m p_m^T) int s U_m ds],
 * Lambda = d (I + p p^T) + 2 (I - p p^T), d = -ln(eps^2 e) (Eq.
 * SBFGeomParam), U_m the velocity (times 8 pi mu) induced by the other
 * fibers.  The interaction integrals are taken with a composite three-point
 * Gauss rule on nq sub-intervals of each fiber (3 nq points per fiber; the
 * paper uses 48); time integration is Adams-Bashforth of second order (the
 * paper asks only for an explicit method of second order with constant dt),
 * started with one Euler step, with p renormalised after every step.
 *
 * Conventions: every call returns lbm_status (include/lbm.h); the context
 * is not thread-safe; work is ordered on its HIP stream; host arrays are
 * FP64 [m][3] in the caller's memory.  sbf_solve waits once per GMRES
 * iteration for the previous iteration's residual (the convergence test)
 * while the next iteration runs, so it may take one iteration more than
 * the tolerance needs.
 */
#ifndef SBF_H
#define SBF_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbf_ctx sbf_ctx;

typedef struct {
    int32_t max_fibers;     /* capacity M (>= 1) */
    int32_t nmodes;         /* N, Legendre modes of the force expansion (1..8) */
    int32_t nq;             /* sub-intervals of the Gauss rule per fiber (1..64) */
    int32_t gmres_restart;  /* Krylov dimension before a restart (1..63) */
    int32_t gmres_maxit;    /* iterations per solve, over all restarts (>= 1) */
    int32_t reserved;       /* 0 */
    double length;          /* L (> 0) */
    double eps;             /* r / L, 0 < eps < 1/2 */
    double mu;              /* dynamic viscosity (> 0) */
    double gmres_tol;       /* relative residual at which GMRES stops (> 0) */
    void *stream;           /* hipStream_t; NULL: a private stream */
} sbf_params;

/* Defaults: 64 fibers, N = 5, nq = 16 (48 points, as in the paper),
 * restart 30, 200 iterations, L = 1, eps = 0.1, mu = 1, tolerance 1e-12. */
lbm_status sbf_params_default(sbf_params *p);

/* Allocate a context for up to max_fibers fibers: the moment matrix (it
 * is symmetric; its upper triangle of 64 x 64 tiles, about
 * (3 M (N + 1))^2 / 2 doubles) and the GMRES basis.  LBM_E_ARG for invalid
 * parameters (including nq and N whose moment workgroup would need more
 * than 64 KiB of LDS: 8 (N + 1)(21 nq + 7 (N + 1)) bytes), LBM_E_NOMEM
 * when the device memory does not suffice. */
lbm_status sbf_create(const sbf_params *p, sbf_ctx **out);
lbm_status sbf_destroy(sbf_ctx *ctx);
const char *sbf_last_error(const sbf_ctx *ctx);

/* Set the configuration: m fibers (1 <= m <= max_fibers), host arrays
 * X[m][3] centres, p[m][3] directions (normalised here; LBM_E_ARG for a
 * zero vector), F[m][3] external forces, M[m][3] external torques (F or M
 * may be NULL: zero).  Resets the time stepping (the next step is an Euler
 * step) and the GMRES start vector. */
lbm_status sbf_set_fibers(sbf_ctx *ctx, int32_t m, const double *X, const double *p, const double *F,
                          const double *M);

/* Velocities of the current configuration (Sec. 3.1: moments of the
 * Green's function, GMRES for the Legendre coefficients, Eqs. xadot,
 * padot).  GMRES starts from the previous solution.  LBM_E_UNSTABLE if it
 * does not reach the tolerance within gmres_maxit iterations (the
 * velocities of the last iterate are kept). */
lbm_status sbf_solve(sbf_ctx *ctx);

/* Results of the last solve (host arrays; any pointer may be NULL):
 * dx/dt [m][3], dp/dt [m][3], coefficients a [m][N][3] (n = 1..N). */
lbm_status sbf_get_velocities(sbf_ctx *ctx, double *V, double *pdot);
lbm_status sbf_get_coefficients(sbf_ctx *ctx, double *a);

/* n time steps of size dt > 0: solve, then Adams-Bashforth 2
 * x += dt (3/2 v_n - 1/2 v_{n-1}) (Euler for the first step after
 * sbf_set_fibers), p likewise and renormalised.  From the third step on,
 * GMRES starts from the linear extrapolation of the two previous steps'
 * coefficients. */
lbm_status sbf_step(sbf_ctx *ctx, int64_t n, double dt);

/* Current centres and directions, host [m][3] each (either may be NULL). */
lbm_status sbf_get_state(sbf_ctx *ctx, double *X, double *p);

/* Iterations and relative residual of the last solve; steps done. */
lbm_status sbf_get_stats(sbf_ctx *ctx, int32_t *iterations, double *residual, int64_t *steps);

/* Device-event timing of the following solves (on != 0; 0 stops it):
 * sbf_get_timing returns the totals since enabling -- milliseconds and
 * launches of the moment kernel and of the products with the moment matrix
 * (any pointer may be NULL). */
lbm_status sbf_enable_timing(sbf_ctx *ctx, int32_t on);
lbm_status sbf_get_timing(sbf_ctx *ctx, double *moments_ms, int64_t *moments_launches, double *gemv_ms,
                          int64_t *gemv_launches);

#ifdef __cplusplus
}
#endif
#endif
