/*
 * lbm_mlp.h -- C ABI of the learned force/torque closure for under-resolved
 * fibers on a coarse lattice.
 *
 * The paper resolves every fiber (Sec. 4.2: cells whose centre lies inside a
 * particle are obstacle cells, forces from the momentum exchange).  On a
 * lattice too coarse for a fiber's diameter that force is biased; this
 * extension adds a correction dF, dM predicted by a small network from the
 * flow around the fiber, trained on pairs of resolved (fine) and coarse runs
 * of the same motion, and falls back to the plain resolved method where the
 * flow lies outside what it was trained on.
 *
 * Network: 247 -> 64 -> 64 -> 6, GELU (exact, erf form) after the two hidden
 * layers, BF16 weights, FP32 activations and accumulation.  Parameters in
 * one vector of LBM_MLP_NPARAM floats: W1[64][247], b1[64], W2[64][64],
 * b2[64], W3[6][64], b3[6].  The kernels use the BF16 copy (round to
 * nearest even of the FP32 master); Adam updates the FP32 master and
 * re-rounds.
 *
 * Features of a fiber (LBM_MLP_IN = 247), in the fiber's body frame R(q)
 * (columns: the axis t = R(q) e_x, R(q) e_y, R(q) e_z): at the points
 * P_k + R(q) o with P0 = X, P1 = X + (L/2) t, P2 = X - (L/2) t and o in
 * {-2, 0, 2}^3 (index m = (iz*3 + iy)*3 + ix, i in {0,1,2} for -2, 0, 2), the
 * fluid velocity (trilinear in the cell-centre velocities; fiber cells
 * contribute the rigid-body velocity; x, y periodic, z clamped to
 * [0, nz-1]) minus the rigid-body velocity V + W x (P_k + R(q) o - X),
 * rotated by R(q)^T and divided by gamma L, with gamma = 2 U / nz the shear
 * rate of the cell: feature (k*27 + m)*3 + c.  Then the orientation
 * quaternion (w, x, y, z) with w >= 0.
 *
 * Outputs (body frame): y[0..2] = R^T dF / (rho0 nu gamma L^2), y[3..5] =
 * R^T dM / (rho0 nu gamma L^3), nu = (tau - 1/2)/3, after multiplication by
 * out_scale.  The inputs are normalised as (x - in_mean) * in_inv_std
 * before the first layer.  Fallback: a fiber with any raw feature outside
 * [env_min, env_max] gets no correction (counted).
 *
 * All x / t / y pointers of the lbm_mlp_* compute calls are device memory;
 * the MLP's work is ordered on its stream.
 */
#ifndef LBM_MLP_H
#define LBM_MLP_H

#include "lbm.h"
#include "lbm_batch.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_IN 247
#define LBM_MLP_HIDDEN 64
#define LBM_MLP_OUT 6
#define LBM_MLP_NPARAM 20422

typedef struct lbm_mlp lbm_mlp;

/* Create a network; weights uniform in +-sqrt(6 / fan_in) (last layer scaled
 * by 0.1), biases 0, from the splitmix64 sequence started at seed.
 * Normalisation: mean 0, inverse std 1, out_scale 1, envelope unbounded. */
lbm_status lbm_mlp_create(uint64_t seed, void *stream, lbm_mlp **out);
lbm_status lbm_mlp_destroy(lbm_mlp *m);
const char *lbm_mlp_last_error(const lbm_mlp *m);

/* FP32 master parameters (host [LBM_MLP_NPARAM]); the BF16 copy is rounded
 * from them.  get: either pointer may be NULL. */
lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *w);
lbm_status lbm_mlp_get_params(lbm_mlp *m, float *w_master, uint16_t *w_bf16);

/* Host arrays: in_mean, in_inv_std, env_min, env_max [LBM_MLP_IN];
 * out_scale [LBM_MLP_OUT].  Any may be NULL (left unchanged). */
lbm_status lbm_mlp_set_norm(lbm_mlp *m, const float *in_mean, const float *in_inv_std,
                            const float *out_scale, const float *env_min, const float *env_max);

/* y[n][6] = out_scale * net((x - in_mean) * in_inv_std) for raw features
 * x[n][247] (device). */
lbm_status lbm_mlp_forward(lbm_mlp *m, const float *x, int32_t n, float *y);

/* Mean squared error between the raw network outputs and t[n][6] (device,
 * network units), *loss (host), and its gradient with respect to the
 * parameters (kept for lbm_mlp_adam; copied to grad[LBM_MLP_NPARAM] on the
 * host when grad is not NULL).  The sum over samples is taken in a fixed
 * order: the result does not depend on timing. */
lbm_status lbm_mlp_loss_grad(lbm_mlp *m, const float *x, const float *t, int32_t n, double *loss,
                             float *grad);

/* One Adam step (Kingma and Ba) on the FP32 master with the last gradient;
 * step counter kept by the network; BF16 copy re-rounded. */
lbm_status lbm_mlp_adam(lbm_mlp *m, float lr, float beta1, float beta2, float eps);

/* Minibatch training: epochs passes over x[n][247], t[n][6] (device) in a
 * splitmix64-shuffled order, batch samples per step, Adam (0.9, 0.999,
 * 1e-8) with learning rate lr.  loss_per_epoch (host [epochs], may be
 * NULL): mean of the minibatch losses of each epoch. */
lbm_status lbm_mlp_train(lbm_mlp *m, const float *x, const float *t, int32_t n, int32_t epochs,
                         int32_t batch, float lr, uint64_t shuffle_seed, double *loss_per_epoch);

/* Attach a trained network to a context (NULL detaches).  Every following
 * step samples the features of each fiber from the populations at the start
 * of the step, evaluates the network and adds dF, dM to the momentum-
 * exchange force and torque before the rigid-body update (to the
 * velocity-free part for implicit coupling).  The context does not own the
 * network; it must stay alive while attached.  LBM_E_ARG when the context
 * has no moving walls (gamma = 0). */
lbm_status lbm_set_closure(lbm_ctx *ctx, lbm_mlp *m);
/* Fibers corrected and fibers that fell back, summed over the steps. */
lbm_status lbm_get_closure_stats(lbm_ctx *ctx, int64_t *applied, int64_t *fallbacks);

/* Features of every fiber at the current state, [nfibers][247] floats,
 * host or device destination. */
lbm_status lbm_sample_features(lbm_ctx *ctx, float *out, int32_t dst_is_device);
/* The same for every case of a batch, [ncases][247]. */
lbm_status lbm_batch_sample_features(lbm_batch *b, float *out, int32_t dst_is_device);

#ifdef __cplusplus
}
#endif
#endif
