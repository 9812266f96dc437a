/*
 * mlp.h -- C ABI of the surrogate network and two-stage unweighting in libme.so.
 *
 * The learned part of the build (not in the paper): a multilayer perceptron
 * that approximates the standardised logarithm of |M|^2 from the momenta,
 * trained on the GPU by the library's own BF16 forward and backward kernels
 * (matrix-core GEMMs with FP32 accumulation, FP32 master weights, Adam), and
 * used to drive a two-stage unweighting in which the exact matrix element is
 * the second stage, so the unweighted sample stays unbiased.
 *
 * Network: n_in inputs -> depth hidden layers of `width` units with SiLU ->
 * one output.  Flat FP32 parameter layout (host copies):
 *   [W_1 (width x n_in, row-major [out][in]), b_1, W_2 (width x width), b_2, ...,
 *    W_depth, b_depth, w_out (width), b_out]
 * Loss: mean squared error.  Adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8
 * and bias correction.
 *
 * Conventions as in me.h: status codes (ME_* from me.h), device pointers owned
 * by the caller, asynchronous on the given stream (NULL = default stream).
 *
 * None of this is in the paper (it has no learned component); the two-stage
 * scheme follows Danziger, Janssen, Schumann, Siegert, SciPost Phys. 12 (2022)
 * 164, and every call below cites that or the network's own definition.
 */
#ifndef MLP_H
#define MLP_H

#include <stdint.h>

#include "me.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct me_mlp me_mlp;

/*
 * mlp_create -- allocate a network on the current device and initialise it
 * (the surrogate of Danziger et al. 2022, here an MLP of the stated shape):
 * weights uniform in +-sqrt(6 / fan_in) (He-uniform), biases 0, from a
 * splitmix64 stream keyed by seed; Adam moments 0, step 0.
 * Constraints: 1 <= n_in <= 32, width a multiple of 64 (<= 1024), depth >= 1.
 * Errors: ME_EINVAL, ME_ENOMEM, ME_EDEVICE.
 */
int mlp_create(int n_in, int width, int depth, uint64_t seed, me_mlp **out);

/* mlp_n_params -- number of FP32 parameters. */
int mlp_n_params(const me_mlp *mlp, int64_t *n);

/* mlp_dims -- the network's input count, hidden width and depth (any output
 * pointer may be NULL). */
int mlp_dims(const me_mlp *mlp, int *n_in, int *width, int *depth);

/* mlp_get_params / mlp_set_params -- copy the FP32 master parameters to / from
 * a host array of n = mlp_n_params entries (flat layout above).  Both
 * synchronise the device; set also refreshes the BF16 working copy. */
int mlp_get_params(me_mlp *mlp, float *host, int64_t n);
int mlp_set_params(me_mlp *mlp, const float *host, int64_t n);

/*
 * mlp_forward -- y[i] = network(x[i]) for i < n (the surrogate's estimate of
 * the standardised log |M|^2, the first stage of Danziger et al. 2022).
 * x: device float32 [n][n_in]; y: device float32 [n].  BF16 operands, FP32
 * accumulation, FP32 bias and activation.  Works in chunks; any n >= 0.
 */
int mlp_forward(me_mlp *mlp, const float *x, int64_t n, float *y, void *stream);

/*
 * mlp_train_step -- one Adam step (Kingma, Ba 2015) on the mini-batch
 * {x[idx[j]], t[idx[j]]},
 * j < n (idx == NULL: the first n rows).
 * x: device float32 [*][n_in]; t: device float32 targets; idx: device int32 [n].
 * n: batch size, a positive multiple of 64.  lr: learning rate of this step.
 * loss_dev: device float32 [1] (may be NULL), receives the batch mean squared
 * error before the update.
 */
int mlp_train_step(me_mlp *mlp, const float *x, const float *t, const int32_t *idx, int64_t n, float lr,
                   float *loss_dev, void *stream);

/*
 * mlp_train_steps -- nsteps consecutive Adam steps as above, step st on the
 * mini-batch {x[idx[st n + j]], t[idx[st n + j]]}, j < n (idx == NULL: rows
 * st n .. st n + n - 1), with learning rate lr_dev[st].
 * idx: device int32 [nsteps n] or NULL; lr_dev: device float32 [nsteps];
 * loss_dev: device float32 [nsteps] (may be NULL), the mean squared error of
 * each step's batch before its update.  Where the one-kernel step applies
 * (see mlp_set_fused_step) all steps run in one cooperative launch, with
 * grid-wide barriers between them; otherwise the steps run one by one after a
 * synchronising read of lr_dev.  The steps are those of nsteps calls of
 * mlp_train_step, except that the bias corrections 1 - beta^t are computed on
 * the device.  Calls on one network must be ordered (one stream): they share
 * its batch buffers.
 */
int mlp_train_steps(me_mlp *mlp, const float *x, const float *t, const int32_t *idx, int64_t n, int64_t nsteps,
                    const float *lr_dev, float *loss_dev, void *stream);

/*
 * mlp_backward -- gradient of the batch loss only (no update), for checks
 * (backpropagation through the network defined above).
 * grad_dev: device float32 [n_params] (flat layout); loss_dev as above.
 */
int mlp_backward(me_mlp *mlp, const float *x, const float *t, const int32_t *idx, int64_t n, float *grad_dev,
                 float *loss_dev, void *stream);

/*
 * mlp_set_fused_step -- choose how mlp_train_step and mlp_backward run.
 * on != 0 (default where it applies): one cooperative kernel per step (width
 * 256, depth <= 4, n_in <= 32, batch a multiple of 128): rows go through the
 * whole forward and backward chain without leaving the block, and the batch
 * sums of the weight gradients and the Adam update follow after grid-wide
 * barriers.  on == 0: the layered GEMM kernels.  Both give the same gradients
 * up to the order of the FP32 sums.  Errors: ME_ESTATE (shape not supported
 * by the fused kernel).
 */
int mlp_set_fused_step(me_mlp *mlp, int on);

int mlp_free(me_mlp *mlp);

/*
 * me_features -- network inputs from momenta: x[i][4 p + c] = momenta[i][p][c]
 * / sqrt(s_i) as float32, with s_i = (p_0 + p_1)^2 of the incoming partons
 * (the points are taken in the partonic centre-of-mass frame).
 * momenta: device float64 [n][npart][4]; x: device float32 [n][4 npart].
 */
int me_features(const double *momenta, int64_t n, int npart, float *x, void *stream);

/*
 * unweight_two_stage -- two-stage unweighting of n points (Danziger, Janssen,
 * Schumann, Siegert 2022).  For point i with phase-space weight w_ps[i]:
 *   surrogate weight  s_i = exp(y_sigma * y_i + y_mu) * w_ps[i]   (y from the network),
 *   stage 1: accept if u[i][0] < min(1, s_i / s_max);
 *   exact weight w_i = |M|^2_i * w_ps[i] (me_eval of ctx, float64) for stage-1
 *   survivors only;
 *   stage 2: accept if u[i][1] < min(1, (w_i / s_i) / r_max);
 *   output weight max(1, s_i/s_max) * max(1, (w_i/s_i)/r_max).
 * momenta: device float64 [n][npart][4]; w_ps: device float64 [n];
 * uniforms: device float64 [n][2] in (0,1).
 * out_idx: device int32 [n], indices of accepted points in increasing order of
 * stage-1 survival (order not guaranteed); out_w: device float64 [n], their
 * weights; out_count: device int32 [2] = {stage-1 survivors (= exact
 * evaluations), accepted}.  Scratch grows on the first call with a larger n
 * (synchronises the device).  Errors: ME_EINVAL, ME_EDEVICE, ME_ENOMEM.
 */
int unweight_two_stage(me_ctx *ctx, me_mlp *mlp, const double *momenta, const double *w_ps, int64_t n,
                       const double *uniforms, double y_mu, double y_sigma, double s_max, double r_max,
                       int32_t *out_idx, double *out_w, int32_t *out_count, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MLP_H */
