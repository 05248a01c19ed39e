/*
 * erf_mlp.h -- learned subgrid closure of liberf.so: a fully connected
 * 10 -> 64 -> 64 -> 64 -> 9 network with ReLU hidden layers that maps the
 * resolved velocity-gradient tensor and dtheta/dz at a cell centre to the
 * kinematic subgrid stresses and heat fluxes, in place of the Smagorinsky
 * closure of Sec. 2.3 (eq. stresstensor).  The paper names learned surrogate
 * models only as future work (Sec. 6); network shape, inputs, fallback rule and
 * training recipe are this library's.
 *
 * Network
 *   inputs  x = (du/dx, du/dy, du/dz, dv/dx, dv/dy, dv/dz, dw/dx, dw/dy, dw/dz,
 *           dtheta/dz), standardised (x - mean_x) / std_x; diagonal terms across
 *           the cell, off-diagonal terms as means of the four edge differences
 *           around the centre (zero on lid edges), dtheta/dz as the mean of the
 *           two face differences (zero through the lids)
 *   outputs y, standardised; tau = y std_y + mean_y gives
 *           (tau_11, tau_22, tau_33, tau_12, tau_13, tau_23, q_1, q_2, q_3)
 *   parameters, float[ERF_MLP_NPARAMS], flat: W1[10][64], b1[64], W2[64][64],
 *           b2[64], W3[64][64], b3[64], W4[64][9], b4[9] (row = input unit)
 *   norm, double[ERF_MLP_NNORM]: mean_x[10], std_x[10], mean_y[9], std_y[9]
 * Arithmetic: every matrix product takes BF16 operands (round to nearest
 * even) and accumulates in FP32 on the matrix cores; inputs, the closure
 * stresses, the fallback test and the divergence are FP64.
 *
 * Closure in the slow right-hand side (erf_params.sgs = ERF_SGS_MLP): the
 * stresses rho tau and heat fluxes rho q are formed at centres and act through
 * 4-cell means on edges and 2-cell means on faces, with tau_13, tau_23 and the
 * vertical heat flux zero on the lids.  A cell falls back to the Smagorinsky
 * values (Cs, Pr_t of the context) when an output is not finite or when its
 * energy transfer -tau:S is below minus twice the Smagorinsky dissipation.
 *
 * Pointers: "host" arguments are read or written before the call returns;
 * "device" arguments are device memory owned by the caller.  Calls enqueue on
 * the context's stream; those that return host values wait for it.
 */
#ifndef ERF_MLP_H
#define ERF_MLP_H

#include "erf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ERF_MLP_NPARAMS 9609
#define ERF_MLP_NNORM 38
#define ERF_MLP_NIN 10
#define ERF_MLP_NOUT 9

/* Set the parameters (host float[ERF_MLP_NPARAMS]) and statistics (host
 * double[ERF_MLP_NNORM]; NULL keeps the current ones, zero means and unit
 * deviations at first), pack them for the matrix cores and reset the Adam
 * state.  Allocates the closure state on first use (ERF_E_NOMEM). */
erf_status erf_mlp_set_weights(erf_ctx *ctx, const float *params, const double *norm);
/* Copy the current parameters and statistics to host arrays (either may be
 * NULL).  Synchronous.  ERF_E_STATE before any erf_mlp_set_weights. */
erf_status erf_mlp_get_weights(erf_ctx *ctx, float *params, double *norm);

/* The network alone on n standardised samples: x device float[n][10] ->
 * y device float[n][9] (standardised outputs). */
erf_status erf_mlp_forward(erf_ctx *ctx, const float *x, int64_t n, float *y);

/* The closure inputs of every cell of state S (raw, not standardised):
 * feat device double[nz*ny*nx][10], cell order x fastest. */
erf_status erf_mlp_features(erf_ctx *ctx, const erf_state *S, double *feat);

/* Box filter of the state S by an integer factor r (nx, ny, nz divisible by
 * r): coarse device arrays (double, full values; rhoq unused) rho and
 * rhotheta as block means, rhou / rhov / rhow as means over the r x r fine faces
 * on each coarse face; targets device double[nc][9] = block covariances of the
 * cell-centre velocities and theta, tau_ij = <u_i u_j> - <u_i><u_j>,
 * q_j = <u_j theta> - <u_j><theta>, plus with Cs > 0 the block mean of the fine
 * grid's own Smagorinsky stresses (Prandtl number Pr_t). */
erf_status erf_box_filter(erf_ctx *ctx, const erf_state *S, int32_t r, double Cs, double Pr_t,
                          erf_state *coarse, double *targets);

/* Statistics of a training set: feat device double[n][10], targets device
 * double[n][9] -> the context's norm (means and population standard
 * deviations, FP64, fixed summation order; a constant column gets deviation
 * 1).  Synchronous. */
erf_status erf_mlp_fit_norm(erf_ctx *ctx, const double *feat, const double *targets, int64_t n);
/* Standardise with the context's norm: x device float[n][10], and t device
 * float[n][9] when targets and t are both non-NULL. */
erf_status erf_mlp_standardize(erf_ctx *ctx, const double *feat, const double *targets, int64_t n,
                               float *x, float *t);

/* Mean-squared error over n samples and 9 outputs of the standardised targets t
 * (device float[n][9]) and its gradient with respect to the parameters (device
 * float[ERF_MLP_NPARAMS]); loss (host, may be NULL) makes the call
 * synchronous. */
erf_status erf_mlp_loss_grad(erf_ctx *ctx, const float *x, const float *t, int64_t n, float *grad,
                             double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the FP32
 * master parameters with the gradient of erf_mlp_loss_grad, then repacking;
 * loss as above.  Training buffers grow on demand (ERF_E_NOMEM). */
erf_status erf_mlp_train_step(erf_ctx *ctx, const float *x, const float *t, int64_t n, double lr,
                              double *loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * erf_mlp_loss_grad without any allocation and without waiting.  The training
 * activations and partial sums live in one fixed scratch array per GPU (about
 * 12 MB, held until the process ends) instead of buffers grown on demand; the
 * kernels and the results are those of erf_mlp_loss_grad, bit for bit.
 * n <= ERF_MLP_NOALLOC_MAX_BATCH (ERF_E_ARG beyond).  loss_dev (device double,
 * may be NULL) receives the loss; the call is asynchronous on the context's
 * stream.  The weights must be set (erf_mlp_set_weights, ERF_E_STATE
 * otherwise).  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (two streams, two threads, two contexts) race and must be
 * serialised by the caller; nothing in the scratch needs clearing between
 * calls. */
#define ERF_MLP_NOALLOC_MAX_BATCH 8192
erf_status erf_mlp_loss_grad_noalloc(erf_ctx *ctx, const float *x, const float *t, int64_t n, float *grad,
                                     double *loss_dev);

/* Number of cells that fell back to Smagorinsky since the closure state was
 * allocated (cumulative over calls).  Synchronous. */
erf_status erf_mlp_fallback_count(erf_ctx *ctx, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* ERF_MLP_H */
