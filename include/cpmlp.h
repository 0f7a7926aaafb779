/*
 * cpmlp.h — C ABI of the learned extrapolation step of libcpgrad.
 *
 * The paper accelerates CP_ALS by making each sweep cheap (Algorithm 2 inside
 * ALS, Section 4) and mentions line-search extrapolation as a known way to
 * cut the number of sweeps (Section 1).  This part adds such a step with a
 * learned step size: after an ALS sweep from A_start to A, a small MLP reads
 * features of the recent cost history and factor updates and proposes
 * sigma >= 0; the extrapolated factors A + sigma (A - A_start) are kept only
 * if their exactly evaluated cost (eq. 2.12) is lower than the sweep's, so the
 * plain ALS step is the fallback.
 *
 * Network: x (n_in) -> tanh(W1 x + b1) (n_hidden) -> tanh(W2 . + b2) (n_hidden)
 *          -> z = w3 . h2 + b3 -> sigma = sigma_max * sigmoid(z), all float32.
 * Parameters: one flat float32 vector [W1 (n_hidden x n_in, row-major), b1,
 * W2 (n_hidden x n_hidden), b2, w3, b3].  Training loss: mean over the batch
 * of (log(1 + sigma) - log(1 + target))^2, optimiser Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8).  All X / sigma / target / grad pointers are DEVICE
 * pointers; parameter transfers use host buffers.
 */
#ifndef CPMLP_H
#define CPMLP_H

#include <stddef.h>
#include <stdint.h>

#include "cpgrad.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CPG_NFEAT 12   /* features of the learned step (cpals_features) */

typedef struct cpmlp_s* cpmlp_t;

/* Create a network with n_in in [1, 32] inputs and n_hidden in [1, 32] units
 * per hidden layer; parameters start at zero (set them with cpmlp_set_params).
 * stream: hipStream_t, NULL for the null stream. */
int cpmlp_create(cpmlp_t* out, int n_in, int n_hidden, float sigma_max, void* stream);

/* Number of float32 parameters. */
int cpmlp_num_params(cpmlp_t m, int64_t* n);

/* Copy n parameters from / to a host buffer (n must equal cpmlp_num_params);
 * set also resets the Adam moments.  Both wait for the stream. */
int cpmlp_set_params(cpmlp_t m, const float* host, int64_t n);
int cpmlp_get_params(cpmlp_t m, float* host, int64_t n);

/* sigma[s] for the batch rows X[s][0..n_in) (device, row-major).  Async. */
int cpmlp_forward(cpmlp_t m, const float* X, int batch, float* sigma);

/* Gradient of the training loss w.r.t. every parameter into grad (device,
 * cpmlp_num_params floats), parameters unchanged; *loss_out (host, may be
 * NULL: then asynchronous) receives the loss. */
int cpmlp_gradients(cpmlp_t m, const float* X, const float* target, int batch, float* grad, double* loss_out);

/* One Adam step with learning rate lr on the batch; *loss_out (host, may be
 * NULL) receives the loss before the step. */
int cpmlp_train_step(cpmlp_t m, const float* X, const float* target, int batch, float lr, double* loss_out);

int cpmlp_destroy(cpmlp_t m);

/* Features of the learned step, written to feat (device, CPG_NFEAT floats):
 * [0..3]  log10 of the relative cost decrease of the last four sweeps / 12,
 *         from costs[0..ncost) (host, oldest first; missing ones count as 1)
 * [4] [5] mean and max over modes of log10(||A - A_start|| / ||A||) / 6
 * [6] [7] mean and min over modes of the cosine between this sweep's update
 *         A - A_start and the previous sweep's update (kept by the plan)
 * [8] R / 20, [9] log10(iteration + 1) / 4,
 * [10] log(1 + last_sigma) / log(1 + 32), [11] last_accept.
 * Then the plan stores A - A_start as the previous update.  Async. */
int cpals_features(cpgrad_plan_t p, const void* const* A, const void* const* A_start, const double* costs,
                   int ncost, int iteration, float last_sigma, int last_accept, float* feat);

/* Cost (eq. 2.12) and fit of the extrapolated model A + sigma (A - A_start)
 * against the bound Y; A is not changed.  Waits for the stream. */
int cp_fit_extrapolated(cpgrad_plan_t p, const void* Y, const void* const* A, const void* const* A_start,
                        double sigma, double* cost_out, double* fit_out);

/* Extrapolation step with a step size the caller chooses (sigma >= 0):
 * A_ext = A_new + sigma (A_new - A_prev); the exact cost of eq. 2.12 of A_ext
 * against the bound Y (one pass over Y plus float64 Grams) is compared with
 * the plan's last cost, which must be the cost of A_new (call this right
 * after the cpals_step or cp_fit that gave A_new).  Only if it is lower is
 * A_new overwritten with A_ext (*accepted = 1) and the plan's last cost
 * replaced; otherwise A_new is unchanged (*accepted = 0).  Returns the cost
 * and fit of the kept factors.  accepted, cost_out, fit_out may be NULL.
 * Waits for the stream.  Errors: CPG_ERR_INVALID (NULL, Y not the bound
 * tensor, sigma negative or not finite), CPG_ERR_NONFINITE, CPG_ERR_HIP. */
int cpals_extrapolate(cpgrad_plan_t p, const void* Y, void* const* A_new, const void* const* A_prev, double sigma,
                      int* accepted, double* cost_out, double* fit_out);

/* One learned-extrapolation ALS step on the bound Y: keeps A as A_start,
 * runs cpals_step, forms the features, lets the network propose sigma,
 * evaluates the exact cost of A + sigma (A - A_start) and keeps it only if
 * it is lower than the sweep's cost.  Returns the cost and fit of the kept
 * factors, whether the extrapolation was kept, and sigma.  costs / ncost /
 * iteration / last_sigma / last_accept feed the features (see above).
 * Waits for the stream.  Errors as cpals_step. */
int cpals_learned_step(cpgrad_plan_t p, cpmlp_t m, const void* Y, void* const* A, const double* costs, int ncost,
                       int iteration, float last_sigma, int last_accept, double* cost_out, double* fit_out,
                       int* accepted, float* sigma_out);

#ifdef __cplusplus
}
#endif

#endif /* CPMLP_H */
