/*
 * ensfem surrogate -- learned form of the ensemble wall solver.
 *
 * A fully connected network maps the leading Karhunen-Loeve coefficients of
 * the log-modulus and log-thickness fields (the stochastic inputs of
 * Sec. 2.1) to the per-node peak radial displacement that the plain solver
 * computes; it serves as the low-fidelity model of a multifidelity control
 * variate whose bias the plain solver corrects.  Hidden layers are
 * z = W h + b, h' = GELU(z) (exact erf form), the output layer is linear;
 * training minimises the mean squared error with Adam (b1 = 0.9, b2 = 0.999,
 * eps = 1e-8, bias-corrected).  Matrix products run on BF16 matrix cores
 * with FP32 accumulation; master weights, biases and Adam moments are FP32.
 *
 * Conventions as in ensfem.h: int32 status codes (ENS_*), the caller
 * allocates the device workspace (sur_info gives its size) and owns every
 * buffer passed in; device arrays are row-major, batch rows outermost.
 * Parameter vector layout (FP32, host): for l = 0 .. n_hidden, W_l
 * [out_l][in_l] row-major then b_l [out_l].
 */
#ifndef ENSFEM_SURROGATE_H
#define ENSFEM_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sur_net sur_net;

/* Network n_in -> n_hidden x width (GELU) -> n_out; batches of at most
 * max_batch rows per pass.  ENS_EINVAL for non-positive sizes, ENS_EDEVICE
 * for a bad device. */
int32_t sur_create(int32_t device, int32_t n_in, int32_t width, int32_t n_hidden, int32_t n_out,
                   int32_t max_batch, sur_net** out);
int32_t sur_destroy(sur_net* s);
const char* sur_last_error(const sur_net* s);
/* parameter count and the workspace size in bytes */
int32_t sur_info(sur_net* s, int64_t* n_params, size_t* workspace_bytes);
/* Device buffer of at least the workspace size, 256-B aligned, borrowed
 * until destroy or re-bind (ENS_EWORKSPACE otherwise). */
int32_t sur_bind_workspace(sur_net* s, void* dptr, size_t bytes);
/* Copy parameters in (host FP32, layout above; resets the Adam state) or
 * out.  ENS_EINVAL on a non-finite value. */
int32_t sur_set_params(sur_net* s, const float* host);
int32_t sur_get_params(sur_net* s, float* host);
/* Copy of the FP32 parameters (layout above) into a caller-owned device
 * buffer of n_params floats, enqueued on `stream` (a snapshot during
 * training without a trip through host memory). */
int32_t sur_get_params_device(sur_net* s, float* dptr, void* stream);
/* Y [batch][n_out] = network(X [batch][n_in]), device FP32 buffers. */
int32_t sur_forward(sur_net* s, const float* X, int32_t batch, float* Y, void* stream);
/* Gradient of the mean squared error against targets T [batch][n_out]
 * (device), written to grad (device FP32, parameter layout); loss (device
 * FP32 scalar) may be NULL.  No update. */
int32_t sur_gradients(sur_net* s, const float* X, const float* T, int32_t batch, float* grad, float* loss,
                      void* stream);
/* Decoupled weight decay for the following Adam steps (AdamW, Loshchilov &
 * Hutter 2019): each step subtracts lr * wd * W from every weight matrix W
 * besides the Adam update; biases are not decayed.  Default 0.  ENS_EINVAL
 * for a negative or non-finite wd. */
int32_t sur_set_weight_decay(sur_net* s, float wd);
/* One Adam step with step size lr on the batch (X, T device FP32); the
 * batch loss before the step goes to *loss (device FP32) if non-NULL. */
int32_t sur_train_step(sur_net* s, const float* X, const float* T, int32_t batch, float lr, float* loss,
                       void* stream);
/* Sums of y and y^2 per output over M input rows X [M][n_in] (device),
 * results to host FP64 arrays [n_out]; the M x n_out outputs are never
 * formed.  The output layer is linear (y = W h + b), so the rows only pass
 * through the hidden layers (4,096 at a time), whose last activations give
 * s = sum_r h_r and G = sum_r h_r h_r^T; then per output j
 * sum y = w_j . s + M b_j and sum y^2 = w_j^T G w_j + 2 b_j w_j . s + M b_j^2
 * (the same sums as a forward pass of every row, up to rounding).
 * Synchronizes. */
int32_t sur_moments(sur_net* s, const float* X, int64_t M, double* sum_host, double* sumsq_host,
                    void* stream);
/* Squared error of the physical-unit predictions against targets:
 * *acc (device FP64 scalar) += sum over the batch rows and outputs j of
 * (mu[j] + sd[j] y[r][j] - Q[r][j])^2, with y = network(X [batch][n_in])
 * and Q [batch][n_out], mu, sd [n_out] device FP64 (the targets'
 * standardization).  Summation order is fixed.  Enqueued on `stream`;
 * ENS_EINVAL for a batch outside 1 .. max_batch. */
int32_t sur_sq_error(sur_net* s, const float* X, int32_t batch, const double* Q, const double* mu, const double* sd,
                     double* acc, void* stream);
/* Row gather for minibatches: dst[r][:] = src[idx[r]][:] for r < n_rows,
 * FP32 rows of n_cols values, idx device int32 (each in range of src, which
 * the caller guarantees).  ENS_EINVAL for n_cols < 1 or n_rows outside
 * 0 .. 65535.  Enqueued on `stream`. */
int32_t sur_gather_rows(const float* src, int64_t n_cols, const int32_t* idx, int32_t n_rows, float* dst,
                        void* stream);
/* Control-variate combination per row (device FP64 arrays):
 * qH, qL [n][N] paired high / low fidelity values, sumL / sumsqL [n] sums
 * of the low-fidelity values and squares over M independent inputs.
 * beta = Cov(qH, qL) / Var(qL); mean = mean(qH) - beta (mean(qL) - sumL/M);
 * the same on the squares gives the second moment, var = m2 - mean^2;
 * rho = the Pearson correlation of qH and qL.  ENS_EINVAL if N < 2. */
int32_t sur_cv_moments(const double* qH, const double* qL, int64_t n, int32_t N, const double* sumL,
                       const double* sumsqL, int64_t M, double* mean, double* var, double* rho, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ENSFEM_SURROGATE_H */
