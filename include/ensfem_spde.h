/*
 * ensfem SPDE sampler -- Gaussian Markov random fields with Matern
 * covariance on the wall mesh (Sec. 2.1), for the material fields of the
 * ensemble solver.
 *
 * With piecewise linear basis functions on the triangles, C~ the lumped
 * mass (C~_ii = sum of A_e / 3 over the elements at node i) and G the
 * surface Laplacian stiffness (G_ij = sum_e A_e grad psi_i . grad psi_j),
 * the alpha = 2 (Matern nu = 1) field has precision K C~^-1 K with
 * K = kappa^2 C~ + G, and x = K^-1 C~^(1/2) z has that distribution for
 * standard normal z.  The continuous field's marginal variance is
 * 1 / (4 pi kappa^2); the correlation length is rho = sqrt(8) / kappa.
 * The S right-hand sides are solved together by conjugate gradients with a
 * diagonal preconditioner, samples fastest in memory.
 *
 * Conventions as in ensfem.h: int32 status codes (ENS_*), host arrays are
 * copied, the caller allocates the device workspace (spde_workspace_size)
 * and keeps ownership; no C++ exception crosses this interface.
 */
#ifndef ENSFEM_SPDE_H
#define ENSFEM_SPDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spde_ctx spde_ctx;

/* Lifetime; ENS_EDEVICE if the device cannot be selected. */
int32_t spde_create(int32_t device, spde_ctx** out);
int32_t spde_destroy(spde_ctx* s);
const char* spde_last_error(const spde_ctx* s);

/* Mesh: xyz [n_nodes*3], tri [n_el*3] (0-based).  Assembles C~ and G on
 * the host (FP64).  ENS_EINVAL for an index out of range or a degenerate
 * triangle. */
int32_t spde_set_mesh(spde_ctx* s, int64_t n_nodes, const double* xyz, int64_t n_el, const int32_t* tri);

/* Device workspace for S samples per call (matrix, preconditioner, four CG
 * block vectors [n_nodes][S_pad] and reduction buffers), and its binding
 * (borrowed until destroy or re-bind; 256-B aligned). */
int32_t spde_workspace_size(spde_ctx* s, int32_t S, size_t* bytes);
int32_t spde_bind_workspace(spde_ctx* s, int32_t S, void* dptr, size_t bytes);

/* x [n_nodes*S] (host, samples fastest) = K^-1 C~^(1/2) z for white noise
 * z [n_nodes*S] (host), kappa > 0.  Conjugate gradients run until every
 * column's residual is at most tol times its right-hand side's norm (checked
 * every 8 iterations) or max_iter iterations; *iterations and the largest
 * relative residual go to the optional outputs.  ENS_ENONFINITE-free: a
 * column that does not converge is reported through max_relres, not as an
 * error.  Synchronizing. */
int32_t spde_sample(spde_ctx* s, double kappa, const double* z, double tol, int32_t max_iter, double* x,
                    int32_t* iterations, double* max_relres);

#ifdef __cplusplus
}
#endif

#endif
