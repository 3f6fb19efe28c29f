/* Finite-element coefficient maps for the RSD library: assembly of the CSR values of
 * K(theta) = sum_e k(theta_e) K_e and the element-wise gradient of a loss through
 * the adjoint solution, for differentiable solves x = K(theta)^{-1} b.
 *
 * Adjoint relation (differentiating K x = b): with lambda = K^{-T} dL/dx, the gradient
 * is dL/db = lambda and dL/dtheta_e = -k'(theta_e) lambda_e^T K_e x_e, where lambda_e,
 * x_e are the element's entries (zero on eliminated dofs).  K is symmetric here, so
 * the adjoint solve reuses the same RSD handle (rsd_solve with right-hand side dL/dx).
 * The operator is the Q1 system of Section 4's model problems with a per-element
 * coefficient; the RSD set-up and apply (Sections 2-3) do not depend on how the
 * values were assembled.
 *
 * All arrays are device pointers on the current HIP device; calls are asynchronous
 * on `stream` (NULL = default stream) and allocate nothing.
 */
#ifndef RSD_FE_H_
#define RSD_FE_H_

#include "rsd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* coef_kind: how the element coefficient depends on the parameter */
enum { RSD_COEF_LINEAR = 0, /* k(theta) = theta      */
       RSD_COEF_EXP = 1 };  /* k(theta) = exp(theta) */

typedef struct {
  int32_t num_elements;        /* E                                                    */
  int32_t dofs_per_element;    /* d, 1 <= d <= 64                                      */
  int64_t nnz;                 /* nonzeros of the assembled CSR matrix                 */
  const int32_t* elem_dofs;    /* E x d, row-major: dof of local index a, -1 when the
                                  dof is eliminated (Dirichlet)                        */
  const double* ke;            /* d x d reference element matrix, column-major,
                                  symmetric; K_e = k(theta_e) * ke                     */
  const int64_t* contrib_ptr;  /* nnz + 1: contributions of CSR entry p are
                                  contrib[contrib_ptr[p] .. contrib_ptr[p + 1])        */
  const int32_t* contrib;      /* packed e * d * d + a * d + b: element e's entry (a, b)
                                  adds to this CSR position; summed in stored order    */
} rsd_fe_map;

/* values[p] = sum over the contributions (e, a, b) of p of k(theta_e) ke[a, b]
 * (the CSR values of K(theta) in the caller's nonzero order, ready for rsd_setup or
 * rsd_update_values).  Deterministic.  Errors: RSD_ERR_INVALID_ARGUMENT for a NULL
 * map / array with a non-zero size, d outside [1, 64] or an unknown coef_kind. */
rsd_status rsd_fe_assemble(const rsd_fe_map* map, const double* theta, int32_t coef_kind,
                           double* values, void* stream);

/* grad[e] = -k'(theta_e) * sum_{a,b} lambda[dof_a] ke[a, b] x[dof_b] over the element's
 * non-eliminated dofs (the theta-gradient of a loss L(x) with lambda = K^{-T} dL/dx).
 * lambda and x: n-vectors in the caller's dof numbering; grad: E values.  Same error
 * behaviour as rsd_fe_assemble. */
rsd_status rsd_fe_grad(const rsd_fe_map* map, const double* theta, int32_t coef_kind,
                       const double* lambda, const double* x, double* grad, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RSD_FE_H_ */
