// Coefficient maps of Q1 systems: CSR values of K(theta) and the element-wise adjoint
// gradient (include/rsd_fe.h).  One thread per nonzero / per element; fixed-order sums.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/rsd_fe.h"

namespace rsd {
void set_thread_error(const std::string& msg);  // capi.cpp
}

namespace {

constexpr int kFeBlock = 256;

__device__ __forceinline__ double coef_of(double t, int kind) { return kind ? exp(t) : t; }

__global__ __launch_bounds__(kFeBlock) void k_fe_assemble(
    int64_t nnz, int d, const int64_t* __restrict__ cptr, const int32_t* __restrict__ contrib,
    const double* __restrict__ ke, const double* __restrict__ theta, int kind,
    double* __restrict__ values) {
  const int64_t p = int64_t(blockIdx.x) * kFeBlock + threadIdx.x;
  if (p >= nnz) return;
  const int dd = d * d;
  double s = 0.0;
  for (int64_t c = cptr[p]; c < cptr[p + 1]; ++c) {
    const int32_t code = contrib[c];
    const int e = code / dd, ab = code % dd, a = ab / d, b = ab % d;
    s += coef_of(theta[e], kind) * ke[a + b * d];
  }
  values[p] = s;
}

__global__ __launch_bounds__(kFeBlock) void k_fe_grad(
    int32_t E, int d, const int32_t* __restrict__ elem_dofs, const double* __restrict__ ke,
    const double* __restrict__ theta, int kind, const double* __restrict__ lam,
    const double* __restrict__ x, double* __restrict__ grad) {
  const int e = int(blockIdx.x) * kFeBlock + threadIdx.x;
  if (e >= E) return;
  const int32_t* dofs = elem_dofs + int64_t(e) * d;
  double s = 0.0;
  for (int a = 0; a < d; ++a) {
    const int32_t da = dofs[a];
    if (da < 0) continue;
    double t = 0.0;
    for (int b = 0; b < d; ++b) {
      const int32_t db = dofs[b];
      if (db >= 0) t += ke[a + b * d] * x[db];
    }
    s += lam[da] * t;
  }
  const double dk = kind ? exp(theta[e]) : 1.0;
  grad[e] = -dk * s;
}

rsd_status check_map(const rsd_fe_map* m, int32_t kind) {
  if (!m) {
    rsd::set_thread_error("map must not be NULL");
    return RSD_ERR_INVALID_ARGUMENT;
  }
  if (m->num_elements < 0 || m->nnz < 0 || m->dofs_per_element < 1 || m->dofs_per_element > 64) {
    rsd::set_thread_error("rsd_fe_map: need num_elements >= 0, nnz >= 0, 1 <= d <= 64");
    return RSD_ERR_INVALID_ARGUMENT;
  }
  if (kind != RSD_COEF_LINEAR && kind != RSD_COEF_EXP) {
    rsd::set_thread_error("unknown coef_kind");
    return RSD_ERR_INVALID_ARGUMENT;
  }
  if (!m->ke || (m->num_elements > 0 && !m->elem_dofs) ||
      (m->nnz > 0 && (!m->contrib_ptr || !m->contrib))) {
    rsd::set_thread_error("rsd_fe_map: NULL array with a non-zero size");
    return RSD_ERR_INVALID_ARGUMENT;
  }
  return RSD_OK;
}

rsd_status launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return RSD_OK;
  rsd::set_thread_error(std::string(what) + ": " + hipGetErrorString(e));
  return RSD_ERR_DEVICE;
}

}  // namespace

extern "C" {

rsd_status rsd_fe_assemble(const rsd_fe_map* map, const double* theta, int32_t coef_kind,
                           double* values, void* stream) {
  const rsd_status st = check_map(map, coef_kind);
  if (st != RSD_OK) return st;
  if (map->nnz == 0) return RSD_OK;
  if (!values || (map->num_elements > 0 && !theta)) {
    rsd::set_thread_error("theta / values must not be NULL");
    return RSD_ERR_INVALID_ARGUMENT;
  }
  const unsigned blocks = unsigned((map->nnz + kFeBlock - 1) / kFeBlock);
  k_fe_assemble<<<blocks, kFeBlock, 0, static_cast<hipStream_t>(stream)>>>(
      map->nnz, map->dofs_per_element, map->contrib_ptr, map->contrib, map->ke, theta, coef_kind,
      values);
  return launched("rsd_fe_assemble");
}

rsd_status rsd_fe_grad(const rsd_fe_map* map, const double* theta, int32_t coef_kind,
                       const double* lambda, const double* x, double* grad, void* stream) {
  const rsd_status st = check_map(map, coef_kind);
  if (st != RSD_OK) return st;
  if (map->num_elements == 0) return RSD_OK;
  if (!theta || !lambda || !x || !grad) {
    rsd::set_thread_error("theta / lambda / x / grad must not be NULL");
    return RSD_ERR_INVALID_ARGUMENT;
  }
  const unsigned blocks = unsigned((map->num_elements + kFeBlock - 1) / kFeBlock);
  k_fe_grad<<<blocks, kFeBlock, 0, static_cast<hipStream_t>(stream)>>>(
      map->num_elements, map->dofs_per_element, map->elem_dofs, map->ke, theta, coef_kind,
      lambda, x, grad);
  return launched("rsd_fe_grad");
}

}  // extern "C"
