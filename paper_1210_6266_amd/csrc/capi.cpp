// extern "C" entry points declared in include/rsd.h.  Nothing throws across the ABI.
#include <cstring>
#include <new>
#include <string>

#include "engine.hpp"

namespace {

thread_local std::string g_last_error = "no error";

rsd_status fail(rsd_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

bool prec_ok(int32_t p) { return p == RSD_PREC_FP64 || p == RSD_PREC_FP32; }
bool leaf_prec_ok(int32_t p) { return prec_ok(p) || p == RSD_PREC_FP16 || p == RSD_PREC_BF16; }

rsd_status check_inputs(const rsd_csr* csr, const rsd_hierarchy* hier) {
  if (!csr || !hier) return fail(RSD_ERR_INVALID_ARGUMENT, "csr and hierarchy must not be NULL");
  if (csr->n <= 0) return fail(RSD_ERR_INVALID_ARGUMENT, "n must be positive");
  if (csr->nnz < 0) return fail(RSD_ERR_INVALID_ARGUMENT, "nnz must be non-negative");
  if (!csr->row_ptr || (csr->nnz > 0 && !csr->col_idx))
    return fail(RSD_ERR_INVALID_ARGUMENT, "row_ptr / col_idx must not be NULL");
  if (hier->num_nodes <= 0 || !hier->parent || !hier->dof_node)
    return fail(RSD_ERR_INVALID_ARGUMENT, "hierarchy needs num_nodes >= 1, parent and dof_node");
  return RSD_OK;
}

}  // namespace

namespace rsd {
void set_thread_error(const std::string& msg) { g_last_error = msg; }
}  // namespace rsd

extern "C" {

void rsd_options_default(rsd_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = int32_t(sizeof(rsd_options));
  o->leaf_prec = RSD_PREC_FP64;
  o->sigma_prec = RSD_PREC_FP64;
  o->iface_prec = RSD_PREC_FP64;
  o->root_prec = RSD_PREC_FP64;
  o->host_pointers = 0;
  o->timing = 0;
  o->iface_mode = RSD_IFACE_DENSE;
  o->gamma = 8;
  o->dense_max = 32768;
  o->graphs = 1;
  o->autotune = 1;
  o->symmetric = 1;
  o->g_coupling = RSD_COUPLING_FULL;
  o->bf16_split = 1;
  o->sym_form = 0;
  o->timing_classes = 0;
  o->dev_alloc = nullptr;
  o->dev_free = nullptr;
  o->alloc_ctx = nullptr;
}

rsd_status rsd_analyze(const rsd_csr* csr, const rsd_hierarchy* hier, rsd_analysis* out) {
  try {
    if (!out) return fail(RSD_ERR_INVALID_ARGUMENT, "out must not be NULL");
    const rsd_status st = check_inputs(csr, hier);
    if (st != RSD_OK) return st;
    rsd::Plan P;
    std::string msg;
    rsd::PlanError e = rsd::build_plan(csr->n, csr->nnz, csr->row_ptr, csr->col_idx,
                                       hier->num_nodes, hier->parent, hier->dof_node, &P, &msg);
    if (e == rsd::PlanError::kOk) e = rsd::build_plan_couplings(csr->row_ptr, csr->col_idx, &P, &msg);
    if (e == rsd::PlanError::kNotSeparable) return fail(RSD_ERR_MAP_NOT_SEPARABLE, msg);
    if (e != rsd::PlanError::kOk) return fail(RSD_ERR_INVALID_ARGUMENT, msg);
    rsd::fill_analysis(P, out);
    return RSD_OK;
  } catch (const std::bad_alloc&) {
    return fail(RSD_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(RSD_ERR_INVALID_ARGUMENT, "unexpected exception in rsd_analyze");
  }
}

rsd_status rsd_setup(const rsd_csr* csr, const rsd_hierarchy* hier, const rsd_options* opt,
                     void* stream, rsd_handle* out) {
  if (!out) return fail(RSD_ERR_INVALID_ARGUMENT, "out must not be NULL");
  *out = nullptr;
  rsd_status st = check_inputs(csr, hier);
  if (st != RSD_OK) return st;
  if (opt) {
    if (opt->struct_size != int32_t(sizeof(rsd_options)))
      return fail(RSD_ERR_INVALID_ARGUMENT, "rsd_options.struct_size mismatch");
    if (!leaf_prec_ok(opt->leaf_prec) || !prec_ok(opt->sigma_prec) || !prec_ok(opt->iface_prec) ||
        !prec_ok(opt->root_prec))
      return fail(RSD_ERR_INVALID_ARGUMENT, "unknown precision code");
    if (opt->host_pointers != 0 && opt->host_pointers != 1)
      return fail(RSD_ERR_INVALID_ARGUMENT, "host_pointers must be 0 or 1");
    if (opt->iface_mode != RSD_IFACE_DENSE && opt->iface_mode != RSD_IFACE_GAMMA &&
        opt->iface_mode != RSD_IFACE_HYBRID)
      return fail(RSD_ERR_INVALID_ARGUMENT, "unknown interface mode");
    if (opt->iface_mode != RSD_IFACE_DENSE && (opt->gamma < 1 || opt->gamma > 64))
      return fail(RSD_ERR_INVALID_ARGUMENT, "gamma must be in 1..64");
    if (opt->iface_mode == RSD_IFACE_HYBRID && opt->dense_max < 0)
      return fail(RSD_ERR_INVALID_ARGUMENT, "dense_max must be >= 0");
    if (opt->graphs != 0 && opt->graphs != 1)
      return fail(RSD_ERR_INVALID_ARGUMENT, "graphs must be 0 or 1");
    if (opt->autotune != 0 && opt->autotune != 1)
      return fail(RSD_ERR_INVALID_ARGUMENT, "autotune must be 0 or 1");
    if (opt->symmetric != 0 && opt->symmetric != 1)
      return fail(RSD_ERR_INVALID_ARGUMENT, "symmetric must be 0 or 1");
    if (opt->bf16_split != 0 && opt->bf16_split != 1)
      return fail(RSD_ERR_INVALID_ARGUMENT, "bf16_split must be 0 or 1");
    if (opt->sym_form != 0 && opt->sym_form != 1)
      return fail(RSD_ERR_INVALID_ARGUMENT, "sym_form must be 0 or 1");
    if (opt->g_coupling != RSD_COUPLING_FULL && opt->g_coupling != RSD_COUPLING_LEAF_ONLY)
      return fail(RSD_ERR_INVALID_ARGUMENT, "g_coupling must be RSD_COUPLING_FULL or "
                                            "RSD_COUPLING_LEAF_ONLY");
    if ((opt->dev_alloc == nullptr) != (opt->dev_free == nullptr))
      return fail(RSD_ERR_INVALID_ARGUMENT, "dev_alloc and dev_free must be set together");
    if (opt->symmetric == 0 && opt->iface_mode != RSD_IFACE_GAMMA)
      return fail(RSD_ERR_UNSUPPORTED,
                  "symmetric = 0 needs iface_mode GAMMA (the interface inverses are symmetric)");
    if (opt->symmetric == 0 && !prec_ok(opt->leaf_prec))
      return fail(RSD_ERR_UNSUPPORTED, "symmetric = 0 needs leaf_prec FP64 or FP32");
  }
  if (!csr->values) return fail(RSD_ERR_INVALID_ARGUMENT, "values must not be NULL");
  rsd_ctx* h = nullptr;
  try {
    h = new rsd_ctx();
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = rsd::engine_init(h, csr, hier, opt, s);
    if (st == RSD_OK) rsd::noalloc_register(h->device);
    if (st == RSD_OK) {
      const double* vals = csr->values;
      double* tmp = nullptr;
      if (h->opt.host_pointers) {
        if (hipMalloc(&tmp, size_t(csr->nnz > 0 ? csr->nnz : 1) * sizeof(double)) != hipSuccess) {
          h->err = "hipMalloc failed for the values";
          st = RSD_ERR_OUT_OF_MEMORY;
        } else if (csr->nnz > 0 &&
                   hipMemcpyAsync(tmp, csr->values, size_t(csr->nnz) * sizeof(double),
                                  hipMemcpyHostToDevice, s) != hipSuccess) {
          h->err = "copy of the values failed";
          st = RSD_ERR_DEVICE;
        }
        vals = tmp;
      }
      if (st == RSD_OK) st = rsd::engine_numeric(h, vals, s);
      if (tmp) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(tmp);
      }
    }
    if (st != RSD_OK) {
      g_last_error = h->err;
      rsd::engine_free(h);
      delete h;
      return st;
    }
    *out = h;
    return RSD_OK;
  } catch (const std::bad_alloc&) {
    if (h) {
      rsd::engine_free(h);
      delete h;
    }
    return fail(RSD_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    if (h) {
      rsd::engine_free(h);
      delete h;
    }
    return fail(RSD_ERR_DEVICE, "unexpected exception in rsd_setup");
  }
}

static rsd_status vec_args(rsd_handle h, int32_t nrhs, const void* a, int64_t lda, const void* b,
                           int64_t ldb) {
  if (!h) return fail(RSD_ERR_INVALID_ARGUMENT, "NULL handle");
  if (nrhs < 0) {
    h->err = "nrhs must be non-negative";
    return RSD_ERR_INVALID_ARGUMENT;
  }
  if (nrhs == 0) return RSD_OK;
  if (!a || !b || lda < h->P.n || ldb < h->P.n) {
    h->err = "vector pointers must not be NULL and leading dimensions must be >= n";
    return RSD_ERR_INVALID_ARGUMENT;
  }
  if (a == b) {
    h->err = "input and output must not overlap";
    return RSD_ERR_INVALID_ARGUMENT;
  }
  return RSD_OK;
}

rsd_status rsd_apply(rsd_handle h, int32_t nrhs, const double* r, int64_t ldr, double* z,
                     int64_t ldz, void* stream) {
  const rsd_status st = vec_args(h, nrhs, r, ldr, z, ldz);
  if (st != RSD_OK || nrhs == 0) return st;
  try {
    return rsd::engine_apply(h, nrhs, r, ldr, z, ldz, static_cast<hipStream_t>(stream));
  } catch (...) {
    h->err = "unexpected exception in rsd_apply";
    return RSD_ERR_DEVICE;
  }
}

rsd_status rsd_spmv(rsd_handle h, int32_t nrhs, const double* x, int64_t ldx, double* y,
                    int64_t ldy, void* stream) {
  const rsd_status st = vec_args(h, nrhs, x, ldx, y, ldy);
  if (st != RSD_OK || nrhs == 0) return st;
  try {
    return rsd::engine_spmv(h, nrhs, x, ldx, y, ldy, static_cast<hipStream_t>(stream));
  } catch (...) {
    h->err = "unexpected exception in rsd_spmv";
    return RSD_ERR_DEVICE;
  }
}

rsd_status rsd_solve(rsd_handle h, int32_t nrhs, const double* b, int64_t ldb, double* x,
                     int64_t ldx, const rsd_solve_options* opt, rsd_solve_info* info,
                     void* stream) {
  const rsd_status st = vec_args(h, nrhs, b, ldb, x, ldx);
  if (st != RSD_OK || nrhs == 0) return st;
  if (opt) {
    if ((opt->method != RSD_SOLVER_FGMRES && opt->method != RSD_SOLVER_PCG) ||
        (opt->method == RSD_SOLVER_FGMRES && (opt->restart < 1 || opt->restart > 256)) ||
        opt->maxit < 0 || !(opt->rtol >= 0.0) || (opt->use_x0 != 0 && opt->use_x0 != 1)) {
      h->err = "invalid rsd_solve_options";
      return RSD_ERR_INVALID_ARGUMENT;
    }
  }
  try {
    return rsd::engine_solve(h, nrhs, b, ldb, x, ldx, opt, info, static_cast<hipStream_t>(stream));
  } catch (...) {
    h->err = "unexpected exception in rsd_solve";
    return RSD_ERR_DEVICE;
  }
}

rsd_status rsd_update_values(rsd_handle h, const double* values, void* stream) {
  if (!h) return fail(RSD_ERR_INVALID_ARGUMENT, "NULL handle");
  if (!values) {
    h->err = "values must not be NULL";
    return RSD_ERR_INVALID_ARGUMENT;
  }
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double* vals = values;
    double* tmp = nullptr;
    if (h->opt.host_pointers) {
      if (hipMalloc(&tmp, size_t(h->P.nnz > 0 ? h->P.nnz : 1) * sizeof(double)) != hipSuccess) {
        h->err = "hipMalloc failed for the values";
        return RSD_ERR_OUT_OF_MEMORY;
      }
      if (h->P.nnz > 0 && hipMemcpyAsync(tmp, values, size_t(h->P.nnz) * sizeof(double),
                                         hipMemcpyHostToDevice, s) != hipSuccess) {
        (void)hipFree(tmp);
        h->err = "copy of the values failed";
        return RSD_ERR_DEVICE;
      }
      vals = tmp;
    }
    const rsd_status st = rsd::engine_numeric(h, vals, s);
    if (tmp) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(tmp);
    }
    return st;
  } catch (...) {
    h->err = "unexpected exception in rsd_update_values";
    return RSD_ERR_DEVICE;
  }
}

rsd_status rsd_get_stats(rsd_handle h, rsd_stats* out, int32_t reset, void* stream) {
  if (!h || !out) return fail(RSD_ERR_INVALID_ARGUMENT, "NULL handle or output");
  try {
    return rsd::engine_stats(h, out, reset, static_cast<hipStream_t>(stream));
  } catch (...) {
    h->err = "unexpected exception in rsd_get_stats";
    return RSD_ERR_DEVICE;
  }
}

void rsd_destroy(rsd_handle h) {
  if (!h) return;
  try {
    rsd::engine_free(h);
  } catch (...) {
  }
  delete h;
}

void rsd_release_cache(int32_t device) {
  try {
    rsd::release_cache(device);
  } catch (...) {
  }
}

const char* rsd_last_error(rsd_handle h) {
  if (h) return h->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
