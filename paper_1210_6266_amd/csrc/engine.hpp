// The RSD engine: device state of one handle, set-up, apply, SpMV and Krylov drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rsd.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace rsd {
// a pinned host block of the library's cache
struct Pinned {
  void* p = nullptr;
  size_t bytes = 0;
};
// Work buffers of one preconditioner application (internal order, nv vectors): the
// handle's own (grown on demand), or carved from caller-independent static memory.
struct ApplyWork {
  double *e = nullptr, *t = nullptr, *xil = nullptr;   // xil: only for nv > 1
  void* sympart = nullptr;                             // symmetric-product partials
  double *gm_V = nullptr, *gm_beta = nullptr, *gm_H = nullptr, *gm_part = nullptr,
         *gm_coef = nullptr;                           // inexact interface solves
  int32_t *gm_steps = nullptr, *gm_stop = nullptr;
};
}  // namespace rsd

struct rsd_ctx {
  rsd::Plan P;
  rsd_options opt{};
  std::string err;
  int device = 0;

  hipStream_t cur = nullptr;      // stream of the running call
  // Ordering between calls on different streams: every call records ev_last on its
  // stream when it ends; a call on another stream first waits for it (calls made while
  // their stream is being captured into a graph are left to the caller's ordering).
  hipEvent_t ev_last = nullptr;
  hipStream_t last_s = nullptr;
  bool has_last = false;
  int no_events = 0;              // 1: the timers count launches but create no events
  // every device allocation of the handle (block, size as allocated)
  std::vector<std::pair<void*, size_t>> allocs;
  int64_t device_bytes = 0;

  // K in internal order and the index structures of the plan
  int64_t *prow = nullptr, *segA = nullptr, *segB = nullptr, *segC = nullptr, *pmap = nullptr;
  int32_t *pcol = nullptr, *perm = nullptr, *iperm = nullptr;
  int32_t *skel_lvl_begin = nullptr, *skel_own_end = nullptr;
  int64_t *kcol_pos = nullptr, *krow_pos = nullptr;   // caller value positions of couplings
  double *kcol_v = nullptr, *krow_v = nullptr;
  double* pval = nullptr;
  int64_t* ell_off = nullptr;       // sliced ELL copy of K (SpMVs)
  int32_t* ell_col = nullptr;
  double* ell_val = nullptr;
  int64_t *B_off = nullptr, *adj_ptr = nullptr, *sig_off_d = nullptr;
  int32_t *B = nullptr, *adj_leaf = nullptr, *adj_pos = nullptr;
  rsd::SigmaArgs sig{};
  void* sigma = nullptr;
  int sigma_fp32 = 0;
  rsd::DevBatch leaf{};
  std::vector<rsd::DevBatch> lev;
  rsd::DevBatch leaf_apply;    // the leaf batch as the applies read it (16-bit copy or leaf)
  int32_t* leaf_row0 = nullptr; // per leaf: its first tile row holding shell rows
  rsd::GenBatch gen;           // symmetric = 0: dense general sub-domain inverses
  int64_t leaf_elems = 0;
  std::vector<rsd::SigmaLevelItems> lev_items;       // Sigma products against deeper levels
  std::vector<rsd::SigmaLevelItems> lev_own_items;   // and against the level itself (gamma)
  int32_t* flags = nullptr;  // one per leaf, then one per interface
  hipStream_t aux = nullptr;          // look-ahead stream of the inversions (held exclusively)
  hipEvent_t ev_main = nullptr, ev_aux = nullptr;
  hipStream_t upl = nullptr;          // the couplings' upload, beside the sub-domain inversion,
  hipEvent_t ev_upl = nullptr;        // and the dense levels' Schur assemblies (held
  hipEvent_t ev_sig = nullptr;        // exclusively, from the same pool as aux): the Sigma
  std::vector<hipEvent_t> ev_lev;     // blocks are done / each level's S~ is assembled
  int group = 0;             // pivot tiles per sweep step (0: by batch size)
  int split16 = 0;           // FP32 batches: sweep updates on the BF16 matrix cores (bf16_split)

  // apply work vectors (internal order)
  double *e = nullptr, *t = nullptr, *rin = nullptr, *zin = nullptr;   // nvec vectors each
  double* xil = nullptr;     // n * kEllVec: interleaved SpMV operand (null while nvec == 1)
  int nvec = 0;
  // inexact interface solves: per level, 1 when its systems get gamma GMRES steps; the
  // GMRES scratch (basis, beta, Hessenberg matrices, steps, stop flags) for nvec vectors
  std::vector<char> gam_level;
  bool any_gamma = false;
  double *gm_V = nullptr, *gm_beta = nullptr, *gm_H = nullptr;
  int32_t *gm_steps = nullptr, *gm_stop = nullptr;
  // levels with systems larger than one chunk: work items of the chunked kernels
  struct GmLevel {
    bool chunked = false;
    int32_t nitems = 0;
    int32_t* item_sys = nullptr;
    int64_t *item_b = nullptr, *item_e = nullptr;
    int32_t* sys_first = nullptr;
  };
  std::vector<GmLevel> gm_lev;
  int32_t gm_max_items = 0;
  // captured preconditioner applications: graph exec per number of columns (index nv),
  // on rin -> zin; dropped whenever a buffer they use is reallocated
  std::vector<hipGraphExec_t> apply_graph;
  hipStream_t cap = nullptr;    // capture stream (the caller's may be the legacy null stream)
  // autotuned vectors per pass of the symmetric products, per column count (index nv):
  // [0] the sub-domain batch, [1 + q] dense interface level q; tuned[nv] once done
  std::vector<std::array<int32_t, 9>> vec_pass;
  std::array<bool, 9> tuned{};
  int32_t last_tuned = 0;
  int32_t setup_variant[8] = {};            // set-up autotuner's candidate + 1 per batch
  double *gm_part = nullptr, *gm_coef = nullptr;
  double* sympart = nullptr;                // partial sums of the symmetric products
  size_t sympart_bytes = 0;

  // Krylov work space (grown on demand)
  int kry_m = 0, kry_nr = 0;   // restart length, right-hand sides in lockstep
  double *V = nullptr, *Z = nullptr, *w = nullptr, *hdev = nullptr, *tmp = nullptr,
         *part = nullptr, *scal = nullptr, *bint = nullptr, *xint = nullptr;
  double* hhost = nullptr;   // pinned (hhost_block): general use, then two halves that
  rsd::Pinned hhost_block;   // take the Hessenberg columns of alternate Arnoldi steps
  hipEvent_t ev_h[2] = {};   // those columns' copies have landed

  // timing
  struct Pending { int cls; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double time_ms[RSD_T_COUNT] = {};
  int64_t launches[RSD_T_COUNT] = {};
  double host_ms = 0.0;
  double setup_wall[4] = {};

  // set-up: the host copy of K's structure kept for the second part of the analysis
  // (build_plan_couplings), which runs while the device inverts the sub-domains, and
  // pinned staging buffers released after the set-up's final synchronisation
  rsd::Pinned csr_stage;
  const int64_t* ana_rp = nullptr;
  const int32_t* ana_ci = nullptr;
  std::vector<rsd::Pinned> held;
  bool couplings_on_device = false;   // upload_couplings has run (once per handle)
};

namespace rsd {

// All return RSD_OK or an error with h->err set.
rsd_status engine_init(rsd_ctx* h, const rsd_csr* csr, const rsd_hierarchy* hier,
                       const rsd_options* opt, hipStream_t s);
rsd_status engine_numeric(rsd_ctx* h, const double* values_dev, hipStream_t s);
rsd_status engine_apply(rsd_ctx* h, int nrhs, const double* r, int64_t ldr, double* z,
                        int64_t ldz, hipStream_t s);
rsd_status engine_spmv(rsd_ctx* h, int nrhs, const double* x, int64_t ldx, double* y,
                       int64_t ldy, hipStream_t s);
rsd_status engine_solve(rsd_ctx* h, int nrhs, const double* b, int64_t ldb, double* x,
                        int64_t ldx, const rsd_solve_options* opt, rsd_solve_info* info,
                        hipStream_t s);
rsd_status engine_stats(rsd_ctx* h, rsd_stats* out, int reset, hipStream_t s);
// rsd_apply on caller-independent memory: every work buffer carved from [area, area +
// cap) (device memory of the handle's device), no allocation, no graph, no autotuning,
// no host synchronisation.  Passes of as many columns (up to 8) as fit;
// RSD_ERR_INVALID_ARGUMENT when one column does not fit.
rsd_status engine_apply_static(rsd_ctx* h, int nrhs, const double* r, int64_t ldr, double* z,
                               int64_t ldz, void* area, size_t cap, hipStream_t s);
// bytes engine_apply_static needs for passes of nv columns
size_t apply_static_bytes(const rsd_ctx* h, int nv);
void engine_free(rsd_ctx* h);
// frees the cached device blocks, pinned staging buffers and idle auxiliary streams
// of `device` (every device when device < 0) that no live handle holds
void release_cache(int device);
void fill_analysis(const Plan& P, rsd_analysis* a);
// looks up the static work area of rsd_apply_noalloc on `device` (current)
void noalloc_register(int device);

}  // namespace rsd
