// Host-side launchers of the HIP kernels (implemented in kernels.hip).
//
// Every launcher enqueues on `s` and returns hipGetLastError() of its launch.
// Dense symmetric blocks are stored as packed lower tiles (see plan.hpp):
// tile (I, J), I >= J, of matrix m starts at tiles + tile_off[m] + (I(I+1)/2 + J)*64*64
// and is column-major 64 x 64; diagonal tiles hold both triangles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace rsd {

// Device view of a SymBatch (arrays live on the device).
struct DevBatch {
  int32_t count = 0;
  int32_t max_nt = 0;
  int64_t max_tiles = 0;
  const int32_t* n = nullptr;
  const int32_t* nt = nullptr;
  const int64_t* tile_off = nullptr;
  const int64_t* vec_off = nullptr;
  int32_t num_items = 0;
  const int32_t* item_mat = nullptr;
  const int32_t* item_BI = nullptr;
  const int32_t* item_BJ = nullptr;
  const int64_t* item_base = nullptr;
  void* tiles = nullptr;  // double* or float* (or 16-bit values, see half)
  int32_t fp32 = 0;
  int32_t half = 0;       // apply-side 16-bit copy of FP32 tiles: 1 FP16, 2 BF16 (0: none)
  int32_t vec_pass = 0;   // vectors per pass of the symmetric product (0: symv_vectors)
  int32_t persist = 0;    // symmetric products as a persistent work-queue launch
  int32_t* queue = nullptr;   // its two counters (zero between launches)
  int32_t split16 = 0;    // FP32 batches: sweep updates on the BF16 matrix cores, operands
                          // split exactly into three BF16 parts (k_sweep_update_bf3s)
  int32_t upd_shape = 0;  // split16 update form, bitwise alike: 0 128 x 128 super-tiles
                          // (k_sweep_update_bf3s), 1 256 x 256 super-tiles in four-tile
                          // groups (k_sweep_update_bf3w)
};

// ---- sparse / vector ------------------------------------------------------------------
hipError_t launch_gather(const double* src, const int64_t* map, int64_t count, double* dst,
                         hipStream_t s);
hipError_t launch_permute(const double* x, int64_t ldx, double* y, int64_t ldy,
                          const int32_t* perm, int64_t n, int32_t nrhs, int32_t inverse,
                          hipStream_t s);
// sliced ELL copy of K (layout in plan.hpp) and the segmented SpMV on it:
// y[r] = (base ? base[r] : 0) + alpha * sum over the entries of row r with CSR positions in
// [s0[r], s1[r]), rows r in [row0, row0 + nrows), entries summed in column order; for
// nv vectors x_k = x + k ld (likewise base, y) the slots are read once per kEllVec vectors,
// and when xil (n * kEllVec doubles of scratch, or null) is given the columns [col0, col1)
// of the vectors -- all that the rows' segments read -- are first interleaved there so that
// the gathers of a column are contiguous.  x, base and y may be the same vectors when the
// columns read are not the rows written.
constexpr int kEllVec = 8;
hipError_t launch_ell_fill(int64_t n, const int64_t* prow, const int32_t* pcol,
                           const double* pval, const int64_t* ell_off, int32_t* ell_col,
                           double* ell_val, hipStream_t s);
hipError_t launch_ell_spmv(int64_t row0, int64_t nrows, const int64_t* s0, const int64_t* s1,
                           const int64_t* prow, const int64_t* ell_off, const int32_t* ell_col,
                           const double* ell_val, const double* x, const double* base,
                           double alpha, double* y, int nv, int64_t ld, double* xil,
                           int64_t col0, int64_t col1, hipStream_t s);
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s);
// K in internal order from the caller's CSR (device arrays): pcol, pmap (caller value
// position of each entry) and the row segments segA / segB / segC
hipError_t launch_permute_csr(int32_t n, int64_t n_leaf, const int32_t* perm, const int32_t* iperm,
                              const int64_t* rp, const int32_t* ci, const int64_t* prow,
                              const int32_t* skel_lvl_begin, const int32_t* skel_own_end,
                              int32_t* pcol, int64_t* pmap, int64_t* segA, int64_t* segB,
                              int64_t* segC, hipStream_t s);

// ---- dense symmetric batches ------------------------------------------------------------
hipError_t launch_sym_fill(const DevBatch& b, hipStream_t s);
// scatters rows' segments [s0[r], s1[r]) of the internal CSR into the batch tiles
hipError_t launch_sym_extract(const DevBatch& b, const int64_t* s0, const int64_t* s1,
                              const int32_t* pcol, const double* pval, int32_t max_n,
                              hipStream_t s);
// In-place inversion by blocked symmetric sweeps, one step over the pivot tile
// columns [c0, c0 + group): stage 0 inverts the pivot block (scalar sweeps in
// registers; flags[m] != 0 marks a non-positive or non-finite pivot of matrix m),
// stage 1 forms the panels C_i = A_ip and B_i = C_i P, stage 2 updates every other
// lower tile (MFMA).  Steps c0 = 0, group, 2 group, ... < max_nt leave -A^{-1}.
// For group = 2 the update can be split: part 1 updates only the tiles in the row
// and column of the next pivot group (what the next pivot and panel read), part 2
// the others; part 0 updates all.
hipError_t launch_sweep_step(const DevBatch& b, int c0, int stage, void* pbuf, void* cbuf,
                             void* bbuf, int32_t* flags, int group, hipStream_t s, int part = 0);
size_t sym_invert_scratch_bytes(const DevBatch& b, int group, size_t* pbytes, size_t* cbytes);
// y_k = base_k + alpha * A x_k for every matrix of the batch and the nv vectors
// x_k = x + k ld (likewise base, y; internal order), read in groups of up to
// symv_vectors(b) vectors per pass over the tiles
// (part: symv_part_bytes(b) of scratch for the per-item partial sums).  base may be y.
// row0 (optional, per matrix): x is zero on the matrix's rows below 64 row0[m], so the
// tile rows I < row0[m] add nothing (their row parts multiply x_J, J <= I, their column
// parts x_I) and are not read
hipError_t launch_symv(const DevBatch& b, const double* x, void* part, double alpha,
                       const double* base, double* y, int nv, int64_t ld, hipStream_t s,
                       const int32_t* row0 = nullptr);
inline int symv_vectors(const DevBatch&) { return 4; }
// dst (count 16-bit values, FP16 for kind 1, BF16 for kind 2) = src rounded to nearest
hipError_t launch_narrow(const float* src, void* dst, int64_t count, int kind, hipStream_t s);
inline size_t symv_part_bytes(const DevBatch& b) {
  return size_t(b.num_items) * 2 * kSymB * kTile * size_t(symv_vectors(b)) *
         (b.fp32 ? sizeof(float) : sizeof(double));
}

// ---- general (non-symmetric) sub-domains: dense column-major inverses ----------------------
constexpr int kGenMax = 2048;   // largest sub-domain (LDS staging of one column and one row)
struct GenBatch {
  int32_t count = 0, max_n = 0, fp32 = 0;
  const int32_t* n = nullptr;
  const int64_t* vec_off = nullptr;
  const int64_t* gen_off = nullptr;   // n_l^2 prefix sums
  const int64_t* perm_off = nullptr;  // n_l prefix sums
  int32_t* perm = nullptr;            // pivot rows of the elimination
  void* A = nullptr;                  // double* or float*
};
// A_l = K_ll (rows' segments [prow[r], segA[r]) of the internal CSR), then A_l <- A_l^{-1}
// by Gauss-Jordan elimination with partial pivoting (flags[l] = k + 1 on a zero pivot)
hipError_t launch_gen_invert(const GenBatch& g, const int64_t* prow, const int64_t* segA,
                             const int32_t* pcol, const double* pval, int32_t* flags,
                             hipStream_t s);
// y_k = alpha A_l x_k on every leaf's rows, nv vectors at stride ld
hipError_t launch_gen_matvec(const GenBatch& g, const double* x, double alpha, double* y,
                             int nv, int64_t ld, hipStream_t s);

// ---- Schur complements --------------------------------------------------------------------
struct SigmaArgs {
  int32_t num_leaves, max_m;
  const int64_t* B_off;
  const int32_t* B;
  const int64_t* shell_off;
  const int32_t* shell;
  const int64_t* kcol_ptr;
  const int32_t* kcol_row;
  const double* kcol_v;     // values of K_{l,B_l} by columns
  const int64_t* krow_ptr;
  const int32_t* krow_col;
  const double* krow_v;     // values of K_{B_l,l} by rows
  const int64_t* w_off;
  const int64_t* sig_off;
  int32_t row_major = 0;    // Sigma_l stored row-major (a K that is not symmetric)
};
// W_l = K_ll^{-1}[shell, :] K_{l,B_l}  (from the leaf batch's -K_ll^{-1} tiles)
hipError_t launch_sigma_w(const DevBatch& leaf, const SigmaArgs& a, double* W, hipStream_t s);
// the same W_l from the dense inverses of a general batch
hipError_t launch_sigma_w_gen(const GenBatch& g, const SigmaArgs& a, double* W, hipStream_t s);
// Sigma_l = K_{B_l,l} W_l   (stored fp64 or fp32; row-major when a.row_major)
hipError_t launch_sigma_s(const SigmaArgs& a, const double* W, void* sigma, int sigma_fp32,
                          hipStream_t s);
// S~ tiles (already holding K_tt) -= sum over adjacent leaves of Sigma_l[I_t, I_t]
hipError_t launch_schur_assemble(const DevBatch& b, const int64_t* adj_ptr,
                                 const int32_t* adj_leaf, const int32_t* adj_pos,
                                 const int64_t* B_off, const int64_t* sig_off,
                                 const void* sigma, int sigma_fp32, int64_t n_leaf,
                                 hipStream_t s);

// ---- apply helpers -------------------------------------------------------------------------
// rows of Sigma_l per work item of the level product: kSigRows for a general Sigma_l (4
// waves, kSigRows / 4 rows each, lanes over columns), kSigRowsWave for a symmetric one
// (one wave, one row per lane).
constexpr int kSigRows = 16;
constexpr int kSigRowsWave = 64;
// longest mean row (columns) of the items given to the one-row-per-lane product: on
// 64^3 diffusion (rows of 721) lanes over columns ran 3x faster, on 48^3 elasticity
// (rows of 291-428) and 256^3 Poisson (rows of at most 386) one row per lane won
constexpr int kSigRowsMaxCols = 512;

// item: rows [a0, a1) of Sigma_l (leaf l) against the columns [c0, c1) of B_l; by_rows
// marks items of up to kSigRowsWave rows of symmetric Sigma blocks
struct SigmaLevelItems {
  int32_t count = 0;
  int32_t by_rows = 0;
  const int32_t* leaf = nullptr;
  const int32_t* c0 = nullptr;
  const int32_t* c1 = nullptr;
  const int32_t* a0 = nullptr;
  const int32_t* a1 = nullptr;
};
// (nv vectors: z_k = z + k ldz, e_k = e + k lde)
hipError_t launch_sigma_level(const SigmaLevelItems& it, const void* sigma, int sigma_fp32,
                              const int64_t* sig_off, const int64_t* B_off, const int32_t* B,
                              const double* z, double* e, int nv, int64_t ldz, int64_t lde,
                              hipStream_t s);
// z[r] += alpha * sum of e over the leaves adjacent to interface dof r (rows
// [row0, row0 + nrows))
hipError_t launch_level_adj(int64_t row0, int64_t nrows, int64_t n_leaf, const int64_t* adj_ptr,
                            const int32_t* adj_leaf, const int32_t* adj_pos, const int64_t* B_off,
                            const double* e, double* z, int nv, int64_t ldz, int64_t lde,
                            double alpha, hipStream_t s);

// gamma steps of unpreconditioned GMRES from zero on S~_t u = g for every system t of a
// level (the batch b gives each system's rows: n, vec_off) and nv vectors.  Basis vector
// j of vector k is V + (j nv + k) ld ((gamma + 1) * nv * ld doubles); per system and
// vector: beta, the (gamma + 1) x gamma Hessenberg matrix H, steps and stop flags
// (nv * count entries each).  start: beta = ||g||, v_0 = g / beta (g at z_k's rows).
// Between orth steps the caller writes w = S~ v_j into basis slot j + 1; orth(j):
// modified Gram-Schmidt, norm, happy-breakdown test, normalisation.  finish: the
// least-squares solution y and u = V y written over g.  gamma in 1..64.
constexpr int kGammaMaxSteps = 64;
// Levels whose systems are larger than one chunk use the chunked kernels (launch_gmc):
// work items of at most kGmChunk rows of one system, any number per system.
constexpr int kGmChunk = 4096;
struct GmArgs {
  int32_t count = 0, nitems = 0, nv = 0, gamma = 0;
  int64_t ld = 0;
  const int32_t* item_sys = nullptr;   // system of each work item
  const int64_t* item_b = nullptr;     // rows [item_b, item_e) (internal positions)
  const int64_t* item_e = nullptr;
  const int32_t* sys_first = nullptr;  // items of system m: sys_first[m] .. sys_first[m + 1]
  double* V = nullptr;                 // basis, as for the one-workgroup kernels
  double* beta = nullptr;
  double* H = nullptr;
  int32_t* steps = nullptr;
  int32_t* stop = nullptr;
  double* part = nullptr;              // nv * nitems * (gamma + 1) chunk partials
  double* coef = nullptr;              // nv * count * (gamma + 2): coefficients, then y
};
// op 0: start (g from zin); op 1: step j (after w = S~ v_j is in basis slot j + 1);
// op 2: finish (u into zout).  Same result as the one-workgroup kernels up to rounding
// (classical Gram-Schmidt twice instead of modified Gram-Schmidt).
hipError_t launch_gmc(const GmArgs& a, int op, int j, const double* zin, double* zout,
                      hipStream_t s);
hipError_t launch_gm_start(const DevBatch& b, int gamma, int nv, const double* z, int64_t ld,
                           double* V, double* beta, double* H, int32_t* steps, int32_t* stop,
                           hipStream_t s);
hipError_t launch_gm_orth(const DevBatch& b, int gamma, int nv, int j, int64_t ld, double* V,
                          const double* beta, double* H, int32_t* steps, int32_t* stop,
                          hipStream_t s);
hipError_t launch_gm_finish(const DevBatch& b, int gamma, int nv, int64_t ld, const double* V,
                            const double* beta, const double* H, const int32_t* steps,
                            double* z, hipStream_t s);

// ---- Krylov ----------------------------------------------------------------------------------
// Each call acts on nb_rhs independent right-hand sides: operand i of right-hand side
// i is its pointer plus i times the stride that follows it (sV, sw, ...).
int mdot_blocks(int64_t n);
// out[c] (c < ncols) = sum_r V[r + c ldv] w[r]  (deterministic two-pass); mode 0 store,
// mode 1 store sqrt (partial: nb_rhs * mdot_blocks(n) * ncols doubles)
hipError_t launch_mdot(int nb_rhs, const double* V, int64_t ldv, int64_t sV, int ncols,
                       const double* w, int64_t sw, int64_t n, double* partial, double* out,
                       int64_t so, int mode, hipStream_t s);
// w += sign * sum_c V[:, c] h[c]
hipError_t launch_gemv_acc(int nb_rhs, const double* V, int64_t ldv, int64_t sV, int ncols,
                           const double* h, int64_t sh, double sign, double* w, int64_t sw,
                           int64_t n, hipStream_t s);
// y = x / d[0]  (y = 0 when d[0] == 0)
hipError_t launch_scale_div(int nb_rhs, const double* x, int64_t sx, const double* d,
                            int64_t sd, double* y, int64_t sy, int64_t n, hipStream_t s);
// a[i] += b[i], i < k
hipError_t launch_small_add(int nb_rhs, double* a, int64_t sa, const double* b, int64_t sb,
                            int k, hipStream_t s);
// y = x + alpha * z  with alpha = num[0] / den[0] * sgn   (device scalars)
hipError_t launch_axpy_ratio(const double* x, const double* z, const double* num,
                             const double* den, double sgn, double* y, int64_t n, hipStream_t s);

}  // namespace rsd
