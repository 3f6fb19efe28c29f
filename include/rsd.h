/*
 * rsd.h -- C ABI of the MI355X Recursive Schur Decomposition (RSD) solver library.
 *
 * The library solves K u = f for a sparse finite-element matrix K -- symmetric
 * positive definite by default, or non-symmetric with a symmetric sparsity pattern
 * (rsd_options.symmetric = 0) -- with a Krylov method preconditioned by RSD
 * (Sampath, Philip, Allu, Simunovic, "Recursive Schur Decomposition"; the
 * problem statement opens Section 3).  The caller describes K in CSR form and
 * the hierarchical domain decomposition of Section 2 as a tree whose leaves
 * are the true sub-domains and whose internal nodes each stand for the
 * interface between their children.
 *
 * Conventions for every entry point
 *   - Every call returns an rsd_status; nothing throws or aborts across the ABI.
 *   - Array arguments are plain pointers.  Unless stated otherwise they are
 *     HIP device pointers owned by the caller; the library never frees them and
 *     keeps no reference after the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *     device work of a call is enqueued on it, in order.  Calls on one handle are
 *     ordered even across streams: each call records an event of the handle on its
 *     stream when it returns, and a call on a different stream first makes its stream
 *     wait for that event (every call on a handle shares the handle's work buffers).
 *     Calls made while their stream is being captured into a graph skip both steps:
 *     inside a capture the caller orders them.
 *   - Vectors are FP64, column-major n x nrhs blocks with leading dimension
 *     ld >= n, in the caller's dof numbering.
 *   - Handles are not thread-safe; distinct handles may be used concurrently (each
 *     holds its own streams, events and device memory).
 *   - Process-wide caches: device blocks and pinned staging buffers released by
 *     handles, and the auxiliary streams and timing events of destroyed handles, are
 *     kept for the next handle (up to 48 GiB of device blocks per device) until
 *     rsd_release_cache.
 */
#ifndef RSD_H_
#define RSD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSD_OK = 0,
  RSD_ERR_INVALID_ARGUMENT = 1,  /* malformed CSR / tree / map, bad sizes or pointers     */
  RSD_ERR_MAP_NOT_SEPARABLE = 2, /* K couples two dofs whose tree nodes are not on one
                                    root-to-leaf path (e.g. two different leaves)        */
  RSD_ERR_NOT_SPD = 3,           /* a sub-domain or interface block has a pivot <= 0 or
                                    a non-finite pivot (symmetric = 0: a zero or
                                    non-finite pivot); rsd_last_error names the block     */
  RSD_ERR_NOT_CONVERGED = 4,     /* Krylov reached maxit; x holds the last iterate       */
  RSD_ERR_BREAKDOWN = 5,         /* NaN/Inf in the Krylov recurrence                     */
  RSD_ERR_OUT_OF_MEMORY = 6,     /* device allocation failed                             */
  RSD_ERR_DEVICE = 7,            /* any other HIP runtime error                          */
  RSD_ERR_UNSUPPORTED = 8        /* valid request the library does not implement         */
} rsd_status;

typedef struct rsd_ctx* rsd_handle;

/* Sparse matrix K (n x n) in CSR form: row_ptr[n+1] (row_ptr[0] = 0,
 * non-decreasing, row_ptr[n] = nnz), col_idx[nnz] strictly increasing within a
 * row, values[nnz].  The sparsity pattern must be symmetric (checked); the values
 * must be too unless rsd_options.symmetric = 0 (not checked). */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* values;
} rsd_csr;

/* The sub-domain hierarchy of Section 2 (Fig. 1): num_nodes tree nodes with
 * parent[0] = -1 and 0 <= parent[t] < t for t > 0 (so ids are topologically
 * ordered).  A node without children is a true sub-domain (leaf).  dof_node[i]
 * (n entries) names the node that owns dof i: a leaf for a dof in the interior
 * of that true sub-domain, an internal node for a dof on the interface that
 * node represents.  Any node may own no dofs. */
typedef struct {
  int32_t num_nodes;
  const int32_t* parent;
  const int32_t* dof_node;
} rsd_hierarchy;

/* Storage / arithmetic precision of a class of dense blocks.  FP16 and BF16 apply to
 * the sub-domain inverses only (leaf_prec): they are formed in FP32 (the Sigma blocks
 * too, from the FP32 inverses) and stored in 16 bits for the applies, whose products
 * accumulate in FP32; the outer FP64 Krylov iteration refines the result. */
enum { RSD_PREC_FP64 = 0, RSD_PREC_FP32 = 1, RSD_PREC_FP16 = 2, RSD_PREC_BF16 = 3 };

/* How the interface systems S~_t u = g of eq. (schur) are solved inside an apply:
 *   RSD_IFACE_DENSE  -- exactly, with the explicit inverse of the assembled S~_t
 *                       (the limit of infinitely many inner iterations);
 *   RSD_IFACE_GAMMA  -- inexactly, as in the paper's experiments (Section 3.1 and
 *                       Section 4): gamma steps of unpreconditioned GMRES from zero
 *                       on S~_t, at every level (happy breakdown stops a system early);
 *   RSD_IFACE_HYBRID -- gamma steps at the levels whose largest interface has more
 *                       than dense_max dofs, exact solves at the others.
 * The preconditioner is then a non-linear function of r: use FGMRES. */
enum { RSD_IFACE_DENSE = 0, RSD_IFACE_GAMMA = 1, RSD_IFACE_HYBRID = 2 };

/* Right-hand side g of each interface system in the recursion of Alg. 2.  The paper
 * writes it for a strip, where an interface couples only to the two sub-domain
 * interiors beside it.  In 3-D an interface also couples directly to deeper interface
 * dofs:
 *   RSD_COUPLING_FULL (default) -- g = f_I - K_{I,V} v over every dof V of the subtree
 *     below the interface (sub-domain interiors and deeper interfaces): the block
 *     elimination of the Schur complement equation with the recursive solution in
 *     place of the exact one;
 *   RSD_COUPLING_LEAF_ONLY -- only the couplings to sub-domain interiors (the strip
 *     formula taken literally); it differs from FULL only where deeper interface dofs
 *     couple to the interface (never in a strip, never with one level).            */
enum { RSD_COUPLING_FULL = 0, RSD_COUPLING_LEAF_ONLY = 1 };

typedef struct {
  int32_t struct_size;   /* sizeof(rsd_options) */
  int32_t leaf_prec;     /* inverses of the true sub-domain matrices K_ll              */
  int32_t sigma_prec;    /* leaf boundary Schur blocks Sigma_l = K_Bl K_ll^-1 K_lB      */
  int32_t iface_prec;    /* inverses of the non-root interface Schur complements       */
  int32_t root_prec;     /* inverse of the root interface Schur complement             */
  int32_t host_pointers; /* 0: csr and hierarchy arrays are device pointers;
                            1: they are host pointers (values are copied to the device) */
  int32_t timing;        /* 1: time every kernel class with HIP events (rsd_get_stats) */
  int32_t iface_mode;    /* RSD_IFACE_DENSE (default), RSD_IFACE_GAMMA or RSD_IFACE_HYBRID  */
  int32_t gamma;         /* inner GMRES steps per interface solve (1..64; gamma modes)      */
  int32_t dense_max;     /* RSD_IFACE_HYBRID: largest interface solved exactly              */
  int32_t graphs;        /* 1: replay each preconditioner application from a HIP graph
                            captured on first use (one per number of columns, 1..8; the
                            one-column graph already during rsd_setup, while the device
                            runs the set-up); ignored while a class of the applications
                            is timed (below)                                              */
  int32_t autotune;      /* 1: before the first application to 2..8 columns, time the
                            candidate numbers of vectors per pass (1, 2, 4) of every dense
                            batch's symmetric product, each with one workgroup per item
                            and as a persistent work-queue launch, on the handle's own
                            blocks and keep the fastest; and on the first set-ups of
                            each batch shape, time in turn the inversion schedules
                            (look-ahead or serial steps;
                            128 x 128 or 256 x 256 update super-tiles for BF16-split
                            batches) and keep the fastest.  Results do not depend on any
                            choice; the choices are remembered per process for batches of
                            the same shape                                                   */
  int32_t symmetric;     /* 1: K is symmetric (sub-domains inverted by symmetric sweeps).
                            0: K may be non-symmetric (pattern still symmetric): dense
                            sub-domain inverses by Gauss-Jordan with partial pivoting (at
                            most 2,048 dofs, leaf_prec FP64 or FP32) and iface_mode GAMMA,
                            i.e. every interface solved by inner GMRES steps              */
  int32_t g_coupling;    /* RSD_COUPLING_FULL (default) or RSD_COUPLING_LEAF_ONLY          */
  int32_t bf16_split;    /* FP32 blocks (leaf_prec, iface_prec FP32 or 16-bit): 1 (default)
                            runs their inversions' trailing updates on the BF16 matrix cores,
                            each FP32 operand split exactly into three BF16 parts and six
                            products accumulated in FP32 (errors of FP32 order); 0 on the
                            FP32 matrix cores.  The FP64 blocks are unaffected.             */
  int32_t sym_form;      /* symmetric products of the applies: 0 (default) one workgroup
                            per 4 x 4 tile block, unless the autotuner picks the persistent
                            form for a batch; 1 always the persistent work-queue form
                            (resident workgroups take the blocks from a counter).  Same
                            results either way                                               */
  int32_t timing_classes; /* with timing = 1: bit mask of the kernel classes timed (bit c for
                            class c of the RSD_T_* list below; the others report 0 ms and
                            add no events between launches); 0 (default): every class.
                            Graphs stay off while a class that the applications launch
                            (leaf or interface apply, coupling, SpMV, Krylov) is timed      */
  /* Optional device allocator for the handle's memory (set both or neither; default
     NULL: the library's own cache of hipMalloc blocks).  dev_alloc(bytes, alloc_ctx)
     returns device memory on the current device, or NULL (RSD_ERR_OUT_OF_MEMORY);
     dev_free(p, alloc_ctx) returns a block once no queued work of the handle uses it.  Both are
     called on the thread that calls rsd_setup, rsd_update_values, rsd_apply, rsd_spmv,
     rsd_solve (workspace for more columns) and rsd_destroy.                         */
  void* (*dev_alloc)(size_t bytes, void* alloc_ctx);
  void (*dev_free)(void* p, void* alloc_ctx);
  void* alloc_ctx;
} rsd_options;

/* Fills *opt with the defaults: all FP64, device pointers, no timing, exact
 * (dense) interface solves, gamma = 8, dense_max = 32768, graphs on, autotune on,
 * symmetric, full interface right-hand sides, BF16-split FP32 updates. */
void rsd_options_default(rsd_options* opt);

enum { RSD_SOLVER_FGMRES = 0, RSD_SOLVER_PCG = 1 };

typedef struct {
  int32_t method;   /* RSD_SOLVER_FGMRES (right-preconditioned, flexible) or RSD_SOLVER_PCG */
  int32_t restart;  /* FGMRES restart length m (1..256)                                       */
  int32_t maxit;    /* maximum number of Krylov iterations per right-hand side               */
  double rtol;      /* stop when ||b - K x||_2 <= rtol ||b||_2 (true residual)               */
  int32_t use_x0;   /* 1: x holds the initial guess on entry; 0: x0 = 0                       */
} rsd_solve_options;

typedef struct {
  int32_t iterations; /* Krylov iterations taken                                        */
  double relres;      /* final true relative residual ||b - K x|| / ||b||               */
  int32_t status;     /* rsd_status of this right-hand side                             */
} rsd_solve_info;

/* Counts produced by the host analysis of the hierarchy (rsd_analyze) and the
 * per-apply / per-setup algorithmic work used for roofline accounting. */
typedef struct {
  int32_t num_leaves;
  int32_t num_levels;           /* interface levels (internal-node depths)              */
  int32_t max_leaf_dofs;
  int32_t max_iface_dofs;
  int32_t max_boundary_dofs;    /* max over leaves of m_l = |B_l|                        */
  int64_t leaf_dofs;            /* dofs in leaf interiors                              */
  int64_t skeleton_dofs;        /* dofs on interfaces                                  */
  int64_t sum_leaf_sq;          /* sum_l n_l^2                                         */
  int64_t sum_iface_sq;         /* sum_t n_t^2                                         */
  int64_t sum_sigma_apply;      /* entries of the Sigma_l blocks read by one apply     */
  int64_t sum_sigma_sq;         /* sum_l m_l^2                                         */
  double leaf_inverse_flops;    /* sum_l n_l^3 (symmetric in-place inversion)          */
  double iface_inverse_flops;   /* sum_t n_t^3                                         */
} rsd_analysis;

/* Host-only analysis of (csr structure, hierarchy): validates the input
 * exactly as rsd_setup does and reports the counts above.  All pointers are
 * HOST pointers; csr->values may be NULL.  Makes no HIP call.
 * Errors: RSD_ERR_INVALID_ARGUMENT, RSD_ERR_MAP_NOT_SEPARABLE. */
rsd_status rsd_analyze(const rsd_csr* csr, const rsd_hierarchy* hier, rsd_analysis* out);

/* Set-up of the RSD preconditioner (Section 3).
 *  1. Host analysis: validates the CSR, the tree and dof_node; checks that the
 *     decomposition separates K (every non-zero K_ij joins dofs whose nodes lie
 *     on one root-to-leaf path -- the block structure of eq. (matPart)); orders
 *     dofs as [leaf interiors | interfaces, deepest level first].  The check of
 *     the pattern's symmetry and the per-sub-domain coupling blocks follow on the
 *     host while the device inverts the sub-domains (a non-symmetric pattern is
 *     reported once that queued work has finished).
 *  2. Device: extracts every true sub-domain matrix K_ll and inverts it exactly
 *     (the direct sub-domain solve of Section 3.1), forms the leaf boundary
 *     blocks Sigma_l = K_Bl K_ll^-1 K_lB, assembles for every internal node t the
 *     interface operator of Alg. 1,
 *        S~_t = K_tt - sum over leaves l of subtree(t) coupled to I_t of Sigma_l[I_t, I_t],
 *     and inverts it (the exact interface solve: the limit of the paper's inner
 *     Krylov iteration).  Dense blocks use the precisions in *opt.
 * csr / hier: device pointers unless opt->host_pointers = 1.  opt may be NULL
 * (defaults).  On success *out receives a new handle; on failure *out = NULL and
 * rsd_last_error(NULL) describes the error (thread-local).  Synchronises `stream`
 * after copying the structure to the host (device pointers) and at the end (pivot
 * status read-back).
 * Errors: INVALID_ARGUMENT, MAP_NOT_SEPARABLE, NOT_SPD, OUT_OF_MEMORY, DEVICE. */
rsd_status rsd_setup(const rsd_csr* csr, const rsd_hierarchy* hier, const rsd_options* opt,
                     void* stream, rsd_handle* out);

/* z = M^{-1} r: one application of the RSD preconditioner (Alg. 2) to each of
 * nrhs columns: all sub-domain solves, then the interface levels from the
 * deepest to the root (right-hand side g of eq. (schur), interface solve,
 * back-substitution of eq. (backSub) onto the adjacent sub-domains), then the
 * final sub-domain solves.  r and z are device arrays (n x nrhs, ld >= n) and
 * must not overlap.  Up to 8 columns go through each step together (each dense
 * block and K read once per 4 columns, the SpMV slots once per 8); every column
 * gets bitwise the result it gets alone.  nrhs = 0 is a no-op.  Asynchronous on
 * `stream`.  Errors: INVALID_ARGUMENT, DEVICE. */
rsd_status rsd_apply(rsd_handle h, int32_t nrhs, const double* r, int64_t ldr, double* z,
                     int64_t ldz, void* stream);

/* rsd_apply for callers that cannot allocate device memory: code being captured into
 * a HIP graph, tight serving loops, harnesses that forbid hipMalloc.  Same arguments and
 * results as rsd_apply (each column bitwise what rsd_apply gives it), but every work
 * buffer of the application comes from one static device area of 256 MiB per GPU
 * (allocated with the library's code on each GPU it runs on and held until the process
 * ends) instead of the handle's memory: the call allocates nothing, replays no graph,
 * runs no autotuning and never waits on the host.  Columns go through in passes of up to
 * 8, fewer when 8 do not fit the area.
 * Ordering: all calls on one GPU share its area.  The library orders them (each call
 * records a per-GPU event; a call on another stream first waits for it), except calls
 * made while their stream is being captured into a graph: such calls, and every replay
 * of the graphs they were captured into, race with any other use of the area on that GPU
 * that can overlap them -- the caller must serialise those.
 * Errors: INVALID_ARGUMENT (as rsd_apply; the handle's device is not current; a single
 * column of this handle needs more than the 256 MiB area, rsd_last_error gives the
 * size), DEVICE. */
rsd_status rsd_apply_noalloc(rsd_handle h, int32_t nrhs, const double* r, int64_t ldr,
                             double* z, int64_t ldz, void* stream);

/* y = K x with the handle's matrix (the Krylov MatVec), x and y device arrays
 * (n x nrhs), not overlapping.  Asynchronous.  Errors: INVALID_ARGUMENT, DEVICE. */
rsd_status rsd_spmv(rsd_handle h, int32_t nrhs, const double* x, int64_t ldx, double* y,
                    int64_t ldy, void* stream);

/* Solves K x = b for each of nrhs columns with RSD-preconditioned Krylov
 * iterations (Section 3: GMRES with RSD as preconditioner; here right-
 * preconditioned flexible GMRES(m), or PCG), in FP64, to the true relative
 * residual ||b - K x||_2 <= rtol ||b||_2.  b and x are device arrays; info is a
 * HOST array of nrhs entries (may be NULL).  opt may be NULL (FGMRES(30),
 * rtol 1e-10, maxit 500, x0 = 0).  FGMRES advances groups of up to 8 columns
 * in lockstep (one preconditioner application and one SpMV for the group per
 * iteration, one host synchronisation of `stream` per iteration); each column
 * keeps its own Krylov basis, stops on its own criterion and gets bitwise the
 * iterate and info of a solve alone.  PCG takes the columns one at a time.
 * Returns the worst per-column status: NOT_CONVERGED (x holds the last
 * iterate), BREAKDOWN, or OK. */
rsd_status rsd_solve(rsd_handle h, int32_t nrhs, const double* b, int64_t ldb, double* x,
                     int64_t ldx, const rsd_solve_options* opt, rsd_solve_info* info,
                     void* stream);

/* Replaces the values of K (same sparsity pattern, `values` in the caller's CSR
 * order, device pointer unless the handle was set up with host_pointers = 1)
 * and recomputes every dense block, skipping the host analysis.
 * Errors: INVALID_ARGUMENT, NOT_SPD, DEVICE. */
rsd_status rsd_update_values(rsd_handle h, const double* values, void* stream);

/* Per-handle statistics.  Times are accumulated device times in milliseconds
 * measured with HIP events when the handle was created with timing = 1 (for the
 * classes selected by timing_classes). */
enum {
  RSD_T_SETUP_EXTRACT = 0, /* value gathers, dense block extraction                    */
  RSD_T_LEAF_INVERSE,      /* batched in-place inversion of the K_ll (all kernels)    */
  RSD_T_LEAF_UPDATE,       /*   of which: the MFMA trailing-update kernels            */
  RSD_T_SIGMA,             /* Sigma_l blocks                                          */
  RSD_T_IFACE_ASSEMBLY,    /* S~_t assembly (extend-add)                              */
  RSD_T_IFACE_INVERSE,     /* batched inversion of the S~_t (all kernels)             */
  RSD_T_IFACE_UPDATE,      /*   of which: MFMA update kernels, non-root levels        */
  RSD_T_ROOT_UPDATE,       /*   of which: MFMA update kernels, root level             */
  RSD_T_LEAF_APPLY,        /* batched symmetric products with K_ll^-1                 */
  RSD_T_IFACE_APPLY,       /* batched symmetric products with S~_t^-1                 */
  RSD_T_COUPLING,          /* sparse couplings, Sigma products, g assembly            */
  RSD_T_SPMV,              /* global SpMV                                             */
  RSD_T_KRYLOV,            /* dots, orthogonalisation, vector updates                 */
  RSD_T_PERMUTE,           /* caller <-> internal dof ordering                        */
  RSD_T_COUNT
};
typedef struct {
  rsd_analysis analysis;
  double time_ms[RSD_T_COUNT];
  int64_t launches[RSD_T_COUNT];
  double host_analysis_ms; /* host time of the analysis (step 1 of rsd_setup;
                              its second part overlaps the device's set-up)     */
  int64_t device_bytes;    /* device memory held by the handle                */
  double setup_wall_ms[4]; /* last rsd_setup / rsd_update_values, host wall time:
                              [0] structure copy to the host and the analysis'
                                  first part, [1] device allocation and index
                                  upload, [2] enqueueing the dense set-up and the
                                  analysis' second part, [3] waiting for the device
                                  and releasing scratch memory                 */
  int32_t vec_pass[8];     /* vectors per pass of the symmetric products chosen by the
                              autotuner (0: not tuned): [0] sub-domains, then the dense
                              interface levels, deepest first                  */
  int32_t setup_variant[8]; /* inversion schedule of the last set-up, same batches:
                              0 none, 1 look-ahead, 2 serial steps, 3 look-ahead with
                              256 x 256 update super-tiles, 4 serial with them (the
                              set-up autotuner's choice, or the candidate it was timing;
                              every variant gives the same bits).  With symmetric K the
                              dense levels other than the shallowest one are inverted
                              beside it on a second stream, in serial steps (2 or 4) */
  int32_t sym_persist[8];   /* the same batches: 1 where the autotuner chose the
                              persistent work-queue form of the symmetric products
                              (resident workgroups taking items from a counter)  */
} rsd_stats;

/* Copies the handle's statistics (synchronises `stream` when timing is on).
 * reset = 1 clears the accumulated times and launch counts afterwards. */
rsd_status rsd_get_stats(rsd_handle h, rsd_stats* out, int32_t reset, void* stream);

/* Frees the handle and its device memory (after its pending work completes: the host
 * waits for the handle's last call, not for the whole device). */
void rsd_destroy(rsd_handle h);

/* Returns to the HIP runtime the device blocks and pinned host buffers that destroyed
 * handles left in the library's caches, and destroys the idle auxiliary streams and
 * timing events, on
 * `device` (every device when device < 0).  Memory and streams held by live handles are
 * not touched.  Safe to call at any time from any thread; later set-ups refill the caches. */
void rsd_release_cache(int32_t device);

/* Message of the last error on h; with h = NULL, of the last failed rsd_setup
 * or rsd_analyze on the calling thread.  Never NULL. */
const char* rsd_last_error(rsd_handle h);

#ifdef __cplusplus
}
#endif
#endif /* RSD_H_ */
