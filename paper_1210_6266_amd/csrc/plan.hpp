// Host analysis of the hierarchical decomposition (no device code).
//
// Given the CSR structure of K and the tree of Section 2 (parent[], dof_node[]),
// this validates the input and derives every index structure the device path
// needs:
//   * the internal dof order [leaf interiors in leaf-id order | interface dofs of
//     the internal nodes, deepest level first]; within a block, caller order;
//   * K in that order (CSR, columns sorted) with a map back to the caller's value
//     positions, and per-row segment boundaries: because columns are sorted and
//     the order is [leaves | deeper interfaces | this interface | shallower], the
//     couplings the apply needs are contiguous row segments;
//   * B_l, the interface dofs coupled to the interior of leaf l (sorted, so the
//     dofs of each interface level are contiguous), and for every interface dof
//     the list of (leaf, position in B_l) pairs -- these define C_t, the leaves
//     coupled to interface t (the generalised V-hat of Section 3.2);
//   * the sparse pieces K_{l,B_l} and K_{B_l,l} used to form Sigma_l;
//   * dense tile layouts and product work lists for the batched blocks.
#pragma once

#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

namespace rsd {

constexpr int kTile = 64;  // dense blocks are stored as kTile x kTile tiles
constexpr int kSymB = 4;   // symmetric products work on kSymB x kSymB blocks of tiles
constexpr int kEllSlice = 64;  // rows per ELL slice (one wave)

// A batch of symmetric matrices stored as packed lower tiles (tile (I, J) with
// I >= J; column-major kTile x kTile each; diagonal tiles hold both triangles).
// A std::vector whose resize() leaves new elements of a trivial type uninitialised.  The
// analysis' large arrays are written in full by their (parallel) producers, which then also
// take the first-touch page faults, instead of a serial zero fill before them.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind { using other = NoInitAlloc<U>; };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept { ::new (static_cast<void*>(p)) U; }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) { ::new (static_cast<void*>(p)) U(std::forward<A>(a)...); }
};
template <typename T>
using hvec = std::vector<T, NoInitAlloc<T>>;

struct SymBatch {
  int32_t count = 0;
  std::vector<int32_t> n;          // order of each matrix
  std::vector<int32_t> nt;         // tiles per side
  std::vector<int64_t> tile_off;   // element offset of tile (0,0)
  std::vector<int64_t> vec_off;    // internal dof of the matrix's first row
  int64_t total_elems = 0;
  int32_t max_nt = 0;
  int64_t max_tiles = 0;           // max over matrices of nt (nt + 1) / 2
  // symmetric product work: item = (matrix, block row BI, block column BJ <= BI) over
  // kSymB x kSymB tiles; the items of matrix m are item_base[m] + tri(BI) + BJ
  std::vector<int32_t> item_mat, item_BI, item_BJ;
  std::vector<int64_t> item_base;
  int64_t num_items = 0;
};

struct LevelSigmaItem {            // rows r0..r1 of Sigma_l (positions in B_l) of one leaf
  int32_t leaf, r0, r1;
};

struct Plan {
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t T = 0;
  std::vector<int32_t> parent, depth;
  std::vector<std::vector<int32_t>> children;

  // leaves (true sub-domains), in node-id order
  std::vector<int32_t> leaf_node;            // leaf index -> node id
  std::vector<int64_t> leaf_off, leaf_n;     // internal dof range of each leaf interior
  std::vector<int32_t> leaf_inner;           // its dofs coupled to no interface dof: they
                                             // come first, the shell (the rest) last
  int64_t n_leaf = 0;                        // sum of leaf sizes: first interface dof

  // internal nodes that own interface dofs, in processing order
  std::vector<int32_t> iface_node;           // iface index -> node id
  std::vector<int64_t> iface_off, iface_n;
  std::vector<int32_t> level_iface_begin;    // per level (deepest first): iface range
  std::vector<int32_t> level_depth;
  std::vector<int64_t> level_dof_begin, level_dof_end;
  std::vector<int32_t> dof_level;            // per interface dof (index - n_leaf): level

  // ordering
  hvec<int32_t> perm, iperm;          // internal -> caller, caller -> internal

  // K in internal order: row pointers here; the columns, the map to the caller's
  // value positions and the row segments are built on the device from perm/iperm
  hvec<int64_t> prow;
  // the same rows as sliced ELL for the SpMV: slices of kEllSlice consecutive rows,
  // slice s padded to its longest row; entry k of row r at ell_off[s] + k kEllSlice + r % kEllSlice
  std::vector<int64_t> ell_off;
  std::vector<int32_t> skel_lvl_begin;       // per interface dof: first dof of its level
  std::vector<int32_t> skel_own_end;         // per interface dof: end of its node's dofs

  // leaf boundaries B_l (internal interface dof indices)
  std::vector<int64_t> B_off;                // per leaf, size num_leaves + 1
  hvec<int32_t> B;
  std::vector<int64_t> sig_off;              // element offset of Sigma_l (m_l x m_l)
  int64_t sig_total = 0;
  // adjacency of interface dofs: (leaf, position in B_l), sorted by leaf
  std::vector<int64_t> adj_ptr;              // size n - n_leaf + 1
  std::vector<int32_t> adj_leaf, adj_pos;

  // Sigma_l = K_{B l} K_ll^{-1} K_{l B}:
  //   shell_l = interior rows of l coupled to B_l (local indices)
  std::vector<int64_t> shell_off;
  hvec<int32_t> shell;
  //   columns of K_{l B}: per flat column (B_off[l] + b): (local row j, caller position)
  std::vector<int64_t> kcol_ptr;
  hvec<int32_t> kcol_row;
  hvec<int64_t> kcol_val;
  //   rows of K_{B l}: per flat row (B_off[l] + a): (shell index, caller position)
  std::vector<int64_t> krow_ptr;
  hvec<int32_t> krow_col;
  hvec<int64_t> krow_val;
  std::vector<int64_t> w_off;                // element offset of W_l (shell_l x m_l)
  int64_t w_total = 0;

  // apply: Sigma products per level (processing order)
  std::vector<std::vector<LevelSigmaItem>> level_sigma;       // cols 0..r0: deeper levels
  std::vector<std::vector<LevelSigmaItem>> level_sigma_own;   // cols r0..r1: the level itself

  SymBatch leaf_batch;
  std::vector<SymBatch> level_batch;         // per level

  // totals for roofline accounting
  bool coupled = false;                      // build_plan_couplings has run
  int64_t sum_leaf_sq = 0, sum_iface_sq = 0, sum_sigma_sq = 0, sum_sigma_apply = 0;
  double leaf_flops = 0.0, iface_flops = 0.0;
  int32_t max_leaf = 0, max_iface = 0, max_m = 0;
};

enum class PlanError { kOk = 0, kInvalid = 1, kNotSeparable = 2 };

// Builds the plan from host arrays (multithreaded).  Returns kOk, or an error with *msg.
// The analysis in two parts.  build_plan validates K and the hierarchy and computes the
// ordering, the internal row pointers, the ELL layout and the dense batches (all the first
// device work needs); build_plan_couplings then adds, from the same (validated) CSR, the
// per-leaf coupling blocks, the adjacency lists and the Sigma layout and apply schedule
// (coupled = true).  A set-up runs the second part on the host while the device inverts
// the sub-domains.
PlanError build_plan(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                     int32_t num_nodes, const int32_t* parent, const int32_t* dof_node,
                     Plan* plan, std::string* msg);
PlanError build_plan_couplings(const int64_t* row_ptr, const int32_t* col_idx, Plan* plan,
                               std::string* msg);

// Tile layout and symmetric-product work items of a batch.
void layout_sym_batch(SymBatch* b);

}  // namespace rsd
