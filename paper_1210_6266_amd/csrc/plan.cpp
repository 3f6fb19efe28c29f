// Host analysis of the hierarchical decomposition: see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <numeric>
#include <utility>

namespace rsd {

namespace {

std::string fmt(const char* f, long long a = 0, long long b = 0, long long c = 0) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), f, a, b, c);
  return buf;
}

int64_t tiles_of(int64_t nt) { return nt * (nt + 1) / 2; }

}  // namespace

void layout_sym_batch(SymBatch* b, int chunk) {
  const int64_t TT = int64_t(kTile) * kTile;
  b->nt.assign(b->count, 0);
  b->tile_off.assign(b->count, 0);
  b->rslot_off.assign(b->count, 0);
  b->cstrip_base.assign(b->count, 0);
  b->item_mat.clear();
  b->item_J.clear();
  b->item_I0.clear();
  b->item_I1.clear();
  b->item_cslot.clear();
  b->cstrip_ptr.clear();
  int64_t off = 0, rs = 0, cs = 0, strips = 0;
  b->max_nt = 0;
  b->max_tiles = 0;
  for (int m = 0; m < b->count; ++m) {
    const int nt = (b->n[m] + kTile - 1) / kTile;
    b->nt[m] = nt;
    b->tile_off[m] = off;
    off += tiles_of(nt) * TT;
    b->rslot_off[m] = rs;
    rs += int64_t(nt) * (nt - 1) / 2;
    b->cstrip_base[m] = strips;
    b->max_nt = std::max(b->max_nt, nt);
    b->max_tiles = std::max<int64_t>(b->max_tiles, tiles_of(nt));
    for (int J = 0; J < nt; ++J) {
      b->cstrip_ptr.push_back(cs);
      for (int I0 = J; I0 < nt; I0 += chunk) {
        b->item_mat.push_back(m);
        b->item_J.push_back(J);
        b->item_I0.push_back(I0);
        b->item_I1.push_back(std::min(nt, I0 + chunk));
        b->item_cslot.push_back(cs++);
      }
    }
    strips += nt;
  }
  b->cstrip_ptr.push_back(cs);
  b->total_elems = off;
  b->num_cslots = cs;
  b->num_rslots = rs;
}

PlanError build_plan(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                     int32_t T, const int32_t* parent, const int32_t* dof_node, Plan* P,
                     std::string* msg) {
  // ---- validation of the CSR --------------------------------------------------------
  if (n <= 0) { *msg = "n must be positive"; return PlanError::kInvalid; }
  if (nnz < 0 || row_ptr == nullptr || (nnz > 0 && col_idx == nullptr)) {
    *msg = "null CSR array or negative nnz";
    return PlanError::kInvalid;
  }
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) {
    *msg = fmt("row_ptr[0] must be 0 and row_ptr[n] = nnz (%lld), got %lld", nnz, row_ptr[n]);
    return PlanError::kInvalid;
  }
  for (int32_t i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) { *msg = fmt("row_ptr decreases at row %lld", i); return PlanError::kInvalid; }
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t c = col_idx[k];
      if (c < 0 || c >= n) { *msg = fmt("column index %lld out of range in row %lld", c, i); return PlanError::kInvalid; }
      if (k > row_ptr[i] && c <= col_idx[k - 1]) {
        *msg = fmt("columns of row %lld not strictly increasing", i);
        return PlanError::kInvalid;
      }
    }
  }
  // structural symmetry
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col_idx[k];
      if (!std::binary_search(col_idx + row_ptr[j], col_idx + row_ptr[j + 1], i)) {
        *msg = fmt("K is not structurally symmetric: (%lld, %lld) present, transpose missing", i, j);
        return PlanError::kInvalid;
      }
    }
  }
  // ---- validation of the tree ----------------------------------------------------------
  if (T <= 0 || parent == nullptr || dof_node == nullptr) {
    *msg = "hierarchy needs num_nodes >= 1, parent and dof_node";
    return PlanError::kInvalid;
  }
  if (parent[0] != -1) { *msg = "parent[0] must be -1"; return PlanError::kInvalid; }
  for (int32_t t = 1; t < T; ++t)
    if (parent[t] < 0 || parent[t] >= t) {
      *msg = fmt("parent[%lld] = %lld must lie in [0, %lld)", t, parent[t], t);
      return PlanError::kInvalid;
    }
  for (int32_t i = 0; i < n; ++i)
    if (dof_node[i] < 0 || dof_node[i] >= T) {
      *msg = fmt("dof_node[%lld] = %lld out of range", i, dof_node[i]);
      return PlanError::kInvalid;
    }

  P->n = n;
  P->nnz = nnz;
  P->T = T;
  P->parent.assign(parent, parent + T);
  P->depth.assign(T, 0);
  P->children.assign(T, {});
  for (int32_t t = 1; t < T; ++t) {
    P->depth[t] = P->depth[parent[t]] + 1;
    P->children[parent[t]].push_back(t);
  }
  // Euler tour for ancestor tests (parent[t] < t: ids are topologically ordered)
  std::vector<int32_t> tin(T), tout(T);
  {
    int32_t clock = 0;
    std::vector<std::pair<int32_t, size_t>> st;
    st.push_back({0, 0});
    tin[0] = clock++;
    while (!st.empty()) {
      auto& top = st.back();
      if (top.second < P->children[top.first].size()) {
        const int32_t c = P->children[top.first][top.second++];
        tin[c] = clock++;
        st.push_back({c, 0});
      } else {
        tout[top.first] = clock++;
        st.pop_back();
      }
    }
  }
  auto anc = [&](int32_t a, int32_t b) {  // a is an ancestor of b, or a == b
    return tin[a] <= tin[b] && tout[b] <= tout[a];
  };
  // separability: every coupling joins nodes on one root-to-leaf path
  for (int32_t i = 0; i < n; ++i) {
    const int32_t a = dof_node[i];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t b = dof_node[col_idx[k]];
      if (!anc(a, b) && !anc(b, a)) {
        *msg = fmt("K couples dof %lld and dof %lld whose tree nodes are not on one root-to-leaf path "
                   "(node %lld)", i, col_idx[k], a);
        return PlanError::kNotSeparable;
      }
    }
  }

  // ---- orderings ---------------------------------------------------------------------
  std::vector<std::vector<int32_t>> owned(T);
  for (int32_t i = 0; i < n; ++i) owned[dof_node[i]].push_back(i);
  std::vector<int32_t> leaf_index(T, -1);
  P->leaf_node.clear();
  for (int32_t t = 0; t < T; ++t)
    if (P->children[t].empty()) {
      leaf_index[t] = int32_t(P->leaf_node.size());
      P->leaf_node.push_back(t);
    }
  const int32_t L = int32_t(P->leaf_node.size());
  P->perm.resize(n);
  P->iperm.resize(n);
  int64_t pos = 0;
  P->leaf_off.assign(L, 0);
  P->leaf_n.assign(L, 0);
  for (int32_t l = 0; l < L; ++l) {
    P->leaf_off[l] = pos;
    P->leaf_n[l] = int64_t(owned[P->leaf_node[l]].size());
    for (int32_t d : owned[P->leaf_node[l]]) P->perm[pos++] = d;
  }
  P->n_leaf = pos;
  std::vector<int32_t> inodes;
  for (int32_t t = 0; t < T; ++t)
    if (!P->children[t].empty() && !owned[t].empty()) inodes.push_back(t);
  std::stable_sort(inodes.begin(), inodes.end(),
                   [&](int32_t a, int32_t b) { return P->depth[a] > P->depth[b]; });
  P->iface_node = inodes;
  const int32_t NI = int32_t(inodes.size());
  P->iface_off.assign(NI, 0);
  P->iface_n.assign(NI, 0);
  P->level_iface_begin.clear();
  P->level_depth.clear();
  P->level_dof_begin.clear();
  P->level_dof_end.clear();
  for (int32_t s = 0; s < NI; ++s) {
    const int32_t t = inodes[s];
    if (s == 0 || P->depth[t] != P->depth[inodes[s - 1]]) {
      if (s > 0) P->level_dof_end.push_back(pos);
      P->level_iface_begin.push_back(s);
      P->level_depth.push_back(P->depth[t]);
      P->level_dof_begin.push_back(pos);
    }
    P->iface_off[s] = pos;
    P->iface_n[s] = int64_t(owned[t].size());
    for (int32_t d : owned[t]) P->perm[pos++] = d;
  }
  if (NI > 0) P->level_dof_end.push_back(pos);
  P->level_iface_begin.push_back(NI);
  const int32_t NL = int32_t(P->level_depth.size());
  for (int32_t i = 0; i < n; ++i) P->iperm[P->perm[i]] = i;
  const int64_t nB = n - P->n_leaf;
  P->dof_level.assign(nB, 0);
  for (int32_t q = 0; q < NL; ++q)
    for (int64_t d = P->level_dof_begin[q]; d < P->level_dof_end[q]; ++d)
      P->dof_level[d - P->n_leaf] = q;
  std::vector<int32_t> dof_iface(nB, -1);
  for (int32_t s = 0; s < NI; ++s)
    for (int64_t d = P->iface_off[s]; d < P->iface_off[s] + P->iface_n[s]; ++d)
      dof_iface[d - P->n_leaf] = s;

  // ---- K in internal order, with segment boundaries -----------------------------------
  P->prow.assign(n + 1, 0);
  P->pcol.resize(nnz);
  P->pmap.resize(nnz);
  P->segA.assign(n, 0);
  P->segB.assign(n, 0);
  P->segC.assign(n, 0);
  {
    std::vector<std::pair<int32_t, int64_t>> row;
    int64_t w = 0;
    for (int32_t r = 0; r < n; ++r) {
      const int32_t o = P->perm[r];
      row.clear();
      for (int64_t k = row_ptr[o]; k < row_ptr[o + 1]; ++k) row.push_back({P->iperm[col_idx[k]], k});
      std::sort(row.begin(), row.end());
      P->prow[r] = w;
      for (auto& e : row) {
        P->pcol[w] = e.first;
        P->pmap[w] = e.second;
        ++w;
      }
    }
    P->prow[n] = w;
    for (int32_t r = 0; r < n; ++r) {
      const int32_t* b = P->pcol.data() + P->prow[r];
      const int32_t* e = P->pcol.data() + P->prow[r + 1];
      P->segA[r] = (std::lower_bound(b, e, int32_t(P->n_leaf)) - P->pcol.data());
      if (r >= P->n_leaf) {
        const int32_t q = P->dof_level[r - P->n_leaf];
        const int32_t s = dof_iface[r - P->n_leaf];
        P->segB[r] = std::lower_bound(b, e, int32_t(P->level_dof_begin[q])) - P->pcol.data();
        P->segC[r] = std::lower_bound(b, e, int32_t(P->iface_off[s] + P->iface_n[s])) - P->pcol.data();
      } else {
        P->segB[r] = P->segC[r] = P->segA[r];
      }
    }
  }

  // ---- leaf boundaries and adjacency ---------------------------------------------------
  P->B_off.assign(L + 1, 0);
  P->B.clear();
  P->shell_off.assign(L + 1, 0);
  P->shell.clear();
  std::vector<int32_t> shell_idx;  // per internal leaf dof: index in its shell or -1
  shell_idx.assign(P->n_leaf, -1);
  for (int32_t l = 0; l < L; ++l) {
    std::vector<int32_t> bl;
    for (int64_t r = P->leaf_off[l]; r < P->leaf_off[l] + P->leaf_n[l]; ++r) {
      if (P->segA[r] < P->prow[r + 1]) {
        shell_idx[r] = int32_t(P->shell.size() - P->shell_off[l]);
        P->shell.push_back(int32_t(r - P->leaf_off[l]));
      }
      for (int64_t k = P->segA[r]; k < P->prow[r + 1]; ++k) bl.push_back(P->pcol[k]);
    }
    std::sort(bl.begin(), bl.end());
    bl.erase(std::unique(bl.begin(), bl.end()), bl.end());
    P->B.insert(P->B.end(), bl.begin(), bl.end());
    P->B_off[l + 1] = int64_t(P->B.size());
    P->shell_off[l + 1] = int64_t(P->shell.size());
  }
  P->adj_ptr.assign(nB + 1, 0);
  for (int32_t p : P->B) P->adj_ptr[p - P->n_leaf + 1]++;
  for (int64_t i = 0; i < nB; ++i) P->adj_ptr[i + 1] += P->adj_ptr[i];
  P->adj_leaf.assign(P->B.size(), 0);
  P->adj_pos.assign(P->B.size(), 0);
  {
    std::vector<int64_t> fill(P->adj_ptr.begin(), P->adj_ptr.end() - 1);
    for (int32_t l = 0; l < L; ++l)
      for (int64_t a = P->B_off[l]; a < P->B_off[l + 1]; ++a) {
        const int64_t p = P->B[a] - P->n_leaf;
        P->adj_leaf[fill[p]] = l;
        P->adj_pos[fill[p]] = int32_t(a - P->B_off[l]);
        ++fill[p];
      }
  }
  // Sigma layouts and the sparse pieces K_{l,B_l}, K_{B_l,l}
  P->sig_off.assign(L + 1, 0);
  P->w_off.assign(L + 1, 0);
  P->max_m = 0;
  P->sum_sigma_sq = 0;
  for (int32_t l = 0; l < L; ++l) {
    const int64_t m = P->B_off[l + 1] - P->B_off[l];
    const int64_t s = P->shell_off[l + 1] - P->shell_off[l];
    P->sig_off[l + 1] = P->sig_off[l] + m * m;
    P->w_off[l + 1] = P->w_off[l] + s * m;
    P->max_m = std::max<int32_t>(P->max_m, int32_t(m));
    P->sum_sigma_sq += m * m;
  }
  P->sig_total = P->sig_off[L];
  P->w_total = P->w_off[L];
  const int64_t nBflat = int64_t(P->B.size());
  P->kcol_ptr.assign(nBflat + 1, 0);
  P->krow_ptr.assign(nBflat + 1, 0);
  // K_{l,B}: columns of the leaf rows' interface suffix
  for (int32_t l = 0; l < L; ++l) {
    const int32_t* Bb = P->B.data() + P->B_off[l];
    const int32_t* Be = P->B.data() + P->B_off[l + 1];
    for (int64_t r = P->leaf_off[l]; r < P->leaf_off[l] + P->leaf_n[l]; ++r)
      for (int64_t k = P->segA[r]; k < P->prow[r + 1]; ++k) {
        const int64_t b = std::lower_bound(Bb, Be, P->pcol[k]) - Bb;
        P->kcol_ptr[P->B_off[l] + b + 1]++;
      }
  }
  for (int64_t i = 0; i < nBflat; ++i) P->kcol_ptr[i + 1] += P->kcol_ptr[i];
  P->kcol_row.assign(P->kcol_ptr[nBflat], 0);
  P->kcol_val.assign(P->kcol_ptr[nBflat], 0);
  {
    std::vector<int64_t> fill(P->kcol_ptr.begin(), P->kcol_ptr.end() - 1);
    for (int32_t l = 0; l < L; ++l) {
      const int32_t* Bb = P->B.data() + P->B_off[l];
      const int32_t* Be = P->B.data() + P->B_off[l + 1];
      for (int64_t r = P->leaf_off[l]; r < P->leaf_off[l] + P->leaf_n[l]; ++r)
        for (int64_t k = P->segA[r]; k < P->prow[r + 1]; ++k) {
          const int64_t f = P->B_off[l] + (std::lower_bound(Bb, Be, P->pcol[k]) - Bb);
          P->kcol_row[fill[f]] = int32_t(r - P->leaf_off[l]);
          P->kcol_val[fill[f]] = k;
          ++fill[f];
        }
    }
  }
  // K_{B,l}: the entries of interface row B_l[a] that fall in leaf l
  for (int32_t l = 0; l < L; ++l)
    for (int64_t a = P->B_off[l]; a < P->B_off[l + 1]; ++a) {
      const int32_t p = P->B[a];
      const int32_t* b = P->pcol.data() + P->prow[p];
      const int32_t* e = P->pcol.data() + P->segA[p];
      const int64_t lo = std::lower_bound(b, e, int32_t(P->leaf_off[l])) - b;
      const int64_t hi = std::lower_bound(b, e, int32_t(P->leaf_off[l] + P->leaf_n[l])) - b;
      P->krow_ptr[a + 1] = hi - lo;
    }
  for (int64_t i = 0; i < nBflat; ++i) P->krow_ptr[i + 1] += P->krow_ptr[i];
  P->krow_col.assign(P->krow_ptr[nBflat], 0);
  P->krow_val.assign(P->krow_ptr[nBflat], 0);
  for (int32_t l = 0; l < L; ++l)
    for (int64_t a = P->B_off[l]; a < P->B_off[l + 1]; ++a) {
      const int32_t p = P->B[a];
      int64_t w = P->krow_ptr[a];
      for (int64_t k = P->prow[p]; k < P->segA[p]; ++k) {
        const int32_t c = P->pcol[k];
        if (c < P->leaf_off[l] || c >= P->leaf_off[l] + P->leaf_n[l]) continue;
        const int32_t si = shell_idx[c];
        if (si < 0) {
          *msg = "internal error: interface row couples to a non-shell interior dof";
          return PlanError::kInvalid;
        }
        P->krow_col[w] = si;
        P->krow_val[w] = k;
        ++w;
      }
    }

  // ---- apply schedule: Sigma products per level --------------------------------------
  P->level_sigma.assign(NL, {});
  P->sum_sigma_apply = 0;
  for (int32_t q = 0; q < NL; ++q)
    for (int32_t l = 0; l < L; ++l) {
      const int32_t* Bb = P->B.data() + P->B_off[l];
      const int32_t* Be = P->B.data() + P->B_off[l + 1];
      const int32_t r0 = int32_t(std::lower_bound(Bb, Be, int32_t(P->level_dof_begin[q])) - Bb);
      const int32_t r1 = int32_t(std::lower_bound(Bb, Be, int32_t(P->level_dof_end[q])) - Bb);
      if (r1 > r0 && r0 > 0) {
        P->level_sigma[q].push_back({l, r0, r1});
        P->sum_sigma_apply += int64_t(r1 - r0) * r0;
      }
    }

  // ---- dense batches ---------------------------------------------------------------
  P->leaf_batch = SymBatch();
  P->leaf_batch.count = L;
  P->leaf_batch.n.resize(L);
  P->leaf_batch.vec_off.resize(L);
  P->sum_leaf_sq = 0;
  P->leaf_flops = 0;
  P->max_leaf = 0;
  for (int32_t l = 0; l < L; ++l) {
    P->leaf_batch.n[l] = int32_t(P->leaf_n[l]);
    P->leaf_batch.vec_off[l] = P->leaf_off[l];
    P->sum_leaf_sq += P->leaf_n[l] * P->leaf_n[l];
    P->leaf_flops += double(P->leaf_n[l]) * P->leaf_n[l] * P->leaf_n[l];
    P->max_leaf = std::max<int32_t>(P->max_leaf, int32_t(P->leaf_n[l]));
  }
  layout_sym_batch(&P->leaf_batch, 8);
  P->level_batch.assign(NL, SymBatch());
  P->sum_iface_sq = 0;
  P->iface_flops = 0;
  P->max_iface = 0;
  for (int32_t q = 0; q < NL; ++q) {
    SymBatch& b = P->level_batch[q];
    b.count = P->level_iface_begin[q + 1] - P->level_iface_begin[q];
    for (int32_t s = P->level_iface_begin[q]; s < P->level_iface_begin[q + 1]; ++s) {
      b.n.push_back(int32_t(P->iface_n[s]));
      b.vec_off.push_back(P->iface_off[s]);
      P->sum_iface_sq += P->iface_n[s] * P->iface_n[s];
      P->iface_flops += double(P->iface_n[s]) * P->iface_n[s] * P->iface_n[s];
      P->max_iface = std::max<int32_t>(P->max_iface, int32_t(P->iface_n[s]));
    }
    layout_sym_batch(&b, 8);
  }
  return PlanError::kOk;
}

}  // namespace rsd
