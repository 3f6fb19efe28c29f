// Host analysis of the hierarchical decomposition: see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <functional>
#include <numeric>
#include <thread>
#include <utility>

namespace rsd {

namespace {

std::string fmt(const char* f, long long a = 0, long long b = 0, long long c = 0) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), f, a, b, c);
  return buf;
}

int64_t tiles_of(int64_t nt) { return nt * (nt + 1) / 2; }

int num_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return int(std::max(1u, std::min(16u, hc)));
}

// Runs fn(lo, hi, worker) over [0, count) split into contiguous chunks, one per worker.
void parallel_for(int64_t count, const std::function<void(int64_t, int64_t, int)>& fn) {
  const int nt = int(std::min<int64_t>(num_threads(), std::max<int64_t>(1, count / 4096 + 1)));
  if (nt <= 1) {
    fn(0, count, 0);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (count + nt - 1) / nt;
  for (int w = 0; w < nt; ++w) {
    const int64_t lo = std::min(count, int64_t(w) * chunk), hi = std::min(count, lo + chunk);
    th.emplace_back(fn, lo, hi, w);
  }
  for (auto& t : th) t.join();
}

typedef std::vector<std::pair<int64_t, std::pair<PlanError, std::string>>> ErrList;

// Runs a row check in parallel; the error of the lowest failing row is reported, so
// the message does not depend on the thread schedule.
PlanError check_rows(int64_t n, const std::function<bool(int64_t, PlanError*, std::string*)>& bad,
                     std::string* msg) {
  std::vector<ErrList> per(16);
  parallel_for(n, [&](int64_t lo, int64_t hi, int w) {
    for (int64_t i = lo; i < hi; ++i) {
      PlanError e;
      std::string m;
      if (bad(i, &e, &m)) {
        per[w].push_back({i, {e, m}});
        return;
      }
    }
  });
  int64_t best = INT64_MAX;
  PlanError code = PlanError::kOk;
  for (auto& p : per)
    for (auto& f : p)
      if (f.first < best) {
        best = f.first;
        code = f.second.first;
        *msg = f.second.second;
      }
  return code;
}

}  // namespace

void layout_sym_batch(SymBatch* b) {
  const int64_t TT = int64_t(kTile) * kTile;
  b->nt.assign(b->count, 0);
  b->tile_off.assign(b->count, 0);
  b->item_base.assign(b->count, 0);
  b->item_mat.clear();
  b->item_BI.clear();
  b->item_BJ.clear();
  int64_t off = 0, items = 0;
  b->max_nt = 0;
  b->max_tiles = 0;
  for (int m = 0; m < b->count; ++m) {
    const int nt = (b->n[m] + kTile - 1) / kTile;
    b->nt[m] = nt;
    b->tile_off[m] = off;
    off += tiles_of(nt) * TT;
    b->max_nt = std::max(b->max_nt, nt);
    b->max_tiles = std::max<int64_t>(b->max_tiles, tiles_of(nt));
    b->item_base[m] = items;
    const int nb = (nt + kSymB - 1) / kSymB;
    for (int BI = 0; BI < nb; ++BI)
      for (int BJ = 0; BJ <= BI; ++BJ) {
        b->item_mat.push_back(m);
        b->item_BI.push_back(BI);
        b->item_BJ.push_back(BJ);
        ++items;
      }
  }
  b->total_elems = off;
  b->num_items = items;
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
  for (int32_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) {
      *msg = fmt("row_ptr decreases at row %lld", i);
      return PlanError::kInvalid;
    }
  PlanError e = check_rows(n, [&](int64_t i, PlanError* code, std::string* m) {
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t c = col_idx[k];
      if (c < 0 || c >= n) {
        *code = PlanError::kInvalid;
        *m = fmt("column index %lld out of range in row %lld", c, i);
        return true;
      }
      if (k > row_ptr[i] && c <= col_idx[k - 1]) {
        *code = PlanError::kInvalid;
        *m = fmt("columns of row %lld not strictly increasing", i);
        return true;
      }
    }
    return false;
  }, msg);
  if (e != PlanError::kOk) return e;
  // structural symmetry: (i, j) present => (j, i) present.  Each entry above the
  // diagonal is looked up in the transposed row; with as many entries below the
  // diagonal as above, that map is a bijection and the lower ones are covered too.
  e = check_rows(n, [&](int64_t i, PlanError* code, std::string* m) {
    for (int64_t k = row_ptr[i + 1] - 1; k >= row_ptr[i] && col_idx[k] > i; --k) {
      const int32_t j = col_idx[k];
      if (!std::binary_search(col_idx + row_ptr[j], col_idx + row_ptr[j + 1], int32_t(i))) {
        *code = PlanError::kInvalid;
        *m = fmt("K is not structurally symmetric: (%lld, %lld) present, transpose missing", i, j);
        return true;
      }
    }
    return false;
  }, msg);
  if (e != PlanError::kOk) return e;
  {
    std::vector<int64_t> upper(16, 0), lower(16, 0);
    parallel_for(n, [&](int64_t lo, int64_t hi, int w) {
      int64_t up = 0, dn = 0;                  // per-thread counts (no shared cache lines)
      for (int64_t i = lo; i < hi; ++i) {
        const int32_t* b = col_idx + row_ptr[i];
        const int32_t* en = col_idx + row_ptr[i + 1];
        const int32_t* d = std::lower_bound(b, en, int32_t(i));   // first column >= i
        dn += d - b;
        up += en - d - (d < en && *d == i ? 1 : 0);
      }
      upper[w] = up;
      lower[w] = dn;
    });
    if (std::accumulate(upper.begin(), upper.end(), int64_t(0)) !=
        std::accumulate(lower.begin(), lower.end(), int64_t(0))) {
      // some entry below the diagonal has no transpose: report the first one
      for (int32_t i = 0; i < n; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1] && col_idx[k] < i; ++k) {
          const int32_t j = col_idx[k];
          if (!std::binary_search(col_idx + row_ptr[j], col_idx + row_ptr[j + 1], i)) {
            *msg = fmt("K is not structurally symmetric: (%lld, %lld) present, transpose missing",
                       i, j);
            return PlanError::kInvalid;
          }
        }
      *msg = "K is not structurally symmetric";
      return PlanError::kInvalid;
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
  e = check_rows(n, [&](int64_t i, PlanError* code, std::string* m) {
    const int32_t a = dof_node[i];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t b = dof_node[col_idx[k]];
      if (!anc(a, b) && !anc(b, a)) {
        *code = PlanError::kNotSeparable;
        *m = fmt("K couples dof %lld and dof %lld whose tree nodes are not on one root-to-leaf "
                 "path (node %lld)", i, col_idx[k], a);
        return true;
      }
    }
    return false;
  }, msg);
  if (e != PlanError::kOk) return e;

  // ---- orderings ---------------------------------------------------------------------
  std::vector<int64_t> own_ptr(size_t(T) + 1, 0);
  std::vector<int32_t> own(n);
  for (int32_t i = 0; i < n; ++i) own_ptr[dof_node[i] + 1]++;
  for (int32_t t = 0; t < T; ++t) own_ptr[t + 1] += own_ptr[t];
  {
    std::vector<int64_t> fill(own_ptr.begin(), own_ptr.end() - 1);
    for (int32_t i = 0; i < n; ++i) own[fill[dof_node[i]]++] = i;
  }
  auto owned_n = [&](int32_t t) { return own_ptr[t + 1] - own_ptr[t]; };
  P->leaf_node.clear();
  for (int32_t t = 0; t < T; ++t)
    if (P->children[t].empty()) P->leaf_node.push_back(t);
  const int32_t L = int32_t(P->leaf_node.size());
  P->perm.resize(n);
  P->iperm.resize(n);
  int64_t pos = 0;
  P->leaf_off.assign(L, 0);
  P->leaf_n.assign(L, 0);
  for (int32_t l = 0; l < L; ++l) {
    const int32_t t = P->leaf_node[l];
    P->leaf_off[l] = pos;
    P->leaf_n[l] = owned_n(t);
    for (int64_t q = own_ptr[t]; q < own_ptr[t + 1]; ++q) P->perm[pos++] = own[q];
  }
  P->n_leaf = pos;
  std::vector<int32_t> inodes;
  for (int32_t t = 0; t < T; ++t)
    if (!P->children[t].empty() && owned_n(t) > 0) inodes.push_back(t);
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
    P->iface_n[s] = owned_n(t);
    for (int64_t q = own_ptr[t]; q < own_ptr[t + 1]; ++q) P->perm[pos++] = own[q];
  }
  if (NI > 0) P->level_dof_end.push_back(pos);
  P->level_iface_begin.push_back(NI);
  const int32_t NL = int32_t(P->level_depth.size());
  for (int32_t i = 0; i < n; ++i) P->iperm[P->perm[i]] = i;
  const int64_t nB = n - P->n_leaf;
  P->dof_level.assign(nB, 0);
  P->skel_lvl_begin.assign(nB, 0);
  P->skel_own_end.assign(nB, 0);
  for (int32_t q = 0; q < NL; ++q)
    for (int64_t d = P->level_dof_begin[q]; d < P->level_dof_end[q]; ++d) {
      P->dof_level[d - P->n_leaf] = q;
      P->skel_lvl_begin[d - P->n_leaf] = int32_t(P->level_dof_begin[q]);
    }
  for (int32_t s = 0; s < NI; ++s)
    for (int64_t d = P->iface_off[s]; d < P->iface_off[s] + P->iface_n[s]; ++d)
      P->skel_own_end[d - P->n_leaf] = int32_t(P->iface_off[s] + P->iface_n[s]);
  // row pointers of K in internal order
  P->prow.assign(size_t(n) + 1, 0);
  for (int32_t r = 0; r < n; ++r) {
    const int32_t o = P->perm[r];
    P->prow[r + 1] = P->prow[r] + (row_ptr[o + 1] - row_ptr[o]);
  }
  {
    const int64_t ns = (int64_t(n) + kEllSlice - 1) / kEllSlice;
    P->ell_off.assign(size_t(ns) + 1, 0);
    for (int64_t sl = 0; sl < ns; ++sl) {
      int64_t w = 0;
      for (int64_t r = sl * kEllSlice; r < std::min<int64_t>(n, (sl + 1) * kEllSlice); ++r)
        w = std::max(w, P->prow[r + 1] - P->prow[r]);
      P->ell_off[sl + 1] = P->ell_off[sl] + w * kEllSlice;
    }
  }

  // ---- per leaf: B_l, shell_l, K_{l,B_l} by columns, K_{B_l,l} by rows ----------------
  // (read from the caller's CSR; value positions are the caller's)
  struct LeafOut {
    std::vector<int32_t> B, shell, kcol_row, krow_col;
    std::vector<int64_t> kcol_ptr, kcol_val, krow_ptr, krow_val;
  };
  std::vector<LeafOut> lo_out(L);
  {
    std::atomic<int32_t> next{0};
    std::vector<std::thread> th;
    const int nw = std::min<int>(num_threads(), std::max(1, L));
    for (int w = 0; w < nw; ++w)
      th.emplace_back([&]() {
        std::vector<int32_t> posB(size_t(std::max<int64_t>(1, nB)), -1);
        std::vector<int32_t> shell_idx;
        for (;;) {
          const int32_t l = next++;
          if (l >= L) break;
          LeafOut& o = lo_out[l];
          const int64_t off = P->leaf_off[l], nl = P->leaf_n[l];
          shell_idx.assign(size_t(nl), -1);
          // B_l and the shell (posB tags the interface dofs already seen in this leaf)
          for (int64_t r = 0; r < nl; ++r) {
            const int32_t orow = P->perm[off + r];
            bool coupled = false;
            for (int64_t k = row_ptr[orow]; k < row_ptr[orow + 1]; ++k) {
              const int32_t c = P->iperm[col_idx[k]];
              if (c < P->n_leaf) continue;
              coupled = true;
              if (posB[c - P->n_leaf] != -2) {
                posB[c - P->n_leaf] = -2;
                o.B.push_back(c);
              }
            }
            if (coupled) {
              shell_idx[r] = int32_t(o.shell.size());
              o.shell.push_back(int32_t(r));
            }
          }
          std::sort(o.B.begin(), o.B.end());
          const int64_t m = int64_t(o.B.size());
          for (int64_t a = 0; a < m; ++a) posB[o.B[a] - P->n_leaf] = int32_t(a);
          // columns of K_{l,B}
          o.kcol_ptr.assign(size_t(m) + 1, 0);
          for (int64_t r = 0; r < nl; ++r) {
            const int32_t orow = P->perm[off + r];
            for (int64_t k = row_ptr[orow]; k < row_ptr[orow + 1]; ++k) {
              const int32_t c = P->iperm[col_idx[k]];
              if (c >= P->n_leaf) o.kcol_ptr[posB[c - P->n_leaf] + 1]++;
            }
          }
          for (int64_t a = 0; a < m; ++a) o.kcol_ptr[a + 1] += o.kcol_ptr[a];
          o.kcol_row.assign(size_t(o.kcol_ptr[m]), 0);
          o.kcol_val.assign(size_t(o.kcol_ptr[m]), 0);
          {
            std::vector<int64_t> fill(o.kcol_ptr.begin(), o.kcol_ptr.end() - 1);
            for (int64_t r = 0; r < nl; ++r) {
              const int32_t orow = P->perm[off + r];
              for (int64_t k = row_ptr[orow]; k < row_ptr[orow + 1]; ++k) {
                const int32_t c = P->iperm[col_idx[k]];
                if (c < P->n_leaf) continue;
                const int64_t f = fill[posB[c - P->n_leaf]]++;
                o.kcol_row[f] = int32_t(r);
                o.kcol_val[f] = k;
              }
            }
          }
          // rows of K_{B,l}
          o.krow_ptr.assign(size_t(m) + 1, 0);
          for (int64_t a = 0; a < m; ++a) {
            const int32_t orow = P->perm[o.B[a]];
            for (int64_t k = row_ptr[orow]; k < row_ptr[orow + 1]; ++k) {
              const int32_t c = P->iperm[col_idx[k]];
              if (c < off || c >= off + nl) continue;
              o.krow_col.push_back(shell_idx[c - off]);
              o.krow_val.push_back(k);
            }
            o.krow_ptr[a + 1] = int64_t(o.krow_col.size());
          }
          for (int64_t a = 0; a < m; ++a) posB[o.B[a] - P->n_leaf] = -1;
        }
      });
    for (auto& t : th) t.join();
  }
  for (int32_t l = 0; l < L; ++l)
    for (int32_t v : lo_out[l].krow_col)
      if (v < 0) {
        *msg = "internal error: interface row couples to a non-shell interior dof";
        return PlanError::kInvalid;
      }
  // concatenate the per-leaf pieces
  P->B_off.assign(L + 1, 0);
  P->shell_off.assign(L + 1, 0);
  int64_t nkc = 0, nkr = 0;
  for (int32_t l = 0; l < L; ++l) {
    P->B_off[l + 1] = P->B_off[l] + int64_t(lo_out[l].B.size());
    P->shell_off[l + 1] = P->shell_off[l] + int64_t(lo_out[l].shell.size());
    nkc += int64_t(lo_out[l].kcol_row.size());
    nkr += int64_t(lo_out[l].krow_col.size());
  }
  const int64_t nBflat = P->B_off[L];
  P->kcol_ptr.assign(nBflat + 1, 0);
  P->krow_ptr.assign(nBflat + 1, 0);
  {
    // per-leaf offsets first, then every leaf's pieces copied in parallel
    std::vector<int64_t> kc_off(size_t(L) + 1, 0), kr_off(size_t(L) + 1, 0);
    for (int32_t l = 0; l < L; ++l) {
      kc_off[l + 1] = kc_off[l] + int64_t(lo_out[l].kcol_row.size());
      kr_off[l + 1] = kr_off[l] + int64_t(lo_out[l].krow_col.size());
    }
    P->B.resize(size_t(nBflat));
    P->shell.resize(size_t(P->shell_off[L]));
    P->kcol_row.resize(size_t(nkc));
    P->kcol_val.resize(size_t(nkc));
    P->krow_col.resize(size_t(nkr));
    P->krow_val.resize(size_t(nkr));
    std::atomic<int32_t> next{0};
    std::vector<std::thread> th;
    const int nw = std::min<int>(num_threads(), std::max(1, L));
    for (int w = 0; w < nw; ++w)
      th.emplace_back([&]() {
        for (;;) {
          const int32_t l = next++;
          if (l >= L) break;
          LeafOut& o = lo_out[l];
          const int64_t base = P->B_off[l];
          for (size_t a = 0; a < o.B.size(); ++a) {
            P->kcol_ptr[base + a + 1] = kc_off[l] + o.kcol_ptr[a + 1];
            P->krow_ptr[base + a + 1] = kr_off[l] + o.krow_ptr[a + 1];
          }
          std::copy(o.B.begin(), o.B.end(), P->B.begin() + base);
          std::copy(o.shell.begin(), o.shell.end(), P->shell.begin() + P->shell_off[l]);
          std::copy(o.kcol_row.begin(), o.kcol_row.end(), P->kcol_row.begin() + kc_off[l]);
          std::copy(o.kcol_val.begin(), o.kcol_val.end(), P->kcol_val.begin() + kc_off[l]);
          std::copy(o.krow_col.begin(), o.krow_col.end(), P->krow_col.begin() + kr_off[l]);
          std::copy(o.krow_val.begin(), o.krow_val.end(), P->krow_val.begin() + kr_off[l]);
          o = LeafOut();
        }
      });
    for (auto& t : th) t.join();
  }
  // adjacency of interface dofs: (leaf, position in B_l), sorted by leaf
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
  // Sigma and W layouts
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

  // ---- apply schedule: Sigma products per level --------------------------------------
  P->level_sigma.assign(NL, {});
  P->level_sigma_own.assign(NL, {});
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
      if (r1 > r0) P->level_sigma_own[q].push_back({l, r0, r1});
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
  layout_sym_batch(&P->leaf_batch);
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
    layout_sym_batch(&b);
  }
  return PlanError::kOk;
}

}  // namespace rsd
