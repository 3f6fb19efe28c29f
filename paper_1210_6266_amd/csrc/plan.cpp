// Host analysis of the hierarchical decomposition: see plan.hpp.
#include "plan.hpp"

#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <functional>
#include <mutex>
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

// Process-wide worker threads for the analysis' parallel loops, started on first use (a
// forked child starts its own).  run(nw, fn) calls fn(w) for w in [0, nw), w = 0 on the
// calling thread, and returns when every call has returned; concurrent callers take
// turns.  Starting threads per loop cost about 1 ms per set-up at 16 threads.
class Pool {
 public:
  static Pool& get() {
    static std::mutex mu;
    static Pool* pool = nullptr;               // never destroyed: its threads are detached
    std::lock_guard<std::mutex> lk(mu);
    if (pool == nullptr || pool->pid_ != getpid()) pool = new Pool(num_threads() - 1);
    return *pool;
  }
  int size() const { return int(nworkers_) + 1; }
  void run(int nw, const std::function<void(int)>& fn) {
    std::lock_guard<std::mutex> turn(run_mu_);
    nw = std::min(nw, size());
    if (nw <= 1) {
      fn(0);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      nw_ = nw;
      pending_ = nw - 1;
      ++gen_;
    }
    cv_.notify_all();
    fn(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return pending_ == 0; });
  }

 private:
  explicit Pool(int nworkers) : pid_(getpid()), nworkers_(std::max(0, nworkers)) {
    for (int w = 1; w <= nworkers_; ++w) std::thread([this, w] { loop(w); }).detach();
  }
  void loop(int w) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* fn;
      int nw;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        fn = fn_;
        nw = nw_;
      }
      if (w >= nw) continue;                   // not needed for this loop
      (*fn)(w);
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) done_.notify_one();
    }
  }
  const pid_t pid_;
  const int nworkers_;
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* fn_ = nullptr;
  int nw_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
};

// Runs fn(lo, hi, worker) over [0, count) split into contiguous chunks, one per worker
// (at most one worker per `grain` items).  The split depends only on count, grain and the
// pool's size: loops over the same count hand worker w the same chunk.
void parallel_for(int64_t count, const std::function<void(int64_t, int64_t, int)>& fn,
                  int64_t grain = 4096) {
  Pool& pool = Pool::get();
  const int nt = int(std::min<int64_t>(pool.size(), std::max<int64_t>(1, count / grain + 1)));
  const int64_t chunk = (count + nt - 1) / nt;
  pool.run(nt, [&](int w) {
    const int64_t lo = std::min(count, int64_t(w) * chunk), hi = std::min(count, lo + chunk);
    fn(lo, hi, w);
  });
}

// Runs fn(item, worker) for every item in [0, count), items taken in turn by the workers.
void parallel_items(int64_t count, const std::function<void(int64_t, int)>& fn) {
  Pool& pool = Pool::get();
  std::atomic<int64_t> next{0};
  pool.run(int(std::min<int64_t>(pool.size(), std::max<int64_t>(1, count))), [&](int w) {
    for (int64_t i = next++; i < count; i = next++) fn(i, w);
  });
}

}  // namespace

namespace {

// Structural symmetry of a CSR whose columns are in range and strictly increasing: every
// entry above the diagonal matched with its transpose, with as many entries below the
// diagonal as above (then that map is a bijection and the lower ones are covered too).  A
// worker's rows come in increasing order, so the transposes it looks for in a row j come
// in increasing column order: one cursor per row j (within the worker's window of rows)
// replaces a search.  If a cursor finds anything else, an exact search over all rows
// names the lowest row with a missing transpose (the message does not depend on the
// thread schedule).
PlanError check_symmetry(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                         std::string* msg) {
  struct Worker {
    int64_t up = 0, dn = 0;
    bool asym = false;
    int64_t row = INT64_MAX;                   // lowest row of an exact search's finding
    std::string msg;
  };
  auto sym_error = [&](int64_t i, Worker* o) {  // the first missing transpose of row i
    for (int64_t k = row_ptr[i + 1] - 1; k >= row_ptr[i] && col_idx[k] > i; --k) {
      const int32_t j = col_idx[k];
      if (!std::binary_search(col_idx + row_ptr[j], col_idx + row_ptr[j + 1], int32_t(i))) {
        o->row = i;
        o->msg = fmt("K is not structurally symmetric: (%lld, %lld) present, transpose missing",
                     i, j);
        return true;
      }
    }
    return false;
  };
  std::vector<Worker> wk(size_t(Pool::get().size()));
  parallel_for(n, [&](int64_t lo, int64_t hi, int w) {
    Worker& o = wk[size_t(w)];
    int64_t jmax = lo;                         // window of rows searched: [lo, jmax]
    for (int64_t i = lo; i < hi; ++i)
      if (row_ptr[i + 1] > row_ptr[i]) jmax = std::max<int64_t>(jmax, col_idx[row_ptr[i + 1] - 1]);
    const bool cursors = jmax - lo < std::max<int64_t>(4 * (hi - lo), int64_t(1) << 20);
    std::vector<int32_t> cur;                  // per row of the window: next position, or -1
    if (cursors) cur.assign(size_t(jmax - lo + 1), -1);
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t* cb = col_idx + row_ptr[i];
      const int32_t* ce = col_idx + row_ptr[i + 1];
      const int32_t* d = std::lower_bound(cb, ce, int32_t(i));   // first column >= i
      const int32_t* u = d < ce && *d == i ? d + 1 : d;          // first column > i
      o.dn += d - cb;
      o.up += ce - u;
      if (!cursors) {
        if (o.row == INT64_MAX) sym_error(i, &o);
        continue;
      }
      if (o.asym) continue;
      for (const int32_t* q = u; q < ce; ++q) {
        const int32_t j = *q;
        const int64_t rj = row_ptr[j];
        int32_t& cj = cur[size_t(j - lo)];
        if (cj < 0)
          cj = int32_t(std::lower_bound(col_idx + rj, col_idx + row_ptr[j + 1], int32_t(lo)) -
                       (col_idx + rj));
        if (rj + cj < row_ptr[j + 1] && col_idx[rj + cj] == i) {
          ++cj;
        } else {
          o.asym = true;
          break;
        }
      }
    }
  });
  bool asym = false;
  for (const Worker& o : wk) asym = asym || o.asym;
  if (asym) {
    for (Worker& o : wk) o.row = INT64_MAX;
    parallel_for(n, [&](int64_t lo, int64_t hi, int w) {
      for (int64_t i = lo; i < hi; ++i)
        if (sym_error(i, &wk[size_t(w)])) return;
    });
  }
  const Worker* best = nullptr;
  for (const Worker& o : wk)
    if (o.row != INT64_MAX && (best == nullptr || o.row < best->row)) best = &o;
  if (best) {
    *msg = best->msg;
    return PlanError::kInvalid;
  }
  int64_t up = 0, dn = 0;
  for (const Worker& o : wk) {
    up += o.up;
    dn += o.dn;
  }
  if (up != dn) {
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
  return PlanError::kOk;
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
  // ---- validation of the CSR (its rows are checked by the passes below) ---------------
  if (n <= 0) { *msg = "n must be positive"; return PlanError::kInvalid; }
  if (nnz < 0 || row_ptr == nullptr || (nnz > 0 && col_idx == nullptr)) {
    *msg = "null CSR array or negative nnz";
    return PlanError::kInvalid;
  }
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) {
    *msg = fmt("row_ptr[0] must be 0 and row_ptr[n] = nnz (%lld), got %lld", nnz, row_ptr[n]);
    return PlanError::kInvalid;
  }
  // ---- validation of the tree (reported after the CSR's errors) ---------------------
  std::string tree_msg;
  if (T <= 0 || parent == nullptr || dof_node == nullptr) {
    tree_msg = "hierarchy needs num_nodes >= 1, parent and dof_node";
  } else if (parent[0] != -1) {
    tree_msg = "parent[0] must be -1";
  } else {
    for (int32_t t = 1; t < T && tree_msg.empty(); ++t)
      if (parent[t] < 0 || parent[t] >= t)
        tree_msg = fmt("parent[%lld] = %lld must lie in [0, %lld)", t, parent[t], t);
  }
  const bool parents_ok = tree_msg.empty();
  // Each check below reports its lowest failing row, so messages do not depend on the
  // thread schedule; the CSR's errors come first, then the tree's, then separability.
  struct RowErr {
    int64_t row = INT64_MAX;
    std::string msg;
  };
  struct Worker {
    RowErr rp, dn, col, sep;
  };
  const int NW = Pool::get().size();
  std::vector<Worker> wk(static_cast<size_t>(NW));
  auto lowest = [&](RowErr Worker::*f) {
    const RowErr* best = nullptr;
    for (const Worker& o : wk)
      if ((o.*f).row != INT64_MAX && (best == nullptr || (o.*f).row < best->row)) best = &(o.*f);
    return best;
  };
  // Per worker (the three passes over the rows split them alike) and node: its rows, and
  // those of them coupled to no dof of another node (rows of TS counts, padded so that no
  // two workers write one cache line).
  const size_t TS = (size_t(T) + 31) / 16 * 16;
  const size_t WT = parents_ok ? size_t(NW) * TS : 0;
  std::vector<int32_t> cnt(WT, 0), icnt(WT, 0);
  // ---- first pass: row_ptr non-decreasing, dof_node in range, the rows of each node ----
  parallel_for(n, [&](int64_t lo, int64_t hi, int w) {
    Worker& o = wk[size_t(w)];
    for (int64_t i = lo; i < hi; ++i)
      if (row_ptr[i + 1] < row_ptr[i]) {
        o.rp = {i, fmt("row_ptr decreases at row %lld", i)};
        break;
      }
    if (!parents_ok) return;
    int32_t* const c = cnt.data() + size_t(w) * TS;
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t t = dof_node[i];
      if (t < 0 || t >= T) {
        o.dn = {i, fmt("dof_node[%lld] = %lld out of range", i, t)};
        break;
      }
      ++c[t];
    }
  });
  if (const RowErr* r = lowest(&Worker::rp)) {   // (then every row lies in [0, nnz])
    *msg = r->msg;
    return PlanError::kInvalid;
  }
  if (parents_ok)
    if (const RowErr* r = lowest(&Worker::dn)) tree_msg = r->msg;
  const bool tree_ok = tree_msg.empty();
  // Euler tour for ancestor tests (parent[t] < t: ids are topologically ordered)
  std::vector<int32_t> tin, tout;
  if (tree_ok) {
    P->parent.assign(parent, parent + T);
    P->depth.assign(T, 0);
    P->children.assign(T, {});
    for (int32_t t = 1; t < T; ++t) {
      P->depth[t] = P->depth[parent[t]] + 1;
      P->children[parent[t]].push_back(t);
    }
    tin.assign(T, 0);
    tout.assign(T, 0);
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
  // ---- second pass: columns in range and strictly increasing; separability ------------
  // (every coupling joins nodes on one root-to-leaf path).  Structural symmetry, which no
  // device work before the couplings relies on, is checked by build_plan_couplings.
  // outer[i] = 1 for a dof coupled to a dof of another tree node (for a leaf's dof: an
  // interface dof, the leaf's shell).
  hvec<uint8_t> outer(static_cast<size_t>(n));
  parallel_for(n, [&](int64_t lo, int64_t hi, int w) {
    Worker& o = wk[size_t(w)];
    const int32_t* const ti = tin.data();
    const int32_t* const to = tout.data();
    auto anc = [&](int32_t a, int32_t b) {  // a is an ancestor of b, or a == b
      return ti[a] <= ti[b] && to[b] <= to[a];
    };
    int32_t* const ic = tree_ok ? icnt.data() + size_t(w) * TS : nullptr;
    uint8_t* const out = outer.data();
    bool sep = tree_ok;                        // no separability error seen yet
    for (int64_t i = lo; i < hi; ++i) {
      const int64_t b = row_ptr[i], en = row_ptr[i + 1];
      bool bad = false;
      int32_t prev = -1;
      for (int64_t k = b; k < en; ++k) {
        const int32_t c = col_idx[k];
        bad |= (c <= prev) | (c >= n);
        prev = c;
      }
      if (bad) {                               // name the first offending entry
        for (int64_t k = b; k < en; ++k) {
          const int32_t c = col_idx[k];
          if (c < 0 || c >= n) {
            o.col = {i, fmt("column index %lld out of range in row %lld", c, i)};
            return;
          }
          if (k > b && c <= col_idx[k - 1]) {
            o.col = {i, fmt("columns of row %lld not strictly increasing", i)};
            return;
          }
        }
      }
      if (!sep) continue;
      const int32_t a = dof_node[i];
      int32_t ok = a;                          // a node of a's path seen last
      bool sh = false;
      for (int64_t k = b; k < en; ++k) {
        const int32_t bn = dof_node[col_idx[k]];
        if (bn == a) continue;
        sh = true;
        if (bn == ok) continue;
        if (!anc(a, bn) && !anc(bn, a)) {
          o.sep = {i, fmt("K couples dof %lld and dof %lld whose tree nodes are not on one "
                          "root-to-leaf path (node %lld)", i, col_idx[k], a)};
          sep = false;
          break;
        }
        ok = bn;
      }
      out[i] = sh;
      ic[a] += !sh;
    }
  });
  if (const RowErr* r = lowest(&Worker::col)) {
    *msg = r->msg;
    return PlanError::kInvalid;
  }
  if (!tree_ok) {
    *msg = tree_msg;
    return PlanError::kInvalid;
  }
  if (const RowErr* r = lowest(&Worker::sep)) {
    *msg = r->msg;
    return PlanError::kNotSeparable;
  }
  P->n = n;
  P->nnz = nnz;
  P->T = T;

  // ---- orderings ---------------------------------------------------------------------
  // Internal order: the leaves in node-id order, each with its dofs coupled to no
  // interface dof first (the back-substitution's correction K_ll^{-1} K_{l,B} u_B then
  // reads only the tile rows of the inverse that hold shell rows: engine's core_apply),
  // then the interface nodes deepest level first; within each group, caller order.
  std::vector<int64_t> owned(size_t(T), 0), inner(size_t(T), 0);
  for (int w = 0; w < NW; ++w)
    for (int32_t t = 0; t < T; ++t) {
      owned[t] += cnt[size_t(w) * TS + t];
      inner[t] += icnt[size_t(w) * TS + t];
    }
  P->leaf_node.clear();
  for (int32_t t = 0; t < T; ++t)
    if (P->children[t].empty()) P->leaf_node.push_back(t);
  const int32_t L = int32_t(P->leaf_node.size());
  // first position of each node's group(s): [2t] its dofs (a leaf's inner ones), [2t + 1]
  // a leaf's shell
  std::vector<int64_t> first(2 * size_t(T), 0);
  std::vector<uint8_t> is_leaf(size_t(T), 0);
  int64_t pos = 0;
  P->leaf_off.assign(L, 0);
  P->leaf_n.assign(L, 0);
  P->leaf_inner.assign(L, 0);
  for (int32_t l = 0; l < L; ++l) {
    const int32_t t = P->leaf_node[l];
    is_leaf[t] = 1;
    P->leaf_off[l] = pos;
    P->leaf_n[l] = owned[t];
    P->leaf_inner[l] = int32_t(inner[t]);
    first[2 * t] = pos;
    first[2 * t + 1] = pos + inner[t];
    pos += owned[t];
  }
  P->n_leaf = pos;
  std::vector<int32_t> inodes;
  for (int32_t t = 0; t < T; ++t)
    if (!P->children[t].empty() && owned[t] > 0) inodes.push_back(t);
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
    P->iface_n[s] = owned[t];
    first[2 * t] = pos;
    pos += owned[t];
  }
  if (NI > 0) P->level_dof_end.push_back(pos);
  P->level_iface_begin.push_back(NI);
  const int32_t NL = int32_t(P->level_depth.size());
  // each worker's first position in each group: the rows of the workers before it come first
  hvec<int64_t> cur(size_t(NW) * 2 * T);
  parallel_for(T, [&](int64_t lo, int64_t hi, int) {
    for (int64_t t = lo; t < hi; ++t) {
      int64_t g0 = first[2 * t], g1 = first[2 * t + 1];
      for (int w = 0; w < NW; ++w) {
        const size_t wt = size_t(w) * TS + t, wc = size_t(w) * T + t;
        cur[2 * wc] = g0;
        cur[2 * wc + 1] = g1;
        g0 += is_leaf[t] ? icnt[wt] : cnt[wt];
        g1 += is_leaf[t] ? cnt[wt] - icnt[wt] : 0;
      }
    }
  }, 256);
  // ---- third pass: perm, iperm and the row lengths in internal order ------------------
  P->perm.resize(n);
  P->iperm.resize(n);
  P->prow.resize(size_t(n) + 1);
  parallel_for(n, [&](int64_t lo, int64_t hi, int w) {
    int64_t* const c = cur.data() + size_t(w) * 2 * T;
    int32_t* const pm = P->perm.data();
    int32_t* const ip = P->iperm.data();
    int64_t* const pr = P->prow.data();
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t t = dof_node[i];
      const int64_t p = c[2 * t + (outer[i] & is_leaf[t])]++;
      pm[p] = int32_t(i);
      ip[i] = int32_t(p);
      pr[p + 1] = row_ptr[i + 1] - row_ptr[i];
    }
  });
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
  // row pointers of K in internal order (a prefix sum of the lengths, by slices of
  // kEllSlice rows), and the sliced ELL layout: slice s padded to its longest row
  {
    const int64_t ns = (int64_t(n) + kEllSlice - 1) / kEllSlice;
    int64_t* const pr = P->prow.data();
    pr[0] = 0;
    P->ell_off.assign(size_t(ns) + 1, 0);
    std::vector<int64_t> part(size_t(NW) + 1, 0);
    parallel_for(ns, [&](int64_t lo, int64_t hi, int w) {
      int64_t sum = 0;
      for (int64_t sl = lo; sl < hi; ++sl) {
        int64_t wd = 0;
        for (int64_t r = sl * kEllSlice; r < std::min<int64_t>(n, (sl + 1) * kEllSlice); ++r) {
          wd = std::max(wd, pr[r + 1]);
          sum += pr[r + 1];
        }
        P->ell_off[sl + 1] = wd * kEllSlice;
      }
      part[size_t(w) + 1] = sum;
    }, 64);
    for (int w = 0; w < NW; ++w) part[size_t(w) + 1] += part[size_t(w)];
    for (int64_t sl = 0; sl < ns; ++sl) P->ell_off[sl + 1] += P->ell_off[sl];
    parallel_for(ns, [&](int64_t lo, int64_t hi, int w) {
      int64_t acc = part[size_t(w)];
      for (int64_t r = lo * kEllSlice; r < std::min<int64_t>(n, hi * kEllSlice); ++r) {
        acc += pr[r + 1];
        pr[r + 1] = acc;
      }
    }, 64);
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
  P->coupled = false;
  return PlanError::kOk;
}

PlanError build_plan_couplings(const int64_t* row_ptr, const int32_t* col_idx, Plan* P,
                               std::string* msg) {
  {
    const PlanError e = check_symmetry(P->n, row_ptr, col_idx, msg);
    if (e != PlanError::kOk) return e;
  }
  const int32_t L = int32_t(P->leaf_node.size());
  const int64_t nB = P->n - P->n_leaf;
  const int32_t NL = int32_t(P->level_depth.size());
  // ---- per leaf: B_l, shell_l, K_{l,B_l} by columns, K_{B_l,l} by rows ----------------
  // (read from the caller's CSR; value positions are the caller's).  Pass 1 finds B_l and
  // the shell and counts the couplings; pass 2 writes both coupling blocks straight into
  // their final place.  K_{B_l,l} has as many entries as K_{l,B_l} (structural symmetry).
  std::vector<std::vector<int32_t>> Bl(L), shl(L), cntl(L);
  std::vector<int64_t> ncpl(size_t(L), 0);
  const int nwk = Pool::get().size();
  std::vector<std::vector<int32_t>> posB_w(static_cast<size_t>(nwk));
  parallel_items(L, [&](int64_t l, int w) {
    std::vector<int32_t>& cntB = posB_w[size_t(w)];   // couplings per interface dof, this leaf
    if (cntB.empty()) cntB.assign(size_t(std::max<int64_t>(1, nB)), 0);
    std::vector<int32_t>& B = Bl[size_t(l)];
    std::vector<int32_t>& sh = shl[size_t(l)];
    const int64_t off = P->leaf_off[l], nl = P->leaf_n[l];
    int64_t cnt = 0;
    for (int64_t r = 0; r < nl; ++r) {
      const int32_t orow = P->perm[off + r];
      const int64_t c0 = cnt;
      for (int64_t k = row_ptr[orow]; k < row_ptr[orow + 1]; ++k) {
        const int32_t c = P->iperm[col_idx[k]];
        if (c < P->n_leaf) continue;
        ++cnt;
        if (cntB[c - P->n_leaf]++ == 0) B.push_back(c);
      }
      if (cnt > c0) sh.push_back(int32_t(r));
    }
    std::sort(B.begin(), B.end());
    std::vector<int32_t>& cn = cntl[size_t(l)];
    cn.resize(B.size());
    for (size_t a = 0; a < B.size(); ++a) {
      cn[a] = cntB[B[a] - P->n_leaf];
      cntB[B[a] - P->n_leaf] = 0;
    }
    ncpl[size_t(l)] = cnt;
  });
  P->B_off.assign(L + 1, 0);
  P->shell_off.assign(L + 1, 0);
  std::vector<int64_t> kc_off(size_t(L) + 1, 0);
  for (int32_t l = 0; l < L; ++l) {
    P->B_off[l + 1] = P->B_off[l] + int64_t(Bl[l].size());
    P->shell_off[l + 1] = P->shell_off[l] + int64_t(shl[l].size());
    kc_off[l + 1] = kc_off[l] + ncpl[l];
  }
  const int64_t nBflat = P->B_off[L], nkc = kc_off[L];
  P->B.resize(size_t(nBflat));
  P->shell.resize(size_t(P->shell_off[L]));
  P->kcol_ptr.assign(nBflat + 1, 0);
  P->krow_ptr.assign(nBflat + 1, 0);
  P->kcol_row.resize(size_t(nkc));
  P->kcol_val.resize(size_t(nkc));
  P->krow_col.resize(size_t(nkc));
  P->krow_val.resize(size_t(nkc));
  std::atomic<bool> bad{false};
  std::vector<std::vector<int32_t>> shidx_w(static_cast<size_t>(nwk));
  std::vector<std::vector<int64_t>> fill_w(static_cast<size_t>(nwk));
  parallel_items(L, [&](int64_t l, int w) {
    std::vector<int32_t>& posB = posB_w[size_t(w)];   // position in B_l of the leaf's columns
    if (posB.empty()) posB.resize(size_t(std::max<int64_t>(1, nB)));
    std::vector<int32_t>& shell_idx = shidx_w[size_t(w)];
    std::vector<int64_t>& fill = fill_w[size_t(w)];
    const std::vector<int32_t>& B = Bl[size_t(l)];
    const std::vector<int32_t>& sh = shl[size_t(l)];
    const int64_t off = P->leaf_off[l], nl = P->leaf_n[l], m = int64_t(B.size());
    const int64_t base = P->B_off[l];
    std::copy(B.begin(), B.end(), P->B.begin() + base);
    std::copy(sh.begin(), sh.end(), P->shell.begin() + P->shell_off[l]);
    for (int64_t a = 0; a < m; ++a) posB[B[a] - P->n_leaf] = int32_t(a);
    shell_idx.assign(size_t(nl), -1);
    for (size_t q = 0; q < sh.size(); ++q) shell_idx[sh[q]] = int32_t(q);
    // columns of K_{l,B}: offsets from the counts of pass 1, then the entries in row order
    const std::vector<int32_t>& cn = cntl[size_t(l)];
    fill.resize(size_t(m) + 1);
    fill[0] = kc_off[l];
    for (int64_t a = 0; a < m; ++a) {
      fill[a + 1] = fill[a] + cn[size_t(a)];
      P->kcol_ptr[base + a + 1] = fill[a + 1];
    }
    for (int64_t r = 0; r < nl; ++r) {
      const int32_t orow = P->perm[off + r];
      for (int64_t k = row_ptr[orow]; k < row_ptr[orow + 1]; ++k) {
        const int32_t c = P->iperm[col_idx[k]];
        if (c < P->n_leaf) continue;
        const int64_t f = fill[posB[c - P->n_leaf]]++;
        P->kcol_row[f] = int32_t(r);
        P->kcol_val[f] = k;
      }
    }
    // rows of K_{B,l}
    int64_t q = kc_off[l];
    for (int64_t a = 0; a < m; ++a) {
      const int32_t orow = P->perm[B[a]];
      for (int64_t k = row_ptr[orow]; k < row_ptr[orow + 1]; ++k) {
        const int32_t c = P->iperm[col_idx[k]];
        if (c < off || c >= off + nl) continue;
        if (q >= kc_off[l + 1] || shell_idx[c - off] < 0) {
          bad = true;
          break;
        }
        P->krow_col[q] = shell_idx[c - off];
        P->krow_val[q] = k;
        ++q;
      }
      P->krow_ptr[base + a + 1] = q;
    }
    if (q != kc_off[l + 1]) bad = true;
  });
  if (bad) {
    *msg = "internal error: interface row couples to a non-shell interior dof";
    return PlanError::kInvalid;
  }
  Bl.clear();
  shl.clear();
  cntl.clear();
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

  P->coupled = true;
  return PlanError::kOk;
}

}  // namespace rsd
