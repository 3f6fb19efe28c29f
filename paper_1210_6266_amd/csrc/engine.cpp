// The RSD engine: set-up (Section 3: exact sub-domain inverses, interface Schur
// complements of Alg. 1, their inverses), the preconditioner apply (Alg. 2 with
// exact interface solves), the MatVec, and FGMRES / PCG drivers.
#include "engine.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>

namespace rsd {

namespace {

struct Fail {
  rsd_status st;
};

void hip_check(rsd_ctx* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  h->err = std::string(what) + ": " + hipGetErrorString(e);
  throw Fail{e == hipErrorOutOfMemory ? RSD_ERR_OUT_OF_MEMORY : RSD_ERR_DEVICE};
}

// Memory recycling.  The library releases device memory only at points where the work
// that used it has completed (after a stream or device synchronization), so released
// blocks go to a per-device cache and serve the next allocation of a similar size
// without a call into the allocator; repeated set-ups reuse the same mappings.  Pinned
// host staging buffers (structure copies) are cached the same way.  Blocks beyond
// kCacheKeepBytes per device are returned to the runtime.
constexpr size_t kCacheKeepBytes = size_t(48) << 30;

struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, void*> blocks;   // size -> block
  size_t bytes = 0;
};

BlockCache& cache_of(int key) {
  static std::mutex mu;
  static std::map<int, BlockCache*> caches;   // device id; -1 - device for pinned host
  std::lock_guard<std::mutex> lock(mu);
  BlockCache*& c = caches[key];
  if (!c) c = new BlockCache();
  return *c;
}

size_t round_block(size_t b) {
  const size_t g = b <= (size_t(1) << 20) ? size_t(4096) : size_t(2) << 20;
  return (std::max<size_t>(b, 1) + g - 1) / g * g;
}

// a cached block of at least `bytes` (and not much larger), or nullptr
void* cache_take(BlockCache& c, size_t bytes, size_t* got) {
  std::lock_guard<std::mutex> lock(c.mu);
  auto it = c.blocks.lower_bound(bytes);
  if (it == c.blocks.end() || it->first > bytes + bytes / 8 + (size_t(4) << 20)) return nullptr;
  void* p = it->second;
  *got = it->first;
  c.bytes -= it->first;
  c.blocks.erase(it);
  return p;
}

void cache_give(BlockCache& c, void* p, size_t bytes, bool pinned) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lock(c.mu);
    c.blocks.insert({bytes, p});
    c.bytes += bytes;
    while (c.bytes > kCacheKeepBytes && !c.blocks.empty()) {
      auto big = std::prev(c.blocks.end());
      c.bytes -= big->first;
      drop.push_back(big->second);
      c.blocks.erase(big);
    }
  }
  for (void* q : drop) (void)(pinned ? hipHostFree(q) : hipFree(q));
}

void cache_drain(BlockCache& c, bool pinned) {
  std::lock_guard<std::mutex> lock(c.mu);
  for (auto& b : c.blocks) (void)(pinned ? hipHostFree(b.second) : hipFree(b.second));
  c.blocks.clear();
  c.bytes = 0;
}

template <typename T>
T* dalloc(rsd_ctx* h, size_t count) {
  const size_t want = round_block(std::max<size_t>(count, 1) * sizeof(T));
  BlockCache& c = cache_of(h->device);
  size_t got = want;
  void* p = cache_take(c, want, &got);
  if (!p) {
    hipError_t st = hipMalloc(&p, want);
    if (st == hipErrorOutOfMemory) {   // give cached blocks back and retry once
      (void)hipGetLastError();
      cache_drain(c, false);
      st = hipMalloc(&p, want);
    }
    hip_check(h, st, "hipMalloc");
  }
  h->allocs.push_back({p, got});
  h->device_bytes += int64_t(got);
  return static_cast<T*>(p);
}

// Releases p; the caller guarantees that no queued work still uses it.
void dfree(rsd_ctx* h, void* p) {
  if (!p) return;
  for (size_t i = 0; i < h->allocs.size(); ++i)
    if (h->allocs[i].first == p) {
      h->device_bytes -= int64_t(h->allocs[i].second);
      cache_give(cache_of(h->device), p, h->allocs[i].second, false);
      h->allocs.erase(h->allocs.begin() + long(i));
      return;
    }
}

// Pinned host staging buffer (released with pfree once the copy has completed).
Pinned palloc(rsd_ctx* h, size_t bytes) {
  Pinned b;
  const size_t want = round_block(bytes);
  BlockCache& c = cache_of(-1 - h->device);
  b.bytes = want;
  b.p = cache_take(c, want, &b.bytes);
  if (!b.p) hip_check(h, hipHostMalloc(&b.p, want, hipHostMallocDefault), "hipHostMalloc");
  return b;
}
void pfree(rsd_ctx* h, Pinned& b) {
  if (b.p) cache_give(cache_of(-1 - h->device), b.p, b.bytes, true);
  b.p = nullptr;
}

// The auxiliary (look-ahead) stream of a device, shared by the handles on it (default
// priority; ordering between streams is carried by each handle's own events).
hipStream_t aux_stream(rsd_ctx* h) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  std::lock_guard<std::mutex> lock(mu);
  hipStream_t& s = streams[h->device];
  if (!s) hip_check(h, hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
  return s;
}

// Packs many host arrays into one device allocation and one host-to-device copy from
// a pinned staging buffer: add() records source and destination pointer (the source
// must stay alive until commit), commit() allocates, copies and patches; the staging
// buffer is released by done() after the stream has been synchronized.
struct Uploader {
  struct Item {
    void** dst;
    const void* src;
    size_t bytes, off;
  };
  std::vector<Item> items;
  size_t total = 0;
  Pinned stage;
  template <typename T, typename P>
  void add(P** dst, const std::vector<T>& v) {
    const size_t off = (total + 255) & ~size_t(255);
    total = off + std::max<size_t>(1, v.size()) * sizeof(T);
    items.push_back({reinterpret_cast<void**>(const_cast<typename std::remove_const<P>::type**>(dst)),
                     v.data(), v.size() * sizeof(T), off});
  }
  void commit(rsd_ctx* h, hipStream_t s) {
    char* d = dalloc<char>(h, total);
    stage = palloc(h, total);
    char* hs = static_cast<char*>(stage.p);
    for (const Item& it : items)
      if (it.bytes) std::memcpy(hs + it.off, it.src, it.bytes);
    hip_check(h, hipMemcpyAsync(d, hs, total, hipMemcpyHostToDevice, s), "hipMemcpyAsync H2D");
    for (const Item& it : items) *it.dst = d + it.off;
  }
  void done(rsd_ctx* h) { pfree(h, stage); }
};

// Times the launches enqueued during its lifetime on stream s (when timing is on).
struct Timer {
  rsd_ctx* h;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Timer(rsd_ctx* h_, int cls_, hipStream_t s_) : h(h_), cls(cls_), s(s_) {
    h->launches[cls]++;
    if (!h->opt.timing) return;
    a = take();
    hip_check(h, hipEventRecord(a, s), "hipEventRecord");
  }
  ~Timer() {
    if (!a) return;
    hipEvent_t b = take();
    (void)hipEventRecord(b, s);
    h->pending.push_back({cls, a, b});
  }
  hipEvent_t take() {
    if (!h->pool.empty()) {
      hipEvent_t e = h->pool.back();
      h->pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hip_check(h, hipEventCreate(&e), "hipEventCreate");
    return e;
  }
};

double ms_since(std::chrono::steady_clock::time_point t) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

void fold_timings(rsd_ctx* h) {
  for (auto& p : h->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess)
      h->time_ms[p.cls] += ms;
    h->pool.push_back(p.a);
    h->pool.push_back(p.b);
  }
  h->pending.clear();
}

void upload_batch(rsd_ctx* h, Uploader& up, DevBatch* d, const SymBatch& b, bool fp32) {
  d->count = b.count;
  d->max_nt = b.max_nt;
  d->max_tiles = b.max_tiles;
  up.add(&d->n, b.n);
  up.add(&d->nt, b.nt);
  up.add(&d->tile_off, b.tile_off);
  up.add(&d->vec_off, b.vec_off);
  d->num_items = int32_t(b.num_items);
  up.add(&d->item_mat, b.item_mat);
  up.add(&d->item_BI, b.item_BI);
  up.add(&d->item_BJ, b.item_BJ);
  up.add(&d->item_base, b.item_base);
  d->fp32 = fp32 ? 1 : 0;
  if (b.total_elems > 0) {
    if (fp32)
      d->tiles = dalloc<float>(h, size_t(b.total_elems));
    else
      d->tiles = dalloc<double>(h, size_t(b.total_elems));
  }
}

// Blocked sweep inversion of a batch; the MFMA update launches are timed as `upd`.
// With two- or four-tile pivot groups the next step's pivot and panel run on the auxiliary
// stream as soon as the tiles they read are updated (look-ahead), overlapping the
// bulk of the current update; the panel buffers alternate between steps.
// Pivot tiles per sweep step: four (K = 256 for the MFMA update, half the passes over
// the matrix) unless the matrices are small; RSD_SWEEP_GROUP overrides.
int group_for(const rsd_ctx* h, const DevBatch& b) {
  if (h->group > 0) return h->group;
  return b.max_nt >= 16 ? 4 : 2;
}

void invert_batch(rsd_ctx* h, const DevBatch& b, void* pbuf, void* cbuf[2], void* bbuf[2],
                  int32_t* flags, int upd, hipStream_t s) {
  const int G = group_for(h, b);
  if (b.count == 0 || b.max_nt == 0) return;
  if (G < 2) {
    for (int c0 = 0; c0 < b.max_nt; c0 += G) {
      hip_check(h, launch_sweep_step(b, c0, 0, pbuf, cbuf[0], bbuf[0], flags, G, s), "sweep pivot");
      hip_check(h, launch_sweep_step(b, c0, 1, pbuf, cbuf[0], bbuf[0], flags, G, s), "sweep panel");
      Timer tm(h, upd, s);
      hip_check(h, launch_sweep_step(b, c0, 2, pbuf, cbuf[0], bbuf[0], flags, G, s), "sweep update");
    }
    return;
  }
  hipStream_t a = h->aux;
  hip_check(h, launch_sweep_step(b, 0, 0, pbuf, cbuf[0], bbuf[0], flags, G, s), "sweep pivot");
  hip_check(h, launch_sweep_step(b, 0, 1, pbuf, cbuf[0], bbuf[0], flags, G, s), "sweep panel");
  int k = 0;
  for (int c0 = 0; c0 < b.max_nt; c0 += G, ++k) {
    const int cur = k & 1, nxt = cur ^ 1;
    const bool more = c0 + G < b.max_nt;
    if (more) {
      {
        Timer tm(h, upd, s);
        hip_check(h, launch_sweep_step(b, c0, 2, pbuf, cbuf[cur], bbuf[cur], flags, G, s, 1),
                  "sweep update (look-ahead part)");
      }
      hip_check(h, hipEventRecord(h->ev_main, s), "hipEventRecord");
      hip_check(h, hipStreamWaitEvent(a, h->ev_main, 0), "hipStreamWaitEvent");
      hip_check(h, launch_sweep_step(b, c0 + G, 0, pbuf, cbuf[nxt], bbuf[nxt], flags, G, a),
                "sweep pivot");
      hip_check(h, launch_sweep_step(b, c0 + G, 1, pbuf, cbuf[nxt], bbuf[nxt], flags, G, a),
                "sweep panel");
      hip_check(h, hipEventRecord(h->ev_aux, a), "hipEventRecord");
    }
    {
      Timer tm(h, upd, s);
      hip_check(h, launch_sweep_step(b, c0, 2, pbuf, cbuf[cur], bbuf[cur], flags, G, s,
                                     more ? 2 : 0), "sweep update");
    }
    if (more) hip_check(h, hipStreamWaitEvent(s, h->ev_aux, 0), "hipStreamWaitEvent");
  }
}

}  // namespace

void fill_analysis(const Plan& P, rsd_analysis* a) {
  std::memset(a, 0, sizeof(*a));
  a->num_leaves = int32_t(P.leaf_node.size());
  a->num_levels = int32_t(P.level_depth.size());
  a->max_leaf_dofs = P.max_leaf;
  a->max_iface_dofs = P.max_iface;
  a->max_boundary_dofs = P.max_m;
  a->leaf_dofs = P.n_leaf;
  a->skeleton_dofs = P.n - P.n_leaf;
  a->sum_leaf_sq = P.sum_leaf_sq;
  a->sum_iface_sq = P.sum_iface_sq;
  a->sum_sigma_apply = P.sum_sigma_apply;
  a->sum_sigma_sq = P.sum_sigma_sq;
  a->leaf_inverse_flops = P.leaf_flops;
  a->iface_inverse_flops = P.iface_flops;
}

rsd_status engine_init(rsd_ctx* h, const rsd_csr* csr, const rsd_hierarchy* hier,
                       const rsd_options* opt, hipStream_t s) {
  try {
    if (opt) {
      h->opt = *opt;
    } else {
      rsd_options_default(&h->opt);
    }
    const auto w0 = std::chrono::steady_clock::now();
    const int32_t n = csr->n;
    const int64_t nnz = csr->nnz;
    const int32_t T = hier->num_nodes;
    h->cur = s;
    // ---- host copies of the structure (pinned staging when it lives on the device)
    const int64_t* rpp = csr->row_ptr;
    const int32_t* cip = csr->col_idx;
    const int32_t* parp = hier->parent;
    const int32_t* dnp = hier->dof_node;
    Pinned stage;
    if (!h->opt.host_pointers) {
      hip_check(h, hipGetDevice(&h->device), "hipGetDevice");
      const size_t b_rp = size_t(n + 1) * 8, b_ci = size_t(nnz) * 4, b_par = size_t(T) * 4;
      const size_t o_ci = b_rp, o_par = o_ci + ((b_ci + 7) & ~size_t(7)), o_dn = o_par + ((b_par + 7) & ~size_t(7));
      stage = palloc(h, o_dn + size_t(n) * 4);
      char* hs = static_cast<char*>(stage.p);
      hip_check(h, hipMemcpyAsync(hs, csr->row_ptr, b_rp, hipMemcpyDeviceToHost, s), "copy row_ptr");
      if (nnz > 0)
        hip_check(h, hipMemcpyAsync(hs + o_ci, csr->col_idx, b_ci, hipMemcpyDeviceToHost, s), "copy col_idx");
      hip_check(h, hipMemcpyAsync(hs + o_par, hier->parent, b_par, hipMemcpyDeviceToHost, s), "copy parent");
      hip_check(h, hipMemcpyAsync(hs + o_dn, hier->dof_node, size_t(n) * 4, hipMemcpyDeviceToHost, s), "copy dof_node");
      hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
      rpp = reinterpret_cast<const int64_t*>(hs);
      cip = reinterpret_cast<const int32_t*>(hs + o_ci);
      parp = reinterpret_cast<const int32_t*>(hs + o_par);
      dnp = reinterpret_cast<const int32_t*>(hs + o_dn);
    }
    const auto t0 = std::chrono::steady_clock::now();
    std::string msg;
    const PlanError pe = build_plan(n, nnz, rpp, cip, T, parp, dnp, &h->P, &msg);
    h->host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    pfree(h, stage);
    if (pe != PlanError::kOk) {
      h->err = msg;
      return pe == PlanError::kNotSeparable ? RSD_ERR_MAP_NOT_SEPARABLE : RSD_ERR_INVALID_ARGUMENT;
    }
    h->setup_wall[0] = ms_since(w0);
    const auto w1 = std::chrono::steady_clock::now();
    hip_check(h, hipGetDevice(&h->device), "hipGetDevice");
    // auxiliary stream (shared, default priority) and events of the inversion look-ahead
    h->aux = aux_stream(h);
    hip_check(h, hipEventCreateWithFlags(&h->ev_main, hipEventDisableTiming), "hipEventCreate");
    hip_check(h, hipEventCreateWithFlags(&h->ev_aux, hipEventDisableTiming), "hipEventCreate");
    const Plan& P = h->P;
    h->group = 0;
    if (const char* g = std::getenv("RSD_SWEEP_GROUP")) {
      const int v = std::atoi(g);
      h->group = (v == 1 || v == 2 || v == 4) ? v : 0;
    }
    // ---- upload structure (one allocation, one copy)
    Uploader up;
    up.add(&h->prow, P.prow);
    up.add(&h->perm, P.perm);
    up.add(&h->iperm, P.iperm);
    up.add(&h->skel_lvl_begin, P.skel_lvl_begin);
    up.add(&h->skel_own_end, P.skel_own_end);
    up.add(&h->ell_off, P.ell_off);
    h->ell_col = dalloc<int32_t>(h, size_t(P.ell_off.back()));
    h->ell_val = dalloc<double>(h, size_t(P.ell_off.back()));
    h->pcol = dalloc<int32_t>(h, size_t(nnz));
    h->pmap = dalloc<int64_t>(h, size_t(nnz));
    h->segA = dalloc<int64_t>(h, size_t(n));
    h->segB = dalloc<int64_t>(h, size_t(n));
    h->segC = dalloc<int64_t>(h, size_t(n));
    h->pval = dalloc<double>(h, size_t(nnz));
    up.add(&h->B_off, P.B_off);
    up.add(&h->B, P.B);
    up.add(&h->adj_ptr, P.adj_ptr);
    up.add(&h->adj_leaf, P.adj_leaf);
    up.add(&h->adj_pos, P.adj_pos);
    up.add(&h->sig_off_d, P.sig_off);
    SigmaArgs& a = h->sig;
    a.num_leaves = int32_t(P.leaf_node.size());
    a.max_m = P.max_m;
    up.add(&a.shell_off, P.shell_off);
    up.add(&a.shell, P.shell);
    up.add(&a.kcol_ptr, P.kcol_ptr);
    up.add(&a.kcol_row, P.kcol_row);
    up.add(&h->kcol_pos, P.kcol_val);
    up.add(&a.krow_ptr, P.krow_ptr);
    up.add(&a.krow_col, P.krow_col);
    up.add(&h->krow_pos, P.krow_val);
    up.add(&a.w_off, P.w_off);
    h->kcol_v = dalloc<double>(h, P.kcol_val.size());
    h->krow_v = dalloc<double>(h, P.krow_val.size());
    a.kcol_v = h->kcol_v;
    a.krow_v = h->krow_v;
    h->sigma_fp32 = h->opt.sigma_prec == RSD_PREC_FP32;
    if (h->sigma_fp32)
      h->sigma = dalloc<float>(h, size_t(P.sig_total));
    else
      h->sigma = dalloc<double>(h, size_t(P.sig_total));
    upload_batch(h, up, &h->leaf, P.leaf_batch, h->opt.leaf_prec == RSD_PREC_FP32);
    const int NL = int(P.level_depth.size());
    h->lev.assign(NL, DevBatch());
    h->lev_items.assign(NL, SigmaLevelItems());

    std::vector<std::vector<int32_t>> il(NL), ir0(NL), ia0(NL), ia1(NL);
    for (int q = 0; q < NL; ++q) {
      const bool root = P.level_depth[q] == 0;
      const int prec = root ? h->opt.root_prec : h->opt.iface_prec;
      upload_batch(h, up, &h->lev[q], P.level_batch[q], prec == RSD_PREC_FP32);
      // Sigma products of this level, split into row chunks of kSigRows
      for (const auto& it : P.level_sigma[q])
        for (int32_t a0 = it.r0; a0 < it.r1; a0 += kSigRows) {
          il[q].push_back(it.leaf);
          ir0[q].push_back(it.r0);
          ia0[q].push_back(a0);
          ia1[q].push_back(std::min(it.r1, a0 + kSigRows));
        }
      SigmaLevelItems& li = h->lev_items[q];
      li.count = int32_t(il[q].size());
      up.add(&li.leaf, il[q]);
      up.add(&li.r0, ir0[q]);
      up.add(&li.a0, ia0[q]);
      up.add(&li.a1, ia1[q]);
    }
    // the caller's CSR structure on the device (copied when given on the host)
    const int64_t* d_rp = csr->row_ptr;
    const int32_t* d_ci = csr->col_idx;
    int64_t* tmp_rp = nullptr;
    int32_t* tmp_ci = nullptr;
    if (h->opt.host_pointers) {
      std::vector<int64_t> vr(csr->row_ptr, csr->row_ptr + n + 1);
      std::vector<int32_t> vc(csr->col_idx, csr->col_idx + nnz);
      up.add(&tmp_rp, vr);
      up.add(&tmp_ci, vc);
      up.commit(h, s);
      d_rp = tmp_rp;
      d_ci = tmp_ci;
    } else {
      up.commit(h, s);
    }
    hip_check(h, launch_permute_csr(n, P.n_leaf, h->perm, h->iperm, d_rp, d_ci, h->prow,
                                    h->skel_lvl_begin, h->skel_own_end, h->pcol, h->pmap,
                                    h->segA, h->segB, h->segC, s), "permute csr");
    a.B_off = h->B_off;
    a.B = h->B;
    a.sig_off = h->sig_off_d;
    const int64_t nflags = int64_t(P.leaf_node.size()) + int64_t(P.iface_node.size());
    h->flags = dalloc<int32_t>(h, size_t(nflags));
    h->e = dalloc<double>(h, std::max<size_t>(1, P.B.size()));
    h->t = dalloc<double>(h, size_t(n));
    h->rin = dalloc<double>(h, size_t(n));
    h->zin = dalloc<double>(h, size_t(n));
    size_t part_bytes = std::max<size_t>(8, symv_part_bytes(h->leaf));
    for (const DevBatch& d : h->lev) part_bytes = std::max(part_bytes, symv_part_bytes(d));
    h->sympart = dalloc<double>(h, (part_bytes + 7) / 8);
    hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
    up.done(h);
    h->setup_wall[1] = ms_since(w1);
    return RSD_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

// Dense set-up from the values of K (caller order, device pointer): Section 3.1's
// exact sub-domain inverses, the Sigma_l blocks, and per interface level the
// operator of Alg. 1 assembled and inverted.
rsd_status engine_numeric(rsd_ctx* h, const double* values, hipStream_t s) {
  try {
    h->cur = s;
    const auto w2 = std::chrono::steady_clock::now();
    const Plan& P = h->P;
    {
      Timer tm(h, RSD_T_SETUP_EXTRACT, s);
      hip_check(h, launch_gather(values, h->pmap, P.nnz, h->pval, s), "gather values");
      hip_check(h, launch_ell_fill(P.n, h->prow, h->pcol, h->pval, h->ell_off, h->ell_col,
                                   h->ell_val, s), "ELL fill");
      hip_check(h, launch_gather(values, h->kcol_pos, int64_t(P.kcol_val.size()), h->kcol_v, s),
                "gather couplings");
      hip_check(h, launch_gather(values, h->krow_pos, int64_t(P.krow_val.size()), h->krow_v, s),
                "gather couplings");
      const int64_t nflags = int64_t(P.leaf_node.size()) + int64_t(P.iface_node.size());
      hip_check(h, hipMemsetAsync(h->flags, 0, size_t(nflags) * 4, s), "hipMemsetAsync flags");
      hip_check(h, launch_sym_fill(h->leaf, s), "leaf fill");
      hip_check(h, launch_sym_extract(h->leaf, h->prow, h->segA, h->pcol, h->pval, P.max_leaf, s),
                "leaf extract");
    }
    // scratch of the sweeps: sized for the largest batch
    size_t pb = 0, cb = 0, need_p = 0, need_c = 0;
    sym_invert_scratch_bytes(h->leaf, group_for(h, h->leaf), &pb, &cb);
    need_p = pb;
    need_c = cb;
    for (const auto& L : h->lev) {
      sym_invert_scratch_bytes(L, group_for(h, L), &pb, &cb);
      need_p = std::max(need_p, pb);
      need_c = std::max(need_c, cb);
    }
    char* pbuf = dalloc<char>(h, need_p);
    void* cbuf[2] = {dalloc<char>(h, need_c), dalloc<char>(h, need_c)};
    void* bbuf[2] = {dalloc<char>(h, need_c), dalloc<char>(h, need_c)};
    {
      Timer tm(h, RSD_T_LEAF_INVERSE, s);
      invert_batch(h, h->leaf, pbuf, cbuf, bbuf, h->flags, RSD_T_LEAF_UPDATE, s);
    }
    double* W = dalloc<double>(h, size_t(std::max<int64_t>(1, P.w_total)));
    {
      Timer tm(h, RSD_T_SIGMA, s);
      hip_check(h, launch_sigma_w(h->leaf, h->sig, W, s), "sigma W");
      hip_check(h, launch_sigma_s(h->sig, W, h->sigma, h->sigma_fp32, s), "sigma S");
    }
    int32_t* iflags = h->flags + P.leaf_node.size();
    for (size_t q = 0; q < h->lev.size(); ++q) {
      {
        Timer tm(h, RSD_T_IFACE_ASSEMBLY, s);
        int32_t maxn = 0;
        for (int32_t v : P.level_batch[q].n) maxn = std::max(maxn, v);
        hip_check(h, launch_sym_fill(h->lev[q], s), "iface fill");
        hip_check(h, launch_sym_extract(h->lev[q], h->segB, h->segC, h->pcol, h->pval, maxn, s),
                  "iface extract");
        hip_check(h, launch_schur_assemble(h->lev[q], h->adj_ptr, h->adj_leaf, h->adj_pos,
                                           h->B_off, h->sig_off_d, h->sigma, h->sigma_fp32,
                                           P.n_leaf, s),
                  "schur assembly");
      }
      {
        Timer tm(h, RSD_T_IFACE_INVERSE, s);
        invert_batch(h, h->lev[q], pbuf, cbuf, bbuf, iflags + P.level_iface_begin[q],
                     P.level_depth[q] == 0 ? RSD_T_ROOT_UPDATE : RSD_T_IFACE_UPDATE, s);
      }
    }
    h->setup_wall[2] = ms_since(w2);
    const auto w3 = std::chrono::steady_clock::now();
    std::vector<int32_t> fl(P.leaf_node.size() + P.iface_node.size());
    if (!fl.empty())
      hip_check(h, hipMemcpyAsync(fl.data(), h->flags, fl.size() * 4, hipMemcpyDeviceToHost, s),
                "flags D2H");
    hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
    dfree(h, W);
    dfree(h, pbuf);
    for (int i = 0; i < 2; ++i) {
      dfree(h, cbuf[i]);
      dfree(h, bbuf[i]);
    }
    h->setup_wall[3] = ms_since(w3);
    for (size_t i = 0; i < fl.size(); ++i)
      if (fl[i]) {
        char buf[256];
        if (i < P.leaf_node.size())
          std::snprintf(buf, sizeof(buf),
                        "sub-domain matrix of leaf node %d is not positive definite "
                        "(non-positive pivot near tile column %d)",
                        P.leaf_node[i], fl[i] - 1);
        else
          std::snprintf(buf, sizeof(buf),
                        "interface Schur complement of node %d is not positive definite "
                        "(non-positive pivot near tile column %d)",
                        P.iface_node[i - P.leaf_node.size()], fl[i] - 1);
        h->err = buf;
        return RSD_ERR_NOT_SPD;
      }
    return RSD_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

namespace {

// z = M^{-1} r on internal-order vectors (Alg. 2 with exact interface solves):
// every sub-domain solve; per interface level from the deepest: right-hand side g
// of eq. (schur) -- the interface part of r minus the couplings to the already
// computed values below it -- and the interface solve; then the back-substitution
// of eq. (backSub) on every sub-domain at once.
void core_apply(rsd_ctx* h, const double* r, double* z, hipStream_t s) {
  const Plan& P = h->P;
  const int64_t n = P.n, nl = P.n_leaf;
  {
    Timer tm(h, RSD_T_LEAF_APPLY, s);
    hip_check(h, launch_symv(h->leaf, r, h->sympart, -1.0, nullptr, z, s), "leaf symv");
  }
  {
    Timer tm(h, RSD_T_COUPLING, s);
    // interface rows: q_B = r_B - K_{B,leaves} y
    hip_check(h, launch_ell_spmv(nl, n - nl, h->prow, h->segA, h->prow, h->ell_off, h->ell_col,
                                 h->ell_val, z, r, -1.0, z, s), "condense");
    hip_check(h, launch_fill(h->e, int64_t(P.B.size()), 0.0, s), "fill e");
  }
  for (size_t q = 0; q < h->lev.size(); ++q) {
    {
      Timer tm(h, RSD_T_COUPLING, s);
      hip_check(h, launch_sigma_level(h->lev_items[q], h->sigma, h->sigma_fp32, h->sig_off_d,
                                      h->B_off, h->B, z, h->e, s), "sigma level");
      const int64_t r0 = P.level_dof_begin[q], r1 = P.level_dof_end[q];
      hip_check(h, launch_level_rhs(r0, r1 - r0, nl, h->pcol, h->pval, h->segA, h->segB,
                                    h->adj_ptr, h->adj_leaf, h->adj_pos, h->B_off, h->e, z, s),
                "level rhs");
    }
    {
      Timer tm(h, RSD_T_IFACE_APPLY, s);
      hip_check(h, launch_symv(h->lev[q], z, h->sympart, -1.0, nullptr, z, s),
                "interface symv");
    }
  }
  {
    Timer tm(h, RSD_T_COUPLING, s);
    // leaf rows: r_l - K_{l,B} u_B
    hip_check(h, launch_ell_spmv(0, nl, h->segA, h->prow + 1, h->prow, h->ell_off, h->ell_col,
                                 h->ell_val, z, r, -1.0, h->t, s), "back-substitution rhs");
  }
  {
    Timer tm(h, RSD_T_LEAF_APPLY, s);
    hip_check(h, launch_symv(h->leaf, h->t, h->sympart, -1.0, nullptr, z, s), "leaf symv");
  }
}

void core_spmv(rsd_ctx* h, const double* x, const double* base, double alpha, double* y,
               hipStream_t s) {
  Timer tm(h, RSD_T_SPMV, s);
  hip_check(h, launch_ell_spmv(0, h->P.n, h->prow, h->prow + 1, h->prow, h->ell_off, h->ell_col,
                               h->ell_val, x, base, alpha, y, s), "spmv");
}

void permute(rsd_ctx* h, const double* x, int64_t ldx, double* y, int64_t ldy, int inverse,
             hipStream_t s) {
  Timer tm(h, RSD_T_PERMUTE, s);
  hip_check(h, launch_permute(x, ldx, y, ldy, h->perm, h->P.n, 1, inverse, s), "permute");
}

void ensure_krylov(rsd_ctx* h, int m) {
  if (h->kry_m >= m && h->V) return;
  if (h->V) hip_check(h, hipStreamSynchronize(h->cur), "hipStreamSynchronize");  // before reuse
  for (double* p : {h->V, h->Z, h->w, h->hdev, h->tmp, h->part, h->scal, h->bint, h->xint})
    dfree(h, p);
  pfree(h, h->hhost_block);
  const size_t n = size_t(h->P.n);
  h->V = dalloc<double>(h, n * size_t(m + 1));
  h->Z = dalloc<double>(h, n * size_t(m));
  h->w = dalloc<double>(h, n);
  h->hdev = dalloc<double>(h, size_t(m + 2));
  h->tmp = dalloc<double>(h, size_t(m + 2));
  h->part = dalloc<double>(h, size_t(mdot_blocks(h->P.n)) * size_t(m + 2));
  h->scal = dalloc<double>(h, 16);
  h->bint = dalloc<double>(h, n);
  h->xint = dalloc<double>(h, n);
  h->hhost_block = palloc(h, sizeof(double) * size_t(m + 16));
  h->hhost = static_cast<double*>(h->hhost_block.p);
  h->kry_m = m;
}

double dev_norm(rsd_ctx* h, const double* v, double* out_dev, hipStream_t s) {
  {
    Timer tm(h, RSD_T_KRYLOV, s);
    hip_check(h, launch_mdot(v, h->P.n, 1, v, h->P.n, h->part, out_dev, 1, s), "norm");
  }
  hip_check(h, hipMemcpyAsync(h->hhost, out_dev, 8, hipMemcpyDeviceToHost, s), "D2H");
  hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
  return h->hhost[0];
}

// Right-preconditioned flexible GMRES(m) in internal order; x (internal) holds the
// initial guess.  Returns the status of this right-hand side.
rsd_status fgmres_one(rsd_ctx* h, const double* b, double* x, const rsd_solve_options& o,
                      rsd_solve_info* info, hipStream_t s) {
  const int64_t n = h->P.n;
  const int m = o.restart;
  double* beta_d = h->scal;      // scal[0]: ||r||, scal[1]: ||b||
  const double bnorm = dev_norm(h, b, h->scal + 1, s);
  if (!(bnorm == bnorm) || std::isinf(bnorm)) {
    info->iterations = 0;
    info->relres = NAN;
    return RSD_ERR_BREAKDOWN;
  }
  if (bnorm == 0.0) {
    hip_check(h, launch_fill(x, n, 0.0, s), "zero x");
    info->iterations = 0;
    info->relres = 0.0;
    return RSD_OK;
  }
  const double tol = o.rtol * bnorm;
  double* r = h->w;
  core_spmv(h, x, b, -1.0, r, s);
  double beta = dev_norm(h, r, beta_d, s);
  int its = 0;
  std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  for (;;) {
    if (beta <= tol) {
      info->iterations = its;
      info->relres = beta / bnorm;
      return RSD_OK;
    }
    if (!(beta == beta)) {
      info->iterations = its;
      info->relres = NAN;
      return RSD_ERR_BREAKDOWN;
    }
    if (its >= o.maxit) {
      info->iterations = its;
      info->relres = beta / bnorm;
      return RSD_ERR_NOT_CONVERGED;
    }
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      hip_check(h, launch_scale_div(r, beta_d, h->V, n, s), "v0");
    }
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool bad = false;
    for (int j = 0; j < m; ++j) {
      double* vj = h->V + size_t(j) * n;
      double* zj = h->Z + size_t(j) * n;
      core_apply(h, vj, zj, s);
      core_spmv(h, zj, nullptr, 1.0, h->w, s);
      {
        Timer tm(h, RSD_T_KRYLOV, s);
        // classical Gram-Schmidt, twice
        hip_check(h, launch_mdot(h->V, n, j + 1, h->w, n, h->part, h->hdev, 0, s), "cgs dots");
        hip_check(h, launch_gemv_acc(h->V, n, j + 1, h->hdev, -1.0, h->w, n, s), "cgs update");
        hip_check(h, launch_mdot(h->V, n, j + 1, h->w, n, h->part, h->tmp, 0, s), "cgs2 dots");
        hip_check(h, launch_gemv_acc(h->V, n, j + 1, h->tmp, -1.0, h->w, n, s), "cgs2 update");
        hip_check(h, launch_small_add(h->hdev, h->tmp, j + 1, s), "h add");
        hip_check(h, launch_mdot(h->w, n, 1, h->w, n, h->part, h->hdev + j + 1, 1, s), "norm");
        hip_check(h, launch_scale_div(h->w, h->hdev + j + 1, h->V + size_t(j + 1) * n, n, s),
                  "normalise");
      }
      hip_check(h, hipMemcpyAsync(h->hhost, h->hdev, sizeof(double) * size_t(j + 2),
                                  hipMemcpyDeviceToHost, s), "h D2H");
      hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
      double* hc = &H[size_t(j) * (m + 1)];
      for (int i = 0; i <= j + 1; ++i) {
        hc[i] = h->hhost[i];
        if (!(hc[i] == hc[i]) || std::isinf(hc[i])) bad = true;
      }
      if (bad) break;
      const double hnext = hc[j + 1];
      for (int i = 0; i < j; ++i) {
        const double t0 = cs[i] * hc[i] + sn[i] * hc[i + 1];
        hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
        hc[i] = t0;
      }
      const double den = std::hypot(hc[j], hc[j + 1]);
      cs[j] = den > 0 ? hc[j] / den : 1.0;
      sn[j] = den > 0 ? hc[j + 1] / den : 0.0;
      hc[j] = den;
      hc[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      k = j + 1;
      if (std::fabs(g[j + 1]) <= tol || its >= o.maxit || hnext == 0.0) break;
    }
    if (bad) {
      info->iterations = its;
      info->relres = NAN;
      return RSD_ERR_BREAKDOWN;
    }
    // y = R^{-1} g (upper triangular k x k)
    for (int i = k - 1; i >= 0; --i) {
      double v = g[i];
      for (int c = i + 1; c < k; ++c) v -= H[size_t(c) * (m + 1) + i] * y[c];
      const double d = H[size_t(i) * (m + 1) + i];
      y[i] = d != 0.0 ? v / d : 0.0;
    }
    for (int i = 0; i < k; ++i) h->hhost[i] = y[i];
    hip_check(h, hipMemcpyAsync(h->tmp, h->hhost, sizeof(double) * size_t(k),
                                hipMemcpyHostToDevice, s), "y H2D");
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      hip_check(h, launch_gemv_acc(h->Z, n, k, h->tmp, 1.0, x, n, s), "x update");
    }
    core_spmv(h, x, b, -1.0, r, s);
    beta = dev_norm(h, r, beta_d, s);
  }
}

// Preconditioned CG in internal order (x holds the initial guess).
rsd_status pcg_one(rsd_ctx* h, const double* b, double* x, const rsd_solve_options& o,
                   rsd_solve_info* info, hipStream_t s) {
  const int64_t n = h->P.n;
  // columns of V: r, z, p, q ; scalars: scal[0..1] rz (ping-pong), scal[2] pq, scal[3] norm
  double* r = h->V;
  double* z = h->V + n;
  double* p = h->V + 2 * n;
  double* q = h->V + 3 * n;
  const double bnorm = dev_norm(h, b, h->scal + 4, s);
  if (!(bnorm == bnorm) || std::isinf(bnorm)) {
    info->iterations = 0;
    info->relres = NAN;
    return RSD_ERR_BREAKDOWN;
  }
  if (bnorm == 0.0) {
    hip_check(h, launch_fill(x, n, 0.0, s), "zero x");
    info->iterations = 0;
    info->relres = 0.0;
    return RSD_OK;
  }
  const double tol = o.rtol * bnorm;
  core_spmv(h, x, b, -1.0, r, s);
  double rn = dev_norm(h, r, h->scal + 3, s);
  int its = 0;
  int cur = 0;
  if (rn <= tol) {
    info->iterations = 0;
    info->relres = rn / bnorm;
    return RSD_OK;
  }
  core_apply(h, r, z, s);
  {
    Timer tm(h, RSD_T_KRYLOV, s);
    hip_check(h, launch_mdot(r, n, 1, z, n, h->part, h->scal + cur, 0, s), "rz");
    hip_check(h, hipMemcpyAsync(p, z, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, s),
              "p = z");
  }
  for (;;) {
    core_spmv(h, p, nullptr, 1.0, q, s);
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      hip_check(h, launch_mdot(p, n, 1, q, n, h->part, h->scal + 2, 0, s), "pq");
      hip_check(h, launch_axpy_ratio(x, p, h->scal + cur, h->scal + 2, 1.0, x, n, s), "x");
      hip_check(h, launch_axpy_ratio(r, q, h->scal + cur, h->scal + 2, -1.0, r, n, s), "r");
      hip_check(h, launch_mdot(r, n, 1, r, n, h->part, h->scal + 3, 1, s), "|r|");
    }
    hip_check(h, hipMemcpyAsync(h->hhost, h->scal, sizeof(double) * 4, hipMemcpyDeviceToHost, s),
              "D2H");
    hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
    ++its;
    rn = h->hhost[3];
    const double pq = h->hhost[2];
    if (!(rn == rn) || !(pq > 0.0) || std::isinf(rn)) {
      info->iterations = its;
      info->relres = NAN;
      return RSD_ERR_BREAKDOWN;
    }
    if (rn <= tol) {
      core_spmv(h, x, b, -1.0, r, s);
      const double rt = dev_norm(h, r, h->scal + 3, s);
      if (rt <= tol) {
        info->iterations = its;
        info->relres = rt / bnorm;
        return RSD_OK;
      }
    }
    if (its >= o.maxit) {
      core_spmv(h, x, b, -1.0, h->w, s);
      info->iterations = its;
      info->relres = dev_norm(h, h->w, h->scal + 5, s) / bnorm;
      return RSD_ERR_NOT_CONVERGED;
    }
    core_apply(h, r, z, s);
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      const int nxt = 1 - cur;
      hip_check(h, launch_mdot(r, n, 1, z, n, h->part, h->scal + nxt, 0, s), "rz");
      hip_check(h, launch_axpy_ratio(z, p, h->scal + nxt, h->scal + cur, 1.0, p, n, s), "p");
      cur = nxt;
    }
  }
}

}  // namespace

rsd_status engine_apply(rsd_ctx* h, int nrhs, const double* r, int64_t ldr, double* z,
                        int64_t ldz, hipStream_t s) {
  try {
    for (int j = 0; j < nrhs; ++j) {
      permute(h, r + size_t(j) * ldr, h->P.n, h->rin, h->P.n, 0, s);
      core_apply(h, h->rin, h->zin, s);
      permute(h, h->zin, h->P.n, z + size_t(j) * ldz, h->P.n, 1, s);
    }
    return RSD_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

rsd_status engine_spmv(rsd_ctx* h, int nrhs, const double* x, int64_t ldx, double* y,
                       int64_t ldy, hipStream_t s) {
  try {
    for (int j = 0; j < nrhs; ++j) {
      permute(h, x + size_t(j) * ldx, h->P.n, h->rin, h->P.n, 0, s);
      core_spmv(h, h->rin, nullptr, 1.0, h->zin, s);
      permute(h, h->zin, h->P.n, y + size_t(j) * ldy, h->P.n, 1, s);
    }
    return RSD_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

rsd_status engine_solve(rsd_ctx* h, int nrhs, const double* b, int64_t ldb, double* x,
                        int64_t ldx, const rsd_solve_options* opt, rsd_solve_info* info,
                        hipStream_t s) {
  try {
    h->cur = s;
    rsd_solve_options o;
    if (opt) {
      o = *opt;
    } else {
      o.method = RSD_SOLVER_FGMRES;
      o.restart = 30;
      o.maxit = 500;
      o.rtol = 1e-10;
      o.use_x0 = 0;
    }
    ensure_krylov(h, o.method == RSD_SOLVER_PCG ? 4 : o.restart);
    rsd_status worst = RSD_OK;
    for (int j = 0; j < nrhs; ++j) {
      rsd_solve_info inf{0, 0.0, RSD_OK};
      permute(h, b + size_t(j) * ldb, h->P.n, h->bint, h->P.n, 0, s);
      if (o.use_x0)
        permute(h, x + size_t(j) * ldx, h->P.n, h->xint, h->P.n, 0, s);
      else
        hip_check(h, launch_fill(h->xint, h->P.n, 0.0, s), "x0");
      const rsd_status st = o.method == RSD_SOLVER_PCG ? pcg_one(h, h->bint, h->xint, o, &inf, s)
                                                       : fgmres_one(h, h->bint, h->xint, o, &inf, s);
      permute(h, h->xint, h->P.n, x + size_t(j) * ldx, h->P.n, 1, s);
      inf.status = st;
      if (info) info[j] = inf;
      if (st == RSD_ERR_BREAKDOWN || (st != RSD_OK && worst == RSD_OK)) worst = st;
    }
    hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
    if (worst == RSD_ERR_NOT_CONVERGED) h->err = "Krylov iteration reached maxit";
    if (worst == RSD_ERR_BREAKDOWN) h->err = "NaN/Inf or breakdown in the Krylov recurrence";
    return worst;
  } catch (const Fail& f) {
    return f.st;
  }
}

rsd_status engine_stats(rsd_ctx* h, rsd_stats* out, int reset, hipStream_t s) {
  try {
    if (h->opt.timing) {
      hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
      fold_timings(h);
    }
    std::memset(out, 0, sizeof(*out));
    fill_analysis(h->P, &out->analysis);
    for (int i = 0; i < RSD_T_COUNT; ++i) {
      out->time_ms[i] = h->time_ms[i];
      out->launches[i] = h->launches[i];
    }
    out->host_analysis_ms = h->host_ms;
    out->device_bytes = h->device_bytes;
    for (int i = 0; i < 4; ++i) out->setup_wall_ms[i] = h->setup_wall[i];
    if (reset) {
      std::memset(h->time_ms, 0, sizeof(h->time_ms));
      std::memset(h->launches, 0, sizeof(h->launches));
    }
    return RSD_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

void engine_free(rsd_ctx* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  for (auto& p : h->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  if (h->ev_main) (void)hipEventDestroy(h->ev_main);
  if (h->ev_aux) (void)hipEventDestroy(h->ev_aux);
  h->ev_main = h->ev_aux = nullptr;
  h->aux = nullptr;                    // shared by the device's handles: not destroyed
  BlockCache& c = cache_of(h->device);
  for (auto& p : h->allocs) cache_give(c, p.first, p.second, false);   // work is complete
  h->allocs.clear();
  h->device_bytes = 0;
  pfree(h, h->hhost_block);
  h->hhost = nullptr;
}

}  // namespace rsd
