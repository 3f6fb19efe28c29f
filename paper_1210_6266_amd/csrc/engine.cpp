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
#include <string>
#include <unordered_map>
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

// Device blocks of the handle: from the caller's allocator when rsd_options gives one,
// else from the process-wide cache of hipMalloc blocks.
template <typename T>
T* dalloc(rsd_ctx* h, size_t count) {
  const size_t want = round_block(std::max<size_t>(count, 1) * sizeof(T));
  if (h->opt.dev_alloc) {
    void* p = h->opt.dev_alloc(want, h->opt.alloc_ctx);
    if (!p) {
      h->err = "the allocator given in rsd_options returned NULL";
      throw Fail{RSD_ERR_OUT_OF_MEMORY};
    }
    h->allocs.push_back({p, want});
    h->device_bytes += int64_t(want);
    return static_cast<T*>(p);
  }
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
      if (h->opt.dev_free)
        h->opt.dev_free(p, h->opt.alloc_ctx);
      else
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

// Auxiliary (look-ahead) streams: each handle holds one exclusively from set-up to
// destroy, so the set-ups of distinct handles never share a stream; streams released by
// destroyed handles wait in a per-device pool for the next handle (creating a stream is
// not free) until release_cache.  Default priority; ordering between a handle's streams
// is carried by its own events.  The timing events of destroyed handles (timing = 1, two
// per timed launch) wait in the same per-device pool.
struct AuxPool {
  std::mutex mu;
  std::map<int, std::vector<hipStream_t>> idle;   // device -> streams no handle holds
  std::map<int, std::vector<hipEvent_t>> events;  // device -> idle timing events
};
AuxPool& aux_pool() {
  static AuxPool* p = new AuxPool();
  return *p;
}

hipStream_t take_aux(rsd_ctx* h) {
  AuxPool& p = aux_pool();
  {
    std::lock_guard<std::mutex> lock(p.mu);
    std::vector<hipStream_t>& v = p.idle[h->device];
    if (!v.empty()) {
      hipStream_t st = v.back();
      v.pop_back();
      return st;
    }
  }
  hipStream_t st = nullptr;
  hip_check(h, hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
  return st;
}

void give_aux(int device, hipStream_t st) {
  AuxPool& p = aux_pool();
  std::lock_guard<std::mutex> lock(p.mu);
  p.idle[device].push_back(st);
}

// ---- ordering of a handle's calls across streams ------------------------------------------
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st == hipStreamCaptureStatusActive;
}

// start of a call on s: wait for the handle's previous call when it ran on another stream
void enter(rsd_ctx* h, hipStream_t s) {
  if (h->has_last && h->last_s != s && !capturing(s))
    hip_check(h, hipStreamWaitEvent(s, h->ev_last, 0), "hipStreamWaitEvent");
}

// end of a call on s
void leave(rsd_ctx* h, hipStream_t s) {
  if (capturing(s)) return;
  hip_check(h, hipEventRecord(h->ev_last, s), "hipEventRecord");
  h->last_s = s;
  h->has_last = true;
}

// the host waits until every call made on the handle so far has completed
void wait_idle(rsd_ctx* h) {
  if (h->has_last) hip_check(h, hipEventSynchronize(h->ev_last), "hipEventSynchronize");
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
  template <typename V, typename P>
  void add(P** dst, const V& v) {
    using T = typename V::value_type;
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

// Is kernel class cls timed with HIP events (timing on, the class selected)?
bool timed(const rsd_ctx* h, int cls) {
  if (!h->opt.timing || h->no_events) return false;
  return h->opt.timing_classes == 0 || ((h->opt.timing_classes >> cls) & 1) != 0;
}
// ...any of the classes the applications launch (they then run eagerly, not from graphs)
bool apply_timed(const rsd_ctx* h) {
  for (int c : {RSD_T_LEAF_APPLY, RSD_T_IFACE_APPLY, RSD_T_COUPLING, RSD_T_SPMV, RSD_T_KRYLOV})
    if (timed(h, c)) return true;
  return false;
}

// Times the launches enqueued during its lifetime on stream s (when its class is timed).
struct Timer {
  rsd_ctx* h;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Timer(rsd_ctx* h_, int cls_, hipStream_t s_) : h(h_), cls(cls_), s(s_) {
    h->launches[cls]++;
    if (!timed(h, cls)) return;
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
    if (h->pool.empty()) {                     // refill from the process-wide pool
      AuxPool& p = aux_pool();
      std::lock_guard<std::mutex> lock(p.mu);
      std::vector<hipEvent_t>& v = p.events[h->device];
      const size_t k = std::min<size_t>(v.size(), 64);
      h->pool.insert(h->pool.end(), v.end() - long(k), v.end());
      v.resize(v.size() - k);
    }
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

// (tiles = false: the systems' sizes and offsets only, for levels solved matrix-free)
void upload_batch(rsd_ctx* h, Uploader& up, DevBatch* d, const SymBatch& b, bool fp32,
                  bool tiles = true) {
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
  d->split16 = fp32 ? h->split16 : 0;
  if (!tiles) d->num_items = 0;
  if (tiles && b.total_elems > 0) {
    if (fp32)
      d->tiles = dalloc<float>(h, size_t(b.total_elems));
    else
      d->tiles = dalloc<double>(h, size_t(b.total_elems));
  }
}

// Blocked sweep inversion of a batch; the MFMA update launches are timed as `upd`.
// With two- or four-tile pivot groups each step's update is split: the part that the
// next step's pivot and panel read runs first on the main stream, then the next pivot
// and panel follow it there while the bulk of the update runs on the auxiliary stream
// (look-ahead); the panel buffers alternate between steps.  The pivot is queued behind
// an in-stream dependency so that its one workgroup per matrix (large LDS) is dispatched
// before the bulk update's workgroups take every compute unit.
// Pivot tiles per sweep step: four (K = 256 for the MFMA update, half the passes over
// the matrix) unless the matrices are small; RSD_SWEEP_GROUP overrides.
int group_for(const rsd_ctx* h, const DevBatch& b) {
  if (h->group > 0) return h->group;
  return b.max_nt >= 16 ? 4 : 2;
}

void invert_batch(rsd_ctx* h, const DevBatch& b, void* pbuf, void* cbuf[2], void* bbuf[2],
                  int32_t* flags, int upd, bool lookahead, hipStream_t s) {
  const int G = group_for(h, b);
  if (b.count == 0 || b.max_nt == 0) return;
  if (G < 2 || !lookahead) {
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
    if (c0 + G >= b.max_nt) {
      Timer tm(h, upd, s);
      hip_check(h, launch_sweep_step(b, c0, 2, pbuf, cbuf[cur], bbuf[cur], flags, G, s, 0),
                "sweep update");
      break;
    }
    {
      Timer tm(h, upd, s);
      hip_check(h, launch_sweep_step(b, c0, 2, pbuf, cbuf[cur], bbuf[cur], flags, G, s, 1),
                "sweep update (look-ahead part)");
    }
    hip_check(h, hipEventRecord(h->ev_main, s), "hipEventRecord");
    hip_check(h, hipStreamWaitEvent(a, h->ev_main, 0), "hipStreamWaitEvent");
    {
      Timer tm(h, upd, a);
      hip_check(h, launch_sweep_step(b, c0, 2, pbuf, cbuf[cur], bbuf[cur], flags, G, a, 2),
                "sweep update");
    }
    hip_check(h, launch_sweep_step(b, c0 + G, 0, pbuf, cbuf[nxt], bbuf[nxt], flags, G, s),
              "sweep pivot");
    hip_check(h, launch_sweep_step(b, c0 + G, 1, pbuf, cbuf[nxt], bbuf[nxt], flags, G, s),
              "sweep panel");
    hip_check(h, hipEventRecord(h->ev_aux, a), "hipEventRecord");
    hip_check(h, hipStreamWaitEvent(s, h->ev_aux, 0), "hipStreamWaitEvent");
  }
}

// ---- set-up autotuner: the schedule and update shape of each batch's inversion ----------
// Candidates, all with bitwise the same results (every tile receives the same updates from
// the same operands in the same order): 0 look-ahead steps (the next pivot and panel run
// beside the bulk update on the auxiliary stream), 1 serial steps (pivot, panel, whole
// update); for BF16-split batches in four-tile groups also 2 / 3, the same with 256 x 256
// update super-tiles.  The first set-ups of a batch shape in the process try the candidates
// in turn, each timed with HIP events around the batch's inversion (read back after the
// set-up's final synchronisation), and then candidate 0 once more: its first timing comes
// from the process's first set-up, slowed by cold caches and first-use costs.  With every
// candidate timed (candidate 0 by the faster of its two) the fastest is kept for the shape
// (a tie keeps the lower index).  With rsd_options.autotune = 0, candidate 0 throughout.
struct InvTune {
  std::vector<float> ms;
  int32_t best = -1;
};
std::mutex g_inv_mu;
std::unordered_map<std::string, InvTune> g_inv;

int inv_candidates(const DevBatch& b, int G) {
  if (G < 2) return 1;
  return b.split16 && b.fp32 && G == 4 ? 4 : 2;
}

std::string inv_key(const SymBatch& sb, const DevBatch& d, int G) {
  uint64_t hsh = 1469598103934665603ull;                 // FNV-1a over the sizes
  for (int32_t v : sb.n) {
    hsh ^= uint64_t(uint32_t(v));
    hsh *= 1099511628211ull;
  }
  return std::to_string(d.fp32) + ":" + std::to_string(d.split16) + ":" + std::to_string(G) +
         ":" + std::to_string(sb.count) + ":" + std::to_string(hsh);
}

// the candidate for this set-up of the batch; *tuning: time it
int inv_pick(rsd_ctx* h, const std::string& key, int ncand, bool* tuning) {
  *tuning = false;
  if (ncand < 2) return 0;
  std::lock_guard<std::mutex> lk(g_inv_mu);
  InvTune& t = g_inv[key];
  if (t.best >= 0) return t.best;
  if (!h->opt.autotune) return 0;
  *tuning = true;
  return int(t.ms.size()) % ncand;      // 0, 1, ..., ncand - 1, then 0 again
}

void inv_record(const std::string& key, int ncand, int cand, float ms) {
  std::lock_guard<std::mutex> lk(g_inv_mu);
  InvTune& t = g_inv[key];
  // another handle timed this candidate first
  if (t.best >= 0 || int(t.ms.size()) % ncand != cand) return;
  t.ms.push_back(ms);
  if (int(t.ms.size()) == ncand + 1) {
    t.ms[0] = std::min(t.ms[0], t.ms[size_t(ncand)]);
    t.best = 0;
    for (int c = 1; c < ncand; ++c)
      if (t.ms[size_t(c)] < t.ms[size_t(t.best)]) t.best = c;
  }
}

void precapture_apply(rsd_ctx* h);

}  // namespace

// Scratch of the inexact interface solves for nv vectors (nothing without gamma levels);
// the caller guarantees that no queued work uses the previous buffers.
void ensure_gamma(rsd_ctx* h, int nv) {
  if (!h->any_gamma) return;
  dfree(h, h->gm_V);
  dfree(h, h->gm_beta);
  dfree(h, h->gm_H);
  dfree(h, h->gm_steps);
  dfree(h, h->gm_stop);
  dfree(h, h->gm_part);
  dfree(h, h->gm_coef);
  int32_t maxc = 1;
  for (const DevBatch& b : h->lev) maxc = std::max(maxc, b.count);
  const size_t g = size_t(h->opt.gamma), sl = size_t(nv) * size_t(maxc);
  h->gm_V = dalloc<double>(h, (g + 1) * size_t(nv) * size_t(h->P.n));
  h->gm_beta = dalloc<double>(h, sl);
  h->gm_H = dalloc<double>(h, sl * (g + 1) * g);
  h->gm_steps = dalloc<int32_t>(h, sl);
  h->gm_stop = dalloc<int32_t>(h, sl);
  h->gm_part = dalloc<double>(h, size_t(nv) * size_t(std::max(1, h->gm_max_items)) * (g + 1));
  h->gm_coef = dalloc<double>(h, sl * (g + 2));
}

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
    h->csr_stage = stage;                      // read again by build_plan_couplings
    h->ana_rp = rpp;
    h->ana_ci = cip;
    if (pe != PlanError::kOk) {
      h->err = msg;
      return pe == PlanError::kNotSeparable ? RSD_ERR_MAP_NOT_SEPARABLE : RSD_ERR_INVALID_ARGUMENT;
    }
    h->setup_wall[0] = ms_since(w0);
    const auto w1 = std::chrono::steady_clock::now();
    hip_check(h, hipGetDevice(&h->device), "hipGetDevice");
    // auxiliary stream (the handle's own, default priority), events of the inversion
    // look-ahead and of the ordering between calls
    h->aux = take_aux(h);
    h->upl = take_aux(h);
    hip_check(h, hipEventCreateWithFlags(&h->ev_upl, hipEventDisableTiming), "hipEventCreate");
    hip_check(h, hipEventCreateWithFlags(&h->ev_sig, hipEventDisableTiming), "hipEventCreate");
    h->ev_lev.assign(h->P.level_depth.size(), nullptr);
    for (hipEvent_t& e : h->ev_lev)
      hip_check(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    hip_check(h, hipEventCreateWithFlags(&h->ev_main, hipEventDisableTiming), "hipEventCreate");
    hip_check(h, hipEventCreateWithFlags(&h->ev_aux, hipEventDisableTiming), "hipEventCreate");
    hip_check(h, hipEventCreateWithFlags(&h->ev_last, hipEventDisableTiming), "hipEventCreate");
    const Plan& P = h->P;
    h->group = 0;
    if (const char* g = std::getenv("RSD_SWEEP_GROUP")) {
      const int v = std::atoi(g);
      h->group = (v == 1 || v == 2 || v == 4) ? v : 0;
    }
    h->split16 = h->opt.bf16_split ? 1 : 0;
    // per leaf, the first tile row that holds shell rows (the leaf's dofs coupled to
    // interface dofs come last): the back-substitution's correction skips those before it
    std::vector<int32_t> row0(P.leaf_inner.size());
    for (size_t l = 0; l < row0.size(); ++l) row0[l] = P.leaf_inner[l] / kTile;
    // ---- upload structure (one allocation, one copy)
    Uploader up;
    up.add(&h->leaf_row0, row0);
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
    const bool general = h->opt.symmetric == 0;
    upload_batch(h, up, &h->leaf, P.leaf_batch, h->opt.leaf_prec != RSD_PREC_FP64, !general);
    // a K that is not symmetric: dense sub-domain inverses (Gauss-Jordan, partial pivoting)
    std::vector<int64_t> gen_off, perm_off;
    if (general) {
      if (P.max_leaf > kGenMax) {
        h->err = "symmetric = 0 supports sub-domains of at most 2048 dofs";
        return RSD_ERR_UNSUPPORTED;
      }
      GenBatch& g = h->gen;
      g.count = P.leaf_batch.count;
      g.max_n = P.max_leaf;
      g.fp32 = h->opt.leaf_prec == RSD_PREC_FP32;
      gen_off.assign(size_t(g.count) + 1, 0);
      perm_off.assign(size_t(g.count) + 1, 0);
      for (int32_t l = 0; l < g.count; ++l) {
        const int64_t nl_ = P.leaf_batch.n[l];
        gen_off[l + 1] = gen_off[l] + nl_ * nl_;
        perm_off[l + 1] = perm_off[l] + nl_;
      }
      up.add(&g.n, P.leaf_batch.n);
      up.add(&g.vec_off, P.leaf_batch.vec_off);
      up.add(&g.gen_off, gen_off);
      up.add(&g.perm_off, perm_off);
      g.perm = dalloc<int32_t>(h, size_t(std::max<int64_t>(1, perm_off[g.count])));
      if (g.fp32)
        g.A = dalloc<float>(h, size_t(std::max<int64_t>(1, gen_off[g.count])));
      else
        g.A = dalloc<double>(h, size_t(std::max<int64_t>(1, gen_off[g.count])));
      h->sig.row_major = 1;     // Sigma_l is not symmetric: the apply reads its rows
    }
    // 16-bit leaves: the apply reads a 16-bit copy of the FP32 inverses
    h->leaf_elems = P.leaf_batch.total_elems;
    void* half_tiles = nullptr;
    const int half = h->opt.leaf_prec == RSD_PREC_FP16 ? 1 : h->opt.leaf_prec == RSD_PREC_BF16 ? 2 : 0;
    if (half) half_tiles = dalloc<uint16_t>(h, size_t(std::max<int64_t>(1, h->leaf_elems)));
    const int NL = int(P.level_depth.size());
    h->lev.assign(NL, DevBatch());
    h->gam_level.assign(NL, 0);
    for (int q = 0; q < NL; ++q) {
      int32_t maxn = 0;
      for (int32_t v : P.level_batch[q].n) maxn = std::max(maxn, v);
      h->gam_level[q] = h->opt.iface_mode == RSD_IFACE_GAMMA ||
                        (h->opt.iface_mode == RSD_IFACE_HYBRID && maxn > h->opt.dense_max);
      h->any_gamma = h->any_gamma || h->gam_level[q];
    }
    for (int q = 0; q < NL; ++q) {
      const bool root = P.level_depth[q] == 0;
      const int prec = root ? h->opt.root_prec : h->opt.iface_prec;
      upload_batch(h, up, &h->lev[q], P.level_batch[q], prec == RSD_PREC_FP32, !h->gam_level[q]);
    }
    // work items of the chunked inner GMRES: levels with a system above one chunk
    h->gm_lev.assign(NL, rsd_ctx::GmLevel());
    struct GmLists { std::vector<int32_t> sys, first; std::vector<int64_t> b, e; };
    std::vector<GmLists> gml(NL);
    for (int q = 0; q < NL; ++q) {
      if (!h->gam_level[q]) continue;
      const SymBatch& sb = P.level_batch[q];
      int32_t maxn = 0;
      for (int32_t v : sb.n) maxn = std::max(maxn, v);
      if (maxn <= kGmChunk) continue;          // one workgroup per system
      GmLists& L = gml[q];
      for (int32_t m = 0; m < sb.count; ++m) {
        L.first.push_back(int32_t(L.sys.size()));
        for (int64_t c = 0; c < sb.n[m]; c += kGmChunk) {
          L.sys.push_back(m);
          L.b.push_back(sb.vec_off[m] + c);
          L.e.push_back(sb.vec_off[m] + std::min<int64_t>(sb.n[m], c + kGmChunk));
        }
      }
      L.first.push_back(int32_t(L.sys.size()));
      rsd_ctx::GmLevel& G = h->gm_lev[q];
      G.chunked = true;
      G.nitems = int32_t(L.sys.size());
      up.add(&G.item_sys, L.sys);
      up.add(&G.item_b, L.b);
      up.add(&G.item_e, L.e);
      up.add(&G.sys_first, L.first);
      h->gm_max_items = std::max(h->gm_max_items, G.nitems);
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
    {                                   // counters of the persistent symmetric products
      int32_t* q = dalloc<int32_t>(h, 2 * (h->lev.size() + 1));
      hip_check(h, hipMemsetAsync(q, 0, sizeof(int32_t) * 2 * (h->lev.size() + 1), s),
                "hipMemsetAsync queues");
      h->leaf.queue = q;
      for (size_t i = 0; i < h->lev.size(); ++i) h->lev[i].queue = q + 2 * (i + 1);
    }
    h->leaf.persist = h->opt.sym_form == 1 ? 1 : 0;
    for (DevBatch& d : h->lev) d.persist = h->leaf.persist;
    h->leaf_apply = h->leaf;            // (device pointers are set by the commit above)
    if (half) {
      h->leaf_apply.half = half;
      h->leaf_apply.tiles = half_tiles;
    }
    hip_check(h, launch_permute_csr(n, P.n_leaf, h->perm, h->iperm, d_rp, d_ci, h->prow,
                                    h->skel_lvl_begin, h->skel_own_end, h->pcol, h->pmap,
                                    h->segA, h->segB, h->segC, s), "permute csr");
    const int64_t nflags = int64_t(P.leaf_node.size()) + int64_t(P.iface_node.size());
    h->flags = dalloc<int32_t>(h, size_t(nflags));
    h->t = dalloc<double>(h, size_t(n));
    h->rin = dalloc<double>(h, size_t(n));
    h->zin = dalloc<double>(h, size_t(n));
    h->nvec = 0;
    ensure_gamma(h, 1);
    h->nvec = 1;
    size_t part_bytes = std::max<size_t>(8, symv_part_bytes(h->leaf));
    for (const DevBatch& d : h->lev) part_bytes = std::max(part_bytes, symv_part_bytes(d));
    // (levels solved matrix-free have num_items = 0: no symmetric product)
    h->sympart = dalloc<double>(h, (part_bytes + 7) / 8);
    h->sympart_bytes = part_bytes;
    h->held.push_back(up.stage);               // released after the set-up's final sync
    up.stage = Pinned();
    h->setup_wall[1] = ms_since(w1);
    return RSD_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

// The second part of the analysis (build_plan_couplings: per-leaf coupling blocks, adjacency,
// Sigma layout and apply schedule) and its upload, for the kernels queued on s after it.  A
// set-up runs it after queueing the sub-domain inversions, so that the host work and the
// copy overlap them.
void upload_couplings(rsd_ctx* h, hipStream_t s) {
  if (h->couplings_on_device) return;          // a refresh of the values: same structure
  const Plan& P = h->P;
  if (!P.coupled) {
    const auto t0 = std::chrono::steady_clock::now();
    std::string msg;
    const PlanError pe = build_plan_couplings(h->ana_rp, h->ana_ci, &h->P, &msg);
    h->host_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    pfree(h, h->csr_stage);
    h->ana_rp = nullptr;
    h->ana_ci = nullptr;
    if (pe != PlanError::kOk) {
      (void)hipStreamSynchronize(s);           // queued work still reads the handle's blocks
      (void)hipStreamSynchronize(h->aux);
      h->err = msg;
      throw Fail{RSD_ERR_INVALID_ARGUMENT};
    }
  }
  const int NL = int(P.level_depth.size());
  Uploader up;
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
  h->lev_items.assign(NL, SigmaLevelItems());
  h->lev_own_items.assign(NL, SigmaLevelItems());
  // Sigma products per level, split into row chunks: against the deeper levels' columns
  // (the apply), and against the level's own columns (the S-MatVec of Alg. 1 for the
  // levels solved with gamma GMRES steps).  Symmetric Sigma blocks whose rows are short
  // (row-weighted mean length <= kSigRowsMaxCols) go one row per lane in chunks of
  // kSigRowsWave; longer rows (and general Sigma) go lanes over columns in chunks of
  // kSigRows, which keeps more waves in flight per row.
  struct ItemLists { std::vector<int32_t> l, c0, c1, a0, a1; };
  std::vector<ItemLists> deep(NL), own(NL);
  auto items = [&](const std::vector<LevelSigmaItem>& src, bool own_cols, ItemLists* o,
                   SigmaLevelItems* li) {
    double rows = 0.0, weighted = 0.0;
    for (const auto& it : src) {
      const double len = own_cols ? double(it.r1 - it.r0) : double(it.r0);
      rows += double(it.r1 - it.r0);
      weighted += len * double(it.r1 - it.r0);
    }
    const bool by_rows = h->opt.symmetric && weighted <= double(kSigRowsMaxCols) * rows;
    const int32_t chunk = by_rows ? kSigRowsWave : kSigRows;
    for (const auto& it : src)
      for (int32_t a0 = it.r0; a0 < it.r1; a0 += chunk) {
        o->l.push_back(it.leaf);
        o->c0.push_back(own_cols ? it.r0 : 0);
        o->c1.push_back(own_cols ? it.r1 : it.r0);
        o->a0.push_back(a0);
        o->a1.push_back(std::min(it.r1, a0 + chunk));
      }
    li->count = int32_t(o->l.size());
    li->by_rows = by_rows ? 1 : 0;
    up.add(&li->leaf, o->l);
    up.add(&li->c0, o->c0);
    up.add(&li->c1, o->c1);
    up.add(&li->a0, o->a0);
    up.add(&li->a1, o->a1);
  };
  for (int q = 0; q < NL; ++q) {
    items(P.level_sigma[q], false, &deep[q], &h->lev_items[q]);
    if (h->gam_level[q]) items(P.level_sigma_own[q], true, &own[q], &h->lev_own_items[q]);
  }
  // the copy runs on the upload stream while s still inverts the sub-domains (queued on s
  // it would wait for them); s waits for it before the first kernel that reads the arrays
  up.commit(h, h->upl);
  hip_check(h, hipEventRecord(h->ev_upl, h->upl), "hipEventRecord");
  hip_check(h, hipStreamWaitEvent(s, h->ev_upl, 0), "hipStreamWaitEvent");
  h->held.push_back(up.stage);                 // released after the set-up's final sync
  up.stage = Pinned();
  a.B_off = h->B_off;
  a.B = h->B;
  a.sig_off = h->sig_off_d;
  h->e = dalloc<double>(h, std::max<size_t>(1, P.B.size()));
  h->couplings_on_device = true;
}

// Dense set-up from the values of K (caller order, device pointer): Section 3.1's
// exact sub-domain inverses, the Sigma_l blocks, and per interface level the
// operator of Alg. 1 assembled and inverted.
rsd_status engine_numeric(rsd_ctx* h, const double* values, hipStream_t s) {
  try {
    h->cur = s;
    enter(h, s);   // applies queued on another stream may still read the old blocks
    const auto w2 = std::chrono::steady_clock::now();
    const Plan& P = h->P;
    {
      Timer tm(h, RSD_T_SETUP_EXTRACT, s);
      hip_check(h, launch_gather(values, h->pmap, P.nnz, h->pval, s), "gather values");
      hip_check(h, launch_ell_fill(P.n, h->prow, h->pcol, h->pval, h->ell_off, h->ell_col,
                                   h->ell_val, s), "ELL fill");
      const int64_t nflags = int64_t(P.leaf_node.size()) + int64_t(P.iface_node.size());
      hip_check(h, hipMemsetAsync(h->flags, 0, size_t(nflags) * 4, s), "hipMemsetAsync flags");
      if (h->opt.symmetric) {
        hip_check(h, launch_sym_fill(h->leaf, s), "leaf fill");
        hip_check(h, launch_sym_extract(h->leaf, h->prow, h->segA, h->pcol, h->pval, P.max_leaf,
                                        s), "leaf extract");
      }
    }
    // scratch of the sweeps: sized for the largest batch
    size_t pb = 0, cb = 0, need_p = 0, need_c = 0;
    if (h->opt.symmetric) {
      sym_invert_scratch_bytes(h->leaf, group_for(h, h->leaf), &pb, &cb);
      need_p = pb;
      need_c = cb;
    }
    // The dense levels other than the shallowest (the last in processing order, the
    // largest systems) are inverted on the upload stream, beside it: each level's S~
    // depends only on K and the Sigma blocks, and the shallowest level's sweep leaves
    // most compute units idle around its pivots.  They take the serial schedule (the
    // auxiliary stream carries the shallowest level's look-ahead) and scratch of their own.
    int last_dense = -1;
    for (size_t q = 0; q < h->lev.size(); ++q)
      if (!h->gam_level[q]) last_dense = int(q);
    size_t side_p = 0, side_c = 0;
    for (size_t q = 0; q < h->lev.size(); ++q) {
      if (h->gam_level[q]) continue;   // no dense factor at the levels solved matrix-free
      const DevBatch& L = h->lev[q];
      sym_invert_scratch_bytes(L, group_for(h, L), &pb, &cb);
      if (int(q) == last_dense || !h->opt.symmetric) {
        need_p = std::max(need_p, pb);
        need_c = std::max(need_c, cb);
      } else {
        side_p = std::max(side_p, pb);
        side_c = std::max(side_c, cb);
      }
    }
    const bool side = side_p > 0 || side_c > 0;
    char* pbuf = dalloc<char>(h, need_p);
    void* cbuf[2] = {dalloc<char>(h, need_c), dalloc<char>(h, need_c)};
    void* bbuf[2] = {dalloc<char>(h, need_c), dalloc<char>(h, need_c)};
    char* side_pbuf = side ? dalloc<char>(h, side_p) : nullptr;
    void* side_cbuf[2] = {side ? dalloc<char>(h, side_c) : nullptr, nullptr};
    void* side_bbuf[2] = {side ? dalloc<char>(h, side_c) : nullptr, nullptr};
    // one batch's inversion with the autotuner's candidate (timed while tuning)
    struct Pending {
      std::string key;
      int ncand, cand;
      hipEvent_t a, b;
    };
    std::vector<Pending> tuned;
    // (on_side: on the upload stream, serial candidates only: 1, 3, ...)
    auto invert = [&](DevBatch bb, const SymBatch& sb, int32_t* fl, int upd, int slot,
                      bool on_side = false) {
      const hipStream_t st = on_side ? h->upl : s;
      const int G = group_for(h, bb);
      const int ncand = on_side ? std::max(1, inv_candidates(bb, G) / 2) : inv_candidates(bb, G);
      const std::string key = inv_key(sb, bb, G) + (on_side ? ":serial" : "");
      bool tuning = false;
      const int pick = inv_pick(h, key, ncand, &tuning);
      const int cand = on_side ? 2 * pick + 1 : pick;
      bb.upd_shape = cand / 2;
      if (slot < 8) h->setup_variant[slot] = cand + 1;
      hipEvent_t a = nullptr, b = nullptr;
      if (tuning) {
        hip_check(h, hipEventCreate(&a), "hipEventCreate");
        hip_check(h, hipEventCreate(&b), "hipEventCreate");
        hip_check(h, hipEventRecord(a, st), "hipEventRecord");
      }
      if (on_side)
        invert_batch(h, bb, side_pbuf, side_cbuf, side_bbuf, fl, upd, false, st);
      else
        invert_batch(h, bb, pbuf, cbuf, bbuf, fl, upd, (cand & 1) == 0, st);
      if (tuning) {
        hip_check(h, hipEventRecord(b, st), "hipEventRecord");
        tuned.push_back({key, ncand, pick, a, b});
      }
    };
    for (int32_t& v : h->setup_variant) v = 0;
    {
      Timer tm(h, RSD_T_LEAF_INVERSE, s);
      if (h->opt.symmetric)
        invert(h->leaf, P.leaf_batch, h->flags, RSD_T_LEAF_UPDATE, 0);
      else
        hip_check(h, launch_gen_invert(h->gen, h->prow, h->segA, h->pcol, h->pval, h->flags, s),
                  "general sub-domain inverses");
    }
    // the couplings (host analysis and upload, while the device inverts the sub-domains)
    upload_couplings(h, s);
    {
      Timer tm(h, RSD_T_SETUP_EXTRACT, s);
      hip_check(h, launch_gather(values, h->kcol_pos, int64_t(P.kcol_val.size()), h->kcol_v, s),
                "gather couplings");
      hip_check(h, launch_gather(values, h->krow_pos, int64_t(P.krow_val.size()), h->krow_v, s),
                "gather couplings");
    }
    double* W = dalloc<double>(h, size_t(std::max<int64_t>(1, P.w_total)));
    {
      Timer tm(h, RSD_T_SIGMA, s);
      if (h->opt.symmetric)
        hip_check(h, launch_sigma_w(h->leaf, h->sig, W, s), "sigma W");
      else
        hip_check(h, launch_sigma_w_gen(h->gen, h->sig, W, s), "sigma W");
      hip_check(h, launch_sigma_s(h->sig, W, h->sigma, h->sigma_fp32, s), "sigma S");
    }
    if (h->leaf_apply.half) {
      Timer tm(h, RSD_T_LEAF_INVERSE, s);
      hip_check(h, launch_narrow(static_cast<const float*>(h->leaf.tiles), h->leaf_apply.tiles,
                                 h->leaf_elems, h->leaf_apply.half, s), "16-bit leaf copy");
    }
    int32_t* iflags = h->flags + P.leaf_node.size();
    // Every dense level's S~ depends only on K and the Sigma blocks: the assemblies run on
    // the upload stream, deepest level first, while s inverts the deeper levels (the
    // inversion of a few interfaces leaves most compute units idle between its pivots).
    hip_check(h, hipEventRecord(h->ev_sig, s), "hipEventRecord");
    hip_check(h, hipStreamWaitEvent(h->upl, h->ev_sig, 0), "hipStreamWaitEvent");
    for (size_t q = 0; q < h->lev.size(); ++q) {
      if (h->gam_level[q]) continue;   // S~ is applied matrix-free (Alg. 1), never formed
      hipStream_t u = h->upl;
      {
        Timer tm(h, RSD_T_IFACE_ASSEMBLY, u);
        int32_t maxn = 0;
        for (int32_t v : P.level_batch[q].n) maxn = std::max(maxn, v);
        hip_check(h, launch_sym_fill(h->lev[q], u), "iface fill");
        hip_check(h, launch_sym_extract(h->lev[q], h->segB, h->segC, h->pcol, h->pval, maxn, u),
                  "iface extract");
        hip_check(h, launch_schur_assemble(h->lev[q], h->adj_ptr, h->adj_leaf, h->adj_pos,
                                           h->B_off, h->sig_off_d, h->sigma, h->sigma_fp32,
                                           P.n_leaf, u),
                  "schur assembly");
      }
      hip_check(h, hipEventRecord(h->ev_lev[q], u), "hipEventRecord");
    }
    for (size_t q = 0; q < h->lev.size(); ++q) {
      if (h->gam_level[q]) continue;
      const bool on_side = side && int(q) != last_dense;
      if (!on_side)      // (the upload stream runs its levels after their assemblies)
        hip_check(h, hipStreamWaitEvent(s, h->ev_lev[q], 0), "hipStreamWaitEvent");
      {
        Timer tm(h, RSD_T_IFACE_INVERSE, on_side ? h->upl : s);
        invert(h->lev[q], P.level_batch[q], iflags + P.level_iface_begin[q],
               P.level_depth[q] == 0 ? RSD_T_ROOT_UPDATE : RSD_T_IFACE_UPDATE, int(1 + q),
               on_side);
      }
    }
    if (side) {        // s waits for the levels on the upload stream
      hip_check(h, hipEventRecord(h->ev_upl, h->upl), "hipEventRecord");
      hip_check(h, hipStreamWaitEvent(s, h->ev_upl, 0), "hipStreamWaitEvent");
    }
    precapture_apply(h);
    h->setup_wall[2] = ms_since(w2);
    const auto w3 = std::chrono::steady_clock::now();
    std::vector<int32_t> fl(P.leaf_node.size() + P.iface_node.size());
    if (!fl.empty())
      hip_check(h, hipMemcpyAsync(fl.data(), h->flags, fl.size() * 4, hipMemcpyDeviceToHost, s),
                "flags D2H");
    hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
    leave(h, s);
    for (Pending& t : tuned) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) inv_record(t.key, t.ncand, t.cand, ms);
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
    dfree(h, W);
    dfree(h, pbuf);
    for (int i = 0; i < 2; ++i) {
      dfree(h, cbuf[i]);
      dfree(h, bbuf[i]);
    }
    if (side) {
      dfree(h, side_pbuf);
      dfree(h, side_cbuf[0]);
      dfree(h, side_bbuf[0]);
    }
    for (Pinned& b : h->held) pfree(h, b);    // the uploads have completed
    h->held.clear();
    h->setup_wall[3] = ms_since(w3);
    for (size_t i = 0; i < fl.size(); ++i)
      if (fl[i]) {
        char buf[256];
        if (i < P.leaf_node.size() && !h->opt.symmetric)
          std::snprintf(buf, sizeof(buf),
                        "sub-domain matrix of leaf node %d is singular "
                        "(zero or non-finite pivot in column %d)",
                        P.leaf_node[i], fl[i] - 1);
        else if (i < P.leaf_node.size())
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

// u = gamma steps of unpreconditioned GMRES from zero on S~_t u = g for every interface
// t of level q and nv vectors (Section 3.1, inexact interface solve); g is read from and
// u written to z at the level's rows.  Each product w = S~_t v is Alg. 1's S-MatVec with
// the Sigma blocks: the own-node columns of K_tt, minus Sigma_l[I_t, I_t] v over every
// leaf adjacent to t (the e buffer is free again once the level's g is formed).
void gamma_solve(rsd_ctx* h, const ApplyWork& wk, size_t q, int nv, double* z, hipStream_t s) {
  const Plan& P = h->P;
  const int64_t n = P.n, nl = P.n_leaf, nB = std::max<int64_t>(1, int64_t(P.B.size()));
  const int64_t r0 = P.level_dof_begin[q], r1 = P.level_dof_end[q];
  const DevBatch& b = h->lev[q];
  const int g = h->opt.gamma;
  const rsd_ctx::GmLevel& G = h->gm_lev[q];
  GmArgs a;                                   // chunked kernels (large systems)
  a.count = b.count;
  a.nitems = G.nitems;
  a.nv = nv;
  a.gamma = g;
  a.ld = n;
  a.item_sys = G.item_sys;
  a.item_b = G.item_b;
  a.item_e = G.item_e;
  a.sys_first = G.sys_first;
  a.V = wk.gm_V;
  a.beta = wk.gm_beta;
  a.H = wk.gm_H;
  a.steps = wk.gm_steps;
  a.stop = wk.gm_stop;
  a.part = wk.gm_part;
  a.coef = wk.gm_coef;
  if (G.chunked)
    hip_check(h, launch_gmc(a, 0, 0, z, nullptr, s), "gmres start");
  else
    hip_check(h, launch_gm_start(b, g, nv, z, n, wk.gm_V, wk.gm_beta, wk.gm_H, wk.gm_steps,
                                 wk.gm_stop, s), "gmres start");
  for (int j = 0; j < g; ++j) {
    const double* vj = wk.gm_V + int64_t(j) * nv * n;
    double* w = wk.gm_V + int64_t(j + 1) * nv * n;
    hip_check(h, launch_ell_spmv(r0, r1 - r0, h->segB, h->segC, h->prow, h->ell_off, h->ell_col,
                                 h->ell_val, vj, nullptr, 1.0, w, nv, n, wk.xil, r0, r1, s),
              "S-MatVec K_tt");
    hip_check(h, launch_sigma_level(h->lev_own_items[q], h->sigma, h->sigma_fp32, h->sig_off_d,
                                    h->B_off, h->B, vj, wk.e, nv, n, nB, s), "S-MatVec Sigma");
    hip_check(h, launch_level_adj(r0, r1 - r0, nl, h->adj_ptr, h->adj_leaf, h->adj_pos, h->B_off,
                                  wk.e, w, nv, n, nB, -1.0, s), "S-MatVec sum");
    if (G.chunked)
      hip_check(h, launch_gmc(a, 1, j, nullptr, nullptr, s), "gmres step");
    else
      hip_check(h, launch_gm_orth(b, g, nv, j, n, wk.gm_V, wk.gm_beta, wk.gm_H, wk.gm_steps,
                                  wk.gm_stop, s), "gmres step");
  }
  if (G.chunked)
    hip_check(h, launch_gmc(a, 2, 0, nullptr, z, s), "gmres finish");
  else
    hip_check(h, launch_gm_finish(b, g, nv, n, wk.gm_V, wk.gm_beta, wk.gm_H, wk.gm_steps, z, s),
              "gmres finish");
}

// the handle's own work buffers (sized for h->nvec vectors)
ApplyWork own_work(const rsd_ctx* h) {
  ApplyWork w;
  w.e = h->e;
  w.t = h->t;
  w.xil = h->xil;
  w.sympart = h->sympart;
  w.gm_V = h->gm_V;
  w.gm_beta = h->gm_beta;
  w.gm_H = h->gm_H;
  w.gm_part = h->gm_part;
  w.gm_coef = h->gm_coef;
  w.gm_steps = h->gm_steps;
  w.gm_stop = h->gm_stop;
  return w;
}

// z = M^{-1} r on internal-order vectors (Alg. 2 with exact interface solves):
// every sub-domain solve; per interface level from the deepest: right-hand side g
// of eq. (schur) -- the interface part of r minus the couplings to the already
// computed values below it -- and the interface solve; then the back-substitution
// of eq. (backSub) on every sub-domain at once.  nv vectors (r_k = r + k n, likewise
// z) go through every step together: the factors and K are read once per group of
// vectors that a kernel holds, and each vector's result is the one it has alone.
void set_vec_pass(rsd_ctx* h, int nv);

void core_apply(rsd_ctx* h, const ApplyWork& wk, int nv, const double* r, double* z,
                hipStream_t s) {
  const Plan& P = h->P;
  set_vec_pass(h, nv);
  const int64_t n = P.n, nl = P.n_leaf, nB = std::max<int64_t>(1, int64_t(P.B.size()));
  {
    Timer tm(h, RSD_T_LEAF_APPLY, s);
    if (h->opt.symmetric)    // tiles hold -K_ll^{-1}
      hip_check(h, launch_symv(h->leaf_apply, r, wk.sympart, -1.0, nullptr, z, nv, n, s),
                "leaf symv");
    else
      hip_check(h, launch_gen_matvec(h->gen, r, 1.0, z, nv, n, s), "leaf matvec");
  }
  {
    Timer tm(h, RSD_T_COUPLING, s);
    // interface rows: q_B = r_B - K_{B,leaves} y
    hip_check(h, launch_ell_spmv(nl, n - nl, h->prow, h->segA, h->prow, h->ell_off, h->ell_col,
                                 h->ell_val, z, r, -1.0, z, nv, n, wk.xil, 0, nl, s), "condense");
    hip_check(h, launch_fill(wk.e, nB * nv, 0.0, s), "fill e");
  }
  for (size_t q = 0; q < h->lev.size(); ++q) {
    {
      Timer tm(h, RSD_T_COUPLING, s);
      hip_check(h, launch_sigma_level(h->lev_items[q], h->sigma, h->sigma_fp32, h->sig_off_d,
                                      h->B_off, h->B, z, wk.e, nv, n, nB, s), "sigma level");
      // g_t = q_t - K_{t, deeper interfaces} u - sum over adjacent leaves of e_l
      const int64_t r0 = P.level_dof_begin[q], r1 = P.level_dof_end[q];
      if (h->opt.g_coupling == RSD_COUPLING_FULL)   // the direct couplings to deeper levels
        hip_check(h, launch_ell_spmv(r0, r1 - r0, h->segA, h->segB, h->prow, h->ell_off,
                                     h->ell_col, h->ell_val, z, z, -1.0, z, nv, n, wk.xil, nl,
                                     r0, s), "level rhs");   // deeper levels come first: [nl, r0)
      hip_check(h, launch_level_adj(r0, r1 - r0, nl, h->adj_ptr, h->adj_leaf, h->adj_pos,
                                    h->B_off, wk.e, z, nv, n, nB, 1.0, s), "level adjacency");
    }
    {
      Timer tm(h, RSD_T_IFACE_APPLY, s);
      if (h->gam_level[q])      // u = gamma GMRES steps on S~ u = g (paper mode)
        gamma_solve(h, wk, q, nv, z, s);
      else                      // u = S~^{-1} g (tiles hold -S~^{-1})
        hip_check(h, launch_symv(h->lev[q], z, wk.sympart, -1.0, nullptr, z, nv, n, s),
                  "interface symv");
    }
  }
  // back-substitution, u_l = K_ll^{-1} (r_l - K_{l,B} u_B).  Symmetric K: the leaf rows of z
  // still hold K_ll^{-1} r_l from the first leaf pass, so u_l = z_l + K_ll^{-1} w with
  // w = -K_{l,B} u_B, which is zero outside the leaf's shell (its last rows): the product
  // skips the tile rows before the shell, whose products with w are zero.
  {
    Timer tm(h, RSD_T_COUPLING, s);
    hip_check(h, launch_ell_spmv(0, nl, h->segA, h->prow + 1, h->prow, h->ell_off, h->ell_col,
                                 h->ell_val, z, h->opt.symmetric ? nullptr : r, -1.0, wk.t, nv,
                                 n, wk.xil, nl, n, s),
              "back-substitution rhs");
  }
  {
    Timer tm(h, RSD_T_LEAF_APPLY, s);
    if (h->opt.symmetric)    // tiles hold -K_ll^{-1}
      hip_check(h, launch_symv(h->leaf_apply, wk.t, wk.sympart, -1.0, z, z, nv, n, s,
                               h->leaf_row0), "leaf symv (correction)");
    else
      hip_check(h, launch_gen_matvec(h->gen, wk.t, 1.0, z, nv, n, s), "leaf matvec");
  }
}

// y_k = base_k + alpha K x_k for nv internal-order vectors (stride n)
void core_spmv(rsd_ctx* h, int nv, const double* x, const double* base, double alpha, double* y,
               hipStream_t s) {
  Timer tm(h, RSD_T_SPMV, s);
  hip_check(h, launch_ell_spmv(0, h->P.n, h->prow, h->prow + 1, h->prow, h->ell_off, h->ell_col,
                               h->ell_val, x, base, alpha, y, nv, h->P.n, h->xil, 0, h->P.n, s),
            "spmv");
}

void permute(rsd_ctx* h, int nv, const double* x, int64_t ldx, double* y, int64_t ldy,
             int inverse, hipStream_t s) {
  Timer tm(h, RSD_T_PERMUTE, s);
  hip_check(h, launch_permute(x, ldx, y, ldy, h->perm, h->P.n, nv, inverse, s), "permute");
}

// Right-hand sides handled together by one apply, SpMV or Krylov iteration.
constexpr int kRhsGroup = 8;

// ---- autotuner: vectors per pass and launch form of the symmetric products --------------
// For a column count nv in 2..8, every dense batch (the sub-domains, each exactly solved
// interface level) times one product of nv vectors with passes of 4, 2 and 1 vectors, each
// as one workgroup per item and as a persistent work-queue launch, on the handle's own
// blocks (one warm-up, two timed runs each) and keeps the fastest; a tie keeps the earlier
// candidate (more vectors per pass, one workgroup per item).  Every choice gives the same
// bits, so only speed depends on it.  Choices (vectors per pass + 16 for the persistent
// form) are remembered per process for batches of the same shape (count, sizes, storage
// type, nv).
std::mutex g_tune_mu;
std::unordered_map<std::string, int32_t> g_tune;

std::string tune_key(const SymBatch& sb, const DevBatch& d, int nv) {
  uint64_t hsh = 1469598103934665603ull;                 // FNV-1a over the sizes
  for (int32_t v : sb.n) {
    hsh ^= uint64_t(uint32_t(v));
    hsh *= 1099511628211ull;
  }
  return std::to_string(d.fp32) + ":" + std::to_string(d.half) + ":" + std::to_string(nv) + ":" +
         std::to_string(sb.count) + ":" + std::to_string(hsh);
}

int32_t tune_batch(rsd_ctx* h, DevBatch& b, const SymBatch& sb, int nv, hipStream_t s) {
  if (b.num_items == 0) return 0;
  const std::string key = tune_key(sb, b, nv);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  const int64_t n = h->P.n;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hip_check(h, hipEventCreate(&e0), "hipEventCreate");
  hip_check(h, hipEventCreate(&e1), "hipEventCreate");
  int32_t best = 4;
  float best_ms = 0.0f;
  for (int32_t cand : {4, 2, 1, 16 + 4, 16 + 2, 16 + 1}) {
    b.vec_pass = cand & 15;
    b.persist = cand >> 4;
    hip_check(h, launch_symv(b, h->rin, h->sympart, -1.0, nullptr, h->zin, nv, n, s), "tune");
    hip_check(h, hipEventRecord(e0, s), "hipEventRecord");
    for (int r = 0; r < 2; ++r)
      hip_check(h, launch_symv(b, h->rin, h->sympart, -1.0, nullptr, h->zin, nv, n, s), "tune");
    hip_check(h, hipEventRecord(e1, s), "hipEventRecord");
    hip_check(h, hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.0f;
    hip_check(h, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (cand == 4 || ms < best_ms) {
      best = cand;
      best_ms = ms;
    }
  }
  b.persist = 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = best;
  return best;
}

void autotune_apply(rsd_ctx* h, int nv, hipStream_t s) {
  if (h->vec_pass.size() < 9) h->vec_pass.assign(9, std::array<int32_t, 9>{});
  std::array<int32_t, 9>& vp = h->vec_pass[size_t(nv)];
  vp.fill(0);
  if (h->opt.symmetric) vp[0] = tune_batch(h, h->leaf_apply, h->P.leaf_batch, nv, s);
  for (size_t q = 0; q < h->lev.size() && q < 8; ++q)
    if (!h->gam_level[q]) vp[1 + q] = tune_batch(h, h->lev[q], h->P.level_batch[q], nv, s);
  h->tuned[size_t(nv)] = true;
  h->last_tuned = nv;
}

// the tuned vectors per pass for nv columns (0: the default) on every dense batch
void set_vec_pass(rsd_ctx* h, int nv) {
  const bool have = nv >= 0 && size_t(nv) < h->vec_pass.size() && h->tuned[size_t(nv)];
  const int32_t forced = h->opt.sym_form == 1 ? 1 : 0;
  const int32_t c0 = have ? h->vec_pass[size_t(nv)][0] : 0;
  h->leaf_apply.vec_pass = c0 & 15;
  h->leaf_apply.persist = forced | (c0 >> 4);
  for (size_t q = 0; q < h->lev.size(); ++q) {
    const int32_t c = have && q < 8 ? h->vec_pass[size_t(nv)][1 + q] : 0;
    h->lev[q].vec_pass = c & 15;
    h->lev[q].persist = forced | (c >> 4);
  }
}

void drop_graphs(rsd_ctx* h) {
  for (hipGraphExec_t& g : h->apply_graph)
    if (g) (void)hipGraphExecDestroy(g);
  h->apply_graph.clear();
}

// The graph of the whole application for nv vectors on the fixed vectors rin -> zin,
// captured on first use (on the handle's own stream: capturing executes nothing).
hipGraphExec_t apply_graph(rsd_ctx* h, int nv) {
  if (int(h->apply_graph.size()) <= nv) h->apply_graph.resize(size_t(nv) + 1, nullptr);
  hipGraphExec_t& ex = h->apply_graph[size_t(nv)];
  if (ex) return ex;
  if (!h->cap)
    hip_check(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking), "hipStreamCreate");
  hipGraph_t g = nullptr;
  hip_check(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    core_apply(h, own_work(h), nv, h->rin, h->zin, h->cap);
  } catch (...) {
    (void)hipStreamEndCapture(h->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_check(h, hipStreamEndCapture(h->cap, &g), "end capture");
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(h, e, "hipGraphInstantiate");
  return ex;
}

// z = M^{-1} r for nv vectors at stride n.  With graphs on (and timing off) the whole
// application is replayed from the graph of this nv on the fixed vectors rin -> zin
// (apply_graph; the one-vector graph is captured during the set-up); r and z are copied
// in and out unless they are those vectors.  The replays run on the caller's stream.
void apply_vectors(rsd_ctx* h, int nv, const double* r, double* z, hipStream_t s) {
  if (h->opt.autotune && nv >= 2 && nv <= kRhsGroup && !h->tuned[size_t(nv)])
    autotune_apply(h, nv, s);            // before this nv's graph is captured
  if (!h->opt.graphs || apply_timed(h)) {
    core_apply(h, own_work(h), nv, r, z, s);
    return;
  }
  const size_t bytes = sizeof(double) * size_t(nv) * size_t(h->P.n);
  if (r != h->rin)
    hip_check(h, hipMemcpyAsync(h->rin, r, bytes, hipMemcpyDeviceToDevice, s), "apply in");
  hip_check(h, hipGraphLaunch(apply_graph(h, nv), s), "hipGraphLaunch");
  if (z != h->zin)
    hip_check(h, hipMemcpyAsync(z, h->zin, bytes, hipMemcpyDeviceToDevice, s), "apply out");
}

// Apply work vectors (e, t, rin, zin, xil, the inner GMRES scratch) for nv vectors.
void ensure_vectors(rsd_ctx* h, int nv) {
  if (h->nvec >= nv) return;
  wait_idle(h);                         // the handle's queued work may use the old buffers
  drop_graphs(h);                       // they refer to the buffers replaced here
  ensure_gamma(h, nv);
  for (double* p : {h->e, h->t, h->rin, h->zin, h->xil}) dfree(h, p);
  const size_t n = size_t(h->P.n), nB = std::max<size_t>(1, h->P.B.size());
  h->xil = dalloc<double>(h, n * size_t(kEllVec));      // interleaved copies for the SpMVs
  h->e = dalloc<double>(h, nB * size_t(nv));
  h->t = dalloc<double>(h, n * size_t(nv));
  h->rin = dalloc<double>(h, n * size_t(nv));
  h->zin = dalloc<double>(h, n * size_t(nv));
  h->nvec = nv;
}

// At the end of a set-up's enqueueing, while the device still runs it: the one-vector
// application's work vectors and graph, which the first apply of a solve would otherwise
// capture with the device idle (a handle whose applies run eagerly, or that has them
// already, is left as it is).
void precapture_apply(rsd_ctx* h) {
  if (!h->opt.graphs || apply_timed(h)) return;
  if (h->apply_graph.size() > 1 && h->apply_graph[1]) return;
  ensure_vectors(h, 1);
  (void)apply_graph(h, 1);
}

// Krylov work space for restart length m and nr right-hand sides in lockstep.
void ensure_krylov(rsd_ctx* h, int m, int nr) {
  if (h->kry_m >= m && h->kry_nr >= nr && h->V) return;
  if (h->V) wait_idle(h);               // the handle's queued work may use the old buffers
  for (double* p : {h->V, h->Z, h->w, h->hdev, h->tmp, h->part, h->scal, h->bint, h->xint})
    dfree(h, p);
  pfree(h, h->hhost_block);
  m = std::max(m, h->kry_m);
  nr = std::max(nr, h->kry_nr);
  const size_t n = size_t(h->P.n), r = size_t(nr);
  h->V = dalloc<double>(h, n * size_t(m + 1) * r);
  h->Z = dalloc<double>(h, n * size_t(m) * r);
  h->w = dalloc<double>(h, n * r);
  h->hdev = dalloc<double>(h, size_t(m + 2) * r);
  h->tmp = dalloc<double>(h, size_t(m + 2) * r);
  h->part = dalloc<double>(h, size_t(mdot_blocks(h->P.n)) * size_t(m + 2) * r);
  h->scal = dalloc<double>(h, 16 * r);
  h->bint = dalloc<double>(h, n * r);
  h->xint = dalloc<double>(h, n * r);
  h->hhost_block = palloc(h, sizeof(double) * (3 * size_t(m + 2) + 16) * r);
  h->hhost = static_cast<double*>(h->hhost_block.p);
  for (hipEvent_t& e : h->ev_h)
    if (!e) hip_check(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  h->kry_m = m;
  h->kry_nr = nr;
}

// ||v_k|| for nv vectors (stride ld) into out_dev[k * so]; returned on the host.
std::vector<double> dev_norms(rsd_ctx* h, int nv, const double* v, int64_t ld, double* out_dev,
                              int64_t so, hipStream_t s) {
  {
    Timer tm(h, RSD_T_KRYLOV, s);
    hip_check(h, launch_mdot(nv, v, h->P.n, ld, 1, v, ld, h->P.n, h->part, out_dev, so, 1, s),
              "norm");
  }
  for (int k = 0; k < nv; ++k)
    hip_check(h, hipMemcpyAsync(h->hhost + k, out_dev + k * so, 8, hipMemcpyDeviceToHost, s),
              "D2H");
  hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
  return std::vector<double>(h->hhost, h->hhost + nv);
}

double dev_norm(rsd_ctx* h, const double* v, double* out_dev, hipStream_t s) {
  return dev_norms(h, 1, v, h->P.n, out_dev, 1, s)[0];
}

// Right-preconditioned flexible GMRES(m) for nr right-hand sides in lockstep, in
// internal order; x holds the initial guesses.  Right-hand side i keeps its own
// Arnoldi basis, Hessenberg matrix and Givens rotations; the preconditioner, the SpMV
// and the Gram-Schmidt kernels take all of them in one launch, and the host waits once
// per iteration for the whole group.  Column j of right-hand side i is V + (j nr + i) n
// (likewise Z).  Kernels run over the range [lo, hi) of right-hand sides still
// iterating; one that has stopped but lies inside the range is carried along, and
// those extra results are never read.  Each right-hand side's arithmetic is that of
// its solve alone.
void fgmres_group(rsd_ctx* h, int nr, const double* b, double* x, const rsd_solve_options& o,
                  rsd_solve_info* info, hipStream_t s) {
  const int64_t n = h->P.n;
  const int m = o.restart;
  const int64_t ldV = int64_t(nr) * n;   // column stride of one right-hand side's basis
  const int64_t hs = m + 2;              // per right-hand side stride of hdev / tmp / hhost
  double* beta_d = h->scal;              // ||r_i||
  double* bnorm_d = h->scal + nr;        // ||b_i||
  double* W = h->w;
  struct Rhs {
    double bnorm = 0, tol = 0, beta = 0;
    double g_prev = 0;                   // residual estimate before the last step
    int its = 0, k = 0;
    bool done = false, stop = false, bad = false;
    std::vector<double> H, cs, sn, g, y;
  };
  std::vector<Rhs> R(static_cast<size_t>(nr));
  auto finish = [&](int i, rsd_status st, double relres) {
    R[i].done = true;
    info[i].iterations = R[i].its;
    info[i].relres = relres;
    info[i].status = st;
  };
  auto range = [&](bool inner, int* lo, int* hi) {
    *lo = nr;
    *hi = 0;
    for (int i = 0; i < nr; ++i)
      if (!R[i].done && !(inner && R[i].stop)) {
        *lo = std::min(*lo, i);
        *hi = i + 1;
      }
    return *lo < *hi;
  };
  {
    const std::vector<double> bn = dev_norms(h, nr, b, n, bnorm_d, 1, s);
    for (int i = 0; i < nr; ++i) {
      Rhs& q = R[i];
      q.bnorm = bn[i];
      q.H.assign(size_t(m + 1) * m, 0.0);
      q.cs.assign(m, 0.0);
      q.sn.assign(m, 0.0);
      q.g.assign(m + 1, 0.0);
      q.y.assign(m, 0.0);
      if (!(q.bnorm == q.bnorm) || std::isinf(q.bnorm)) {
        finish(i, RSD_ERR_BREAKDOWN, NAN);
      } else if (q.bnorm == 0.0) {
        hip_check(h, launch_fill(x + i * n, n, 0.0, s), "zero x");
        finish(i, RSD_OK, 0.0);
      } else {
        q.tol = o.rtol * q.bnorm;
      }
    }
  }
  // true residuals r_i = b_i - K x_i (in W) and their norms
  auto residuals = [&]() {
    int lo, hi;
    if (!range(false, &lo, &hi)) return;
    core_spmv(h, hi - lo, x + lo * n, b + lo * n, -1.0, W + lo * n, s);
    const std::vector<double> bt = dev_norms(h, hi - lo, W + lo * n, n, beta_d + lo, 1, s);
    for (int i = lo; i < hi; ++i) R[i].beta = bt[i - lo];
  };
  residuals();
  for (;;) {
    for (int i = 0; i < nr; ++i) {
      Rhs& q = R[i];
      if (q.done) continue;
      if (q.beta <= q.tol) finish(i, RSD_OK, q.beta / q.bnorm);
      else if (!(q.beta == q.beta)) finish(i, RSD_ERR_BREAKDOWN, NAN);
      else if (q.its >= o.maxit) finish(i, RSD_ERR_NOT_CONVERGED, q.beta / q.bnorm);
    }
    int lo, hi;
    if (!range(false, &lo, &hi)) return;
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      hip_check(h, launch_scale_div(hi - lo, W + lo * n, n, beta_d + lo, 1, h->V + lo * n, n, n, s),
                "v0");
    }
    for (int i = lo; i < hi; ++i) {
      Rhs& q = R[i];
      if (q.done) continue;
      std::fill(q.H.begin(), q.H.end(), 0.0);
      std::fill(q.g.begin(), q.g.end(), 0.0);
      q.g[0] = q.beta;
      q.k = 0;
      q.stop = q.bad = false;
    }
    // Arnoldi step j on the device: apply, SpMV, classical Gram-Schmidt twice, the new
    // basis vector, and the Hessenberg columns copied to pinned half j % 2 of hhost.  Step
    // j + 1 depends only on v_{j+1}, which the device forms, so it is queued before the
    // host waits for step j's columns (the host's Givens rotations then overlap it),
    // unless every right-hand side is expected to reach its tolerance at step j (its
    // residual estimate falling at the rate of the last step).  A step queued ahead that
    // is not needed is carried along like a stopped right-hand side: nothing reads it.
    struct Queued { int lo = 0, hi = 0; bool on = false; };
    Queued qd[2];
    auto half = [&](int j) { return h->hhost + size_t(nr) * size_t(hs) * size_t(1 + (j & 1)); };
    auto step = [&](int j, int slo, int shi) {
      const int nv = shi - slo;
      const double* Vb = h->V + slo * n;                // column 0 of right-hand side slo
      double* Wb = W + slo * n;
      apply_vectors(h, nv, h->V + (int64_t(j) * nr + slo) * n, h->Z + (int64_t(j) * nr + slo) * n,
                    s);
      core_spmv(h, nv, h->Z + (int64_t(j) * nr + slo) * n, nullptr, 1.0, Wb, s);
      {
        Timer tm(h, RSD_T_KRYLOV, s);
        double* hd = h->hdev + slo * hs;
        double* td = h->tmp + slo * hs;
        // classical Gram-Schmidt, twice
        hip_check(h, launch_mdot(nv, Vb, ldV, n, j + 1, Wb, n, n, h->part, hd, hs, 0, s),
                  "cgs dots");
        hip_check(h, launch_gemv_acc(nv, Vb, ldV, n, j + 1, hd, hs, -1.0, Wb, n, n, s),
                  "cgs update");
        hip_check(h, launch_mdot(nv, Vb, ldV, n, j + 1, Wb, n, n, h->part, td, hs, 0, s),
                  "cgs2 dots");
        hip_check(h, launch_gemv_acc(nv, Vb, ldV, n, j + 1, td, hs, -1.0, Wb, n, n, s),
                  "cgs2 update");
        hip_check(h, launch_small_add(nv, hd, hs, td, hs, j + 1, s), "h add");
        hip_check(h, launch_mdot(nv, Wb, n, n, 1, Wb, n, n, h->part, hd + j + 1, hs, 1, s),
                  "norm");
        hip_check(h, launch_scale_div(nv, Wb, n, hd + j + 1, hs,
                                      h->V + (int64_t(j + 1) * nr + slo) * n, n, n, s),
                  "normalise");
      }
      hip_check(h, hipMemcpyAsync(half(j), h->hdev + slo * hs, sizeof(double) * size_t(nv * hs),
                                  hipMemcpyDeviceToHost, s), "h D2H");
      hip_check(h, hipEventRecord(h->ev_h[j & 1], s), "hipEventRecord");
      qd[j & 1] = {slo, shi, true};
    };
    for (int j = 0; j < m; ++j) {
      if (!range(true, &lo, &hi)) break;
      if (!qd[j & 1].on) step(j, lo, hi);
      if (j + 1 < m) {                   // queue step j + 1 ahead?
        bool ahead = false;
        for (int i = lo; i < hi; ++i) {
          const Rhs& q = R[i];
          if (q.done || q.stop || q.its + 1 >= o.maxit) continue;
          const double r1 = std::fabs(q.g[j]);
          const double r0 = j > 0 ? std::fabs(q.g_prev) : 0.0;
          ahead = ahead || j == 0 || !(r0 > 0.0) || r1 * (r1 / r0) > q.tol;
        }
        if (ahead) step(j + 1, lo, hi);
      }
      hip_check(h, hipEventSynchronize(h->ev_h[j & 1]), "hipEventSynchronize");
      const Queued cur = qd[j & 1];
      qd[j & 1].on = false;
      for (int i = lo; i < hi; ++i) {
        Rhs& q = R[i];
        if (q.done || q.stop) continue;
        double* hc = &q.H[size_t(j) * (m + 1)];
        const double* src = half(j) + (i - cur.lo) * hs;
        for (int t = 0; t <= j + 1; ++t) {
          hc[t] = src[t];
          if (!(hc[t] == hc[t]) || std::isinf(hc[t])) q.bad = true;
        }
        if (q.bad) {
          q.stop = true;
          continue;
        }
        const double hnext = hc[j + 1];
        for (int t = 0; t < j; ++t) {
          const double t0 = q.cs[t] * hc[t] + q.sn[t] * hc[t + 1];
          hc[t + 1] = -q.sn[t] * hc[t] + q.cs[t] * hc[t + 1];
          hc[t] = t0;
        }
        const double den = std::hypot(hc[j], hc[j + 1]);
        q.cs[j] = den > 0 ? hc[j] / den : 1.0;
        q.sn[j] = den > 0 ? hc[j + 1] / den : 0.0;
        hc[j] = den;
        hc[j + 1] = 0.0;
        q.g_prev = q.g[j];
        q.g[j + 1] = -q.sn[j] * q.g[j];
        q.g[j] = q.cs[j] * q.g[j];
        ++q.its;
        q.k = j + 1;
        if (std::fabs(q.g[j + 1]) <= q.tol || q.its >= o.maxit || hnext == 0.0) q.stop = true;
      }
    }
    qd[0].on = qd[1].on = false;         // (a step queued ahead and not needed)
    // x_i += Z_i y_i with y_i = R_i^{-1} g_i (upper triangular k x k)
    bool any = false;
    for (int i = 0; i < nr; ++i) {
      Rhs& q = R[i];
      if (q.done) continue;
      if (q.bad) {
        finish(i, RSD_ERR_BREAKDOWN, NAN);
        continue;
      }
      for (int t = q.k - 1; t >= 0; --t) {
        double v = q.g[t];
        for (int c = t + 1; c < q.k; ++c) v -= q.H[size_t(c) * (m + 1) + t] * q.y[c];
        const double d = q.H[size_t(t) * (m + 1) + t];
        q.y[t] = d != 0.0 ? v / d : 0.0;
      }
      for (int t = 0; t < q.k; ++t) h->hhost[i * hs + t] = q.y[t];
      any = true;
    }
    if (!any) return;
    hip_check(h, hipMemcpyAsync(h->tmp, h->hhost, sizeof(double) * size_t(nr * hs),
                                hipMemcpyHostToDevice, s), "y H2D");
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      for (int i = 0; i < nr; ++i)
        if (!R[i].done)
          hip_check(h, launch_gemv_acc(1, h->Z + i * n, ldV, 0, R[i].k, h->tmp + i * hs, 0, 1.0,
                                       x + i * n, 0, n, s), "x update");
    }
    residuals();
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
  core_spmv(h, 1, x, b, -1.0, r, s);
  double rn = dev_norm(h, r, h->scal + 3, s);
  int its = 0;
  int cur = 0;
  if (rn <= tol) {
    info->iterations = 0;
    info->relres = rn / bnorm;
    return RSD_OK;
  }
  apply_vectors(h, 1, r, z, s);
  {
    Timer tm(h, RSD_T_KRYLOV, s);
    hip_check(h, launch_mdot(1, r, n, 0, 1, z, 0, n, h->part, h->scal + cur, 0, 0, s), "rz");
    hip_check(h, hipMemcpyAsync(p, z, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, s),
              "p = z");
  }
  for (;;) {
    core_spmv(h, 1, p, nullptr, 1.0, q, s);
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      hip_check(h, launch_mdot(1, p, n, 0, 1, q, 0, n, h->part, h->scal + 2, 0, 0, s), "pq");
      hip_check(h, launch_axpy_ratio(x, p, h->scal + cur, h->scal + 2, 1.0, x, n, s), "x");
      hip_check(h, launch_axpy_ratio(r, q, h->scal + cur, h->scal + 2, -1.0, r, n, s), "r");
      hip_check(h, launch_mdot(1, r, n, 0, 1, r, 0, n, h->part, h->scal + 3, 0, 1, s), "|r|");
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
      core_spmv(h, 1, x, b, -1.0, r, s);
      const double rt = dev_norm(h, r, h->scal + 3, s);
      if (rt <= tol) {
        info->iterations = its;
        info->relres = rt / bnorm;
        return RSD_OK;
      }
    }
    if (its >= o.maxit) {
      core_spmv(h, 1, x, b, -1.0, h->w, s);
      info->iterations = its;
      info->relres = dev_norm(h, h->w, h->scal + 5, s) / bnorm;
      return RSD_ERR_NOT_CONVERGED;
    }
    apply_vectors(h, 1, r, z, s);
    {
      Timer tm(h, RSD_T_KRYLOV, s);
      const int nxt = 1 - cur;
      hip_check(h, launch_mdot(1, r, n, 0, 1, z, 0, n, h->part, h->scal + nxt, 0, 0, s), "rz");
      hip_check(h, launch_axpy_ratio(z, p, h->scal + nxt, h->scal + cur, 1.0, p, n, s), "p");
      cur = nxt;
    }
  }
}

}  // namespace

rsd_status engine_apply(rsd_ctx* h, int nrhs, const double* r, int64_t ldr, double* z,
                        int64_t ldz, hipStream_t s) {
  try {
    const int64_t n = h->P.n;
    enter(h, s);
    for (int j0 = 0; j0 < nrhs; j0 += kRhsGroup) {
      const int c = std::min(kRhsGroup, nrhs - j0);
      ensure_vectors(h, c);
      permute(h, c, r + size_t(j0) * ldr, ldr, h->rin, n, 0, s);
      apply_vectors(h, c, h->rin, h->zin, s);
      permute(h, c, h->zin, n, z + size_t(j0) * ldz, ldz, 1, s);
    }
    leave(h, s);
    return RSD_OK;
  } catch (const Fail& f) {
    return f.st;
  }
}

namespace {

// consecutive 256-byte aligned pieces of one block (sizes only while base is null)
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

// the apply work of nv vectors laid out in a Carver: the permuted input and output, then
// the buffers of ApplyWork sized as ensure_vectors / ensure_gamma size the handle's own
void carve_apply(const rsd_ctx* h, int nv, Carver& c, double** rin, double** zin,
                 ApplyWork* w) {
  const size_t n = size_t(h->P.n), nB = std::max<size_t>(1, h->P.B.size());
  *rin = c.take<double>(n * size_t(nv));
  *zin = c.take<double>(n * size_t(nv));
  w->t = c.take<double>(n * size_t(nv));
  w->e = c.take<double>(nB * size_t(nv));
  w->xil = nv > 1 ? c.take<double>(n * size_t(kEllVec)) : nullptr;
  w->sympart = c.take<char>(h->sympart_bytes);
  if (h->any_gamma) {
    int32_t maxc = 1;
    for (const DevBatch& b : h->lev) maxc = std::max(maxc, b.count);
    const size_t g = size_t(h->opt.gamma), sl = size_t(nv) * size_t(maxc);
    w->gm_V = c.take<double>((g + 1) * size_t(nv) * n);
    w->gm_beta = c.take<double>(sl);
    w->gm_H = c.take<double>(sl * (g + 1) * g);
    w->gm_steps = c.take<int32_t>(sl);
    w->gm_stop = c.take<int32_t>(sl);
    w->gm_part = c.take<double>(size_t(nv) * size_t(std::max(1, h->gm_max_items)) * (g + 1));
    w->gm_coef = c.take<double>(sl * (g + 2));
  }
}

}  // namespace

size_t apply_static_bytes(const rsd_ctx* h, int nv) {
  Carver c;
  double *rin = nullptr, *zin = nullptr;
  ApplyWork w;
  carve_apply(h, nv, c, &rin, &zin, &w);
  return c.off;
}

rsd_status engine_apply_static(rsd_ctx* h, int nrhs, const double* r, int64_t ldr, double* z,
                               int64_t ldz, void* area, size_t cap, hipStream_t s) {
  try {
    int c = std::min(kRhsGroup, nrhs);
    while (c > 1 && apply_static_bytes(h, c) > cap) --c;
    const size_t need = apply_static_bytes(h, c);
    if (need > cap) {
      h->err = "rsd_apply_noalloc: one column of this handle needs " + std::to_string(need) +
               " bytes of work memory; the static area holds " + std::to_string(cap);
      return RSD_ERR_INVALID_ARGUMENT;
    }
    const int64_t n = h->P.n;
    enter(h, s);
    h->no_events = 1;   // the timers count launches only: no event objects are created
    for (int j0 = 0; j0 < nrhs; j0 += c) {
      const int cc = std::min(c, nrhs - j0);
      Carver cv;
      cv.base = static_cast<char*>(area);
      double *rin = nullptr, *zin = nullptr;
      ApplyWork w;
      carve_apply(h, cc, cv, &rin, &zin, &w);
      permute(h, cc, r + size_t(j0) * ldr, ldr, rin, n, 0, s);
      core_apply(h, w, cc, rin, zin, s);
      permute(h, cc, zin, n, z + size_t(j0) * ldz, ldz, 1, s);
    }
    h->no_events = 0;
    leave(h, s);
    return RSD_OK;
  } catch (const Fail& f) {
    h->no_events = 0;
    return f.st;
  }
}

rsd_status engine_spmv(rsd_ctx* h, int nrhs, const double* x, int64_t ldx, double* y,
                       int64_t ldy, hipStream_t s) {
  try {
    const int64_t n = h->P.n;
    enter(h, s);
    for (int j0 = 0; j0 < nrhs; j0 += kRhsGroup) {
      const int c = std::min(kRhsGroup, nrhs - j0);
      ensure_vectors(h, c);
      permute(h, c, x + size_t(j0) * ldx, ldx, h->rin, n, 0, s);
      core_spmv(h, c, h->rin, nullptr, 1.0, h->zin, s);
      permute(h, c, h->zin, n, y + size_t(j0) * ldy, ldy, 1, s);
    }
    leave(h, s);
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
    const bool pcg = o.method == RSD_SOLVER_PCG;
    const int group = pcg ? 1 : std::min(kRhsGroup, std::max(nrhs, 1));
    enter(h, s);
    ensure_krylov(h, pcg ? 4 : o.restart, group);
    ensure_vectors(h, group);
    const int64_t n = h->P.n;
    rsd_status worst = RSD_OK;
    std::vector<rsd_solve_info> inf(static_cast<size_t>(group));
    for (int j0 = 0; j0 < nrhs; j0 += group) {
      const int c = std::min(group, nrhs - j0);
      permute(h, c, b + size_t(j0) * ldb, ldb, h->bint, n, 0, s);
      if (o.use_x0)
        permute(h, c, x + size_t(j0) * ldx, ldx, h->xint, n, 0, s);
      else
        hip_check(h, launch_fill(h->xint, n * c, 0.0, s), "x0");
      if (pcg)
        inf[0].status = pcg_one(h, h->bint, h->xint, o, &inf[0], s);
      else
        fgmres_group(h, c, h->bint, h->xint, o, inf.data(), s);
      permute(h, c, h->xint, n, x + size_t(j0) * ldx, ldx, 1, s);
      for (int k = 0; k < c; ++k) {
        const rsd_status st = static_cast<rsd_status>(inf[k].status);
        if (info) info[j0 + k] = inf[k];
        if (st == RSD_ERR_BREAKDOWN || (st != RSD_OK && worst == RSD_OK)) worst = st;
      }
    }
    hip_check(h, hipStreamSynchronize(s), "hipStreamSynchronize");
    leave(h, s);
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
    if (h->last_tuned > 0)
      for (int i = 0; i < 8; ++i) {
        out->vec_pass[i] = h->vec_pass[size_t(h->last_tuned)][size_t(i)] & 15;
        out->sym_persist[i] = h->vec_pass[size_t(h->last_tuned)][size_t(i)] >> 4;
      }
    for (int i = 0; i < 8; ++i) out->setup_variant[i] = h->setup_variant[i];
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
  // every call of the handle ends with its work joined onto the call's stream and ev_last
  // recorded there (set-up and solves also synchronise), so this waits for all of it
  if (h->has_last) (void)hipEventSynchronize(h->ev_last);
  drop_graphs(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  h->cap = nullptr;
  {                                            // completed: back to the process-wide pool
    AuxPool& ap = aux_pool();
    std::lock_guard<std::mutex> lock(ap.mu);
    std::vector<hipEvent_t>& v = ap.events[h->device];
    for (auto& p : h->pending) {
      v.push_back(p.a);
      v.push_back(p.b);
    }
    v.insert(v.end(), h->pool.begin(), h->pool.end());
  }
  h->pending.clear();
  h->pool.clear();
  if (h->ev_main) (void)hipEventDestroy(h->ev_main);
  if (h->ev_aux) (void)hipEventDestroy(h->ev_aux);
  if (h->ev_upl) (void)hipEventDestroy(h->ev_upl);
  if (h->ev_sig) (void)hipEventDestroy(h->ev_sig);
  h->ev_upl = h->ev_sig = nullptr;
  for (hipEvent_t& e : h->ev_lev)
    if (e) (void)hipEventDestroy(e);
  h->ev_lev.clear();
  if (h->ev_last) (void)hipEventDestroy(h->ev_last);
  h->ev_main = h->ev_aux = h->ev_last = nullptr;
  h->has_last = false;
  if (h->aux) give_aux(h->device, h->aux);   // idle: its work was joined and completed
  h->aux = nullptr;
  if (h->upl) {                                // (its work, the couplings' copy and the
    (void)hipStreamSynchronize(h->upl);        // Schur assemblies, was joined onto the
    give_aux(h->device, h->upl);               // set-up's stream; a failed set-up may have
  }                                            // stopped before those waits)
  h->upl = nullptr;
  BlockCache& c = cache_of(h->device);
  for (auto& p : h->allocs) {                                           // work is complete
    if (h->opt.dev_free)
      h->opt.dev_free(p.first, h->opt.alloc_ctx);
    else
      cache_give(c, p.first, p.second, false);
  }
  h->allocs.clear();
  h->device_bytes = 0;
  pfree(h, h->hhost_block);
  h->hhost = nullptr;
  for (hipEvent_t& e : h->ev_h) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  pfree(h, h->csr_stage);
  for (Pinned& b : h->held) pfree(h, b);
  h->held.clear();
}

void release_cache(int device) {
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return;
  for (int d = 0; d < count; ++d) {
    if (device >= 0 && d != device) continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    {
      AuxPool& p = aux_pool();
      std::lock_guard<std::mutex> lock(p.mu);
      for (hipStream_t st : p.idle[d]) (void)hipStreamDestroy(st);
      p.idle[d].clear();
      for (hipEvent_t e : p.events[d]) (void)hipEventDestroy(e);
      p.events[d].clear();
    }
    cache_drain(cache_of(d), false);
    cache_drain(cache_of(-1 - d), true);
  }
  (void)hipSetDevice(cur);
}

}  // namespace rsd
