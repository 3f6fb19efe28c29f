// HIP kernels for gfx950 (CDNA4): sparse couplings, batched dense symmetric
// blocks (in-place inversion on MFMA, symmetric products), Schur complements of
// the sub-domain hierarchy, and the Krylov vector kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"

namespace rsd {

namespace {

constexpr int TS = 64;            // tile side
constexpr int TT = TS * TS;       // tile elements
constexpr int kBlock = 256;

// partial sums of the symmetric products: FP32 for FP32 and 16-bit factors, FP64 otherwise
template <typename T>
struct SymPart { using type = double; };
template <>
struct SymPart<float> { using type = float; };
template <>
struct SymPart<_Float16> { using type = float; };
template <>
struct SymPart<__bf16> { using type = float; };

__host__ __device__ __forceinline__ int64_t tri(int64_t I) { return I * (I + 1) / 2; }
__device__ __forceinline__ int64_t tile_index(int I, int J) { return tri(I) + J; }

// (I, J) of the t-th lower tile in row-major tile order
__host__ __device__ __forceinline__ void tile_ij(int64_t t, int* I, int* J) {
  int i = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (tri(i) > t) --i;
  while (tri(i + 1) <= t) ++i;
  *I = i;
  *J = int(t - tri(i));
}

// (I, J) of the s-th lower tile of an n x n tile triangle in band order: bands of
// kBand tile rows, each band walked kBand x kBand block by block (left to right,
// the diagonal triangle last).  The lower tiles of any kBand x kBand block are
// consecutive, so workgroups that run at the same time share kBand row panels and
// kBand column panels instead of one row panel and many column panels.
constexpr int kBand = 8;
__host__ __device__ __forceinline__ void band_ij(int64_t s, int n, int* I, int* J) {
  int i, j;
  tile_ij(s, &i, &j);                          // row in plain order picks the band
  const int r0 = (i / kBand) * kBand, h = min(kBand, n - r0);
  const int64_t t = s - tri(r0), full = int64_t(r0) * h;
  if (t < full) {
    const int64_t cb = t / (int64_t(kBand) * h), u = t % (int64_t(kBand) * h);
    *I = r0 + int(u % h);
    *J = int(cb) * kBand + int(u / h);
  } else {
    tile_ij(t - full, &i, &j);
    *I = r0 + i;
    *J = r0 + j;
  }
}

// a load of data streamed once per use (matrix tiles, Sigma blocks, sparse slots): the
// non-temporal hint keeps it from displacing reused data in the caches
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}

// element (r, c) of the symmetric matrix whose lower tiles start at base
template <typename T>
__device__ __forceinline__ T sym_elem(const T* base, int r, int c) {
  const int I = r / TS, J = c / TS;
  if (I >= J) return base[tile_index(I, J) * TT + (r % TS) + (c % TS) * TS];
  return base[tile_index(J, I) * TT + (c % TS) + (r % TS) * TS];
}

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// 64 x 64 block product on MFMA 16x16x4 by 4 waves (each wave a 32 x 32 quadrant):
// acc += A(64 x K) * B(K x 64).  A(r, k) = lda(r, k), B(k, c) = ldb(k, c).
// The position of accumulator element acc[bi][bj][v] is given by acc_pos<T>.
template <typename T, int K, typename LA, typename LB>
__device__ __forceinline__ void mfma_block(LA lda, LB ldb, typename Mfma<T>::v4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 8
  for (int k = 0; k < K; k += 4) {
    const T a0 = lda(r0 + li, k + lk), a1 = lda(r0 + 16 + li, k + lk);
    const T b0 = ldb(k + lk, c0 + li), b1 = ldb(k + lk, c0 + 16 + li);
    acc[0][0] = Mfma<T>::op(a0, b0, acc[0][0]);
    acc[0][1] = Mfma<T>::op(a0, b1, acc[0][1]);
    acc[1][0] = Mfma<T>::op(a1, b0, acc[1][0]);
    acc[1][1] = Mfma<T>::op(a1, b1, acc[1][1]);
  }
}

// Position in the 64 x 64 block of accumulator element acc[bi][bj][v].  Both
// instructions take A(i, k) from lane i + 16 k and B(k, j) from lane j + 16 k; the
// 16 x 16 result lies in lane j + 16 g, element v, with row i = 4 g + v for FP32 but
// row i = 4 v + g for FP64 (checked on gfx950).
template <typename T>
__device__ __forceinline__ void acc_pos(int bi, int bj, int v, int* r, int* c) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int i = (sizeof(T) == 8) ? 4 * v + g : 4 * g + v;
  *r = (w >> 1) * 32 + 16 * bi + i;
  *c = (w & 1) * 32 + 16 * bj + (lane & 15);
}

// ================================================================ sparse / vectors
__global__ void k_gather(const double* __restrict__ src, const int64_t* __restrict__ map,
                         int64_t count, double* __restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[map[i]];
}

__global__ void k_permute(const double* __restrict__ x, int64_t ldx, double* __restrict__ y,
                          int64_t ldy, const int32_t* __restrict__ perm, int64_t n,
                          int inverse) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  if (inverse)
    y[int64_t(perm[i]) + j * ldy] = x[i + j * ldx];   // internal -> caller
  else
    y[i + j * ldy] = x[int64_t(perm[i]) + j * ldx];   // caller -> internal
}

// ---- sliced ELL copy of K (internal order) for the SpMVs -------------------------------
// Entry k of row r sits at ell_off[r / 64] + 64 k + r % 64: a wave's 64 rows read each
// k as one coalesced load, one thread per row, no cross-lane reduction.  Padding
// entries hold column r and value 0.
__global__ __launch_bounds__(kEllSlice) void k_ell_fill(int64_t n, const int64_t* __restrict__ prow,
                                                        const int32_t* __restrict__ pcol,
                                                        const double* __restrict__ pval,
                                                        const int64_t* __restrict__ ell_off,
                                                        int32_t* __restrict__ ell_col,
                                                        double* __restrict__ ell_val) {
  // one wave per slice: the slice's CSR entries are contiguous, read coalesced; each
  // finds its row by bisection over the slice's row starts (LDS) and is written to its
  // slot; then the padding slots of each row
  const int64_t sl = blockIdx.x, r0 = sl * kEllSlice;
  const int rows = int(min<int64_t>(kEllSlice, n - r0)), l = threadIdx.x;
  __shared__ int64_t rs[kEllSlice + 1];     // row starts of the slice and its end
  if (l < rows) rs[l] = prow[r0 + l];
  if (l == 0) rs[rows] = prow[r0 + rows];
  __syncthreads();
  const int64_t w = (ell_off[sl + 1] - ell_off[sl]) / kEllSlice;
  int32_t* col = ell_col + ell_off[sl];
  double* val = ell_val + ell_off[sl];
  for (int64_t q = rs[0] + l; q < rs[rows]; q += kEllSlice) {
    int lo = 0, hi = rows;                     // rs[lo] <= q < rs[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (rs[mid] <= q) lo = mid; else hi = mid;
    }
    const int64_t k = q - rs[lo];
    col[k * kEllSlice + lo] = pcol[q];
    val[k * kEllSlice + lo] = pval[q];
  }
  if (l < rows)
    for (int64_t k = rs[l + 1] - rs[l]; k < w; ++k) {
      col[k * kEllSlice + l] = int32_t(r0 + l);
      val[k * kEllSlice + l] = 0.0;
    }
}

// xil[i KV + k] = x_k[i] (k < nv), 0 for nv <= k < KV: the vectors of a column side by
// side, so that one lane's gather for all of them is KV contiguous doubles.
template <int KV>
__global__ __launch_bounds__(kBlock) void k_interleave(const double* __restrict__ x, int nv,
                                                       int64_t ld, int64_t col0, int64_t col1,
                                                       double* __restrict__ xil) {
  const int64_t i = col0 + int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= col1) return;
  typedef double D2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int k = 0; k < KV; k += 2) {
    D2 v;
    v.x = k < nv ? x[k * ld + i] : 0.0;
    v.y = k + 1 < nv ? x[(k + 1) * ld + i] : 0.0;
    *(D2*)(xil + i * KV + k) = v;
  }
}

// y_k[r] = (base ? base_k[r] : 0) + alpha * sum over the entries of row r with CSR
// positions in [s0[r], s1[r]) (contiguous: columns are sorted), rows r in
// [row0, row0 + nrows), for the nv <= KV vectors x_k = x + k ld (likewise base, y).
// The slots are read once for all vectors; with IL the gathers read the interleaved
// copy xil of x.  Each vector's sum has the same order whatever KV is.  x, base and y
// may be the same vectors when the columns read are not the rows written.
template <int KV, bool IL>
__global__ __launch_bounds__(kBlock) void k_ell_spmv(
    int64_t row0, int64_t nrows, const int64_t* __restrict__ s0, const int64_t* __restrict__ s1,
    const int64_t* __restrict__ prow, const int64_t* __restrict__ ell_off,
    const int32_t* __restrict__ ell_col, const double* __restrict__ ell_val,
    const double* x, const double* __restrict__ xil, const double* base, double alpha,
    double* y, int nv, int64_t ld) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nrows) return;
  const int64_t r = row0 + i;
  const int64_t p0 = prow[r];
  const int64_t k0 = s0[r] - p0, k1 = s1[r] - p0;
  const int64_t o = ell_off[r / kEllSlice] + r % kEllSlice;
  const int32_t* c = ell_col + o;
  const double* v = ell_val + o;
  // eight slots at a time: their column and value loads are independent, then the
  // eight gathers of x; out-of-range slots read slot k0 with a zero weight
  double acc[KV];
#pragma unroll
  for (int k = 0; k < KV; ++k) acc[k] = 0.0;
  for (int64_t kb = k0; kb < k1; kb += 8) {
    int32_t ci[8];
    double vi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t kk = kb + u < k1 ? kb + u : k0;
      ci[u] = ld_stream(c + kk * kEllSlice);
      vi[u] = kb + u < k1 ? ld_stream(v + kk * kEllSlice) : 0.0;
    }
    if constexpr (IL) {
      typedef double D2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const D2* xp = (const D2*)(xil + int64_t(ci[u]) * KV);
#pragma unroll
        for (int k = 0; k < KV; k += 2) {
          const D2 xv = xp[k / 2];
          acc[k] += vi[u] * xv.x;
          acc[k + 1] += vi[u] * xv.y;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int k = 0; k < KV; ++k)
          if (KV == 1 || k < nv) acc[k] += vi[u] * x[k * ld + ci[u]];
    }
  }
#pragma unroll
  for (int k = 0; k < KV; ++k)
    if (KV == 1 || k < nv) y[k * ld + r] = (base ? base[k * ld + r] : 0.0) + alpha * acc[k];
}

// Row r of K in internal order: row perm[r] of the caller's CSR with columns renamed by
// iperm and sorted, the caller's value position of each entry, and the row segments:
// first interface column (segA); for interface rows the end of the deeper-level columns
// (segB) and of the own node's columns (segC).  One wave per row: lane l holds entries
// l, l + 64, ... (up to kPermSlots each); the columns are distinct, so an entry's place
// is the number of smaller columns, counted by broadcasting every column once, and a
// segment bound is the number of columns below it (ballots).  Longer rows: one lane
// sorts by insertion.
constexpr int kPermSlots = 4;
constexpr int kPermRows = kBlock / 64;         // rows per workgroup
__global__ __launch_bounds__(kBlock) void k_permute_csr(
    int32_t n, int64_t n_leaf, const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const int64_t* __restrict__ prow, const int32_t* __restrict__ skel_lvl_begin,
    const int32_t* __restrict__ skel_own_end, int32_t* __restrict__ pcol,
    int64_t* __restrict__ pmap, int64_t* __restrict__ segA, int64_t* __restrict__ segB,
    int64_t* __restrict__ segC) {
  const int64_t r = int64_t(blockIdx.x) * kPermRows + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (r >= n) return;                          // (the same for the whole wave)
  const int32_t o = perm[r];
  const int64_t k0 = rp[o], len = rp[o + 1] - k0, base = prow[r];
  const int32_t lb = r < n_leaf ? 0 : skel_lvl_begin[r - n_leaf];
  const int32_t oe = r < n_leaf ? 0 : skel_own_end[r - n_leaf];
  int64_t na = 0, nb = 0, nc = 0;              // columns below n_leaf, lb, oe
  if (len <= 64 * kPermSlots) {
    int32_t key[kPermSlots];
    int32_t rank[kPermSlots];
#pragma unroll
    for (int sl = 0; sl < kPermSlots; ++sl) {
      const int64_t e = int64_t(sl) * 64 + lane;
      key[sl] = e < len ? iperm[ci[k0 + e]] : INT32_MAX;
      rank[sl] = 0;
    }
#pragma unroll
    for (int sj = 0; sj < kPermSlots; ++sj) {
      const int cnt = int(min<int64_t>(64, len - int64_t(sj) * 64));
      for (int j = 0; j < cnt; ++j) {
        const int32_t kj = __shfl(key[sj], j, 64);
#pragma unroll
        for (int sl = 0; sl < kPermSlots; ++sl) rank[sl] += kj < key[sl] ? 1 : 0;
      }
    }
#pragma unroll
    for (int sl = 0; sl < kPermSlots; ++sl) {
      const int64_t e = int64_t(sl) * 64 + lane;
      const bool ok = e < len;
      if (ok) {
        pcol[base + rank[sl]] = key[sl];
        pmap[base + rank[sl]] = k0 + e;
      }
      na += __popcll(__ballot(ok && key[sl] < n_leaf));
      nb += __popcll(__ballot(ok && key[sl] < lb));
      nc += __popcll(__ballot(ok && key[sl] < oe));
    }
  } else {
    if (lane != 0) return;
    int32_t* c = pcol + base;
    int64_t* v = pmap + base;
    for (int64_t e = 0; e < len; ++e) {
      const int32_t kc = iperm[ci[k0 + e]];
      int64_t w = e;
      while (w > 0 && c[w - 1] > kc) {
        c[w] = c[w - 1];
        v[w] = v[w - 1];
        --w;
      }
      c[w] = kc;
      v[w] = k0 + e;
    }
    for (int64_t e = 0; e < len; ++e) {
      na += c[e] < n_leaf;
      nb += c[e] < lb;
      nc += c[e] < oe;
    }
  }
  if (lane != 0) return;
  segA[r] = base + na;
  if (r < n_leaf) {
    segB[r] = segC[r] = base + na;
    return;
  }
  // (sorted columns: the deeper-level segment starts at the first interface column)
  const int64_t b = na > nb ? na : nb;
  segB[r] = base + b;
  segC[r] = base + (b > nc ? b : nc);
}

__global__ void k_fill(double* p, int64_t count, double v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// ================================================================ dense batches
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sym_fill(T* tiles, const int64_t* tile_off,
                                                     const int32_t* n_arr,
                                                     const int32_t* nt_arr) {
  const int m = blockIdx.y;
  const int nt = nt_arr[m];
  const int64_t t = blockIdx.x;
  if (t >= tri(nt)) return;
  int I, J;
  tile_ij(t, &I, &J);
  T* p = tiles + tile_off[m] + t * TT;
  const int n = n_arr[m];
  for (int e = threadIdx.x; e < TT; e += kBlock) {
    const int r = I * TS + (e % TS), c = J * TS + (e / TS);
    p[e] = (r == c && r >= n) ? T(1) : T(0);   // padding: identity
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sym_extract(T* tiles, const int64_t* tile_off,
                                                        const int32_t* n_arr,
                                                        const int64_t* vec_off,
                                                        const int64_t* s0, const int64_t* s1,
                                                        const int32_t* pcol,
                                                        const double* pval) {
  const int m = blockIdx.y;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int n = n_arr[m];
  if (i >= n) return;
  const int64_t off = vec_off[m];
  const int64_t r = off + i;
  T* base = tiles + tile_off[m];
  for (int64_t k = s0[r]; k < s1[r]; ++k) {
    const int64_t j = int64_t(pcol[k]) - off;
    if (j < 0 || j >= n) continue;
    const int I = i / TS, J = int(j) / TS;
    if (I < J) continue;
    base[tile_index(I, J) * TT + (i % TS) + (j % TS) * TS] = T(pval[k]);
  }
}

// ---- blocked symmetric sweep (in-place inversion) --------------------------------------
// Step over pivot tile columns [c0, c0 + g): with the pivot block P = A_pp^{-1},
//   A_ij -= A_ip P A_pj  (i, j outside the pivot group),
//   A_ip <- A_ip P,  A_pj <- P A_pj,  A_pp <- -P.
// After all steps the tiles hold -A^{-1}.

// (1) pivot block: scalar sweeps of the G*64 x G*64 block held in registers by
// 1024 threads (a 32 x 32 grid of R x R sub-blocks).  Each pivot p applies the
// rank-one update to every element (branch-free), then the owners of row p and
// column p overwrite them with the scaled pivot column and -1/d.
constexpr int kPivotThreads = 1024;
template <typename T, int G>
__global__ __launch_bounds__(kPivotThreads) void k_sweep_pivot(T* tiles, const int64_t* tile_off,
                                                               const int32_t* nt_arr, int c0,
                                                               T* pbuf, int32_t* flags) {
  constexpr int PB = G * TS, R = PB / 32;
  const int m = blockIdx.x;
  const int nt = nt_arr[m];
  if (c0 >= nt) return;
  const int g = min(G, nt - c0), pbm = g * TS;
  T* base = tiles + tile_off[m];
  const int ty = threadIdx.x / 32, tx = threadIdx.x % 32;
  T a[R][R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int gi = ty * R + i, gj = tx * R + j;
      if (gi < pbm && gj < pbm)
        a[i][j] = sym_elem(base, c0 * TS + gi, c0 * TS + gj);
      else
        a[i][j] = (gi == gj) ? T(1) : T(0);
    }
  __shared__ T colbuf[2][PB];
  int fail = 0;
  for (int p = 0; p < pbm; ++p) {
    T* cb = colbuf[p & 1];
    const int owner = p / R, pp = p % R;
    if (tx == owner) {   // owner of column p publishes it (select keeps a[][] in VGPRs)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        T v = a[i][0];
#pragma unroll
        for (int j = 1; j < R; ++j) v = (j == pp) ? a[i][j] : v;
        cb[ty * R + i] = v;
      }
    }
    __syncthreads();
    T d = cb[p];
    if (!(d > T(0)) || !(d < T(INFINITY))) {
      fail = 1;
      d = T(1);
    }
    const T inv = T(1) / d;
    T ci[R], cj[R];
#pragma unroll
    for (int i = 0; i < R; ++i) ci[i] = cb[ty * R + i];
#pragma unroll
    for (int j = 0; j < R; ++j) cj[j] = cb[tx * R + j];
    // (c_i c_j) inv is symmetric in (i, j), so an exactly symmetric block stays so
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) a[i][j] -= (ci[i] * cj[j]) * inv;
    if (ty == owner) {   // row p: c_j / d
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) a[i][j] = (i == pp) ? cj[j] * inv : a[i][j];
    }
    if (tx == owner) {   // column p: c_i / d, and -1/d on the diagonal
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j)
          a[i][j] = (j == pp) ? ((ty == owner && i == pp) ? -inv : ci[i] * inv) : a[i][j];
    }
  }
  T* P = pbuf + int64_t(m) * PB * PB;
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int gi = ty * R + i, gj = tx * R + j;
      P[gi + gj * PB] = -a[i][j];
      if (gi < pbm && gj < pbm) {
        const int I = c0 + gi / TS, J = c0 + gj / TS;
        if (I >= J) base[tile_index(I, J) * TT + (gi % TS) + (gj % TS) * TS] = a[i][j];
      }
    }
  if (fail && threadIdx.x == 0) flags[m] = c0 + 1;
}

// ---- blocked pivot: the pivot group (G tiles) inverted by one workgroup in 64-wide
// sub-steps.  Each diagonal 64 x 64 block is swept by a single wave (wave-synchronous:
// the pivot column is broadcast through LDS without workgroup barriers); the panel and
// the update inside the group are single-wave 64 x 64 x 64 MFMA products.

// ordering of a wave's LDS writes before its later reads (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 64 scalar sweeps of the symmetric 64 x 64 block at A (column-major, ld 64) by one
// wave, lanes on an 8 x 8 grid holding 8 x 8 each: A <- -A^{-1}, P <- A^{-1} (ld 64).
// The inner eight pivots are unrolled so that every register index is static: the
// owners of row / column p overwrite one row / column of their block directly.
template <typename T>
__device__ __forceinline__ void wave_sweep64(T* A, T* P, T* col, int* fail) {
  const int lane = threadIdx.x & 63, ly = lane >> 3, lx = lane & 7;
  T a[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) a[i][j] = A[(ly * 8 + i) + (lx * 8 + j) * TS];
  int f = 0;
  for (int ob = 0; ob < 8; ++ob) {
#pragma unroll
    for (int pp = 0; pp < 8; ++pp) {
      const int p = ob * 8 + pp;
      T* cb = col + (pp & 1) * TS;
      if (lx == ob) {
#pragma unroll
        for (int i = 0; i < 8; ++i) cb[ly * 8 + i] = a[i][pp];
      }
      wave_sync();
      T d = cb[p];
      if (!(d > T(0)) || !(d < T(INFINITY))) {
        f = 1;
        d = T(1);
      }
      const T inv = T(1) / d;
      T ci[8], cs[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) ci[i] = cb[ly * 8 + i];
#pragma unroll
      for (int j = 0; j < 8; ++j) cs[j] = cb[lx * 8 + j] * inv;
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[i][j] = fma(-ci[i], cs[j], a[i][j]);
      if (ly == ob) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[pp][j] = cs[j];           // row p: c_j / d
      }
      if (lx == ob) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i][pp] = ci[i] * inv;     // column p: c_i / d
        if (ly == ob) a[pp][pp] = -inv;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      A[(ly * 8 + i) + (lx * 8 + j) * TS] = a[i][j];
      P[(ly * 8 + i) + (lx * 8 + j) * TS] = -a[i][j];
    }
  if (f) *fail = 1;
}

// one wave: acc += A(64 x 64) B(64 x 64) on MFMA 16x16x4, acc[bi][bj] at acc_pos64
template <typename T, typename LA, typename LB>
__device__ __forceinline__ void wave_gemm64(LA lda, LB ldb, typename Mfma<T>::v4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < TS; k += 4) {
    T a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = lda(16 * q + li, k + lk);
      b[q] = ldb(k + lk, 16 * q + li);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = Mfma<T>::op(a[bi], b[bj], acc[bi][bj]);
  }
}


template <typename T>
__device__ __forceinline__ int acc_row64(int bi, int v) {
  const int g = (threadIdx.x & 63) >> 4;
  return 16 * bi + ((sizeof(T) == 8) ? 4 * v + g : 4 * g + v);
}

// threads of the blocked pivot: 8 waves for FP32, 4 for FP64 (register budget)
template <typename T>
struct PivCfg { static constexpr int threads = sizeof(T) == 8 ? 256 : 512; };
template <typename T, int G>
__global__ __launch_bounds__(PivCfg<T>::threads) void k_sweep_pivot_blk(
    T* tiles, const int64_t* tile_off, const int32_t* nt_arr, int c0, T* pbuf, int32_t* flags) {
  constexpr int PB = G * TS, NTH = PivCfg<T>::threads, NW = NTH / 64;
  // on the critical path while the bulk update of the previous step shares the compute
  // units: its waves take issue priority over the update's
  __builtin_amdgcn_s_setprio(3);
  const int m = blockIdx.x;
  const int nt = nt_arr[m];
  if (c0 >= nt) return;
  const int g = min(G, nt - c0);
  T* base = tiles + tile_off[m];
  T* P = pbuf + int64_t(m) * PB * PB;          // written during the last sub-step
  __shared__ T Ps[TT];
  __shared__ T Bs[(G > 1 ? G - 1 : 1) * TT];
  __shared__ T col[2 * TS];
  __shared__ int fail;
  // FP32: the sub-step's pivot-column tiles C_r (r != s) are staged in LDS by the other
  // waves while wave 0 sweeps the diagonal tile, for the panel and the in-group update
  // (FP64 reads them from global memory: 96 KB more would not fit).  Cs[r'][k][row] with
  // k-rows padded to LDC (conflict-free reads of 16 rows x 4 k-rows per instruction).
  constexpr bool kStageC = sizeof(T) == 4 && G > 1;
  constexpr int LDC = TS + 16, CST = TS * LDC;
  __shared__ T Cs[kStageC ? (G - 1) * CST : 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15;
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  auto tl = [&](int r, int c) { return base + tile_index(c0 + r, c0 + c) * TT; };
  auto pel = [&](int I, int J, int r, int c) -> T& { return P[(I * TS + r) + int64_t(J * TS + c) * PB]; };
  for (int s = 0; s < g; ++s) {
    const bool last = s == g - 1;
    if (w == 0) {
      wave_sweep64(tl(s, s), Ps, col, &fail);
    } else if constexpr (kStageC) {
      // C_r(row, k) = A[r][s](row, k) for r > s, A[s][r](k, row) for r < s (r' = the index
      // of r among the group's rows other than s)
      for (int e = threadIdx.x - 64; e < (g - 1) * TT; e += NTH - 64) {
        const int rr = e / TT, x = e % TT, row = x % TS, k = x / TS;
        const int r = rr < s ? rr : rr + 1;
        Cs[rr * CST + k * LDC + row] = r > s ? tl(r, s)[row + k * TS] : tl(s, r)[k + row * TS];
      }
    }
    __syncthreads();
    if (last)                                  // P_ss = -(swept diagonal tile) = Ps
      for (int e = threadIdx.x; e < TT; e += NTH) pel(s, s, e % TS, e / TS) = Ps[e];
    // panel of the group: B_r = C_r P_s, C_r = A[r][s] (tile (r,s) or (s,r)^T); work
    // item it: column half it % 2 of the (it / 2)-th row r != s
    for (int it = w; it < 2 * (g - 1); it += NW) {
      const int rr = it >> 1, hf = it & 1;
      const int r = rr < s ? rr : rr + 1;
      const T* Cr = r > s ? tl(r, s) : tl(s, r);
      const bool tr = r < s;
      typename Mfma<T>::v4 acc[4][2];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = typename Mfma<T>::v4{0, 0, 0, 0};
      const int lk = lane >> 4;
#pragma unroll 4
      for (int k = 0; k < TS; k += 4) {
        T a[4], b[2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * q + li, kk = k + lk;
          if constexpr (kStageC)
            a[q] = Cs[rr * CST + kk * LDC + row];
          else
            a[q] = tr ? Cr[kk + row * TS] : Cr[row + kk * TS];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) b[q] = Ps[(32 * hf + 16 * q + li) + (k + lk) * TS];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mfma<T>::op(a[bi], b[bj], acc[bi][bj]);
      }
      T* Br = Bs + rr * TT;
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            Br[acc_row64<T>(bi, v) + (32 * hf + 16 * bj + li) * TS] = acc[bi][bj][v];
    }
    __syncthreads();
    // update inside the group: A_rq -= B_r C_q^T for r >= q, r, q != s
    {
      int item = 0;
      for (int r = 0; r < g; ++r)
        for (int q = 0; q <= r; ++q) {
          if (r == s || q == s) continue;
          if ((item++ % NW) != w) continue;
          T* A = tl(r, q);
          const T* Cq = q > s ? tl(q, s) : tl(s, q);
          const bool tq = q < s;
          const T* Br = Bs + (r < s ? r : r - 1) * TT;
          typename Mfma<T>::v4 acc[4][4];
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[bi][bj][v] = A[acc_row64<T>(bi, v) + (16 * bj + li) * TS];
          const T* Cqs = Cs + (kStageC ? (q < s ? q : q - 1) * CST : 0);
          wave_gemm64<T>([&](int row, int k) { return -Br[row + k * TS]; },
                         [&](int k, int c) {
                           if constexpr (kStageC) return Cqs[k * LDC + c];
                           else return tq ? Cq[k + c * TS] : Cq[c + k * TS];
                         }, acc);
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int rw = acc_row64<T>(bi, v), cl = 16 * bj + li;
                A[rw + cl * TS] = acc[bi][bj][v];
                if (last) {
                  pel(r, q, rw, cl) = -acc[bi][bj][v];
                  if (r != q) pel(q, r, cl, rw) = -acc[bi][bj][v];
                }
              }
        }
    }
    __syncthreads();
    // row and column s of the group: A[r][s] <- B_r (r > s), A[s][q] <- B_q^T (q < s)
    for (int r = 0; r < g; ++r) {
      if (r == s) continue;
      const T* Br = Bs + (r < s ? r : r - 1) * TT;
      T* A = r > s ? tl(r, s) : tl(s, r);
      if (r > s)
        for (int e = threadIdx.x; e < TT; e += NTH) A[e] = Br[e];
      else
        for (int e = threadIdx.x; e < TT; e += NTH) A[e] = Br[(e / TS) + (e % TS) * TS];
      if (last)                                // P_rs = -B_r, P_sr = -B_r^T
        for (int e = threadIdx.x; e < TT; e += NTH) {
          const int i = e % TS, j = e / TS;
          pel(r, s, i, j) = -Br[e];
          pel(s, r, i, j) = -Br[j + i * TS];
        }
    }
    __syncthreads();
  }
  // P on the padding tiles of a short last group: identity on the diagonal
  for (int t = w; t < G * G; t += NW) {
    const int I = t % G, J = t / G;
    if (I < g && J < g) continue;
#pragma unroll 8
    for (int u = 0; u < TS; ++u) pel(I, J, lane, u) = (I == J && lane == u) ? T(1) : T(0);
  }
  if (fail && threadIdx.x == 0) flags[m] = c0 + 1;
}

// (2) panel: C_i = A_{i,p} (64 x PB), B_i = C_i P, with C_i staged through LDS one
// 64-column chunk at a time (P is symmetric: its columns are read as rows, coalesced)
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_sweep_panel(const T* tiles, const int64_t* tile_off,
                                                        const int32_t* nt_arr, int c0,
                                                        const T* pbuf, T* cbuf, T* bbuf,
                                                        int64_t stride) {
  constexpr int PB = G * TS;
  const int m = blockIdx.y, i = blockIdx.x;
  const int nt = nt_arr[m];
  if (c0 >= nt || i >= nt) return;
  const int g = min(G, nt - c0);
  if (i >= c0 && i < c0 + g) return;
  const T* base = tiles + tile_off[m];
  __shared__ T C[TS * TS];
  T* Cout = cbuf + int64_t(m) * stride + int64_t(i) * TS * PB;
  T* Bout = bbuf + int64_t(m) * stride + int64_t(i) * TS * PB;
  const T* P = pbuf + int64_t(m) * PB * PB;
  typename Mfma<T>::v4 acc[G][2][2];
#pragma unroll
  for (int cb = 0; cb < G; ++cb)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[cb][bi][bj] = typename Mfma<T>::v4{0, 0, 0, 0};
#pragma unroll
  for (int kc = 0; kc < G; ++kc) {
    const int J = c0 + kc;
    for (int e = threadIdx.x; e < TT; e += kBlock) {
      const int r = e % TS, cc = e / TS;
      T v = T(0);
      if (kc < g)
        v = (i > J) ? base[tile_index(i, J) * TT + r + cc * TS]
                    : base[tile_index(J, i) * TT + cc + r * TS];
      C[e] = v;
      Cout[int64_t(kc) * TT + e] = v;
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < G; ++cb)
      mfma_block<T, TS>([&](int r, int k) { return C[r + k * TS]; },
                        [&](int k, int c) { return P[(cb * TS + c) + (kc * TS + k) * PB]; },
                        acc[cb]);
    __syncthreads();
  }
#pragma unroll
  for (int cb = 0; cb < G; ++cb)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int r, c;
          acc_pos<T>(bi, bj, v, &r, &c);
          Bout[r + (cb * TS + c) * TS] = acc[cb][bi][bj][v];
        }
}

// (2') panel for two- and four-tile groups: B_i = C_i P with C_i (64 x PB) and the
// rows of P (= its columns: P is symmetric) streamed through double-buffered LDS in
// k-chunks; wave w owns output columns ob .. ob + NB - 1 (64 x NB, NB / 4 MFMA
// accumulators).  FP32: NB = 64, one workgroup per row tile.  FP64: NB = 32, a workgroup
// per 128 output columns (two per row tile in four-tile groups): its waves then need at
// most 166 registers, so that a workgroup starts in the place of any one finished
// workgroup of a running FP64 update (a 64-column FP64 wave needs 192 and waited for two).
template <typename T>
struct PanelCfg;
template <>
struct PanelCfg<double> { static constexpr int KC = 8, NB = 32; };
template <>
struct PanelCfg<float> { static constexpr int KC = 16, NB = 64; };
// workgroups of k_sweep_panel2 per row tile
template <typename T>
constexpr int panel_wgs(int G) {
  return G * TS > 4 * PanelCfg<T>::NB ? G * TS / (4 * PanelCfg<T>::NB) : 1;
}

template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_sweep_panel2(const T* tiles, const int64_t* tile_off,
                                                         const int32_t* nt_arr, int c0,
                                                         const T* pbuf, T* cbuf, T* bbuf,
                                                         int64_t stride) {
  constexpr int PB = G * TS, KC = PanelCfg<T>::KC, NCH = PB / KC, NB = PanelCfg<T>::NB;
  constexpr int NWG = panel_wgs<T>(G), WC = PB / NWG;  // output columns per workgroup
  constexpr int LDC = TS + 16, LDP = WC + 16;         // padded LDS rows (bank-spread)
  constexpr int NC = KC * TS / kBlock, NP = KC * WC / kBlock;   // loads per thread and chunk
  static_assert(WC <= 4 * NB && WC % NB == 0, "panel columns per workgroup");
  __builtin_amdgcn_s_setprio(3);               // critical path, as the pivot
  const int m = blockIdx.y, i = blockIdx.x / NWG, hb = blockIdx.x % NWG;
  const int nt = nt_arr[m];
  if (c0 >= nt || i >= nt) return;
  const int g = min(G, nt - c0);
  if (i >= c0 && i < c0 + g) return;
  const T* base = tiles + tile_off[m];
  T* Cout = cbuf + int64_t(m) * stride + int64_t(i) * TS * PB;
  T* Bout = bbuf + int64_t(m) * stride + int64_t(i) * TS * PB;
  const T* P = pbuf + int64_t(m) * PB * PB + hb * WC;
  __shared__ T sC[2][KC * LDC], sP[2][KC * LDP];
  T rc[NC], rp[NP];
  auto gload = [&](int ch) {
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const int r = e % TS, kk = e / TS, k = ch * KC + kk;
      const int J = c0 + k / TS, kl = k % TS;
      T v = T(0);
      if (k < g * TS)
        v = (i > J) ? base[tile_index(i, J) * TT + r + kl * TS]
                    : base[tile_index(J, i) * TT + kl + r * TS];
      rc[u] = v;
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const int c = e % WC, kk = e / WC;
      rp[u] = P[c + int64_t(ch * KC + kk) * PB];
    }
  };
  auto sstore = [&](int ch, int buf) {
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int e = threadIdx.x + u * kBlock;
      const int r = e % TS, kk = e / TS;
      sC[buf][kk * LDC + r] = rc[u];
      if (hb == 0) Cout[r + int64_t(ch * KC + kk) * TS] = rc[u];
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = threadIdx.x + u * kBlock;
      sP[buf][(e / WC) * LDP + (e % WC)] = rp[u];
    }
  };
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  constexpr int NJ = NB / 16;                  // accumulator columns per wave
  typename Mfma<T>::v4 acc[4][NJ];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < NJ; ++bj) acc[bi][bj] = typename Mfma<T>::v4{0, 0, 0, 0};
  const bool active = NB * w < WC;
  const int ol = NB * (active ? w : 0);        // the wave's first column in the workgroup's
  const int ob = hb * WC + ol;                 // and in the panel
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int ch = 0; ch < NCH; ++ch) {
    if (ch + 1 < NCH) gload(ch + 1);
    const T* C_ = sC[ch & 1];
    const T* P_ = sP[ch & 1];
    if (active) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        T a[4], b[NJ];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = C_[(kk + lk) * LDC + 16 * q + li];
#pragma unroll
        for (int q = 0; q < NJ; ++q) b[q] = P_[(kk + lk) * LDP + ol + 16 * q + li];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int bj = 0; bj < NJ; ++bj) acc[bi][bj] = Mfma<T>::op(a[bi], b[bj], acc[bi][bj]);
      }
    }
    if (ch + 1 < NCH) sstore(ch + 1, (ch + 1) & 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Bout[acc_row64<T>(bi, v) + int64_t(ob + 16 * bj + li) * TS] = acc[bi][bj][v];
}

// (3) update of every lower tile outside the pivot group
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_sweep_update(T* tiles, const int64_t* tile_off,
                                                         const int32_t* nt_arr, int c0,
                                                         const T* cbuf, const T* bbuf,
                                                         int64_t stride) {
  constexpr int PB = G * TS;
  const int m = blockIdx.y;
  const int nt = nt_arr[m];
  const int64_t t = blockIdx.x;
  if (c0 >= nt || t >= tri(nt)) return;
  int i, j;
  tile_ij(t, &i, &j);
  const int g = min(G, nt - c0);
  const bool in_i = i >= c0 && i < c0 + g, in_j = j >= c0 && j < c0 + g;
  if (in_i && in_j) return;
  T* A = tiles + tile_off[m] + t * TT;
  const T* Bb = bbuf + int64_t(m) * stride;
  const T* Cb = cbuf + int64_t(m) * stride;
  if (in_i) {   // row of the pivot group, j < c0:  A_ij <- (B_j[:, i block])^T
    const T* Bj = Bb + int64_t(j) * TS * PB + int64_t(i - c0) * TS * TS;
    for (int e = threadIdx.x; e < TT; e += kBlock) {
      const int r = e % TS, c = e / TS;
      A[e] = Bj[c + r * TS];
    }
    return;
  }
  if (in_j) {   // column of the pivot group, i >= c0 + g:  A_ij <- B_i[:, j block]
    const T* Bi = Bb + int64_t(i) * TS * PB + int64_t(j - c0) * TS * TS;
    for (int e = threadIdx.x; e < TT; e += kBlock) A[e] = Bi[e];
    return;
  }
  const T* Bi = Bb + int64_t(i) * TS * PB;
  const T* Cj = Cb + int64_t(j) * TS * PB;
  typename Mfma<T>::v4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = typename Mfma<T>::v4{0, 0, 0, 0};
  mfma_block<T, PB>([&](int r, int k) { return Bi[r + k * TS]; },
                    [&](int k, int c) { return Cj[c + k * TS]; }, acc);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r, c;
        acc_pos<T>(bi, bj, v, &r, &c);
        A[r + c * TS] -= acc[bi][bj][v];
      }
}

// (3') the update for two-tile pivot groups, by 128 x 128 super-tiles: a workgroup
// of 4 waves owns super-tile (BI, BJ) (tiles 2BI..2BI+1 x 2BJ..2BJ+1), each wave one
// 64 x 64 tile with 16 MFMA accumulators; the operand panels B_i (128 x 128) and
// C_j (128 x 128) stream through double-buffered, bank-padded LDS in k-chunks.
// Super-tile ids are spread so that each XCD (every 8th workgroup) owns a
// contiguous range, i.e. shares the panels of a few super-rows in its L2.
// KC k-rows per LDS chunk, LD padded k-row length, NS ring stages, minb(G) workgroups per
// compute unit: FP64 in four-tile groups runs three (4-deep chunks, 37 KB of LDS, at most
// 168 registers), the rest two.
template <typename T>
struct Upd2Cfg;
template <>
struct Upd2Cfg<double> {
  static constexpr int KC = 4, LD = 144, NS = 4;
  static constexpr int minb(int g) { return g >= 4 ? 3 : 2; }
};
template <>
struct Upd2Cfg<float> {
  static constexpr int KC = 8, LD = 144, NS = 4;
  static constexpr int minb(int) { return 2; }
};

// s_waitcnt for vmcnt <= N (expcnt and lgkmcnt unconstrained; gfx9 field layout)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}
// wait for the oldest chunk of an LDS ring with `younger` chunks (PERW loads per wave
// each) issued after it
template <int PERW, int NS>
__device__ __forceinline__ void wait_ring(int younger) {
  if constexpr (NS >= 4) {
    if (younger >= 2) {
      wait_vmcnt<2 * PERW>();
      return;
    }
  }
  if constexpr (NS >= 3) {
    if (younger >= 1) {
      wait_vmcnt<PERW>();
      return;
    }
  }
  wait_vmcnt<0>();
}

template <typename T, int G>
__global__ __launch_bounds__(kBlock, Upd2Cfg<T>::minb(G)) void k_sweep_update2(T* tiles, const int64_t* tile_off,
                                                          const int32_t* nt_arr, int c0,
                                                          const T* cbuf, const T* bbuf,
                                                          int64_t stride, int64_t per_xcd,
                                                          int part, int count) {
  constexpr int PB = G * TS, KC = Upd2Cfg<T>::KC, LD = Upd2Cfg<T>::LD, NS = Upd2Cfg<T>::NS;
  constexpr int NCH = PB / KC;
  constexpr int GS = G / 2;                    // super-rows per pivot group
  // Workgroups are dealt to the 8 XCDs round-robin by linear id.  With 8 or more
  // matrices (part 0 or 2, 1-D grid) each XCD takes whole matrices, one after the
  // other: matrix 8 q + x on XCD x, its super-tiles at slots s < per_xcd.  Otherwise
  // (grid y = matrix) XCD x takes the contiguous slot range [x, x + 1) * per_xcd.
  int m;
  int64_t s = 0;
  if (part != 1 && count >= 8) {
    const int64_t q = blockIdx.x / 8;
    m = int(8 * (q / per_xcd)) + int(blockIdx.x % 8);
    s = q % per_xcd;
    if (m >= count) return;
  } else {
    m = blockIdx.y;
    s = int64_t(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  }
  const int nt = nt_arr[m];
  if (c0 >= nt) return;
  const int nsb = (nt + 1) / 2;
  const int gN = c0 / 2 + GS;                  // first super index of the next pivot group
  auto in_next = [&](int X) { return X >= gN && X < gN + GS; };
  int BI, BJ;
  if (part == 1) {                             // only the next group's rows and columns
    const int t = blockIdx.x / GS, sub = blockIdx.x % GS;
    const int gx = gN + sub;
    if (t >= nsb || gx >= nsb) return;
    BI = t <= gx ? gx : t;
    BJ = t <= gx ? t : gx;
    if (t < gx && t >= gN) return;             // (gx, t), t an earlier super of the group:
                                               // handled as (t', gx) by its own sub-row
  } else {
    if (s >= tri(nsb)) return;
    band_ij(s, nsb, &BI, &BJ);
    if (part == 2 && (in_next(BI) || in_next(BJ))) return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = 2 * BI + (w >> 1), tj = 2 * BJ + (w & 1);
  const bool valid = ti < nt && tj <= ti;
  const T* Bb = bbuf + int64_t(m) * stride;
  const T* Cb = cbuf + int64_t(m) * stride;
  T* base = tiles + tile_off[m];
  const int gB = c0 / 2;
  auto in_cur = [&](int X) { return X >= gB && X < gB + GS; };
  if (in_cur(BI) || in_cur(BJ)) {
    const bool ii = ti >= c0 && ti < c0 + G, jj = tj >= c0 && tj < c0 + G;
    if (ii && jj) return;                      // pivot tiles: written by the pivot kernel
    if (!valid) return;
    T* A = base + tile_index(ti, tj) * TT;
    if (ii) {                                  // pivot-group row: A_ij <- (B_j[:, i block])^T
      const T* Bj = Bb + int64_t(tj) * TS * PB + int64_t(ti - c0) * TS * TS;
      for (int e = lane; e < TT; e += 64) A[e] = Bj[(e / TS) + (e % TS) * TS];
    } else {                                   // pivot-group column: A_ij <- B_i[:, j block]
      const T* Bi = Bb + int64_t(ti) * TS * PB + int64_t(tj - c0) * TS * TS;
      for (int e = lane; e < TT; e += 64) A[e] = Bi[e];
    }
    return;
  }
  // Panels B_i, C_j stream straight from global memory into an NS-stage LDS ring
  // (global_load_lds: each wave instruction fills one padded k-row; FP64 16 bytes per
  // lane for all 128 rows, FP32 4 bytes per lane for one tile's 64 rows), so NS - 1
  // chunks are in flight while one is multiplied, with one barrier per chunk.
  constexpr int IPR = sizeof(T) == 8 ? 1 : 2;  // load instructions per k-row and panel
  constexpr int PERW = 2 * KC * IPR / 4;       // load instructions per wave and chunk
  __shared__ __attribute__((aligned(16))) T ring[NS][2][KC * LD];
  auto issue = [&](int ch) {
    const int st = ch % NS;
#pragma unroll
    for (int u = 0; u < KC * IPR / 4; ++u) {
      const int idx = w + 4 * u, kk = idx / IPR, hf = idx % IPR, k = ch * KC + kk;
      const int r = sizeof(T) == 8 ? 2 * lane : 64 * hf + lane;   // first row of the lane
      // a row block past the matrix reads its super-row's first tile (finite data that
      // only reaches accumulators of tiles that are never stored)
      const int iA = 2 * BI + r / 64 < nt ? 2 * BI + r / 64 : 2 * BI;
      const int iB = 2 * BJ + r / 64 < nt ? 2 * BJ + r / 64 : 2 * BJ;
      const int lo = sizeof(T) == 8 ? 0 : 64 * hf;
      const void* ga = Bb + int64_t(iA) * TS * PB + (r % 64) + int64_t(k) * TS;
      const void* gb = Cb + int64_t(iB) * TS * PB + (r % 64) + int64_t(k) * TS;
      auto la = (__attribute__((address_space(3))) void*)&ring[st][0][kk * LD + lo];
      auto lb = (__attribute__((address_space(3))) void*)&ring[st][1][kk * LD + lo];
      if constexpr (sizeof(T) == 8) {
        __builtin_amdgcn_global_load_lds(ga, la, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(gb, lb, 16, 0, 0);
      } else {
        __builtin_amdgcn_global_load_lds(ga, la, 4, 0, 0);
        __builtin_amdgcn_global_load_lds(gb, lb, 4, 0, 0);
      }
    }
  };
  // the accumulators start from A_ij (the MFMA's C operand), with the panel of B_i
  // negated: D = A_ij - B_i C_j^T.  The MFMA computes the transposed product (the C_j
  // operand first), so a lane's accumulator holds 16 consecutive rows of a column:
  // the old tile is read, and the new one written, in whole cache lines.
  const int li = lane & 15, lk = lane >> 4, g = lane >> 4;
  T* At = base + tile_index(valid ? ti : 0, valid ? tj : 0) * TT;
  auto acc_col = [&](int bj, int v) { return 16 * bj + ((sizeof(T) == 8) ? 4 * v + g : 4 * g + v); };
  typename Mfma<T>::v4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc[bi][bj][v] = valid ? At[(16 * bi + li) + acc_col(bj, v) * TS] : T(0);
  const int oa = 64 * (w >> 1) + li, ob = 64 * (w & 1) + li;
#pragma unroll
  for (int c = 0; c < NS - 1; ++c)
    if (c < NCH) issue(c);
  for (int ch = 0; ch < NCH; ++ch) {
    // chunk ch has landed once at most the younger chunks' loads are outstanding
    wait_ring<PERW, NS>(min(NS - 2, NCH - 1 - ch));
    __syncthreads();
    if (ch + NS - 1 < NCH) issue(ch + NS - 1);   // into the stage freed by chunk ch - 1
    const T* A_ = ring[ch % NS][0];
    const T* B_ = ring[ch % NS][1];
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = -A_[(kk + lk) * LD + oa + 16 * q];
        b[q] = B_[(kk + lk) * LD + ob + 16 * q];
      }
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = Mfma<T>::op(b[bj], a[bi], acc[bi][bj]);
    }
  }
  if (!valid) return;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) At[(16 * bi + li) + acc_col(bj, v) * TS] = acc[bi][bj][v];
}

// (3f) the look-ahead part of a step (the next group's tile rows and columns) for batches
// of few matrices, whose 128 x 128 super-tiles leave most compute units idle while the
// part runs alone on the critical path: one workgroup per 64 x 64 tile, each wave a
// 32 x 32 quadrant.  Every tile element receives the MFMA products of k_sweep_update2 in
// the same order (same instruction, operands and k-steps), so the results are the same
// bits.  The operand rows of the tile pair stream through a double-buffered LDS area,
// staged in registers two chunks ahead.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_sweep_update_la(T* tiles, const int64_t* tile_off,
                                                         const int32_t* nt_arr, int c0,
                                                         const T* cbuf, const T* bbuf,
                                                         int64_t stride) {
  constexpr int PB = G * TS, KC = 16, NCH = PB / KC;
  constexpr int LDF = TS + 16;                 // padded k-row (conflict-free 8-byte reads)
  const int m = blockIdx.y, t = blockIdx.x / G, x = c0 + G + int(blockIdx.x % G);
  const int nt = nt_arr[m];
  if (x >= nt || t >= nt) return;
  if (t >= c0 + G && t < c0 + 2 * G && t > x) return;   // counted as (t, x)
  T* base = tiles + tile_off[m];
  const T* Bb = bbuf + int64_t(m) * stride;
  const T* Cb = cbuf + int64_t(m) * stride;
  if (t >= c0 && t < c0 + G) {                 // pivot-group column: A_xt <- B_x[:, t block]
    T* A = base + tile_index(x, t) * TT;
    const T* Bx = Bb + int64_t(x) * TS * PB + int64_t(t - c0) * TS * TS;
    for (int e = threadIdx.x; e < TT; e += kBlock) A[e] = Bx[e];
    return;
  }
  const int I = x > t ? x : t, J = x > t ? t : x;
  T* A = base + tile_index(I, J) * TT;
  const T* gB = Bb + int64_t(I) * TS * PB;     // rows of B_I, k-major
  const T* gC = Cb + int64_t(J) * TS * PB;     // rows of C_J
  __shared__ T sB[2][KC * LDF], sC[2][KC * LDF];
  const int r = threadIdx.x % TS, kq = threadIdx.x / TS;
  T rb[2][KC / 4], rc[2][KC / 4];              // two chunks in flight: [chunk % 2]
  auto gload = [&](int ch, T (&pb)[KC / 4], T (&pc)[KC / 4]) {
#pragma unroll
    for (int u = 0; u < KC / 4; ++u) {
      const int k = ch * KC + kq + 4 * u;
      pb[u] = gB[r + int64_t(k) * TS];
      pc[u] = gC[r + int64_t(k) * TS];
    }
  };
  auto sstore = [&](int buf, const T (&pb)[KC / 4], const T (&pc)[KC / 4]) {
#pragma unroll
    for (int u = 0; u < KC / 4; ++u) {
      sB[buf][(kq + 4 * u) * LDF + r] = pb[u];
      sC[buf][(kq + 4 * u) * LDF + r] = pc[u];
    }
  };
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int qr = 32 * (w >> 1), qc = 32 * (w & 1);
  auto acc_col = [&](int bj, int v) { return 16 * bj + ((sizeof(T) == 8) ? 4 * v + g : 4 * g + v); };
  typename Mfma<T>::v4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[bi][bj][v] = A[(qr + 16 * bi + li) + (qc + acc_col(bj, v)) * TS];
  static_assert(NCH % 2 == 0 && NCH >= 2, "chunks are taken in pairs");
  gload(0, rb[0], rc[0]);
  gload(1, rb[1], rc[1]);
  sstore(0, rb[0], rc[0]);
  __syncthreads();
  // chunk ch is in LDS buffer ch % 2 and chunk ch + 1 in registers p (set ch % 2 ^ 1);
  // the registers of chunk ch (set ch % 2) take chunk ch + 2
  auto step = [&](int ch, T (&pb)[KC / 4], T (&pc)[KC / 4], T (&nb)[KC / 4], T (&nc)[KC / 4]) {
    if (ch + 2 < NCH) gload(ch + 2, pb, pc);
    const T* B_ = sB[ch & 1];
    const T* C_ = sC[ch & 1];
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T a[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        a[q] = -B_[(kk + g) * LDF + qr + 16 * q + li];
        b[q] = C_[(kk + g) * LDF + qc + 16 * q + li];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mfma<T>::op(b[bj], a[bi], acc[bi][bj]);
    }
    if (ch + 1 < NCH) sstore((ch + 1) & 1, nb, nc);
    __syncthreads();
  };
  for (int ch = 0; ch < NCH; ch += 2) {
    step(ch, rb[0], rc[0], rb[1], rc[1]);
    step(ch + 1, rb[1], rc[1], rb[0], rc[0]);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(qr + 16 * bi + li) + (qc + acc_col(bj, v)) * TS] = acc[bi][bj][v];
}

// (3'') the update of an FP32 batch on the BF16 matrix cores.  Same super-tiles, XCD
// dealing, band order and look-ahead parts as k_sweep_update2<float>, 32-deep k-chunks.
// Each operand value x is split exactly into three BF16 parts (split_bf3; BF16 has FP32's
// exponent range, so no scaling is needed), and each 16 x 16 x 32 block takes six MFMAs,
// hi hi + hi mid + mid hi + hi lo + mid mid + lo hi, accumulated in FP32 from A_ij; the
// three dropped products (mid lo, lo mid, lo lo) are below 2^-21 of |x y|.  Lane group lk
// of an MFMA operand holds the k-values lk, lk + 4, ..., lk + 28 of the chunk (the same
// permutation of k for both operands leaves the sum unchanged).
using bf8 = __bf16 __attribute__((ext_vector_type(8)));
using f4v = float __attribute__((ext_vector_type(4)));

// x = hi + mid + lo exactly: hi and mid keep the upper 16 bits of x and of r = x - hi
// (both subtractions are exact); r - mid has at most 8 significant bits, a BF16 value
__device__ __forceinline__ void split_bf3(const float (&x)[8], bf8& h, bf8& m, bf8& l) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float a = __uint_as_float(__float_as_uint(x[e]) & 0xffff0000u);
    const float r = x[e] - a;
    const float b = __uint_as_float(__float_as_uint(r) & 0xffff0000u);
    h[e] = __builtin_bit_cast(__bf16, uint16_t(__float_as_uint(a) >> 16));
    m[e] = __builtin_bit_cast(__bf16, uint16_t(__float_as_uint(b) >> 16));
    l[e] = __builtin_bit_cast(__bf16, uint16_t(__float_as_uint(r - b) >> 16));
  }
}

// (3w) the BF16-split update of an FP32 batch for four-tile pivot groups by 256 x 256
// super-tiles: eight waves, wave w owning tile row 4 BI + w / 2 and the two tiles
// 4 BJ + 2 (w % 2) + {0, 1} of it (a 64 x 128 block, 32 accumulators).  Twice the work per
// operand byte of the 128 x 128 form: the panels of four tile rows (256 rows) stream
// through a two-stage LDS ring, one 16-byte direct load per lane filling a whole k-row
// (four tile rows' 64-row segments side by side).  Per 32-deep chunk a wave splits its
// four B row blocks once and each C row block once (split_bf3), and issues 192 MFMAs in
// groups of four independent accumulators.  Pivot group = one super-row (G = 4).
template <int NS>
__global__ __launch_bounds__(512, 1) void k_sweep_update_bf3w(float* tiles, const int64_t* tile_off,
                                                           const int32_t* nt_arr, int c0,
                                                           const float* cbuf, const float* bbuf,
                                                           int64_t stride, int64_t per_xcd,
                                                           int part, int count) {
  constexpr int G = 4, PB = G * TS, KC = 32, LD = 4 * TS + 16, NCH = PB / KC;
  int m;
  int64_t s = 0;
  if (part != 1 && count >= 8) {
    const int64_t q = blockIdx.x / 8;
    m = int(8 * (q / per_xcd)) + int(blockIdx.x % 8);
    s = q % per_xcd;
    if (m >= count) return;
  } else {
    m = blockIdx.y;
    s = int64_t(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  }
  const int nt = nt_arr[m];
  if (c0 >= nt) return;
  const int nsb = (nt + 3) / 4;
  const int gB = c0 / 4, gN = gB + 1;          // super-rows of this and the next pivot group
  int BI, BJ;
  if (part == 1) {                             // only the next group's super-row and column
    const int t = blockIdx.x;
    if (t >= nsb || gN >= nsb) return;
    BI = t <= gN ? gN : t;
    BJ = t <= gN ? t : gN;
  } else {
    if (s >= tri(nsb)) return;
    band_ij(s, nsb, &BI, &BJ);
    if (part == 2 && (BI == gN || BJ == gN)) return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = 4 * BI + (w >> 1), tj0 = 4 * BJ + 2 * (w & 1);
  const float* Bb = bbuf + int64_t(m) * stride;
  const float* Cb = cbuf + int64_t(m) * stride;
  float* base = tiles + tile_off[m];
  if (BI == gB || BJ == gB) {                  // the pivot group's tile rows and columns
    if (BI == gB && BJ == gB) return;          // pivot tiles: written by the pivot kernel
    for (int h = 0; h < 2; ++h) {
      const int tj = tj0 + h;
      if (!(ti < nt && tj <= ti)) continue;
      float* A = base + tile_index(ti, tj) * TT;
      if (BI == gB) {                          // row of the group: A_ij <- (B_j[:, i block])^T
        const float* Bj = Bb + int64_t(tj) * TS * PB + int64_t(ti - c0) * TS * TS;
        for (int e = lane; e < TT; e += 64) A[e] = Bj[(e / TS) + (e % TS) * TS];
      } else {                                 // column of the group: A_ij <- B_i[:, j block]
        const float* Bi = Bb + int64_t(ti) * TS * PB + int64_t(tj - c0) * TS * TS;
        for (int e = lane; e < TT; e += 64) A[e] = Bi[e];
      }
    }
    return;
  }
  // ring: [stage][panel][k-row * LD + row], 256 rows of a k-row filled by one wave load
  // (lane l: four consecutive rows of tile row 4 X + l / 16); a tile row past the matrix
  // reads the super-row's first tile (finite data reaching only tiles never stored)
  constexpr int PERW = 2 * KC / 8;             // load instructions per wave and chunk
  __shared__ __attribute__((aligned(16))) float ring[NS][2][KC * LD];
  const int lq = lane >> 4, lr = 4 * (lane & 15);
  const int iA = 4 * BI + lq < nt ? 4 * BI + lq : 4 * BI;
  const int iB = 4 * BJ + lq < nt ? 4 * BJ + lq : 4 * BJ;
  const float* gA = Bb + int64_t(iA) * TS * PB + lr;
  const float* gC = Cb + int64_t(iB) * TS * PB + lr;
  auto issue = [&](int ch) {
    const int st = ch % NS;
#pragma unroll
    for (int u = 0; u < PERW; ++u) {
      const int idx = w + 8 * u, kk = idx >> 1, pp = idx & 1, k = ch * KC + kk;
      const void* gp = (pp == 0 ? gA : gC) + int64_t(k) * TS;
      auto l = (__attribute__((address_space(3))) void*)&ring[st][pp][kk * LD];
      __builtin_amdgcn_global_load_lds(gp, l, 16, 0, 0);
    }
  };
  const int li = lane & 15, lk = lane >> 4, g = lane >> 4;
  bool valid[2];
  float* At[2];
  f4v acc[2][4][4];                            // [tile][bi][bj]
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    valid[h] = ti < nt && tj0 + h <= ti;
    At[h] = base + tile_index(valid[h] ? ti : 0, valid[h] ? tj0 + h : 0) * TT;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[h][bi][bj][v] =
              valid[h] ? At[h][(16 * bi + li) + (16 * bj + 4 * g + v) * TS] : 0.0f;
  }
  const int oa = 64 * (w >> 1) + li, ob = 128 * (w & 1) + li;
#pragma unroll
  for (int c = 0; c < NS - 1; ++c)
    if (c < NCH) issue(c);
  for (int ch = 0; ch < NCH; ++ch) {
    wait_ring<PERW, NS>(min(NS - 2, NCH - 1 - ch));
    __syncthreads();
    if (ch + NS - 1 < NCH) issue(ch + NS - 1);
    const float* A_ = ring[ch % NS][0];
    const float* B_ = ring[ch % NS][1];
    bf8 bh[4], bm[4], bl[4];                   // the wave's B_i row blocks (negated)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = -A_[(lk + 4 * e) * LD + oa + 16 * q];
      split_bf3(x, bh[q], bm[q], bl[q]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) {         // C row block bj of tile h
        bf8 chh, cmm, cll;
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = B_[(lk + 4 * e) * LD + ob + 64 * h + 16 * bj];
        split_bf3(x, chh, cmm, cll);
#define RSD_BF3W_TERM(CA, BB)                                                                   \
  _Pragma("unroll") for (int q = 0; q < 4; ++q)                                                 \
      acc[h][q][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(CA, BB[q], acc[h][q][bj], 0, 0, 0);
        RSD_BF3W_TERM(cll, bh)
        RSD_BF3W_TERM(cmm, bm)
        RSD_BF3W_TERM(chh, bl)
        RSD_BF3W_TERM(cmm, bh)
        RSD_BF3W_TERM(chh, bm)
        RSD_BF3W_TERM(chh, bh)
#undef RSD_BF3W_TERM
      }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!valid[h]) continue;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          At[h][(16 * bi + li) + (16 * bj + 4 * g + v) * TS] = acc[h][bi][bj][v];
  }
}

// (3s) the BF16-split update by 128 x 128 super-tiles, each operand value split once per
// workgroup (its four waves read every panel row twice; splitting where the values are
// read cost three times the vector instructions and ran 25% slower).  Per 32-deep chunk
// each thread loads eight k-values of one panel row (value e of k-group q is k = q + 4 e)
// into registers, one chunk ahead;
// after the previous chunk's products the workgroup splits them and writes the three
// BF16 parts straight into the MFMA operand layout in LDS ([panel][part][row block]
// [k-group][row] of 16-byte fragments), so each MFMA operand is one conflict-free 16-byte
// LDS read.  48 KB of LDS, one stage; three workgroups per compute unit in four-tile
// groups (168 registers: the LDS stores and operand reads are constant offsets from one
// base address each), two in two-tile groups.
template <int G>
__global__ __launch_bounds__(kBlock, G >= 4 ? 3 : 2) void k_sweep_update_bf3s(float* tiles, const int64_t* tile_off,
                                                              const int32_t* nt_arr, int c0,
                                                              const float* cbuf, const float* bbuf,
                                                              int64_t stride, int64_t per_xcd,
                                                              int part, int count) {
  constexpr int PB = G * TS, KC = 32, NCH = PB / KC;
  constexpr int GS = G / 2;
  int m;
  int64_t s = 0;
  if (part != 1 && count >= 8) {
    const int64_t q = blockIdx.x / 8;
    m = int(8 * (q / per_xcd)) + int(blockIdx.x % 8);
    s = q % per_xcd;
    if (m >= count) return;
  } else {
    m = blockIdx.y;
    s = int64_t(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  }
  const int nt = nt_arr[m];
  if (c0 >= nt) return;
  const int nsb = (nt + 1) / 2;
  const int gN = c0 / 2 + GS;
  auto in_next = [&](int X) { return X >= gN && X < gN + GS; };
  int BI, BJ;
  if (part == 1) {
    const int t = blockIdx.x / GS, sub = blockIdx.x % GS;
    const int gx = gN + sub;
    if (t >= nsb || gx >= nsb) return;
    BI = t <= gx ? gx : t;
    BJ = t <= gx ? t : gx;
    if (t < gx && t >= gN) return;
  } else {
    if (s >= tri(nsb)) return;
    band_ij(s, nsb, &BI, &BJ);
    if (part == 2 && (in_next(BI) || in_next(BJ))) return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = 2 * BI + (w >> 1), tj = 2 * BJ + (w & 1);
  const bool valid = ti < nt && tj <= ti;
  const float* Bb = bbuf + int64_t(m) * stride;
  const float* Cb = cbuf + int64_t(m) * stride;
  float* base = tiles + tile_off[m];
  const int gB = c0 / 2;
  auto in_cur = [&](int X) { return X >= gB && X < gB + GS; };
  if (in_cur(BI) || in_cur(BJ)) {
    const bool ii = ti >= c0 && ti < c0 + G, jj = tj >= c0 && tj < c0 + G;
    if (ii && jj) return;
    if (!valid) return;
    float* A = base + tile_index(ti, tj) * TT;
    if (ii) {
      const float* Bj = Bb + int64_t(tj) * TS * PB + int64_t(ti - c0) * TS * TS;
      for (int e = lane; e < TT; e += 64) A[e] = Bj[(e / TS) + (e % TS) * TS];
    } else {
      const float* Bi = Bb + int64_t(ti) * TS * PB + int64_t(tj - c0) * TS * TS;
      for (int e = lane; e < TT; e += 64) A[e] = Bi[e];
    }
    return;
  }
  // this thread's panel row r (the same for both panels) and k-groups kq, kq + 2; a tile
  // row past the matrix reads the super-row's first tile (finite data reaching only tiles
  // never stored)
  const int r = threadIdx.x & 127, kq = threadIdx.x >> 7;
  const int iA = 2 * BI + r / 64 < nt ? 2 * BI + r / 64 : 2 * BI;
  const int iB = 2 * BJ + r / 64 < nt ? 2 * BJ + r / 64 : 2 * BJ;
  const float* gp[2] = {Bb + int64_t(iA) * TS * PB + (r % 64),
                        Cb + int64_t(iB) * TS * PB + (r % 64)};
  float pre[4][8];                             // [panel * 2 + k-group half][e]
  auto load = [&](int ch) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        pre[u][e] = gp[u >> 1][int64_t(ch * KC + kq + 2 * (u & 1) + 4 * e) * TS];
  };
  // operand fragments: [panel][part][row block][k-group][row in block]
  __shared__ bf8 frag[2 * 3 * 8 * 4 * 16];
  auto fidx = [](int pp, int pt, int rb, int q, int ri) {
    return (((pp * 3 + pt) * 8 + rb) * 4 + q) * 16 + ri;
  };
  const int li = lane & 15, lk = lane >> 4, g = lane >> 4;
  float* At = base + tile_index(valid ? ti : 0, valid ? tj : 0) * TT;
  f4v acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc[bi][bj][v] = valid ? At[(16 * bi + li) + (16 * bj + 4 * g + v) * TS] : 0.0f;
  const int ra = 4 * (w >> 1), rbb = 4 * (w & 1);   // the wave's first row block per panel
  // one base address for this thread's fragment stores and one for the wave's operand
  // reads; every other position is a constant offset from them
  bf8* const fw = frag + fidx(0, 0, r >> 4, kq, r & 15);
  const bf8* const fa = frag + fidx(0, 0, ra, lk, li);
  load(0);
  for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (u >> 1) == 0 ? -pre[u][e] : pre[u][e];
      bf8 h, md, lo;
      split_bf3(x, h, md, lo);
      const int pp = u >> 1, dq = 2 * (u & 1);
      fw[fidx(pp, 0, 0, dq, 0)] = h;
      fw[fidx(pp, 1, 0, dq, 0)] = md;
      fw[fidx(pp, 2, 0, dq, 0)] = lo;
    }
    __syncthreads();
    if (ch + 1 < NCH) load(ch + 1);
    bf8 bh[4], bm[4], bl[4];                   // the wave's B_i row blocks (negated)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bh[q] = fa[fidx(0, 0, q, 0, 0)];
      bm[q] = fa[fidx(0, 1, q, 0, 0)];
      bl[q] = fa[fidx(0, 2, q, 0, 0)];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {              // C row block j
      const bf8 chh = fa[fidx(1, 0, rbb - ra + j, 0, 0)];
      const bf8 cmm = fa[fidx(1, 1, rbb - ra + j, 0, 0)];
      const bf8 cll = fa[fidx(1, 2, rbb - ra + j, 0, 0)];
#define RSD_BF3S_TERM(CA, BB)                                                                   \
  _Pragma("unroll") for (int q = 0; q < 4; ++q)                                                 \
      acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(CA, BB[q], acc[q][j], 0, 0, 0);
      RSD_BF3S_TERM(cll, bh)
      RSD_BF3S_TERM(cmm, bm)
      RSD_BF3S_TERM(chh, bl)
      RSD_BF3S_TERM(cmm, bh)
      RSD_BF3S_TERM(chh, bm)
      RSD_BF3S_TERM(chh, bh)
#undef RSD_BF3S_TERM
    }
    __syncthreads();
  }
  if (!valid) return;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) At[(16 * bi + li) + (16 * bj + 4 * g + v) * TS] = acc[bi][bj][v];
}

// ---- symmetric products y = base + alpha A x -------------------------------------------
// Work item = a kSymB x kSymB block of tiles (block row BI, block column BJ <= BI) of
// one matrix.  Phase 1 streams the block's lower tiles once, row by row of tiles.  The
// row part sum_J A_IJ x_J of tile row I (the full diagonal tile included) is folded
// across the wave and parked in LDS when its row is done.  The column parts
// sum_{I > J} A_IJ^T x_I of the block's tile columns either stay in registers until
// the end of the item (FP32 tiles), or (FP64 tiles, whose 16-byte loads hold half as
// many entries) are folded across the row lanes after every tile and added into LDS
// by the one lane that owns the column, which frees the registers for four vectors
// per pass.  P = float for FP32 factors, as accurate as the factor.
// Phase 2 adds, for every tile row, the row parts of its block row and the column parts
// of its block column, in a fixed order.  No atomics: results are reproducible.  With
// several vectors (KV per launch, x_k = x + k ld) the tiles are read once for all of
// them; each vector's sums have the same order whatever KV is.
template <int N, typename P>
__device__ __forceinline__ void xor_fold(P* a, int lane, int o) {
  // trade half of a[0..N) with the lane `lane ^ o`; the lane with bit o set keeps the
  // upper half, so after folds over bits b1 > b2 > ... a lane holds the block of
  // entries selected by its own bits (N is a constant so that a[] stays in registers)
  const bool up = (lane & o) != 0;
#pragma unroll
  for (int j = 0; j < N / 2; ++j) {
    const P give = up ? a[j] : a[j + N / 2];
    const P keep = up ? a[j + N / 2] : a[j];
    a[j] = keep + __shfl_xor(give, o, 64);
  }
}

// PERSIST: a persistent work-queue form of the same kernel for uneven batches.  A grid
// of about one resident workgroup per slot takes items from a counter (queue[0]) until
// the items run out; the last workgroup to finish (queue[1] counts them) resets both
// counters for the next launch.  Every item writes its own partial sums, so the results
// do not depend on which workgroup computed an item.
template <typename T, int KV, bool PERSIST = false>
__global__ __launch_bounds__(kBlock) void k_symv1(
    const T* __restrict__ tiles, const int64_t* __restrict__ tile_off,
    const int32_t* __restrict__ n_arr, const int32_t* __restrict__ nt_arr,
    const int64_t* __restrict__ vec_off, const int32_t* __restrict__ item_mat,
    const int32_t* __restrict__ item_BI, const int32_t* __restrict__ item_BJ,
    const double* __restrict__ x, int64_t ldx, int nv,
    typename SymPart<T>::type* __restrict__ part, int32_t* __restrict__ queue,
    int64_t num_items, const int32_t* __restrict__ row0) {
  using P = typename SymPart<T>::type;
  constexpr int B = kSymB;
  // elements per load: 16-byte loads of FP64 / FP32, 8-byte loads of 16-bit values
  constexpr int VEC = sizeof(T) == 8 ? 2 : 4;
  constexpr int LPC = 4 / VEC;                 // loads per column (four rows per thread)
  typedef T V __attribute__((ext_vector_type(VEC)));
  constexpr bool kColLds = sizeof(T) == 8;
  __shared__ P xs[KV][2][B][TS];               // x in the product's precision
  __shared__ P red[KV][4][B][TS];
  __shared__ P colr[kColLds ? KV : 1][B][TS];
  __shared__ int s_item;
  for (int round = 0;; ++round) {
    int it;
    if constexpr (PERSIST) {
      if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
      __syncthreads();
      it = s_item;
      if (int64_t(it) >= num_items) break;       // the same for the whole workgroup
    } else {
      if (round > 0) break;
      it = blockIdx.x;
    }
    const int m = item_mat[it], BI = item_BI[it], BJ = item_BJ[it];
    const int n = n_arr[m], nt = nt_arr[m];
    const int r0 = row0 ? row0[m] : 0;         // tile rows below r0 meet only zeros of x
    if ((BI + 1) * B <= r0) {                  // the whole item: no partial sums (k_symv2
      if constexpr (PERSIST) {                 // skips them), next item
        __syncthreads();                       // (s_item read by every thread)
        continue;
      } else {
        return;
      }
    }
    const int64_t xo = vec_off[m];
    // thread t: rows q4(v) of the tile (q = t % 16), columns g + 16 u (g = t / 16, u < 4);
    // FP32 and 16-bit: rows 4q .. 4q + 3 (one load per column); FP64: rows 2q, 2q + 1,
    // 32 + 2q, 33 + 2q (two loads per column, each contiguous over 16 lanes)
    const int t = threadIdx.x, q = t & 15, g = t >> 4, w = t >> 6, lane = t & 63;
    auto q4 = [&](int v) { return sizeof(T) <= 4 ? 4 * q + v : (v < 2 ? 2 * q + v : 30 + 2 * q + v); };
    for (int e = t; e < KV * 2 * B * TS; e += kBlock) {
      const int k = e / (2 * B * TS), sd = (e / (B * TS)) % 2, b = (e / TS) % B, r = e % TS;
      const int idx = ((sd == 0 ? BI : BJ) * B + b) * TS + r;
      xs[k][sd][b][r] = P(idx < n && k < nv ? x[k * ldx + xo + idx] : 0.0);
    }
    if (kColLds)
      for (int e = t; e < KV * B * TS; e += kBlock) (&colr[0][0][0])[e] = P(0);
    __syncthreads();
    P cacc[kColLds ? 1 : KV][B * 4];             // [vector][block column b][column u]
    #pragma unroll
    for (int k = 0; k < (kColLds ? 1 : KV); ++k)
      #pragma unroll
      for (int i = 0; i < B * 4; ++i) cacc[k][i] = P(0);
    const int usel = (q >> 2) & 3;               // LDS columns: column g + 16 usel after the fold
    const T* base = tiles + tile_off[m] + q4(0) + g * TS;
    #pragma unroll
    for (int bi = 0; bi < B; ++bi) {
      const int I = BI * B + bi;
      P ra[KV][4];                               // row part of tile row I, rows q4(v)
      #pragma unroll
      for (int k = 0; k < KV; ++k)
        #pragma unroll
        for (int v = 0; v < 4; ++v) ra[k][v] = P(0);
      if (I < nt && I >= r0) {
        // x_I: in registers for FP32 tiles, read from LDS at each use for FP64 tiles
        P xi[kColLds ? 1 : KV][4];
        if constexpr (!kColLds)
          #pragma unroll
          for (int k = 0; k < KV; ++k)
            #pragma unroll
            for (int v = 0; v < 4; ++v) xi[k][v] = xs[k][0][bi][q4(v)];
        #pragma unroll
        for (int bj = 0; bj < B; ++bj) {
          const int J = BJ * B + bj;
          if (J > I) break;
          const T* tl = base + tile_index(I, J) * TT;
          V a[4][LPC];
          #pragma unroll
          for (int u = 0; u < 4; ++u)
            #pragma unroll
            for (int h = 0; h < LPC; ++h) a[u][h] = ld_stream((const V*)(tl + 16 * u * TS + 32 * h));
          P cf[KV][4];                           // column parts of this tile, columns g + 16 u
          #pragma unroll
          for (int u = 0; u < 4; ++u) {
            P xk[KV];
            #pragma unroll
            for (int k = 0; k < KV; ++k) {
              xk[k] = xs[k][1][bj][g + 16 * u];
              cf[k][u] = P(0);
            }
            #pragma unroll
            for (int v = 0; v < 4; ++v) {
              const P av = P(a[u][v / VEC][v % VEC]);
              #pragma unroll
              for (int k = 0; k < KV; ++k) {
                const P xv = kColLds ? xs[k][0][bi][q4(v)] : xi[kColLds ? 0 : k][v];
                cf[k][u] = fma(av, xv, cf[k][u]);
                ra[k][v] = fma(av, xk[k], ra[k][v]);
              }
            }
            if (!kColLds && J < I)
              #pragma unroll
              for (int k = 0; k < KV; ++k) cacc[kColLds ? 0 : k][bj * 4 + u] += cf[k][u];
          }
          if (J < I) {
            if constexpr (kColLds) {
              // fold over the 16 row lanes (bits 3..0): lanes q with q % 4 == 0 then hold
              // column g + 16 usel of this tile, which only they update
              #pragma unroll
              for (int k = 0; k < KV; ++k) {
                xor_fold<4>(cf[k], lane, 8);
                xor_fold<2>(cf[k], lane, 4);
                P c = cf[k][0];
                c += __shfl_xor(c, 2, 64);
                c += __shfl_xor(c, 1, 64);
                if ((q & 3) == 0) colr[k][bj][g + 16 * usel] += c;
              }
            }
          }
        }
      }
      // fold over the wave's four column groups (lane bits 5, 4): lane (q, g) then holds
      // row q4(g % 4) of tile row I; the four waves are summed in LDS at the end
      #pragma unroll
      for (int k = 0; k < KV; ++k) {
        xor_fold<4>(ra[k], lane, 32);
        xor_fold<2>(ra[k], lane, 16);
        red[k][w][bi][q4(g & 3)] = ra[k][0];
      }
    }
    // part of item it, side sd (0 rows, 1 columns), vector k
    auto partp = [&](int sd, int k) { return part + ((int64_t(2 * it + sd) * KV + k) * B) * TS; };
    if constexpr (!kColLds) {
      #pragma unroll
      for (int k = 0; k < KV; ++k) {
        // columns: fold over the 16 row lanes (bits 3..0); lane q holds block column q / 4,
        // column g + 16 (q % 4), summed over the block's rows -- written directly
        xor_fold<B * 4>(cacc[k], lane, 8);
        xor_fold<B * 2>(cacc[k], lane, 4);
        xor_fold<B>(cacc[k], lane, 2);
        xor_fold<B / 2>(cacc[k], lane, 1);
        if (k < nv) partp(1, k)[(q >> 2) * TS + g + 16 * (q & 3)] = cacc[k][0];
      }
    }
    __syncthreads();
    for (int e = t; e < KV * B * TS; e += kBlock) {
      const int k = e / (B * TS), b = (e / TS) % B, r = e % TS;
      if (k < nv) {
        partp(0, k)[b * TS + r] = (red[k][0][b][r] + red[k][1][b][r]) + (red[k][2][b][r] + red[k][3][b][r]);
        if constexpr (kColLds) partp(1, k)[b * TS + r] = colr[k][b][r];
      }
    }
    __syncthreads();                             // LDS (and s_item) free for the next item
  }
  if constexpr (PERSIST) {
    if (threadIdx.x == 0) {
      __threadfence();
      if (atomicAdd(queue + 1, 1) == int(gridDim.x) - 1) {   // the last workgroup: reset
        atomicExch(queue, 0);
        atomicExch(queue + 1, 0);
      }
    }
  }
}

template <typename P>
__global__ __launch_bounds__(kBlock) void k_symv2(
    const int32_t* __restrict__ n_arr, const int32_t* __restrict__ nt_arr,
    const int64_t* __restrict__ vec_off, const int64_t* __restrict__ item_base,
    const P* __restrict__ part, int kv, double alpha, const double* base, double* y,
    int64_t ld, const int32_t* __restrict__ row0) {
  // block (tile row I, matrix m, vector k); the parts of phase 1 hold kv vectors
  constexpr int B = kSymB;
  const int m = blockIdx.y, I = blockIdx.x, k = blockIdx.z, r = threadIdx.x & 63,
            prt = threadIdx.x >> 6;
  const int nt = nt_arr[m];
  if (I >= nt) return;
  const int nb = (nt + B - 1) / B, BI = I / B, b = I % B;
  const int64_t ib = item_base[m];
  const int r0 = row0 ? row0[m] : 0;           // items of block rows below r0: no parts
  double s = 0.0;
  if ((BI + 1) * B > r0)
    for (int BJ = prt; BJ <= BI; BJ += 4)      // row parts of block row BI
      s += double(part[((2 * (ib + tri(BI) + BJ) * kv + k) * B + b) * TS + r]);
  for (int B2 = BI + prt; B2 < nb; B2 += 4)    // column parts of block column BI
    if ((B2 + 1) * B > r0)
      s += double(part[(((2 * (ib + tri(B2) + BI) + 1) * kv + k) * B + b) * TS + r]);
  __shared__ double red[4][TS];
  red[prt][r] = s;
  __syncthreads();
  const int row = I * TS + r;
  if (prt == 0 && row < n_arr[m]) {
    const int64_t o = k * ld + vec_off[m] + row;
    const double v = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
    y[o] = (base ? base[o] : 0.0) + alpha * v;
  }
}

// ================================================================ Schur complements
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sigma_w(const T* __restrict__ tiles,
                                                    const int64_t* __restrict__ tile_off,
                                                    SigmaArgs a, double* __restrict__ W) {
  const int l = blockIdx.y, b = blockIdx.x;
  const int64_t m = a.B_off[l + 1] - a.B_off[l];
  if (b >= m) return;
  const int64_t s = a.shell_off[l + 1] - a.shell_off[l];
  const T* base = tiles + tile_off[l];
  const int64_t f = a.B_off[l] + b;
  double* Wc = W + a.w_off[l] + int64_t(b) * s;
  const int32_t* sh = a.shell + a.shell_off[l];
  for (int64_t si = threadIdx.x; si < s; si += kBlock) {
    const int i = sh[si];
    double v = 0.0;
    for (int64_t e = a.kcol_ptr[f]; e < a.kcol_ptr[f + 1]; ++e)
      v -= double(sym_elem(base, i, a.kcol_row[e])) * a.kcol_v[e];   // tiles hold -K^-1
    Wc[si] = v;
  }
}

constexpr int kSigmaRow = 32;   // max non-zeros of a row of K_{B_l, l} kept in registers
template <typename S>
__global__ __launch_bounds__(kBlock) void k_sigma_s(SigmaArgs a, const double* __restrict__ W,
                                                    S* __restrict__ sigma, int col_chunk) {
  // block (row chunk, column chunk, leaf): Sigma_l[a, b] = sum_e K[B_l[a], i_e] W_l[i_e, b]
  const int l = blockIdx.z;
  const int64_t m = a.B_off[l + 1] - a.B_off[l];
  const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t b0 = int64_t(blockIdx.y) * col_chunk;
  if (b0 >= m) return;
  const int64_t b1 = min<int64_t>(m, b0 + col_chunk);
  const int64_t s = a.shell_off[l + 1] - a.shell_off[l];
  int32_t col[kSigmaRow];
  double val[kSigmaRow];
  int cnt = 0;
  if (r < m) {
    const int64_t f = a.B_off[l] + r;
    const int64_t e0 = a.krow_ptr[f], e1 = a.krow_ptr[f + 1];
    cnt = int(min<int64_t>(e1 - e0, kSigmaRow));
#pragma unroll
    for (int e = 0; e < kSigmaRow; ++e)
      if (e < cnt) {
        col[e] = a.krow_col[e0 + e];
        val[e] = a.krow_v[e0 + e];
      }
    // rows with more couplings than fit in registers take the slow path below
    if (e1 - e0 > kSigmaRow) cnt = -1;
  }
  if (r >= m) return;
  const double* Wl = W + a.w_off[l];
  S* out = sigma + a.sig_off[l];
  for (int64_t b = b0; b < b1; ++b) {
    const double* Wc = Wl + b * s;
    double v = 0.0;
    if (cnt >= 0) {
#pragma unroll
      for (int e = 0; e < kSigmaRow; ++e)
        if (e < cnt) v += val[e] * Wc[col[e]];
    } else {
      const int64_t f = a.B_off[l] + r;
      for (int64_t e = a.krow_ptr[f]; e < a.krow_ptr[f + 1]; ++e)
        v += a.krow_v[e] * Wc[a.krow_col[e]];
    }
    out[a.row_major ? r * m + b : r + b * m] = S(v);
  }
}

template <typename T, typename S>
__global__ __launch_bounds__(kBlock) void k_schur_assemble(
    T* tiles, const int64_t* tile_off, const int32_t* n_arr, const int32_t* nt_arr,
    const int64_t* vec_off, const int64_t* __restrict__ adj_ptr,
    const int32_t* __restrict__ adj_leaf, const int32_t* __restrict__ adj_pos,
    const int64_t* __restrict__ B_off, const int64_t* __restrict__ sig_off,
    const S* __restrict__ sigma, int64_t n_leaf) {
  const int m = blockIdx.y;
  const int64_t t = blockIdx.x;
  if (t >= tri(nt_arr[m])) return;
  int I, J;
  tile_ij(t, &I, &J);
  const int n = n_arr[m];
  T* tl = tiles + tile_off[m] + t * TT;
  for (int e = threadIdx.x; e < TT; e += kBlock) {
    const int p = I * TS + (e % TS), q = J * TS + (e / TS);
    if (p >= n || q >= n) continue;
    const int64_t P = vec_off[m] + p - n_leaf, Q = vec_off[m] + q - n_leaf;
    int64_t ip = adj_ptr[P];
    const int64_t ep = adj_ptr[P + 1];
    int64_t iq = adj_ptr[Q];
    const int64_t eq = adj_ptr[Q + 1];
    double v = double(tl[e]);
    while (ip < ep && iq < eq) {   // leaves adjacent to both dofs (lists sorted by leaf)
      const int lp = adj_leaf[ip], lq = adj_leaf[iq];
      if (lp < lq) {
        ++ip;
      } else if (lq < lp) {
        ++iq;
      } else {
        const int64_t mm = B_off[lp + 1] - B_off[lp];
        v -= double(sigma[sig_off[lp] + adj_pos[ip] + int64_t(adj_pos[iq]) * mm]);
        ++ip;
        ++iq;
      }
    }
    tl[e] = T(v);
  }
}

// ================================================================ apply helpers
template <typename S, int KV>
__global__ __launch_bounds__(kBlock) void k_sigma_level(
    const int32_t* __restrict__ it_leaf, const int32_t* __restrict__ it_c0,
    const int32_t* __restrict__ it_c1, const int32_t* __restrict__ it_a0,
    const int32_t* __restrict__ it_a1,
    const S* __restrict__ sigma, const int64_t* __restrict__ sig_off,
    const int64_t* __restrict__ B_off, const int32_t* __restrict__ B,
    const double* __restrict__ z, double* __restrict__ e, int nv, int64_t ldz, int64_t lde) {
  // e_l[a] = sum_{c0 <= b < c1} Sigma_l[a, b] u[B_l[b]] for rows a in [a0, a1)
  // (<= kSigRows), for nv <= KV vectors (u_k = z + k ldz, e_k = e + k lde).  Row a of
  // Sigma_l is read contiguously in b (a symmetric Sigma_l is stored by columns, which
  // are its rows; a general one is stored by rows), one wave per kSigRows / 4 rows, the
  // gathered u staged in LDS; each row's sum is taken in a fixed order that does not
  // depend on KV.
  const int it = blockIdx.x;
  const int l = it_leaf[it], c0 = it_c0[it], c1 = it_c1[it], a0 = it_a0[it], a1 = it_a1[it];
  const int64_t m = B_off[l + 1] - B_off[l];
  const S* Sg = sigma + sig_off[l];
  const int32_t* Bl = B + B_off[l];
  constexpr int kSigStage = 1024;              // u values staged per pass and vector (8 KB)
  __shared__ double ub[KV][kSigStage];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int RW = kSigRows / 4;             // rows per wave
  double acc[RW][KV];
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int k = 0; k < KV; ++k) acc[q][k] = 0.0;
  for (int b0 = c0; b0 < c1; b0 += kSigStage) {
    const int nb = min(kSigStage, c1 - b0);
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kBlock) {
      const int32_t gi = Bl[b0 + b];
#pragma unroll
      for (int k = 0; k < KV; ++k) ub[k][b] = k < nv ? z[k * ldz + gi] : 0.0;
    }
    __syncthreads();
    const S* col[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int a = min(a0 + w * RW + q, a1 - 1);   // rows past a1 repeat a valid row
      col[q] = Sg + int64_t(a) * m + b0;
    }
    int b = lane;
    for (; b + 64 < nb; b += 128) {
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        const double s0 = double(ld_stream(col[q] + b)), s1 = double(ld_stream(col[q] + b + 64));
#pragma unroll
        for (int k = 0; k < KV; ++k) acc[q][k] += s0 * ub[k][b] + s1 * ub[k][b + 64];
      }
    }
    if (b < nb) {
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        const double s0 = double(ld_stream(col[q] + b));
#pragma unroll
        for (int k = 0; k < KV; ++k) acc[q][k] += s0 * ub[k][b];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int k = 0; k < KV; ++k) {
      double v = acc[q][k];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      const int a = a0 + w * RW + q;
      if (lane == 0 && a < a1 && k < nv) e[k * lde + B_off[l] + a] = v;
    }
}

// The same product for a symmetric Sigma_l (stored by columns: Sigma_l[a, b] at b m + a)
// and items of up to 64 rows: one wave per item, lane = row a, so each load of a column
// segment is coalesced and each row's sum runs over b in ascending order in one lane (no
// cross-lane reduction, no workgroup barrier).  The gathered u of 64 columns at a time
// is staged in the wave's own LDS slice and read back as broadcasts.  Small blocks (the
// face blocks of small sub-domains) keep the whole wave busy on one item.
template <typename S, int KV>
__global__ __launch_bounds__(kBlock) void k_sigma_rows(
    const int32_t* __restrict__ it_leaf, const int32_t* __restrict__ it_c0,
    const int32_t* __restrict__ it_c1, const int32_t* __restrict__ it_a0,
    const int32_t* __restrict__ it_a1, int count,
    const S* __restrict__ sigma, const int64_t* __restrict__ sig_off,
    const int64_t* __restrict__ B_off, const int32_t* __restrict__ B,
    const double* __restrict__ z, double* __restrict__ e, int nv, int64_t ldz, int64_t lde) {
  constexpr int NWV = kBlock / 64;
  __shared__ double ub[NWV][64][KV];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int it = blockIdx.x * NWV + w;
  if (it >= count) return;                     // wave-uniform: no block barrier below
  const int l = it_leaf[it], c0 = it_c0[it], c1 = it_c1[it], a0 = it_a0[it], a1 = it_a1[it];
  const int64_t m = B_off[l + 1] - B_off[l];
  const S* Sg = sigma + sig_off[l];
  const int32_t* Bl = B + B_off[l];
  const int a = min(a0 + lane, a1 - 1);        // lanes past a1 repeat a valid row
  double (*u)[KV] = ub[w];
  double acc[KV];
#pragma unroll
  for (int k = 0; k < KV; ++k) acc[k] = 0.0;
  for (int b0 = c0; b0 < c1; b0 += 64) {
    const int nb = min(64, c1 - b0);
    wave_sync();                               // the previous chunk's broadcasts are read
    if (lane < nb) {
      const int32_t gi = Bl[b0 + lane];
#pragma unroll
      for (int k = 0; k < KV; ++k) u[lane][k] = k < nv ? z[k * ldz + gi] : 0.0;
    }
    wave_sync();
    const S* col = Sg + int64_t(b0) * m + a;
    int j = 0;
    for (; j + 8 <= nb; j += 8) {
      S sv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) sv[q] = ld_stream(col + int64_t(j + q) * m);
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int k = 0; k < KV; ++k) acc[k] = fma(double(sv[q]), u[j + q][k], acc[k]);
    }
    for (; j < nb; ++j) {
      const double sv = double(ld_stream(col + int64_t(j) * m));
#pragma unroll
      for (int k = 0; k < KV; ++k) acc[k] = fma(sv, u[j][k], acc[k]);
    }
  }
  if (lane < a1 - a0) {
#pragma unroll
    for (int k = 0; k < KV; ++k)
      if (k < nv) e[k * lde + B_off[l] + a] = acc[k];
  }
}

// z_v[r] += alpha * sum over the leaves l adjacent to interface dof r of e_l[position of
// r in B_l], rows r in [row0, row0 + nrows), for nv vectors (z_v = z + v ldz, e_v = e +
// v lde)
__global__ __launch_bounds__(kBlock) void k_level_adj(
    int64_t row0, int64_t nrows, int64_t n_leaf, const int64_t* __restrict__ adj_ptr,
    const int32_t* __restrict__ adj_leaf, const int32_t* __restrict__ adj_pos,
    const int64_t* __restrict__ B_off, const double* __restrict__ e, double* __restrict__ z,
    int nv, int64_t ldz, int64_t lde, double alpha) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int v = blockIdx.y;                    // vector
  if (i >= nrows || v >= nv) return;
  const int64_t r = row0 + i;
  const int64_t p = r - n_leaf;
  const double* ev = e + v * lde;
  double s = z[v * ldz + r];
  for (int64_t k = adj_ptr[p]; k < adj_ptr[p + 1]; ++k)
    s += alpha * ev[B_off[adj_leaf[k]] + adj_pos[k]];
  z[v * ldz + r] = s;
}

// ================================================================ Krylov
constexpr int kDotCols = 8;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = sh[0] + sh[1] + sh[2] + sh[3];
  return t;
}

// The Krylov kernels below act on a batch of right-hand sides, one per grid row
// (blockIdx.y): operand i is the base pointer plus i times its batch stride.
__global__ __launch_bounds__(kBlock) void k_mdot_partial(const double* __restrict__ V,
                                                         int64_t ldv, int64_t sV, int ncols,
                                                         const double* __restrict__ w,
                                                         int64_t sw, int64_t n,
                                                         double* __restrict__ part) {
  __shared__ double sh[4];
  V += blockIdx.y * sV;
  w += blockIdx.y * sw;
  part += int64_t(blockIdx.y) * gridDim.x * ncols;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = min(n, lo + chunk);
  for (int c0 = 0; c0 < ncols; c0 += kDotCols) {
    double acc[kDotCols];
#pragma unroll
    for (int u = 0; u < kDotCols; ++u) acc[u] = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
      const double wr = w[r];
#pragma unroll
      for (int u = 0; u < kDotCols; ++u)
        if (c0 + u < ncols) acc[u] += V[r + (c0 + u) * ldv] * wr;
    }
#pragma unroll
    for (int u = 0; u < kDotCols; ++u) {
      if (c0 + u >= ncols) break;
      const double t = block_sum(acc[u], sh);
      if (threadIdx.x == 0) part[int64_t(blockIdx.x) * ncols + c0 + u] = t;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_mdot_final(const double* __restrict__ part,
                                                       int nblocks, int ncols,
                                                       double* __restrict__ out, int64_t so,
                                                       int mode) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  part += int64_t(blockIdx.y) * nblocks * ncols;
  out += blockIdx.y * so;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) v += part[int64_t(b) * ncols + c];
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) out[c] = (mode == 1) ? sqrt(t) : t;
}

__global__ __launch_bounds__(kBlock) void k_gemv_acc(const double* __restrict__ V, int64_t ldv,
                                                     int64_t sV, int ncols,
                                                     const double* __restrict__ h, int64_t sh,
                                                     double sign, double* __restrict__ w,
                                                     int64_t sw, int64_t n) {
  const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (r >= n) return;
  V += blockIdx.y * sV;
  h += blockIdx.y * sh;
  w += blockIdx.y * sw;
  double s = 0.0;
  for (int c = 0; c < ncols; ++c) s += V[r + c * ldv] * h[c];
  w[r] += sign * s;
}

__global__ void k_scale_div(const double* __restrict__ x, int64_t sx,
                            const double* __restrict__ d, int64_t sd, double* __restrict__ y,
                            int64_t sy, int64_t n) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  x += blockIdx.y * sx;
  y += blockIdx.y * sy;
  const double dv = d[blockIdx.y * sd];
  y[r] = dv != 0.0 ? x[r] / dv : 0.0;
}

__global__ void k_small_add(double* a, int64_t sa, const double* b, int64_t sb, int k) {
  const int i = threadIdx.x;
  if (i < k) a[blockIdx.y * sa + i] += b[blockIdx.y * sb + i];
}

__global__ void k_axpy_ratio(const double* __restrict__ x, const double* __restrict__ z,
                             const double* __restrict__ num, const double* __restrict__ den,
                             double sgn, double* __restrict__ y, int64_t n) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double dn = den[0];
  const double alpha = dn != 0.0 ? sgn * num[0] / dn : 0.0;
  y[r] = x[r] + alpha * z[r];
}


// ================================================================ inexact interface solves
// gamma steps of unpreconditioned GMRES from zero on S~_t u = g for every system m of a
// level and every vector k: one block per (m, k); the products w = S~ v_j between the
// steps are the caller's (Alg. 1's operator, applied matrix-free).  Basis vector j of vector k is V + (j nv + k) ld, used at the matrix's rows
// vec_off[m] .. vec_off[m] + n[m]; slot = k count + m indexes the per-system state:
// beta = ||g||, the (gamma + 1) x gamma Hessenberg matrix H (column-major), the steps
// taken and a stop flag (happy breakdown, or g = 0).
__device__ __forceinline__ double block_allsum(double v, double* sh) {
  // sum over the kBlock threads, returned to every thread (fixed order)
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(kBlock) void k_gm_start(
    const int32_t* __restrict__ n_arr, const int64_t* __restrict__ vec_off, int count,
    const double* __restrict__ z, int64_t ld, int nv, int gamma, double* __restrict__ V,
    double* __restrict__ beta, double* __restrict__ H, int32_t* __restrict__ steps,
    int32_t* __restrict__ stop) {
  __shared__ double sh[4];
  const int m = blockIdx.x, k = blockIdx.y;
  const int n = n_arr[m];
  const int64_t o = vec_off[m];
  const double* g = z + k * ld + o;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += g[i] * g[i];
  const double b = sqrt(block_allsum(s, sh));
  double* v0 = V + int64_t(k) * ld + o;
  for (int i = threadIdx.x; i < n; i += kBlock) v0[i] = b > 0.0 ? g[i] / b : 0.0;
  const int64_t slot = int64_t(k) * count + m;
  double* Hs = H + slot * (gamma + 1) * gamma;
  for (int i = threadIdx.x; i < (gamma + 1) * gamma; i += kBlock) Hs[i] = 0.0;
  if (threadIdx.x == 0) {
    beta[slot] = b;
    steps[slot] = 0;
    stop[slot] = b > 0.0 ? 0 : 1;
  }
}

// Step j after w = S~ v_j has been written to basis slot j + 1: modified Gram-Schmidt
// against v_0 .. v_j, the norm, and the normalisation unless the norm is at most
// 1e-14 beta (happy breakdown: the system stops with j + 1 steps).
__global__ __launch_bounds__(kBlock) void k_gm_orth(
    const int32_t* __restrict__ n_arr, const int64_t* __restrict__ vec_off, int count, int j,
    int64_t ld, int nv, int gamma, double* __restrict__ V, const double* __restrict__ beta,
    double* __restrict__ H, int32_t* __restrict__ steps, int32_t* __restrict__ stop) {
  __shared__ double sh[4];
  const int m = blockIdx.x, k = blockIdx.y;
  const int64_t slot = int64_t(k) * count + m;
  if (stop[slot] || steps[slot] != j) return;
  const int n = n_arr[m];
  const int64_t o = vec_off[m];
  double* Hs = H + slot * (gamma + 1) * gamma;
  double* w = V + (int64_t(j + 1) * nv + k) * ld + o;
  for (int i = 0; i <= j; ++i) {
    const double* vi = V + (int64_t(i) * nv + k) * ld + o;
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += kBlock) s += vi[r] * w[r];
    const double hij = block_allsum(s, sh);
    for (int r = threadIdx.x; r < n; r += kBlock) w[r] -= hij * vi[r];
    if (threadIdx.x == 0) Hs[i + j * (gamma + 1)] = hij;
  }
  double s = 0.0;
  for (int r = threadIdx.x; r < n; r += kBlock) s += w[r] * w[r];
  const double hn = sqrt(block_allsum(s, sh));
  if (threadIdx.x == 0) {
    Hs[j + 1 + j * (gamma + 1)] = hn;
    steps[slot] = j + 1;
  }
  if (hn <= 1e-14 * beta[slot]) {
    if (threadIdx.x == 0) stop[slot] = 1;
    return;
  }
  for (int r = threadIdx.x; r < n; r += kBlock) w[r] /= hn;
}

// u = V_k y with y the least-squares solution of min || beta e1 - H y || over the
// steps taken (Givens QR of the Hessenberg matrix), written over g in z.
constexpr int kGammaMax = kGammaMaxSteps;
__global__ __launch_bounds__(kBlock) void k_gm_finish(
    const int32_t* __restrict__ n_arr, const int64_t* __restrict__ vec_off, int count,
    int64_t ld, int nv, int gamma, const double* __restrict__ V,
    const double* __restrict__ beta, const double* __restrict__ H,
    const int32_t* __restrict__ steps, double* __restrict__ z) {
  __shared__ double R[(kGammaMax + 1) * kGammaMax];
  __shared__ double y[kGammaMax + 1];
  const int m = blockIdx.x, k = blockIdx.y;
  const int64_t slot = int64_t(k) * count + m;
  const int n = n_arr[m];
  const int64_t o = vec_off[m];
  const int ks = beta[slot] > 0.0 ? steps[slot] : 0;
  const double* Hs = H + slot * (gamma + 1) * gamma;
  for (int i = threadIdx.x; i < (gamma + 1) * gamma; i += kBlock) R[i] = Hs[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int L = gamma + 1;
    for (int i = 0; i <= ks; ++i) y[i] = i == 0 ? beta[slot] : 0.0;
    for (int c = 0; c < ks; ++c) {
      // rotation c acts on rows c, c + 1 of the remaining columns and zeroes R[c + 1, c]
      const double a = R[c + c * L], b = R[c + 1 + c * L];
      const double d = hypot(a, b);
      const double cs = d > 0.0 ? a / d : 1.0, sn = d > 0.0 ? b / d : 0.0;
      for (int cc = c; cc < ks; ++cc) {
        const double t0 = R[c + cc * L], t1 = R[c + 1 + cc * L];
        R[c + cc * L] = cs * t0 + sn * t1;
        R[c + 1 + cc * L] = -sn * t0 + cs * t1;
      }
      const double g0 = y[c], g1 = y[c + 1];
      y[c] = cs * g0 + sn * g1;
      y[c + 1] = -sn * g0 + cs * g1;
    }
    for (int c = ks - 1; c >= 0; --c) {
      double v = y[c];
      for (int cc = c + 1; cc < ks; ++cc) v -= R[c + cc * L] * y[cc];
      const double dg = R[c + c * L];
      y[c] = dg != 0.0 ? v / dg : 0.0;
    }
  }
  __syncthreads();
  double* u = z + k * ld + o;
  for (int r = threadIdx.x; r < n; r += kBlock) {
    double s = 0.0;
    for (int c = 0; c < ks; ++c) s += y[c] * V[(int64_t(c) * nv + k) * ld + o + r];
    u[r] = s;
  }
}

// ---- the same steps for levels with large systems: each system's rows are cut into
// chunks of at most kGmChunk entries (work items); a (chunk, vector) pair is one
// workgroup, so one large interface spreads over the whole GPU.  Gram-Schmidt is
// classical and done twice (two reductions per step instead of j + 1); every sum is a
// fixed-order two-pass reduction (per chunk, then per system in chunk order).  The
// state per (system, vector) slot is that of the one-workgroup kernels above, plus
// coef[slot][0 .. gamma + 1]: the current projection coefficients, then y; the last
// entry holds beta (start) or the new norm (step).
constexpr int kGmPer = kGmChunk / kBlock;       // rows per thread in a chunk

// partial sums of one chunk, mode 0: ||g||^2 of the right-hand side (z); mode 1: the
// projections v_i . w (i < ncols) of w = basis slot ncols; mode 2: ||w||^2 (w = slot j + 1)
__global__ __launch_bounds__(kBlock) void k_gmc_dots(GmArgs a, const double* __restrict__ z,
                                                     int j, int mode) {
  __shared__ double sh[4];
  const int it = blockIdx.x, k = blockIdx.y;
  const int m = a.item_sys[it];
  const int64_t slot = int64_t(k) * a.count + m;
  if (mode != 0 && (a.stop[slot] || a.steps[slot] != j)) return;
  const int64_t b = a.item_b[it], e = a.item_e[it];
  const double* w = mode == 0 ? z + k * a.ld : a.V + (int64_t(j + 1) * a.nv + k) * a.ld;
  double wv[kGmPer];
#pragma unroll
  for (int u = 0; u < kGmPer; ++u) {
    const int64_t r = b + threadIdx.x + int64_t(u) * kBlock;
    wv[u] = r < e ? w[r] : 0.0;
  }
  double* out = a.part + (int64_t(k) * a.nitems + it) * (a.gamma + 1);
  const int ncols = mode == 1 ? j + 1 : 1;
  for (int i = 0; i < ncols; ++i) {
    const double* vi = mode == 1 ? a.V + (int64_t(i) * a.nv + k) * a.ld : nullptr;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kGmPer; ++u) {
      const int64_t r = b + threadIdx.x + int64_t(u) * kBlock;
      if (r < e) s += (mode == 1 ? vi[r] : wv[u]) * wv[u];
    }
    const double t = block_allsum(s, sh);
    if (threadIdx.x == 0) out[i] = t;
  }
}

// per slot: sum the chunk partials in chunk order.  mode 0: beta, v_0 scale, reset of the
// state; mode 1 / 2: first / second Gram-Schmidt pass (H column j set / incremented,
// coefficients for the update); mode 3: the new norm, steps, happy-breakdown test.
__global__ void k_gmc_reduce(GmArgs a, int j, int mode) {
  const int m = blockIdx.x, k = blockIdx.y;
  const int64_t slot = int64_t(k) * a.count + m;
  const int L = a.gamma + 1;
  double* Hs = a.H + slot * L * a.gamma;
  double* cf = a.coef + slot * (L + 1);
  const int f = a.sys_first[m], l = a.sys_first[m + 1];
  const double* part = a.part + int64_t(k) * a.nitems * L;
  if (mode == 0) {
    for (int i = threadIdx.x; i < L * a.gamma; i += blockDim.x) Hs[i] = 0.0;
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int it = f; it < l; ++it) s += part[int64_t(it) * L];
      const double b = sqrt(s);
      a.beta[slot] = b;
      a.steps[slot] = 0;
      a.stop[slot] = b > 0.0 ? 0 : 1;
      cf[L] = b;
    }
    return;
  }
  if (a.stop[slot] || a.steps[slot] != j) return;
  if (mode == 3) {
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int it = f; it < l; ++it) s += part[int64_t(it) * L];
      const double hn = sqrt(s);
      Hs[j + 1 + j * L] = hn;
      cf[L] = hn;
      a.steps[slot] = j + 1;
      if (hn <= 1e-14 * a.beta[slot]) a.stop[slot] = 1;
    }
    return;
  }
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    double s = 0.0;
    for (int it = f; it < l; ++it) s += part[int64_t(it) * L + i];
    Hs[i + j * L] = mode == 1 ? s : Hs[i + j * L] + s;
    cf[i] = s;
  }
}

// mode 0: v_0 = g / beta (0 when beta = 0); mode 1: w -= sum_{i <= j} coef_i v_i
// (active slots of step j); mode 2: w /= norm unless the slot stopped at step j
__global__ __launch_bounds__(kBlock) void k_gmc_update(GmArgs a, const double* __restrict__ z,
                                                       int j, int mode) {
  const int it = blockIdx.x, k = blockIdx.y;
  const int m = a.item_sys[it];
  const int64_t slot = int64_t(k) * a.count + m;
  const int L = a.gamma + 1;
  const double* cf = a.coef + slot * (L + 1);
  const int64_t b = a.item_b[it], e = a.item_e[it];
  if (mode == 0) {
    const double bt = cf[L];
    const double* g = z + k * a.ld;
    double* v0 = a.V + int64_t(k) * a.ld;
    for (int64_t r = b + threadIdx.x; r < e; r += kBlock) v0[r] = bt > 0.0 ? g[r] / bt : 0.0;
    return;
  }
  double* w = a.V + (int64_t(j + 1) * a.nv + k) * a.ld;
  if (mode == 1) {
    if (a.stop[slot] || a.steps[slot] != j) return;
    for (int64_t r = b + threadIdx.x; r < e; r += kBlock) {
      double s = w[r];
      for (int i = 0; i <= j; ++i) s -= cf[i] * a.V[(int64_t(i) * a.nv + k) * a.ld + r];
      w[r] = s;
    }
    return;
  }
  if (a.stop[slot] || a.steps[slot] != j + 1) return;
  const double hn = cf[L];
  for (int64_t r = b + threadIdx.x; r < e; r += kBlock) w[r] /= hn;
}

// least squares of each slot (one thread, Givens QR as in k_gm_finish): y into coef
__global__ void k_gmc_lsq(GmArgs a) {
  __shared__ double R[(kGammaMax + 1) * kGammaMax];
  const int m = blockIdx.x, k = blockIdx.y;
  const int64_t slot = int64_t(k) * a.count + m;
  const int L = a.gamma + 1;
  const double* Hs = a.H + slot * L * a.gamma;
  for (int i = threadIdx.x; i < L * a.gamma; i += blockDim.x) R[i] = Hs[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* y = a.coef + slot * (L + 1);
  const int ks = a.beta[slot] > 0.0 ? a.steps[slot] : 0;
  for (int i = 0; i <= ks; ++i) y[i] = i == 0 ? a.beta[slot] : 0.0;
  for (int c = 0; c < ks; ++c) {
    const double p = R[c + c * L], q = R[c + 1 + c * L];
    const double d = hypot(p, q);
    const double cs = d > 0.0 ? p / d : 1.0, sn = d > 0.0 ? q / d : 0.0;
    for (int cc = c; cc < ks; ++cc) {
      const double t0 = R[c + cc * L], t1 = R[c + 1 + cc * L];
      R[c + cc * L] = cs * t0 + sn * t1;
      R[c + 1 + cc * L] = -sn * t0 + cs * t1;
    }
    const double g0 = y[c], g1 = y[c + 1];
    y[c] = cs * g0 + sn * g1;
    y[c + 1] = -sn * g0 + cs * g1;
  }
  for (int c = ks - 1; c >= 0; --c) {
    double v = y[c];
    for (int cc = c + 1; cc < ks; ++cc) v -= R[c + cc * L] * y[cc];
    const double dg = R[c + c * L];
    y[c] = dg != 0.0 ? v / dg : 0.0;
  }
}

// u = V_k y over a chunk, written over g in z
__global__ __launch_bounds__(kBlock) void k_gmc_combine(GmArgs a, double* __restrict__ z) {
  const int it = blockIdx.x, k = blockIdx.y;
  const int m = a.item_sys[it];
  const int64_t slot = int64_t(k) * a.count + m;
  const int L = a.gamma + 1;
  const double* y = a.coef + slot * (L + 1);
  const int ks = a.beta[slot] > 0.0 ? a.steps[slot] : 0;
  const int64_t b = a.item_b[it], e = a.item_e[it];
  double* u = z + k * a.ld;
  for (int64_t r = b + threadIdx.x; r < e; r += kBlock) {
    double s = 0.0;
    for (int c = 0; c < ks; ++c) s += y[c] * a.V[(int64_t(c) * a.nv + k) * a.ld + r];
    u[r] = s;
  }
}

// ================================================================ general sub-domains
// For a K that is not symmetric (the paper's two-field Problems 2 and 3) each leaf
// matrix is kept dense, column-major (n x n at gen_off[l]), and inverted by Gauss-Jordan
// elimination with partial pivoting -- the explicit-inverse counterpart of an LU solve.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gen_extract(
    T* __restrict__ A, const int64_t* __restrict__ gen_off, const int32_t* __restrict__ n_arr,
    const int64_t* __restrict__ vec_off, const int64_t* __restrict__ s0,
    const int64_t* __restrict__ s1, const int32_t* __restrict__ pcol,
    const double* __restrict__ pval) {
  const int m = blockIdx.y;
  const int n = n_arr[m];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  T* Am = A + gen_off[m];
  if (i >= n) return;
  for (int j = 0; j < n; ++j) Am[i + int64_t(j) * n] = T(0);
  const int64_t off = vec_off[m], r = off + i;
  for (int64_t k = s0[r]; k < s1[r]; ++k) {
    const int64_t j = int64_t(pcol[k]) - off;
    if (j >= 0 && j < n) Am[i + j * n] = T(pval[k]);
  }
}

// One workgroup per matrix; column k and the scaled pivot row are staged in LDS for
// each step (n <= kGenMax).  Arithmetic in FP64, storage T.  flags[m] = k + 1 when the
// largest candidate pivot of column k is zero or not finite.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gen_invert(T* __restrict__ A,
                                                       const int64_t* __restrict__ gen_off,
                                                       const int32_t* __restrict__ n_arr,
                                                       const int64_t* __restrict__ perm_off,
                                                       int32_t* __restrict__ perm,
                                                       int32_t* __restrict__ flags) {
  __shared__ double colk[kGenMax], rowk[kGenMax];
  __shared__ double rv[4];
  __shared__ int ri[4];
  const int m = blockIdx.x;
  const int n = n_arr[m];
  T* Am = A + gen_off[m];
  int32_t* pm = perm + perm_off[m];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = 0; k < n; ++k) {
    // pivot: largest |A[i, k]|, i >= k (smallest index among equals)
    double best = -1.0;
    int bi = n;
    for (int i = k + threadIdx.x; i < n; i += kBlock) {
      const double v = fabs(double(Am[i + int64_t(k) * n]));
      if (v > best || (v == best && i < bi)) { best = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    __syncthreads();
    if (lane == 0) { rv[w] = best; ri[w] = bi; }
    __syncthreads();
    best = rv[0];
    bi = ri[0];
    for (int q = 1; q < 4; ++q)
      if (rv[q] > best || (rv[q] == best && ri[q] < bi)) { best = rv[q]; bi = ri[q]; }
    if (!(best > 0.0) || best > 1.7e308) {      // zero, NaN or infinite pivot
      if (threadIdx.x == 0) flags[m] = k + 1;
      return;
    }
    if (bi != k)
      for (int j = threadIdx.x; j < n; j += kBlock) {
        const T t = Am[k + int64_t(j) * n];
        Am[k + int64_t(j) * n] = Am[bi + int64_t(j) * n];
        Am[bi + int64_t(j) * n] = t;
      }
    if (threadIdx.x == 0) pm[k] = bi;
    __syncthreads();
    const double d = double(Am[k + int64_t(k) * n]);
    for (int i = threadIdx.x; i < n; i += kBlock) {
      colk[i] = double(Am[i + int64_t(k) * n]);
      rowk[i] = (i == k ? 1.0 : double(Am[k + int64_t(i) * n])) / d;
    }
    __syncthreads();
    // A[k, :] <- row k / d (with A[k, k] = 1 / d); A[i, :] -= A[i, k] row_k otherwise
    // (A[i, k] <- -A[i, k] / d)
    const int64_t nn = int64_t(n) * n;
    for (int64_t e = threadIdx.x; e < nn; e += kBlock) {
      const int i = int(e % n), j = int(e / n);
      if (i == k) {
        Am[e] = T(rowk[j]);
      } else {
        const double a = j == k ? 0.0 : double(Am[e]);
        Am[e] = T(a - colk[i] * rowk[j]);
      }
    }
    __syncthreads();
  }
  // the row interchanges of the elimination become column interchanges of the inverse
  for (int k = n - 1; k >= 0; --k) {
    const int p = pm[k];
    if (p != k)
      for (int i = threadIdx.x; i < n; i += kBlock) {
        const T t = Am[i + int64_t(k) * n];
        Am[i + int64_t(k) * n] = Am[i + int64_t(p) * n];
        Am[i + int64_t(p) * n] = t;
      }
    __syncthreads();
  }
}

// y_k = alpha A_m x_k on every leaf's rows (one thread per row, x staged in LDS)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gen_matvec(
    const T* __restrict__ A, const int64_t* __restrict__ gen_off,
    const int32_t* __restrict__ n_arr, const int64_t* __restrict__ vec_off,
    const double* __restrict__ x, double alpha, double* __restrict__ y, int64_t ld) {
  __shared__ double xs[1024];
  const int m = blockIdx.y, k = blockIdx.z;
  const int n = n_arr[m];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (blockIdx.x * kBlock >= n) return;
  const T* Am = A + gen_off[m];
  const double* xv = x + k * ld + vec_off[m];
  double s = 0.0;
  for (int j0 = 0; j0 < n; j0 += 1024) {
    const int nb = min(1024, n - j0);
    __syncthreads();
    for (int j = threadIdx.x; j < nb; j += kBlock) xs[j] = xv[j0 + j];
    __syncthreads();
    if (i < n)
      for (int j = 0; j < nb; ++j) s += double(Am[i + int64_t(j0 + j) * n]) * xs[j];
  }
  if (i < n) y[k * ld + vec_off[m] + i] = alpha * s;
}

// W_l = K_ll^{-1}[shell, :] K_{l,B_l} from the dense inverses (cf. k_sigma_w)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sigma_w_gen(const T* __restrict__ A,
                                                        const int64_t* __restrict__ gen_off,
                                                        const int32_t* __restrict__ n_arr,
                                                        SigmaArgs a, double* __restrict__ W) {
  const int l = blockIdx.y, b = blockIdx.x;
  const int64_t m = a.B_off[l + 1] - a.B_off[l];
  if (b >= m) return;
  const int64_t s = a.shell_off[l + 1] - a.shell_off[l];
  const int n = n_arr[l];
  const T* Al = A + gen_off[l];
  const int64_t f = a.B_off[l] + b;
  double* Wc = W + a.w_off[l] + int64_t(b) * s;
  const int32_t* sh = a.shell + a.shell_off[l];
  for (int64_t si = threadIdx.x; si < s; si += kBlock) {
    const int i = sh[si];
    double v = 0.0;
    for (int64_t e = a.kcol_ptr[f]; e < a.kcol_ptr[f + 1]; ++e)
      v += double(Al[i + int64_t(a.kcol_row[e]) * n]) * a.kcol_v[e];
    Wc[si] = v;
  }
}

// 16-bit copy of FP32 tiles (round to nearest)
template <typename H>
__global__ __launch_bounds__(kBlock) void k_narrow(const float* __restrict__ src,
                                                   H* __restrict__ dst, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) dst[i] = H(src[i]);
}

inline unsigned blocks_for(int64_t n, int per = kBlock) { return unsigned((n + per - 1) / per); }

}  // namespace

// ================================================================ launchers
hipError_t launch_gather(const double* src, const int64_t* map, int64_t count, double* dst,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_gather<<<blocks_for(count), kBlock, 0, s>>>(src, map, count, dst);
  return hipGetLastError();
}

hipError_t launch_permute(const double* x, int64_t ldx, double* y, int64_t ldy,
                          const int32_t* perm, int64_t n, int32_t nrhs, int32_t inverse,
                          hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  k_permute<<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(x, ldx, y, ldy, perm, n, inverse);
  return hipGetLastError();
}

hipError_t launch_ell_fill(int64_t n, const int64_t* prow, const int32_t* pcol,
                           const double* pval, const int64_t* ell_off, int32_t* ell_col,
                           double* ell_val, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t ns = (n + kEllSlice - 1) / kEllSlice;
  k_ell_fill<<<unsigned(ns), kEllSlice, 0, s>>>(n, prow, pcol, pval, ell_off, ell_col, ell_val);
  return hipGetLastError();
}

hipError_t launch_ell_spmv(int64_t row0, int64_t nrows, const int64_t* s0, const int64_t* s1,
                           const int64_t* prow, const int64_t* ell_off, const int32_t* ell_col,
                           const double* ell_val, const double* x, const double* base,
                           double alpha, double* y, int nv, int64_t ld, double* xil,
                           int64_t col0, int64_t col1, hipStream_t s) {
  if (nrows <= 0 || nv <= 0) return hipSuccess;
  for (int v0 = 0; v0 < nv; v0 += kEllVec) {
    const int c = nv - v0 < kEllVec ? nv - v0 : kEllVec;
    const int kv = c == 1 ? 1 : c == 2 ? 2 : c <= 4 ? 4 : 8;
    const double* xb = x + v0 * ld;
    const double* bb = base ? base + v0 * ld : nullptr;
    double* yb = y + v0 * ld;
    const bool il = kv > 1 && xil != nullptr;
#define RSD_ELL(KV, IL)                                                                        \
  k_ell_spmv<KV, IL><<<blocks_for(nrows), kBlock, 0, s>>>(row0, nrows, s0, s1, prow, ell_off, \
                                                          ell_col, ell_val, xb, xil, bb, alpha, \
                                                          yb, c, ld)
#define RSD_IL(KV)                                                                         \
  if (col1 > col0)                                                                         \
  k_interleave<KV><<<blocks_for(col1 - col0), kBlock, 0, s>>>(xb, c, ld, col0, col1, xil)
    if (kv == 1) {
      RSD_ELL(1, false);
    } else if (!il) {
      if (kv == 2) RSD_ELL(2, false); else if (kv == 4) RSD_ELL(4, false); else RSD_ELL(8, false);
    } else if (kv == 2) {
      RSD_IL(2);
      RSD_ELL(2, true);
    } else if (kv == 4) {
      RSD_IL(4);
      RSD_ELL(4, true);
    } else {
      RSD_IL(8);
      RSD_ELL(8, true);
    }
#undef RSD_IL
#undef RSD_ELL
  }
  return hipGetLastError();
}

hipError_t launch_permute_csr(int32_t n, int64_t n_leaf, const int32_t* perm, const int32_t* iperm,
                              const int64_t* rp, const int32_t* ci, const int64_t* prow,
                              const int32_t* skel_lvl_begin, const int32_t* skel_own_end,
                              int32_t* pcol, int64_t* pmap, int64_t* segA, int64_t* segB,
                              int64_t* segC, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_permute_csr<<<unsigned((int64_t(n) + kPermRows - 1) / kPermRows), kBlock, 0, s>>>(
      n, n_leaf, perm, iperm, rp, ci, prow,
                                                 skel_lvl_begin, skel_own_end, pcol, pmap, segA,
                                                 segB, segC);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill<<<blocks_for(count), kBlock, 0, s>>>(p, count, v);
  return hipGetLastError();
}

hipError_t launch_sym_fill(const DevBatch& b, hipStream_t s) {
  if (b.count == 0 || b.max_tiles == 0) return hipSuccess;
  dim3 grid(unsigned(b.max_tiles), b.count);
  if (b.fp32)
    k_sym_fill<float><<<grid, kBlock, 0, s>>>((float*)b.tiles, b.tile_off, b.n, b.nt);
  else
    k_sym_fill<double><<<grid, kBlock, 0, s>>>((double*)b.tiles, b.tile_off, b.n, b.nt);
  return hipGetLastError();
}

hipError_t launch_sym_extract(const DevBatch& b, const int64_t* s0, const int64_t* s1,
                              const int32_t* pcol, const double* pval, int32_t max_n,
                              hipStream_t s) {
  if (b.count == 0 || max_n == 0) return hipSuccess;
  dim3 grid(blocks_for(max_n), b.count);
  if (b.fp32)
    k_sym_extract<float><<<grid, kBlock, 0, s>>>((float*)b.tiles, b.tile_off, b.n, b.vec_off,
                                                  s0, s1, pcol, pval);
  else
    k_sym_extract<double><<<grid, kBlock, 0, s>>>((double*)b.tiles, b.tile_off, b.n, b.vec_off,
                                                   s0, s1, pcol, pval);
  return hipGetLastError();
}

size_t sym_invert_scratch_bytes(const DevBatch& b, int group, size_t* pbytes, size_t* cbytes) {
  const size_t es = b.fp32 ? 4 : 8;
  const size_t PB = size_t(group) * TS;
  *pbytes = size_t(b.count) * PB * PB * es;
  *cbytes = size_t(b.count) * size_t(b.max_nt) * TS * PB * es;
  return *pbytes + 2 * *cbytes;
}

// FP64 look-ahead parts use k_sweep_update_la (a workgroup per tile) while the batch has
// at most this many 128 x 128 super-tiles in the next group's rows and columns
constexpr int64_t kFineLookAhead = 1024;

hipError_t launch_sweep_step(const DevBatch& b, int c0, int stage, void* pbuf, void* cbuf,
                             void* bbuf, int32_t* flags, int group, hipStream_t s, int part) {
  if (b.count == 0 || b.max_nt == 0) return hipSuccess;
  const int64_t stride = int64_t(b.max_nt) * TS * group * TS;
  if (b.split16 && b.fp32 && group >= 2 && stage == 2) {
    const int64_t nsb = (b.max_nt + 1) / 2, ns = nsb * (nsb + 1) / 2;
    const bool major = part != 1 && b.count >= 8;
    const int64_t per_xcd = major ? ns : (ns + 7) / 8;
    const dim3 grid = part == 1 ? dim3(unsigned(nsb * (group / 2)), b.count)
                      : major   ? dim3(unsigned(8 * ((b.count + 7) / 8) * ns), 1)
                                : dim3(unsigned(8 * per_xcd), b.count);
    if (group == 4 && b.upd_shape == 1) {
      const int64_t nsw = (b.max_nt + 3) / 4, nw = nsw * (nsw + 1) / 2;
      const int64_t pxw = major ? nw : (nw + 7) / 8;
      const dim3 gw = part == 1 ? dim3(unsigned(nsw), b.count)
                      : major   ? dim3(unsigned(8 * ((b.count + 7) / 8) * nw), 1)
                                : dim3(unsigned(8 * pxw), b.count);
      k_sweep_update_bf3w<2><<<gw, 512, 0, s>>>((float*)b.tiles, b.tile_off, b.nt, c0,
                                                (const float*)cbuf, (const float*)bbuf, stride, pxw,
                                                part, b.count);
    } else if (group == 4)
      k_sweep_update_bf3s<4><<<grid, kBlock, 0, s>>>((float*)b.tiles, b.tile_off, b.nt, c0,
                                                     (const float*)cbuf, (const float*)bbuf, stride,
                                                     per_xcd, part, b.count);
    else
      k_sweep_update_bf3s<2><<<grid, kBlock, 0, s>>>((float*)b.tiles, b.tile_off, b.nt, c0,
                                                     (const float*)cbuf, (const float*)bbuf, stride,
                                                     per_xcd, part, b.count);
    return hipGetLastError();
  }
#define RSD_STEP(T, G)                                                                          \
  do {                                                                                          \
    if (stage == 0 && G == 1)                                                                   \
      k_sweep_pivot<T, G><<<b.count, kPivotThreads, 0, s>>>((T*)b.tiles, b.tile_off, b.nt, c0,   \
                                                            (T*)pbuf, flags);                   \
    else if (stage == 0)                                                                        \
      k_sweep_pivot_blk<T, G><<<b.count, PivCfg<T>::threads, 0, s>>>(                          \
          (T*)b.tiles, b.tile_off, b.nt, c0, (T*)pbuf, flags);                                  \
    else if (stage == 1 && G >= 2)                                                              \
      k_sweep_panel2<T, (G >= 2 ? G : 2)><<<dim3(b.max_nt * panel_wgs<T>(G), b.count), kBlock, 0, s>>>( \
          (const T*)b.tiles, b.tile_off, b.nt, c0, (const T*)pbuf, (T*)cbuf, (T*)bbuf, stride); \
    else if (stage == 1)                                                                        \
      k_sweep_panel<T, G><<<dim3(b.max_nt, b.count), kBlock, 0, s>>>(                           \
          (const T*)b.tiles, b.tile_off, b.nt, c0, (const T*)pbuf, (T*)cbuf, (T*)bbuf, stride); \
    else if (G >= 2 && part == 1 && sizeof(T) == 8 &&                                         \
             int64_t(b.count) * ((b.max_nt + 1) / 2) * (G / 2) <= kFineLookAhead)               \
      k_sweep_update_la<T, (G >= 2 ? G : 2)><<<dim3(unsigned(b.max_nt * G), b.count), kBlock, 0, \
                                               s>>>((T*)b.tiles, b.tile_off, b.nt, c0,          \
                                                    (const T*)cbuf, (const T*)bbuf, stride);    \
    else if (G >= 2) {                                                                          \
      const int64_t nsb = (b.max_nt + 1) / 2, ns = nsb * (nsb + 1) / 2;                         \
      const bool major = part != 1 && b.count >= 8;                                             \
      const int64_t per_xcd = major ? ns : (ns + 7) / 8;                                        \
      const dim3 grid = part == 1 ? dim3(unsigned(nsb * (G / 2)), b.count)                      \
                        : major   ? dim3(unsigned(8 * ((b.count + 7) / 8) * ns), 1)             \
                                  : dim3(unsigned(8 * per_xcd), b.count);                       \
      k_sweep_update2<T, (G >= 2 ? G : 2)><<<grid, kBlock, 0, s>>>(                             \
          (T*)b.tiles, b.tile_off, b.nt, c0, (const T*)cbuf, (const T*)bbuf, stride, per_xcd,   \
          part, b.count);                                                                       \
    } else                                                                                      \
      k_sweep_update<T, G><<<dim3(unsigned(b.max_tiles), b.count), kBlock, 0, s>>>(             \
          (T*)b.tiles, b.tile_off, b.nt, c0, (const T*)cbuf, (const T*)bbuf, stride);           \
  } while (0)
  if (b.fp32) {
    if (group == 4) RSD_STEP(float, 4); else if (group == 2) RSD_STEP(float, 2); else RSD_STEP(float, 1);
  } else {
    if (group == 4) RSD_STEP(double, 4); else if (group == 2) RSD_STEP(double, 2); else RSD_STEP(double, 1);
  }
#undef RSD_STEP
  return hipGetLastError();
}

// workgroups of a persistent launch: as many as the device holds at once (occupancy of
// the kernel times the compute units, looked up once per kernel), at most one per item
template <typename K>
unsigned persistent_grid(K kernel, int64_t items) {
  static const int64_t slots = [&] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess)
      return int64_t(256);
    return int64_t(std::max(1, cus)) * std::max(1, per);
  }();
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(items, slots)));
}

hipError_t launch_symv(const DevBatch& b, const double* x, void* part, double alpha,
                       const double* base, double* y, int nv, int64_t ld, hipStream_t s,
                       const int32_t* row0) {
  if (b.count == 0 || b.num_items == 0 || nv <= 0) return hipSuccess;
  const int kmax = b.vec_pass > 0 ? min(b.vec_pass, symv_vectors(b)) : symv_vectors(b);
  for (int v0 = 0; v0 < nv; v0 += kmax) {
    const int c = nv - v0 < kmax ? nv - v0 : kmax;
    const int kv = c == 1 ? 1 : c == 2 ? 2 : 4;
    const double* xb = x + v0 * ld;
    const double* bb = base ? base + v0 * ld : nullptr;
    double* yb = y + v0 * ld;
#define RSD_SYMV(T, KV)                                                                         \
  do {                                                                                          \
    if (b.persist && b.queue)                                                                   \
      k_symv1<T, KV, true><<<persistent_grid(k_symv1<T, KV, true>, b.num_items), kBlock, 0, s>>>( \
          (const T*)b.tiles, b.tile_off, b.n, b.nt, b.vec_off, b.item_mat, b.item_BI,           \
          b.item_BJ, xb, ld, c, (typename SymPart<T>::type*)part, b.queue, b.num_items, row0);  \
    else                                                                                        \
      k_symv1<T, KV><<<b.num_items, kBlock, 0, s>>>((const T*)b.tiles, b.tile_off, b.n, b.nt,   \
                                                    b.vec_off, b.item_mat, b.item_BI, b.item_BJ, \
                                                    xb, ld, c, (typename SymPart<T>::type*)part, \
                                                    nullptr, b.num_items, row0);                \
  } while (0)
    if (b.half) {
      if (b.half == 1) {
        if (kv == 1) RSD_SYMV(_Float16, 1); else if (kv == 2) RSD_SYMV(_Float16, 2); else RSD_SYMV(_Float16, 4);
      } else {
        if (kv == 1) RSD_SYMV(__bf16, 1); else if (kv == 2) RSD_SYMV(__bf16, 2); else RSD_SYMV(__bf16, 4);
      }
      k_symv2<float><<<dim3(b.max_nt, b.count, c), kBlock, 0, s>>>(
          b.n, b.nt, b.vec_off, b.item_base, (const float*)part, kv, alpha, bb, yb, ld, row0);
    } else if (b.fp32) {
      if (kv == 1) RSD_SYMV(float, 1); else if (kv == 2) RSD_SYMV(float, 2); else RSD_SYMV(float, 4);
      k_symv2<float><<<dim3(b.max_nt, b.count, c), kBlock, 0, s>>>(
          b.n, b.nt, b.vec_off, b.item_base, (const float*)part, kv, alpha, bb, yb, ld, row0);
    } else {
      if (kv == 1) RSD_SYMV(double, 1); else if (kv == 2) RSD_SYMV(double, 2); else RSD_SYMV(double, 4);
      k_symv2<double><<<dim3(b.max_nt, b.count, c), kBlock, 0, s>>>(
          b.n, b.nt, b.vec_off, b.item_base, (const double*)part, kv, alpha, bb, yb, ld, row0);
    }
#undef RSD_SYMV
  }
  return hipGetLastError();
}

hipError_t launch_gen_invert(const GenBatch& g, const int64_t* prow, const int64_t* segA,
                             const int32_t* pcol, const double* pval, int32_t* flags,
                             hipStream_t s) {
  if (g.count == 0) return hipSuccess;
  if (g.max_n > kGenMax) return hipErrorInvalidValue;
  const dim3 grid(blocks_for(g.max_n), unsigned(g.count));
  if (g.fp32) {
    k_gen_extract<float><<<grid, kBlock, 0, s>>>((float*)g.A, g.gen_off, g.n, g.vec_off, prow,
                                                 segA, pcol, pval);
    k_gen_invert<float><<<g.count, kBlock, 0, s>>>((float*)g.A, g.gen_off, g.n, g.perm_off,
                                                   g.perm, flags);
  } else {
    k_gen_extract<double><<<grid, kBlock, 0, s>>>((double*)g.A, g.gen_off, g.n, g.vec_off, prow,
                                                  segA, pcol, pval);
    k_gen_invert<double><<<g.count, kBlock, 0, s>>>((double*)g.A, g.gen_off, g.n, g.perm_off,
                                                    g.perm, flags);
  }
  return hipGetLastError();
}

hipError_t launch_gen_matvec(const GenBatch& g, const double* x, double alpha, double* y,
                             int nv, int64_t ld, hipStream_t s) {
  if (g.count == 0 || nv <= 0) return hipSuccess;
  const dim3 grid(blocks_for(g.max_n), unsigned(g.count), unsigned(nv));
  if (g.fp32)
    k_gen_matvec<float><<<grid, kBlock, 0, s>>>((const float*)g.A, g.gen_off, g.n, g.vec_off, x,
                                                alpha, y, ld);
  else
    k_gen_matvec<double><<<grid, kBlock, 0, s>>>((const double*)g.A, g.gen_off, g.n, g.vec_off,
                                                 x, alpha, y, ld);
  return hipGetLastError();
}

hipError_t launch_sigma_w_gen(const GenBatch& g, const SigmaArgs& a, double* W, hipStream_t s) {
  if (a.num_leaves == 0 || a.max_m == 0) return hipSuccess;
  dim3 grid(a.max_m, a.num_leaves);
  if (g.fp32)
    k_sigma_w_gen<float><<<grid, kBlock, 0, s>>>((const float*)g.A, g.gen_off, g.n, a, W);
  else
    k_sigma_w_gen<double><<<grid, kBlock, 0, s>>>((const double*)g.A, g.gen_off, g.n, a, W);
  return hipGetLastError();
}

hipError_t launch_narrow(const float* src, void* dst, int64_t count, int kind, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (kind == 1)
    k_narrow<_Float16><<<blocks_for(count), kBlock, 0, s>>>(src, (_Float16*)dst, count);
  else if (kind == 2)
    k_narrow<__bf16><<<blocks_for(count), kBlock, 0, s>>>(src, (__bf16*)dst, count);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sigma_w(const DevBatch& leaf, const SigmaArgs& a, double* W, hipStream_t s) {
  if (a.num_leaves == 0 || a.max_m == 0) return hipSuccess;
  dim3 grid(a.max_m, a.num_leaves);
  if (leaf.fp32)
    k_sigma_w<float><<<grid, kBlock, 0, s>>>((const float*)leaf.tiles, leaf.tile_off, a, W);
  else
    k_sigma_w<double><<<grid, kBlock, 0, s>>>((const double*)leaf.tiles, leaf.tile_off, a, W);
  return hipGetLastError();
}

hipError_t launch_sigma_s(const SigmaArgs& a, const double* W, void* sigma, int sigma_fp32,
                          hipStream_t s) {
  if (a.num_leaves == 0 || a.max_m == 0) return hipSuccess;
  const int chunk = 64;
  dim3 grid(blocks_for(a.max_m), unsigned((a.max_m + chunk - 1) / chunk), a.num_leaves);
  if (sigma_fp32)
    k_sigma_s<float><<<grid, kBlock, 0, s>>>(a, W, (float*)sigma, chunk);
  else
    k_sigma_s<double><<<grid, kBlock, 0, s>>>(a, W, (double*)sigma, chunk);
  return hipGetLastError();
}

hipError_t launch_schur_assemble(const DevBatch& b, const int64_t* adj_ptr,
                                 const int32_t* adj_leaf, const int32_t* adj_pos,
                                 const int64_t* B_off, const int64_t* sig_off,
                                 const void* sigma, int sigma_fp32, int64_t n_leaf,
                                 hipStream_t s) {
  if (b.count == 0 || b.max_tiles == 0) return hipSuccess;
  dim3 grid(unsigned(b.max_tiles), b.count);
#define RSD_ASM(T, S)                                                                       \
  k_schur_assemble<T, S><<<grid, kBlock, 0, s>>>((T*)b.tiles, b.tile_off, b.n, b.nt, b.vec_off, \
                                                 adj_ptr, adj_leaf, adj_pos, B_off, sig_off, \
                                                 (const S*)sigma, n_leaf)
  if (b.fp32) {
    if (sigma_fp32) RSD_ASM(float, float); else RSD_ASM(float, double);
  } else {
    if (sigma_fp32) RSD_ASM(double, float); else RSD_ASM(double, double);
  }
#undef RSD_ASM
  return hipGetLastError();
}

hipError_t launch_sigma_level(const SigmaLevelItems& it, const void* sigma, int sigma_fp32,
                              const int64_t* sig_off, const int64_t* B_off, const int32_t* B,
                              const double* z, double* e, int nv, int64_t ldz, int64_t lde,
                              hipStream_t s) {
  if (it.count == 0 || nv <= 0) return hipSuccess;
  constexpr int kmax = 4;
  for (int v0 = 0; v0 < nv; v0 += kmax) {
    const int c = nv - v0 < kmax ? nv - v0 : kmax;
    const double* zb = z + v0 * ldz;
    double* eb = e + v0 * lde;
#define RSD_SIGL(S, KV)                                                                     \
  do {                                                                                      \
    if (it.by_rows)                                                                         \
      k_sigma_rows<S, KV><<<(it.count + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, s>>>(  \
          it.leaf, it.c0, it.c1, it.a0, it.a1, it.count, (const S*)sigma, sig_off, B_off, B, \
          zb, eb, c, ldz, lde);                                                             \
    else                                                                                    \
      k_sigma_level<S, KV><<<it.count, kBlock, 0, s>>>(it.leaf, it.c0, it.c1, it.a0, it.a1, \
                                                       (const S*)sigma, sig_off, B_off, B, zb, \
                                                       eb, c, ldz, lde);                    \
  } while (0)
    if (sigma_fp32) {
      if (c == 1) RSD_SIGL(float, 1); else if (c == 2) RSD_SIGL(float, 2); else RSD_SIGL(float, 4);
    } else {
      if (c == 1) RSD_SIGL(double, 1); else if (c == 2) RSD_SIGL(double, 2); else RSD_SIGL(double, 4);
    }
#undef RSD_SIGL
  }
  return hipGetLastError();
}

hipError_t launch_level_adj(int64_t row0, int64_t nrows, int64_t n_leaf, const int64_t* adj_ptr,
                            const int32_t* adj_leaf, const int32_t* adj_pos, const int64_t* B_off,
                            const double* e, double* z, int nv, int64_t ldz, int64_t lde,
                            double alpha, hipStream_t s) {
  if (nrows <= 0 || nv <= 0) return hipSuccess;
  k_level_adj<<<dim3(blocks_for(nrows), nv), kBlock, 0, s>>>(row0, nrows, n_leaf, adj_ptr,
                                                             adj_leaf, adj_pos, B_off, e, z, nv,
                                                             ldz, lde, alpha);
  return hipGetLastError();
}

hipError_t launch_gm_start(const DevBatch& b, int gamma, int nv, const double* z, int64_t ld,
                           double* V, double* beta, double* H, int32_t* steps, int32_t* stop,
                           hipStream_t s) {
  if (b.count == 0 || nv <= 0) return hipSuccess;
  if (gamma < 1 || gamma > kGammaMax) return hipErrorInvalidValue;
  k_gm_start<<<dim3(unsigned(b.count), unsigned(nv)), kBlock, 0, s>>>(
      b.n, b.vec_off, b.count, z, ld, nv, gamma, V, beta, H, steps, stop);
  return hipGetLastError();
}

hipError_t launch_gm_orth(const DevBatch& b, int gamma, int nv, int j, int64_t ld, double* V,
                          const double* beta, double* H, int32_t* steps, int32_t* stop,
                          hipStream_t s) {
  if (b.count == 0 || nv <= 0) return hipSuccess;
  if (gamma < 1 || gamma > kGammaMax || j < 0 || j >= gamma) return hipErrorInvalidValue;
  k_gm_orth<<<dim3(unsigned(b.count), unsigned(nv)), kBlock, 0, s>>>(
      b.n, b.vec_off, b.count, j, ld, nv, gamma, V, beta, H, steps, stop);
  return hipGetLastError();
}

hipError_t launch_gmc(const GmArgs& a, int op, int j, const double* zin, double* zout,
                      hipStream_t s) {
  if (a.count == 0 || a.nv <= 0 || a.nitems == 0) return hipSuccess;
  if (a.gamma < 1 || a.gamma > kGammaMax || j < 0 || j >= a.gamma) return hipErrorInvalidValue;
  const dim3 gi(unsigned(a.nitems), unsigned(a.nv)), gs(unsigned(a.count), unsigned(a.nv));
  switch (op) {
    case 0:   // start: beta = ||g||, v_0 = g / beta
      k_gmc_dots<<<gi, kBlock, 0, s>>>(a, zin, 0, 0);
      k_gmc_reduce<<<gs, 64, 0, s>>>(a, 0, 0);
      k_gmc_update<<<gi, kBlock, 0, s>>>(a, zin, 0, 0);
      break;
    case 1:   // step j after w = S~ v_j: classical Gram-Schmidt twice, norm, normalisation
      for (int pass = 1; pass <= 2; ++pass) {
        k_gmc_dots<<<gi, kBlock, 0, s>>>(a, nullptr, j, 1);
        k_gmc_reduce<<<gs, 64, 0, s>>>(a, j, pass);
        k_gmc_update<<<gi, kBlock, 0, s>>>(a, nullptr, j, 1);
      }
      k_gmc_dots<<<gi, kBlock, 0, s>>>(a, nullptr, j, 2);
      k_gmc_reduce<<<gs, 64, 0, s>>>(a, j, 3);
      k_gmc_update<<<gi, kBlock, 0, s>>>(a, nullptr, j, 2);
      break;
    default:  // finish: least squares, u = V y
      k_gmc_lsq<<<gs, 64, 0, s>>>(a);
      k_gmc_combine<<<gi, kBlock, 0, s>>>(a, zout);
  }
  return hipGetLastError();
}

hipError_t launch_gm_finish(const DevBatch& b, int gamma, int nv, int64_t ld, const double* V,
                            const double* beta, const double* H, const int32_t* steps,
                            double* z, hipStream_t s) {
  if (b.count == 0 || nv <= 0) return hipSuccess;
  if (gamma < 1 || gamma > kGammaMax) return hipErrorInvalidValue;
  k_gm_finish<<<dim3(unsigned(b.count), unsigned(nv)), kBlock, 0, s>>>(
      b.n, b.vec_off, b.count, ld, nv, gamma, V, beta, H, steps, z);
  return hipGetLastError();
}

int mdot_blocks(int64_t n) {
  int64_t b = (n + 511) / 512;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return int(b);
}

hipError_t launch_mdot(int nb_rhs, const double* V, int64_t ldv, int64_t sV, int ncols,
                       const double* w, int64_t sw, int64_t n, double* partial, double* out,
                       int64_t so, int mode, hipStream_t s) {
  if (ncols <= 0 || nb_rhs <= 0) return hipSuccess;
  const int nb = mdot_blocks(n);
  k_mdot_partial<<<dim3(nb, nb_rhs), kBlock, 0, s>>>(V, ldv, sV, ncols, w, sw, n, partial);
  k_mdot_final<<<dim3(ncols, nb_rhs), kBlock, 0, s>>>(partial, nb, ncols, out, so, mode);
  return hipGetLastError();
}

hipError_t launch_gemv_acc(int nb_rhs, const double* V, int64_t ldv, int64_t sV, int ncols,
                           const double* h, int64_t sh, double sign, double* w, int64_t sw,
                           int64_t n, hipStream_t s) {
  if (ncols <= 0 || n <= 0 || nb_rhs <= 0) return hipSuccess;
  k_gemv_acc<<<dim3(blocks_for(n), nb_rhs), kBlock, 0, s>>>(V, ldv, sV, ncols, h, sh, sign, w,
                                                            sw, n);
  return hipGetLastError();
}

hipError_t launch_scale_div(int nb_rhs, const double* x, int64_t sx, const double* d,
                            int64_t sd, double* y, int64_t sy, int64_t n, hipStream_t s) {
  if (n <= 0 || nb_rhs <= 0) return hipSuccess;
  k_scale_div<<<dim3(blocks_for(n), nb_rhs), kBlock, 0, s>>>(x, sx, d, sd, y, sy, n);
  return hipGetLastError();
}

hipError_t launch_small_add(int nb_rhs, double* a, int64_t sa, const double* b, int64_t sb,
                            int k, hipStream_t s) {
  if (k <= 0 || nb_rhs <= 0) return hipSuccess;
  k_small_add<<<dim3(1, nb_rhs), 512, 0, s>>>(a, sa, b, sb, k);
  return hipGetLastError();
}

hipError_t launch_axpy_ratio(const double* x, const double* z, const double* num,
                             const double* den, double sgn, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axpy_ratio<<<blocks_for(n), kBlock, 0, s>>>(x, z, num, den, sgn, y, n);
  return hipGetLastError();
}

}  // namespace rsd
