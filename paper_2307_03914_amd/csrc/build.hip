// bspai_build / bspai_import: SPAI on a fixed pattern (Algorithm 1's least
// squares with no pattern augmentation, run on A^T as in Algorithm 4 step 1),
// ||M||_inf, bucketing (Algorithm 2, eq. (nint)) and per-bucket packing.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "formats.h"

namespace bspai {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// sums and square roots in the construction precision T: shuffled values are
// widened exactly to float (fp16) and every addition is rounded to T
template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
  if constexpr (sizeof(T) == 8) {
    return wave_sum_d(v);
  } else {
    for (int o = 32; o > 0; o >>= 1) v = (T)(v + (T)__shfl_xor((float)v, o));
    return v;
  }
}

template <typename T>
__device__ __forceinline__ T sqrt_t(T v) {
  if constexpr (sizeof(T) == 8) return sqrt(v);
  else return (T)sqrtf((float)v);  // correctly rounded in float, then in fp16
}

template <typename T>
constexpr double unit_roundoff_t() {
  return sizeof(T) == 8 ? 0x1p-53 : sizeof(T) == 4 ? 0x1p-24 : 0x1p-11;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lower_bound_i(const int32_t *a, int len, int key) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Limits of the one-wavefront path (least-squares tile in LDS).
constexpr int kSmallJ = 64;
constexpr int kSmallCand = 1024;
constexpr int kSmallTile = 8192;  // doubles

// per row k of the pattern: |J_k| and the number of candidate shadow indices;
// rows beyond the wavefront path's limits are appended to the block path list
__global__ void k_spai_sizes(int n, const int32_t *arp, const int32_t *prp, const int32_t *pcol, int32_t *out_max,
                             int8_t *is_big, int32_t *big_list, int32_t *big_count, int32_t *cand_of) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int s = prp[k], e = prp[k + 1];
  int cand = 0;
  for (int p = s; p < e; p++) cand += arp[pcol[p] + 1] - arp[pcol[p]];
  int nJ = e - s;
  cand_of[k] = cand;
  bool big = nJ > kSmallJ || cand > kSmallCand || (int64_t)cand * nJ > kSmallTile;
  is_big[k] = big ? 1 : 0;
  if (big) {
    big_list[atomicAdd(big_count, 1)] = k;
    atomicMax(&out_max[2], nJ);
    atomicMax(&out_max[3], cand);
  } else {
    atomicMax(&out_max[0], nJ);
    atomicMax(&out_max[1], cand);
  }
}

// d_j = 1 / max_l |a_jl|: scales column j of A^T to unit max (Section 4)
__global__ void k_row_maxabs_inv(int n, const int32_t *arp, const double *aval, double *d) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double mx = 0;
  for (int p = arp[j]; p < arp[j + 1]; p++) mx = fmax(mx, fabs(aval[p]));
  d[j] = mx > 0 ? 1.0 / mx : 1.0;
}

struct SpaiArgs {
  int n;
  const int32_t *arp, *acol;
  const double *aval;
  const int32_t *prp, *pcol;
  const double *dscale;  // null: no scaling
  double *mval;
  int cand_p2;  // capacity of the index lists (power of two)
  int tile_cap; // capacity of the dense tile in doubles
  int32_t *err; // [0] first zero row, [1] first rank-deficient row, [2] first oversized row,
                // [3] first row whose least squares overflows the construction precision
  const int8_t *is_big;  // rows left to the block path
};

// One wavefront per row k of M:
//   J = P(k,:); I = sorted union of the nonzero columns of the rows J of A
//   (the shadow of J in A^T); Abar(l, c) = a_{J_c, I_l}; ebar = e_k(I);
//   Householder QR of Abar, mbar = R^{-1} (Q^T ebar)(1:|J|); M(k, J) = mbar.
// T is the construction precision u_f (Section 4: double, single or half):
// the tile holds a_{J_c, I_l} d_j rounded to T, every operation of the QR
// and the back substitution is done in T and rounded separately (the library
// is built without implicit multiply-add fusion; sums run as wavefront
// trees), and M(k, j) is mbar_j d_j rounded to T, stored in FP64.
template <typename T>
__global__ void __launch_bounds__(64) k_spai(SpaiArgs a) {
  extern __shared__ double lds_d[];
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  if (a.is_big[k]) return;
  const int ps = a.prp[k], nJ = a.prp[k + 1] - ps;
  int32_t *cand = reinterpret_cast<int32_t *>(lds_d);  // cand_p2
  int32_t *I = cand + a.cand_p2;                        // cand_p2
  T *Ab = reinterpret_cast<T *>(lds_d + a.cand_p2);    // tile_cap (after the two int lists)
  T *eb = Ab + a.tile_cap;                              // cand_p2
  T *mv = eb + a.cand_p2;                               // 64 + nJ

  // gather candidate columns (nonzero values only), compacted with ballots
  int nc = 0;
  for (int c = 0; c < nJ; c++) {
    int j = a.pcol[ps + c];
    int s = a.arp[j], e = a.arp[j + 1];
    for (int base = s; base < e; base += 64) {
      int p = base + lane;
      bool pred = p < e && a.aval[p] != 0.0;
      uint64_t mask = __ballot(pred);
      if (nc + __popcll(mask) > a.cand_p2) {
        if (lane == 0) atomicMin(&a.err[2], k);
        return;
      }
      int pos = nc + __popcll(mask & ((1ull << lane) - 1ull));
      if (pred) cand[pos] = a.acol[p];
      nc += __popcll(mask);
    }
  }
  int S = 1;
  while (S < nc) S <<= 1;
  for (int p = nc + lane; p < S; p += 64) cand[p] = INT_MAX;
  wave_sync();
  // bitonic sort of cand[0..S)
  for (int size = 2; size <= S; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = lane; t < S / 2; t += 64) {
        int lo = 2 * stride * (t / stride) + (t % stride);
        int hi = lo + stride;
        bool up = ((lo & size) == 0);
        int x = cand[lo], y = cand[hi];
        if ((x > y) == up) {
          cand[lo] = y;
          cand[hi] = x;
        }
      }
      wave_sync();
    }
  }
  // unique -> I
  int nI = 0;
  for (int base = 0; base < nc; base += 64) {
    int p = base + lane;
    bool pred = p < nc && (p == 0 || cand[p] != cand[p - 1]);
    uint64_t mask = __ballot(pred);
    int pos = nI + __popcll(mask & ((1ull << lane) - 1ull));
    if (pred) I[pos] = cand[p];
    nI += __popcll(mask);
  }
  wave_sync();
  for (int c = lane; c < nJ; c += 64) a.mval[ps + c] = 0.0;
  int lk = lower_bound_i(I, nI, k);
  if (lk >= nI || I[lk] != k) {
    if (lane == 0) atomicMin(&a.err[0], k);
    return;
  }
  if (nI < nJ) {
    if (lane == 0) atomicMin(&a.err[1], k);
    return;
  }
  if ((int64_t)nI * nJ > a.tile_cap || nJ > 64) {
    if (lane == 0) atomicMin(&a.err[2], k);
    return;
  }
  // dense tile, column-major with leading dimension nI
  for (int p = lane; p < nI * nJ; p += 64) Ab[p] = (T)0;
  for (int p = lane; p < nI; p += 64) eb[p] = (p == lk) ? (T)1 : (T)0;
  wave_sync();
  for (int c = 0; c < nJ; c++) {
    int j = a.pcol[ps + c];
    double dj = a.dscale ? a.dscale[j] : 1.0;
    for (int p = a.arp[j] + lane; p < a.arp[j + 1]; p += 64) {
      double v = a.aval[p];
      if (v != 0.0) Ab[lower_bound_i(I, nI, a.acol[p]) + c * nI] = (T)(v * dj);
    }
  }
  wave_sync();
  T fro2 = 0;
  for (int p = lane; p < nI * nJ; p += 64) fro2 += Ab[p] * Ab[p];
  const double fro = (double)sqrt_t(wave_sum_t(fro2));
  if (!isfinite(fro)) {  // an entry or ||Abar||_F overflows T
    if (lane == 0) atomicMin(&a.err[3], k);
    return;
  }
  T *diagR = mv + 64;
  // Householder QR: reflector v = a + sign(a_1) ||a|| e_1 kept in column c
  for (int c = 0; c < nJ; c++) {
    T *col = Ab + c * nI;
    T s2 = 0;
    for (int l = c + lane; l < nI; l += 64) s2 += col[l] * col[l];
    const T nrm = sqrt_t(wave_sum_t(s2));
    const T alpha = col[c];
    const T beta = (T)-copysign((double)nrm, (double)alpha);
    if (nrm == (T)0 || fabs((double)beta) <= (double)nJ * unit_roundoff_t<T>() * fro) {
      if (lane == 0) atomicMin(&a.err[1], k);
      return;
    }
    wave_sync();
    if (lane == 0) col[c] = (T)(alpha - beta);
    wave_sync();
    T vt = 0;
    for (int l = c + lane; l < nI; l += 64) vt += col[l] * col[l];
    const T vtv = wave_sum_t(vt);
    for (int jj = c + 1; jj <= nJ; jj++) {  // jj == nJ is the right-hand side
      T *cj = (jj < nJ) ? Ab + jj * nI : eb;
      T w = 0;
      for (int l = c + lane; l < nI; l += 64) w += col[l] * cj[l];
      const T f = (T)((T)2 * wave_sum_t(w)) / vtv;
      for (int l = c + lane; l < nI; l += 64) cj[l] -= f * col[l];
      wave_sync();
    }
    if (lane == 0) diagR[c] = beta;
    wave_sync();
  }
  // back substitution R m = (Q^T ebar)(1:nJ), one lane
  if (lane == 0) {
    bool finite = true;
    for (int c = nJ - 1; c >= 0; c--) {
      T t = eb[c];
      for (int jj = c + 1; jj < nJ; jj++) t -= Ab[c + jj * nI] * mv[jj];
      mv[c] = t / diagR[c];
      finite = finite && isfinite((double)mv[c]);
    }
    if (!finite) atomicMin(&a.err[3], k);
  }
  wave_sync();
  for (int c = lane; c < nJ; c += 64) {
    double dj = a.dscale ? a.dscale[a.pcol[ps + c]] : 1.0;
    a.mval[ps + c] = (double)(T)((double)mv[c] * dj);
  }
}


// ------------------------------------------------------------------ block path
//
// One block per row k whose least-squares tile is too large for a wavefront.
// The candidate shadow indices are sorted in LDS; a shadow row l with a single
// nonzero (in column c) only enters the objective as (a_l m_c - e_l)^2, so all
// such rows of column c are replaced by one row with entry ||a||_2 and right
// side (sum_l a_l e_l) / ||a||_2 (an orthogonal reduction; the least-squares
// solution is unchanged).  Rows with several nonzeros are kept.  The reduced
// tile (multi rows, then one folded row per column) is factored by Householder
// QR in global memory, columns spread over the waves.

constexpr int kBigThreads = 256;
constexpr int kBigCand = 16384;  // LDS capacity for the sorted candidates

struct SpaiBigArgs {
  const int32_t *arp, *acol;
  const double *aval;
  const int32_t *prp, *pcol;
  const double *dscale;
  double *mval;
  const int32_t *rows;       // rows of this batch
  const int64_t *tile_off;   // per row: offset of its tile in tiles (doubles)
  const int64_t *rhs_off;    // per row: offset of its right side in rhs (doubles)
  double *tiles, *rhs;
  int32_t *err;
};

__device__ __forceinline__ double block_sum_big(double v, double *sh) {
  v = wave_sum_d(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kBigThreads / 64; w++) t += sh[w];
  return t;
}

__global__ void __launch_bounds__(kBigThreads) k_spai_big(SpaiBigArgs a) {
  extern __shared__ double lds_b[];
  int32_t *S = reinterpret_cast<int32_t *>(lds_b);  // kBigCand sorted candidates
  int32_t *code = S + kBigCand;                       // per sorted position: multi row index, -1 single
  double *diagR = lds_b + kBigCand;                   // after the two int arrays (8 * kBigCand bytes)
  double *yv = diagR + 1024;
  __shared__ double sh[kBigThreads / 64];
  __shared__ int s_nc, s_nmulti, s_flag;
  const int tid = threadIdx.x;
  const int k = a.rows[blockIdx.x];
  const int ps = a.prp[k], nJ = a.prp[k + 1] - ps;
  const int *J = a.pcol + ps;
  for (int c = tid; c < nJ; c += kBigThreads) a.mval[ps + c] = 0.0;
  if (tid == 0) {
    // candidate count (all entries of the rows J; zeros are marked below)
    int nc = 0;
    for (int c = 0; c < nJ; c++) nc += a.arp[J[c] + 1] - a.arp[J[c]];
    s_nc = nc;
  }
  __syncthreads();
  const int nc = s_nc;
  if (nc > kBigCand || nJ > 1024) {
    if (tid == 0) atomicMin(&a.err[2], k);
    return;
  }
  // gather: segment offsets by one thread, then one thread per column copies
  // its row's column indices (explicit zeros become INT_MAX, sorted last)
  if (tid == 0) {
    int off = 0;
    for (int c = 0; c < nJ; c++) {
      code[c] = off;
      off += a.arp[J[c] + 1] - a.arp[J[c]];
    }
  }
  __syncthreads();
  for (int c = tid; c < nJ; c += kBigThreads) {
    int j = J[c], off = code[c];
    for (int p = a.arp[j]; p < a.arp[j + 1]; p++) S[off++] = a.aval[p] != 0.0 ? a.acol[p] : INT_MAX;
  }
  int P2 = 1;
  while (P2 < nc) P2 <<= 1;
  __syncthreads();
  for (int p = nc + tid; p < P2; p += kBigThreads) S[p] = INT_MAX;
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < P2 / 2; t += kBigThreads) {
        int lo = 2 * stride * (t / stride) + (t % stride);
        int hi = lo + stride;
        bool up = ((lo & size) == 0);
        int x = S[lo], y = S[hi];
        if ((x > y) == up) {
          S[lo] = y;
          S[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  // runs of equal indices: multi rows get consecutive indices in sorted order
  if (tid == 0) {
    int nm = 0, found_k = 0;
    for (int p = 0; p < nc && S[p] != INT_MAX;) {
      int q = p + 1;
      while (q < nc && S[q] == S[p]) q++;
      int c = (q - p >= 2) ? nm++ : -1;
      for (int t = p; t < q; t++) code[t] = c;
      if (S[p] == k) found_k = 1;
      p = q;
    }
    s_nmulti = nm;
    s_flag = found_k;
  }
  __syncthreads();
  if (!s_flag) {
    if (tid == 0) atomicMin(&a.err[0], k);
    return;
  }
  const int nm = s_nmulti;
  const int T = nm + nJ;  // tile rows: multi rows, then one folded row per column
  double *tile = a.tiles + a.tile_off[blockIdx.x];
  double *rhs = a.rhs + a.rhs_off[blockIdx.x];
  for (int64_t p = tid; p < (int64_t)T * nJ; p += kBigThreads) tile[p] = 0.0;
  for (int p = tid; p < T; p += kBigThreads) rhs[p] = 0.0;
  __syncthreads();
  // scatter the entries: thread per column, entries in row order (deterministic)
  int valid = nc;
  while (valid > 0 && S[valid - 1] == INT_MAX) valid--;
  for (int c = tid; c < nJ; c += kBigThreads) {
    int j = J[c];
    double dj = a.dscale ? a.dscale[j] : 1.0;
    double f2 = 0.0, fk = 0.0;
    for (int p = a.arp[j]; p < a.arp[j + 1]; p++) {
      double v = a.aval[p];
      if (v == 0.0) continue;
      v *= dj;
      int i = a.acol[p];
      int lo = lower_bound_i(S, valid, i);
      int cd = code[lo];
      if (cd >= 0) {
        tile[cd + (int64_t)c * T] = v;
        if (i == k) rhs[cd] = 1.0;
      } else {
        f2 += v * v;
        if (i == k) fk = v;
      }
    }
    if (f2 > 0.0) {
      double nrm = sqrt(f2);
      tile[nm + c + (int64_t)c * T] = nrm;
      rhs[nm + c] = fk / nrm;
    }
  }
  __syncthreads();
  // Frobenius norm for the rank test
  double fl = 0.0;
  for (int64_t p = tid; p < (int64_t)T * nJ; p += kBigThreads) fl += tile[p] * tile[p];
  const double fro = sqrt(block_sum_big(fl, sh));
  const int lane = tid & 63, w = tid >> 6;
  for (int c = 0; c < nJ; c++) {
    double *col = tile + (int64_t)c * T;
    double s2 = 0.0;
    for (int l = c + tid; l < T; l += kBigThreads) s2 += col[l] * col[l];
    double nrm = sqrt(block_sum_big(s2, sh));
    double alpha = col[c];
    double beta = -copysign(nrm, alpha);
    if (nrm == 0.0 || fabs(beta) <= (double)nJ * 0x1p-53 * fro) {
      if (tid == 0) atomicMin(&a.err[1], k);
      return;
    }
    __syncthreads();
    if (tid == 0) {
      col[c] = alpha - beta;
      diagR[c] = beta;
    }
    __syncthreads();
    double vt = 0.0;
    for (int l = c + tid; l < T; l += kBigThreads) vt += col[l] * col[l];
    const double vtv = block_sum_big(vt, sh);
    // trailing columns and the right side: one wave per column
    for (int jj = c + 1 + w; jj <= nJ; jj += kBigThreads / 64) {
      double *cj = (jj < nJ) ? tile + (int64_t)jj * T : rhs;
      double d = 0.0;
      for (int l = c + lane; l < T; l += 64) d += col[l] * cj[l];
      double f = 2.0 * wave_sum_d(d) / vtv;
      for (int l = c + lane; l < T; l += 64) cj[l] -= f * col[l];
    }
    __syncthreads();
  }
  // back substitution, column by column
  for (int c = tid; c < nJ; c += kBigThreads) yv[c] = rhs[c];
  __syncthreads();
  for (int c = nJ - 1; c >= 0; c--) {
    double yc = yv[c] / diagR[c];
    __syncthreads();
    if (tid == 0) yv[c] = yc;
    const double *Rc = tile + (int64_t)c * T;
    for (int i = tid; i < c; i += kBigThreads) yv[i] -= Rc[i] * yc;
    __syncthreads();
  }
  for (int c = tid; c < nJ; c += kBigThreads) {
    double dj = a.dscale ? a.dscale[J[c]] : 1.0;
    a.mval[ps + c] = yv[c] * dj;
  }
}

// ------------------------------------------------------------------ adaptive SPAI
//
// Algorithm 1 with its augmentation loop, run on A^T: one block per row k of
// M.  Each round rebuilds the shadow of J_k, solves the least squares
// problem by Householder QR in global scratch, forms the residual, and (if
// it is above eps and rounds remain) scores the candidates from the columns
// of A over the residual's support by the univariate minimisation
// rho_j^2 = ||s||^2 - (s . a_j)^2 / ||a_j||^2 (a_j the whole row j of A),
// rounded to fp32; the candidates at or below the mean (summed in ascending
// j), ordered by (rho_j, j), join J_k up to beta of them.

constexpr int kAdThreads = 256;
constexpr int kAdCand = 8192;    // candidate entries per round (LDS)
constexpr int kAdShadow = 4096;  // shadow rows (LDS)
constexpr int kAdJ = 64;         // pattern entries per row of M

struct AdaptiveArgs {
  int n, alpha, beta, jmax;
  double eps;
  const double *dscale;         // column scaling of A^T (null: none)
  const int32_t *arp, *acol;
  const double *aval;
  const int32_t *atrp, *atcol;  // pattern of A^T (columns of A)
  const int32_t *j0rp, *j0col;  // initial pattern (null: identity)
  const double *rownorm2;       // sum of a_jl^2 over row j of A, in CSR order
  const int32_t *rows;          // rows of this batch
  double *tiles, *rhs;          // per block: kAdShadow * jmax and kAdShadow doubles
  int32_t *cnt, *cols, *steps;
  double *vals;
  int32_t *err;                 // [0] zero row, [1] rank, [2] limits, [3] u_f overflow: smallest row
};

// Sum over the block (kBigThreads) in the construction precision T: FP64 as
// block_sum_big; fp32 and fp16 as wavefront trees, then the waves in order,
// every addition rounded to T.
template <typename T>
__device__ __forceinline__ T block_sum_t(T v, double *sh) {
  if constexpr (sizeof(T) == 8) {
    return block_sum_big(v, sh);
  } else {
    v = wave_sum_t<T>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = (double)v;
    __syncthreads();
    T t = (T)sh[0];
    for (int w = 1; w < kBigThreads / 64; w++) t = (T)(t + (T)sh[w]);
    return t;
  }
}

__global__ void k_rownorm2(int n, const int32_t *rp, const double *v, double *out) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int e = rp[j]; e < rp[j + 1]; e++) s += v[e] * v[e];
  out[j] = s;
}

// ascending sort of len (a power of two) keys in LDS by the whole block
template <typename K>
__device__ void block_bitonic(K *S, int len) {
  for (int size = 2; size <= len; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < len / 2; t += kAdThreads) {
        int lo = 2 * stride * (t / stride) + (t % stride);
        int hi = lo + stride;
        bool up = ((lo & size) == 0);
        K x = S[lo], y = S[hi];
        if ((x > y) == up) {
          S[lo] = y;
          S[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// T: the construction precision u_f of the least squares solves (Section 4:
// double, single or half).  The tile holds a_{J_c, I_l} d_{J_c} rounded to
// T, the QR and back substitution round every operation to T, and
// M(k, J_c) = m_c d_{J_c} rounded to T; the residual and the candidate
// scores are formed in FP64 from the unscaled A and those values.  With
// T = double and no scaling this is the FP64 construction, operation for
// operation.
template <typename T>
__global__ void __launch_bounds__(kAdThreads) k_spai_adaptive(AdaptiveArgs a) {
  extern __shared__ double lds_a[];
  unsigned long long *key = reinterpret_cast<unsigned long long *>(lds_a);  // kAdCand
  int32_t *S = reinterpret_cast<int32_t *>(lds_a);                          // aliases key
  int32_t *I = reinterpret_cast<int32_t *>(lds_a + kAdCand);                // kAdShadow
  double *sv = lds_a + kAdCand + kAdShadow / 2;                             // kAdShadow
  __shared__ int32_t J[kAdJ], off[kAdJ + 1];
  __shared__ T yv[kAdJ], diagR[kAdJ];
  __shared__ double md[kAdJ];  // M(k, J): the solution rounded to T, in FP64
  __shared__ double sh[kAdThreads / 64];
  __shared__ int s_n, s_nI, s_kpos, s_nJ, s_done, s_nsolve;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = a.rows[blockIdx.x];
  // the scratch tile: T values for the least squares, FP64 for the residual
  double *tiled = a.tiles + (int64_t)blockIdx.x * kAdShadow * a.jmax;
  T *tile = reinterpret_cast<T *>(tiled);
  T *rhs = reinterpret_cast<T *>(a.rhs + (int64_t)blockIdx.x * kAdShadow);
  auto fail_row = [&](int slot) {
    if (tid == 0) atomicMin(&a.err[slot], k);
  };
  if (tid == 0) {
    int nJ = 0;
    if (a.j0rp) {
      for (int e = a.j0rp[k]; e < a.j0rp[k + 1] && nJ < a.jmax; e++) {
        int v = a.j0col[e], p = nJ++;  // insertion sort
        while (p > 0 && J[p - 1] > v) J[p] = J[p - 1], p--;
        J[p] = v;
      }
    } else {
      J[nJ++] = k;
    }
    s_nJ = nJ;
    s_nsolve = 0;
  }
  __syncthreads();
  for (int step = 0; step <= a.alpha; step++) {
    const int nJ = s_nJ;
    // ---- shadow: the nonzero columns of the rows J of A, sorted, unique
    if (tid == 0) {
      int o = 0;
      for (int c = 0; c < nJ; c++) {
        off[c] = o;
        o += a.arp[J[c] + 1] - a.arp[J[c]];
      }
      off[nJ] = o;
      s_n = o;
    }
    __syncthreads();
    const int nc = s_n;
    if (nc > kAdCand) return fail_row(2);
    for (int c = tid; c < nJ; c += kAdThreads) {
      int o = off[c];
      for (int p = a.arp[J[c]]; p < a.arp[J[c] + 1]; p++) S[o++] = a.aval[p] != 0.0 ? a.acol[p] : INT_MAX;
    }
    int P2 = 1;
    while (P2 < nc) P2 <<= 1;
    __syncthreads();
    for (int p = nc + tid; p < P2; p += kAdThreads) S[p] = INT_MAX;
    __syncthreads();
    block_bitonic<int32_t>(S, P2);
    if (w == 0) {  // compaction of the distinct indices by one wavefront
      int cntI = 0;
      for (int b0 = 0; b0 < nc; b0 += 64) {
        int p = b0 + lane;
        int v = p < nc ? S[p] : INT_MAX;
        bool keep = v != INT_MAX && (p == 0 || S[p - 1] != v);
        unsigned long long m = __ballot(keep);
        int pos = cntI + __popcll(m & ((1ull << lane) - 1ull));
        if (keep && pos < kAdShadow) I[pos] = v;
        cntI += __popcll(m);
      }
      if (lane == 0) s_nI = cntI;
    }
    __syncthreads();
    const int nI = s_nI;
    if (nI > kAdShadow) return fail_row(2);
    if (tid == 0) {
      int p = lower_bound_i(I, nI, k);
      s_kpos = (p < nI && I[p] == k) ? p : -1;
    }
    __syncthreads();
    const int kpos = s_kpos;
    if (kpos < 0) return fail_row(0);
    if (nI < nJ) return fail_row(1);
    // ---- tile A(J, I)^T in scratch, column c = row J[c] of A: for the least
    // squares scaled and rounded to T, for the residual the FP64 values
    auto scatter_t = [&]() {
      for (int64_t p = tid; p < (int64_t)nI * nJ; p += kAdThreads) tile[p] = (T)0;
      __syncthreads();
      for (int c = tid; c < nJ; c += kAdThreads) {
        const double dj = a.dscale ? a.dscale[J[c]] : 1.0;
        for (int p = a.arp[J[c]]; p < a.arp[J[c] + 1]; p++)
          if (a.aval[p] != 0.0) tile[lower_bound_i(I, nI, a.acol[p]) + (int64_t)c * nI] = (T)(a.aval[p] * dj);
      }
      __syncthreads();
    };
    auto scatter_d = [&]() {
      for (int64_t p = tid; p < (int64_t)nI * nJ; p += kAdThreads) tiled[p] = 0.0;
      __syncthreads();
      for (int c = tid; c < nJ; c += kAdThreads)
        for (int p = a.arp[J[c]]; p < a.arp[J[c] + 1]; p++)
          if (a.aval[p] != 0.0) tiled[lower_bound_i(I, nI, a.acol[p]) + (int64_t)c * nI] = a.aval[p];
      __syncthreads();
    };
    scatter_t();
    for (int l = tid; l < nI; l += kAdThreads) rhs[l] = (l == kpos) ? (T)1 : (T)0;
    T fl = (T)0;
    for (int64_t p = tid; p < (int64_t)nI * nJ; p += kAdThreads) fl = fl + tile[p] * tile[p];
    const T fro = sqrt_t<T>(block_sum_t<T>(fl, sh));
    if (!isfinite((double)fro)) return fail_row(3);
    for (int c = 0; c < nJ; c++) {
      T *col = tile + (int64_t)c * nI;
      T s2 = (T)0;
      for (int l = c + tid; l < nI; l += kAdThreads) s2 = s2 + col[l] * col[l];
      T nrm = sqrt_t<T>(block_sum_t<T>(s2, sh));
      T al = col[c];
      T be = (T)(-copysign((double)nrm, (double)al));
      if (nrm == (T)0 || fabs((double)be) <= (double)nJ * unit_roundoff_t<T>() * (double)fro) return fail_row(1);
      __syncthreads();
      if (tid == 0) {
        col[c] = al - be;
        diagR[c] = be;
      }
      __syncthreads();
      T vt = (T)0;
      for (int l = c + tid; l < nI; l += kAdThreads) vt = vt + col[l] * col[l];
      const T vtv = block_sum_t<T>(vt, sh);
      for (int jj = c + 1 + w; jj <= nJ; jj += kAdThreads / 64) {
        T *cj = (jj < nJ) ? tile + (int64_t)jj * nI : rhs;
        T d = (T)0;
        for (int l = c + lane; l < nI; l += 64) d = d + col[l] * cj[l];
        T f = (T)2 * wave_sum_t<T>(d) / vtv;
        for (int l = c + lane; l < nI; l += 64) cj[l] = cj[l] - f * col[l];
      }
      __syncthreads();
    }
    for (int c = tid; c < nJ; c += kAdThreads) yv[c] = rhs[c];
    __syncthreads();
    for (int c = nJ - 1; c >= 0; c--) {
      T yc = yv[c] / diagR[c];
      __syncthreads();
      if (tid == 0) yv[c] = yc;
      const T *Rc = tile + (int64_t)c * nI;
      for (int i = tid; i < c; i += kAdThreads) yv[i] = yv[i] - Rc[i] * yc;
      __syncthreads();
    }
    for (int c = tid; c < nJ; c += kAdThreads) {
      const double dj = a.dscale ? a.dscale[J[c]] : 1.0;
      md[c] = (double)(T)((double)yv[c] * dj);
    }
    if (tid == 0) s_nsolve++;
    __syncthreads();
    // ---- residual s = Abar m - e_k on the shadow (FP64 tile rebuilt)
    scatter_d();
    double q2 = 0.0;
    for (int l = tid; l < nI; l += kAdThreads) {
      double t = 0.0;
      for (int c = 0; c < nJ; c++) t += tiled[l + (int64_t)c * nI] * md[c];
      t -= (l == kpos) ? 1.0 : 0.0;
      sv[l] = t;
      q2 += t * t;
    }
    const double ns2 = block_sum_big(q2, sh);
    if (tid == 0) s_done = (sqrt(ns2) <= a.eps || step == a.alpha) ? 1 : 0;
    __syncthreads();
    if (s_done) break;
    // ---- candidates: columns l of A over the residual's support, minus J
    if (tid == 0) s_n = 0;
    __syncthreads();
    for (int l = tid; l < nI; l += kAdThreads) {
      if (!(fabs(sv[l]) > 0x1p-40)) continue;  // rounding noise of an exact fit counts as zero
      const int i = I[l];
      const int len = a.atrp[i + 1] - a.atrp[i];
      int o = atomicAdd(&s_n, len);
      for (int e = 0; e < len && o + e < kAdCand; e++) S[o + e] = a.atcol[a.atrp[i] + e];
    }
    __syncthreads();
    const int ncand = s_n;
    if (ncand > kAdCand) return fail_row(2);
    P2 = 1;
    while (P2 < ncand) P2 <<= 1;
    for (int p = ncand + tid; p < P2; p += kAdThreads) S[p] = INT_MAX;
    __syncthreads();
    block_bitonic<int32_t>(S, P2);
    // distinct candidates not in J, ascending, moved to the upper half of the
    // key area as int32 (keys are written below them)
    int32_t *C = S + kAdCand;  // second half of the 64-bit key array, as ints
    if (w == 0) {
      int nC = 0;
      for (int b0 = 0; b0 < ncand; b0 += 64) {
        int p = b0 + lane;
        int v = p < ncand ? S[p] : INT_MAX;
        bool keep = v != INT_MAX && (p == 0 || S[p - 1] != v);
        if (keep) {
          for (int c = 0; c < nJ; c++) keep = keep && (J[c] != v);
        }
        unsigned long long m = __ballot(keep);
        int pos = nC + __popcll(m & ((1ull << lane) - 1ull));
        if (keep && pos < kAdCand / 2) C[pos] = v;  // C and rho share the upper half
        nC += __popcll(m);
      }
      if (lane == 0) s_n = nC;
    }
    __syncthreads();
    const int nC = s_n;
    if (nC > kAdCand / 2) return fail_row(2);
    // rho_j rounded to fp32, kept as its bit pattern beside j
    float *rho = reinterpret_cast<float *>(C + nC);
    for (int t = tid; t < nC; t += kAdThreads) {
      const int j = C[t];
      double dot = 0.0;
      for (int e = a.arp[j]; e < a.arp[j + 1]; e++) {
        int p = lower_bound_i(I, nI, a.acol[e]);
        if (p < nI && I[p] == a.acol[e]) dot += sv[p] * a.aval[e];
      }
      const double nrm = a.rownorm2[j];
      const double r2 = nrm > 0.0 ? ns2 - dot * dot / nrm : ns2;
      rho[t] = (float)sqrt(r2 > 0.0 ? r2 : 0.0);
    }
    __syncthreads();
    if (tid == 0) {  // mean over the candidates, ascending j, in FP64
      double sum = 0.0;
      for (int t = 0; t < nC; t++) sum += (double)rho[t];
      sh[0] = nC > 0 ? sum / nC : 0.0;
      s_n = 0;
    }
    __syncthreads();
    const double mean = sh[0];
    __syncthreads();
    // acceptable candidates as 64-bit keys (rho bits, j) in the lower half
    for (int t = tid; t < nC; t += kAdThreads) {
      if ((double)rho[t] <= mean) {
        int o = atomicAdd(&s_n, 1);
        key[o] = ((unsigned long long)__float_as_uint(rho[t]) << 32) | (unsigned)C[t];
      }
    }
    __syncthreads();
    const int nacc = s_n;
    int P = 1;
    while (P < nacc) P <<= 1;
    for (int p = nacc + tid; p < P; p += kAdThreads) key[p] = ~0ull;
    __syncthreads();
    block_bitonic<unsigned long long>(key, P);
    if (tid == 0) {
      int add = nacc < a.beta ? nacc : a.beta;
      if (add > a.jmax - nJ) add = a.jmax - nJ;
      int cntJ = nJ;
      for (int t = 0; t < add; t++) {
        int v = (int)(key[t] & 0xFFFFFFFFull), p = cntJ++;
        while (p > 0 && J[p - 1] > v) J[p] = J[p - 1], p--;
        J[p] = v;
      }
      s_nJ = cntJ;
      s_done = add == 0;
    }
    __syncthreads();
    if (s_done) break;
  }
  // the last solve belongs to the final J (a round that added entries always
  // solves again before it can end)
  const int nJ = s_nJ;
  for (int c = tid; c < nJ; c += kAdThreads) {
    a.cols[(int64_t)k * a.jmax + c] = J[c];
    a.vals[(int64_t)k * a.jmax + c] = md[c];
  }
  if (tid == 0) {
    a.cnt[k] = nJ;
    a.steps[k] = s_nsolve;
  }
}

// ------------------------------------------------------------------ buckets

// ||M||_inf: each row summed left to right in CSR order; the maximum of the
// (non-negative) row sums and of |m| via integer max on their bit patterns.
__global__ void k_row_abs(int n, const int32_t *rp, const double *v, unsigned long long *mx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0, m = 0;
  for (int p = rp[i]; p < rp[i + 1]; p++) {
    s += fabs(v[p]);
    m = fmax(m, fabs(v[p]));
  }
  atomicMax(&mx[0], (unsigned long long)__double_as_longlong(s));
  atomicMax(&mx[1], (unsigned long long)__double_as_longlong(m));
}

struct BucketArgs {
  int n, q;
  int prec[kMaxBuckets];
  double t[kMaxBuckets];
  double inv_scale[kMaxBuckets];
  double scale[kMaxBuckets];
  const int32_t *rp, *col;
  const double *v;
  int8_t *bid;
  double *stored;
  int32_t *cnt;  // [q][n]
  int32_t *brp[kMaxBuckets];
  int32_t *bcol[kMaxBuckets];
  void *bval[kMaxBuckets];
};

// Algorithm 2 / eq. (nint): bucket 1 if |m| > t_2, bucket q if |m| <= t_q,
// otherwise the k with t_{k+1} < |m| <= t_k.
__device__ __forceinline__ int classify(const BucketArgs &a, double m) {
  double x = fabs(m);
  if (a.q == 1) return 0;
  if (x > a.t[1]) return 0;
  if (x <= a.t[a.q - 1]) return a.q - 1;
  for (int k = 1; k <= a.q - 2; k++)
    if (x > a.t[k + 1] && x <= a.t[k]) return k;
  return a.q - 1;
}

__global__ void k_classify(BucketArgs a) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  int c[kMaxBuckets] = {0, 0, 0, 0, 0, 0};
  for (int p = a.rp[i]; p < a.rp[i + 1]; p++) {
    int k = classify(a, a.v[p]);
    a.bid[p] = (int8_t)k;
    c[k]++;
  }
  for (int k = 0; k < a.q; k++) a.cnt[(int64_t)k * a.n + i] = c[k];
}

__global__ void k_pack(BucketArgs a) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  int pos[kMaxBuckets];
  for (int k = 0; k < a.q; k++) pos[k] = a.brp[k] ? a.brp[k][i] : 0;
  for (int p = a.rp[i]; p < a.rp[i + 1]; p++) {
    int k = a.bid[p];
    double m = a.v[p];
    double y = m * a.inv_scale[k];  // exact: power-of-two scale
    double st = 0.0;
    switch (a.prec[k]) {
      case BSPAI_FP64:
        static_cast<double *>(a.bval[k])[pos[k]] = m;
        st = m;
        break;
      case BSPAI_FP32: {
        float f = encode_f32(y);
        static_cast<float *>(a.bval[k])[pos[k]] = f;
        st = (double)f * a.scale[k];
      } break;
      case BSPAI_FP16: {
        uint16_t h = encode_f16(y);
        static_cast<uint16_t *>(a.bval[k])[pos[k]] = h;
        st = (double)decode_f16(h) * a.scale[k];
      } break;
      case BSPAI_BF16: {
        uint16_t h = encode_bf16(y);
        static_cast<uint16_t *>(a.bval[k])[pos[k]] = h;
        st = (double)decode_bf16(h) * a.scale[k];
      } break;
      case BSPAI_FP8_E4M3: {
        uint8_t h = encode_e4m3(y);
        static_cast<uint8_t *>(a.bval[k])[pos[k]] = h;
        st = (double)decode_e4m3(h) * a.scale[k];
      } break;
      default:  // dropped
        break;
    }
    if (a.prec[k] != BSPAI_DROP) {
      a.bcol[k][pos[k]] = a.col[p];
      pos[k]++;
    }
    a.stored[p] = st;
  }
}

static int ceil_log2(double t) {
  int e;
  double f = frexp(t, &e);
  return (f == 0.5) ? e - 1 : e;
}

static unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

static int check_precs(const bspai_prec *precs, int q) {
  if (!precs || q < 1 || q > kMaxBuckets) return fail(BSPAI_EINVAL, "precision set: need 1 <= q <= 6");
  for (int k = 0; k < q; k++)
    if (precs[k] < BSPAI_FP64 || precs[k] > BSPAI_DROP) return fail(BSPAI_EINVAL, "precision %d unknown", precs[k]);
  for (int k = 1; k < q; k++)
    if (!(unit_roundoff(precs[k - 1]) < unit_roundoff(precs[k])))
      return fail(BSPAI_EINVAL, "precisions must have strictly increasing unit roundoff (got %d before %d)",
                  precs[k - 1], precs[k]);
  for (int k = 0; k + 1 < q; k++)
    if (precs[k] == BSPAI_DROP) return fail(BSPAI_EINVAL, "DROP must be the last precision");
  if (precs[0] == BSPAI_DROP) return fail(BSPAI_EINVAL, "the first bucket cannot be DROP");
  return BSPAI_OK;
}

static int check_csr(const char *what, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col) {
  if (n < 0 || nnz < 0 || nnz > INT32_MAX) return fail(BSPAI_EINVAL, "%s: bad sizes n=%d nnz=%lld", what, n, (long long)nnz);
  if (n > 0 && (!rp || (nnz > 0 && !col))) return fail(BSPAI_EINVAL, "%s: null pointer", what);
  return BSPAI_OK;
}

static void free_handle_memory(bspai_handle *h) {
  for (int k = 0; k < kMaxBuckets; k++) {
    dfree(h->b[k].rp), dfree(h->b[k].col), dfree(h->b[k].val);
    dfree(h->b[k].rpT), dfree(h->b[k].colT), dfree(h->b[k].valT);
    dfree(h->b[k].sptr), dfree(h->b[k].scol), dfree(h->b[k].sval);
    dfree(h->b[k].sptrT), dfree(h->b[k].scolT), dfree(h->b[k].svalT);
    dfree(h->b[k].ecol), dfree(h->b[k].eval), dfree(h->b[k].ecolT), dfree(h->b[k].evalT);
    dfree(h->b[k].ecode), dfree(h->b[k].ecodeT), dfree(h->b[k].edict), dfree(h->b[k].edictT);
  }
  dfree(h->m_rp), dfree(h->m_col), dfree(h->m_val);
  dfree(h->mT_rp), dfree(h->mT_col), dfree(h->mT_val);
  dfree(h->bucket_id), dfree(h->stored);
  dfree(h->seg_rows), dfree(h->seg_rowsT);
}

// Buckets, packing and (optionally) transposed packing of h->m_* (FP64 M).
static int bucketize(bspai_handle *h, const bspai_prec *precs, int q, double eps, const bspai_opts &o,
                     hipStream_t s) {
  const int n = h->n;
  const int64_t nnz = h->nnz;
  h->q = q;
  h->eps = eps;
  for (int k = 0; k < q; k++) h->precs[k] = precs[k];
  unsigned long long *mx = nullptr;
  int rc;
  if ((rc = dalloc_t(&mx, 2))) return rc;
  unsigned long long hm[2] = {0, 0};
  BSPAI_HIP(hipMemsetAsync(mx, 0, sizeof(hm), s));
  if (n > 0) {
    hipLaunchKernelGGL(k_row_abs, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, h->m_rp, h->m_val, mx);
    BSPAI_CHECK_LAUNCH();
  }
  BSPAI_HIP(hipMemcpyAsync(hm, mx, sizeof(hm), hipMemcpyDeviceToHost, s));
  BSPAI_HIP(hipStreamSynchronize(s));
  dfree(mx);
  double normM, maxabs;
  memcpy(&normM, &hm[0], 8);
  memcpy(&maxabs, &hm[1], 8);
  h->normM = normM;
  BucketArgs a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.q = q;
  const double base = eps * normM;
  for (int k = 0; k < q; k++) {
    a.prec[k] = precs[k];
    a.t[k] = base / unit_roundoff(precs[k]);
    double tk = (k == 0) ? maxabs : a.t[k];
    double sc = 1.0;
    if ((precs[k] == BSPAI_FP16 || precs[k] == BSPAI_FP8_E4M3) && tk > 0)
      sc = ldexp(1.0, ceil_log2(tk) - (precs[k] == BSPAI_FP16 ? 15 : 8));
    a.scale[k] = sc;
    a.inv_scale[k] = 1.0 / sc;
    h->b[k].prec = precs[k];
    h->b[k].t = a.t[k];
    h->b[k].scale = sc;
  }
  a.rp = h->m_rp;
  a.col = h->m_col;
  a.v = h->m_val;
  if ((rc = dalloc_t(&h->bucket_id, (size_t)nnz + 1)) || (rc = dalloc_t(&h->stored, (size_t)nnz + 1))) return rc;
  a.bid = h->bucket_id;
  a.stored = h->stored;
  int32_t *cnt = nullptr;
  void *tmp = nullptr;
  if ((rc = dalloc_t(&cnt, (size_t)q * n + 1)) || (rc = dalloc(&tmp, scan_tmp_bytes(n)))) {
    dfree(cnt), dfree(tmp);
    return rc;
  }
  auto body = [&]() -> int {
    a.cnt = cnt;
    if (n > 0) {
      hipLaunchKernelGGL(k_classify, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
      BSPAI_CHECK_LAUNCH();
    }
    for (int k = 0; k < q; k++) {
      int32_t *rp = nullptr;
      int r;
      if ((r = dalloc_t(&rp, (size_t)n + 1))) return r;
      h->b[k].rp = rp;
      if ((r = exclusive_scan(cnt + (int64_t)k * n, rp, n, tmp, s))) return r;
      int32_t tot = 0;
      BSPAI_HIP(hipMemcpyAsync(&tot, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      BSPAI_HIP(hipStreamSynchronize(s));
      h->b[k].nnz = tot;
      if (precs[k] != BSPAI_DROP) {
        if ((r = dalloc_t(&h->b[k].col, (size_t)tot + 1))) return r;
        if ((r = dalloc(&h->b[k].val, (size_t)value_bytes(precs[k]) * (tot + 1)))) return r;
        a.brp[k] = rp;
        a.bcol[k] = h->b[k].col;
        a.bval[k] = h->b[k].val;
      }
    }
    if (n > 0) {
      hipLaunchKernelGGL(k_pack, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
      BSPAI_CHECK_LAUNCH();
    }
    BSPAI_HIP(hipStreamSynchronize(s));
    return BSPAI_OK;
  };
  rc = body();
  dfree(cnt), dfree(tmp);
  if (rc) return rc;
  // kernel view: stored buckets from the least to the most precise
  BMat &M = h->mat;
  memset(&M, 0, sizeof(M));
  M.n = n;
  for (int k = q - 1; k >= 0; k--) {
    if (precs[k] == BSPAI_DROP || h->b[k].nnz == 0) continue;
    M.prec[M.nb] = precs[k];
    M.scale[M.nb] = h->b[k].scale;
    M.rp[M.nb] = h->b[k].rp;
    M.col[M.nb] = h->b[k].col;
    M.val[M.nb] = h->b[k].val;
    M.nnz += h->b[k].nnz;
    M.nb++;
  }
  M.lanes = pick_lanes(M, M.nnz);
  M.aligned = bmat_aligned(M);
  {  // SELL-64 copies of the stored buckets for the products
    int j = 0;
    for (int k = q - 1; k >= 0; k--) {
      if (precs[k] == BSPAI_DROP || h->b[k].nnz == 0) continue;
      Bucket &B = h->b[k];
      int32_t w = 0;
      int r = csr_to_sell(n, B.rp, B.col, B.val, value_bytes(B.prec), &B.sptr, &B.scol, &B.sval, &w, s);
      if (r) return r;
      M.sell_w[j] = w;
      if ((r = csr_to_ell(n, B.rp, B.col, B.val, value_bytes(B.prec), &B.ecol, &B.eval, &w, s))) return r;
      if (w && (r = ell_codes(n, w, B.ecol, &B.ecode, &B.edict, &B.ecw, s))) return r;
      if (B.ecw) {  // the codes replace the int32 columns
        dfree(B.ecol);
        B.ecol = nullptr;
      }
      M.ell_w[j] = w;
      M.ell_col[j] = B.ecol;
      M.ell_val[j] = B.eval;
      M.ell_code[j] = B.ecode;
      M.ell_dict[j] = B.edict;
      M.ell_cw[j] = B.ecw;
      M.sell_ptr[j] = B.sptr;
      M.sell_col[j] = B.scol;
      M.sell_val[j] = B.sval;
      j++;
    }
  }
  if (o.build_T) {
    BMat &T = h->matT;
    T = M;
    int j = 0;
    for (int k = q - 1; k >= 0; k--) {
      if (precs[k] == BSPAI_DROP || h->b[k].nnz == 0) continue;
      Bucket &B = h->b[k];
      int r;
      if ((r = dalloc_t(&B.rpT, (size_t)n + 1)) || (r = dalloc_t(&B.colT, (size_t)B.nnz + 1)) ||
          (r = dalloc(&B.valT, (size_t)value_bytes(B.prec) * (B.nnz + 1))))
        return r;
      if ((r = csr_transpose(n, B.nnz, B.rp, B.col, B.val, value_bytes(B.prec), B.rpT, B.colT, B.valT, s))) return r;
      T.rp[j] = B.rpT;
      T.col[j] = B.colT;
      T.val[j] = B.valT;
      int32_t w = 0;
      if ((r = csr_to_sell(n, B.rpT, B.colT, B.valT, value_bytes(B.prec), &B.sptrT, &B.scolT, &B.svalT, &w, s)))
        return r;
      T.sell_w[j] = w;
      if ((r = csr_to_ell(n, B.rpT, B.colT, B.valT, value_bytes(B.prec), &B.ecolT, &B.evalT, &w, s))) return r;
      if (w && (r = ell_codes(n, w, B.ecolT, &B.ecodeT, &B.edictT, &B.ecwT, s))) return r;
      if (B.ecwT) {
        dfree(B.ecolT);
        B.ecolT = nullptr;
      }
      T.ell_w[j] = w;
      T.ell_col[j] = B.ecolT;
      T.ell_val[j] = B.evalT;
      T.ell_code[j] = B.ecodeT;
      T.ell_dict[j] = B.edictT;
      T.ell_cw[j] = B.ecwT;
      T.sell_ptr[j] = B.sptrT;
      T.sell_col[j] = B.scolT;
      T.sell_val[j] = B.svalT;
      j++;
    }
    T.aligned = bmat_aligned(T);
    if (h->has_fp64) {
      int r;
      if ((r = dalloc_t(&h->mT_rp, (size_t)n + 1)) || (r = dalloc_t(&h->mT_col, (size_t)nnz + 1)) ||
          (r = dalloc_t(&h->mT_val, (size_t)nnz + 1)))
        return r;
      if ((r = csr_transpose(n, nnz, h->m_rp, h->m_col, h->m_val, 8, h->mT_rp, h->mT_col, h->mT_val, s))) return r;
    }
    h->has_T = 1;
  }
  {  // entry-balanced tile plans for the segmented product (after matT copied mat)
    int r;
    if ((r = build_seg_plan(h->mat, &h->seg_rows, s))) return r;
    if (h->has_T && (r = build_seg_plan(h->matT, &h->seg_rowsT, s))) return r;
  }
  return BSPAI_OK;
}

static bspai_opts default_opts() {
  bspai_opts o;
  o.build_T = 1;
  o.keep_fp64_M = 1;
  o.scale = 0;
  o.u_f = BSPAI_FP64;
  return o;
}

static int finish_build(bspai_handle *h, const bspai_prec *precs, int q, double eps, const bspai_opts &o,
                        hipStream_t s, bspai_handle **out) {
  h->has_fp64 = 1;  // the FP64 M is needed while packing; dropped below unless kept
  int rc = bucketize(h, precs, q, eps, o, s);
  if (rc) {
    free_handle_memory(h);
    delete h;
    return rc;
  }
  if (!o.keep_fp64_M) {
    (void)hipStreamSynchronize(s);
    dfree(h->m_val);
    h->m_val = nullptr;
    dfree(h->mT_val);
    h->mT_val = nullptr;
    h->has_fp64 = 0;
  }
  *out = h;
  return BSPAI_OK;
}

}  // namespace bspai

using namespace bspai;

extern "C" int bspai_build(const bspai_csr *A, const bspai_pattern *P, double eps_b, const bspai_prec *precs, int q,
                           const bspai_opts *opts, bspai_handle **out, void *stream) {
  if (!out) return fail(BSPAI_EINVAL, "bspai_build: null output");
  *out = nullptr;
  if (!A) return fail(BSPAI_EINVAL, "bspai_build: null A");
  int rc;
  if ((rc = check_csr("A", A->n, A->nnz, A->row_ptr, A->col))) return rc;
  if (A->n > 0 && A->nnz > 0 && !A->val) return fail(BSPAI_EINVAL, "A: null values");
  bspai_pattern Pd;
  if (P) {
    Pd = *P;
    if (Pd.n != A->n) return fail(BSPAI_EINVAL, "pattern size %d != n %d", Pd.n, A->n);
    if ((rc = check_csr("P", Pd.n, Pd.nnz, Pd.row_ptr, Pd.col))) return rc;
  } else {
    Pd.n = A->n;
    Pd.nnz = A->nnz;
    Pd.row_ptr = A->row_ptr;
    Pd.col = A->col;
  }
  if ((rc = check_precs(precs, q))) return rc;
  if (!(eps_b >= 0) || !std::isfinite(eps_b)) return fail(BSPAI_EINVAL, "eps_b must be finite and >= 0");
  bspai_opts o = opts ? *opts : default_opts();
  if (o.u_f != BSPAI_FP64 && o.u_f != BSPAI_FP32 && o.u_f != BSPAI_FP16)
    return fail(BSPAI_EINVAL, "bspai_build: u_f must be FP64, FP32 or FP16");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = A->n;
  bspai_handle *h = new bspai_handle();
  BSPAI_HIP(hipGetDevice(&h->device));
  h->n = n;
  h->nnz = Pd.nnz;
  int32_t *mx = nullptr, *err = nullptr, *biglist = nullptr, *candof = nullptr;
  int8_t *isbig = nullptr;
  double *dsc = nullptr, *tiles = nullptr, *rhsb = nullptr;
  int64_t *offs = nullptr;
  int32_t *brows = nullptr;
  int nbig = 0;
  auto body = [&]() -> int {
    int r;
    if ((r = dalloc_t(&h->m_rp, (size_t)n + 1)) || (r = dalloc_t(&h->m_col, (size_t)Pd.nnz + 1)) ||
        (r = dalloc_t(&h->m_val, (size_t)Pd.nnz + 1)))
      return r;
    BSPAI_HIP(hipMemcpyAsync(h->m_rp, Pd.row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (Pd.nnz) BSPAI_HIP(hipMemcpyAsync(h->m_col, Pd.col, sizeof(int32_t) * Pd.nnz, hipMemcpyDeviceToDevice, s));
    if (n == 0) return BSPAI_OK;
    if ((r = dalloc_t(&mx, 5)) || (r = dalloc_t(&err, 4)) || (r = dalloc_t(&isbig, (size_t)n)) ||
        (r = dalloc_t(&biglist, (size_t)n)) || (r = dalloc_t(&candof, (size_t)n)))
      return r;
    int32_t hmx[5] = {0, 0, 0, 0, 0};
    BSPAI_HIP(hipMemsetAsync(mx, 0, sizeof(hmx), s));
    hipLaunchKernelGGL(k_spai_sizes, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, A->row_ptr, Pd.row_ptr, Pd.col,
                       mx, isbig, biglist, mx + 4, candof);
    BSPAI_CHECK_LAUNCH();
    BSPAI_HIP(hipMemcpyAsync(hmx, mx, sizeof(hmx), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    int nJmax = hmx[0], candmax = hmx[1];
    nbig = hmx[4];
    if (nbig > 0 && o.u_f != BSPAI_FP64)
      return fail(BSPAI_EINVAL, "bspai_build: u_f below FP64 covers rows whose least squares fit one wavefront "
                                "(|J| <= %d, <= %d shadow candidates, tile <= %d values); %d rows need more",
                  kSmallJ, kSmallCand, kSmallTile, nbig);
    int cand_p2 = 64;
    while (cand_p2 < candmax) cand_p2 <<= 1;
    // the maxima may come from different rows; no row of this path exceeds kSmallTile
    int64_t tile = std::min<int64_t>((int64_t)std::max(candmax, 1) * std::max(nJmax, 1), kSmallTile);
    size_t lds = sizeof(double) * ((size_t)cand_p2 /* two int lists */ + tile + cand_p2 + 64 + 64 + 64);
    if (o.scale) {
      if ((r = dalloc_t(&dsc, (size_t)n))) return r;
      hipLaunchKernelGGL(k_row_maxabs_inv, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, A->row_ptr, A->val, dsc);
      BSPAI_CHECK_LAUNCH();
    }
    int32_t herr[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    BSPAI_HIP(hipMemcpyAsync(err, herr, sizeof(herr), hipMemcpyHostToDevice, s));
    SpaiArgs sa;
    sa.n = n;
    sa.arp = A->row_ptr;
    sa.acol = A->col;
    sa.aval = A->val;
    sa.prp = Pd.row_ptr;
    sa.pcol = Pd.col;
    sa.dscale = dsc;
    sa.mval = h->m_val;
    sa.cand_p2 = cand_p2;
    sa.tile_cap = (int)tile;
    sa.err = err;
    sa.is_big = isbig;
    if (nbig < n) {
      const void *fn = o.u_f == BSPAI_FP32   ? (const void *)k_spai<float>
                       : o.u_f == BSPAI_FP16 ? (const void *)k_spai<_Float16>
                                             : (const void *)k_spai<double>;
      if (lds > 64 * 1024) BSPAI_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      if (o.u_f == BSPAI_FP32) hipLaunchKernelGGL(k_spai<float>, dim3(n), dim3(64), lds, s, sa);
      else if (o.u_f == BSPAI_FP16) hipLaunchKernelGGL(k_spai<_Float16>, dim3(n), dim3(64), lds, s, sa);
      else hipLaunchKernelGGL(k_spai<double>, dim3(n), dim3(64), lds, s, sa);
      BSPAI_CHECK_LAUNCH();
    }
    if (nbig > 0) {
      // rows left to the block path, in batches whose tiles fit a scratch budget
      std::vector<int32_t> hb(nbig), hcand(n), hprp(n + 1);
      BSPAI_HIP(hipMemcpyAsync(hb.data(), biglist, sizeof(int32_t) * nbig, hipMemcpyDeviceToHost, s));
      BSPAI_HIP(hipMemcpyAsync(hcand.data(), candof, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
      BSPAI_HIP(hipMemcpyAsync(hprp.data(), Pd.row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
      BSPAI_HIP(hipStreamSynchronize(s));
      std::sort(hb.begin(), hb.end());
      const int64_t budget = (int64_t)1 << 27;  // doubles of tile scratch per batch (1 GiB)
      int64_t cap_tiles = 0, cap_rhs = 0;
      std::vector<int64_t> toff, roff;
      std::vector<std::pair<int, int>> batches;  // [first, last) into hb
      {
        int first = 0;
        int64_t acc_t = 0, acc_r = 0;
        for (int b = 0; b < nbig; b++) {
          int k = hb[b];
          int64_t nJ = hprp[k + 1] - hprp[k];
          int64_t rows = hcand[k] / 2 + nJ + 1;  // multi rows <= candidates / 2, plus one folded row per column
          int64_t t = rows * nJ, rr = rows;
          if (b > first && (acc_t + t > budget || b - first >= 4096)) {
            batches.push_back({first, b});
            cap_tiles = std::max(cap_tiles, acc_t);
            cap_rhs = std::max(cap_rhs, acc_r);
            first = b;
            acc_t = acc_r = 0;
          }
          toff.push_back(acc_t);
          roff.push_back(acc_r);
          acc_t += t;
          acc_r += rr;
        }
        batches.push_back({first, nbig});
        cap_tiles = std::max(cap_tiles, acc_t);
        cap_rhs = std::max(cap_rhs, acc_r);
      }
      if ((r = dalloc_t(&tiles, (size_t)cap_tiles + 1)) || (r = dalloc_t(&rhsb, (size_t)cap_rhs + 1)) ||
          (r = dalloc_t(&offs, 2 * (size_t)std::min(nbig, 4096) + 2)) ||
          (r = dalloc_t(&brows, (size_t)std::min(nbig, 4096) + 1)))
        return r;
      const size_t lds_big = 8 * (size_t)kBigCand + 2 * 1024 * sizeof(double);
      BSPAI_HIP(hipFuncSetAttribute((const void *)k_spai_big, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds_big));
      for (auto &bt : batches) {
        int cnt = bt.second - bt.first;
        std::vector<int64_t> ho(2 * (size_t)cnt);
        for (int t = 0; t < cnt; t++) {
          ho[t] = toff[bt.first + t];
          ho[cnt + t] = roff[bt.first + t];
        }
        BSPAI_HIP(hipMemcpyAsync(brows, hb.data() + bt.first, sizeof(int32_t) * cnt, hipMemcpyHostToDevice, s));
        BSPAI_HIP(hipMemcpyAsync(offs, ho.data(), sizeof(int64_t) * 2 * cnt, hipMemcpyHostToDevice, s));
        SpaiBigArgs ba;
        ba.arp = A->row_ptr;
        ba.acol = A->col;
        ba.aval = A->val;
        ba.prp = Pd.row_ptr;
        ba.pcol = Pd.col;
        ba.dscale = dsc;
        ba.mval = h->m_val;
        ba.rows = brows;
        ba.tile_off = offs;
        ba.rhs_off = offs + cnt;
        ba.tiles = tiles;
        ba.rhs = rhsb;
        ba.err = err;
        hipLaunchKernelGGL(k_spai_big, dim3(cnt), dim3(kBigThreads), lds_big, s, ba);
        BSPAI_CHECK_LAUNCH();
        BSPAI_HIP(hipStreamSynchronize(s));  // host arrays above are reused per batch
      }
    }
    BSPAI_HIP(hipMemcpyAsync(herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    if (herr[2] != INT_MAX) return fail(BSPAI_EINVAL, "row %d: least-squares tile exceeds its capacity", herr[2]);
    if (herr[0] != INT_MAX || herr[1] != INT_MAX) {
      if (herr[0] < herr[1]) return fail(BSPAI_EZEROROW, "row %d of M is zero: %d is not in its shadow", herr[0], herr[0]);
      return fail(BSPAI_ERANK, "row %d: reduced least-squares problem is rank deficient", herr[1]);
    }
    if (herr[3] != INT_MAX)
      return fail(BSPAI_ENAN, "row %d: the least squares overflows u_f (the column scaling avoids this)", herr[3]);
    return BSPAI_OK;
  };
  rc = body();
  dfree(mx), dfree(err), dfree(dsc), dfree(isbig), dfree(biglist), dfree(candof);
  dfree(tiles), dfree(rhsb), dfree(offs), dfree(brows);
  if (rc) {
    free_handle_memory(h);
    delete h;
    return rc;
  }
  return finish_build(h, precs, q, eps_b, o, s, out);
}

extern "C" int bspai_import(const bspai_csr *M, double eps_b, const bspai_prec *precs, int q, const bspai_opts *opts,
                            bspai_handle **out, void *stream) {
  if (!out) return fail(BSPAI_EINVAL, "bspai_import: null output");
  *out = nullptr;
  if (!M) return fail(BSPAI_EINVAL, "bspai_import: null M");
  int rc;
  if ((rc = check_csr("M", M->n, M->nnz, M->row_ptr, M->col))) return rc;
  if (M->nnz > 0 && !M->val) return fail(BSPAI_EINVAL, "M: null values");
  if ((rc = check_precs(precs, q))) return rc;
  if (!(eps_b >= 0) || !std::isfinite(eps_b)) return fail(BSPAI_EINVAL, "eps_b must be finite and >= 0");
  bspai_opts o = opts ? *opts : default_opts();
  hipStream_t s = static_cast<hipStream_t>(stream);
  bspai_handle *h = new bspai_handle();
  BSPAI_HIP(hipGetDevice(&h->device));
  h->n = M->n;
  h->nnz = M->nnz;
  auto body = [&]() -> int {
    int r;
    if ((r = dalloc_t(&h->m_rp, (size_t)M->n + 1)) || (r = dalloc_t(&h->m_col, (size_t)M->nnz + 1)) ||
        (r = dalloc_t(&h->m_val, (size_t)M->nnz + 1)))
      return r;
    BSPAI_HIP(hipMemcpyAsync(h->m_rp, M->row_ptr, sizeof(int32_t) * (M->n + 1), hipMemcpyDeviceToDevice, s));
    if (M->nnz) {
      BSPAI_HIP(hipMemcpyAsync(h->m_col, M->col, sizeof(int32_t) * M->nnz, hipMemcpyDeviceToDevice, s));
      BSPAI_HIP(hipMemcpyAsync(h->m_val, M->val, sizeof(double) * M->nnz, hipMemcpyDeviceToDevice, s));
    }
    return BSPAI_OK;
  };
  rc = body();
  if (rc) {
    free_handle_memory(h);
    delete h;
    return rc;
  }
  return finish_build(h, precs, q, eps_b, o, s, out);
}

namespace bspai {
__global__ void k_iota(int n, int32_t *o) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = i;
}

// rows of width jmax (cnt[k] used) into CSR at rp
__global__ void k_compact_rows(int n, int jmax, const int32_t *cnt, const int32_t *cols, const double *vals,
                               const int32_t *rp, int32_t *col, double *val) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  for (int c = 0; c < cnt[k]; c++) {
    col[rp[k] + c] = cols[(int64_t)k * jmax + c];
    val[rp[k] + c] = vals[(int64_t)k * jmax + c];
  }
}
}  // namespace bspai

extern "C" int bspai_build_adaptive(const bspai_csr *A, const bspai_pattern *J0, const bspai_adaptive_opts *ad,
                                    double eps_b, const bspai_prec *precs, int q, const bspai_opts *opts,
                                    bspai_handle **out, int32_t *steps_host, void *stream) {
  using namespace bspai;
  if (!out) return fail(BSPAI_EINVAL, "bspai_build_adaptive: null output");
  *out = nullptr;
  if (!A || !ad) return fail(BSPAI_EINVAL, "bspai_build_adaptive: null argument");
  int rc;
  if ((rc = check_csr("A", A->n, A->nnz, A->row_ptr, A->col))) return rc;
  if (A->n < 1 || (A->nnz > 0 && !A->val)) return fail(BSPAI_EINVAL, "bspai_build_adaptive: empty A or null values");
  if (J0 && (rc = check_csr("J0", J0->n, J0->nnz, J0->row_ptr, J0->col))) return rc;
  if (J0 && J0->n != A->n) return fail(BSPAI_EINVAL, "bspai_build_adaptive: J0 is %d x %d, A %d x %d", J0->n, J0->n,
                                       A->n, A->n);
  if (ad->alpha < 0 || ad->beta < 0 || !(ad->eps >= 0) || !std::isfinite(ad->eps))
    return fail(BSPAI_EINVAL, "bspai_build_adaptive: need alpha >= 0, beta >= 0 and a finite eps >= 0");
  if ((rc = check_precs(precs, q))) return rc;
  if (!(eps_b >= 0) || !std::isfinite(eps_b)) return fail(BSPAI_EINVAL, "eps_b must be finite and >= 0");
  const int uf = opts ? (int)opts->u_f : (int)BSPAI_FP64;
  if (uf != BSPAI_FP64 && uf != BSPAI_FP32 && uf != BSPAI_FP16)
    return fail(BSPAI_EINVAL, "bspai_build_adaptive: u_f must be FP64, FP32 or FP16");
  const bool scale = opts && opts->scale;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = A->n;
  const int64_t nnz = A->nnz;
  int j0max = 1;
  if (J0) {
    std::vector<int32_t> h(n + 1);
    BSPAI_HIP(hipMemcpy(h.data(), J0->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    j0max = 0;
    for (int i = 0; i < n; i++) j0max = std::max(j0max, h[i + 1] - h[i]);
  }
  const int64_t jmax64 = (int64_t)j0max + (int64_t)ad->alpha * ad->beta;
  if (jmax64 > kAdJ)
    return fail(BSPAI_EINVAL, "bspai_build_adaptive: initial entries + alpha * beta = %lld exceeds %d per row",
                (long long)jmax64, kAdJ);
  const int jmax = (int)std::max<int64_t>(jmax64, 1);
  const int batch = std::min(n, 512);
  int32_t *trp = nullptr, *tcol = nullptr, *iota = nullptr, *cnt = nullptr, *cols = nullptr, *stp = nullptr,
          *err = nullptr, *mrp = nullptr, *mcol = nullptr;
  double *rn2 = nullptr, *vals = nullptr, *tiles = nullptr, *rhs = nullptr, *mval = nullptr, *dsc = nullptr;
  void *tmp = nullptr;
  auto body = [&]() -> int {
    int r;
    if ((r = dalloc_t(&trp, (size_t)n + 1)) || (r = dalloc_t(&tcol, (size_t)nnz + 1)) ||
        (r = dalloc_t(&iota, (size_t)n)) || (r = dalloc_t(&cnt, (size_t)n)) ||
        (r = dalloc_t(&cols, (size_t)n * jmax)) || (r = dalloc_t(&stp, (size_t)n)) || (r = dalloc_t(&err, 4)) ||
        (scale && (r = dalloc_t(&dsc, (size_t)n))) ||
        (r = dalloc_t(&rn2, (size_t)n)) || (r = dalloc_t(&vals, (size_t)n * jmax)) ||
        (r = dalloc_t(&tiles, (size_t)batch * kAdShadow * jmax)) || (r = dalloc_t(&rhs, (size_t)batch * kAdShadow)))
      return r;
    if ((r = csr_transpose(n, nnz, A->row_ptr, A->col, nullptr, 0, trp, tcol, nullptr, s))) return r;
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_rownorm2, dim3(g), dim3(256), 0, s, n, A->row_ptr, A->val, rn2);
    hipLaunchKernelGGL(k_iota, dim3(g), dim3(256), 0, s, n, iota);
    if (scale) hipLaunchKernelGGL(k_row_maxabs_inv, dim3(g), dim3(256), 0, s, n, A->row_ptr, A->val, dsc);
    BSPAI_CHECK_LAUNCH();
    BSPAI_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, s));
    const int32_t init[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
    BSPAI_HIP(hipMemcpyAsync(err, init, sizeof(init), hipMemcpyHostToDevice, s));
    const size_t lds = sizeof(double) * ((size_t)kAdCand + kAdShadow / 2 + kAdShadow);
    const void *kern = uf == BSPAI_FP32   ? (const void *)k_spai_adaptive<float>
                       : uf == BSPAI_FP16 ? (const void *)k_spai_adaptive<_Float16>
                                          : (const void *)k_spai_adaptive<double>;
    BSPAI_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    AdaptiveArgs a;
    a.n = n;
    a.alpha = ad->alpha;
    a.beta = ad->beta;
    a.jmax = jmax;
    a.eps = ad->eps;
    a.dscale = dsc;
    a.arp = A->row_ptr;
    a.acol = A->col;
    a.aval = A->val;
    a.atrp = trp;
    a.atcol = tcol;
    a.j0rp = J0 ? J0->row_ptr : nullptr;
    a.j0col = J0 ? J0->col : nullptr;
    a.rownorm2 = rn2;
    a.tiles = tiles;
    a.rhs = rhs;
    a.cnt = cnt;
    a.cols = cols;
    a.steps = stp;
    a.vals = vals;
    a.err = err;
    for (int r0 = 0; r0 < n; r0 += batch) {
      a.rows = iota + r0;
      const int nb = std::min(batch, n - r0);
      void *args[] = {&a};
      BSPAI_HIP(hipLaunchKernel(kern, dim3(nb), dim3(kAdThreads), args, lds, s));
    }
    int32_t he[4];
    BSPAI_HIP(hipMemcpyAsync(he, err, sizeof(he), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    if (he[0] != INT32_MAX) return fail(BSPAI_EZEROROW, "bspai_build_adaptive: row %d of M is zero (a_kk = 0?)", he[0]);
    if (he[1] != INT32_MAX) return fail(BSPAI_ERANK, "bspai_build_adaptive: rank-deficient least squares in row %d", he[1]);
    if (he[2] != INT32_MAX)
      return fail(BSPAI_EINVAL, "bspai_build_adaptive: row %d exceeds %d shadow rows or %d candidates", he[2],
                  kAdShadow, kAdCand / 2);
    if (he[3] != INT32_MAX)
      return fail(BSPAI_ENAN, "bspai_build_adaptive: the least squares of row %d overflow u_f (use scale)", he[3]);
    if (steps_host) BSPAI_HIP(hipMemcpy(steps_host, stp, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    // CSR of M
    if ((r = dalloc_t(&mrp, (size_t)n + 1)) || (r = dalloc(&tmp, scan_tmp_bytes(n)))) return r;
    if ((r = exclusive_scan(cnt, mrp, n, tmp, s))) return r;
    int32_t mnnz = 0;
    BSPAI_HIP(hipMemcpyAsync(&mnnz, mrp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    if ((r = dalloc_t(&mcol, (size_t)mnnz + 1)) || (r = dalloc_t(&mval, (size_t)mnnz + 1))) return r;
    hipLaunchKernelGGL(k_compact_rows, dim3(g), dim3(256), 0, s, n, jmax, cnt, cols, vals, mrp, mcol, mval);
    BSPAI_CHECK_LAUNCH();
    BSPAI_HIP(hipStreamSynchronize(s));
    bspai_csr Mc;
    Mc.n = n;
    Mc.nnz = mnnz;
    Mc.row_ptr = mrp;
    Mc.col = mcol;
    Mc.val = mval;
    return bspai_import(&Mc, eps_b, precs, q, opts, out, stream);
  };
  rc = body();
  (void)hipStreamSynchronize(s);
  dfree(trp), dfree(tcol), dfree(iota), dfree(cnt), dfree(cols), dfree(stp), dfree(err), dfree(rn2), dfree(vals);
  dfree(tiles), dfree(rhs), dfree(mrp), dfree(mcol), dfree(mval), dfree(tmp), dfree(dsc);
  return rc;
}

extern "C" int bspai_export_pattern(const bspai_handle *M, int32_t *row_ptr_host, int32_t *col_host) {
  using namespace bspai;
  if (!M) return fail(BSPAI_EINVAL, "bspai_export_pattern: null handle");
  if (row_ptr_host) BSPAI_HIP(hipMemcpy(row_ptr_host, M->m_rp, sizeof(int32_t) * ((size_t)M->n + 1), hipMemcpyDeviceToHost));
  if (col_host && M->nnz) BSPAI_HIP(hipMemcpy(col_host, M->m_col, sizeof(int32_t) * (size_t)M->nnz, hipMemcpyDeviceToHost));
  return BSPAI_OK;
}

extern "C" int bspai_stats(const bspai_handle *M, bspai_bucket_stats *o) {
  if (!M || !o) return fail(BSPAI_EINVAL, "bspai_stats: null argument");
  memset(o, 0, sizeof(*o));
  o->n = M->n;
  o->q = M->q;
  o->nnz = M->nnz;
  o->norm_inf = M->normM;
  o->eps_b = M->eps;
  double num = 0;
  for (int k = 0; k < M->q; k++) {
    o->precs[k] = (bspai_prec)M->precs[k];
    o->count[k] = M->b[k].nnz;
    o->threshold[k] = M->b[k].t;
    o->scale[k] = M->b[k].scale;
    int vb = value_bytes(M->precs[k]);
    o->bytes_values += (int64_t)vb * M->b[k].nnz;
    if (M->precs[k] != BSPAI_DROP && M->b[k].nnz > 0) o->bytes_indices += 4 * M->b[k].nnz + 4 * ((int64_t)M->n + 1);
    num += (double)vb * M->b[k].nnz;
    o->col_bytes[k] = M->b[k].ecw ? M->b[k].ecw : 4;
  }
  // ELL widths are kept in the kernel view (stored buckets, least precise first)
  for (int k = M->q - 1, j = 0; k >= 0; k--) {
    if (M->precs[k] == BSPAI_DROP || M->b[k].nnz == 0) continue;
    o->ell_width[k] = M->mat.ell_w[j++];
  }
  o->storage_pct = M->nnz ? 100.0 * num / ((double)M->nnz * value_bytes(M->precs[0])) : 100.0;
  o->apply_kind[0] = M->mat.nb ? apply_kind_resolved(M->mat) : 0;
  o->apply_kind[1] = M->has_T && M->matT.nb ? apply_kind_resolved(M->matT) : 0;
  return BSPAI_OK;
}

extern "C" int bspai_export(const bspai_handle *M, int8_t *bucket_host, double *stored_host, double *m64_host) {
  if (!M) return fail(BSPAI_EINVAL, "bspai_export: null handle");
  size_t nnz = (size_t)M->nnz;
  if (bucket_host && nnz) BSPAI_HIP(hipMemcpy(bucket_host, M->bucket_id, nnz, hipMemcpyDeviceToHost));
  if (stored_host && nnz) BSPAI_HIP(hipMemcpy(stored_host, M->stored, nnz * 8, hipMemcpyDeviceToHost));
  if (m64_host && nnz) {
    if (!M->has_fp64) return fail(BSPAI_EINVAL, "bspai_export: the FP64 M was not kept");
    BSPAI_HIP(hipMemcpy(m64_host, M->m_val, nnz * 8, hipMemcpyDeviceToHost));
  }
  return BSPAI_OK;
}

extern "C" void bspai_free(bspai_handle *M) {
  if (!M) return;
  (void)hipDeviceSynchronize();
  free_handle_memory(M);
  delete M;
}
