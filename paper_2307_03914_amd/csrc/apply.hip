// Public bucketed products: bspai_apply (M_b X) and bspai_apply_T (M_b^T X).
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "spmv_dev.h"

namespace bspai {

constexpr int kApplyThreads = 256;

// Blocks are dispatched round-robin over the 8 XCDs; remap so that each XCD
// works on one contiguous range of rows (neighbouring rows share x in its L2).
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  constexpr int kXcd = 8;
  int per = nblocks / kXcd;
  if (per == 0 || nblocks % kXcd) return b;
  return (b % kXcd) * per + b / kXcd;
}

// one row per group of L lanes; rows_per_block consecutive rows per block
template <int L, typename XT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv(BMat M, const XT *__restrict__ x, XT *__restrict__ y,
                                                         int rows_per_block) {
  int b = xcd_block(blockIdx.x, gridDim.x);
  int r0 = b * rows_per_block;
  int r1 = min(M.n, r0 + rows_per_block);
  bspmv_rows<L, XT, XT>(M, x, y, r0, r1);
}

// two-phase tile product: a block per range of rows_per_block rows
template <typename XT, typename PT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_tile(BMat M, const XT *__restrict__ x, XT *__restrict__ y,
                                                              int rows_per_block, int cap) {
  extern __shared__ double lds_tile[];
  PT *prod = reinterpret_cast<PT *>(lds_tile);
  double *acc = lds_tile + (cap * sizeof(PT) + 7) / 8;
  int32_t *rps = reinterpret_cast<int32_t *>(acc + rows_per_block);
  int b = xcd_block(blockIdx.x, gridDim.x);
  int r0 = b * rows_per_block;
  int r1 = min(M.n, r0 + rows_per_block);
  bspmv_tile_rows<XT, XT, PT>(M, x, y, r0, r1, prod, cap, acc, rows_per_block, rps);
}

// one wavefront per 64-row slice (SELL-64)
template <typename XT, typename PT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_sell(BMat M, const XT *__restrict__ x, XT *__restrict__ y) {
  constexpr int kWavesPerBlock = kApplyThreads / 64;
  int sl = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (sl * kSlice >= M.n) return;
  double v = bspmv_sell_row<XT, PT>(M, x, sl, lane);
  int row = sl * kSlice + lane;
  if (row < M.n) y[row] = (XT)v;
}

template <typename XT, typename PT>
static int launch_sell(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  int64_t ns = (M.n + kSlice - 1) / kSlice;
  int64_t nblk = (ns + kApplyThreads / 64 - 1) / (kApplyThreads / 64);
  hipLaunchKernelGGL((k_bspmv_sell<XT, PT>), dim3((unsigned)nblk), dim3(kApplyThreads), 0, s, M, x, y);
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

// one thread per row
template <typename XT, typename PT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_row(BMat M, const XT *__restrict__ x, XT *__restrict__ y) {
  int i = xcd_block(blockIdx.x, gridDim.x) * kApplyThreads + threadIdx.x;
  if (i < M.n) y[i] = (XT)bspmv_row_thread<XT, XT, PT>(M, x, i);
}

// RT rows per thread: rows b * RT * T + r * T + t of block b (coalesced per r)
template <int RT, typename XT, typename PT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_rows(BMat M, const XT *__restrict__ x, XT *__restrict__ y) {
  int base = xcd_block(blockIdx.x, gridDim.x) * kApplyThreads * RT + threadIdx.x;
  int rows[RT];
#pragma unroll
  for (int r = 0; r < RT; r++) rows[r] = base + r * kApplyThreads < M.n ? base + r * kApplyThreads : -1;
  double out[RT];
  bspmv_rows_thread<RT, XT, PT>(M, x, rows, out);
#pragma unroll
  for (int r = 0; r < RT; r++)
    if (rows[r] >= 0) y[rows[r]] = (XT)out[r];
}

template <typename XT, typename PT>
static int launch_rowthread(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  int rt = 2;
  if (const char *e = getenv("BSPAI_APPLY_RT")) rt = atoi(e);
  if (rt <= 1) {
    int64_t nblk = (M.n + kApplyThreads - 1) / kApplyThreads;
    hipLaunchKernelGGL((k_bspmv_row<XT, PT>), dim3((unsigned)nblk), dim3(kApplyThreads), 0, s, M, x, y);
  } else if (rt == 2) {
    int64_t nblk = (M.n + 2 * kApplyThreads - 1) / (2 * kApplyThreads);
    hipLaunchKernelGGL((k_bspmv_rows<2, XT, PT>), dim3((unsigned)nblk), dim3(kApplyThreads), 0, s, M, x, y);
  } else {
    int64_t nblk = (M.n + 4 * kApplyThreads - 1) / (4 * kApplyThreads);
    hipLaunchKernelGGL((k_bspmv_rows<4, XT, PT>), dim3((unsigned)nblk), dim3(kApplyThreads), 0, s, M, x, y);
  }
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

template <typename XT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmm(BMat M, const XT *__restrict__ x, XT *__restrict__ y,
                                                         int64_t ld, int nrhs, int group) {
  int lane = threadIdx.x & (group - 1);
  int rows_per_block = kApplyThreads / group;
  int i = xcd_block(blockIdx.x, gridDim.x) * rows_per_block + threadIdx.x / group;
  if (i >= M.n) return;
  for (int c0 = 0; c0 < nrhs; c0 += group) {
    int c = c0 + lane;
    bspmm_row<XT>(M, x, y, ld, i, c, c < nrhs);
  }
}

int bmat_aligned(const BMat &M) {
  for (int k = 0; k < M.nb; k++)
    if ((reinterpret_cast<uintptr_t>(M.col[k]) & 15) || (reinterpret_cast<uintptr_t>(M.val[k]) & 15)) return 0;
  return 1;
}

static bool has_fp64_bucket(const BMat &M) {
  for (int k = 0; k < M.nb; k++)
    if (M.prec[k] == BSPAI_FP64) return true;
  return false;
}

// products held in LDS per block, and rows per block sized so that a block's
// entries of one bucket usually fit
template <typename XT, typename PT>
static int launch_tile(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  const int cap = 16384 / (int)sizeof(PT);
  double avg = M.n ? (double)M.nnz / M.n : 1.0;
  int rows = (int)(cap / (1.3 * std::max(avg, 1.0)));
  rows = std::max(32, std::min(1024, rows & ~31));
  if (const char *e = getenv("BSPAI_TILE_ROWS")) rows = std::max(32, std::min(1024, atoi(e) & ~31));
  int64_t nblk = (M.n + rows - 1) / rows;
  size_t lds = (size_t)cap * sizeof(PT) + (size_t)rows * sizeof(double) + 4 * ((size_t)rows + 1) + 16;
  hipLaunchKernelGGL((k_bspmv_tile<XT, PT>), dim3((unsigned)nblk), dim3(kApplyThreads), lds, s, M, x, y, rows, cap);
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

int pick_lanes(const BMat &M, int64_t nnz) {
  double avg = M.n ? (double)nnz / M.n : 0;
  if (avg <= 3) return 2;
  if (avg <= 6) return 4;
  if (avg <= 14) return 8;
  if (avg <= 40) return 16;
  return 32;
}

template <typename XT>
static int launch_vec(const BMat &M, const XT *x, XT *y, int lanes, hipStream_t s) {
  // about 4 rows per group per block, blocks a multiple of 8 (XCDs)
  int groups = kApplyThreads / lanes;
  int rows_per_block = groups * 4;
  int64_t nblk = (M.n + rows_per_block - 1) / rows_per_block;
  if (nblk == 0) return BSPAI_OK;
  dim3 grid((unsigned)nblk), block(kApplyThreads);
  switch (lanes) {
    case 2: hipLaunchKernelGGL((k_bspmv<2, XT>), grid, block, 0, s, M, x, y, rows_per_block); break;
    case 4: hipLaunchKernelGGL((k_bspmv<4, XT>), grid, block, 0, s, M, x, y, rows_per_block); break;
    case 8: hipLaunchKernelGGL((k_bspmv<8, XT>), grid, block, 0, s, M, x, y, rows_per_block); break;
    case 16: hipLaunchKernelGGL((k_bspmv<16, XT>), grid, block, 0, s, M, x, y, rows_per_block); break;
    default: hipLaunchKernelGGL((k_bspmv<32, XT>), grid, block, 0, s, M, x, y, rows_per_block); break;
  }
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

int launch_bspmv(const BMat &M, const void *x, void *y, int nrhs, int64_t ld, int fp64, hipStream_t s) {
  if (M.n == 0) return BSPAI_OK;
  if (nrhs == 1) {
    double avg = M.n ? (double)M.nnz / M.n : 0.0;
    const char *kind = getenv("BSPAI_APPLY_KERNEL");
    if (M.sell_ptr[0] && !(kind && (kind[0] == 't' || kind[0] == 'r'))) {
      if (fp64) return launch_sell<double, double>(M, static_cast<const double *>(x), static_cast<double *>(y), s);
      if (has_fp64_bucket(M))
        return launch_sell<float, double>(M, static_cast<const float *>(x), static_cast<float *>(y), s);
      return launch_sell<float, float>(M, static_cast<const float *>(x), static_cast<float *>(y), s);
    }
    if (avg <= 24 && !(kind && kind[0] == 't')) {
      if (fp64) return launch_rowthread<double, double>(M, static_cast<const double *>(x), static_cast<double *>(y), s);
      if (has_fp64_bucket(M))
        return launch_rowthread<float, double>(M, static_cast<const float *>(x), static_cast<float *>(y), s);
      return launch_rowthread<float, float>(M, static_cast<const float *>(x), static_cast<float *>(y), s);
    }
    if (M.aligned && avg <= 48) {
      if (fp64) return launch_tile<double, double>(M, static_cast<const double *>(x), static_cast<double *>(y), s);
      if (has_fp64_bucket(M))
        return launch_tile<float, double>(M, static_cast<const float *>(x), static_cast<float *>(y), s);
      return launch_tile<float, float>(M, static_cast<const float *>(x), static_cast<float *>(y), s);
    }
    int lanes = M.lanes > 0 ? M.lanes : pick_lanes(M, M.nnz);
    return fp64 ? launch_vec<double>(M, static_cast<const double *>(x), static_cast<double *>(y), lanes, s)
                : launch_vec<float>(M, static_cast<const float *>(x), static_cast<float *>(y), lanes, s);
  }
  int group = 1;
  while (group < nrhs && group < 64) group <<= 1;
  int rows_per_block = kApplyThreads / group;
  int64_t nblk = (M.n + rows_per_block - 1) / rows_per_block;
  dim3 grid((unsigned)nblk), block(kApplyThreads);
  if (fp64)
    hipLaunchKernelGGL(k_bspmm<double>, grid, block, 0, s, M, static_cast<const double *>(x),
                       static_cast<double *>(y), ld, nrhs, group);
  else
    hipLaunchKernelGGL(k_bspmm<float>, grid, block, 0, s, M, static_cast<const float *>(x), static_cast<float *>(y),
                       ld, nrhs, group);
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

static int apply_common(const bspai_handle *M, const void *x, void *y, int nrhs, int64_t ld, bspai_prec xy_prec,
                        void *stream, bool trans) {
  if (!M) return fail(BSPAI_EINVAL, "apply: null handle");
  if (trans && !M->has_T) return fail(BSPAI_EINVAL, "apply_T: handle built without build_T");
  if (nrhs < 1) return fail(BSPAI_EINVAL, "apply: nrhs must be >= 1");
  if (nrhs > 1 && ld < nrhs) return fail(BSPAI_EINVAL, "apply: ld < nrhs");
  if (xy_prec != BSPAI_FP32 && xy_prec != BSPAI_FP64) return fail(BSPAI_EINVAL, "apply: xy_prec must be FP32 or FP64");
  if (M->n > 0 && (!x || !y)) return fail(BSPAI_EINVAL, "apply: null vector");
  if (x == y) return fail(BSPAI_EINVAL, "apply: x and y must not overlap");
  int dev = 0;
  BSPAI_HIP(hipGetDevice(&dev));
  if (dev != M->device) return fail(BSPAI_EINVAL, "apply: handle lives on device %d, current is %d", M->device, dev);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return launch_bspmv(trans ? M->matT : M->mat, x, y, nrhs, nrhs == 1 ? 1 : ld, xy_prec == BSPAI_FP64, s);
}

}  // namespace bspai

extern "C" int bspai_apply(const bspai_handle *M, const void *x, void *y, int nrhs, int64_t ld, bspai_prec xy_prec,
                           void *stream) {
  return bspai::apply_common(M, x, y, nrhs, ld, xy_prec, stream, false);
}

extern "C" int bspai_apply_T(const bspai_handle *M, const void *x, void *y, int nrhs, int64_t ld,
                             bspai_prec xy_prec, void *stream) {
  return bspai::apply_common(M, x, y, nrhs, ld, xy_prec, stream, true);
}

// ------------------------------------------------------------------ adjoint

namespace bspai {
__global__ void k_grad_vals(int n, const int32_t *rp, const int32_t *col, const double *lam, const double *x,
                            double *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double li = lam[i];
  for (int p = rp[i]; p < rp[i + 1]; p++) out[p] = -li * x[col[p]];
}
}  // namespace bspai

// dL/da_ij = -lambda_i x_j for the entries of A (adjoint of A x = b).
extern "C" int bspai_grad_vals(const bspai_pattern *A, const double *lam, const double *x, double *out,
                               void *stream) {
  using namespace bspai;
  if (!A || A->n < 0 || (A->n > 0 && (!A->row_ptr || !lam || !x || (A->nnz > 0 && (!A->col || !out)))))
    return fail(BSPAI_EINVAL, "bspai_grad_vals: bad argument");
  if (A->n == 0) return BSPAI_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_grad_vals, dim3((A->n + 255) / 256), dim3(256), 0, s, A->n, A->row_ptr, A->col, lam, x, out);
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}
