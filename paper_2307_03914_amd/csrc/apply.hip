// Public bucketed products: bspai_apply (M_b X) and bspai_apply_T (M_b^T X).
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
