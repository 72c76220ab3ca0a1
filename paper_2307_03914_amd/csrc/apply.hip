// Public bucketed products: bspai_apply (M_b X) and bspai_apply_T (M_b^T X).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

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

// one wavefront per 64-row slice (SELL-64 or ELL copies); the offset tables of
// byte-coded ELL columns are staged in LDS first
template <typename XT, typename PT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_sell(BMat M, const XT *__restrict__ x, XT *__restrict__ y) {
  constexpr int kWavesPerBlock = kApplyThreads / 64;
  __shared__ int32_t sdict[kMaxBuckets * 256];
  bool staged = false;
  for (int k = 0; k < M.nb; k++) {
    if (M.ell_w[k] && M.ell_cw[k] == 1) {
      for (int t = threadIdx.x; t < 256; t += blockDim.x) sdict[256 * k + t] = M.ell_dict[k][t];
      staged = true;
    }
  }
  if (staged) __syncthreads();
  int sl = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (sl * kSlice >= M.n) return;
  double v = bspmv_sell_row<XT, PT>(M, x, sl, lane, sdict);
  int row = sl * kSlice + lane;
  if (row < M.n) y[row] = (XT)v;
}

// RT rows per thread, every stored bucket in ELL form: rows b RT T + r T + t
// of block b (coalesced per r); invalid rows read row 0's entries and are not
// stored
template <int RT, typename XT, typename PT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_ell(BMat M, const XT *__restrict__ x, XT *__restrict__ y) {
  __shared__ int32_t sdict[kMaxBuckets * 256];
  bool staged = false;
  for (int k = 0; k < M.nb; k++) {
    if (M.ell_cw[k] == 1) {
      for (int t = threadIdx.x; t < 256; t += blockDim.x) sdict[256 * k + t] = M.ell_dict[k][t];
      staged = true;
    }
  }
  if (staged) __syncthreads();
  const int base = xcd_block(blockIdx.x, gridDim.x) * kApplyThreads * RT + threadIdx.x;
  int rows[RT];
#pragma unroll
  for (int r = 0; r < RT; r++) rows[r] = base + r * kApplyThreads < M.n ? base + r * kApplyThreads : -1;
  double out[RT];
  bspmv_ell_rows<RT, XT, PT>(M, x, rows, sdict, out);
#pragma unroll
  for (int r = 0; r < RT; r++)
    if (rows[r] >= 0) y[rows[r]] = (XT)out[r];
}

// One stored bucket of known format FMT in ELL form, one row per thread: the
// format switch is resolved at compile time so the kernel stays small enough
// for full occupancy.  NT: stream the codes and values with non-temporal
// loads (they are read once; x stays in L2).

template <typename XT, typename PT, int FMT, bool NT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_ell1(BMat M, const XT *__restrict__ x, XT *__restrict__ y) {
  __shared__ int32_t sdict[256];
  const int cw = M.ell_cw[0], ew = M.ell_w[0];
  if (cw == 1) {
    sdict[threadIdx.x] = M.ell_dict[0][threadIdx.x];  // kApplyThreads == 256
    __syncthreads();
  }
  const int row = xcd_block(blockIdx.x, gridDim.x) * kApplyThreads + threadIdx.x;
  if (row >= M.n) return;
  constexpr bool wide = FMT == BSPAI_FP64 || sizeof(PT) == 8;
  double accd = 0.0;
  float accf = 0.f;
  for (int c0 = 0; c0 < ew; c0 += 8) {
    const int64_t e = (int64_t)row * ew + c0;
    const int nc = ew - c0 < 8 ? 4 : 8;  // widths are 4, 8 or 16
    int cc[8];
    if (cw == 1) {
      const uint8_t *p = static_cast<const uint8_t *>(M.ell_code[0]) + e;
      uint32_t q0, q1 = 0;
      if (nc == 8) {
        u32x2 t = ld_stream<NT, u32x2>(p);
        q0 = t.x, q1 = t.y;
      } else {
        q0 = ld_stream<NT, uint32_t>(p);
      }
#pragma unroll
      for (int t = 0; t < 4; t++) cc[t] = row + sdict[(q0 >> (8 * t)) & 0xFFu];
#pragma unroll
      for (int t = 0; t < 4; t++) cc[4 + t] = row + sdict[(q1 >> (8 * t)) & 0xFFu];
    } else if (cw == 2) {
      const int16_t *p = static_cast<const int16_t *>(M.ell_code[0]) + e;
      int32_t q[4] = {0, 0, 0, 0};
      if (nc == 8) {
        i32x4 t = ld_stream<NT, i32x4>(p);
        q[0] = t.x, q[1] = t.y, q[2] = t.z, q[3] = t.w;
      } else {
        i32x2 t = ld_stream<NT, i32x2>(p);
        q[0] = t.x, q[1] = t.y;
      }
#pragma unroll
      for (int t = 0; t < 8; t++) cc[t] = row + ((t & 1) ? (q[t / 2] >> 16) : (int32_t)(int16_t)(q[t / 2] & 0xFFFF));
    } else {
      const int32_t *p = M.ell_col[0] + e;
      i32x4 a = ld_stream<NT, i32x4>(p);
      i32x4 b = nc == 8 ? ld_stream<NT, i32x4>(p + 4) : i32x4{row, row, row, row};
      cc[0] = a.x, cc[1] = a.y, cc[2] = a.z, cc[3] = a.w, cc[4] = b.x, cc[5] = b.y, cc[6] = b.z, cc[7] = b.w;
    }
    PT vv[8];
    if (FMT == BSPAI_FP16 || FMT == BSPAI_BF16) {
      const uint16_t *p = static_cast<const uint16_t *>(M.ell_val[0]) + e;
      uint32_t w4[4] = {0, 0, 0, 0};
      if (nc == 8) {
        u32x4 a = ld_stream<NT, u32x4>(p);
        w4[0] = a.x, w4[1] = a.y, w4[2] = a.z, w4[3] = a.w;
      } else {
        u32x2 a = ld_stream<NT, u32x2>(p);
        w4[0] = a.x, w4[1] = a.y;
      }
#pragma unroll
      for (int t = 0; t < 4; t++) {
        vv[2 * t] = FMT == BSPAI_FP16 ? decode_f16(w4[t] & 0xFFFFu) : decode_bf16(w4[t] & 0xFFFFu);
        vv[2 * t + 1] = FMT == BSPAI_FP16 ? decode_f16(w4[t] >> 16) : decode_bf16(w4[t] >> 16);
      }
    } else if (FMT == BSPAI_FP8_E4M3) {
      const uint8_t *p = static_cast<const uint8_t *>(M.ell_val[0]) + e;
      uint32_t q0, q1 = 0;
      if (nc == 8) {
        u32x2 a = ld_stream<NT, u32x2>(p);
        q0 = a.x, q1 = a.y;
      } else {
        q0 = ld_stream<NT, uint32_t>(p);
      }
#pragma unroll
      for (int t = 0; t < 4; t++) vv[t] = decode_e4m3((q0 >> (8 * t)) & 0xFFu), vv[4 + t] = decode_e4m3((q1 >> (8 * t)) & 0xFFu);
    } else if (FMT == BSPAI_FP32) {
      const float *p = static_cast<const float *>(M.ell_val[0]) + e;
      f32x4 a = ld_stream<NT, f32x4>(p);
      f32x4 b = nc == 8 ? ld_stream<NT, f32x4>(p + 4) : f32x4{0.f, 0.f, 0.f, 0.f};
      vv[0] = a.x, vv[1] = a.y, vv[2] = a.z, vv[3] = a.w, vv[4] = b.x, vv[5] = b.y, vv[6] = b.z, vv[7] = b.w;
    } else {
      const double *p = static_cast<const double *>(M.ell_val[0]) + e;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        f64x2 a = (2 * t < nc) ? ld_stream<NT, f64x2>(p + 2 * t) : f64x2{0.0, 0.0};
        vv[2 * t] = (PT)a.x, vv[2 * t + 1] = (PT)a.y;
      }
    }
    PT xv[8];
#pragma unroll
    for (int u = 0; u < 8; u++) xv[u] = u < nc ? (PT)x[cc[u]] : (PT)0;
#pragma unroll
    for (int u = 0; u < 8; u++) {
      if (u < nc) {
        if (wide)
          accd = fma((double)vv[u], (double)xv[u], accd);
        else
          accf = fmaf((float)vv[u], (float)xv[u], accf);
      }
    }
  }
  y[row] = (XT)((wide ? accd : (double)accf) * M.scale[0]);
}

template <typename XT, typename PT, bool NT>
static int launch_ell1_nt(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  const unsigned nblk = (unsigned)((M.n + kApplyThreads - 1) / kApplyThreads);
  switch (M.prec[0]) {
    case BSPAI_FP64: hipLaunchKernelGGL((k_bspmv_ell1<XT, PT, BSPAI_FP64, NT>), dim3(nblk), dim3(kApplyThreads), 0, s, M, x, y); break;
    case BSPAI_FP32: hipLaunchKernelGGL((k_bspmv_ell1<XT, PT, BSPAI_FP32, NT>), dim3(nblk), dim3(kApplyThreads), 0, s, M, x, y); break;
    case BSPAI_FP16: hipLaunchKernelGGL((k_bspmv_ell1<XT, PT, BSPAI_FP16, NT>), dim3(nblk), dim3(kApplyThreads), 0, s, M, x, y); break;
    case BSPAI_BF16: hipLaunchKernelGGL((k_bspmv_ell1<XT, PT, BSPAI_BF16, NT>), dim3(nblk), dim3(kApplyThreads), 0, s, M, x, y); break;
    default: hipLaunchKernelGGL((k_bspmv_ell1<XT, PT, BSPAI_FP8_E4M3, NT>), dim3(nblk), dim3(kApplyThreads), 0, s, M, x, y); break;
  }
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

// measured on the 128^3 operator (bf16 bucket, byte-coded columns, MI355X):
// 18.1 us with plain loads, 17.1 us with non-temporal ones
template <typename XT, typename PT>
static int launch_ell1(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  return launch_ell1_nt<XT, PT, true>(M, x, y, s);
}

static bool all_ell(const BMat &M) {
  for (int k = 0; k < M.nb; k++)
    if (!M.ell_w[k]) return false;
  return M.nb > 0;
}

// one bucket: the format-specialised kernel; several: the generic one (one
// row per thread measured faster than 2 or 4: 23.0, 27.0, 37.0 us on the
// 128^3 operator, as more rows per thread cost occupancy)
template <typename XT, typename PT>
static int launch_ell(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  if (M.nb == 1) return launch_ell1<XT, PT>(M, x, y, s);
  const unsigned nblk = (unsigned)((M.n + kApplyThreads - 1) / kApplyThreads);
  hipLaunchKernelGGL((k_bspmv_ell<1, XT, PT>), dim3(nblk), dim3(kApplyThreads), 0, s, M, x, y);
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

template <typename XT, typename PT>
static int launch_sell(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  if (all_ell(M)) return launch_ell<XT, PT>(M, x, y, s);
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

// two rows per thread (one row per thread and four measured slower: four
// costs occupancy)
template <typename XT, typename PT>
static int launch_rowthread(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  int64_t nblk = (M.n + 2 * kApplyThreads - 1) / (2 * kApplyThreads);
  hipLaunchKernelGGL((k_bspmv_rows<2, XT, PT>), dim3((unsigned)nblk), dim3(kApplyThreads), 0, s, M, x, y);
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

// Many right-hand sides with R a multiple of 4 (row-major, ld a multiple of
// 4): R / 4 lanes per row, each owning 4 consecutive columns, so a wavefront
// works on several rows; per bucket a row's columns and values are loaded 8
// at a time ahead of their 16-byte gathers of x.  Same order of operations as
// bspmm_row (entries in CSR order, per-bucket FP32 or FP64 accumulation,
// buckets added in FP64 from the least precise).
template <typename XT>
__device__ __forceinline__ void ld4(const XT *p, double (&v)[4]) {
  if (sizeof(XT) == 4) {
    float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
  } else {
    double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
  }
}

template <typename XT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmm4(BMat M, const XT *__restrict__ x, XT *__restrict__ y,
                                                          int64_t ld, int nrhs) {
  const int tpr = nrhs / 4, rpb = kApplyThreads / tpr;
  const int g = threadIdx.x / tpr, c0 = 4 * (threadIdx.x % tpr);
  const int i = xcd_block(blockIdx.x, gridDim.x) * rpb + g;
  if (g >= rpb || i >= M.n) return;
  double total[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < M.nb; k++) {
    const int s = M.rp[k][i], e = M.rp[k][i + 1];
    const int32_t *col = M.col[k];
    const bool wide = M.prec[k] == BSPAI_FP64 || sizeof(XT) == 8;
    double accd[4] = {0.0, 0.0, 0.0, 0.0};
    float accf[4] = {0.f, 0.f, 0.f, 0.f};
    for (int p0 = s; p0 < e; p0 += 8) {
      int cc[8];
      double vv[8];
#pragma unroll
      for (int t = 0; t < 8; t++) {
        const int p = p0 + t < e ? p0 + t : s;
        cc[t] = col[p];
        vv[t] = M.prec[k] == BSPAI_FP64 ? static_cast<const double *>(M.val[k])[p] : (double)load_value_f32(M, k, p);
      }
      double xv[8][4];
#pragma unroll
      for (int t = 0; t < 8; t++) ld4<XT>(x + (int64_t)cc[t] * ld + c0, xv[t]);
#pragma unroll
      for (int t = 0; t < 8; t++) {
        if (p0 + t < e) {
#pragma unroll
          for (int u = 0; u < 4; u++) {
            if (wide)
              accd[u] = fma(vv[t], xv[t][u], accd[u]);
            else
              accf[u] = fmaf((float)vv[t], (float)xv[t][u], accf[u]);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; u++) total[u] += (wide ? accd[u] : (double)accf[u]) * M.scale[k];
  }
  XT o[4];
#pragma unroll
  for (int u = 0; u < 4; u++) o[u] = (XT)total[u];
  XT *yp = y + (int64_t)i * ld + c0;
  if (sizeof(XT) == 4) {
    *reinterpret_cast<float4 *>(yp) = make_float4((float)o[0], (float)o[1], (float)o[2], (float)o[3]);
  } else {
    reinterpret_cast<double2 *>(yp)[0] = make_double2((double)o[0], (double)o[1]);
    reinterpret_cast<double2 *>(yp)[1] = make_double2((double)o[2], (double)o[3]);
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

// ------------------------------------------------------------------ segmented tiles
//
// For rows of very different lengths with scattered columns (a power-law
// matrix): the rows are cut into tiles of whole rows holding about
// kSegTile entries over all buckets (a plan built with the handle), one
// block per tile.  Phase 1 streams every bucket's entries of the tile with
// 8-wide aligned non-temporal loads (each thread keeps 8 gathers of x in
// flight) and writes the products to LDS; phase 2 adds each row's products
// in CSR order, one thread per row, except rows of more than kSegLong
// entries, which a whole wavefront adds (lane l takes products l, l + 64,
// ..., then a fixed butterfly), so a long row does not hold its block.
// Measured on a 2^20-row power-law matrix: kSegLong 16 / 32 / 64 / 128 /
// 256 gave 137 / 114 / 104 / 104 / 116 us, tiles of 2048 / 4096 / 8192
// entries 118 / 114 / 154 us, one chunk per round instead of two 110 us,
// one chunk with kSegLong 64: 101 us.
// Per-bucket sums in FP32 (FP64 for wide products), scaled and added in FP64
// from the least to the most precise bucket, as in the other kernels; the
// order of additions inside a row is fixed by the plan, so repeated products
// give identical bits.
constexpr int kSegTile = 4096;
constexpr int kSegLong = 64;
constexpr int kSegMaxLong = 2 * kSegTile / (kSegLong + 1) + 1;

template <typename T>
__device__ __forceinline__ T wave_butterfly_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// one bucket's entries [b0, b1) of a tile into LDS products (pk indexed by
// entry), the value format fixed at compile time: each thread takes up to
// kSegChunks aligned 8-entry chunks, issues all their column and value loads,
// then all their gathers, then writes the products of the entries inside
// [b0, b1).  Loads go through buffer resources whose extent is the 16-byte
// granule holding entry b1 - 1 (a 16-byte load that crosses the extent
// returns zero as a whole; the granule never crosses a page), so chunks past
// the tile read zero without a branch around a load; entries at or past b1
// gather x[t] of their lane (coalesced, never written).  The chunk loop runs
// the same number of times in every thread of the block.
constexpr int kSegChunks = 1;  // 8-entry chunks per thread per round
template <int FMT, typename XT, typename PT>
__device__ __forceinline__ void seg_stream(const BMat &M, int k, int b0, int b1, const XT *__restrict__ x,
                                           PT *pk) {
  constexpr int VB = FMT == BSPAI_FP64 ? 8 : FMT == BSPAI_FP32 ? 4 : (FMT == BSPAI_FP8_E4M3 ? 1 : 2);
  const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(M.col[k]), (short)0,
                                                                      (4 * b1 + 15) & ~15, 0x00020000);
  const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(M.val[k]), (short)0,
                                                                      (VB * b1 + 15) & ~15, 0x00020000);
  const int a0 = b0 & ~(kTileVec - 1), first = a0 + threadIdx.x * kTileVec;
  constexpr int kStride = kApplyThreads * kTileVec;
  const int groups = (b1 - a0 + kSegChunks * kStride - 1) / (kSegChunks * kStride);
  const int spare = min((int)threadIdx.x, M.n - 1);
  for (int g = 0, base0 = first; g < groups; g++, base0 += kSegChunks * kStride) {
    int cc[kSegChunks][kTileVec];
    PT vv[kSegChunks][kTileVec];
#pragma unroll
    for (int u = 0; u < kSegChunks; u++) {
      const unsigned base = (unsigned)(base0 + u * kStride);
      const auto c0 = __builtin_amdgcn_raw_buffer_load_b128(rc, 4u * base, 0u, 2);
      const auto c1 = __builtin_amdgcn_raw_buffer_load_b128(rc, 4u * base + 16u, 0u, 2);
#pragma unroll
      for (int t = 0; t < 4; t++) {
        cc[u][t] = (int)base + t < b1 ? (int)c0[t] : spare;
        cc[u][4 + t] = (int)base + 4 + t < b1 ? (int)c1[t] : spare;
      }
      if constexpr (FMT == BSPAI_FP8_E4M3) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(rv, base, 0u, 2);
#pragma unroll
        for (int t = 0; t < 8; t++) vv[u][t] = (PT)decode_e4m3((uint8_t)((w[t >> 2] >> (8 * (t & 3))) & 0xFFu));
      } else if constexpr (FMT == BSPAI_FP16 || FMT == BSPAI_BF16) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(rv, 2u * base, 0u, 2);
#pragma unroll
        for (int t = 0; t < 8; t++) {
          const uint16_t h = (uint16_t)((w[t >> 1] >> (16 * (t & 1))) & 0xFFFFu);
          vv[u][t] = (PT)(FMT == BSPAI_FP16 ? decode_f16(h) : decode_bf16(h));
        }
      } else if constexpr (FMT == BSPAI_FP32) {
        const auto w0 = __builtin_amdgcn_raw_buffer_load_b128(rv, 4u * base, 0u, 2);
        const auto w1 = __builtin_amdgcn_raw_buffer_load_b128(rv, 4u * base + 16u, 0u, 2);
#pragma unroll
        for (int t = 0; t < 4; t++) vv[u][t] = (PT)__uint_as_float(w0[t]), vv[u][4 + t] = (PT)__uint_as_float(w1[t]);
      } else {
#pragma unroll
        for (int h2 = 0; h2 < 4; h2++) {
          const auto w = __builtin_amdgcn_raw_buffer_load_b128(rv, 8u * base + 16u * h2, 0u, 2);
          vv[u][2 * h2] = (PT)__longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
          vv[u][2 * h2 + 1] = (PT)__longlong_as_double((long long)(((unsigned long long)w[3] << 32) | w[2]));
        }
      }
    }
    PT xv[kSegChunks][kTileVec];
#pragma unroll
    for (int u = 0; u < kSegChunks; u++)
#pragma unroll
      for (int t = 0; t < kTileVec; t++) xv[u][t] = (PT)x[cc[u][t]];
#pragma unroll
    for (int u = 0; u < kSegChunks; u++)
#pragma unroll
      for (int t = 0; t < kTileVec; t++) {
        const int e = base0 + u * kStride + t;
        if (e >= b0 && e < b1) pk[e] = vv[u][t] * xv[u][t];
      }
  }
}

template <typename XT, typename PT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmv_seg(BMat M, const XT *__restrict__ x, XT *__restrict__ y) {
  extern __shared__ double seg_lds[];
  PT *prod = reinterpret_cast<PT *>(seg_lds);
  __shared__ int nlong;
  __shared__ int longrow[kSegMaxLong];
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, nb = M.nb;
  // the tile's rows and each bucket's entry range, from the plan in one round
  const int r0 = M.seg_rows[tile], r1 = M.seg_rows[tile + 1];
  int e0[kMaxBuckets], off[kMaxBuckets + 1];
  off[0] = 0;
#pragma unroll
  for (int k = 0; k < kMaxBuckets; k++) {
    if (k < nb) {
      e0[k] = M.seg_off[tile * nb + k];
      off[k + 1] = off[k] + (M.seg_off[(tile + 1) * nb + k] - e0[k]);
    } else {
      e0[k] = 0;
      off[k + 1] = off[k];
    }
  }
  // row pointers of the thread's first two rows, loaded under the gathers
  constexpr int RR = 2;
  int ra[RR][kMaxBuckets], rb[RR][kMaxBuckets];
#pragma unroll
  for (int r = 0; r < RR; r++) {
    const int i = r0 + tid + r * kApplyThreads;
#pragma unroll
    for (int k = 0; k < kMaxBuckets; k++) {
      const bool ok = k < nb && i < r1;
      ra[r][k] = ok ? M.rp[k][i] : 0;
      rb[r][k] = ok ? M.rp[k][i + 1] : 0;
    }
  }
  if (tid == 0) nlong = 0;
#pragma unroll
  for (int k = 0; k < kMaxBuckets; k++) {
    if (k >= nb) break;
    const int b0 = e0[k], b1 = b0 + (off[k + 1] - off[k]);
    PT *pk = prod + off[k] - b0;
    switch (M.prec[k]) {
      case BSPAI_FP64: seg_stream<BSPAI_FP64, XT, PT>(M, k, b0, b1, x, pk); break;
      case BSPAI_FP32: seg_stream<BSPAI_FP32, XT, PT>(M, k, b0, b1, x, pk); break;
      case BSPAI_FP16: seg_stream<BSPAI_FP16, XT, PT>(M, k, b0, b1, x, pk); break;
      case BSPAI_BF16: seg_stream<BSPAI_BF16, XT, PT>(M, k, b0, b1, x, pk); break;
      default: seg_stream<BSPAI_FP8_E4M3, XT, PT>(M, k, b0, b1, x, pk); break;
    }
  }
  __syncthreads();
  for (int r = 0, i = r0 + tid; i < r1; r++, i += kApplyThreads) {
    int a[kMaxBuckets], b[kMaxBuckets], len = 0;
#pragma unroll
    for (int k = 0; k < kMaxBuckets; k++) {
      if (r < RR) {
        a[k] = r == 0 ? ra[0][k] : ra[1][k];
        b[k] = r == 0 ? rb[0][k] : rb[1][k];
      } else {
        a[k] = k < nb ? M.rp[k][i] : 0;
        b[k] = k < nb ? M.rp[k][i + 1] : 0;
      }
      len += b[k] - a[k];
    }
    if (len > kSegLong) {
      longrow[atomicAdd(&nlong, 1)] = i;
      continue;
    }
    double total = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxBuckets; k++) {
      if (k >= nb) break;
      const PT *pk = prod + off[k] - e0[k];
      if (M.prec[k] == BSPAI_FP64 || sizeof(PT) == 8) {
        double sum = 0.0;
        for (int q = a[k]; q < b[k]; q++) sum += (double)pk[q];
        total += sum * M.scale[k];
      } else {
        float sum = 0.f;
        for (int q = a[k]; q < b[k]; q++) sum += (float)pk[q];
        total += (double)sum * M.scale[k];
      }
    }
    y[i] = (XT)total;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  for (int q = wv; q < nlong; q += kApplyThreads / 64) {
    const int i = longrow[q];
    double total = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxBuckets; k++) {
      if (k >= nb) break;
      const int a = M.rp[k][i], b = M.rp[k][i + 1];
      const PT *pk = prod + off[k] - e0[k];
      if (M.prec[k] == BSPAI_FP64 || sizeof(PT) == 8) {
        double sum = 0.0;
        for (int p = a + lane; p < b; p += 64) sum += (double)pk[p];
        total += wave_butterfly_sum(sum) * M.scale[k];
      } else {
        float sum = 0.f;
        for (int p = a + lane; p < b; p += 64) sum += (float)pk[p];
        total += (double)wave_butterfly_sum(sum) * M.scale[k];
      }
    }
    if (lane == 0) y[i] = (XT)total;
  }
}

template <typename XT, typename PT>
static int launch_seg(const BMat &M, const XT *x, XT *y, hipStream_t s) {
  if (M.seg_ntiles == 0) return BSPAI_OK;
  const size_t lds = (size_t)M.seg_cap * sizeof(PT);
  static bool attr = false;  // raise the dynamic LDS limit once per instantiation
  if (!attr) {
    BSPAI_HIP(hipFuncSetAttribute((const void *)k_bspmv_seg<XT, PT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((k_bspmv_seg<XT, PT>), dim3((unsigned)M.seg_ntiles), dim3(kApplyThreads), lds, s, M, x, y);
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

// entries of row i over all buckets, and the longest row
__global__ void k_seg_len(BMat M, int32_t *len, int32_t *mx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.n) return;
  int l = 0;
  for (int k = 0; k < M.nb; k++) l += M.rp[k][i + 1] - M.rp[k][i];
  len[i] = l;
  atomicMax(mx, l);
}

// rows[t] = the first row whose entries start at or after t kSegTile
// (pre: exclusive prefix of the row lengths, n + 1 entries); rows[nt] = n;
// off[t nb + k] = the first entry of bucket k in tile t
__global__ void k_seg_bounds(BMat M, const int32_t *pre, int nt, int32_t *rows, int32_t *off) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > nt) return;
  const int n = M.n;
  int lo = n;
  if (t < nt) {
    const int64_t target = (int64_t)t * kSegTile;
    int hi = n;  // smallest r in [0, n] with pre[r] >= target
    lo = 0;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      if (pre[mid] >= target)
        hi = mid;
      else
        lo = mid + 1;
    }
  }
  rows[t] = lo;
  for (int k = 0; k < M.nb; k++) off[(int64_t)t * M.nb + k] = M.rp[k][lo];
}

int build_seg_plan(BMat &M, int32_t **rows, hipStream_t s) {
  *rows = nullptr;
  M.seg_rows = nullptr;
  M.seg_off = nullptr;
  M.seg_ntiles = 0;
  M.seg_cap = 0;
  if (M.n == 0 || M.nb == 0) return BSPAI_OK;
  const int n = M.n;
  int32_t *len = nullptr, *pre = nullptr, *mx = nullptr;
  void *tmp = nullptr;
  int rc;
  if ((rc = dalloc_t(&len, (size_t)n)) || (rc = dalloc_t(&pre, (size_t)n + 1)) || (rc = dalloc_t(&mx, 1)) ||
      (rc = dalloc(&tmp, scan_tmp_bytes(n)))) {
    dfree(len), dfree(pre), dfree(mx), dfree(tmp);
    return rc;
  }
  int32_t hmx = 0, total = 0;
  auto body = [&]() -> int {
    BSPAI_HIP(hipMemsetAsync(mx, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_seg_len, dim3((n + 255) / 256), dim3(256), 0, s, M, len, mx);
    BSPAI_CHECK_LAUNCH();
    int r = exclusive_scan(len, pre, n, tmp, s);
    if (r) return r;
    BSPAI_HIP(hipMemcpyAsync(&hmx, mx, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipMemcpyAsync(&total, pre + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    // no plan for a row longer than a tile, or for byte offsets of the
    // buffer loads (8 per FP64 entry) that would not fit 31 bits
    if (hmx > kSegTile || total > (1 << 28)) return BSPAI_OK;
    const int nt = std::max(1, (total + kSegTile - 1) / kSegTile);
    // one allocation: nt + 1 tile rows, then (nt + 1) nb bucket offsets
    if ((r = dalloc_t(rows, (size_t)(nt + 1) * (1 + M.nb)))) return r;
    int32_t *off = *rows + nt + 1;
    hipLaunchKernelGGL(k_seg_bounds, dim3((nt + 1 + 255) / 256), dim3(256), 0, s, M, pre, nt, *rows, off);
    BSPAI_CHECK_LAUNCH();
    BSPAI_HIP(hipStreamSynchronize(s));
    M.seg_rows = *rows;
    M.seg_off = off;
    M.seg_ntiles = nt;
    M.seg_cap = 2 * kSegTile;  // a tile holds fewer than kSegTile + (longest row) entries
    return BSPAI_OK;
  };
  rc = body();
  dfree(len), dfree(pre), dfree(mx), dfree(tmp);
  if (rc) {
    dfree(*rows);
    *rows = nullptr;
    M.seg_rows = nullptr;
    M.seg_off = nullptr;
    M.seg_ntiles = 0;
  }
  return rc;
}

// every stored bucket has an ELL or a SELL copy
static bool sell_ok(const BMat &M) {
  for (int k = 0; k < M.nb; k++)
    if (!M.ell_w[k] && !M.sell_ptr[k]) return false;
  return M.nb > 0;
}

bool apply_kind_ok(const BMat &M, int kind) {
  switch (kind) {
    case kApplyAuto: return true;
    case kApplySell: return sell_ok(M);
    case kApplyTile: return M.aligned != 0;
    case kApplyRows:
    case kApplyLanes: return true;
    case kApplySeg: return M.seg_rows != nullptr && M.aligned != 0;
  }
  return false;
}

// the padded copies when every bucket has one, else LDS tiles (balanced for
// rows of any length), else one group of lanes per row
int apply_kind_resolved(const BMat &M) {
  if (M.apply_kind > 0 && apply_kind_ok(M, M.apply_kind)) return M.apply_kind;
  if (sell_ok(M)) return kApplySell;
  if (M.aligned) return kApplyTile;
  return kApplyLanes;
}

template <typename XT, typename PT>
static int launch_one(const BMat &M, const XT *x, XT *y, int kind, hipStream_t s) {
  switch (kind) {
    case kApplySell: return launch_sell<XT, PT>(M, x, y, s);
    case kApplyTile: return launch_tile<XT, PT>(M, x, y, s);
    case kApplyRows: return launch_rowthread<XT, PT>(M, x, y, s);
    case kApplySeg: return launch_seg<XT, PT>(M, x, y, s);
    default: return launch_vec<XT>(M, x, y, M.lanes > 0 ? M.lanes : pick_lanes(M, M.nnz), s);
  }
}

// Many right-hand sides (R a multiple of 4, as k_bspmm4) when every stored
// bucket has an ELL copy: a row's column codes and values arrive in the ELL
// copies' vector loads (byte or int16 codes where the bucket has them: 1 or
// 2 bytes per entry instead of 4), then their 16-byte gathers of x.  Same
// order of operations as k_bspmm4; padding entries add +0.
template <int U, typename PT, typename XT>
__device__ __forceinline__ void bspmm4_ell_chunk(const BMat &M, int k, int64_t e, int row, const int32_t *dict,
                                                 const XT *__restrict__ x, int64_t ld, int c0, PT (&acc)[4]) {
  int cc[U];
  PT vv[U];
  ell_cols<U>(M, k, e, row, dict, cc);
  if constexpr (U == 4)
    ell_vals4<PT>(M, k, e, vv);
  else
    ell_vals8<PT>(M, k, e, vv);
  double xv[U][4];
#pragma unroll
  for (int t = 0; t < U; t++) ld4<XT>(x + (int64_t)cc[t] * ld + c0, xv[t]);
#pragma unroll
  for (int t = 0; t < U; t++)
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if constexpr (sizeof(PT) == 8)
        acc[u] = fma(vv[t], xv[t][u], acc[u]);
      else
        acc[u] = fmaf(vv[t], (float)xv[t][u], acc[u]);
    }
}

template <typename XT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmm4_ell(BMat M, const XT *__restrict__ x, XT *__restrict__ y,
                                                              int64_t ld, int nrhs) {
  __shared__ int32_t sdict[kMaxBuckets * 256];
  bool staged = false;
  for (int k = 0; k < M.nb; k++) {
    if (M.ell_cw[k] == 1) {
      for (int t = threadIdx.x; t < 256; t += blockDim.x) sdict[256 * k + t] = M.ell_dict[k][t];
      staged = true;
    }
  }
  if (staged) __syncthreads();
  const int tpr = nrhs / 4, rpb = kApplyThreads / tpr;
  const int g = threadIdx.x / tpr, c0 = 4 * (threadIdx.x % tpr);
  const int i = xcd_block(blockIdx.x, gridDim.x) * rpb + g;
  if (g >= rpb || i >= M.n) return;
  double total[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < M.nb; k++) {
    const int ew = M.ell_w[k];
    const int64_t e0 = (int64_t)i * ew;
    const int32_t *dict = sdict + 256 * k;
    if (M.prec[k] == BSPAI_FP64 || sizeof(XT) == 8) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (ew == 4)
        bspmm4_ell_chunk<4, double, XT>(M, k, e0, i, dict, x, ld, c0, acc);
      else
        for (int q = 0; q < ew; q += 8) bspmm4_ell_chunk<8, double, XT>(M, k, e0 + q, i, dict, x, ld, c0, acc);
#pragma unroll
      for (int u = 0; u < 4; u++) total[u] += acc[u] * M.scale[k];
    } else {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      if (ew == 4)
        bspmm4_ell_chunk<4, float, XT>(M, k, e0, i, dict, x, ld, c0, acc);
      else
        for (int q = 0; q < ew; q += 8) bspmm4_ell_chunk<8, float, XT>(M, k, e0 + q, i, dict, x, ld, c0, acc);
#pragma unroll
      for (int u = 0; u < 4; u++) total[u] += (double)acc[u] * M.scale[k];
    }
  }
  XT *yp = y + (int64_t)i * ld + c0;
  if (sizeof(XT) == 4) {
    *reinterpret_cast<float4 *>(yp) = make_float4((float)total[0], (float)total[1], (float)total[2], (float)total[3]);
  } else {
    reinterpret_cast<double2 *>(yp)[0] = make_double2(total[0], total[1]);
    reinterpret_cast<double2 *>(yp)[1] = make_double2(total[2], total[3]);
  }
}

// One stored bucket in ELL form (the common case of a stencil operator):
// k_bspmm4_ell with the value format fixed at compile time, so the kernel
// keeps few registers and many waves in flight; codes and values are read
// once, with non-temporal loads.  Same order of operations.
template <int U, int FMT, typename PT>
__device__ __forceinline__ void ell1_vals(const void *val, int64_t e, PT (&v)[U]) {
  if constexpr (FMT == BSPAI_FP64) {
#pragma unroll
    for (int t = 0; t < U; t += 2) {
      const f64x2 a = ld_stream<true, f64x2>(static_cast<const double *>(val) + e + t);
      v[t] = (PT)a.x, v[t + 1] = (PT)a.y;
    }
  } else if constexpr (FMT == BSPAI_FP32) {
#pragma unroll
    for (int t = 0; t < U; t += 4) {
      const f32x4 a = ld_stream<true, f32x4>(static_cast<const float *>(val) + e + t);
      v[t] = a.x, v[t + 1] = a.y, v[t + 2] = a.z, v[t + 3] = a.w;
    }
  } else if constexpr (FMT == BSPAI_FP16 || FMT == BSPAI_BF16) {
    uint32_t w[U / 2];
    if constexpr (U == 8) {
      const u32x4 a = ld_stream<true, u32x4>(static_cast<const uint16_t *>(val) + e);
      w[0] = a.x, w[1] = a.y, w[2] = a.z, w[3] = a.w;
    } else {
      const u32x2 a = ld_stream<true, u32x2>(static_cast<const uint16_t *>(val) + e);
      w[0] = a.x, w[1] = a.y;
    }
#pragma unroll
    for (int t = 0; t < U; t++) {
      const uint16_t h = (uint16_t)((w[t >> 1] >> (16 * (t & 1))) & 0xFFFFu);
      v[t] = (PT)(FMT == BSPAI_FP16 ? decode_f16(h) : decode_bf16(h));
    }
  } else {
    uint32_t w[2] = {0u, 0u};
    if constexpr (U == 8) {
      const u32x2 a = ld_stream<true, u32x2>(static_cast<const uint8_t *>(val) + e);
      w[0] = a.x, w[1] = a.y;
    } else {
      w[0] = ld_stream<true, uint32_t>(static_cast<const uint8_t *>(val) + e);
    }
#pragma unroll
    for (int t = 0; t < U; t++) v[t] = (PT)decode_e4m3((uint8_t)((w[t >> 2] >> (8 * (t & 3))) & 0xFFu));
  }
}

template <int U>
__device__ __forceinline__ void ell1_cols(const BMat &M, int cw, int64_t e, int row, const int32_t *dict,
                                          int (&c)[U]) {
  if (cw == 1) {
    uint32_t q[2] = {0u, 0u};
    if constexpr (U == 8) {
      const u32x2 a = ld_stream<true, u32x2>(static_cast<const uint8_t *>(M.ell_code[0]) + e);
      q[0] = a.x, q[1] = a.y;
    } else {
      q[0] = ld_stream<true, uint32_t>(static_cast<const uint8_t *>(M.ell_code[0]) + e);
    }
#pragma unroll
    for (int t = 0; t < U; t++) c[t] = row + dict[(q[t >> 2] >> (8 * (t & 3))) & 0xFFu];
  } else if (cw == 2) {
    uint32_t q[4] = {0u, 0u, 0u, 0u};
    if constexpr (U == 8) {
      const u32x4 a = ld_stream<true, u32x4>(static_cast<const int16_t *>(M.ell_code[0]) + e);
      q[0] = a.x, q[1] = a.y, q[2] = a.z, q[3] = a.w;
    } else {
      const u32x2 a = ld_stream<true, u32x2>(static_cast<const int16_t *>(M.ell_code[0]) + e);
      q[0] = a.x, q[1] = a.y;
    }
#pragma unroll
    for (int t = 0; t < U; t++) c[t] = row + (int32_t)(int16_t)((q[t >> 1] >> (16 * (t & 1))) & 0xFFFFu);
  } else {
#pragma unroll
    for (int t = 0; t < U; t += 4) {
      const i32x4 a = ld_stream<true, i32x4>(M.ell_col[0] + e + t);
      c[t] = a.x, c[t + 1] = a.y, c[t + 2] = a.z, c[t + 3] = a.w;
    }
  }
}

template <int U, int FMT, typename XT, typename PT>
__device__ __forceinline__ void bspmm4_ell1_chunk(const BMat &M, int cw, int64_t e, int row, const int32_t *dict,
                                                  const XT *__restrict__ x, int64_t ld, int c0, PT (&acc)[4]) {
  int cc[U];
  PT vv[U];
  ell1_cols<U>(M, cw, e, row, dict, cc);
  ell1_vals<U, FMT, PT>(M.ell_val[0], e, vv);
  double xv[U][4];
#pragma unroll
  for (int t = 0; t < U; t++) ld4<XT>(x + (int64_t)cc[t] * ld + c0, xv[t]);
#pragma unroll
  for (int t = 0; t < U; t++)
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if constexpr (sizeof(PT) == 8)
        acc[u] = fma(vv[t], xv[t][u], acc[u]);
      else
        acc[u] = fmaf(vv[t], (float)xv[t][u], acc[u]);
    }
}

template <typename XT, int FMT>
__global__ void __launch_bounds__(kApplyThreads) k_bspmm4_ell1(BMat M, const XT *__restrict__ x, XT *__restrict__ y,
                                                               int64_t ld, int nrhs) {
  using PT = typename std::conditional<FMT == BSPAI_FP64 || sizeof(XT) == 8, double, float>::type;
  __shared__ int32_t sdict[256];
  const int cw = M.ell_cw[0], ew = M.ell_w[0];
  if (cw == 1) {
    sdict[threadIdx.x] = M.ell_dict[0][threadIdx.x];  // kApplyThreads == 256
    __syncthreads();
  }
  const int tpr = nrhs / 4, rpb = kApplyThreads / tpr;
  const int g = threadIdx.x / tpr, c0 = 4 * (threadIdx.x % tpr);
  const int i = xcd_block(blockIdx.x, gridDim.x) * rpb + g;
  if (g >= rpb || i >= M.n) return;
  PT acc[4] = {(PT)0, (PT)0, (PT)0, (PT)0};
  const int64_t e0 = (int64_t)i * ew;
  if (ew == 4)
    bspmm4_ell1_chunk<4, FMT, XT, PT>(M, cw, e0, i, sdict, x, ld, c0, acc);
  else
    for (int q = 0; q < ew; q += 8) bspmm4_ell1_chunk<8, FMT, XT, PT>(M, cw, e0 + q, i, sdict, x, ld, c0, acc);
  double total[4];
#pragma unroll
  for (int u = 0; u < 4; u++) total[u] = (double)acc[u] * M.scale[0];
  XT *yp = y + (int64_t)i * ld + c0;
  if (sizeof(XT) == 4) {
    *reinterpret_cast<float4 *>(yp) = make_float4((float)total[0], (float)total[1], (float)total[2], (float)total[3]);
  } else {
    reinterpret_cast<double2 *>(yp)[0] = make_double2(total[0], total[1]);
    reinterpret_cast<double2 *>(yp)[1] = make_double2(total[2], total[3]);
  }
}

template <typename XT>
static void *bspmm4_ell1_kernel(int fmt) {
  switch (fmt) {
    case BSPAI_FP64: return (void *)k_bspmm4_ell1<XT, BSPAI_FP64>;
    case BSPAI_FP32: return (void *)k_bspmm4_ell1<XT, BSPAI_FP32>;
    case BSPAI_FP16: return (void *)k_bspmm4_ell1<XT, BSPAI_FP16>;
    case BSPAI_BF16: return (void *)k_bspmm4_ell1<XT, BSPAI_BF16>;
    default: return (void *)k_bspmm4_ell1<XT, BSPAI_FP8_E4M3>;
  }
}

int launch_bspmv(const BMat &M, const void *x, void *y, int nrhs, int64_t ld, int fp64, hipStream_t s) {
  if (M.n == 0) return BSPAI_OK;
  if (nrhs == 1) {
    const int kind = apply_kind_resolved(M);
    if (fp64) return launch_one<double, double>(M, static_cast<const double *>(x), static_cast<double *>(y), kind, s);
    if (has_fp64_bucket(M))
      return launch_one<float, double>(M, static_cast<const float *>(x), static_cast<float *>(y), kind, s);
    return launch_one<float, float>(M, static_cast<const float *>(x), static_cast<float *>(y), kind, s);
  }
  if (nrhs % 4 == 0 && nrhs <= 64 && ld % 4 == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0 &&
      (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
    const int rpb = kApplyThreads / (nrhs / 4);
    const int64_t nblk = (M.n + rpb - 1) / rpb;
    const bool ell = all_ell(M);
    if (ell && M.nb == 1) {  // one ELL bucket: the format-specialised kernel
      BMat Mc = M;
      int nr = nrhs;
      void *args[] = {&Mc, const_cast<void **>(&x), &y, &ld, &nr};
      void *fn = fp64 ? bspmm4_ell1_kernel<double>(M.prec[0]) : bspmm4_ell1_kernel<float>(M.prec[0]);
      BSPAI_HIP(hipLaunchKernel(fn, dim3((unsigned)nblk), dim3(kApplyThreads), args, 0, s));
    } else if (fp64)
      hipLaunchKernelGGL(ell ? k_bspmm4_ell<double> : k_bspmm4<double>, dim3((unsigned)nblk), dim3(kApplyThreads),
                         0, s, M, static_cast<const double *>(x), static_cast<double *>(y), ld, nrhs);
    else
      hipLaunchKernelGGL(ell ? k_bspmm4_ell<float> : k_bspmm4<float>, dim3((unsigned)nblk), dim3(kApplyThreads), 0,
                         s, M, static_cast<const float *>(x), static_cast<float *>(y), ld, nrhs);
    BSPAI_CHECK_LAUNCH();
    return BSPAI_OK;
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

// ------------------------------------------------------------------ kernel choice

namespace bspai {

__global__ void k_fill_pattern(int n, float *x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 1.0f + 0.125f * (float)(i % 13);
}

// average time of `reps` products with kernel `kind` (fp32 vectors)
static int time_kind(const BMat &M, int kind, const float *x, float *y, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                     float *ms) {
  BMat T = M;
  T.apply_kind = kind;
  constexpr int kWarm = 2, kReps = 20;
  for (int r = 0; r < kWarm; r++) {
    int rc = launch_bspmv(T, x, y, 1, 1, 0, s);
    if (rc) return rc;
  }
  BSPAI_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < kReps; r++) {
    int rc = launch_bspmv(T, x, y, 1, 1, 0, s);
    if (rc) return rc;
  }
  BSPAI_HIP(hipEventRecord(e1, s));
  BSPAI_HIP(hipEventSynchronize(e1));
  BSPAI_HIP(hipEventElapsedTime(ms, e0, e1));
  *ms /= kReps;
  return BSPAI_OK;
}

static int tune_one(BMat &M, const float *x, float *y, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  int best = kApplyAuto;
  float best_ms = 0.f;
  for (int kind : {kApplySell, kApplyTile, kApplyRows, kApplyLanes, kApplySeg}) {
    if (!apply_kind_ok(M, kind)) continue;
    float ms = 0.f;
    int rc = time_kind(M, kind, x, y, s, e0, e1, &ms);
    if (rc) return rc;
    if (best == kApplyAuto || ms < best_ms) best = kind, best_ms = ms;
  }
  M.apply_kind = best;
  return BSPAI_OK;
}

}  // namespace bspai

extern "C" int bspai_set_apply_kind(bspai_handle *M, int trans, int kind) {
  using namespace bspai;
  if (!M) return fail(BSPAI_EINVAL, "bspai_set_apply_kind: null handle");
  if (trans && !M->has_T) return fail(BSPAI_EINVAL, "bspai_set_apply_kind: handle built without build_T");
  BMat &B = trans ? M->matT : M->mat;
  if (kind < kApplyAuto || kind > kApplySeg || !apply_kind_ok(B, kind))
    return fail(BSPAI_EINVAL, "bspai_set_apply_kind: kernel %d is not available for this matrix", kind);
  B.apply_kind = kind;
  return BSPAI_OK;
}

extern "C" int bspai_tune_apply(bspai_handle *M, void *stream) {
  using namespace bspai;
  if (!M) return fail(BSPAI_EINVAL, "bspai_tune_apply: null handle");
  if (M->n == 0 || M->mat.nb == 0) return BSPAI_OK;
  int dev = 0;
  BSPAI_HIP(hipGetDevice(&dev));
  if (dev != M->device) return fail(BSPAI_EINVAL, "bspai_tune_apply: handle lives on device %d", M->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *x = nullptr, *y = nullptr;
  int rc;
  if ((rc = dalloc_t(&x, (size_t)M->n)) || (rc = dalloc_t(&y, (size_t)M->n))) {
    dfree(x);
    return rc;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto body = [&]() -> int {
    BSPAI_HIP(hipEventCreate(&e0));
    BSPAI_HIP(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_fill_pattern, dim3((M->n + 255) / 256), dim3(256), 0, s, M->n, x);
    BSPAI_CHECK_LAUNCH();
    int r = tune_one(M->mat, x, y, s, e0, e1);
    if (!r && M->has_T) r = tune_one(M->matT, x, y, s, e0, e1);
    return r;
  };
  rc = body();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  dfree(x), dfree(y);
  return rc;
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
