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
    if (fp64)
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
  for (int kind : {kApplySell, kApplyTile, kApplyRows, kApplyLanes}) {
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
  if (kind < kApplyAuto || kind > kApplyLanes || !apply_kind_ok(B, kind))
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
