// Device routines for the bucketed product y = M_b x (Algorithm 3 with the
// storage precision of each bucket decoupled from the arithmetic).
//
// Each stored bucket is its own CSR (row pointers, int32 columns, values of
// the bucket's width).  A group of L consecutive lanes handles one row: the
// lanes stride over the row's entries of a bucket, decode each stored value
// exactly to binary32, multiply by x and accumulate; the group then reduces
// with cross-lane shuffles.  The partial sum of a bucket is accumulated in
// FP32 (FP64 for the fp64 bucket, and for everything when the vectors are
// FP64), scaled by the bucket's power-of-two storage scale (exact), and the
// partials are added in FP64 from the least to the most precise bucket.
#pragma once

#include "common.h"
#include "formats.h"

namespace bspai {

template <typename T>
__device__ __forceinline__ T group_sum(T v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

// value of entry p of bucket k as float (exact for every narrow format)
__device__ __forceinline__ float load_value_f32(const BMat &M, int k, int64_t p) {
  switch (M.prec[k]) {
    case BSPAI_FP32: return static_cast<const float *>(M.val[k])[p];
    case BSPAI_FP16: return decode_f16(static_cast<const uint16_t *>(M.val[k])[p]);
    case BSPAI_BF16: return decode_bf16(static_cast<const uint16_t *>(M.val[k])[p]);
    case BSPAI_FP8_E4M3: return decode_e4m3(static_cast<const uint8_t *>(M.val[k])[p]);
  }
  return 0.f;
}

// y_i for one row with L lanes; XT = float (FP32 vectors) or double.
// Returns the row value in FP64 on every lane of the group.
template <int L, typename XT>
__device__ __forceinline__ double bspmv_row(const BMat &M, const XT *__restrict__ x, int i, int lane) {
  double total = 0.0;
  for (int k = 0; k < M.nb; k++) {
    const int32_t *rp = M.rp[k];
    const int32_t *col = M.col[k];
    int s = rp[i], e = rp[i + 1];
    if (M.prec[k] == BSPAI_FP64 || sizeof(XT) == 8) {
      double acc = 0.0;
      if (M.prec[k] == BSPAI_FP64) {
        const double *v = static_cast<const double *>(M.val[k]);
        for (int p = s + lane; p < e; p += L) acc = fma(v[p], (double)x[col[p]], acc);
      } else {
        for (int p = s + lane; p < e; p += L) acc = fma((double)load_value_f32(M, k, p), (double)x[col[p]], acc);
      }
      acc = group_sum(acc, L);
      total += acc * M.scale[k];
    } else {
      float acc = 0.f;
      switch (M.prec[k]) {
        case BSPAI_FP32: {
          const float *v = static_cast<const float *>(M.val[k]);
          for (int p = s + lane; p < e; p += L) acc = fmaf(v[p], (float)x[col[p]], acc);
        } break;
        case BSPAI_FP16: {
          const uint16_t *v = static_cast<const uint16_t *>(M.val[k]);
          for (int p = s + lane; p < e; p += L) acc = fmaf(decode_f16(v[p]), (float)x[col[p]], acc);
        } break;
        case BSPAI_BF16: {
          const uint16_t *v = static_cast<const uint16_t *>(M.val[k]);
          for (int p = s + lane; p < e; p += L) acc = fmaf(decode_bf16(v[p]), (float)x[col[p]], acc);
        } break;
        case BSPAI_FP8_E4M3: {
          const uint8_t *v = static_cast<const uint8_t *>(M.val[k]);
          for (int p = s + lane; p < e; p += L) acc = fmaf(decode_e4m3(v[p]), (float)x[col[p]], acc);
        } break;
      }
      acc = group_sum(acc, L);
      total += (double)acc * M.scale[k];
    }
  }
  return total;
}

// Rows [r0, r1) of y = M_b x, one group of L lanes per row, groups of the
// calling block striding over the rows.
template <int L, typename XT, typename YT>
__device__ __forceinline__ void bspmv_rows(const BMat &M, const XT *__restrict__ x, YT *__restrict__ y, int r0,
                                           int r1) {
  const int lane = threadIdx.x & (L - 1);
  const int ngroups = blockDim.x / L;
  for (int i = r0 + (int)threadIdx.x / L; i < r1; i += ngroups) {
    double v = bspmv_row<L, XT>(M, x, i, lane);
    if (lane == 0) y[i] = (YT)v;
  }
}

// Y = M_b X for nrhs right-hand sides stored row-major (leading dimension ld):
// a group of G lanes (G >= nrhs, power of two) per row, one lane per column.
template <typename XT>
__device__ __forceinline__ void bspmm_row(const BMat &M, const XT *__restrict__ x, XT *__restrict__ y, int64_t ld,
                                          int i, int c, bool active) {
  double total = 0.0;
  for (int k = 0; k < M.nb; k++) {
    int s = M.rp[k][i], e = M.rp[k][i + 1];
    const int32_t *col = M.col[k];
    if (M.prec[k] == BSPAI_FP64 || sizeof(XT) == 8) {
      double acc = 0.0;
      for (int p = s; p < e; p++) {
        double v = M.prec[k] == BSPAI_FP64 ? static_cast<const double *>(M.val[k])[p]
                                           : (double)load_value_f32(M, k, p);
        if (active) acc = fma(v, (double)x[(int64_t)col[p] * ld + c], acc);
      }
      total += acc * M.scale[k];
    } else {
      float acc = 0.f;
      for (int p = s; p < e; p++) {
        float v = load_value_f32(M, k, p);
        if (active) acc = fmaf(v, (float)x[(int64_t)col[p] * ld + c], acc);
      }
      total += (double)acc * M.scale[k];
    }
  }
  if (active) y[(int64_t)i * ld + c] = (XT)total;
}

}  // namespace bspai
