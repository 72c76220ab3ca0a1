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

// ---------------------------------------------------------------- tiles
//
// Two-phase product for a contiguous range of rows (used when a row has few
// entries).  Phase 1: the block streams the entries of the range, which are
// contiguous in each bucket's arrays, with wide aligned loads (8 entries per
// thread and pass), gathers x and writes each product to LDS.  Phase 2: one
// thread per row adds its products from LDS in CSR order.  The per-bucket row
// sums are then scaled and added from the least to the most precise bucket in
// FP64, as in bspmv_row.  Many independent loads per thread keep enough bytes
// in flight to stream HBM; the per-row order stays fixed (deterministic).

constexpr int kTileVec = 8;  // entries per thread and pass

// vector loads, optionally non-temporal (data read once: leave the caches to
// the gathered vector)
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <bool NT, typename V>
__device__ __forceinline__ V ld_stream(const void *p) {
  const V *q = static_cast<const V *>(p);
  if (NT) return __builtin_nontemporal_load(q);
  return *q;
}

template <typename PT, bool NT = false>
__device__ __forceinline__ void load_vals8(const BMat &M, int k, int64_t base, PT (&v)[kTileVec]) {
  // base is a multiple of 8 entries: every load below is naturally aligned
  switch (M.prec[k]) {
    case BSPAI_FP64: {
      const double *p = static_cast<const double *>(M.val[k]) + base;
      f64x4 a = ld_stream<NT, f64x4>(p), b = ld_stream<NT, f64x4>(p + 4);
      v[0] = (PT)a.x; v[1] = (PT)a.y; v[2] = (PT)a.z; v[3] = (PT)a.w;
      v[4] = (PT)b.x; v[5] = (PT)b.y; v[6] = (PT)b.z; v[7] = (PT)b.w;
    } break;
    case BSPAI_FP32: {
      const float *p = static_cast<const float *>(M.val[k]) + base;
      f32x4 a = ld_stream<NT, f32x4>(p), b = ld_stream<NT, f32x4>(p + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } break;
    case BSPAI_FP16: {
      u32x4 a = ld_stream<NT, u32x4>(static_cast<const uint16_t *>(M.val[k]) + base);
      uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int t = 0; t < 4; t++) {
        v[2 * t] = decode_f16((uint16_t)(w[t] & 0xFFFFu));
        v[2 * t + 1] = decode_f16((uint16_t)(w[t] >> 16));
      }
    } break;
    case BSPAI_BF16: {
      u32x4 a = ld_stream<NT, u32x4>(static_cast<const uint16_t *>(M.val[k]) + base);
      uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int t = 0; t < 4; t++) {
        v[2 * t] = decode_bf16((uint16_t)(w[t] & 0xFFFFu));
        v[2 * t + 1] = decode_bf16((uint16_t)(w[t] >> 16));
      }
    } break;
    case BSPAI_FP8_E4M3: {
      u32x2 a = ld_stream<NT, u32x2>(static_cast<const uint8_t *>(M.val[k]) + base);
      uint32_t w[2] = {a.x, a.y};
#pragma unroll
      for (int t = 0; t < 8; t++) v[t] = decode_e4m3((uint8_t)((w[t >> 2] >> (8 * (t & 3))) & 0xFFu));
    } break;
    default:
#pragma unroll
      for (int t = 0; t < kTileVec; t++) v[t] = (PT)0;
  }
}

// Rows [r0, r1) of y = M_b x with the two-phase tile method; sub-ranges of
// at most `rows_cap` rows whose entries of a bucket exceed `cap` products fall
// back to the L-lane method for that bucket.  prod: LDS [cap] of PT,
// acc: LDS [rows_cap] doubles, rps: LDS [rows_cap + 1] ints.  All threads of
// the block must call this.
template <typename XT, typename YT, typename PT>
__device__ void bspmv_tile_rows(const BMat &M, const XT *__restrict__ x, YT *__restrict__ y, int r0, int r1,
                                PT *prod, int cap, double *acc, int rows_cap, int32_t *rps) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int s0 = r0; s0 < r1; s0 += rows_cap) {
    const int s1 = min(r1, s0 + rows_cap);
    for (int i = s0 + tid; i < s1; i += nt) acc[i - s0] = 0.0;
    for (int k = 0; k < M.nb; k++) {
      const int32_t *col = M.col[k];
      // the sub-range's row pointers of this bucket, staged in LDS
      for (int i = s0 + tid; i <= s1; i += nt) rps[i - s0] = M.rp[k][i];
      __syncthreads();
      const int32_t *rp = rps - s0;
      const int e0 = rp[s0], e1 = rp[s1];
      const double sc = M.scale[k];
      const bool wide = (M.prec[k] == BSPAI_FP64) || sizeof(PT) == 8;
      if (e1 - e0 <= cap) {
        const int eb = e0 & ~(kTileVec - 1);
        for (int base = eb + tid * kTileVec; base < e1; base += nt * kTileVec) {
          if (base >= e0 && base + kTileVec <= e1) {
            // 8 entries inside the range: aligned non-temporal vector loads
            // (read once, so x keeps the caches), 8 gathers in flight
            i32x4 ca = ld_stream<true, i32x4>(col + base);
            i32x4 cb = ld_stream<true, i32x4>(col + base + 4);
            int cc[kTileVec] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
            PT vv[kTileVec];
            load_vals8<PT, true>(M, k, base, vv);
            PT xv[kTileVec];
#pragma unroll
            for (int t = 0; t < kTileVec; t++) xv[t] = (PT)x[cc[t]];
#pragma unroll
            for (int t = 0; t < kTileVec; t++) prod[base + t - e0] = vv[t] * xv[t];
          } else {
            // the ends of the range: element by element, never outside [e0, e1)
            for (int t = 0; t < kTileVec; t++) {
              int e = base + t;
              if (e >= e0 && e < e1) {
                PT v = M.prec[k] == BSPAI_FP64 ? (PT) static_cast<const double *>(M.val[k])[e]
                                               : (PT)load_value_f32(M, k, e);
                prod[e - e0] = v * (PT)x[col[e]];
              }
            }
          }
        }
        __syncthreads();
        for (int i = s0 + tid; i < s1; i += nt) {
          int a = rp[i] - e0, b = rp[i + 1] - e0;
          if (wide) {
            double sum = 0.0;
            for (int q = a; q < b; q++) sum += (double)prod[q];
            acc[i - s0] += sum * sc;
          } else {
            float sum = 0.f;
            for (int q = a; q < b; q++) sum += (float)prod[q];
            acc[i - s0] += (double)sum * sc;
          }
        }
        __syncthreads();
      } else {
        // long rows: one group of 8 lanes per row (this bucket only)
        const int lane = tid & 7;
        for (int i = s0 + tid / 8; i < s1; i += nt / 8) {
          double v;
          int a = rp[i], b = rp[i + 1];
          if (wide) {
            double sum = 0.0;
            for (int q = a + lane; q < b; q += 8)
              sum = fma(M.prec[k] == BSPAI_FP64 ? static_cast<const double *>(M.val[k])[q]
                                                : (double)load_value_f32(M, k, q),
                        (double)x[col[q]], sum);
            v = group_sum(sum, 8);
          } else {
            float sum = 0.f;
            for (int q = a + lane; q < b; q += 8) sum = fmaf(load_value_f32(M, k, q), (float)x[col[q]], sum);
            v = (double)group_sum(sum, 8);
          }
          if (lane == 0) acc[i - s0] += v * sc;
        }
        __syncthreads();
      }
    }
    for (int i = s0 + tid; i < s1; i += nt) y[i] = (YT)acc[i - s0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- rows
//
// One thread per row: the row's entries of a bucket are fetched 8 at a time
// with independent (predicated) loads of columns and values, then 8 gathers of
// x, then the FMAs in CSR order.  No LDS and no block barrier: every wave
// streams on its own, with up to 8 entries x 3 loads in flight per lane.

template <typename PT>
__device__ __forceinline__ PT value_at(const BMat &M, int k, int64_t p) {
  if (M.prec[k] == BSPAI_FP64) return (PT) static_cast<const double *>(M.val[k])[p];
  return (PT)load_value_f32(M, k, p);
}

template <typename XT, typename YT, typename PT>
__device__ __forceinline__ double bspmv_row_thread(const BMat &M, const XT *__restrict__ x, int i) {
  constexpr int U = 8;
  double total = 0.0;
  for (int k = 0; k < M.nb; k++) {
    const int32_t *col = M.col[k];
    const int s = M.rp[k][i], e = M.rp[k][i + 1];
    const bool wide = (M.prec[k] == BSPAI_FP64) || sizeof(PT) == 8;
    double accd = 0.0;
    float accf = 0.f;
    for (int p = s; p < e; p += U) {
      int cc[U];
      PT vv[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        bool ok = p + u < e;
        cc[u] = ok ? col[p + u] : 0;
        vv[u] = ok ? value_at<PT>(M, k, p + u) : (PT)0;
      }
      PT xv[U];
#pragma unroll
      for (int u = 0; u < U; u++) xv[u] = (p + u < e) ? (PT)x[cc[u]] : (PT)0;
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (p + u < e) {
          if (wide)
            accd = fma((double)vv[u], (double)xv[u], accd);
          else
            accf = fmaf((float)vv[u], (float)xv[u], accf);
        }
      }
    }
    total += (wide ? accd : (double)accf) * M.scale[k];
  }
  return total;
}

// RT rows per thread (rows i0 + r * stride): the load chains of the rows are
// interleaved so that RT times as many bytes are in flight per lane.
template <int RT, typename XT, typename PT>
__device__ __forceinline__ void bspmv_rows_thread(const BMat &M, const XT *__restrict__ x, const int (&rows)[RT],
                                                  double (&out)[RT]) {
  constexpr int U = 8;
#pragma unroll
  for (int r = 0; r < RT; r++) out[r] = 0.0;
  for (int k = 0; k < M.nb; k++) {
    const int32_t *col = M.col[k];
    const int32_t *rp = M.rp[k];
    const bool wide = (M.prec[k] == BSPAI_FP64) || sizeof(PT) == 8;
    int s[RT], e[RT];
#pragma unroll
    for (int r = 0; r < RT; r++) {
      bool ok = rows[r] >= 0;
      s[r] = ok ? rp[rows[r]] : 0;
      e[r] = ok ? rp[rows[r] + 1] : 0;
    }
    int len = 0;
#pragma unroll
    for (int r = 0; r < RT; r++) len = max(len, e[r] - s[r]);
    double accd[RT];
    float accf[RT];
#pragma unroll
    for (int r = 0; r < RT; r++) {
      accd[r] = 0.0;
      accf[r] = 0.f;
    }
    for (int o = 0; o < len; o += U) {
      int cc[RT][U];
      PT vv[RT][U];
#pragma unroll
      for (int r = 0; r < RT; r++)
#pragma unroll
        for (int u = 0; u < U; u++) {
          int p = s[r] + o + u;
          bool ok = p < e[r];
          cc[r][u] = ok ? col[p] : 0;
          vv[r][u] = ok ? value_at<PT>(M, k, p) : (PT)0;
        }
      PT xv[RT][U];
#pragma unroll
      for (int r = 0; r < RT; r++)
#pragma unroll
        for (int u = 0; u < U; u++) xv[r][u] = (s[r] + o + u < e[r]) ? (PT)x[cc[r][u]] : (PT)0;
#pragma unroll
      for (int r = 0; r < RT; r++)
#pragma unroll
        for (int u = 0; u < U; u++) {
          if (s[r] + o + u < e[r]) {
            if (wide)
              accd[r] = fma((double)vv[r][u], (double)xv[r][u], accd[r]);
            else
              accf[r] = fmaf((float)vv[r][u], (float)xv[r][u], accf[r]);
          }
        }
    }
#pragma unroll
    for (int r = 0; r < RT; r++) out[r] += (wide ? accd[r] : (double)accf[r]) * M.scale[k];
  }
}

// ---------------------------------------------------------------- SELL-64
//
// One wavefront per 64-row slice, lane r on row 64 s + r.  Entry u of the
// slice's rows is one contiguous 64-wide column, so every load instruction of
// columns (256 B) and values (64 x width) is contiguous; the slice's columns
// are fetched 8 at a time before their gathers of x.  Short rows are padded
// with zero values (adding +0 leaves the FP sum unchanged).  Per row the
// entries are added in CSR order.

template <typename PT>
__device__ __forceinline__ PT sell_value(const BMat &M, int k, int64_t p) {
  if (M.prec[k] == BSPAI_FP64) return (PT) static_cast<const double *>(M.sell_val[k])[p];
  switch (M.prec[k]) {
    case BSPAI_FP32: return (PT) static_cast<const float *>(M.sell_val[k])[p];
    case BSPAI_FP16: return (PT)decode_f16(static_cast<const uint16_t *>(M.sell_val[k])[p]);
    case BSPAI_BF16: return (PT)decode_bf16(static_cast<const uint16_t *>(M.sell_val[k])[p]);
    case BSPAI_FP8_E4M3: return (PT)decode_e4m3(static_cast<const uint8_t *>(M.sell_val[k])[p]);
  }
  return (PT)0;
}

// 4 consecutive stored values of an ELL bucket (entry e a multiple of 4)
template <typename PT>
__device__ __forceinline__ void ell_vals4(const BMat &M, int k, int64_t e, PT (&v)[4]) {
  switch (M.prec[k]) {
    case BSPAI_FP64: {
      const double2 *p = reinterpret_cast<const double2 *>(static_cast<const double *>(M.ell_val[k]) + e);
      double2 a = p[0], b = p[1];
      v[0] = (PT)a.x; v[1] = (PT)a.y; v[2] = (PT)b.x; v[3] = (PT)b.y;
    } break;
    case BSPAI_FP32: {
      float4 a = *reinterpret_cast<const float4 *>(static_cast<const float *>(M.ell_val[k]) + e);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } break;
    case BSPAI_FP16: {
      uint2 a = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(M.ell_val[k]) + e);
      v[0] = decode_f16(a.x & 0xFFFFu); v[1] = decode_f16(a.x >> 16);
      v[2] = decode_f16(a.y & 0xFFFFu); v[3] = decode_f16(a.y >> 16);
    } break;
    case BSPAI_BF16: {
      uint2 a = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(M.ell_val[k]) + e);
      v[0] = decode_bf16(a.x & 0xFFFFu); v[1] = decode_bf16(a.x >> 16);
      v[2] = decode_bf16(a.y & 0xFFFFu); v[3] = decode_bf16(a.y >> 16);
    } break;
    case BSPAI_FP8_E4M3: {
      uint32_t a = *reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(M.ell_val[k]) + e);
      v[0] = decode_e4m3(a & 0xFFu); v[1] = decode_e4m3((a >> 8) & 0xFFu);
      v[2] = decode_e4m3((a >> 16) & 0xFFu); v[3] = decode_e4m3(a >> 24);
    } break;
    default:
      v[0] = v[1] = v[2] = v[3] = (PT)0;
  }
}

// entries e .. e + 7 of bucket k's ELL values (e a multiple of 8): one
// 16-byte load for the 2-byte formats
template <typename PT>
__device__ __forceinline__ void ell_vals8(const BMat &M, int k, int64_t e, PT (&v)[8]) {
  switch (M.prec[k]) {
    case BSPAI_FP64: {
      const double2 *p = reinterpret_cast<const double2 *>(static_cast<const double *>(M.ell_val[k]) + e);
#pragma unroll
      for (int t = 0; t < 4; t++) {
        double2 a = p[t];
        v[2 * t] = (PT)a.x, v[2 * t + 1] = (PT)a.y;
      }
    } break;
    case BSPAI_FP32: {
      const float4 *p = reinterpret_cast<const float4 *>(static_cast<const float *>(M.ell_val[k]) + e);
      float4 a = p[0], b = p[1];
      v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
    } break;
    case BSPAI_FP16:
    case BSPAI_BF16: {
      uint4 a = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(M.ell_val[k]) + e);
      const uint32_t w4[4] = {a.x, a.y, a.z, a.w};
      const bool h = M.prec[k] == BSPAI_FP16;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        v[2 * t] = h ? decode_f16(w4[t] & 0xFFFFu) : decode_bf16(w4[t] & 0xFFFFu);
        v[2 * t + 1] = h ? decode_f16(w4[t] >> 16) : decode_bf16(w4[t] >> 16);
      }
    } break;
    case BSPAI_FP8_E4M3: {
      uint2 a = *reinterpret_cast<const uint2 *>(static_cast<const uint8_t *>(M.ell_val[k]) + e);
#pragma unroll
      for (int t = 0; t < 4; t++) {
        v[t] = decode_e4m3((a.x >> (8 * t)) & 0xFFu);
        v[4 + t] = decode_e4m3((a.y >> (8 * t)) & 0xFFu);
      }
    } break;
    default:
#pragma unroll
      for (int t = 0; t < 8; t++) v[t] = (PT)0;
  }
}

// columns of entries e .. e + N - 1 (N = 4 or 8, e a multiple of N) of row
// `row` in bucket k's ELL copy, from its byte codes (dict: the 256 offsets),
// int16 offsets or int32 columns
template <int N>
__device__ __forceinline__ void ell_cols(const BMat &M, int k, int64_t e, int row, const int32_t *dict, int (&c)[N]) {
  const int cw = M.ell_cw[k];
  if (cw == 1) {
    const uint8_t *p = static_cast<const uint8_t *>(M.ell_code[k]) + e;
    uint32_t q[2];
    if (N == 8) {
      uint2 t = *reinterpret_cast<const uint2 *>(p);
      q[0] = t.x, q[1] = t.y;
    } else {
      q[0] = *reinterpret_cast<const uint32_t *>(p), q[1] = 0;
    }
#pragma unroll
    for (int t = 0; t < N; t++) c[t] = row + dict[(q[t / 4] >> (8 * (t % 4))) & 0xFFu];
  } else if (cw == 2) {
    const int16_t *p = static_cast<const int16_t *>(M.ell_code[k]) + e;
    int32_t q[4];
    if (N == 8) {
      int4 t = *reinterpret_cast<const int4 *>(p);
      q[0] = t.x, q[1] = t.y, q[2] = t.z, q[3] = t.w;
    } else {
      int2 t = *reinterpret_cast<const int2 *>(p);
      q[0] = t.x, q[1] = t.y, q[2] = 0, q[3] = 0;
    }
#pragma unroll
    for (int t = 0; t < N; t++) c[t] = row + ((t & 1) ? (q[t / 2] >> 16) : (int32_t)(int16_t)(q[t / 2] & 0xFFFF));
  } else {
    const int4 *p = reinterpret_cast<const int4 *>(M.ell_col[k] + e);
#pragma unroll
    for (int t = 0; t < N / 4; t++) {
      int4 a = p[t];
      c[4 * t] = a.x, c[4 * t + 1] = a.y, c[4 * t + 2] = a.z, c[4 * t + 3] = a.w;
    }
  }
}

// row 64 sl + lane of M_b x: each bucket from its ELL copy (the row's own
// entries with 16-byte vector loads, narrow column codes) when present, else
// from its SELL-64 copy.  Entries are added in CSR order, padding adds +0.
// sdict: the buckets' offset tables staged in LDS (256 per bucket), or null.
template <typename XT, typename PT>
__device__ __forceinline__ double bspmv_sell_row(const BMat &M, const XT *__restrict__ x, int sl, int lane,
                                                 const int32_t *sdict) {
  constexpr int U = 8;
  const int row = sl * kSlice + lane;
  double total = 0.0;
  for (int k = 0; k < M.nb; k++) {
    const bool wide = (M.prec[k] == BSPAI_FP64) || sizeof(PT) == 8;
    double accd = 0.0;
    float accf = 0.f;
    const int ew = M.ell_w[k];
    if (ew) {
      if (row < M.n) {
        const int64_t e0 = (int64_t)row * ew;
        const int32_t *dict = sdict ? sdict + 256 * k : M.ell_dict[k];
        if (ew == 4) {
          int cc[4];
          PT vv[4];
          ell_cols<4>(M, k, e0, row, dict, cc);
          ell_vals4<PT>(M, k, e0, vv);
          PT xv[4];
#pragma unroll
          for (int u = 0; u < 4; u++) xv[u] = (PT)x[cc[u]];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            if (wide)
              accd = fma((double)vv[u], (double)xv[u], accd);
            else
              accf = fmaf((float)vv[u], (float)xv[u], accf);
          }
        } else {
          for (int c0 = 0; c0 < ew; c0 += U) {
            int cc[U];
            PT vv[U];
            ell_cols<U>(M, k, e0 + c0, row, dict, cc);
            ell_vals8<PT>(M, k, e0 + c0, vv);
            PT xv[U];
#pragma unroll
            for (int u = 0; u < U; u++) xv[u] = (PT)x[cc[u]];
#pragma unroll
            for (int u = 0; u < U; u++) {
              if (wide)
                accd = fma((double)vv[u], (double)xv[u], accd);
              else
                accf = fmaf((float)vv[u], (float)xv[u], accf);
            }
          }
        }
      }
    } else {
      const int w = M.sell_w[k];
      const int p0 = w ? sl * kSlice * w : M.sell_ptr[k][sl];
      const int len = w ? w : (M.sell_ptr[k][sl + 1] - p0) / kSlice;
      const int32_t *col = M.sell_col[k] + p0 + lane;
      const int64_t vbase = (int64_t)p0 + lane;
      for (int u0 = 0; u0 < len; u0 += U) {
        int cc[U];
        PT vv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          bool ok = u0 + u < len;  // uniform over the wavefront
          cc[u] = ok ? col[(u0 + u) * kSlice] : 0;
          vv[u] = ok ? sell_value<PT>(M, k, vbase + (int64_t)(u0 + u) * kSlice) : (PT)0;
        }
        PT xv[U];
#pragma unroll
        for (int u = 0; u < U; u++) xv[u] = (u0 + u < len) ? (PT)x[cc[u]] : (PT)0;
#pragma unroll
        for (int u = 0; u < U; u++) {
          if (u0 + u < len) {
            if (wide)
              accd = fma((double)vv[u], (double)xv[u], accd);
            else
              accf = fmaf((float)vv[u], (float)xv[u], accf);
          }
        }
      }
    }
    total += (wide ? accd : (double)accf) * M.scale[k];
  }
  return total;
}

// RT rows per thread when every stored bucket has an ELL copy: for each
// bucket and each 8-entry chunk, the column codes and values of all RT rows
// are loaded first, then their x entries, then the products are added, so a
// thread keeps RT independent load chains in flight.  rows[r] < 0: no row.
// Same order of operations per row as bspmv_sell_row.
template <int RT, typename XT, typename PT>
__device__ __forceinline__ void bspmv_ell_rows(const BMat &M, const XT *__restrict__ x, const int (&rows)[RT],
                                               const int32_t *sdict, double (&out)[RT]) {
#pragma unroll
  for (int r = 0; r < RT; r++) out[r] = 0.0;
  for (int k = 0; k < M.nb; k++) {
    const bool wide = (M.prec[k] == BSPAI_FP64) || sizeof(PT) == 8;
    const int ew = M.ell_w[k];
    const int32_t *dict = sdict ? sdict + 256 * k : M.ell_dict[k];
    double accd[RT];
    float accf[RT];
#pragma unroll
    for (int r = 0; r < RT; r++) accd[r] = 0.0, accf[r] = 0.f;
    if (ew == 4) {
      int cc[RT][4];
      PT vv[RT][4];
#pragma unroll
      for (int r = 0; r < RT; r++) {
        const int row = rows[r] < 0 ? 0 : rows[r];
        ell_cols<4>(M, k, (int64_t)row * 4, row, dict, cc[r]);
        ell_vals4<PT>(M, k, (int64_t)row * 4, vv[r]);
      }
      PT xv[RT][4];
#pragma unroll
      for (int r = 0; r < RT; r++)
#pragma unroll
        for (int u = 0; u < 4; u++) xv[r][u] = (PT)x[cc[r][u]];
#pragma unroll
      for (int r = 0; r < RT; r++)
#pragma unroll
        for (int u = 0; u < 4; u++) {
          if (wide)
            accd[r] = fma((double)vv[r][u], (double)xv[r][u], accd[r]);
          else
            accf[r] = fmaf((float)vv[r][u], (float)xv[r][u], accf[r]);
        }
    } else {
      for (int c0 = 0; c0 < ew; c0 += 8) {
        int cc[RT][8];
        PT vv[RT][8];
#pragma unroll
        for (int r = 0; r < RT; r++) {
          const int row = rows[r] < 0 ? 0 : rows[r];
          ell_cols<8>(M, k, (int64_t)row * ew + c0, row, dict, cc[r]);
          ell_vals8<PT>(M, k, (int64_t)row * ew + c0, vv[r]);
        }
        PT xv[RT][8];
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
          for (int u = 0; u < 8; u++) xv[r][u] = (PT)x[cc[r][u]];
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
          for (int u = 0; u < 8; u++) {
            if (wide)
              accd[r] = fma((double)vv[r][u], (double)xv[r][u], accd[r]);
            else
              accf[r] = fmaf((float)vv[r][u], (float)xv[r][u], accf[r]);
          }
      }
    }
#pragma unroll
    for (int r = 0; r < RT; r++) out[r] += (wide ? accd[r] : (double)accf[r]) * M.scale[k];
  }
}

// ---------------------------------------------------------------- tile, all buckets
//
// All buckets of a sub-range of rows in one pass: the bucket bounds of the
// sub-range are loaded together, every bucket's entries are streamed into LDS
// products with aligned 8-wide loads in the same phase, the row pointers of
// the thread's row are fetched meanwhile, and after one barrier each thread
// adds its row's products bucket by bucket (CSR order, least to most precise
// bucket).  Three dependent memory rounds per sub-range whatever the number of
// buckets.  rows_cap <= RPT * blockDim.x (RPT rows per thread: rows s0 + tid
// and s0 + tid + blockDim.x, each summed exactly as with one row per thread).
// A sub-range whose entries exceed cap is computed row by row from global
// memory instead.
template <typename XT, typename YT, typename PT, int RPT = 1>
__device__ void bspmv_tile_all(const BMat &M, const XT *__restrict__ x, YT *__restrict__ y, int r0, int r1,
                               PT *prod, int cap, int rows_cap) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = M.nb;
  for (int s0 = r0; s0 < r1; s0 += rows_cap) {
    const int s1 = min(r1, s0 + rows_cap);
    int e0[kMaxBuckets], off[kMaxBuckets + 1];
    off[0] = 0;
#pragma unroll
    for (int k = 0; k < kMaxBuckets; k++) {
      if (k < nb) {
        e0[k] = M.rp[k][s0];
        off[k + 1] = off[k] + (M.rp[k][s1] - e0[k]);
      } else {
        e0[k] = 0;
        off[k + 1] = off[k];
      }
    }
    const bool fits = off[nb] <= cap;
    int ra[RPT][kMaxBuckets], rb[RPT][kMaxBuckets];
#pragma unroll
    for (int r = 0; r < RPT; r++) {
      const int i = s0 + tid + r * nt;
#pragma unroll
      for (int k = 0; k < kMaxBuckets; k++) {
        bool ok = k < nb && i < s1;
        ra[r][k] = ok ? M.rp[k][i] : 0;
        rb[r][k] = ok ? M.rp[k][i + 1] : 0;
      }
    }
    if (fits) {
#pragma unroll
      for (int k = 0; k < kMaxBuckets; k++) {
        if (k >= nb) break;
        const int32_t *col = M.col[k];
        const int b0 = e0[k], b1 = b0 + (off[k + 1] - off[k]);
        PT *pk = prod + off[k] - b0;
        for (int base = (b0 & ~(kTileVec - 1)) + tid * kTileVec; base < b1; base += nt * kTileVec) {
          if (base >= b0 && base + kTileVec <= b1) {
            int4 ca = *reinterpret_cast<const int4 *>(col + base);
            int4 cb = *reinterpret_cast<const int4 *>(col + base + 4);
            int cc[kTileVec] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
            PT vv[kTileVec];
            load_vals8<PT>(M, k, base, vv);
            PT xv[kTileVec];
#pragma unroll
            for (int t = 0; t < kTileVec; t++) xv[t] = (PT)x[cc[t]];
#pragma unroll
            for (int t = 0; t < kTileVec; t++) pk[base + t] = vv[t] * xv[t];
          } else {
            for (int t = 0; t < kTileVec; t++) {
              int e = base + t;
              if (e >= b0 && e < b1) pk[e] = value_at<PT>(M, k, e) * (PT)x[col[e]];
            }
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPT; r++) {
      const int i = s0 + tid + r * nt;
      if (i >= s1) continue;
      double total = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxBuckets; k++) {
        if (k >= nb) break;
        const bool wide = (M.prec[k] == BSPAI_FP64) || sizeof(PT) == 8;
        const PT *pk = prod + off[k] - e0[k];
        if (fits) {
          if (wide) {
            double sum = 0.0;
            for (int q = ra[r][k]; q < rb[r][k]; q++) sum += (double)pk[q];
            total += sum * M.scale[k];
          } else {
            float sum = 0.f;
            for (int q = ra[r][k]; q < rb[r][k]; q++) sum += (float)pk[q];
            total += (double)sum * M.scale[k];
          }
        } else {
          const int32_t *col = M.col[k];
          if (wide) {
            double sum = 0.0;
            for (int q = ra[r][k]; q < rb[r][k]; q++) sum += (double)(value_at<PT>(M, k, q) * (PT)x[col[q]]);
            total += sum * M.scale[k];
          } else {
            float sum = 0.f;
            for (int q = ra[r][k]; q < rb[r][k]; q++) sum += (float)(value_at<PT>(M, k, q) * (PT)x[col[q]]);
            total += (double)sum * M.scale[k];
          }
        }
      }
      y[i] = (YT)total;
    }
    __syncthreads();
  }
}

}  // namespace bspai
