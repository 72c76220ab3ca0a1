// gmres_ir_solve with several right-hand sides (Algorithm 4 for each column).
//
// The columns share every pass over the data: one bucketed product serves all
// of them (M_b's bytes are read once per product, not once per column), and
// each kernel below streams the n x R row-major vectors once.  At the sizes
// where batching pays (n R of tens of millions) every MGS pass moves hundreds
// of megabytes, so the passes are separate kernels driven from the host; the
// per-column scalars (dots, norms, Givens state) stay on the device and are
// reduced in a fixed order.  Each column keeps its own refinement state and
// stops on its own; a column that is done contributes a zero right-hand side
// to the remaining corrections.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"
#include "spmv_dev.h"

namespace bspai {

constexpr int kBT = 256;       // threads per block
constexpr int kBGrid = 2048;   // blocks of the streaming kernels (grid-stride): 8 per CU

// Thread t handles column t % Rp of rows t / Rp + g * (kBT / Rp) ...; Rp is R
// rounded up to a power of two (<= 64), lanes c >= R idle.
struct Cols {
  int R, Rp;
};

__device__ __forceinline__ void col_mapping(const Cols &c, int &col, int64_t &row0, int64_t &stride) {
  col = threadIdx.x % c.Rp;
  int64_t groups = (int64_t)gridDim.x * (kBT / c.Rp);
  row0 = (int64_t)blockIdx.x * (kBT / c.Rp) + threadIdx.x / c.Rp;
  stride = groups;
}

// block partial per column (fixed order): part[blockIdx][col]
template <bool MAX>
__device__ __forceinline__ void block_cols(const Cols &c, double v, double *sh, double *part) {
  sh[threadIdx.x] = v;
  __syncthreads();
  if ((int)threadIdx.x < c.R) {
    double a = sh[threadIdx.x];
    for (int g = 1; g < kBT / c.Rp; g++) {
      double t = sh[g * c.Rp + threadIdx.x];
      a = MAX ? fmax(a, t) : a + t;
    }
    part[(int64_t)blockIdx.x * c.R + threadIdx.x] = a;
  }
}

// out[c] = fixed-order reduction of the nblk block partials of column c (one
// block per column: a strided sum per thread, then a tree in LDS); also stored
// at out2[c * stride2] when out2 is given
template <bool MAX>
__global__ void __launch_bounds__(kBT) k_finish(int R, int nblk, const double *part, double *out, int sqrt_out,
                                               double *out2, int64_t stride2) {
  __shared__ double sh[kBT];
  const int c = blockIdx.x, t = threadIdx.x;
  double a = 0.0;
  for (int b = t; b < nblk; b += kBT) {
    double v = part[(int64_t)b * R + c];
    a = MAX ? fmax(a, v) : a + v;
  }
  sh[t] = a;
  __syncthreads();
  for (int o = kBT / 2; o > 0; o >>= 1) {
    if (t < o) sh[t] = MAX ? fmax(sh[t], sh[t + o]) : sh[t] + sh[t + o];
    __syncthreads();
  }
  if (t == 0) {
    double r = sqrt_out ? sqrt(sh[0]) : sh[0];
    out[c] = r;
    if (out2) out2[(int64_t)c * stride2] = r;
  }
}

// residual r = b - A x (double-double or FP64) per column, max|r| and max|x|
__global__ void __launch_bounds__(kBT) k_b_residual(Cols cc, int n, const int32_t *rp, const int32_t *col,
                                                    const double *val, const double *b, const double *x, double *r,
                                                    int dd, double *part_r, double *part_x) {
  __shared__ double sh[kBT];
  int c;
  int64_t i, stride;
  col_mapping(cc, c, i, stride);
  double mr = 0.0, mx = 0.0;
  const int R = cc.R;
  for (; i < n; i += stride) {
    if (c >= R) continue;
    double s = b[i * R + c];
    if (dd) {
      double comp = 0.0;
      for (int p = rp[i]; p < rp[i + 1]; p++) {
        double a = -val[p], xv = x[(int64_t)col[p] * R + c];
        double pr = __dmul_rn(a, xv);
        double pe = fma(a, xv, -pr);
        double t = __dadd_rn(s, pr);
        double z = __dsub_rn(t, s);
        double se = __dadd_rn(__dsub_rn(s, __dsub_rn(t, z)), __dsub_rn(pr, z));
        s = t;
        comp = __dadd_rn(comp, __dadd_rn(pe, se));
      }
      s = __dadd_rn(s, comp);
    } else {
      for (int p = rp[i]; p < rp[i + 1]; p++) s = __dsub_rn(s, __dmul_rn(val[p], x[(int64_t)col[p] * R + c]));
    }
    r[i * R + c] = s;
    mr = fmax(mr, isfinite(s) ? fabs(s) : INFINITY);
    double xv = x[i * R + c];
    mx = fmax(mx, isfinite(xv) ? fabs(xv) : INFINITY);
  }
  block_cols<true>(cc, mr, sh, part_r);
  __syncthreads();
  block_cols<true>(cc, mx, sh, part_x);
}

// ||A||_inf (rows summed left to right) and max|b| per column
__global__ void __launch_bounds__(kBT) k_b_norms(Cols cc, int n, const int32_t *rp, const double *val,
                                                 const double *b, double *part_a, double *part_b) {
  __shared__ double sh[kBT];
  int c;
  int64_t i, stride;
  col_mapping(cc, c, i, stride);
  double ma = 0.0, mb = 0.0;
  for (; i < n; i += stride) {
    if (c >= cc.R) continue;
    if (c == 0) {
      double s = 0.0;
      for (int p = rp[i]; p < rp[i + 1]; p++) s += fabs(val[p]);
      ma = fmax(ma, s);
    }
    mb = fmax(mb, fabs(b[i * cc.R + c]));
  }
  block_cols<true>(cc, ma, sh, part_a);
  __syncthreads();
  block_cols<true>(cc, mb, sh, part_b);
}

// x_0 = M b column by column with the FP64 M (rows in CSR order)
__global__ void k_b_x0(int R, int n, const int32_t *rp, const int32_t *col, const double *val, const double *b,
                       double *x) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * R) return;
  int64_t i = t / R;
  int c = (int)(t % R);
  double acc = 0.0;
  for (int p = rp[i]; p < rp[i + 1]; p++) acc = __dadd_rn(acc, __dmul_rn(val[p], b[(int64_t)col[p] * R + c]));
  x[t] = acc;
}

// rv = (VT) r for active columns, 0 otherwise
template <typename VT>
__global__ void k_b_to_vt(int R, int64_t nr, const double *r, const int *active, VT *rv) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nr) rv[t] = active[t % R] ? (VT)r[t] : (VT)0;
}

// sum of squares per column of a VT block
template <typename VT>
__global__ void __launch_bounds__(kBT) k_b_sumsq(Cols cc, int n, const VT *v, double *part) {
  __shared__ double sh[kBT];
  int c;
  int64_t i, stride;
  col_mapping(cc, c, i, stride);
  double s = 0.0;
  for (; i < n; i += stride)
    if (c < cc.R) {
      double t = (double)v[i * cc.R + c];
      s = fma(t, t, s);
    }
  block_cols<false>(cc, s, sh, part);
}

// v = z / h per column (0 where h = 0); in place allowed
template <typename VT>
__global__ void k_b_scale(int R, int64_t nr, const VT *z, const double *h, VT *v) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr) return;
  double hh = h[t % R];
  v[t] = hh > 0.0 ? (VT)((double)z[t] / hh) : (VT)0;
}

// MGS pass: z -= hprev * vprev (when vprev), then partial dots with vcur
template <typename VT>
__global__ void __launch_bounds__(kBT) k_b_mgs(Cols cc, int n, VT *z, const VT *vprev, const double *hprev,
                                               const VT *vcur, double *part) {
  __shared__ double sh[kBT];
  int c;
  int64_t i, stride;
  col_mapping(cc, c, i, stride);
  const int R = cc.R;
  double hp = (vprev && c < R) ? hprev[c] : 0.0;
  double s = 0.0;
  for (; i < n; i += stride) {
    if (c >= R) continue;
    int64_t e = i * R + c;
    double zz = (double)z[e];
    if (vprev) {
      zz = (double)(VT)fma(-hp, (double)vprev[e], zz);
      z[e] = (VT)zz;
    }
    if (vcur) s = fma((double)vcur[e], zz, s);
    else s = fma(zz, zz, s);
  }
  block_cols<false>(cc, s, sh, part);
}

// 4 consecutive columns per thread (R a multiple of 4): 16-byte loads and
// stores of z and the basis (two per 4 doubles).  Threads t < rpp * tpr work:
// tpr = R / 4 threads per row, rpp rows per block and pass.
template <typename VT>
struct Vec4;
template <>
struct Vec4<float> {
  __device__ static void load(const float *p, double (&v)[4]) {
    float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
  }
  __device__ static void store(float *p, const float (&v)[4]) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};
template <>
struct Vec4<double> {
  __device__ static void load(const double *p, double (&v)[4]) {
    double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
  }
  __device__ static void store(double *p, const double (&v)[4]) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
  }
};

// the per-column partials (sums, or maxima with MAX) of a block of 4-column
// threads, fixed order
template <bool MAX = false>
__device__ __forceinline__ void block_cols4(int R, int tpr, int rpp, const double (&acc)[4], double *sh, double *part) {
  const int t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; u++) sh[4 * t + u] = acc[u];
  __syncthreads();
  if (t < R) {
    const int cg = t / 4, u = t % 4;
    double a = sh[4 * cg + u];
    for (int g = 1; g < rpp; g++) {
      const double v = sh[4 * (g * tpr + cg) + u];
      a = MAX ? fmax(a, v) : a + v;
    }
    part[(int64_t)blockIdx.x * R + t] = a;
  }
}

template <typename VT>
__global__ void __launch_bounds__(kBT) k_b_mgs4(int R, int n, VT *z, const VT *vprev, const double *hprev,
                                                const VT *vcur, double *part) {
  __shared__ double sh[4 * kBT];
  const int tpr = R / 4, rpp = kBT / tpr;
  const int g = threadIdx.x / tpr, c0 = 4 * (threadIdx.x % tpr);
  double hp[4] = {0.0, 0.0, 0.0, 0.0}, acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (vprev && g < rpp)
#pragma unroll
    for (int u = 0; u < 4; u++) hp[u] = hprev[c0 + u];
  if (g < rpp) {
    for (int64_t i = (int64_t)blockIdx.x * rpp + g; i < n; i += (int64_t)gridDim.x * rpp) {
      const int64_t e = i * R + c0;
      double zz[4];
      Vec4<VT>::load(z + e, zz);
      if (vprev) {
        double vp[4];
        Vec4<VT>::load(vprev + e, vp);
        VT zo[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          zo[u] = (VT)fma(-hp[u], vp[u], zz[u]);
          zz[u] = (double)zo[u];
        }
        Vec4<VT>::store(z + e, zo);
      }
      if (vcur) {
        double vc[4];
        Vec4<VT>::load(vcur + e, vc);
#pragma unroll
        for (int u = 0; u < 4; u++) acc[u] = fma(vc[u], zz[u], acc[u]);
      } else {
#pragma unroll
        for (int u = 0; u < 4; u++) acc[u] = fma(zz[u], zz[u], acc[u]);
      }
    }
  }
  block_cols4(R, tpr, rpp, acc, sh, part);
}

// v = z / h per column, 4 columns per thread
template <typename VT>
__global__ void k_b_scale4(int R, int64_t nr, const VT *z, const double *h, VT *v) {
  int64_t e = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= nr) return;
  const int c0 = (int)(e % R);
  double zz[4];
  Vec4<VT>::load(z + e, zz);
  VT o[4];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const double hh = h[c0 + u];
    o[u] = hh > 0.0 ? (VT)(zz[u] / hh) : (VT)0;
  }
  Vec4<VT>::store(v + e, o);
}

// Givens step j, one block of 64 threads per column (grid R; dynamic LDS
// (3 m + 1) doubles).  H column j holds h_{0..j+1, j} on entry; rotated in
// place.  Writes res[c] = |g_{j+1}|.  The column and the earlier rotations
// are staged in LDS by the whole block; lane 0 then applies rotations
// 0..j-1 carrying the rotated entry in a register (the chain of dependent
// products never goes through global memory) and forms rotation j.
// hn non-null: the column's GMRES stops here (gm_active[c] = 0) when
// |g_{j+1}| <= tau beta[c], h_{j+1,j} = hn[c] = 0 or j + 1 = m, the test the
// host repeats on the same values, so that steps queued ahead see it.
// The host's copy of the step (pinned host memory hq, read once a later
// event has completed): hq[c] = hrow[c] (h_{j+1,j}), hq[R + c] = |g_{j+1}|
// and, from block 0, the MGS abort word *abortf at hq + 3 R (an unsigned).
__global__ void __launch_bounds__(64) k_b_givens(int R, int m, int j, double *H, double *cs, double *sn, double *g,
                                                 int *gm_active, double *res, const double *hn, const double *beta,
                                                 double tau, const double *hrow, const unsigned *abortf,
                                                 double *hq) {
  extern __shared__ double gsh[];
  const int c = blockIdx.x;
  if (c >= R) return;
  double *h = H + ((int64_t)c * m + j) * (m + 1);
  double *cc = cs + (int64_t)c * m, *ss = sn + (int64_t)c * m, *gg = g + (int64_t)c * (m + 1);
  auto to_host = [&](double r) {
    hq[c] = hrow[c];
    hq[R + c] = r;
    if (c == 0) *reinterpret_cast<unsigned *>(hq + 3 * R) = *abortf;
    __threadfence_system();
  };
  if (!gm_active[c]) {
    if (threadIdx.x == 0) {
      res[c] = 0.0;
      to_host(0.0);
    }
    return;
  }
  double *lh = gsh, *lc = gsh + (m + 1), *ls = lc + m;
  for (int i = threadIdx.x; i <= j + 1; i += 64) lh[i] = h[i];
  for (int i = threadIdx.x; i < j; i += 64) {
    lc[i] = cc[i];
    ls[i] = ss[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = lh[0];
#pragma unroll 4
    for (int i = 0; i < j; i++) {
      const double b = lh[i + 1], ci = lc[i], si = ls[i];
      lh[i] = ci * a + si * b;
      a = -si * a + ci * b;
    }
    const double b = lh[j + 1];
    const double rho = hypot(a, b);
    const double cj = rho == 0.0 ? 1.0 : a / rho;
    const double sj = rho == 0.0 ? 0.0 : b / rho;
    cc[j] = cj;
    ss[j] = sj;
    lh[j] = rho;
    lh[j + 1] = 0.0;
    const double gj = gg[j];
    gg[j + 1] = -sj * gj;
    gg[j] = cj * gj;
    const double hres = fabs(-sj * gj);
    res[c] = hres;
    if (hn && (hres <= tau * beta[c] || hn[c] == 0.0 || j + 1 == m)) gm_active[c] = 0;
    to_host(hres);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += 64) h[i] = lh[i];
}

// y = R^{-1} g for every column (k[c] iterations): one 64-thread block per
// column (grid R, dynamic LDS 3 m doubles, m <= kBacksubMaxM).  For row i the
// lanes form the rounded products h_{i,j} y_j (j > i) in parallel and lane 0
// subtracts them from g_i in increasing j, the order of the row recurrence;
// the entries of row i - 1 are loaded while lane 0 works on row i.
constexpr int kBacksubMaxM = 192;
// Arnoldi steps of the column-group path queued ahead of the host's
// stopping decisions, and the steps per completion event the host waits on
// (each event recorded on the stream delays the next dispatch by a few
// microseconds; twice as many steps queued as one event covers keep the
// stream busy while the host reads them)
constexpr int kStepLag = 8;
constexpr int kStepsPerEvent = 4;
__global__ void __launch_bounds__(64) k_b_backsub(int R, int m, const double *H, const double *g, const int *kc,
                                                  double *y) {
  constexpr int Q = kBacksubMaxM / 64;
  extern __shared__ double bsh[];
  const int c = blockIdx.x;
  if (c >= R) return;
  const int k = kc[c], lane = threadIdx.x;
  if (k <= 0) return;
  const double *Hc = H + (int64_t)c * m * (m + 1);
  double *ly = bsh, *lp = bsh + m, *lh = bsh + 2 * m;  // y, products, row i (entries j >= i)
  double r[Q];
  auto load_row = [&](int i) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
      const int j = i + lane + 64 * q;
      r[q] = j < k ? Hc[(int64_t)j * (m + 1) + i] : 0.0;
    }
  };
  auto store_row = [&](int i) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
      const int j = i + lane + 64 * q;
      if (j < k) lh[j] = r[q];
    }
  };
  load_row(k - 1);
  store_row(k - 1);
  __syncthreads();
  for (int i = k - 1; i >= 0; i--) {
    for (int j = i + 1 + lane; j < k; j += 64) lp[j] = lh[j] * ly[j];
    const double diag = lh[i];
    __syncthreads();
    if (i > 0) load_row(i - 1);
    if (lane == 0) {
      double t = g[(int64_t)c * (m + 1) + i];
      for (int j = i + 1; j < k; j++) t -= lp[j];
      ly[i] = t / diag;
    }
    if (i > 0) store_row(i - 1);
    __syncthreads();
  }
  for (int i = lane; i < k; i += 64) y[(int64_t)c * m + i] = ly[i];
}

// d = V y per column (FP64); add mode: x += d, else out = d; max|d|, max|x|
template <typename VT>
__global__ void __launch_bounds__(kBT) k_b_update(Cols cc, int n, int m, const VT *V, int64_t vstride, const double *y,
                                                  const int *kc, double *x, double *dout, double *part_d,
                                                  double *part_x) {
  __shared__ double sh[kBT];
  int c;
  int64_t i, stride;
  col_mapping(cc, c, i, stride);
  const int R = cc.R;
  const int k = c < R ? kc[c] : 0;
  const double *yy = y + (int64_t)(c < R ? c : 0) * m;
  double md = 0.0, mx = 0.0;
  for (; i < n; i += stride) {
    if (c >= R) continue;
    int64_t e = i * R + c;
    double d = 0.0;
    for (int t = 0; t < k; t++) d = fma((double)V[(int64_t)t * vstride + e], yy[t], d);
    if (dout) {
      dout[e] = d;
    } else {
      double xn = x[e] + d;
      x[e] = xn;
      md = fmax(md, fabs(d));
      mx = fmax(mx, fabs(xn));
    }
  }
  block_cols<true>(cc, md, sh, part_d);
  __syncthreads();
  block_cols<true>(cc, mx, sh, part_x);
}

// k_b_update with four adjacent columns per thread (R % 4 == 0): one 16-byte
// load of V per basis vector instead of four.  Each column's sum runs over t
// in the order of k_b_update and the maxima are exact, so the results are
// the same bits.
template <typename VT>
__global__ void __launch_bounds__(kBT) k_b_update4(int R, int n, int m, const VT *V, int64_t vstride,
                                                   const double *y, const int *kc, double *x, double *dout,
                                                   double *part_d, double *part_x) {
  __shared__ double sh[4 * kBT];
  const int tpr = R / 4, rpp = kBT / tpr;
  const int g = threadIdx.x / tpr, c0 = 4 * (threadIdx.x % tpr);
  double md[4] = {0.0, 0.0, 0.0, 0.0}, mx[4] = {0.0, 0.0, 0.0, 0.0};
  if (g < rpp) {
    int k[4], kmax = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      k[u] = kc[c0 + u];
      kmax = max(kmax, k[u]);
    }
    const double *yy = y + (int64_t)c0 * m;  // column c0 + u at yy + u m
    for (int64_t i = (int64_t)blockIdx.x * rpp + g; i < n; i += (int64_t)gridDim.x * rpp) {
      const int64_t e = i * R + c0;
      double d[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < kmax; t++) {
        double v[4];
        Vec4<VT>::load(V + (int64_t)t * vstride + e, v);
#pragma unroll
        for (int u = 0; u < 4; u++)
          if (t < k[u]) d[u] = fma(v[u], yy[(int64_t)u * m + t], d[u]);
      }
      if (dout) {
        Vec4<double>::store(dout + e, d);
      } else {
        double xv[4];
        Vec4<double>::load(x + e, xv);
#pragma unroll
        for (int u = 0; u < 4; u++) {
          xv[u] = xv[u] + d[u];
          md[u] = fmax(md[u], fabs(d[u]));
          mx[u] = fmax(mx[u], fabs(xv[u]));
        }
        Vec4<double>::store(x + e, xv);
      }
    }
  }
  block_cols4<true>(R, tpr, rpp, md, sh, part_d);
  __syncthreads();
  block_cols4<true>(R, tpr, rpp, mx, sh, part_x);
}

// x += d (d FP64, computed by the transposed apply) with max|d|, max|x|
__global__ void __launch_bounds__(kBT) k_b_add(Cols cc, int n, const double *d, double *x, double *part_d,
                                               double *part_x) {
  __shared__ double sh[kBT];
  int c;
  int64_t i, stride;
  col_mapping(cc, c, i, stride);
  double md = 0.0, mx = 0.0;
  for (; i < n; i += stride) {
    if (c >= cc.R) continue;
    int64_t e = i * cc.R + c;
    double xn = x[e] + d[e];
    x[e] = xn;
    md = fmax(md, fabs(d[e]));
    mx = fmax(mx, fabs(xn));
  }
  block_cols<true>(cc, md, sh, part_d);
  __syncthreads();
  block_cols<true>(cc, mx, sh, part_x);
}

template <typename VT>
__global__ void k_to_vt_vals(int64_t nnz, const double *a, VT *o) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) o[e] = (VT)a[e];
}

// ------------------------------------------------------------------ host

struct DevBuf {
  void *p = nullptr;
  bool own = true;  // false: carved from the grow-only block below
  ~DevBuf() {
    if (own) dfree(p);
  }
};

// The column-group solve's per-call buffers come from one grow-only device
// block that the library keeps between calls (bspai_release_workspace frees
// it).  A call holds the block's lock from start to end, so such solves from
// several threads run one after another (their MGS kernels each need every
// compute unit); the holder's stream is idle whenever the lock is free.
static struct {
  std::mutex mu;
  void *ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
} g_bws;

int release_batched_workspace() {
  std::lock_guard<std::mutex> lock(g_bws.mu);
  if (!g_bws.ptr) return BSPAI_OK;
  int cur = 0;
  BSPAI_HIP(hipGetDevice(&cur));
  const int dev = g_bws.device;
  if (cur != dev) BSPAI_HIP(hipSetDevice(dev));
  const hipError_t e = hipDeviceSynchronize();
  dfree(g_bws.ptr);
  g_bws.ptr = nullptr;
  g_bws.bytes = 0;
  g_bws.device = -1;
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess) return fail(BSPAI_EHIP, "bspai_release_workspace: %s", hipGetErrorString(e));
  return BSPAI_OK;
}

template <typename VT>
int solve_batched(const bspai_csr *A, const bspai_handle *Ab, const double *b, const bspai_handle *M,
                  const gmres_ir_tol *tol, double *x, int R, int m, gmres_ir_stats *st_host, hipStream_t s,
                  bool mgs1) {
  if (m > kBacksubMaxM) return fail(BSPAI_EINVAL, "gmres_ir_solve: gmres_max %d above %d", m, kBacksubMaxM);
  if (mgs1 && (R * (int)sizeof(VT) != 16 || !mgs_persist_rpt(A->n)))
    return fail(BSPAI_EINVAL, "gmres_ir_solve: the one-launch MGS needs %d columns and at most %d rows",
                16 / (int)sizeof(VT), 256 * 512 * 16);
  const int n = A->n;
  const int64_t nnz = A->nnz, nr = (int64_t)n * R;
  const bool tr = tol->trans != 0;
  const double stag_ratio = tol->stag_ratio == 0.0 ? 0.5 : tol->stag_ratio;
  Cols cc{R, 1};
  while (cc.Rp < R) cc.Rp <<= 1;
  const int nblk = (int)std::min<int64_t>(kBGrid, (n + (kBT / cc.Rp) - 1) / (kBT / cc.Rp));
  const unsigned eg = (unsigned)((nr + 255) / 256);
  // 4-column kernels for the per-iteration passes when R is a multiple of 4
  // (rows of R values then start 16-byte aligned); they use the same
  // fixed-order per-column reduction
  const bool vec4 = R % 4 == 0;
  const int rpp4 = vec4 ? kBT / (R / 4) : 1;
  const int nblk4 = (int)std::min<int64_t>(kBGrid, (n + rpp4 - 1) / rpp4);

  // operators: A (or A^T) in FP64 and, inside GMRES, in u_g or bucketed (A_b
  // or A_b^T), M_b (or M_b^T), FP64 M for x_0
  // the grow-only block's lock while this call uses the block; the stream
  // drains before it is released (drain is destroyed first)
  std::unique_lock<std::mutex> bws_lock;
  struct Drain {
    hipStream_t s;
    const std::unique_lock<std::mutex> *l;
    ~Drain() {
      if (l->owns_lock()) (void)hipStreamSynchronize(s);
    }
  } drain{s, &bws_lock};
  DevBuf trp, tcol, tval, apv, rbuf, rv, wv, zv, Vb, dtmp, parts, scal, Hb, csb, snb, gb, yb, kcb, actb, mgsws;
  int rc;
  {
    const std::pair<DevBuf *, size_t> want[] = {
        {&mgsws, mgs1 ? mgs_persist_ws_bytes() : 0},
        {&trp, tr ? 4 * ((size_t)n + 1) : 0},
        {&tcol, tr ? 4 * (size_t)(nnz + 1) : 0},
        {&tval, tr ? 8 * (size_t)(nnz + 1) : 0},
        {&apv, !Ab ? sizeof(VT) * (size_t)(nnz + 1) : 0},
        {&rbuf, 8 * (size_t)nr},
        {&rv, sizeof(VT) * (size_t)nr},
        {&wv, sizeof(VT) * (size_t)nr},
        {&zv, sizeof(VT) * (size_t)nr},
        {&Vb, sizeof(VT) * (size_t)nr * (m + 1)},
        {&dtmp, 8 * (size_t)nr},
        {&parts, 2 * 8 * (size_t)kBGrid * R},
        {&scal, 8 * (8 * (size_t)R + 1)},
        {&Hb, 8 * (size_t)R * m * (m + 1)},
        {&csb, 8 * (size_t)R * m},
        {&snb, 8 * (size_t)R * m},
        {&gb, 8 * (size_t)R * (m + 1)},
        {&yb, 8 * (size_t)R * m},
        {&kcb, 4 * (size_t)R},
        {&actb, 4 * (size_t)R}};
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t total = 0;
    for (const auto &w : want) total += a256(w.second);
    bws_lock = std::unique_lock<std::mutex>(g_bws.mu);
    int dev = 0;
    BSPAI_HIP(hipGetDevice(&dev));
    if (g_bws.bytes < total || g_bws.device != dev) {
      if (g_bws.ptr) {
        (void)hipDeviceSynchronize();
        dfree(g_bws.ptr);
        g_bws.ptr = nullptr;
        g_bws.bytes = 0;
      }
      if ((rc = dalloc(&g_bws.ptr, total))) return rc;
      g_bws.bytes = total;
      g_bws.device = dev;
    }
    char *base = static_cast<char *>(g_bws.ptr);
    for (const auto &w : want) {
      if (!w.second) continue;
      w.first->p = base;
      w.first->own = false;
      base += a256(w.second);
    }
  }
  if (mgs1) BSPAI_HIP(hipMemsetAsync(mgsws.p, 0, mgs_persist_ws_bytes(), s));
  unsigned mgs_rounds = 0;  // exchange rounds of the MGS launches so far
  // per queued step: pinned host memory that the step's rotation kernel
  // fills with h_{j+1,j} and |g_{j+1}| of every column and the MGS abort
  // word, a completion event (recorded after every kStepsPerEvent-th step),
  // and (when profiling) HIP events around its MGS launch
  const bool prof = mgs1 && profiling_on();
  struct StepRing {
    void *pin = nullptr, *dpin = nullptr;  // host and device addresses
    int R = 0;
    hipStream_t st = nullptr;
    hipEvent_t done[kStepLag] = {};
    hipEvent_t prof[2 * kStepLag] = {};
    bool timed[kStepLag] = {};  // the slot's MGS launch has events around it
    double *hq(int k) { return static_cast<double *>(pin) + (size_t)k * (3 * R + 1); }
    unsigned *abort(int k) { return reinterpret_cast<unsigned *>(hq(k) + 3 * R); }
    double *dhq(int k) { return static_cast<double *>(dpin) + (size_t)k * (3 * R + 1); }
    ~StepRing() {
      if (pin) (void)hipStreamSynchronize(st);  // kernels writing into pin may still be queued on an error return
      for (auto q : done)
        if (q) (void)hipEventDestroy(q);
      for (auto q : prof)
        if (q) (void)hipEventDestroy(q);
      if (pin) (void)hipHostFree(pin);
    }
  } ring;
  ring.R = R;
  ring.st = s;
  BSPAI_HIP(hipHostMalloc(&ring.pin, sizeof(double) * (size_t)kStepLag * (3 * R + 1),
                          hipHostMallocMapped | hipHostMallocCoherent));
  BSPAI_HIP(hipHostGetDevicePointer(&ring.dpin, ring.pin, 0));
  for (int k = 0; k < kStepLag; k++) {
    BSPAI_HIP(hipEventCreateWithFlags(&ring.done[k], hipEventDisableTiming));
    if (prof) {
      BSPAI_HIP(hipEventCreate(&ring.prof[2 * k]));
      BSPAI_HIP(hipEventCreate(&ring.prof[2 * k + 1]));
    }
  }
  const int32_t *arp = A->row_ptr, *acol = A->col;
  const double *aval = A->val;
  if (tr) {
    if ((rc = csr_transpose(n, nnz, arp, acol, aval, 8, (int32_t *)trp.p, (int32_t *)tcol.p, tval.p, s))) return rc;
    arp = (const int32_t *)trp.p, acol = (const int32_t *)tcol.p, aval = (const double *)tval.p;
  }
  VT *Ap = (VT *)apv.p, *RV = (VT *)rv.p, *W = (VT *)wv.p, *Z = (VT *)zv.p, *V = (VT *)Vb.p;
  double *r64 = (double *)rbuf.p, *D = (double *)dtmp.p, *P1 = (double *)parts.p, *P2 = P1 + (int64_t)kBGrid * R;
  double *S = (double *)scal.p;  // 8 rows of R scalars, then the MGS abort word
  unsigned *mgs_abortf = reinterpret_cast<unsigned *>(S + 8 * R);
  BSPAI_HIP(hipMemsetAsync(mgs_abortf, 0, sizeof(double), s));
  double *H = (double *)Hb.p, *CS = (double *)csb.p, *SN = (double *)snb.p, *G = (double *)gb.p, *Y = (double *)yb.p;
  int *KC = (int *)kcb.p, *ACT = (int *)actb.p;
  if (nnz > 0 && !Ab) {
    hipLaunchKernelGGL(k_to_vt_vals<VT>, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, aval, Ap);
    BSPAI_CHECK_LAUNCH();
  }
  BMat Apm;
  memset(&Apm, 0, sizeof(Apm));
  Apm.n = n;
  Apm.nb = 1;
  Apm.nnz = nnz;
  Apm.prec[0] = sizeof(VT) == 8 ? BSPAI_FP64 : BSPAI_FP32;
  Apm.scale[0] = 1.0;
  Apm.rp[0] = arp;
  Apm.col[0] = acol;
  Apm.val[0] = Ap;
  // A's ELL copy (byte or int16 column codes where they fit) for the
  // many-column products: 5 instead of 8 bytes per FP32 entry
  DevBuf aecol, aeval, aecode, aedict;
  if (!Ab && nnz > 0 && R % 4 == 0) {
    int32_t w = 0, cw = 0, *ecol = nullptr, *edict = nullptr;
    void *eval = nullptr, *ecode = nullptr;
    rc = csr_to_ell(n, arp, acol, Ap, (int)sizeof(VT), &ecol, &eval, &w, s);
    aecol.p = ecol, aeval.p = eval;
    if (rc) return rc;
    if (w) {
      rc = ell_codes(n, w, ecol, &ecode, &edict, &cw, s);
      aecode.p = ecode, aedict.p = edict;
      if (rc) return rc;
      Apm.ell_w[0] = w;
      Apm.ell_cw[0] = cw;
      Apm.ell_col[0] = cw ? nullptr : ecol;
      Apm.ell_val[0] = eval;
      Apm.ell_code[0] = ecode;
      Apm.ell_dict[0] = edict;
    }
  }
  if (Ab) Apm = tr ? Ab->matT : Ab->mat;
  const BMat &Mb = tr ? M->matT : M->mat;
  const int fp64 = sizeof(VT) == 8;

  auto finish = [&](bool mx, const double *part, double *out, int sq, double *out2 = nullptr,
                    int64_t stride2 = 0, int nparts = 0) -> int {
    const int np = nparts > 0 ? nparts : nblk;  // blocks that wrote partials
    if (mx)
      hipLaunchKernelGGL(k_finish<true>, dim3(R), dim3(kBT), 0, s, R, np, part, out, sq, out2, stride2);
    else
      hipLaunchKernelGGL(k_finish<false>, dim3(R), dim3(kBT), 0, s, R, np, part, out, sq, out2, stride2);
    BSPAI_CHECK_LAUNCH();
    return BSPAI_OK;
  };
  auto to_host = [&](const double *d, std::vector<double> &h, int rows = 1) -> int {
    h.resize((size_t)R * rows);
    BSPAI_HIP(hipMemcpyAsync(h.data(), d, 8 * (size_t)R * rows, hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    return BSPAI_OK;
  };

  // norms of A and b, x_0
  hipLaunchKernelGGL(k_b_norms, dim3(nblk), dim3(kBT), 0, s, cc, n, arp, aval, b, P1, P2);
  BSPAI_CHECK_LAUNCH();
  if ((rc = finish(true, P1, S + 0 * R, 0)) || (rc = finish(true, P2, S + 1 * R, 0))) return rc;
  std::vector<double> hnA, hnb;
  if ((rc = to_host(S + 0 * R, hnA)) || (rc = to_host(S + 1 * R, hnb))) return rc;
  const double normA = hnA[0];
  if (tol->x0_mode == 0) {
    const int32_t *frp = tr ? M->mT_rp : M->m_rp, *fcol = tr ? M->mT_col : M->m_col;
    const double *fval = tr ? M->mT_val : M->m_val;
    hipLaunchKernelGGL(k_b_x0, dim3(eg), dim3(256), 0, s, R, n, frp, fcol, fval, b, x);
    BSPAI_CHECK_LAUNCH();
  } else if (tol->x0_mode == 1) {
    if ((rc = launch_bspmv(Mb, b, x, R, R, 1, s))) return rc;
  } else if (tol->x0_mode == 2) {
    BSPAI_HIP(hipMemsetAsync(x, 0, 8 * (size_t)nr, s));
  }

  std::vector<gmres_ir_stats> st(R);
  for (auto &q : st) memset(&q, 0, sizeof(q));
  std::vector<int> active(R, 1), stag(R, 0), status(R, BSPAI_OK);
  std::vector<double> dx_prev(R, 0.0), hr, hbeta;
  int it = 0;
  for (;;) {
    // residuals and stopping tests per column
    hipLaunchKernelGGL(k_b_residual, dim3(nblk), dim3(kBT), 0, s, cc, n, arp, acol, aval, b, x, r64, tol->ur_dd, P1,
                       P2);
    BSPAI_CHECK_LAUNCH();
    if ((rc = finish(true, P1, S + 2 * R, 0)) || (rc = finish(true, P2, S + 3 * R, 0))) return rc;
    if ((rc = to_host(S + 2 * R, hr, 2))) return rc;  // rows 2 and 3: max|r|, max|x| per column
    int nact = 0;
    for (int c = 0; c < R; c++) {
      if (!active[c]) continue;
      double nr_ = hr[c], nx = hr[R + c], nb_ = hnb[c];
      double eta = nr_ / (normA * nx + nb_);
      double rho = nb_ > 0 ? nr_ / nb_ : nr_;
      if (it <= 64) {
        st[c].eta[it] = eta;
        st[c].relres[it] = rho;
      }
      int reason = 0;
      if (!std::isfinite(nr_) || !std::isfinite(nx)) {
        reason = 5;
        status[c] = BSPAI_ENAN;
      } else if (rho <= tol->tol_rr) reason = 1;
      else if (eta <= tol->tol_be) reason = 2;
      else if (stag[c]) {
        reason = 3;
        status[c] = BSPAI_ESTAG;
      } else if (it >= tol->i_max || it >= 64) {
        reason = 4;
        status[c] = BSPAI_ENOCONV;
      }
      if (reason) {
        active[c] = 0;
        st[c].stop_reason = reason;
        st[c].steps = it;
      } else {
        nact++;
      }
    }
    if (nact == 0) break;
    BSPAI_HIP(hipMemcpyAsync(ACT, active.data(), 4 * (size_t)R, hipMemcpyHostToDevice, s));
    // right-hand side of the Krylov solve
    hipLaunchKernelGGL(k_b_to_vt<VT>, dim3(eg), dim3(256), 0, s, R, nr, r64, ACT, RV);
    BSPAI_CHECK_LAUNCH();
    if (!tr) {
      if ((rc = launch_bspmv(Mb, RV, V, R, R, fp64, s))) return rc;
    } else {
      BSPAI_HIP(hipMemcpyAsync(V, RV, sizeof(VT) * (size_t)nr, hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_b_sumsq<VT>, dim3(nblk), dim3(kBT), 0, s, cc, n, V, P1);
    BSPAI_CHECK_LAUNCH();
    if ((rc = finish(false, P1, S + 4 * R, 1))) return rc;  // beta
    if ((rc = to_host(S + 4 * R, hbeta))) return rc;
    hipLaunchKernelGGL(k_b_scale<VT>, dim3(eg), dim3(256), 0, s, R, nr, V, S + 4 * R, V);
    BSPAI_CHECK_LAUNCH();
    std::vector<int> gm_active(R), kc(R, 0);
    std::vector<double> g0(R * (size_t)(m + 1), 0.0);
    for (int c = 0; c < R; c++) {
      gm_active[c] = active[c] && hbeta[c] > 0.0;
      g0[(size_t)c * (m + 1)] = hbeta[c];
    }
    BSPAI_HIP(hipMemcpyAsync(G, g0.data(), 8 * g0.size(), hipMemcpyHostToDevice, s));
    int *GMA = ACT;  // reuse: active GMRES columns
    BSPAI_HIP(hipMemcpyAsync(GMA, gm_active.data(), 4 * (size_t)R, hipMemcpyHostToDevice, s));
    int nrun = 0;
    for (int c = 0; c < R; c++) nrun += gm_active[c];
    // Steps are queued up to `lag` ahead of the host.  On the column-group
    // path the Givens kernel applies each column's stopping test on the
    // device (a step queued after every column stopped finds no active
    // column: its MGS launch returns at once and its rotations are skipped),
    // and the host repeats the test on the same values when the step's event
    // completes.  The per-pass path decides on the host after every step.
    const int lag = mgs1 ? kStepLag : 1, every = mgs1 ? kStepsPerEvent : 1;
    int jq = 0;  // steps queued
    for (int jd = 0; jd < m && nrun > 0; jd++) {
      for (; jq < m && jq < jd + lag; jq++) {
        const int j = jq, slot = j % lag;
        VT *vj = V + (int64_t)j * nr;
        if (!tr) {
          if ((rc = launch_bspmv(Apm, vj, W, R, R, fp64, s)) || (rc = launch_bspmv(Mb, W, Z, R, R, fp64, s)))
            return rc;
        } else {
          if ((rc = launch_bspmv(Mb, vj, W, R, R, fp64, s)) || (rc = launch_bspmv(Apm, W, Z, R, R, fp64, s)))
            return rc;
        }
        if (mgs1) {
          // the whole step's MGS in one cooperative launch (h_{i,j} to H, the
          // norms to S row 5, v_{j+1} written)
          ring.timed[slot] = prof && mgs_profile_sample();
          if (ring.timed[slot]) BSPAI_HIP(hipEventRecord(ring.prof[2 * slot], s));
          if ((rc = launch_mgs_persist<VT>(n, j, m, Z, V, nr, H, S + 5 * R, GMA, mgsws.p, mgs_rounds, mgs_abortf,
                                           s)))
            return rc;
          mgs_rounds += (unsigned)(j + 2);
          if (ring.timed[slot]) BSPAI_HIP(hipEventRecord(ring.prof[2 * slot + 1], s));
        }
        // MGS: pass i removes v_{i-1}, measures v_i; h_{i,j} lands in H column j
        for (int i = 0; !mgs1 && i <= j + 1; i++) {
          const VT *vprev = i > 0 ? V + (int64_t)(i - 1) * nr : nullptr;
          const VT *vcur = i <= j ? V + (int64_t)i * nr : nullptr;
          const double *hprev = S + 5 * R;
          if (vec4)
            hipLaunchKernelGGL(k_b_mgs4<VT>, dim3(nblk4), dim3(kBT), 0, s, R, n, Z, vprev, hprev, vcur, P1);
          else
            hipLaunchKernelGGL(k_b_mgs<VT>, dim3(nblk), dim3(kBT), 0, s, cc, n, Z, vprev, hprev, vcur, P1);
          BSPAI_CHECK_LAUNCH();
          // the finished scalar goes to S row 5 (next pass) and into H column j
          if ((rc = finish(false, P1, S + 5 * R, i > j, H + (int64_t)j * (m + 1) + i, (int64_t)m * (m + 1),
                           vec4 ? nblk4 : nblk)))
            return rc;
        }
        // v_{j+1} = z / h_{j+1,j} (written by the one-launch MGS itself)
        if (mgs1) {
        } else if (vec4)
          hipLaunchKernelGGL(k_b_scale4<VT>, dim3((unsigned)((nr / 4 + 255) / 256)), dim3(256), 0, s, R, nr, Z,
                             S + 5 * R, V + (int64_t)(j + 1) * nr);
        else
          hipLaunchKernelGGL(k_b_scale<VT>, dim3(eg), dim3(256), 0, s, R, nr, Z, S + 5 * R,
                             V + (int64_t)(j + 1) * nr);
        BSPAI_CHECK_LAUNCH();
        // the rotations; h_{j+1,j}, |g_{j+1}| and the MGS abort word go
        // straight to the step's pinned slot
        hipLaunchKernelGGL(k_b_givens, dim3(R), dim3(64), (size_t)(3 * m + 1) * sizeof(double), s, R, m, j, H, CS,
                           SN, G, GMA, S + 6 * R, mgs1 ? S + 5 * R : nullptr, S + 4 * R, tol->tau, S + 5 * R,
                           mgs_abortf, ring.dhq(slot));
        BSPAI_CHECK_LAUNCH();
        if (j % every == every - 1 || j == m - 1) BSPAI_HIP(hipEventRecord(ring.done[slot], s));
      }
      const int slot = jd % lag;
      // the first event recorded at or after step jd (queued: it is less
      // than jd + lag)
      const int je = std::min(m - 1, jd - jd % every + every - 1);
      BSPAI_HIP(hipEventSynchronize(ring.done[je % lag]));
      if (mgs1 && *ring.abort(slot))
        return fail(BSPAI_EHIP, "gmres_ir_solve: a grid exchange of the MGS kernel timed out");
      if (prof && ring.timed[slot]) {
        float ms = 0.f;
        BSPAI_HIP(hipEventElapsedTime(&ms, ring.prof[2 * slot], ring.prof[2 * slot + 1]));
        // algorithmic bytes of MGS step j: v_0..v_j read and v_{j+1} written,
        // (j + 2) vectors of u_g per column (z, read once more by the kernel,
        // is not counted)
        add_mgs_profile(ms, (double)(jd + 2) * (double)nr * sizeof(VT));
      }
      const double *hn = ring.hq(slot), *hres = hn + R;
      bool changed = false;
      for (int c = 0; c < R; c++) {
        if (!gm_active[c]) continue;
        kc[c] = jd + 1;
        if (hres[c] <= tol->tau * hbeta[c] || hn[c] == 0.0 || jd + 1 == m) {
          gm_active[c] = 0;
          nrun--;
          changed = true;
        }
      }
      if (changed && !mgs1) BSPAI_HIP(hipMemcpyAsync(GMA, gm_active.data(), 4 * (size_t)R, hipMemcpyHostToDevice, s));
    }
    BSPAI_HIP(hipMemcpyAsync(KC, kc.data(), 4 * (size_t)R, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_b_backsub, dim3(R), dim3(64), (size_t)3 * m * sizeof(double), s, R, m, H, G, KC, Y);
    BSPAI_CHECK_LAUNCH();
    if (vec4)
      hipLaunchKernelGGL(k_b_update4<VT>, dim3(nblk), dim3(kBT), 0, s, R, n, m, V, nr, Y, KC, x, tr ? r64 : nullptr,
                         P1, P2);
    else
      hipLaunchKernelGGL(k_b_update<VT>, dim3(nblk), dim3(kBT), 0, s, cc, n, m, V, nr, Y, KC, x, tr ? r64 : nullptr,
                         P1, P2);
    BSPAI_CHECK_LAUNCH();
    if (tr) {
      if ((rc = launch_bspmv(Mb, r64, D, R, R, 1, s))) return rc;  // d = M_b^T (V y) in FP64
      hipLaunchKernelGGL(k_b_add, dim3(nblk), dim3(kBT), 0, s, cc, n, D, x, P1, P2);
      BSPAI_CHECK_LAUNCH();
    }
    if ((rc = finish(true, P1, S + 6 * R, 0)) || (rc = finish(true, P2, S + 7 * R, 0))) return rc;
    std::vector<double> hdx;
    if ((rc = to_host(S + 6 * R, hdx, 2))) return rc;  // rows 6 and 7: max|d|, max|x|
    const double *hdn = hdx.data(), *hxn = hdx.data() + R;
    for (int c = 0; c < R; c++) {
      if (!active[c]) continue;
      if (it < 64) st[c].its[it] = kc[c];
      st[c].its_total += kc[c];
      double dx = hxn[c] > 0 ? hdn[c] / hxn[c] : 0.0;
      if (it >= 1 && stag_ratio > 0.0 && dx > stag_ratio * dx_prev[c]) stag[c] = 1;
      dx_prev[c] = dx;
    }
    it++;
  }
  int worst = BSPAI_OK;
  for (int c = 0; c < R; c++) {
    st[c].status = status[c];
    worst = worse_status(worst, status[c]);
  }
  if (st_host) memcpy(st_host, st.data(), sizeof(gmres_ir_stats) * R);
  BSPAI_HIP(hipStreamSynchronize(s));
  if (worst == BSPAI_ENOCONV) return fail(BSPAI_ENOCONV, "gmres_ir_solve: some right-hand side reached i_max");
  if (worst == BSPAI_ESTAG)
    return fail(BSPAI_ESTAG, "gmres_ir_solve: some right-hand side stagnated before meeting a tolerance");
  if (worst == BSPAI_ENAN) return fail(BSPAI_ENAN, "gmres_ir_solve: NaN or infinity in a residual");
  return BSPAI_OK;
}

// columns [c0, c0 + g) of an n x R row-major array to an n x g one and back
__global__ void k_gather_cols(int64_t n, int R, int c0, int g, const double *src, double *dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * g) dst[t] = src[(t / g) * R + c0 + t % g];
}
__global__ void k_scatter_cols(int64_t n, int R, int c0, int g, const double *src, double *dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * g) dst[(t / g) * R + c0 + t % g] = src[t];
}

// When the column groups pay: from n R u_g values of 64 MiB every pass is
// bound by the bytes it moves (the groups move a quarter of them); below,
// a pass of the per-pass kernels costs two launches shared by all columns and
// a group pass one grid exchange, so the groups pay while there are at most
// four of them
constexpr double kGroupBytes = 64.0 * 1024 * 1024;
constexpr int kMaxLaunchBoundGroups = 4;

template <typename VT>
int solve_many(const bspai_csr *A, const bspai_handle *Ab, const double *b, const bspai_handle *M,
               const gmres_ir_tol *tol, double *x, int R, int m, gmres_ir_stats *st_host, hipStream_t s) {
  constexpr int C = 16 / (int)sizeof(VT);
  const int n = A->n;
  const int mode = batch_mode();
  const bool fits = mgs_persist_rpt(n) > 0 && R >= C;
  const bool big = (double)n * R * sizeof(VT) >= kGroupBytes;
  const bool grouped = mode == 2 ? fits : (mode == 1 ? false : fits && (big || R <= kMaxLaunchBoundGroups * C));
  if (!grouped) return solve_batched<VT>(A, Ab, b, M, tol, x, R, m, st_host, s, false);
  if (R == C) return solve_batched<VT>(A, Ab, b, M, tol, x, R, m, st_host, s, true);
  // consecutive groups of C columns (a trailing C + 1 or fewer than C go
  // together through the per-pass kernels), each solved on its own
  std::vector<gmres_ir_stats> st(R);
  DevBuf bg, xg;
  int rc;
  if ((rc = dalloc(&bg.p, 8 * (size_t)n * (C + 1))) || (rc = dalloc(&xg.p, 8 * (size_t)n * (C + 1)))) return rc;
  int worst = BSPAI_OK;
  for (int c0 = 0; c0 < R;) {
    const int left = R - c0;
    const int g = left == C + 1 ? C + 1 : (left < C ? left : C);
    const unsigned eg = (unsigned)(((int64_t)n * g + 255) / 256);
    hipLaunchKernelGGL(k_gather_cols, dim3(eg), dim3(256), 0, s, (int64_t)n, R, c0, g, b, (double *)bg.p);
    BSPAI_CHECK_LAUNCH();
    if (tol->x0_mode == 3) {
      hipLaunchKernelGGL(k_gather_cols, dim3(eg), dim3(256), 0, s, (int64_t)n, R, c0, g, x, (double *)xg.p);
      BSPAI_CHECK_LAUNCH();
    }
    rc = solve_batched<VT>(A, Ab, (const double *)bg.p, M, tol, (double *)xg.p, g, m, st.data() + c0, s, g == C);
    if (rc != BSPAI_OK && rc != BSPAI_ENOCONV && rc != BSPAI_ESTAG && rc != BSPAI_ENAN) return rc;
    worst = worse_status(worst, rc);
    hipLaunchKernelGGL(k_scatter_cols, dim3(eg), dim3(256), 0, s, (int64_t)n, R, c0, g, (const double *)xg.p, x);
    BSPAI_CHECK_LAUNCH();
    c0 += g;
  }
  BSPAI_HIP(hipStreamSynchronize(s));
  if (st_host) memcpy(st_host, st.data(), sizeof(gmres_ir_stats) * R);
  if (worst == BSPAI_ENAN) return fail(BSPAI_ENAN, "gmres_ir_solve: NaN or infinity in a residual");
  if (worst == BSPAI_ENOCONV) return fail(BSPAI_ENOCONV, "gmres_ir_solve: some right-hand side reached i_max");
  if (worst == BSPAI_ESTAG)
    return fail(BSPAI_ESTAG, "gmres_ir_solve: some right-hand side stagnated before meeting a tolerance");
  return BSPAI_OK;
}

template int solve_many<float>(const bspai_csr *, const bspai_handle *, const double *, const bspai_handle *,
                               const gmres_ir_tol *, double *, int, int, gmres_ir_stats *, hipStream_t);
template int solve_many<double>(const bspai_csr *, const bspai_handle *, const double *, const bspai_handle *,
                                const gmres_ir_tol *, double *, int, int, gmres_ir_stats *, hipStream_t);
template int solve_batched<float>(const bspai_csr *, const bspai_handle *, const double *, const bspai_handle *,
                                  const gmres_ir_tol *, double *, int, int, gmres_ir_stats *, hipStream_t, bool);
template int solve_batched<double>(const bspai_csr *, const bspai_handle *, const double *, const bspai_handle *,
                                   const gmres_ir_tol *, double *, int, int, gmres_ir_stats *, hipStream_t, bool);

}  // namespace bspai
