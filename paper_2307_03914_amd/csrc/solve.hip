// gmres_ir_solve: BSPAI-GMRES-IR (Algorithm 4) as one persistent cooperative
// kernel per solve.
//
// G co-resident blocks of 512 threads each own a contiguous range of rows.
// Everything of Algorithm 4 after the SPAI build runs inside the kernel: x_0,
// the refinement residual (FP64 or double-double), the stopping tests, the
// preconditioned operator z = M_b (A_p v) (or A_p^T (M_b^T v) for the
// transposed solve), modified Gram-Schmidt, Givens rotations, the update
// d = V y and x = x + d.  The only cross-block communication is a per-block
// epoch flag barrier and fixed-order all-reductions of FP64 partials, so every
// block takes identical decisions and the result is deterministic.
//
// Modified Gram-Schmidt is kept literal: the projection on v_i uses z already
// orthogonalised against v_1..v_{i-1}, so step j needs j+1 dependent
// reductions.  Each pass fuses the update with v_{i-1} and the dot with v_i.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"
#include "spmv_dev.h"

namespace bspai {

constexpr int kSolveThreads = 512;
constexpr int kWaves = kSolveThreads / 64;
constexpr int kNumSlots = 4;
constexpr int kMaxBlocks = 256;
constexpr int kMaxSlotWidth = 2;
// Largest GMRES cap whose packed triangular R and rotation state fit in LDS
// next to the product tile.
constexpr int kMaxGmres = 160;
constexpr int kTileBytes = 49152;  // least LDS for the products of one sub-range of rows
// dynamic LDS of a solver block: all of the CU's 160 KB but 1 KB for the
// kernels' static arrays; the products take what the GMRES state leaves
constexpr size_t kLdsBytes = 160 * 1024 - 1024;
constexpr unsigned kSpinLimit = 1u << 27;  // ~ seconds: a bound, never reached by a healthy run

struct Grid {
  unsigned *flags;  // [G] epoch reached by each block
  unsigned *abortf; // set when a wait exceeds the spin bound
  double *slots;    // [kNumSlots][kMaxBlocks][kMaxSlotWidth][2] tagged 64-bit words
  unsigned long long *wide;  // [kNumSlots][G][kMaxGmres + 1][2] for vector reductions (or null)
  int G;
};

// bytes of the vector-reduction words of a grid of G blocks
constexpr size_t wide_bytes(int G) { return 16 * (size_t)kNumSlots * G * (kMaxGmres + 1); }
constexpr size_t kWideBytes = wide_bytes(kMaxBlocks);

template <typename VT>
struct SolveParams {
  int n, G, rows_per_block, m_max;
  int lanes_a, lanes_m;
  int rows_a, rows_m;  // rows per sub-range of the tile products (up to 2 per thread)
  int tile_bytes;      // LDS for the products
  const int32_t *a_rp, *a_col;
  const double *a_val;  // A (A^T for trans) in FP64, for the residual and ||A||_inf
  BMat Ap;              // the same matrix with values rounded to u_p = u_g
  BMat Mb;              // bucketed M (M^T for trans)
  const int32_t *f_rp, *f_col;
  const double *f_val;  // FP64 M (M^T for trans), x0_mode 0
  int x0_mode, trans, ur_dd, i_max;
  int orth;  // 0 MGS, 1 CGS2
  double tau, tol_rr, tol_be;
  double stag;  // stagnation ratio (<= 0: no stagnation stop)
  const double *b;
  double *x;
  VT *rv, *w, *zg, *V;
  double *dv, *dv2;
  Grid grid;
  gmres_ir_stats *stats;
};

// ------------------------------------------------------------------ sync

// bid: index of the calling block among the G blocks that share `g`
__device__ bool grid_sync(const Grid &g, unsigned &epoch, int bid) {
  epoch++;
  __syncthreads();
  if (g.G == 1) return true;
  if (threadIdx.x == 0) __hip_atomic_store(&g.flags[bid], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  int bad = 0;
  if ((int)threadIdx.x < g.G) {
    unsigned spins = 0;
    while (__hip_atomic_load(&g.flags[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      if (++spins > kSpinLimit || __hip_atomic_load(g.abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        bad = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  bad = __syncthreads_or(bad);
  if (bad && threadIdx.x == 0) __hip_atomic_store(g.abortf, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return !bad;
}

// DPP move of a double (two 32-bit halves); lanes whose row is masked off or
// whose source lane is out of range receive 0
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, BOUND);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, BOUND);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront with DPP row shifts and row
// broadcasts (register-to-register, no LDS permutes): row_shr 1, 2, 4, 8
// leave each row's sum in its lane 15, row_bcast:15 adds row 0 into row 1 and
// row 2 into row 3, row_bcast:31 adds lane 31 into rows 2 and 3, and lane 63
// holds the total, which every lane reads back.  Fixed order: identical bits
// in every lane and every call.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_mov<0x111, 0xf, true>(v);
  v += dpp_mov<0x112, 0xf, true>(v);
  v += dpp_mov<0x114, 0xf, true>(v);
  v += dpp_mov<0x118, 0xf, true>(v);
  v += dpp_mov<0x142, 0xa, false>(v);
  v += dpp_mov<0x143, 0xc, false>(v);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

template <bool MAX>
__device__ __forceinline__ double wave_red(double v) {
  if constexpr (!MAX) {
    return wave_sum_dpp(v);
  } else {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
  }
}

// A scalar exchange needs no fences: every block publishes its FP64 partial as
// two 64-bit words (payload in the upper 48 bits, the low 16 bits carry the
// exchange's sequence tag) with relaxed agent-scope atomic stores, and readers
// poll the words with relaxed atomic loads until both tags match.  Atomicity of
// each word is all the protocol relies on; no cache is written back or
// invalidated, so the blocks keep their basis slices in L2.
// exchange round -> 16-bit tag; never 0, the value of cleared slot words
__device__ __forceinline__ unsigned long long tag16(unsigned rtag) { return rtag % 65535u + 1u; }

__device__ __forceinline__ void publish_partial(unsigned long long *w, double v, unsigned rtag) {
  unsigned long long b = __double_as_longlong(v);
  unsigned long long t = tag16(rtag);
  __hip_atomic_store(&w[0], (b & ~0xFFFFull) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&w[1], ((b & 0xFFFFull) << 16) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// returns false when the wait exceeds the bound or another block aborted
__device__ __forceinline__ bool collect_partial(unsigned long long *w, unsigned rtag, const unsigned *abortf,
                                                double *out) {
  const unsigned long long t = tag16(rtag);
  unsigned long long a, b;
  unsigned spins = 0;
  for (;;) {
    a = __hip_atomic_load(&w[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b = __hip_atomic_load(&w[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((a & 0xFFFFull) == t && (b & 0xFFFFull) == t) break;
    if (++spins > kSpinLimit || __hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
  }
  *out = __longlong_as_double((long long)((a & ~0xFFFFull) | ((b >> 16) & 0xFFFFull)));
  return true;
}

// Workgroup barrier that orders LDS only: global loads still in flight (the
// prefetched basis slice of the next MGS pass) stay in flight across it,
// where __syncthreads would first wait for every outstanding memory access.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// XCC_ID hardware register (hwreg 20, bits 3:0): the accelerator complex die
// (XCD) the wave runs on.
__device__ __forceinline__ unsigned xcd_id() { return __builtin_amdgcn_s_getreg(6164) & 0xFu; }

// Puts a cooperative grid's work on one XCD.  Every block registers its XCD;
// once all gridDim.x blocks have registered (a cooperative launch keeps them
// all resident), the lowest-numbered XCD with at least `want` blocks is
// chosen and its first `want` arrivals take ranks 0..want-1.  Returns the
// block's rank, or -1 for a block that is not used (all blocks get -1, and
// the abort flag is set, when no XCD holds `want` blocks or a wait runs out).
// reg: 9 words cleared before the launch ([0..7] arrivals per XCD, [8] blocks
// registered).  One-off cost per launch: one registration round trip.
__device__ int one_xcd_rank(unsigned *reg, int want, unsigned *abortf) {
  __shared__ int s_rank;
  if (threadIdx.x == 0) {
    const unsigned x = xcd_id() & 7u;
    const unsigned r = __hip_atomic_fetch_add(&reg[x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&reg[8], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    bool ok = true;
    while (__hip_atomic_load(&reg[8], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
      if (++spins > kSpinLimit || __hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    int target = -1;
    if (ok)
      for (int k = 0; k < 8 && target < 0; k++)
        if (__hip_atomic_load(&reg[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)want) target = k;
    if (target < 0) __hip_atomic_store(abortf, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_rank = ((int)x == target && r < (unsigned)want) ? (int)r : -1;
  }
  __syncthreads();
  return s_rank;
}

// All-reduction of W values over the grid (sum or max).  Every block combines
// the same G partials in the same order, so all blocks obtain identical
// results.  Two LDS-only workgroup barriers: it orders no global memory
// between the block's threads and publishes nothing but the scalars (use
// grid_sync or __syncthreads for that).  sh: kWaves kMaxSlotWidth +
// kMaxSlotWidth + 1 doubles.
template <int W, bool MAX>
__device__ bool grid_reduce(const Grid &g, unsigned &rtag, double (&v)[W], double *sh, int bid) {
  static_assert(W >= 1 && W <= kMaxSlotWidth, "grid_reduce handles 1..kMaxSlotWidth values");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double part[W];
#pragma unroll
  for (int c = 0; c < W; c++) part[c] = wave_red<MAX>(v[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < W; c++) sh[wv * W + c] = part[c];
  }
  lds_barrier();
  // results and abort flag at a fixed place past every call's wave partials:
  // the next call's partials (written before its first barrier, while other
  // waves may still read these results) never overlap them
  double *res = sh + kWaves * kMaxSlotWidth;
  int bad = 0;
  rtag++;
  if (g.G == 1) {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < W; c++) {
        double a = sh[c];
        for (int k = 1; k < kWaves; k++) a = MAX ? fmax(a, sh[k * W + c]) : a + sh[k * W + c];
        res[c] = a;
      }
    }
  } else {
    unsigned long long *set = reinterpret_cast<unsigned long long *>(g.slots) +
                              (size_t)(rtag % kNumSlots) * kMaxBlocks * kMaxSlotWidth * 2;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < W; c++) {
        double a = sh[c];
        for (int k = 1; k < kWaves; k++) a = MAX ? fmax(a, sh[k * W + c]) : a + sh[k * W + c];
        publish_partial(set + ((size_t)bid * kMaxSlotWidth + c) * 2, a, rtag);
      }
    }
    if (wv == 0) {
#pragma unroll
      for (int c = 0; c < W; c++) {
        double acc = MAX ? 0.0 : 0.0;
        for (int t = lane; t < g.G; t += 64) {
          double x;
          if (!collect_partial(set + ((size_t)t * kMaxSlotWidth + c) * 2, rtag, g.abortf, &x)) {
            bad = 1;
            break;
          }
          acc = MAX ? fmax(acc, x) : acc + x;
        }
        acc = wave_red<MAX>(acc);
        if (lane == 0) res[c] = acc;
      }
    }
  }
  // only wave 0 polls: its vote is the block's abort flag
  if (wv == 0) {
    const bool any_bad = __any(bad);
    if (lane == 0) res[W] = any_bad ? 1.0 : 0.0;
  }
  lds_barrier();
  if (res[W] != 0.0) {
    if (threadIdx.x == 0) __hip_atomic_store(g.abortf, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
#pragma unroll
  for (int c = 0; c < W; c++) v[c] = res[c];
  return true;
}

// All-reduction (sum) of W <= kMaxGmres + 1 values over the grid, for CGS2.
// in: the block's W partials (LDS); out: the grid sums (LDS); tmp: blockDim
// doubles of LDS.  Thread t*tpv + q sums value t over blocks q, q + tpv, ...
// (tpv a power of two, the most that fit the block), issuing the loads of
// kVecBatch blocks at once, and the tpv sums are then added in order q = 0,
// 1, ...: every block obtains identical bits.  Ends with a workgroup barrier.
constexpr int kVecBatch = 16;
__device__ bool grid_reduce_vec(const Grid &g, unsigned &rtag, int W, const double *in, double *out, double *tmp,
                                int bid) {
  const int tid = threadIdx.x, nt = blockDim.x;
  rtag++;
  if (g.G == 1) {
    for (int t = tid; t < W; t += nt) out[t] = in[t];
    __syncthreads();
    return true;
  }
  constexpr size_t kStride = kMaxGmres + 1;
  unsigned long long *set = g.wide + (size_t)(rtag % kNumSlots) * g.G * kStride * 2;
  for (int t = tid; t < W; t += nt) publish_partial(set + ((size_t)bid * kStride + t) * 2, in[t], rtag);
  int tpv = 1;
  while (2 * tpv * W <= nt && 2 * tpv <= g.G) tpv *= 2;
  const int t = tid / tpv, q = tid % tpv;
  const unsigned long long tg = tag16(rtag);
  int bad = 0;
  if (t < W) {
    double acc = 0.0;
    for (int b0 = q; b0 < g.G && !bad; b0 += tpv * kVecBatch) {
      unsigned long long wa[kVecBatch], wb[kVecBatch];
#pragma unroll
      for (int u = 0; u < kVecBatch; u++) {
        const int b = b0 + u * tpv;
        wa[u] = wb[u] = 0;
        if (b < g.G) {
          unsigned long long *w = set + ((size_t)b * kStride + t) * 2;
          wa[u] = __hip_atomic_load(&w[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          wb[u] = __hip_atomic_load(&w[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
#pragma unroll
      for (int u = 0; u < kVecBatch; u++) {
        const int b = b0 + u * tpv;
        if (b >= g.G || bad) continue;
        double x;
        if ((wa[u] & 0xFFFFull) == tg && (wb[u] & 0xFFFFull) == tg) {
          x = __longlong_as_double((long long)((wa[u] & ~0xFFFFull) | ((wb[u] >> 16) & 0xFFFFull)));
        } else if (!collect_partial(set + ((size_t)b * kStride + t) * 2, rtag, g.abortf, &x)) {
          bad = 1;
          continue;
        }
        acc += x;
      }
    }
    tmp[tid] = acc;
  }
  bad = __syncthreads_or(bad);
  if (bad) {
    if (tid == 0) __hip_atomic_store(g.abortf, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  for (int t2 = tid; t2 < W; t2 += nt) {
    double a = tmp[t2 * tpv];
    for (int q2 = 1; q2 < tpv; q2++) a += tmp[t2 * tpv + q2];
    out[t2] = a;
  }
  __syncthreads();
  return true;
}

// ------------------------------------------------------------------ rows

template <typename XT, typename YT>
__device__ __forceinline__ void spmv_rows_dispatch(int lanes, const BMat &M, const XT *x, YT *y, int r0, int r1) {
  switch (lanes) {
    case 4: bspmv_rows<4, XT, YT>(M, x, y, r0, r1); break;
    case 16: bspmv_rows<16, XT, YT>(M, x, y, r0, r1); break;
    default: bspmv_rows<8, XT, YT>(M, x, y, r0, r1); break;
  }
}

// rows [r0, r1) of a CSR product, rows t and t + blockDim of each pass
// interleaved in one thread
template <typename XT, typename PT>
__device__ __forceinline__ void csr_rows2(const BMat &M, const XT *__restrict__ x, XT *__restrict__ y, int r0,
                                          int r1) {
  const int nt = blockDim.x;
  for (int i = r0 + (int)threadIdx.x; i < r1; i += 2 * nt) {
    int rows[2] = {i, i + nt < r1 ? i + nt : -1};
    double out[2];
    bspmv_rows_thread<2, XT, PT>(M, x, rows, out);
    y[i] = (XT)out[0];
    if (rows[1] >= 0) y[rows[1]] = (XT)out[1];
  }
}

// r_i = b_i - sum_j a_ij x_j: double-double (TwoProd with FMA, TwoSum,
// compensation summed in FP64, as in Ogita-Rump-Oishi's Dot2) or plain FP64,
// entries in CSR order.  The file is compiled without FMA contraction, so
// the products and sums here are rounded separately, as TwoSum requires.
__device__ __forceinline__ double residual_row(const int32_t *rp, const int32_t *col, const double *val,
                                               const double *b, const double *x, int i, int dd) {
  double s = b[i];
  if (dd) {
    double c = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; p++) {
      double a = -val[p], xv = x[col[p]];
      double pr = __dmul_rn(a, xv);
      double pe = fma(a, xv, -pr);
      double t = __dadd_rn(s, pr);
      double z = __dsub_rn(t, s);
      double se = __dadd_rn(__dsub_rn(s, __dsub_rn(t, z)), __dsub_rn(pr, z));
      s = t;
      c = __dadd_rn(c, __dadd_rn(pe, se));
    }
    return __dadd_rn(s, c);
  }
  for (int p = rp[i]; p < rp[i + 1]; p++) s = __dsub_rn(s, __dmul_rn(val[p], x[col[p]]));
  return s;
}

// ------------------------------------------------------------------ kernel

// Algorithm 4 for one system by the G blocks of `G`; bid is the calling
// block's index among them.  epoch and rtag carry on from earlier calls by
// the same blocks.  Returns false when a wait timed out (G.abortf is set).
template <typename VT, typename PT, int ZR, bool CGS2 = false>
__device__ bool gmres_ir_body(const SolveParams<VT> &p, const Grid &G, int bid, unsigned &epoch, unsigned &rtag,
                              double *sm, double *sh, int &s_flag) {
  const int kCap = p.tile_bytes / (int)sizeof(PT);
  const int m = p.m_max;
  double *cs = sm;            // m
  double *sn = cs + m;        // m
  double *g = sn + m;         // m + 1
  double *hcol = g + m + 1;   // m + 1
  double *y = hcol + m + 1;   // m
  double *Rp = y + m;         // m (m + 1) / 2, column c holds R(0..c, c) at c (c + 1) / 2
  PT *tprod = reinterpret_cast<PT *>(Rp + (size_t)m * (m + 1) / 2);  // kCap products
  // products of both operators: all buckets of a sub-range of rows at once
#define SPMV_ROWS(Mat, in, out, rows)                                                   \
  do {                                                                                  \
    if ((rows) > (int)blockDim.x)                                                       \
      bspmv_tile_all<VT, VT, PT, 2>(Mat, in, out, r0, r1, tprod, kCap, rows);           \
    else                                                                                \
      bspmv_tile_all<VT, VT, PT, 1>(Mat, in, out, r0, r1, tprod, kCap, rows);           \
  } while (0)
#define SPMV_M(Mat, in, out) SPMV_ROWS(Mat, in, out, p.rows_m)
#define SPMV_A(Mat, in, out) SPMV_ROWS(Mat, in, out, p.rows_a)
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = p.n;
  const int r0 = min(n, bid * p.rows_per_block);  // blocks past the last row own none
  const int r1 = min(n, r0 + p.rows_per_block);
  const bool rec = (bid == 0 && tid == 0);

#define OWN_ROWS(k, i) \
  _Pragma("unroll") for (int k = 0; k < ZR; k++) if (int i = r0 + k * nt + tid; i < r1)

  // ||A||_inf (rows summed left to right) and ||b||_inf
  double normA, normb;
  {
    double v[2] = {0.0, 0.0};
    OWN_ROWS(k, i) {
      double s = 0.0;
      for (int q = p.a_rp[i]; q < p.a_rp[i + 1]; q++) s += fabs(p.a_val[q]);
      v[0] = fmax(v[0], s);
      v[1] = fmax(v[1], fabs(p.b[i]));
    }
    if (!grid_reduce<2, true>(G, rtag, v, sh, bid)) return false;
    normA = v[0];
    normb = v[1];
  }
  // x_0 (Algorithm 4 step 2)
  if (p.x0_mode == 0) {
    OWN_ROWS(k, i) {
      double acc = 0.0;
      for (int q = p.f_rp[i]; q < p.f_rp[i + 1]; q++) acc = __dadd_rn(acc, __dmul_rn(p.f_val[q], p.b[p.f_col[q]]));
      p.x[i] = acc;
    }
  } else if (p.x0_mode == 1) {
    bspmv_tile_all<double, double, double>(p.Mb, p.b, p.x, r0, r1, reinterpret_cast<double *>(tprod),
                                           p.tile_bytes / 8, min(p.rows_m / 2 > 0 ? p.rows_m / 2 : 1, nt));
  } else if (p.x0_mode == 2) {
    OWN_ROWS(k, i) { p.x[i] = 0.0; }
  }
  if (!grid_sync(G, epoch, bid)) return false;

  int it = 0, stag = 0, status = BSPAI_OK, reason = 0, its_total = 0;
  double dx_prev = 0.0;
  for (;;) {
    // residual (u_r), backward error and relative residual
    double rr[ZR];
    double nv[2] = {0.0, 0.0};
    OWN_ROWS(k, i) {
      double r = residual_row(p.a_rp, p.a_col, p.a_val, p.b, p.x, i, p.ur_dd);
      rr[k] = r;
      nv[0] = fmax(nv[0], isfinite(r) ? fabs(r) : INFINITY);
      double xv = p.x[i];
      nv[1] = fmax(nv[1], isfinite(xv) ? fabs(xv) : INFINITY);
    }
    if (!grid_reduce<2, true>(G, rtag, nv, sh, bid)) return false;
    const double nr = nv[0], nx = nv[1];
    const double eta = nr / (normA * nx + normb);
    const double rho = normb > 0 ? nr / normb : nr;
    if (rec && it <= 64) {
      p.stats->eta[it] = eta;
      p.stats->relres[it] = rho;
    }
    if (!isfinite(nr) || !isfinite(nx)) { status = BSPAI_ENAN; reason = 5; break; }
    if (rho <= p.tol_rr) { reason = 1; break; }
    if (eta <= p.tol_be) { reason = 2; break; }
    if (stag) { status = BSPAI_ESTAG; reason = 3; break; }
    if (it >= p.i_max || it >= 64) { status = BSPAI_ENOCONV; reason = 4; break; }

    // ---------------- GMRES on M_b A d = M_b r (left) / A^T M_b^T w = r (right)
    OWN_ROWS(k, i) { p.rv[i] = (VT)rr[k]; }
    VT *V0 = p.V;
    double ss[1] = {0.0};
    if (!p.trans) {
      if (!grid_sync(G, epoch, bid)) return false;
      SPMV_M(p.Mb, p.rv, V0);
      __syncthreads();
      OWN_ROWS(k, i) {
        double s = (double)V0[i];
        ss[0] += s * s;
      }
    } else {
      OWN_ROWS(k, i) {
        double s = (double)p.rv[i];
        V0[i] = p.rv[i];
        ss[0] += s * s;
      }
    }
    if (!grid_reduce<1, false>(G, rtag, ss, sh, bid)) return false;
    const double beta = sqrt(ss[0]);
    int kdone = 0;
    if (beta > 0.0) {
      OWN_ROWS(k, i) { V0[i] = (VT)((double)V0[i] / beta); }
      if (tid == 0) g[0] = beta;
      if (!grid_sync(G, epoch, bid)) return false;
      for (int j = 0; j < m; j++) {
        const VT *vj = p.V + (size_t)j * n;
        if (!p.trans) {
          SPMV_A(p.Ap, vj, p.w);
          if (!grid_sync(G, epoch, bid)) return false;
          SPMV_M(p.Mb, p.w, p.zg);
        } else {
          SPMV_M(p.Mb, vj, p.w);
          if (!grid_sync(G, epoch, bid)) return false;
          SPMV_A(p.Ap, p.w, p.zg);
        }
        __syncthreads();
        VT zr[ZR];
        OWN_ROWS(k, i) { zr[k] = p.zg[i]; }
        if constexpr (!CGS2) {
          // modified Gram-Schmidt: pass i removes the v_{i-1} component and
          // measures the v_i component of the updated z.  The slice of v_{i+1}
          // does not depend on h_i, so it is loaded before the reduction of
          // pass i and arrives while the blocks exchange their partials.
          double hprev = 0.0;
          VT vprev[ZR], vcur[ZR], vnext[ZR];
          OWN_ROWS(k, i) { vnext[k] = p.V[i]; }
          for (int i2 = 0; i2 <= j; i2++) {
#pragma unroll
            for (int k = 0; k < ZR; k++) {
              vprev[k] = vcur[k];
              vcur[k] = vnext[k];
            }
            if (i2 < j) {
              const VT *vn2 = p.V + (size_t)(i2 + 1) * n;
              OWN_ROWS(k, i) { vnext[k] = vn2[i]; }
            }
            double part[1] = {0.0};
            OWN_ROWS(k, i) {
              if (i2 > 0) zr[k] = (VT)fma(-hprev, (double)vprev[k], (double)zr[k]);
              part[0] = fma((double)vcur[k], (double)zr[k], part[0]);
            }
            if (!grid_reduce<1, false>(G, rtag, part, sh, bid)) return false;
            hprev = part[0];
            if (tid == 0) hcol[i2] = hprev;
          }
          OWN_ROWS(k, i) { zr[k] = (VT)fma(-hprev, (double)vcur[k], (double)zr[k]); }
        } else {
          // CGS2: two passes, each taking all j + 1 coefficients against the
          // same z in one vector all-reduction, then z - V h formed in FP64
          // (FMAs in the order i = 0..j) and rounded once.  The product tile
          // is free here and holds the reduction's scratch.
          const int W = j + 1, lane = tid & 63, wv = tid >> 6;
          double *wpart = reinterpret_cast<double *>(tprod);  // [kWaves][W]
          double *bpart = wpart + kWaves * (kMaxGmres + 1);   // [W]
          double *tmp = bpart + (kMaxGmres + 1);              // [blockDim]
          double *hv = tmp + kSolveThreads;                   // [W]
          // basis slices are loaded kCh vectors at a time so that the loads
          // are in flight together rather than one latency per vector
          constexpr int kCh = ZR <= 2 ? 8 : (ZR <= 4 ? 4 : 2);    // dot products
          constexpr int kChU = ZR <= 2 ? 16 : (ZR <= 4 ? 8 : 4);  // update
          for (int pass = 0; pass < 2; pass++) {
            for (int i0 = 0; i0 < W; i0 += kCh) {
              VT vv[kCh][ZR];
#pragma unroll
              for (int u = 0; u < kCh; u++) {
                const VT *vi = p.V + (size_t)(i0 + u) * n;
                OWN_ROWS(k, i) { vv[u][k] = i0 + u < W ? vi[i] : (VT)0; }
              }
              double part[kCh];
#pragma unroll
              for (int u = 0; u < kCh; u++) {
                part[u] = 0.0;
                OWN_ROWS(k, i) { part[u] = fma((double)vv[u][k], (double)zr[k], part[u]); }
              }
#pragma unroll
              for (int u = 0; u < kCh; u++) part[u] = wave_red<false>(part[u]);
              if (lane == 0) {
#pragma unroll
                for (int u = 0; u < kCh; u++)
                  if (i0 + u < W) wpart[wv * W + i0 + u] = part[u];
              }
            }
            __syncthreads();
            for (int t = tid; t < W; t += nt) {
              double a = wpart[t];
              for (int w = 1; w < kWaves; w++) a += wpart[w * W + t];
              bpart[t] = a;
            }
            __syncthreads();
            if (!grid_reduce_vec(G, rtag, W, bpart, hv, tmp, bid)) return false;
            double acc[ZR];
            OWN_ROWS(k, i) { acc[k] = (double)zr[k]; }
            for (int i0 = 0; i0 < W; i0 += kChU) {
              VT vv[kChU][ZR];
#pragma unroll
              for (int u = 0; u < kChU; u++) {
                const VT *vi = p.V + (size_t)(i0 + u) * n;
                OWN_ROWS(k, i) { vv[u][k] = i0 + u < W ? vi[i] : (VT)0; }
              }
#pragma unroll
              for (int u = 0; u < kChU; u++) {
                if (i0 + u < W) {
                  const double h = hv[i0 + u];
                  OWN_ROWS(k, i) { acc[k] = fma(-h, (double)vv[u][k], acc[k]); }
                }
              }
            }
            OWN_ROWS(k, i) { zr[k] = (VT)acc[k]; }
            for (int t = tid; t < W; t += nt) hcol[t] = pass == 0 ? hv[t] : hcol[t] + hv[t];
            __syncthreads();
          }
        }
        double nz[1] = {0.0};
        OWN_ROWS(k, i) { nz[0] = fma((double)zr[k], (double)zr[k], nz[0]); }
        if (!grid_reduce<1, false>(G, rtag, nz, sh, bid)) return false;
        const double hn = sqrt(nz[0]);
        VT *vn = p.V + (size_t)(j + 1) * n;
        OWN_ROWS(k, i) { vn[i] = hn > 0.0 ? (VT)((double)zr[k] / hn) : (VT)0; }
        // Givens rotations on the new Hessenberg column (identical in every block)
        // (the rotated entry i2 + 1 is carried to the next rotation in a
        // register rather than through LDS)
        if (tid == 0) {
          double a = hcol[0];
          for (int i2 = 0; i2 < j; i2++) {
            const double bb = hcol[i2 + 1];
            hcol[i2] = cs[i2] * a + sn[i2] * bb;
            a = -sn[i2] * a + cs[i2] * bb;
          }
          const double bb = hn;
          double rho2 = hypot(a, bb);
          cs[j] = rho2 == 0.0 ? 1.0 : a / rho2;
          sn[j] = rho2 == 0.0 ? 0.0 : bb / rho2;
          hcol[j] = rho2;
          hcol[j + 1] = hn;
          g[j + 1] = -sn[j] * g[j];
          g[j] = cs[j] * g[j];
          s_flag = (fabs(g[j + 1]) <= p.tau * beta) || (hn == 0.0);
        }
        __syncthreads();
        {
          double *Rc = Rp + (size_t)j * (j + 1) / 2;
          for (int i2 = tid; i2 <= j; i2 += nt) Rc[i2] = hcol[i2];
        }
        __syncthreads();
        kdone = j + 1;
        if (s_flag || kdone == m) break;
        if (!grid_sync(G, epoch, bid)) return false;
      }
      // y = R^{-1} g by one wavefront (column-oriented back substitution)
      if (tid < 64) {
        constexpr int kPer = (kMaxGmres + 63) / 64;
        double gg[kPer];
#pragma unroll
        for (int t = 0; t < kPer; t++) {
          int c = tid + 64 * t;
          gg[t] = c < kdone ? g[c] : 0.0;
        }
        for (int c = kdone - 1; c >= 0; c--) {
          const double *Rc = Rp + (size_t)c * (c + 1) / 2;
          double gsel = 0.0;
#pragma unroll
          for (int t = 0; t < kPer; t++)
            if (t == c / 64) gsel = gg[t];
          double gc = __shfl(gsel, c % 64);
          double yc = gc / Rc[c];
          if (tid == 0) y[c] = yc;
#pragma unroll
          for (int t = 0; t < kPer; t++) {
            int r = tid + 64 * t;
            if (r < c) gg[t] -= Rc[r] * yc;
          }
        }
      }
      __syncthreads();
    }
    // d = V y in FP64; x = x + d (M_b^T applied to V y first for the right-preconditioned solve)
    double dn[2] = {0.0, 0.0};
    if (!p.trans) {
      OWN_ROWS(k, i) {
        double d = 0.0;
        for (int c = 0; c < kdone; c++) d = fma((double)p.V[(size_t)c * n + i], y[c], d);
        double xn = p.x[i] + d;
        p.x[i] = xn;
        dn[0] = fmax(dn[0], fabs(d));
        dn[1] = fmax(dn[1], fabs(xn));
      }
    } else {
      OWN_ROWS(k, i) {
        double d = 0.0;
        for (int c = 0; c < kdone; c++) d = fma((double)p.V[(size_t)c * n + i], y[c], d);
        p.dv[i] = d;
      }
      if (!grid_sync(G, epoch, bid)) return false;
      bspmv_tile_all<double, double, double>(p.Mb, p.dv, p.dv2, r0, r1, reinterpret_cast<double *>(tprod),
                                             p.tile_bytes / 8, min(p.rows_m / 2 > 0 ? p.rows_m / 2 : 1, nt));
      __syncthreads();
      OWN_ROWS(k, i) {
        double d = p.dv2[i];
        double xn = p.x[i] + d;
        p.x[i] = xn;
        dn[0] = fmax(dn[0], fabs(d));
        dn[1] = fmax(dn[1], fabs(xn));
      }
    }
    if (!grid_reduce<2, true>(G, rtag, dn, sh, bid)) return false;
    if (!grid_sync(G, epoch, bid)) return false;  // publish x for the next residual
    const double dx = dn[1] > 0 ? dn[0] / dn[1] : 0.0;
    if (it >= 1 && p.stag > 0.0 && dx > p.stag * dx_prev) stag = 1;
    dx_prev = dx;
    if (rec && it < 64) p.stats->its[it] = kdone;
    its_total += kdone;
    it++;
  }
  if (rec) {
    p.stats->steps = it;
    p.stats->its_total = its_total;
    p.stats->stop_reason = reason;
    p.stats->status = status;
  }
  return true;
#undef OWN_ROWS
#undef SPMV_M
#undef SPMV_A
}

// one system on the whole grid
template <typename VT, typename PT, int ZR, bool CGS2>
__global__ void __launch_bounds__(kSolveThreads) k_gmres_ir(const SolveParams<VT> *__restrict__ pp) {
  extern __shared__ double sm[];
  __shared__ double sh[kWaves * kMaxSlotWidth + kMaxSlotWidth + 1];
  __shared__ int s_flag;
  unsigned epoch = 0, rtag = 0;
  (void)gmres_ir_body<VT, PT, ZR, CGS2>(*pp, pp->grid, blockIdx.x, epoch, rtag, sm, sh, s_flag);
}

template <typename VT>
__global__ void k_to_prec(int64_t nnz, const double *a, VT *o) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) o[e] = (VT)a[e];
}

// ------------------------------------------------------------------ host

// optional timing of the solver kernel with HIP events on the solve's stream
static int g_profile = 0;
static double g_last_ms = 0.0;

struct Workspace {
  std::mutex mu;
  void *ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
};
static Workspace g_ws;

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr size_t kSlotBytes = 16 * (size_t)kNumSlots * kMaxBlocks * kMaxSlotWidth;

// device memory of one system's solve, as offsets from a base address
struct SysLayout {
  size_t ap, rv, w, zg, V, dv, dv2, flags, abort, slots, wide, stats, params, acol, trp, tcol, tval, total;
  bool has_wide;
};

template <typename VT>
static SysLayout sys_layout(int n, int64_t nnz, int m, bool tr, bool wide_slots = false) {
  SysLayout L{};
  L.has_wide = wide_slots;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.ap = take(sizeof(VT) * (size_t)(nnz + 1));
  L.rv = take(sizeof(VT) * n);
  L.w = take(sizeof(VT) * n);
  L.zg = take(sizeof(VT) * n);
  L.V = take(sizeof(VT) * (size_t)n * (m + 1));
  L.dv = take(8 * (size_t)n);
  L.dv2 = take(8 * (size_t)n);
  L.flags = take(4 * kMaxBlocks);
  L.abort = take(4);
  L.slots = take(kSlotBytes);
  if (wide_slots) L.wide = take(kWideBytes);
  L.stats = take(sizeof(gmres_ir_stats));
  L.params = take(sizeof(SolveParams<VT>));
  L.acol = take(4 * (size_t)(nnz + 1));
  if (tr) {
    L.trp = take(4 * ((size_t)n + 1));
    L.tcol = take(4 * (size_t)(nnz + 1));
    L.tval = take(8 * (size_t)(nnz + 1));
  }
  L.total = off;
  return L;
}

// LDS of the GMRES state (rotations, g, the Hessenberg column, y, packed R)
constexpr size_t solve_head(int m) { return sizeof(double) * ((size_t)5 * m + 2 + (size_t)m * (m + 1) / 2); }
// the products get the rest of kLdsBytes, so every block takes kLdsBytes
// whatever m is (systems of different m share one multi-system launch)
constexpr size_t tile_bytes(int m) { return (kLdsBytes - solve_head(m)) / 256 * 256; }
static_assert(tile_bytes(kMaxGmres) >= kTileBytes, "GMRES state leaves too little LDS for the products");
static size_t solve_lds(int) { return kLdsBytes; }

// Parameters of one system whose workspace starts at `base` (rows split into
// blocks of rpb rows): A rounded to u_g, A^T and its copy for trans; with Ab
// the GMRES products use the bucketed A_b (A_b^T) instead of A rounded to u_g.
// `wide` is set when the products need FP64 partials.  Enqueues work on s.
template <typename VT>
static int sys_setup(const bspai_csr *A, const bspai_handle *Ab, const double *b, const bspai_handle *M,
                     const gmres_ir_tol *tol, double *x, int m, int G, int rpb, char *base, const SysLayout &L,
                     SolveParams<VT> &p, bool &wide, hipStream_t s) {
  const int n = A->n;
  const int64_t nnz = A->nnz;
  const bool tr = tol->trans != 0;
  memset(&p, 0, sizeof(p));
  p.n = n;
  p.G = G;
  p.rows_per_block = rpb;
  p.m_max = m;
  const int32_t *arp = A->row_ptr, *acol = A->col;
  const double *aval = A->val;
  if (tr) {
    int32_t *trp = reinterpret_cast<int32_t *>(base + L.trp);
    int32_t *tcol = reinterpret_cast<int32_t *>(base + L.tcol);
    double *tval = reinterpret_cast<double *>(base + L.tval);
    int rc = csr_transpose(n, nnz, arp, acol, aval, 8, trp, tcol, tval, s);
    if (rc) return rc;
    arp = trp, acol = tcol, aval = tval;
  }
  if (reinterpret_cast<uintptr_t>(acol) & 15) {  // the tile product loads 16-byte column vectors
    int32_t *ac = reinterpret_cast<int32_t *>(base + L.acol);
    if (nnz) BSPAI_HIP(hipMemcpyAsync(ac, acol, 4 * (size_t)nnz, hipMemcpyDeviceToDevice, s));
    acol = ac;
  }
  p.a_rp = arp;
  p.a_col = acol;
  p.a_val = aval;
  VT *apv = reinterpret_cast<VT *>(base + L.ap);
  if (nnz > 0 && !Ab) {
    hipLaunchKernelGGL(k_to_prec<VT>, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, aval, apv);
    BSPAI_CHECK_LAUNCH();
  }
  BMat Ap;
  memset(&Ap, 0, sizeof(Ap));
  Ap.n = n;
  Ap.nb = 1;
  Ap.nnz = nnz;
  Ap.prec[0] = sizeof(VT) == 8 ? BSPAI_FP64 : BSPAI_FP32;
  Ap.scale[0] = 1.0;
  Ap.rp[0] = arp;
  Ap.col[0] = acol;
  Ap.val[0] = apv;
  Ap.lanes = pick_lanes(Ap, nnz);
  Ap.aligned = 1;
  if (Ab) Ap = tr ? Ab->matT : Ab->mat;
  p.Ap = Ap;
  p.Mb = tr ? M->matT : M->mat;
  auto clamp_lanes = [](int l) { return l <= 4 ? 4 : (l >= 16 ? 16 : 8); };
  p.lanes_a = clamp_lanes(Ap.lanes);
  p.lanes_m = clamp_lanes(p.Mb.lanes);
  p.f_rp = tr ? M->mT_rp : M->m_rp;
  p.f_col = tr ? M->mT_col : M->m_col;
  p.f_val = tr ? M->mT_val : M->m_val;
  p.x0_mode = tol->x0_mode;
  p.orth = tol->orth;
  p.trans = tr;
  p.ur_dd = tol->ur_dd;
  p.i_max = tol->i_max;
  p.tau = tol->tau;
  p.tol_rr = tol->tol_rr;
  p.tol_be = tol->tol_be;
  p.stag = tol->stag_ratio == 0.0 ? 0.5 : tol->stag_ratio;
  p.b = b;
  p.x = x;
  p.rv = reinterpret_cast<VT *>(base + L.rv);
  p.w = reinterpret_cast<VT *>(base + L.w);
  p.zg = reinterpret_cast<VT *>(base + L.zg);
  p.V = reinterpret_cast<VT *>(base + L.V);
  p.dv = reinterpret_cast<double *>(base + L.dv);
  p.dv2 = reinterpret_cast<double *>(base + L.dv2);
  p.grid.flags = reinterpret_cast<unsigned *>(base + L.flags);
  p.grid.abortf = reinterpret_cast<unsigned *>(base + L.abort);
  p.grid.slots = reinterpret_cast<double *>(base + L.slots);
  p.grid.wide = L.has_wide ? reinterpret_cast<unsigned long long *>(base + L.wide) : nullptr;
  p.grid.G = G;
  p.stats = reinterpret_cast<gmres_ir_stats *>(base + L.stats);
  wide = sizeof(VT) == 8;
  for (int k = 0; k < p.Mb.nb; k++) wide = wide || p.Mb.prec[k] == BSPAI_FP64;
  for (int k = 0; k < p.Ap.nb; k++) wide = wide || p.Ap.prec[k] == BSPAI_FP64;
  {
    p.tile_bytes = (int)tile_bytes(m);
    const int cap = p.tile_bytes / (wide ? 8 : 4);
    // sub-ranges of up to two rows per thread for short rows (fewer
    // dependent rounds: A's 5-point rows on the 256^2 system, 10.9 -> 8.3 us
    // per product); longer rows keep one row per thread, where the longer
    // per-thread sums cost more than the saved round (M's 13-entry rows:
    // 13.6 -> 20.3 us with two)
    auto rows_for_avg = [&](double avg) {
      int r = (int)(cap / (1.25 * std::max(avg, 1.0)));
      return std::max(1, std::min((avg <= 8.0 ? 2 : 1) * kSolveThreads, r));
    };
    p.rows_a = rows_for_avg((double)p.Ap.nnz / n);
    p.rows_m = rows_for_avg((double)p.Mb.nnz / n);
  }
  return BSPAI_OK;
}

// rows per block (a multiple of 64) when n rows are split over g blocks
static int rows_for(int n, int g) { return ((n + g - 1) / g + kSlice - 1) / kSlice * kSlice; }

template <typename VT, bool CGS2>
static void *pick_single_o(bool wide, int ZR) {
  if (wide) {
    switch (ZR) {
      case 1: return (void *)k_gmres_ir<VT, double, 1, CGS2>;
      case 2: return (void *)k_gmres_ir<VT, double, 2, CGS2>;
      case 4: return (void *)k_gmres_ir<VT, double, 4, CGS2>;
      case 8: return (void *)k_gmres_ir<VT, double, 8, CGS2>;
      default: return (void *)k_gmres_ir<VT, double, 16, CGS2>;
    }
  }
  switch (ZR) {
    case 1: return (void *)k_gmres_ir<VT, float, 1, CGS2>;
    case 2: return (void *)k_gmres_ir<VT, float, 2, CGS2>;
    case 4: return (void *)k_gmres_ir<VT, float, 4, CGS2>;
    case 8: return (void *)k_gmres_ir<VT, float, 8, CGS2>;
    default: return (void *)k_gmres_ir<VT, float, 16, CGS2>;
  }
}

template <typename VT>
static void *pick_single(bool wide, int ZR, bool cgs2) {
  return cgs2 ? pick_single_o<VT, true>(wide, ZR) : pick_single_o<VT, false>(wide, ZR);
}

// One system, one right-hand side, as one persistent kernel.  The workspace
// is the library's grow-only block (g_ws) or, when ext_base is given, the
// caller-side block of ext_cap bytes at that device address (nothing is
// allocated then, and the solver kernel is not timed).
template <typename VT>
static int solve_typed(const bspai_csr *A, const bspai_handle *Ab, const double *b, const bspai_handle *M,
                       const gmres_ir_tol *tol, double *x, gmres_ir_stats *st_host, hipStream_t s,
                       char *ext_base = nullptr, size_t ext_cap = 0, const char *who = "gmres_ir_solve") {
  const int n = A->n;
  const int64_t nnz = A->nnz;
  int m = std::min(std::max(tol->gmres_max, 1), std::min(n, kMaxGmres));
  // about two rows per thread: each MGS pass is bound by the latency of
  // loading a basis slice and exchanging a partial, not by bandwidth, and more
  // blocks make every exchange wait for more partials (measured on MI355X at
  // n = 65,536: 32 blocks 10.5, 64 blocks 13.0, 128 blocks 11.3 solves/s).
  // CGS2 has five exchanges per iteration whatever j is, and its basis
  // sweeps gain from more compute units: about one row per thread (64 blocks
  // 18.8, 128 blocks 21.6 solves/s)
  const int rpt = tol->orth ? 1 : 2;
  int G = std::min(kMaxBlocks, std::max(1, (n + rpt * kSolveThreads - 1) / (rpt * kSolveThreads)));
  if (const char *e = getenv("BSPAI_SOLVE_BLOCKS")) G = std::min(kMaxBlocks, std::max(1, atoi(e)));
  int rpb = rows_for(n, G);
  int zr = (rpb + kSolveThreads - 1) / kSolveThreads;
  while (zr > 16 && G < kMaxBlocks) {
    G = std::min(kMaxBlocks, G * 2);
    rpb = rows_for(n, G);
    zr = (rpb + kSolveThreads - 1) / kSolveThreads;
  }
  if (zr > 16) return fail(BSPAI_EINVAL, "%s: n = %d exceeds %d rows", who, n, kMaxBlocks * kSolveThreads * 16);
  int ZR = 1;
  while (ZR < zr) ZR <<= 1;
  G = (n + rpb - 1) / rpb;
  if (G < 1) G = 1;

  const SysLayout L = sys_layout<VT>(n, nnz, m, tol->trans != 0, tol->orth != 0);
  std::unique_lock<std::mutex> lock(g_ws.mu, std::defer_lock);
  char *base = ext_base;
  if (ext_base) {
    if (L.total > ext_cap)
      return fail(BSPAI_EINVAL, "%s: n = %d, nnz = %lld, gmres_max %d need %zu bytes of workspace; the limit is %zu",
                  who, n, (long long)nnz, m, L.total, ext_cap);
  } else {
    lock.lock();
    int dev = 0;
    BSPAI_HIP(hipGetDevice(&dev));
    if (g_ws.bytes < L.total || g_ws.device != dev) {
      if (g_ws.ptr) {
        (void)hipDeviceSynchronize();
        dfree(g_ws.ptr);
        g_ws.ptr = nullptr;
        g_ws.bytes = 0;
      }
      int rc = dalloc(&g_ws.ptr, L.total);
      if (rc) return rc;
      g_ws.bytes = L.total;
      g_ws.device = dev;
    }
    base = static_cast<char *>(g_ws.ptr);
  }
  const bool prof = g_profile && !ext_base;
  SolveParams<VT> p;
  bool wide = false;
  int rc = sys_setup<VT>(A, Ab, b, M, tol, x, m, G, rpb, base, L, p, wide, s);
  if (rc) return rc;
  BSPAI_HIP(hipMemsetAsync(p.grid.flags, 0, 4 * kMaxBlocks, s));
  BSPAI_HIP(hipMemsetAsync(p.grid.abortf, 0, 4, s));
  // tags restart at 1 every launch: clear the exchange words of the last one
  BSPAI_HIP(hipMemsetAsync(p.grid.slots, 0, kSlotBytes, s));
  if (p.grid.wide) BSPAI_HIP(hipMemsetAsync(p.grid.wide, 0, wide_bytes(p.grid.G), s));
  BSPAI_HIP(hipMemsetAsync(p.stats, 0, sizeof(gmres_ir_stats), s));
  const size_t lds = solve_lds(m);
  void *fn = pick_single<VT>(wide, ZR, tol->orth != 0);
  BSPAI_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  SolveParams<VT> *pdev = reinterpret_cast<SolveParams<VT> *>(base + L.params);
  BSPAI_HIP(hipMemcpyAsync(pdev, &p, sizeof(p), hipMemcpyHostToDevice, s));
  void *args[] = {&pdev};
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (prof) {
    BSPAI_HIP(hipEventCreate(&ev[0]));
    BSPAI_HIP(hipEventCreate(&ev[1]));
    BSPAI_HIP(hipEventRecord(ev[0], s));
  }
  BSPAI_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(kSolveThreads), args, (unsigned)lds, s));
  if (prof) BSPAI_HIP(hipEventRecord(ev[1], s));
  gmres_ir_stats hs;
  unsigned aborted = 0;
  BSPAI_HIP(hipMemcpyAsync(&hs, p.stats, sizeof(hs), hipMemcpyDeviceToHost, s));
  BSPAI_HIP(hipMemcpyAsync(&aborted, p.grid.abortf, 4, hipMemcpyDeviceToHost, s));
  BSPAI_HIP(hipStreamSynchronize(s));
  if (prof) {
    float ms = 0.f;
    BSPAI_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    g_last_ms = ms;
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
  }
  if (aborted) return fail(BSPAI_EHIP, "%s: grid synchronisation timed out", who);
  if (st_host) *st_host = hs;
  if (hs.status == BSPAI_ENOCONV)
    return fail(BSPAI_ENOCONV, "%s: %d refinement steps without meeting a tolerance", who, hs.steps);
  if (hs.status == BSPAI_ENAN) return fail(BSPAI_ENAN, "%s: NaN or infinity in the residual", who);
  if (hs.status == BSPAI_ESTAG)
    return fail(BSPAI_ESTAG, "%s: corrections stagnated after %d steps before meeting a tolerance "
                             "(relres %.3e, eta %.3e)", who, hs.steps, hs.relres[hs.steps < 64 ? hs.steps : 64],
                hs.eta[hs.steps < 64 ? hs.steps : 64]);
  return hs.status;
}

// ------------------------------------------------------------------ many systems

// Several independent systems in one persistent launch.  The systems fall
// into classes by the group size that solves them; the grid is cut into
// groups of those sizes, each group belonging to one class.  A group takes
// the next system of its class off that class's device queue (largest
// first), solves it with the single-system body on its own barrier and
// exchange words, and goes back to the queue until it is empty.  Results do
// not depend on which group solves a system: all groups of a class have the
// same size, so the row split and the reduction order of a system are fixed
// by the plan.
template <typename VT>
struct MultiParams {
  const SolveParams<VT> *sys;  // [nsys]
  const int *order;            // systems by class, each class largest first
  const int *class_off;        // [nclass + 1]: class c owns order[class_off[c] .. class_off[c + 1])
  const Grid *grids;           // [ngroups]
  const int *group_class;      // [ngroups]
  const int *block_group;      // [grid size]: group of each block
  const int *block_local;      // [grid size]: index of the block within its group
  unsigned *queues;            // [nclass]: next queue position per class (cleared per launch)
  unsigned *groups_done;       // groups that have left their queue (cleared per launch)
  const unsigned *seq;         // launches so far (advanced by the clear kernel)
  unsigned *done_host;         // host word: seq of the last launch that has finished
  int ngroups;
};

template <typename VT, typename PT, int ZR, bool CGS2>
__global__ void __launch_bounds__(kSolveThreads) k_gmres_multi(const MultiParams<VT> *__restrict__ mp) {
  extern __shared__ double sm[];
  __shared__ double sh[kWaves * kMaxSlotWidth + kMaxSlotWidth + 1];
  __shared__ int s_flag;
  const int group = mp->block_group[blockIdx.x], bid = mp->block_local[blockIdx.x];
  const int cls = mp->group_class[group];
  const int first = mp->class_off[cls], count = mp->class_off[cls + 1] - first;
  const Grid G = mp->grids[group];
  unsigned epoch = 0, rtag = 0;
  for (;;) {
    // the group's first block takes a queue position; the all-reduction (max
    // of it and zeros) hands it to every block of the group
    double q[1] = {0.0};
    if (bid == 0 && threadIdx.x == 0) q[0] = (double)atomicAdd(&mp->queues[cls], 1u);
    if (!grid_reduce<1, true>(G, rtag, q, sh, bid)) break;
    const int k = (int)q[0];
    if (k >= count) break;
    if (!gmres_ir_body<VT, PT, ZR, CGS2>(mp->sys[mp->order[first + k]], G, bid, epoch, rtag, sm, sh, s_flag))
      break;
  }
  if (bid == 0 && threadIdx.x == 0) {
    unsigned d = atomicAdd(mp->groups_done, 1u);
    if (d + 1 == (unsigned)mp->ngroups)
      __hip_atomic_store(mp->done_host, *mp->seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// zero the per-launch state (a kernel, not a memset node, so that graph
// replays clear it reliably) and advance the launch counter
__global__ void k_multi_clear(unsigned *words, int64_t nwords, unsigned *seq) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
    words[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *seq += 1u;
}

template <typename VT, bool CGS2>
static void *pick_multi_o(bool wide, int ZR) {
  if (wide) {
    switch (ZR) {
      case 1: return (void *)k_gmres_multi<VT, double, 1, CGS2>;
      case 2: return (void *)k_gmres_multi<VT, double, 2, CGS2>;
      case 4: return (void *)k_gmres_multi<VT, double, 4, CGS2>;
      case 8: return (void *)k_gmres_multi<VT, double, 8, CGS2>;
      default: return (void *)k_gmres_multi<VT, double, 16, CGS2>;
    }
  }
  switch (ZR) {
    case 1: return (void *)k_gmres_multi<VT, float, 1, CGS2>;
    case 2: return (void *)k_gmres_multi<VT, float, 2, CGS2>;
    case 4: return (void *)k_gmres_multi<VT, float, 4, CGS2>;
    case 8: return (void *)k_gmres_multi<VT, float, 8, CGS2>;
    default: return (void *)k_gmres_multi<VT, float, 16, CGS2>;
  }
}

template <typename VT>
static void *pick_multi(bool wide, int ZR, bool cgs2) {
  return cgs2 ? pick_multi_o<VT, true>(wide, ZR) : pick_multi_o<VT, false>(wide, ZR);
}

}  // namespace bspai

struct bspai_multi {
  int nsys = 0, ngroups = 0, group_blocks = 0, device = 0;
  void *mem = nullptr;             // every system's workspace, the parameters and the per-launch state
  unsigned *done_host = nullptr;   // pinned host word
  unsigned launches = 0;
  gmres_ir_stats *stats = nullptr; // [nsys], device
  unsigned *aborts = nullptr;      // [ngroups], device
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace bspai {

static void multi_release(bspai_multi *P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->mem) {
    (void)hipDeviceSynchronize();
    dfree(P->mem);
  }
  if (P->done_host) (void)hipHostFree(P->done_host);
  delete P;
}

// smallest power-of-two group that keeps n rows within 8 rows per thread
static int class_blocks(int n) {
  const int need = (n + 8 * kSolveThreads - 1) / (8 * kSolveThreads);
  int g = 1;
  while (g < need) g <<= 1;
  return std::min(g, kMaxBlocks);
}

// rough cost of one exchange by a group of g blocks (microseconds, measured
// on MI355X: 1.3 for one block ... 2.5 for 48); only ratios matter
static double exchange_cost(int g) { return 1.3 + 0.25 * std::log2((double)std::max(g, 1)); }

template <typename VT>
static int multi_plan_typed(const bspai_system *sys, int nsys, const gmres_ir_tol *tol, int group_blocks,
                            int max_groups, bspai_multi **out, hipStream_t s) {
  const bool tr = tol->trans != 0;
  int nmax = 0;
  for (int k = 0; k < nsys; k++) nmax = std::max(nmax, sys[k].A.n);
  // smallest group that keeps every system within 16 rows per thread
  const int gmin = (nmax + kSolveThreads * 16 - 1) / (kSolveThreads * 16);
  if (group_blocks > 0 && (group_blocks < gmin || group_blocks > kMaxBlocks))
    return fail(BSPAI_EINVAL, "bspai_multi_plan: group_blocks must be in %d..%d for n up to %d", gmin, kMaxBlocks,
                nmax);
  if (nmax > kMaxBlocks * kSolveThreads * 16)
    return fail(BSPAI_EINVAL, "bspai_multi_plan: n = %d exceeds %d rows", nmax, kMaxBlocks * kSolveThreads * 16);
  // group size of each system: one size for all (group_blocks > 0) or its class
  std::vector<int> gs(nsys);
  for (int k = 0; k < nsys; k++)
    gs[k] = group_blocks > 0 ? group_blocks : class_blocks(sys[k].A.n);
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  BSPAI_HIP(hipGetDevice(&dev));
  BSPAI_HIP(hipGetDeviceProperties(&prop, dev));
  // kernel variant and residency (needs the row split: settle the classes first)
  auto classes_of = [&](std::vector<int> &sizes) {
    std::vector<int> c(sizes);
    std::sort(c.begin(), c.end(), std::greater<int>());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    return c;
  };
  std::vector<int> csize = classes_of(gs);
  int ZR = 1, mmax = 1;
  bool wide = sizeof(VT) == 8;
  void *fn = nullptr;
  size_t lds = 0;
  int resident = 0;
  auto settle_kernel = [&]() -> int {
    ZR = 1, mmax = 1;
    for (int k = 0; k < nsys; k++) {
      const int n = sys[k].A.n;
      mmax = std::max(mmax, std::min(std::max(tol->gmres_max, 1), std::min(n, kMaxGmres)));
      while (ZR * kSolveThreads < rows_for(n, gs[k])) ZR <<= 1;
      const BMat &Mb = tr ? sys[k].M->matT : sys[k].M->mat;
      for (int q = 0; q < Mb.nb; q++) wide = wide || Mb.prec[q] == BSPAI_FP64;
    }
    lds = solve_lds(mmax);
    fn = pick_multi<VT>(wide, ZR, tol->orth != 0);
    BSPAI_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    BSPAI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSolveThreads, lds));
    // every block of the grid must be resident at once (a group waits on its blocks)
    resident = per_cu * prop.multiProcessorCount;
    return BSPAI_OK;
  };
  int rc = settle_kernel();
  if (rc) return rc;
  // one group per class must fit (and no more classes than max_groups):
  // otherwise the smallest class joins the next larger one
  auto fits = [&]() {
    int need = 0;
    for (int g : csize) need += g;
    return need <= resident && (max_groups <= 0 || (int)csize.size() <= max_groups);
  };
  while (!fits() && csize.size() > 1) {
    const int small = csize.back(), next = csize[csize.size() - 2];
    for (int &g : gs)
      if (g == small) g = next;
    csize.pop_back();
  }
  if (!fits())
    return fail(BSPAI_EINVAL, "bspai_multi_plan: a group of %d blocks does not fit on the device (%d resident)",
                csize[0], resident);
  if ((rc = settle_kernel())) return rc;  // the row split may have changed
  const int nclass = (int)csize.size();
  std::vector<int> cls(nsys), ccount(nclass, 0);
  std::vector<double> cload(nclass, 0.0);
  for (int k = 0; k < nsys; k++) {
    cls[k] = (int)(std::find(csize.begin(), csize.end(), gs[k]) - csize.begin());
    ccount[cls[k]]++;
    // a system's cost: iterations grow about like the grid side, each costs
    // a few exchanges of its group
    cload[cls[k]] += std::sqrt((double)sys[k].A.n) * exchange_cost(gs[k]);
  }
  // groups per class: start with one each, then give groups to the class
  // with the largest load per group while blocks remain
  std::vector<int> kc(nclass, 1);
  int blocks = 0, ngroups = nclass;
  for (int c = 0; c < nclass; c++) blocks += csize[c];
  for (;;) {
    int best = -1;
    double bl = 0.0;
    for (int c = 0; c < nclass; c++) {
      if (kc[c] >= ccount[c] || blocks + csize[c] > resident) continue;
      if (max_groups > 0 && ngroups >= max_groups) continue;
      const double l = cload[c] / kc[c];
      if (best < 0 || l > bl) best = c, bl = l;
    }
    if (best < 0) break;
    kc[best]++, ngroups++, blocks += csize[best];
  }
  // systems by class, largest first within a class
  std::vector<int> order(nsys), coff(nclass + 1, 0);
  for (int k = 0; k < nsys; k++) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (cls[a] != cls[b]) return cls[a] < cls[b];
    return sys[a].A.n > sys[b].A.n;
  });
  for (int c = 0; c < nclass; c++) coff[c + 1] = coff[c] + ccount[c];
  std::vector<int> gclass(ngroups), bgroup(blocks), blocal(blocks), gfirst(ngroups);
  for (int c = 0, gi = 0, fb = 0; c < nclass; c++) {
    for (int i = 0; i < kc[c]; i++, gi++) {
      gclass[gi] = c;
      gfirst[gi] = fb;
      for (int t = 0; t < csize[c]; t++, fb++) bgroup[fb] = gi, blocal[fb] = t;
    }
  }

  // memory: per-system workspaces, parameters, maps, then the per-launch state
  std::vector<SysLayout> L(nsys);
  std::vector<size_t> base(nsys);
  size_t off = 0;
  for (int k = 0; k < nsys; k++) {
    L[k] = sys_layout<VT>(sys[k].A.n, sys[k].A.nnz, std::min(std::max(tol->gmres_max, 1), std::min(sys[k].A.n, kMaxGmres)), tr);
    base[k] = off;
    off += L[k].total;
  }
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t o_params = take(sizeof(SolveParams<VT>) * nsys);
  const size_t o_order = take(4 * (size_t)nsys);
  const size_t o_coff = take(4 * (size_t)(nclass + 1));
  const size_t o_grids = take(sizeof(Grid) * ngroups);
  const size_t o_gclass = take(4 * (size_t)ngroups);
  const size_t o_bgroup = take(4 * (size_t)blocks);
  const size_t o_blocal = take(4 * (size_t)blocks);
  const size_t o_mp = take(sizeof(MultiParams<VT>));
  const size_t o_seq = take(4);
  // per-launch state, cleared by k_multi_clear: queues and the group counter,
  // aborts, stats, flags, exchange words
  const size_t o_state = off;
  const size_t o_queues = take(4 * (size_t)(nclass + 1));
  const size_t o_aborts = take(4 * (size_t)ngroups);
  const size_t o_stats = take(sizeof(gmres_ir_stats) * nsys);
  const size_t o_flags = take(4 * (size_t)kMaxBlocks * ngroups);
  const size_t o_slots = take(kSlotBytes * ngroups);
  size_t wide_total = 0;
  if (tol->orth)
    for (int g = 0; g < ngroups; g++) wide_total += wide_bytes(csize[gclass[g]]);
  const size_t o_wide = take(wide_total);
  const size_t state_bytes = off - o_state;

  bspai_multi *P = new bspai_multi;
  P->nsys = nsys;
  P->ngroups = ngroups;
  P->group_blocks = nclass == 1 ? csize[0] : 0;
  P->device = dev;
  rc = dalloc(&P->mem, off);
  if (rc) {
    multi_release(P);
    return rc;
  }
  char *mem = static_cast<char *>(P->mem);
  auto bail = [&](int code) {
    multi_release(P);
    return code;
  };
  if (hipHostMalloc((void **)&P->done_host, 4, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
    return bail(fail(BSPAI_EHIP, "bspai_multi_plan: hipHostMalloc failed"));
  *P->done_host = 0u;
  unsigned *done_dev = nullptr;
  if (hipHostGetDevicePointer((void **)&done_dev, P->done_host, 0) != hipSuccess)
    return bail(fail(BSPAI_EHIP, "bspai_multi_plan: hipHostGetDevicePointer failed"));

  std::vector<SolveParams<VT>> ps(nsys);
  gmres_ir_stats *stats = reinterpret_cast<gmres_ir_stats *>(mem + o_stats);
  for (int k = 0; k < nsys; k++) {
    bool w = false;
    const int m = std::min(std::max(tol->gmres_max, 1), std::min(sys[k].A.n, kMaxGmres));
    rc = sys_setup<VT>(&sys[k].A, nullptr, sys[k].b, sys[k].M, tol, sys[k].x, m, gs[k], rows_for(sys[k].A.n, gs[k]),
                       mem + base[k], L[k], ps[k], w, s);
    if (rc) return bail(rc);
    ps[k].stats = stats + k;
  }
  std::vector<Grid> grids(ngroups);
  unsigned *aborts = reinterpret_cast<unsigned *>(mem + o_aborts);
  size_t wide_off = o_wide;
  for (int g = 0; g < ngroups; g++) {
    grids[g].flags = reinterpret_cast<unsigned *>(mem + o_flags) + (size_t)kMaxBlocks * g;
    grids[g].abortf = aborts + g;
    grids[g].slots = reinterpret_cast<double *>(mem + o_slots + kSlotBytes * g);
    grids[g].G = csize[gclass[g]];
    grids[g].wide = nullptr;  // vector-reduction words: CGS2 only
    if (tol->orth) {
      grids[g].wide = reinterpret_cast<unsigned long long *>(mem + wide_off);
      wide_off += wide_bytes(grids[g].G);
    }
  }
  MultiParams<VT> mp;
  memset(&mp, 0, sizeof(mp));
  mp.sys = reinterpret_cast<const SolveParams<VT> *>(mem + o_params);
  mp.order = reinterpret_cast<const int *>(mem + o_order);
  mp.class_off = reinterpret_cast<const int *>(mem + o_coff);
  mp.grids = reinterpret_cast<const Grid *>(mem + o_grids);
  mp.group_class = reinterpret_cast<const int *>(mem + o_gclass);
  mp.block_group = reinterpret_cast<const int *>(mem + o_bgroup);
  mp.block_local = reinterpret_cast<const int *>(mem + o_blocal);
  mp.queues = reinterpret_cast<unsigned *>(mem + o_queues);
  mp.groups_done = mp.queues + nclass;
  mp.seq = reinterpret_cast<const unsigned *>(mem + o_seq);
  mp.done_host = done_dev;
  mp.ngroups = ngroups;
  // pageable host copies: synchronise before the vectors go out of scope
  if (hipMemcpyAsync(mem + o_params, ps.data(), sizeof(SolveParams<VT>) * nsys, hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(mem + o_order, order.data(), 4 * (size_t)nsys, hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(mem + o_coff, coff.data(), 4 * (size_t)(nclass + 1), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(mem + o_grids, grids.data(), sizeof(Grid) * ngroups, hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(mem + o_gclass, gclass.data(), 4 * (size_t)ngroups, hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(mem + o_bgroup, bgroup.data(), 4 * (size_t)blocks, hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(mem + o_blocal, blocal.data(), 4 * (size_t)blocks, hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(mem + o_mp, &mp, sizeof(mp), hipMemcpyHostToDevice, s) ||
      hipMemsetAsync(mem + o_seq, 0, 4, s) || hipStreamSynchronize(s))
    return bail(fail(BSPAI_EHIP, "bspai_multi_plan: setting up the parameters failed"));
  P->stats = stats;
  P->aborts = aborts;
  const int gb = blocks;  // grid size of the launch

  // capture clear + solve into a graph on a private stream
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(BSPAI_EHIP, "bspai_multi_plan: stream creation failed"));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const int64_t nwords = (int64_t)(state_bytes / 4);
    hipLaunchKernelGGL(k_multi_clear, dim3(256), dim3(256), 0, cs, reinterpret_cast<unsigned *>(mem + o_state),
                       nwords, reinterpret_cast<unsigned *>(mem + o_seq));
    const MultiParams<VT> *mpd = reinterpret_cast<const MultiParams<VT> *>(mem + o_mp);
    void *args[] = {&mpd};
    hipError_t el = hipLaunchKernel(fn, dim3(gb), dim3(kSolveThreads), args, lds, cs);
    hipError_t ee = hipStreamEndCapture(cs, &P->graph);
    e = el != hipSuccess ? el : ee;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return bail(fail(BSPAI_EHIP, "bspai_multi_plan: graph capture failed: %s", hipGetErrorString(e)));
  *out = P;
  return BSPAI_OK;
}

// ------------------------------------------------- batched MGS, one launch
// One Arnoldi step's modified Gram-Schmidt for the C columns of an n x C
// row-major block of u_g values (16 bytes per row: C = 4 in FP32, 2 in FP64)
// as one cooperative kernel (used by the many-right-hand-side solve, which
// runs its columns in such groups).  Grid thread t owns rows t, t + T, ...
// (RPT of them, T threads in the grid).  Its slice of z stays in registers
// across the j + 2 passes and its slice of v_{i-1} is kept from the pass
// before, so each basis vector is read once per step.  Pass i <= j subtracts
// h_{i-1} v_{i-1} from z (i > 0) and forms the dots with v_i, pass j + 1
// subtracts h_j v_j and forms ||z||^2; every pass is one grid-wide
// all-reduction of the C column sums.  Then v_{j+1} = z / ||z|| (0 where
// ||z|| = 0).  The arithmetic is that of the per-pass kernels (each update
// one FMA rounded to u_g, products summed in FP64), reduced in a fixed order:
// per thread over its rows, DPP wave sums, waves in order, blocks in order.
constexpr int kMgsCols = 4;  // column sums per exchange (FP32: 4, FP64: 2 used)

struct MgsGrid {
  // [kNumSlots][kMaxBlocks][kMgsCols][2] tagged words, cleared once per solve:
  // each block's words share one 64-byte line, written by one instruction
  // (column-major slots, whose polls coalesce, measured 4% slower per pass:
  // four blocks then write into every line)
  unsigned long long *slots;
  unsigned *abortf;
};

template <typename VT>
struct BMgsParams {
  int n, j, m;
  const VT *z;       // n x C: M_b (A v_j) (or A (M_b v_j)) on entry
  VT *V;             // v_i at V + i * vstride; v_{j+1} is written
  int64_t vstride;
  double *H;         // h_{i,j} of column c at H + (c * m + j) * (m + 1) + i, i <= j + 1
  double *hn;        // [C]: h_{j+1,j}
  const int *gma;    // [C] GMRES-active flags, or null: with none set the launch does nothing
  unsigned rtag0;    // exchange rounds before this launch (its first round is rtag0 + 1)
  MgsGrid grid;
};

template <typename VT>
struct Row16;
template <>
struct Row16<float> {
  __device__ static void load(const float *p, float (&v)[4]) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
  }
  __device__ static void store(float *p, const float (&v)[4]) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
  __device__ static void unpack(const unsigned (&u)[4], float (&v)[4]) {
    for (int c = 0; c < 4; c++) v[c] = __uint_as_float(u[c]);
  }
  __device__ static void pack(const float (&v)[4], unsigned (&u)[4]) {
    for (int c = 0; c < 4; c++) u[c] = __float_as_uint(v[c]);
  }
};
template <>
struct Row16<double> {
  __device__ static void load(const double *p, double (&v)[2]) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    v[0] = a.x, v[1] = a.y;
  }
  __device__ static void store(double *p, const double (&v)[2]) {
    *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
  }
  __device__ static void unpack(const unsigned (&u)[4], double (&v)[2]) {
    for (int c = 0; c < 2; c++)
      v[c] = __longlong_as_double((long long)(((unsigned long long)u[2 * c + 1] << 32) | u[2 * c]));
  }
  __device__ static void pack(const double (&v)[2], unsigned (&u)[4]) {
    for (int c = 0; c < 2; c++) {
      const unsigned long long b = (unsigned long long)__double_as_longlong(v[c]);
      u[2 * c] = (unsigned)b, u[2 * c + 1] = (unsigned)(b >> 32);
    }
  }
};

// A buffer resource over `bytes` bytes at p (raw: no stride, no swizzle):
// loads through it take a uniform row offset in an SGPR and the thread's
// offset in one VGPR, instead of a 64-bit address per row.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const void *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename VT, int C>
__device__ __forceinline__ void load_row16(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, VT (&o)[C]) {
  const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
  const unsigned u[4] = {w[0], w[1], w[2], w[3]};
  Row16<VT>::unpack(u, o);
}

template <typename VT, int C>
__device__ __forceinline__ void store_row16(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const VT (&v)[C]) {
  unsigned u[4];
  Row16<VT>::pack(v, u);
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 w = {u[0], u[1], u[2], u[3]};
  __builtin_amdgcn_raw_buffer_store_b128(w, rs, voff, soff, 0);
}

// Sum over the grid of the C column values `part` (per thread); every block
// obtains the same bits.  Two halves, so that a caller can issue independent
// loads while the other blocks' partials arrive: mgs_post publishes this
// block's sums, mgs_collect waits for all of them.  Wave c < C collects column
// c: lane l adds the partials of blocks l, l + 64, ... in that order, issuing
// all of its loads before checking any tag.
template <int C>
__device__ void mgs_post(const MgsGrid &g, unsigned &rtag, const double (&part)[C], double *wpart) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < C; c++) {
    const double w = wave_sum_dpp(part[c]);
    if (lane == 0) wpart[wv * C + c] = w;
  }
  lds_barrier();
  rtag++;
  unsigned long long *set = g.slots + (size_t)(rtag % kNumSlots) * kMaxBlocks * kMgsCols * 2;
  if (threadIdx.x < C) {
    double a = wpart[threadIdx.x];
    for (int k = 1; k < kWaves; k++) a += wpart[k * C + threadIdx.x];
    publish_partial(set + ((size_t)blockIdx.x * kMgsCols + threadIdx.x) * 2, a, rtag);
  }
}

// Returns false (and raises the abort flag) when a wait exceeds the bound or
// a block aborted; otherwise part holds the grid sums.
template <int C>
__device__ bool mgs_collect(const MgsGrid &g, unsigned rtag, double (&part)[C], double *res) {
  constexpr int K = kMaxBlocks / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, G = gridDim.x;
  const unsigned long long tg = tag16(rtag);
  const unsigned long long *set = g.slots + (size_t)(rtag % kNumSlots) * kMaxBlocks * kMgsCols * 2;
  int bad = 0;
  if (wv < C) {
    unsigned long long a[K], b[K];
    unsigned spins = 0;
    for (;;) {
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int blk = lane + 64 * k;
        if (blk < G) {
          const unsigned long long *w = set + ((size_t)blk * kMgsCols + wv) * 2;
          a[k] = __hip_atomic_load(&w[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          b[k] = __hip_atomic_load(&w[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      bool ok = true;
#pragma unroll
      for (int k = 0; k < K; k++)
        if (lane + 64 * k < G) ok = ok && (a[k] & 0xFFFFull) == tg && (b[k] & 0xFFFFull) == tg;
      if (ok) break;
      if (++spins > kSpinLimit || __hip_atomic_load(g.abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        bad = 1;
        break;
      }
    }
    double s = 0.0;
    if (!bad) {
#pragma unroll
      for (int k = 0; k < K; k++)
        if (lane + 64 * k < G) s += __longlong_as_double((long long)((a[k] & ~0xFFFFull) | ((b[k] >> 16) & 0xFFFFull)));
    }
    s = wave_sum_dpp(s);
    const bool any_bad = __any(bad);
    if (lane == 0) {
      res[wv] = s;
      res[C + wv] = any_bad ? 1.0 : 0.0;
    }
  }
  lds_barrier();
  bool fail_any = false;
#pragma unroll
  for (int c = 0; c < C; c++) fail_any = fail_any || res[C + c] != 0.0;
  if (fail_any) {
    if (threadIdx.x == 0) __hip_atomic_store(g.abortf, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
#pragma unroll
  for (int c = 0; c < C; c++) part[c] = res[c];
  return true;
}

// ZL: z lives in LDS (8 or more rows per thread: z and two basis slices would
// not all fit in registers); each thread touches only its own 16-byte entries.
//
// Pass i (0 <= i <= j + 1) of the step: z -= h_{i-1,j} v_{i-1} (i > 0), then
// the grid sum of v_i . z (i <= j) or of z . z (i = j + 1), one row at a time
// in that order.  The basis slices alternate between two register sets: while
// pass i's sums travel between the blocks, v_{i+1} is already being loaded
// into the set that held v_{i-1}.
template <typename VT, int RPT, bool ZL>
__global__ void __launch_bounds__(kSolveThreads) k_b_mgs_persist(BMgsParams<VT> p) {
  constexpr int C = 16 / (int)sizeof(VT);
  extern __shared__ double zdyn[];  // ZL: [RPT][kSolveThreads] rows of 16 bytes
  // per-wave partials, then the column sums and abort votes; two halves so
  // that one exchange's results are never overwritten by the next one's
  // partials while slower waves still read them
  __shared__ double wpart[2][kWaves * C];
  __shared__ double res[2][2 * C];
  // rows t0 + r T, 16 bytes each (byte offsets fit 32 bits: n <= 2^21).
  // Every access goes through a buffer resource of n rows, whose range check
  // (on the thread offset plus the uniform row offset) reads rows past n - 1
  // as zero and drops stores to them: no load or store sits behind a branch,
  // so the wait counts stay exact and loads issued early stay in flight.
  const unsigned T = gridDim.x * kSolveThreads;
  const unsigned t0 = blockIdx.x * kSolveThreads + threadIdx.x;
  const int n = p.n, j = p.j;
  const unsigned b0 = t0 * 16u, bs = T * 16u, nbytes = (unsigned)n * 16u;
  auto load_rows = [&](const VT *base, VT (&dst)[RPT][C]) {
    const __amdgpu_buffer_rsrc_t rs = rows_rsrc(base, nbytes);
#pragma unroll
    for (int r = 0; r < RPT; r++) load_row16<VT, C>(rs, b0, (unsigned)r * bs, dst[r]);
  };
  VT va[RPT][C], vb[RPT][C];
  VT zreg[ZL ? 1 : RPT][C];
  VT *zl = reinterpret_cast<VT *>(zdyn) + threadIdx.x * C;
  auto zget = [&](int r, VT (&o)[C]) {
    if constexpr (ZL) {
      Row16<VT>::load(zl + r * kSolveThreads * C, o);
    } else {
#pragma unroll
      for (int c = 0; c < C; c++) o[c] = zreg[r][c];
    }
  };
  auto zput = [&](int r, const VT (&o)[C]) {
    if constexpr (ZL) {
      Row16<VT>::store(zl + r * kSolveThreads * C, o);
    } else {
#pragma unroll
      for (int c = 0; c < C; c++) zreg[r][c] = o[c];
    }
  };
  // z enters through the first register set while v_0 loads into the second
  load_rows(p.z, va);
  load_rows(p.V, vb);
  if (p.gma) {  // a step queued after every column stopped: nothing to do
    int any = 0;
#pragma unroll
    for (int c = 0; c < C; c++) any |= p.gma[c];
    if (!any) return;
  }
#pragma unroll
  for (int r = 0; r < RPT; r++) zput(r, va[r]);
  unsigned rtag = p.rtag0;
  double h[C];
#pragma unroll
  for (int c = 0; c < C; c++) h[c] = 0.0;
  // one pass; vp holds v_{i-1} (refilled with v_{i+1}), vc holds v_i.  The
  // first pass (no update) is a separate instance.  Each row of v_{i+1} is
  // requested as soon as the row of v_{i-1} in its registers has been used,
  // so the loads run under this pass's arithmetic and exchange (the last two
  // passes have no v_{i+1}: an empty resource, whose loads return zero
  // without touching memory).
  auto pass = [&](auto first, int i2, VT (&vp)[RPT][C], const VT (&vc)[RPT][C]) -> bool {
    const bool pre = i2 + 1 <= j;
    const __amdgpu_buffer_rsrc_t rs = rows_rsrc(p.V + (int64_t)(pre ? i2 + 1 : 0) * p.vstride, pre ? nbytes : 0u);
    double part[C];
#pragma unroll
    for (int c = 0; c < C; c++) part[c] = 0.0;
#pragma unroll
    for (int r = 0; r < RPT; r++) {
      VT zr[C];
      zget(r, zr);
      if constexpr (!decltype(first)::value) {
#pragma unroll
        for (int c = 0; c < C; c++) zr[c] = (VT)fma(-h[c], (double)vp[r][c], (double)zr[c]);
        zput(r, zr);
      }
      load_row16<VT, C>(rs, b0, (unsigned)r * bs, vp[r]);
#pragma unroll
      for (int c = 0; c < C; c++) {
        const double w = i2 <= j ? (double)vc[r][c] : (double)zr[c];
        part[c] = fma(w, (double)zr[c], part[c]);
      }
    }
    mgs_post<C>(p.grid, rtag, part, wpart[i2 & 1]);
    if (!mgs_collect<C>(p.grid, rtag, part, res[i2 & 1])) return false;
    if (i2 <= j) {
#pragma unroll
      for (int c = 0; c < C; c++) h[c] = part[c];
      if (blockIdx.x == 0 && threadIdx.x < C) p.H[((int64_t)threadIdx.x * p.m + j) * (p.m + 1) + i2] = part[threadIdx.x];
    } else {
      double hn[C];
#pragma unroll
      for (int c = 0; c < C; c++) hn[c] = sqrt(part[c]);
      if (blockIdx.x == 0 && threadIdx.x < C) {
        p.H[((int64_t)threadIdx.x * p.m + j) * (p.m + 1) + j + 1] = hn[threadIdx.x];
        p.hn[threadIdx.x] = hn[threadIdx.x];
      }
      const __amdgpu_buffer_rsrc_t rs = rows_rsrc(p.V + (int64_t)(j + 1) * p.vstride, nbytes);
#pragma unroll
      for (int r = 0; r < RPT; r++) {
        VT zr[C], o[C];
        zget(r, zr);
#pragma unroll
        for (int c = 0; c < C; c++) o[c] = hn[c] > 0.0 ? (VT)((double)zr[c] / hn[c]) : (VT)0;
        store_row16<VT, C>(rs, b0, (unsigned)r * bs, o);
      }
    }
    return true;
  };
  if (!pass(std::true_type{}, 0, va, vb)) return;
  for (int i2 = 1; i2 <= j + 1; i2 += 2) {
    if (!pass(std::false_type{}, i2, vb, va)) return;
    if (i2 + 1 <= j + 1 && !pass(std::false_type{}, i2 + 1, va, vb)) return;
  }
}

// rows per thread of the batched MGS kernel for n rows: the smallest power of
// two <= 16 with n <= kMaxBlocks * kSolveThreads * RPT (0: n too large)
int mgs_persist_rpt(int n) {
  for (int r = 1; r <= 16; r *= 2)
    if ((int64_t)n <= (int64_t)kMaxBlocks * kSolveThreads * r) return r;
  return 0;
}

size_t mgs_persist_ws_bytes() { return 16 * (size_t)kNumSlots * kMaxBlocks * kMgsCols; }

template <typename VT, int RPT>
static int launch_mgs_rpt(BMgsParams<VT> &p, int G, hipStream_t s) {
  constexpr bool ZL = RPT >= 8;
  const unsigned lds = ZL ? (unsigned)(RPT * kSolveThreads * 16) : 0u;
  void *fn = (void *)k_b_mgs_persist<VT, RPT, ZL>;
  // per device: the attribute set once, and whether G blocks are co-resident
  // (blocks per compute unit from the occupancy API times the units)
  static std::mutex mu;
  static int resident[16] = {0};  // 0 unknown, else blocks that fit + 1
  int dev = 0;
  BSPAI_HIP(hipGetDevice(&dev));
  int fit = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 16 && resident[dev]) {
      fit = resident[dev] - 1;
    } else {
      if (ZL) BSPAI_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      int per_cu = 0, cus = 0;
      BSPAI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSolveThreads, lds));
      BSPAI_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      fit = per_cu * cus;
      if (dev < 16) resident[dev] = fit + 1;
    }
  }
  void *args[] = {&p};
  // A plain launch when every block is resident at once (the exchanges'
  // waits are bounded: a grid that were not would end with the abort flag,
  // not hang): the cooperative launch measured 11 us of idle before and
  // 15 us after each MGS kernel, against a few for a plain one.
  if (G <= fit)
    BSPAI_HIP(hipLaunchKernel(fn, dim3(G), dim3(kSolveThreads), args, lds, s));
  else
    BSPAI_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(kSolveThreads), args, lds, s));
  return BSPAI_OK;
}

// One Arnoldi step's MGS (see k_b_mgs_persist) for the n x (16 / sizeof(VT))
// block z, basis V (v_i at V + i * vstride), H columns of step j; gma: the
// columns' GMRES-active flags (the launch returns at once when none is set),
// or null; ws: mgs_persist_ws_bytes() of device memory holding the exchange
// words, zeroed by the caller before the first launch on it; rtag0: the
// exchange rounds of all earlier launches on ws (j + 2 per launch), so that
// words left by them never carry a current tag; abortf: a zeroed word that a
// timed-out exchange sets.  Enqueued on s.
template <typename VT>
int launch_mgs_persist(int n, int j, int m, const VT *z, VT *V, int64_t vstride, double *H, double *hn,
                       const int *gma, void *ws, unsigned rtag0, unsigned *abortf, hipStream_t s) {
  const int rpt = mgs_persist_rpt(n);
  if (!rpt) return fail(BSPAI_EINVAL, "batched MGS: n = %d exceeds %d rows", n, kMaxBlocks * kSolveThreads * 16);
  const int G = (int)(((int64_t)n + (int64_t)kSolveThreads * rpt - 1) / ((int64_t)kSolveThreads * rpt));
  // layout check: every grid thread t owns rows t + r T, r < rpt - 1, below n
  // (the kernel's range-checked accesses would also cover rows past n)
  if ((int64_t)(rpt - 1) * G * kSolveThreads > n)
    return fail(BSPAI_EINVAL, "batched MGS: %d rows per thread on %d blocks overrun n = %d", rpt, G, n);
  BMgsParams<VT> p;
  p.n = n;
  p.j = j;
  p.m = m;
  p.z = z;
  p.V = V;
  p.vstride = vstride;
  p.H = H;
  p.hn = hn;
  p.gma = gma;
  p.rtag0 = rtag0;
  p.grid.slots = static_cast<unsigned long long *>(ws);
  p.grid.abortf = abortf;
  switch (rpt) {
    case 1: return launch_mgs_rpt<VT, 1>(p, G, s);
    case 2: return launch_mgs_rpt<VT, 2>(p, G, s);
    case 4: return launch_mgs_rpt<VT, 4>(p, G, s);
    case 8: return launch_mgs_rpt<VT, 8>(p, G, s);
    default: return launch_mgs_rpt<VT, 16>(p, G, s);
  }
}

template int launch_mgs_persist<float>(int, int, int, const float *, float *, int64_t, double *, double *,
                                       const int *, void *, unsigned, unsigned *, hipStream_t);
template int launch_mgs_persist<double>(int, int, int, const double *, double *, int64_t, double *, double *,
                                        const int *, void *, unsigned, unsigned *, hipStream_t);

}  // namespace bspai

using namespace bspai;

// Instrumentation: `iters` back-to-back all-reductions of one FP64 value by G
// blocks of the solver's size, with the solver's own grid_reduce.
__global__ void __launch_bounds__(kSolveThreads) k_exchange_probe(Grid g, int iters, double *out) {
  __shared__ double sh[kWaves * kMaxSlotWidth + kMaxSlotWidth + 1];
  unsigned rtag = 0;
  double acc = 0.0;
  for (int it = 0; it < iters; it++) {
    double v[1] = {(double)((threadIdx.x + it) & 7)};
    if (!grid_reduce<1, false>(g, rtag, v, sh, blockIdx.x)) return;
    acc += v[0];
  }
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// The same probe with the solver's LDS footprint (one block per compute
// unit) and placement: one_xcd = 0 launches G blocks (the dispatcher spreads
// them over the XCDs), one_xcd = 1 launches 8 G blocks and keeps the G that
// share one XCD.
__global__ void __launch_bounds__(kSolveThreads) k_exchange_probe_placed(Grid g, unsigned *reg, int one_xcd,
                                                                          int iters, double *out) {
  extern __shared__ double dyn[];
  __shared__ double sh[kWaves * kMaxSlotWidth + kMaxSlotWidth + 1];
  int bid = blockIdx.x;
  if (one_xcd) {
    bid = one_xcd_rank(reg, g.G, g.abortf);
    if (bid < 0) return;
  }
  if (threadIdx.x == 0) dyn[0] = 0.0;  // the dynamic LDS only sets the occupancy
  unsigned rtag = 0;
  double acc = 0.0;
  for (int it = 0; it < iters; it++) {
    double v[1] = {(double)((threadIdx.x + it) & 7)};
    if (!grid_reduce<1, false>(g, rtag, v, sh, bid)) return;
    acc += v[0];
  }
  if (threadIdx.x == 0) {
    out[bid] = acc;
    out[kMaxBlocks + bid] = (double)xcd_id();
  }
}

extern "C" int bspai_exchange_latency_placed(int G, int iters, int one_xcd, double *us_out, int *xcd_out,
                                             void *stream) {
  const int grid = one_xcd ? 8 * G : G;
  if (G < 1 || iters < 1 || !us_out || grid > kMaxBlocks)
    return fail(BSPAI_EINVAL, "bspai_exchange_latency_placed: need 1 <= G, iters >= 1 and %d blocks <= %d",
                grid, kMaxBlocks);
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *mem = nullptr;
  const size_t bytes = kSlotBytes + 256 + 256 + 16 * (size_t)kMaxBlocks;
  int rc = dalloc(&mem, bytes);
  if (rc) return rc;
  char *base = static_cast<char *>(mem);
  Grid g;
  g.slots = reinterpret_cast<double *>(base);
  g.wide = nullptr;
  g.abortf = reinterpret_cast<unsigned *>(base + kSlotBytes);
  g.flags = nullptr;
  g.G = G;
  unsigned *reg = reinterpret_cast<unsigned *>(base + kSlotBytes + 256);
  double *out = reinterpret_cast<double *>(base + kSlotBytes + 512);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto body = [&]() -> int {
    BSPAI_HIP(hipMemsetAsync(mem, 0, bytes, s));
    BSPAI_HIP(hipFuncSetAttribute((const void *)k_exchange_probe_placed, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kLdsBytes));
    BSPAI_HIP(hipEventCreate(&e0));
    BSPAI_HIP(hipEventCreate(&e1));
    void *args[] = {&g, &reg, &one_xcd, &iters, &out};
    BSPAI_HIP(hipEventRecord(e0, s));
    BSPAI_HIP(hipLaunchCooperativeKernel((void *)k_exchange_probe_placed, dim3(grid), dim3(kSolveThreads), args,
                                         (unsigned)kLdsBytes, s));
    BSPAI_HIP(hipEventRecord(e1, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    BSPAI_HIP(hipEventElapsedTime(&ms, e0, e1));
    unsigned ab = 0;
    BSPAI_HIP(hipMemcpy(&ab, g.abortf, 4, hipMemcpyDeviceToHost));
    if (ab) return fail(BSPAI_EHIP, "bspai_exchange_latency_placed: placement or an exchange failed");
    if (xcd_out) {
      std::vector<double> h(G);
      BSPAI_HIP(hipMemcpy(h.data(), out + kMaxBlocks, 8 * (size_t)G, hipMemcpyDeviceToHost));
      for (int k = 0; k < G; k++) xcd_out[k] = (int)h[k];
    }
    *us_out = ms * 1e3 / iters;
    return BSPAI_OK;
  };
  rc = body();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dfree(mem);
  return rc;
}

extern "C" int bspai_exchange_latency(int G, int iters, double *us_out, void *stream) {
  if (G < 1 || G > kMaxBlocks || iters < 1 || !us_out)
    return fail(BSPAI_EINVAL, "bspai_exchange_latency: need 1 <= G <= %d, iters >= 1", kMaxBlocks);
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *mem = nullptr;
  const size_t bytes = kSlotBytes + 256 + 8 * (size_t)kMaxBlocks;
  int rc = dalloc(&mem, bytes);
  if (rc) return rc;
  Grid g;
  g.slots = static_cast<double *>(mem);
  g.wide = nullptr;
  g.abortf = reinterpret_cast<unsigned *>(static_cast<char *>(mem) + kSlotBytes);
  g.flags = nullptr;
  g.G = G;
  double *out = reinterpret_cast<double *>(static_cast<char *>(mem) + kSlotBytes + 256);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto body = [&]() -> int {
    BSPAI_HIP(hipMemsetAsync(mem, 0, bytes, s));
    BSPAI_HIP(hipEventCreate(&e0));
    BSPAI_HIP(hipEventCreate(&e1));
    void *args[] = {&g, &iters, &out};
    BSPAI_HIP(hipEventRecord(e0, s));
    BSPAI_HIP(hipLaunchCooperativeKernel((void *)k_exchange_probe, dim3(G), dim3(kSolveThreads), args, 0, s));
    BSPAI_HIP(hipEventRecord(e1, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    BSPAI_HIP(hipEventElapsedTime(&ms, e0, e1));
    unsigned ab = 0;
    BSPAI_HIP(hipMemcpy(&ab, g.abortf, 4, hipMemcpyDeviceToHost));
    if (ab) return fail(BSPAI_EHIP, "bspai_exchange_latency: an exchange timed out");
    *us_out = ms * 1e3 / iters;
    return BSPAI_OK;
  };
  rc = body();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dfree(mem);
  return rc;
}

extern "C" int bspai_solve_blocks(int n) {
  if (n < 1) return fail(BSPAI_EINVAL, "bspai_solve_blocks: n < 1");
  int G = std::min(kMaxBlocks, std::max(1, (n + 2 * kSolveThreads - 1) / (2 * kSolveThreads)));
  if (const char *e = getenv("BSPAI_SOLVE_BLOCKS")) G = std::min(kMaxBlocks, std::max(1, atoi(e)));
  int rpb = rows_for(n, G);
  while ((rpb + kSolveThreads - 1) / kSolveThreads > 16 && G < kMaxBlocks) {
    G = std::min(kMaxBlocks, G * 2);
    rpb = rows_for(n, G);
  }
  return (n + rpb - 1) / rpb;
}

extern "C" void bspai_set_profiling(int on) { g_profile = on ? 1 : 0; }

static std::mutex g_mgs_mu;
static double g_mgs_ms = 0.0, g_mgs_bytes = 0.0;
static long long g_mgs_launches = 0, g_mgs_all = 0;
static int g_batch_mode = 0;
namespace bspai {
bool profiling_on() { return g_profile != 0; }
// One launch in kMgsProfEvery is timed: the two events around a launch delay
// the next dispatch by several microseconds each.  The counter runs across
// launches and solves, so with correction lengths prime to 7 the sample
// covers every step index j evenly.
constexpr unsigned kMgsProfEvery = 7;
static std::atomic<unsigned> g_mgs_seq{0};
bool mgs_profile_sample() {
  {
    std::lock_guard<std::mutex> lock(g_mgs_mu);
    g_mgs_all++;
  }
  return g_mgs_seq.fetch_add(1, std::memory_order_relaxed) % kMgsProfEvery == 0;
}
void add_mgs_profile(double ms, double bytes) {
  std::lock_guard<std::mutex> lock(g_mgs_mu);
  g_mgs_ms += ms;
  g_mgs_bytes += bytes;
  g_mgs_launches++;
}
int batch_mode() { return g_batch_mode; }
}  // namespace bspai

extern "C" void bspai_batched_mgs_profile(int reset, double *ms_total, long long *launches, double *bytes,
                                          long long *all_launches) {
  std::lock_guard<std::mutex> lock(g_mgs_mu);
  if (ms_total) *ms_total = g_mgs_ms;
  if (launches) *launches = g_mgs_launches;
  if (bytes) *bytes = g_mgs_bytes;
  if (all_launches) *all_launches = g_mgs_all;
  if (reset) {
    g_mgs_ms = g_mgs_bytes = 0.0;
    g_mgs_launches = g_mgs_all = 0;
  }
}

extern "C" int bspai_set_batch_mode(int mode) {
  if (mode < 0 || mode > 2) return fail(BSPAI_EINVAL, "bspai_set_batch_mode: mode must be 0, 1 or 2");
  g_batch_mode = mode;
  return BSPAI_OK;
}
extern "C" double bspai_last_solve_kernel_ms(void) { return g_last_ms; }

static int check_system(const bspai_csr *A, const double *b, const bspai_handle *M, const gmres_ir_tol *tol,
                        const double *x, const char *who) {
  if (!A || !M || !tol) return fail(BSPAI_EINVAL, "%s: null argument", who);
  if (A->n != M->n) return fail(BSPAI_EINVAL, "%s: A is %d x %d but M is %d x %d", who, A->n, A->n, M->n, M->n);
  if (A->n < 1) return fail(BSPAI_EINVAL, "%s: empty system", who);
  if (!A->row_ptr || (A->nnz > 0 && (!A->col || !A->val)) || !b || !x)
    return fail(BSPAI_EINVAL, "%s: null device pointer", who);
  if (tol->u_g != BSPAI_FP32 && tol->u_g != BSPAI_FP64) return fail(BSPAI_EINVAL, "%s: u_g must be FP32 or FP64", who);
  if (tol->x0_mode < 0 || tol->x0_mode > 3) return fail(BSPAI_EINVAL, "%s: x0_mode must be 0..3", who);
  if (tol->i_max < 0) return fail(BSPAI_EINVAL, "%s: i_max < 0", who);
  if (tol->orth != 0 && tol->orth != 1) return fail(BSPAI_EINVAL, "%s: orth must be 0 (MGS) or 1 (CGS2)", who);
  if (tol->trans && !M->has_T) return fail(BSPAI_EINVAL, "%s: trans needs a handle built with build_T", who);
  if (tol->x0_mode == 0 && !M->has_fp64) return fail(BSPAI_EINVAL, "%s: x0_mode 0 needs keep_fp64_M", who);
  int dev = 0;
  BSPAI_HIP(hipGetDevice(&dev));
  if (dev != M->device) return fail(BSPAI_EINVAL, "%s: handle lives on device %d", who, M->device);
  return BSPAI_OK;
}

extern "C" int bspai_multi_plan(const bspai_system *sys, int nsys, const gmres_ir_tol *tol, int group_blocks,
                                int max_groups, bspai_multi **plan_out, void *stream) {
  if (!plan_out) return fail(BSPAI_EINVAL, "bspai_multi_plan: null plan_out");
  *plan_out = nullptr;
  if (!sys || nsys < 1 || !tol) return fail(BSPAI_EINVAL, "bspai_multi_plan: need at least one system and tolerances");
  if (group_blocks < -1 || max_groups < 0) return fail(BSPAI_EINVAL, "bspai_multi_plan: bad group size or count");
  for (int k = 0; k < nsys; k++) {
    int rc = check_system(&sys[k].A, sys[k].b, sys[k].M, tol, sys[k].x, "bspai_multi_plan");
    if (rc) return rc;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto plan = [&](int gb, bspai_multi **out) {
    return tol->u_g == BSPAI_FP64 ? multi_plan_typed<double>(sys, nsys, tol, gb, max_groups, out, s)
                                  : multi_plan_typed<float>(sys, nsys, tol, gb, max_groups, out, s);
  };
  if (group_blocks >= 0) return plan(group_blocks, plan_out);
  // autotune: size classes, then one group size for all systems (the
  // smallest that holds the largest system, then doubled); one timed launch
  // of each, keep the fastest plan
  int nmax = 0;
  for (int k = 0; k < nsys; k++) nmax = std::max(nmax, sys[k].A.n);
  const int gmin = std::max(1, (nmax + kSolveThreads * 16 - 1) / (kSolveThreads * 16));
  bspai_multi *best = nullptr;
  float best_ms = 0.f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BSPAI_HIP(hipEventCreate(&e0));
  BSPAI_HIP(hipEventCreate(&e1));
  int rc = BSPAI_OK;
  // the timed launches write every x_k; with x0_mode 3 x_k is also the
  // caller's starting point, so it is saved here and put back before each
  // timed launch and once more at the end
  double *x0_save = nullptr;
  std::vector<size_t> x0_off(nsys + 1, 0);
  for (int k = 0; k < nsys; k++) x0_off[k + 1] = x0_off[k] + (size_t)sys[k].A.n;
  auto restore_x0 = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    for (int k = 0; k < nsys && e == hipSuccess; k++)
      e = hipMemcpyAsync(sys[k].x, x0_save + x0_off[k], 8 * (size_t)sys[k].A.n, hipMemcpyDeviceToDevice, s);
    return e;
  };
  if (tol->x0_mode == 3) {
    if ((rc = dalloc_t(&x0_save, x0_off[nsys]))) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
    for (int k = 0; k < nsys; k++) {
      hipError_t e = hipMemcpyAsync(x0_save + x0_off[k], sys[k].x, 8 * (size_t)sys[k].A.n, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) {
        rc = fail(BSPAI_EHIP, "bspai_multi_plan: saving x_0: %s", hipGetErrorString(e));
        break;
      }
    }
  }
  std::vector<int> cands = {0};
  for (int gb = gmin; gb <= kMaxBlocks; gb *= 2) cands.push_back(gb);
  for (int gb : cands) {
    if (rc) break;
    bspai_multi *cand = nullptr;
    rc = plan(gb, &cand);
    if (rc) {
      if (best) {  // a larger group no longer fits: keep what we have
        rc = BSPAI_OK;
        break;
      }
      break;
    }
    float ms = 0.f;
    hipError_t e = x0_save ? restore_x0() : hipSuccess;
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = hipGraphLaunch(cand->exec, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    cand->launches++;
    if (e != hipSuccess) {
      multi_release(cand);
      rc = fail(BSPAI_EHIP, "bspai_multi_plan: timing a candidate failed: %s", hipGetErrorString(e));
      break;
    }
    if (!best || ms < best_ms) {
      multi_release(best);
      best = cand;
      best_ms = ms;
    } else {
      multi_release(cand);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (x0_save) {
    hipError_t e = restore_x0();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(x0_save);
    if (e != hipSuccess && !rc) rc = fail(BSPAI_EHIP, "bspai_multi_plan: restoring x_0: %s", hipGetErrorString(e));
  }
  if (rc) {
    multi_release(best);
    return rc;
  }
  *plan_out = best;
  return BSPAI_OK;
}

extern "C" int bspai_multi_group_blocks(const bspai_multi *plan) {
  if (!plan) return fail(BSPAI_EINVAL, "bspai_multi_group_blocks: no plan");
  return plan->group_blocks;
}

extern "C" int bspai_multi_launch(bspai_multi *plan, void *stream) {
  if (!plan || !plan->exec) return fail(BSPAI_EINVAL, "bspai_multi_launch: no plan");
  int dev = 0;
  BSPAI_HIP(hipGetDevice(&dev));
  if (dev != plan->device) return fail(BSPAI_EINVAL, "bspai_multi_launch: plan lives on device %d", plan->device);
  BSPAI_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
  plan->launches++;
  return BSPAI_OK;
}

extern "C" int bspai_multi_poll(const bspai_multi *plan) {
  if (!plan) return fail(BSPAI_EINVAL, "bspai_multi_poll: no plan");
  return __atomic_load_n(plan->done_host, __ATOMIC_ACQUIRE) == plan->launches ? 1 : 0;
}

extern "C" int bspai_multi_wait(bspai_multi *plan, gmres_ir_stats *st_host, void *stream) {
  if (!plan) return fail(BSPAI_EINVAL, "bspai_multi_wait: no plan");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<gmres_ir_stats> st(plan->nsys);
  std::vector<unsigned> ab(plan->ngroups);
  BSPAI_HIP(hipMemcpyAsync(st.data(), plan->stats, sizeof(gmres_ir_stats) * plan->nsys, hipMemcpyDeviceToHost, s));
  BSPAI_HIP(hipMemcpyAsync(ab.data(), plan->aborts, 4 * (size_t)plan->ngroups, hipMemcpyDeviceToHost, s));
  BSPAI_HIP(hipStreamSynchronize(s));
  if (st_host) memcpy(st_host, st.data(), sizeof(gmres_ir_stats) * plan->nsys);
  for (unsigned a : ab)
    if (a) return fail(BSPAI_EHIP, "bspai_multi_wait: a group's synchronisation timed out");
  int worst = BSPAI_OK;
  for (const auto &q : st) worst = worse_status(worst, q.status);
  if (worst == BSPAI_ENOCONV) return fail(BSPAI_ENOCONV, "bspai_multi_wait: some system reached i_max");
  if (worst == BSPAI_ESTAG)
    return fail(BSPAI_ESTAG, "bspai_multi_wait: some system stagnated before meeting a tolerance");
  if (worst == BSPAI_ENAN) return fail(BSPAI_ENAN, "bspai_multi_wait: NaN or infinity in a residual");
  return BSPAI_OK;
}

extern "C" void bspai_multi_free(bspai_multi *plan) { multi_release(plan); }

extern "C" int bspai_release_workspace(void) {
  if (int rc = release_batched_workspace()) return rc;
  std::lock_guard<std::mutex> lock(g_ws.mu);
  if (!g_ws.ptr) return BSPAI_OK;
  int cur = 0;
  const int dev = g_ws.device;
  BSPAI_HIP(hipGetDevice(&cur));
  if (cur != dev) BSPAI_HIP(hipSetDevice(dev));
  hipError_t e = hipDeviceSynchronize();
  dfree(g_ws.ptr);
  g_ws.ptr = nullptr;
  g_ws.bytes = 0;
  g_ws.device = -1;
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess) return fail(BSPAI_EHIP, "bspai_release_workspace: %s", hipGetErrorString(e));
  return BSPAI_OK;
}

static int solve_entry(const bspai_csr *A, const bspai_handle *Ab, const double *b, const bspai_handle *M,
                       const gmres_ir_tol *tol, double *x, int nrhs, gmres_ir_stats *st_host, void *stream,
                       const char *who) {
  if (nrhs < 1 || nrhs > 64) return fail(BSPAI_EINVAL, "%s: nrhs must be in 1..64 (got %d)", who, nrhs);
  int rc = check_system(A, b, M, tol, x, who);
  if (rc) return rc;
  if (Ab) {
    if (Ab->n != A->n) return fail(BSPAI_EINVAL, "%s: A is %d x %d but A_b is %d x %d", who, A->n, A->n, Ab->n, Ab->n);
    if (tol->trans && !Ab->has_T) return fail(BSPAI_EINVAL, "%s: trans needs A_b built with build_T", who);
    if (Ab->device != M->device) return fail(BSPAI_EINVAL, "%s: A_b lives on device %d", who, Ab->device);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (nrhs > 1) {
    if (tol->orth != 0) return fail(BSPAI_EINVAL, "%s: orth = 1 (CGS2) needs nrhs = 1", who);
    const int m = std::min(std::max(tol->gmres_max, 1), std::min(A->n, kMaxGmres));
    if (tol->u_g == BSPAI_FP64) return solve_many<double>(A, Ab, b, M, tol, x, nrhs, m, st_host, s);
    return solve_many<float>(A, Ab, b, M, tol, x, nrhs, m, st_host, s);
  }
  if (tol->u_g == BSPAI_FP64) return solve_typed<double>(A, Ab, b, M, tol, x, st_host, s);
  return solve_typed<float>(A, Ab, b, M, tol, x, st_host, s);
}

extern "C" int gmres_ir_solve(const bspai_csr *A, const double *b, const bspai_handle *M, const gmres_ir_tol *tol,
                              double *x, int nrhs, gmres_ir_stats *st_host, void *stream) {
  return solve_entry(A, nullptr, b, M, tol, x, nrhs, st_host, stream, "gmres_ir_solve");
}

// ---------------------------------------------- solve without allocation
// Workspace of gmres_ir_solve_noalloc: a file-scope device array.  Every GPU
// the library runs on holds its own copy until the process ends.  Host code
// never uses the array's name (a host-side stand-in): the device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is passed to kernels and copies.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxScratchDevices];

static int scratch_address(char **out, const char *who) {
  int dev = 0;
  BSPAI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(BSPAI_EINVAL, "%s: device %d is out of range", who, dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BSPAI_EHIP, "%s: device address of the scratch array: %s", who, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return BSPAI_OK;
}

extern "C" int gmres_ir_solve_noalloc(const bspai_csr *A, const double *b, const bspai_handle *M,
                                      const gmres_ir_tol *tol, double *x, gmres_ir_stats *st_host, void *stream) {
  const char *who = "gmres_ir_solve_noalloc";
  int rc = check_system(A, b, M, tol, x, who);
  if (rc) return rc;
  if (tol->trans)
    return fail(BSPAI_EINVAL, "%s: the transposed solve forms A^T in temporary storage; use gmres_ir_solve", who);
  char *base = nullptr;
  if ((rc = scratch_address(&base, who))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (tol->u_g == BSPAI_FP64) return solve_typed<double>(A, nullptr, b, M, tol, x, st_host, s, base, kScratchBytes, who);
  return solve_typed<float>(A, nullptr, b, M, tol, x, st_host, s, base, kScratchBytes, who);
}

extern "C" int gmres_ir_solve_ab(const bspai_csr *A, const bspai_handle *A_b, const double *b, const bspai_handle *M,
                                 const gmres_ir_tol *tol, double *x, int nrhs, gmres_ir_stats *st_host, void *stream) {
  if (!A_b) return fail(BSPAI_EINVAL, "gmres_ir_solve_ab: null A_b");
  return solve_entry(A, A_b, b, M, tol, x, nrhs, st_host, stream, "gmres_ir_solve_ab");
}
