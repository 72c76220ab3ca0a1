// Error reporting, device allocation, prefix sums and CSR transposition.
#include <cstdarg>
#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "common.h"

namespace bspai {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int dalloc(void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? BSPAI_ENOMEM : BSPAI_EHIP, "hipMalloc(%zu bytes): %s", bytes,
                hipGetErrorString(e));
  }
  return BSPAI_OK;
}

void dfree(void *p) {
  if (p) (void)hipFree(p);
}

// ------------------------------------------------------------------ scan
// Three passes: per-block sums, a scan of the block sums (one block, looping
// over chunks), then the block-local scans plus their offsets.

constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(kScanBlock) k_scan_block_sums(const int32_t *in, int64_t n, int32_t *bsum) {
  __shared__ int32_t sh[kScanBlock / 64];
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int32_t v = i < n ? in[i] : 0;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int w = 0; w < kScanBlock / 64; w++) t += sh[w];
    bsum[blockIdx.x] = t;
  }
}

// inclusive scan of one block of values held one per thread; returns the
// exclusive prefix of this thread and the block total in *total
__device__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
  __shared__ int32_t wsum[kScanBlock / 64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    int32_t t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) {
      int32_t t = wsum[k];
      wsum[k] = acc;
      acc += t;
    }
    wsum[0] = wsum[0];
    *total = acc;
  }
  __syncthreads();
  int32_t ex = inc - v + wsum[w];
  __syncthreads();
  return ex;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_bsums(int32_t *bsum, int64_t nb) {
  __shared__ int32_t total;
  int32_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanBlock) {
    int64_t i = base + threadIdx.x;
    int32_t v = i < nb ? bsum[i] : 0;
    int32_t ex = block_exclusive_scan(v, &total);
    if (i < nb) bsum[i] = ex + carry;
    __syncthreads();
    carry += total;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_final(const int32_t *in, int64_t n, const int32_t *bsum,
                                                          int32_t *out) {
  __shared__ int32_t total;
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int32_t v = i < n ? in[i] : 0;
  int32_t ex = block_exclusive_scan(v, &total) + bsum[blockIdx.x];
  if (i < n) out[i] = ex;
  if (i == n - 1) out[n] = ex + v;
}

size_t scan_tmp_bytes(int64_t n) { return sizeof(int32_t) * (size_t)((n + kScanBlock - 1) / kScanBlock + 1); }

int exclusive_scan(const int32_t *in, int32_t *out, int64_t n, void *tmp, hipStream_t s) {
  if (n <= 0) {
    BSPAI_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
    return BSPAI_OK;
  }
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  int32_t *bsum = static_cast<int32_t *>(tmp);
  hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, bsum);
  BSPAI_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kScanBlock), 0, s, bsum, nb);
  BSPAI_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, bsum, out);
  BSPAI_CHECK_LAUNCH();
  return BSPAI_OK;
}

// ------------------------------------------------------------------ transpose

__global__ void k_count_cols(const int32_t *col, int64_t nnz, int32_t *cnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[col[e]], 1);
}

// Scatter entry e of row i to column col[e]; the slot within the column is
// taken with an atomic, then every column is sorted by source row below.
__global__ void k_scatter_T(int n, const int32_t *rp, const int32_t *col, int32_t *fill, const int32_t *trp,
                            int32_t *tsrc, int32_t *trow) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; e++) {
    int c = col[e];
    int pos = trp[c] + atomicAdd(&fill[c], 1);
    trow[pos] = i;
    tsrc[pos] = e;
  }
}

// insertion sort of each output row by source row (rows are short)
__global__ void k_sort_T(int n, const int32_t *trp, int32_t *trow, int32_t *tsrc) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int s = trp[c], e = trp[c + 1];
  for (int a = s + 1; a < e; a++) {
    int kr = trow[a], ks = tsrc[a];
    int b = a - 1;
    while (b >= s && trow[b] > kr) {
      trow[b + 1] = trow[b];
      tsrc[b + 1] = tsrc[b];
      b--;
    }
    trow[b + 1] = kr;
    tsrc[b + 1] = ks;
  }
}

__global__ void k_gather_vals(int64_t nnz, const int32_t *tsrc, const uint8_t *val, int vbytes, uint8_t *tval) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const uint8_t *src = val + (int64_t)tsrc[p] * vbytes;
  uint8_t *dst = tval + p * vbytes;
  for (int b = 0; b < vbytes; b++) dst[b] = src[b];
}

int csr_transpose(int n, int64_t nnz, const int32_t *rp, const int32_t *col, const void *val, int vbytes,
                  int32_t *trp, int32_t *tcol, void *tval, hipStream_t s) {
  int32_t *cnt = nullptr, *fill = nullptr, *tsrc = nullptr;
  void *tmp = nullptr;
  int rc = BSPAI_OK;
  if ((rc = dalloc_t(&cnt, (size_t)n)) || (rc = dalloc_t(&fill, (size_t)n)) || (rc = dalloc_t(&tsrc, (size_t)nnz + 1)) ||
      (rc = dalloc(&tmp, scan_tmp_bytes(n)))) {
    dfree(cnt), dfree(fill), dfree(tsrc), dfree(tmp);
    return rc;
  }
  auto body = [&]() -> int {
    BSPAI_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, s));
    BSPAI_HIP(hipMemsetAsync(fill, 0, sizeof(int32_t) * n, s));
    if (nnz > 0) {
      hipLaunchKernelGGL(k_count_cols, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, col, nnz, cnt);
      BSPAI_CHECK_LAUNCH();
    }
    int r = exclusive_scan(cnt, trp, n, tmp, s);
    if (r) return r;
    unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_scatter_T, dim3(g), dim3(256), 0, s, n, rp, col, fill, trp, tsrc, tcol);
    BSPAI_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sort_T, dim3(g), dim3(256), 0, s, n, trp, tcol, tsrc);
    BSPAI_CHECK_LAUNCH();
    if (val && nnz > 0) {
      hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, tsrc,
                         static_cast<const uint8_t *>(val), vbytes, static_cast<uint8_t *>(tval));
      BSPAI_CHECK_LAUNCH();
    }
    BSPAI_HIP(hipStreamSynchronize(s));
    return BSPAI_OK;
  };
  rc = body();
  dfree(cnt), dfree(fill), dfree(tsrc), dfree(tmp);
  return rc;
}

// ------------------------------------------------------------------ SELL-64

__global__ void k_slice_len(int n, const int32_t *rp, int32_t *len) {
  int sl = blockIdx.x * blockDim.x + threadIdx.x;
  int ns = (n + kSlice - 1) / kSlice;
  if (sl >= ns) return;
  int mx = 0;
  for (int r = sl * kSlice; r < min(n, (sl + 1) * kSlice); r++) mx = max(mx, rp[r + 1] - rp[r]);
  len[sl] = mx * kSlice;
}

__global__ void k_sell_fill(int n, const int32_t *rp, const int32_t *col, const uint8_t *val, int vbytes,
                            const int32_t *sptr, int32_t *scol, uint8_t *sval) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int ns = (n + kSlice - 1) / kSlice;
  if (i >= ns * kSlice) return;
  int sl = i / kSlice, r = i % kSlice;
  int len = (sptr[sl + 1] - sptr[sl]) / kSlice;
  int s = i < n ? rp[i] : 0, e = i < n ? rp[i + 1] : 0;
  int pad_col = i < n ? i : 0;
  for (int u = 0; u < len; u++) {
    int64_t dst = (int64_t)sptr[sl] + (int64_t)u * kSlice + r;
    if (s + u < e) {
      scol[dst] = col[s + u];
      for (int b = 0; b < vbytes; b++) sval[dst * vbytes + b] = val[(int64_t)(s + u) * vbytes + b];
    } else {
      scol[dst] = pad_col;
      for (int b = 0; b < vbytes; b++) sval[dst * vbytes + b] = 0;  // +0 in every format
    }
  }
}

__global__ void k_fill_value(int32_t *a, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

int csr_to_sell(int n, const int32_t *rp, const int32_t *col, const void *val, int vbytes, int32_t **sptr,
                int32_t **scol, void **sval, int32_t *width, hipStream_t s) {
  *sptr = nullptr, *scol = nullptr, *sval = nullptr;
  *width = 0;
  int ns = (n + kSlice - 1) / kSlice;
  int32_t *len = nullptr;
  void *tmp = nullptr;
  int rc;
  if ((rc = dalloc_t(&len, (size_t)ns + 1)) || (rc = dalloc(&tmp, scan_tmp_bytes(ns))) ||
      (rc = dalloc_t(sptr, (size_t)ns + 1))) {
    dfree(len), dfree(tmp), dfree(*sptr);
    *sptr = nullptr;
    return rc;
  }
  auto body = [&]() -> int {
    if (ns > 0) {
      hipLaunchKernelGGL(k_slice_len, dim3((ns + 255) / 256), dim3(256), 0, s, n, rp, len);
      BSPAI_CHECK_LAUNCH();
    }
    int32_t total = 0, wmax = 0;
    if (ns > 0) {
      std::vector<int32_t> hl((size_t)ns);
      BSPAI_HIP(hipMemcpyAsync(hl.data(), len, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
      BSPAI_HIP(hipStreamSynchronize(s));
      int64_t tot = 0;
      for (int32_t v : hl) {
        tot += v;
        wmax = std::max(wmax, v / kSlice);
      }
      // slices of rows with very different lengths (power-law matrices) pad
      // each row to the longest of its slice: no SELL copy when that more
      // than 1.5x the entries
      int32_t nnz = 0;
      BSPAI_HIP(hipMemcpyAsync(&nnz, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      BSPAI_HIP(hipStreamSynchronize(s));
      if ((double)tot > 1.5 * (double)std::max(nnz, 1) || tot >= INT32_MAX) return 1;  // no copy
      if ((double)ns * kSlice * wmax <= 1.15 * (double)tot && (int64_t)ns * kSlice * wmax < INT32_MAX) {
        *width = wmax;  // one width for all slices
        hipLaunchKernelGGL(k_fill_value, dim3((ns + 255) / 256), dim3(256), 0, s, len, (int64_t)ns, wmax * kSlice);
        BSPAI_CHECK_LAUNCH();
      }
    }
    int r = exclusive_scan(len, *sptr, ns, tmp, s);
    if (r) return r;
    BSPAI_HIP(hipMemcpyAsync(&total, *sptr + ns, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    if ((r = dalloc_t(scol, (size_t)total + kSlice)) || (r = dalloc(sval, (size_t)vbytes * (total + kSlice))))
      return r;
    if (ns > 0) {
      hipLaunchKernelGGL(k_sell_fill, dim3((ns * kSlice + 255) / 256), dim3(256), 0, s, n, rp, col,
                         static_cast<const uint8_t *>(val), vbytes, *sptr, *scol, static_cast<uint8_t *>(*sval));
      BSPAI_CHECK_LAUNCH();
    }
    BSPAI_HIP(hipStreamSynchronize(s));
    return BSPAI_OK;
  };
  rc = body();
  dfree(len), dfree(tmp);
  if (rc) {
    dfree(*sptr), dfree(*scol), dfree(*sval);
    *sptr = nullptr, *scol = nullptr, *sval = nullptr;
    *width = 0;
  }
  return rc == 1 ? BSPAI_OK : rc;
}

// ------------------------------------------------------------------ ELL

// the longest row: a grid-stride maximum, one atomic per block
__global__ void __launch_bounds__(256) k_row_len_max(int n, const int32_t *rp, int32_t *mx) {
  int v = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v = max(v, rp[i + 1] - rp[i]);
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  __shared__ int32_t sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); k++) v = max(v, sh[k]);
    atomicMax(mx, v);
  }
}

// one thread per ELL entry (row i = dst / w, slot u = dst % w), so that the
// stores of a wave are contiguous; values move as whole 2-, 4- or 8-byte words.
// Slots past the row's length hold column i and value 0.
__global__ void k_ell_fill(int n, const int32_t *rp, const int32_t *col, const uint8_t *val, int vbytes, int w,
                           int32_t *ecol, uint8_t *eval) {
  const int64_t dst = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dst >= (int64_t)n * w) return;
  const int i = (int)(dst / w), u = (int)(dst % w);
  const int s = rp[i], e = rp[i + 1];
  const bool in = s + u < e;
  const int64_t src = (int64_t)s + u;
  ecol[dst] = in ? col[src] : i;
  if (vbytes == 8) {
    reinterpret_cast<uint64_t *>(eval)[dst] = in ? reinterpret_cast<const uint64_t *>(val)[src] : 0ull;
  } else if (vbytes == 4) {
    reinterpret_cast<uint32_t *>(eval)[dst] = in ? reinterpret_cast<const uint32_t *>(val)[src] : 0u;
  } else if (vbytes == 2) {
    reinterpret_cast<uint16_t *>(eval)[dst] = in ? reinterpret_cast<const uint16_t *>(val)[src] : (uint16_t)0;
  } else {
    for (int b = 0; b < vbytes; b++) eval[dst * vbytes + b] = in ? val[src * vbytes + b] : (uint8_t)0;
  }
}

int csr_to_ell(int n, const int32_t *rp, const int32_t *col, const void *val, int vbytes, int32_t **ecol,
               void **evalp, int32_t *width, hipStream_t s) {
  *ecol = nullptr, *evalp = nullptr, *width = 0;
  if (n == 0) return BSPAI_OK;
  int32_t *mx = nullptr;
  int rc;
  if ((rc = dalloc_t(&mx, 1))) return rc;
  int32_t hmx = 0, nnz = 0;
  auto body = [&]() -> int {
    BSPAI_HIP(hipMemsetAsync(mx, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_row_len_max, dim3((unsigned)std::min(1024, (n + 255) / 256)), dim3(256), 0, s, n, rp, mx);
    BSPAI_CHECK_LAUNCH();
    BSPAI_HIP(hipMemcpyAsync(&hmx, mx, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipMemcpyAsync(&nnz, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    return BSPAI_OK;
  };
  rc = body();
  dfree(mx);
  if (rc) return rc;
  int w = hmx <= 4 ? 4 : (hmx <= 8 ? 8 : (hmx <= 16 ? 16 : 0));
  if (w == 0 || (double)n * w > 1.25 * (double)std::max(nnz, 1) || (int64_t)n * w >= INT32_MAX) return BSPAI_OK;
  if ((rc = dalloc_t(ecol, (size_t)n * w)) || (rc = dalloc(evalp, (size_t)n * w * vbytes))) {
    dfree(*ecol), dfree(*evalp);
    *ecol = nullptr, *evalp = nullptr;
    return rc;
  }
  hipLaunchKernelGGL(k_ell_fill, dim3((unsigned)(((int64_t)n * w + 255) / 256)), dim3(256), 0, s, n, rp, col,
                     static_cast<const uint8_t *>(val), vbytes, w, *ecol, static_cast<uint8_t *>(*evalp));
  BSPAI_CHECK_LAUNCH();
  BSPAI_HIP(hipStreamSynchronize(s));
  *width = w;
  return BSPAI_OK;
}

// ------------------------------------------------------------------ ELL column codes
//
// Entry u of row i of an ELL copy sits at i W + u, so its column can be stored
// as the offset col - i.  Structured operators have few distinct offsets (7
// for a 3D 7-point stencil): with at most 256 of them the columns become one
// byte each, an index into a per-bucket table of offsets; otherwise, when every
// offset fits 16 bits, two bytes each.

constexpr int kDeltaWaves = 4;  // waves per block of k_delta_range (256 threads)
__global__ void __launch_bounds__(256) k_delta_range(int64_t ne, int w, const int32_t *ecol, int32_t *mm) {
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t d = ecol[e] - (int32_t)(e / w);
    lo = min(lo, d);
    hi = max(hi, d);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o));
    hi = max(hi, __shfl_xor(hi, o));
  }
  // one pair of atomics per block (every wave's would queue on two words)
  __shared__ int32_t sh[2][kDeltaWaves];
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = lo;
    sh[1][threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); k++) {
      lo = min(lo, sh[0][k]);
      hi = max(hi, sh[1][k]);
    }
    atomicMin(&mm[0], lo);
    atomicMax(&mm[1], hi);
  }
}

__global__ void k_delta_mark(int64_t ne, int w, const int32_t *ecol, int32_t lo, int32_t *flags) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x)
    flags[ecol[e] - (int32_t)(e / w) - lo] = 1;
}

__global__ void k_dict_fill(int32_t range, const int32_t *flags, const int32_t *pos, int32_t lo, int32_t *dict) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < range && flags[i]) dict[pos[i]] = i + lo;
}

__global__ void k_code8(int64_t ne, int w, const int32_t *ecol, int32_t lo, const int32_t *pos, uint8_t *code) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x)
    code[e] = (uint8_t)pos[ecol[e] - (int32_t)(e / w) - lo];
}

__global__ void k_code16(int64_t ne, int w, const int32_t *ecol, int16_t *code) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x)
    code[e] = (int16_t)(ecol[e] - (int32_t)(e / w));
}

int ell_codes(int n, int w, const int32_t *ecol, void **code, int32_t **dict, int32_t *cw, hipStream_t s) {
  *code = nullptr, *dict = nullptr, *cw = 0;
  const int64_t ne = (int64_t)n * w;
  if (ne == 0) return BSPAI_OK;
  constexpr int64_t kMaxRange = 1 << 22;
  const unsigned grid = (unsigned)std::min<int64_t>(4096, (ne + 255) / 256);
  int32_t *mm = nullptr, *flags = nullptr, *pos = nullptr;
  void *tmp = nullptr;
  int rc = dalloc_t(&mm, 2);
  if (rc) return rc;
  auto body = [&]() -> int {
    const int32_t init[2] = {INT32_MAX, INT32_MIN};
    int32_t hm[2];
    BSPAI_HIP(hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_delta_range, dim3(std::min(grid, 1024u)), dim3(256), 0, s, ne, w, ecol, mm);
    BSPAI_CHECK_LAUNCH();
    BSPAI_HIP(hipMemcpyAsync(hm, mm, sizeof(hm), hipMemcpyDeviceToHost, s));
    BSPAI_HIP(hipStreamSynchronize(s));
    const int32_t lo = hm[0], hi = hm[1];
    const int64_t range = (int64_t)hi - lo + 1;
    if (range <= kMaxRange) {
      int r;
      if ((r = dalloc_t(&flags, (size_t)range)) || (r = dalloc_t(&pos, (size_t)range + 1)) ||
          (r = dalloc(&tmp, scan_tmp_bytes(range))))
        return r;
      BSPAI_HIP(hipMemsetAsync(flags, 0, 4 * (size_t)range, s));
      hipLaunchKernelGGL(k_delta_mark, dim3(grid), dim3(256), 0, s, ne, w, ecol, lo, flags);
      BSPAI_CHECK_LAUNCH();
      if ((r = exclusive_scan(flags, pos, range, tmp, s))) return r;
      int32_t total = 0;
      BSPAI_HIP(hipMemcpyAsync(&total, pos + range, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      BSPAI_HIP(hipStreamSynchronize(s));
      if (total <= 256) {
        if ((r = dalloc_t(dict, 256)) || (r = dalloc(code, (size_t)ne + 16))) return r;
        BSPAI_HIP(hipMemsetAsync(*dict, 0, 4 * 256, s));
        hipLaunchKernelGGL(k_dict_fill, dim3((unsigned)((range + 255) / 256)), dim3(256), 0, s, (int32_t)range, flags,
                           pos, lo, *dict);
        BSPAI_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_code8, dim3(grid), dim3(256), 0, s, ne, w, ecol, lo, pos, static_cast<uint8_t *>(*code));
        BSPAI_CHECK_LAUNCH();
        *cw = 1;
      }
    }
    if (*cw == 0 && lo >= -32768 && hi <= 32767) {
      int r;
      if ((r = dalloc(code, 2 * (size_t)ne + 16))) return r;
      hipLaunchKernelGGL(k_code16, dim3(grid), dim3(256), 0, s, ne, w, ecol, static_cast<int16_t *>(*code));
      BSPAI_CHECK_LAUNCH();
      *cw = 2;
    }
    BSPAI_HIP(hipStreamSynchronize(s));
    return BSPAI_OK;
  };
  rc = body();
  dfree(mm), dfree(flags), dfree(pos), dfree(tmp);
  if (rc) {
    dfree(*code), dfree(*dict);
    *code = nullptr, *dict = nullptr, *cw = 0;
  }
  return rc;
}

}  // namespace bspai

extern "C" const char *bspai_last_error(void) { return bspai::g_err; }
