// Error reporting, device allocation, prefix sums and CSR transposition.
#include <cstdarg>
#include <cstring>

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

}  // namespace bspai

extern "C" const char *bspai_last_error(void) { return bspai::g_err; }
