// Internal declarations shared by the HIP sources of libbspai.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "bspai.h"

namespace bspai {

constexpr int kMaxBuckets = 6;

// Unit roundoff of each storage precision (Table 2; u = 1 for the drop bucket).
inline double unit_roundoff(int p) {
  switch (p) {
    case BSPAI_FP64: return 0x1p-53;
    case BSPAI_FP32: return 0x1p-24;
    case BSPAI_FP16: return 0x1p-11;
    case BSPAI_BF16: return 0x1p-8;
    case BSPAI_FP8_E4M3: return 0x1p-4;
    case BSPAI_DROP: return 1.0;
  }
  return -1.0;
}

inline int value_bytes(int p) {
  switch (p) {
    case BSPAI_FP64: return 8;
    case BSPAI_FP32: return 4;
    case BSPAI_FP16: return 2;
    case BSPAI_BF16: return 2;
    case BSPAI_FP8_E4M3: return 1;
  }
  return 0;
}

// A bucketed sparse matrix as the kernels see it: one CSR per stored bucket,
// ordered from the least precise bucket to the most precise one (the order
// in which the partial sums are added).
struct BMat {
  int32_t n;
  int32_t nb;
  int32_t lanes;    // lanes per row chosen for the single-vector product
  int32_t aligned;  // every col / val array is 16-byte aligned (tile product allowed)
  int64_t nnz;      // stored entries (all buckets)
  int32_t prec[kMaxBuckets];
  double scale[kMaxBuckets];
  const int32_t *rp[kMaxBuckets];
  const int32_t *col[kMaxBuckets];
  const void *val[kMaxBuckets];
  // the same buckets in SELL-64 form (64-row slices stored column by column,
  // short rows padded with zero values): entry u of row 64 s + r of bucket k
  // is at sell_ptr[k][s] + 64 u + r.  sell_ptr null: not available.
  const int32_t *sell_ptr[kMaxBuckets];
  const int32_t *sell_col[kMaxBuckets];
  const void *sell_val[kMaxBuckets];
  // > 0: every slice of the bucket has this width (ELL), so slice s starts at
  // 64 s w and the kernels need not load sell_ptr
  int32_t sell_w[kMaxBuckets];
  // row-major padded copy (ELL): row i's entries at i W .. i W + W - 1, W in
  // {4, 8, 16}, padding entries with value 0; ell_w 0: not available
  const int32_t *ell_col[kMaxBuckets];
  const void *ell_val[kMaxBuckets];
  int32_t ell_w[kMaxBuckets];
  // narrow columns of the ELL copy (then ell_col is null): ell_cw 1: ell_code
  // holds one byte per entry, an index into ell_dict (256 offsets col - row);
  // 2: ell_code holds the int16 offset col - row; 0: int32 ell_col
  const void *ell_code[kMaxBuckets];
  const int32_t *ell_dict[kMaxBuckets];
  int32_t ell_cw[kMaxBuckets];
  // kernel of the single-vector product: 0 chosen from the layout, else one
  // of the ApplyKind values (set by bspai_set_apply_kind / bspai_tune_apply)
  int32_t apply_kind;
  // entry-balanced tiles of whole rows for the segmented product: tile t
  // holds rows seg_rows[t] .. seg_rows[t + 1] - 1, with fewer than seg_cap
  // entries over all buckets, whose entries of bucket k start at
  // seg_off[t nb + k]; seg_rows null: no plan
  const int32_t *seg_rows;
  const int32_t *seg_off;
  int32_t seg_ntiles;
  int32_t seg_cap;
};

// kernels of the single-vector bucketed product
enum ApplyKind { kApplyAuto = 0, kApplySell = 1, kApplyTile = 2, kApplyRows = 3, kApplyLanes = 4, kApplySeg = 5 };

constexpr int kSlice = 64;

struct Bucket {
  int prec = BSPAI_FP64;
  int64_t nnz = 0;
  double t = 0, scale = 1;
  int32_t *rp = nullptr, *col = nullptr;
  void *val = nullptr;
  int32_t *rpT = nullptr, *colT = nullptr;
  void *valT = nullptr;
  int32_t *sptr = nullptr, *scol = nullptr, *sptrT = nullptr, *scolT = nullptr;
  void *sval = nullptr, *svalT = nullptr;
  int32_t *ecol = nullptr, *ecolT = nullptr;
  void *eval = nullptr, *evalT = nullptr;
  void *ecode = nullptr, *ecodeT = nullptr;
  int32_t *edict = nullptr, *edictT = nullptr;
  int32_t ecw = 0, ecwT = 0;
};

}  // namespace bspai

struct bspai_handle {
  int32_t n = 0;
  int64_t nnz = 0;
  int q = 0;
  int precs[bspai::kMaxBuckets] = {0};
  double eps = 0, normM = 0;
  bspai::Bucket b[bspai::kMaxBuckets];
  // FP64 M in CSR (pattern order) and, with build_T, its transpose
  int32_t *m_rp = nullptr, *m_col = nullptr;
  double *m_val = nullptr;
  int32_t *mT_rp = nullptr, *mT_col = nullptr;
  double *mT_val = nullptr;
  int8_t *bucket_id = nullptr;  // per entry of M, CSR order
  double *stored = nullptr;     // decoded stored value per entry (FP64), CSR order
  int has_T = 0, has_fp64 = 0;
  bspai::BMat mat, matT;
  int32_t *seg_rows = nullptr, *seg_rowsT = nullptr;  // tile plans of mat and matT
  int device = 0;
};

namespace bspai {

void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// The more severe of two per-right-hand-side solve statuses, in the order
// ENAN > ENOCONV > ESTAG > OK (a call reports the worst of its columns).
inline int worse_status(int a, int b) {
  auto rank = [](int c) { return c == BSPAI_ENAN ? 3 : c == BSPAI_ENOCONV ? 2 : c == BSPAI_ESTAG ? 1 : 0; };
  return rank(b) > rank(a) ? b : a;
}

#define BSPAI_HIP(expr)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return ::bspai::fail(e_ == hipErrorOutOfMemory ? BSPAI_ENOMEM : BSPAI_EHIP, "%s: %s (%s:%d)", \
                           #expr, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define BSPAI_CHECK_LAUNCH() BSPAI_HIP(hipGetLastError())

// Device memory helpers (hipMalloc with error reporting).
int dalloc(void **p, size_t bytes);
template <typename T>
int dalloc_t(T **p, size_t count) {
  return dalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}
void dfree(void *p);

// Exclusive prefix sum of n int32 counts into out[0..n] (out[n] = total),
// on device; the total must fit int32.  tmp needs scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
int exclusive_scan(const int32_t *in, int32_t *out, int64_t n, void *tmp, hipStream_t s);

// CSR transpose on the device: entries of each output row sorted by source
// row (deterministic).  Values of `vbytes` bytes each are moved when val != null.
int csr_transpose(int n, int64_t nnz, const int32_t *rp, const int32_t *col, const void *val, int vbytes,
                  int32_t *trp, int32_t *tcol, void *tval, hipStream_t s);

// SELL-64 copy of one CSR (values of vbytes bytes); allocates *sptr (n/64+1),
// *scol and *sval (padded length).  No copy (null pointers, BSPAI_OK) when
// the padding would exceed half the entries.
// *width gets the common slice width when all slices are padded to the
// widest one (chosen when that pads at most 15% more than per-slice widths),
// else 0.
int csr_to_sell(int n, const int32_t *rp, const int32_t *col, const void *val, int vbytes, int32_t **sptr,
                int32_t **scol, void **sval, int32_t *width, hipStream_t s);

// Row-major padded (ELL) copy of one CSR when every row has at most 16
// entries and padding to W in {4, 8, 16} adds at most 25% entries; *width
// gets W, or 0 (and nothing allocated) otherwise.
int csr_to_ell(int n, const int32_t *rp, const int32_t *col, const void *val, int vbytes, int32_t **ecol,
               void **evalp, int32_t *width, hipStream_t s);

// Narrow column codes of an ELL copy (n rows of width w): *cw = 1 with
// *code one byte per entry and *dict 256 int32 offsets col - row when the
// copy has at most 256 distinct offsets; *cw = 2 with *code int16 offsets
// when they all fit; else *cw = 0 and nothing allocated.
int ell_codes(int n, int w, const int32_t *ecol, void **code, int32_t **dict, int32_t *cw, hipStream_t s);

// Bucketed product kernels (apply.hip), used by the public apply and the build.
int pick_lanes(const BMat &M, int64_t nnz);
int bmat_aligned(const BMat &M);
int launch_bspmv(const BMat &M, const void *x, void *y, int nrhs, int64_t ld, int fp64, hipStream_t s);
// whether M has what kernel `kind` needs, and the kernel used when none is set
bool apply_kind_ok(const BMat &M, int kind);
int apply_kind_resolved(const BMat &M);
// Entry-balanced tile plan of M for the segmented product (sets M.seg_*);
// *rows is allocated here and owned by the caller.  No plan (and BSPAI_OK)
// when some row has more entries than a tile holds.
int build_seg_plan(BMat &M, int32_t **rows, hipStream_t s);

// One Arnoldi step's MGS over an n x (16 / sizeof(VT)) row-major column
// group as one cooperative kernel (solve.hip).  mgs_persist_rpt(n) is 0 when
// n is too large for it; ws needs mgs_persist_ws_bytes() bytes of exchange
// words, zeroed once before the first launch (see launch_mgs_persist).
int mgs_persist_rpt(int n);
size_t mgs_persist_ws_bytes();
template <typename VT>
int launch_mgs_persist(int n, int j, int m, const VT *z, VT *V, int64_t vstride, double *H, double *hn,
                       const int *gma, void *ws, unsigned rtag0, unsigned *abortf, hipStream_t s);

// Instrumentation shared by the solvers (solve.hip): the profiling switch
// (bspai_set_profiling) and the totals of the one-launch MGS kernel.
bool profiling_on();
int release_batched_workspace();  // frees the column-group solve's kept device block
bool mgs_profile_sample();  // whether to time the next one-launch MGS (one in seven)
void add_mgs_profile(double ms, double bytes);
// How the many-right-hand-side solve runs its columns (bspai_set_batch_mode):
// 0 automatic, 1 every column in each pass kernel, 2 column groups with the
// one-launch MGS.
int batch_mode();

// gmres_ir_solve for 2 <= R <= 64 right-hand sides (solve_batched.hip);
// arguments already validated, m the GMRES cap, Ab the bucketed A used inside
// GMRES (NULL: A rounded to u_g).  solve_many picks between all columns
// together (solve_batched with the per-pass kernels) and consecutive groups
// of 16 / sizeof(VT) columns (solve_batched with mgs1, one MGS launch per
// Arnoldi step).
template <typename VT>
int solve_many(const bspai_csr *A, const bspai_handle *Ab, const double *b, const bspai_handle *M,
               const gmres_ir_tol *tol, double *x, int R, int m, gmres_ir_stats *st_host, hipStream_t s);
template <typename VT>
int solve_batched(const bspai_csr *A, const bspai_handle *Ab, const double *b, const bspai_handle *M,
                  const gmres_ir_tol *tol, double *x, int R, int m, gmres_ir_stats *st_host, hipStream_t s,
                  bool mgs1);

}  // namespace bspai
