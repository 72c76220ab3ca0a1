/*
 * CPU oracle for BSPAI-GMRES-IR (Khan & Carson, arXiv 2307.03914).
 *
 * TEST INFRASTRUCTURE.  This library is the plain, slow reference that the HIP
 * implementation is checked against.  Only the test-suite, the package smoke
 * check and the benchmark's CPU-baseline leg load it; the product path never
 * does.  It shares no code, header, table or helper with the HIP sources.
 *
 * Every function follows a passage of the paper and says which.  Arithmetic is
 * FP64 unless the paper fixes another precision.  The working precision of
 * GMRES (u_g) and of the operator (u_p) is emulated by rounding every FP64
 * operation result to that format (for binary32 this reproduces native single
 * arithmetic exactly, since 53 >= 2*24+2).  Build with -ffp-contract=off so
 * that the compiler adds no fused multiply-adds.
 *
 * Each part is pinned against something other than itself (exact rational
 * arithmetic, NumPy/torch casts and dense solvers, closed forms, the numbers
 * printed in Tables 3 and 4); the pins are the tests/test_oracle_*.py files and
 * the package docstring lists them per function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <fenv.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Interface numbering of precisions and status codes (same values as the C
 * interface of the library; defined here independently). */
enum { OP_FP64 = 0, OP_FP32 = 1, OP_FP16 = 2, OP_BF16 = 3, OP_FP8 = 4, OP_DROP = 5 };
enum {
    ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EZEROROW = -4,
    ORC_ERANK = -5, ORC_ENOCONV = -6, ORC_ENAN = -7, ORC_ESTAG = -8
};

int orc_num_threads(int req) {
#ifdef _OPENMP
    if (req > 0) omp_set_num_threads(req);
    return omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Floating-point formats (Table 2 of the paper for half/single/double; the
 * bfloat16 and OCP FP8 E4M3FN formats from their published definitions).
 * ---------------------------------------------------------------------- */

/* unit roundoff u = 2^-p for a format with p significand bits (Table 2);
 * the "drop" pseudo-precision has u = 1 (Section 4, the choice u_q = 1). */
double orc_unit_roundoff(int prec) {
    switch (prec) {
    case OP_FP64: return ldexp(1.0, -53);
    case OP_FP32: return ldexp(1.0, -24);
    case OP_FP16: return ldexp(1.0, -11);
    case OP_BF16: return ldexp(1.0, -8);
    case OP_FP8: return ldexp(1.0, -4);
    case OP_DROP: return 1.0;
    }
    return NAN;
}

/* significand bits (with the hidden bit), minimum normal exponent, largest
 * finite value, exponent field width and bias of each stored format */
static int fmt_params(int prec, int *p, int *emin, double *maxf, int *ebits, int *bias) {
    switch (prec) {
    case OP_FP32: *p = 24; *emin = -126; *maxf = ldexp(2.0 - ldexp(1.0, -23), 127); *ebits = 8; *bias = 127; return 0;
    case OP_FP16: *p = 11; *emin = -14; *maxf = 65504.0; *ebits = 5; *bias = 15; return 0;
    case OP_BF16: *p = 8; *emin = -126; *maxf = ldexp(2.0 - ldexp(1.0, -7), 127); *ebits = 8; *bias = 127; return 0;
    case OP_FP8: *p = 4; *emin = -6; *maxf = 448.0; *ebits = 4; *bias = 7; return 0;
    }
    return -1;
}

/* Round x to the nearest value of the format, ties to even (IEEE default
 * rounding), keeping subnormals.  Overflow returns +-inf (never reached by
 * the scaled bucket values).  FP64 is the identity, DROP gives 0. */
double orc_round(int prec, double x) {
    int p, emin, ebits, bias;
    double maxf;
    if (prec == OP_FP64) return x;
    if (prec == OP_DROP) return 0.0;
    if (fmt_params(prec, &p, &emin, &maxf, &ebits, &bias)) return NAN;
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);          /* |x| = f 2^e, f in [1/2, 1) */
    int lead = e - 1;      /* 2^lead <= |x| < 2^(lead+1) */
    if (lead < emin) lead = emin;           /* subnormal range: fixed spacing */
    double q = ldexp(1.0, lead - (p - 1));  /* spacing of the format near x */
    double r = nearbyint(x / q) * q;        /* x / q is exact: q is a power of 2 */
    if (fabs(r) > maxf) return copysign(INFINITY, x);
    return r;
}

/* value of a bit pattern of the format (sign, biased exponent, fraction) */
double orc_decode(int prec, uint32_t code) {
    int p, emin, ebits, bias;
    double maxf;
    if (fmt_params(prec, &p, &emin, &maxf, &ebits, &bias)) return NAN;
    int fbits = p - 1;
    uint32_t frac = code & ((1u << fbits) - 1u);
    uint32_t ex = (code >> fbits) & ((1u << ebits) - 1u);
    int sign = (code >> (fbits + ebits)) & 1u;
    double v;
    if (prec == OP_FP8) {
        /* E4M3FN: no infinities, NaN only at exponent 1111 with fraction 111 */
        if (ex == 15u && frac == 7u) return NAN;
    } else if (ex == (1u << ebits) - 1u) {
        v = frac ? NAN : INFINITY;
        return sign ? -v : v;
    }
    if (ex == 0u)
        v = ldexp((double)frac, emin - fbits);
    else
        v = ldexp(1.0 + ldexp((double)frac, -fbits), (int)ex - bias);
    return sign ? -v : v;
}

/* bit pattern of orc_round(prec, x) */
uint32_t orc_encode(int prec, double x) {
    int p, emin, ebits, bias;
    double maxf;
    if (fmt_params(prec, &p, &emin, &maxf, &ebits, &bias)) return 0;
    int fbits = p - 1;
    double r = orc_round(prec, x);
    uint32_t sign = signbit(r) ? 1u : 0u;
    uint32_t code;
    double a = fabs(r);
    if (isnan(r)) {
        code = (prec == OP_FP8) ? 0x7Fu : ((((1u << ebits) - 1u) << fbits) | (1u << (fbits - 1)));
    } else if (isinf(r)) {
        code = (prec == OP_FP8) ? 0x7Fu : (((1u << ebits) - 1u) << fbits);
    } else if (a == 0.0) {
        code = 0;
    } else {
        int e;
        frexp(a, &e);
        int lead = e - 1;
        if (lead < emin) { /* subnormal */
            code = (uint32_t)ldexp(a, fbits - emin);
        } else {
            uint32_t fr = (uint32_t)(ldexp(a, fbits - lead) - ldexp(1.0, fbits));
            code = ((uint32_t)(lead + bias) << fbits) | fr;
        }
    }
    return code | (sign << (fbits + ebits));
}

/* element-wise helpers over arrays (for exhaustive format tests) */
void orc_round_array(int prec, int64_t n, const double *x, double *y) {
    for (int64_t i = 0; i < n; i++) y[i] = orc_round(prec, x[i]);
}
void orc_encode_array(int prec, int64_t n, const double *x, uint32_t *c) {
    for (int64_t i = 0; i < n; i++) c[i] = orc_encode(prec, x[i]);
}
void orc_decode_array(int prec, int64_t n, const uint32_t *c, double *x) {
    for (int64_t i = 0; i < n; i++) x[i] = orc_decode(prec, c[i]);
}

/* storage bytes of one value in the format (values only) */
static double fmt_bytes(int prec, double drop_bytes) {
    switch (prec) {
    case OP_FP64: return 8; case OP_FP32: return 4; case OP_FP16: return 2;
    case OP_BF16: return 2; case OP_FP8: return 1; case OP_DROP: return drop_bytes;
    }
    return 0;
}

/* Storage of the bucketed M as a percentage of storing all nnz entries in
 * u_1 (the "str." column of Tables 3 and 4).  drop_bytes charges entries of
 * the u = 1 bucket; with_index adds a 4-byte column index to every stored
 * entry. */
double orc_storage_pct(const int64_t *counts, const int *precs, int q, double drop_bytes, int with_index) {
    double num = 0, tot = 0;
    for (int k = 0; k < q; k++) {
        double b = fmt_bytes(precs[k], drop_bytes);
        if (with_index && precs[k] != OP_DROP) b += 4;
        num += (double)counts[k] * b;
        tot += (double)counts[k];
    }
    double b1 = fmt_bytes(precs[0], drop_bytes) + (with_index ? 4 : 0);
    return tot > 0 ? 100.0 * num / (tot * b1) : 100.0;
}

/* ------------------------------------------------------------------------
 * Householder least squares: min || b - A x ||_2 for a dense m x n matrix,
 * m >= n, column-major with leading dimension m; A and b are overwritten.
 * Unpivoted Householder QR (reflector v = a + sign(a_1)||a|| e_1), then
 * x = R^{-1} (Q^T b)(1:n).  Used for the reduced problem of the SPAI
 * construction (Section 2.2, eq. (redprob)).
 * Returns ORC_ERANK when some |r_cc| <= n u ||A||_F.
 * ---------------------------------------------------------------------- */
/* Householder least squares with every elementary operation (+, -, *, /,
 * sqrt) rounded to precision `prec` (FP64: plain double arithmetic), sums
 * taken left to right: the QR factorisation "in u_f" of Section 2.2.  Every
 * operation on two u_f numbers done in FP64 and then rounded is correctly
 * rounded in u_f for fp32 and fp16 (53 >= 2p + 2 bits).  A rank-deficiency
 * test uses n u_f ||A||_F; a non-finite result (overflow in u_f) is ENAN. */
int orc_householder_ls_prec(int m, int n, double *A, double *b, double *x, int prec) {
#define R_(v) orc_round(prec, (v))
    if (m < n || n <= 0) return ORC_ERANK;
    double fro = 0;
    for (int j = 0; j < n; j++)
        for (int i = 0; i < m; i++) fro = R_(fro + R_(A[i + (size_t)j * m] * A[i + (size_t)j * m]));
    fro = R_(sqrt(fro));
    if (!isfinite(fro)) return ORC_ENAN;  /* an entry or ||A||_F overflows u_f */
    double *v = (double *)malloc(sizeof(double) * (size_t)m);
    if (!v) return ORC_ENOMEM;
    int status = ORC_OK;
    for (int c = 0; c < n; c++) {
        double *col = A + (size_t)c * m;
        double nrm2 = 0;
        for (int i = c; i < m; i++) nrm2 = R_(nrm2 + R_(col[i] * col[i]));
        double nrm = R_(sqrt(nrm2));
        if (nrm == 0.0) { status = ORC_ERANK; break; }
        double alpha = col[c];
        double beta = -copysign(nrm, alpha);
        int len = m - c;
        for (int i = 0; i < len; i++) v[i] = col[c + i];
        v[0] = R_(alpha - beta);
        double vtv = 0;
        for (int i = 0; i < len; i++) vtv = R_(vtv + R_(v[i] * v[i]));
        /* apply H = I - 2 v v^T / (v^T v) to the trailing columns and to b */
        for (int j = c + 1; j < n; j++) {
            double *cj = A + (size_t)j * m + c;
            double w = 0;
            for (int i = 0; i < len; i++) w = R_(w + R_(v[i] * cj[i]));
            double f = R_(2.0 * w / vtv);
            for (int i = 0; i < len; i++) cj[i] = R_(cj[i] - R_(f * v[i]));
        }
        {
            double w = 0;
            for (int i = 0; i < len; i++) w = R_(w + R_(v[i] * b[c + i]));
            double f = R_(2.0 * w / vtv);
            for (int i = 0; i < len; i++) b[c + i] = R_(b[c + i] - R_(f * v[i]));
        }
        col[c] = beta;
        for (int i = c + 1; i < m; i++) col[i] = 0.0;
        if (fabs(beta) <= (double)n * orc_unit_roundoff(prec) * fro) { status = ORC_ERANK; break; }
    }
    if (status == ORC_OK) {
        for (int c = n - 1; c >= 0; c--) {
            double s = b[c];
            for (int j = c + 1; j < n; j++) s = R_(s - R_(A[c + (size_t)j * m] * x[j]));
            x[c] = R_(s / A[c + (size_t)c * m]);
            if (!isfinite(x[c])) { status = ORC_ENAN; break; }
        }
    }
    free(v);
    return status;
#undef R_
}

int orc_householder_ls(int m, int n, double *A, double *b, double *x) {
    return orc_householder_ls_prec(m, n, A, b, x, OP_FP64);
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static int find_sorted(const int *a, int len, int key) {
    int lo = 0, hi = len - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (a[mid] == key) return mid;
        if (a[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------
 * SPAI on a fixed pattern, run on A^T and transposed (Algorithm 4 step 1
 * with Algorithm 1's least-squares solve and no pattern augmentation; the
 * reduced problem of eq. (redprob)).
 *
 * Row k of M is column k of the SPAI of A^T:  J = pattern row k (sorted),
 * I = { i : sum_{j in J} |a_{ji}| != 0 } (the shadow of J in A^T),
 * Abar(l, c) = a_{J_c, I_l}, ebar = e_k(I), mbar = argmin ||ebar - Abar m||,
 * M(k, J) = mbar.  With `scale` set, the columns of A^T are first scaled by
 * d_j = 1 / max_l |a_{jl}| and M(k, j) = mbar_j d_j (the one-sided scaling
 * of Section 4).
 *
 * uf is the construction precision u_f (Section 4's settings use double,
 * single and half): each entry of Abar is a_{J_c, I_l} d_j computed in FP64
 * and rounded once to u_f, the least squares runs with every operation in
 * u_f (orc_householder_ls_prec), and M(k, j) is mbar_j d_j computed in FP64
 * and rounded once to u_f.  orc_spai is uf = FP64.
 *
 * rows/nrows select a subset of rows (NULL: all).  On failure bad_row gets
 * the first failing row and the status is ORC_EZEROROW (k not in I: the
 * zero-row case of Section 4), ORC_ERANK or ORC_ENAN (overflow in u_f).
 * ---------------------------------------------------------------------- */
int orc_spai_prec(int n, const int *Arp, const int *Aci, const double *Av,
                  const int *Prp, const int *Pci, double *Mv,
                  const int *rows, int nrows, int scale, int uf, int *bad_row) {
    int status = ORC_OK;
    int first_bad = n;
    int count = rows ? nrows : n;
    double *dscale = NULL;
    if (scale) {
        dscale = (double *)malloc(sizeof(double) * (size_t)n);
        for (int j = 0; j < n; j++) {
            double mx = 0;
            for (int e = Arp[j]; e < Arp[j + 1]; e++) mx = fmax(mx, fabs(Av[e]));
            dscale[j] = mx > 0 ? 1.0 / mx : 1.0;
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int t = 0; t < count; t++) {
        int k = rows ? rows[t] : t;
        int nJ = Prp[k + 1] - Prp[k];
        const int *J = Pci + Prp[k];
        int cand = 0;
        for (int c = 0; c < nJ; c++) cand += Arp[J[c] + 1] - Arp[J[c]];
        int *I = (int *)malloc(sizeof(int) * (size_t)(cand > 0 ? cand : 1));
        int nI = 0;
        for (int c = 0; c < nJ; c++)
            for (int e = Arp[J[c]]; e < Arp[J[c] + 1]; e++)
                if (Av[e] != 0.0) I[nI++] = Aci[e];
        qsort(I, (size_t)nI, sizeof(int), cmp_int);
        int u = 0;
        for (int l = 0; l < nI; l++)
            if (u == 0 || I[l] != I[u - 1]) I[u++] = I[l];
        nI = u;
        for (int c = 0; c < nJ; c++) Mv[Prp[k] + c] = 0.0;
        int st = ORC_OK;
        if (find_sorted(I, nI, k) < 0) {
            st = ORC_EZEROROW;
        } else if (nI < nJ) {
            st = ORC_ERANK;
        } else {
            double *Ab = (double *)calloc((size_t)nI * nJ, sizeof(double));
            double *eb = (double *)calloc((size_t)nI, sizeof(double));
            double *m = (double *)calloc((size_t)nJ, sizeof(double));
            for (int c = 0; c < nJ; c++) {
                double dj = scale ? dscale[J[c]] : 1.0;
                for (int e = Arp[J[c]]; e < Arp[J[c] + 1]; e++) {
                    if (Av[e] == 0.0) continue;
                    int l = find_sorted(I, nI, Aci[e]);
                    Ab[l + (size_t)c * nI] = orc_round(uf, Av[e] * dj);
                }
            }
            eb[find_sorted(I, nI, k)] = 1.0;
            st = orc_householder_ls_prec(nI, nJ, Ab, eb, m, uf);
            if (st == ORC_OK)
                for (int c = 0; c < nJ; c++) Mv[Prp[k] + c] = orc_round(uf, m[c] * (scale ? dscale[J[c]] : 1.0));
            free(Ab); free(eb); free(m);
        }
        free(I);
        if (st != ORC_OK) {
#pragma omp critical
            {
                if (status == ORC_OK || k < first_bad) { status = st; first_bad = k; }
            }
        }
    }
    free(dscale);
    if (bad_row) *bad_row = (status == ORC_OK) ? -1 : first_bad;
    return status;
}

int orc_spai(int n, const int *Arp, const int *Aci, const double *Av,
             const int *Prp, const int *Pci, double *Mv,
             const int *rows, int nrows, int scale, int *bad_row) {
    return orc_spai_prec(n, Arp, Aci, Av, Prp, Pci, Mv, rows, nrows, scale, OP_FP64, bad_row);
}

/* ------------------------------------------------------------------------
 * Adaptive SPAI: Algorithm 1 with its augmentation loop, run on A^T (row k
 * of M is column k of SPAI(A^T), as in orc_spai).  Row k starts from
 * J_k = J0(k,:) (the identity when J0rp is NULL) and for step = 0..alpha:
 *   - I_k is the shadow of J_k (the nonzero columns of the rows j in J_k of
 *     A); the least squares problem (redprob) with Abar = A(J_k, I_k)^T is
 *     solved by Householder QR from scratch (the QR update of the paper gives
 *     the same solution up to rounding);
 *   - s = Abar m - e_k(I_k) is the residual; the row is done when
 *     ||s||_2 <= eps or after the last solve (step = alpha);
 *   - L_k holds the rows l of I_k with s(l) != 0, "nonzero" meaning
 *     |s(l)| > 2^-40 (||e_k|| = 1: where the fit is exact, s(l) is rounding
 *     noise whose exact zeros depend on the summation order); the candidates
 *     are the j with a_jl != 0 for some l in L_k (column l of A), minus J_k;
 *   - for a candidate j, rho_j^2 = ||s||^2 - (s . a_j)^2 / ||a_j||^2, with
 *     a_j the whole row j of A (as a vector over l): the residual norm
 *     after adding j alone with its best coefficient;
 *   - rho_j is compared after rounding to fp32, the mean is the FP64 sum of
 *     the rounded values in ascending j divided by the number of candidates;
 *     the candidates with rho_j <= mean, ordered by (rho_j, j), join J_k up
 *     to beta of them (J_k is kept sorted).  No candidate left: the row is
 *     done.
 * Out: cnt[k] = |J_k|, its columns (ascending) and values at k*jmax ..,
 * steps[k] = least squares solves made.  |J_k| never exceeds jmax (further
 * candidates are not added).  Errors as orc_spai (EZEROROW, ERANK).
 * ---------------------------------------------------------------------- */
typedef struct { float rho; int j; } orc_cand;

static int cmp_cand(const void *a, const void *b) {
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    if (x->rho != y->rho) return (x->rho > y->rho) - (x->rho < y->rho);
    return (x->j > y->j) - (x->j < y->j);
}

/* With a construction precision uf (Section 4's single and half settings,
 * orc_spai_adaptive_prec) every least squares solve is that of orc_spai_prec:
 * the reduced matrix a_{J_c, I_l} d_{J_c} rounded to uf (d from the optional
 * column scaling of A^T), Householder QR and back substitution in uf, and
 * M(k, J_c) = m_c d_{J_c} rounded to uf.  The residual s and the candidate
 * scores are then formed in FP64 from the unscaled A and those rounded
 * values, so the pattern decisions see the uf solution but add no rounding
 * of their own.  uf = FP64 without scaling is orc_spai_adaptive. */
int orc_spai_adaptive_prec(int n, const int *Arp, const int *Aci, const double *Av,
                           const int *ATrp, const int *ATci, const int *J0rp, const int *J0ci,
                           int alpha, int beta, double eps, int jmax, int scale, int uf,
                           int *cnt, int *cols, double *vals, int *steps, int *bad_row) {
    int status = ORC_OK;
    int first_bad = n;
    const int plain = uf == OP_FP64 && !scale;
    double *dscale = NULL;
    if (scale) {
        dscale = (double *)malloc(sizeof(double) * (size_t)n);
        for (int j = 0; j < n; j++) {
            double mx = 0;
            for (int e = Arp[j]; e < Arp[j + 1]; e++) mx = fmax(mx, fabs(Av[e]));
            dscale[j] = mx > 0 ? 1.0 / mx : 1.0;
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < n; k++) {
        int *J = (int *)malloc(sizeof(int) * (size_t)jmax);
        int nJ = 0;
        if (J0rp) {
            for (int e = J0rp[k]; e < J0rp[k + 1] && nJ < jmax; e++) J[nJ++] = J0ci[e];
            qsort(J, (size_t)nJ, sizeof(int), cmp_int);
        } else {
            J[nJ++] = k;
        }
        int st = ORC_OK, nsolve = 0;
        double *m = NULL;
        for (int step = 0; step <= alpha; step++) {
            /* shadow */
            int cap = 0;
            for (int c = 0; c < nJ; c++) cap += Arp[J[c] + 1] - Arp[J[c]];
            int *I = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
            int nI = 0;
            for (int c = 0; c < nJ; c++)
                for (int e = Arp[J[c]]; e < Arp[J[c] + 1]; e++)
                    if (Av[e] != 0.0) I[nI++] = Aci[e];
            qsort(I, (size_t)nI, sizeof(int), cmp_int);
            int u = 0;
            for (int l = 0; l < nI; l++)
                if (u == 0 || I[l] != I[u - 1]) I[u++] = I[l];
            nI = u;
            const int kpos = find_sorted(I, nI, k);
            if (kpos < 0) { st = ORC_EZEROROW; free(I); break; }
            if (nI < nJ) { st = ORC_ERANK; free(I); break; }
            double *Ab = (double *)calloc((size_t)nI * nJ, sizeof(double));
            double *A0 = (double *)calloc((size_t)nI * nJ, sizeof(double));
            double *eb = (double *)calloc((size_t)nI, sizeof(double));
            free(m);
            m = (double *)calloc((size_t)nJ, sizeof(double));
            for (int c = 0; c < nJ; c++) {
                const double dj = scale ? dscale[J[c]] : 1.0;
                for (int e = Arp[J[c]]; e < Arp[J[c] + 1]; e++) {
                    if (Av[e] == 0.0) continue;
                    const size_t at = find_sorted(I, nI, Aci[e]) + (size_t)c * nI;
                    A0[at] = Av[e];
                    Ab[at] = plain ? Av[e] : orc_round(uf, Av[e] * dj);
                }
            }
            eb[kpos] = 1.0;
            st = plain ? orc_householder_ls(nI, nJ, Ab, eb, m) : orc_householder_ls_prec(nI, nJ, Ab, eb, m, uf);
            nsolve++;
            if (st != ORC_OK) { free(Ab); free(A0); free(eb); free(I); break; }
            if (!plain)
                for (int c = 0; c < nJ; c++) m[c] = orc_round(uf, m[c] * (scale ? dscale[J[c]] : 1.0));
            /* residual on the shadow */
            double *sv = (double *)malloc(sizeof(double) * (size_t)nI);
            double ns2 = 0.0;
            for (int l = 0; l < nI; l++) {
                double t = 0.0;
                for (int c = 0; c < nJ; c++) t += A0[l + (size_t)c * nI] * m[c];
                sv[l] = t - (l == kpos ? 1.0 : 0.0);
                ns2 += sv[l] * sv[l];
            }
            free(Ab); free(A0); free(eb);
            int done = sqrt(ns2) <= eps || step == alpha;
            if (!done) {
                /* candidates: columns l of A over the residual's support */
                int ccap = 0;
                for (int l = 0; l < nI; l++)
                    if (fabs(sv[l]) > 0x1p-40) ccap += ATrp[I[l] + 1] - ATrp[I[l]];
                int *C = (int *)malloc(sizeof(int) * (size_t)(ccap > 0 ? ccap : 1));
                int nC = 0;
                for (int l = 0; l < nI; l++)
                    if (fabs(sv[l]) > 0x1p-40)
                        for (int e = ATrp[I[l]]; e < ATrp[I[l] + 1]; e++) C[nC++] = ATci[e];
                qsort(C, (size_t)nC, sizeof(int), cmp_int);
                u = 0;
                for (int t = 0; t < nC; t++)
                    if ((u == 0 || C[t] != C[u - 1]) && find_sorted(J, nJ, C[t]) < 0) C[u++] = C[t];
                nC = u;
                orc_cand *cd = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(nC > 0 ? nC : 1));
                double sum = 0.0;
                for (int t = 0; t < nC; t++) {
                    const int j = C[t];
                    double dot = 0.0, nrm = 0.0;
                    for (int e = Arp[j]; e < Arp[j + 1]; e++) {
                        const int l = find_sorted(I, nI, Aci[e]);
                        if (l >= 0) dot += sv[l] * Av[e];
                        nrm += Av[e] * Av[e];
                    }
                    double r2 = nrm > 0.0 ? ns2 - dot * dot / nrm : ns2;
                    cd[t].rho = (float)sqrt(r2 > 0.0 ? r2 : 0.0);
                    cd[t].j = j;
                    sum += (double)cd[t].rho;
                }
                int nacc = 0;
                if (nC > 0) {
                    const double mean = sum / nC;
                    for (int t = 0; t < nC; t++)
                        if ((double)cd[t].rho <= mean) cd[nacc++] = cd[t];
                    qsort(cd, (size_t)nacc, sizeof(orc_cand), cmp_cand);
                }
                int add = nacc < beta ? nacc : beta;
                if (add > jmax - nJ) add = jmax - nJ;
                for (int t = 0; t < add; t++) J[nJ++] = cd[t].j;
                qsort(J, (size_t)nJ, sizeof(int), cmp_int);
                free(cd); free(C);
                if (add == 0) done = 1;
                else { free(m); m = NULL; }  /* J changed: solve again */
            }
            free(sv); free(I);
            if (done) break;
        }
        cnt[k] = nJ;
        steps[k] = nsolve;
        for (int c = 0; c < nJ; c++) {
            cols[(size_t)k * jmax + c] = J[c];
            vals[(size_t)k * jmax + c] = (st == ORC_OK && m) ? m[c] : 0.0;
        }
        free(m); free(J);
        if (st != ORC_OK) {
#pragma omp critical
            {
                if (status == ORC_OK || k < first_bad) { status = st; first_bad = k; }
            }
        }
    }
    free(dscale);
    if (bad_row) *bad_row = (status == ORC_OK) ? -1 : first_bad;
    return status;
}

int orc_spai_adaptive(int n, const int *Arp, const int *Aci, const double *Av,
                      const int *ATrp, const int *ATci, const int *J0rp, const int *J0ci,
                      int alpha, int beta, double eps, int jmax,
                      int *cnt, int *cols, double *vals, int *steps, int *bad_row) {
    return orc_spai_adaptive_prec(n, Arp, Aci, Av, ATrp, ATci, J0rp, J0ci, alpha, beta, eps, jmax, 0, OP_FP64, cnt,
                                  cols, vals, steps, bad_row);
}

/* ------------------------------------------------------------------------
 * ||M||_inf = max_i sum_j |m_ij| (the default norm of Section 2.1), each row
 * summed left to right in CSR order.
 * ---------------------------------------------------------------------- */
double orc_norm_inf(int n, const int *rp, const double *v) {
    double mx = 0;
    for (int i = 0; i < n; i++) {
        double s = 0;
        for (int e = rp[i]; e < rp[i + 1]; e++) s += fabs(v[e]);
        if (s > mx) mx = s;
    }
    return mx;
}

/* ceil(log2 t) for t > 0 */
static int ceil_log2(double t) {
    int e;
    double f = frexp(t, &e);
    return (f == 0.5) ? e - 1 : e;
}

/* ------------------------------------------------------------------------
 * Bucketing (Algorithm 2, intervals of eq. (nint)) plus the stored values.
 *
 * precs[0..q-1] are sorted so that u_1 < ... < u_q.  With t_k = fl(eps ||M||) / u_k
 * (an exact power-of-two division), an entry a goes to bucket 1 if |a| > t_2,
 * to bucket q if |a| <= t_q, otherwise to the k with t_{k+1} < |a| <= t_k.
 * q = 1 puts everything in bucket 1.
 *
 * Stored value (range handling for the narrow formats, not in the paper):
 * mt = round_k(a / s_k) s_k with the power-of-two scale
 * s_k = 2^(ceil(log2 t_k) - E_k), E_k = 15 for fp16, 8 for fp8, s_k = 1 for
 * the other formats; bucket 1 uses t_1 = max |a| for its scale.  Entries of a
 * u = 1 bucket store 0 (they are dropped).
 *
 * Outputs: bucket[e] in 0..q-1, mt[e], t[q], s[q], counts[q].
 * ---------------------------------------------------------------------- */
int orc_bucketize(int n, const int *rp, const double *v, double eps, const int *precs, int q,
                  signed char *bucket, double *mt, double *t, double *s, int64_t *counts) {
    if (q < 1 || q > 6) return ORC_EINVAL;
    for (int k = 1; k < q; k++)
        if (!(orc_unit_roundoff(precs[k - 1]) < orc_unit_roundoff(precs[k]))) return ORC_EINVAL;
    for (int k = 0; k < q - 1; k++)
        if (precs[k] == OP_DROP) return ORC_EINVAL;
    double normM = orc_norm_inf(n, rp, v);
    double base = eps * normM;
    int64_t nnz = rp[n];
    for (int k = 0; k < q; k++) t[k] = base / orc_unit_roundoff(precs[k]);
    for (int k = 0; k < q; k++) counts[k] = 0;
    double maxabs = 0;
    for (int64_t e = 0; e < nnz; e++) maxabs = fmax(maxabs, fabs(v[e]));
    for (int64_t e = 0; e < nnz; e++) {
        double a = fabs(v[e]);
        int b;
        if (q == 1) b = 0;
        else if (a > t[1]) b = 0;
        else if (a <= t[q - 1]) b = q - 1;
        else {
            b = -1;
            for (int k = 1; k <= q - 2; k++)
                if (a > t[k + 1] && a <= t[k]) { b = k; break; }
        }
        bucket[e] = (signed char)b;
        counts[b]++;
    }
    for (int k = 0; k < q; k++) {
        int pk = precs[k];
        double tk = (k == 0) ? maxabs : t[k];
        if ((pk == OP_FP16 || pk == OP_FP8) && tk > 0)
            s[k] = ldexp(1.0, ceil_log2(tk) - (pk == OP_FP16 ? 15 : 8));
        else
            s[k] = 1.0;
    }
    for (int64_t e = 0; e < nnz; e++) {
        int k = bucket[e];
        mt[e] = (precs[k] == OP_DROP) ? 0.0 : orc_round(precs[k], v[e] / s[k]) * s[k];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Bucketed product y = M_b x (Algorithm 3 with storage and compute precision
 * decoupled, as the conclusions propose): per row, the partial sums
 * y_i^(k) = sum_{j in B_ik} mt_ij x_j in FP64 in CSR order, then
 * y_i = sum over k = q..1 of y_i^(k) in FP64, rounded to out_prec.
 * ---------------------------------------------------------------------- */
void orc_apply(int n, const int *rp, const int *ci, const double *mt, const signed char *bucket, int q,
               const double *x, double *y, int out_prec) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double part[6] = {0, 0, 0, 0, 0, 0};
        for (int e = rp[i]; e < rp[i + 1]; e++) part[bucket[e]] += mt[e] * x[ci[e]];
        double acc = 0;
        for (int k = q - 1; k >= 0; k--) acc += part[k];
        y[i] = orc_round(out_prec, acc);
    }
}

/* Transpose of a CSR matrix with values and bucket ids, entries of each
 * output row in increasing source-row order. */
void orc_transpose(int n, const int *rp, const int *ci, const double *v, const signed char *bk,
                   int *trp, int *tci, double *tv, signed char *tbk) {
    for (int i = 0; i <= n; i++) trp[i] = 0;
    for (int e = 0; e < rp[n]; e++) trp[ci[e] + 1]++;
    for (int i = 0; i < n; i++) trp[i + 1] += trp[i];
    int *pos = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; i++) pos[i] = trp[i];
    for (int i = 0; i < n; i++)
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            int p = pos[ci[e]]++;
            tci[p] = i;
            if (tv) tv[p] = v[e];
            if (tbk) tbk[p] = bk[e];
        }
    free(pos);
}

/* Algorithm 3 as printed: the partial sum of bucket k is accumulated in
 * precision u_k (each product and each addition rounded to u_k, the way the
 * chop emulation of Section 4 rounds), the partials are then summed in u_1
 * for k = q..1.  Entries of a u = 1 bucket are skipped. */
void orc_apply_paper(int n, const int *rp, const int *ci, const double *mt, const signed char *bucket,
                     const int *precs, int q, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double part[6] = {0, 0, 0, 0, 0, 0};
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            int k = bucket[e];
            if (precs[k] == OP_DROP) continue;
            double prod = orc_round(precs[k], mt[e] * x[ci[e]]);
            part[k] = orc_round(precs[k], part[k] + prod);
        }
        double acc = 0;
        for (int k = q - 1; k >= 0; k--) acc = orc_round(precs[0], acc + part[k]);
        y[i] = acc;
    }
}

/* y = fl_p(A_p x): values rounded to precision p (u_p of Algorithm 4), the
 * product accumulated in FP64 and rounded to out_prec. */
void orc_spmv(int n, const int *rp, const int *ci, const double *v, int val_prec,
              const double *x, double *y, int out_prec) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double acc = 0;
        for (int e = rp[i]; e < rp[i + 1]; e++) acc += orc_round(val_prec, v[e]) * x[ci[e]];
        y[i] = orc_round(out_prec, acc);
    }
}

/* ------------------------------------------------------------------------
 * Refinement residual r = b - A x (Algorithm 4, "in precision u_r").
 * dd = 1: double-double accumulation (Dekker/Knuth TwoSum and TwoProd with
 * an exact FMA, compensated as in Ogita-Rump-Oishi Dot2), standing in for
 * the paper's quadruple precision; dd = 0: plain FP64.  Result stored FP64.
 * ---------------------------------------------------------------------- */
static inline void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

void orc_residual(int n, const int *rp, const int *ci, const double *v, const double *b,
                  const double *x, double *r, int dd) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        if (dd) {
            double s = b[i], c = 0, p, pe, se;
            for (int e = rp[i]; e < rp[i + 1]; e++) {
                two_prod(-v[e], x[ci[e]], &p, &pe);
                two_sum(s, p, &s, &se);
                c += pe + se;
            }
            r[i] = s + c;
        } else {
            double s = b[i];
            for (int e = rp[i]; e < rp[i + 1]; e++) s -= v[e] * x[ci[e]];
            r[i] = s;
        }
    }
}

static double vec_norm_inf(int n, const double *x) {
    double m = 0;
    for (int i = 0; i < n; i++) m = fmax(m, fabs(x[i]));
    return m;
}

/* ------------------------------------------------------------------------
 * Preconditioned MGS-GMRES in working precision u_g (Algorithm 4 step 5 and
 * Section 3).  The operator is z = M_b (A_p v) with A rounded to u_p and M
 * applied as its buckets (orc_apply); the vector operations (dots, axpys,
 * norms, scaling) are rounded to u_g after every operation, dot products are
 * sequential.  The Hessenberg matrix, Givens rotations and the projected
 * right-hand side are FP64; d = V y is formed in FP64.
 *
 * dot64 = 1 selects the other realisation of "vector operations in u_g" that
 * keeps the vectors in u_g: each dot product and squared norm is a sum of the
 * (exact) products of u_g numbers accumulated in FP64, h_ij, beta and
 * h_{j+1,j} stay FP64, and each axpy z - h v is formed with one FMA in FP64
 * and then rounded to u_g.  Sequential recursive summation in u_g has an
 * error bound growing with n u_g; this one stays near u_g, which is what a
 * reduction over FP64 partials gives.
 *
 * Left preconditioning (trans = 0): solves M A d = M r,  stop when
 * |g_{j+1}| <= tau ||M r||_2.
 * Right preconditioning on the transposed system (trans = 1, used by the
 * adjoint): solves A^T M^T w = r, d = M^T w,  stop when |g_{j+1}| <= tau ||r||_2.
 * In that case (rp, ci, v) and (mrp, mci, mt, mb) describe A^T and M^T.
 *
 * orth = 1 replaces modified Gram-Schmidt by classical Gram-Schmidt run
 * twice (CGS2, "twice is enough": Giraud, Langou, Rozloznik and van den
 * Eshof, Numer. Math. 101, 2005): each pass takes all coefficients
 * h_i = v_i . z against the same z, then forms z - sum_i h_i v_i (with
 * dot64: the sum in FP64 by FMAs in the order i = 0..j, rounded once to u_g;
 * otherwise each term subtracted in u_g); the Hessenberg column is the sum
 * of both passes' coefficients.  In exact arithmetic it is the same Arnoldi
 * process; it trades the j dependent reductions of MGS for two.
 *
 * Stops also on h_{j+1,j} = 0 (the Krylov space is invariant: exact
 * solution) or after max_it iterations.  V_out (n x (max_it+1), column-major)
 * and H_out ((max_it+1) x max_it, column-major) receive the Arnoldi basis and
 * Hessenberg matrix when non-NULL.
 * ---------------------------------------------------------------------- */
typedef struct {
    int ug, up;       /* working / operator precision (OP_FP32 or OP_FP64) */
    double tau;       /* relative tolerance */
    int max_it;       /* iteration cap (<= n) */
    int trans;        /* 0: left-preconditioned M A, 1: right-preconditioned A^T M^T */
    int dot64;        /* 1: dots and norms accumulated in FP64 (see above) */
    /* A applied bucketed too (eqs. (nbe2), (fe2)): CSR, stored values and
     * bucket ids of A (of A^T when trans), q buckets; arp_b NULL: A rounded
     * to u_p as above */
    const int *arp_b, *aci_b;
    const double *at_b;
    const signed char *ab_b;
    int qa;
    int orth;         /* 0: modified Gram-Schmidt (the paper's), 1: CGS2 */
} orc_gmres_opts;

static inline double wp(int prec, double x) {
    if (prec == OP_FP32) return (double)(float)x;
    return x;
}

int orc_gmres(int n, const int *rp, const int *ci, const double *v,
              const int *mrp, const int *mci, const double *mt, const signed char *mb, int q,
              const double *r, double *d, int *its_out, double *relres_out, const orc_gmres_opts *o,
              double *V_out, double *H_out) {
    int ug = o->ug, up = o->up, m = o->max_it;
    if (m > n) m = n;
    if (m < 1) m = 1;
    int ld = m + 1;
    double *V = (double *)malloc(sizeof(double) * (size_t)n * (m + 1));
    double *H = (double *)calloc((size_t)ld * m, sizeof(double));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *rr = (double *)malloc(sizeof(double) * (size_t)n);
    double *cg = (double *)calloc((size_t)m + 1, sizeof(double)); /* one CGS pass's coefficients */
    if (!V || !H || !cs || !sn || !g || !w || !z || !rr || !cg) return ORC_ENOMEM;

    /* right-hand side of the Krylov solve, in u_g */
    for (int i = 0; i < n; i++) rr[i] = wp(ug, r[i]);
    double *s = V; /* v_1 is built in place */
    if (o->trans == 0) {
        orc_apply(n, mrp, mci, mt, mb, q, rr, s, ug);
    } else {
        for (int i = 0; i < n; i++) s[i] = rr[i];
    }
    const int d64 = o->dot64;
    double acc = 0;
    if (d64) {
        for (int i = 0; i < n; i++) acc += s[i] * s[i];
    } else {
        for (int i = 0; i < n; i++) acc = wp(ug, acc + wp(ug, s[i] * s[i]));
    }
    double beta = d64 ? sqrt(acc) : wp(ug, sqrt(acc));
    for (int i = 0; i < n; i++) d[i] = 0.0;
    if (beta == 0.0) {
        *its_out = 0;
        if (relres_out) *relres_out = 0.0;
        free(V); free(H); free(cs); free(sn); free(g); free(w); free(z); free(rr); free(cg);
        return ORC_OK;
    }
    for (int i = 0; i < n; i++) s[i] = wp(ug, s[i] / beta);
    g[0] = beta;
    int k = 0;
    double res = beta;
    for (int j = 0; j < m; j++) {
        double *vj = V + (size_t)j * n;
        if (o->trans == 0) {
            if (o->arp_b) orc_apply(n, o->arp_b, o->aci_b, o->at_b, o->ab_b, o->qa, vj, w, ug);  /* w = A_b v_j */
            else orc_spmv(n, rp, ci, v, up, vj, w, ug);           /* w = A_p v_j */
            orc_apply(n, mrp, mci, mt, mb, q, w, z, ug);          /* z = M_b w   */
        } else {
            orc_apply(n, mrp, mci, mt, mb, q, vj, w, ug);         /* w = M_b^T v_j */
            if (o->arp_b) orc_apply(n, o->arp_b, o->aci_b, o->at_b, o->ab_b, o->qa, w, z, ug);   /* z = A_b^T w */
            else orc_spmv(n, rp, ci, v, up, w, z, ug);            /* z = A_p^T w   */
        }
        double *hj = H + (size_t)j * ld;
        if (o->orth == 1) {                                        /* CGS2 */
            for (int i = 0; i <= j; i++) hj[i] = 0.0;
            for (int pass = 0; pass < 2; pass++) {
                for (int i = 0; i <= j; i++) {
                    const double *vi = V + (size_t)i * n;
                    double h = 0;
                    if (d64) for (int l = 0; l < n; l++) h += vi[l] * z[l];
                    else for (int l = 0; l < n; l++) h = wp(ug, h + wp(ug, vi[l] * z[l]));
                    cg[i] = h;
                    hj[i] += h;
                }
                for (int l = 0; l < n; l++) {
                    double t = z[l];
                    if (d64) {
                        for (int i = 0; i <= j; i++) t = fma(-cg[i], V[(size_t)i * n + l], t);
                        z[l] = wp(ug, t);
                    } else {
                        for (int i = 0; i <= j; i++) t = wp(ug, t - wp(ug, cg[i] * V[(size_t)i * n + l]));
                        z[l] = t;
                    }
                }
            }
        } else
        for (int i = 0; i <= j; i++) {                             /* modified Gram-Schmidt */
            const double *vi = V + (size_t)i * n;
            double h = 0;
            if (d64) {
                for (int l = 0; l < n; l++) h += vi[l] * z[l];
                hj[i] = h;
                for (int l = 0; l < n; l++) z[l] = wp(ug, fma(-h, vi[l], z[l]));
            } else {
                for (int l = 0; l < n; l++) h = wp(ug, h + wp(ug, vi[l] * z[l]));
                hj[i] = h;
                for (int l = 0; l < n; l++) z[l] = wp(ug, z[l] - wp(ug, h * vi[l]));
            }
        }
        acc = 0;
        if (d64) {
            for (int l = 0; l < n; l++) acc += z[l] * z[l];
        } else {
            for (int l = 0; l < n; l++) acc = wp(ug, acc + wp(ug, z[l] * z[l]));
        }
        double hn = d64 ? sqrt(acc) : wp(ug, sqrt(acc));
        hj[j + 1] = hn;
        if (H_out) for (int i = 0; i <= j + 1; i++) H_out[(size_t)j * ld + i] = hj[i];
        if (hn != 0.0) {
            double *vn = V + (size_t)(j + 1) * n;
            for (int l = 0; l < n; l++) vn[l] = wp(ug, z[l] / hn);
        }
        /* apply the previous rotations to column j, then a new one */
        for (int i = 0; i < j; i++) {
            double a = hj[i], b = hj[i + 1];
            hj[i] = cs[i] * a + sn[i] * b;
            hj[i + 1] = -sn[i] * a + cs[i] * b;
        }
        {
            double a = hj[j], b = hj[j + 1];
            double rho = hypot(a, b);
            cs[j] = (rho == 0.0) ? 1.0 : a / rho;
            sn[j] = (rho == 0.0) ? 0.0 : b / rho;
            hj[j] = rho;
            hj[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
        }
        k = j + 1;
        res = fabs(g[j + 1]);
        if (res <= o->tau * beta || hn == 0.0) break;
    }
    /* y = R^{-1} g, d = V y (FP64) */
    double *y = (double *)calloc((size_t)k, sizeof(double));
    for (int i = k - 1; i >= 0; i--) {
        double t = g[i];
        for (int c = i + 1; c < k; c++) t -= H[(size_t)c * ld + i] * y[c];
        y[i] = t / H[(size_t)i * ld + i];
    }
    double *dv = (o->trans == 0) ? d : w;
    for (int l = 0; l < n; l++) {
        double t = 0;
        for (int c = 0; c < k; c++) t += V[(size_t)c * n + l] * y[c];
        dv[l] = t;
    }
    if (o->trans == 1) orc_apply(n, mrp, mci, mt, mb, q, w, d, OP_FP64); /* d = M_b^T (V y) */
    if (V_out) memcpy(V_out, V, sizeof(double) * (size_t)n * (k + 1));
    *its_out = k;
    if (relres_out) *relres_out = res / beta;
    free(y); free(V); free(H); free(cs); free(sn); free(g); free(w); free(z); free(rr); free(cg);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * BSPAI-GMRES-IR (Algorithm 4).
 *
 * x_0 = M b with the unbucketed FP64 M (x0_mode 0), with the buckets
 * (x0_mode 1), x_0 = 0 (x0_mode 2) or the x_0 the caller left in x
 * (x0_mode 3).  Each refinement step: r = b - A x in
 * u_r (double-double when ur_dd, else FP64), stored FP64; the normwise
 * backward error eta = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) and
 * rho = ||r||_inf / ||b||_inf are recorded; then GMRES (orc_gmres) gives d
 * and x = x + d in FP64.
 *
 * The paper gives no stopping rule for the refinement loop; this one stops
 * when rho <= tol_rr (reason 1), eta <= tol_be (2), when the correction
 * stagnates: ||d_i||/||x_{i+1}|| > s ||d_{i-1}||/||x_i|| for i >= 1 (3; s = stag,
 * 0 meaning 0.5 and a negative value switching the test off), or
 * after i_max corrections (4, status ORC_ENOCONV).
 *
 * trans = 1 solves A^T x = b (the adjoint): the caller passes A^T as (rp,ci,v),
 * M^T as (mrp, mci, mt, mb) and the FP64 M^T as (frp, fci, fv); GMRES is then
 * right-preconditioned.
 * ---------------------------------------------------------------------- */
typedef struct {
    int ug, up, ur_dd;
    double tau, tol_rr, tol_be;
    int i_max, gmres_max, x0_mode, trans;
    int dot64;  /* GMRES dot products accumulated in FP64 (orc_gmres) */
    double stag;  /* stagnation ratio: 0 means 0.5, negative: no stagnation stop */
    const int *arp_b, *aci_b;  /* bucketed A for GMRES, as in orc_gmres_opts */
    const double *at_b;
    const signed char *ab_b;
    int qa;
    int orth;   /* Gram-Schmidt variant of GMRES, as in orc_gmres_opts */
} orc_ir_opts;

typedef struct {
    int steps, its_total, stop_reason, pad;
    int its[64];
    double eta[65];
    double relres[65];
} orc_ir_stats;

int orc_gmres_ir(int n, const int *rp, const int *ci, const double *v,
                 const int *frp, const int *fci, const double *fv,
                 const int *mrp, const int *mci, const double *mt, const signed char *mb, int q,
                 const double *b, double *x, const orc_ir_opts *o, orc_ir_stats *st) {
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !d) return ORC_ENOMEM;
    memset(st, 0, sizeof(*st));
    /* ||A||_inf */
    double normA = orc_norm_inf(n, rp, v); /* of A^T when trans = 1 */
    double normb = vec_norm_inf(n, b);
    if (o->x0_mode == 0) {
        orc_spmv(n, frp, fci, fv, OP_FP64, b, x, OP_FP64);
    } else if (o->x0_mode == 1) {
        orc_apply(n, mrp, mci, mt, mb, q, b, x, OP_FP64);
    } else if (o->x0_mode == 2) {
        for (int i = 0; i < n; i++) x[i] = 0.0;
    } /* x0_mode 3: x holds the caller's x_0 */
    orc_gmres_opts go = {o->ug, o->up, o->tau, o->gmres_max, o->trans, o->dot64,
                         o->arp_b, o->aci_b, o->at_b, o->ab_b, o->qa, o->orth};
    int status = ORC_OK, stagnated = 0;
    double dx_prev = 0;
    int i = 0;
    for (;;) {
        orc_residual(n, rp, ci, v, b, x, r, o->ur_dd);
        double nr = vec_norm_inf(n, r), nx = vec_norm_inf(n, x);
        double eta = nr / (normA * nx + normb);
        double rho = normb > 0 ? nr / normb : nr;
        if (i <= 64) { st->eta[i] = eta; st->relres[i] = rho; }
        if (!isfinite(nr)) { status = ORC_ENAN; st->stop_reason = 5; break; }
        if (rho <= o->tol_rr) { st->stop_reason = 1; break; }
        if (eta <= o->tol_be) { st->stop_reason = 2; break; }
        if (stagnated) { status = ORC_ESTAG; st->stop_reason = 3; break; }
        if (i >= o->i_max || i >= 64) { status = ORC_ENOCONV; st->stop_reason = 4; break; }
        int its = 0;
        int gs = orc_gmres(n, rp, ci, v, mrp, mci, mt, mb, q, r, d, &its, NULL, &go, NULL, NULL);
        if (gs != ORC_OK) { status = gs; break; }
        st->its[i] = its;
        st->its_total += its;
        for (int l = 0; l < n; l++) x[l] += d[l];
        double dx = vec_norm_inf(n, d) / vec_norm_inf(n, x);
        const double sr = o->stag == 0.0 ? 0.5 : o->stag;
        if (i >= 1 && sr > 0.0 && dx > sr * dx_prev) stagnated = 1;
        dx_prev = dx;
        i++;
    }
    st->steps = i;
    free(r);
    free(d);
    return status;
}
