/*
 * CPU oracle for threshold-detector click probabilities of zero-mean Gaussian
 * states.  TEST INFRASTRUCTURE ONLY: it exists to check the GPU library.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the library never calls it.  It shares no code, header or table with the
 * GPU path.
 *
 * What it computes (Sec. II of arXiv:1810.00900, "The Algorithm"):
 *   A click is the POVM element I - |0><0|, a difference of two Gaussian
 *   operators, so by linearity the probability of a pattern with clicked modes
 *   C, no-click modes N and unobserved modes U is a signed sum over the subsets
 *   Y of C of vacuum probabilities:
 *
 *       p(C, N) = sum_{Y subset of C} (-1)^{|Y|} P_vac(Y u N),
 *
 *   where the vacuum probability of a mode set A of a zero-mean state is the
 *   q_k of Eq. (prob) at zero mean.  With hbar = 1 (V = 2 sigma) the paper's
 *   2 / sqrt(det(V_B + 1)) equals det(sigma_Q[A])^{-1/2} with
 *   sigma_Q = sigma + I/2.  Unobserved modes are dropped (the marginal of a
 *   Gaussian state is its sub-covariance, as in the block split of Sec. II).
 *
 * Routes:
 *   form P  the definition above: one Cholesky of sigma_Q[Y u N] per subset.
 *   form S  the same sum after conditioning on vacuum at N once: the Schur
 *           complement Sigma_C = sigma_Q[C] - sigma_Q[C,N] sigma_Q[N]^-1 sigma_Q[N,C]
 *           (Eq. MatrixUpdate iterated over N), using
 *           det sigma_Q[Y u N] = det sigma_Q[N] * det Sigma_C[Y].
 *
 * Precision: the paper reports that quadruple precision is required for
 * accurate probabilities (Sec. III, "Memory"), so all arithmetic here is
 * IEEE binary128 (__float128, libquadmath).  Each term is an independent
 * unblocked Cholesky; subset sums are plain binary128 sums per thread, merged
 * in thread order (deterministic for a fixed thread count).
 *
 * Input conventions: sigma is 2m x 2m, row-major, interleaved (x1,p1,...),
 * hbar = 1; only the lower triangle (row >= column) is read.  pattern[i] is
 * 1 (click), 0 (no click) or -1 (unobserved).
 */
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 qf;

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOTPD = -2, OR_ETOOBIG = -3, OR_ENOMEM = -4 };

/* Results, all as doubles.  Quantities that need more than 53 bits are split
 * into (hi, lo) with hi + lo equal to the binary128 value to ~106 bits. */
typedef struct {
    double p_hi, p_lo;       /* p(C, N) */
    double t_hi, t_lo;       /* T = sum_Y (-1)^|Y| det(Sigma_C[Y])^-1/2 (form S), p / P_vac(N) */
    double abs_sum;          /* sum_Y P_vac(Y u N) (no signs), for the cancellation ratio */
    double pvac_n;           /* P_vac(N) */
    double n_terms;          /* number of subsets summed */
} oracle_result;

static inline double q_hi(qf x) { return (double)x; }
static inline double q_lo(qf x) { return (double)(x - (qf)(double)x); }

/* sigma_Q entry for global quadrature indices (ga, gb): lower triangle of
 * sigma plus 1/2 on the diagonal, formed exactly in binary128. */
static inline qf sigq(const double *cov, int m, int ga, int gb) {
    int r = ga > gb ? ga : gb;
    int c = ga > gb ? gb : ga;
    qf v = (qf)cov[(size_t)r * (size_t)(2 * m) + (size_t)c];
    if (ga == gb) v += (qf)0.5;
    return v;
}

/* In-place unblocked Cholesky of the k x k symmetric matrix A (row-major, full
 * storage, lower triangle used).  Returns 0 and sets *inv_sqrt_det =
 * prod_i 1/L_ii = det(A)^-1/2, or -1 if a pivot is not positive. */
static int chol_inv_sqrt_det(qf *A, int k, qf *inv_sqrt_det) {
    qf prod = 1;
    for (int j = 0; j < k; j++) {
        qf s = A[j * k + j];
        for (int t = 0; t < j; t++) s -= A[j * k + t] * A[j * k + t];
        if (!(s > 0)) return -1;
        qf ljj = sqrtq(s);
        A[j * k + j] = ljj;
        prod /= ljj;
        for (int i = j + 1; i < k; i++) {
            qf v = A[i * k + j];
            for (int t = 0; t < j; t++) v -= A[i * k + t] * A[j * k + t];
            A[i * k + j] = v / ljj;
        }
    }
    *inv_sqrt_det = prod;
    return 0;
}

static int validate(const double *cov, int m, const int8_t *pattern) {
    if (!cov || !pattern || m <= 0) return OR_EINVAL;
    for (int i = 0; i < m; i++)
        if (pattern[i] < -1 || pattern[i] > 1) return OR_EINVAL;
    for (size_t i = 0; i < (size_t)(4 * (size_t)m * m); i++) {
        double v = cov[i];
        if (v != v || v - v != 0) return OR_EINVAL; /* NaN or inf */
    }
    return OR_OK;
}

/* Sum over subsets Y = {Cidx[i] : bit i of mask} for masks
 * mask = begin + j*stride (j = 0..count-1, mask < 2^n), of sign * f(Y), where
 * f is computed by the callback-free inner routine below.  Thread partials are
 * merged in thread order. */

/* ---------------- form P ---------------- */

/* Displaced states (mean mu, hbar = 1, interleaved): the vacuum probability
 * of a mode set A becomes det(sigma_Q[A])^-1/2 exp(-mu_A^T sigma_Q[A]^-1 mu_A / 2),
 * the overlap of a Gaussian state with the vacuum (a coherent state |alpha>
 * gives exp(-|alpha|^2)).  Sec. II prints the exponent of q_k without the
 * factor 1/2 (hbar = 2 there); this follows the overlap formula.  With
 * sigma_Q[A] = L L^T the quadratic form is |L^-1 mu_A|^2. */
static qf mean_factor(const qf *L, int d, const qf *mu, qf *z) {
    qf s = 0;
    for (int i = 0; i < d; i++) {
        qf v = mu[i];
        for (int t = 0; t < i; t++) v -= L[i * d + t] * z[t];
        z[i] = v / L[i * d + i];
        s += z[i] * z[i];
    }
    return expq(-s / 2);
}

static int term_formP(const double *cov, const double *mean, int m, const int *cidx, int n,
                      const int *nidx, int nn, uint64_t mask, qf *work, qf *vec, int *modes,
                      qf *term) {
    int k = 0;
    /* Y u N in ascending mode order (the determinant does not depend on the
     * order as long as both quadratures of a mode move together). */
    int ci = 0, ni = 0;
    while (ci < n || ni < nn) {
        int takec;
        if (ci >= n) takec = 0;
        else if (ni >= nn) takec = 1;
        else takec = cidx[ci] < nidx[ni];
        if (takec) {
            if ((mask >> ci) & 1u) modes[k++] = cidx[ci];
            ci++;
        } else {
            modes[k++] = nidx[ni++];
        }
    }
    int d = 2 * k;
    for (int a = 0; a < d; a++)
        for (int b = 0; b <= a; b++) {
            int ga = 2 * modes[a / 2] + (a & 1);
            int gb = 2 * modes[b / 2] + (b & 1);
            qf v = sigq(cov, m, ga, gb);
            work[a * d + b] = v;
            work[b * d + a] = v;
        }
    if (k == 0) { *term = 1; return 0; }
    if (chol_inv_sqrt_det(work, d, term)) return -1;
    if (mean) {  /* vec holds 2d scalars: mu_A, then the solve */
        for (int a = 0; a < d; a++) vec[a] = (qf)mean[2 * modes[a / 2] + (a & 1)];
        *term *= mean_factor(work, d, vec, vec + d);
    }
    return 0;
}

static int split_pattern(int m, const int8_t *pattern, int **cidx, int *n, int **nidx, int *nn) {
    *cidx = (int *)malloc(sizeof(int) * (size_t)(m + 1));
    *nidx = (int *)malloc(sizeof(int) * (size_t)(m + 1));
    if (!*cidx || !*nidx) { free(*cidx); free(*nidx); return OR_ENOMEM; }
    *n = 0; *nn = 0;
    for (int i = 0; i < m; i++) {
        if (pattern[i] == 1) (*cidx)[(*n)++] = i;
        else if (pattern[i] == 0) (*nidx)[(*nn)++] = i;
    }
    return OR_OK;
}

/* Form P over a strided range of subset masks (the full sum is begin = 0,
 * stride = 1, count = 2^n).  threads <= 0 means the OpenMP default. */
int oracle_formP_mean_range(const double *cov, const double *mean, int m, const int8_t *pattern,
                            uint64_t begin, uint64_t stride, uint64_t count, int threads,
                            oracle_result *out) {
    int rc = validate(cov, m, pattern);
    if (rc) return rc;
    int *cidx, *nidx, n, nn;
    if ((rc = split_pattern(m, pattern, &cidx, &n, &nidx, &nn))) return rc;
    if (n > 40) { free(cidx); free(nidx); return OR_ETOOBIG; }
    int nthr = 1;
#ifdef _OPENMP
    nthr = threads > 0 ? threads : omp_get_max_threads();
#endif
    qf *part_s = (qf *)calloc((size_t)nthr, sizeof(qf));
    qf *part_a = (qf *)calloc((size_t)nthr, sizeof(qf));
    int *bad = (int *)calloc((size_t)nthr, sizeof(int));
    int dmax = 2 * (n + nn);
    int err = 0;
#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        qf *work = (qf *)malloc(sizeof(qf) * (size_t)(dmax > 0 ? dmax * dmax : 1));
        qf *vec = (qf *)malloc(sizeof(qf) * (size_t)(2 * dmax + 2));
        int *modes = (int *)malloc(sizeof(int) * (size_t)(n + nn + 1));
        qf s = 0, a = 0;
        int mybad = (!work || !modes || !vec);
        /* static contiguous chunks: thread t takes j in [lo, hi) */
        uint64_t lo = count * (uint64_t)tid / (uint64_t)nthr;
        uint64_t hi = count * (uint64_t)(tid + 1) / (uint64_t)nthr;
        for (uint64_t j = lo; j < hi && !mybad; j++) {
            uint64_t mask = begin + j * stride;
            if (n < 64) mask &= ((uint64_t)1 << n) - 1;
            qf t;
            if (term_formP(cov, mean, m, cidx, n, nidx, nn, mask, work, vec, modes, &t)) { mybad = 1; break; }
            if (__builtin_popcountll(mask) & 1) s -= t; else s += t;
            a += t;
        }
        part_s[tid] = s; part_a[tid] = a; bad[tid] = mybad;
        free(work); free(vec); free(modes);
    }
    qf S = 0, A = 0;
    for (int t = 0; t < nthr; t++) { S += part_s[t]; A += part_a[t]; err |= bad[t]; }
    free(part_s); free(part_a); free(bad);

    qf pvn = 1;
    if (!err && nn > 0) {
        /* P_vac(N) alone (the empty subset of C), for reporting */
        int *modes = (int *)malloc(sizeof(int) * (size_t)(nn + 1));
        qf *work = (qf *)malloc(sizeof(qf) * (size_t)(4 * nn * nn));
        qf *vec = (qf *)malloc(sizeof(qf) * (size_t)(4 * nn + 2));
        if (!modes || !work || !vec || term_formP(cov, mean, m, cidx, n, nidx, nn, 0, work, vec, modes, &pvn))
            err = 1;
        free(modes); free(work); free(vec);
    }
    free(cidx); free(nidx);
    if (err) return OR_ENOTPD;
    out->p_hi = q_hi(S); out->p_lo = q_lo(S);
    qf T = S / pvn;
    out->t_hi = q_hi(T); out->t_lo = q_lo(T);
    out->abs_sum = (double)A;
    out->pvac_n = (double)pvn;
    out->n_terms = (double)count;
    return OR_OK;
}

int oracle_formP_range(const double *cov, int m, const int8_t *pattern,
                       uint64_t begin, uint64_t stride, uint64_t count, int threads,
                       oracle_result *out) {
    return oracle_formP_mean_range(cov, NULL, m, pattern, begin, stride, count, threads, out);
}

/* Form P of a displaced state (mean: 2m doubles, hbar = 1, interleaved). */
int oracle_formP_mean(const double *cov, const double *mean, int m, const int8_t *pattern, int threads,
                      oracle_result *out) {
    int n = 0;
    if (!pattern || m <= 0 || !mean) return OR_EINVAL;
    for (int i = 0; i < 2 * m; i++)
        if (mean[i] != mean[i] || mean[i] - mean[i] != 0) return OR_EINVAL;
    for (int i = 0; i < m; i++) n += pattern[i] == 1;
    if (n > 40) return OR_ETOOBIG;
    return oracle_formP_mean_range(cov, mean, m, pattern, 0, 1, (uint64_t)1 << n, threads, out);
}

int oracle_formP(const double *cov, int m, const int8_t *pattern, int threads, oracle_result *out) {
    int n = 0;
    if (!pattern || m <= 0) return OR_EINVAL;
    for (int i = 0; i < m; i++) n += pattern[i] == 1;
    if (n > 40) return OR_ETOOBIG;
    return oracle_formP_range(cov, m, pattern, 0, 1, (uint64_t)1 << n, threads, out);
}

/* ---------------- form S ---------------- */

/* Sigma_C (2n x 2n, full storage, binary128) and P_vac(N) for a pattern:
 * Cholesky sigma_Q[N] = L L^T, W = L^-1 sigma_Q[N, C], Sigma_C = sigma_Q[C] - W^T W. */
static int condition_on_vacuum(const double *cov, int m, const int *cidx, int n,
                               const int *nidx, int nn, qf *sig_c, qf *pvac_n) {
    int dc = 2 * n, dn = 2 * nn;
    for (int a = 0; a < dc; a++)
        for (int b = 0; b <= a; b++) {
            qf v = sigq(cov, m, 2 * cidx[a / 2] + (a & 1), 2 * cidx[b / 2] + (b & 1));
            sig_c[a * dc + b] = v;
            sig_c[b * dc + a] = v;
        }
    *pvac_n = 1;
    if (nn == 0) return 0;
    qf *L = (qf *)malloc(sizeof(qf) * (size_t)dn * (size_t)dn);
    qf *W = (qf *)malloc(sizeof(qf) * (size_t)dn * (size_t)(dc > 0 ? dc : 1));
    if (!L || !W) { free(L); free(W); return -2; }
    for (int a = 0; a < dn; a++)
        for (int b = 0; b <= a; b++) {
            qf v = sigq(cov, m, 2 * nidx[a / 2] + (a & 1), 2 * nidx[b / 2] + (b & 1));
            L[(size_t)a * dn + b] = v;
            L[(size_t)b * dn + a] = v;
        }
    if (chol_inv_sqrt_det(L, dn, pvac_n)) { free(L); free(W); return -1; }
    /* forward substitution L W = sigma_Q[N, C] */
    for (int c = 0; c < dc; c++) {
        int gc = 2 * cidx[c / 2] + (c & 1);
        for (int i = 0; i < dn; i++) {
            qf v = sigq(cov, m, 2 * nidx[i / 2] + (i & 1), gc);
            for (int t = 0; t < i; t++) v -= L[(size_t)i * dn + t] * W[(size_t)t * dc + c];
            W[(size_t)i * dc + c] = v / L[(size_t)i * dn + i];
        }
    }
    for (int a = 0; a < dc; a++)
        for (int b = 0; b <= a; b++) {
            qf v = 0;
            for (int t = 0; t < dn; t++) v += W[(size_t)t * dc + a] * W[(size_t)t * dc + b];
            sig_c[a * dc + b] -= v;
            if (a != b) sig_c[b * dc + a] = sig_c[a * dc + b];
        }
    free(L); free(W);
    return 0;
}

int oracle_formS_range(const double *cov, int m, const int8_t *pattern,
                       uint64_t begin, uint64_t stride, uint64_t count, int threads,
                       oracle_result *out) {
    int rc = validate(cov, m, pattern);
    if (rc) return rc;
    int *cidx, *nidx, n, nn;
    if ((rc = split_pattern(m, pattern, &cidx, &n, &nidx, &nn))) return rc;
    if (n > 40) { free(cidx); free(nidx); return OR_ETOOBIG; }
    int dc = 2 * n;
    qf *sig_c = (qf *)malloc(sizeof(qf) * (size_t)(dc > 0 ? dc * dc : 1));
    qf pvn;
    if (!sig_c) { free(cidx); free(nidx); return OR_ENOMEM; }
    int crc = condition_on_vacuum(cov, m, cidx, n, nidx, nn, sig_c, &pvn);
    free(cidx); free(nidx);
    if (crc) { free(sig_c); return crc == -2 ? OR_ENOMEM : OR_ENOTPD; }

    int nthr = 1;
#ifdef _OPENMP
    nthr = threads > 0 ? threads : omp_get_max_threads();
#endif
    qf *part_s = (qf *)calloc((size_t)nthr, sizeof(qf));
    qf *part_a = (qf *)calloc((size_t)nthr, sizeof(qf));
    int *bad = (int *)calloc((size_t)nthr, sizeof(int));
#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        qf *work = (qf *)malloc(sizeof(qf) * (size_t)(dc > 0 ? dc * dc : 1));
        int sel[64];
        qf s = 0, a = 0;
        int mybad = !work;
        uint64_t lo = count * (uint64_t)tid / (uint64_t)nthr;
        uint64_t hi = count * (uint64_t)(tid + 1) / (uint64_t)nthr;
        for (uint64_t j = lo; j < hi && !mybad; j++) {
            uint64_t mask = begin + j * stride;
            if (n < 64) mask &= ((uint64_t)1 << n) - 1;
            int k = 0;
            for (int i = 0; i < n; i++)
                if ((mask >> i) & 1u) sel[k++] = i;
            int d = 2 * k;
            for (int x = 0; x < d; x++)
                for (int y = 0; y < d; y++)
                    work[x * d + y] = sig_c[(2 * sel[x / 2] + (x & 1)) * dc + 2 * sel[y / 2] + (y & 1)];
            qf t = 1;
            if (k > 0 && chol_inv_sqrt_det(work, d, &t)) { mybad = 1; break; }
            if (k & 1) s -= t; else s += t;
            a += t;
        }
        part_s[tid] = s; part_a[tid] = a; bad[tid] = mybad;
        free(work);
    }
    qf T = 0, A = 0;
    int err = 0;
    for (int t = 0; t < nthr; t++) { T += part_s[t]; A += part_a[t]; err |= bad[t]; }
    free(part_s); free(part_a); free(bad); free(sig_c);
    if (err) return OR_ENOTPD;
    qf P = pvn * T;
    out->p_hi = q_hi(P); out->p_lo = q_lo(P);
    out->t_hi = q_hi(T); out->t_lo = q_lo(T);
    out->abs_sum = (double)(pvn * A);
    out->pvac_n = (double)pvn;
    out->n_terms = (double)count;
    return OR_OK;
}

int oracle_formS(const double *cov, int m, const int8_t *pattern, int threads, oracle_result *out) {
    int n = 0;
    if (!pattern || m <= 0) return OR_EINVAL;
    for (int i = 0; i < m; i++) n += pattern[i] == 1;
    if (n > 40) return OR_ETOOBIG;
    return oracle_formS_range(cov, m, pattern, 0, 1, (uint64_t)1 << n, threads, out);
}

/* Sigma_C in binary128, exported as (hi, lo) double pairs (2n x 2n full), and
 * P_vac(N): lets tests compare the library's conditioned matrix. */
int oracle_conditioned(const double *cov, int m, const int8_t *pattern,
                       double *sig_hi, double *sig_lo, double *pvac_n) {
    int rc = validate(cov, m, pattern);
    if (rc) return rc;
    int *cidx, *nidx, n, nn;
    if ((rc = split_pattern(m, pattern, &cidx, &n, &nidx, &nn))) return rc;
    int dc = 2 * n;
    qf *sig_c = (qf *)malloc(sizeof(qf) * (size_t)(dc > 0 ? dc * dc : 1));
    qf pvn;
    int crc = sig_c ? condition_on_vacuum(cov, m, cidx, n, nidx, nn, sig_c, &pvn) : -2;
    free(cidx); free(nidx);
    if (crc) { free(sig_c); return crc == -2 ? OR_ENOMEM : OR_ENOTPD; }
    for (int i = 0; i < dc * dc; i++) { sig_hi[i] = q_hi(sig_c[i]); sig_lo[i] = q_lo(sig_c[i]); }
    *pvac_n = (double)pvn;
    free(sig_c);
    return OR_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
