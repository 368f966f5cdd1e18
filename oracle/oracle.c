/*
 * Plain FP64 CPU oracle for the two-table Figaro computation of R and sigma.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library: it is a separate, slow and
 * obviously correct restatement of the paper's definitions.
 *
 * What it computes ("Figaro on GPUs: Two Tables", Section 1, Theory):
 *   - the natural join of two relations, read as the union over join-key
 *     groups of per-group Cartesian products (the Cartesian product C = A x B
 *     is the single-group case);
 *   - the QR head H(A) = (1/sqrt m) sum_i A_i and the QR tail
 *     T(A)_i = (sqrt(i) A_{i+1} - S_i / sqrt(i)) / sqrt(i+1), S_i = sum_{k<=i} A_k;
 *   - the compact matrix of Claim 1, per group g:
 *       [ sqrt(m2_g) A_g | H(B_g) ]   (one row per A row, H(B_g) repeated)
 *       [ 0              | sqrt(m1_g) T(B_g) ]
 *   - R, the upper-triangular factor of the Householder QR of that matrix
 *     (Experiments section: the dense QR is Householder), rows normalised to a
 *     non-negative diagonal;
 *   - sigma, the singular values of R (Related Works: SVD through QR; the
 *     singular values of the join equal those of R), by one-sided Jacobi.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - Claim 1's zero block under A sqrt(m2) has m2-1 rows, not one;
 *   - a key group exists iff the key occurs in both tables; unmatched rows
 *     contribute nothing;
 *   - rows of the compact matrix: all region-1 rows (groups ascending, A
 *     order), then all region-2 rows (groups ascending, B order);
 *   - sums run in input row order with Neumaier compensation.
 *
 * Parity status: every function here is pinned by CPU tests against brute
 * force (explicit join, explicit Givens sequence, LAPACK QR/SVD of the
 * explicit join, Gram-Cholesky, closed-form invariants).  Rank-deficient
 * inputs have no unique R beyond the rank: parity unpinned there.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_EUNSORTED -2
#define ORACLE_ECAP -3

/* group table columns */
enum { G_KEY = 0, G_OFFA, G_M1, G_OFFB, G_M2, G_R1, G_R2, G_COLS };

/* ---------------------------------------------------------------- groups */

/*
 * Key grouping (Experiments section: relations sorted by join attribute).
 * keys may be NULL for both tables (Cartesian product: one group).
 * tab is cap x 7 int64, row g = {key, offA, m1_g, offB, m2_g, r1_g, r2_g}.
 * counts[0..3] = {G, R1 = sum m1_g, R2 = sum (m2_g - 1), join_rows = sum m1_g m2_g}.
 */
int oracle_groups(const int32_t *kA, int64_t m1, const int32_t *kB, int64_t m2,
                  int64_t cap, int64_t *tab, int64_t *counts)
{
    if (m1 < 0 || m2 < 0 || !counts) return ORACLE_EINVAL;
    if ((kA == NULL) != (kB == NULL)) return ORACLE_EINVAL;
    int64_t G = 0, R1 = 0, R2 = 0, J = 0;
    if (kA == NULL) {
        if (m1 > 0 && m2 > 0) {
            if (cap < 1) return ORACLE_ECAP;
            int64_t *t = tab;
            t[G_KEY] = 0; t[G_OFFA] = 0; t[G_M1] = m1; t[G_OFFB] = 0; t[G_M2] = m2;
            t[G_R1] = 0; t[G_R2] = 0;
            G = 1; R1 = m1; R2 = m2 - 1; J = m1 * m2;
        }
    } else {
        for (int64_t i = 1; i < m1; i++) if (kA[i] < kA[i - 1]) return ORACLE_EUNSORTED;
        for (int64_t i = 1; i < m2; i++) if (kB[i] < kB[i - 1]) return ORACLE_EUNSORTED;
        int64_t a = 0, b = 0;
        while (a < m1 && b < m2) {
            /* run lengths at the current positions */
            int64_t ea = a; while (ea < m1 && kA[ea] == kA[a]) ea++;
            int64_t eb = b; while (eb < m2 && kB[eb] == kB[b]) eb++;
            if (kA[a] < kB[b]) { a = ea; continue; }
            if (kB[b] < kA[a]) { b = eb; continue; }
            if (G >= cap) return ORACLE_ECAP;
            int64_t *t = tab + G * G_COLS;
            t[G_KEY] = kA[a]; t[G_OFFA] = a; t[G_M1] = ea - a; t[G_OFFB] = b; t[G_M2] = eb - b;
            t[G_R1] = R1; t[G_R2] = R2;
            R1 += ea - a; R2 += (eb - b) - 1; J += (ea - a) * (eb - b);
            G++;
            a = ea; b = eb;
        }
    }
    counts[0] = G; counts[1] = R1; counts[2] = R2; counts[3] = J;
    return ORACLE_OK;
}

/* --------------------------------------------------------- compact matrix */

/* Neumaier compensated accumulation: s + c is the running sum. */
static inline void neumaier_add(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/*
 * Claim 1 compact matrix, generalised per key group.
 * M is (R1 + R2) x (n1 + n2) row-major with leading dimension ldm; it is
 * fully written (the zero block included).  heads (G x n2) receives H(B_g).
 */
int oracle_compact(const double *A, int64_t m1, int64_t n1, int64_t lda,
                   const double *B, int64_t m2, int64_t n2, int64_t ldb,
                   const int64_t *tab, int64_t G, int64_t R1,
                   double *M, int64_t ldm, double *heads)
{
    (void)m1; (void)m2;
    const int64_t N = n1 + n2;
    if (ldm < N) return ORACLE_EINVAL;
    double *s = (double *)malloc(sizeof(double) * (size_t)(n2 > 0 ? n2 : 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(n2 > 0 ? n2 : 1));
    for (int64_t g = 0; g < G; g++) {
        const int64_t *t = tab + g * G_COLS;
        const int64_t offA = t[G_OFFA], mg1 = t[G_M1], offB = t[G_OFFB], mg2 = t[G_M2];
        const int64_t r1 = t[G_R1], r2 = t[G_R2];
        /* Region 2: tails of B_g, scaled by sqrt(m1_g).  The prefix S_i covers
           the group's first i rows (1-based i), the tail row i uses row i+1. */
        for (int64_t j = 0; j < n2; j++) { s[j] = 0.0; c[j] = 0.0; }
        for (int64_t i = 1; i <= mg2; i++) {
            const double *row = B + (offB + i - 1) * ldb;      /* row i (1-based) */
            if (i >= 2) {
                /* tail index i-1 uses S_{i-1} and row i */
                const double ii = (double)(i - 1);
                double *out = M + (R1 + r2 + (i - 2)) * ldm;
                for (int64_t j = 0; j < n1; j++) out[j] = 0.0;
                for (int64_t j = 0; j < n2; j++) {
                    const double S = s[j] + c[j];
                    const double tail = (sqrt(ii) * row[j] - S / sqrt(ii)) / sqrt(ii + 1.0);
                    out[n1 + j] = sqrt((double)mg1) * tail;
                }
            }
            for (int64_t j = 0; j < n2; j++) neumaier_add(&s[j], &c[j], row[j]);
        }
        /* Head of B_g: (1/sqrt m2_g) * sum of the group's rows. */
        double *h = heads + g * n2;
        for (int64_t j = 0; j < n2; j++) h[j] = (s[j] + c[j]) / sqrt((double)mg2);
        /* Region 1: [sqrt(m2_g) A_r | H(B_g)] for each A row of the group. */
        for (int64_t r = 0; r < mg1; r++) {
            const double *arow = A + (offA + r) * lda;
            double *out = M + (r1 + r) * ldm;
            for (int64_t j = 0; j < n1; j++) out[j] = sqrt((double)mg2) * arow[j];
            for (int64_t j = 0; j < n2; j++) out[n1 + j] = h[j];
        }
    }
    free(s); free(c);
    return ORACLE_OK;
}

/* ---------------------------------------------------------- Householder QR */

static int nthreads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Householder QR of X (rows x N, row-major, ld), overwritten; on return the
 * upper triangle of the first min(rows, N) rows holds R.  Conventions of the
 * textbook unblocked algorithm: for column j with alpha = X_jj and x the
 * entries below, beta = -sign(alpha) * ||(alpha, x)||, tau = (beta-alpha)/beta,
 * v = x / (alpha - beta) with v_0 = 1; tau = 0 when x = 0.  The reflector
 * I - tau v v^T is then applied to the trailing columns.  Rows are split over
 * threads for the two reductions and the update; nothing else is reordered.
 */
int oracle_householder(double *X, int64_t rows, int64_t N, int64_t ld)
{
    if (rows < 0 || N < 0 || ld < N) return ORACLE_EINVAL;
    const int nt = nthreads();
    double *wpart = (double *)calloc((size_t)nt * (size_t)(N > 0 ? N : 1), sizeof(double));
    double *spart = (double *)calloc((size_t)nt, sizeof(double));
    double *w = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    const int64_t kmax = rows < N ? rows : N;
    for (int64_t j = 0; j < kmax; j++) {
        const double alpha = X[j * ld + j];
        /* ||x||, scaled by the largest magnitude against overflow */
        double scale = 0.0;
        for (int64_t i = j + 1; i < rows; i++) {
            const double a = fabs(X[i * ld + j]);
            if (a > scale) scale = a;
        }
        double xnorm = 0.0;
        if (scale > 0.0) {
            for (int t = 0; t < nt; t++) spart[t] = 0.0;
#pragma omp parallel num_threads(nt)
            {
#ifdef _OPENMP
                const int t = omp_get_thread_num();
#else
                const int t = 0;
#endif
                double acc = 0.0;
#pragma omp for schedule(static)
                for (int64_t i = j + 1; i < rows; i++) {
                    const double q = X[i * ld + j] / scale;
                    acc += q * q;
                }
                spart[t] = acc;
            }
            double ssq = 0.0;
            for (int t = 0; t < nt; t++) ssq += spart[t];
            xnorm = scale * sqrt(ssq);
        }
        if (xnorm == 0.0) continue; /* tau = 0: H_j = I */
        const double h = hypot(alpha, xnorm);
        const double beta = alpha >= 0.0 ? -h : h;
        const double tau = (beta - alpha) / beta;
        const double vscale = 1.0 / (alpha - beta);
        X[j * ld + j] = beta;
        for (int64_t i = j + 1; i < rows; i++) X[i * ld + j] *= vscale; /* v below the unit entry */
        const int64_t nk = N - j - 1;
        if (nk == 0) continue;
        /* w = X[j, j+1:] + v^T X[j+1:, j+1:] */
        memset(wpart, 0, sizeof(double) * (size_t)nt * (size_t)N);
#pragma omp parallel num_threads(nt)
        {
#ifdef _OPENMP
            const int t = omp_get_thread_num();
#else
            const int t = 0;
#endif
            double *wp = wpart + (size_t)t * (size_t)N;
#pragma omp for schedule(static)
            for (int64_t i = j + 1; i < rows; i++) {
                const double vi = X[i * ld + j];
                const double *xr = X + i * ld + j + 1;
                for (int64_t k = 0; k < nk; k++) wp[k] += vi * xr[k];
            }
        }
        for (int64_t k = 0; k < nk; k++) {
            double acc = X[j * ld + j + 1 + k];
            for (int t = 0; t < nt; t++) acc += wpart[(size_t)t * (size_t)N + k];
            w[k] = acc;
        }
        /* X[j, :] -= tau w ; X[i, :] -= tau v_i w */
        for (int64_t k = 0; k < nk; k++) X[j * ld + j + 1 + k] -= tau * w[k];
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t i = j + 1; i < rows; i++) {
            const double tv = tau * X[i * ld + j];
            double *xr = X + i * ld + j + 1;
            for (int64_t k = 0; k < nk; k++) xr[k] -= tv * w[k];
        }
    }
    free(wpart); free(spart); free(w);
    return ORACLE_OK;
}

/*
 * Row-sign normalisation of an upper-triangular R (N x N, row-major, ldr):
 * R is unique only up to the sign of each row.  A row with a negative
 * diagonal is negated; a row with a zero diagonal is negated iff its first
 * nonzero entry is negative; -0.0 becomes +0.0.
 */
void oracle_sign_normalise(double *R, int64_t N, int64_t ldr)
{
    for (int64_t i = 0; i < N; i++) {
        double *row = R + i * ldr;
        int neg = 0;
        if (row[i] < 0.0) neg = 1;
        else if (row[i] == 0.0) {
            for (int64_t k = i; k < N; k++) {
                if (row[k] != 0.0) { neg = row[k] < 0.0; break; }
            }
        }
        for (int64_t k = 0; k < N; k++) {
            double v = (k < i) ? 0.0 : (neg ? -row[k] : row[k]);
            row[k] = v + 0.0; /* -0.0 + 0.0 == +0.0 */
        }
    }
}

/* Extract R (N x N, zeros below the diagonal) from a factored X. */
void oracle_extract_r(const double *X, int64_t rows, int64_t N, int64_t ld, double *R, int64_t ldr)
{
    for (int64_t i = 0; i < N; i++)
        for (int64_t k = 0; k < N; k++)
            R[i * ldr + k] = (i < rows && k >= i) ? X[i * ld + k] : 0.0;
}

/* ------------------------------------------------------------ full chain */

/*
 * R of the join matrix of (A, B) through the compact matrix: groups, Claim 1
 * assembly, Householder QR of the compact matrix, sign normalisation.
 * A, B are FP64 row-major.  keys NULL = Cartesian product.
 * R (N x N, ldr) and counts[4] are outputs; returns an ORACLE_* code.
 */
int oracle_r(const double *A, int64_t m1, int64_t n1, int64_t lda, const int32_t *kA,
             const double *B, int64_t m2, int64_t n2, int64_t ldb, const int32_t *kB,
             double *R, int64_t ldr, int64_t *counts)
{
    const int64_t N = n1 + n2;
    if (N <= 0) return ORACLE_EINVAL;
    int64_t cap = (m1 < m2 ? m1 : m2);
    if (cap < 1) cap = 1;
    int64_t *tab = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap * G_COLS);
    int rc = oracle_groups(kA, m1, kB, m2, cap, tab, counts);
    if (rc != ORACLE_OK) { free(tab); return rc; }
    const int64_t G = counts[0], R1 = counts[1], R2 = counts[2];
    const int64_t rows = R1 + R2;
    double *M = (double *)calloc((size_t)(rows > 0 ? rows : 1) * (size_t)N, sizeof(double));
    double *heads = (double *)calloc((size_t)(G > 0 ? G : 1) * (size_t)(n2 > 0 ? n2 : 1), sizeof(double));
    oracle_compact(A, m1, n1, lda, B, m2, n2, ldb, tab, G, R1, M, N, heads);
    oracle_householder(M, rows, N, N);
    oracle_extract_r(M, rows, N, N, R, ldr);
    oracle_sign_normalise(R, N, ldr);
    free(M); free(heads); free(tab);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------- sigma */

static int cmp_desc(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/*
 * Singular values of R (N x N, row-major, ldr) by one-sided (Hestenes)
 * Jacobi on its columns, cyclic-by-rows pair order.  For the pair (p, q) with
 * alpha = |c_p|^2, beta = |c_q|^2, gamma = c_p . c_q the pair is skipped when
 * |gamma| <= N * 2^-53 * sqrt(alpha beta); otherwise zeta = (beta-alpha)/(2 gamma),
 * t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1+t^2), s = c t and
 * (c_p, c_q) <- (c c_p - s c_q, s c_p + c c_q).  Sweeps stop after one with no
 * rotation (at most max_sweeps).  sigma = column norms, descending.
 * Returns the number of sweeps taken, or a negative code.
 */
int oracle_sigma(const double *R, int64_t N, int64_t ldr, double *sigma, int max_sweeps)
{
    if (N <= 0 || ldr < N) return ORACLE_EINVAL;
    /* columns of R stored contiguously */
    double *C = (double *)malloc(sizeof(double) * (size_t)N * (size_t)N);
    for (int64_t i = 0; i < N; i++)
        for (int64_t k = 0; k < N; k++) C[k * N + i] = R[i * ldr + k];
    const double tol = (double)N * ldexp(1.0, -53);
    int sweeps = 0;
    for (; sweeps < max_sweeps;) {
        int64_t rotations = 0;
        for (int64_t p = 0; p < N - 1; p++) {
            for (int64_t q = p + 1; q < N; q++) {
                double *cp = C + p * N, *cq = C + q * N;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t i = 0; i < N; i++) {
                    alpha += cp[i] * cp[i];
                    beta += cq[i] * cq[i];
                    gamma += cp[i] * cq[i];
                }
                if (fabs(gamma) <= tol * sqrt(alpha * beta)) continue;
                const double zeta = (beta - alpha) / (2.0 * gamma);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = c * t;
                for (int64_t i = 0; i < N; i++) {
                    const double xp = cp[i], xq = cq[i];
                    cp[i] = c * xp - s * xq;
                    cq[i] = s * xp + c * xq;
                }
                rotations++;
            }
        }
        sweeps++;
        if (rotations == 0) break;
    }
    for (int64_t k = 0; k < N; k++) {
        double acc = 0.0;
        for (int64_t i = 0; i < N; i++) acc += C[k * N + i] * C[k * N + i];
        sigma[k] = sqrt(acc);
    }
    qsort(sigma, (size_t)N, sizeof(double), cmp_desc);
    free(C);
    return sweeps;
}

/*
 * Right singular vectors (Abstract: the right singular vectors of the join;
 * Related Works: the SVD of the join through its R).  The one-sided Jacobi of
 * oracle_sigma, with every rotation also applied to the columns of V, which
 * starts as the identity, so that on exit R V has orthogonal columns of norms
 * sigma and V is orthogonal.  Outputs sigma descending (equal values in column
 * order) and V row-major (ldv): V[i * ldv + j] is component i of the right
 * singular vector of sigma[j].  Returns the sweeps taken or a negative code.
 */
int oracle_svd_v(const double *R, int64_t N, int64_t ldr, double *sigma, double *V, int64_t ldv, int max_sweeps)
{
    if (N <= 0 || ldr < N || ldv < N) return ORACLE_EINVAL;
    double *C = (double *)malloc(sizeof(double) * (size_t)N * (size_t)N);
    double *Q = (double *)malloc(sizeof(double) * (size_t)N * (size_t)N);
    double *nrm = (double *)malloc(sizeof(double) * (size_t)N);
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    for (int64_t i = 0; i < N; i++)
        for (int64_t k = 0; k < N; k++) {
            C[k * N + i] = R[i * ldr + k];
            Q[k * N + i] = (i == k) ? 1.0 : 0.0;
        }
    const double tol = (double)N * ldexp(1.0, -53);
    int sweeps = 0;
    for (; sweeps < max_sweeps;) {
        int64_t rotations = 0;
        for (int64_t p = 0; p < N - 1; p++) {
            for (int64_t q = p + 1; q < N; q++) {
                double *cp = C + p * N, *cq = C + q * N;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t i = 0; i < N; i++) {
                    alpha += cp[i] * cp[i];
                    beta += cq[i] * cq[i];
                    gamma += cp[i] * cq[i];
                }
                if (fabs(gamma) <= tol * sqrt(alpha * beta)) continue;
                const double zeta = (beta - alpha) / (2.0 * gamma);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = c * t;
                double *vp = Q + p * N, *vq = Q + q * N;
                for (int64_t i = 0; i < N; i++) {
                    const double xp = cp[i], xq = cq[i];
                    cp[i] = c * xp - s * xq;
                    cq[i] = s * xp + c * xq;
                    const double yp = vp[i], yq = vq[i];
                    vp[i] = c * yp - s * yq;
                    vq[i] = s * yp + c * yq;
                }
                rotations++;
            }
        }
        sweeps++;
        if (rotations == 0) break;
    }
    for (int64_t k = 0; k < N; k++) {
        double acc = 0.0;
        for (int64_t i = 0; i < N; i++) acc += C[k * N + i] * C[k * N + i];
        nrm[k] = sqrt(acc);
        ord[k] = k;
    }
    /* descending by norm, equal norms in column order (insertion sort: stable) */
    for (int64_t a = 1; a < N; a++) {
        const int64_t x = ord[a];
        int64_t b = a - 1;
        while (b >= 0 && nrm[ord[b]] < nrm[x]) {
            ord[b + 1] = ord[b];
            b--;
        }
        ord[b + 1] = x;
    }
    for (int64_t j = 0; j < N; j++) {
        sigma[j] = nrm[ord[j]];
        for (int64_t i = 0; i < N; i++) V[i * ldv + j] = Q[ord[j] * N + i];
    }
    free(C);
    free(Q);
    free(nrm);
    free(ord);
    return sweeps;
}

int oracle_num_threads(void) { return nthreads(); }
