/*
 * lagp_oracle.c -- FP64 CPU oracle for local approximate Gaussian-process
 * prediction with greedy ALC local designs (Gramacy & Apley, "Local Gaussian
 * process approximation for large computer experiments").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg load this library.  It shares no code,
 * header or table with the GPU path; the product never calls it.
 *
 * It is deliberately plain and slow.  At every greedy step the local
 * covariance matrix K_j is rebuilt and factorised from scratch, every
 * candidate is solved against that factor, and the final prediction uses a
 * fresh factorisation of K_n.  Nothing is carried from one step to the next
 * except the list of chosen design indices.
 *
 * Model (Section 2): zero-mean GP, isotropic Gaussian correlation
 *   K(a,b) = exp(-||a-b||^2 / theta)   for two distinct points,
 * and the nugget eta is added on the diagonal of every design covariance
 * matrix and to the self-covariance K(x,x) = 1 + eta of the predictive
 * location and of a candidate.  Cross-covariances never carry the nugget,
 * even where coordinates coincide (the Kronecker delta is taken on indices).
 *
 * Greedy local design (Section 3 with the criterion of Sections 3.2-3.3):
 * start from the n0 nearest neighbours of x, then for j = n0..n-1 add the
 * candidate with the largest reduction in predictive variance at x,
 *   ALC_j(c) = v_j(x) - v_{j+1}(x | c) = cov_j(x,c)^2 / v_j(c)
 * (eq dxy, and its partial-correlation form eq dxy2 of SM Section 4), where
 *   v_j(c)     = 1 + eta - k_j(c)' K_j^{-1} k_j(c),
 *   cov_j(x,c) = K(x,c)  - k_j(x)' K_j^{-1} k_j(c).
 * Candidates are the N' nearest design points of x (Section 6).
 *
 * Prediction (eqs predgp and preds2 with N -> n): mean k'K^{-1}Y, scale
 * s2 = psi * v_n(x) / n with psi = Y'K^{-1}Y, df = n, variance
 * V = s2 * n / (n-2) = psi * v_n(x) / (n-2).
 *
 * Local lengthscale inference (Sections 3.2 and 4.2): the concentrated log
 * likelihood of a local design (eq gpk of Section 2, constants dropped)
 *   l(theta) = -1/2 log|K| - n/2 log psi,   psi = Y'K^{-1}Y,
 * its first and second derivatives in theta (eqs dl and d2l of SM Section 2,
 * with the entrywise derivatives of K for the isotropic Gaussian kernel), a Newton
 * search for its maximum inside (tmin, tmax), and the two-stage scheme of
 * Section 4.2 with one repetition.  Every evaluation forms K^{-1} explicitly
 * from a fresh Cholesky factor.
 *
 * MSPE criterion (Section 3.1, eq mspe): the alternative greedy rule that
 * minimises the approximate mean-squared predictive error, which adds to the
 * reduced variance the theta-uncertainty term (dmu/dtheta)^2 / G with the
 * expected Fisher information G, at fixed theta.
 *
 * Augmentation and stopping (Section 6's discussion): a saved design may
 * replace the n0 nearest neighbours as the starting design, and the greedy
 * search may stop once the best candidate's variance ratio v_j(x)/v_{j+1}(x)
 * (V_j/V_{j+1} with psi cancelled) falls below a threshold.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 * distances are summed over coordinates left to right with no fused
 * multiply-add; nearest neighbours are ordered by (squared distance, index);
 * argmax ties go to the smaller design index; a candidate whose v_j(c) is
 * not positive scores -infinity; a failed factorisation flags the location.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_NOTPD 1
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* ||a-b||^2, coordinates summed left to right. */
static double sqdist(const double *a, const double *b, int p)
{
    double s = 0.0;
    for (int k = 0; k < p; k++) {
        double t = a[k] - b[k];
        s += t * t;
    }
    return s;
}

/* Isotropic Gaussian correlation of two distinct points (Section 2). */
static double corr(const double *a, const double *b, int p, double theta)
{
    return exp(-sqdist(a, b, p) / theta);
}

static double dot(const double *a, const double *b, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* Lower Cholesky factor L (row-major n x n) of the symmetric matrix A,
 * computed row by row: L[i][m] = (A[i][m] - sum_{l<m} L[i][l] L[m][l]) / L[m][m]
 * and L[i][i] = sqrt(A[i][i] - sum_{l<i} L[i][l]^2).  Returns -1 when a
 * pivot is not positive. */
static int cholesky(const double *A, int n, double *L)
{
    for (int i = 0; i < n; i++) {
        for (int m = 0; m <= i; m++) {
            double s = A[(size_t)i * n + m];
            for (int l = 0; l < m; l++) s -= L[(size_t)i * n + l] * L[(size_t)m * n + l];
            if (m == i) {
                if (!(s > 0.0)) return -1;
                L[(size_t)i * n + i] = sqrt(s);
            } else {
                L[(size_t)i * n + m] = s / L[(size_t)m * n + m];
            }
        }
        for (int m = i + 1; m < n; m++) L[(size_t)i * n + m] = 0.0;
    }
    return 0;
}

/* Solve L w = b by forward substitution. */
static void forward_solve(const double *L, int n, const double *b, double *w)
{
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int l = 0; l < i; l++) s -= L[(size_t)i * n + l] * w[l];
        w[i] = s / L[(size_t)i * n + i];
    }
}

/* K_j = K(D, D) + eta I for the j design indices D. */
static void design_cov(const double *X, int p, const int32_t *D, int j, double theta,
                       double eta, double *K)
{
    for (int a = 0; a < j; a++) {
        for (int b = 0; b < j; b++) {
            K[(size_t)a * j + b] = (a == b) ? 1.0 + eta
                                            : corr(X + (size_t)D[a] * p, X + (size_t)D[b] * p, p, theta);
        }
    }
}

typedef struct {
    double d2;
    int64_t i;
} keyed;

static int keyed_cmp(const void *pa, const void *pb)
{
    const keyed *a = (const keyed *)pa, *b = (const keyed *)pb;
    if (a->d2 < b->d2) return -1;
    if (a->d2 > b->d2) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

/* The M nearest design points of x, ascending by (squared distance, index)
 * (Section 3: nearest-neighbour sub-design; Section 6: N' nearest candidates). */
int lagp_oracle_knn(const double *X, int64_t N, int32_t p, const double *x, int64_t M,
                    int32_t *idx, double *d2_out)
{
    if (N < 1 || p < 1 || M < 1 || M > N) return ORACLE_EINVAL;
    keyed *all = (keyed *)malloc((size_t)N * sizeof(keyed));
    if (!all) return ORACLE_ENOMEM;
    for (int64_t i = 0; i < N; i++) {
        all[i].d2 = sqdist(X + (size_t)i * p, x, p);
        all[i].i = i;
    }
    qsort(all, (size_t)N, sizeof(keyed), keyed_cmp);
    for (int64_t m = 0; m < M; m++) {
        idx[m] = (int32_t)all[m].i;
        if (d2_out) d2_out[m] = all[m].d2;
    }
    free(all);
    return ORACLE_OK;
}

/* Local GP prediction at x from the design indices D (eqs predgp, preds2),
 * through a fresh Cholesky factor of K_n.  out = {mean, s2, var, v_n(x), psi}. */
int lagp_oracle_predict(const double *X, const double *y, int32_t p, const double *x,
                        const int32_t *D, int32_t n, double theta, double eta, double *out)
{
    if (n < 1) return ORACLE_EINVAL;
    double *K = (double *)malloc((size_t)n * n * sizeof(double));
    double *L = (double *)malloc((size_t)n * n * sizeof(double));
    double *kx = (double *)malloc((size_t)n * sizeof(double));
    double *wx = (double *)malloc((size_t)n * sizeof(double));
    double *yd = (double *)malloc((size_t)n * sizeof(double));
    double *u = (double *)malloc((size_t)n * sizeof(double));
    int rc = ORACLE_OK;
    if (!K || !L || !kx || !wx || !yd || !u) { rc = ORACLE_ENOMEM; goto done; }
    design_cov(X, p, D, n, theta, eta, K);
    if (cholesky(K, n, L) != 0) {
        for (int i = 0; i < 5; i++) out[i] = NAN;
        rc = ORACLE_NOTPD;
        goto done;
    }
    for (int a = 0; a < n; a++) {
        kx[a] = corr(X + (size_t)D[a] * p, x, p, theta);
        yd[a] = y[D[a]];
    }
    forward_solve(L, n, kx, wx);   /* wx = L^{-1} k_n(x) */
    forward_solve(L, n, yd, u);    /* u  = L^{-1} Y_n    */
    {
        double mean = dot(wx, u, n);            /* k' K^{-1} Y   */
        double psi = dot(u, u, n);              /* Y' K^{-1} Y   */
        double vx = (1.0 + eta) - dot(wx, wx, n); /* K(x,x) - k' K^{-1} k */
        out[0] = mean;
        out[1] = psi * vx / n;
        out[2] = (n > 2) ? psi * vx / (n - 2) : NAN;
        out[3] = vx;
        out[4] = psi;
    }
done:
    free(K); free(L); free(kx); free(wx); free(yd); free(u);
    return rc;
}

/* ALC scores of the candidates cand[0..nc-1] given the current local design
 * D (j points): ALC(c) = cov_j(x,c)^2 / v_j(c), from a fresh Cholesky of K_j.
 * Also returns v_j(c), cov_j(x,c) and v_j(x).  A candidate with v_j(c) <= 0
 * scores -infinity. */
int lagp_oracle_alc(const double *X, int32_t p, const double *x, const int32_t *D, int32_t j,
                    const int32_t *cand, int64_t nc, double theta, double eta,
                    double *alc, double *vc_out, double *cov_out, double *vx_out)
{
    if (j < 1) return ORACLE_EINVAL;
    double *K = (double *)malloc((size_t)j * j * sizeof(double));
    double *L = (double *)malloc((size_t)j * j * sizeof(double));
    double *kx = (double *)malloc((size_t)j * sizeof(double));
    double *wx = (double *)malloc((size_t)j * sizeof(double));
    double *kc = (double *)malloc((size_t)j * sizeof(double));
    double *wc = (double *)malloc((size_t)j * sizeof(double));
    int rc = ORACLE_OK;
    if (!K || !L || !kx || !wx || !kc || !wc) { rc = ORACLE_ENOMEM; goto done; }
    design_cov(X, p, D, j, theta, eta, K);
    if (cholesky(K, j, L) != 0) { rc = ORACLE_NOTPD; goto done; }
    for (int a = 0; a < j; a++) kx[a] = corr(X + (size_t)D[a] * p, x, p, theta);
    forward_solve(L, j, kx, wx);
    if (vx_out) *vx_out = (1.0 + eta) - dot(wx, wx, j);
    for (int64_t ci = 0; ci < nc; ci++) {
        const double *xc = X + (size_t)cand[ci] * p;
        for (int a = 0; a < j; a++) kc[a] = corr(X + (size_t)D[a] * p, xc, p, theta);
        forward_solve(L, j, kc, wc);
        double vc = (1.0 + eta) - dot(wc, wc, j);
        double cov = corr(x, xc, p, theta) - dot(wx, wc, j);
        alc[ci] = (vc > 0.0) ? cov * cov / vc : -INFINITY;
        if (vc_out) vc_out[ci] = vc;
        if (cov_out) cov_out[ci] = cov;
    }
done:
    free(K); free(L); free(kx); free(wx); free(kc); free(wc);
    return rc;
}

/* v_j(x) for the design D, from a fresh Cholesky of K_j (eq newv). */
static int variance_at(const double *X, int p, const double *x, const int32_t *D, int j,
                       double theta, double eta, double *K, double *L, double *kx,
                       double *wx, double *out)
{
    design_cov(X, p, D, j, theta, eta, K);
    if (cholesky(K, j, L) != 0) return ORACLE_NOTPD;
    for (int a = 0; a < j; a++) kx[a] = corr(X + (size_t)D[a] * p, x, p, theta);
    forward_solve(L, j, kx, wx);
    *out = (1.0 + eta) - dot(wx, wx, j);
    return ORACLE_OK;
}

/* Brute-force ALC: v_j(x) - v_{j+1}(x | c), each variance from its own fresh
 * Cholesky factor (K_j, then K_{j+1} with c appended).  Non-positive-definite
 * augmented matrices score NaN. */
int lagp_oracle_alc_brute(const double *X, int32_t p, const double *x, const int32_t *D,
                          int32_t j, const int32_t *cand, int64_t nc, double theta,
                          double eta, double *alc)
{
    if (j < 1) return ORACLE_EINVAL;
    int j1 = j + 1;
    double *K = (double *)malloc((size_t)j1 * j1 * sizeof(double));
    double *L = (double *)malloc((size_t)j1 * j1 * sizeof(double));
    double *kx = (double *)malloc((size_t)j1 * sizeof(double));
    double *wx = (double *)malloc((size_t)j1 * sizeof(double));
    int32_t *D1 = (int32_t *)malloc((size_t)j1 * sizeof(int32_t));
    int rc = ORACLE_OK;
    double v0;
    if (!K || !L || !kx || !wx || !D1) { rc = ORACLE_ENOMEM; goto done; }
    if (variance_at(X, p, x, D, j, theta, eta, K, L, kx, wx, &v0) != 0) { rc = ORACLE_NOTPD; goto done; }
    memcpy(D1, D, (size_t)j * sizeof(int32_t));
    for (int64_t ci = 0; ci < nc; ci++) {
        double v1;
        D1[j] = cand[ci];
        if (variance_at(X, p, x, D1, j1, theta, eta, K, L, kx, wx, &v1) != 0)
            alc[ci] = NAN;
        else
            alc[ci] = v0 - v1;
    }
done:
    free(K); free(L); free(kx); free(wx); free(D1);
    return rc;
}

/* Greedy ALC local design and prediction at one location x.
 *
 *   sel[0..n-1]   chosen design indices in order (the first n0 are the
 *                 nearest neighbours in (distance, index) order);
 *   out[0..4]     {mean, s2, var, v_n(x), psi};
 *   diag[3*j..]   for each greedy step j >= n0: {largest ALC, second largest
 *                 ALC, ALC of the chosen candidate}; NaN for the n0 initial
 *                 steps (nullable);
 *   replay        if non-NULL, the n indices to follow instead of the
 *                 argmax (the first n0 must be the nearest neighbours);
 *                 diag then reports how far each followed choice falls short
 *                 of the oracle's own largest ALC.
 *
 * Returns ORACLE_OK, ORACLE_NOTPD (outputs NaN) or a negative error. */
/* The general form of lagp_oracle_local with the extensions of Section 6's
 * discussion:
 *   start (nullable): a saved local design of n0 indices that replaces the
 *     n0 nearest neighbours, so the greedy search picks up where an earlier
 *     one left off (augmentation); every start index must be one of x's M
 *     candidates and appear once, else ORACLE_EINVAL;
 *   vratio: when > 0, stop before greedy step j (j >= n0) once the best
 *     candidate's variance ratio v_j(x) / v_{j+1}(x) = v_j(x) / (v_j(x) -
 *     ALC_j) is below vratio (psi cancels in the ratio V_j / V_{j+1}), so
 *     the design has n_used <= n points;
 *   n_used (nullable) receives the final design size. */
int lagp_oracle_local_ex(const double *X, const double *y, int64_t N, int32_t p, const double *x,
                         int32_t n0, int32_t n, int64_t M, double theta, double eta,
                         const int32_t *replay, const int32_t *start, double vratio, int32_t *sel,
                         int32_t *n_used, double *out, double *diag)
{
    if (N < 1 || p < 1 || n0 < 1 || n0 > n || (int64_t)n > M || M > N || !(theta > 0.0) ||
        !(eta >= 0.0) || !(vratio >= 0.0))
        return ORACLE_EINVAL;
    int32_t *C = (int32_t *)malloc((size_t)M * sizeof(int32_t));
    char *used = (char *)calloc((size_t)M, 1);
    double *K = (double *)malloc((size_t)n * n * sizeof(double));
    double *L = (double *)malloc((size_t)n * n * sizeof(double));
    double *kx = (double *)malloc((size_t)n * sizeof(double));
    double *wx = (double *)malloc((size_t)n * sizeof(double));
    double *kc = (double *)malloc((size_t)n * sizeof(double));
    double *wc = (double *)malloc((size_t)n * sizeof(double));
    int rc = ORACLE_OK;
    if (!C || !used || !K || !L || !kx || !wx || !kc || !wc) { rc = ORACLE_ENOMEM; goto done; }
    rc = lagp_oracle_knn(X, N, p, x, M, C, NULL);
    if (rc != ORACLE_OK) goto done;

    for (int j = 0; j < n0; j++) {
        int64_t ci = j;
        if (start) {   /* the saved design's j-th point, found among the candidates */
            for (ci = 0; ci < M && C[ci] != start[j]; ci++) {}
            if (ci == M || used[ci]) { rc = ORACLE_EINVAL; goto done; }
        }
        if (replay && replay[j] != C[ci]) { rc = ORACLE_EINVAL; goto done; }
        sel[j] = C[ci];
        used[ci] = 1;
        if (diag) diag[3 * j] = diag[3 * j + 1] = diag[3 * j + 2] = NAN;
    }

    int32_t nu = n;
    for (int j = n0; j < n; j++) {
        /* K_j and its Cholesky factor, from scratch. */
        design_cov(X, p, sel, j, theta, eta, K);
        if (cholesky(K, j, L) != 0) { rc = ORACLE_NOTPD; break; }
        for (int a = 0; a < j; a++) kx[a] = corr(X + (size_t)sel[a] * p, x, p, theta);
        forward_solve(L, j, kx, wx);

        double a1 = -INFINITY, a2 = -INFINITY, a_follow = NAN;
        int64_t best = -1, follow = -1;
        for (int64_t ci = 0; ci < M; ci++) {
            if (used[ci]) continue;
            const double *xc = X + (size_t)C[ci] * p;
            for (int a = 0; a < j; a++) kc[a] = corr(X + (size_t)sel[a] * p, xc, p, theta);
            forward_solve(L, j, kc, wc);
            double vc = (1.0 + eta) - dot(wc, wc, j);
            double cov = corr(x, xc, p, theta) - dot(wx, wc, j);
            double alc = (vc > 0.0) ? cov * cov / vc : -INFINITY;
            if (best < 0 || alc > a1 || (alc == a1 && C[ci] < C[best])) {
                a2 = a1;
                a1 = alc;
                best = ci;
            } else if (alc > a2) {
                a2 = alc;
            }
            if (replay && C[ci] == replay[j]) { follow = ci; a_follow = alc; }
        }
        if (best < 0 || a1 == -INFINITY) { rc = ORACLE_NOTPD; break; }
        if (vratio > 0.0) {
            const double vx = (1.0 + eta) - dot(wx, wx, j);
            const double vnext = vx - a1;
            if (vnext > 0.0 && vx / vnext < vratio) { nu = j; break; }
        }
        int64_t take = best;
        if (replay) {
            if (follow < 0) { rc = ORACLE_EINVAL; goto done; }
            take = follow;
        }
        if (diag) {
            diag[3 * j] = a1;
            diag[3 * j + 1] = a2;
            diag[3 * j + 2] = replay ? a_follow : a1;
        }
        sel[j] = C[take];
        used[take] = 1;
    }

    if (rc == ORACLE_OK) rc = lagp_oracle_predict(X, y, p, x, sel, nu, theta, eta, out);
    if (rc == ORACLE_NOTPD) {
        for (int i = 0; i < 5; i++) out[i] = NAN;
    }
    for (int j = nu; j < n; j++) sel[j] = -1;
    if (n_used) *n_used = nu;
done:
    free(C); free(used); free(K); free(L); free(kx); free(wx); free(kc); free(wc);
    return rc;
}

int lagp_oracle_local(const double *X, const double *y, int64_t N, int32_t p, const double *x,
                      int32_t n0, int32_t n, int64_t M, double theta, double eta,
                      const int32_t *replay, int32_t *sel, double *out, double *diag)
{
    return lagp_oracle_local_ex(X, y, N, p, x, n0, n, M, theta, eta, replay, NULL, 0.0, sel, NULL, out, diag);
}

/* Independent local designs over T predictive locations (Section 4.1),
 * parallel over locations with OpenMP.  n_per / M_per (nullable) override
 * n / M per location; sel is T x sel_stride.  out5 is T x 5 as in
 * lagp_oracle_local.  status[t] receives each location's return code.
 * Returns the first negative error, else 0. */
int lagp_oracle_batch(const double *X, const double *y, int64_t N, int32_t p, const double *XX,
                      int64_t T, int32_t n0, int32_t n, int64_t M, const int32_t *n_per,
                      const int32_t *M_per, double theta, double eta, int32_t *sel,
                      int64_t sel_stride, double *out5, int32_t *status, int32_t nthreads)
{
    int err = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t t = 0; t < T; t++) {
        int32_t nt = n_per ? n_per[t] : n;
        int64_t Mt = M_per ? M_per[t] : M;
        int rc = lagp_oracle_local(X, y, N, p, XX + (size_t)t * p, n0, nt, Mt, theta, eta, NULL,
                                   sel + (size_t)t * sel_stride, out5 + (size_t)t * 5, NULL);
        status[t] = rc;
        if (rc < 0) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            err = rc;
        }
    }
    (void)nthreads;
    return err;
}

/* ---- local lengthscale inference (Section 3.2, last paragraph, and the
 * two-stage scheme of Section 4.2; derivatives from SM Section 2, eqs dl and d2l).
 *
 * For the local design D (n indices) and lengthscale theta, with
 * K = K(D,D) + eta I, psi = Y'K^{-1}Y, the log marginal likelihood of eq gpk
 * (N -> n, dropping the theta-free constant) is
 *   l(theta) = -1/2 log|K| - n/2 log psi,
 * and with Kd = dK/dtheta, Kdd = d2K/dtheta2 (zero on the diagonal, whose
 * entries 1 + eta do not depend on theta; off the diagonal
 * dK/dtheta = K d^2/theta^2 and d2K/dtheta2 = K (d^4/theta^4 - 2 d^2/theta^3)):
 *   l'  = -1/2 tr(K^{-1} Kd) + n/2 Y'K^{-1}Kd K^{-1}Y / psi                 (eq dl)
 *   l'' = -1/2 tr(K^{-1} (Kdd - Kd K^{-1} Kd))
 *         + n/(2 psi) Y'K^{-1} (Kdd - 2 Kd K^{-1} Kd) K^{-1}Y
 *         + n/(2 psi^2) (Y'K^{-1}Kd K^{-1}Y)^2                             (eq d2l)
 * computed here from the explicit inverse K^{-1} = L^{-T} L^{-1}.
 * out3 = {l, l', l''}. */
int lagp_oracle_loglik(const double *X, const double *y, int32_t p, const int32_t *D, int32_t n,
                       double theta, double eta, double *out3)
{
    if (n < 1 || !(theta > 0.0)) return ORACLE_EINVAL;
    const size_t nn = (size_t)n * n;
    double *K = (double *)malloc(nn * sizeof(double));
    double *L = (double *)malloc(nn * sizeof(double));
    double *Li = (double *)calloc(nn, sizeof(double));
    double *Ki = (double *)malloc(nn * sizeof(double));
    double *Kd = (double *)malloc(nn * sizeof(double));
    double *Kdd = (double *)malloc(nn * sizeof(double));
    double *B = (double *)malloc(nn * sizeof(double));
    double *e = (double *)malloc((size_t)n * sizeof(double));
    double *col = (double *)malloc((size_t)n * sizeof(double));
    double *Yd = (double *)malloc((size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *v = (double *)malloc((size_t)n * sizeof(double));
    double *z = (double *)malloc((size_t)n * sizeof(double));
    int rc = ORACLE_OK;
    if (!K || !L || !Li || !Ki || !Kd || !Kdd || !B || !e || !col || !Yd || !w || !v || !z) {
        rc = ORACLE_ENOMEM;
        goto done;
    }
    design_cov(X, p, D, n, theta, eta, K);
    for (int a = 0; a < n; a++) {
        Yd[a] = y[D[a]];
        for (int b = 0; b < n; b++) {
            if (a == b) {
                Kd[(size_t)a * n + b] = 0.0;
                Kdd[(size_t)a * n + b] = 0.0;
            } else {
                const double d2 = sqdist(X + (size_t)D[a] * p, X + (size_t)D[b] * p, p);
                const double k = K[(size_t)a * n + b];
                Kd[(size_t)a * n + b] = k * d2 / (theta * theta);
                Kdd[(size_t)a * n + b] = k * (d2 * d2 / (theta * theta * theta * theta) - 2.0 * d2 / (theta * theta * theta));
            }
        }
    }
    if (cholesky(K, n, L) != 0) { rc = ORACLE_NOTPD; goto done; }
    /* L^{-1} column by column, then K^{-1} = L^{-T} L^{-1}. */
    for (int c = 0; c < n; c++) {
        for (int a = 0; a < n; a++) e[a] = (a == c) ? 1.0 : 0.0;
        forward_solve(L, n, e, col);
        for (int a = 0; a < n; a++) Li[(size_t)a * n + c] = col[a];
    }
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            double s = 0.0;
            for (int k = 0; k < n; k++) s += Li[(size_t)k * n + a] * Li[(size_t)k * n + b];
            Ki[(size_t)a * n + b] = s;
        }
    for (int a = 0; a < n; a++) w[a] = dot(Ki + (size_t)a * n, Yd, n);   /* K^{-1} Y */
    {
        double logdet = 0.0;
        for (int a = 0; a < n; a++) logdet += 2.0 * log(L[(size_t)a * n + a]);
        const double psi = dot(Yd, w, n);
        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++) {
                t1 += Ki[(size_t)a * n + b] * Kd[(size_t)b * n + a];
                t2 += Ki[(size_t)a * n + b] * Kdd[(size_t)b * n + a];
                double s = 0.0;
                for (int k = 0; k < n; k++) s += Ki[(size_t)a * n + k] * Kd[(size_t)k * n + b];
                B[(size_t)a * n + b] = s;                                     /* K^{-1} Kd */
            }
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++) t3 += B[(size_t)a * n + b] * B[(size_t)b * n + a];
        for (int a = 0; a < n; a++) v[a] = dot(Kd + (size_t)a * n, w, n);     /* Kd K^{-1} Y */
        for (int a = 0; a < n; a++) z[a] = dot(Kdd + (size_t)a * n, w, n);    /* Kdd K^{-1} Y */
        const double q = dot(w, v, n);
        const double r = dot(w, z, n);
        for (int a = 0; a < n; a++) e[a] = dot(Ki + (size_t)a * n, v, n);     /* K^{-1} Kd K^{-1} Y */
        const double sq = dot(v, e, n);
        out3[0] = -0.5 * logdet - 0.5 * n * log(psi);
        out3[1] = -0.5 * t1 + 0.5 * n * q / psi;
        out3[2] = -0.5 * (t2 - t3) + 0.5 * n * (r - 2.0 * sq) / psi + 0.5 * n * q * q / (psi * psi);
    }
done:
    free(K); free(L); free(Li); free(Ki); free(Kd); free(Kdd); free(B); free(e); free(col);
    free(Yd); free(w); free(v); free(z);
    return rc;
}

/* Maximum-likelihood lengthscale for the local design D by Newton's method
 * on l(theta) (the paper asks for a Newton-like method with the analytic
 * derivatives and leaves the details open).  From theta0 (or sqrt(tmin tmax)
 * when theta0 is outside (tmin, tmax)): where l'' < 0 the step is -l'/l''; elsewhere it is theta
 * in the direction of l' (doubling or zeroing theta).  A step that would
 * leave (tmin, tmax) goes half way to the bound instead.  Iteration stops
 * when a step moves theta by at most tol * theta, or after maxit steps.
 * Returns the final theta in *theta_hat and the step count in *iters. */
int lagp_oracle_mle(const double *X, const double *y, int32_t p, const int32_t *D, int32_t n,
                    double theta0, double eta, double tmin, double tmax, int32_t maxit, double tol,
                    double *theta_hat, int32_t *iters)
{
    if (n < 2 || !(tmin > 0.0) || !(tmax > tmin) || maxit < 1 || !(tol > 0.0)) return ORACLE_EINVAL;
    double theta = (theta0 > tmin && theta0 < tmax) ? theta0 : sqrt(tmin * tmax);
    int it = 0, rc = ORACLE_OK;
    while (it < maxit) {
        double l[3];
        rc = lagp_oracle_loglik(X, y, p, D, n, theta, eta, l);
        if (rc != ORACLE_OK) break;
        ++it;
        const double step = (l[2] < 0.0) ? -l[1] / l[2] : (l[1] > 0.0 ? theta : -theta);
        double next = theta + step;
        if (!(next > tmin)) next = 0.5 * (theta + tmin);
        if (!(next < tmax)) next = 0.5 * (theta + tmax);
        const int done = fabs(next - theta) <= tol * theta;
        theta = next;
        if (done) break;
    }
    *theta_hat = theta;
    *iters = it;
    return rc;
}

/* The two-stage scheme of Section 4.2 with one repetition (the paper's
 * "alc2"): designs at theta0, the local MLE theta1 from them, designs again
 * at theta1, the local MLE theta2 from those, and the prediction from the
 * second designs at theta2.  thetas = {theta1, theta2}; sel1, sel2 receive
 * the two designs; out5 as in lagp_oracle_local. */
int lagp_oracle_alc2(const double *X, const double *y, int64_t N, int32_t p, const double *x, int32_t n0,
                     int32_t n, int64_t M, double theta0, double eta, double tmin, double tmax,
                     int32_t maxit, double tol, int32_t *sel1, int32_t *sel2, double *thetas, double *out5)
{
    double o[5];
    int32_t its;
    int rc = lagp_oracle_local(X, y, N, p, x, n0, n, M, theta0, eta, NULL, sel1, o, NULL);
    if (rc != ORACLE_OK) return rc;
    rc = lagp_oracle_mle(X, y, p, sel1, n, theta0, eta, tmin, tmax, maxit, tol, &thetas[0], &its);
    if (rc != ORACLE_OK) return rc;
    rc = lagp_oracle_local(X, y, N, p, x, n0, n, M, thetas[0], eta, NULL, sel2, o, NULL);
    if (rc != ORACLE_OK) return rc;
    rc = lagp_oracle_mle(X, y, p, sel2, n, thetas[0], eta, tmin, tmax, maxit, tol, &thetas[1], &its);
    if (rc != ORACLE_OK) return rc;
    return lagp_oracle_predict(X, y, p, x, sel2, n, thetas[1], eta, out5);
}

/* ---- MSPE criterion (Section 3.1, eq mspe; expressions of Section 3.1 and
 * SM Section 2), at fixed theta as Section 3.2 recommends.
 *
 * For the design D (j >= 3 points) and each candidate c:
 *   J(c) = V_j(x|c) + (dmu_j(x)/dtheta)^2 / G_{j+1}(c),
 *   V_j(x|c)   = psi/(j-2) * v_{j+1}(x|c),  v_{j+1}(x|c) = v_j(x) - cov_j(x,c)^2 / v_j(c),
 *   dmu_j(z)   = (kd_j(z) - Kd K^{-1} k_j(z))' K^{-1} Y          (z = x or c),
 *   G_{j+1}(c) = F_j + dV_j(c)^2 / (2 V_j(c)^2) + dmu_j(c)^2 / V_j(c),
 *   V_j(c)     = psi/(j-2) * v_j(c),  F_j = -l''(theta) of the design (eq d2l),
 *   dV_j(c)    = d V_j(c) / dtheta = [-q v_j(c) - psi (2 kd_j(c)'K^{-1}k_j(c)
 *                                      - k_j(c)'K^{-1} Kd K^{-1} k_j(c))] / (j-2),
 * with q = Y'K^{-1} Kd K^{-1} Y = -dpsi/dtheta and kd_j(z) the derivatives of
 * K(x_i, z) in theta.  (The printed dV carries +q; the derivative of
 * psi v / (j-2) has -q, which is the reading taken.)  Everything is formed
 * from an explicit K^{-1} of a fresh Cholesky factor.  A candidate with
 * v_j(c) <= 0 scores +infinity.
 *   J[ncand]; parts (nullable) ncand x 5 = {V_j(x|c), dmu_j(c), dV_j(c), V_j(c), G};
 *   scal (nullable) = {F_j, dmu_j(x), psi, q, v_j(x)}. */
int lagp_oracle_mspe(const double *X, const double *y, int32_t p, const double *x, const int32_t *D, int32_t j,
                     const int32_t *cand, int32_t ncand, double theta, double eta, double *J, double *parts,
                     double *scal)
{
    if (j < 3 || ncand < 0 || !(theta > 0.0)) return ORACLE_EINVAL;
    double l3[3];
    int rc = lagp_oracle_loglik(X, y, p, D, j, theta, eta, l3);
    if (rc != ORACLE_OK) return rc;
    const size_t jj = (size_t)j * j;
    double *K = (double *)malloc(jj * sizeof(double));
    double *L = (double *)malloc(jj * sizeof(double));
    double *Ki = (double *)malloc(jj * sizeof(double));
    double *Kd = (double *)malloc(jj * sizeof(double));
    double *e = (double *)malloc((size_t)j * sizeof(double));
    double *col = (double *)malloc((size_t)j * sizeof(double));
    double *Yd = (double *)malloc((size_t)j * sizeof(double));
    double *al = (double *)malloc((size_t)j * sizeof(double));    /* K^{-1} Y */
    double *Kal = (double *)malloc((size_t)j * sizeof(double));   /* Kd K^{-1} Y */
    double *k = (double *)malloc((size_t)j * sizeof(double));
    double *kd = (double *)malloc((size_t)j * sizeof(double));
    double *kt = (double *)malloc((size_t)j * sizeof(double));    /* K^{-1} k */
    double *Kkt = (double *)malloc((size_t)j * sizeof(double));   /* Kd K^{-1} k */
    double *Li = (double *)calloc(jj, sizeof(double));
    if (!K || !L || !Ki || !Kd || !e || !col || !Yd || !al || !Kal || !k || !kd || !kt || !Kkt || !Li) {
        rc = ORACLE_ENOMEM;
        goto done;
    }
    design_cov(X, p, D, j, theta, eta, K);
    for (int a = 0; a < j; a++) {
        Yd[a] = y[D[a]];
        for (int b = 0; b < j; b++) {
            const double d2 = sqdist(X + (size_t)D[a] * p, X + (size_t)D[b] * p, p);
            Kd[(size_t)a * j + b] = (a == b) ? 0.0 : K[(size_t)a * j + b] * d2 / (theta * theta);
        }
    }
    if (cholesky(K, j, L) != 0) { rc = ORACLE_NOTPD; goto done; }
    for (int c = 0; c < j; c++) {
        for (int a = 0; a < j; a++) e[a] = (a == c) ? 1.0 : 0.0;
        forward_solve(L, j, e, col);
        for (int a = 0; a < j; a++) Li[(size_t)a * j + c] = col[a];
    }
    for (int a = 0; a < j; a++)
        for (int b = 0; b < j; b++) {
            double s = 0.0;
            for (int m = 0; m < j; m++) s += Li[(size_t)m * j + a] * Li[(size_t)m * j + b];
            Ki[(size_t)a * j + b] = s;
        }
    for (int a = 0; a < j; a++) al[a] = dot(Ki + (size_t)a * j, Yd, j);
    for (int a = 0; a < j; a++) Kal[a] = dot(Kd + (size_t)a * j, al, j);
    {
        const double psi = dot(Yd, al, j);
        const double q = dot(al, Kal, j);
        const double F = -l3[2];
        const double sc = psi / (j - 2);
        /* the predictive location */
        for (int a = 0; a < j; a++) {
            const double d2 = sqdist(X + (size_t)D[a] * p, x, p);
            k[a] = exp(-d2 / theta);
            kd[a] = k[a] * d2 / (theta * theta);
        }
        for (int a = 0; a < j; a++) kt[a] = dot(Ki + (size_t)a * j, k, j);
        const double vx = (1.0 + eta) - dot(k, kt, j);
        const double dmux = dot(kd, al, j) - dot(kt, Kal, j);
        double *kxs = (double *)malloc((size_t)j * sizeof(double));   /* k_j(x) */
        if (!kxs) { rc = ORACLE_ENOMEM; goto done; }
        memcpy(kxs, k, (size_t)j * sizeof(double));
        for (int ci = 0; ci < ncand; ci++) {
            const double *xc = X + (size_t)cand[ci] * p;
            for (int a = 0; a < j; a++) {
                const double d2 = sqdist(X + (size_t)D[a] * p, xc, p);
                k[a] = exp(-d2 / theta);
                kd[a] = k[a] * d2 / (theta * theta);
            }
            for (int a = 0; a < j; a++) kt[a] = dot(Ki + (size_t)a * j, k, j);
            for (int a = 0; a < j; a++) Kkt[a] = dot(Kd + (size_t)a * j, kt, j);
            const double vc = (1.0 + eta) - dot(k, kt, j);
            const double cov = exp(-sqdist(x, xc, p) / theta) - dot(kxs, kt, j);
            double Jc = INFINITY, vxc = NAN, dmuc = NAN, dVc = NAN, Vc = NAN, G = NAN;
            if (vc > 0.0) {
                vxc = sc * (vx - cov * cov / vc);
                Vc = sc * vc;
                dmuc = dot(kd, al, j) - dot(kt, Kal, j);
                dVc = (-q * vc - psi * (2.0 * dot(kd, kt, j) - dot(kt, Kkt, j))) / (j - 2);
                G = F + dVc * dVc / (2.0 * Vc * Vc) + dmuc * dmuc / Vc;
                Jc = vxc + dmux * dmux / G;
            }
            J[ci] = Jc;
            if (parts) {
                parts[5 * ci] = vxc;
                parts[5 * ci + 1] = dmuc;
                parts[5 * ci + 2] = dVc;
                parts[5 * ci + 3] = Vc;
                parts[5 * ci + 4] = G;
            }
        }
        if (scal) {
            scal[0] = F;
            scal[1] = dmux;
            scal[2] = psi;
            scal[3] = q;
            scal[4] = vx;
        }
        free(kxs);
    }
done:
    free(K); free(L); free(Ki); free(Kd); free(e); free(col); free(Yd); free(al); free(Kal);
    free(k); free(kd); free(kt); free(Kkt); free(Li);
    return rc;
}

/* Greedy MSPE local design (Section 3.1): from the n0 >= 3 nearest
 * neighbours, add the candidate with the smallest J(c) until n points (ties
 * to the smaller design index), then predict as lagp_oracle_local does.
 * diag (nullable, n x 2): the smallest and second smallest J per step. */
int lagp_oracle_mspe_local(const double *X, const double *y, int64_t N, int32_t p, const double *x, int32_t n0,
                           int32_t n, int64_t M, double theta, double eta, int32_t *sel, double *out, double *diag)
{
    if (N < 1 || p < 1 || n0 < 3 || n0 > n || (int64_t)n > M || M > N || !(theta > 0.0) || !(eta >= 0.0))
        return ORACLE_EINVAL;
    int32_t *C = (int32_t *)malloc((size_t)M * sizeof(int32_t));
    int32_t *live = (int32_t *)malloc((size_t)M * sizeof(int32_t));
    char *used = (char *)calloc((size_t)M, 1);
    double *J = (double *)malloc((size_t)M * sizeof(double));
    int rc = ORACLE_OK;
    if (!C || !live || !used || !J) { rc = ORACLE_ENOMEM; goto done; }
    rc = lagp_oracle_knn(X, N, p, x, M, C, NULL);
    if (rc != ORACLE_OK) goto done;
    for (int j = 0; j < n0; j++) {
        sel[j] = C[j];
        used[j] = 1;
        if (diag) diag[2 * j] = diag[2 * j + 1] = NAN;
    }
    for (int j = n0; j < n; j++) {
        int32_t nl = 0;
        for (int64_t ci = 0; ci < M; ci++)
            if (!used[ci]) live[nl++] = C[ci];
        rc = lagp_oracle_mspe(X, y, p, x, sel, j, live, nl, theta, eta, J, NULL, NULL);
        if (rc != ORACLE_OK) break;
        double j1 = INFINITY, j2 = INFINITY;
        int32_t best = -1;
        for (int32_t a = 0; a < nl; a++) {
            if (best < 0 || J[a] < j1 || (J[a] == j1 && live[a] < live[best])) {
                j2 = j1;
                j1 = J[a];
                best = a;
            } else if (J[a] < j2) {
                j2 = J[a];
            }
        }
        if (best < 0 || j1 == INFINITY) { rc = ORACLE_NOTPD; break; }
        if (diag) { diag[2 * j] = j1; diag[2 * j + 1] = j2; }
        sel[j] = live[best];
        for (int64_t ci = 0; ci < M; ci++)
            if (C[ci] == live[best]) used[ci] = 1;
    }
    if (rc == ORACLE_OK) rc = lagp_oracle_predict(X, y, p, x, sel, n, theta, eta, out);
    if (rc == ORACLE_NOTPD)
        for (int i = 0; i < 5; i++) out[i] = NAN;
done:
    free(C); free(live); free(used); free(J);
    return rc;
}

int lagp_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
