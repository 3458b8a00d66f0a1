/*
 * CPU FP64 ORACLE for the generalized shifted equations (zB - A) x = e_j.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the tests, the smoke check
 * and the CPU-baseline leg of the benchmark; the product path never links or
 * calls it.  It shares no code with the GPU library.
 *
 * What it computes (paper Sec. III-A, Eqs. 9, 10 and 13): for every requested
 * column j and every complex energy z_k (Im z_k > 0) the vector
 *     x_{j,k} = (z_k B - A)^{-1} e_j,
 * where A is real symmetric and B is real symmetric positive definite
 * (Sec. II-A).  The solver is a plain Krylov method on the shifted family
 * (Sec. III-B, Eq. 14): all shifts share one Krylov subspace.
 *
 * Method (written from the mathematics, no listing exists in the paper):
 *  - Left-preconditioning by B turns the family into truly shifted systems
 *        (z_k I - B^{-1} A) x = B^{-1} e_j,
 *    whose matrices differ only by multiples of the identity, so their
 *    Krylov subspaces coincide.
 *  - A seed system z_s (the shift with the median real part) is solved with
 *    the conjugate orthogonal CG method (COCG: CG with the unconjugated
 *    bilinear form u^T r, valid because z_s B - A is complex symmetric), with
 *    B^{-1} as preconditioner.  B^{-1} is applied by plain CG on B
 *    (real and imaginary parts separately) to a tight relative tolerance.
 *  - Shifted residuals stay collinear with the seed residual,
 *        r_k = r / pi_k,
 *    where pi_k = R_n(-sigma_k) is the seed's COCG residual polynomial
 *    evaluated at minus the shift difference sigma_k = z_k - z_s.  The
 *    three-term recurrence of that polynomial gives pi_k, and from it the
 *    step lengths alpha_k and beta_k of each shifted system.
 *  - Convergence per (j,k): ||r|| / |pi_k| <= tol (||e_j|| = 1); converged
 *    shifts are frozen.  The final true residual ||e_j - (z_k B - A) x||_2
 *    is recomputed with this file's own CSR product.
 *
 * Everything is FP64 (complex as two doubles), scalar CSR, one column per
 * OpenMP thread (the paper computes each projected quantity single-threaded,
 * Sec. III-C).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int n;
    const int64_t *rp;
    const int32_t *ci;
    const double *v;
} csr_t;

/* y = X v (real) */
static void spmv(const csr_t *X, const double *v, double *y) {
    for (int i = 0; i < X->n; ++i) {
        double s = 0.0;
        for (int64_t p = X->rp[i]; p < X->rp[i + 1]; ++p) s += X->v[p] * v[X->ci[p]];
        y[i] = s;
    }
}

static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Plain CG on B x = s (x0 = 0).  Stops when ||s - Bx|| <= tol ||s||.
 * Returns the number of iterations, or -1 if max_it was reached.
 * work: 3n doubles. */
static int cg_B(const csr_t *B, const double *s, double *x, double tol, int max_it, double *work) {
    const int n = B->n;
    double *r = work, *p = work + n, *q = work + 2 * n;
    double ss = dot(n, s, s);
    memset(x, 0, sizeof(double) * n);
    if (ss == 0.0) return 0;
    memcpy(r, s, sizeof(double) * n);
    memcpy(p, s, sizeof(double) * n);
    double rr = ss;
    const double stop = tol * tol * ss;
    for (int it = 1; it <= max_it; ++it) {
        spmv(B, p, q);
        double pq = dot(n, p, q);
        double a = rr / pq;
        for (int i = 0; i < n; ++i) {
            x[i] += a * p[i];
            r[i] -= a * q[i];
        }
        double rr2 = dot(n, r, r);
        if (rr2 <= stop) return it;
        double b = rr2 / rr;
        rr = rr2;
        for (int i = 0; i < n; ++i) p[i] = r[i] + b * p[i];
    }
    return -1;
}

int oracle_cg_B(int n, const int64_t *rp, const int32_t *ci, const double *v, const double *s, double *x,
                double tol, int max_it) {
    csr_t B = {n, rp, ci, v};
    double *w = (double *)malloc(sizeof(double) * 3 * n);
    int it = cg_B(&B, s, x, tol, max_it, w);
    free(w);
    return it;
}

/* complex u = B^{-1} r, solving the real and imaginary parts separately */
static int cg_B_cplx(const csr_t *B, const cplx *r, cplx *u, double tol, int max_it, double *work) {
    const int n = B->n;
    double *sr = work, *si = work + n, *xr = work + 2 * n, *xi = work + 3 * n, *w = work + 4 * n;
    for (int i = 0; i < n; ++i) {
        sr[i] = creal(r[i]);
        si[i] = cimag(r[i]);
    }
    int a = cg_B(B, sr, xr, tol, max_it, w);
    int b = cg_B(B, si, xi, tol, max_it, w);
    for (int i = 0; i < n; ++i) u[i] = xr[i] + I * xi[i];
    if (a < 0 || b < 0) return -1;
    return a > b ? a : b;
}

/* bilinear (unconjugated) complex dot */
static cplx bdot(int n, const cplx *a, const cplx *b) {
    cplx s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double cnorm(int n, const cplx *a) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return sqrt(s);
}

/* Seed: index of the shift with the median real part (ties -> lower index). */
static int median_seed(int K, const cplx *z) {
    int *idx = (int *)malloc(sizeof(int) * K);
    for (int k = 0; k < K; ++k) idx[k] = k;
    for (int a = 1; a < K; ++a) { /* insertion sort by (Re z, index) */
        int t = idx[a], b = a - 1;
        while (b >= 0 && (creal(z[idx[b]]) > creal(z[t]) || (creal(z[idx[b]]) == creal(z[t]) && idx[b] > t))) {
            idx[b + 1] = idx[b];
            --b;
        }
        idx[b + 1] = t;
    }
    int s = idx[(K - 1) / 2];
    free(idx);
    return s;
}

/* True residual norm ||e_j - (z B - A) x||_2 for one complex x. work: 4n doubles */
static double true_residual(const csr_t *A, const csr_t *B, int j, cplx z, const cplx *x, double *work) {
    const int n = A->n;
    double *xr = work, *xi = work + n, *t1 = work + 2 * n, *t2 = work + 3 * n;
    for (int i = 0; i < n; ++i) {
        xr[i] = creal(x[i]);
        xi[i] = cimag(x[i]);
    }
    /* (zB - A) x = z (B x) - A x ; compute real and imaginary parts */
    double *bxr = (double *)malloc(sizeof(double) * n * 4);
    double *bxi = bxr + n, *axr = bxr + 2 * n, *axi = bxr + 3 * n;
    spmv(B, xr, bxr);
    spmv(B, xi, bxi);
    spmv(A, xr, axr);
    spmv(A, xi, axi);
    (void)t1;
    (void)t2;
    const double zr = creal(z), zi = cimag(z);
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        double re = zr * bxr[i] - zi * bxi[i] - axr[i];
        double im = zr * bxi[i] + zi * bxr[i] - axi[i];
        re = (i == j ? 1.0 : 0.0) - re;
        im = -im;
        s += re * re + im * im;
    }
    free(bxr);
    return sqrt(s);
}

/*
 * Solve one column j for all K shifts.  xs: K*n complex (full vectors, output).
 * conv_it[k]: iteration at which shift k converged (-1 if never).
 * est[k]: final residual estimate ||r|| / |pi_k|.
 * Returns the number of outer iterations, negative on inner-solve failure.
 */
static int cocg_column(const csr_t *A, const csr_t *B, int j, int K, const cplx *z, double tol, int max_it,
                       double inner_tol, int inner_max, cplx *xs, int *conv_it, double *est, int *inner_fail) {
    const int n = A->n;
    const int s_idx = median_seed(K, z);
    const cplx zs = z[s_idx];
    cplx *r = (cplx *)calloc((size_t)n, sizeof(cplx));
    cplx *u = (cplx *)calloc((size_t)n, sizeof(cplx));
    cplx *p = (cplx *)calloc((size_t)n, sizeof(cplx));
    cplx *q = (cplx *)calloc((size_t)n, sizeof(cplx));
    cplx *ps = (cplx *)calloc((size_t)K * n, sizeof(cplx));
    double *work = (double *)malloc(sizeof(double) * 8 * n);
    double *pr = (double *)malloc(sizeof(double) * n), *pi_ = (double *)malloc(sizeof(double) * n);
    double *bpr = (double *)malloc(sizeof(double) * n), *bpi = (double *)malloc(sizeof(double) * n);
    double *apr = (double *)malloc(sizeof(double) * n), *api = (double *)malloc(sizeof(double) * n);
    cplx *pik = (cplx *)malloc(sizeof(cplx) * K), *pik_old = (cplx *)malloc(sizeof(cplx) * K);
    cplx *sig = (cplx *)malloc(sizeof(cplx) * K);
    char *done = (char *)calloc((size_t)K, 1);

    memset(xs, 0, sizeof(cplx) * (size_t)K * n);
    r[j] = 1.0;
    if (cg_B_cplx(B, r, u, inner_tol, inner_max, work) < 0) (*inner_fail)++;
    for (int i = 0; i < n; ++i) p[i] = u[i];
    for (int k = 0; k < K; ++k) {
        memcpy(ps + (size_t)k * n, u, sizeof(cplx) * n);
        pik[k] = 1.0;
        pik_old[k] = 1.0;
        sig[k] = z[k] - zs;
        conv_it[k] = -1;
        est[k] = 1.0;
    }
    cplx gamma = bdot(n, u, r);
    cplx alpha_old = 1.0, beta_old = 0.0;
    int it = 0;
    int remaining = K;
    while (remaining > 0 && it < max_it) {
        ++it;
        /* q = (zs B - A) p */
        for (int i = 0; i < n; ++i) {
            pr[i] = creal(p[i]);
            pi_[i] = cimag(p[i]);
        }
        spmv(B, pr, bpr);
        spmv(B, pi_, bpi);
        spmv(A, pr, apr);
        spmv(A, pi_, api);
        for (int i = 0; i < n; ++i) q[i] = zs * (bpr[i] + I * bpi[i]) - (apr[i] + I * api[i]);
        cplx delta = bdot(n, p, q);
        cplx alpha = gamma / delta;
        /* shifted systems: new collinearity factors and step lengths */
        for (int k = 0; k < K; ++k) {
            if (done[k]) continue;
            cplx pnew = (1.0 + alpha * sig[k]) * pik[k] + (alpha * beta_old / alpha_old) * (pik[k] - pik_old[k]);
            cplx ak = alpha * pik[k] / pnew;
            cplx *xk = xs + (size_t)k * n, *pk = ps + (size_t)k * n;
            for (int i = 0; i < n; ++i) xk[i] += ak * pk[i];
            pik_old[k] = pik[k];
            pik[k] = pnew;
        }
        /* seed residual and preconditioned residual */
        for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];
        if (cg_B_cplx(B, r, u, inner_tol, inner_max, work) < 0) (*inner_fail)++;
        cplx gamma_new = bdot(n, u, r);
        cplx beta = gamma_new / gamma;
        for (int k = 0; k < K; ++k) {
            if (done[k]) continue;
            cplx ratio = pik_old[k] / pik[k];
            cplx bk = ratio * ratio * beta;
            cplx *pk = ps + (size_t)k * n;
            cplx inv = 1.0 / pik[k];
            for (int i = 0; i < n; ++i) pk[i] = inv * u[i] + bk * pk[i];
        }
        for (int i = 0; i < n; ++i) p[i] = u[i] + beta * p[i];
        alpha_old = alpha;
        beta_old = beta;
        gamma = gamma_new;
        double rn = cnorm(n, r);
        for (int k = 0; k < K; ++k) {
            if (done[k]) continue;
            est[k] = rn / cabs(pik[k]);
            if (est[k] <= tol) {
                done[k] = 1;
                conv_it[k] = it;
                --remaining;
            }
        }
    }
    free(r); free(u); free(p); free(q); free(ps); free(work);
    free(pr); free(pi_); free(bpr); free(bpi); free(apr); free(api);
    free(pik); free(pik_old); free(sig); free(done);
    return it;
}

/*
 * Solve columns cols[0..ncols) for shifts z (K complex, re/im interleaved).
 *
 *   full_out = 1 : x_out holds [ncols][K][n] complex (re, im interleaved)
 *   full_out = 0 : x_out holds, for column c, the entries on the pattern
 *                  P_j = { i : B_ij structurally present } in ascending i,
 *                  laid out [K][|P_j|] at complex offset pat_off[c] * K.
 * iters_out[c] : outer iterations; conv_it_out[c*K+k]: iteration of
 * convergence (-1: not converged); est_out/true_out[c*K+k]: residual
 * estimate and recomputed true residual.  max_it caps the outer iterations
 * (used to time a bounded sample).  Returns the number of inner-solve
 * failures (0 on success).
 */
int oracle_shifted_solve(int n, const int64_t *rpA, const int32_t *ciA, const double *vA, const int64_t *rpB,
                         const int32_t *ciB, const double *vB, int ncols, const int32_t *cols, int K,
                         const double *zri, double tol, int max_it, double inner_tol, int inner_max, int full_out,
                         const int64_t *pat_off, double *x_out, int32_t *iters_out, int32_t *conv_it_out,
                         double *est_out, double *true_out, int nthreads) {
    csr_t A = {n, rpA, ciA, vA}, B = {n, rpB, ciB, vB};
    cplx *z = (cplx *)malloc(sizeof(cplx) * K);
    for (int k = 0; k < K; ++k) z[k] = zri[2 * k] + I * zri[2 * k + 1];
    int fails = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
    for (int c = 0; c < ncols; ++c) {
        const int j = cols[c];
        cplx *xs = (cplx *)malloc(sizeof(cplx) * (size_t)K * n);
        int *cit = (int *)malloc(sizeof(int) * K);
        double *est = (double *)malloc(sizeof(double) * K);
        double *work = (double *)malloc(sizeof(double) * 4 * n);
        int f = 0;
        int it = cocg_column(&A, &B, j, K, z, tol, max_it, inner_tol, inner_max, xs, cit, est, &f);
        fails += f;
        iters_out[c] = it;
        for (int k = 0; k < K; ++k) {
            conv_it_out[(size_t)c * K + k] = cit[k];
            est_out[(size_t)c * K + k] = est[k];
            if (true_out) true_out[(size_t)c * K + k] = true_residual(&A, &B, j, z[k], xs + (size_t)k * n, work);
        }
        if (full_out) {
            memcpy(x_out + (size_t)2 * c * K * n, xs, sizeof(cplx) * (size_t)K * n);
        } else {
            const int64_t b0 = B.rp[j], b1 = B.rp[j + 1];
            const int64_t plen = b1 - b0;
            double *dst = x_out + 2 * pat_off[c] * K;
            for (int k = 0; k < K; ++k)
                for (int64_t p = 0; p < plen; ++p) {
                    cplx v = xs[(size_t)k * n + B.ci[b0 + p]];
                    dst[2 * (k * plen + p)] = creal(v);
                    dst[2 * (k * plen + p) + 1] = cimag(v);
                }
        }
        free(xs); free(cit); free(est); free(work);
    }
    free(z);
    return fails;
}

/* y = X v for tests of the CSR product itself */
void oracle_spmv(int n, const int64_t *rp, const int32_t *ci, const double *v, const double *x, double *y) {
    csr_t X = {n, rp, ci, v};
    spmv(&X, x, y);
}

/* residual of a caller-supplied full x (complex, re/im interleaved) */
double oracle_true_residual(int n, const int64_t *rpA, const int32_t *ciA, const double *vA, const int64_t *rpB,
                            const int32_t *ciB, const double *vB, int j, double zr, double zi, const double *x) {
    csr_t A = {n, rpA, ciA, vA}, B = {n, rpB, ciB, vB};
    double *work = (double *)malloc(sizeof(double) * 4 * n);
    double r = true_residual(&A, &B, j, zr + I * zi, (const cplx *)x, work);
    free(work);
    return r;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
