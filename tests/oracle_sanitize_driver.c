/*
 * Runs every routine of oracle/oracle.c on small symmetric-definite pencils
 * (orders 1..40) so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks their memory accesses and arithmetic; also
 * checks A Y = B Y Lambda and Y^T B Y = I so that the run computes something.
 * Exit status 0 on success.  Built and run by tests/test_oracle_sanitize.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_threads(void);
void orc_symmetrize_lower(int64_t n, const double *a, int64_t lda, double *s);
int64_t orc_cholesky(int64_t n, double *l, int64_t ld);
void orc_reduce(int64_t n, const double *a, int64_t lda, const double *l, int64_t ldl, double *c);
void orc_back_transform(int64_t n, int64_t ncol, const double *l, int64_t ldl, double *z,
                        int64_t ldz);
void orc_tridiagonalize(int64_t n, double *c, double *d, double *e, double *beta);
void orc_form_q(int64_t n, const double *c, const double *beta, double *q);
int64_t orc_sturm_count(int64_t n, const double *d, const double *e, double x);
void orc_bisect_all(int64_t n, const double *d, const double *e, double *w);
int64_t orc_tql(int64_t n, double *d, double *e_in, double *z, int64_t ldz);

static double urand(uint64_t *s) {
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

static int run(int64_t n, uint64_t seed) {
    size_t nn = (size_t)n * (size_t)n;
    double *a = malloc(nn * sizeof(double)), *b = malloc(nn * sizeof(double));
    double *l = malloc(nn * sizeof(double)), *c = malloc(nn * sizeof(double));
    double *q = malloc(nn * sizeof(double)), *y = malloc(nn * sizeof(double));
    double *d = malloc((size_t)n * sizeof(double)), *e = malloc((size_t)(n > 1 ? n : 1) * sizeof(double));
    double *beta = calloc((size_t)n, sizeof(double)), *w = malloc((size_t)n * sizeof(double));
    double *d2 = malloc((size_t)n * sizeof(double)), *e2 = malloc((size_t)(n > 1 ? n : 1) * sizeof(double));
    uint64_t s = seed;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i < n; ++i) {
            double x = urand(&s), z = (i == j) ? 1.0 + 0.2 * fabs(urand(&s)) : 0.3 * urand(&s) / (double)n;
            a[i + j * n] = a[j + i * n] = x;
            b[i + j * n] = b[j + i * n] = z;
        }
    for (size_t k = 0; k < nn; ++k) l[k] = b[k];
    if (orc_cholesky(n, l, n) != 0) return 1;
    orc_reduce(n, a, n, l, n, c);
    orc_tridiagonalize(n, c, d, e, beta);
    for (int64_t i = 0; i < n; ++i) d2[i] = d[i];
    for (int64_t i = 0; i + 1 < n; ++i) e2[i] = e[i];
    orc_bisect_all(n, d, e, w);
    if (n > 0 && orc_sturm_count(n, d, e, w[n - 1] + 1.0) != n) return 2;
    orc_form_q(n, c, beta, q);
    if (orc_tql(n, d2, e2, q, n) != 0) return 3;
    for (size_t k = 0; k < nn; ++k) y[k] = q[k];
    orc_back_transform(n, n, l, n, y, n);
    /* residual and B-orthogonality (d2 holds the QL eigenvalues, unsorted) */
    double res = 0.0, orth = 0.0;
    for (int64_t k = 0; k < n; ++k)
        for (int64_t i = 0; i < n; ++i) {
            double ay = 0.0, by = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                ay += a[i + j * n] * y[j + k * n];
                by += b[i + j * n] * y[j + k * n];
            }
            double r = fabs(ay - d2[k] * by);
            if (r > res) res = r;
        }
    for (int64_t k = 0; k < n; ++k)
        for (int64_t m = 0; m < n; ++m) {
            double g = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double by = 0.0;
                for (int64_t j = 0; j < n; ++j) by += b[i + j * n] * y[j + m * n];
                g += y[i + k * n] * by;
            }
            g -= (k == m) ? 1.0 : 0.0;
            if (fabs(g) > orth) orth = fabs(g);
        }
    free(a); free(b); free(l); free(c); free(q); free(y); free(d); free(e); free(beta); free(w);
    free(d2); free(e2);
    if (!(res < 1e-12 && orth < 1e-12)) {
        fprintf(stderr, "n=%lld res=%g orth=%g\n", (long long)n, res, orth);
        return 4;
    }
    return 0;
}

int main(void) {
    for (int64_t n = 1; n <= 40; n += (n < 10 ? 1 : 7)) {
        int rc = run(n, 1000 + (uint64_t)n);
        if (rc) {
            fprintf(stderr, "order %lld failed (%d)\n", (long long)n, rc);
            return rc;
        }
    }
    printf("sanitized oracle run ok (%d threads)\n", orc_threads());
    return 0;
}
