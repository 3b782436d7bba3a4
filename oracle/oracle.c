/*
 * Plain, slow, FP64 CPU oracle for the generalized symmetric-definite eigenproblem
 *     A y_k = lambda_k B y_k          (section 1, Eq. 1)
 *     A Y = B Y Lambda,  Y^T B Y = I  (section 3.1, Eq. 2)
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls this
 * file; it exists so that tests and the benchmark's CPU baseline can check the GPU
 * library against an independent computation.  It shares no code with the GPU path.
 *
 * Route (deliberately different from the GPU route so that a shared mistake is
 * unlikely): textbook Cholesky, two forward substitutions for the reduced matrix,
 * one-stage unblocked Householder tridiagonalisation, Sturm bisection for the
 * eigenvalues, implicit QL with accumulated rotations for the eigenvectors, and a
 * back substitution for Y.  No blocking, no fusion.  Built with
 * -O2 -ffp-contract=off and no fast-math.
 *
 * Storage: column-major, element (i, j) at a[i + j*ld].  Only the lower triangle of
 * the symmetric inputs is read.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(a, i, j, ld) ((a)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Copy the lower triangle of a into both triangles of s (ld = n). */
void orc_symmetrize_lower(int64_t n, const double *a, int64_t lda, double *s) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            AT(s, i, j, n) = (i >= j) ? AT(a, i, j, lda) : AT(a, j, i, lda);
}

/*
 * Cholesky factorisation B = L L^T (section 3.1, Eq. 4, written with L = U^T).
 * Outer-product form: for each column j, take the square root of the pivot, scale
 * the column below it, and subtract the rank-one term from the trailing columns.
 * On entry l holds B (lower triangle read); on exit its lower triangle is L and its
 * strict upper triangle is zero.  Returns 0, or k (1-based) if the k-th pivot is not
 * positive (the leading minor of order k is not positive definite).
 */
int64_t orc_cholesky(int64_t n, double *l, int64_t ld) {
    for (int64_t j = 0; j < n; ++j) {
        double piv = AT(l, j, j, ld);
        if (!(piv > 0.0)) return j + 1;
        double ljj = sqrt(piv);
        AT(l, j, j, ld) = ljj;
        for (int64_t i = j + 1; i < n; ++i) AT(l, i, j, ld) /= ljj;
#pragma omp parallel for schedule(static) if (n - j > 256)
        for (int64_t k = j + 1; k < n; ++k) {
            double lkj = AT(l, k, j, ld);
            for (int64_t i = k; i < n; ++i) AT(l, i, k, ld) -= AT(l, i, j, ld) * lkj;
        }
    }
    for (int64_t j = 1; j < n; ++j)
        for (int64_t i = 0; i < j; ++i) AT(l, i, j, ld) = 0.0;
    return 0;
}

/* x <- L^{-1} x for one column, column-oriented forward substitution. */
static void fwd_subst(int64_t n, const double *l, int64_t ld, double *x) {
    for (int64_t k = 0; k < n; ++k) {
        double xk = x[k] / AT(l, k, k, ld);
        x[k] = xk;
        const double *col = &AT(l, 0, k, ld);
        for (int64_t i = k + 1; i < n; ++i) x[i] -= col[i] * xk;
    }
}

/* x <- L^{-T} x for one column: back substitution with the rows of L^T, which are
 * the columns of L. */
static void bwd_subst_t(int64_t n, const double *l, int64_t ld, double *x) {
    for (int64_t k = n - 1; k >= 0; --k) {
        const double *col = &AT(l, 0, k, ld);
        double s = x[k];
        for (int64_t i = k + 1; i < n; ++i) s -= col[i] * x[i];
        x[k] = s / col[k];
    }
}

/*
 * Reduced matrix C = L^{-1} A L^{-T} (section 3.1, Eq. 5, with L = U^T), formed
 * without an explicit inverse: X = L^{-1} A column by column, then, because A is
 * symmetric, C = L^{-1} X^T column by column.  The result is symmetrised as
 * (C + C^T)/2.  a: lower triangle read; c: n x n output (ld n).
 */
void orc_reduce(int64_t n, const double *a, int64_t lda, const double *l, int64_t ldl,
                double *c) {
    double *x = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    orc_symmetrize_lower(n, a, lda, x);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < n; ++j) fwd_subst(n, l, ldl, &AT(x, 0, j, n));
    /* c = x^T */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) AT(c, i, j, n) = AT(x, j, i, n);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < n; ++j) fwd_subst(n, l, ldl, &AT(c, 0, j, n));
    /* symmetrise */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j + 1; i < n; ++i) {
            double v = 0.5 * (AT(c, i, j, n) + AT(c, j, i, n));
            AT(c, i, j, n) = v;
            AT(c, j, i, n) = v;
        }
    free(x);
}

/* Y = L^{-T} Z, column by column (section 3.1, Eq. 6 with U^{-1} = L^{-T}). */
void orc_back_transform(int64_t n, int64_t ncol, const double *l, int64_t ldl, double *z,
                        int64_t ldz) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < ncol; ++j) bwd_subst_t(n, l, ldl, &AT(z, 0, j, ldz));
}

/*
 * One-stage Householder tridiagonalisation of the full symmetric matrix c (ld n):
 * c = Q T Q^T, Q = H_0 H_1 ... H_{n-3}, H_k = I - beta_k v_k v_k^T acting on rows
 * k+1..n-1.  Step k: v from column k below the diagonal (v_0 = 1), p = beta C22 v,
 * w = p - (beta p^T v / 2) v, C22 <- C22 - v w^T - w v^T.  On exit d[0..n-1] is the
 * diagonal of T, e[0..n-2] the subdiagonal, v_k is stored in c[k+2.., k] and beta_k
 * in beta[k].
 */
void orc_tridiagonalize(int64_t n, double *c, double *d, double *e, double *beta) {
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t k = 0; k + 2 < n; ++k) {
        int64_t m = n - k - 1; /* length of x = c[k+1.., k] */
        double *x = &AT(c, k + 1, k, n);
        double sigma = 0.0;
        for (int64_t i = 1; i < m; ++i) sigma += x[i] * x[i];
        double x0 = x[0];
        double b = 0.0;
        v[0] = 1.0;
        for (int64_t i = 1; i < m; ++i) v[i] = x[i];
        double alpha;
        if (sigma == 0.0) {
            b = 0.0;
            alpha = x0;
        } else {
            double mu = sqrt(x0 * x0 + sigma);
            /* v0 = x0 - mu computed without cancellation */
            double v0 = (x0 <= 0.0) ? x0 - mu : -sigma / (x0 + mu);
            b = 2.0 * v0 * v0 / (sigma + v0 * v0);
            for (int64_t i = 1; i < m; ++i) v[i] = x[i] / v0;
            alpha = mu;
        }
        beta[k] = b;
        /* H x = alpha e_1 */
        x[0] = alpha;
        for (int64_t i = 1; i < m; ++i) x[i] = v[i];
        AT(c, k, k + 1, n) = alpha;
        if (b == 0.0) continue;
        double *c22 = &AT(c, k + 1, k + 1, n);
        /* p = b * C22 v  (C22 full symmetric, column-major, ld n) */
#pragma omp parallel for schedule(static) if (m > 256)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < m; ++j) s += AT(c22, j, i, n) * v[j]; /* row i = column i */
            p[i] = b * s;
        }
        double pv = 0.0;
        for (int64_t i = 0; i < m; ++i) pv += p[i] * v[i];
        double half = 0.5 * b * pv;
        for (int64_t i = 0; i < m; ++i) p[i] -= half * v[i]; /* p is now w */
#pragma omp parallel for schedule(static) if (m > 256)
        for (int64_t j = 0; j < m; ++j) {
            double vj = v[j], wj = p[j];
            double *col = &AT(c22, 0, j, n);
            for (int64_t i = 0; i < m; ++i) col[i] -= v[i] * wj + p[i] * vj;
        }
    }
    for (int64_t k = 0; k < n; ++k) d[k] = AT(c, k, k, n);
    for (int64_t k = 0; k + 1 < n; ++k) e[k] = AT(c, k + 1, k, n);
    free(v);
    free(p);
}

/* Q = H_0 H_1 ... H_{n-3} formed explicitly from the reflectors left in c by
 * orc_tridiagonalize (backward accumulation: Q <- H_k Q for k = n-3 .. 0). */
void orc_form_q(int64_t n, const double *c, const double *beta, double *q) {
    memset(q, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int64_t i = 0; i < n; ++i) AT(q, i, i, n) = 1.0;
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t k = n - 3; k >= 0; --k) {
        double b = beta[k];
        if (b == 0.0) continue;
        int64_t m = n - k - 1;
        v[0] = 1.0;
        for (int64_t i = 1; i < m; ++i) v[i] = AT(c, k + 1 + i, k, n);
#pragma omp parallel for schedule(static) if (m > 256)
        for (int64_t j = k + 1; j < n; ++j) {
            double *col = &AT(q, k + 1, j, n);
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += v[i] * col[i];
            s *= b;
            for (int64_t i = 0; i < m; ++i) col[i] -= s * v[i];
        }
    }
    free(v);
}

/* Number of eigenvalues of the symmetric tridiagonal (d, e) that are < x: the number
 * of negative pivots of the LDL^T factorisation of T - x I (Sylvester's law of
 * inertia).  A zero pivot is replaced by a tiny negative number. */
int64_t orc_sturm_count(int64_t n, const double *d, const double *e, double x) {
    int64_t cnt = 0;
    double q = d[0] - x;
    const double tiny = DBL_MIN / DBL_EPSILON;
    if (q == 0.0) q = -tiny;
    if (q < 0.0) ++cnt;
    for (int64_t i = 1; i < n; ++i) {
        q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
        if (q == 0.0) q = -tiny;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

/* All eigenvalues of the tridiagonal (d, e), ascending, by bisection on Sturm counts
 * inside the Gershgorin interval.  Each interval is halved until its width is below
 * 2 eps max(|lo|, |hi|) or an absolute floor of eps * ||T||_1. */
void orc_bisect_all(int64_t n, const double *d, const double *e, double *w) {
    double lo = INFINITY, hi = -INFINITY, tnorm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = 0.0;
        if (i > 0) r += fabs(e[i - 1]);
        if (i + 1 < n) r += fabs(e[i]);
        if (d[i] - r < lo) lo = d[i] - r;
        if (d[i] + r > hi) hi = d[i] + r;
        if (fabs(d[i]) + r > tnorm) tnorm = fabs(d[i]) + r;
    }
    double pad = 2.0 * DBL_EPSILON * tnorm + DBL_MIN;
    lo -= pad;
    hi += pad;
    const double floor_abs = DBL_EPSILON * tnorm;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        /* find x with count(x) <= k < count(hi): lambda_k in [a, b) */
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (a + b);
            double tol = 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b));
            if (tol < floor_abs) tol = floor_abs;
            if (b - a <= tol || mid <= a || mid >= b) break;
            if (orc_sturm_count(n, d, e, mid) > k)
                b = mid;
            else
                a = mid;
        }
        w[k] = 0.5 * (a + b);
    }
}

/*
 * Implicit QL iteration with Wilkinson shifts on the tridiagonal (d, e), accumulating
 * the plane rotations into the columns of z (n rows, ld ldz): on exit d holds the
 * eigenvalues (unordered) and column k of z is multiplied on the right by all the
 * rotations, so if z = Q on entry then z = Q Z_T.  e[0..n-2] is the subdiagonal;
 * it is destroyed.  Returns 0, or the index+1 of an eigenvalue that did not converge.
 */
int64_t orc_tql(int64_t n, double *d, double *e_in, double *z, int64_t ldz) {
    if (n <= 1) return 0;
    double *e = (double *)calloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    double *cs = (double *)malloc(sizeof(double) * (size_t)n);
    double *sn = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t fail = 0;
    for (int64_t l = 0; l < n && !fail; ++l) {
        int iter = 0;
        for (;;) {
            int64_t m = l;
            for (; m + 1 < n; ++m) {
                double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= DBL_EPSILON * dd || fabs(e[m]) < DBL_MIN) break;
            }
            if (m == l) break;
            if (++iter > 60) {
                fail = l + 1;
                break;
            }
            /* Wilkinson-type shift from the leading 2x2 block at l */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int64_t i;
            int64_t nrot = 0;
            int early = 0;
            for (i = m - 1; i >= l; --i) {
                double f = s * e[i];
                double bb = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) { /* the rotation vanishes: split here */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = 1;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * bb;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - bb;
                cs[nrot] = c;
                sn[nrot] = s;
                ++nrot;
            }
            /* apply the rotations of this sweep to the columns of z, row-parallel */
            if (nrot > 0) {
                int64_t top = m - 1;
#pragma omp parallel for schedule(static) if (n > 256)
                for (int64_t row = 0; row < n; ++row) {
                    for (int64_t t = 0; t < nrot; ++t) {
                        int64_t ii = top - t;
                        double *zi = &AT(z, row, ii, ldz);
                        double *zi1 = &AT(z, row, ii + 1, ldz);
                        double f = *zi1;
                        *zi1 = sn[t] * (*zi) + cs[t] * f;
                        *zi = cs[t] * (*zi) - sn[t] * f;
                    }
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    free(e);
    free(cs);
    free(sn);
    return fail;
}

/*
 * Number of negative eigenvalues of the symmetric matrix whose lower triangle is
 * in a (n x n, ld; destroyed), from a symmetric indefinite factorisation
 * P a P^T = L D L^T with diagonal pivoting (Bunch-Kaufman, Golub and Van Loan,
 * "Matrix Computations", section 4.4): D is block diagonal with 1 x 1 and 2 x 2
 * blocks, and by Sylvester's law of inertia a has as many negative eigenvalues as
 * D (a 1 x 1 block by its sign; a 2 x 2 block one if its determinant is negative,
 * two if it is positive with a negative trace).  Only D's blocks are needed, so L
 * is not kept.  Returns -1 if an exactly singular pivot occurs.
 */
static void sym_swap_lower(int64_t n, double *a, int64_t ld, int64_t k, int64_t kk, int64_t p) {
    /* swap rows/columns kk < p of the trailing part (indices >= k), lower storage */
    double t;
    t = AT(a, kk, kk, ld); AT(a, kk, kk, ld) = AT(a, p, p, ld); AT(a, p, p, ld) = t;
    for (int64_t j = k; j < kk; ++j) {
        t = AT(a, kk, j, ld); AT(a, kk, j, ld) = AT(a, p, j, ld); AT(a, p, j, ld) = t;
    }
    for (int64_t i = kk + 1; i < p; ++i) {
        t = AT(a, i, kk, ld); AT(a, i, kk, ld) = AT(a, p, i, ld); AT(a, p, i, ld) = t;
    }
    for (int64_t i = p + 1; i < n; ++i) {
        t = AT(a, i, kk, ld); AT(a, i, kk, ld) = AT(a, i, p, ld); AT(a, i, p, ld) = t;
    }
}

int64_t orc_ldlt_inertia(int64_t n, double *a, int64_t ld) {
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    int64_t neg = 0, k = 0;
    while (k < n) {
        const double akk = fabs(AT(a, k, k, ld));
        int64_t r = k;
        double colmax = 0.0;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(AT(a, i, k, ld)) > colmax) {
                colmax = fabs(AT(a, i, k, ld));
                r = i;
            }
        if (akk == 0.0 && colmax == 0.0) return -1;
        int size = 1;
        int64_t piv = k;
        if (!(akk >= alpha * colmax)) {
            double rowmax = 0.0;
            for (int64_t j = k; j < r; ++j)
                if (fabs(AT(a, r, j, ld)) > rowmax) rowmax = fabs(AT(a, r, j, ld));
            for (int64_t i = r + 1; i < n; ++i)
                if (fabs(AT(a, i, r, ld)) > rowmax) rowmax = fabs(AT(a, i, r, ld));
            if (akk * rowmax >= alpha * colmax * colmax) {
                piv = k;
            } else if (fabs(AT(a, r, r, ld)) >= alpha * rowmax) {
                piv = r;
            } else {
                size = 2;
                piv = r;
            }
        }
        const int64_t kk = (size == 1) ? k : k + 1;
        if (piv != kk) sym_swap_lower(n, a, ld, k, kk, piv);
        if (size == 1) {
            const double d = AT(a, k, k, ld);
            if (d == 0.0) return -1;
            if (d < 0.0) ++neg;
            /* trailing lower triangle -= l l^T d, l = a(k+1:, k) / d */
#pragma omp parallel for schedule(dynamic, 16) if (n - k > 256)
            for (int64_t j = k + 1; j < n; ++j) {
                const double f = AT(a, j, k, ld) / d;
                for (int64_t i = j; i < n; ++i) AT(a, i, j, ld) -= AT(a, i, k, ld) * f;
            }
            k += 1;
        } else {
            const double d11 = AT(a, k, k, ld), d21 = AT(a, k + 1, k, ld), d22 = AT(a, k + 1, k + 1, ld);
            const double det = d11 * d22 - d21 * d21;
            if (det == 0.0) return -1;
            if (det < 0.0) neg += 1;
            else if (d11 + d22 < 0.0) neg += 2;
            /* trailing -= [a_k a_k1] D^{-1} [a_k a_k1]^T */
            const double e11 = d22 / det, e21 = -d21 / det, e22 = d11 / det;
#pragma omp parallel for schedule(dynamic, 16) if (n - k > 256)
            for (int64_t j = k + 2; j < n; ++j) {
                const double xj = AT(a, j, k, ld), yj = AT(a, j, k + 1, ld);
                const double fj = e11 * xj + e21 * yj, gj = e21 * xj + e22 * yj;
                for (int64_t i = j; i < n; ++i)
                    AT(a, i, j, ld) -= AT(a, i, k, ld) * fj + AT(a, i, k + 1, ld) * gj;
            }
            k += 2;
        }
    }
    return neg;
}
