/*
 * neig_oracle.c -- CPU reference for the Schur reduction of a real upper
 * Hessenberg matrix.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the benchmark's CPU-baseline leg call it; the GPU library never links or
 * calls anything in this directory, and nothing here calls the GPU library.
 *
 * Plain, slow, single-threaded, IEEE binary64, no BLAS.  Every routine follows
 * a textbook definition written out directly:
 *
 *   neig_oracle_hessenberg  Householder reduction A = Q1 H Q1^T (the reduction
 *                           phase of Section 2, eq. 3; unblocked, one reflector
 *                           per column).
 *   neig_oracle_francis_step one implicit double-shift QR iteration with a given
 *                           shift polynomial x^2 - tr x + det: bulge created from
 *                           the first column of (H - l1 I)(H - l2 I) and chased
 *                           with overlapping 3-element reflectors (Section 3.2,
 *                           "Bulge chasing step", the two-shift case).
 *   neig_oracle_schur       the double-shift Francis QR algorithm (the m = 2 case
 *                           of Section 3.2) producing the real Schur form of
 *                           Section 2, eq. 4: H = Z S Z^T, S upper
 *                           quasi-triangular with 1x1 and standardised 2x2
 *                           diagonal blocks, Z_out = Z_in * Q.
 *   neig_oracle_std2x2      closed-form standardisation of one 2x2 block.
 *   neig_oracle_cond        eigenvalue condition numbers |x| |y| / |y^H x| of a
 *                           quasi-triangular S from its left and right
 *                           eigenvectors (substitution).
 *   neig_oracle_swap        exchange of two adjacent diagonal blocks (Bai and
 *                           Demmel's Sylvester-equation construction, which
 *                           the paper cites for its reordering phase).
 *   neig_oracle_reorder     selected eigenvalues moved to the leading block by
 *                           adjacent swaps, in order.
 *
 * Readings where the paper is silent (listed again in the design notes):
 *   - negligible subdiagonal: |h(k,k-1)| <= max(smlnum, eps(|h(k-1,k-1)|+|h(k,k)|)),
 *     with ||H||_F in place of the sum when the sum is 0, smlnum = DBL_MIN*n/eps;
 *   - exceptional shifts after 10 and 20 iterations without deflation: a double
 *     shift centred at h(i,i) with trace offset 1.5 s and determinant offset s^2,
 *     s = |h(i,i-1)| + |h(i-1,i-2)| (the ad hoc shift of the Handbook procedure hqr);
 *   - iteration limit 30 * max(10, n) double-shift iterations; on hitting it the
 *     return value is i+1 where rows/cols 0..i are not yet reduced;
 *   - 2x2 blocks with real eigenvalues are split into two 1x1 blocks; blocks with
 *     complex eigenvalues get equal diagonal entries and off-diagonal entries of
 *     opposite sign.
 *
 * Matrices are column-major with a leading dimension.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define EL(M, ld, i, j) (M)[(size_t)(j) * (size_t)(ld) + (size_t)(i)]

static int g_last_iterations = 0;

int neig_oracle_last_iterations(void) { return g_last_iterations; }

/* Householder vector for x[0..m-1]: P = I - tau v v^T, v[0] = 1, P x = beta e1.
 * On return x[0] = beta, x[1..m-1] = v[1..m-1]; returns tau (0 means P = I). */
static double house(int m, double *x) {
    double alpha = x[0], sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma = hypot(sigma, x[i]);
    if (sigma == 0.0) return 0.0;
    double norm = hypot(alpha, sigma);
    double beta = alpha >= 0.0 ? -norm : norm;
    double tau = (beta - alpha) / beta;
    double scal = 1.0 / (alpha - beta);
    for (int i = 1; i < m; ++i) x[i] *= scal;
    x[0] = beta;
    return tau;
}

/* rows r..r+m-1 of M, columns c0..c1, from the left by P = I - tau v v^T (v[0] = 1) */
static void apply_left(double *M, int ld, int r, int m, int c0, int c1, double tau, const double *v) {
    if (tau == 0.0) return;
    for (int j = c0; j <= c1; ++j) {
        double t = EL(M, ld, r, j);
        for (int i = 1; i < m; ++i) t += v[i] * EL(M, ld, r + i, j);
        t *= tau;
        EL(M, ld, r, j) -= t;
        for (int i = 1; i < m; ++i) EL(M, ld, r + i, j) -= t * v[i];
    }
}

/* columns c..c+m-1 of M, rows r0..r1, from the right by P */
static void apply_right(double *M, int ld, int c, int m, int r0, int r1, double tau, const double *v) {
    if (tau == 0.0) return;
    for (int i = r0; i <= r1; ++i) {
        double t = EL(M, ld, i, c);
        for (int k = 1; k < m; ++k) t += v[k] * EL(M, ld, i, c + k);
        t *= tau;
        EL(M, ld, i, c) -= t;
        for (int k = 1; k < m; ++k) EL(M, ld, i, c + k) -= t * v[k];
    }
}

int neig_oracle_hessenberg(int n, double *A, int lda, double *Q, int ldq) {
    if (n < 0) return -1;
    if (!A && n > 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (!Q && n > 0) return -4;
    if (ldq < (n > 1 ? n : 1)) return -5;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) EL(Q, ldq, i, j) = (i == j) ? 1.0 : 0.0;
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int k = 0; k + 2 < n; ++k) {
        int m = n - k - 1;
        for (int i = 0; i < m; ++i) v[i] = EL(A, lda, k + 1 + i, k);
        double tau = house(m, v);
        if (tau == 0.0) continue;
        double beta = v[0];
        v[0] = 1.0;
        apply_left(A, lda, k + 1, m, k + 1, n - 1, tau, v);
        EL(A, lda, k + 1, k) = beta;
        for (int i = k + 2; i < n; ++i) EL(A, lda, i, k) = 0.0;
        apply_right(A, lda, k + 1, m, 0, n - 1, tau, v);
        apply_right(Q, ldq, k + 1, m, 0, n - 1, tau, v);
    }
    free(v);
    return 0;
}

/*
 * Standardise B = [[a b][c d]]: find G = [[cs -sn][sn cs]] with G^T B G either
 * upper triangular (real eigenvalues) or of the form [[m b'][c' m]] with
 * b' c' < 0 (complex pair m +- i sqrt(|b'| |c'|)).  Derivation: write
 * B = m I + [[p q+k][q-k -p]] with m = (a+d)/2, p = (a-d)/2, q = (b+c)/2,
 * k = (b-c)/2.  A rotation by theta leaves m and k unchanged and rotates the
 * pair (p, q) by 2 theta.  The discriminant is p^2 + bc.
 *   - real: the first column of G is the eigenvector (z, c) of eigenvalue
 *     d + z, z = p + sign(p) sqrt(p^2 + bc); the other eigenvalue is d - bc/z.
 *   - complex: choose (cos 2t, sin 2t) = (q, -p)/hypot(p, q), which zeroes p and
 *     makes the off-diagonal entries r + k and r - k, r = hypot(p, q).
 * On return (a, b, c, d) hold the standardised block.
 */
void neig_oracle_std2x2(double *a, double *b, double *c, double *d, double *cs, double *sn,
                        double *rt1r, double *rt1i, double *rt2r, double *rt2i) {
    double A = *a, B = *b, C = *c, D = *d;
    *rt1i = *rt2i = 0.0;
    if (C == 0.0) {
        *cs = 1.0; *sn = 0.0;
        *rt1r = A; *rt2r = D;
        return;
    }
    if (B == 0.0) {
        /* a quarter turn swaps the diagonal entries and makes the block upper triangular */
        *cs = 0.0; *sn = 1.0;
        *a = D; *b = -C; *c = 0.0; *d = A;
        *rt1r = D; *rt2r = A;
        return;
    }
    double p = 0.5 * (A - D);
    double bc = B * C;
    double disc = p * p + bc;
    if (disc >= 0.0) {
        double r = sqrt(disc);
        double z = p + (p >= 0.0 ? r : -r);
        if (z == 0.0) { /* p = 0 and bc underflowed: treat as triangular */
            *cs = 1.0; *sn = 0.0; *c = 0.0;
            *rt1r = A; *rt2r = D;
            return;
        }
        double t = hypot(z, C);
        double c_ = z / t, s_ = C / t;
        double l1 = D + z, l2 = D - bc / z;
        double bnew = (D - A) * c_ * s_ + B * c_ * c_ - C * s_ * s_;
        *cs = c_; *sn = s_;
        *a = l1; *b = bnew; *c = 0.0; *d = l2;
        *rt1r = l1; *rt2r = l2;
        return;
    }
    double q = 0.5 * (B + C), k = 0.5 * (B - C);
    double r = hypot(p, q);
    double c_ = 1.0, s_ = 0.0;
    if (r != 0.0) {
        double c2 = q / r, s2 = -p / r;
        if (c2 >= 0.0) {
            c_ = sqrt(0.5 * (1.0 + c2));
            s_ = s2 / (2.0 * c_);
        } else {
            s_ = copysign(sqrt(0.5 * (1.0 - c2)), s2);
            c_ = s2 / (2.0 * s_);
        }
    }
    double m = 0.5 * (A + D);
    double bn = r + k, cn = r - k;
    *cs = c_; *sn = s_;
    *a = m; *b = bn; *c = cn; *d = m;
    *rt1r = *rt2r = m;
    *rt1i = sqrt(fabs(bn)) * sqrt(fabs(cn));
    *rt2i = -*rt1i;
}

/* rotate rows/columns i, i+1 of the whole matrix (and the columns of Z) by G */
static void rotate_pair(int n, double *H, int ldh, double *Z, int ldz, int i, double cs, double sn) {
    for (int j = i + 2; j < n; ++j) {
        double x = EL(H, ldh, i, j), y = EL(H, ldh, i + 1, j);
        EL(H, ldh, i, j) = cs * x + sn * y;
        EL(H, ldh, i + 1, j) = -sn * x + cs * y;
    }
    for (int r = 0; r < i; ++r) {
        double x = EL(H, ldh, r, i), y = EL(H, ldh, r, i + 1);
        EL(H, ldh, r, i) = cs * x + sn * y;
        EL(H, ldh, r, i + 1) = -sn * x + cs * y;
    }
    for (int r = 0; r < n; ++r) {
        double x = EL(Z, ldz, r, i), y = EL(Z, ldz, r, i + 1);
        EL(Z, ldz, r, i) = cs * x + sn * y;
        EL(Z, ldz, r, i + 1) = -sn * x + cs * y;
    }
}

static void finish_2x2(int n, double *H, int ldh, double *Z, int ldz, int i, double *wr, double *wi) {
    double a = EL(H, ldh, i, i), b = EL(H, ldh, i, i + 1);
    double c = EL(H, ldh, i + 1, i), d = EL(H, ldh, i + 1, i + 1);
    double cs, sn, r1, i1, r2, i2;
    neig_oracle_std2x2(&a, &b, &c, &d, &cs, &sn, &r1, &i1, &r2, &i2);
    if (!(cs == 1.0 && sn == 0.0)) rotate_pair(n, H, ldh, Z, ldz, i, cs, sn);
    EL(H, ldh, i, i) = a; EL(H, ldh, i, i + 1) = b;
    EL(H, ldh, i + 1, i) = c; EL(H, ldh, i + 1, i + 1) = d;
    wr[i] = r1; wi[i] = i1; wr[i + 1] = r2; wi[i + 1] = i2;
}

/*
 * One double-shift iteration on the active block [l, i] (0-based, i - l >= 2),
 * with full-width updates of H (all columns to the right, all rows above) and Z.
 * The shift polynomial is x^2 - tr x + det.
 */
static void francis_double_step(int n, double *H, int ldh, double *Z, int ldz, int l, int i, double tr, double det) {
    double h00 = EL(H, ldh, l, l), h01 = EL(H, ldh, l, l + 1);
    double h10 = EL(H, ldh, l + 1, l), h11 = EL(H, ldh, l + 1, l + 1);
    double h21 = EL(H, ldh, l + 2, l + 1);
    /* first column of H^2 - tr H + det I restricted to the block: three nonzeros */
    double v[3];
    v[0] = h00 * h00 + h01 * h10 - tr * h00 + det;
    v[1] = h10 * (h00 + h11 - tr);
    v[2] = h10 * h21;
    for (int k = l; k <= i - 1; ++k) {
        int m = (k <= i - 2) ? 3 : 2;
        if (k > l) {
            v[0] = EL(H, ldh, k, k - 1);
            v[1] = EL(H, ldh, k + 1, k - 1);
            v[2] = (m == 3) ? EL(H, ldh, k + 2, k - 1) : 0.0;
        }
        double tau = house(m, v);
        double beta = v[0];
        v[0] = 1.0;
        if (tau != 0.0) {
            int c0 = (k > l) ? k : l;
            apply_left(H, ldh, k, m, c0, n - 1, tau, v);
            if (k > l) {
                EL(H, ldh, k, k - 1) = beta;
                EL(H, ldh, k + 1, k - 1) = 0.0;
                if (m == 3) EL(H, ldh, k + 2, k - 1) = 0.0;
            }
            int r1 = (k + 3 < i) ? k + 3 : i;
            apply_right(H, ldh, k, m, 0, r1, tau, v);
            apply_right(Z, ldz, k, m, 0, n - 1, tau, v);
        }
    }
}

int neig_oracle_francis_step(int n, double *H, int ldh, double *Z, int ldz, int ilo, int ihi, double tr, double det) {
    if (n < 3 || ilo < 0 || ihi >= n || ihi - ilo < 2) return -1;
    francis_double_step(n, H, ldh, Z, ldz, ilo, ihi, tr, det);
    return 0;
}

static int negligible(const double *H, int ldh, int k, double hnorm, double smlnum) {
    double h = fabs(EL(H, ldh, k, k - 1));
    double s = fabs(EL(H, ldh, k - 1, k - 1)) + fabs(EL(H, ldh, k, k));
    if (s == 0.0) s = hnorm;
    double tol = DBL_EPSILON * s;
    if (tol < smlnum) tol = smlnum;
    return h <= tol;
}

int neig_oracle_schur(int n, double *H, int ldh, double *Z, int ldz, double *wr, double *wi, int maxit) {
    g_last_iterations = 0;
    if (n < 0) return -1;
    if (!H && n > 0) return -2;
    if (ldh < (n > 1 ? n : 1)) return -3;
    if (!Z && n > 0) return -4;
    if (ldz < (n > 1 ? n : 1)) return -5;
    if ((!wr || !wi) && n > 0) return -6;
    if (n == 0) return 0;
    double hnorm = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            if (i > j + 1) EL(H, ldh, i, j) = 0.0;
            double x = EL(H, ldh, i, j);
            if (!isfinite(x)) return -2;
            hnorm = hypot(hnorm, x);
        }
    double smlnum = DBL_MIN * ((double)n / DBL_EPSILON);
    if (maxit <= 0) maxit = 30 * (n > 10 ? n : 10);
    int total = 0, its = 0;
    int i = n - 1;
    while (i >= 0) {
        int l = i;
        while (l > 0) {
            if (negligible(H, ldh, l, hnorm, smlnum)) {
                EL(H, ldh, l, l - 1) = 0.0;
                break;
            }
            --l;
        }
        if (l == i) {
            wr[i] = EL(H, ldh, i, i);
            wi[i] = 0.0;
            --i;
            its = 0;
            continue;
        }
        if (l == i - 1) {
            finish_2x2(n, H, ldh, Z, ldz, i - 1, wr, wi);
            i -= 2;
            its = 0;
            continue;
        }
        if (total >= maxit) {
            g_last_iterations = total;
            return i + 1;
        }
        ++total;
        ++its;
        double tr, det;
        if (its == 10 || its == 20) {
            double s = fabs(EL(H, ldh, i, i - 1)) + fabs(EL(H, ldh, i - 1, i - 2));
            double x = EL(H, ldh, i, i);
            tr = 2.0 * x + 1.5 * s;
            det = x * x + 1.5 * s * x + s * s;
        } else {
            double a = EL(H, ldh, i - 1, i - 1), b = EL(H, ldh, i - 1, i);
            double c = EL(H, ldh, i, i - 1), d = EL(H, ldh, i, i);
            tr = a + d;
            det = a * d - b * c;
        }
        francis_double_step(n, H, ldh, Z, ldz, l, i, tr, det);
    }
    g_last_iterations = total;
    /* structural zeros: everything below the subdiagonal, and every subdiagonal
     * entry that is not inside a 2x2 block */
    for (int j = 0; j < n; ++j)
        for (int r = j + 2; r < n; ++r) EL(H, ldh, r, j) = 0.0;
    for (int k = 0; k + 1 < n; ++k)
        if (!(wi[k] > 0.0)) EL(H, ldh, k + 1, k) = 0.0;
    return 0;
}

/* ---- eigenvalue condition numbers ------------------------------------- */

static double complex csafe_div(double complex num, double complex den, double floor) {
    if (cabs(den) < floor) den = floor;
    return num / den;
}

/* solve (B - lam I) u = r for a 2x2 real block B, complex lam, by Cramer's rule */
static void solve2(double b00, double b01, double b10, double b11, double complex lam, double complex r0,
                   double complex r1, double floor, double complex *u0, double complex *u1) {
    double complex a00 = b00 - lam, a11 = b11 - lam;
    double complex det = a00 * a11 - b01 * b10;
    if (cabs(det) < floor) det = floor;
    *u0 = (r0 * a11 - b01 * r1) / det;
    *u1 = (a00 * r1 - b10 * r0) / det;
}

static void rescale(double complex *x, int lo, int hi) {
    double m = 0.0;
    for (int i = lo; i <= hi; ++i) if (cabs(x[i]) > m) m = cabs(x[i]);
    if (m > 1e100) for (int i = lo; i <= hi; ++i) x[i] /= m;
}

/*
 * cond[j] for every diagonal position j of the quasi-triangular S: the
 * reciprocal of |y^H x| / (|x| |y|) for the right (S x = lam x) and left
 * (y^H S = lam y^H) eigenvectors of the eigenvalue read off the block
 * containing j.  Capped at 1/eps.  2x2 blocks are recognised by a nonzero
 * subdiagonal entry.
 */
static int neig_oracle_cond_select(int n, const double *S, int lds, const int *idx, int nidx, double *cond) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    double snorm = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= (j + 1 < n ? j + 1 : j); ++i) snorm = hypot(snorm, EL(S, lds, i, j));
    double floor = DBL_EPSILON * (snorm > 0 ? snorm : 1.0);
    double cap = 1.0 / DBL_EPSILON;
    double complex *x = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *w = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    int *bstart = (int *)malloc(sizeof(int) * (size_t)n); /* first index of the block holding i */
    for (int i = 0; i < n;) {
        if (i + 1 < n && EL(S, lds, i + 1, i) != 0.0) { bstart[i] = bstart[i + 1] = i; i += 2; }
        else { bstart[i] = i; i += 1; }
    }
    char *want = (char *)calloc((size_t)n, 1);
    if (idx) {
        for (int t = 0; t < nidx; ++t)
            if (idx[t] >= 0 && idx[t] < n) want[idx[t]] = 1;
    }
    for (int j = 0; j < n;) {
        int bs = (j + 1 < n && EL(S, lds, j + 1, j) != 0.0) ? 2 : 1;
        if (idx && !want[j] && !(bs == 2 && want[j + 1])) {
            for (int t = 0; t < bs; ++t) cond[j + t] = 0.0;
            j += bs;
            continue;
        }
        double complex lam;
        for (int i = 0; i < n; ++i) x[i] = w[i] = 0.0;
        int top = j + bs - 1; /* last row of the block */
        if (bs == 1) {
            lam = EL(S, lds, j, j);
            x[j] = 1.0;
            w[j] = 1.0;
        } else {
            double a = EL(S, lds, j, j), b = EL(S, lds, j, j + 1), c = EL(S, lds, j + 1, j), d = EL(S, lds, j + 1, j + 1);
            double tr = a + d, dt = a * d - b * c;
            double disc = 0.25 * tr * tr - dt;
            lam = 0.5 * tr + I * sqrt(fabs(disc));
            if (disc > 0) lam = 0.5 * tr + sqrt(disc); /* not a genuine complex block */
            /* right: (B - lam) u = 0 -> u = (b, lam - a); left: w^T (B - lam) = 0 -> w = (c, lam - a) */
            if (fabs(b) + cabs(lam - a) > 0) { x[j] = b; x[j + 1] = lam - a; }
            else { x[j] = lam - d; x[j + 1] = c; }
            if (fabs(c) + cabs(lam - a) > 0) { w[j] = c; w[j + 1] = lam - a; }
            else { w[j] = lam - d; w[j + 1] = b; }
        }
        /* back substitution for x above the block: rows j-1 .. 0 */
        for (int i = j - 1; i >= 0;) {
            int b0 = bstart[i];
            if (b0 == i) {
                double complex r = 0.0;
                for (int k = i + 1; k <= top; ++k) r += EL(S, lds, i, k) * x[k];
                x[i] = csafe_div(-r, EL(S, lds, i, i) - lam, floor);
                --i;
            } else { /* 2x2 block rows b0, b0+1 = i */
                double complex r0 = 0.0, r1 = 0.0;
                for (int k = i + 1; k <= top; ++k) {
                    r0 += EL(S, lds, b0, k) * x[k];
                    r1 += EL(S, lds, i, k) * x[k];
                }
                solve2(EL(S, lds, b0, b0), EL(S, lds, b0, i), EL(S, lds, i, b0), EL(S, lds, i, i), lam, -r0, -r1,
                       floor, &x[b0], &x[i]);
                i -= 2;
            }
            rescale(x, (i + 1 > 0 ? i + 1 : 0), top);
        }
        /* forward substitution for w below the block: w^T (S - lam I) = 0, columns top+1 .. n-1 */
        for (int i = top + 1; i < n;) {
            int b0 = bstart[i];
            if (b0 == i && !(i + 1 < n && bstart[i + 1] == i)) {
                double complex r = 0.0;
                for (int k = j; k < i; ++k) r += w[k] * EL(S, lds, k, i);
                w[i] = csafe_div(-r, EL(S, lds, i, i) - lam, floor);
                ++i;
            } else { /* 2x2 block columns i, i+1: (B - lam)^T (w_i, w_i1) = -(r0, r1) */
                double complex r0 = 0.0, r1 = 0.0;
                for (int k = j; k < i; ++k) {
                    r0 += w[k] * EL(S, lds, k, i);
                    r1 += w[k] * EL(S, lds, k, i + 1);
                }
                solve2(EL(S, lds, i, i), EL(S, lds, i + 1, i), EL(S, lds, i, i + 1), EL(S, lds, i + 1, i + 1), lam,
                       -r0, -r1, floor, &w[i], &w[i + 1]);
                i += 2;
            }
            rescale(w, j, i - 1);
        }
        double nx = 0.0, nw = 0.0;
        double complex dot = 0.0;
        for (int i = 0; i < n; ++i) {
            nx = hypot(nx, cabs(x[i]));
            nw = hypot(nw, cabs(w[i]));
            dot += w[i] * x[i];
        }
        double c = (cabs(dot) > 0) ? nx * nw / cabs(dot) : cap;
        if (!(c <= cap)) c = cap;
        for (int t = 0; t < bs; ++t) cond[j + t] = c;
        j += bs;
    }
    free(x); free(w); free(bstart); free(want);
    return 0;
}

int neig_oracle_cond(int n, const double *S, int lds, double *cond) {
    return neig_oracle_cond_select(n, S, lds, 0, 0, cond);
}

/*
 * Condition numbers for selected diagonal positions only (each O(n^2)): for
 * position j the block containing j is used; results in cond[0..nidx-1].
 */
int neig_oracle_cond_subset(int n, const double *S, int lds, const int *idx, int nidx, double *cond) {
    if (n < 0 || nidx < 0) return -1;
    double *all = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int rc = neig_oracle_cond_select(n, S, lds, idx, nidx, all);
    for (int t = 0; t < nidx; ++t) cond[t] = all[idx[t]];
    free(all);
    return rc;
}


/* ------------------------------------------------------------------------
 * Eigenvalue reordering (the reordering phase the paper runs after the Schur
 * reduction: an orthogonal similarity that moves chosen eigenvalues to the
 * leading diagonal block).  Adjacent diagonal blocks A (p x p) and C (q x q)
 * with coupling B are exchanged by the construction the paper cites (Bai and
 * Demmel): solve the Sylvester equation A X - X C = B, take Q from the QR
 * factorisation of [-X; I] (its first q columns span the invariant subspace of
 * C), and apply Q^T (.) Q.  The lower-left block of the result is set to zero;
 * the swap is rejected when that block or the reconstruction error exceeds
 * 20 eps ||block||.
 * ---------------------------------------------------------------------- */

/* Solve the k x k system M y = r (k <= 4) by Gaussian elimination with partial
 * pivoting; M and r are overwritten.  Returns 0, or 1 for a zero pivot. */
static int solve_small(int k, double M[4][4], double r[4]) {
    for (int s = 0; s < k; ++s) {
        int piv = s;
        for (int i = s + 1; i < k; ++i)
            if (fabs(M[i][s]) > fabs(M[piv][s])) piv = i;
        if (M[piv][s] == 0.0) return 1;
        for (int j = 0; j < k; ++j) {
            double t = M[s][j]; M[s][j] = M[piv][j]; M[piv][j] = t;
        }
        double t = r[s]; r[s] = r[piv]; r[piv] = t;
        for (int i = s + 1; i < k; ++i) {
            const double f = M[i][s] / M[s][s];
            for (int j = s; j < k; ++j) M[i][j] -= f * M[s][j];
            r[i] -= f * r[s];
        }
    }
    for (int s = k - 1; s >= 0; --s) {
        double t = r[s];
        for (int j = s + 1; j < k; ++j) t -= M[s][j] * r[j];
        r[s] = t / M[s][s];
    }
    return 0;
}

/* Swap the adjacent blocks at st (sizes p then q) of the n x n quasi-triangular
 * S, applying the transformation to all of S and to the columns of Z.  Returns
 * 0, or 1 if the swap is rejected (S and Z unchanged). */
int neig_oracle_swap(int n, double *S, int lds, double *Z, int ldz, int st, int p, int q) {
    const int N = p + q;
    if (p < 1 || p > 2 || q < 1 || q > 2 || st < 0 || st + N > n) return 2;
    double B[4][4];
    double bnorm = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            B[i][j] = S[(st + i) + (size_t)(st + j) * lds];
            bnorm += B[i][j] * B[i][j];
        }
    bnorm = sqrt(bnorm);
    /* Sylvester A X - X C = B12 with X p x q: unknown X(i,j) at index i + p j */
    double M[4][4] = {{0}}, r[4] = {0};
    const int K = p * q;
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < p; ++i) {
            const int row = i + p * j;
            r[row] = B[i][p + j];
            for (int k = 0; k < p; ++k) M[row][k + p * j] += B[i][k];
            for (int k = 0; k < q; ++k) M[row][i + p * k] -= B[p + k][p + j];
        }
    if (solve_small(K, M, r)) return 1;
    /* Y = [-X; I] (N x q), Householder QR, Q accumulated (N x N) */
    double Y[4][2], Q[4][4];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < q; ++j) Y[i][j] = (i < p) ? -r[i + p * j] : ((i - p == j) ? 1.0 : 0.0);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Q[i][j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < q; ++c) {
        double v[4];
        for (int t = 0; t < N - c; ++t) v[t] = Y[c + t][c];
        const double tau = house(N - c, v);
        if (tau == 0.0) continue;
        v[0] = 1.0;
        /* Y <- (I - tau v v^T) Y on rows c.., Q <- Q (I - tau v v^T) on columns c.. */
        for (int j = c; j < q; ++j) {
            double d = 0.0;
            for (int t = 0; t < N - c; ++t) d += v[t] * Y[c + t][j];
            for (int t = 0; t < N - c; ++t) Y[c + t][j] -= tau * d * v[t];
        }
        for (int i = 0; i < N; ++i) {
            double d = 0.0;
            for (int t = 0; t < N - c; ++t) d += Q[i][c + t] * v[t];
            for (int t = 0; t < N - c; ++t) Q[i][c + t] -= tau * d * v[t];
        }
    }
    /* Bn = Q^T B Q; tests on the lower-left q... block */
    double W[4][4], Bn[4][4];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
            for (int k = 0; k < N; ++k) d += B[i][k] * Q[k][j];
            W[i][j] = d;
        }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
            for (int k = 0; k < N; ++k) d += Q[k][i] * W[k][j];
            Bn[i][j] = d;
        }
    const double thresh = fmax(20.0 * DBL_EPSILON * bnorm, DBL_MIN);
    double low = 0.0;
    for (int i = q; i < N; ++i)
        for (int j = 0; j < q; ++j) {
            low = fmax(low, fabs(Bn[i][j]));
            Bn[i][j] = 0.0;
        }
    if (low > thresh) return 1;
    double err = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
            for (int k = 0; k < N; ++k)
                for (int l = 0; l < N; ++l) d += Q[i][k] * Bn[k][l] * Q[j][l];
            err = fmax(err, fabs(d - B[i][j]));
        }
    if (err > thresh) return 1;
    /* apply: rows st..st+N-1 right of the pair, columns above it, Z, the block */
    for (int j = st + N; j < n; ++j) {
        double o[4];
        for (int i = 0; i < N; ++i) o[i] = S[(st + i) + (size_t)j * lds];
        for (int i = 0; i < N; ++i) {
            double d = 0.0;
            for (int k = 0; k < N; ++k) d += Q[k][i] * o[k];
            S[(st + i) + (size_t)j * lds] = d;
        }
    }
    for (int i = 0; i < st; ++i) {
        double o[4];
        for (int k = 0; k < N; ++k) o[k] = S[i + (size_t)(st + k) * lds];
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
            for (int k = 0; k < N; ++k) d += o[k] * Q[k][j];
            S[i + (size_t)(st + j) * lds] = d;
        }
    }
    for (int i = 0; i < n; ++i) {
        double o[4];
        for (int k = 0; k < N; ++k) o[k] = Z[i + (size_t)(st + k) * ldz];
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
            for (int k = 0; k < N; ++k) d += o[k] * Q[k][j];
            Z[i + (size_t)(st + j) * ldz] = d;
        }
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) S[(st + i) + (size_t)(st + j) * lds] = Bn[i][j];
    /* the new 2x2 blocks in standard form */
    if (q == 2) {
        double cs, sn, r1, i1, r2, i2;
        double *a = &S[st + (size_t)st * lds], *b = &S[st + (size_t)(st + 1) * lds];
        double *c = &S[(st + 1) + (size_t)st * lds], *d = &S[(st + 1) + (size_t)(st + 1) * lds];
        neig_oracle_std2x2(a, b, c, d, &cs, &sn, &r1, &i1, &r2, &i2);
        /* rows st, st+1 right of the block and columns above it, Z */
        for (int j = st + 2; j < n; ++j) {
            const double x = S[st + (size_t)j * lds], y = S[st + 1 + (size_t)j * lds];
            S[st + (size_t)j * lds] = cs * x + sn * y;
            S[st + 1 + (size_t)j * lds] = -sn * x + cs * y;
        }
        for (int i = 0; i < st; ++i) {
            const double x = S[i + (size_t)st * lds], y = S[i + (size_t)(st + 1) * lds];
            S[i + (size_t)st * lds] = cs * x + sn * y;
            S[i + (size_t)(st + 1) * lds] = -sn * x + cs * y;
        }
        for (int i = 0; i < n; ++i) {
            const double x = Z[i + (size_t)st * ldz], y = Z[i + (size_t)(st + 1) * ldz];
            Z[i + (size_t)st * ldz] = cs * x + sn * y;
            Z[i + (size_t)(st + 1) * ldz] = -sn * x + cs * y;
        }
    }
    if (p == 2) {
        const int s2 = st + q;
        double cs, sn, r1, i1, r2, i2;
        double *a = &S[s2 + (size_t)s2 * lds], *b = &S[s2 + (size_t)(s2 + 1) * lds];
        double *c = &S[(s2 + 1) + (size_t)s2 * lds], *d = &S[(s2 + 1) + (size_t)(s2 + 1) * lds];
        neig_oracle_std2x2(a, b, c, d, &cs, &sn, &r1, &i1, &r2, &i2);
        for (int j = s2 + 2; j < n; ++j) {
            const double x = S[s2 + (size_t)j * lds], y = S[s2 + 1 + (size_t)j * lds];
            S[s2 + (size_t)j * lds] = cs * x + sn * y;
            S[s2 + 1 + (size_t)j * lds] = -sn * x + cs * y;
        }
        for (int i = 0; i < s2; ++i) {
            const double x = S[i + (size_t)s2 * lds], y = S[i + (size_t)(s2 + 1) * lds];
            S[i + (size_t)s2 * lds] = cs * x + sn * y;
            S[i + (size_t)(s2 + 1) * lds] = -sn * x + cs * y;
        }
        for (int i = 0; i < n; ++i) {
            const double x = Z[i + (size_t)s2 * ldz], y = Z[i + (size_t)(s2 + 1) * ldz];
            Z[i + (size_t)s2 * ldz] = cs * x + sn * y;
            Z[i + (size_t)(s2 + 1) * ldz] = -sn * x + cs * y;
        }
    }
    return 0;
}

/* Reorder the standardised real Schur form S (n x n) so that the eigenvalues
 * with select[j] != 0 (either entry of a 2x2 block selects the pair) occupy the
 * leading diagonal block, keeping their relative order: each selected block,
 * top to bottom, is moved up by adjacent swaps to just below the ones already
 * placed.  Z_out = Z_in Q.  *m receives the number of selected eigenvalues;
 * (wr, wi) are read off the reordered S.  Returns 0, or 1 if a swap was
 * rejected (S, Z then hold the partly reordered, still valid Schur form). */
int neig_oracle_reorder(int n, double *S, int lds, double *Z, int ldz, const int *select, double *wr, double *wi,
                        int *m) {
    /* block starts and sizes, with their selection */
    int *bsel = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int info = 0, placed = 0;
    for (int j = 0; j < n; ++j) bsel[j] = select[j] != 0;
    for (int j = 0; j + 1 < n; ++j)
        if (S[(j + 1) + (size_t)j * lds] != 0.0) {
            const int s2 = bsel[j] || bsel[j + 1];
            bsel[j] = bsel[j + 1] = s2;
            ++j;
        }
    int j = 0;
    while (j < n) {
        const int bs = (j + 1 < n && S[(j + 1) + (size_t)j * lds] != 0.0) ? 2 : 1;
        if (!bsel[j]) {
            j += bs;
            continue;
        }
        /* move the block at j up to position placed */
        int pos = j;
        while (pos > placed) {
            const int ba = (pos - 2 >= placed && S[(pos - 1) + (size_t)(pos - 2) * lds] != 0.0) ? 2 : 1;
            const int st = pos - ba;
            if (neig_oracle_swap(n, S, lds, Z, ldz, st, ba, bs)) {
                info = 1;
                break;
            }
            /* the selection flags travel with the blocks */
            for (int t = 0; t < bs; ++t) bsel[st + t] = 1;
            for (int t = 0; t < ba; ++t) bsel[st + bs + t] = 0;
            pos = st;
        }
        if (info) break;
        placed += bs;
        j += bs;
    }
    *m = placed;
    free(bsel);
    /* eigenvalues in diagonal order */
    for (int k = 0; k < n;) {
        if (k + 1 < n && S[(k + 1) + (size_t)k * lds] != 0.0) {
            const double a = S[k + (size_t)k * lds], b = S[k + (size_t)(k + 1) * lds];
            const double c = S[(k + 1) + (size_t)k * lds];
            const double im = sqrt(fabs(b)) * sqrt(fabs(c));
            wr[k] = wr[k + 1] = a;
            wi[k] = im;
            wi[k + 1] = -im;
            k += 2;
        } else {
            wr[k] = S[k + (size_t)k * lds];
            wi[k] = 0.0;
            ++k;
        }
    }
    return info;
}
