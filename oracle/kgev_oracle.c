/*
 * kgev_oracle.c -- plain FP64 CPU oracle for the per-k-point generalized
 * Hermitian eigensolve H(k) C = S(k) C Lambda of Band_DFT_Col.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, and by nothing
 * else.  The GPU library shares no code, header, table or helper with it.
 *
 * Source: J.-H. Parq, E. Sevre, S.-M. Lee, "Effects of Easy Hybrid
 * Parallelization with CUDA for Numerical-Atomic-Orbital Density Functional
 * Theory Calculation", arXiv:1402.4247, Section III ("Application to
 * OpenMX"):
 *   - Part 2: diagonalise S and use its eigenpairs to rearrange S;
 *   - Part 3: matrix products forming S^dagger H S (with the rearranged S);
 *   - Part 4: diagonalise S^dagger H S (Eigen_HH) and one ZGEMM;
 *   - Eigen_HH = Householder tridiagonalisation (Procedures 1-6), a LAPACK
 *     tridiagonal eigensolver, rearrangement (back-transformation) of the
 *     eigenvectors, normalisation.
 *
 * Readings of passages the paper leaves open:
 *   - "rearrange S" is canonical orthogonalisation X = U diag(s)^(-1/2) where
 *     S = U diag(s) U^dagger; "S^dagger H S" is X^dagger H X.
 *   - Procedure 2 "subtract s" is taken with the stable sign: the reflector
 *     maps the column onto beta e_1 with beta = -sign(Re alpha) ||x|| real
 *     (sign(0) = +1), so T comes out real; H_i = I - tau_i v_i v_i^dagger with
 *     v_i(0) = 1.  Procedures 4-6 are the standard two-sided update
 *     y = tau A22 v, w = y - (tau/2)(y^dagger v) v, A22 -= v w^dagger + w v^dagger.
 *   - The tridiagonal solver (the paper names dstevx/dstegr/dstedc without
 *     choosing) is implicit QL with Wilkinson shifts; Sturm-count bisection is
 *     provided as an independent second opinion for eigenvalues.
 *   - Normalisation is to unit 2-norm per column; eigenvalues ascending.
 *
 * Conventions: column-major, element (i,j) of a matrix with leading
 * dimension ld at a[i + j*ld]; Hermitian inputs are read from the LOWER
 * triangle only and the imaginary part of the diagonal is ignored.
 * Built with -O2 -ffp-contract=off and no fast-math.  OpenMP is used only on
 * loops whose iterations are independent, so every result is the same as the
 * serial loop's.
 *
 * Parity pins: every exported function is pinned by the CPU tests
 * (closed forms, known spectra, invariants, brute force, LAPACK as a third
 * opinion); see tests/test_oracle_*.py.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex zc;

#define IX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

enum { OR_OK = 0, OR_ENOTPD = 1, OR_ENOCONV = 2, OR_ENONFINITE = 3, OR_EARG = -1, OR_ENOMEM = -100 };

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Full Hermitian copy of the lower triangle of src (diagonal made real). */
static void herm_full(int n, const zc* src, int lds, zc* dst)
{
    for (int j = 0; j < n; ++j) {
        dst[IX(j, j, n)] = creal(src[IX(j, j, lds)]);
        for (int i = j + 1; i < n; ++i) {
            zc a = src[IX(i, j, lds)];
            dst[IX(i, j, n)] = a;
            dst[IX(j, i, n)] = conj(a);
        }
    }
}

static int lower_finite(int n, const zc* a, int lda)
{
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) {
            zc x = a[IX(i, j, lda)];
            if (!isfinite(creal(x)) || !isfinite(cimag(x))) return 0;
        }
    return 1;
}

/*
 * Plain matrix product C = alpha op(A) op(B) + beta C, op in {'N','C'}
 * ('C' = conjugate transpose).  C is m x n, the inner dimension is k.
 * Used for Part 3 (S^dagger H S) and the final ZGEMM of Part 4.
 */
void or_zgemm(char ta, char tb, int m, int n, int k, zc alpha, const zc* A, int lda,
              const zc* B, int ldb, zc beta, zc* C, int ldc)
{
#pragma omp parallel
    {
        zc* acc = (zc*)malloc(sizeof(zc) * (size_t)(m > 0 ? m : 1));
#pragma omp for schedule(static)
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < m; ++i) acc[i] = 0;
            for (int p = 0; p < k; ++p) {
                zc b = (tb == 'N') ? B[IX(p, j, ldb)] : conj(B[IX(j, p, ldb)]);
                if (ta == 'N') {
                    for (int i = 0; i < m; ++i) acc[i] += A[IX(i, p, lda)] * b;
                } else {
                    for (int i = 0; i < m; ++i) acc[i] += conj(A[IX(p, i, lda)]) * b;
                }
            }
            for (int i = 0; i < m; ++i) {
                zc c = (beta == 0) ? 0 : beta * C[IX(i, j, ldc)];
                C[IX(i, j, ldc)] = alpha * acc[i] + c;
            }
        }
        free(acc);
    }
}

/* or_zgemm with alpha and beta passed as (re, im) pairs (for FFI callers). */
void or_zgemm_ri(char ta, char tb, int m, int n, int k, double ar, double ai, const zc* A, int lda,
                 const zc* B, int ldb, double br, double bi, zc* C, int ldc)
{
    or_zgemm(ta, tb, m, n, k, ar + ai * I, A, lda, B, ldb, br + bi * I, C, ldc);
}

/*
 * Householder tridiagonalisation, Section III Procedures 1-6, one reflector
 * per column i = 0 .. n-2 (unblocked, textbook order).
 *   A   : in: Hermitian matrix (lower triangle read), n x n, leading dim lda;
 *         out: overwritten by a full working copy (T on the band).
 *   V   : out, n x n (ld n): column i holds v_i in rows i+1..n-1 (v_i(i+1) = 1)
 *         and zeros elsewhere.  May be NULL.
 *   d,e : out, diagonal (n) and sub-diagonal (n-1) of the real tridiagonal T.
 *   tau : out, n-1 reflector scalars.
 * T = Q^dagger A Q with Q = H_0 H_1 ... H_{n-2}, H_i = I - tau_i v_i v_i^dagger.
 */
int or_zhetrd(int n, zc* A, int lda, zc* V, double* d, double* e, zc* tau)
{
    if (n < 1) return OR_EARG;
    zc* B = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* v = (zc*)malloc(sizeof(zc) * (size_t)n);
    zc* y = (zc*)malloc(sizeof(zc) * (size_t)n);
    if (!B || !v || !y) { free(B); free(v); free(y); return OR_ENOMEM; }
    herm_full(n, A, lda, B);
    if (V) memset(V, 0, sizeof(zc) * (size_t)n * n);

    for (int i = 0; i + 1 < n; ++i) {
        const int o = i + 1;          /* first row of the reflector */
        const int m = n - o;          /* reflector length */
        /* Procedure 1: u = column i below the diagonal. */
        zc alpha = B[IX(o, i, n)];
        double sigma2 = 0.0;
        for (int r = 1; r < m; ++r) {
            zc x = B[IX(o + r, i, n)];
            sigma2 += creal(x) * creal(x) + cimag(x) * cimag(x);
        }
        /* Procedure 2: norm and the reflector (stable sign, real beta). */
        zc t;
        double beta;
        if (sigma2 == 0.0 && cimag(alpha) == 0.0) {
            t = 0;
            beta = creal(alpha);
            v[0] = 1;
            for (int r = 1; r < m; ++r) v[r] = 0;
        } else {
            double nrm = sqrt(creal(alpha) * creal(alpha) + cimag(alpha) * cimag(alpha) + sigma2);
            beta = (creal(alpha) >= 0.0) ? -nrm : nrm;
            t = (beta - alpha) / beta;
            zc sc = 1.0 / (alpha - beta);
            v[0] = 1;
            for (int r = 1; r < m; ++r) v[r] = B[IX(o + r, i, n)] * sc;
        }
        /* Procedure 3: keep what the back-transformation needs. */
        tau[i] = t;
        e[i] = beta;
        if (V)
            for (int r = 0; r < m; ++r) V[IX(o + r, i, n)] = v[r];
        /* Column i and row i of the working copy become tridiagonal. */
        B[IX(o, i, n)] = beta;
        B[IX(i, o, n)] = beta;
        for (int r = 1; r < m; ++r) { B[IX(o + r, i, n)] = 0; B[IX(i, o + r, n)] = 0; }
        if (t == 0) continue;
        /* Procedure 4: y = tau * A22 v. */
        /* B is kept exactly Hermitian (both triangles are updated with
         * conjugate-symmetric terms), so row r of A22 is the conjugate of
         * column r; reading the column keeps the loop contiguous. */
#pragma omp parallel for schedule(static)
        for (int r = 0; r < m; ++r) {
            zc acc = 0;
            for (int c = 0; c < m; ++c) acc += conj(B[IX(o + c, o + r, n)]) * v[c];
            y[r] = t * acc;
        }
        /* Procedure 5: w = y - (tau/2) (y^dagger v) v  (stored over y). */
        zc yv = 0;
        for (int r = 0; r < m; ++r) yv += conj(y[r]) * v[r];
        zc a2 = -0.5 * t * yv;
        for (int r = 0; r < m; ++r) y[r] += a2 * v[r];
        /* Procedure 6: A22 -= v w^dagger + w v^dagger. */
#pragma omp parallel for schedule(static)
        for (int c = 0; c < m; ++c) {
            zc wc = conj(y[c]), vc = conj(v[c]);
            for (int r = 0; r < m; ++r) B[IX(o + r, o + c, n)] -= v[r] * wc + y[r] * vc;
        }
    }
    for (int i = 0; i < n; ++i) d[i] = creal(B[IX(i, i, n)]);
    /* Hand the working copy back (T on the band, zeros elsewhere). */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) A[IX(i, j, lda)] = B[IX(i, j, n)];
    free(B); free(v); free(y);
    return OR_OK;
}


/*
 * Sturm count: number of eigenvalues of the symmetric tridiagonal T(d, e)
 * strictly below x, i.e. the number of negative pivots q_i of the LDL^T
 * factorisation of T - xI (q_0 = d_0 - x, q_i = d_i - x - e_{i-1}^2 / q_{i-1}).
 * A zero pivot is replaced by -pivmin (Kahan's safeguard).
 */
int or_sturm_count(int n, const double* d, const double* e, double x)
{
    double emax2 = 0.0;
    for (int i = 0; i + 1 < n; ++i) emax2 = fmax(emax2, e[i] * e[i]);
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    int cnt = 0;
    double q = 0.0;
    for (int i = 0; i < n; ++i) {
        q = (d[i] - x) - ((i > 0) ? (e[i - 1] * e[i - 1]) / q : 0.0);
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

/*
 * All eigenvalues of T(d, e) by bisection on the Sturm count, ascending.
 * Eigenvalue j is the point where the count steps from j to j+1; the
 * bracket starts from the Gershgorin interval and is halved until it is a
 * few ulps wide.
 */
void or_bisect_eigs(int n, const double* d, const double* e, double* w)
{
    double lo0 = INFINITY, hi0 = -INFINITY;
    for (int i = 0; i < n; ++i) {
        double r = ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < n) ? fabs(e[i]) : 0.0);
        lo0 = fmin(lo0, d[i] - r);
        hi0 = fmax(hi0, d[i] + r);
    }
    double span = fmax(fabs(lo0), fabs(hi0));
    lo0 -= 4.0 * 2.220446049250313e-16 * span + 1e-300;
    hi0 += 4.0 * 2.220446049250313e-16 * span + 1e-300;
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < n; ++j) {
        double lo = lo0, hi = hi0;
        for (int it = 0; it < 2000; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (hi - lo <= 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi))) break;
            if (or_sturm_count(n, d, e, mid) <= j) lo = mid; else hi = mid;
        }
        w[j] = 0.5 * (lo + hi);
    }
}

typedef struct { double val; int idx; } keyed;

static int keyed_cmp(const void* a, const void* b)
{
    const keyed* x = (const keyed*)a;
    const keyed* y = (const keyed*)b;
    if (x->val < y->val) return -1;
    if (x->val > y->val) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);   /* ties keep input order */
}

/*
 * Implicit QL iteration with Wilkinson-type shifts for the real symmetric
 * tridiagonal T(d, e) (Bowdler, Martin, Reinsch & Wilkinson 1968; Golub &
 * Van Loan, Matrix Computations, Sec. 8.3).  d (n) is overwritten by the
 * eigenvalues in ascending order; e (n-1) is read only.  If Z is not NULL it
 * receives the orthonormal eigenvectors (column j for eigenvalue j), n x n
 * with leading dimension ldz.  A sub-diagonal entry counts as zero when
 * |e_m| <= eps * tst1, tst1 the running maximum of |d_l| + |e_l| over the rows
 * reached so far (the normwise test of the published algorithm, tql2).
 * Returns OR_ENOCONV after 30 sweeps on one eigenvalue without convergence.
 */
int or_tridiag_ql(int n, double* d, const double* e_in, double* Z, int ldz)
{
    const double eps = 2.220446049250313e-16;
    double* e = (double*)calloc((size_t)n + 1, sizeof(double));
    double* rc = (double*)malloc(sizeof(double) * (size_t)n);
    double* rs = (double*)malloc(sizeof(double) * (size_t)n);
    if (!e || !rc || !rs) { free(e); free(rc); free(rs); return OR_ENOMEM; }
    for (int i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    if (Z)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) Z[IX(i, j, ldz)] = (i == j) ? 1.0 : 0.0;

    int status = OR_OK;
    /* Deflation is tested against the running norm tst1 = max(|d_l| + |e_l|)
     * over the rows reached so far, as in the published QL algorithm (tql2):
     * a coupling below eps * tst1 is within the rounding already committed,
     * and clusters of eigenvalues near zero deflate as readily as others. */
    double tst1 = 0.0;
    for (int l = 0; l < n && status == OR_OK; ++l) {
        int sweeps = 0;
        tst1 = fmax(tst1, fabs(d[l]) + fabs(e[l]));
        for (;;) {
            /* Smallest m >= l whose coupling to m+1 is negligible. */
            int m = l;
            while (m < n - 1 && fabs(e[m]) > eps * tst1) ++m;
            if (m == l) break;
            if (++sweeps > 30) { status = OR_ENOCONV; break; }
            /* Shift: eigenvalue of the leading 2x2 block nearer d_l. */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int nrot = 0, underflow = 0;
            /* Chase the bulge from the bottom (row m) up to row l. */
            for (int i = m - 1; i >= l; --i) {
                double f = s * e[i], b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {            /* deflate early on exact zero */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    underflow = 1;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                rc[nrot] = c;
                rs[nrot] = s;
                ++nrot;
            }
            /* Apply this sweep's rotations (in order) to the columns of Z;
             * rows are independent, so they are split across threads. */
            if (Z && nrot > 0) {
#pragma omp parallel for schedule(static)
                for (int k = 0; k < n; ++k) {
                    for (int q = 0; q < nrot; ++q) {
                        int i = m - 1 - q;
                        double zi = Z[IX(k, i, ldz)], zi1 = Z[IX(k, i + 1, ldz)];
                        Z[IX(k, i + 1, ldz)] = rs[q] * zi + rc[q] * zi1;
                        Z[IX(k, i, ldz)] = rc[q] * zi - rs[q] * zi1;
                    }
                }
            }
            if (underflow) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    free(e); free(rc); free(rs);
    if (status != OR_OK) return status;

    /* Stable ascending sort of the eigenvalues, carrying Z's columns. */
    keyed* kv = (keyed*)malloc(sizeof(keyed) * (size_t)n);
    double* dcopy = (double*)malloc(sizeof(double) * (size_t)n);
    double* zcopy = Z ? (double*)malloc(sizeof(double) * (size_t)n * n) : NULL;
    if (!kv || !dcopy || (Z && !zcopy)) { free(kv); free(dcopy); free(zcopy); return OR_ENOMEM; }
    for (int i = 0; i < n; ++i) { kv[i].val = d[i]; kv[i].idx = i; dcopy[i] = d[i]; }
    qsort(kv, (size_t)n, sizeof(keyed), keyed_cmp);
    for (int j = 0; j < n; ++j) d[j] = dcopy[kv[j].idx];
    if (Z) {
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) zcopy[IX(i, j, n)] = Z[IX(i, kv[j].idx, ldz)];
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) Z[IX(i, j, ldz)] = zcopy[IX(i, j, n)];
    }
    free(kv); free(dcopy); free(zcopy);
    return OR_OK;
}

/*
 * "Rearrangement of eigenvectors" (back-transformation): U <- Q U with
 * Q = H_0 H_1 ... H_{n-2}, applying H_{n-2} first.  V and tau are those of
 * or_zhetrd; U is n x ncols with leading dimension ldu.
 */
void or_apply_q(int n, const zc* V, const zc* tau, int ncols, zc* U, int ldu)
{
    for (int i = n - 2; i >= 0; --i) {
        const zc t = tau[i];
        if (t == 0) continue;
        const int o = i + 1;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < ncols; ++c) {
            zc s = 0;
            for (int r = o; r < n; ++r) s += conj(V[IX(r, i, n)]) * U[IX(r, c, ldu)];
            s *= t;
            for (int r = o; r < n; ++r) U[IX(r, c, ldu)] -= V[IX(r, i, n)] * s;
        }
    }
}

/*
 * Normalisation (Eigen_HH's last step): each column j of U (nrows x ncols)
 * is divided by its 2-norm.
 */
void or_normalize_cols(int nrows, int ncols, zc* U, int ldu)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ncols; ++j) {
        double ss = 0.0;
        for (int i = 0; i < nrows; ++i) {
            zc x = U[IX(i, j, ldu)];
            ss += creal(x) * creal(x) + cimag(x) * cimag(x);
        }
        const double f = 1.0 / sqrt(ss);
        for (int i = 0; i < nrows; ++i) U[IX(i, j, ldu)] *= f;
    }
}

/*
 * Eigen_HH (Section III): Householder tridiagonalisation, tridiagonal
 * eigensolve, rearrangement (back-transformation) and normalisation of the
 * eigenvectors of the Hermitian matrix whose lower triangle is A (n x n, ld
 * lda; A is not modified).  w receives the ascending eigenvalues; Y (n x n,
 * ld n) the eigenvectors, or nothing when Y is NULL (eigenvalues only).
 * Optional stage outputs d, e (the tridiagonal T) may be NULL.
 */
int or_eigen_hh(int n, const zc* A, int lda, double* w, zc* Y, double* d_out, double* e_out)
{
    if (n < 1) return OR_EARG;
    zc* B = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* V = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* tau = (zc*)malloc(sizeof(zc) * (size_t)n);
    double* e = (double*)calloc((size_t)n, sizeof(double));
    double* Z = Y ? (double*)malloc(sizeof(double) * (size_t)n * n) : NULL;
    int st = OR_ENOMEM;
    if (!B || !V || !tau || !e || (Y && !Z)) goto out;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) B[IX(i, j, n)] = A[IX(i, j, lda)];
    st = or_zhetrd(n, B, n, V, w, e, tau);
    if (st != OR_OK) goto out;
    if (d_out) memcpy(d_out, w, sizeof(double) * (size_t)n);
    if (e_out && n > 1) memcpy(e_out, e, sizeof(double) * (size_t)(n - 1));
    st = or_tridiag_ql(n, w, e, Z, n);
    if (st != OR_OK || !Y) goto out;
    for (size_t q = 0; q < (size_t)n * n; ++q) Y[q] = Z[q];
    or_apply_q(n, V, tau, n, Y, n);
    or_normalize_cols(n, n, Y, n);
out:
    free(B); free(V); free(tau); free(e); free(Z);
    return st;
}

/*
 * The per-k solve, Parts 2-4 of Band_DFT_Col (Section III), for one k-point:
 *   Part 2: S = U diag(s) U^dagger by Eigen_HH; check s_min > s_tol s_max;
 *           rearrange S into X = U diag(s)^(-1/2).
 *   Part 3: A = X^dagger H X by two plain matrix products.
 *   Part 4: A = Y diag(lambda) Y^dagger by Eigen_HH; C = X Y.
 * H, S: lower triangles read (ld ldh, lds).  w: n eigenvalues ascending.
 * C: n x n (ld ldc), S-orthonormal generalized eigenvectors, or NULL for
 * eigenvalues only.  Stage outputs (any may be NULL): dS, eS (T of S), sS
 * (eigenvalues of S), X (n x n, ld n), Am (X^dagger H X, n x n, ld n),
 * dA, eA (T of A).
 * Returns OR_OK, OR_ENONFINITE, OR_ENOTPD, OR_ENOCONV or OR_ENOMEM.
 */
int or_solve_k(int n, const zc* H, int ldh, const zc* S, int lds, double s_tol, double* w, zc* C,
               int ldc, double* dS, double* eS, double* sS, zc* X_out, zc* A_out, double* dA,
               double* eA)
{
    if (n < 1) return OR_EARG;
    if (!lower_finite(n, H, ldh) || !lower_finite(n, S, lds)) return OR_ENONFINITE;
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    zc* X = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* Hf = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* G = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* A = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* Y = C ? (zc*)malloc(sizeof(zc) * (size_t)n * n) : NULL;
    int st = OR_ENOMEM;
    if (!s || !X || !Hf || !G || !A || (C && !Y)) goto out;

    /* Part 2 */
    st = or_eigen_hh(n, S, lds, s, X, dS, eS);
    if (st != OR_OK) goto out;
    if (sS) memcpy(sS, s, sizeof(double) * (size_t)n);
    if (!(s[0] > s_tol * s[n - 1])) { st = OR_ENOTPD; goto out; }
    for (int j = 0; j < n; ++j) {
        double f = 1.0 / sqrt(s[j]);
        for (int i = 0; i < n; ++i) X[IX(i, j, n)] *= f;
    }
    if (X_out) memcpy(X_out, X, sizeof(zc) * (size_t)n * n);

    /* Part 3 */
    herm_full(n, H, ldh, Hf);
    or_zgemm('N', 'N', n, n, n, 1.0, Hf, n, X, n, 0.0, G, n);
    or_zgemm('C', 'N', n, n, n, 1.0, X, n, G, n, 0.0, A, n);
    if (A_out) memcpy(A_out, A, sizeof(zc) * (size_t)n * n);

    /* Part 4 */
    st = or_eigen_hh(n, A, n, w, Y, dA, eA);
    if (st != OR_OK || !C) goto out;
    zc* Ct = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    if (!Ct) { st = OR_ENOMEM; goto out; }
    or_zgemm('N', 'N', n, n, n, 1.0, X, n, Y, n, 0.0, Ct, n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) C[IX(i, j, ldc)] = Ct[IX(i, j, n)];
    free(Ct);
out:
    free(s); free(X); free(Hf); free(G); free(A); free(Y);
    return st;
}

/* ------------------------------------------------------------------------
 * Band_DFT_Col Part 5: chemical potential and band energy.
 * The paper names the step only; the reading followed here is the usual one
 * for a finite electronic temperature: occupation of state j at k-point k is
 * f_kj = 1 / (1 + exp((lambda_kj - mu) / kT)); mu is the root of
 *   N(mu) = g * sum_k wk_k * sum_j f_kj  =  nelec
 * (g = electrons per state), found by bisection on a bracket whose ends
 * are 50 kT beyond the extreme eigenvalues; the band energy is
 *   E_band = g * sum_k wk_k * sum_j f_kj lambda_kj.
 * Plain loops in the order written; sums in index order.
 * ---------------------------------------------------------------------- */
static double or_fd(double x, double mu, double kT)
{
    const double t = (x - mu) / kT;
    if (t > 0.0) {
        const double e = exp(-t);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(t));
}

static double or_count(int nk, int n, const double* w, int ldw, const double* wk, double g, double mu, double kT)
{
    double N = 0.0;
    for (int k = 0; k < nk; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += or_fd(w[(size_t)k * ldw + j], mu, kT);
        N += wk[k] * s;
    }
    return g * N;
}

/* returns 0, or -1 for invalid arguments (kT <= 0, nelec outside (0, g n sum wk)) */
int or_fermi(int nk, int n, const double* w, int ldw, const double* wk, double nelec, double kT, double g,
             double* out3, double* occ, int ldo)
{
    if (nk < 1 || n < 1 || !(kT > 0.0) || !(g > 0.0)) return -1;
    double wsum = 0.0, lo = w[0], hi = w[0];
    for (int k = 0; k < nk; ++k) {
        wsum += wk[k];
        for (int j = 0; j < n; ++j) {
            const double x = w[(size_t)k * ldw + j];
            if (x < lo) lo = x;
            if (x > hi) hi = x;
        }
    }
    if (!(nelec > 0.0) || !(nelec < g * n * wsum)) return -1;
    lo -= 50.0 * kT;
    hi += 50.0 * kT;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (or_count(nk, n, w, ldw, wk, g, mid, kT) < nelec) lo = mid;
        else hi = mid;
    }
    const double mu = 0.5 * (lo + hi);
    double eb = 0.0;
    for (int k = 0; k < nk; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            const double x = w[(size_t)k * ldw + j];
            const double f = or_fd(x, mu, kT);
            s += f * x;
            if (occ) occ[(size_t)k * ldo + j] = f;
        }
        eb += wk[k] * s;
    }
    out3[0] = mu;
    out3[1] = g * eb;
    out3[2] = or_count(nk, n, w, ldw, wk, g, mu, kT);
    return 0;
}

/* ------------------------------------------------------------------------
 * Band_DFT_Col Part 6: charge density matrix and energy density matrix,
 *   rho = g * sum_k wk_k * sum_{j < nocc} f_kj c_kj c_kj^H,
 *   edm = g * sum_k wk_k * sum_{j < nocc} f_kj lambda_kj c_kj c_kj^H,
 * with c_kj column j of the k-th eigenvector matrix (C_k, column-major, ld
 * ldc, k-stride sc).  Full n x n results, column-major with ld n; edm may be
 * NULL.  Triple loops, sums in index order (k outer, then j).
 * ---------------------------------------------------------------------- */
void or_density(int nk, int n, int nocc, const zc* C, int ldc, long sc, const double* w, int ldw, const double* occ,
                int ldo, const double* wk, double g, zc* rho, zc* edm)
{
#pragma omp parallel for schedule(static)
    for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
            zc sr = 0.0, se = 0.0;
            for (int k = 0; k < nk; ++k) {
                const zc* Ck = C + (size_t)k * sc;
                zc tr = 0.0, te = 0.0;
                for (int j = 0; j < nocc; ++j) {
                    const zc t = Ck[IX(a, j, ldc)] * conj(Ck[IX(b, j, ldc)]);
                    const double f = occ[(size_t)k * ldo + j];
                    tr += f * t;
                    te += f * w[(size_t)k * ldw + j] * t;
                }
                sr += wk[k] * tr;
                se += wk[k] * te;
            }
            rho[IX(a, b, n)] = g * sr;
            if (edm) edm[IX(a, b, n)] = g * se;
        }
}

/* Part 6 at selected entries (a_q, b_q), q < npairs: the same sums as
 * or_density, for sizes where the full matrices are too costly here. */
void or_density_entries(int nk, int n, int nocc, const zc* C, int ldc, long sc, const double* w, int ldw,
                        const double* occ, int ldo, const double* wk, double g, int npairs, const int* ab,
                        zc* rho, zc* edm)
{
    (void)n;
#pragma omp parallel for schedule(static)
    for (int q = 0; q < npairs; ++q) {
        const int a = ab[2 * q], b = ab[2 * q + 1];
        zc sr = 0.0, se = 0.0;
        for (int k = 0; k < nk; ++k) {
            const zc* Ck = C + (size_t)k * sc;
            zc tr = 0.0, te = 0.0;
            for (int j = 0; j < nocc; ++j) {
                const zc t = Ck[IX(a, j, ldc)] * conj(Ck[IX(b, j, ldc)]);
                const double f = occ[(size_t)k * ldo + j];
                tr += f * t;
                te += f * w[(size_t)k * ldw + j] * t;
            }
            sr += wk[k] * tr;
            se += wk[k] * te;
        }
        rho[q] = g * sr;
        edm[q] = g * se;
    }
}

/* ------------------------------------------------------------------------
 * Part 2 variant (not the paper's method): S = L L^H by the textbook
 * column-oriented Cholesky factorisation (lower, real positive diagonal),
 * and the lower-triangular inverse L^{-1} by forward substitution on the
 * identity.  X = L^{-H} satisfies X^H S X = I, so Parts 3 and 4 are then the
 * same as with X = U diag(s)^{-1/2}.  S is read from its lower triangle.
 * Returns OR_ENOTPD when a pivot d_j <= s_tol * max_i S_ii (or is not
 * positive); L and Linv are full n x n, column-major, ld n, zero above the
 * diagonal.
 * ---------------------------------------------------------------------- */
int or_cholesky_inv(int n, const zc* S, int lds, double s_tol, zc* L, zc* Linv)
{
    if (n < 1) return OR_EARG;
    double smax = 0.0;
    for (int i = 0; i < n; ++i) {
        const double d = creal(S[IX(i, i, lds)]);
        if (d > smax) smax = d;
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) L[IX(i, j, n)] = (i >= j) ? S[IX(i, j, lds)] : 0.0;
    for (int j = 0; j < n; ++j) {
        double d = creal(L[IX(j, j, n)]);
        for (int k = 0; k < j; ++k) {
            const zc l = L[IX(j, k, n)];
            d -= creal(l * conj(l));
        }
        if (!(d > s_tol * smax)) return OR_ENOTPD;
        const double ljj = sqrt(d);
        L[IX(j, j, n)] = ljj;
        for (int i = j + 1; i < n; ++i) {
            zc s = L[IX(i, j, n)];
            for (int k = 0; k < j; ++k) s -= L[IX(i, k, n)] * conj(L[IX(j, k, n)]);
            L[IX(i, j, n)] = s / ljj;
        }
    }
    /* L Linv = I, column c: forward substitution */
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            if (i < c) { Linv[IX(i, c, n)] = 0.0; continue; }
            zc s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[IX(i, k, n)] * Linv[IX(k, c, n)];
            Linv[IX(i, c, n)] = s / L[IX(i, i, n)];
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Part 2 variant (not the paper's method): canonical orthogonalisation with
 * pruning.  S = U diag(s) U^H as in Part 2; the directions with
 * s_j <= s_tol * s_max are dropped, X' = U(:, keep) diag(s_keep)^(-1/2)
 * (n x n' with n' kept columns, taken in ascending order of s); then Parts 3
 * and 4 on the reduced n' x n' matrix A' = X'^H H X': A' = Y' diag(w') Y'^H,
 * C' = X' Y'.  Outputs: *nkeep = n', w[0:n'] ascending and w[n':n] = +inf,
 * C (n x n, ld ldc) with columns 0..n'-1 = C' and the rest zero.
 * ---------------------------------------------------------------------- */
int or_solve_k_prune(int n, const zc* H, int ldh, const zc* S, int lds, double s_tol, double* w, zc* C, int ldc,
                     int* nkeep)
{
    if (n < 1) return OR_EARG;
    if (!lower_finite(n, H, ldh) || !lower_finite(n, S, lds)) return OR_ENONFINITE;
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    zc* U = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* Hf = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* G = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* A = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    zc* Y = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    double* wr = (double*)malloc(sizeof(double) * (size_t)n);
    int st = OR_ENOMEM;
    if (!s || !U || !Hf || !G || !A || !Y || !wr) goto out;
    st = or_eigen_hh(n, S, lds, s, U, NULL, NULL);
    if (st != OR_OK) goto out;
    int j0 = 0;
    while (j0 < n && !(s[j0] > s_tol * s[n - 1])) ++j0;      /* s ascending: dropped ones first */
    const int m = n - j0;
    *nkeep = m;
    for (int j = 0; j < m; ++j) {
        const double f = 1.0 / sqrt(s[j0 + j]);
        for (int i = 0; i < n; ++i) U[IX(i, j, n)] = U[IX(i, j0 + j, n)] * f;   /* X' in the first m columns */
    }
    herm_full(n, H, ldh, Hf);
    if (m > 0) {
        or_zgemm('N', 'N', n, m, n, 1.0, Hf, n, U, n, 0.0, G, n);
        or_zgemm('C', 'N', m, m, n, 1.0, U, n, G, n, 0.0, A, m);
        st = or_eigen_hh(m, A, m, wr, Y, NULL, NULL);
        if (st != OR_OK) goto out;
        or_zgemm('N', 'N', n, m, m, 1.0, U, n, Y, m, 0.0, G, n);
    }
    for (int j = 0; j < n; ++j) {
        w[j] = j < m ? wr[j] : INFINITY;
        if (C)
            for (int i = 0; i < n; ++i) C[IX(i, j, ldc)] = j < m ? G[IX(i, j, n)] : 0.0;
    }
    st = OR_OK;
out:
    free(s); free(U); free(Hf); free(G); free(A); free(Y); free(wr);
    return st;
}

/* ------------------------------------------------------------------------
 * Band_DFT_Col Part 1 (k-point dependence of H and S).  The paper names the
 * step only; the reading is the Bloch sum over real-space blocks,
 *   M(k)_{IJ} = sum over the blocks (I, J, R) of exp(2 pi i k.R) M_{IJ}(R),
 * with k and R in fractional (reciprocal / direct lattice) coordinates.
 * Atoms I have orbitals off[I] .. off[I+1]-1.  Block q (q < nblocks) is the
 * pair (bi[q], bj[q]) at lattice vector R[rid[q]] (3 doubles), with data at
 * data + doff[q] (n_I x n_J, column-major).  Out: nk matrices n x n (ld n),
 * zero where no block contributes; blocks are added in index order.
 * ---------------------------------------------------------------------- */
void or_bloch(int natom, const int* off, int nblocks, const int* bi, const int* bj, const int* rid,
              const long* doff, const zc* data, const double* R, int nk, const double* kf, zc* out)
{
    const int n = off[natom];
    for (size_t q = 0; q < (size_t)nk * n * n; ++q) out[q] = 0.0;
    for (int k = 0; k < nk; ++k) {
        zc* Ok = out + (size_t)k * n * n;
        for (int q = 0; q < nblocks; ++q) {
            const double* r = R + 3 * (size_t)rid[q];
            const double ph = 2.0 * M_PI * (kf[3 * k] * r[0] + kf[3 * k + 1] * r[1] + kf[3 * k + 2] * r[2]);
            const zc e = cos(ph) + I * sin(ph);
            const int I0 = off[bi[q]], ni = off[bi[q] + 1] - I0;
            const int J0 = off[bj[q]], nj = off[bj[q] + 1] - J0;
            const zc* M = data + doff[q];
            for (int c = 0; c < nj; ++c)
                for (int a = 0; a < ni; ++a) Ok[IX(I0 + a, J0 + c, n)] += e * M[IX(a, c, ni)];
        }
    }
}
