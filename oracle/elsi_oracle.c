/*
 * elsi_oracle.c -- plain, slow, FP64 CPU reference for the dense Kohn-Sham path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and must never serve as a
 * fallback for it.
 *
 * What it computes (ELSI paper, Sec. 2 and Sec. 3.1):
 *   - the generalized eigenproblem H c = eps S c, Eq. (6), for real symmetric
 *     H and symmetric positive definite S;
 *   - by the route the paper describes for ELPA: Cholesky S = L L^T, Eq. (10);
 *     H~ = L^-1 H L^-T, Eq. (11); one-stage Householder tridiagonalization
 *     T = Q^T H~ Q, Eq. (12); a tridiagonal eigensolver (implicit QL here);
 *     back substitution c = L^-T c~ (Sec. 3.1, below Eq. (11));
 *   - Fermi-Dirac occupations, Eq. (17), with the chemical potential fixed by
 *     the electron count, Eq. (18), found by bisection from an interval spanned
 *     by the lowest and highest eigenvalue and widened when needed, followed by
 *     removal of the remaining electron surplus from the highest occupied
 *     states downward (Sec. 4.5, elsi_dm_real);
 *   - the density matrix n_ij = sum_l f_l c_il c_jl, Eq. (9), and the band
 *     energy sum_l f_l eps_l (Sec. 4.5, "energy" output of elsi_dm_real).
 *   - FP64 refinement sweeps (CholeskyQR twice, Rayleigh-Ritz, residuals
 *     and a Newton correction through an approximate factorization of H~)
 *     of an approximate invariant subspace of H~, the last stage of the GPU
 *     library's mixed-precision mode (orc_refine);
 *   - the same steps for complex Hermitian H and Hermitian positive definite
 *     S (the complex interface of Sec. 4.3, the k-point problems of periodic
 *     systems), the Householder tridiagonal made real by a diagonal unitary
 *     scaling, and n_ij = sum_l f_l c_il conj(c_jl) (see the end of the file).
 *
 * Matrices are column-major with a leading dimension; the lower triangle of
 * the symmetric inputs is the one that is read.
 *
 * Sources for the textbook steps: Golub & Van Loan, "Matrix Computations"
 * (column Cholesky; Householder tridiagonalization; symmetric QR/QL step with
 * Wilkinson shift); Bowdler, Martin, Reinsch & Wilkinson (1968), the implicit
 * QL algorithm.  Every loop below follows the definition directly: there is
 * no blocking, and OpenMP only splits loops whose iterations write disjoint
 * outputs, each in a fixed order, so results do not depend on thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define IDX(i, j, ld) ((size_t)(j) * (size_t)(ld) + (size_t)(i))

/* ------------------------------------------------------------------------- */
/* Cholesky S = L L^T (Eq. (10)), column by column.  Returns 0, or j+1 when   */
/* the j-th pivot is not positive (S not positive definite).  L overwrites   */
/* the lower triangle; the strict upper triangle is set to zero.             */
/* ------------------------------------------------------------------------- */
int orc_potrf(int n, double *A, int lda)
{
    for (int j = 0; j < n; ++j) {
        double s = A[IDX(j, j, lda)];
        for (int k = 0; k < j; ++k) s -= A[IDX(j, k, lda)] * A[IDX(j, k, lda)];
        if (!(s > 0.0) || !isfinite(s)) return j + 1;
        double ljj = sqrt(s);
        A[IDX(j, j, lda)] = ljj;
        /* L_ij = (S_ij - sum_k L_ik L_jk) / L_jj for i > j */
#pragma omp parallel for schedule(static)
        for (int i = j + 1; i < n; ++i) {
            double t = A[IDX(i, j, lda)];
            for (int k = 0; k < j; ++k) t -= A[IDX(i, k, lda)] * A[IDX(j, k, lda)];
            A[IDX(i, j, lda)] = t / ljj;
        }
    }
    for (int j = 1; j < n; ++j)
        for (int i = 0; i < j; ++i) A[IDX(i, j, lda)] = 0.0;
    return 0;
}

/* x <- L^-1 x, forward substitution with the lower triangle of L. */
static void fwd_subst(int n, const double *L, int ldl, double *x)
{
    for (int k = 0; k < n; ++k) {
        x[k] /= L[IDX(k, k, ldl)];
        double xk = x[k];
        const double *col = L + IDX(0, k, ldl);
        for (int i = k + 1; i < n; ++i) x[i] -= col[i] * xk;
    }
}

/* x <- L^-T x, back substitution with the lower triangle of L. */
static void back_subst_t(int n, const double *L, int ldl, double *x)
{
    for (int i = n - 1; i >= 0; --i) {
        const double *col = L + IDX(0, i, ldl);
        double t = x[i];
        for (int j = i + 1; j < n; ++j) t -= col[j] * x[j];
        x[i] = t / col[i];
    }
}

/* ------------------------------------------------------------------------- */
/* Reduction to standard form, Eq. (11):  H <- L^-1 H L^-T (full symmetric). */
/* W = L^-1 H column by column; then H~ = L^-1 W^T (= L^-1 H L^-T since H is */
/* symmetric), again column by column; finally H~ <- (H~ + H~^T) / 2.        */
/* ------------------------------------------------------------------------- */
void orc_reduce(int n, double *H, int ldh, const double *L, int ldl)
{
    double *W = (double *)malloc(sizeof(double) * (size_t)n * n);
    /* symmetric input: expand the lower triangle into W's columns */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double *w = W + (size_t)j * n;
        for (int i = 0; i < n; ++i) w[i] = (i >= j) ? H[IDX(i, j, ldh)] : H[IDX(j, i, ldh)];
        fwd_subst(n, L, ldl, w);
    }
    /* H~(:, j) = L^-1 (row j of W)^T */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double *x = (double *)malloc(sizeof(double) * n);
        for (int i = 0; i < n; ++i) x[i] = W[(size_t)i * n + j];
        fwd_subst(n, L, ldl, x);
        for (int i = 0; i < n; ++i) H[IDX(i, j, ldh)] = x[i];
        free(x);
    }
    free(W);
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i) {
            double a = 0.5 * (H[IDX(i, j, ldh)] + H[IDX(j, i, ldh)]);
            H[IDX(i, j, ldh)] = a;
            H[IDX(j, i, ldh)] = a;
        }
}

/* ------------------------------------------------------------------------- */
/* Householder tridiagonalization with Q accumulated (one-stage, Eq. (12)).  */
/* On entry A is full symmetric (both triangles).  On exit d (n), e (n-1)    */
/* hold T, and Q (n x n) satisfies A = Q T Q^T.  A is destroyed.             */
/* Step k: v = house(A(k+1:n, k)), p = beta A22 v, w = p - (beta p^T v / 2) v */
/* and A22 <- A22 - v w^T - w v^T (Golub & Van Loan, Householder            */
/* tridiagonalization).  Q = H_0 H_1 ... H_{n-3} by backward accumulation.   */
/* ------------------------------------------------------------------------- */
void orc_tred(int n, double *A, int lda, double *d, double *e, double *Q, int ldq)
{
    double *beta = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int k = 0; k + 2 < n; ++k) {
        int m = n - k - 1;                       /* length of the vector below row k */
        double *x = A + IDX(k + 1, k, lda);     /* A(k+1:n, k), overwritten by v */
        double tail = 0.0;
        for (int i = 1; i < m; ++i) tail += x[i] * x[i];
        double x0 = x[0];
        if (tail == 0.0) {                       /* already reduced: H_k = I */
            beta[k] = 0.0;
            e[k] = x0;
            for (int i = 1; i < m; ++i) x[i] = 0.0;
            continue;
        }
        double nrm = sqrt(x0 * x0 + tail);
        double alpha = (x0 >= 0.0) ? -nrm : nrm; /* (I - beta v v^T) x = alpha e_1 */
        double v0 = x0 - alpha;
        for (int i = 1; i < m; ++i) x[i] /= v0;  /* v = [1, x(1:)/v0] */
        x[0] = 1.0;
        double vtv = 1.0 + tail / (v0 * v0);
        double b = 2.0 / vtv;
        beta[k] = b;
        e[k] = alpha;
        double *A22 = A + IDX(k + 1, k + 1, lda);
        /* p = beta * A22 v (A22 symmetric, columns read contiguously) */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < m; ++j) {
            const double *col = A22 + (size_t)j * lda;
            double t = 0.0;
            for (int i = 0; i < m; ++i) t += col[i] * x[i];
            p[j] = b * t;
        }
        double ptv = 0.0;
        for (int i = 0; i < m; ++i) ptv += p[i] * x[i];
        double half = 0.5 * b * ptv;
        for (int i = 0; i < m; ++i) p[i] -= half * x[i]; /* p is now w */
        /* A22 <- A22 - v w^T - w v^T */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < m; ++j) {
            double *col = A22 + (size_t)j * lda;
            double vj = x[j], wj = p[j];
            for (int i = 0; i < m; ++i) col[i] -= x[i] * wj + p[i] * vj;
        }
    }
    for (int i = 0; i < n; ++i) d[i] = A[IDX(i, i, lda)];
    if (n >= 2) e[n - 2] = A[IDX(n - 1, n - 2, lda)];

    /* Q = H_0 H_1 ... H_{n-3}: start from I and apply H_k to Q(k+1:, k+1:), k descending */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) Q[IDX(i, j, ldq)] = (i == j) ? 1.0 : 0.0;
    for (int k = n - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        int m = n - k - 1;
        const double *v = A + IDX(k + 1, k, lda);
        double b = beta[k];
#pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {
            double *col = Q + IDX(k + 1, j, ldq);
            double t = 0.0;
            for (int i = 0; i < m; ++i) t += v[i] * col[i];
            t *= b;
            for (int i = 0; i < m; ++i) col[i] -= t * v[i];
        }
    }
    free(beta);
    free(p);
}

/* ------------------------------------------------------------------------- */
/* Implicit QL on a symmetric tridiagonal (d, e) with eigenvector update.    */
/* e[i] couples rows i and i+1.  Each sweep on an unreduced block [l, m]     */
/* takes the shift from the leading 2x2 (the eigenvalue of it nearer to      */
/* d[l]), starts with the rotation fixed by the last column of T - mu I, and */
/* chases the bulge upward; the top off-diagonal converges and deflates.     */
/* A rotation in plane (p, p+1) maps a pair (x_p, x_q) to                    */
/* (c x_p - s x_q, s x_p + c x_q); it acts the same way on the rows of Q.    */
/* Q is held row-major in Qr (n x n) so that each row is contiguous.         */
/* Returns 0, or 2 when more than 30 n sweeps were needed.                   */
/* ------------------------------------------------------------------------- */
static void rot_apply(double *xp, double *xq, double c, double s)
{
    double a = *xp, b = *xq;
    *xp = c * a - s * b;
    *xq = s * a + c * b;
}

int orc_tql(int n, double *d, double *e, double *Qr, int with_vectors)
{
    if (n <= 1) return 0;
    int *rp = (int *)malloc(sizeof(int) * n);
    double *rc = (double *)malloc(sizeof(double) * n);
    double *rs = (double *)malloc(sizeof(double) * n);
    long iter = 0, max_iter = 30L * n;
    int status = 0;
    int l = 0;
    while (l < n) {
        int m = l;
        while (m < n - 1) {
            double dd = fabs(d[m]) + fabs(d[m + 1]);
            if (fabs(e[m]) <= DBL_EPSILON * dd) break;
            ++m;
        }
        if (m == l) { ++l; continue; }
        if (++iter > max_iter) { status = 2; break; }
        if (m < n - 1) e[m] = 0.0;   /* the split is exact from here on */
        /* shift: eigenvalue of [[d_l, e_l], [e_l, d_{l+1}]] nearer to d_l */
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = hypot(g, 1.0);
        double mu = d[l] - e[l] / (g + (g >= 0.0 ? r : -r));
        int nrot = 0;
        double bulge = 0.0;
        for (int p = m - 1; p >= l; --p) {
            int q = p + 1;
            double xp, xq;
            if (p == m - 1) { xp = e[p]; xq = d[q] - mu; }   /* last column of T - mu I */
            else            { xp = bulge; xq = e[q]; }       /* (T_{p,q+1}, T_{q,q+1})  */
            double rr = hypot(xp, xq);
            double c, s;
            if (rr == 0.0) { c = 1.0; s = 0.0; }
            else { c = xq / rr; s = xp / rr; }
            if (p != m - 1) e[q] = rr;                       /* bulge annihilated */
            /* 2x2 block M [[a, b], [b, cq]] M^T with M = [[c, -s], [s, c]] */
            double a = d[p], b = e[p], cq = d[q];
            d[p] = c * c * a - 2.0 * c * s * b + s * s * cq;
            e[p] = c * s * a + (c * c - s * s) * b - c * s * cq;
            d[q] = s * s * a + 2.0 * c * s * b + c * c * cq;
            if (p > l) {                                     /* row p-1 couples to p and q */
                double ep = e[p - 1];
                e[p - 1] = c * ep;
                bulge = s * ep;
            }
            rp[nrot] = p; rc[nrot] = c; rs[nrot] = s; ++nrot;
        }
        if (with_vectors) {
#pragma omp parallel for schedule(static)
            for (int row = 0; row < n; ++row) {
                double *qrow = Qr + (size_t)row * n;
                for (int t = 0; t < nrot; ++t)
                    rot_apply(&qrow[rp[t]], &qrow[rp[t] + 1], rc[t], rs[t]);
            }
        }
    }
    free(rp); free(rc); free(rs);
    return status;
}

/* stable ascending order of w: perm[0..n-1] (merge sort on indices) */
static void stable_argsort(int n, const double *w, int *perm)
{
    int *tmp = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int width = 1; width < n; width *= 2) {
        for (int lo = 0; lo < n; lo += 2 * width) {
            int mid = lo + width < n ? lo + width : n;
            int hi = lo + 2 * width < n ? lo + 2 * width : n;
            int a = lo, b = mid, o = lo;
            while (a < mid && b < hi) tmp[o++] = (w[perm[b]] < w[perm[a]]) ? perm[b++] : perm[a++];
            while (a < mid) tmp[o++] = perm[a++];
            while (b < hi) tmp[o++] = perm[b++];
        }
        memcpy(perm, tmp, sizeof(int) * n);
    }
    free(tmp);
}

/* ------------------------------------------------------------------------- */
/* Back substitution c = L^-T c~ for k columns (Sec. 3.1, below Eq. (11)).   */
/* ------------------------------------------------------------------------- */
void orc_backsub(int n, int k, const double *L, int ldl, double *Z, int ldz)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < k; ++j) back_subst_t(n, L, ldl, Z + (size_t)j * ldz);
}

/* Sign convention: the largest-magnitude entry of each column is positive. */
static void normalize_sign(int n, int k, double *C, int ldc)
{
    for (int j = 0; j < k; ++j) {
        double *c = C + (size_t)j * ldc;
        int imax = 0;
        for (int i = 1; i < n; ++i) if (fabs(c[i]) > fabs(c[imax])) imax = i;
        if (c[imax] < 0.0) for (int i = 0; i < n; ++i) c[i] = -c[i];
    }
}

/* ------------------------------------------------------------------------- */
/* Full generalized eigensolve, Eq. (6):  eval (n, ascending), evec n x      */
/* n_state (column-major, ldc = n).  H and S are destroyed (S -> L).         */
/* Returns 0, 1 (S not positive definite; *fail_col = pivot), 2 (QL failed). */
/* ------------------------------------------------------------------------- */
int orc_gevp(int n, int n_state, double *H, int ldh, double *S, int lds,
             double *eval, double *evec, int *fail_col)
{
    if (fail_col) *fail_col = 0;
    int info = orc_potrf(n, S, lds);
    if (info) { if (fail_col) *fail_col = info; return 1; }
    orc_reduce(n, H, ldh, S, lds);
    double *d = (double *)malloc(sizeof(double) * n);
    double *e = (double *)calloc((size_t)n, sizeof(double));
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * n);
    orc_tred(n, H, ldh, d, e, Q, n);
    /* QL works on Q's rows: Qr = Q^T in column-major == Q in row-major */
    double *Qr = (double *)malloc(sizeof(double) * (size_t)n * n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Qr[(size_t)i * n + j] = Q[IDX(i, j, n)];
    int st = orc_tql(n, d, e, Qr, 1);
    if (st) { free(d); free(e); free(Q); free(Qr); return st; }
    int *perm = (int *)malloc(sizeof(int) * n);
    stable_argsort(n, d, perm);
    for (int j = 0; j < n; ++j) eval[j] = d[perm[j]];
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n_state; ++j)
        for (int i = 0; i < n; ++i) evec[IDX(i, j, n)] = Qr[(size_t)i * n + perm[j]];
    orc_backsub(n, n_state, S, lds, evec, n);
    normalize_sign(n, n_state, evec, n);
    free(perm); free(d); free(e); free(Q); free(Qr);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Singularity check of the overlap and the eigendecomposition transform     */
/* (Sec. 4.5, Eq. (20)).  All eigenvalues lam of S are compared with the     */
/* tolerance tau; when the smallest is >= tau (S well conditioned) the call   */
/* is orc_gevp.  Otherwise S = x diag(lam) x^T = X X^T with X = x sqrt(lam), */
/* and the N_nonsing = m eigenvectors with lam >= tau are kept: with          */
/* Y = x_keep diag(lam_keep)^(-1/2) (n x m),                                  */
/*   H~ = Y^T H Y (m x m),  H~ c~ = eps c~,  c = Y c~   (c^T S c = I).        */
/* eval[0 .. m) receives the m eigenvalues ascending and eval[m .. n) the     */
/* value +HUGE_VAL (no state there); evec (n x n_state) the first             */
/* min(n_state, m) vectors c (largest |component| positive), later columns   */
/* zero; S is overwritten by X's kept columns [0 .. m) (the rest zero).       */
/* *n_nonsing = m (n on the Cholesky route).  Returns as orc_gevp.           */
/* ------------------------------------------------------------------------- */
int orc_gevp_checked(int n, int n_state, double *H, int ldh, double *S, int lds, double tau, double *eval,
                     double *evec, int *n_nonsing, int *fail_col)
{
    double *Sc = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *I = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *lam = (double *)malloc(sizeof(double) * n);
    double *xv = (double *)malloc(sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            Sc[IDX(i, j, n)] = (i >= j) ? S[IDX(i, j, lds)] : S[IDX(j, i, lds)];
            I[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
        }
    int st = orc_gevp(n, n, Sc, n, I, n, lam, xv, NULL);   /* S = x diag(lam) x^T */
    if (st) { free(Sc); free(I); free(lam); free(xv); return st; }
    if (lam[0] >= tau) {
        free(Sc); free(I); free(lam); free(xv);
        if (n_nonsing) *n_nonsing = n;
        return orc_gevp(n, n_state, H, ldh, S, lds, eval, evec, fail_col);
    }
    if (fail_col) *fail_col = 0;
    int m = 0;
    for (int l = 0; l < n; ++l) if (lam[l] >= tau) ++m;
    const int first = n - m;   /* lam ascending: the kept ones are the last m */
    if (n_nonsing) *n_nonsing = m;
    double *Y = (double *)malloc(sizeof(double) * (size_t)n * (m > 0 ? m : 1));
    for (int j = 0; j < m; ++j) {
        const double sc = 1.0 / sqrt(lam[first + j]);
        for (int i = 0; i < n; ++i) Y[IDX(i, j, n)] = xv[IDX(i, first + j, n)] * sc;
    }
    /* H~ = Y^T H Y, lower triangle of H read */
    double *HY = (double *)malloc(sizeof(double) * (size_t)n * (m > 0 ? m : 1));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) {
            double t = 0.0;
            for (int c = 0; c < n; ++c) {
                const double h = (i >= c) ? H[IDX(i, c, ldh)] : H[IDX(c, i, ldh)];
                t += h * Y[IDX(c, j, n)];
            }
            HY[IDX(i, j, n)] = t;
        }
    double *Ht = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (m > 0 ? m : 1));
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            double t = 0.0;
            for (int r = 0; r < n; ++r) t += Y[IDX(r, i, n)] * HY[IDX(r, j, n)];
            Ht[IDX(i, j, m)] = t;
        }
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < j; ++i) {
            const double a = 0.5 * (Ht[IDX(i, j, m)] + Ht[IDX(j, i, m)]);
            Ht[IDX(i, j, m)] = a;
            Ht[IDX(j, i, m)] = a;
        }
    double *Im = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (m > 0 ? m : 1));
    double *ct = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (m > 0 ? m : 1));
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) Im[IDX(i, j, m)] = (i == j) ? 1.0 : 0.0;
    st = (m > 0) ? orc_gevp(m, m, Ht, m, Im, m, eval, ct, NULL) : 0;
    if (!st) {
        for (int l = m; l < n; ++l) eval[l] = HUGE_VAL;
        const int kk = n_state < m ? n_state : m;
#pragma omp parallel for schedule(static)
        for (int j = 0; j < n_state; ++j)
            for (int i = 0; i < n; ++i) {
                double t = 0.0;
                if (j < kk)
                    for (int c = 0; c < m; ++c) t += Y[IDX(i, c, n)] * ct[IDX(c, j, m)];
                evec[IDX(i, j, n)] = t;
            }
        normalize_sign(n, kk, evec, n);
        /* S <- X = x_keep diag(sqrt(lam_keep)) */
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                S[IDX(i, j, lds)] = (j < m) ? xv[IDX(i, first + j, n)] * sqrt(lam[first + j]) : 0.0;
    }
    free(Sc); free(I); free(lam); free(xv); free(Y); free(HY); free(Ht); free(Im); free(ct);
    return st;
}

/* Tridiagonal eigenvalues only (QL without vectors), ascending. */
int orc_tridiag_eigvals(int n, double *d, double *e, double *w)
{
    int st = orc_tql(n, d, e, NULL, 0);
    if (st) return st;
    int *perm = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    stable_argsort(n, d, perm);
    for (int j = 0; j < n; ++j) w[j] = d[perm[j]];
    free(perm);
    return 0;
}

/* Tridiagonal eigenpairs: Z (n x n, column-major) holds the eigenvectors. */
int orc_tridiag_eig(int n, double *d, double *e, double *w, double *Z)
{
    double *Qr = (double *)malloc(sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Qr[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    int st = orc_tql(n, d, e, Qr, 1);
    if (!st) {
        int *perm = (int *)malloc(sizeof(int) * n);
        stable_argsort(n, d, perm);
        for (int j = 0; j < n; ++j) {
            w[j] = d[perm[j]];
            for (int i = 0; i < n; ++i) Z[IDX(i, j, n)] = Qr[(size_t)i * n + perm[j]];
        }
        normalize_sign(n, n, Z, n);
        free(perm);
    }
    free(Qr);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Occupation of one state, x = (eps - mu) / width, for the broadening       */
/* schemes of Sec. 4.6 (broadening_scheme):                                  */
/*   1 Fermi-Dirac, Eq. (17), written so that no exponential overflows:      */
/*       f = spin e^-x / (1 + e^-x) for x >= 0, spin / (1 + e^x) for x < 0;  */
/*   2 Gaussian, Eq. (21): f = spin (1 - erf x) / 2, evaluated as            */
/*       spin erfc(x) / 2 (the same function, without the cancellation);     */
/*   3 Methfessel-Paxton of order 0: the Gaussian step;                      */
/*   4 Methfessel-Paxton of order 1 (Methfessel & Paxton, Phys. Rev. B 40,   */
/*       3616 (1989): S_N = S_0 + sum_{n=1..N} A_n H_{2n-1}(x) e^{-x^2},     */
/*       A_n = (-1)^n / (n! 4^n sqrt(pi)); for N = 1, A_1 H_1(x) =           */
/*       -x / (2 sqrt(pi))):  f = spin (erfc(x)/2 - x e^{-x^2}/(2 sqrt(pi))).*/
/*       These occupations leave [0, spin] near mu.                          */
/* ------------------------------------------------------------------------- */
double orc_occupation_value(int scheme, double eps, double mu, double width, double spin)
{
    const double x = (eps - mu) / width;
    switch (scheme) {
    case 2:
    case 3:
        return spin * 0.5 * erfc(x);
    case 4:
        return spin * (0.5 * erfc(x) - x * exp(-x * x) / (2.0 * sqrt(3.14159265358979323846)));
    default:
        if (x >= 0.0) { double t = exp(-x); return spin * t / (1.0 + t); }
        return spin / (1.0 + exp(x));
    }
}

/* electrons at mu: sum_l w_l f_l (w NULL: all 1) */
static double electron_count(int n, const double *eps, const double *w, int scheme, double mu, double width,
                             double spin)
{
    double s = 0.0;
    for (int l = 0; l < n; ++l) s += (w ? w[l] : 1.0) * orc_occupation_value(scheme, eps[l], mu, width, spin);
    return s;
}

/* ------------------------------------------------------------------------- */
/* Chemical potential by bisection on  sum_l w_l f_l(mu) - N_e, Eq. (18)     */
/* (Sec. 4.5; with weights the sum runs over k-points and spin channels):    */
/* interval [min eps - 10 width, max eps + 10 width], widened (the step      */
/* doubling each time) until it brackets the root; halved until the electron */
/* count is within occ_accuracy, the interval cannot shrink any further in   */
/* floating point, or max_steps halvings were made.  mu is the upper bound   */
/* (surplus >= 0); f_l = w_l f(eps_l); the surplus is then removed from the  */
/* highest-index states with f > 0 downward so that sum f = N_e.             */
/* eps ascending within each problem; w (per state, may be NULL).  Returns   */
/* 0, or 4 when max_steps ran out first.                                     */
/* ------------------------------------------------------------------------- */
int orc_occupations_scheme(int n, const double *eps, const double *w, int scheme, double n_electron,
                           double width, double spin, double occ_accuracy, int max_steps, double *f,
                           double *mu_out)
{
    double emin = eps[0], emax = eps[0];
    for (int l = 1; l < n; ++l) {
        if (eps[l] < emin) emin = eps[l];
        if (eps[l] > emax) emax = eps[l];
    }
    double lo = emin - 10.0 * width, hi = emax + 10.0 * width;
    double step = hi - lo;
    for (int t = 0; t < 64 && electron_count(n, eps, w, scheme, lo, width, spin) - n_electron > 0.0; ++t) {
        lo -= step; step *= 2.0;
    }
    step = hi - lo;
    for (int t = 0; t < 64 && electron_count(n, eps, w, scheme, hi, width, spin) - n_electron < 0.0; ++t) {
        hi += step; step *= 2.0;
    }
    /* the upper bound always carries a surplus g(hi) >= 0; stop once it is    */
    /* within occ_accuracy or the midpoint no longer differs from the bounds   */
    int status = 0, steps = 0;
    for (;;) {
        double mid = 0.5 * (lo + hi);
        if (!(lo < mid && mid < hi)) break;
        if (steps >= max_steps) { status = 4; break; }
        ++steps;
        double g = electron_count(n, eps, w, scheme, mid, width, spin) - n_electron;
        if (g >= 0.0) {
            hi = mid;
            if (g <= occ_accuracy) break;
        } else {
            lo = mid;
        }
    }
    double mu = hi;
    for (int l = 0; l < n; ++l) f[l] = (w ? w[l] : 1.0) * orc_occupation_value(scheme, eps[l], mu, width, spin);
    double surplus = electron_count(n, eps, w, scheme, mu, width, spin) - n_electron;
    for (int l = n - 1; l >= 0 && surplus > 0.0; --l) {
        if (f[l] <= 0.0) continue;
        double take = f[l] < surplus ? f[l] : surplus;
        f[l] -= take;
        surplus -= take;
    }
    *mu_out = mu;
    return status;
}

/* Fermi-Dirac occupations of one problem (scheme 1, no weights). */
int orc_occupations(int n, const double *eps, double n_electron, double kT, double spin,
                    double occ_accuracy, int max_steps, double *f, double *mu_out)
{
    return orc_occupations_scheme(n, eps, NULL, 1, n_electron, kT, spin, occ_accuracy, max_steps, f, mu_out);
}

/* ------------------------------------------------------------------------- */
/* Density matrix, Eq. (9):  D_ij = sum_l f_l c_il c_jl over every state     */
/* with f_l != 0 (Methfessel-Paxton occupations can be negative).            */
/* C is n x k (column-major, ldc), D is n x n (ldd), both triangles written. */
/* ------------------------------------------------------------------------- */
void orc_density(int n, int k, const double *C, int ldc, const double *f, double *D, int ldd)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double *dcol = D + (size_t)j * ldd;
        for (int i = 0; i < n; ++i) dcol[i] = 0.0;
        for (int l = 0; l < k; ++l) {
            if (f[l] == 0.0) continue;
            const double *c = C + (size_t)l * ldc;
            double w = f[l] * c[j];
            for (int i = 0; i < n; ++i) dcol[i] += w * c[i];
        }
    }
}

/* Band energy (Sec. 4.5):  E = sum_l f_l eps_l. */
double orc_band_energy(int n, const double *f, const double *eps)
{
    double s = 0.0;
    for (int l = 0; l < n; ++l) s += f[l] * eps[l];
    return s;
}

/* ------------------------------------------------------------------------- */
/* Density-matrix driver: eigensolve, occupations, D and energy.             */
/* Returns 0 / 1 / 2 as orc_gevp, or 4 when the bisection ran out of steps.  */
/* ------------------------------------------------------------------------- */
int orc_dm_scheme(int n, double *H, int ldh, double *S, int lds, int scheme, double n_electron, double kT,
                  double spin, double occ_accuracy, int max_steps, double *D, int ldd,
                  double *eval, double *occ, double *energy, double *mu, int *fail_col)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)n * n);
    int st = orc_gevp(n, n, H, ldh, S, lds, eval, C, fail_col);
    if (st) { free(C); return st; }
    st = orc_occupations_scheme(n, eval, NULL, scheme, n_electron, kT, spin, occ_accuracy, max_steps, occ, mu);
    orc_density(n, n, C, n, occ, D, ldd);
    *energy = orc_band_energy(n, occ, eval);
    free(C);
    return st;
}

/* Density matrix with the singularity check (Eq. (20)): the occupations and  */
/* D run over the n_nonsing states of orc_gevp_checked.                       */
int orc_dm_checked(int n, double *H, int ldh, double *S, int lds, double tau, int scheme, double n_electron,
                   double kT, double spin, double occ_accuracy, int max_steps, double *D, int ldd, double *eval,
                   double *occ, double *energy, double *mu, int *n_nonsing, int *fail_col)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)n * n);
    int m = n;
    int st = orc_gevp_checked(n, n, H, ldh, S, lds, tau, eval, C, &m, fail_col);
    if (st) { free(C); return st; }
    if (n_nonsing) *n_nonsing = m;
    for (int l = 0; l < n; ++l) occ[l] = 0.0;
    st = orc_occupations_scheme(m, eval, NULL, scheme, n_electron, kT, spin, occ_accuracy, max_steps, occ, mu);
    orc_density(n, m, C, n, occ, D, ldd);
    *energy = orc_band_energy(m, occ, eval);
    free(C);
    return st;
}

int orc_dm(int n, double *H, int ldh, double *S, int lds, double n_electron, double kT,
           double spin, double occ_accuracy, int max_steps, double *D, int ldd,
           double *eval, double *occ, double *energy, double *mu, int *fail_col)
{
    return orc_dm_scheme(n, H, ldh, S, lds, 1, n_electron, kT, spin, occ_accuracy, max_steps, D, ldd, eval, occ,
                         energy, mu, fail_col);
}

/* ------------------------------------------------------------------------- */
/* Residual certificate in extended precision: for each of the k columns x   */
/* of X with value lam, r = H x - lam S x; writes ||r||_2 into res.  H and S */
/* are the original (symmetric, lower triangle read) matrices.               */
/* ------------------------------------------------------------------------- */
void orc_residual_norms(int n, int k, const double *H, int ldh, const double *S, int lds,
                        const double *X, int ldx, const double *lam, double *res)
{
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < k; ++j) {
        const double *x = X + (size_t)j * ldx;
        long double acc = 0.0L;
        for (int i = 0; i < n; ++i) {
            long double r = 0.0L;
            for (int c = 0; c < n; ++c) {
                long double h = (i >= c) ? H[IDX(i, c, ldh)] : H[IDX(c, i, ldh)];
                long double s = (i >= c) ? S[IDX(i, c, lds)] : S[IDX(c, i, lds)];
                r += (h - (long double)lam[j] * s) * (long double)x[c];
            }
            acc += r * r;
        }
        res[j] = (double)sqrtl(acc);
    }
}

/* ------------------------------------------------------------------------- */
/* (T - shift I) x = b for the symmetric tridiagonal T = tridiag(e, d, e)    */
/* (d: n, e: n-1) by Gaussian elimination with partial (row) pivoting: at    */
/* step k the row with the larger |entry| in column k (the current row on a  */
/* tie) becomes the pivot row, so U has at most two superdiagonals.  A pivot */
/* that is exactly zero is replaced by DBL_EPSILON times the largest row sum */
/* of |T - shift I|, the usual guard of inverse iteration.                   */
/* ------------------------------------------------------------------------- */
void orc_tridiag_shift_solve(int n, const double *d, const double *e, double shift, const double *b,
                             double *x)
{
    if (n <= 0) return;
    double *u0 = (double *)malloc(sizeof(double) * n);
    double *u1 = (double *)malloc(sizeof(double) * n);
    double *u2 = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * n);
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = fabs(d[i] - shift);
        if (i > 0) r += fabs(e[i - 1]);
        if (i + 1 < n) r += fabs(e[i]);
        if (r > tnorm) tnorm = r;
        y[i] = b[i];
    }
    double tiny = DBL_EPSILON * tnorm;
    if (tiny == 0.0) tiny = DBL_MIN;
    double p = d[0] - shift;                 /* current row: (p, q) in columns k, k+1 */
    double q = (n > 1) ? e[0] : 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        const double a = e[k];               /* row k+1: (a, bb, c) in columns k, k+1, k+2 */
        const double bb = d[k + 1] - shift;
        const double c = (k + 2 < n) ? e[k + 1] : 0.0;
        if (fabs(p) >= fabs(a)) {
            if (p == 0.0) p = tiny;
            const double m = a / p;
            u0[k] = p; u1[k] = q; u2[k] = 0.0;
            y[k + 1] -= m * y[k];
            p = bb - m * q;
            q = c;
        } else {
            const double m = p / a;
            u0[k] = a; u1[k] = bb; u2[k] = c;
            const double yk = y[k], yk1 = y[k + 1];
            y[k] = yk1;
            y[k + 1] = yk - m * yk1;
            const double pn = q - m * bb;
            q = -m * c;
            p = pn;
        }
    }
    if (p == 0.0) p = tiny;
    u0[n - 1] = p; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
    for (int k = n - 1; k >= 0; --k) {
        double t = y[k];
        if (k + 1 < n) t -= u1[k] * x[k + 1];
        if (k + 2 < n) t -= u2[k] * x[k + 2];
        x[k] = t / u0[k];
    }
    free(u0); free(u1); free(u2); free(y);
}

/* X <- X L_G^-T with G = X^T X = L_G L_G^T (CholeskyQR), `passes` times.   */
/* Returns 0, or 1 when a Gram matrix is not positive definite (X untouched  */
/* then, or after the first pass).                                           */
static int cholesky_qr(int n, int k, double *X, int ldx, double *G, int passes)
{
    for (int pass = 0; pass < passes; ++pass) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i) {
                double t = 0.0;
                for (int r = 0; r < n; ++r) t += X[IDX(r, i, ldx)] * X[IDX(r, j, ldx)];
                G[IDX(i, j, k)] = t;
            }
        if (orc_potrf(k, G, k)) return 1;
#pragma omp parallel for schedule(static)
        for (int r = 0; r < n; ++r) {
            double *row = (double *)malloc(sizeof(double) * k);
            for (int j = 0; j < k; ++j) row[j] = X[IDX(r, j, ldx)];
            fwd_subst(k, G, k, row);   /* L_G y = x^T  <=>  y^T = x L_G^-T */
            for (int j = 0; j < k; ++j) X[IDX(r, j, ldx)] = row[j];
            free(row);
        }
    }
    return 0;
}

/* ========================================================================= */
/* FP64 refinement of an approximate invariant subspace of the standard-form */
/* matrix H~ = L^-1 H L^-T (Eq. (11)): the last stage of the GPU library's   */
/* mixed-precision mode (the paper's solvers run in one precision, so this   */
/* stage has no passage of its own).  X is n x k (ldx), approximating the    */
/* invariant subspace of the k lowest eigenvalues; on return it holds the    */
/* refined vectors.                                                          */
/*                                                                           */
/* Each sweep:                                                               */
/*   (1) CholeskyQR: G = X^T X = L_G L_G^T, X <- X L_G^-T (twice in the first */
/*       sweep, once after a correction);                                     */
/*   (2) Rayleigh-Ritz: A = X^T H~ X = W diag(theta) W^T (orc_gevp, S = I),  */
/*       X <- X W;                                                           */
/*   (3) residuals r_l = H~ x_l - theta_l x_l, res_l = ||r_l||_2.            */
/* Rayleigh-Ritz picks the best vectors inside span(X) but never moves that  */
/* span, so without more information one sweep is all that can be done: the */
/* call then ends with 0 when max res_l <= tol over the first kw states, 3   */
/* otherwise (Qp == NULL).                                                   */
/*                                                                           */
/* With an approximate factorization H~ ~ Qp T Qp^T (Qp n x n orthogonal,   */
/* T = tridiag(eT, dT, eT); in the mixed mode these are the reduced-         */
/* precision reduction's own Q1 Q2 and T) each sweep also forms the Newton   */
/* correction of the subspace: with Z the eigenvectors of T for its k lowest */
/* eigenvalues (computed here by QL) and P = I - Z Z^T,                      */
/*   (4) y_l = -P (T - theta_l I)^-1 P Qp^T r_l,   step_l = ||y_l||_2;        */
/* this solves the correction equation (H~ - theta_l) d_l = -r_l on the      */
/* complement of the subspace with T standing in for Qp^T H~ Qp, so it       */
/* removes the subspace's error up to the factorization's error over the     */
/* gap between theta_l and the complement's spectrum.  Unless it was the     */
/* last allowed sweep (status 3, X as that sweep's Rayleigh-Ritz left it),   */
/* X_l += Qp y_l for every l with step_l <= 1/2 (a larger step lies outside  */
/* the region where the linear model holds and is not taken) and the next    */
/* sweep starts.  When the largest weighted step W_s = max_{l<kw} w_l step_l */
/* (weight NULL: w_l = 1) is <= tol, or when 10 (W_s / W_{s-1}) W_s <= tol   */
/* (the contraction measured over the last two steps predicts that taking    */
/* W_s leaves less than tol), that step is still taken and the next sweep,   */
/* steps (1)-(3) only, closes the call with 0 (the untaken step would be     */
/* amplified by L^-T in c = L^-T x).                                         */
/* Dependent columns (G not positive definite)                               */
/* end the call with 3 and leave X as the last completed sweep left it.      */
/* step (k, may be NULL) receives the last computed steps (0 without Qp).    */
/* ========================================================================= */
int orc_refine(int n, int k, int kw, const double *Ht, int ldh, double *X, int ldx, const double *Qp,
               int ldq, const double *dT, const double *eT, const double *weight, double *theta, double *res,
               double *step, double tol, int max_sweeps, int *sweeps)
{
    if (sweeps) *sweeps = 0;
    if (n <= 0 || k <= 0) return 0;
    if (kw > k) kw = k;
    if (kw < 0) kw = 0;
    double *G = (double *)malloc(sizeof(double) * (size_t)k * k);
    double *I = (double *)malloc(sizeof(double) * (size_t)k * k);
    double *Wq = (double *)malloc(sizeof(double) * (size_t)k * k);
    double *Xs = (double *)malloc(sizeof(double) * (size_t)n * k);
    double *R = (double *)malloc(sizeof(double) * (size_t)n * k);
    double *Y = (double *)malloc(sizeof(double) * (size_t)n * k);
    double *stp = (double *)malloc(sizeof(double) * (size_t)k);
    double *Z = NULL;
    for (int j = 0; j < k; ++j) if (step) step[j] = 0.0;
    if (Qp) {
        /* Z: eigenvectors of T for its k lowest eigenvalues */
        double *dd = (double *)malloc(sizeof(double) * n);
        double *ee = (double *)malloc(sizeof(double) * n);
        double *wt = (double *)malloc(sizeof(double) * n);
        double *Zt = (double *)malloc(sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; ++i) { dd[i] = dT[i]; ee[i] = (i + 1 < n) ? eT[i] : 0.0; }
        int st = orc_tridiag_eig(n, dd, ee, wt, Zt);
        if (!st) {
            Z = (double *)malloc(sizeof(double) * (size_t)n * k);
            memcpy(Z, Zt, sizeof(double) * (size_t)n * k);
        }
        free(dd); free(ee); free(wt); free(Zt);
        if (st) { free(G); free(I); free(Wq); free(Xs); free(R); free(Y); free(stp); return 3; }
    }
    int status = 3, finishing = 0;
    double prev_worst = 0.0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        /* (1) orthonormalize a copy, so that a failure leaves X as it was */
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < n; ++i) Xs[IDX(i, j, n)] = X[IDX(i, j, ldx)];
        /* twice for the starting vectors; once after a correction, which leaves */
        /* them orthonormal to O(step) */
        if (cholesky_qr(n, k, Xs, n, G, sweep == 0 ? 2 : 1)) { status = 3; break; }
        /* (2) A = X^T (H~ X), lower triangle of H~ read */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < n; ++i) {
                double t = 0.0;
                for (int c = 0; c < n; ++c) {
                    const double h = (i >= c) ? Ht[IDX(i, c, ldh)] : Ht[IDX(c, i, ldh)];
                    t += h * Xs[IDX(c, j, n)];
                }
                Y[IDX(i, j, n)] = t;
            }
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i) {
                double t = 0.0;
                for (int r = 0; r < n; ++r) t += Xs[IDX(r, i, n)] * Y[IDX(r, j, n)];
                G[IDX(i, j, k)] = t;
            }
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < j; ++i) {
                const double a = 0.5 * (G[IDX(i, j, k)] + G[IDX(j, i, k)]);
                G[IDX(i, j, k)] = a;
                G[IDX(j, i, k)] = a;
            }
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i) I[IDX(i, j, k)] = (i == j) ? 1.0 : 0.0;
        if (orc_gevp(k, k, G, k, I, k, theta, Wq, NULL)) { status = 3; break; }
        /* X <- X W */
#pragma omp parallel for schedule(static)
        for (int r = 0; r < n; ++r)
            for (int j = 0; j < k; ++j) {
                double t = 0.0;
                for (int c = 0; c < k; ++c) t += Xs[IDX(r, c, n)] * Wq[IDX(c, j, k)];
                X[IDX(r, j, ldx)] = t;
            }
        /* (3) r_l = H~ x_l - theta_l x_l from the definition */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < k; ++j) {
            double acc = 0.0;
            for (int i = 0; i < n; ++i) {
                double t = -theta[j] * X[IDX(i, j, ldx)];
                for (int c = 0; c < n; ++c) {
                    const double h = (i >= c) ? Ht[IDX(i, c, ldh)] : Ht[IDX(c, i, ldh)];
                    t += h * X[IDX(c, j, ldx)];
                }
                R[IDX(i, j, n)] = t;
                acc += t * t;
            }
            res[j] = sqrt(acc);
        }
        if (sweeps) *sweeps = sweep + 1;
        if (finishing) { status = 0; break; }   /* the closing Rayleigh-Ritz sweep */
        if (!Qp) {
            double rmax = 0.0;
            for (int l = 0; l < kw; ++l) if (res[l] > rmax) rmax = res[l];
            status = (rmax <= tol) ? 0 : 3;
            break;
        }
        /* (4) y_l = -P (T - theta_l)^-1 P Qp^T r_l */
#pragma omp parallel for schedule(dynamic)
        for (int j = 0; j < k; ++j) {
            double *rho = (double *)malloc(sizeof(double) * n);
            double *yv = (double *)malloc(sizeof(double) * n);
            double *cz = (double *)malloc(sizeof(double) * k);
            for (int i = 0; i < n; ++i) {
                double t = 0.0;
                for (int r = 0; r < n; ++r) t += Qp[IDX(r, i, ldq)] * R[IDX(r, j, n)];
                rho[i] = -t;
            }
            for (int c = 0; c < k; ++c) {
                double t = 0.0;
                for (int i = 0; i < n; ++i) t += Z[IDX(i, c, n)] * rho[i];
                cz[c] = t;
            }
            for (int i = 0; i < n; ++i) {
                double t = rho[i];
                for (int c = 0; c < k; ++c) t -= Z[IDX(i, c, n)] * cz[c];
                rho[i] = t;
            }
            orc_tridiag_shift_solve(n, dT, eT, theta[j], rho, yv);
            for (int c = 0; c < k; ++c) {
                double t = 0.0;
                for (int i = 0; i < n; ++i) t += Z[IDX(i, c, n)] * yv[i];
                cz[c] = t;
            }
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) {
                double t = yv[i];
                for (int c = 0; c < k; ++c) t -= Z[IDX(i, c, n)] * cz[c];
                Y[IDX(i, j, n)] = t;
                nrm += t * t;
            }
            stp[j] = sqrt(nrm);
            free(rho); free(yv); free(cz);
        }
        double worst = 0.0;
        for (int l = 0; l < k; ++l) {
            if (step) step[l] = stp[l];
            if (l < kw) {
                const double w = weight ? weight[l] : 1.0;
                if (w * stp[l] > worst) worst = w * stp[l];
            }
        }
        if (sweep == max_sweeps - 1) { status = 3; break; }
        /* take this last step, then one closing sweep, when it is within tol or */
        /* when the contraction measured from the previous step predicts what it */
        /* leaves within tol (with a safety factor of 10)                        */
        if (worst <= tol) finishing = 1;
        if (prev_worst > 0.0) {
            double rate = worst / prev_worst;
            if (rate > 1.0) rate = 1.0;
            if (10.0 * rate * worst <= tol) finishing = 1;
        }
        prev_worst = worst;
        /* X_l += Qp y_l for the steps inside the linear region */
#pragma omp parallel for schedule(static)
        for (int r = 0; r < n; ++r)
            for (int j = 0; j < k; ++j) {
                if (!(stp[j] <= 0.5)) continue;
                double t = 0.0;
                for (int c = 0; c < n; ++c) t += Qp[IDX(r, c, ldq)] * Y[IDX(c, j, n)];
                X[IDX(r, j, ldx)] += t;
            }
    }
    free(G); free(I); free(Wq); free(Xs); free(R); free(Y); free(stp); free(Z);
    return status;
}

/* ========================================================================= */
/* Complex Hermitian path (the complex eigensolver interface of Sec. 4.3,    */
/* the k-point problems of periodic systems): the same steps in complex      */
/* arithmetic.  Complex matrices are column-major arrays of double complex   */
/* (real and imaginary parts interleaved); the lower triangle of the         */
/* Hermitian inputs is the one that is read.  Eq. (9) becomes                */
/* D_ij = sum_l f_l c_il conj(c_jl), so that D is Hermitian.                 */
/* ========================================================================= */
#include <complex.h>
typedef double complex zc;

/* Cholesky S = L L^H, column by column.  Returns 0 or j+1 (pivot j not       */
/* positive).  The strict upper triangle is set to zero.                     */
int orc_zpotrf(int n, zc *A, int lda)
{
    for (int j = 0; j < n; ++j) {
        double s = creal(A[IDX(j, j, lda)]);
        for (int k = 0; k < j; ++k) {
            zc l = A[IDX(j, k, lda)];
            s -= creal(l) * creal(l) + cimag(l) * cimag(l);
        }
        if (!(s > 0.0) || !isfinite(s)) return j + 1;
        double ljj = sqrt(s);
        A[IDX(j, j, lda)] = ljj;
        /* L_ij = (S_ij - sum_k L_ik conj(L_jk)) / L_jj for i > j */
#pragma omp parallel for schedule(static)
        for (int i = j + 1; i < n; ++i) {
            zc t = A[IDX(i, j, lda)];
            for (int k = 0; k < j; ++k) t -= A[IDX(i, k, lda)] * conj(A[IDX(j, k, lda)]);
            A[IDX(i, j, lda)] = t / ljj;
        }
    }
    for (int j = 1; j < n; ++j)
        for (int i = 0; i < j; ++i) A[IDX(i, j, lda)] = 0.0;
    return 0;
}

/* x <- L^-1 x (forward substitution, lower triangle of L). */
static void zfwd_subst(int n, const zc *L, int ldl, zc *x)
{
    for (int k = 0; k < n; ++k) {
        x[k] /= L[IDX(k, k, ldl)];
        zc xk = x[k];
        const zc *col = L + IDX(0, k, ldl);
        for (int i = k + 1; i < n; ++i) x[i] -= col[i] * xk;
    }
}

/* x <- L^-H x (back substitution with the conjugate transpose of L). */
static void zback_subst_h(int n, const zc *L, int ldl, zc *x)
{
    for (int i = n - 1; i >= 0; --i) {
        const zc *col = L + IDX(0, i, ldl);
        zc t = x[i];
        for (int j = i + 1; j < n; ++j) t -= conj(col[j]) * x[j];
        x[i] = t / creal(col[i]);
    }
}

/* Eq. (11) for the Hermitian pencil: W = L^-1 H column by column; then       */
/* H~ = W L^-H = L^-1 W^H (H~ Hermitian), whose column j is L^-1 applied to   */
/* the conjugated row j of W; finally H~ <- (H~ + H~^H) / 2.                 */
void orc_zreduce(int n, zc *H, int ldh, const zc *L, int ldl)
{
    zc *W = (zc *)malloc(sizeof(zc) * (size_t)n * n);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        zc *w = W + (size_t)j * n;
        for (int i = 0; i < n; ++i) w[i] = (i >= j) ? H[IDX(i, j, ldh)] : conj(H[IDX(j, i, ldh)]);
        zfwd_subst(n, L, ldl, w);
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        zc *x = (zc *)malloc(sizeof(zc) * n);
        for (int i = 0; i < n; ++i) x[i] = conj(W[(size_t)i * n + j]);
        zfwd_subst(n, L, ldl, x);
        for (int i = 0; i < n; ++i) H[IDX(i, j, ldh)] = x[i];
        free(x);
    }
    free(W);
    for (int j = 0; j < n; ++j) {
        H[IDX(j, j, ldh)] = creal(H[IDX(j, j, ldh)]);
        for (int i = j + 1; i < n; ++i) {
            zc a = 0.5 * (H[IDX(i, j, ldh)] + conj(H[IDX(j, i, ldh)]));
            H[IDX(i, j, ldh)] = a;
            H[IDX(j, i, ldh)] = conj(a);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Hermitian Householder tridiagonalization, Eq. (12) in complex arithmetic: */
/* A = Q T Q^H with T Hermitian tridiagonal, then T = P T_r P^H with the     */
/* diagonal unitary P (p_0 = 1, p_{k+1} = p_k e_k / |e_k|) so that T_r is    */
/* real symmetric with off-diagonal |e_k|.  On exit d (n), e (n-1) hold T_r  */
/* and Q (n x n) is replaced by Q P.  Step k: alpha = -e^{i arg x_0} ||x||   */
/* for x = A(k+1:n, k), v = (x - alpha e_1) / (x_0 - alpha), beta = 2 /      */
/* v^H v, p = beta A22 v, w = p - (beta (v^H p) / 2) v (v^H p is real) and   */
/* A22 <- A22 - v w^H - w v^H.  A (both triangles) is destroyed.             */
/* ------------------------------------------------------------------------- */
void orc_ztred(int n, zc *A, int lda, double *d, double *e, zc *Q, int ldq)
{
    double *beta = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    zc *p = (zc *)malloc(sizeof(zc) * (size_t)(n > 0 ? n : 1));
    zc *ec = (zc *)calloc((size_t)(n > 0 ? n : 1), sizeof(zc));
    for (int k = 0; k + 2 < n; ++k) {
        int m = n - k - 1;
        zc *x = A + IDX(k + 1, k, lda);
        double tail = 0.0;
        for (int i = 1; i < m; ++i) tail += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
        zc x0 = x[0];
        if (tail == 0.0) {   /* already reduced: H_k = I */
            beta[k] = 0.0;
            ec[k] = x0;
            for (int i = 1; i < m; ++i) x[i] = 0.0;
            continue;
        }
        double ax0 = cabs(x0);
        double nrm = sqrt(ax0 * ax0 + tail);
        zc ph = (ax0 > 0.0) ? x0 / ax0 : 1.0;
        zc alpha = -ph * nrm;
        zc v0 = x0 - alpha;
        for (int i = 1; i < m; ++i) x[i] /= v0;
        x[0] = 1.0;
        double av0 = cabs(v0);
        double vhv = 1.0 + tail / (av0 * av0);
        double b = 2.0 / vhv;
        beta[k] = b;
        ec[k] = alpha;
        zc *A22 = A + IDX(k + 1, k + 1, lda);
        /* p = beta A22 v: row j of A22 is conj of column j (Hermitian) */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < m; ++j) {
            const zc *col = A22 + (size_t)j * lda;
            zc t = 0.0;
            for (int i = 0; i < m; ++i) t += conj(col[i]) * x[i];
            p[j] = b * t;
        }
        zc vhp = 0.0;
        for (int i = 0; i < m; ++i) vhp += conj(x[i]) * p[i];
        double half = 0.5 * b * creal(vhp);
        for (int i = 0; i < m; ++i) p[i] -= half * x[i];   /* p is now w */
        /* A22 <- A22 - v w^H - w v^H */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < m; ++j) {
            zc *col = A22 + (size_t)j * lda;
            zc vj = conj(x[j]), wj = conj(p[j]);
            for (int i = 0; i < m; ++i) col[i] -= x[i] * wj + p[i] * vj;
        }
    }
    for (int i = 0; i < n; ++i) d[i] = creal(A[IDX(i, i, lda)]);
    if (n >= 2) ec[n - 2] = A[IDX(n - 1, n - 2, lda)];

    /* Q = H_0 H_1 ... H_{n-3} (H_k = I - beta_k v_k v_k^H), backward accumulation */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) Q[IDX(i, j, ldq)] = (i == j) ? 1.0 : 0.0;
    for (int k = n - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        int m = n - k - 1;
        const zc *v = A + IDX(k + 1, k, lda);
        double b = beta[k];
#pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {
            zc *col = Q + IDX(k + 1, j, ldq);
            zc t = 0.0;
            for (int i = 0; i < m; ++i) t += conj(v[i]) * col[i];
            t *= b;
            for (int i = 0; i < m; ++i) col[i] -= t * v[i];
        }
    }
    /* the diagonal unitary P: T(k+1, k) = e_k = p_{k+1} |e_k| conj(p_k) */
    zc pk = 1.0;
    for (int k = 0; k < n; ++k) {
        if (k > 0) {
            double a = cabs(ec[k - 1]);
            if (a > 0.0) pk = pk * (ec[k - 1] / a);
            e[k - 1] = a;
        }
        zc *col = Q + IDX(0, k, ldq);
        for (int i = 0; i < n; ++i) col[i] *= pk;
    }
    free(beta);
    free(p);
    free(ec);
}

/* Phase convention: the largest-magnitude entry of each column is real > 0. */
static void znormalize_phase(int n, int k, zc *C, int ldc)
{
    for (int j = 0; j < k; ++j) {
        zc *c = C + (size_t)j * ldc;
        int imax = 0;
        for (int i = 1; i < n; ++i) if (cabs(c[i]) > cabs(c[imax])) imax = i;
        double a = cabs(c[imax]);
        if (a == 0.0) continue;
        zc ph = conj(c[imax]) / a;
        for (int i = 0; i < n; ++i) c[i] *= ph;
        c[imax] = a;
    }
}

/* Complex generalized eigensolve: eval (n, ascending), evec n x n_state     */
/* (complex, ldc = n).  H and S are destroyed (S -> L).  Returns as orc_gevp. */
int orc_zgevp(int n, int n_state, zc *H, int ldh, zc *S, int lds, double *eval, zc *evec, int *fail_col)
{
    if (fail_col) *fail_col = 0;
    int info = orc_zpotrf(n, S, lds);
    if (info) { if (fail_col) *fail_col = info; return 1; }
    orc_zreduce(n, H, ldh, S, lds);
    double *d = (double *)malloc(sizeof(double) * n);
    double *e = (double *)calloc((size_t)n, sizeof(double));
    zc *Q = (zc *)malloc(sizeof(zc) * (size_t)n * n);
    orc_ztred(n, H, ldh, d, e, Q, n);
    /* eigenvectors Z of the real tridiagonal (row-major for the QL sweeps) */
    double *Zr = (double *)malloc(sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Zr[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    int st = orc_tql(n, d, e, Zr, 1);
    if (st) { free(d); free(e); free(Q); free(Zr); return st; }
    int *perm = (int *)malloc(sizeof(int) * n);
    stable_argsort(n, d, perm);
    for (int j = 0; j < n; ++j) eval[j] = d[perm[j]];
    /* evec = (Q P) Z for the wanted columns, then L^-H */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n_state; ++j) {
        zc *c = evec + (size_t)j * n;
        for (int i = 0; i < n; ++i) c[i] = 0.0;
        for (int k = 0; k < n; ++k) {
            double z = Zr[(size_t)k * n + perm[j]];
            const zc *q = Q + (size_t)k * n;
            for (int i = 0; i < n; ++i) c[i] += q[i] * z;
        }
        zback_subst_h(n, S, lds, c);
    }
    znormalize_phase(n, n_state, evec, n);
    free(perm); free(d); free(e); free(Q); free(Zr);
    return 0;
}

/* Eq. (9) for complex coefficients: D_ij = sum_{l: f_l > 0} f_l c_il conj(c_jl). */
void orc_zdensity(int n, int k, const zc *C, int ldc, const double *f, zc *D, int ldd)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        zc *dcol = D + (size_t)j * ldd;
        for (int i = 0; i < n; ++i) dcol[i] = 0.0;
        for (int l = 0; l < k; ++l) {
            if (f[l] == 0.0) continue;
            const zc *c = C + (size_t)l * ldc;
            zc w = f[l] * conj(c[j]);
            for (int i = 0; i < n; ++i) dcol[i] += c[i] * w;
        }
    }
}

/* Complex density-matrix driver (returns as orc_dm). */
int orc_zdm(int n, zc *H, int ldh, zc *S, int lds, double n_electron, double kT, double spin,
            double occ_accuracy, int max_steps, zc *D, int ldd, double *eval, double *occ,
            double *energy, double *mu, int *fail_col)
{
    zc *C = (zc *)malloc(sizeof(zc) * (size_t)n * n);
    int st = orc_zgevp(n, n, H, ldh, S, lds, eval, C, fail_col);
    if (st) { free(C); return st; }
    st = orc_occupations(n, eval, n_electron, kT, spin, occ_accuracy, max_steps, occ, mu);
    orc_zdensity(n, n, C, n, occ, D, ldd);
    *energy = orc_band_energy(n, occ, eval);
    free(C);
    return st;
}
