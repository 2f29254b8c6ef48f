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
 *   - FP64 refinement sweeps (CholeskyQR twice, Rayleigh-Ritz, residual
 *     norms) of an approximate invariant subspace of H~, the last stage of
 *     the GPU library's mixed-precision mode (orc_refine);
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
/* Fermi-Dirac occupations, Eq. (17), written so that no exponential         */
/* overflows:  x = (eps - mu) / kT;  f = spin * e^-x / (1 + e^-x), x >= 0;   */
/*                                   f = spin / (1 + e^x),          x <  0.  */
/* ------------------------------------------------------------------------- */
static double fermi(double eps, double mu, double kT, double spin)
{
    double x = (eps - mu) / kT;
    if (x >= 0.0) { double t = exp(-x); return spin * t / (1.0 + t); }
    return spin / (1.0 + exp(x));
}

static double electron_count(int n, const double *eps, double mu, double kT, double spin)
{
    double s = 0.0;
    for (int l = 0; l < n; ++l) s += fermi(eps[l], mu, kT, spin);
    return s;
}

/* ------------------------------------------------------------------------- */
/* Chemical potential by bisection on  sum_l f_l(mu) - N_e, Eq. (18)         */
/* (Sec. 4.5): interval [eps_min - 10 kT, eps_max + 10 kT], widened (the     */
/* step doubling each time) until it brackets the root; halved until the     */
/* electron count is within occ_accuracy, the interval cannot shrink any     */
/* further in floating point, or max_steps halvings were made.  mu is the    */
/* upper bound (surplus >= 0), and the surplus is then removed from the      */
/* highest occupied states downward so that sum f = N_e.                     */
/* eps must be ascending.  Returns 0, or 4 when max_steps ran out first.     */
/* ------------------------------------------------------------------------- */
int orc_occupations(int n, const double *eps, double n_electron, double kT, double spin,
                    double occ_accuracy, int max_steps, double *f, double *mu_out)
{
    double lo = eps[0] - 10.0 * kT, hi = eps[n - 1] + 10.0 * kT;
    double step = hi - lo;
    while (electron_count(n, eps, lo, kT, spin) - n_electron > 0.0) { lo -= step; step *= 2.0; }
    step = hi - lo;
    while (electron_count(n, eps, hi, kT, spin) - n_electron < 0.0) { hi += step; step *= 2.0; }
    /* the upper bound always carries a surplus g(hi) >= 0; stop once it is    */
    /* within occ_accuracy or the midpoint no longer differs from the bounds   */
    int status = 0, steps = 0;
    for (;;) {
        double mid = 0.5 * (lo + hi);
        if (!(lo < mid && mid < hi)) break;
        if (steps >= max_steps) { status = 4; break; }
        ++steps;
        double g = electron_count(n, eps, mid, kT, spin) - n_electron;
        if (g >= 0.0) {
            hi = mid;
            if (g <= occ_accuracy) break;
        } else {
            lo = mid;
        }
    }
    double mu = hi;
    for (int l = 0; l < n; ++l) f[l] = fermi(eps[l], mu, kT, spin);
    double surplus = electron_count(n, eps, mu, kT, spin) - n_electron;
    for (int l = n - 1; l >= 0 && surplus > 0.0; --l) {
        if (f[l] <= 0.0) continue;
        double take = f[l] < surplus ? f[l] : surplus;
        f[l] -= take;
        surplus -= take;
    }
    *mu_out = mu;
    return status;
}

/* ------------------------------------------------------------------------- */
/* Density matrix, Eq. (9):  D_ij = sum_{l: f_l > 0} f_l c_il c_jl.          */
/* C is n x k (column-major, ldc), D is n x n (ldd), both triangles written. */
/* ------------------------------------------------------------------------- */
void orc_density(int n, int k, const double *C, int ldc, const double *f, double *D, int ldd)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double *dcol = D + (size_t)j * ldd;
        for (int i = 0; i < n; ++i) dcol[i] = 0.0;
        for (int l = 0; l < k; ++l) {
            if (!(f[l] > 0.0)) continue;
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
int orc_dm(int n, double *H, int ldh, double *S, int lds, double n_electron, double kT,
           double spin, double occ_accuracy, int max_steps, double *D, int ldd,
           double *eval, double *occ, double *energy, double *mu, int *fail_col)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)n * n);
    int st = orc_gevp(n, n, H, ldh, S, lds, eval, C, fail_col);
    if (st) { free(C); return st; }
    st = orc_occupations(n, eval, n_electron, kT, spin, occ_accuracy, max_steps, occ, mu);
    orc_density(n, n, C, n, occ, D, ldd);
    *energy = orc_band_energy(n, occ, eval);
    free(C);
    return st;
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

/* ========================================================================= */
/* FP64 refinement of an approximate invariant subspace of the standard-form */
/* matrix H~ = L^-1 H L^-T (Eq. (11)): the last stage of the GPU library's   */
/* mixed-precision mode (the paper's solvers run in one precision, so this   */
/* stage has no passage of its own; each step below is the textbook          */
/* definition).  X is n x k (ldx); on return it holds the refined vectors.    */
/* One sweep:                                                                */
/*   CholeskyQR, twice: G = X^T X = L_G L_G^T, X <- X L_G^-T (row by row,     */
/*   forward substitution with L_G);                                         */
/*   Rayleigh-Ritz: A = X^T H~ X, A = Q diag(theta) Q^T (orc_gevp with S = I),*/
/*   X <- X Q;                                                               */
/*   residuals res_l = ||H~ x_l - theta_l x_l||_2, from the definition.      */
/* The first kw states decide: stop with 0 when max res_l <= tol; otherwise  */
/* stop with 3 after that sweep (its Rayleigh-Ritz step leaves the subspace   */
/* unchanged, so a further sweep cannot lower the residual), and with 3 when  */
/* G is not positive definite (dependent columns) or max_sweeps is 0.         */
/* ========================================================================= */
int orc_refine(int n, int k, int kw, const double *Ht, int ldh, double *X, int ldx, double *theta,
               double *res, double tol, int max_sweeps, int *sweeps)
{
    if (sweeps) *sweeps = 0;
    if (n <= 0 || k <= 0) return 0;
    if (kw > k) kw = k;
    double *G = (double *)malloc(sizeof(double) * (size_t)k * k);
    double *I = (double *)malloc(sizeof(double) * (size_t)k * k);
    double *Q = (double *)malloc(sizeof(double) * (size_t)k * k);
    double *Y = (double *)malloc(sizeof(double) * (size_t)n * k);
    int status = 3;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        int bad = 0;
        for (int pass = 0; pass < 2 && !bad; ++pass) {
#pragma omp parallel for schedule(static)
            for (int j = 0; j < k; ++j)
                for (int i = 0; i < k; ++i) {
                    double t = 0.0;
                    for (int r = 0; r < n; ++r) t += X[IDX(r, i, ldx)] * X[IDX(r, j, ldx)];
                    G[IDX(i, j, k)] = t;
                }
            if (orc_potrf(k, G, k)) { bad = 1; break; }
#pragma omp parallel for schedule(static)
            for (int r = 0; r < n; ++r) {
                double *row = (double *)malloc(sizeof(double) * k);
                for (int j = 0; j < k; ++j) row[j] = X[IDX(r, j, ldx)];
                fwd_subst(k, G, k, row);   /* L_G y = x^T  <=>  y^T = x L_G^-T */
                for (int j = 0; j < k; ++j) X[IDX(r, j, ldx)] = row[j];
                free(row);
            }
        }
        if (bad) { status = 3; break; }
        /* A = X^T (H~ X), lower triangle of H~ read */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < n; ++i) {
                double t = 0.0;
                for (int c = 0; c < n; ++c) {
                    const double h = (i >= c) ? Ht[IDX(i, c, ldh)] : Ht[IDX(c, i, ldh)];
                    t += h * X[IDX(c, j, ldx)];
                }
                Y[IDX(i, j, n)] = t;
            }
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i) {
                double t = 0.0;
                for (int r = 0; r < n; ++r) t += X[IDX(r, i, ldx)] * Y[IDX(r, j, n)];
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
        if (orc_gevp(k, k, G, k, I, k, theta, Q, NULL)) { status = 3; break; }
        /* X <- X Q */
#pragma omp parallel for schedule(static)
        for (int r = 0; r < n; ++r) {
            double *row = (double *)malloc(sizeof(double) * k);
            for (int j = 0; j < k; ++j) {
                double t = 0.0;
                for (int c = 0; c < k; ++c) t += X[IDX(r, c, ldx)] * Q[IDX(c, j, k)];
                row[j] = t;
            }
            for (int j = 0; j < k; ++j) X[IDX(r, j, ldx)] = row[j];
            free(row);
        }
        /* res_l = || H~ x_l - theta_l x_l || */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < k; ++j) {
            double acc = 0.0;
            for (int i = 0; i < n; ++i) {
                double t = -theta[j] * X[IDX(i, j, ldx)];
                for (int c = 0; c < n; ++c) {
                    const double h = (i >= c) ? Ht[IDX(i, c, ldh)] : Ht[IDX(c, i, ldh)];
                    t += h * X[IDX(c, j, ldx)];
                }
                acc += t * t;
            }
            res[j] = sqrt(acc);
        }
        if (sweeps) *sweeps = sweep + 1;
        double rmax = 0.0;
        for (int l = 0; l < kw; ++l) if (res[l] > rmax) rmax = res[l];
        status = (rmax <= tol) ? 0 : 3;
        break;
    }
    free(G); free(I); free(Q); free(Y);
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
            if (!(f[l] > 0.0)) continue;
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
