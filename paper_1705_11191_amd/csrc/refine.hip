// FP64 refinement of an approximate invariant subspace of the standard-form
// matrix H~ = L^-1 H L^-T (Eq. (11)), used after the steps of Fig. 1 ran
// with FP32 matrix-core arithmetic.  The paper's solvers work in one
// precision; this stage is this library's addition.  One sweep:
//   (1) orthonormalize X (n x k) by CholeskyQR (twice in the first sweep,
//       once after a correction): G = X^T X = R^T R, X <- X R^-1;
//   (2) Rayleigh-Ritz: A = X^T H~ X (k x k), A = W Theta W^T by the FP64
//       solver of this library (S = I), X <- X W;
//   (3) residuals r_l = H~ x_l - theta_l x_l (the pencil residual
//       H c - theta S c equals L r for c = L^-T x), with their norms.
// Rayleigh-Ritz alone never moves span(X); what moves it is
//   (4) the Newton correction through the approximate factorization
//       H~ ~ Q T Q^T that the reduced-precision steps produced (Q = Q1 Q2,
//       T tridiagonal): with Z the eigenvectors of T for its k lowest
//       eigenvalues and P = I - Z Z^T,
//           y_l = -P (T - theta_l)^-1 P Q^T r_l,    step_l = ||y_l||_2,
//       which solves the correction equation (H~ - theta_l) d_l = -r_l on the
//       complement of the subspace with T standing in for Q^T H~ Q.  The
//       per-column shifted solves run by Gaussian elimination with partial
//       pivoting, one lane per column.
// After each sweep x_l += Q y_l (for steps <= 1/2, inside the region where
// the linear model holds) and the next sweep starts.  Once the largest
// weighted step W_s over the wanted states is <= tol, or the contraction
// measured over the last two steps predicts that taking it leaves less than
// tol (10 (W_s / W_{s-1}) W_s <= tol), that step is still taken and one
// closing sweep of steps (1)-(3) ends the call converged: the step left
// untaken would be amplified by L^-T in the pencil's eigenvectors.
#include "api_internal.h"

#include <algorithm>
#include <cfloat>
#include <vector>

namespace eg {
namespace {

constexpr double kStepCap = 0.5;   // larger steps are measured but not taken

// W(:, l) <- W(:, l) - theta_l X(:, l) and r_l = its 2-norm; one workgroup per
// column with a fixed-order tree sum.
__global__ __launch_bounds__(256) void residual_kernel(int n, double* __restrict__ W, int ldw,
                                                       const double* __restrict__ X, int ldx,
                                                       const double* __restrict__ theta, double* r)
{
    __shared__ double red[256];
    const int l = blockIdx.x;
    const double t = theta[l];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double v = W[cm(i, l, ldw)] - t * X[cm(i, l, ldx)];
        W[cm(i, l, ldw)] = v;
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) r[l] = sqrt(red[0]);
}

// out_l = ||Y(:, l)||_2, one workgroup per column.
__global__ __launch_bounds__(256) void column_norms_kernel(int n, const double* __restrict__ Y, int ldy,
                                                           double* out)
{
    __shared__ double red[256];
    const int l = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double v = Y[cm(i, l, ldy)];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[l] = sqrt(red[0]);
}

// Y(:, l) <- (T - theta_l I)^-1 (-Y(:, l)), T = tridiag(e, d, e), for l < k:
// Gaussian elimination with partial pivoting (the row with the larger entry
// in the pivot column leads, the current row on a tie; an exactly zero pivot
// becomes DBL_EPSILON times the largest row sum of |T - theta_l I|).  One
// lane per column; the factors U0, U1 (the pivot row's first two entries;
// its third is e[r + 1] after a row exchange, else 0) and the exchange flags
// are stored row by row with the columns adjacent (row r at r * k).
__global__ __launch_bounds__(64) void tri_shift_solve_kernel(int n, int k, const double* __restrict__ d,
                                                             const double* __restrict__ e,
                                                             const double* __restrict__ theta, double* Y, int ldy,
                                                             double* __restrict__ U0, double* __restrict__ U1,
                                                             unsigned char* __restrict__ SW)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= k) return;
    const double s = theta[j];
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = fabs(d[i] - s);
        if (i > 0) r += fabs(e[i - 1]);
        if (i + 1 < n) r += fabs(e[i]);
        tnorm = fmax(tnorm, r);
    }
    double tiny = DBL_EPSILON * tnorm;
    if (tiny == 0.0) tiny = DBL_MIN;
    double* y = Y + (size_t)j * ldy;
    double p = d[0] - s;                      // current row: (p, q) in columns r, r+1
    double q = (n > 1) ? e[0] : 0.0;
    double yr = -y[0];                        // right-hand side of the current row
    for (int r = 0; r + 1 < n; ++r) {
        const double a = e[r];                // row r+1: (a, bb, c) in columns r, r+1, r+2
        const double bb = d[r + 1] - s;
        const double c = (r + 2 < n) ? e[r + 1] : 0.0;
        const double yn = -y[r + 1];
        const size_t o = (size_t)r * k + j;
        if (fabs(p) >= fabs(a)) {
            if (p == 0.0) p = tiny;
            const double m = a / p;
            U0[o] = p;
            U1[o] = q;
            SW[o] = 0;
            y[r] = yr;
            yr = yn - m * yr;
            p = bb - m * q;
            q = c;
        } else {
            const double m = p / a;
            U0[o] = a;
            U1[o] = bb;
            SW[o] = 1;
            y[r] = yn;
            yr = yr - m * yn;
            const double pn = q - m * bb;
            q = -m * c;
            p = pn;
        }
    }
    if (p == 0.0) p = tiny;
    double x1 = yr / p;   // x[r + 1]
    double x2 = 0.0;      // x[r + 2]
    y[n - 1] = x1;
    for (int r = n - 2; r >= 0; --r) {
        const size_t o = (size_t)r * k + j;
        const double u2 = (SW[o] && r + 2 < n) ? e[r + 1] : 0.0;
        double t = y[r];
        t -= U1[o] * x1;
        t -= u2 * x2;
        const double x = t / U0[o];
        y[r] = x;
        x2 = x1;
        x1 = x;
    }
}

// X(:, l) += Y(:, l) for the columns whose step is <= cap.
__global__ __launch_bounds__(256) void masked_add_kernel(int n, double* __restrict__ X, int ldx,
                                                         const double* __restrict__ Y, int ldy,
                                                         const double* __restrict__ step, double cap)
{
    const int l = blockIdx.y;
    if (!(step[l] <= cap)) return;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        X[cm(i, l, ldx)] += Y[cm(i, l, ldy)];
}

// Y <- P Y with P = I - Z Z^T (Z n x k orthonormal), G: k x k scratch.
void project_out(hipStream_t st, int n, int k, const double* Z, int ldz, double* Y, int ldy, double* G,
                 double* part, size_t npart)
{
    dgemm_splitk(st, 'T', 'N', k, k, n, 1.0, Z, ldz, Y, ldy, 0.0, G, k, part, npart);
    dgemm(st, 'N', 'N', n, k, k, -1.0, Z, ldz, G, k, 1.0, Y, ldy);
}

}  // namespace

size_t refine_scratch_doubles(int n, int k)
{
    (void)n;
    const size_t kk = (size_t)std::max(k, 1);
    return 2 * kk * kk + (size_t)ceil_div(std::max(k, 1), 64) * 4096 + 3 * kk + 64;
}

int refine_subspace(hipStream_t st, int n, int k, int kw, const double* Ht, int ldh, const RefineBuffers& B,
                    RefinePrecond* pc, const double* weight, double tol, int max_sweeps, RefineOutcome* out)
{
    out->x_buf = 0;
    out->sweeps = 0;
    out->rmax = -1.0;
    out->smax = -1.0;
    out->converged = 0;
    if (n <= 0 || k <= 0) {
        out->converged = 1;
        return 0;
    }
    kw = std::min(std::max(kw, 0), k);
    const int ldb = B.ldb;
    int xi = 0;
    std::vector<double> hr((size_t)k), hs((size_t)k), hw((size_t)k, 1.0);
    if (weight && kw > 0) {
        if (hipMemcpyAsync(hw.data(), weight, sizeof(double) * k, hipMemcpyDeviceToHost, st) != hipSuccess)
            return kStatusHip;
        if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
    }
    if (pc) fill_d(st, B.step, (size_t)k, 0.0);
    // the k x k eigensolver of the Rayleigh-Ritz step (S = I), kept for all sweeps
    struct SubSolver {
        elsi_gpu_handle h = nullptr;
        ~SubSolver() { if (h) elsi_gpu_finalize(&h); }
    } sub;
    if (max_sweeps > 0) {
        int rc = elsi_gpu_init(&sub.h, ELSI_GPU_REAL64, k, k, 0.0, st);
        if (!rc) rc = elsi_gpu_set_overlap_is_unit(sub.h, 1);
        if (rc) return rc > 0 ? rc : kStatusHip;
    }
    bool finishing = false;
    double prev_smax = 0.0;
    for (int l = 0; l < (int)(sizeof(out->hist) / sizeof(out->hist[0])); ++l) out->hist[l] = 0.0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double* X = B.X[xi];
        double* W = B.X[(xi + 1) % 3];
        double* X2 = B.X[(xi + 2) % 3];
        // (1) CholeskyQR: twice for the starting vectors, once after a
        // correction (which leaves them orthonormal to O(step)); each
        // factorization is checked before X is touched, so that a failure
        // leaves the vectors of the last completed sweep (or the starting
        // ones) in B.X[out->x_buf]
        fill_i(st, B.dinfo, 1, 0);
        const int passes = (sweep == 0) ? 2 : 1;
        for (int pass = 0; pass < passes; ++pass) {
            dgemm_splitk(st, 'T', 'N', k, k, n, 1.0, X, ldb, X, ldb, 0.0, B.G, k, B.part, B.npart);
            dpotrf(st, k, B.G, k, B.Linv, B.dinfo);
            int hinfo = 0;
            if (hipMemcpyAsync(&hinfo, B.dinfo, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
                return kStatusHip;
            if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
            if (hinfo) return kStatusRefine;   // the columns of X are numerically dependent
            dtrsm_right_lower_t(st, n, k, B.G, k, B.Linv, X, ldb);
        }
        // (2) Rayleigh-Ritz
        dgemm(st, 'N', 'N', n, k, n, 1.0, Ht, ldh, X, ldb, 0.0, W, ldb);
        dgemm_splitk(st, 'T', 'N', k, k, n, 1.0, X, ldb, W, ldb, 0.0, B.G, k, B.part, B.npart);
        symmetrize_average(st, k, B.G, k);
        {
            const int rc = elsi_gpu_ev(sub.h, B.G, nullptr, B.theta, B.Qm);
            if (rc) return rc > 0 ? rc : kStatusHip;
        }
        dgemm(st, 'N', 'N', n, k, k, 1.0, X, ldb, B.Qm, k, 0.0, X2, ldb);   // refined vectors
        dgemm(st, 'N', 'N', n, k, k, 1.0, W, ldb, B.Qm, k, 0.0, X, ldb);    // H~ times them
        // (3) residuals, in the buffer that held the start of the sweep
        hipLaunchKernelGGL(residual_kernel, dim3(k), dim3(256), 0, st, n, X, ldb, X2, ldb, B.theta, B.r);
        double* R = X;
        double* tmp = W;
        xi = (xi + 2) % 3;
        out->sweeps = sweep + 1;
        out->x_buf = xi;
        if (hipMemcpyAsync(hr.data(), B.r, sizeof(double) * k, hipMemcpyDeviceToHost, st) != hipSuccess)
            return kStatusHip;
        if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
        double rmax = 0.0;
        for (int l = 0; l < kw; ++l) rmax = std::max(rmax, hr[l]);
        out->rmax = rmax;
        if (finishing) {   // the closing sweep after a step within tol
            out->converged = 1;
            break;
        }
        if (!pc) {   // Rayleigh-Ritz alone: one sweep decides
            out->converged = (rmax <= tol) ? 1 : 0;
            break;
        }
        // (4) Newton correction in the basis of T.  P commutes with (T - theta)^-1
        // (Z holds eigenvectors of T), so one projection after the solves gives
        // P (T - theta)^-1 P rho; the rounding a solve adds along an eigenvector
        // of T whose eigenvalue is near theta is removed by that projection
        pc->apply_qt(st, R, ldb, k, tmp);
        hipLaunchKernelGGL(tri_shift_solve_kernel, dim3(ceil_div(k, 64)), dim3(64), 0, st, n, k, pc->d, pc->e,
                           B.theta, R, ldb, tmp, B.U1, B.SW);
        project_out(st, n, k, pc->Z, pc->ldz, R, ldb, B.G, B.part, B.npart);
        hipLaunchKernelGGL(column_norms_kernel, dim3(k), dim3(256), 0, st, n, R, ldb, B.step);
        if (hipMemcpyAsync(hs.data(), B.step, sizeof(double) * k, hipMemcpyDeviceToHost, st) != hipSuccess)
            return kStatusHip;
        if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
        double smax = 0.0;
        for (int l = 0; l < kw; ++l) smax = std::max(smax, hw[l] * hs[l]);
        out->smax = smax;
        if (sweep < (int)(sizeof(out->hist) / sizeof(out->hist[0]))) out->hist[sweep] = smax;
        if (sweep == max_sweeps - 1) break;
        // a step within tol is still taken, and one closing Rayleigh-Ritz
        // sweep follows: left untaken, it would be amplified by L^-T in the
        // pencil's eigenvectors.  The same holds when the contraction measured
        // over the last two steps predicts that taking this one leaves less
        // than tol (safety factor 10).
        if (smax <= tol) finishing = true;
        if (prev_smax > 0.0 && 10.0 * std::min(1.0, smax / prev_smax) * smax <= tol) finishing = true;
        prev_smax = smax;
        pc->apply_q(st, R, ldb, k, tmp);
        masked_add_kernel<<<dim3(std::max(1, std::min(ceil_div(n, 256), 64)), k), dim3(256), 0, st>>>(
            n, B.X[xi], ldb, R, ldb, B.step, kStepCap);
    }
    return 0;
}

}  // namespace eg

using namespace eg;

namespace {

// The factorization of the stage entry point: Q given as a dense n x n matrix.
struct DensePrecond : RefinePrecond {
    const double* Q = nullptr;
    int ldq = 0, n = 0;
    void apply_qt(hipStream_t st, double* X, int ld, int ncol, double* tmp) override
    {
        dgemm(st, 'T', 'N', n, ncol, n, 1.0, Q, ldq, X, ld, 0.0, tmp, ld);
        copy_matrix(st, n, ncol, tmp, ld, X, ld);
    }
    void apply_q(hipStream_t st, double* X, int ld, int ncol, double* tmp) override
    {
        dgemm(st, 'N', 'N', n, ncol, n, 1.0, Q, ldq, X, ld, 0.0, tmp, ld);
        copy_matrix(st, n, ncol, tmp, ld, X, ld);
    }
};

}  // namespace

extern "C" int elsi_gpu_x_refine(int n, int k, int kw, const double* Ht, int ldh, double* X, int ldx,
                                 const double* Q, int ldq, const double* d, const double* e, const double* weight,
                                 double* theta, double* resid, double* step, double tol, int max_sweeps,
                                 int* sweeps, void* hip_stream)
{
    if (n < 0) return -1;
    if (k < 0 || k > n) return -2;
    if (kw < 0 || kw > k) return -3;
    if ((!Ht && n > 0) || ldh < std::max(1, n)) return -4;
    if ((!X && k > 0) || ldx < std::max(1, n)) return -6;
    if (Q && ldq < std::max(1, n)) return -9;
    if (Q && !d) return -10;
    if (Q && !e && n > 1) return -11;
    if (!theta && k > 0) return -13;
    if (!resid && k > 0) return -14;
    if (!(tol >= 0.0)) return -16;
    if (max_sweeps < 0) return -17;
    if (sweeps) *sweeps = 0;
    if (n == 0 || k == 0) return 0;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t nk = (size_t)n * k;
    const size_t npart = (size_t)8 * n * 64;
    const size_t kk = (size_t)k * k;
    DevBuf<double> b1, b2, scratch, part, u1, zall, z2, zu, dd, ee;
    DevBuf<unsigned char> sw;
    DevBuf<char> dcwork;
    DevBuf<int> dinfo;
    if (!b1.alloc(nk) || !b2.alloc(nk) || !scratch.alloc(refine_scratch_doubles(n, k)) || !part.alloc(npart) ||
        !dinfo.alloc(4))
        return kStatusOom;
    double* b0 = X;
    DevBuf<double> xcopy;
    if (ldx != n) {   // the sweeps keep their three column blocks at leading dimension n
        if (!xcopy.alloc(nk)) return kStatusOom;
        copy_matrix(st, n, k, X, ldx, xcopy.p, n);
        b0 = xcopy.p;
    }
    RefineBuffers B{};
    B.X[0] = b0;
    B.X[1] = b1.p;
    B.X[2] = b2.p;
    B.ldb = n;
    B.G = scratch.p;
    B.Qm = B.G + kk;
    B.Linv = B.Qm + kk;
    double* sc = B.Linv + (size_t)ceil_div(k, 64) * 4096;
    B.r = sc;
    B.step = sc + k;
    B.theta = theta;
    B.dinfo = dinfo.p;
    B.part = part.p;
    B.npart = npart;
    DensePrecond pc;
    if (Q) {
        // Z: the eigenvectors of T for its k lowest eigenvalues (divide and conquer)
        if (!u1.alloc(nk) || !sw.alloc(nk) || !zall.alloc((size_t)n * n) || !z2.alloc((size_t)n * n) ||
            !zu.alloc((size_t)n * n) || !dd.alloc(n) || !ee.alloc(n) || !dcwork.alloc(stedc_workspace_bytes(n)))
            return kStatusOom;
        (void)hipMemcpyAsync(dd.p, d, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
        fill_d(st, ee.p, (size_t)n, 0.0);
        if (n > 1) (void)hipMemcpyAsync(ee.p, e, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, st);
        DevBuf<double> wall;
        if (!wall.alloc(n)) return kStatusOom;
        int rc = stedc(st, n, dd.p, ee.p, wall.p, zall.p, z2.p, zu.p, n, k, dcwork.p, dinfo.p + 1, nullptr);
        if (rc) return rc;
        int herr = 0;
        (void)hipMemcpyAsync(&herr, dinfo.p + 1, sizeof(int), hipMemcpyDeviceToHost, st);
        rc = sync_status(st);
        if (rc) return rc;
        if (herr) return ELSI_GPU_ERR_NO_CONV;
        pc.Q = Q;
        pc.ldq = ldq;
        pc.n = n;
        pc.Z = zall.p;
        pc.ldz = n;
        pc.d = dd.p;
        pc.e = ee.p;
        B.U1 = u1.p;
        B.SW = sw.p;
    }
    RefineOutcome out{};
    int rc = refine_subspace(st, n, k, kw, Ht, ldh, B, Q ? &pc : nullptr, weight, tol, max_sweeps, &out);
    if (rc && rc != kStatusRefine) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    const bool dependent = (rc == kStatusRefine);
    if (out.sweeps > 0) {
        copy_matrix(st, n, k, B.X[out.x_buf], n, X, ldx);
        (void)hipMemcpyAsync(resid, B.r, sizeof(double) * k, hipMemcpyDeviceToDevice, st);
        if (step) {
            if (Q)
                (void)hipMemcpyAsync(step, B.step, sizeof(double) * k, hipMemcpyDeviceToDevice, st);
            else
                fill_d(st, step, (size_t)k, 0.0);
        }
    }
    if (sweeps) *sweeps = out.sweeps;
    rc = sync_status(st);
    if (rc) return rc;
    return (out.converged && !dependent) ? 0 : kStatusRefine;
}
