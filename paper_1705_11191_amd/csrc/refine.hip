// FP64 refinement of an approximate invariant subspace of the standard-form
// matrix H~ = L^-1 H L^-T (Eq. (11)), used after the steps of Fig. 1 ran
// with FP32 matrix-core arithmetic.  The paper's solvers work in one
// precision; this stage is this library's addition.  One sweep:
//   (1) orthonormalize X (n x k) by CholeskyQR twice: G = X^T X = R^T R,
//       X <- X R^-1;
//   (2) Rayleigh-Ritz: A = X^T H~ X (k x k), A = Q Theta Q^T by the FP64
//       solver of this library (S = I), X <- X Q;
//   (3) residuals r_l = || H~ x_l - theta_l x_l ||_2, which bound the error of
//       theta_l (the pencil residual H c - theta S c equals L r for c = L^-T x).
// A sweep that leaves the wanted states' largest residual above tol ends the
// refinement (not converged): its Rayleigh-Ritz step does not change the
// subspace, so a further sweep could not lower the residual.
#include "api_internal.h"

#include <algorithm>
#include <vector>

namespace eg {
namespace {

// r_l = || W(:, l) - theta_l X(:, l) ||_2, one workgroup per column with a
// fixed-order tree sum.
__global__ __launch_bounds__(256) void residual_norms_kernel(int n, const double* __restrict__ W, int ldw,
                                                             const double* __restrict__ X, int ldx,
                                                             const double* __restrict__ theta, double* r)
{
    __shared__ double red[256];
    const int l = blockIdx.x;
    const double t = theta[l];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double v = W[cm(i, l, ldw)] - t * X[cm(i, l, ldx)];
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

}  // namespace

size_t refine_scratch_doubles(int n, int k)
{
    (void)n;
    const size_t kk = (size_t)std::max(k, 1);
    return 2 * kk * kk + (size_t)ceil_div(std::max(k, 1), 64) * 4096 + 2 * kk + 64;
}

int refine_subspace(hipStream_t st, int n, int k, int kw, const double* Ht, int ldh, double* const bufs[3], int ldb,
                    double* G, double* Qm, double* Linv, int* dinfo, double* part, size_t npart, double* theta,
                    double* r, double tol, int max_sweeps, RefineOutcome* out)
{
    out->x_buf = 0;
    out->sweeps = 0;
    out->rmax = -1.0;
    out->converged = 0;
    if (n <= 0 || k <= 0) {
        out->converged = 1;
        return 0;
    }
    kw = std::min(std::max(kw, 0), k);
    int xi = 0;
    std::vector<double> hr((size_t)k);
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
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double* X = bufs[xi];
        double* W = bufs[(xi + 1) % 3];
        double* X2 = bufs[(xi + 2) % 3];
        // (1) two CholeskyQR passes; each factorization is checked before X is
        // touched, so that a failure leaves the vectors of the last completed
        // sweep (or the starting ones) in bufs[out->x_buf]
        fill_i(st, dinfo, 1, 0);
        for (int pass = 0; pass < 2; ++pass) {
            dgemm_splitk(st, 'T', 'N', k, k, n, 1.0, X, ldb, X, ldb, 0.0, G, k, part, npart);
            dpotrf(st, k, G, k, Linv, dinfo);
            int hinfo = 0;
            if (hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
                return kStatusHip;
            if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
            if (hinfo) return kStatusRefine;   // the columns of X are numerically dependent
            dtrsm_right_lower_t(st, n, k, G, k, Linv, X, ldb);
        }
        // (2) Rayleigh-Ritz
        dgemm(st, 'N', 'N', n, k, n, 1.0, Ht, ldh, X, ldb, 0.0, W, ldb);
        dgemm_splitk(st, 'T', 'N', k, k, n, 1.0, X, ldb, W, ldb, 0.0, G, k, part, npart);
        symmetrize_average(st, k, G, k);
        {
            const int rc = elsi_gpu_ev(sub.h, G, nullptr, theta, Qm);
            if (rc) return rc > 0 ? rc : kStatusHip;
        }
        dgemm(st, 'N', 'N', n, k, k, 1.0, X, ldb, Qm, k, 0.0, X2, ldb);   // refined vectors
        dgemm(st, 'N', 'N', n, k, k, 1.0, W, ldb, Qm, k, 0.0, X, ldb);    // H~ times them
        // (3) residual norms
        hipLaunchKernelGGL(residual_norms_kernel, dim3(k), dim3(256), 0, st, n, X, ldb, X2, ldb, theta, r);
        xi = (xi + 2) % 3;
        out->sweeps = sweep + 1;
        out->x_buf = xi;
        if (hipMemcpyAsync(hr.data(), r, sizeof(double) * k, hipMemcpyDeviceToHost, st) != hipSuccess)
            return kStatusHip;
        if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
        double rmax = 0.0;
        for (int l = 0; l < kw; ++l) rmax = std::max(rmax, hr[l]);
        out->rmax = rmax;
        out->converged = (rmax <= tol) ? 1 : 0;
        break;
    }
    return 0;
}

}  // namespace eg

using namespace eg;

extern "C" int elsi_gpu_x_refine(int n, int k, int kw, const double* Ht, int ldh, double* X, int ldx,
                                 double* theta, double* resid, double tol, int max_sweeps, int* sweeps,
                                 void* hip_stream)
{
    if (n < 0) return -1;
    if (k < 0 || k > n) return -2;
    if (kw < 0 || kw > k) return -3;
    if ((!Ht && n > 0) || ldh < std::max(1, n)) return -4;
    if ((!X && k > 0) || ldx < std::max(1, n)) return -6;
    if (!theta && k > 0) return -8;
    if (!resid && k > 0) return -9;
    if (!(tol >= 0.0)) return -10;
    if (max_sweeps < 0) return -11;
    if (sweeps) *sweeps = 0;
    if (n == 0 || k == 0) return 0;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t nk = (size_t)n * k;
    const size_t npart = (size_t)8 * n * 64;
    DevBuf<double> b1, b2, scratch, part;
    DevBuf<int> dinfo;
    if (!b1.alloc(nk) || !b2.alloc(nk) || !scratch.alloc(refine_scratch_doubles(n, k)) || !part.alloc(npart) ||
        !dinfo.alloc(1))
        return kStatusOom;
    double* b0 = X;
    DevBuf<double> xcopy;
    if (ldx != n) {   // the sweeps keep their three column blocks at leading dimension n
        if (!xcopy.alloc(nk)) return kStatusOom;
        copy_matrix(st, n, k, X, ldx, xcopy.p, n);
        b0 = xcopy.p;
    }
    double* const bufs[3] = {b0, b1.p, b2.p};
    const size_t kk = (size_t)k * k;
    double* G = scratch.p;
    double* Qm = G + kk;
    double* Linv = Qm + kk;
    double* r = Linv + (size_t)ceil_div(k, 64) * 4096;
    RefineOutcome out{};
    int rc = refine_subspace(st, n, k, kw, Ht, ldh, bufs, n, G, Qm, Linv, dinfo.p, part.p, npart, theta, r, tol,
                             max_sweeps, &out);
    if (rc && rc != kStatusRefine) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    const bool dependent = (rc == kStatusRefine);
    if (out.sweeps > 0) {
        copy_matrix(st, n, k, bufs[out.x_buf], n, X, ldx);
        (void)hipMemcpyAsync(resid, r, sizeof(double) * k, hipMemcpyDeviceToDevice, st);
    }
    if (sweeps) *sweeps = out.sweeps;
    rc = sync_status(st);
    if (rc) return rc;
    return (out.converged && !dependent) ? 0 : kStatusRefine;
}
