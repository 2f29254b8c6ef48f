// C ABI of libelsi_gpu: handle management, argument checking, workspace and
// the stage entry points.  The solver drivers elsi_gpu_ev / elsi_gpu_dm live
// in solver.hip.
#include "api_internal.h"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

using namespace eg;

extern "C" {

const char* elsi_gpu_strerror(int status)
{
    if (status == 0) return "success";
    if (status < 0) return "invalid argument";
    switch (status) {
        case ELSI_GPU_ERR_NOT_PD: return "overlap matrix is not positive definite";
        case ELSI_GPU_ERR_NO_CONV: return "tridiagonal eigensolver did not converge";
        case ELSI_GPU_ERR_REFINE: return "refinement tolerance not reached";
        case ELSI_GPU_ERR_MU: return "chemical potential bisection ran out of steps";
        case ELSI_GPU_ERR_HIP: return "HIP runtime error";
        case ELSI_GPU_ERR_OOM: return "out of device memory";
        case ELSI_GPU_ERR_NONFINITE: return "input holds NaN or Inf";
        default: return "unknown status";
    }
}

int elsi_gpu_init(elsi_gpu_handle* h, int dtype, int n_basis, int n_state, double n_electron,
                  void* hip_stream)
{
    if (!h) return -1;
    *h = nullptr;
    if (dtype != ELSI_GPU_REAL64 && dtype != ELSI_GPU_COMPLEX128) return -2;
    if (n_basis < 1) return -3;
    if (n_state < 1 || n_state > n_basis) return -4;
    if (!(n_electron >= 0.0) || n_electron > (double)n_basis * 2.0) return -5;
    elsi_gpu_handle_s* p = new (std::nothrow) elsi_gpu_handle_s();
    if (!p) return ELSI_GPU_ERR_OOM;
    p->dtype = dtype;
    p->n = n_basis;
    p->n_state = n_state;
    p->n_electron = n_electron;
    p->stream = (hipStream_t)hip_stream;
    std::memset(&p->info, 0, sizeof(p->info));
    p->info.n_basis = n_basis;
    // second stream and events for full -> band; without them the solve runs
    // on the one stream
    if (hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking) != hipSuccess) p->aux_stream = nullptr;
    for (auto& ev : p->aux_ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
    (void)hipGetLastError();
    *h = p;
    return 0;
}

int elsi_gpu_workspace_size(elsi_gpu_handle h, size_t* bytes)
{
    if (!h) return -1;
    if (!bytes) return -2;
    *bytes = workspace_bytes(h);
    return 0;
}

int elsi_gpu_set_workspace(elsi_gpu_handle h, void* dev_ptr, size_t bytes)
{
    if (!h) return -1;
    if (!dev_ptr) return -2;
    if (bytes < workspace_bytes(h)) return -3;
    release_workspace(h);
    h->ws = dev_ptr;
    h->ws_bytes = bytes;
    h->ws_owned = 0;
    return 0;
}

int elsi_gpu_set_occupation(elsi_gpu_handle h, int scheme, double width, double occ_accuracy,
                            int mu_max_steps, double spin_factor)
{
    if (!h) return -1;
    if (scheme < ELSI_GPU_OCC_EXPLICIT || scheme > ELSI_GPU_OCC_MP1) return -2;
    if (!(width > 0.0)) return -3;
    if (!(occ_accuracy > 0.0)) return -4;
    if (mu_max_steps < 1) return -5;
    if (!(spin_factor > 0.0)) return -6;
    h->occ_scheme = scheme;
    h->kT = width;
    h->occ_accuracy = occ_accuracy;
    h->mu_max_steps = mu_max_steps;
    h->spin = spin_factor;
    return 0;
}

int elsi_gpu_set_singularity(elsi_gpu_handle h, int check, double tolerance)
{
    if (!h) return -1;
    if (check != 0 && check != 1) return -2;
    if (check && h->dtype != ELSI_GPU_REAL64) return -2;
    if (!(tolerance > 0.0)) return -3;
    h->sing_check = check;
    h->sing_tol = tolerance;
    return 0;
}

int elsi_gpu_set_overlap_is_unit(elsi_gpu_handle h, int flag)
{
    if (!h) return -1;
    h->overlap_is_unit = flag ? 1 : 0;
    return 0;
}

int elsi_gpu_set_overlap_factored(elsi_gpu_handle h, int flag)
{
    if (!h) return -1;
    h->overlap_factored = flag ? 1 : 0;
    return 0;
}

int elsi_gpu_set_band_width(elsi_gpu_handle h, int b)
{
    if (!h) return -1;
    if (b < 8 || b > 64 || (b % 8) != 0) return -2;
    h->band_width = b;
    return 0;
}

int elsi_gpu_set_precision(elsi_gpu_handle h, int prec, double refine_tol, int max_refine)
{
    if (!h) return -1;
    if (prec != ELSI_GPU_PREC_FP64 && prec != ELSI_GPU_PREC_MIXED) return -2;
    if (!(refine_tol >= 0.0)) return -3;
    if (max_refine < 0) return -4;
    h->precision = prec;
    h->refine_tol = refine_tol;
    h->max_refine = max_refine;
    return 0;
}

int elsi_gpu_set_launch_timing(elsi_gpu_handle h, int on)
{
    if (!h) return -1;
    if (on != 0 && on != 1) return -2;
    launch_probe::enable(on != 0);
    if (on) launch_probe::reset_totals();
    h->info.probe_launches = 0;
    h->info.probe_ms = 0.0;
    h->info.probe_flops = 0.0;
    h->info.probe_kernel[0] = '\0';
    return 0;
}

int elsi_gpu_get_info(elsi_gpu_handle h, elsi_gpu_info* out)
{
    if (!h) return -1;
    if (!out) return -2;
    *out = h->info;
    return 0;
}

int elsi_gpu_finalize(elsi_gpu_handle* h)
{
    if (!h || !*h) return -1;
    if ((*h)->aux_stream) {
        (void)hipStreamSynchronize((*h)->aux_stream);
        (void)hipStreamDestroy((*h)->aux_stream);
    }
    for (auto ev : (*h)->aux_ev)
        if (ev) (void)hipEventDestroy(ev);
    release_workspace(*h);
    delete *h;
    *h = nullptr;
    return 0;
}

// ---------------------------------------------------------------------------
// stage entry points
// ---------------------------------------------------------------------------
int elsi_gpu_x_dgemm(char ta, char tb, int m, int n, int k, double alpha, const double* A, int lda,
                     const double* B, int ldb, double beta, double* C, int ldc, void* hip_stream)
{
    if (ta != 'N' && ta != 'T' && ta != 'S') return -1;
    if (tb != 'N' && tb != 'T') return -2;
    if (ta == 'S' && tb != 'N') return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0 || (ta == 'S' && k != m)) return -5;
    if (m == 0 || n == 0) return 0;
    if (!C) return -12;
    if (k > 0 && (!A || !B)) return !A ? -7 : -9;
    hipStream_t st = (hipStream_t)hip_stream;
    dgemm(st, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, 0);
    return sync_status(st);
}

int elsi_gpu_x_gemm_fp32(char ta, char tb, int m, int n, int k, double alpha, const double* A, int lda,
                         const double* B, int ldb, double beta, double* C, int ldc, int uplo, void* hip_stream)
{
    if (ta != 'N' && ta != 'T' && ta != 'S') return -1;
    if (tb != 'N' && tb != 'T') return -2;
    if (ta == 'S' && tb != 'N') return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0 || (ta == 'S' && k != m)) return -5;
    if (uplo != 0 && uplo != 1) return -14;
    if (m == 0 || n == 0) return 0;
    if (!C) return -12;
    if (k > 0 && (!A || !B)) return !A ? -7 : -9;
    hipStream_t st = (hipStream_t)hip_stream;
    {
        Fp32GemmScope fp32(true);
        dgemm(st, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, uplo);
    }
    return sync_status(st);
}

int elsi_gpu_x_cholesky(int n, double* S, int lds, int* fail_col, void* hip_stream)
{
    if (n < 0) return -1;
    if (n == 0) return 0;
    if (!S) return -2;
    if (lds < n) return -3;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf<double> Linv;
    DevBuf<int> info;
    if (!Linv.alloc((size_t)ceil_div(n, 64) * 64 * 64) || !info.alloc(1)) return ELSI_GPU_ERR_OOM;
    fill_i(st, info.p, 1, 0);
    dpotrf(st, n, S, lds, Linv.p, info.p);
    int hinfo = 0;
    if (hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
        return ELSI_GPU_ERR_HIP;
    int rc = sync_status(st);
    if (rc) return rc;
    if (fail_col) *fail_col = hinfo;
    return hinfo ? ELSI_GPU_ERR_NOT_PD : 0;
}

int elsi_gpu_x_reduce(int n, double* H, int ldh, const double* L, int ldl, void* hip_stream)
{
    if (n < 0) return -1;
    if (n == 0) return 0;
    if (!H) return -2;
    if (ldh < n) return -3;
    if (!L) return -4;
    if (ldl < n) return -5;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf<double> Linv;
    if (!Linv.alloc((size_t)ceil_div(n, 64) * 64 * 64)) return ELSI_GPU_ERR_OOM;
    reduce_to_standard(st, n, H, ldh, L, ldl, Linv.p);
    return sync_status(st);
}

int elsi_gpu_x_backsub(int n, int k, const double* L, int ldl, double* X, int ldx, void* hip_stream)
{
    if (n < 0) return -1;
    if (k < 0) return -2;
    if (n == 0 || k == 0) return 0;
    if (!L) return -3;
    if (ldl < n) return -4;
    if (!X) return -5;
    if (ldx < n) return -6;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf<double> Linv;
    if (!Linv.alloc((size_t)ceil_div(n, 64) * 64 * 64)) return ELSI_GPU_ERR_OOM;
    dtrtri_diag_blocks(st, n, L, ldl, Linv.p);
    dtrsm_left_lower_t(st, n, k, L, ldl, Linv.p, X, ldx);
    return sync_status(st);
}

int elsi_gpu_x_occupations(int n, const double* eps, const double* weight, int scheme, double n_electron,
                           double width, double spin, double occ_accuracy, int mu_max_steps, double* f, double* mu,
                           int* k_s, void* hip_stream)
{
    if (n < 1) return -1;
    if (!eps) return -2;
    if (scheme < ELSI_GPU_OCC_FERMI || scheme > ELSI_GPU_OCC_MP1) return -4;
    if (!(n_electron >= 0.0)) return -5;
    if (!(width > 0.0)) return -6;
    if (!(spin > 0.0)) return -7;
    if (!(occ_accuracy > 0.0)) return -8;
    if (mu_max_steps < 1) return -9;
    if (!f) return -10;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf<double> scal;
    if (!scal.alloc(8)) return ELSI_GPU_ERR_OOM;
    occupations(st, n, eps, weight, scheme, n_electron, width, spin, occ_accuracy, mu_max_steps, kFCut, f, scal.p);
    double hs[8];
    if (hipMemcpyAsync(hs, scal.p, 6 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
        return ELSI_GPU_ERR_HIP;
    int rc = sync_status(st);
    if (rc) return rc;
    if (mu) *mu = hs[0];
    if (k_s) *k_s = (int)hs[2];
    return (int)hs[1];
}

int elsi_gpu_x_density(int n, int k, const double* C, int ldc, const double* f, double* D, int ldd,
                       void* hip_stream)
{
    if (n < 0) return -1;
    if (k < 0) return -2;
    if (n == 0) return 0;
    if (k > 0 && !C) return -3;
    if (ldc < n) return -4;
    if (k > 0 && !f) return -5;
    if (!D) return -6;
    if (ldd < n) return -7;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf<double> W, W2;
    if (k > 0 && (!W.alloc((size_t)n * k) || !W2.alloc((size_t)n * k))) return ELSI_GPU_ERR_OOM;
    density_matrix(st, n, k, C, ldc, f, W.p, W2.p, D, ldd);
    return sync_status(st);
}

int elsi_gpu_x_band_reduce(int n, int b, double* A, int lda, double* band, int ldband, void* hip_stream)
{
    if (n < 1) return -1;
    if (b < 1 || b > 64) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!band) return -5;
    if (ldband < b + 1) return -6;
    hipStream_t st = (hipStream_t)hip_stream;
    const int bb = std::min(b, std::max(1, n - 1));
    DevBuf<double> Vall, Tall, Bd, work, Acopy;
    if (!Vall.alloc((size_t)n * n) || !Tall.alloc((size_t)ceil_div(n, bb) * bb * bb) ||
        !Bd.alloc((size_t)2 * bb * n) || !work.alloc(sy2sb_workspace_doubles(n, bb)) || !Acopy.alloc((size_t)n * n))
        return ELSI_GPU_ERR_OOM;
    copy_matrix(st, n, n, A, lda, Acopy.p, n);
    mirror_lower_to_upper(st, n, Acopy.p, n);
    sy2sb(st, n, bb, Acopy.p, n, Vall.p, Tall.p, Bd.p, 2 * bb, work.p);
    for (int c = 0; c < n; ++c) fill_d(st, band + (size_t)c * ldband, (size_t)(b + 1), 0.0);
    copy_matrix(st, bb + 1, n, Bd.p, 2 * bb, band, ldband);
    return sync_status(st);
}

int elsi_gpu_x_tridiagonalize(int n, int b, double* A, int lda, double* d, double* e, void* hip_stream)
{
    if (n < 1) return -1;
    if (b < 1 || b > 64) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!d) return -5;
    if (!e && n > 1) return -6;
    hipStream_t st = (hipStream_t)hip_stream;
    const int bb = std::min(b, std::max(1, n - 1));
    DevBuf<double> Vall, Tall, Bd, work, Acopy, V2, tau2, ee, mbox;
    DevBuf<int> ints;
    if (!Vall.alloc((size_t)n * n) || !Tall.alloc((size_t)ceil_div(n, bb) * bb * bb) ||
        !Bd.alloc((size_t)2 * bb * n) || !work.alloc(sy2sb_workspace_doubles(n, bb)) ||
        !Acopy.alloc((size_t)n * n) || !V2.alloc((size_t)n * n) ||
        !tau2.alloc((size_t)std::max(n - 2, 1) * sb2st_kmax(n, bb)) || !ee.alloc((size_t)n) ||
        !ints.alloc((size_t)n + 64) || !mbox.alloc(sb2st_mailbox_doubles(n, bb)))
        return ELSI_GPU_ERR_OOM;
    copy_matrix(st, n, n, A, lda, Acopy.p, n);
    mirror_lower_to_upper(st, n, Acopy.p, n);
    sy2sb(st, n, bb, Acopy.p, n, Vall.p, Tall.p, Bd.p, 2 * bb, work.p);
    int rc = sb2st(st, n, bb, Bd.p, 2 * bb, d, ee.p, V2.p, tau2.p, ints.p + 64, ints.p, mbox.p);
    if (rc) return rc;
    if (n > 1) (void)hipMemcpyAsync(e, ee.p, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, st);
    int herr = 0;
    (void)hipMemcpyAsync(&herr, ints.p, sizeof(int), hipMemcpyDeviceToHost, st);
    rc = sync_status(st);
    if (rc) return rc;
    return herr ? ELSI_GPU_ERR_NO_CONV : 0;
}

int elsi_gpu_x_set_bulge_path(int path)
{
    if (path < 0 || path > 2) return -1;
    set_bulge_path(path);
    return 0;
}

int elsi_gpu_x_backtransform(int n, int b, const double* A, int lda, double* d, double* e, double* X, int ldx,
                             int ncol, int trans, int slab, void* hip_stream)
{
    if (n < 1) return -1;
    if (b < 1 || b > 64) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!d) return -5;
    if (!e && n > 1) return -6;
    if (!X && ncol > 0) return -7;
    if (ldx < n) return -8;
    if (ncol < 0) return -9;
    if (trans != 0 && trans != 1) return -10;
    if (slab != 0 && slab != 128 && slab != 256 && slab != 512) return -11;
    hipStream_t st = (hipStream_t)hip_stream;
    const int bb = std::min(b, std::max(1, n - 1));
    const int kmax = sb2st_kmax(n, bb);
    DevBuf<double> Vall, Tall, Bd, work, Acopy, V2, tau2, ee, Tq, q1work, mbox;
    DevBuf<int> ints;
    if (!Vall.alloc((size_t)n * n) || !Tall.alloc((size_t)ceil_div(n, bb) * bb * bb) ||
        !Bd.alloc((size_t)2 * bb * n) || !work.alloc(sy2sb_workspace_doubles(n, bb)) ||
        !Acopy.alloc((size_t)n * n) || !V2.alloc((size_t)n * n) ||
        !tau2.alloc((size_t)std::max(n - 2, 1) * kmax) || !ee.alloc((size_t)n) ||
        !ints.alloc((size_t)n + 64) || !Tq.alloc(apply_q2_workspace_doubles(n, bb)) ||
        !mbox.alloc(sb2st_mailbox_doubles(n, bb)) ||
        !q1work.alloc(apply_q1_workspace_doubles(n, std::max(ncol, 1))))
        return ELSI_GPU_ERR_OOM;
    copy_matrix(st, n, n, A, lda, Acopy.p, n);
    mirror_lower_to_upper(st, n, Acopy.p, n);
    sy2sb(st, n, bb, Acopy.p, n, Vall.p, Tall.p, Bd.p, 2 * bb, work.p);
    int rc = sb2st(st, n, bb, Bd.p, 2 * bb, d, ee.p, V2.p, tau2.p, ints.p + 64, ints.p, mbox.p);
    if (rc) return rc;
    if (n > 1) (void)hipMemcpyAsync(e, ee.p, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, st);
    if (ncol > 0) {
        if (trans) {
            apply_q1(st, n, bb, ncol, Vall.p, Tall.p, X, ldx, q1work.p, true);
            apply_q2(st, n, bb, ncol, V2.p, tau2.p, kmax, X, ldx, Tq.p, true, false, slab);
        } else {
            apply_q2(st, n, bb, ncol, V2.p, tau2.p, kmax, X, ldx, Tq.p, false, false, slab);
            apply_q1(st, n, bb, ncol, Vall.p, Tall.p, X, ldx, q1work.p, false);
        }
    }
    int herr = 0;
    (void)hipMemcpyAsync(&herr, ints.p, sizeof(int), hipMemcpyDeviceToHost, st);
    rc = sync_status(st);
    if (rc) return rc;
    return herr ? ELSI_GPU_ERR_NO_CONV : 0;
}

int elsi_gpu_x_tridiag_eig(int n, const double* d, const double* e, double* w, double* Z, int ldz,
                           void* hip_stream)
{
    if (n < 1) return -1;
    if (!d) return -2;
    if (!e && n > 1) return -3;
    if (!w) return -4;
    if (!Z) return -5;
    if (ldz < n) return -6;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf<double> Z1, Z2, U, ee;
    DevBuf<char> work;
    DevBuf<int> err;
    if (!Z1.alloc((size_t)n * n) || !Z2.alloc((size_t)n * n) || !U.alloc((size_t)n * n) ||
        !work.alloc(stedc_workspace_bytes(n)) || !err.alloc(4) || !ee.alloc((size_t)n))
        return ELSI_GPU_ERR_OOM;
    fill_d(st, ee.p, (size_t)n, 0.0);
    if (n > 1) (void)hipMemcpyAsync(ee.p, e, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, st);
    int rc = stedc(st, n, d, ee.p, w, Z1.p, Z2.p, U.p, n, n, work.p, err.p, nullptr);
    if (rc) return rc;
    copy_matrix(st, n, n, Z1.p, n, Z, ldz);
    int herr = 0;
    (void)hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, st);
    rc = sync_status(st);
    if (rc) return rc;
    return herr ? ELSI_GPU_ERR_NO_CONV : 0;
}

}  // extern "C"
