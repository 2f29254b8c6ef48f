// Drivers of the dense path: reduction to standard form, density matrix, and
// (below) the eigensolver / density-matrix entry points.
#include "api_internal.h"

#include <cstdio>

#include <algorithm>
#include <cstring>
#include <vector>

namespace eg {

// Eq. (11): W = L^-1 H, then the lower triangle of H~ = W L^-T, mirrored.
// (The blocked two-sided recurrence needs only n^3 flops against 4n^3/3 here,
// but its intermediate H21 L11^-T - L21 H~11 carries the large entries of H~
// that an ill-conditioned S creates and loses accuracy to cancellation.)
void reduce_to_standard(hipStream_t st, int n, double* H, int ldh, const double* L, int ldl, double* Linv)
{
    dtrtri_diag_blocks(st, n, L, ldl, Linv);
    mirror_lower_to_upper(st, n, H, ldh);   // only the lower triangle of H is read
    dtrsm_left_lower_n(st, n, n, L, ldl, Linv, H, ldh);
    dtrsm_right_lower_t_lowerpart(st, n, L, ldl, Linv, H, ldh);
    mirror_lower_to_upper(st, n, H, ldh);
}

// Eq. (9): D = sum_l f_l c_l c_l^T = (C |F|^1/2)(C sign(F) |F|^1/2)^T (the
// two factors are equal when every f_l >= 0), lower tiles on the matrix
// cores, then mirrored.
void density_matrix(hipStream_t st, int n, int k, const double* C, int ldc, const double* f, double* W, double* W2,
                    double* D, int ldd)
{
    if (k <= 0) {
        for (int j = 0; j < n; ++j) fill_d(st, D + cm(0, j, ldd), (size_t)n, 0.0);
        return;
    }
    scale_columns_signed(st, n, k, C, ldc, f, W, W2, n);
    dgemm(st, 'N', 'T', n, n, k, 1.0, W, n, W2, n, 0.0, D, ldd, 1);
    mirror_lower_to_upper(st, n, D, ldd);
}

// ---------------------------------------------------------------------------
// workspace layout (all sub-buffers 256-byte aligned)
// ---------------------------------------------------------------------------
struct Layout {
    size_t linv, bd, vall, tall, v2, tau2, tq2, tq1, d, e, w, z, z2, u, sywork, dcwork, q1work, f, scal, ints, mbox;
    int q1ncol;   // columns the Q1 workspace is sized for
    // mixed precision: the band reduction's copy of H~ (H keeps H~ for the
    // refinement), which afterwards holds the eigenvectors of T of the carried
    // states; the refinement's k' x k' blocks, per-state values and the
    // factors of its tridiagonal solves
    size_t hcopy, rg, rq, rtheta, rres, rstep, tri1, trisw;
    size_t hv, sv;   // eigenvalue pass of a shared-mu batch: copies of H and S (the inputs stay intact)
    size_t total;
};

static Layout make_layout(int n, int b, int ncol, bool mixed = false, bool vcopy = false)
{
    Layout L{};
    size_t off = 0;
    auto put = [&](size_t bytes) { size_t r = off; off += align_up(std::max<size_t>(bytes, 8), 256); return r; };
    const size_t nn = (size_t)n * n;
    L.linv = put(sizeof(double) * (size_t)ceil_div(n, 64) * 4096);
    L.bd = put(sizeof(double) * (size_t)2 * b * n);
    L.vall = put(sizeof(double) * nn);
    L.tall = put(sizeof(double) * (size_t)ceil_div(n, b) * b * b);
    L.v2 = put(sizeof(double) * nn);
    L.tau2 = put(sizeof(double) * (size_t)std::max(n - 2, 1) * sb2st_kmax(n, b));
    L.tq2 = put(sizeof(double) * apply_q2_workspace_doubles(n, b));
    L.tq1 = put(sizeof(double) * q1_tfactor_doubles(n, b));
    L.d = put(sizeof(double) * n);
    L.e = put(sizeof(double) * n);
    L.w = put(sizeof(double) * n);
    L.z = put(sizeof(double) * nn);
    L.z2 = put(sizeof(double) * nn);
    L.u = put(sizeof(double) * nn);
    L.sywork = put(sizeof(double) * sy2sb_workspace_doubles(n, b));
    L.dcwork = put(stedc_workspace_bytes(n));
    L.q1work = put(sizeof(double) * apply_q1_workspace_doubles(n, ncol));
    L.q1ncol = ncol;
    L.f = put(sizeof(double) * n);
    L.scal = put(sizeof(double) * 16);
    L.ints = put(sizeof(int) * ((size_t)n + 64));
    L.mbox = put(sizeof(double) * sb2st_mailbox_doubles(n, b));
    if (mixed) {
        L.hcopy = put(sizeof(double) * nn);
        L.rg = put(sizeof(double) * nn);
        L.rq = put(sizeof(double) * nn);
        L.rtheta = put(sizeof(double) * n);
        L.rres = put(sizeof(double) * n);
        L.rstep = put(sizeof(double) * n);
        L.tri1 = put(sizeof(double) * nn);
        L.trisw = put(nn);
    }
    if (vcopy) {
        L.hv = put(sizeof(double) * nn);
        L.sv = put(sizeof(double) * nn);
    }
    L.total = off;
    return L;
}

// Complex handles solve the real 2n x 2n image of their pencil: the real
// layout for 2n, then the images of H, S and of the result (D, or the chosen
// eigenvectors), the doubled occupations and a small index list.
struct CLayout {
    size_t h2, s2, x2, f2, idx;
    size_t total;
};

static CLayout make_clayout(size_t base, int n)
{
    CLayout C{};
    size_t off = base;
    auto put = [&](size_t bytes) { size_t r = off; off += align_up(std::max<size_t>(bytes, 8), 256); return r; };
    const size_t n2 = (size_t)2 * n;
    C.h2 = put(sizeof(double) * n2 * n2);
    C.s2 = put(sizeof(double) * n2 * n2);
    C.x2 = put(sizeof(double) * n2 * n2);
    C.f2 = put(sizeof(double) * n2);
    C.idx = put(sizeof(int) * (size_t)n);
    C.total = off;
    return C;
}

size_t workspace_bytes(const elsi_gpu_handle_s* h)
{
    if (h->dtype == ELSI_GPU_COMPLEX128) {
        const size_t base =
            make_layout(2 * h->n, h->band_width, 2 * h->n, h->precision == ELSI_GPU_PREC_MIXED).total;
        return make_clayout(base, h->n).total;
    }
    return make_layout(h->n, h->band_width, h->n, h->precision == ELSI_GPU_PREC_MIXED, h->values_copies != 0).total;
}

void release_workspace(elsi_gpu_handle_s* h)
{
    if (h->ws && h->ws_owned) (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
    h->ws_owned = 0;
}

static int ensure_workspace(elsi_gpu_handle_s* h)
{
    size_t need = workspace_bytes(h);
    if (h->ws && h->ws_bytes >= need) return 0;
    if (h->ws && !h->ws_owned) return -1;   // caller-provided buffer became too small
    release_workspace(h);
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
        (void)hipGetLastError();
        return kStatusOom;
    }
    h->ws = p;
    h->ws_bytes = need;
    h->ws_owned = 1;
    return 0;
}

// Per-stage device time: each mark() closes the interval since the previous
// mark (or the start) and charges it to the given stage.
struct Timer {
    static constexpr int kMax = 32;
    hipEvent_t start, stop;
    hipEvent_t ev[kMax];
    int stage[kMax];
    int nmark = 0;
    hipStream_t st;
    explicit Timer(hipStream_t s) : st(s) {
        (void)hipEventCreate(&start);
        (void)hipEventCreate(&stop);
        (void)hipEventRecord(start, st);
    }
    void mark(int stg) {
        if (nmark >= kMax) return;
        (void)hipEventCreate(&ev[nmark]);
        (void)hipEventRecord(ev[nmark], st);
        stage[nmark++] = stg;
    }
    void finish(elsi_gpu_info* info) {
        (void)hipEventRecord(stop, st);
        (void)hipEventSynchronize(stop);
        for (int i = 0; i < ELSI_GPU_NSTAGES; ++i) info->stage_ms[i] = 0.0;
        hipEvent_t prev = start;
        for (int i = 0; i < nmark; ++i) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, prev, ev[i]);
            info->stage_ms[stage[i]] += ms;
            prev = ev[i];
        }
        float tot = 0.f;
        (void)hipEventElapsedTime(&tot, start, stop);
        info->total_ms = tot;
    }
    ~Timer() {
        for (int i = 0; i < nmark; ++i) (void)hipEventDestroy(ev[i]);
        (void)hipEventDestroy(start);
        (void)hipEventDestroy(stop);
    }
};

// Steps common to ev and dm: finiteness check, Cholesky (Eq. (10)),
// reduction (Eq. (11)), full -> band and band -> tridiagonal (Eq. (13)), and
// the tridiagonal eigenpairs (divide and conquer).  On success w holds all
// eigenvalues ascending and Z the eigenvectors of T (first ncol columns).
// vectors: back_half follows, so the block T factors of Q2 and the group T'
// factors of Q1 are built on the handle's second stream while the tridiagonal
// problem is solved.
static int front_half(elsi_gpu_handle_s* h, double* H, double* S, char* ws, const Layout& L, Timer& tm,
                      DcState* dc, bool vectors)
{
    hipStream_t st = h->stream;
    const int n = h->n, b = std::min(h->band_width, std::max(1, n - 1));
    int* ints = (int*)(ws + L.ints);
    int* info = ints;        // Cholesky pivot
    int* flag = ints + 1;    // non-finite input
    int* err = ints + 2;     // sb2st / stedc failure flags
    int* err2 = ints + 3;
    int* progress = ints + 64;
    double* Linv = (double*)(ws + L.linv);
    fill_i(st, ints, 64, 0);
    check_finite(st, n, n, H, n, flag);
    if (!h->overlap_is_unit) check_finite(st, n, n, S, n, flag);
    int hflags[2] = {0, 0};
    if (hipMemcpyAsync(hflags, ints, 2 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return kStatusHip;
    if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
    if (hflags[1]) return 7;
    if (!h->overlap_is_unit) {
        if (!h->overlap_factored) {
            dpotrf(st, n, S, n, Linv, info);
            if (hipMemcpyAsync(hflags, info, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return kStatusHip;
            if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
            if (hflags[0]) {
                h->info.fail_col = hflags[0];
                return kStatusNotPD;
            }
        }
        tm.mark(ELSI_GPU_ST_CHOLESKY);
        reduce_to_standard(st, n, H, n, S, n, Linv);
    } else {
        tm.mark(ELSI_GPU_ST_CHOLESKY);
        mirror_lower_to_upper(st, n, H, n);
    }
    tm.mark(ELSI_GPU_ST_REDUCE);
    double* Bd = (double*)(ws + L.bd);
    double* Vall = (double*)(ws + L.vall);
    double* Tall = (double*)(ws + L.tall);
    const bool mixed = h->precision == ELSI_GPU_PREC_MIXED;
    double* A = H;
    if (mixed) {   // the refinement needs H~ after step (1) has consumed its copy
        A = (double*)(ws + L.hcopy);
        copy_matrix(st, n, n, H, n, A, n);
    }
    {
        // outside batched calls (whose workers keep one stream each) the panel
        // T factors run on the handle's second stream
        Sy2sbAux aux{nullptr, nullptr, nullptr};
        if (!batch_mode_active()) aux = Sy2sbAux{h->aux_stream, h->aux_ev[0], h->aux_ev[1]};
        Fp32GemmScope fp32(mixed);
        sy2sb(st, n, b, A, n, Vall, Tall, Bd, 2 * b, (double*)(ws + L.sywork), &aux);
    }
    tm.mark(ELSI_GPU_ST_BAND);
    double* d = (double*)(ws + L.d);
    double* e = (double*)(ws + L.e);
    int rc = sb2st(st, n, b, Bd, 2 * b, d, e, (double*)(ws + L.v2), (double*)(ws + L.tau2), progress, err,
                   (double*)(ws + L.mbox));
    if (rc) return rc;
    tm.mark(ELSI_GPU_ST_BULGE);
    // the T factors of Q2 need only the reflectors of step (2), the group T'
    // factors of Q1 only those of step (1); outside batched calls (whose workers
    // keep one stream each) both are built beside the tridiagonal solve
    bool q2t_built = false;
    hipEvent_t q2t_ev = nullptr;
    if (vectors && !batch_mode_active() && h->aux_stream && h->aux_ev[0] && h->aux_ev[1] &&
        hipEventRecord(h->aux_ev[0], st) == hipSuccess &&
        hipStreamWaitEvent(h->aux_stream, h->aux_ev[0], 0) == hipSuccess) {
        build_q2_t(h->aux_stream, n, b, (double*)(ws + L.v2), (double*)(ws + L.tau2), sb2st_kmax(n, b),
                   (double*)(ws + L.tq2));
        build_q1_t(h->aux_stream, n, b, L.q1ncol, Vall, Tall, (double*)(ws + L.tq1), (double*)(ws + L.q1work));
        if (hipEventRecord(h->aux_ev[1], h->aux_stream) == hipSuccess)
            q2t_ev = h->aux_ev[1];
        else if (hipStreamSynchronize(h->aux_stream) != hipSuccess)
            return kStatusHip;
        q2t_built = true;
    }
    double* w = (double*)(ws + L.w);
    rc = stedc_values(st, n, d, e, w, (double*)(ws + L.z), (double*)(ws + L.z2), (double*)(ws + L.u), n,
                      ws + L.dcwork, err2, dc);
    if (rc) {
        // no back half follows: keep later work on the stream behind the reads of the reflectors
        if (q2t_ev) (void)hipStreamWaitEvent(st, q2t_ev, 0);
        return rc;
    }
    dc->q2t_built = q2t_built;
    dc->q2t_ev = q2t_ev;
    dc->q1t = q2t_built ? (const double*)(ws + L.tq1) : nullptr;
    tm.mark(ELSI_GPU_ST_TRIDIAG);
    return 0;
}

// X (n x k, in Z) <- L^-T X.
static void back_substitute(elsi_gpu_handle_s* h, double* S, char* ws, const Layout& L, Timer& tm, int k)
{
    hipStream_t st = h->stream;
    const int n = h->n;
    if (!h->overlap_is_unit) {
        double* Linv = (double*)(ws + L.linv);
        dtrtri_diag_blocks(st, n, S, n, Linv);
        dtrsm_left_lower_t(st, n, k, S, n, Linv, (double*)(ws + L.z), n);
    }
    tm.mark(ELSI_GPU_ST_BACKSUB);
}

// X (n x k, in Z) <- L^-T Q1 Q2 X: steps (4), (5) and the back substitution.
// zsave (n x k, may be NULL) receives the eigenvectors of T before step (4).
static void back_half(elsi_gpu_handle_s* h, double* S, char* ws, const Layout& L, Timer& tm, int k, DcState* dc,
                      bool backsub = true, double* zsave = nullptr)
{
    hipStream_t st = h->stream;
    const int n = h->n, b = std::min(h->band_width, std::max(1, n - 1));
    double* X = (double*)(ws + L.z);
    stedc_vectors(st, *dc, k);   // top merge of step (3) restricted to the k wanted columns
    if (zsave) copy_matrix(st, n, k, X, n, zsave, n);
    tm.mark(ELSI_GPU_ST_TRIDIAG);
    if (dc->q2t_ev) (void)hipStreamWaitEvent(st, dc->q2t_ev, 0);
    apply_q2(st, n, b, k, (double*)(ws + L.v2), (double*)(ws + L.tau2), sb2st_kmax(n, b), X, n,
             (double*)(ws + L.tq2), false, dc->q2t_built);
    dc->q2t_built = false;
    dc->q2t_ev = nullptr;
    tm.mark(ELSI_GPU_ST_BACK_Q2);
    {
        Fp32GemmScope fp32(h->precision == ELSI_GPU_PREC_MIXED);
        apply_q1(st, n, b, k, (double*)(ws + L.vall), (double*)(ws + L.tall), X, n, (double*)(ws + L.q1work), false,
                 dc->q1t);
    }
    tm.mark(ELSI_GPU_ST_BACK_Q1);
    if (backsub) back_substitute(h, S, ws, L, tm, k);
}

// The factorization H~ ~ (Q1 Q2) T (Q1 Q2)^T left by steps (1) and (2): Q1 from
// the panel reflectors, Q2 from the bulge-chasing reflectors (their block T
// factors already built by the forward application of step (4)).
struct ReflectorPrecond : RefinePrecond {
    int n = 0, b = 0, kmax = 0;
    const double *Vall = nullptr, *Tall = nullptr, *V2 = nullptr, *tau2 = nullptr;
    const double* Tq1 = nullptr;   // Q1's group T' factors when built beforehand
    double *Tq = nullptr, *q1work = nullptr;
    // Q1's products run on the FP32 matrix cores, as in step (5) of this mode:
    // the correction only needs its own size to a few digits
    void apply_qt(hipStream_t st, double* X, int ld, int ncol, double* tmp) override
    {
        (void)tmp;
        {
            Fp32GemmScope fp32(true);
            apply_q1(st, n, b, ncol, Vall, Tall, X, ld, q1work, true, Tq1);
        }
        apply_q2(st, n, b, ncol, V2, tau2, kmax, X, ld, Tq, true, true);
    }
    void apply_q(hipStream_t st, double* X, int ld, int ncol, double* tmp) override
    {
        (void)tmp;
        apply_q2(st, n, b, ncol, V2, tau2, kmax, X, ld, Tq, false, true);
        Fp32GemmScope fp32(true);
        apply_q1(st, n, b, ncol, Vall, Tall, X, ld, q1work, false, Tq1);
    }
};

// Mixed precision: FP64 refinement of the k' columns in Z against H~ (held in
// H), with the Newton correction through the reduced-precision factorization;
// the eigenvectors of T of the k' states are in hcopy.  On return Z holds the
// refined vectors and w[0 .. k') their Ritz values.  kw leading states decide
// convergence, each step weighted by weight[l] (device; NULL: 1).  q1t: Q1's
// group T' factors when the front half built them (NULL: built per application).
// Returns 0, kStatusRefine (outputs usable, tolerance not reached) or an error.
static int refine_states(elsi_gpu_handle_s* h, const double* Ht, char* ws, const Layout& L, Timer& tm, int kp,
                         int kw, const double* weight, const double* q1t)
{
    hipStream_t st = h->stream;
    const int n = h->n, b = std::min(h->band_width, std::max(1, n - 1));
    RefineBuffers B{};
    B.X[0] = (double*)(ws + L.z);
    B.X[1] = (double*)(ws + L.z2);
    B.X[2] = (double*)(ws + L.u);
    B.ldb = n;
    B.G = (double*)(ws + L.rg);
    B.Qm = (double*)(ws + L.rq);
    B.Linv = (double*)(ws + L.linv);   // rebuilt for the back substitution
    B.theta = (double*)(ws + L.rtheta);
    B.r = (double*)(ws + L.rres);
    B.step = (double*)(ws + L.rstep);
    B.dinfo = (int*)(ws + L.ints) + 8;
    B.part = (double*)(ws + L.sywork);   // free after step (1)
    B.npart = sy2sb_workspace_doubles(n, b);
    B.U1 = (double*)(ws + L.tri1);
    B.SW = (unsigned char*)(ws + L.trisw);
    ReflectorPrecond pc;
    pc.n = n;
    pc.b = b;
    pc.kmax = sb2st_kmax(n, b);
    pc.Vall = (const double*)(ws + L.vall);
    pc.Tall = (const double*)(ws + L.tall);
    pc.V2 = (const double*)(ws + L.v2);
    pc.tau2 = (const double*)(ws + L.tau2);
    pc.Tq = (double*)(ws + L.tq2);
    pc.q1work = (double*)(ws + L.q1work);
    pc.Tq1 = q1t;
    pc.Z = (const double*)(ws + L.hcopy);
    pc.ldz = n;
    pc.d = (const double*)(ws + L.d);
    pc.e = (const double*)(ws + L.e);
    RefineOutcome out{};
    int rc = refine_subspace(st, n, kp, kw, Ht, n, B, &pc, weight, h->refine_tol, h->max_refine, &out);
    if (rc && rc != kStatusRefine) return rc;
    if (out.sweeps > 0) {
        if (out.x_buf != 0) copy_matrix(st, n, kp, B.X[out.x_buf], n, B.X[0], n);
        if (hipMemcpyAsync(ws + L.w, B.theta, sizeof(double) * kp, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return kStatusHip;
    }
    h->info.refine_sweeps = out.sweeps;
    h->info.refine_states = kp;
    h->info.refine_resid = out.rmax;
    h->info.refine_step = out.smax;
    for (int l = 0; l < 8; ++l) h->info.refine_hist[l] = out.hist[l];
    tm.mark(ELSI_GPU_ST_REFINE);
    return (rc == kStatusRefine || !out.converged) ? kStatusRefine : 0;
}

// Fold the launch timings of the finished call into the info record.
static void harvest_launch_probe(elsi_gpu_handle_s* h)
{
    if (!launch_probe::enabled()) return;
    launch_probe::harvest();
    int nl = 0;
    double ms = 0.0, fl = 0.0;
    const char* name = "";
    if (launch_probe::dominant(&nl, &ms, &fl, &name)) {
        h->info.probe_launches = nl;
        h->info.probe_ms = ms;
        h->info.probe_flops = fl;
        std::snprintf(h->info.probe_kernel, sizeof(h->info.probe_kernel), "%s", name);
    }
}

static int read_flags(hipStream_t st, char* ws, const Layout& L)
{
    int f[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(f, ws + L.ints, 4 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return kStatusHip;
    if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
    if (f[2] || f[3]) return kStatusNoConv;
    return 0;
}

}  // namespace eg

using namespace eg;

static int ev_real(elsi_gpu_handle_s* h, double* H, double* S, double* eval, double* evec)
{
    if (!h) return -1;
    if (!H) return -2;
    if (!S && !h->overlap_is_unit) return -3;
    if (!eval) return -4;
    if (!evec) return -5;
    int rc = ensure_workspace(h);
    if (rc) return rc < 0 ? -1 : rc;
    hipStream_t st = h->stream;
    const int n = h->n, k = h->n_state;
    const bool mixed = h->precision == ELSI_GPU_PREC_MIXED;
    char* ws = (char*)h->ws;
    const Layout L = make_layout(n, h->band_width, n, mixed);
    std::memset(h->info.stage_ms, 0, sizeof(h->info.stage_ms));
    h->info.fail_col = 0;
    h->info.band_width = std::min(h->band_width, std::max(1, n - 1));
    h->info.refine_sweeps = 0;
    h->info.refine_states = 0;
    h->info.refine_resid = 0.0;
    h->info.refine_step = 0.0;
    for (int l = 0; l < 8; ++l) h->info.refine_hist[l] = 0.0;
    Timer tm(st);
    DcState dc;
    rc = front_half(h, H, S, ws, L, tm, &dc, true);
    if (rc) { tm.finish(&h->info); return rc; }
    int rstat = 0;
    if (mixed) {
        const int kp = refine_columns(n, k);
        back_half(h, S, ws, L, tm, kp, &dc, false, (double*)(ws + L.hcopy));
        rstat = refine_states(h, H, ws, L, tm, kp, k, nullptr, dc.q1t);
        if (rstat && rstat != kStatusRefine) { tm.finish(&h->info); return rstat; }
        back_substitute(h, S, ws, L, tm, k);
    } else {
        back_half(h, S, ws, L, tm, k, &dc);
    }
    copy_matrix(st, n, k, (double*)(ws + L.z), n, evec, n);
    (void)hipMemcpyAsync(eval, ws + L.w, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    rc = sync_status(st);
    if (rc) return rc;
    tm.finish(&h->info);
    harvest_launch_probe(h);
    rc = read_flags(st, ws, L);
    return rc ? rc : rstat;
}

static int dm_real(elsi_gpu_handle_s* h, double* H, double* S, double* occ, double* D, double* eval,
                   double* energy, double* mu)
{
    if (!h) return -1;
    if (!H) return -2;
    if (!S && !h->overlap_is_unit) return -3;
    if (!occ && h->occ_scheme == ELSI_GPU_OCC_EXPLICIT) return -4;
    if (!D) return -5;
    if (!energy) return -7;
    int rc = ensure_workspace(h);
    if (rc) return rc < 0 ? -1 : rc;
    hipStream_t st = h->stream;
    const int n = h->n;
    const bool mixed = h->precision == ELSI_GPU_PREC_MIXED;
    char* ws = (char*)h->ws;
    const Layout L = make_layout(n, h->band_width, n, mixed);
    std::memset(h->info.stage_ms, 0, sizeof(h->info.stage_ms));
    h->info.fail_col = 0;
    h->info.band_width = std::min(h->band_width, std::max(1, n - 1));
    h->info.refine_sweeps = 0;
    h->info.refine_states = 0;
    h->info.refine_resid = 0.0;
    h->info.refine_step = 0.0;
    for (int l = 0; l < 8; ++l) h->info.refine_hist[l] = 0.0;
    Timer tm(st);
    DcState dc;
    rc = front_half(h, H, S, ws, L, tm, &dc, true);
    if (rc) { tm.finish(&h->info); return rc; }
    double* w = (double*)(ws + L.w);
    double* f = occ ? occ : (double*)(ws + L.f);
    double* scal = (double*)(ws + L.scal);
    int status = 0;
    int ks = 0;
    double hs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto occupy = [&]() -> int {
        if (h->occ_scheme != ELSI_GPU_OCC_EXPLICIT)
            occupations(st, n, w, nullptr, h->occ_scheme, h->n_electron, h->kT, h->spin, h->occ_accuracy,
                        h->mu_max_steps, kFCut, f, scal);
        else
            explicit_occupations(st, n, h->n_state, w, f, kFCut, scal);
        if (hipMemcpyAsync(hs, scal, 6 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return kStatusHip;
        if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
        status = (h->occ_scheme != ELSI_GPU_OCC_EXPLICIT) ? (int)hs[1] : 0;
        ks = (int)hs[2];
        return 0;
    };
    if ((rc = occupy())) return rc;
    tm.mark(ELSI_GPU_ST_OCC);
    int rstat = 0;
    if (mixed) {
        // refine k_s states plus guards, then take the occupations again from
        // the refined eigenvalues
        const int kp = refine_columns(n, ks);
        back_half(h, S, ws, L, tm, kp, &dc, false, (double*)(ws + L.hcopy));
        rstat = refine_states(h, H, ws, L, tm, kp, ks, f, dc.q1t);   // each state weighted by its occupation
        if (rstat && rstat != kStatusRefine) { tm.finish(&h->info); return rstat; }
        if ((rc = occupy())) return rc;
        ks = std::min(ks, kp);
        tm.mark(ELSI_GPU_ST_OCC);
        back_substitute(h, S, ws, L, tm, ks);
    } else {
        back_half(h, S, ws, L, tm, ks, &dc);
    }
    density_matrix(st, n, ks, (double*)(ws + L.z), n, f, (double*)(ws + L.z2), (double*)(ws + L.u), D, n);
    tm.mark(ELSI_GPU_ST_DENSITY);
    if (eval) (void)hipMemcpyAsync(eval, w, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    rc = sync_status(st);
    if (rc) return rc;
    tm.finish(&h->info);
    harvest_launch_probe(h);
    *energy = hs[3];
    if (mu) *mu = hs[0];
    h->info.mu = hs[0];
    h->info.energy = hs[3];
    h->info.k_s = ks;
    h->info.mu_steps = (int)hs[4];
    h->info.charge_residual = hs[5];
    rc = read_flags(st, ws, L);
    if (rc) return rc;
    return status ? status : rstat;
}


// ---------------------------------------------------------------------------
// complex Hermitian pencils: the real 2n x 2n image (complex.hip) through the
// real drivers, results read back
// ---------------------------------------------------------------------------
static elsi_gpu_handle_s inner_handle(const elsi_gpu_handle_s* h, int n_state2)
{
    elsi_gpu_handle_s r;
    r.dtype = ELSI_GPU_REAL64;
    r.n = 2 * h->n;
    r.n_state = n_state2;
    r.n_electron = 2.0 * h->n_electron;   // every level appears twice
    r.stream = h->stream;
    r.occ_scheme = h->occ_scheme;
    r.kT = h->kT;
    r.occ_accuracy = 2.0 * h->occ_accuracy;
    r.mu_max_steps = h->mu_max_steps;
    r.spin = h->spin;
    r.overlap_is_unit = h->overlap_is_unit;
    r.overlap_factored = h->overlap_factored;
    r.band_width = h->band_width;
    r.batch_workers = 1;
    r.precision = h->precision;
    r.refine_tol = h->refine_tol;
    r.max_refine = h->max_refine;
    r.ws = h->ws;
    r.ws_bytes = make_layout(r.n, r.band_width, r.n, r.precision == ELSI_GPU_PREC_MIXED).total;
    r.ws_owned = 0;
    r.aux_stream = h->aux_stream;   // borrowed: the outer handle releases them
    r.aux_ev[0] = h->aux_ev[0];
    r.aux_ev[1] = h->aux_ev[1];
    std::memset(&r.info, 0, sizeof(r.info));
    r.info.n_basis = r.n;
    return r;
}

static void complex_info(elsi_gpu_handle_s* h, const elsi_gpu_handle_s& r)
{
    h->info = r.info;
    h->info.n_basis = h->n;
    h->info.k_s = (r.info.k_s + 1) / 2;
    h->info.fail_col = (r.info.fail_col + 1) / 2;   // real pivot 2j+1 or 2j+2 -> complex column j+1
    h->info.energy = 0.5 * r.info.energy;
    h->info.charge_residual = 0.5 * r.info.charge_residual;
}

static int ev_complex(elsi_gpu_handle_s* h, double* H, double* S, double* eval, double* evec)
{
    if (!H) return -2;
    if (!S && !h->overlap_is_unit) return -3;
    if (!eval) return -4;
    if (!evec) return -5;
    int rc = ensure_workspace(h);
    if (rc) return rc < 0 ? -1 : rc;
    hipStream_t st = h->stream;
    const int n = h->n, n2 = 2 * n, k = h->n_state, k2 = std::min(n2, 2 * k);
    char* ws = (char*)h->ws;
    const Layout L = make_layout(n2, h->band_width, n2);
    const CLayout C = make_clayout(L.total, n);
    double* H2 = (double*)(ws + C.h2);
    double* S2 = h->overlap_is_unit ? nullptr : (double*)(ws + C.s2);
    double* U = (double*)(ws + C.x2);
    embed_complex(st, n, H, n, H2, n2, false);
    if (S2) embed_complex(st, n, S, n, S2, n2, h->overlap_factored != 0);
    elsi_gpu_handle_s r = inner_handle(h, k2);
    r.precision = ELSI_GPU_PREC_FP64;   // complex eigenvectors are computed in FP64
    r.info.band_width = std::min(r.band_width, std::max(1, n2 - 1));
    Timer tm(st);
    DcState dc;
    rc = front_half(&r, H2, S2, ws, L, tm, &dc, true);
    if (rc) {
        tm.finish(&r.info);
        complex_info(h, r);
        return rc;
    }
    back_half(&r, S2, ws, L, tm, k2, &dc, false);   // standard-form vectors, n2 x k2, in ws + L.z
    std::vector<double> w2(n2);
    if (hipMemcpyAsync(w2.data(), ws + L.w, sizeof(double) * n2, hipMemcpyDeviceToHost, st) != hipSuccess)
        return kStatusHip;
    if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;
    rc = select_complex_states(st, n, k, w2.data(), (const double*)(ws + L.z), n2, k2, U, n2, (int*)(ws + C.idx));
    if (rc) return rc;
    // the standard-form vectors X are consumed: their buffers serve as scratch
    orthonormalize_complex_images(st, n, k, U, n2, (double*)(ws + L.z), (double*)(ws + L.z2));
    if (S2) {
        double* Linv = (double*)(ws + L.linv);
        dtrtri_diag_blocks(st, n2, S2, n2, Linv);
        dtrsm_left_lower_t(st, n2, k, S2, n2, Linv, U, n2);
    }
    tm.mark(ELSI_GPU_ST_BACKSUB);
    extract_vectors(st, n, k, U, n2, evec, n);
    pair_values(st, n, (const double*)(ws + L.w), eval);
    if (S2 && !h->overlap_factored) extract_complex(st, n, S2, n2, S, n, true);
    rc = sync_status(st);
    if (rc) return rc;
    tm.finish(&r.info);
    harvest_launch_probe(&r);
    complex_info(h, r);
    return read_flags(st, ws, L);
}

static int dm_complex(elsi_gpu_handle_s* h, double* H, double* S, double* occ, double* D, double* eval,
                      double* energy, double* mu)
{
    if (!H) return -2;
    if (!S && !h->overlap_is_unit) return -3;
    if (!occ && h->occ_scheme == ELSI_GPU_OCC_EXPLICIT) return -4;
    if (!D) return -5;
    if (!energy) return -7;
    int rc = ensure_workspace(h);
    if (rc) return rc < 0 ? -1 : rc;
    hipStream_t st = h->stream;
    const int n = h->n, n2 = 2 * n;
    char* ws = (char*)h->ws;
    const Layout L = make_layout(n2, h->band_width, n2, h->precision == ELSI_GPU_PREC_MIXED);
    const CLayout C = make_clayout(L.total, n);
    double* H2 = (double*)(ws + C.h2);
    double* S2 = h->overlap_is_unit ? nullptr : (double*)(ws + C.s2);
    double* D2 = (double*)(ws + C.x2);
    double* occ2 = nullptr;
    embed_complex(st, n, H, n, H2, n2, false);
    if (S2) embed_complex(st, n, S, n, S2, n2, h->overlap_factored != 0);
    if (h->occ_scheme == ELSI_GPU_OCC_EXPLICIT) {
        occ2 = (double*)(ws + C.f2);
        duplicate_values(st, h->n_state, occ, occ2);
    }
    elsi_gpu_handle_s r = inner_handle(h, 2 * h->n_state);
    double e2 = 0.0, mu2 = 0.0;
    const int rc2 = dm_real(&r, H2, S2, occ2, D2, nullptr, &e2, &mu2);
    complex_info(h, r);
    if (rc2 != 0 && rc2 != ELSI_GPU_ERR_MU && rc2 != ELSI_GPU_ERR_REFINE) return rc2;
    extract_complex(st, n, D2, n2, D, n, false);
    if (eval) pair_values(st, n, (const double*)(ws + L.w), eval);
    // Fermi-Dirac occupations of the states: the mean over each real pair
    if (occ && h->occ_scheme != ELSI_GPU_OCC_EXPLICIT) pair_values(st, n, (const double*)(ws + L.f), occ);
    if (S2 && !h->overlap_factored) extract_complex(st, n, S2, n2, S, n, true);
    rc = sync_status(st);
    if (rc) return rc;
    *energy = 0.5 * e2;
    if (mu) *mu = mu2;
    h->info.mu = mu2;
    return rc2;
}

// All n eigenvalues of the pencil (ascending), with H and S only read: the
// steps up to divide and conquer run on copies (real handles; the handle must
// carry values_copies for the workspace), or on the real image (complex
// handles, R8: each value the mean of its pair).
int eg::eigenvalues_only(elsi_gpu_handle_s* h, const double* H, const double* S, double* eval)
{
    if (!H) return -2;
    if (!S && !h->overlap_is_unit) return -3;
    if (!eval) return -4;
    int rc = ensure_workspace(h);
    if (rc) return rc < 0 ? -1 : rc;
    hipStream_t st = h->stream;
    const int n = h->n;
    char* ws = (char*)h->ws;
    std::memset(h->info.stage_ms, 0, sizeof(h->info.stage_ms));
    h->info.fail_col = 0;
    if (h->dtype == ELSI_GPU_COMPLEX128) {
        const int n2 = 2 * n;
        const Layout L = make_layout(n2, h->band_width, n2);
        const CLayout C = make_clayout(L.total, n);
        double* H2 = (double*)(ws + C.h2);
        double* S2 = h->overlap_is_unit ? nullptr : (double*)(ws + C.s2);
        embed_complex(st, n, H, n, H2, n2, false);
        if (S2) embed_complex(st, n, S, n, S2, n2, h->overlap_factored != 0);
        elsi_gpu_handle_s r = inner_handle(h, n2);
        r.precision = ELSI_GPU_PREC_FP64;
        r.info.band_width = std::min(r.band_width, std::max(1, n2 - 1));
        Timer tm(st);
        DcState dc;
        rc = front_half(&r, H2, S2, ws, L, tm, &dc, false);
        tm.finish(&r.info);
        complex_info(h, r);
        if (rc) return rc;
        pair_values(st, n, (const double*)(ws + L.w), eval);
        rc = sync_status(st);
        if (rc) return rc;
        return read_flags(st, ws, L);
    }
    const Layout L = make_layout(n, h->band_width, n, false, true);
    double* Hc = (double*)(ws + L.hv);
    double* Sc = h->overlap_is_unit ? nullptr : (double*)(ws + L.sv);
    copy_matrix(st, n, n, H, n, Hc, n);
    if (Sc) copy_matrix(st, n, n, S, n, Sc, n);
    h->info.band_width = std::min(h->band_width, std::max(1, n - 1));
    Timer tm(st);
    DcState dc;
    rc = front_half(h, Hc, Sc, ws, L, tm, &dc, false);
    tm.finish(&h->info);
    if (rc) return rc;
    (void)hipMemcpyAsync(eval, ws + L.w, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    rc = sync_status(st);
    if (rc) return rc;
    return read_flags(st, ws, L);
}

// ---------------------------------------------------------------------------
// Singularity check of the overlap and the eigendecomposition transform
// (Sec. 4.5, Eq. (20)): when S has an eigenvalue below tau, S = x lam x^T =
// X X^T replaces the Cholesky factor, and only the m = N_nonsing eigenvectors
// with lam >= tau are kept: Y = x_keep lam_keep^(-1/2) (n x m), the standard
// problem H~ = Y^T H Y of size m is solved, and c = Y c~.
// ---------------------------------------------------------------------------
namespace {

__global__ void scale_cols_kernel(int n, int m, const double* A, int lda, const double* v, int first, int mode,
                                  double* B, int ldb)
{
    // mode 0: B(:, j) = A(:, first + j) / sqrt(v[first + j]);  mode 1: times sqrt;
    // mode 2: B(:, j) = A(:, j) / v[j]
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n || j >= m) return;
    if (mode == 2) {
        B[cm(i, j, ldb)] = A[cm(i, j, lda)] / v[j];
        return;
    }
    const double s = sqrt(v[first + j]);
    B[cm(i, j, ldb)] = (mode == 0) ? A[cm(i, first + j, lda)] / s : A[cm(i, first + j, lda)] * s;
}

__global__ void col_sqnorm_kernel(int n, const double* A, int lda, double* out)
{
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += A[cm(i, j, lda)] * A[cm(i, j, lda)];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

// A sub-handle for a standard (S = I) problem of size m on the caller's stream,
// with the caller's occupation settings.
int standard_subhandle(const elsi_gpu_handle_s* h, int m, int n_state, elsi_gpu_handle* out)
{
    int rc = elsi_gpu_init(out, ELSI_GPU_REAL64, m, n_state, std::min(h->n_electron, (double)m * h->spin), h->stream);
    if (rc) return rc > 0 ? rc : kStatusHip;
    (*out)->overlap_is_unit = 1;
    (*out)->occ_scheme = h->occ_scheme;
    (*out)->kT = h->kT;
    (*out)->occ_accuracy = h->occ_accuracy;
    (*out)->mu_max_steps = h->mu_max_steps;
    (*out)->spin = h->spin;
    (*out)->band_width = h->band_width;
    return 0;
}

struct SubHandle {
    elsi_gpu_handle h = nullptr;
    ~SubHandle() { if (h) elsi_gpu_finalize(&h); }
};

// Decide the route and, for the eigendecomposition one, build Y (n x m).
// Returns 0 with *m = 0 for the Cholesky route, 0 with *m > 0 and Y filled,
// or an error.  S is overwritten by X on the eigendecomposition route.
int overlap_transform(elsi_gpu_handle_s* h, double* S, DevBuf<double>& Y, int* m_out)
{
    hipStream_t st = h->stream;
    const int n = h->n;
    *m_out = 0;
    if (h->overlap_factored) {
        const int m = h->sing_m;
        if (m <= 0) return 0;   // S holds L
        // S holds X (n x m): lam_j = ||X_j||^2, Y_j = X_j / lam_j
        DevBuf<double> lam;
        if (!Y.alloc((size_t)n * m) || !lam.alloc(m)) return kStatusOom;
        hipLaunchKernelGGL(col_sqnorm_kernel, dim3(m), dim3(256), 0, st, n, S, n, lam.p);
        hipLaunchKernelGGL(scale_cols_kernel, dim3(ceil_div(n, 256), m), dim3(256), 0, st, n, m, S, n, lam.p, 0, 2,
                           Y.p, n);
        *m_out = m;
        return sync_status(st);
    }
    if (!h->sing_check) {
        h->sing_m = 0;
        return 0;
    }
    // all eigenvalues of S, by the library's own path with S as a standard matrix
    DevBuf<double> Sc, lam, xv;
    if (!Sc.alloc((size_t)n * n) || !lam.alloc(n) || !xv.alloc((size_t)n * n)) return kStatusOom;
    copy_matrix(st, n, n, S, n, Sc.p, n);
    SubHandle sub;
    int rc = standard_subhandle(h, n, n, &sub.h);
    if (rc) return rc;
    rc = elsi_gpu_ev(sub.h, Sc.p, nullptr, lam.p, xv.p);
    if (rc) return rc;
    std::vector<double> hl((size_t)n);
    if (hipMemcpyAsync(hl.data(), lam.p, sizeof(double) * n, hipMemcpyDeviceToHost, st) != hipSuccess)
        return kStatusHip;
    rc = sync_status(st);
    if (rc) return rc;
    h->info.overlap_min_eig = hl[0];
    if (hl[0] >= h->sing_tol) {   // not singular: the Cholesky route
        h->sing_m = 0;
        return 0;
    }
    int m = 0;
    for (int l = 0; l < n; ++l) m += (hl[l] >= h->sing_tol) ? 1 : 0;
    if (m == 0) return kStatusNotPD;
    const int first = n - m;
    if (!Y.alloc((size_t)n * m)) return kStatusOom;
    hipLaunchKernelGGL(scale_cols_kernel, dim3(ceil_div(n, 256), m), dim3(256), 0, st, n, m, xv.p, n, lam.p, first, 0,
                       Y.p, n);
    // S <- X = x_keep lam_keep^(1/2), the remaining columns zero
    fill_d(st, S, (size_t)n * n, 0.0);
    hipLaunchKernelGGL(scale_cols_kernel, dim3(ceil_div(n, 256), m), dim3(256), 0, st, n, m, xv.p, n, lam.p, first, 1,
                       S, n);
    h->sing_m = m;
    *m_out = m;
    return sync_status(st);
}

// H~ = Y^T H Y (m x m, full) into Ht; H symmetric, lower triangle read.
void transform_h(hipStream_t st, int n, int m, const double* H, const double* Y, double* W, double* Ht)
{
    dgemm(st, 'S', 'N', n, m, n, 1.0, H, n, Y, n, 0.0, W, n);
    dgemm(st, 'T', 'N', m, m, n, 1.0, Y, n, W, n, 0.0, Ht, m);
    symmetrize_average(st, m, Ht, m);
}

int ev_singular(elsi_gpu_handle_s* h, double* H, const DevBuf<double>& Y, int m, double* eval, double* evec)
{
    hipStream_t st = h->stream;
    const int n = h->n, k = h->n_state, km = std::min(k, m);
    DevBuf<double> W, Ht, Ct;
    if (!W.alloc((size_t)n * m) || !Ht.alloc((size_t)m * m) || !Ct.alloc((size_t)m * km)) return kStatusOom;
    transform_h(st, n, m, H, Y.p, W.p, Ht.p);
    SubHandle sub;
    int rc = standard_subhandle(h, m, km, &sub.h);
    if (rc) return rc;
    rc = elsi_gpu_ev(sub.h, Ht.p, nullptr, W.p, Ct.p);   // eigenvalues into W (m doubles)
    if (rc) return rc;
    (void)hipMemcpyAsync(eval, W.p, sizeof(double) * m, hipMemcpyDeviceToDevice, st);
    if (m < n) fill_d(st, eval + m, (size_t)(n - m), HUGE_VAL);
    dgemm(st, 'N', 'N', n, km, m, 1.0, Y.p, n, Ct.p, m, 0.0, evec, n);   // c = Y c~
    if (km < k) fill_d(st, evec + (size_t)n * km, (size_t)n * (k - km), 0.0);
    h->info.n_nonsing = m;
    return sync_status(st);
}

int dm_singular(elsi_gpu_handle_s* h, double* H, const DevBuf<double>& Y, int m, double* occ, double* D, double* eval,
                double* energy, double* mu)
{
    hipStream_t st = h->stream;
    const int n = h->n;
    DevBuf<double> W, Ht, Dt, ev, f, T1;
    if (!W.alloc((size_t)n * m) || !Ht.alloc((size_t)m * m) || !Dt.alloc((size_t)m * m) || !ev.alloc(m) ||
        !f.alloc(m) || !T1.alloc((size_t)m * n))
        return kStatusOom;
    transform_h(st, n, m, H, Y.p, W.p, Ht.p);
    SubHandle sub;
    int rc = standard_subhandle(h, m, m, &sub.h);
    if (rc) return rc;
    const bool explicit_occ = h->occ_scheme == ELSI_GPU_OCC_EXPLICIT;
    if (explicit_occ) (void)hipMemcpyAsync(f.p, occ, sizeof(double) * m, hipMemcpyDeviceToDevice, st);
    double e = 0.0, mm = 0.0;
    const int rcd = elsi_gpu_dm(sub.h, Ht.p, nullptr, f.p, Dt.p, ev.p, &e, &mm);
    if (rcd != 0 && rcd != ELSI_GPU_ERR_MU) return rcd;
    // D = Y D~ Y^T: T1 = D~ Y^T, then the lower tiles of Y T1, mirrored
    dgemm(st, 'N', 'T', m, n, m, 1.0, Dt.p, m, Y.p, n, 0.0, T1.p, m);
    dgemm(st, 'N', 'N', n, n, m, 1.0, Y.p, n, T1.p, m, 0.0, D, n, 1);
    mirror_lower_to_upper(st, n, D, n);
    if (eval) {
        (void)hipMemcpyAsync(eval, ev.p, sizeof(double) * m, hipMemcpyDeviceToDevice, st);
        if (m < n) fill_d(st, eval + m, (size_t)(n - m), HUGE_VAL);
    }
    if (occ && !explicit_occ) {
        (void)hipMemcpyAsync(occ, f.p, sizeof(double) * m, hipMemcpyDeviceToDevice, st);
        if (m < n) fill_d(st, occ + m, (size_t)(n - m), 0.0);
    }
    elsi_gpu_info sinfo;
    elsi_gpu_get_info(sub.h, &sinfo);
    h->info.mu = sinfo.mu;
    h->info.energy = sinfo.energy;
    h->info.k_s = sinfo.k_s;
    h->info.mu_steps = sinfo.mu_steps;
    h->info.charge_residual = sinfo.charge_residual;
    h->info.n_nonsing = m;
    *energy = e;
    if (mu) *mu = mm;
    rc = sync_status(st);
    return rc ? rc : rcd;
}

}  // namespace

extern "C" {

int elsi_gpu_ev(elsi_gpu_handle h, double* H, double* S, double* eval, double* evec)
{
    if (!h) return -1;
    if (h->dtype == ELSI_GPU_COMPLEX128) return ev_complex(h, H, S, eval, evec);
    h->info.n_nonsing = h->n;
    h->info.overlap_min_eig = 0.0;
    if (!h->overlap_is_unit && S && (h->sing_check || (h->overlap_factored && h->sing_m > 0))) {
        if (!H) return -2;
        if (!eval) return -4;
        if (!evec) return -5;
        DevBuf<double> Y;
        int m = 0;
        const int rc = overlap_transform(h, S, Y, &m);
        if (rc) return rc;
        if (m > 0) return ev_singular(h, H, Y, m, eval, evec);
    }
    return ev_real(h, H, S, eval, evec);
}

int elsi_gpu_dm(elsi_gpu_handle h, double* H, double* S, double* occ, double* D, double* eval, double* energy,
                double* mu)
{
    if (!h) return -1;
    if (h->dtype == ELSI_GPU_COMPLEX128) return dm_complex(h, H, S, occ, D, eval, energy, mu);
    h->info.n_nonsing = h->n;
    h->info.overlap_min_eig = 0.0;
    if (!h->overlap_is_unit && S && (h->sing_check || (h->overlap_factored && h->sing_m > 0))) {
        if (!H) return -2;
        if (!occ && h->occ_scheme == ELSI_GPU_OCC_EXPLICIT) return -4;
        if (!D) return -5;
        if (!energy) return -7;
        DevBuf<double> Y;
        int m = 0;
        const int rc = overlap_transform(h, S, Y, &m);
        if (rc) return rc;
        if (m > 0) return dm_singular(h, H, Y, m, occ, D, eval, energy, mu);
    }
    return dm_real(h, H, S, occ, D, eval, energy, mu);
}

}  // extern "C"
