// Many independent eigenproblems in one call (ELSI paper, Sec. 4.3: k-points
// and spin channels are independent problems that ELSI distributes over
// process groups; here they share one GPU).
//
// A pool of host worker threads, each with its own non-blocking stream and its
// own workspace, takes problems largest first (longest-processing-time order)
// and runs the single-problem driver on them, so that the many small kernels of
// small problems overlap on the device.  The panel factorization of step (1)
// takes its per-column path there (kernels that never wait on each other).
//
// Kernels whose workgroups wait on each other pass a gate while a batch is
// active.  The runtime runs cooperative launches one at a time across all
// streams, which would put every problem's bulge chasing in one line, so a
// kernel with at least three workgroups per compute unit takes an ordinary
// launch instead and the gate keeps it fully resident.  The argument: the
// workgroups of a launch go to the XCDs in turn, so an XCD of C compute units
// receives at most ceil(w / X) of a kernel's w workgroups (X XCDs), each using
// at most 1/p <= 1/3 of every resource of a compute unit.  With the admitted
// kernels' shares summing to at most half of the device and at most C / 2 of
// them admitted, an XCD carries less than C/2 + (C/2)(1/3) = 2C/3 compute
// units' worth of waiting workgroups, so one of its compute units is loaded to
// at most 2/3 and takes the next one as soon as the kernels that do not wait
// (which always finish) have left.  Every wait in those kernels is bounded
// as well: an expired wait sets the kernel's error flag instead of hanging.
#include "api_internal.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdint>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

namespace eg {
namespace {

std::atomic<int> g_batch_depth{0};
std::mutex g_persistent_mu;
std::condition_variable g_persistent_cv;
constexpr long long kDevice = 1LL << 30;   // the whole device, in share units
long long g_persistent_used = 0;           // shares of the admitted kernels
int g_persistent_kernels = 0;              // admitted kernels

struct BatchDepth {
    BatchDepth() { g_batch_depth.fetch_add(1); }
    ~BatchDepth() { g_batch_depth.fetch_sub(1); }
};

// Worker-local copy of the caller's handle: settings shared, stream and
// workspace private (the band width is set per problem).
elsi_gpu_handle_s worker_handle(const elsi_gpu_handle_s* proto, hipStream_t st)
{
    elsi_gpu_handle_s w;
    w.dtype = proto->dtype;
    w.occ_scheme = proto->occ_scheme;
    w.kT = proto->kT;
    w.occ_accuracy = proto->occ_accuracy;
    w.mu_max_steps = proto->mu_max_steps;
    w.spin = proto->spin;
    w.overlap_is_unit = proto->overlap_is_unit;
    w.overlap_factored = proto->overlap_factored;
    w.band_width = proto->band_width;
    w.batch_workers = 1;
    w.stream = st;
    std::memset(&w.info, 0, sizeof(w.info));
    return w;
}

// Band width of a problem of size n in a batched call: the first table entry
// that covers n, else the handle's own.
int batch_band(const elsi_gpu_handle_s* h, int n)
{
    for (int i = 0; i < h->band_tab_count; ++i)
        if (n <= h->band_tab_nmax[i]) return h->band_tab_b[i];
    return h->band_width;
}

// Run fn(worker handle, problem index) over all problems with the pool.
template <typename Fn>
int run_pool(elsi_gpu_handle_s* h, int count, const int* n, int* status, Fn fn)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kStatusHip;
    // the caller's inputs must be complete before other streams read them
    if (hipStreamSynchronize(h->stream) != hipSuccess) return kStatusHip;
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
    std::atomic<int> next{0};
    const int nworkers = std::max(1, std::min(h->batch_workers, count));
    BatchDepth depth;
    auto work = [&]() {
        (void)hipSetDevice(dev);
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (int q = next.fetch_add(1); q < count; q = next.fetch_add(1)) status[order[q]] = kStatusHip;
            return;
        }
        elsi_gpu_handle_s w = worker_handle(h, st);
        for (int q = next.fetch_add(1); q < count; q = next.fetch_add(1)) status[order[q]] = fn(&w, order[q]);
        release_workspace(&w);
        (void)hipStreamDestroy(st);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nworkers; ++t) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    for (int p = 0; p < count; ++p)
        if (status[p] != 0) return status[p];
    return 0;
}

}  // namespace

bool batch_mode_active() { return g_batch_depth.load(std::memory_order_relaxed) > 0; }

namespace {
// compute units of the current device, and per XCD
void device_cus(int& cus, int& per_xcd)
{
    int dev = 0, xcds = 0;
    cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipDeviceGetAttribute(&xcds, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || xcds < 1) xcds = 1;
    cus = std::max(1, cus);
    per_xcd = std::max(1, cus / xcds);
}
}  // namespace

bool persistent_plain_ok(int per_cu) { return batch_mode_active() && per_cu >= 3; }

long long persistent_enter(int workgroups, int per_cu)
{
    if (!batch_mode_active()) return 0;
    int cus = 1, per_xcd = 1;
    device_cus(cus, per_xcd);
    const long long capacity = (long long)cus * std::max(1, per_cu);
    // a kernel with fewer than three workgroups per compute unit falls outside
    // the residency argument above and is admitted alone
    const long long share = per_cu >= 3
                                ? std::max(1LL, ((long long)workgroups * kDevice + capacity - 1) / capacity)
                                : kDevice / 2;
    const int max_kernels = std::max(1, per_xcd / 2);
    std::unique_lock<std::mutex> lk(g_persistent_mu);
    // a kernel larger than the budget is admitted alone
    g_persistent_cv.wait(lk, [&] {
        return g_persistent_kernels == 0 ||
               (g_persistent_used + share <= kDevice / 2 && g_persistent_kernels < max_kernels);
    });
    g_persistent_used += share;
    ++g_persistent_kernels;
    return share;
}

void persistent_leave(hipStream_t st, long long share)
{
    if (share == 0) return;
    (void)hipStreamSynchronize(st);
    {
        std::lock_guard<std::mutex> lk(g_persistent_mu);
        g_persistent_used -= share;
        --g_persistent_kernels;
    }
    g_persistent_cv.notify_all();
}

}  // namespace eg

using namespace eg;

extern "C" {

int elsi_gpu_set_batch_workers(elsi_gpu_handle h, int workers)
{
    if (!h) return -1;
    if (workers < 1 || workers > 16) return -2;
    h->batch_workers = workers;
    return 0;
}

int elsi_gpu_set_batch_band_table(elsi_gpu_handle h, int count, const int* n_max, const int* b)
{
    if (!h) return -1;
    if (count < 0 || count > 16) return -2;
    if (count > 0 && !n_max) return -3;
    if (count > 0 && !b) return -4;
    for (int i = 0; i < count; ++i) {
        if (n_max[i] < 1 || (i > 0 && n_max[i] <= n_max[i - 1])) return -3;
        if (b[i] < 8 || b[i] > 64 || b[i] % 8 != 0) return -4;
    }
    for (int i = 0; i < count; ++i) {
        h->band_tab_nmax[i] = n_max[i];
        h->band_tab_b[i] = b[i];
    }
    h->band_tab_count = count;
    return 0;
}

int elsi_gpu_ev_batched(elsi_gpu_handle h, int count, const int* n, const int* n_state, double* const* H,
                        double* const* S, double* const* eval, double* const* evec, int* status)
{
    if (!h) return -1;
    if (count < 0) return -2;
    if (count == 0) return 0;
    if (!n) return -3;
    if (!n_state) return -4;
    if (!H) return -5;
    if (!S && !h->overlap_is_unit) return -6;
    if (!eval) return -7;
    if (!evec) return -8;
    if (!status) return -9;
    for (int p = 0; p < count; ++p)
        if (n[p] < 1 || n_state[p] < 1 || n_state[p] > n[p] || !H[p] || (!h->overlap_is_unit && !S[p]) ||
            !eval[p] || !evec[p])
            return -3;
    return run_pool(h, count, n, status, [&](elsi_gpu_handle_s* w, int p) {
        w->n = n[p];
        w->band_width = batch_band(h, n[p]);
        w->n_state = n_state[p];
        w->n_electron = 0.0;
        return elsi_gpu_ev(w, H[p], S ? S[p] : nullptr, eval[p], evec[p]);
    });
}

int elsi_gpu_dm_batched(elsi_gpu_handle h, int count, const int* n, const double* n_electron,
                        const double* kweight, double* const* H, double* const* S, double* const* D,
                        double* const* eval, double* energy, double* mu, int* status)
{
    if (!h) return -1;
    if (h->occ_scheme == ELSI_GPU_OCC_EXPLICIT) return -1;
    if (count < 0) return -2;
    if (count == 0) return 0;
    if (!n) return -3;
    if (!n_electron) return -4;
    if (!H) return -6;
    if (!S && !h->overlap_is_unit) return -7;
    if (!D) return -8;
    if (!energy) return -10;
    if (!status) return -12;
    for (int p = 0; p < count; ++p)
        if (n[p] < 1 || !(n_electron[p] >= 0.0) || n_electron[p] > 2.0 * n[p] || !H[p] ||
            (!h->overlap_is_unit && !S[p]) || !D[p])
            return -3;
    if (kweight)
        for (int p = 0; p < count; ++p)
            if (!(kweight[p] > 0.0)) return -5;
    if (!kweight)
        return run_pool(h, count, n, status, [&](elsi_gpu_handle_s* w, int p) {
            w->n = n[p];
            w->band_width = batch_band(h, n[p]);
            w->n_state = n[p];
            w->n_electron = n_electron[p];
            double e = 0.0, m = 0.0;
            const int rc = elsi_gpu_dm(w, H[p], S ? S[p] : nullptr, nullptr, D[p], eval ? eval[p] : nullptr, &e, &m);
            energy[p] = e;
            if (mu) mu[p] = m;
            return rc;
        });

    // One chemical potential for all problems (k-points and spin channels of
    // one system, Sec. 4.5): every problem's eigenvalues first, then mu over
    // all of them with each state weighted by its problem's weight, then each
    // problem's density matrix with those occupations fixed.
    std::vector<size_t> off((size_t)count + 1, 0);
    for (int p = 0; p < count; ++p) off[p + 1] = off[p] + (size_t)n[p];
    const size_t ntot = off[count];
    if (ntot > (size_t)INT32_MAX) return -3;
    DevBuf<double> E, Wt, F, scal;
    if (!E.alloc(ntot) || !Wt.alloc(ntot) || !F.alloc(ntot) || !scal.alloc(8)) return kStatusOom;
    int rc = run_pool(h, count, n, status, [&](elsi_gpu_handle_s* w, int p) {
        w->n = n[p];
        w->band_width = batch_band(h, n[p]);
        w->n_state = n[p];
        w->values_copies = 1;
        return eigenvalues_only(w, H[p], S ? S[p] : nullptr, E.p + off[p]);
    });
    if (rc) return rc;
    hipStream_t st = h->stream;
    double ne = 0.0;
    for (int p = 0; p < count; ++p) {
        fill_d(st, Wt.p + off[p], (size_t)n[p], kweight[p]);
        ne += kweight[p] * n_electron[p];
    }
    occupations(st, (int)ntot, E.p, Wt.p, h->occ_scheme, ne, h->kT, h->spin, h->occ_accuracy, h->mu_max_steps, kFCut,
                F.p, scal.p);
    double hs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (hipMemcpyAsync(hs, scal.p, 6 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return kStatusHip;
    rc = sync_status(st);
    if (rc) return rc;
    const double mu_all = hs[0];
    const int mu_status = (int)hs[1];
    return run_pool(h, count, n, status, [&](elsi_gpu_handle_s* w, int p) {
        w->n = n[p];
        w->band_width = batch_band(h, n[p]);
        w->n_state = n[p];
        w->n_electron = n_electron[p];
        w->occ_scheme = ELSI_GPU_OCC_EXPLICIT;
        w->values_copies = 0;
        double e = 0.0, m = 0.0;
        const int r = elsi_gpu_dm(w, H[p], S ? S[p] : nullptr, F.p + off[p], D[p], eval ? eval[p] : nullptr, &e, &m);
        energy[p] = e;
        if (mu) mu[p] = mu_all;
        return r ? r : mu_status;
    });
}

}  // extern "C"
