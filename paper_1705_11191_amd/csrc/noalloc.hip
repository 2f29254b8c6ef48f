// Allocation-free variant of the Cholesky stage entry point (Eq. (10)) for
// callers that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// Its scratch -- the inverses of the 64 x 64 diagonal blocks of L and the
// first-bad-pivot flag -- lives in a file-scope device array of fixed size.
// Each device holds its own copy of the array at its own address; the host
// learns that address once per device with hipGetSymbolAddress and passes it
// to the kernels (the array's name is not a device address in host code).
// Every call on one device shares that device's array: calls that overlap on
// one device race.
#include "api_internal.h"

#include <mutex>

namespace {

constexpr int kMaxN = ELSI_GPU_NOALLOC_MAX_N;
constexpr size_t kLinvDoubles = (size_t)((kMaxN + 63) / 64) * 64 * 64;   // diagonal-block inverses
constexpr size_t kFlagOffset = kLinvDoubles * sizeof(double);             // pivot flag (one int)
constexpr size_t kScratchBytes = kFlagOffset + 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

// Device address of this device's scratch array (looked up on the first call
// on the device, with that device current).
int scratch_address(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ELSI_GPU_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return ELSI_GPU_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return ELSI_GPU_ERR_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return 0;
}

}  // namespace

using namespace eg;

extern "C" int elsi_gpu_x_cholesky_noalloc(int n, double* S, int lds, int* fail_col, void* hip_stream)
{
    if (n < 0 || n > kMaxN) return -1;
    if (n == 0) {
        if (fail_col) *fail_col = 0;
        return 0;
    }
    if (!S) return -2;
    if (lds < n) return -3;
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    double* Linv = (double*)base;
    int* info = (int*)((char*)base + kFlagOffset);
    hipStream_t st = (hipStream_t)hip_stream;
    fill_i(st, info, 1, 0);   // the previous call's flag stays in the array
    dpotrf(st, n, S, lds, Linv, info);
    int hinfo = 0;
    if (hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
        return ELSI_GPU_ERR_HIP;
    rc = sync_status(st);
    if (rc) return rc;
    if (fail_col) *fail_col = hinfo;
    return hinfo ? ELSI_GPU_ERR_NOT_PD : 0;
}
