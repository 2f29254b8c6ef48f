// Step (2) of the two-stage tridiagonalization (ELSI paper, Sec. 3.1,
// Eq. (13) and Fig. 1): T = Q2^T B Q2 by Householder bulge chasing on the
// band (successive band reduction).
//
// Storage: lower band with room for the bulge, Bd(r, c) = A(c + r, c) for
// 0 <= r < 2b (ld = 2b).  Sweep s annihilates column s below its first
// subdiagonal.  Its task 0 reflects A(s+1:s+b, s) and updates the diagonal
// block A(J0, J0) from both sides; task k >= 1 works on rows J_k = [s+1+kb,
// s+(k+1)b]: it applies the previous reflector from the right to the block
// A(J_k, J_{k-1}) (which fills it), takes a new reflector from the block's
// first column, applies it from the left to the block and from both sides to
// A(J_k, J_k).  The fill left in the other columns of the block is removed by
// the following sweeps.
//
// Parallel schedule: one workgroup per sweep, sweeps dealt round-robin to a
// grid that is entirely resident (cooperative launch).  Task k of sweep s
// touches only rows J_k(s); it overlaps task k+1 of sweep s-1 and nothing
// later, so it starts once sweep s-1 reports k+2 finished tasks.
//
// Hand-off between workgroups: the band is only ever read and written with
// device-scope (agent) relaxed atomic accesses, which are coherent across the
// XCDs without writing back or invalidating their L2 caches.  A task's stores
// complete (s_waitcnt) before the workgroup barrier, after which one lane
// publishes the progress counter; waiting lanes poll the counter with the same
// kind of access.  Every wait is bounded and an expired wait aborts the whole
// grid with an error flag.
#include "common.h"

namespace eg {
namespace {

constexpr int SB = 64;          // maximum bandwidth
constexpr int SBT = 256;        // threads per workgroup
constexpr int kDone = 0x3fffffff;

struct SbArgs {
    int n, b, ldb, nsweeps, kmax;
    double* Bd;
    double* V2;      // n x nsweeps, ld n: reflector of task (s, k) at rows J_k(s) of column s
    double* tau2;    // nsweeps x kmax
    int* progress;   // nsweeps
    int* err;
    long long spin_limit;
};

__device__ inline int ntasks(int n, int b, int s) { return (n - 2 - s) / b + 1; }

__device__ inline int ld_flag(int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_flag(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// coherent (device-scope) band accesses
__device__ inline double ldc(const double* p)
{
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void stc(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double wave_sum64(double v) { return wave_sum_dpp(v); }

// One task runs in a workgroup of 256 threads: thread (i, q) = (tid % 64,
// tid / 64) keeps entries (i, 16q .. 16q+15) of both blocks in registers.
// Band traffic uses pipelined buffer loads and stores with device-scope
// coherence (sc1), so no cache writeback or invalidate is needed at the
// hand-off; dot products along a row are 16-long register chains combined
// through LDS, and column sums are wave reductions inside each wave.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kSc1 = 16;   // cache-policy bit: device-scope coherence

__device__ inline double bld(__amdgpu_buffer_rsrc_t r, int elem)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, elem * 8, 0, kSc1));
}

__device__ inline void bst(__amdgpu_buffer_rsrc_t r, int elem, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, elem * 8, 0, kSc1);
}

__global__ __launch_bounds__(SBT) void sb2st_kernel(SbArgs a)
{
    __shared__ double LW[SB][SB + 1];      // lower triangle of the diagonal block
    __shared__ double red[4][SB];
    __shared__ double vs[SB], vps[SB], ws[SB];
    __shared__ double sh[4];
    __shared__ int abort_flag;
    const int tid = threadIdx.x;
    const int i = tid & 63, q = tid >> 6;
    const int n = a.n, b = a.b, ldb = a.ldb;
    const __amdgpu_buffer_rsrc_t band =
        __builtin_amdgcn_make_buffer_rsrc(a.Bd, (short)0, (int)((size_t)ldb * n * 8), 0x00020000);

    for (int s = blockIdx.x; s < a.nsweeps; s += gridDim.x) {
        const int nt = ntasks(n, b, s);
        double tp = 0.0;
        for (int k = 0; k < nt; ++k) {
            // ---- wait for sweep s-1 to have finished tasks 0 .. k+1
            if (tid == 0) {
                abort_flag = 0;
                if (s > 0) {
                    const int need = min(k + 2, ntasks(n, b, s - 1));
                    long long spins = 0;
                    for (;;) {
                        if (ld_flag(&a.progress[s - 1]) >= need) break;
                        if (ld_flag(a.err)) { abort_flag = 1; break; }
                        if (++spins > a.spin_limit) {
                            st_flag(a.err, 1);
                            abort_flag = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
            }
            __syncthreads();
            if (abort_flag) return;

            const int rk = s + 1 + k * b;                 // first row of J_k
            const int Lk = min(b, n - rk);
            // ---- loads: off-diagonal block row (k >= 1) and the diagonal block's lower triangle
            double ob[16], dg[16];
#pragma unroll
            for (int cq = 0; cq < 16; ++cq) {
                const int c = 16 * q + cq;
                ob[cq] = (k > 0 && i < Lk && c < b) ? bld(band, cm(b + i - c, rk - b + c, ldb)) : 0.0;
                dg[cq] = (i < Lk && c <= i) ? bld(band, cm(i - c, rk + c, ldb)) : 0.0;
            }
            double xi = 0.0;
            if (k == 0 && q == 0) xi = (i < Lk) ? bld(band, cm(1 + i, s, ldb)) : 0.0;
#pragma unroll
            for (int cq = 0; cq < 16; ++cq) LW[i][16 * q + cq] = dg[cq];
            __syncthreads();
            // full rows of the symmetric diagonal block
#pragma unroll
            for (int cq = 0; cq < 16; ++cq) {
                const int c = 16 * q + cq;
                dg[cq] = (c <= i) ? LW[i][c] : LW[c][i];
                if (c >= Lk || i >= Lk) dg[cq] = 0.0;
            }
            if (k > 0) {
                // ---- right application of the previous reflector: ob <- ob (I - tp vp vp^T)
                if (tp != 0.0) {
                    double part = 0.0;
#pragma unroll
                    for (int cq = 0; cq < 16; ++cq) part += ob[cq] * vps[16 * q + cq];
                    red[q][i] = part;
                    __syncthreads();
                    const double wr = tp * (red[0][i] + red[1][i] + red[2][i] + red[3][i]);
#pragma unroll
                    for (int cq = 0; cq < 16; ++cq) ob[cq] -= wr * vps[16 * q + cq];
                }
                if (q == 0) xi = ob[0];
            }
            // ---- Householder vector of column 0 (k >= 1) or of column s (k == 0), wave 0
            if (q == 0) {
                const double tail = wave_sum64((i >= 1 && i < Lk) ? xi * xi : 0.0);
                const double x0 = __shfl(xi, 0, 64);
                double t = 0.0, den = 1.0, alpha = x0;
                if (tail > 0.0) {
                    const double nrm = sqrt(x0 * x0 + tail);
                    alpha = (x0 >= 0.0) ? -nrm : nrm;
                    t = (alpha - x0) / alpha;
                    den = x0 - alpha;
                }
                vs[i] = (i == 0) ? 1.0 : ((i < Lk && tail > 0.0) ? xi / den : 0.0);
                if (i == 0) { sh[0] = t; sh[1] = alpha; }
            }
            __syncthreads();
            const double t = sh[0], alpha = sh[1];
            const double vi = vs[i];
            if (k == 0) {
                if (q == 0 && i < Lk) bst(band, cm(1 + i, s, ldb), (i == 0) ? alpha : 0.0);
            } else {
                // ---- left application: ob <- (I - t v v^T) ob, column sums inside each wave
                if (t != 0.0) {
#pragma unroll
                    for (int cq = 0; cq < 16; ++cq) {
                        const double uc = t * wave_sum64(vi * ob[cq]);
                        ob[cq] -= vi * uc;
                    }
                    if (q == 0) ob[0] = (i == 0) ? alpha : 0.0;
                }
#pragma unroll
                for (int cq = 0; cq < 16; ++cq) {
                    const int c = 16 * q + cq;
                    if (i < Lk && c < b) bst(band, cm(b + i - c, rk - b + c, ldb), ob[cq]);
                }
            }
            // ---- two-sided update of the diagonal block: dg <- H dg H
            if (t != 0.0) {
                double part = 0.0;
#pragma unroll
                for (int cq = 0; cq < 16; ++cq) part += dg[cq] * vs[16 * q + cq];
                red[q][i] = part;
                __syncthreads();
                const double pi = t * (red[0][i] + red[1][i] + red[2][i] + red[3][i]);
                const double beta = 0.5 * t * wave_sum64(pi * vi);
                const double wi = pi - beta * vi;
                if (q == 0) ws[i] = wi;
                __syncthreads();
#pragma unroll
                for (int cq = 0; cq < 16; ++cq) {
                    const int c = 16 * q + cq;
                    dg[cq] -= vi * ws[c] + wi * vs[c];
                }
            }
#pragma unroll
            for (int cq = 0; cq < 16; ++cq) {
                const int c = 16 * q + cq;
                if (i < Lk && c <= i) bst(band, cm(i - c, rk + c, ldb), dg[cq]);
            }
            if (q == 0 && i < Lk) a.V2[cm(rk + i, s, n)] = vi;
            if (tid == 0) a.tau2[(size_t)s * a.kmax + k] = t;
            if (q == 0) vps[i] = vi;
            tp = t;
            __builtin_amdgcn_s_waitcnt(0);   // this thread's band stores have completed
            __syncthreads();
            if (tid == 0) st_flag(&a.progress[s], (k + 1 == nt) ? kDone : k + 1);
        }
    }
}

__global__ void extract_tridiag_kernel(int n, const double* Bd, int ldb, double* d, double* e)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    d[i] = Bd[cm(0, i, ldb)];
    if (i + 1 < n) e[i] = Bd[cm(1, i, ldb)];
}

}  // namespace

int sb2st_kmax(int n, int b) { return n >= 2 ? (n - 2) / b + 1 : 1; }

// Bd (ldb = 2b) -> (d, e); reflectors into V2 (n x n, ld n) and tau2
// (nsweeps x kmax).  progress: n ints of scratch.  Returns 0, or 2 when a
// wait expired (the grid was aborted).
int sb2st(hipStream_t st, int n, int b, double* Bd, int ldb, double* d, double* e, double* V2, double* tau2,
          int* progress, int* err)
{
    const int nsweeps = n - 2;
    fill_i(st, err, 1, 0);
    if (nsweeps > 0) {
        fill_i(st, progress, (size_t)nsweeps, 0);
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sb2st_kernel, SBT, 0);
        int resident = std::max(1, cus * std::max(1, per_cu));
        // sweep s starts two tasks after sweep s-1, so a workgroup that takes
        // sweep s + grid after finishing sweep s (ntasks(0) tasks) never holds the
        // pipeline back once grid >= ntasks(0) / 2; a few spare workgroups absorb
        // uneven timing
        const int need = ((n - 2) / b + 1) / 2 + 8;
        int grid = std::min(nsweeps, std::min(std::min(resident, cus > 0 ? cus : 1), need));
        SbArgs a;
        a.n = n; a.b = b; a.ldb = ldb; a.nsweeps = nsweeps; a.kmax = sb2st_kmax(n, b);
        a.Bd = Bd; a.V2 = V2; a.tau2 = tau2; a.progress = progress; a.err = err;
        a.spin_limit = 1LL << 22;
        void* args[] = {&a};
        const bool gated = persistent_enter(grid, resident);
        hipError_t rc = hipLaunchCooperativeKernel((const void*)sb2st_kernel, dim3(grid), dim3(SBT), args, 0, st);
        persistent_leave(st, gated, grid);
        if (rc != hipSuccess) return kStatusHip;
    }
    hipLaunchKernelGGL(extract_tridiag_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, Bd, ldb, d, e);
    return 0;
}

}  // namespace eg
