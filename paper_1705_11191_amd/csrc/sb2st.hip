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
// later, so it starts once sweep s-1 reports k+2 finished tasks.  Progress
// counters are published with agent-scope release and read with acquire; every
// wait is bounded and an expired wait aborts the whole grid with an error flag.
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

__device__ inline int load_acquire(int* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void store_release(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Householder vector of x (length L in xs[0..L)): on exit v in vs (v0 = 1),
// returns tau, writes alpha.  tail == 0 gives tau = 0, v = e0.
__device__ void house(int L, const double* xs, double* vs, double* sh, int tid)
{
    if (tid == 0) {
        double x0 = xs[0], tail = 0.0;
        for (int i = 1; i < L; ++i) tail += xs[i] * xs[i];
        double t = 0.0, alpha = x0, den = 1.0;
        if (tail > 0.0) {
            double nrm = sqrt(x0 * x0 + tail);
            alpha = (x0 >= 0.0) ? -nrm : nrm;
            t = (alpha - x0) / alpha;
            den = x0 - alpha;
        }
        sh[0] = t;
        sh[1] = alpha;
        sh[2] = (tail > 0.0) ? 1.0 / den : 0.0;
    }
    __syncthreads();
    double inv = sh[2];
    for (int i = tid; i < SB; i += SBT) vs[i] = (i == 0) ? 1.0 : ((i < L) ? xs[i] * inv : 0.0);
    __syncthreads();
}

// DG <- H DG H for the symmetric L x L block in LDS, H = I - t v v^T.
__device__ void two_sided(int L, double (*DG)[SB + 1], const double* v, double t, double* p, double* sh,
                          int tid)
{
    if (t == 0.0) return;
    if (tid < L) {
        double s = 0.0;
        for (int j = 0; j < L; ++j) s += DG[tid][j] * v[j];
        p[tid] = t * s;
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < L; ++i) s += p[i] * v[i];
        sh[3] = 0.5 * t * s;
    }
    __syncthreads();
    double beta = sh[3];
    if (tid < L) p[tid] -= beta * v[tid];   // p is now w
    __syncthreads();
    for (int e = tid; e < L * L; e += SBT) {
        int i = e % L, j = e / L;
        DG[i][j] -= v[i] * p[j] + p[i] * v[j];
    }
    __syncthreads();
}

__global__ __launch_bounds__(SBT) void sb2st_kernel(SbArgs a)
{
    __shared__ double DG[SB][SB + 1];
    __shared__ double OB[SB][SB + 1];
    __shared__ double v[SB], vp[SB], xs[SB], p[SB], u[SB];
    __shared__ double sh[8];
    __shared__ int abort_flag;
    const int tid = threadIdx.x;
    const int n = a.n, b = a.b, ldb = a.ldb;
    double* Bd = a.Bd;

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
                        int pr = load_acquire(&a.progress[s - 1]);
                        if (pr >= need) break;
                        if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            abort_flag = 1;
                            break;
                        }
                        if (++spins > a.spin_limit) {
                            __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            abort_flag = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            }
            __syncthreads();
            if (abort_flag) return;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

            const int rk = s + 1 + k * b;                 // first row of J_k
            const int Lk = min(b, n - rk);
            double t = 0.0;
            if (k == 0) {
                // column s, rows J0
                for (int i = tid; i < Lk; i += SBT) xs[i] = Bd[cm(1 + i, s, ldb)];
                for (int e = tid; e < SB * SB; e += SBT) {
                    int i = e % SB, c = e / SB;
                    if (i < Lk && c < Lk && i >= c) {
                        double val = Bd[cm(i - c, rk + c, ldb)];
                        DG[i][c] = val;
                        DG[c][i] = val;
                    }
                }
                __syncthreads();
                house(Lk, xs, v, sh, tid);
                t = sh[0];
                const double alpha = sh[1];
                for (int i = tid; i < Lk; i += SBT) Bd[cm(1 + i, s, ldb)] = (i == 0) ? alpha : 0.0;
                two_sided(Lk, DG, v, t, p, sh, tid);
            } else {
                // block A(J_k, J_{k-1}): rows rk + i, columns rk - b + c
                for (int e = tid; e < SB * SB; e += SBT) {
                    int i = e % SB, c = e / SB;
                    if (i < Lk && c < b) OB[i][c] = Bd[cm(b + i - c, rk - b + c, ldb)];
                    if (i < Lk && c < Lk && i >= c) {
                        double val = Bd[cm(i - c, rk + c, ldb)];
                        DG[i][c] = val;
                        DG[c][i] = val;
                    }
                }
                __syncthreads();
                // right application of the previous reflector: OB <- OB (I - tp vp vp^T)
                if (tp != 0.0) {
                    if (tid < Lk) {
                        double s2 = 0.0;
                        for (int c = 0; c < b; ++c) s2 += OB[tid][c] * vp[c];
                        p[tid] = tp * s2;
                    }
                    __syncthreads();
                    for (int e = tid; e < Lk * b; e += SBT) {
                        int i = e % Lk, c = e / Lk;
                        OB[i][c] -= p[i] * vp[c];
                    }
                    __syncthreads();
                }
                // new reflector from the block's first column
                for (int i = tid; i < Lk; i += SBT) xs[i] = OB[i][0];
                __syncthreads();
                house(Lk, xs, v, sh, tid);
                t = sh[0];
                const double alpha = sh[1];
                if (t != 0.0) {
                    if (tid < b && tid > 0) {
                        double s2 = 0.0;
                        for (int i = 0; i < Lk; ++i) s2 += v[i] * OB[i][tid];
                        u[tid] = t * s2;
                    }
                    __syncthreads();
                    for (int e = tid; e < Lk * b; e += SBT) {
                        int i = e % Lk, c = e / Lk;
                        if (c == 0) OB[i][0] = (i == 0) ? alpha : 0.0;
                        else OB[i][c] -= v[i] * u[c];
                    }
                    __syncthreads();
                }
                two_sided(Lk, DG, v, t, p, sh, tid);
                for (int e = tid; e < SB * SB; e += SBT) {
                    int i = e % SB, c = e / SB;
                    if (i < Lk && c < b) Bd[cm(b + i - c, rk - b + c, ldb)] = OB[i][c];
                }
            }
            // write back the diagonal block and the reflector
            for (int e = tid; e < SB * SB; e += SBT) {
                int i = e % SB, c = e / SB;
                if (i < Lk && c < Lk && i >= c) Bd[cm(i - c, rk + c, ldb)] = DG[i][c];
            }
            for (int i = tid; i < Lk; i += SBT) a.V2[cm(rk + i, s, n)] = v[i];
            if (tid == 0) a.tau2[(size_t)s * a.kmax + k] = t;
            for (int i = tid; i < SB; i += SBT) vp[i] = v[i];
            tp = t;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0) store_release(&a.progress[s], (k + 1 == nt) ? kDone : k + 1);
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
        int grid = std::min(nsweeps, std::min(resident, cus > 0 ? cus : 1));
        SbArgs a;
        a.n = n; a.b = b; a.ldb = ldb; a.nsweeps = nsweeps; a.kmax = sb2st_kmax(n, b);
        a.Bd = Bd; a.V2 = V2; a.tau2 = tau2; a.progress = progress; a.err = err;
        a.spin_limit = 1LL << 22;
        void* args[] = {&a};
        hipError_t rc = hipLaunchCooperativeKernel((const void*)sb2st_kernel, dim3(grid), dim3(SBT), args, 0, st);
        if (rc != hipSuccess) return kStatusHip;
    }
    hipLaunchKernelGGL(extract_tridiag_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, Bd, ldb, d, e);
    return 0;
}

}  // namespace eg
