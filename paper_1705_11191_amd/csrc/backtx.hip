// Steps (4) and (5) of Fig. 1 (ELSI paper, Sec. 3.1): eigenvectors of T are
// carried back to the band form (X <- Q2 X) and then to the full standard
// form (X <- Q1 X).
//
// Step (4).  Q2 is the product of the bulge-chasing reflectors in execution
// order (sweep s ascending, block k ascending), so X <- Q2 X applies them in
// the reverse order.  Reflector (s, k) touches rows J_k(s) = [s+1+kb,
// s+(k+1)b]; two reflectors only fail to commute when their rows overlap.
// Grouping b consecutive sweeps g, the order "groups descending, inside a
// group k ascending, inside (g, k) sweeps descending" keeps every overlapping
// pair in its reverse-execution order, and the reflectors of one (g, k) all
// live in a window of 2b-1 rows.  One workgroup owns a slab of columns of X,
// stages each window in LDS and applies the reflectors there.
//
// Step (5).  Q1 = Q_0 Q_1 ... with Q_p = I - V_p T_p V_p^T from the panels of
// step (1); X <- Q1 X applies the panels last to first as three FP64
// matrix-core products (V^T X with a deterministic split over rows).
#include "common.h"

namespace eg {
namespace {

constexpr int NB2 = 64;     // maximum band width
constexpr int NC = 64;      // columns of X per workgroup

__global__ __launch_bounds__(256) void apply_q2_kernel(int n, int b, int ncol, const double* __restrict__ V2,
                                                       const double* __restrict__ tau2, int kmax, double* X,
                                                       int ldx)
{
    __shared__ double W[2 * NB2][NC + 1];
    __shared__ double vs[NB2];
    __shared__ double red[4][NC + 1];
    const int tid = threadIdx.x;
    const int c = tid & 63, part = tid >> 6;
    const int col0 = blockIdx.x * NC;
    const int gc = col0 + c;
    const int nsweeps = n - 2;
    if (nsweeps <= 0) return;
    const int ngroups = ceil_div(nsweeps, b);
    for (int g = ngroups - 1; g >= 0; --g) {
        const int s_lo = g * b;
        const int s_hi = min(nsweeps - 1, s_lo + b - 1);
        const int nt_max = (n - 2 - s_lo) / b + 1;
        for (int k = 0; k < nt_max; ++k) {
            const int base = s_lo + 1 + k * b;
            if (base >= n) break;
            const int wrows = min(2 * b - 1, n - base);
            // stage the window
            for (int r = part; r < wrows; r += 4)
                W[r][c] = (gc < ncol) ? X[cm(base + r, gc, ldx)] : 0.0;
            __syncthreads();
            for (int s = s_hi; s >= s_lo; --s) {
                if (k > (n - 2 - s) / b) continue;   // sweep s has no task k
                const double t = tau2[(size_t)s * kmax + k];
                if (t == 0.0) continue;
                const int r0 = s + 1 + k * b;
                const int L = min(b, n - r0);
                const int off = r0 - base;
                if (tid < L) vs[tid] = V2[cm(r0 + tid, s, n)];
                __syncthreads();
                double acc = 0.0;
                for (int i = part; i < L; i += 4) acc += vs[i] * W[off + i][c];
                red[part][c] = acc;
                __syncthreads();
                const double u = t * (red[0][c] + red[1][c] + red[2][c] + red[3][c]);
                for (int i = part; i < L; i += 4) W[off + i][c] -= vs[i] * u;
                __syncthreads();
            }
            for (int r = part; r < wrows; r += 4)
                if (gc < ncol) X[cm(base + r, gc, ldx)] = W[r][c];
            __syncthreads();
        }
    }
}

// partial W = A^T B over one chunk of rows for a 64-column tile of B (A has m <= 64 columns)
__global__ __launch_bounds__(256) void tn_tile_partial(int m, int ncol, int k, const double* __restrict__ A,
                                                       int lda, const double* __restrict__ B, int ldb,
                                                       double* __restrict__ part, int chunk)
{
    __shared__ double As[32][65];
    __shared__ double Bs[32][65];
    const int r0 = blockIdx.x * chunk;
    const int r1 = min(k, r0 + chunk);
    const int c0 = blockIdx.y * 64;
    const int tid = threadIdx.x;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int rr = r0; rr < r1; rr += 32) {
        for (int e = tid; e < 32 * 64; e += 256) {
            int kk = e % 32, cc = e / 32;
            int gk = rr + kk;
            As[kk][cc] = (gk < r1 && cc < m) ? A[cm(gk, cc, lda)] : 0.0;
            Bs[kk][cc] = (gk < r1 && c0 + cc < ncol) ? B[cm(gk, c0 + cc, ldb)] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int e = tid + q * 256;
            int i = e % 64, j = e / 64;
            double s = acc[q];
#pragma unroll 8
            for (int kk = 0; kk < 32; ++kk) s += As[kk][i] * Bs[kk][j];
            acc[q] = s;
        }
        __syncthreads();
    }
    double* P = part + ((size_t)blockIdx.x * gridDim.y + blockIdx.y) * 4096;
#pragma unroll
    for (int q = 0; q < 16; ++q) P[tid + q * 256] = acc[q];
}

__global__ void tn_tile_reduce(int m, int ncol, int nchunks, int ntiles, const double* __restrict__ part,
                               double* C, int ldc)
{
    const int tile = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4096) return;
    const int i = e % 64, j = tile * 64 + e / 64;
    if (i >= m || j >= ncol) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[((size_t)c * ntiles + tile) * 4096 + e];
    C[cm(i, j, ldc)] = s;
}

}  // namespace

void apply_q2(hipStream_t st, int n, int b, int ncol, const double* V2, const double* tau2, int kmax, double* X,
              int ldx)
{
    if (n <= 2 || ncol <= 0) return;
    hipLaunchKernelGGL(apply_q2_kernel, dim3(ceil_div(ncol, NC)), dim3(256), 0, st, n, b, ncol, V2, tau2, kmax,
                       X, ldx);
}

size_t apply_q1_workspace_doubles(int n, int ncol)
{
    const int chunk = 1024;
    return (size_t)ceil_div(n, chunk) * ceil_div(std::max(ncol, 1), 64) * 4096 + (size_t)2 * 64 * std::max(ncol, 1);
}

// X (n x ncol) <- Q1 X with the panel reflectors of step (1).
void apply_q1(hipStream_t st, int n, int b, int ncol, const double* Vall, const double* Tall, double* X, int ldx,
              double* work)
{
    if (ncol <= 0) return;
    const int chunk = 1024;
    const int npanel = ceil_div(n, b);
    double* W = work;                        // 64 x ncol
    double* W2 = W + (size_t)64 * ncol;      // 64 x ncol
    double* part = W2 + (size_t)64 * ncol;
    const int ntiles = ceil_div(ncol, 64);
    for (int p = npanel - 1; p >= 0; --p) {
        const int j = p * b;
        const int r0 = j + b;
        const int m = n - r0;
        if (m < 2) continue;
        const int bw = std::min(b, n - j);
        const double* V = Vall + cm(r0, j, n);
        const double* T = Tall + (size_t)p * b * b;
        const int nchunks = ceil_div(m, chunk);
        hipLaunchKernelGGL(tn_tile_partial, dim3(nchunks, ntiles), dim3(256), 0, st, bw, ncol, m, V, n,
                           X + r0, ldx, part, chunk);
        hipLaunchKernelGGL(tn_tile_reduce, dim3(16, ntiles), dim3(256), 0, st, bw, ncol, nchunks, ntiles, part, W,
                           64);
        dgemm(st, 'N', 'N', bw, ncol, bw, 1.0, T, b, W, 64, 0.0, W2, 64);
        dgemm(st, 'N', 'N', m, ncol, bw, -1.0, V, n, W2, 64, 1.0, X + r0, ldx);
    }
}

}  // namespace eg
