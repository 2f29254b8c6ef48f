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
// live in a window of 2b-1 rows.  The b reflectors of (g, k), applied sweeps
// descending, form one block reflector H_{s_lo} ... H_{s_hi} = I - V T V^T
// (T formed once per (g, k) by a separate kernel), applied to a slab of 32
// columns as three FP64 matrix-core products (V^T X_W, T W, X_W - V W2) on
// the window staged in LDS.  Blocks run in anti-diagonal steps t = (G-1-g)+k:
// the windows of (g, k) and (g', k') overlap only when |(g+k) - (g'+k')| <= 1,
// so blocks of one step are independent and overlapping pairs keep their
// order; each step is one launch over all of its blocks and column slabs.
//
// Step (5).  Q1 = Q_0 Q_1 ... with Q_p = I - V_p T_p V_p^T from the panels of
// step (1); X <- Q1 X applies the panels last to first as three FP64
// matrix-core products (V^T X with a deterministic split over rows).
#include "common.h"

namespace eg {
namespace {

constexpr int NB2 = 64;     // maximum band width
constexpr int NCB = 32;     // columns of X per workgroup in the blocked Q2 application

__device__ inline int q2_ntasks(int n, int b, int s) { return (n - 2 - s) / b + 1; }

// Stage the reflectors of group (g, k) in LDS: column i is the reflector of
// sweep s_lo + i at rows [i, i + L_i) of the window that starts at base.
// Thread t always handles window row t % 128 and columns t / 128 + 2 j; all of
// its loads are issued before any LDS store so that their latencies overlap.
__device__ void q2_load_v(int n, int b, int g, int k, const double* __restrict__ V2, double (*Vs)[NB2 + 1])
{
    const int nsweeps = n - 2;
    const int s_lo = g * b;
    const int base = s_lo + 1 + k * b;
    const int r = threadIdx.x & 127, i0 = threadIdx.x >> 7;
    double v[NB2 / 2];
#pragma unroll
    for (int j = 0; j < NB2 / 2; ++j) {
        const int i = i0 + 2 * j;
        const int s = s_lo + i;
        v[j] = 0.0;
        if (i < b && s < nsweeps) {
            const int r0 = s + 1 + k * b;          // first row of this reflector
            const int L = min(b, n - r0);
            const int qq = r - i;
            if (r0 < n && qq >= 0 && qq < L) v[j] = V2[cm(base + r, s, n)];
        }
    }
#pragma unroll
    for (int j = 0; j < NB2 / 2; ++j) Vs[r][i0 + 2 * j] = v[j];
}

// T of P = H_{s_lo} H_{s_lo+1} ... H_{s_hi} = I - V T V^T for every (g, k)
// (forward accumulation from G = V^T V and the tau's).
__global__ __launch_bounds__(256) void q2_build_t_kernel(int n, int b, const double* __restrict__ V2,
                                                         const double* __restrict__ tau2, int kmax, double* Tq)
{
    __shared__ double Vs[2 * NB2][NB2 + 1];
    __shared__ double Gs[NB2][NB2 + 1];
    __shared__ double Ts[NB2][NB2 + 1];
    __shared__ double tau[NB2];
    const int g = blockIdx.x, k = blockIdx.y;
    const int nsweeps = n - 2;
    const int s_lo = g * b;
    if (k >= q2_ntasks(n, b, s_lo)) return;
    const int tid = threadIdx.x;
    q2_load_v(n, b, g, k, V2, Vs);
    if (tid < NB2) {
        const int s = s_lo + tid;
        tau[tid] = (tid < b && s < nsweeps && k < q2_ntasks(n, b, s)) ? tau2[(size_t)s * kmax + k] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < NB2 * NB2; e += 256) {
        const int i = e % NB2, j = e / NB2;
        double acc = 0.0;
        if (i < j) {
            for (int r = 0; r < 2 * NB2; ++r) acc += Vs[r][i] * Vs[r][j];
        }
        Gs[i][j] = acc;
        Ts[i][j] = 0.0;
    }
    __syncthreads();
    for (int c = 0; c < b; ++c) {
        if (tid < c) {
            double acc = 0.0;
            for (int j = tid; j < c; ++j) acc += Ts[tid][j] * Gs[j][c];
            Ts[tid][c] = -tau[c] * acc;
        }
        if (tid == c) Ts[c][c] = tau[c];
        __syncthreads();
    }
    double* T = Tq + ((size_t)g * kmax + k) * NB2 * NB2;
    for (int e = tid; e < NB2 * NB2; e += 256) T[e] = Ts[e % NB2][e / NB2];   // column-major, ld 64
}

// acc (16 x 16 block) += A (16 x 4K) B (4K x 16) with A(i, kk) = fa(i, kk), B(kk, j) = fb(kk, j)
// D layout: lane l, element r -> row 4 r + l / 16, column l % 16.

// One block reflector (g, k) on one 32-column slab of X per workgroup; the
// launch covers every (g, k) on the anti-diagonal step t = (G-1-g) + k.
// Blocks on one step touch disjoint row windows, and every pair of blocks
// whose windows overlap lands on different steps in the reverse-execution
// order (windows overlap only when g + k differ by at most one).
__global__ __launch_bounds__(256) void q2_apply_step_kernel(int n, int b, int ncol, int t,
                                                            const double* __restrict__ V2,
                                                            const double* __restrict__ Tq, int kmax, double* X,
                                                            int ldx)
{
    __shared__ double Vs[2 * NB2][NB2 + 1];
    __shared__ double Xs[2 * NB2][NCB + 1];
    __shared__ double Ws[NB2][NCB + 1];
    __shared__ double W2s[NB2][NCB + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nsweeps = n - 2;
    const int ngroups = ceil_div(nsweeps, b);
    const int g = ngroups - 1 - (int)blockIdx.x;
    const int k = t - (int)blockIdx.x;
    if (g < 0 || k < 0 || k >= q2_ntasks(n, b, g * b)) return;
    const int col0 = blockIdx.y * NCB;
    const int li = lane & 15, lk = lane >> 4;
    const int s_lo = g * b;
    const int base = s_lo + 1 + k * b;
    const int wrows = min(2 * b - 1, n - base);
    const double* T = Tq + ((size_t)g * kmax + k) * NB2 * NB2;
    double treg[NB2 / 4];
#pragma unroll
    for (int q4 = 0; q4 < NB2 / 4; ++q4) treg[q4] = T[(wave * 16 + li) + (size_t)(4 * q4 + lk) * NB2];
    {
        const int r = tid & 127, c0 = tid >> 7;
        double xv[NCB / 2];
#pragma unroll
        for (int j = 0; j < NCB / 2; ++j) {
            const int gc = col0 + c0 + 2 * j;
            xv[j] = (r < wrows && gc < ncol) ? X[cm(base + r, gc, ldx)] : 0.0;
        }
        q2_load_v(n, b, g, k, V2, Vs);
#pragma unroll
        for (int j = 0; j < NCB / 2; ++j) Xs[r][c0 + 2 * j] = xv[j];
    }
    __syncthreads();
    // W = V^T X_W (64 x 32): wave w owns rows 16w .. 16w+15, both column blocks
    {
        double4_t a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
        const int i0 = wave * 16;
        for (int kk = 0; kk < 2 * NB2; kk += 4) {
            const double av = Vs[kk + lk][i0 + li];
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Xs[kk + lk][li], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Xs[kk + lk][16 + li], a1, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Ws[i0 + 4 * r + lk][li] = a0[r];
            Ws[i0 + 4 * r + lk][16 + li] = a1[r];
        }
    }
    __syncthreads();
    // W2 = T W (64 x 32), T operands from registers
    {
        double4_t a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
        const int i0 = wave * 16;
#pragma unroll
        for (int q4 = 0; q4 < NB2 / 4; ++q4) {
            const int kk = 4 * q4;
            const double av = treg[q4];
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ws[kk + lk][li], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ws[kk + lk][16 + li], a1, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            W2s[i0 + 4 * r + lk][li] = a0[r];
            W2s[i0 + 4 * r + lk][16 + li] = a1[r];
        }
    }
    __syncthreads();
    // X_W -= V W2 (128 x 32): wave w owns rows 32w .. 32w+31
    {
        double4_t acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[a][c] = (double4_t){0, 0, 0, 0};
        const int i0 = wave * 32;
        for (int kk = 0; kk < NB2; kk += 4) {
            const double b0 = W2s[kk + lk][li], b1 = W2s[kk + lk][16 + li];
            const double v0 = Vs[i0 + li][kk + lk], v1 = Vs[i0 + 16 + li][kk + lk];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(v0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(v0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(v1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(v1, b1, acc[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) Xs[i0 + 16 * a + 4 * r + lk][16 * c + li] -= acc[a][c][r];
    }
    __syncthreads();
    {
        const int r = tid & 127, c0 = tid >> 7;
#pragma unroll
        for (int j = 0; j < NCB / 2; ++j) {
            const int gc = col0 + c0 + 2 * j;
            if (r < wrows && gc < ncol) X[cm(base + r, gc, ldx)] = Xs[r][c0 + 2 * j];
        }
    }
}

}  // namespace

size_t apply_q2_workspace_doubles(int n, int b)
{
    const int ngroups = std::max(1, ceil_div(std::max(n - 2, 1), b));
    const int kmax = n >= 2 ? (n - 2) / b + 1 : 1;
    return (size_t)ngroups * kmax * NB2 * NB2;
}

// X (n x ncol) <- Q2 X; Tq: apply_q2_workspace_doubles(n, b) doubles.
void apply_q2(hipStream_t st, int n, int b, int ncol, const double* V2, const double* tau2, int kmax, double* X,
              int ldx, double* Tq)
{
    if (n <= 2 || ncol <= 0) return;
    const int ngroups = ceil_div(n - 2, b);
    hipLaunchKernelGGL(q2_build_t_kernel, dim3(ngroups, kmax), dim3(256), 0, st, n, b, V2, tau2, kmax, Tq);
    const int nslab = ceil_div(ncol, NCB);
    const int tmax = (ngroups - 1) + kmax;   // last step: g = 0 with its last block
    for (int t = 0; t < tmax; ++t) {
        const int nb = std::min(ngroups, t + 1);   // blockIdx.x = G-1-g ranges over 0 .. min(G-1, t)
        hipLaunchKernelGGL(q2_apply_step_kernel, dim3(nb, nslab), dim3(256), 0, st, n, b, ncol, t, V2, Tq, kmax,
                           X, ldx);
    }
}

size_t apply_q1_workspace_doubles(int n, int ncol)
{
    return (size_t)8 * 64 * std::max(ncol, 1) + (size_t)2 * 64 * std::max(ncol, 1);
}

// X (n x ncol) <- Q1 X with the panel reflectors of step (1).
void apply_q1(hipStream_t st, int n, int b, int ncol, const double* Vall, const double* Tall, double* X, int ldx,
              double* work)
{
    if (ncol <= 0) return;
    const int npanel = ceil_div(n, b);
    double* W = work;                        // 64 x ncol
    double* W2 = W + (size_t)64 * ncol;      // 64 x ncol
    double* part = W2 + (size_t)64 * ncol;
    const size_t npart = apply_q1_workspace_doubles(n, ncol) - (size_t)2 * 64 * ncol;
    for (int p = npanel - 1; p >= 0; --p) {
        const int j = p * b;
        const int r0 = j + b;
        const int m = n - r0;
        if (m < 2) continue;
        const int bw = std::min(b, n - j);
        const double* V = Vall + cm(r0, j, n);
        const double* T = Tall + (size_t)p * b * b;
        dgemm_splitk(st, 'T', 'N', bw, ncol, m, 1.0, V, n, X + r0, ldx, 0.0, W, 64, part, npart);
        dgemm(st, 'N', 'N', bw, ncol, bw, 1.0, T, b, W, 64, 0.0, W2, 64);
        dgemm(st, 'N', 'N', m, ncol, bw, -1.0, V, n, W2, 64, 1.0, X + r0, ldx);
    }
}

}  // namespace eg
