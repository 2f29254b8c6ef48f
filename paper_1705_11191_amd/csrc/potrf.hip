// Cholesky factorization S = L L^T (ELSI paper, Sec. 3.1, Eq. (10)) and the
// triangular solves that use L (Eq. (11) and the back substitution c = L^-T c~).
//
// Blocking: 64 x 64 diagonal blocks are factored (and inverted) by one
// workgroup entirely in LDS; inside a 1024-wide outer panel the 64-column
// steps update only the panel, and the trailing matrix receives one K = 1024
// update per outer panel on the matrix cores (1024 beats 512 and 2048: the
// products run faster at larger K while the K = 64 work inside the panel grows).  Triangular solves multiply by
// the inverted 64 x 64 diagonal blocks and update with the same two-level
// scheme.
#include "common.h"

namespace eg {
namespace {

constexpr int NB = 64;     // diagonal block
constexpr int NBO = 2048;   // outer panel
constexpr int NBM = 256;    // middle panel: inside an outer panel the updates take K = 256 rather than 64

__device__ inline double lane_value(double v, int l)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// Orders one wave's LDS accesses across its lanes (no workgroup barrier needed).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Factor the jb x jb diagonal block at (j0, j0) and write L and L^-1.  The
// factorization is done by one wave with lane r holding row r in registers
// (column c: the pivot is read from lane c, the new column is broadcast
// through LDS); the inverse by the whole workgroup in LDS.
__global__ __launch_bounds__(256) void potf2_inv_kernel(int jb, int j0, double* A, int lda,
                                                        double* Linv, int* info)
{
    __shared__ double L[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    __shared__ double Y[NB][NB + 1];
    __shared__ double col[NB];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = (*info != 0);
    {
        // a thread's 16 loads are all in flight before its first LDS store
        double v[NB * NB / 256];
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int e = tid + 256 * u, i = e % NB, c = e / NB;
            v[u] = (i < jb && c < jb && i >= c) ? A[cm(j0 + i, j0 + c, lda)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int e = tid + 256 * u;
            L[e % NB][e / NB] = v[u];
        }
    }
    __syncthreads();
    if (bad) return;
    if (tid < 64) {
        // rows and columns beyond jb are padded with the identity, so all 64
        // steps run unconditionally (the loop unrolls and g stays in registers);
        // after a non-positive pivot the remaining steps only produce values
        // that are discarded
        const int lane = tid;
        double g[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) g[q] = (lane >= jb && q == lane) ? 1.0 : L[lane][q];
        int fail = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const double s = lane_value(g[c], c);
            if (!fail && (!(s > 0.0) || !isfinite(s))) fail = c + 1;
            const double d = sqrt(s);
            const double l = (lane == c) ? d : g[c] / d;   // rows below c: L(r, c)
            if (lane >= c) g[c] = l;
            col[lane] = (lane > c) ? l : 0.0;
            wave_lds_sync();
            // the column into registers first, so that its LDS reads are all in
            // flight together instead of one round trip per pair of entries
            double cv[NB];
#pragma unroll
            for (int q = c + 1; q < NB; ++q) cv[q] = col[q];
#pragma unroll
            for (int q = c + 1; q < NB; ++q) g[q] -= l * cv[q];   // only q <= r is kept
            wave_lds_sync();
        }
        if (!fail) {
#pragma unroll
            for (int q = 0; q < NB; ++q) L[lane][q] = (q <= lane && lane < jb) ? g[q] : 0.0;
        } else if (lane == 0) {
            atomicCAS(info, 0, j0 + fail);
            bad = 1;
        }
    }
    __syncthreads();
    if (bad) return;
    tri_inverse_lower64<256>(jb, L, X, Y);
    for (int e = tid; e < NB * NB; e += 256) {
        int i = e % NB, c = e / NB;
        if (i < jb && c < jb && i >= c) A[cm(j0 + i, j0 + c, lda)] = L[i][c];
        Linv[e] = X[i][c];
    }
}

// Inverse of each 64 x 64 diagonal block of an already factored L.
__global__ __launch_bounds__(256) void trtri_blocks_kernel(int n, const double* L, int ldl, double* Linv)
{
    __shared__ double Ls[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    __shared__ double Y[NB][NB + 1];
    const int blk = blockIdx.x;
    const int j0 = blk * NB;
    const int jb = min(NB, n - j0);
    const int tid = threadIdx.x;
    {
        double v[NB * NB / 256];
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int e = tid + 256 * u, i = e % NB, c = e / NB;
            v[u] = (i < jb && c < jb && i >= c) ? L[cm(j0 + i, j0 + c, ldl)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int e = tid + 256 * u;
            Ls[e % NB][e / NB] = v[u];
        }
    }
    __syncthreads();
    tri_inverse_lower64<256>(jb, Ls, X, Y);
    double* out = Linv + (size_t)blk * NB * NB;
    for (int e = tid; e < NB * NB; e += 256) out[e] = X[e % NB][e / NB];
}

__global__ void zero_strict_upper_kernel(int n, double* A, int lda)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)n * n;
    if (e >= total) return;
    int i = (int)(e % n), j = (int)(e / n);
    if (i < j) A[cm(i, j, lda)] = 0.0;
}

}  // namespace

void dtrtri_diag_blocks(hipStream_t st, int n, const double* L, int ldl, double* Linv)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(trtri_blocks_kernel, dim3(ceil_div(n, NB)), dim3(256), 0, st, n, L, ldl, Linv);
}

void dpotrf(hipStream_t st, int n, double* A, int lda, double* Linv, int* info)
{
    for (int J0 = 0; J0 < n; J0 += NBO) {
        const int JB = std::min(NBO, n - J0);
        for (int M0 = J0; M0 < J0 + JB; M0 += NBM) {
            const int MB = std::min(NBM, J0 + JB - M0);
            for (int j0 = M0; j0 < M0 + MB; j0 += NB) {
                const int jb = std::min(NB, M0 + MB - j0);
                double* Lj = Linv + (size_t)(j0 / NB) * NB * NB;
                hipLaunchKernelGGL(potf2_inv_kernel, dim3(1), dim3(256), 0, st, jb, j0, A, lda, Lj, info);
                const int r0 = j0 + jb;
                if (r0 >= n) break;
                double* P = A + cm(r0, j0, lda);
                // panel rows below the block: P <- P L_jj^-T
                dgemm(st, 'N', 'T', n - r0, jb, jb, 1.0, P, lda, Lj, NB, 0.0, P, lda);
                // update the rest of this middle panel (columns r0 .. M0+MB-1)
                const int wc = M0 + MB - r0;
                if (wc > 0)
                    dgemm(st, 'N', 'T', n - r0, wc, jb, -1.0, P, lda, A + cm(r0, j0, lda), lda, 1.0,
                          A + cm(r0, r0, lda), lda, 1);
            }
            // update the rest of this outer panel (columns M0+MB .. J0+JB-1), K = MB
            const int m0 = M0 + MB, mc = J0 + JB - m0;
            if (mc > 0 && m0 < n)
                dgemm(st, 'N', 'T', n - m0, mc, MB, -1.0, A + cm(m0, M0, lda), lda, A + cm(m0, M0, lda), lda, 1.0,
                      A + cm(m0, m0, lda), lda, 1);
        }
        const int t0 = J0 + JB;
        if (t0 < n) {
            // trailing matrix: A22 -= P P^T (lower tiles), K = outer panel width
            const double* P = A + cm(t0, J0, lda);
            dgemm(st, 'N', 'T', n - t0, n - t0, JB, -1.0, P, lda, P, lda, 1.0, A + cm(t0, t0, lda), lda, 1);
        }
    }
    size_t total = (size_t)n * n;
    hipLaunchKernelGGL(zero_strict_upper_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       n, A, lda);
}

// B <- L^-1 B, L lower (n x n), B n x ncol.
void dtrsm_left_lower_n(hipStream_t st, int n, int ncol, const double* L, int ldl,
                        const double* Linv, double* B, int ldb)
{
    for (int I0 = 0; I0 < n; I0 += NBO) {
        const int IB = std::min(NBO, n - I0);
        for (int M0 = I0; M0 < I0 + IB; M0 += NBM) {
            const int MB = std::min(NBM, I0 + IB - M0);
            for (int i0 = M0; i0 < M0 + MB; i0 += NB) {
                const int ib = std::min(NB, M0 + MB - i0);
                const double* Li = Linv + (size_t)(i0 / NB) * NB * NB;
                dgemm(st, 'N', 'N', ib, ncol, ib, 1.0, Li, NB, B + i0, ldb, 0.0, B + i0, ldb);
                const int r0 = i0 + ib, rn = M0 + MB - r0;
                if (rn > 0)
                    dgemm(st, 'N', 'N', rn, ncol, ib, -1.0, L + cm(r0, i0, ldl), ldl, B + i0, ldb, 1.0,
                          B + r0, ldb);
            }
            const int m0 = M0 + MB, mn = I0 + IB - m0;
            if (mn > 0)
                dgemm(st, 'N', 'N', mn, ncol, MB, -1.0, L + cm(m0, M0, ldl), ldl, B + M0, ldb, 1.0, B + m0, ldb);
        }
        const int t0 = I0 + IB;
        if (t0 < n)
            dgemm(st, 'N', 'N', n - t0, ncol, IB, -1.0, L + cm(t0, I0, ldl), ldl, B + I0, ldb, 1.0,
                  B + t0, ldb);
    }
}

// Lower triangle only of X = B L^-T (n x n): column block j of X needs rows
// >= j of B's column block j and of the earlier X blocks, so every product
// is restricted to rows at or below its column block (upper entries of B are
// left in an unspecified state).
void dtrsm_right_lower_t_lowerpart(hipStream_t st, int n, const double* L, int ldl, const double* Linv,
                                   double* B, int ldb)
{
    for (int J0 = 0; J0 < n; J0 += NBO) {
        const int JB = std::min(NBO, n - J0);
        for (int M0 = J0; M0 < J0 + JB; M0 += NBM) {
            const int MB = std::min(NBM, J0 + JB - M0);
            for (int j0 = M0; j0 < M0 + MB; j0 += NB) {
                const int jb = std::min(NB, M0 + MB - j0);
                const double* Lj = Linv + (size_t)(j0 / NB) * NB * NB;
                double* Bj = B + cm(j0, j0, ldb);
                dgemm(st, 'N', 'T', n - j0, jb, jb, 1.0, Bj, ldb, Lj, NB, 0.0, Bj, ldb);
                const int c0 = j0 + jb, cn = M0 + MB - c0;
                if (cn > 0)
                    dgemm(st, 'N', 'T', n - c0, cn, jb, -1.0, B + cm(c0, j0, ldb), ldb, L + cm(c0, j0, ldl), ldl,
                          1.0, B + cm(c0, c0, ldb), ldb, 1);
            }
            const int m0 = M0 + MB, mc = J0 + JB - m0;
            if (mc > 0)
                dgemm(st, 'N', 'T', n - m0, mc, MB, -1.0, B + cm(m0, M0, ldb), ldb, L + cm(m0, M0, ldl), ldl, 1.0,
                      B + cm(m0, m0, ldb), ldb, 1);
        }
        const int t0 = J0 + JB;
        if (t0 < n)
            dgemm(st, 'N', 'T', n - t0, n - t0, JB, -1.0, B + cm(t0, J0, ldb), ldb, L + cm(t0, J0, ldl), ldl,
                  1.0, B + cm(t0, t0, ldb), ldb, 1);
    }
}

// B <- B L^-T, B nrow x n: solve X L^T = B column block by column block.
void dtrsm_right_lower_t(hipStream_t st, int nrow, int n, const double* L, int ldl,
                         const double* Linv, double* B, int ldb)
{
    for (int J0 = 0; J0 < n; J0 += NBO) {
        const int JB = std::min(NBO, n - J0);
        for (int j0 = J0; j0 < J0 + JB; j0 += NB) {
            const int jb = std::min(NB, J0 + JB - j0);
            const double* Lj = Linv + (size_t)(j0 / NB) * NB * NB;
            double* Bj = B + cm(0, j0, ldb);
            dgemm(st, 'N', 'T', nrow, jb, jb, 1.0, Bj, ldb, Lj, NB, 0.0, Bj, ldb);
            const int c0 = j0 + jb, cn = J0 + JB - c0;
            if (cn > 0)
                dgemm(st, 'N', 'T', nrow, cn, jb, -1.0, Bj, ldb, L + cm(c0, j0, ldl), ldl, 1.0,
                      B + cm(0, c0, ldb), ldb);
        }
        const int t0 = J0 + JB;
        if (t0 < n)
            dgemm(st, 'N', 'T', nrow, n - t0, JB, -1.0, B + cm(0, J0, ldb), ldb, L + cm(t0, J0, ldl), ldl,
                  1.0, B + cm(0, t0, ldb), ldb);
    }
}

// B <- L^-T B, B n x ncol: solve L^T X = B from the bottom block upward.
void dtrsm_left_lower_t(hipStream_t st, int n, int ncol, const double* L, int ldl,
                        const double* Linv, double* B, int ldb)
{
    const int nouter = ceil_div(n, NBO);
    for (int ob = nouter - 1; ob >= 0; --ob) {
        const int I0 = ob * NBO;
        const int IB = std::min(NBO, n - I0);
        const int nmid = ceil_div(IB, NBM);
        for (int mb = nmid - 1; mb >= 0; --mb) {
            const int M0 = I0 + mb * NBM;
            const int MB = std::min(NBM, I0 + IB - M0);
            const int ninner = ceil_div(MB, NB);
            for (int q = ninner - 1; q >= 0; --q) {
                const int i0 = M0 + q * NB;
                const int ib = std::min(NB, M0 + MB - i0);
                const double* Li = Linv + (size_t)(i0 / NB) * NB * NB;
                dgemm(st, 'T', 'N', ib, ncol, ib, 1.0, Li, NB, B + i0, ldb, 0.0, B + i0, ldb);
                const int rn = i0 - M0;   // rows of this middle block above the inner block
                if (rn > 0)
                    dgemm(st, 'T', 'N', rn, ncol, ib, -1.0, L + cm(i0, M0, ldl), ldl, B + i0, ldb, 1.0,
                          B + M0, ldb);
            }
            const int mn = M0 - I0;       // rows of this outer block above the middle block
            if (mn > 0)
                dgemm(st, 'T', 'N', mn, ncol, MB, -1.0, L + cm(M0, I0, ldl), ldl, B + M0, ldb, 1.0, B + I0, ldb);
        }
        if (I0 > 0)
            dgemm(st, 'T', 'N', I0, ncol, IB, -1.0, L + cm(I0, 0, ldl), ldl, B + I0, ldb, 1.0, B, ldb);
    }
}

}  // namespace eg
