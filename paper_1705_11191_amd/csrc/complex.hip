// Complex Hermitian pencils (the complex eigensolver interface of the ELSI
// paper, Sec. 4.3: the k-point problems of periodic systems) through their
// real image.  A complex n x n matrix Z = X + iY maps to the real 2n x 2n
// matrix with the 2 x 2 block [[x, -y], [y, x]] at rows and columns 2j, 2j+1
// for z_jk = x + iy (interleaved ordering).  The map is a ring homomorphism
// (products, inverses and conjugate transposes map to products, inverses and
// transposes), so:
//   - a Hermitian H maps to a symmetric H2 and an HPD S to an SPD S2;
//   - the Cholesky factor of S2 is the image of the complex factor L (its
//     2 x 2 diagonal blocks are l_jj I), so L can be read back from it;
//   - H2 x = lam S2 x has every eigenvalue of the complex pencil twice, with
//     the eigenvectors [Re c; Im c] and J [Re c; Im c], J the image of i;
//   - the complex D = sum f c c^H has the real image sum f (v v^T + Jv (Jv)^T),
//     i.e. the real density matrix of the doubled spectrum.
// These kernels build the images and read the complex results back.
#include "api_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace eg {
namespace {

// z_jk of a Hermitian matrix from its lower triangle (interleaved storage).
__device__ inline void herm_entry(const double* Z, int ldz, int j, int k, double& x, double& y)
{
    if (j >= k) {
        const size_t e = 2 * cm(j, k, ldz);
        x = Z[e];
        y = (j == k) ? 0.0 : Z[e + 1];
    } else {
        const size_t e = 2 * cm(k, j, ldz);
        x = Z[e];
        y = -Z[e + 1];
    }
}

// factor = 0: R = image of the Hermitian Z (lower triangle read), both
// triangles written; factor = 1: R = image of the lower triangular Z, zero
// above the diagonal.
__global__ void embed_kernel(int n, const double* Z, int ldz, double* R, int ldr, int factor)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;   // row block
    const int k = blockIdx.y;                              // column block
    if (j >= n) return;
    double x = 0.0, y = 0.0;
    if (!factor) {
        herm_entry(Z, ldz, j, k, x, y);
    } else if (j >= k) {
        const size_t e = 2 * cm(j, k, ldz);
        x = Z[e];
        y = (j == k) ? 0.0 : Z[e + 1];
    }
    R[cm(2 * j, 2 * k, ldr)] = x;
    R[cm(2 * j + 1, 2 * k, ldr)] = y;
    R[cm(2 * j, 2 * k + 1, ldr)] = -y;
    R[cm(2 * j + 1, 2 * k + 1, ldr)] = x;
}

// Z = the complex matrix nearest to the image R: each 2 x 2 block
// [[a, b], [c, d]] gives x = (a + d) / 2, y = (c - b) / 2 (for a symmetric R
// this makes Z exactly Hermitian); lower = 1 writes the lower triangle (real
// diagonal) and zeros above it.
__global__ void extract_kernel(int n, const double* R, int ldr, double* Z, int ldz, int lower)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (j >= n) return;
    double x = 0.0, y = 0.0;
    if (!lower || j >= k) {
        x = 0.5 * (R[cm(2 * j, 2 * k, ldr)] + R[cm(2 * j + 1, 2 * k + 1, ldr)]);
        y = (lower && j == k) ? 0.0 : 0.5 * (R[cm(2 * j + 1, 2 * k, ldr)] - R[cm(2 * j, 2 * k + 1, ldr)]);
    }
    const size_t e = 2 * cm(j, k, ldz);
    Z[e] = x;
    Z[e + 1] = y;
}

// The eigenvalues of the complex pencil from the doubled real spectrum.
__global__ void pair_values_kernel(int n, const double* w2, double* w)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) w[l] = 0.5 * (w2[2 * l] + w2[2 * l + 1]);
}

// Complex columns c_l = U(0::2, l) + i U(1::2, l).
__global__ void extract_vectors_kernel(int n, int k, const double* U, int ldu, double* C, int ldc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (i >= n || l >= k) return;
    const size_t e = 2 * cm(i, l, ldc);
    C[e] = U[cm(2 * i, l, ldu)];
    C[e + 1] = U[cm(2 * i + 1, l, ldu)];
}

// U(:, l) = X(:, src[l]).
__global__ void gather_columns_kernel(int rows, int k, const double* X, int ldx, const int* src, double* U, int ldu)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (i >= rows || l >= k) return;
    U[cm(i, l, ldu)] = X[cm(i, src[l], ldx)];
}

// JU: the image of i times each column (rows 2i, 2i+1: (-u_{2i+1}, u_{2i})).
__global__ void apply_j_kernel(int n, int k, const double* U, int ldu, double* JU, int ldj)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (i >= n || l >= k) return;
    const double u0 = U[cm(2 * i, l, ldu)], u1 = U[cm(2 * i + 1, l, ldu)];
    JU[cm(2 * i, l, ldj)] = -u1;
    JU[cm(2 * i + 1, l, ldj)] = u0;
}

__global__ void duplicate_kernel(int k, const double* f, double* f2)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < k) {
        f2[2 * l] = f[l];
        f2[2 * l + 1] = f[l];
    }
}

// Fixed-order sum over the 256 threads of the workgroup (red: 4 doubles of LDS).
__device__ inline double block_sum(double v, double* red)
{
    v = wave_sum_dpp(v);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// One cluster of m numerically equal complex eigenvalues: the ncand real
// standard-form eigenvectors X(:, 0:ncand) (2n rows, ld ldx) span a subspace
// that J maps onto itself.  Greedily take m of them, each time the candidate
// with the largest component outside span{u_s, J u_s} of those already taken,
// orthogonalized against that span twice; U(:, 0:m) gets the results, whose
// complex images are then orthonormal (u_s and J u_s are orthogonal for every
// real u).  One workgroup of 256 threads.
constexpr int kMaxCand = 64;
__global__ __launch_bounds__(256) void select_cluster_kernel(int rows, const double* X, int ldx, int ncand, int m,
                                                             double* U, int ldu)
{
    __shared__ double red[4];
    __shared__ double coef[2 * kMaxCand];
    __shared__ int used[kMaxCand];
    const int tid = threadIdx.x;
    const int half = rows / 2;
    if (tid < kMaxCand) used[tid] = 0;
    __syncthreads();
    for (int t = 0; t < m; ++t) {
        int best = -1;
        double bestn = -1.0;
        for (int j = 0; j < ncand; ++j) {
            if (used[j]) continue;
            const double* x = X + (size_t)j * ldx;
            // coefficients <u_s, x>, <J u_s, x>
            for (int s = 0; s < t; ++s) {
                const double* u = U + (size_t)s * ldu;
                double a = 0.0, b = 0.0;
                for (int i = tid; i < half; i += 256) {
                    const double u0 = u[2 * i], u1 = u[2 * i + 1], x0 = x[2 * i], x1 = x[2 * i + 1];
                    a += u0 * x0 + u1 * x1;
                    b += -u1 * x0 + u0 * x1;
                }
                a = block_sum(a, red);
                b = block_sum(b, red);
                if (tid == 0) {
                    coef[2 * s] = a;
                    coef[2 * s + 1] = b;
                }
            }
            __syncthreads();
            double q = 0.0;
            for (int i = tid; i < half; i += 256) {
                double r0 = x[2 * i], r1 = x[2 * i + 1];
                for (int s = 0; s < t; ++s) {
                    const double* u = U + (size_t)s * ldu;
                    const double a = coef[2 * s], b = coef[2 * s + 1];
                    r0 -= a * u[2 * i] - b * u[2 * i + 1];
                    r1 -= a * u[2 * i + 1] + b * u[2 * i];
                }
                q += r0 * r0 + r1 * r1;
            }
            q = block_sum(q, red);
            if (q > bestn) {
                bestn = q;
                best = j;
            }
        }
        if (best < 0) return;
        // u_t = the chosen candidate, projected out of the earlier span twice
        double* ut = U + (size_t)t * ldu;
        const double* x = X + (size_t)best * ldx;
        for (int i = tid; i < rows; i += 256) ut[i] = x[i];
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int s = 0; s < t; ++s) {
                const double* u = U + (size_t)s * ldu;
                double a = 0.0, b = 0.0;
                for (int i = tid; i < half; i += 256) {
                    const double u0 = u[2 * i], u1 = u[2 * i + 1], x0 = ut[2 * i], x1 = ut[2 * i + 1];
                    a += u0 * x0 + u1 * x1;
                    b += -u1 * x0 + u0 * x1;
                }
                a = block_sum(a, red);
                b = block_sum(b, red);
                for (int i = tid; i < half; i += 256) {
                    const double u0 = u[2 * i], u1 = u[2 * i + 1];
                    ut[2 * i] -= a * u0 - b * u1;
                    ut[2 * i + 1] -= a * u1 + b * u0;
                }
                __syncthreads();
            }
        }
        double q = 0.0;
        for (int i = tid; i < rows; i += 256) q += ut[i] * ut[i];
        q = block_sum(q, red);
        const double inv = 1.0 / sqrt(q);
        for (int i = tid; i < rows; i += 256) ut[i] *= inv;
        if (tid == 0) used[best] = 1;
        __syncthreads();
    }
}

}  // namespace

void embed_complex(hipStream_t st, int n, const double* Z, int ldz, double* R, int ldr, bool lower_factor)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(embed_kernel, dim3(ceil_div(n, 256), n), dim3(256), 0, st, n, Z, ldz, R, ldr,
                       lower_factor ? 1 : 0);
}

void extract_complex(hipStream_t st, int n, const double* R, int ldr, double* Z, int ldz, bool lower_factor)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(extract_kernel, dim3(ceil_div(n, 256), n), dim3(256), 0, st, n, R, ldr, Z, ldz,
                       lower_factor ? 1 : 0);
}

void pair_values(hipStream_t st, int n, const double* w2, double* w)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(pair_values_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, w2, w);
}

void extract_vectors(hipStream_t st, int n, int k, const double* U, int ldu, double* C, int ldc)
{
    if (n <= 0 || k <= 0) return;
    hipLaunchKernelGGL(extract_vectors_kernel, dim3(ceil_div(n, 256), k), dim3(256), 0, st, n, k, U, ldu, C, ldc);
}

// The complex images c_l of the columns of U (real-orthonormal, 2n rows) have
// the Gram matrix C^H C = U^T U - i B, B = U^T (J U); U^T U is the identity to
// rounding, and B is of the order of the eigensolver's subspace errors.  One
// Loewdin step, C <- C (I - i B)^-1/2 = C (I + i B / 2) + O(|B|^2), is
// U <- U + (J U)(B / 2) in real arithmetic.  JU and Bm are scratch (2n x k,
// k x k).
void orthonormalize_complex_images(hipStream_t st, int n, int k, double* U, int ldu, double* JU, double* Bm)
{
    if (n <= 0 || k <= 0) return;
    const int n2 = 2 * n;
    hipLaunchKernelGGL(apply_j_kernel, dim3(ceil_div(n, 256), k), dim3(256), 0, st, n, k, U, ldu, JU, n2);
    dgemm(st, 'T', 'N', k, k, n2, 1.0, U, ldu, JU, n2, 0.0, Bm, k);
    dgemm(st, 'N', 'N', n2, k, k, 0.5, JU, n2, Bm, k, 1.0, U, ldu);
}

void duplicate_values(hipStream_t st, int k, const double* f, double* f2)
{
    if (k <= 0) return;
    hipLaunchKernelGGL(duplicate_kernel, dim3(ceil_div(k, 256)), dim3(256), 0, st, k, f, f2);
}

int select_complex_states(hipStream_t st, int n, int k, const double* w2, const double* X, int ldx, int k2,
                          double* U, int ldu, int* dsrc)
{
    // complex state l stands for the real pair (2l, 2l+1); consecutive states
    // whose values agree to 1e-9 (relative above 1 Ha) form a cluster
    std::vector<int> src(k);
    std::vector<double> mu(n);
    for (int l = 0; l < n; ++l) mu[l] = 0.5 * (w2[2 * l] + w2[2 * l + 1]);
    auto close = [&](int a, int b) {
        return std::fabs(mu[b] - mu[a]) <= 1e-9 * std::max(1.0, std::max(std::fabs(mu[a]), std::fabs(mu[b])));
    };
    struct Cluster { int l0, m, ncand; };
    std::vector<Cluster> multi;
    int l0 = 0;
    while (l0 < k) {
        int lend = l0 + 1;
        while (lend < n && close(lend - 1, lend)) ++lend;
        const int m = std::min(lend, k) - l0;              // wanted states in the cluster
        const int ncand = std::min(2 * lend, k2) - 2 * l0;  // computed real vectors of it
        if (m == 1 || ncand > kMaxCand) {
            // a single state: either vector of its pair; a cluster too large for
            // the selection kernel keeps every other vector
            for (int q = 0; q < m; ++q) src[l0 + q] = 2 * (l0 + q);
        } else {
            multi.push_back({l0, m, ncand});
            for (int q = 0; q < m; ++q) src[l0 + q] = 2 * (l0 + q);
        }
        l0 += m;
    }
    if (hipMemcpyAsync(dsrc, src.data(), sizeof(int) * (size_t)k, hipMemcpyHostToDevice, st) != hipSuccess)
        return kStatusHip;
    if (hipStreamSynchronize(st) != hipSuccess) return kStatusHip;   // src is host memory of this frame
    const int rows = 2 * n;
    hipLaunchKernelGGL(gather_columns_kernel, dim3(ceil_div(rows, 256), k), dim3(256), 0, st, rows, k, X, ldx, dsrc,
                       U, ldu);
    for (const Cluster& c : multi)
        hipLaunchKernelGGL(select_cluster_kernel, dim3(1), dim3(256), 0, st, rows, X + (size_t)2 * c.l0 * ldx, ldx,
                           c.ncand, c.m, U + (size_t)c.l0 * ldu, ldu);
    return 0;
}

}  // namespace eg
