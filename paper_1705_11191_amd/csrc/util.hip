// Element-wise helpers, the density-matrix column scaling and the chemical
// potential / occupation kernel.
#include "common.h"
#include "../../include/elsi_gpu.h"

namespace eg {
namespace {

__global__ void fill_d_kernel(double* p, size_t count, double v)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; e < count; e += stride) p[e] = v;
}

__global__ void fill_i_kernel(int* p, size_t count, int v)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; e < count; e += stride) p[e] = v;
}

__global__ void copy_matrix_kernel(int m, int n, const double* A, int lda, double* B, int ldb)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    for (; j < n; j += gridDim.y)
        if (i < m) B[cm(i, j, ldb)] = A[cm(i, j, lda)];
}

// Several independent column-major copies in one launch (blockIdx.z picks the
// copy); the packing of the update operands takes one launch instead of one
// per block.
__global__ void copy_batch_kernel(CopyBatch cb)
{
    const CopyDesc d = cb.d[blockIdx.z];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.m) return;
    for (int j = blockIdx.y; j < d.n; j += gridDim.y) d.B[cm(i, j, d.ldb)] = d.A[cm(i, j, d.lda)];
}

// Copy the lower triangle onto the upper one through a 32 x 32 LDS tile so
// that both the reads and the writes are coalesced.
__global__ void mirror_kernel(int n, double* A, int lda)
{
    __shared__ double t[32][33];
    int bi = blockIdx.x, bj = blockIdx.y;   // source tile (bi, bj) with bi >= bj
    if (bi < bj) return;
    int tx = threadIdx.x, ty = threadIdx.y; // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        int gi = bi * 32 + tx, gj = bj * 32 + r;
        t[r][tx] = (gi < n && gj < n) ? A[cm(gi, gj, lda)] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        // destination (row = bj*32 + tx, col = bi*32 + r) = source (bi*32 + r, bj*32 + tx)
        int di = bj * 32 + tx, dj = bi * 32 + r;
        if (di < n && dj < n && di < dj) A[cm(di, dj, lda)] = t[tx][r];
    }
}

// A <- (A + A^T) / 2 for one pair of 32 x 32 tiles (bi, bj), bi >= bj.
__global__ void symmetrize_kernel(int n, double* A, int lda)
{
    __shared__ double lo[32][33];
    __shared__ double up[32][33];
    int bi = blockIdx.x, bj = blockIdx.y;
    if (bi < bj) return;
    int tx = threadIdx.x, ty = threadIdx.y;
    for (int r = ty; r < 32; r += 8) {
        int gi = bi * 32 + tx, gj = bj * 32 + r;          // lower tile element (gi, gj)
        lo[r][tx] = (gi < n && gj < n) ? A[cm(gi, gj, lda)] : 0.0;
        int ui = bj * 32 + tx, uj = bi * 32 + r;          // upper tile element (ui, uj)
        up[r][tx] = (ui < n && uj < n) ? A[cm(ui, uj, lda)] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        // lower (bi*32+tx, bj*32+r) pairs with upper (bj*32+r, bi*32+tx) = up[tx][r]
        int gi = bi * 32 + tx, gj = bj * 32 + r;
        if (gi < n && gj < n && gi > gj) {
            double v = 0.5 * (lo[r][tx] + up[tx][r]);
            A[cm(gi, gj, lda)] = v;
        }
        int ui = bj * 32 + tx, uj = bi * 32 + r;           // upper (ui, uj) pairs with lo[tx][r]
        if (ui < n && uj < n && ui < uj) {
            double v = 0.5 * (up[r][tx] + lo[tx][r]);
            A[cm(ui, uj, lda)] = v;
        }
    }
}

__global__ void identity_kernel(int n, double* A, int lda)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    for (; j < n; j += gridDim.y)
        if (i < n) A[cm(i, j, lda)] = (i == j) ? 1.0 : 0.0;
}

__global__ void scale_sqrt_kernel(int n, int k, const double* C, int ldc, const double* f, double* out,
                                  int ldo)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    for (; j < k; j += gridDim.y) {
        double s = sqrt(fmax(f[j], 0.0));
        if (i < n) out[cm(i, j, ldo)] = s * C[cm(i, j, ldc)];
    }
}

// out = C sqrt|f| and out2 = C sign(f) sqrt|f| (columnwise), so that
// out out2^T = C diag(f) C^T for occupations of either sign
__global__ void scale_signed_kernel(int n, int k, const double* C, int ldc, const double* f, double* out,
                                   double* out2, int ldo)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    for (; j < k; j += gridDim.y) {
        const double fj = f[j];
        const double s = sqrt(fabs(fj));
        if (i < n) {
            const double v = s * C[cm(i, j, ldc)];
            out[cm(i, j, ldo)] = v;
            out2[cm(i, j, ldo)] = (fj < 0.0) ? -v : v;
        }
    }
}

__global__ void finite_kernel(int m, int n, const double* A, int lda, int* flag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    for (; j < n; j += gridDim.y)
        if (i < m && !isfinite(A[cm(i, j, lda)])) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Occupations (Eq. (17)) and chemical potential (Eq. (18)) by bisection, as
// described for elsi_dm_real (Sec. 4.5): start from [eps_min - 10 kT,
// eps_max + 10 kT], widen each side (doubling the step) until the electron
// count brackets N_e, halve keeping a surplus at the upper bound until that
// surplus is within occ_accuracy or the midpoint stops moving, take mu at the
// upper bound and strip the remaining surplus from the highest occupied
// states downward.  One workgroup; electron counts are block reductions in a
// fixed order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int FD_THREADS = 1024;

// Occupation of one state, x = (eps - mu) / width, for the broadening schemes
// (Sec. 4.6): Fermi-Dirac, Eq. (17), without overflowing exponentials;
// Gaussian, Eq. (21), f = spin (1 - erf x) / 2 = spin erfc(x) / 2;
// Methfessel-Paxton order 0 (the Gaussian step) and order 1,
// f = spin (erfc(x) / 2 - x e^{-x^2} / (2 sqrt(pi))) (Methfessel & Paxton,
// Phys. Rev. B 40, 3616 (1989)), which leaves [0, spin] near mu.
__device__ inline double occ_value(int scheme, double eps, double mu, double width, double spin)
{
    const double x = (eps - mu) / width;
    if (scheme == ELSI_GPU_OCC_GAUSSIAN || scheme == ELSI_GPU_OCC_MP0) return spin * 0.5 * erfc(x);
    if (scheme == ELSI_GPU_OCC_MP1)
        return spin * (0.5 * erfc(x) - x * exp(-x * x) / (2.0 * sqrt(3.14159265358979323846)));
    if (x >= 0.0) {
        double t = exp(-x);
        return spin * t / (1.0 + t);
    }
    return spin / (1.0 + exp(x));
}

__device__ double block_sum(double v, double* red)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
        for (int w = 0; w < FD_THREADS / 64; ++w) s += red[w];
        red[FD_THREADS / 64] = s;
    }
    __syncthreads();
    return red[FD_THREADS / 64];
}

// max (is_max) or min of v over the block
__device__ double block_extreme(double v, double* red, bool is_max)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(v, off, 64);
        v = is_max ? fmax(v, o) : fmin(v, o);
    }
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = red[0];
        for (int w = 1; w < FD_THREADS / 64; ++w) s = is_max ? fmax(s, red[w]) : fmin(s, red[w]);
        red[FD_THREADS / 64] = s;
    }
    __syncthreads();
    return red[FD_THREADS / 64];
}

// electrons at mu: sum_l w_l f_l (w NULL: all 1)
__device__ double count_electrons(int n, const double* eps, const double* w, int scheme, double mu, double width,
                                  double spin, double* red)
{
    double s = 0.0;
    for (int l = threadIdx.x; l < n; l += FD_THREADS) s += (w ? w[l] : 1.0) * occ_value(scheme, eps[l], mu, width, spin);
    return block_sum(s, red);
}

// The chemical potential by bisection (Eq. (18), Sec. 4.5; with per-state
// weights the electron count runs over k-points and spin channels): the
// interval [min eps - 10 width, max eps + 10 width] is widened (the step
// doubling, at most 64 times per side) until it brackets N_e, then halved
// keeping a surplus at the upper bound until that surplus is within
// occ_accuracy, the midpoint stops moving, or max_steps halvings were made;
// mu is the upper bound, f_l = w_l f(eps_l), and the remaining surplus is
// stripped from the highest-index states with f > 0 downward.  k_s: one past
// the last state with |f| > f_cut.
__global__ __launch_bounds__(FD_THREADS) void occupations_kernel(int n, const double* eps, const double* w, int scheme,
                                                                double ne, double width, double spin, double acc,
                                                                int max_steps, double f_cut, double* f, double* scal)
{
    __shared__ double red[FD_THREADS / 64 + 1];
    __shared__ double sh_surplus;
    double vmin = INFINITY, vmax = -INFINITY;
    for (int l = threadIdx.x; l < n; l += FD_THREADS) {
        vmin = fmin(vmin, eps[l]);
        vmax = fmax(vmax, eps[l]);
    }
    vmin = block_extreme(vmin, red, false);
    vmax = block_extreme(vmax, red, true);
    double lo = vmin - 10.0 * width, hi = vmax + 10.0 * width;
    double step = hi - lo;
    for (int t = 0; t < 64 && count_electrons(n, eps, w, scheme, lo, width, spin, red) - ne > 0.0; ++t) {
        lo -= step;
        step *= 2.0;
    }
    step = hi - lo;
    for (int t = 0; t < 64 && count_electrons(n, eps, w, scheme, hi, width, spin, red) - ne < 0.0; ++t) {
        hi += step;
        step *= 2.0;
    }
    int status = 0, steps = 0;
    for (;;) {
        double mid = 0.5 * (lo + hi);
        if (!(lo < mid && mid < hi)) break;
        if (steps >= max_steps) { status = kStatusMu; break; }
        ++steps;
        double g = count_electrons(n, eps, w, scheme, mid, width, spin, red) - ne;
        if (g >= 0.0) {
            hi = mid;
            if (g <= acc) break;
        } else {
            lo = mid;
        }
    }
    const double mu = hi;
    for (int l = threadIdx.x; l < n; l += FD_THREADS) f[l] = (w ? w[l] : 1.0) * occ_value(scheme, eps[l], mu, width, spin);
    double total = count_electrons(n, eps, w, scheme, mu, width, spin, red);
    __syncthreads();
    if (threadIdx.x == 0) {
        double surplus = total - ne;
        for (int l = n - 1; l >= 0 && surplus > 0.0; --l) {
            double fl = f[l];
            if (fl <= 0.0) continue;
            double take = fl < surplus ? fl : surplus;
            f[l] = fl - take;
            surplus -= take;
        }
        sh_surplus = surplus;
    }
    __syncthreads();
    double last = -1.0, en = 0.0;
    for (int l = threadIdx.x; l < n; l += FD_THREADS) {
        double fl = f[l];
        if (fabs(fl) > f_cut) last = fmax(last, (double)l);
        en += fl * eps[l];
    }
    double ks = block_extreme(last, red, true) + 1.0;
    double energy = block_sum(en, red);
    if (threadIdx.x == 0) {
        scal[0] = mu;
        scal[1] = (double)status;
        scal[2] = ks;
        scal[3] = energy;
        scal[4] = (double)steps;
        scal[5] = sh_surplus;
    }
}

__global__ __launch_bounds__(FD_THREADS) void explicit_occ_kernel(int n, const double* eps, const double* f,
                                                                  double f_cut, double* scal)
{
    __shared__ double red[FD_THREADS / 64 + 1];
    double en = 0.0, last = -1.0;
    for (int l = threadIdx.x; l < n; l += FD_THREADS) {
        en += f[l] * eps[l];
        if (fabs(f[l]) > f_cut) last = fmax(last, (double)l);
    }
    double energy = block_sum(en, red);
    // maximum of `last` through the same reduction shape
    for (int off = 32; off > 0; off >>= 1) last = fmax(last, __shfl_down(last, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = last;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = -1.0;
        for (int w = 0; w < FD_THREADS / 64; ++w) m = fmax(m, red[w]);
        scal[0] = 0.0;
        scal[1] = 0.0;
        scal[2] = m + 1.0;
        scal[3] = energy;
        scal[4] = 0.0;
        scal[5] = 0.0;
    }
}

}  // namespace

void explicit_occupations(hipStream_t st, int n, int n_state, const double* eps, const double* f,
                          double f_cut, double* scal)
{
    (void)n_state;
    hipLaunchKernelGGL(explicit_occ_kernel, dim3(1), dim3(FD_THREADS), 0, st, n, eps, f, f_cut, scal);
}

void fill_d(hipStream_t st, double* p, size_t count, double v)
{
    if (!count) return;
    unsigned g = (unsigned)std::min<size_t>((count + 255) / 256, 65535);
    hipLaunchKernelGGL(fill_d_kernel, dim3(g), dim3(256), 0, st, p, count, v);
}

void fill_i(hipStream_t st, int* p, size_t count, int v)
{
    if (!count) return;
    unsigned g = (unsigned)std::min<size_t>((count + 255) / 256, 65535);
    hipLaunchKernelGGL(fill_i_kernel, dim3(g), dim3(256), 0, st, p, count, v);
}

void copy_matrix(hipStream_t st, int m, int n, const double* A, int lda, double* B, int ldb)
{
    if (m <= 0 || n <= 0) return;
    dim3 grid(ceil_div(m, 256), std::min(n, 65535));
    hipLaunchKernelGGL(copy_matrix_kernel, grid, dim3(256), 0, st, m, n, A, lda, B, ldb);
}

void copy_matrices(hipStream_t st, const CopyBatch& cb)
{
    int mmax = 0, nmax = 0;
    for (int c = 0; c < cb.count; ++c) {
        mmax = std::max(mmax, cb.d[c].m);
        nmax = std::max(nmax, cb.d[c].n);
    }
    if (cb.count <= 0 || mmax <= 0 || nmax <= 0) return;
    dim3 grid(ceil_div(mmax, 256), std::min(nmax, 65535), cb.count);
    hipLaunchKernelGGL(copy_batch_kernel, grid, dim3(256), 0, st, cb);
}

void mirror_lower_to_upper(hipStream_t st, int n, double* A, int lda)
{
    if (n <= 1) return;
    int t = ceil_div(n, 32);
    hipLaunchKernelGGL(mirror_kernel, dim3(t, t), dim3(32, 8), 0, st, n, A, lda);
}

void symmetrize_average(hipStream_t st, int n, double* A, int lda)
{
    if (n <= 1) return;
    int t = ceil_div(n, 32);
    hipLaunchKernelGGL(symmetrize_kernel, dim3(t, t), dim3(32, 8), 0, st, n, A, lda);
}

void set_identity(hipStream_t st, int n, double* A, int lda)
{
    if (n <= 0) return;
    dim3 grid(ceil_div(n, 256), std::min(n, 65535));
    hipLaunchKernelGGL(identity_kernel, grid, dim3(256), 0, st, n, A, lda);
}

void scale_columns_sqrt(hipStream_t st, int n, int k, const double* C, int ldc, const double* f,
                        double* out, int ldo)
{
    if (n <= 0 || k <= 0) return;
    dim3 grid(ceil_div(n, 256), std::min(k, 65535));
    hipLaunchKernelGGL(scale_sqrt_kernel, grid, dim3(256), 0, st, n, k, C, ldc, f, out, ldo);
}

void scale_columns_signed(hipStream_t st, int n, int k, const double* C, int ldc, const double* f, double* out,
                          double* out2, int ldo)
{
    if (n <= 0 || k <= 0) return;
    dim3 grid(ceil_div(n, 256), std::min(k, 65535));
    hipLaunchKernelGGL(scale_signed_kernel, grid, dim3(256), 0, st, n, k, C, ldc, f, out, out2, ldo);
}

void check_finite(hipStream_t st, int m, int n, const double* A, int lda, int* flag)
{
    if (m <= 0 || n <= 0) return;
    dim3 grid(ceil_div(m, 256), std::min(n, 65535));
    hipLaunchKernelGGL(finite_kernel, grid, dim3(256), 0, st, m, n, A, lda, flag);
}

void occupations(hipStream_t st, int n, const double* eps, const double* weight, int scheme, double n_electron,
                 double width, double spin, double occ_accuracy, int max_steps, double f_cut, double* f, double* scal)
{
    hipLaunchKernelGGL(occupations_kernel, dim3(1), dim3(FD_THREADS), 0, st, n, eps, weight, scheme, n_electron,
                       width, spin, occ_accuracy, max_steps, f_cut, f, scal);
}

}  // namespace eg
