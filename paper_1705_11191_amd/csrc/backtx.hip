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
// (T formed once per (g, k) by a separate kernel), applied to a slab of X
// columns as three FP64 matrix-core products (V^T X_W, T W, X_W - V W2).  Blocks run in anti-diagonal steps t = (G-1-g)+k:
// the windows of (g, k) and (g', k') overlap only when |(g+k) - (g'+k')| <= 1,
// so blocks of one step are independent and overlapping pairs keep their
// order; each step is one launch over all of its blocks and column slabs.
//
// Step (5).  Q1 = Q_0 Q_1 ... with Q_p = I - V_p T_p V_p^T from the panels of
// step (1); X <- Q1 X applies groups of panels last to first, each as three
// FP64 matrix-core products (V^T X with a deterministic split over rows).
//
// The transposed applications (X <- Q2^T X, X <- Q1^T X, in the reverse order
// and with each block's T transposed) carry residuals into the basis of the
// tridiagonal matrix for the refinement of the mixed-precision mode.
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
// (from G = V^T V and the tau's, by block doubling).
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
    // G = V^T V above the diagonal on the matrix cores: the ten 16 x 16 tiles on
    // and above the diagonal, each summed only over the window rows where both
    // of its column ranges can be nonzero (reflector i lives in rows
    // i .. i+b-1)
    {
        const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
        for (int t = wave; t < 10; t += 4) {
            const int I = t < 4 ? 0 : (t < 7 ? 1 : (t < 9 ? 2 : 3));
            const int J = t < 4 ? t : (t < 7 ? t - 3 : (t < 9 ? t - 5 : 3));
            const int k_hi = min(2 * NB2, 16 * I + 15 + b);
            double4_t acc = {0.0, 0.0, 0.0, 0.0};
            for (int kk = 16 * J; kk < k_hi; kk += 4)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[kk + lk][16 * I + li], Vs[kk + lk][16 * J + li], acc, 0,
                                                           0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * I + 4 * r + lk, j = 16 * J + li;
                Gs[i][j] = (i < j) ? acc[r] : 0.0;
            }
        }
    }
    for (int e = tid; e < NB2 * NB2; e += 256) {
        const int i = e % NB2, j = e / NB2;
        Ts[i][j] = (i == j) ? tau[i] : 0.0;   // tau is zero beyond the block's reflectors
    }
    __syncthreads();
    // T by doubling: for adjacent reflector blocks A, B (A first),
    // T_AB = -T_AA G_AB T_BB; blocks of 1, 2, 4, ... 32, each level two
    // parallel small products.  Y reuses the V area (V is no longer needed).
    double(*Ys)[NB2 + 1] = Vs;
    for (int sz = 1; sz < NB2; sz *= 2) {
        const int nout = (NB2 / (2 * sz)) * sz * sz;
        for (int e = tid; e < nout; e += 256) {
            const int pr = e / (sz * sz), rem = e % (sz * sz);
            const int a = rem % sz, bb = rem / sz;
            const int p0 = pr * 2 * sz, pb = p0 + sz;
            double y = 0.0;
            for (int jj = 0; jj <= bb; ++jj) y += Gs[p0 + a][pb + jj] * Ts[pb + jj][pb + bb];
            Ys[p0 + a][pb + bb] = y;
        }
        __syncthreads();
        for (int e = tid; e < nout; e += 256) {
            const int pr = e / (sz * sz), rem = e % (sz * sz);
            const int a = rem % sz, bb = rem / sz;
            const int p0 = pr * 2 * sz, pb = p0 + sz;
            double t = 0.0;
            for (int ii = a; ii < sz; ++ii) t += Ts[p0 + a][p0 + ii] * Ys[p0 + ii][pb + bb];
            Ts[p0 + a][pb + bb] = -t;
        }
        __syncthreads();
    }
    double* T = Tq + ((size_t)g * kmax + k) * NB2 * NB2;
    for (int e = tid; e < NB2 * NB2; e += 256) T[e] = Ts[e % NB2][e / NB2];   // column-major, ld 64
}

// One block reflector (g, k) applied to a slab of X columns per workgroup,
// 32 columns at a time; the launch covers every (g, k) on the
// anti-diagonal step t = (G-1-g) + k.  Blocks on one step touch disjoint row
// windows, and every pair of blocks whose windows overlap lands on different
// steps in the reverse-execution order (windows overlap only when g + k
// differ by at most one).
//
// Reflector i of the block is nonzero only in window rows i .. i+b-1, so V is
// a 128 x 64 parallelogram: the products skip the 16 x 4 MFMA blocks that lie
// outside it.  V and T sit in registers as MFMA operands for the whole slab;
// LDS holds only the current 32-column chunk of X and the two 64 x 32
// intermediates, which lets two workgroups share a CU.  Workgroups are
// numbered so that all slabs of one block run on one XCD (one L2 copy of V).
// Phase-3 row blocks of each wave (16-row blocks of the 128-row window with
// their first nonzero 4-column step), balanced to 20 MFMA steps per wave.
__device__ __forceinline__ void q2_rowblocks(int wave, int& rbA, int& kA0, int& nA, int& rbB, int& kB0)
{
    switch (wave) {
    case 0: rbA = 3; kA0 = 0; nA = 16; rbB = 0; kB0 = 0; break;
    case 1: rbA = 4; kA0 = 0; nA = 16; rbB = 7; kB0 = 48; break;
    case 2: rbA = 2; kA0 = 0; nA = 12; rbB = 1; kB0 = 0; break;
    default: rbA = 5; kA0 = 16; nA = 12; rbB = 6; kB0 = 32; break;
    }
}

// TRANS: apply the transposed block I - V T^T V^T (Q2^T runs the anti-diagonal
// steps in the opposite order); T^T is lower triangular, so row block rb of
// T^T W needs the K steps 0 .. 4 rb + 3, and the same row-block pairs keep 20
// MFMA steps per wave.
template <bool TRANS>
__global__ __launch_bounds__(256, 2) void q2_apply_step_kernel(int n, int b, int ncol, int qw, int t, int nb, int nslab,
                                                               const double* __restrict__ V2,
                                                               const double* __restrict__ Tq, int kmax, double* X,
                                                               int ldx)
{
    // phase 0: V (128 x 65); afterwards X chunk (128 x 33), W and W2 (64 x 33 each)
    __shared__ double lds[2 * NB2 * (NCB + 1) + 2 * NB2 * (NCB + 1)];
    double(*Vs)[NB2 + 1] = (double(*)[NB2 + 1])lds;
    double(*Xs)[NCB + 1] = (double(*)[NCB + 1])lds;
    double(*Ws)[NCB + 1] = (double(*)[NCB + 1])(lds + 2 * NB2 * (NCB + 1));
    double(*W2s)[NCB + 1] = (double(*)[NCB + 1])(lds + 3 * NB2 * (NCB + 1));

    const int bid = blockIdx.x;
    const int q = bid >> 3;
    const int slab = q % nslab;
    const int blk = (q / nslab) * 8 + (bid & 7);
    if (blk >= nb) return;
    const int nsweeps = n - 2;
    const int ngroups = ceil_div(nsweeps, b);
    const int g = ngroups - 1 - blk;
    const int k = t - blk;
    if (g < 0 || k < 0 || k >= q2_ntasks(n, b, g * b)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int s_lo = g * b;
    const int base = s_lo + 1 + k * b;
    const int wrows = min(2 * b - 1, n - base);
    const int cbeg = slab * qw, cend = min(ncol, cbeg + qw);

    // W2 = T W with T upper triangular: row block rb needs K from 16 rb.  Wave w
    // forms column block w & 1 of two row blocks with complementary K ranges
    // (rows 0 and 3, or 1 and 2): 20 MFMA steps each.
    const int t_cb = wave & 1;
    const int t_rb0 = (wave >> 1) ? 1 : 0, t_rb1 = 3 - t_rb0;
    double treg[20];
    const int tA = TRANS ? 4 * t_rb0 + 4 : 0;   // (TRANS) steps of the first row block (4 or 8)
    {
        const double* T = Tq + ((size_t)g * kmax + k) * NB2 * NB2;
        if (TRANS) {
#pragma unroll
            for (int q = 0; q < 20; ++q) {
                const int rb = (q < tA) ? t_rb0 : t_rb1;
                const int kq = (q < tA) ? q : q - tA;
                treg[q] = T[(4 * kq + lk) + (size_t)(rb * 16 + li) * NB2];   // T^T(16 rb + li, 4 kq + lk)
            }
        } else {
            const int n0 = 16 - 4 * t_rb0;   // steps of the first row block (16 or 12)
#pragma unroll
            for (int q = 0; q < 20; ++q) {
                const int rb = (q < n0) ? t_rb0 : t_rb1;
                const int kq = (q < n0) ? 4 * t_rb0 + q : 4 * t_rb1 + (q - n0);
                treg[q] = T[(rb * 16 + li) + (size_t)(4 * kq + lk) * NB2];
            }
        }
    }
    const int xr = tid & 127, xc = tid >> 7;
    double xv[NCB / 2];
    auto load_x = [&](int c0) {
#pragma unroll
        for (int j = 0; j < NCB / 2; ++j) {
            const int gc = c0 + xc + 2 * j;
            xv[j] = (xr < wrows && gc < cend) ? X[cm(base + xr, gc, ldx)] : 0.0;
        }
    };
    load_x(cbeg);
    q2_load_v(n, b, g, k, V2, Vs);
    __syncthreads();

    // phase-1 operand: V^T rows 16w.., window rows 16w .. 16w+79
    double va1[20];
#pragma unroll
    for (int j = 0; j < 20; ++j) va1[j] = Vs[16 * wave + 4 * j + lk][16 * wave + li];
    int rbA, kA0, nA, rbB, kB0;
    q2_rowblocks(wave, rbA, kA0, nA, rbB, kB0);
    double va3[20];
#pragma unroll
    for (int j = 0; j < 20; ++j)
        va3[j] = (j < nA) ? Vs[16 * rbA + li][kA0 + 4 * j + lk] : Vs[16 * rbB + li][kB0 + 4 * (j - nA) + lk];
    __syncthreads();   // the V area now holds X chunks

    for (int c0 = cbeg; c0 < cend; c0 += NCB) {
#pragma unroll
        for (int j = 0; j < NCB / 2; ++j) Xs[xr][xc + 2 * j] = xv[j];
        __syncthreads();
        if (c0 + NCB < cend) load_x(c0 + NCB);
        // W = V^T X (64 x 32): wave w owns rows 16w .. 16w+15
        {
            double4_t a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < 20; ++j) {
                const int kk = 16 * wave + 4 * j + lk;
                a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(va1[j], Xs[kk][li], a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(va1[j], Xs[kk][16 + li], a1, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Ws[16 * wave + 4 * r + lk][li] = a0[r];
                Ws[16 * wave + 4 * r + lk][16 + li] = a1[r];
            }
        }
        __syncthreads();
        // W2 = T W (64 x 32), or T^T W
        if (TRANS) {
            double4_t a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
            const int cc = 16 * t_cb + li;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[4 * q + lk][cc], a0, 0, 0, 0);
            if (tA == 8) {
#pragma unroll
                for (int q = 4; q < 8; ++q)
                    a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[4 * q + lk][cc], a0, 0, 0, 0);
            } else {
#pragma unroll
                for (int q = 4; q < 8; ++q)
                    a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[4 * (q - 4) + lk][cc], a1, 0, 0, 0);
            }
#pragma unroll
            for (int q = 8; q < 20; ++q)
                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[4 * (q - tA) + lk][cc], a1, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                W2s[16 * t_rb0 + 4 * r + lk][cc] = a0[r];
                W2s[16 * t_rb1 + 4 * r + lk][cc] = a1[r];
            }
        } else {
            double4_t a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
            const int n0 = 16 - 4 * t_rb0;
            const int cc = 16 * t_cb + li;
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const int kk = 4 * (4 * t_rb0 + q) + lk;
                a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[kk][cc], a0, 0, 0, 0);
            }
            if (n0 == 16) {
#pragma unroll
                for (int q = 12; q < 16; ++q) {
                    const int kk = 4 * q + lk;
                    a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[kk][cc], a0, 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int q = 12; q < 16; ++q) {
                    const int kk = 4 * (4 * t_rb1 + (q - 12)) + lk;
                    a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[kk][cc], a1, 0, 0, 0);
                }
            }
#pragma unroll
            for (int q = 16; q < 20; ++q) {
                const int kk = 4 * (4 * t_rb1 + (q - n0)) + lk;
                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(treg[q], Ws[kk][cc], a1, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                W2s[16 * t_rb0 + 4 * r + lk][cc] = a0[r];
                W2s[16 * t_rb1 + 4 * r + lk][cc] = a1[r];
            }
        }
        __syncthreads();
        // X -= V W2 on the wave's two row blocks; operands swapped so that a
        // lane's results run down a column: lane l, element r holds
        // (V W2)(16 rb + l % 16, 16 cb + 4 r + l / 16)
        {
            double4_t A0 = {0, 0, 0, 0}, A1 = {0, 0, 0, 0}, B0 = {0, 0, 0, 0}, B1 = {0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const int kk = kA0 + 4 * j + lk;
                A0 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][li], va3[j], A0, 0, 0, 0);
                A1 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][16 + li], va3[j], A1, 0, 0, 0);
            }
            if (nA == 16) {
#pragma unroll
                for (int j = 12; j < 16; ++j) {
                    const int kk = kA0 + 4 * j + lk;
                    A0 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][li], va3[j], A0, 0, 0, 0);
                    A1 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][16 + li], va3[j], A1, 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int j = 12; j < 16; ++j) {
                    const int kk = kB0 + 4 * (j - 12) + lk;
                    B0 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][li], va3[j], B0, 0, 0, 0);
                    B1 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][16 + li], va3[j], B1, 0, 0, 0);
                }
            }
#pragma unroll
            for (int j = 16; j < 20; ++j) {
                const int kk = kB0 + 4 * (j - nA) + lk;
                B0 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][li], va3[j], B0, 0, 0, 0);
                B1 = __builtin_amdgcn_mfma_f64_16x16x4f64(W2s[kk][16 + li], va3[j], B1, 0, 0, 0);
            }
            const int ra = 16 * rbA + li, rb = 16 * rbB + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 4 * r + lk;
                if (ra < wrows && c0 + c < cend) X[cm(base + ra, c0 + c, ldx)] = Xs[ra][c] - A0[r];
                if (ra < wrows && c0 + 16 + c < cend) X[cm(base + ra, c0 + 16 + c, ldx)] = Xs[ra][16 + c] - A1[r];
                if (rb < wrows && c0 + c < cend) X[cm(base + rb, c0 + c, ldx)] = Xs[rb][c] - B0[r];
                if (rb < wrows && c0 + 16 + c < cend) X[cm(base + rb, c0 + 16 + c, ldx)] = Xs[rb][16 + c] - B1[r];
            }
        }
        __syncthreads();   // Xs, W, W2 free for the next chunk
    }
}

}  // namespace

// Columns of X per workgroup: wide slabs amortize the loads of V and T, narrow
// ones keep enough workgroups in flight.  The width follows the column count,
// halved while the busiest step (about half of the row groups active) would
// have fewer than about 1024 workgroups: N = 8,192 with 2,050 columns takes
// 128 (Q2 18.3 -> 16.6 ms against 256), N = 32,768 with 8,194 columns 512.
int q2_slab_width(int n, int b, int ncol)
{
    int w = ncol >= 8192 ? 512 : (ncol >= 2048 ? 256 : 128);
    const long long busy = std::max(1, ceil_div(std::max(n - 2, 1), b) / 2);
    while (w > 128 && busy * ceil_div(ncol, w) < 1024) w /= 2;
    return w;
}

size_t apply_q2_workspace_doubles(int n, int b)
{
    const int ngroups = std::max(1, ceil_div(std::max(n - 2, 1), b));
    const int kmax = n >= 2 ? (n - 2) / b + 1 : 1;
    return (size_t)ngroups * kmax * NB2 * NB2;
}

void build_q2_t(hipStream_t st, int n, int b, const double* V2, const double* tau2, int kmax, double* Tq)
{
    if (n <= 2) return;
    hipLaunchKernelGGL(q2_build_t_kernel, dim3(ceil_div(n - 2, b), kmax), dim3(256), 0, st, n, b, V2, tau2, kmax, Tq);
}

// X (n x ncol) <- Q2 X, or Q2^T X (trans); Tq: apply_q2_workspace_doubles(n, b)
// doubles, rebuilt from the reflectors unless tq_ready says a previous call on
// the same reflectors left it there.  slab: columns per workgroup (0 picks
// q2_slab_width(n, b, ncol); otherwise 128, 256 or 512).
void apply_q2(hipStream_t st, int n, int b, int ncol, const double* V2, const double* tau2, int kmax, double* X,
              int ldx, double* Tq, bool trans, bool tq_ready, int slab)
{
    if (n <= 2 || ncol <= 0) return;
    const int ngroups = ceil_div(n - 2, b);
    if (!tq_ready) build_q2_t(st, n, b, V2, tau2, kmax, Tq);
    const int qw = slab > 0 ? slab : q2_slab_width(n, b, ncol);
    const int nslab = ceil_div(ncol, qw);
    const int tmax = (ngroups - 1) + kmax;   // last step: g = 0 with its last block
    for (int s = 0; s < tmax; ++s) {
        const int t = trans ? tmax - 1 - s : s;
        const int nb = std::min(ngroups, t + 1);   // block index G-1-g ranges over 0 .. min(G-1, t)
        const int nwg = ceil_div(nb, 8) * 8 * nslab;
        if (trans)
            hipLaunchKernelGGL(q2_apply_step_kernel<true>, dim3(nwg), dim3(256), 0, st, n, b, ncol, qw, t, nb, nslab,
                               V2, Tq, kmax, X, ldx);
        else
            hipLaunchKernelGGL(q2_apply_step_kernel<false>, dim3(nwg), dim3(256), 0, st, n, b, ncol, qw, t, nb, nslab,
                               V2, Tq, kmax, X, ldx);
    }
}

// Q1 is applied in groups of Q1G consecutive panels: their product
// Q_p ... Q_{p+Q1G-1} = I - V' T' V'^T with V' = [V_p ... V_{p+Q1G-1}] (the
// later panels' columns are zero above their first row) and T' upper
// triangular, built block column by block column from
//   T'(0:c, block q) = -T'(0:c, 0:c) (V'(:, 0:c)^T V_q) T_q,
// so that every application is a product with K = Q1G b.
constexpr int Q1G = kQ1Group;

// panels with at least two rows below them carry reflectors (full width b)
static int q1_panels(int n, int b)
{
    int nvalid = 0;
    while (n - (nvalid + 1) * b >= 2) ++nvalid;
    return nvalid;
}

size_t apply_q1_workspace_doubles(int n, int ncol)
{
    const size_t w = (size_t)Q1G * 64;
    const size_t c = (size_t)std::max(ncol, 1);
    (void)n;
    return 2 * w * c + 8 * w * c + 2 * w * w + w * 64;
}

size_t q1_tfactor_doubles(int n, int b)
{
    const size_t w = (size_t)Q1G * 64;
    return (size_t)std::max(1, ceil_div(q1_panels(n, b), Q1G)) * w * w;
}

// T' of group g (two panels or more) into Tg (ld Q1G*64), block column by
// block column; Gg (Q1G*64 square) and tmp (Q1G*64 x 64) are scratch, part
// the split-K partials of the Gram matrix V'^T V'.
static void q1_group_t(hipStream_t st, int n, int b, int g, int nvalid, const double* Vall, const double* Tall,
                       double* Tg, double* Gg, double* tmp, double* part, size_t npart)
{
    const int wmax = Q1G * 64;
    const int p0 = g * Q1G;
    const int np = std::min(Q1G, nvalid - p0);
    const int w = np * b;
    const int j0 = p0 * b;
    const int r0 = j0 + b;
    const int m = n - r0;
    const double* V = Vall + cm(r0, j0, n);
    const double* T = Tall + (size_t)p0 * b * b;
    dgemm_splitk(st, 'T', 'N', w, w, m, 1.0, V, n, V, n, 0.0, Gg, wmax, part, npart);
    fill_d(st, Tg, (size_t)wmax * w, 0.0);
    for (int q = 0; q < np; ++q)
        copy_matrix(st, b, b, T + (size_t)q * b * b, b, Tg + cm(q * b, q * b, wmax), wmax);
    for (int q = 1; q < np; ++q) {
        const int c = q * b;
        dgemm(st, 'N', 'N', c, b, b, 1.0, Gg + cm(0, c, wmax), wmax, T + (size_t)q * b * b, b, 0.0, tmp, wmax);
        dgemm(st, 'N', 'N', c, b, c, -1.0, Tg, wmax, tmp, wmax, 0.0, Tg + cm(0, c, wmax), wmax);
    }
}

void build_q1_t(hipStream_t st, int n, int b, int ncol, const double* Vall, const double* Tall, double* Tq1,
                double* work)
{
    // the scratch apply_q1 uses for its own T' with ncol columns
    const int wmax = Q1G * 64;
    const size_t c = (size_t)std::max(ncol, 1);
    double* part = work + 2 * (size_t)wmax * c;
    const size_t npart = (size_t)8 * wmax * c;
    double* Gg = part + npart + (size_t)wmax * wmax;
    double* tmp = Gg + (size_t)wmax * wmax;
    const int nvalid = q1_panels(n, b);
    const int ngroups = ceil_div(nvalid, Q1G);
    for (int g = 0; g < ngroups; ++g)
        if (std::min(Q1G, nvalid - g * Q1G) >= 2)
            q1_group_t(st, n, b, g, nvalid, Vall, Tall, Tq1 + (size_t)g * wmax * wmax, Gg, tmp, part, npart);
}

// X (n x ncol) <- Q1 X with the panel reflectors of step (1), or Q1^T X
// (trans: the groups first to last, each with its T'^T).
void apply_q1(hipStream_t st, int n, int b, int ncol, const double* Vall, const double* Tall, double* X, int ldx,
              double* work, bool trans, const double* Tq1)
{
    if (ncol <= 0) return;
    const int wmax = Q1G * 64;
    double* W = work;                                // wmax x ncol
    double* W2 = W + (size_t)wmax * ncol;            // wmax x ncol
    double* part = W2 + (size_t)wmax * ncol;         // split-K partials
    const size_t npart = (size_t)8 * wmax * ncol;
    double* Tg = part + npart;                       // wmax x wmax
    double* Gg = Tg + (size_t)wmax * wmax;           // wmax x wmax
    double* tmp = Gg + (size_t)wmax * wmax;          // wmax x 64
    const int nvalid = q1_panels(n, b);
    const int ngroups = ceil_div(nvalid, Q1G);
    const char tt = trans ? 'T' : 'N';
    for (int gi = 0; gi < ngroups; ++gi) {
        const int g = trans ? gi : ngroups - 1 - gi;
        const int p0 = g * Q1G;
        const int np = std::min(Q1G, nvalid - p0);
        const int w = np * b;
        const int j0 = p0 * b;
        const int r0 = j0 + b;
        const int m = n - r0;
        const double* V = Vall + cm(r0, j0, n);
        const double* T = Tall + (size_t)p0 * b * b;
        if (np == 1) {
            dgemm_splitk(st, 'T', 'N', b, ncol, m, 1.0, V, n, X + r0, ldx, 0.0, W, wmax, part, npart);
            dgemm(st, tt, 'N', b, ncol, b, 1.0, T, b, W, wmax, 0.0, W2, wmax);
            dgemm(st, 'N', 'N', m, ncol, b, -1.0, V, n, W2, wmax, 1.0, X + r0, ldx);
            continue;
        }
        // T' of the group: built beforehand, or here
        const double* Tp = Tg;
        if (Tq1)
            Tp = Tq1 + (size_t)g * wmax * wmax;
        else
            q1_group_t(st, n, b, g, nvalid, Vall, Tall, Tg, Gg, tmp, part, npart);
        dgemm_splitk(st, 'T', 'N', w, ncol, m, 1.0, V, n, X + r0, ldx, 0.0, W, wmax, part, npart);
        dgemm(st, tt, 'N', w, ncol, w, 1.0, Tp, wmax, W, wmax, 0.0, W2, wmax);
        dgemm(st, 'N', 'N', m, ncol, w, -1.0, V, n, W2, wmax, 1.0, X + r0, ldx);
    }
}

}  // namespace eg
