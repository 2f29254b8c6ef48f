// Step (1) of the two-stage tridiagonalization (ELSI paper, Sec. 3.1,
// Eq. (13) and Fig. 1): B = Q1^T H~ Q1 with bandwidth b.
//
// Panel p covers columns j .. j+b-1.  Its sub-band block P = A(j+b:n, j:j+b)
// (m x b) is reduced to upper triangular form by b Householder reflectors
// H_c = I - tau_c v_c v_c^T, and the trailing matrix A22 = A(j+b:n, j+b:n)
// receives the two-sided block update Q^T A22 Q with Q = I - V T V^T:
//     Y = A22 V,  X = Y T,  W = X - 1/2 V (T^T (V^T X)),
//     A22 <- A22 - V W^T - W V^T,
// all as FP64 matrix-core products.  Only the lower triangle of A22 is read
// (Y by a symmetric product) and updated (the rank-2b update skips tiles
// above the diagonal).
//
// The panel QR uses one kernel launch per column.  A reflector for column c
// needs x = P(c:m, c) only through x^T P(c:m, r) (r >= c), so each launch
// (1) reduces the per-workgroup partial Gram row of column c left by the
// previous launch, (2) applies reflector c to its rows, and (3) forms the
// partial Gram row of column c+1 -- one grid-wide reduction per column.
#include "common.h"

namespace eg {
namespace {

constexpr int PR = 256;    // panel rows per workgroup (one row per thread)
constexpr int BMAX = 64;
constexpr int GS = BMAX + 2;   // per-block partial record: Gram row (64), tail, spare

__device__ inline double wave_sum(double v) { return wave_sum_dpp(v); }

// c >= 0: apply reflector c (its Gram row is in gin, row c in rin) and form the
// Gram record of column c+1.  c == -1: only form the record of column 0.
__global__ __launch_bounds__(PR) void panel_step_kernel(int m, int bw, int c, double* P, int ldp,
                                                        const double* __restrict__ gin, double* gout,
                                                        const double* __restrict__ rin, double* rout,
                                                        double* tau, int nblk)
{
    __shared__ double G[BMAX + 1];
    __shared__ double scoef[BMAX];
    __shared__ double red[PR / 64][BMAX + 1];
    __shared__ double sh[4];
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const int i = blk * PR + tid;
    const int lane = tid & 63, wave = tid >> 6;

    double rowv[BMAX];
    const bool have_row = (i < m) && (i >= (c < 0 ? 0 : c));
#pragma unroll
    for (int r = 0; r < BMAX; ++r) {
        rowv[r] = 0.0;
        if (r < bw && r >= (c < 0 ? 0 : c) && have_row) rowv[r] = P[cm(i, r, ldp)];
    }

    if (c >= 0) {
        // (1) Gram row of column c over rows >= c, and the squared tail over rows > c
        for (int r = tid; r <= BMAX; r += PR) {
            if ((r >= c && r < bw) || r == BMAX) {
                double s = 0.0;
                for (int b = 0; b < nblk; ++b) s += gin[(size_t)b * GS + r];
                G[r] = s;
            }
        }
        __syncthreads();
        if (tid == 0) {
            double x0 = rin[c];
            double tail = G[BMAX];
            double t = 0.0, alpha = x0, den = 1.0;
            if (tail > 0.0) {
                double nrm = sqrt(x0 * x0 + tail);
                alpha = (x0 >= 0.0) ? -nrm : nrm;
                t = (alpha - x0) / alpha;
                den = x0 - alpha;
            }
            sh[0] = t; sh[1] = alpha; sh[2] = den;
            if (blk == 0) tau[c] = t;
        }
        __syncthreads();
        const double t = sh[0], alpha = sh[1], den = sh[2];
        for (int r = tid; r < bw; r += PR)
            if (r > c) scoef[r] = (t != 0.0) ? (G[r] - alpha * rin[r]) / den : 0.0;
        __syncthreads();
        // (2) apply H_c = I - t v v^T to this block's rows (v_c = 1, v_i = x_i / den)
        if (have_row) {
            double xc = 0.0;
#pragma unroll
            for (int r = 0; r < BMAX; ++r) if (r == c) xc = rowv[r];
            double vi = (i == c) ? 1.0 : ((t != 0.0) ? xc / den : 0.0);
#pragma unroll
            for (int r = 0; r < BMAX; ++r) {
                if (r > c && r < bw) {
                    rowv[r] -= t * vi * scoef[r];
                    P[cm(i, r, ldp)] = rowv[r];
                }
            }
            if (i == c) P[cm(i, c, ldp)] = alpha;
            else P[cm(i, c, ldp)] = vi;
        }
    }

    // (3) record of column cn = c+1: Gram row over rows >= cn, tail over rows > cn
    const int cn = c + 1;
    if (cn >= bw) return;
    double xn = 0.0;
#pragma unroll
    for (int r = 0; r < BMAX; ++r) if (r == cn) xn = rowv[r];
    if (!(i < m && i >= cn)) xn = 0.0;
#pragma unroll
    for (int r = 0; r < BMAX; ++r) {
        if (r >= cn && r < bw) {
            double s = wave_sum(xn * rowv[r]);
            if (lane == 0) red[wave][r] = s;
        }
    }
    {
        double tl = (i > cn && i < m) ? xn * xn : 0.0;
        double s = wave_sum(tl);
        if (lane == 0) red[wave][BMAX] = s;
    }
    __syncthreads();
    for (int r = tid; r <= BMAX; r += PR) {
        if ((r >= cn && r < bw) || r == BMAX) {
            double s = 0.0;
            for (int w = 0; w < PR / 64; ++w) s += red[w][r];
            gout[(size_t)blk * GS + r] = s;
        }
    }
    if (i == cn && i < m) {
#pragma unroll
        for (int r = 0; r < BMAX; ++r)
            if (r >= cn && r < bw) rout[r] = rowv[r];
    }
}

// Pipelined buffer loads and stores with device-scope coherence (sc1): the
// cross-workgroup records need no cache writeback or invalidate.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kSc1 = 16;

__device__ inline double bld(__amdgpu_buffer_rsrc_t r, int elem)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, elem * 8, 0, kSc1));
}

__device__ inline void bst(__amdgpu_buffer_rsrc_t r, int elem, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, elem * 8, 0, kSc1);
}

// Whole panel QR in one cooperative launch: every workgroup keeps its PR
// panel rows in registers across all columns; the per-column Gram records and
// the pivot row cross workgroups through device-coherent accesses, separated
// by a grid barrier (a monotonic arrival counter with a bounded wait).
__global__ __launch_bounds__(PR) void panel_qr_coop_kernel(int m, int bw, int nr, double* P, int ldp,
                                                           double* gbuf, double* rbuf, double* tau,
                                                           int* counter, int* err, int nblk)
{
    __shared__ double G[BMAX + 1];
    __shared__ double scoef[BMAX];
    __shared__ double red[PR / 64][BMAX + 1];
    __shared__ double sh[4];
    __shared__ double prow[BMAX];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const int i = blk * PR + tid;
    const int lane = tid & 63, wave = tid >> 6;
    const __amdgpu_buffer_rsrc_t grs =
        __builtin_amdgcn_make_buffer_rsrc(gbuf, (short)0, (int)((size_t)2 * nblk * GS * 8), 0x00020000);
    const __amdgpu_buffer_rsrc_t rrs = __builtin_amdgcn_make_buffer_rsrc(rbuf, (short)0, 2 * 64 * 8, 0x00020000);

    double rowv[BMAX];
#pragma unroll
    for (int r = 0; r < BMAX; ++r) rowv[r] = (r < bw && i < m) ? P[cm(i, r, ldp)] : 0.0;
    int arrive = 0;
    double xn = 0.0;   // this row's entry in the column the next step reflects

    for (int c = -1; c < nr; ++c) {
        const int gin = ((c + 2) & 1) * nblk * GS;    // element offsets into gbuf / rbuf
        const int gout = ((c + 1) & 1) * nblk * GS;
        const int rin = ((c + 2) & 1) * 64;
        const int rout = ((c + 1) & 1) * 64;
        if (c >= 0) {
            // everything column c needs from other workgroups, loaded at once:
            // the per-block records (wave w takes blocks w, w+4, ..., lane r
            // entry r) and the pivot row (thread r entry r)
            {
                // loads are unconditional and issued in batches of RU so that they
                // are in flight together (a guarded load would wait by itself); the
                // entries a lane does not need are dropped by a select
                constexpr int RU = 16;
                const double pv = bld(rrs, rin + lane);
                double s = 0.0, st = 0.0;
                const bool need = lane >= c && lane < bw;
                int b = wave;
                for (; b + (RU - 1) * (PR / 64) < nblk; b += RU * (PR / 64)) {
                    double v[RU], vt[RU];
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        v[u] = bld(grs, gin + (b + u * (PR / 64)) * GS + lane);
                        vt[u] = bld(grs, gin + (b + u * (PR / 64)) * GS + BMAX);
                    }
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        s += need ? v[u] : 0.0;
                        st += vt[u];
                    }
                }
                for (; b < nblk; b += PR / 64) {
                    const double v = bld(grs, gin + b * GS + lane);
                    const double vt = bld(grs, gin + b * GS + BMAX);
                    s += need ? v : 0.0;
                    st += vt;
                }
                red[wave][lane] = s;
                if (lane == 0) red[wave][BMAX] = st;
                if (tid < BMAX) prow[tid] = (lane < bw) ? pv : 0.0;
            }
            __syncthreads();
            if (tid <= BMAX) {
                double s = 0.0;
                for (int w = 0; w < PR / 64; ++w) s += red[w][tid];
                G[tid] = s;
            }
            __syncthreads();
            if (tid == 0) {
                double x0 = prow[c];
                double tail = G[BMAX];
                double t = 0.0, alpha = x0, den = 1.0;
                if (tail > 0.0) {
                    double nrm = sqrt(x0 * x0 + tail);
                    alpha = (x0 >= 0.0) ? -nrm : nrm;
                    t = (alpha - x0) / alpha;
                    den = x0 - alpha;
                }
                sh[0] = t; sh[1] = alpha; sh[2] = den;
                if (blk == 0) tau[c] = t;
            }
            __syncthreads();
            const double t = sh[0], alpha = sh[1], den = sh[2];
            // coefficients of the update, zero outside columns c+1 .. bw-1 so that
            // the update below needs no per-column condition
            if (tid < BMAX)
                scoef[tid] = (tid > c && tid < bw && t != 0.0) ? (G[tid] - alpha * prow[tid]) / den : 0.0;
            __syncthreads();
            if (i < m && i >= c) {
                // xn of the previous step is this row's entry in column c
                const double vi = (i == c) ? 1.0 : ((t != 0.0) ? xn / den : 0.0);
                const double tv = t * vi;
#pragma unroll
                for (int r = 0; r < BMAX; ++r) rowv[r] -= tv * scoef[r];
                // column c is final for this row: alpha on the diagonal, v below it
                P[cm(i, c, ldp)] = (i == c) ? alpha : vi;
            }
        }
        const int cn = c + 1;
        if (cn < nr) {
            {
                // rowv[cn] for the uniform cn in two levels (eight group
                // conditions, then eight entry conditions), so that rowv stays
                // in registers and few condition masks are live
                double g8[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) g8[q] = 0.0;
                const int hi = cn >> 3, lo = cn & 7;
#pragma unroll
                for (int g = 0; g < 8; ++g)
                    if (g == hi) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) g8[q] = rowv[8 * g + q];
                    }
                xn = 0.0;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q == lo) xn = g8[q];
            }
            if (!(i < m && i >= cn)) xn = 0.0;
            // Gram row of column cn over the wave's rows by a butterfly
            // transpose-reduction: after the step with offset h a lane keeps the
            // half of its partial sums selected by lane bit h, so that at the end
            // lane l holds the wave total of entry l
            {
                double v[BMAX];
#pragma unroll
                for (int r = 0; r < BMAX; ++r) v[r] = xn * rowv[r];   // entries r < cn are never read
#pragma unroll
                for (int h = BMAX / 2; h >= 1; h >>= 1) {
                    const bool up = (lane & h) != 0;
#pragma unroll
                    for (int j = 0; j < h; ++j) {
                        const double send = up ? v[j] : v[j + h];
                        const double keep = up ? v[j + h] : v[j];
                        v[j] = keep + __shfl_xor(send, h, 64);
                    }
                }
                red[wave][lane] = v[0];
                double tl = (i > cn && i < m) ? xn * xn : 0.0;
                double s = wave_sum(tl);
                if (lane == 0) red[wave][BMAX] = s;
            }
            __syncthreads();
            for (int r = tid; r <= BMAX; r += PR) {
                if ((r >= cn && r < bw) || r == BMAX) {
                    double s = 0.0;
                    for (int w = 0; w < PR / 64; ++w) s += red[w][r];
                    bst(grs, gout + blk * GS + r, s);
                }
            }
            if (i == cn && i < m) {
#pragma unroll
                for (int r = 0; r < BMAX; ++r) bst(rrs, rout + r, rowv[r]);   // entries r < cn are never read
            }
            // grid barrier
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            arrive += nblk;
            if (tid == 0) {
                bad = 0;
                __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                long long spins = 0;
                while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < arrive) {
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { bad = 1; break; }
                    if (++spins > (1LL << 22)) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        bad = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
            if (bad) return;
        }
    }
    // write back the entries not yet final in P: R above the diagonal and the
    // columns that needed no reflector
    if (i < m) {
#pragma unroll
        for (int r = 0; r < BMAX; ++r)
            if (r < bw && !(r < nr && i >= r)) P[cm(i, r, ldp)] = rowv[r];
    }
}

// Explicit V (m x bw, unit lower trapezoidal) of the panel into V (ld ldv),
// and zeros into the zpad rows above it (so that V of several consecutive
// panels reads as one matrix with the later panels zero above their rows).
__global__ void panel_store_v_kernel(int m, int bw, int nr, const double* P, int ldp, double* V, int ldv,
                                     int zpad)
{
    int i = (int)(blockIdx.x * blockDim.x + threadIdx.x) - zpad;
    int c = blockIdx.y;
    if (i >= m || c >= bw) return;
    double v = 0.0;
    if (i >= 0 && c < nr) v = (i == c) ? 1.0 : (i > c ? P[cm(i, c, ldp)] : 0.0);
    V[(ptrdiff_t)c * ldv + i] = v;
}

// T (upper triangular, bw x bw, ld ldt) of Q = H_0 ... H_{bw-1} = I - V T V^T
// from G = V^T V and tau.  T_cc = tau_c, and for two adjacent blocks of
// reflectors A, B (A first) T_AB = -T_AA G_AB T_BB; the blocks double in size
// from 1 to 32, each level two parallel small products over 256 threads.
__global__ __launch_bounds__(256) void build_t_kernel(int bw, const double* G, int ldg, const double* tau,
                                                       double* T, int ldt)
{
    __shared__ double Ts[BMAX][BMAX + 1];
    __shared__ double Gs[BMAX][BMAX + 1];
    __shared__ double Ys[BMAX][BMAX + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < BMAX * BMAX; e += 256) {
        const int r = e % BMAX, c = e / BMAX;
        Gs[r][c] = (r < bw && c < bw) ? G[cm(r, c, ldg)] : 0.0;
        Ts[r][c] = (r == c && r < bw) ? tau[r] : 0.0;
    }
    __syncthreads();
    for (int sz = 1; sz < BMAX; sz *= 2) {
        const int nout = (BMAX / (2 * sz)) * sz * sz;   // entries of all off-diagonal blocks
        // Y = G_AB T_BB (row a of A, column b of B)
        for (int e = tid; e < nout; e += 256) {
            const int pr = e / (sz * sz), rem = e % (sz * sz);
            const int a = rem % sz, bb = rem / sz;
            const int p0 = pr * 2 * sz, pb = p0 + sz;
            double y = 0.0;
            for (int jj = 0; jj <= bb; ++jj) y += Gs[p0 + a][pb + jj] * Ts[pb + jj][pb + bb];
            Ys[p0 + a][pb + bb] = y;
        }
        __syncthreads();
        // T_AB = -T_AA Y
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
    for (int e = tid; e < bw * bw; e += 256) {
        const int r = e % bw, c = e / bw;
        T[cm(r, c, ldt)] = Ts[r][c];
    }
}

// Band of the reduced matrix: Bd(r, c) = A(c + r, c) for 0 <= r <= b, zero for b < r < ldb.
__global__ void extract_band_kernel(int n, int b, const double* A, int lda, double* Bd, int ldb)
{
    int r = threadIdx.x;   // blockDim.x == ldb
    int c = blockIdx.x;
    if (c >= n || r >= ldb) return;
    double v = 0.0;
    if (r <= b && c + r < n) v = A[cm(c + r, c, lda)];
    Bd[cm(r, c, ldb)] = v;
}

int coop_max_blocks()
{
    static const int cached = [] {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, panel_qr_coop_kernel, PR, 0);
        return std::max(0, cus * per_cu);
    }();
    return cached;
}

}  // namespace

size_t sy2sb_workspace_doubles(int n, int b)
{
    size_t nblk = (size_t)ceil_div(n, PR);
    size_t w = 0;
    w += (size_t)n * b * 3;          // Y, W of the first and of the second panel of a pair
    w += (size_t)n * 4 * b * 2;      // VW, WV (up to four b-wide blocks each)
    w += 2 * nblk * GS;              // Gram records (ping-pong)
    w += 2 * 64 + 64;                // pivot rows, tau
    w += 3 * 64 * 64;                // Gram of V, Z, U
    w += 2 * 64 * 64;                // correction coefficients of a pair (2b x b)
    w += (size_t)8 * n * 64;         // split-K partials
    w += 64;                         // barrier counter and error flag
    return w;
}

// A (n x n symmetric, lower triangle read; the strict upper part is left
// stale) -> band in Bd (ldbd = 2b rows), reflectors in
// Vall (n x n, ld n: panel p occupies rows j+b.., columns j..j+b-1) and
// T factors in Tall (b x b per panel).
//
// Panels are taken in pairs so that the trailing matrix receives one update
// of rank 4b instead of two of rank 2b (the matrix cores run much closer to
// peak at K = 4b).  With A1 = A - V1 W1^T - W1 V1^T the update of the first
// panel, the second panel needs
//   (a) its own columns of A1, formed directly: A(R1, J2) -= [V1 W1] [W1 V1]^T
//       restricted to the rows of J2;
//   (b) Y2 = A1(R2, R2) V2 = A(R2, R2) V2 - V1' (W1'^T V2) - W1' (V1'^T V2),
//       with V1', W1' the rows of V1, W1 in R2, so A(R2, R2) is never formed
//       in between;
// and A(R2, R2) -= [V1' W1' V2 W2] [W1' V1' W2 V2]^T applies both panels.
void sy2sb(hipStream_t st, int n, int b, double* A, int lda, double* Vall, double* Tall, double* Bd,
           int ldbd, double* work)
{
    const int nblk_max = ceil_div(n, PR);
    double* Y = work;
    double* W1 = Y + (size_t)n * b;
    double* W2 = W1 + (size_t)n * b;
    double* VW = W2 + (size_t)n * b;
    double* WV = VW + (size_t)n * 4 * b;
    double* gbuf0 = WV + (size_t)n * 4 * b;
    double* gbuf1 = gbuf0 + (size_t)nblk_max * GS;
    double* rbuf0 = gbuf1 + (size_t)nblk_max * GS;
    double* rbuf1 = rbuf0 + 64;
    double* tau = rbuf1 + 64;
    double* Gv = tau + 64;
    double* Z = Gv + 64 * 64;
    double* U = Z + 64 * 64;
    double* Gc = U + 64 * 64;
    double* part = Gc + 2 * 64 * 64;
    int* ibuf = (int*)(part + (size_t)8 * n * 64);
    const size_t npart = (size_t)8 * n * 64;

    // QR of panel p (columns j .. j+bw-1, rows j+b ..): V into Vall, T into Tall.
    auto factor_panel = [&](int p, int m, int bw, int nr) {
        const int j = p * b;
        const int r0 = j + b;
        double* P = A + cm(r0, j, lda);
        const int nblk = ceil_div(m, PR);
        bool coop_done = false;
        // batched calls take the per-column path: its kernels never wait on each other
        if (!batch_mode_active() && nblk <= coop_max_blocks()) {
            fill_i(st, ibuf, 2, 0);
            int mm = m, bww = bw, nrr = nr, ld = lda, nb = nblk;
            double* Pp = P;
            double* gb = gbuf0;
            double* rb = rbuf0;
            double* tp = tau;
            int* cnt = ibuf;
            int* er = ibuf + 1;
            void* args[] = {&mm, &bww, &nrr, &Pp, &ld, &gb, &rb, &tp, &cnt, &er, &nb};
            coop_done = hipLaunchCooperativeKernel((const void*)panel_qr_coop_kernel, dim3(nblk), dim3(PR), args, 0,
                                                   st) == hipSuccess;
            if (!coop_done) (void)hipGetLastError();
        }
        if (!coop_done) {
            double* gi = gbuf0; double* go = gbuf1;
            double* ri = rbuf0; double* ro = rbuf1;
            hipLaunchKernelGGL(panel_step_kernel, dim3(nblk), dim3(PR), 0, st, m, bw, -1, P, lda, gi, go, ri, ro,
                               tau, nblk);
            for (int c = 0; c < nr; ++c) {
                std::swap(gi, go);
                std::swap(ri, ro);
                hipLaunchKernelGGL(panel_step_kernel, dim3(nblk), dim3(PR), 0, st, m, bw, c, P, lda, gi, go, ri,
                                   ro, tau, nblk);
            }
        }
        if (nr < bw) fill_d(st, tau + nr, (size_t)(bw - nr), 0.0);
        double* V = Vall + cm(r0, j, n);
        const int zpad = std::min(3 * b, r0);
        hipLaunchKernelGGL(panel_store_v_kernel, dim3(ceil_div(m + zpad, 256), bw), dim3(256), 0, st, m, bw, nr, P,
                           lda, V, n, zpad);
        double* T = Tall + (size_t)p * b * b;
        dgemm_splitk(st, 'T', 'N', bw, bw, m, 1.0, V, n, V, n, 0.0, Gv, 64, part, npart);
        hipLaunchKernelGGL(build_t_kernel, dim3(1), dim3(256), 0, st, bw, Gv, 64, tau, T, b);
    };
    // Y = A22 V (A22 = A(r0.., r0..), symmetric, lower triangle read)
    auto form_y = [&](int r0, int m, int bw, const double* V) {
        dgemm_splitk(st, 'S', 'N', m, bw, m, 1.0, A + cm(r0, r0, lda), lda, V, n, 0.0, Y, m, part, npart);
    };
    // W = X - 1/2 V (T^T (V^T X)) with X = Y T
    auto finish_w = [&](int m, int bw, const double* V, const double* T, double* W) {
        dgemm(st, 'N', 'N', m, bw, bw, 1.0, Y, m, T, b, 0.0, W, m);
        dgemm_splitk(st, 'T', 'N', bw, bw, m, 1.0, V, n, W, m, 0.0, Z, 64, part, npart);
        dgemm(st, 'T', 'N', bw, bw, bw, 1.0, T, b, Z, 64, 0.0, U, 64);
        dgemm(st, 'N', 'N', m, bw, bw, -0.5, V, n, U, 64, 1.0, W, m);
    };

    const int npanel = ceil_div(n, b);
    int p = 0;
    while (p < npanel) {
        const int j = p * b;
        const int r0 = j + b;
        const int m = n - r0;
        const int bw = std::min(b, n - j);
        if (m < 2) break;
        const int nr = std::min(bw, m - 1);
        const int m2 = m - b;
        const bool pair = (p + 1 < npanel) && bw == b && m2 > 2 * b;
        factor_panel(p, m, bw, nr);
        const double* V1 = Vall + cm(r0, j, n);
        const double* T1 = Tall + (size_t)p * b * b;
        form_y(r0, m, bw, V1);
        finish_w(m, bw, V1, T1, W1);
        if (!pair) {
            // A22 -= [V W] [W V]^T, lower tiles
            copy_matrix(st, m, bw, V1, n, VW, m);
            copy_matrix(st, m, bw, W1, m, VW + (size_t)m * bw, m);
            copy_matrix(st, m, bw, W1, m, WV, m);
            copy_matrix(st, m, bw, V1, n, WV + (size_t)m * bw, m);
            dgemm(st, 'N', 'T', m, m, 2 * bw, -1.0, VW, m, WV, m, 1.0, A + cm(r0, r0, lda), lda, 1);
            ++p;
            continue;
        }
        // (a) the second panel's columns J2 = [r0, r0+b) over rows r0..: -= [V1 W1] [W1 V1]^T
        copy_matrix(st, m, b, V1, n, VW, m);
        copy_matrix(st, m, b, W1, m, VW + (size_t)m * b, m);
        copy_matrix(st, b, b, W1, m, WV, b);
        copy_matrix(st, b, b, V1, n, WV + (size_t)b * b, b);
        dgemm(st, 'N', 'T', m, b, 2 * b, -1.0, VW, m, WV, b, 1.0, A + cm(r0, r0, lda), lda);
        // second panel
        const int r2 = r0 + b;
        const int nr2 = std::min(b, m2 - 1);
        factor_panel(p + 1, m2, b, nr2);
        const double* V2 = Vall + cm(r2, r0, n);
        const double* T2 = Tall + (size_t)(p + 1) * b * b;
        const double* V1s = V1 + b;          // rows of V1 in R2 (ld n)
        const double* W1s = W1 + b;          // rows of W1 in R2 (ld m)
        form_y(r2, m2, b, V2);
        // (b) Y2 -= [V1' W1'] [W1'^T V2 ; V1'^T V2]
        dgemm_splitk(st, 'T', 'N', b, b, m2, 1.0, W1s, m, V2, n, 0.0, Gc, 2 * b, part, npart);
        dgemm_splitk(st, 'T', 'N', b, b, m2, 1.0, V1s, n, V2, n, 0.0, Gc + b, 2 * b, part, npart);
        copy_matrix(st, m2, b, V1s, n, VW, m2);
        copy_matrix(st, m2, b, W1s, m, VW + (size_t)m2 * b, m2);
        dgemm(st, 'N', 'N', m2, b, 2 * b, -1.0, VW, m2, Gc, 2 * b, 1.0, Y, m2);
        finish_w(m2, b, V2, T2, W2);
        // A(R2, R2) -= [V1' W1' V2 W2] [W1' V1' W2 V2]^T, lower tiles
        copy_matrix(st, m2, b, V2, n, VW + (size_t)2 * m2 * b, m2);
        copy_matrix(st, m2, b, W2, m2, VW + (size_t)3 * m2 * b, m2);
        copy_matrix(st, m2, b, W1s, m, WV, m2);
        copy_matrix(st, m2, b, V1s, n, WV + (size_t)m2 * b, m2);
        copy_matrix(st, m2, b, W2, m2, WV + (size_t)2 * m2 * b, m2);
        copy_matrix(st, m2, b, V2, n, WV + (size_t)3 * m2 * b, m2);
        dgemm(st, 'N', 'T', m2, m2, 4 * b, -1.0, VW, m2, WV, m2, 1.0, A + cm(r2, r2, lda), lda, 1);
        p += 2;
    }
    hipLaunchKernelGGL(extract_band_kernel, dim3(n), dim3(ldbd), 0, st, n, b, A, lda, Bd, ldbd);
}

}  // namespace eg
