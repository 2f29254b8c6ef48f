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
// The panel QR first tries two CholeskyQR passes with Householder
// reconstruction in one cooperative launch (five grid-wide reductions per
// panel), accepted only for well-conditioned panels.  Otherwise it takes
// Householder reflectors column by column: a reflector for column c needs
// x = P(c:m, c) only through x^T P(c:m, r) (r >= c), so each step (1) reduces
// the per-workgroup partial Gram row of column c left by the previous step,
// (2) applies reflector c to its rows, and (3) forms the partial Gram row of
// column c+1 -- one grid-wide reduction per column, in one cooperative launch
// (or one launch per column in batched calls).
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
                                                        double* tau, int nblk, const int* skip)
{
    if (*skip) return;   // the panel was already factored by the CholeskyQR2 kernel
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
                                                           int* counter, int* err, int nblk, const int* skip)
{
    if (*skip) return;   // the panel was already factored by the CholeskyQR2 kernel
    __shared__ double G[BMAX + 1];
    __shared__ double scoef[BMAX];
    __shared__ double red[PR / 64][BMAX + 1];
    __shared__ double sh[4];
    __shared__ double prow[BMAX];
    __shared__ double tau_sh[BMAX];
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
                tau_sh[c] = t;
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
                // column c is final for this row: alpha on the diagonal, v below
                // it.  It stays in rowv[c] (no later update touches it, scoef[c]
                // being zero) and reaches P with the rest of the row at the end: a
                // store here would make the next step wait for its completion.
                const double fin = (i == c) ? alpha : vi;
#pragma unroll
                for (int r = 0; r < BMAX; ++r) rowv[r] = (r == c) ? fin : rowv[r] - tv * scoef[r];
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
    // the row into P: R above the diagonal, alpha on it, v below it, and the
    // columns that needed no reflector; the reflector factors of workgroup 0
    if (i < m) {
#pragma unroll
        for (int r = 0; r < BMAX; ++r)
            if (r < bw) P[cm(i, r, ldp)] = rowv[r];
    }
    if (blk == 0 && tid < nr) tau[tid] = tau_sh[tid];
}

// ---------------------------------------------------------------------------
// Panel QR in a few grid-wide steps: CholeskyQR2 and Householder reconstruction
// ---------------------------------------------------------------------------
// For a well-conditioned panel P (m x 64), two CholeskyQR passes give P = Q R
// with Q orthonormal to working precision: G = P^T P = L L^T, Q' = P L^-T,
// then the same for Q' (R = R2 R1 with R_i = L_i^T).  The reflectors follow
// from Q alone (Householder reconstruction): the LU factorization without
// pivoting Q1 - S = L U of the top 64 x 64 block, with the sign S_cc = -sign
// of the c-th pivot chosen during the elimination so that every pivot has
// magnitude at least 1, gives V = [L; Q2 U^-1] (unit lower trapezoidal) with
// (I - V T V^T)[:, 0:64] = Q S, hence P = (I - V T V^T) [S R; 0].  The output
// has the layout of the column-by-column kernel: S R on and above the
// diagonal of the top block, V below it; T follows from V (tau_c = 2 / v_c^T v_c).
//
// The whole panel takes five grid barriers instead of one per column.  Every
// workgroup factors the 64 x 64 Gram matrices itself (identical inputs and
// code, so identical bits everywhere); workgroup 0 forms R and the LU and
// shares U^T.
//
// Gram-matrix methods lose the small components of panels whose rows differ
// greatly in size (the reduced matrix of an ill-conditioned overlap is such a
// case), where Householder QR keeps them; accepting every panel whose first
// pass left the columns within 0.1 of orthonormal cost five orders of
// magnitude in the density matrix of such pencils.  So a panel is taken only
// when the first pass already left them orthonormal to kCholQrAccept (a panel
// condition number of order 100 or less); any other panel (and one whose
// Cholesky factorization breaks down) is left untouched with *status at 0,
// and the column-by-column kernel factors it.
constexpr double kCholQrAccept = 1e-12;
constexpr int CQ_TILES = 10;               // 16 x 16 tiles on and above the diagonal of a 64 x 64 Gram
constexpr int CQ_REC = CQ_TILES * 256;     // doubles per partial Gram record
constexpr int LP = BMAX + 1;               // LDS pitch

__device__ inline void cq_tile(int t, int& I, int& J)
{
    I = t < 4 ? 0 : (t < 7 ? 1 : (t < 9 ? 2 : 3));
    J = t < 4 ? t : (t < 7 ? t - 3 : (t < 9 ? t - 5 : 3));
}

// Grid barrier (monotonic arrival counter, bounded wait).  False on a
// time-out or when another workgroup reported one.
__device__ inline bool cq_grid_sync(int* counter, int* err, int& arrive, int nblk, int* bad)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    arrive += nblk;
    if (threadIdx.x == 0) {
        *bad = 0;
        __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        long long spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < arrive) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { *bad = 1; break; }
            if (++spins > (1LL << 22)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                *bad = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    return *bad == 0;
}

constexpr int CQ_NT = 128;   // panel rows (threads) per workgroup

__device__ inline double cq_readlane(double v, int l)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// Orders a wave's LDS accesses across lanes (one wave needs no workgroup barrier).
__device__ inline void cq_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky G = L L^T of the symmetric 64 x 64 matrix in LDS by one wave, lane
// r holding row r in registers; each step broadcasts its scaled column
// through col.  L (lower, with its diagonal) replaces the lower triangle of G.
// False at a pivot that is not positive and finite (the same in every lane).
__device__ bool cq_cholesky_wave(double (*__restrict__ G)[LP], double* __restrict__ col)
{
    const int lane = threadIdx.x & 63;
    double g[BMAX];
#pragma unroll
    for (int q = 0; q < BMAX; ++q) g[q] = G[lane][q];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < BMAX; ++c) {
        const double d = cq_readlane(g[c], c);
        if (!(d > 0.0) || !isfinite(d)) {
            ok = false;
            break;
        }
        const double s = sqrt(d);
        const double l = (lane == c) ? s : g[c] / s;   // lanes below c: L(r, c)
        g[c] = l;
        col[lane] = (lane > c) ? l : 0.0;
        cq_wave_sync();
#pragma unroll
        for (int q = c + 1; q < BMAX; ++q) g[q] -= l * col[q];   // only q <= r is kept
        cq_wave_sync();
    }
    if (ok) {
#pragma unroll
        for (int q = 0; q < BMAX; ++q)
            if (q <= lane) G[lane][q] = g[q];
    }
    return ok;
}

// LU without pivoting of A - S by one wave (lane r holding row r of A in a),
// S_cc = -sign of the c-th pivot (+1 taken as the sign of 0); the pivot row
// of each step is read from lane c.  On return a holds L strictly below the
// diagonal (unit diagonal implied) and U on and above it; sgn gets S.
__device__ void cq_signed_lu_wave(double (&a)[BMAX], double* __restrict__ sgn)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < BMAX; ++c) {
        const double u = cq_readlane(a[c], c);
        const double s = (u >= 0.0) ? -1.0 : 1.0;
        const double pv = u - s;   // |pv| = |u| + 1
        const double lm = (lane > c) ? a[c] / pv : 0.0;
        a[c] = (lane > c) ? lm : ((lane == c) ? pv : a[c]);
        if (lane == 0) sgn[c] = s;
#pragma unroll
        for (int q = c + 1; q < BMAX; ++q) a[q] -= lm * cq_readlane(a[q], c);
    }
}

// The wave's 64 rows of St <- Z with Z M^T = St for a lower triangular M in
// LDS (dinv holding 1 / M_kk): with M = L one CholeskyQR step X L^-T, with
// M = U^T the product X U^-1.  Blocked by 16 columns J: the update
// Y_J = X_J - Z_{<J} M_{J,<J}^T on the matrix cores, then Z_J from
// Z_J M_JJ^T = Y_J by substitution, each lane taking its own row.  Only the
// wave's own rows are read or written.
__device__ void cq_rows_solve(double (*__restrict__ St)[LP], const double (*__restrict__ M)[LP],
                              const double* __restrict__ dinv)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r0 = 64 * wave;
#pragma unroll
    for (int J = 0; J < 4; ++J) {
        const int o = 16 * J;
        if (J > 0) {
            double4_t acc[4];
#pragma unroll
            for (int R = 0; R < 4; ++R)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[R][r] = St[r0 + 16 * R + 4 * r + lk][o + li];
#pragma unroll
            for (int kk = 0; kk < o; kk += 4) {
                const double bm = M[o + li][kk + lk];
#pragma unroll
                for (int R = 0; R < 4; ++R)
                    acc[R] = __builtin_amdgcn_mfma_f64_16x16x4f64(-St[r0 + 16 * R + li][kk + lk], bm, acc[R], 0, 0,
                                                                  0);
            }
#pragma unroll
            for (int R = 0; R < 4; ++R)
#pragma unroll
                for (int r = 0; r < 4; ++r) St[r0 + 16 * R + 4 * r + lk][o + li] = acc[R][r];
            cq_wave_sync();
        }
        double y[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) y[c] = St[r0 + lane][o + c];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            double t = y[c];
#pragma unroll
            for (int k = 0; k < c; ++k) t -= y[k] * M[o + c][o + k];
            y[c] = t * dinv[o + c];
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) St[r0 + lane][o + c] = y[c];
        cq_wave_sync();
    }
}

// The wave's 64 rows of St <- St (I - F^T) with F = L - I for a lower
// triangular L in LDS whose strict upper triangle is zero: X L^-T to first
// order in F.  Column block J takes the products over columns 0 .. 16J+15 of
// the rows as they were; blocks are formed last to first so that no block
// reads a column already replaced.
// (Not inlined: inlined into the panel kernel, it pushes the kernel's other
// phases past their register budget.)
__device__ __attribute__((noinline)) void cq_rows_first_order(double (*__restrict__ St)[LP],
                                                              const double (*__restrict__ L)[LP])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r0 = 64 * wave;
#pragma unroll 1
    for (int J = 3; J >= 0; --J) {
        const int o = 16 * J;
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const int ra = r0 + 32 * h;
            double4_t acc[2];
#pragma unroll
            for (int R = 0; R < 2; ++R)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[R][r] = St[ra + 16 * R + 4 * r + lk][o + li];
            for (int kk = 0; kk < o + 16; kk += 4) {
                const int kq = kk + lk, c = o + li;
                const double f = (kq <= c) ? L[c][kq] - ((kq == c) ? 1.0 : 0.0) : 0.0;   // F(c, kq)
#pragma unroll
                for (int R = 0; R < 2; ++R)
                    acc[R] = __builtin_amdgcn_mfma_f64_16x16x4f64(-St[ra + 16 * R + li][kq], f, acc[R], 0, 0, 0);
            }
#pragma unroll
            for (int R = 0; R < 2; ++R)
#pragma unroll
                for (int r = 0; r < 4; ++r) St[ra + 16 * R + 4 * r + lk][o + li] = acc[R][r];
        }
        cq_wave_sync();
    }
}

// One thread per panel row (CQ_NT rows per workgroup, m >= 64, 64 columns).
// rec holds nblk partial Gram records, the summed record, U^T and the
// first-pass factor L1 (written and read by workgroup 0 only).
__global__ __launch_bounds__(CQ_NT, 1) void panel_cholqr_kernel(int m, double* P, int ldp, double* rec,
                                                                int* counter, int* err, int* status, int nblk,
                                                                double thr)
{
    constexpr int NT = CQ_NT;
    constexpr int NW = NT / 64;
    constexpr int TPW = (CQ_TILES + NW - 1) / NW;   // Gram tiles per wave
    __shared__ double Gb[BMAX][LP];   // Gram matrix, then its Cholesky factor; the LU (workgroup 0)
    __shared__ double Xb[BMAX][LP];   // R (workgroup 0), then U^T
    __shared__ double St[NT][LP];     // the rows: operand staging of the Gram products, parking
    __shared__ double red[NT];
    __shared__ double sgn[BMAX];
    __shared__ double colv[BMAX];
    __shared__ double dinv[BMAX];
    __shared__ int bad;
    __shared__ int flag;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int blk = blockIdx.x;
    const int i = blk * NT + tid;
    const int gfin = nblk * CQ_REC;   // element offsets: summed record, U^T, L1
    const int mgo = gfin + CQ_REC;
    const int l1o = mgo + BMAX * BMAX;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        rec, (short)0, (int)(((size_t)l1o + BMAX * BMAX) * 8), 0x00020000);

    // the rows stay in LDS through all three phases; all 64 loads of a row
    // are issued before the first store, so that they are in flight together
    {
        double x[BMAX];
#pragma unroll
        for (int r = 0; r < BMAX; ++r) x[r] = (i < m) ? P[cm(i, r, ldp)] : 0.0;
#pragma unroll
        for (int r = 0; r < BMAX; ++r) St[tid][r] = x[r];
    }
    __syncthreads();
    int arrive = 0;

    for (int ph = 0; ph < 3; ++ph) {
        if (ph < 2) {
            // partial Gram matrix of this workgroup's rows on the matrix cores
            double4_t acc[TPW];
#pragma unroll
            for (int s = 0; s < TPW; ++s) acc[s] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int kk = 0; kk < NT; kk += 4) {
                const int kr = kk + (lane >> 4);
#pragma unroll
                for (int s = 0; s < TPW; ++s) {
                    const int t = wave + NW * s;
                    if (t < CQ_TILES) {
                        int I, J;
                        cq_tile(t, I, J);
                        const double a = St[kr][16 * I + (lane & 15)];
                        const double b = St[kr][16 * J + (lane & 15)];
                        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < TPW; ++s) {
                const int t = wave + NW * s;
                if (t < CQ_TILES) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) bst(rs, blk * CQ_REC + t * 256 + r * 64 + lane, acc[s][r]);
                }
            }
            if (!cq_grid_sync(counter, err, arrive, nblk, &bad)) return;
            // fixed-order sums of the records: this workgroup takes entries
            // [e0, e0 + E), each split over S threads by record index mod S
            {
                const int E = (CQ_REC + nblk - 1) / nblk;
                const int S = (E <= NT) ? NT / E : 1;
                const int e0 = blk * E;
                for (int w = tid; w < E * S; w += NT) {
                    const int el = w % E, sp = w / E, e = e0 + el;
                    double sum = 0.0;
                    if (e < CQ_REC) {
                        int p = sp;
                        for (; p + 7 * S < nblk; p += 8 * S) {
                            double v[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) v[u] = bld(rs, (p + u * S) * CQ_REC + e);
#pragma unroll
                            for (int u = 0; u < 8; ++u) sum += v[u];
                        }
                        for (; p < nblk; p += S) sum += bld(rs, p * CQ_REC + e);
                    }
                    if (S > 1) red[w] = sum;
                    else if (e < CQ_REC) bst(rs, gfin + e, sum);
                }
                if (S > 1) {
                    __syncthreads();
                    if (tid < E && e0 + tid < CQ_REC) {
                        double sum = 0.0;
                        for (int sp = 0; sp < S; ++sp) sum += red[sp * E + tid];
                        bst(rs, gfin + e0 + tid, sum);
                    }
                }
            }
            if (!cq_grid_sync(counter, err, arrive, nblk, &bad)) return;
            {
                // the summed record, all loads in flight together
                constexpr int PER = CQ_REC / NT;
                double v[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) v[u] = bld(rs, gfin + tid + u * NT);
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = tid + u * NT;
                    const int t = e >> 8, r = (e >> 6) & 3, l = e & 63;
                    int I, J;
                    cq_tile(t, I, J);
                    const int row = 16 * I + 4 * r + (l >> 4), col = 16 * J + (l & 15);
                    if (I != J || row >= col) {
                        Gb[row][col] = v[u];
                        Gb[col][row] = v[u];
                    }
                }
            }
            __syncthreads();
            if (ph == 1) {
                double dev = 0.0;
                for (int e = tid; e < BMAX * BMAX; e += NT) {
                    const int r = e & 63, c = e >> 6;
                    const double d = fabs(Gb[r][c] - (r == c ? 1.0 : 0.0));
                    dev = (d > dev || d != d) ? d : dev;   // a NaN counts as a large deviation
                }
                // largest deviation over the workgroup (a NaN wins every comparison)
#pragma unroll
                for (int h = 1; h < 64; h <<= 1) {
                    const double o = __shfl_xor(dev, h, 64);
                    dev = (o > dev || o != o) ? o : dev;
                }
                if (lane == 0) red[wave] = dev;
                __syncthreads();
                if (tid == 0) {
                    double mx = 0.0;
                    for (int t = 0; t < NW; ++t) mx = (red[t] > mx || red[t] != red[t]) ? red[t] : mx;
                    flag = (mx <= thr) ? 1 : 0;
                }
                __syncthreads();
                if (!flag) return;
            }
            if (ph == 1 && thr <= 1e-9) {
                // The second pass starts from columns orthonormal to thr: G =
                // I + E with |E_ij| <= thr, so chol(G) = I + F with F the lower
                // triangle of E and half its diagonal, and L^-T = I - F^T, both
                // up to terms of order 64 thr^2, far below the rounding of
                // entries of order one.  No factorization or substitution chain.
                for (int e = tid; e < BMAX * BMAX; e += NT) {
                    const int r = e & 63, c = e >> 6;
                    const double g = Gb[r][c];
                    Gb[r][c] = (r > c) ? g : ((r == c) ? 1.0 + 0.5 * (g - 1.0) : 0.0);
                }
                __syncthreads();
                cq_rows_first_order(St, Gb);   // rows <- rows (I - F^T)
            } else {
                if (wave == 0) {
                    const bool ok = cq_cholesky_wave(Gb, colv);
                    if (lane == 0) flag = ok ? 1 : 0;
                }
                __syncthreads();
                if (!flag) return;
                if (tid < BMAX) dinv[tid] = 1.0 / Gb[tid][tid];
                if (ph == 0 && blk == 0) {
                    for (int e = tid; e < BMAX * BMAX; e += NT) {
                        const int r = e & 63, c = e >> 6;
                        bst(rs, l1o + e, (r >= c) ? Gb[r][c] : 0.0);
                    }
                }
                __syncthreads();
                cq_rows_solve(St, Gb, dinv);   // rows <- rows L^-T
            }
        } else {
            if (blk == 0 && wave == 0) {
                // Q1 = rows 0..63 of the panel = the rows of wave 0
                double a[BMAX];
#pragma unroll
                for (int q = 0; q < BMAX; ++q) a[q] = St[lane][q];
                cq_signed_lu_wave(a, sgn);
#pragma unroll
                for (int q = 0; q < BMAX; ++q) Xb[lane][q] = a[q];
            }
            __syncthreads();
            if (blk == 0) {
                // L below the diagonal of the top block (R goes on and above it
                // after the barrier), and U^T for every workgroup
                for (int e = tid; e < BMAX * BMAX; e += NT) {
                    const int r = e & 63, c = e >> 6;
                    if (r > c && r < m) P[cm(r, c, ldp)] = Xb[r][c];
                    bst(rs, mgo + e, (r >= c) ? Xb[c][r] : 0.0);   // U^T
                }
            }
            if (!cq_grid_sync(counter, err, arrive, nblk, &bad)) return;
            {
                constexpr int PER = BMAX * BMAX / NT;
                double v[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) v[u] = bld(rs, mgo + tid + u * NT);
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = tid + u * NT;
                    Xb[e & 63][e >> 6] = v[u];
                }
            }
            __syncthreads();
            if (tid < BMAX) dinv[tid] = 1.0 / Xb[tid][tid];
            __syncthreads();
            if (blk > 0 || wave > 0) {
                cq_rows_solve(St, Xb, dinv);   // V2 = Q2 U^-1 (rows 64 and on)
            } else {
                // off the other workgroups' path: R = R2 R1 = L2^T L1^T into P
                // as S R on and above the diagonal, on the matrix cores.  A =
                // L2^T from Gb (which still holds L2 below its diagonal and the
                // Gram matrix above it, hence the mask), B = L1^T from L1 staged
                // in this wave's own rows of St (free once the LU has read them).
#pragma unroll
                for (int k0 = 0; k0 < BMAX; k0 += 16) {
                    double l1[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) l1[k] = bld(rs, l1o + lane + 64 * (k0 + k));   // L1(lane, k)
#pragma unroll
                    for (int k = 0; k < 16; ++k) St[lane][k0 + k] = l1[k];
                }
                cq_wave_sync();
                const int li = lane & 15, lk = lane >> 4;
#pragma unroll 1   // rolled: unrolled, it pushes the kernel past its register budget
                for (int I = 0; I < 4; ++I) {
                    double4_t acc[4];
#pragma unroll
                    for (int J = 0; J < 4; ++J) acc[J] = (double4_t){0.0, 0.0, 0.0, 0.0};
                    // tile (I, J) needs k from 16 I (L2(k, i) = 0 for k < i) to
                    // 16 J + 15 (L1(j, k) = 0 for k > j)
#pragma unroll
                    for (int kk = 16 * I; kk < BMAX; kk += 4) {
                        const int k = kk + lk, ii = 16 * I + li;
                        const double a = (k >= ii) ? Gb[k][ii] : 0.0;
#pragma unroll
                        for (int J = I; J < 4; ++J)
                            if (kk < 16 * J + 16)
                                acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, St[16 * J + li][k], acc[J], 0, 0, 0);
                    }
#pragma unroll
                    for (int J = I; J < 4; ++J)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = 16 * I + 4 * r + lk, col = 16 * J + li;
                            if (row <= col && row < m) P[cm(row, col, ldp)] = sgn[row] * acc[J][r];
                        }
                }
            }
        }
        __syncthreads();
    }
    if (i >= BMAX && i < m) {
#pragma unroll 8
        for (int c = 0; c < BMAX; ++c) P[cm(i, c, ldp)] = St[tid][c];
    }
    if (blk == 0 && tid == 0) *status = 1;
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
// from G = V^T V and tau (or 2 / G_cc when *gram_tau is set).  T_cc = tau_c, and for two adjacent blocks of
// reflectors A, B (A first) T_AB = -T_AA G_AB T_BB; the blocks double in size
// from 1 to 32, each level two parallel small products over 256 threads.
__global__ __launch_bounds__(256) void build_t_kernel(int bw, const double* G, int ldg, const double* tau,
                                                       double* T, int ldt, int* flags, int nflags)
{
    __shared__ double Ts[BMAX][BMAX + 1];
    __shared__ double Gs[BMAX][BMAX + 1];
    __shared__ double Ys[BMAX][BMAX + 1];
    const int tid = threadIdx.x;
    {
        // a thread's loads are all in flight before its first LDS store;
        // flags[2] is the CholeskyQR2 status of the panel
        const bool gt = flags[2] != 0;
        double v[BMAX * BMAX / 256];
#pragma unroll
        for (int u = 0; u < BMAX * BMAX / 256; ++u) {
            const int e = tid + 256 * u, r = e % BMAX, c = e / BMAX;
            v[u] = (r < bw && c < bw) ? G[cm(r, c, ldg)] : 0.0;
        }
        const double td = (tid < bw && !gt) ? tau[tid] : 0.0;
#pragma unroll
        for (int u = 0; u < BMAX * BMAX / 256; ++u) {
            const int e = tid + 256 * u, r = e % BMAX, c = e / BMAX;
            Gs[r][c] = v[u];
            Ts[r][c] = 0.0;
        }
        // reflectors from the reconstruction take tau_c = 2 / v_c^T v_c, which
        // makes each one exactly orthogonal for the stored v_c
        __syncthreads();
        if (tid < bw) Ts[tid][tid] = gt ? 2.0 / Gs[tid][tid] : td;
    }
    __syncthreads();
    // each dot product's LDS operands are loaded into registers before its
    // multiply-adds, so that the loads are in flight together (the sums keep
    // their order: entries 0 .. bb, and a .. sz-1)
#pragma unroll
    for (int lg = 0; lg < 6; ++lg) {
        const int sz = 1 << lg;
        const int nout = (BMAX / (2 * sz)) * sz * sz;   // entries of all off-diagonal blocks
        // Y = G_AB T_BB (row a of A, column b of B)
        for (int e = tid; e < nout; e += 256) {
            const int pr = e / (sz * sz), rem = e % (sz * sz);
            const int a = rem % sz, bb = rem / sz;
            const int p0 = pr * 2 * sz, pb = p0 + sz;
            double gv[32], tv[32];
#pragma unroll
            for (int jj = 0; jj < (1 << lg); ++jj) {
                gv[jj] = Gs[p0 + a][pb + jj];
                tv[jj] = Ts[pb + jj][pb + bb];
            }
            double y = 0.0;
#pragma unroll
            for (int jj = 0; jj < (1 << lg); ++jj)
                if (jj <= bb) y += gv[jj] * tv[jj];
            Ys[p0 + a][pb + bb] = y;
        }
        __syncthreads();
        // T_AB = -T_AA Y
        for (int e = tid; e < nout; e += 256) {
            const int pr = e / (sz * sz), rem = e % (sz * sz);
            const int a = rem % sz, bb = rem / sz;
            const int p0 = pr * 2 * sz, pb = p0 + sz;
            double tv[32], yv[32];
#pragma unroll
            for (int ii = 0; ii < (1 << lg); ++ii) {
                tv[ii] = Ts[p0 + a][p0 + ii];
                yv[ii] = Ys[p0 + ii][pb + bb];
            }
            double t = 0.0;
#pragma unroll
            for (int ii = 0; ii < (1 << lg); ++ii)
                if (ii >= a) t += tv[ii] * yv[ii];
            Ts[p0 + a][pb + bb] = -t;
        }
        __syncthreads();
    }
    for (int e = tid; e < bw * bw; e += 256) {
        const int r = e % bw, c = e / bw;
        T[cm(r, c, ldt)] = Ts[r][c];
    }
    // the panel's counters, error flags and status start at zero for the next
    // panel (every thread has read the status above)
    if (tid < nflags) flags[tid] = 0;
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

int cholqr_max_blocks()
{
    static const int cached = [] {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, panel_cholqr_kernel, CQ_NT, 0);
        return std::max(0, cus * per_cu);
    }();
    return cached;
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
    w += (size_t)128 * 64 * 64;      // split-K partials of V^T V on the second stream
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
           int ldbd, double* work, const Sy2sbAux* aux)
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
    double* part2 = part + npart + 64;
    const size_t npart2 = (size_t)128 * 64 * 64;
    // each panel's V^T V and T factor on a second stream, beside Y = A22 V
    // (which needs only V); the W formation waits for T
    const bool fork = aux && aux->st2 && aux->ev_v && aux->ev_t;
    hipStream_t sv = fork ? aux->st2 : st;

    // QR of panel p (columns j .. j+bw-1, rows j+b ..): V into Vall, T into Tall.
    auto factor_panel = [&](int p, int m, int bw, int nr) {
        const int j = p * b;
        const int r0 = j + b;
        double* P = A + cm(r0, j, lda);
        const int nblk = ceil_div(m, PR);
        bool coop_done = false;
        // ibuf: per-column kernel counter and error flag, CholeskyQR2 status,
        // counter and error flag; zero on entry (cleared before the first panel,
        // and by build_t_kernel at the end of every panel)
        int* cq_status = ibuf + 2;
        // batched calls take the per-column path: its kernels never wait on each other
        if (!batch_mode_active() && bw == BMAX && nr == BMAX && m >= 2 * BMAX) {
            int mm = m, ld = lda, nb = 0;
            double* Pp = P;
            double* rec = part;
            int* cnt = ibuf + 3;
            int* er = ibuf + 4;
            int* stp = cq_status;
            double thr = kCholQrAccept;
            void* args[] = {&mm, &Pp, &ld, &rec, &cnt, &er, &stp, &nb, &thr};
            nb = ceil_div(m, CQ_NT);
            if (nb <= cholqr_max_blocks() &&
                hipLaunchCooperativeKernel((const void*)panel_cholqr_kernel, dim3(nb), dim3(CQ_NT), args, 0, st) !=
                    hipSuccess)
                (void)hipGetLastError();
        }
        if (!batch_mode_active() && nblk <= coop_max_blocks()) {
            int mm = m, bww = bw, nrr = nr, ld = lda, nb = nblk;
            double* Pp = P;
            double* gb = gbuf0;
            double* rb = rbuf0;
            double* tp = tau;
            int* cnt = ibuf;
            int* er = ibuf + 1;
            const int* skp = cq_status;
            void* args[] = {&mm, &bww, &nrr, &Pp, &ld, &gb, &rb, &tp, &cnt, &er, &nb, &skp};
            coop_done = hipLaunchCooperativeKernel((const void*)panel_qr_coop_kernel, dim3(nblk), dim3(PR), args, 0,
                                                   st) == hipSuccess;
            if (!coop_done) (void)hipGetLastError();
        }
        if (!coop_done) {
            double* gi = gbuf0; double* go = gbuf1;
            double* ri = rbuf0; double* ro = rbuf1;
            hipLaunchKernelGGL(panel_step_kernel, dim3(nblk), dim3(PR), 0, st, m, bw, -1, P, lda, gi, go, ri, ro,
                               tau, nblk, (const int*)cq_status);
            for (int c = 0; c < nr; ++c) {
                std::swap(gi, go);
                std::swap(ri, ro);
                hipLaunchKernelGGL(panel_step_kernel, dim3(nblk), dim3(PR), 0, st, m, bw, c, P, lda, gi, go, ri,
                                   ro, tau, nblk, (const int*)cq_status);
            }
        }
        if (nr < bw) fill_d(st, tau + nr, (size_t)(bw - nr), 0.0);
        double* V = Vall + cm(r0, j, n);
        const int zpad = std::min((kQ1Group - 1) * b, r0);
        hipLaunchKernelGGL(panel_store_v_kernel, dim3(ceil_div(m + zpad, 256), bw), dim3(256), 0, st, m, bw, nr, P,
                           lda, V, n, zpad);
        double* T = Tall + (size_t)p * b * b;
        if (fork) {
            (void)hipEventRecord(aux->ev_v, st);
            (void)hipStreamWaitEvent(sv, aux->ev_v, 0);
        }
        dgemm_splitk(sv, 'T', 'N', bw, bw, m, 1.0, V, n, V, n, 0.0, Gv, 64, fork ? part2 : part,
                     fork ? npart2 : npart);
        hipLaunchKernelGGL(build_t_kernel, dim3(1), dim3(256), 0, sv, bw, Gv, 64, tau, T, b, ibuf, 5);
        if (fork) (void)hipEventRecord(aux->ev_t, sv);
    };
    // Y = A22 V (A22 = A(r0.., r0..), symmetric, lower triangle read)
    auto form_y = [&](int r0, int m, int bw, const double* V) {
        dgemm_splitk(st, 'S', 'N', m, bw, m, 1.0, A + cm(r0, r0, lda), lda, V, n, 0.0, Y, m, part, npart);
    };
    // W = X - 1/2 V (T^T (V^T X)) with X = Y T
    auto finish_w = [&](int m, int bw, const double* V, const double* T, double* W) {
        if (fork) (void)hipStreamWaitEvent(st, aux->ev_t, 0);   // T, and the panel's flags cleared
        dgemm(st, 'N', 'N', m, bw, bw, 1.0, Y, m, T, b, 0.0, W, m);
        dgemm_splitk(st, 'T', 'N', bw, bw, m, 1.0, V, n, W, m, 0.0, Z, 64, part, npart);
        dgemm(st, 'T', 'N', bw, bw, bw, 1.0, T, b, Z, 64, 0.0, U, 64);
        dgemm(st, 'N', 'N', m, bw, bw, -0.5, V, n, U, 64, 1.0, W, m);
    };

    const int npanel = ceil_div(n, b);
    fill_i(st, ibuf, 5, 0);
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
            CopyBatch cb;
            cb.add(m, bw, V1, n, VW, m);
            cb.add(m, bw, W1, m, VW + (size_t)m * bw, m);
            cb.add(m, bw, W1, m, WV, m);
            cb.add(m, bw, V1, n, WV + (size_t)m * bw, m);
            copy_matrices(st, cb);
            dgemm(st, 'N', 'T', m, m, 2 * bw, -1.0, VW, m, WV, m, 1.0, A + cm(r0, r0, lda), lda, 1);
            ++p;
            continue;
        }
        // (a) the second panel's columns J2 = [r0, r0+b) over rows r0..: -= [V1 W1] [W1 V1]^T
        {
            CopyBatch cb;
            cb.add(m, b, V1, n, VW, m);
            cb.add(m, b, W1, m, VW + (size_t)m * b, m);
            cb.add(b, b, W1, m, WV, b);
            cb.add(b, b, V1, n, WV + (size_t)b * b, b);
            copy_matrices(st, cb);
        }
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
        {
            CopyBatch cb;
            cb.add(m2, b, V1s, n, VW, m2);
            cb.add(m2, b, W1s, m, VW + (size_t)m2 * b, m2);
            copy_matrices(st, cb);
        }
        dgemm(st, 'N', 'N', m2, b, 2 * b, -1.0, VW, m2, Gc, 2 * b, 1.0, Y, m2);
        finish_w(m2, b, V2, T2, W2);
        // A(R2, R2) -= [V1' W1' V2 W2] [W1' V1' W2 V2]^T, lower tiles
        {
            CopyBatch cb;
            cb.add(m2, b, V2, n, VW + (size_t)2 * m2 * b, m2);
            cb.add(m2, b, W2, m2, VW + (size_t)3 * m2 * b, m2);
            cb.add(m2, b, W1s, m, WV, m2);
            cb.add(m2, b, V1s, n, WV + (size_t)m2 * b, m2);
            cb.add(m2, b, W2, m2, WV + (size_t)2 * m2 * b, m2);
            cb.add(m2, b, V2, n, WV + (size_t)3 * m2 * b, m2);
            copy_matrices(st, cb);
        }
        dgemm(st, 'N', 'T', m2, m2, 4 * b, -1.0, VW, m2, WV, m2, 1.0, A + cm(r2, r2, lda), lda, 1);
        p += 2;
    }
    hipLaunchKernelGGL(extract_band_kernel, dim3(n), dim3(ldbd), 0, st, n, b, A, lda, Bd, ldbd);
}

}  // namespace eg
