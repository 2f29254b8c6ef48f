// Step (2) of the two-stage tridiagonalization (ELSI paper, Sec. 3.1,
// Eq. (13) and Fig. 1): T = Q2^T B Q2 by Householder bulge chasing on the
// band (successive band reduction).
//
// Sweep s annihilates column s below its first subdiagonal.  Its task 0
// reflects A(s+1:s+b, s) and updates the diagonal block A(J0, J0) from both
// sides; task k >= 1 works on rows J_k = [s+1+kb, s+(k+1)b]: it applies the
// previous reflector from the right to the block A(J_k, J_{k-1}) (which fills
// it), takes a new reflector from the block's first column, applies it from
// the left to the block and from both sides to A(J_k, J_k).  The fill left in
// the other columns of the block is removed by the following sweeps.
//
// Row-window schedule (the default).  Workgroup k owns rows J_k(s) in every
// sweep: the off-diagonal block A(J_k, J_{k-1}) and the full symmetric
// diagonal block A(J_k, J_k) stay in its registers for the whole chase.  From
// sweep s to s+1 the window moves down one row.  Its top row is final for the
// sweep and becomes the bottom row of workgroup k-1's next window; the new
// bottom row comes from workgroup k+1.  Entries are indexed by absolute row
// and column mod b, so the move copies no data: the leaving row's slot takes
// the entering row, the off-diagonal slot of the leaving column takes the
// column that leaves the diagonal block, and that diagonal slot takes the
// entering column.  An entering row needs only its b+1 entries nearest the
// diagonal: further out, earlier sweeps have annihilated every entry.  Task
// (s, k) publishes its reflector as soon as it is formed (for the right
// application in task (s, k+1)) and its top row after its two-sided update;
// it waits for the reflector of (s, k-1) and the row of (s-1, k+1), so it
// runs at pipeline step 2s + k.  Messages are b+1 doubles in two-slot
// mailboxes.  Each double travels as two 64-bit words, one per 32-bit half,
// each word tagged with the sweep in its upper 32 bits: 64-bit atomic stores
// are single-copy atomic, so a word whose tag matches holds its half of this
// sweep's value, and a consumer wave that finds every tag current has the
// whole message.  The producer therefore stores and moves on (no wait for its
// stores, no counter), and the consumer's poll of the message is also its
// load.
//
// Pipelined-sweep schedule (used when the row-window grid does not fit the
// device at once).  One workgroup per sweep, sweeps dealt round-robin to a
// grid that is entirely resident (cooperative launch).  Task k of sweep s
// touches only rows J_k(s); it overlaps task k+1 of sweep s-1 and nothing
// later, so it starts once sweep s-1 reports k+2 finished tasks.  Each task
// loads its two blocks from the band and stores them back.
//
// Hand-off between workgroups (both schedules): data shared between
// workgroups is only read and written with device-scope (agent) coherent
// accesses, which are coherent across the XCDs without writing back or
// invalidating their L2 caches.  In the pipelined-sweep schedule a producer's
// stores complete (s_waitcnt) before one lane publishes a progress counter;
// waiting lanes poll the counter with the same kind of access.  Every wait is
// bounded and an expired wait aborts the whole grid with an error flag.
#include "common.h"

#include <atomic>

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

// ---------------------------------------------------------------------------
// Row-window schedule
// ---------------------------------------------------------------------------
struct SbWinArgs {
    int n, b, nsweeps, kmax, ldb;
    const double* Bd;   // the band on entry (read once)
    double* V2;
    double* tau2;
    double* d;
    double* e;
    unsigned long long* vbox;   // kmax x 2 slots x kBoxWords: reflector by absolute row mod b, tau, alpha
    unsigned long long* rbox;   // kmax x 2 slots x kBoxWords: top row by absolute column mod b, then its diagonal
    int* err;
    long long spin_limit;
};

constexpr int kBoxWords = 2 * 66;   // value i in words 2i (upper half) and 2i+1 (lower half); i = 64, 65: extra values

__device__ inline unsigned long long ld_word(const unsigned long long* p)
{
    return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void put_value(unsigned long long* box, int i, double x, unsigned tag)
{
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long t = (unsigned long long)tag << 32;
    __hip_atomic_store(box + 2 * i, t | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(box + 2 * i + 1, t | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave polls values 0 .. b-1 of a message (lane l taking value l) until
// they carry `tag`.
__device__ inline bool poll_row(const unsigned long long* box, int b, unsigned tag, int* err, long long limit,
                                double& val)
{
    const int lane = threadIdx.x & 63;
    long long spins = 0;
    for (;;) {
        bool ok = true;
        if (lane < b) {
            const unsigned long long w0 = ld_word(box + 2 * lane), w1 = ld_word(box + 2 * lane + 1);
            ok = (unsigned)(w0 >> 32) == tag && (unsigned)(w1 >> 32) == tag;
            val = __builtin_bit_cast(double, (w0 << 32) | (w1 & 0xffffffffull));
        }
        if (__all(ok)) return true;
        if ((++spins & 63) == 0) {
            int bad = 0;
            if (lane == 0) {
                bad = ld_flag(err);
                if (!bad && spins > limit) {
                    st_flag(err, 1);
                    bad = 1;
                }
            }
            if (__shfl(bad, 0, 64)) return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// One wave polls 16 values of a message (values i0 .. i0+15 below b, lane l
// taking value i0 + l % 16; 0 for the others) and, when `with_extra` (uniform),
// the extra value 64 (every lane) until all carry `tag`.  Every poll returns
// false when the grid's error flag is set or its spin limit expires (then it
// sets the flag).
__device__ inline bool poll_part(const unsigned long long* box, int i0, int b, bool with_extra, unsigned tag,
                                 int* err, long long limit, double& val, double& extra)
{
    const int lane = threadIdx.x & 63;
    const int i = i0 + (lane & 15);
    const bool mine = i < b;
    long long spins = 0;
    for (;;) {
        const unsigned long long w0 = mine ? ld_word(box + 2 * i) : 0, w1 = mine ? ld_word(box + 2 * i + 1) : 0;
        const unsigned long long x0 = with_extra ? ld_word(box + 128) : 0, x1 = with_extra ? ld_word(box + 129) : 0;
        const bool ok = (!mine || ((unsigned)(w0 >> 32) == tag && (unsigned)(w1 >> 32) == tag)) &&
                        (!with_extra || ((unsigned)(x0 >> 32) == tag && (unsigned)(x1 >> 32) == tag));
        if (__all(ok)) {
            val = mine ? __builtin_bit_cast(double, (w0 << 32) | (w1 & 0xffffffffull)) : 0.0;
            extra = with_extra ? __builtin_bit_cast(double, (x0 << 32) | (x1 & 0xffffffffull)) : 0.0;
            return true;
        }
        if ((++spins & 63) == 0) {
            int bad = 0;
            if (lane == 0) {
                bad = ld_flag(err);
                if (!bad && spins > limit) {
                    st_flag(err, 1);
                    bad = 1;
                }
            }
            if (__shfl(bad, 0, 64)) return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// The whole wave polls one value of a message (value i) until it carries
// `tag`.
__device__ inline bool poll_value(const unsigned long long* box, int i, unsigned tag, int* err, long long limit,
                                  double& val)
{
    const int lane = threadIdx.x & 63;
    long long spins = 0;
    for (;;) {
        const unsigned long long w0 = ld_word(box + 2 * i), w1 = ld_word(box + 2 * i + 1);
        const bool ok = (unsigned)(w0 >> 32) == tag && (unsigned)(w1 >> 32) == tag;
        if (__all(ok)) {
            val = __builtin_bit_cast(double, (w0 << 32) | (w1 & 0xffffffffull));
            return true;
        }
        if ((++spins & 63) == 0) {
            int bad = 0;
            if (lane == 0) {
                bad = ld_flag(err);
                if (!bad && spins > limit) {
                    st_flag(err, 1);
                    bad = 1;
                }
            }
            if (__shfl(bad, 0, 64)) return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Offset of A(R, C) in the band on entry (bandwidth b, lower storage
// Bd(r, c) = A(c + r, c)), or -1 outside the band.  Branch-free, so that the
// window's 32 loads issue back to back.
__device__ inline long band_offset(int n, int b, int ldb, int R, int C)
{
    const int lo = min(R, C), dist = abs(R - C);
    const bool in = R >= 0 && C >= 0 && R < n && C < n && dist <= b;
    return in ? (long)lo * ldb + dist : -1;
}

// Value of v in lane `lane` (wave-uniform) in every lane, through two scalar
// register reads rather than a cross-lane permute through the LDS unit.
__device__ __forceinline__ double lane_value(double v, int lane)
{
    const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)w, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(w >> 32), lane);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// One-hot mask of column slot `slot` among the wave's slots 16q .. 16q+15
// (0 when another wave holds it).  The mask is made opaque to the compiler so
// that the per-slot selects below stay selects on fixed registers instead of
// being turned into indexed vector accesses.
__device__ __forceinline__ unsigned slot_mask(int slot, int q)
{
    const int j = slot - 16 * q;
    unsigned m = __builtin_amdgcn_readfirstlane((j >= 0 && j < 16) ? (1u << j) : 0u);
    asm volatile("" : "+s"(m));
    return m;
}

__device__ __forceinline__ bool has(unsigned m, int j) { return (m >> j) & 1u; }

// Thread (l, q) = (tid % 64, tid / 64) holds the window row in slot l, in the
// column slots 16q .. 16q+15: ob (off-diagonal block) and dg (diagonal block,
// both triangles).  Slots >= b stay zero.
__global__ __launch_bounds__(256) void sb2st_window_kernel(SbWinArgs a)
{
    __shared__ double vps[SB], vs[SB], ws[SB], rowm[SB];
    __shared__ double red[4][SB];
    __shared__ double colbuf[4][16][SB + 1];   // per wave: the left application's products by column (padded)
    __shared__ double sh[2];   // tau, alpha
    __shared__ int abort_flag;
    const int tid = threadIdx.x;
    const int l = tid & 63;
    const int q = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n, b = a.b;
    const int k = blockIdx.x;
    double ob[16], dg[16];
    {
        const int R0 = 1 + k * b, p0 = R0 % b;
        const int R = (l < b) ? R0 + ((l - p0 + b) % b) : n;   // n: no row
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int c = 16 * q + j;
            const int cc = (c - p0 + b) % b;
            const long oo = (c < b) ? band_offset(n, b, a.ldb, R, R0 - b + cc) : -1;
            const long od = (c < b) ? band_offset(n, b, a.ldb, R, R0 + cc) : -1;
            const double xo = a.Bd[oo < 0 ? 0 : oo];
            const double xd = a.Bd[od < 0 ? 0 : od];
            ob[j] = (oo < 0) ? 0.0 : xo;
            dg[j] = (od < 0) ? 0.0 : xd;
        }
    }
    if (tid == 0) {
        abort_flag = 0;
        if (k == 0) a.d[0] = a.Bd[0];
    }
    __syncthreads();

    for (int s = 0; s < a.nsweeps && k < ntasks(n, b, s); ++s) {
        const int r0 = s + 1 + k * b;
        const int p = r0 % b;                  // slot of the top row
        const int pm = (p == 0) ? b - 1 : p - 1;   // slot of the row (and column) that left
        const int rowabs = r0 + ((l >= p) ? l - p : l - p + b);
        const bool valid = l < b && rowabs < n;
        const bool need_row = s > 0 && k + 1 < ntasks(n, b, s - 1);
        const bool need_v = k > 0;
        // ---- messages needed first, each wave polling what it uses itself (no
        // workgroup barrier before the right application): the reflector of
        // (s, k-1) (tag s+1), every wave its 16 entries and tau, and the alpha
        // of (s-1, k+1) (tag s), the entering row's entry in the column leaving
        // the diagonal block, by the wave holding that column.  The entering
        // row's other entries are needed only by the two-sided update and are
        // polled there.
        const unsigned mpm = slot_mask(pm, q);
        bool fail = false;
        double tp = 0.0;
        if (need_v) {
            const unsigned long long* box = a.vbox + ((size_t)(k - 1) * 2 + (s & 1)) * kBoxWords;
            double val = 0.0;
            fail = !poll_part(box, 16 * q, b, true, (unsigned)s + 1, a.err, a.spin_limit, val, tp);
            if (l < 16) vps[16 * q + l] = val;
            __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS stores are done
            __builtin_amdgcn_wave_barrier();
        }
        double alpha_in = 0.0;
        if (need_row && mpm)
            fail = !poll_value(a.vbox + ((size_t)(k + 1) * 2 + ((s - 1) & 1)) * kBoxWords, 65, (unsigned)s, a.err,
                               a.spin_limit, alpha_in) || fail;
        if (fail && l == 0) abort_flag = 1;
        // ---- move the window down one row: the column leaving the diagonal
        // block joins the off-diagonal block, and the entering row's only
        // nonzero there is alpha_in (its diagonal-block entries come later)
        if (s > 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (has(mpm, j)) ob[j] = dg[j];
            if (l == pm) {
#pragma unroll
                for (int j = 0; j < 16; ++j) ob[j] = has(mpm, j) ? alpha_in : 0.0;
            }
        }
        // ---- right application of the previous reflector: ob <- ob (I - tp vp vp^T)
        // (the barrier also settles a failed poll in every wave)
        {
            double part = 0.0;
            if (need_v) {
#pragma unroll
                for (int j = 0; j < 16; ++j) part += ob[j] * vps[16 * q + j];
            }
            red[q][l] = part;
            __syncthreads();
            if (abort_flag) return;
            if (need_v && tp != 0.0) {
                const double w = tp * (red[0][l] + red[1][l] + red[2][l] + red[3][l]);
#pragma unroll
                for (int j = 0; j < 16; ++j) ob[j] -= w * vps[16 * q + j];
            }
        }
        // ---- reflector of the block's first column (k >= 1) or of column s (k == 0)
        const int hc = (k > 0) ? p : pm;
        const int hq = hc >> 4;
        const unsigned mhc = slot_mask(hc, q);
        if (q == hq) {
            double x = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (has(mhc, j)) x = ob[j];
            if (!valid) x = 0.0;
            const double tail = wave_sum64((l != p) ? x * x : 0.0);
            const double x0 = lane_value(x, p);
            double t = 0.0, den = 1.0, alpha = x0;
            if (tail > 0.0) {
                const double nrm = sqrt(x0 * x0 + tail);
                alpha = (x0 >= 0.0) ? -nrm : nrm;
                t = (alpha - x0) / alpha;
                den = x0 - alpha;
            }
            const double v = (l == p) ? 1.0 : ((valid && tail > 0.0) ? x / den : 0.0);
            vs[l] = v;
            if (l == 0) {
                sh[0] = t;
                sh[1] = alpha;
            }
            unsigned long long* box = a.vbox + ((size_t)k * 2 + (s & 1)) * kBoxWords;
            if (k + 1 < ntasks(n, b, s)) {   // for the right application in task (s, k+1)
                if (l < b) put_value(box, l, v, (unsigned)s + 1);
                if (l == 0) put_value(box, 64, t, (unsigned)s + 1);
            }
            // alpha opens task (s+1, k-1): the entry of this window's top row
            // in the column just reflected
            if (k > 0 && s + 1 < a.nsweeps && k - 1 < ntasks(n, b, s + 1) && l == 0)
                put_value(box, 65, alpha, (unsigned)s + 1);
        }
        __syncthreads();
        const double t = sh[0], alpha = sh[1];
        const double v = vs[l];
        // ---- left application to the off-diagonal block.  The wave's 16 column
        // sums go through its own LDS block: lanes 4c .. 4c+3 sum a quarter of
        // column c each, a quad reduction completes it, and the 16 sums return
        // as scalars.
        if (k > 0 && t != 0.0) {
            double(*cb)[SB + 1] = colbuf[q];
#pragma unroll
            for (int j = 0; j < 16; ++j) cb[j][l] = v * ob[j];
            __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS stores are done
            __builtin_amdgcn_wave_barrier();
            const int c = l >> 2, r0q = (l & 3) * 16;
            double part = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) part += cb[c][r0q + i];
            part += __shfl_xor(part, 1, 64);
            part += __shfl_xor(part, 2, 64);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const double u = t * lane_value(part, 4 * j);
                ob[j] -= v * u;
            }
        }
        {
            const double col_out = (l == p) ? alpha : 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (has(mhc, j)) ob[j] = col_out;
        }
        // ---- the top row's entries left of the diagonal block are final now:
        // to workgroup k-1 for task (s+1, k-1) (its diagonal entry follows the
        // two-sided update).  The row sits in lane p; lanes 0 .. 15 each take
        // one of the wave's 16 values by a scalar read and store it.
        const bool row_out = k > 0 && s + 1 < a.nsweeps && k - 1 < ntasks(n, b, s + 1);
        unsigned long long* rbx = a.rbox + ((size_t)k * 2 + (s & 1)) * kBoxWords;
        if (row_out) {
            double mine = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const double x = lane_value(ob[j], p);
                if (l == j) mine = x;
            }
            if (l < 16 && 16 * q + l < b) put_value(rbx, 16 * q + l, mine, (unsigned)s + 1);
        }
        // ---- the entering row (of (s-1, k+1), tag s) into the diagonal block:
        // its entries as the new column and as its own lane's row; its
        // diagonal entry, published later, only by the wave holding that slot
        if (s > 0) {
            // wave 0 polls the entries; after the barrier the wave holding the
            // leaving slot polls the diagonal entry, the last value its sender
            // publishes, while the others go on
            const unsigned long long* box = a.rbox + ((size_t)(k + 1) * 2 + ((s - 1) & 1)) * kBoxWords;
            if (q == 0) {
                double val = 0.0;
                if (need_row && !poll_row(box, b, (unsigned)s, a.err, a.spin_limit, val) && l == 0) abort_flag = 1;
                rowm[l] = (l < b) ? val : 0.0;
            }
            __syncthreads();
            if (abort_flag) return;
            double rd = 0.0;
            if (mpm && need_row && !poll_value(box, 64, (unsigned)s, a.err, a.spin_limit, rd) && l == 0)
                abort_flag = 1;
            const double col_in = (l == pm) ? rd : rowm[l];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (has(mpm, j)) dg[j] = col_in;
            if (l == pm) {
#pragma unroll
                for (int j = 0; j < 16; ++j) dg[j] = has(mpm, j) ? rd : rowm[16 * q + j];
            }
        }
        // ---- two-sided update of the diagonal block: dg <- H dg H.  The top
        // row's diagonal entry goes to workgroup k-1 as soon as it is known:
        // with v_p = 1 it is dg_pp - (w_p + w_p), the value the update below
        // leaves there.
        const unsigned mp = slot_mask(p, q);
        double dpp = 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (has(mp, j)) dpp = dg[j];
        if (t != 0.0) {
            double part = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) part += dg[j] * vs[16 * q + j];
            red[q][l] = part;
            __syncthreads();
            const double pi = t * (red[0][l] + red[1][l] + red[2][l] + red[3][l]);
            const double beta = 0.5 * t * wave_sum64(pi * v);
            const double w = pi - beta * v;
            if (row_out && mp && l == p) put_value(rbx, 64, dpp - (v * w + w * v), (unsigned)s + 1);
            if (q == 0) ws[l] = w;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; ++j) dg[j] -= v * ws[16 * q + j] + w * vs[16 * q + j];
        } else if (row_out && mp && l == p) {
            put_value(rbx, 64, dpp, (unsigned)s + 1);
        }
        // ---- outputs: the reflector for Q2, and T's entries that are final
        if (q == 0 && valid) a.V2[cm(rowabs, s, n)] = v;
        if (tid == 0) a.tau2[(size_t)s * a.kmax + k] = t;
        if (k == 0) {
            if (tid == 0) a.e[s] = alpha;
            const int l1 = (p + 1 == b) ? 0 : p + 1;
            const unsigned ml1 = slot_mask(l1, q);
            double dp = 0.0, dl1 = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (has(mp, j)) dp = dg[j];
                if (has(ml1, j)) dl1 = dg[j];
            }
            if (l == p && mp) a.d[r0] = dp;
            if (s == a.nsweeps - 1 && l == l1) {
                if (ml1) a.d[n - 1] = dl1;
                if (mp) a.e[n - 2] = dp;
            }
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

size_t sb2st_mailbox_doubles(int n, int b) { return (size_t)sb2st_kmax(n, b) * 4 * kBoxWords; }

namespace {
std::atomic<int> g_bulge_path{0};   // 0: automatic, 1: row window (if it fits), 2: pipelined sweeps
}

void set_bulge_path(int path) { g_bulge_path.store(path); }

// Bd (ldb = 2b) -> (d, e); reflectors into V2 (n x n, ld n) and tau2
// (nsweeps x kmax).  progress: n ints of scratch (pipelined-sweep schedule);
// mbox: sb2st_mailbox_doubles (row-window schedule).
// Returns 0 (an expired wait sets *err and aborts the grid; the caller reports
// it), or kStatusHip when the launch fails.
int sb2st(hipStream_t st, int n, int b, double* Bd, int ldb, double* d, double* e, double* V2, double* tau2,
          int* progress, int* err, double* mbox)
{
    const int nsweeps = n - 2;
    fill_i(st, err, 1, 0);
    if (nsweeps <= 0) {
        hipLaunchKernelGGL(extract_tridiag_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, Bd, ldb, d, e);
        return 0;
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    cus = std::max(cus, 1);
    const int kmax = sb2st_kmax(n, b);
    const int path = g_bulge_path.load();
    int per_cu_w = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_w, sb2st_window_kernel, SBT, 0);
    const int resident_w = cus * std::max(0, per_cu_w);
    if (path != 2 && kmax <= resident_w) {
        // tag 0 everywhere: no word of a previous call can pass for a current one
        fill_d(st, mbox, sb2st_mailbox_doubles(n, b), 0.0);
        SbWinArgs a;
        a.n = n; a.b = b; a.nsweeps = nsweeps; a.kmax = kmax; a.ldb = ldb;
        a.Bd = Bd; a.V2 = V2; a.tau2 = tau2; a.d = d; a.e = e;
        a.vbox = (unsigned long long*)mbox;
        a.rbox = (unsigned long long*)mbox + (size_t)kmax * 2 * kBoxWords;
        a.err = err;
        a.spin_limit = 1LL << 22;
        void* args[] = {&a};
        // inside a batched call an ordinary launch, kept resident by the gate
        // (cooperative launches would run one problem's bulge chasing at a time)
        const long long share = persistent_enter(kmax, per_cu_w);
        const hipError_t rc =
            persistent_plain_ok(per_cu_w)
                ? hipLaunchKernel((const void*)sb2st_window_kernel, dim3(kmax), dim3(SBT), args, 0, st)
                : hipLaunchCooperativeKernel((const void*)sb2st_window_kernel, dim3(kmax), dim3(SBT), args, 0, st);
        persistent_leave(st, share);
        return rc == hipSuccess ? 0 : kStatusHip;
    }
    fill_i(st, progress, (size_t)nsweeps, 0);
    int per_cu = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sb2st_kernel, SBT, 0);
    int resident = std::max(1, cus * std::max(1, per_cu));
    // sweep s starts two tasks after sweep s-1, so a workgroup that takes
    // sweep s + grid after finishing sweep s (ntasks(0) tasks) never holds the
    // pipeline back once grid >= ntasks(0) / 2; a few spare workgroups absorb
    // uneven timing
    const int need = ((n - 2) / b + 1) / 2 + 8;
    int grid = std::min(nsweeps, std::min(std::min(resident, cus), need));
    SbArgs a;
    a.n = n; a.b = b; a.ldb = ldb; a.nsweeps = nsweeps; a.kmax = kmax;
    a.Bd = Bd; a.V2 = V2; a.tau2 = tau2; a.progress = progress; a.err = err;
    a.spin_limit = 1LL << 22;
    void* args[] = {&a};
    const long long share = persistent_enter(grid, std::max(1, per_cu));
    hipError_t rc = hipLaunchCooperativeKernel((const void*)sb2st_kernel, dim3(grid), dim3(SBT), args, 0, st);
    persistent_leave(st, share);
    if (rc != hipSuccess) return kStatusHip;
    hipLaunchKernelGGL(extract_tridiag_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, Bd, ldb, d, e);
    return 0;
}

}  // namespace eg
