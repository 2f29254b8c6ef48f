// Internal helpers shared by the HIP translation units of libelsi_gpu.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <algorithm>
#include <cstdint>
#include <vector>

namespace eg {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kStatusOk = 0;
constexpr int kStatusNotPD = 1;
constexpr int kStatusNoConv = 2;
constexpr int kStatusRefine = 3;
constexpr int kStatusMu = 4;
constexpr int kStatusHip = 5;
constexpr int kStatusOom = 6;

// Record the first HIP error; launchers return it as status 5.
struct HipCheck {
    hipError_t err = hipSuccess;
    inline bool ok(hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) err = e;
        return e == hipSuccess;
    }
};

// Panels per block reflector in the back-transformation with Q1; the
// full -> band stage stores each panel's V with (kQ1Group - 1) b zero rows
// above it so that a group reads as one matrix.
constexpr int kQ1Group = 8;

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Column-major element address.
__host__ __device__ inline size_t cm(int i, int j, int ld) {
    return (size_t)j * (size_t)ld + (size_t)i;
}

// ---------------------------------------------------------------------------
// Sum over the 64 lanes of a wave with DPP lane moves (no LDS round trips):
// swaps inside quads, rotations inside rows of 16, then row broadcasts, which
// leave the total in lane 63; it is read from there, so every lane gets the
// same bits.  Each double moves as two 32-bit halves.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add_f64(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    const unsigned long long o = (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32);
    return v + __builtin_bit_cast(double, o);
}

__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v = dpp_add_f64<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
    v = dpp_add_f64<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
    v = dpp_add_f64<0x124, 0xf>(v);   // row_ror:4
    v = dpp_add_f64<0x128, 0xf>(v);   // row_ror:8
    v = dpp_add_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// X = L^-1 for the lower triangular jb x jb block L (zero beyond jb, jb <= 64,
// LDS arrays of pitch 65), by the NT threads of one workgroup: X_cc = 1 / L_cc,
// then for adjacent blocks A (first) and B of doubling size 2^lg
// X_BA = -X_BB (L_BA X_AA); Y is LDS scratch.  Only the lower triangle of L is
// read.
template <int NT>
__device__ __forceinline__ void tri_inverse_lower64(int jb, double (*Lm)[65], double (*X)[65], double (*Y)[65])
{
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 * 64; e += NT) {
        const int r = e & 63, c = e >> 6;
        X[r][c] = (r == c && r < jb) ? 1.0 / Lm[r][r] : 0.0;
    }
    __syncthreads();
    // each dot product's LDS operands are loaded into registers before its
    // multiply-adds, so that the loads are in flight together (the sums keep
    // their order: entries a .. sz-1, and 0 .. bb)
#pragma unroll
    for (int lg = 0; lg < 6; ++lg) {
        const int sz = 1 << lg;
        const int nout = 32 << lg;   // (64 / 2sz) pairs of sz x sz blocks
        for (int e = tid; e < nout; e += NT) {
            const int pr = e >> (2 * lg), rem = e & (sz * sz - 1);
            const int bb = rem & (sz - 1), a = rem >> lg;
            const int p0 = pr << (lg + 1), pb = p0 + sz;
            double lv[32], xv[32];
#pragma unroll
            for (int ii = 0; ii < (1 << lg); ++ii) {
                lv[ii] = Lm[pb + bb][p0 + ii];
                xv[ii] = X[p0 + ii][p0 + a];
            }
            double y = 0.0;
#pragma unroll
            for (int ii = 0; ii < (1 << lg); ++ii)
                if (ii >= a) y += lv[ii] * xv[ii];
            Y[pb + bb][p0 + a] = y;
        }
        __syncthreads();
        for (int e = tid; e < nout; e += NT) {
            const int pr = e >> (2 * lg), rem = e & (sz * sz - 1);
            const int bb = rem & (sz - 1), a = rem >> lg;
            const int p0 = pr << (lg + 1), pb = p0 + sz;
            double xv[32], yv[32];
#pragma unroll
            for (int jj = 0; jj < (1 << lg); ++jj) {
                xv[jj] = X[pb + bb][pb + jj];
                yv[jj] = Y[pb + jj][p0 + a];
            }
            double t = 0.0;
#pragma unroll
            for (int jj = 0; jj < (1 << lg); ++jj)
                if (jj <= bb) t += xv[jj] * yv[jj];
            X[pb + bb][p0 + a] = -t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host-side launchers implemented in the .hip files
// ---------------------------------------------------------------------------

// Batched calls run several problems at once from host worker threads on
// their own streams.  While such a call is active, kernels whose workgroups
// wait on one another are admitted to the device through a gate counted in
// shares of the device: a kernel of w workgroups of which p fit on one compute
// unit takes w / (p x compute units), and the admitted kernels together take
// at most half (a kernel with p < 3 is admitted alone).  The runtime runs
// cooperative launches one at a time across all streams, so inside a batch a
// kernel with p >= 3 takes an ordinary launch (persistent_plain_ok); the gate
// is what keeps every admitted one fully resident then (batched.hip gives the
// argument).  enter() blocks until the kernel fits and returns its share;
// leave() waits for the kernel on its stream and returns the share.  Outside
// batched calls enter() returns 0 and both are no-ops.
bool batch_mode_active();
long long persistent_enter(int workgroups, int per_cu);
void persistent_leave(hipStream_t st, long long share);
bool persistent_plain_ok(int per_cu);

// Optional device timing of individual launches (off by default).  While it is
// enabled, the GEMM launchers bracket every launch with a pair of events on the
// launch stream and record the launch's algorithmic flops under the id of the
// kernel instantiation; harvest() waits for the events and folds them into
// per-instantiation totals.
namespace launch_probe {
void enable(bool on);
bool enabled();
int begin(hipStream_t st);   // returns a slot (or -1 when disabled / pool exhausted)
void end(hipStream_t st, int slot, int kernel_id, double flops);
void harvest();              // synchronizes the recorded events
void reset_totals();
// instantiation with the largest summed device time since reset_totals()
bool dominant(int* launches, double* ms, double* flops, const char** name);
}  // namespace launch_probe

// C = alpha * op(A) op(B) + beta * C (FP64 MFMA).  op = 'N' or 'T'; for A
// also 'S': A is symmetric (m == k) and only its lower triangle is read
// (op(B) must then be 'N').
// uplo: 0 = all tiles, 1 = only tiles that touch the lower triangle (i >= j).
// C may alias A only when n <= 64 (each workgroup then reads exactly the A rows
// it writes) and beta == 0; C may alias B only when m <= 64 and beta == 0.
void dgemm(hipStream_t st, char ta, char tb, int m, int n, int k, double alpha,
           const double* A, int lda, const double* B, int ldb, double beta,
           double* C, int ldc, int uplo = 0);

// While an Fp32GemmScope(true) lives, the products that dgemm and dgemm_splitk
// launch from this host thread round their FP64 operands to FP32 and multiply
// and accumulate in FP32 on the matrix cores; inputs and outputs stay FP64.
// (dgemm_tn_small is not affected.)
class Fp32GemmScope {
public:
    explicit Fp32GemmScope(bool on);
    ~Fp32GemmScope();
    Fp32GemmScope(const Fp32GemmScope&) = delete;
    Fp32GemmScope& operator=(const Fp32GemmScope&) = delete;

private:
    bool on_;
};

// As dgemm, split over K into partial products (summed in a fixed order) when
// the output has too few tiles to fill the GPU; `work` holds the partials.
void dgemm_splitk(hipStream_t st, char ta, char tb, int m, int n, int k, double alpha,
                  const double* A, int lda, const double* B, int ldb, double beta, double* C,
                  int ldc, double* work, size_t work_doubles);

// C(:, cmap[j]) = alpha A B(:, j) + beta C(:, cmap[j]) for j < n (op = 'N' for
// both; cmap on the device, a map into C's columns without repeats).
void dgemm_colmap(hipStream_t st, int m, int n, int k, double alpha, const double* A, int lda, const double* B,
                  int ldb, double beta, double* C, int ldc, const int* cmap);

// Deterministic split-K product W = A^T B for tall A (k x m), B (k x n),
// m, n <= 64: partial products over row chunks are summed in a fixed order.
// `part` needs ceil(k / chunk) * m * n doubles.
void dgemm_tn_small(hipStream_t st, int m, int n, int k, double alpha, const double* A, int lda,
                    const double* B, int ldb, double beta, double* C, int ldc, double* part,
                    int chunk = 2048);

// Cholesky S = L L^T in place (lower).  Linv receives the inverses of the
// nb x nb diagonal blocks (nb = 64), laid out block after block (64 x 64 each).
// info (device int) is set to j+1 for the first non-positive pivot j, else left 0.
void dpotrf(hipStream_t st, int n, double* A, int lda, double* Linv, int* info);

// Inverses of the 64 x 64 diagonal blocks of a lower triangular L.
void dtrtri_diag_blocks(hipStream_t st, int n, const double* L, int ldl, double* Linv);

// Triangular solves with the lower Cholesky factor, using the block inverses.
//   left_lower_n : B <- L^-1 B     (n x ncol)
//   right_lower_t: B <- B L^-T     (nrow x n)
//   left_lower_t : B <- L^-T B     (n x ncol)
void dtrsm_left_lower_n(hipStream_t st, int n, int ncol, const double* L, int ldl,
                        const double* Linv, double* B, int ldb);
void dtrsm_right_lower_t(hipStream_t st, int nrow, int n, const double* L, int ldl,
                         const double* Linv, double* B, int ldb);
void dtrsm_left_lower_t(hipStream_t st, int n, int ncol, const double* L, int ldl,
                        const double* Linv, double* B, int ldb);
//   right_lower_t_lowerpart: lower triangle of B <- B L^-T (B n x n)
void dtrsm_right_lower_t_lowerpart(hipStream_t st, int n, const double* L, int ldl,
                                   const double* Linv, double* B, int ldb);

// Utility kernels.
void fill_d(hipStream_t st, double* p, size_t count, double v);
void fill_i(hipStream_t st, int* p, size_t count, int v);
void copy_matrix(hipStream_t st, int m, int n, const double* A, int lda, double* B, int ldb);
// up to kMaxCopies independent copies B_c = A_c (m_c x n_c) in one launch
struct CopyDesc {
    int m, n;
    const double* A;
    int lda;
    double* B;
    int ldb;
};
constexpr int kMaxCopies = 8;
struct CopyBatch {
    int count = 0;
    CopyDesc d[kMaxCopies];
    void add(int m, int n, const double* A, int lda, double* B, int ldb)
    {
        if (m > 0 && n > 0) d[count++] = CopyDesc{m, n, A, lda, B, ldb};
    }
};
void copy_matrices(hipStream_t st, const CopyBatch& cb);
void mirror_lower_to_upper(hipStream_t st, int n, double* A, int lda);
void symmetrize_average(hipStream_t st, int n, double* A, int lda);
void set_identity(hipStream_t st, int n, double* A, int lda);
void scale_columns_sqrt(hipStream_t st, int n, int k, const double* C, int ldc, const double* f,
                        double* out, int ldo);
void check_finite(hipStream_t st, int m, int n, const double* A, int lda, int* flag);

// Occupations and chemical potential on the device (one workgroup) for a
// broadening scheme (ELSI_GPU_OCC_FERMI, _GAUSSIAN, _MP0, _MP1) of width
// `width`: eps (n; ascending within each problem), weight (n per-state
// weights for a mu shared by several problems, or NULL); f (n) out, w_l f_l;
// scal (device, 6 doubles) out: mu, status, k_s (one past the last |f| >
// f_cut), energy sum f eps, bisection steps, surplus left.
void occupations(hipStream_t st, int n, const double* eps, const double* weight, int scheme, double n_electron,
                 double width, double spin, double occ_accuracy, int max_steps, double f_cut, double* f,
                 double* scal);
// out = C sqrt|f|, out2 = C sign(f) sqrt|f| (n x k, ldo): out out2^T = C F C^T.
void scale_columns_signed(hipStream_t st, int n, int k, const double* C, int ldc, const double* f, double* out,
                          double* out2, int ldo);

// Explicit occupations: f given for all n states; scal: mu (0), status (0),
// k_s (1 + last index with f > f_cut), energy (sum f eps).
void explicit_occupations(hipStream_t st, int n, int n_state, const double* eps, const double* f,
                          double f_cut, double* scal);

// Step (1): full (n x n, full symmetric) -> band; see sy2sb.hip.
size_t sy2sb_workspace_doubles(int n, int b);
// A second stream and two events for full -> band: when given, each panel's
// Gram matrix V^T V and T factor run on st2 while st forms Y = A22 V.
struct Sy2sbAux {
    hipStream_t st2;
    hipEvent_t ev_v, ev_t;
};
void sy2sb(hipStream_t st, int n, int b, double* A, int lda, double* Vall, double* Tall, double* Bd,
           int ldbd, double* work, const Sy2sbAux* aux = nullptr);

// Step (2): band -> tridiagonal; see sb2st.hip.
int sb2st_kmax(int n, int b);
size_t sb2st_mailbox_doubles(int n, int b);
int sb2st(hipStream_t st, int n, int b, double* Bd, int ldb, double* d, double* e, double* V2, double* tau2,
          int* progress, int* err, double* mbox);
// 0: automatic (row window when its grid fits the device), 1: row window
// when it fits, 2: pipelined sweeps; process-wide, for tests
void set_bulge_path(int path);

// Step (3): tridiagonal divide and conquer; see stedc.hip.
struct MergeDescH {
    int o, n1, n2;
};
struct DcState {
    int n = 0, ldz = 0;
    double* Z = nullptr;      // where the eigenvectors end up
    double* Zin = nullptr;    // solved halves of the last merge
    double* Zout = nullptr;
    double* U = nullptr;      // coefficient blocks of the last merge (root columns first)
    bool have_last = false;
    std::vector<MergeDescH> last;
    const MergeDescH* last_dev = nullptr;   // the last merge's descriptor on the device
    void* work = nullptr;                   // the solver's scratch (merge bookkeeping)
    // Q2's block T factors were launched beside this solve (on another stream):
    // the stream that applies Q2 waits on q2t_ev (if set) and skips the build
    bool q2t_built = false;
    hipEvent_t q2t_ev = nullptr;
    const double* q1t = nullptr;   // Q1's group T' factors, built on the same stream before q2t_ev
};
size_t stedc_workspace_bytes(int n);
int stedc_values(hipStream_t st, int n, const double* d, const double* e, double* w, double* Z, double* Z2,
                 double* U, int ldz, void* work, int* err, DcState* state);
void stedc_vectors(hipStream_t st, DcState& state, int ncol);
int stedc(hipStream_t st, int n, const double* d, const double* e, double* w, double* Z, double* Z2,
          double* U, int ldz, int ncol_final, void* work, int* err, int* err_host_copy);

// Steps (4) and (5): back-transformations; see backtx.hip.
size_t apply_q2_workspace_doubles(int n, int b);
// The block T factors of Q2 (apply_q2_workspace_doubles(n, b) doubles at Tq),
// built from the bulge-chasing reflectors alone; apply_q2 with tq_ready uses them.
void build_q2_t(hipStream_t st, int n, int b, const double* V2, const double* tau2, int kmax, double* Tq);
void apply_q2(hipStream_t st, int n, int b, int ncol, const double* V2, const double* tau2, int kmax,
              double* X, int ldx, double* Tq, bool trans = false, bool tq_ready = false, int slab = 0);
int q2_slab_width(int n, int b, int ncol);
size_t apply_q1_workspace_doubles(int n, int ncol);
// The group T' factors of Q1 (q1_tfactor_doubles(n, b) doubles at Tq1), built
// from the panel reflectors alone, with the scratch of an apply_q1 workspace
// for ncol columns; apply_q1 given Tq1 uses them instead of building its own.
size_t q1_tfactor_doubles(int n, int b);
void build_q1_t(hipStream_t st, int n, int b, int ncol, const double* Vall, const double* Tall, double* Tq1,
                double* work);
void apply_q1(hipStream_t st, int n, int b, int ncol, const double* Vall, const double* Tall, double* X,
              int ldx, double* work, bool trans = false, const double* Tq1 = nullptr);

}  // namespace eg
