// Handle layout and internal driver declarations shared by api.hip and solver.hip.
#pragma once
#include "../../include/elsi_gpu.h"
#include "common.h"

#include <algorithm>

namespace eg {

constexpr double kFCut = 1e-20;   // eigenvectors with f_l <= kFCut do not enter D

// RAII device buffer for the stage entry points.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    bool alloc(size_t count) {
        if (count == 0) count = 1;
        return hipMalloc((void**)&p, count * sizeof(T)) == hipSuccess;
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

inline int sync_status(hipStream_t st)
{
    hipError_t e = hipGetLastError();
    if (e == hipErrorOutOfMemory) return kStatusOom;
    if (e != hipSuccess) return kStatusHip;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return kStatusHip;
    return 0;
}

// H <- L^-1 H L^-T (full symmetric on exit); Linv receives the 64 x 64 block inverses.
void reduce_to_standard(hipStream_t st, int n, double* H, int ldh, const double* L, int ldl, double* Linv);

// D = C diag(f) C^T, both triangles, for occupations of either sign; W and W2
// are n x k scratch.
void density_matrix(hipStream_t st, int n, int k, const double* C, int ldc, const double* f, double* W, double* W2,
                    double* D, int ldd);

// Complex Hermitian pencils through their real 2n x 2n image (complex.hip):
// complex matrices are interleaved (real, imaginary) doubles, column-major.
void embed_complex(hipStream_t st, int n, const double* Z, int ldz, double* R, int ldr, bool lower_factor);
void extract_complex(hipStream_t st, int n, const double* R, int ldr, double* Z, int ldz, bool lower_factor);
void pair_values(hipStream_t st, int n, const double* w2, double* w);
void extract_vectors(hipStream_t st, int n, int k, const double* U, int ldu, double* C, int ldc);
void duplicate_values(hipStream_t st, int k, const double* f, double* f2);
void orthonormalize_complex_images(hipStream_t st, int n, int k, double* U, int ldu, double* JU, double* Bm);
// One real standard-form eigenvector per wanted complex state (k of them) from
// the k2 computed ones X (2n rows), w2 the doubled spectrum on the host; dsrc
// is device scratch of k ints.
int select_complex_states(hipStream_t st, int n, int k, const double* w2, const double* X, int ldx, int k2,
                          double* U, int ldu, int* dsrc);

// FP64 refinement of an approximate invariant subspace of the standard-form
// matrix (refine.hip).
//
// An approximate factorization H~ ~ Q T Q^T (T = tridiag(e, d, e)) with Z,
// the eigenvectors of T for its k lowest eigenvalues (n x k, ldz): the
// refinement's Newton correction goes through it.  apply_qt / apply_q
// overwrite X (n x ncol, ld) with Q^T X / Q X; tmp is n x ncol scratch of the
// same leading dimension.
struct RefinePrecond {
    const double* Z = nullptr;
    int ldz = 0;
    const double* d = nullptr;
    const double* e = nullptr;
    virtual ~RefinePrecond() = default;
    virtual void apply_qt(hipStream_t st, double* X, int ld, int ncol, double* tmp) = 0;
    virtual void apply_q(hipStream_t st, double* X, int ld, int ncol, double* tmp) = 0;
};

// Device buffers of one refinement: X[0] holds the start (n x k, ld ldb),
// X[1] and X[2] are scratch of the same shape; G, Qm: k x k; Linv:
// ceil(k / 64) * 4096 doubles; theta, r, step: k each; dinfo: one int; part:
// npart doubles of split-K scratch; U1 (n x k doubles) and SW (n x k bytes):
// the tridiagonal solves' factors (only with a factorization).
struct RefineBuffers {
    double* X[3];
    int ldb;
    double* G;
    double* Qm;
    double* Linv;
    double* theta;
    double* r;
    double* step;
    int* dinfo;
    double* part;
    size_t npart;
    double* U1;
    unsigned char* SW;
};

// On return X[out->x_buf] holds the refined vectors, theta the Ritz values
// ascending, r their residual norms and step the last computed Newton steps.
// kw: leading states that decide convergence, each step weighted by
// weight[l] (device, k values; NULL: 1).  pc NULL: one Rayleigh-Ritz sweep,
// converged when the residual norms are <= tol.
struct RefineOutcome {
    int x_buf;
    int sweeps;
    int converged;
    double rmax;   // largest residual norm of the first kw states after the last sweep
    double smax;   // largest weighted step of the first kw states (-1: none computed)
    double hist[8];   // smax of each of the first eight sweeps
};
size_t refine_scratch_doubles(int n, int k);
int refine_subspace(hipStream_t st, int n, int k, int kw, const double* Ht, int ldh, const RefineBuffers& B,
                    RefinePrecond* pc, const double* weight, double tol, int max_sweeps, RefineOutcome* out);

// Guard states carried beyond the kw wanted ones in the mixed path.
inline int refine_columns(int n, int kw)
{
    const int g = std::max(64, (kw + 9) / 10);
    return std::min(n, kw + g);
}

}  // namespace eg

struct elsi_gpu_handle_s {
    int dtype = 0;
    int n = 0;
    int n_state = 0;
    double n_electron = 0.0;
    hipStream_t stream = nullptr;
    int occ_scheme = ELSI_GPU_OCC_FERMI;
    double kT = 0.01;
    double occ_accuracy = 1e-13;
    int mu_max_steps = 100;
    double spin = 1.0;
    int overlap_is_unit = 0;
    int overlap_factored = 0;
    int band_width = 64;
    int batch_workers = 8;
    int band_tab_count = 0;       // per-size band widths of the batched calls
    int band_tab_nmax[16] = {};
    int band_tab_b[16] = {};
    int values_copies = 0;         // workspace holds copies of H and S (eigenvalue pass of a batch)
    int sing_check = 0;            // singularity check of S (Eq. (20)) before the transformation
    double sing_tol = 1e-5;        // its tolerance tau
    int sing_m = 0;                // > 0: the last call took the eigendecomposition route, S holds X (n x m)
    int precision = ELSI_GPU_PREC_FP64;
    double refine_tol = 1e-10;
    int max_refine = 6;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int ws_owned = 0;
    // second stream and events of full -> band (created by elsi_gpu_init,
    // released by elsi_gpu_finalize; batch workers and inner handles borrow
    // or leave them null)
    hipStream_t aux_stream = nullptr;
    hipEvent_t aux_ev[2] = {nullptr, nullptr};
    elsi_gpu_info info;
};

namespace eg {
size_t workspace_bytes(const elsi_gpu_handle_s* h);
void release_workspace(elsi_gpu_handle_s* h);
// All eigenvalues of the handle's pencil with H and S left intact (solver.hip).
int eigenvalues_only(elsi_gpu_handle_s* h, const double* H, const double* S, double* eval);
}  // namespace eg
