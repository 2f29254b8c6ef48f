// Drivers of the dense path: reduction to standard form, density matrix, and
// (below) the eigensolver / density-matrix entry points.
#include "api_internal.h"

#include <algorithm>

namespace eg {

// Eq. (11): W = L^-1 H, then H~ = W L^-T, then H~ <- (H~ + H~^T)/2.
void reduce_to_standard(hipStream_t st, int n, double* H, int ldh, const double* L, int ldl, double* Linv)
{
    dtrtri_diag_blocks(st, n, L, ldl, Linv);
    mirror_lower_to_upper(st, n, H, ldh);   // only the lower triangle of H is read
    dtrsm_left_lower_n(st, n, n, L, ldl, Linv, H, ldh);
    dtrsm_right_lower_t(st, n, n, L, ldl, Linv, H, ldh);
    symmetrize_average(st, n, H, ldh);
}

// Eq. (9): D = sum_l f_l c_l c_l^T = (C F^1/2)(C F^1/2)^T, lower tiles on the
// matrix cores, then mirrored.
void density_matrix(hipStream_t st, int n, int k, const double* C, int ldc, const double* f, double* W,
                    double* D, int ldd)
{
    if (k <= 0) {
        for (int j = 0; j < n; ++j) fill_d(st, D + cm(0, j, ldd), (size_t)n, 0.0);
        return;
    }
    scale_columns_sqrt(st, n, k, C, ldc, f, W, n);
    dgemm(st, 'N', 'T', n, n, k, 1.0, W, n, W, n, 0.0, D, ldd, 1);
    mirror_lower_to_upper(st, n, D, ldd);
}

size_t workspace_bytes(const elsi_gpu_handle_s* h)
{
    (void)h;
    return 0;
}

void release_workspace(elsi_gpu_handle_s* h)
{
    if (h->ws && h->ws_owned) (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
    h->ws_owned = 0;
}

}  // namespace eg

extern "C" {

int elsi_gpu_ev(elsi_gpu_handle h, double* H, double* S, double* eval, double* evec)
{
    (void)H; (void)S; (void)eval; (void)evec;
    if (!h) return -1;
    return ELSI_GPU_ERR_HIP;
}

int elsi_gpu_dm(elsi_gpu_handle h, double* H, double* S, double* occ, double* D, double* eval,
                double* energy, double* mu)
{
    (void)H; (void)S; (void)occ; (void)D; (void)eval; (void)energy; (void)mu;
    if (!h) return -1;
    return ELSI_GPU_ERR_HIP;
}

}  // extern "C"
