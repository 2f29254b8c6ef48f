/*
 * elsi_gpu.h -- C ABI of libelsi_gpu, a single-GPU (AMD Instinct MI355X,
 * gfx950) solver for the dense Kohn-Sham generalized eigenproblem and the
 * density matrix built from it.
 *
 * What is computed (ELSI paper, arXiv 1705.11191):
 *   - H c = eps S c for real symmetric H and symmetric positive definite S,
 *     Sec. 2, Eq. (6);
 *   - by Cholesky S = L L^T, Eq. (10); reduction H~ = L^-1 H L^-T and
 *     back substitution c = L^-T c~, Eq. (11); two-stage tridiagonalization
 *     B = Q1 H~ Q1^T, T = Q2 B Q2^T, Eq. (13); divide and conquer on T and
 *     back-transformation through Q2 and Q1 -- the five steps of Fig. 1
 *     (Sec. 3.1);
 *   - Fermi-Dirac occupations, Eq. (17), with the chemical potential fixed by
 *     the electron count, Eq. (18), found by bisection and followed by the
 *     exact charge fix-up described for elsi_dm_real (Sec. 4.5);
 *   - the density matrix n_ij = sum_l f_l c_il c_jl, Eq. (9), and the band
 *     energy sum_l f_l eps_l (Sec. 4.5).
 *
 * Conventions for every entry point:
 *   - matrices are column-major; the leading dimension equals n_basis unless
 *     an argument says otherwise; only the lower triangle of a symmetric
 *     input is read;
 *   - "device" pointers point to GPU memory on the current HIP device, "host"
 *     pointers to CPU memory; the caller owns every buffer it passes; the
 *     library keeps no caller pointer after a call returns, except a
 *     workspace registered with elsi_gpu_set_workspace;
 *   - calls are synchronous: they return after the handle's stream has
 *     finished the work;
 *   - return value: 0 success; -i the i-th argument is invalid (LAPACK style,
 *     counted from 1, nothing was launched); a positive value is a numerical
 *     or runtime failure (ELSI_GPU_ERR_*), see elsi_gpu_strerror.
 *   - energies are in Hartree; the library does no unit conversion.
 * One handle serves one host thread at a time; several handles may be used
 * concurrently (the paper's opaque handle without globals, Sec. 4.3).
 */
#ifndef ELSI_GPU_H
#define ELSI_GPU_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct elsi_gpu_handle_s *elsi_gpu_handle;

/* scalar type of H, S, eigenvectors and D (Sec. 4.5: elsi_ev_real / _complex).
 * ELSI_GPU_COMPLEX128: complex Hermitian H, Hermitian positive definite S
 * (the k-point problems of periodic systems, Sec. 4.3).  Every matrix argument
 * of elsi_gpu_ev / elsi_gpu_dm (and of the batched calls) is then an array of
 * complex doubles, real and imaginary parts interleaved, column-major with the
 * same leading dimension n; eigenvalues, occupations, energy and mu stay real.
 * The library solves the real symmetric 2n x 2n image of the pencil (each
 * entry x + iy becomes the block [[x, -y], [y, x]]), which holds every complex
 * eigenvalue twice; D, the eigenvectors and L are read back from it.  This
 * costs 8x the real n x n flops (a native complex path would cost 4x).  The
 * stage entry points (elsi_gpu_x_*) are real only. */
enum { ELSI_GPU_REAL64 = 0, ELSI_GPU_COMPLEX128 = 1 };

/* occupation scheme (Sec. 4.6, broadening_scheme): explicit values given by
 * the caller, or a broadening of width w with x = (eps - mu) / w:
 *   FERMI     Fermi-Dirac, Eq. (17): f = spin / (1 + e^x);
 *   GAUSSIAN  Gaussian, Eq. (21): f = spin (1 - erf x) / 2;
 *   MP0       Methfessel-Paxton of order 0 (the Gaussian step);
 *   MP1       Methfessel-Paxton of order 1 (Phys. Rev. B 40, 3616 (1989)):
 *             f = spin (erfc(x) / 2 - x e^{-x^2} / (2 sqrt(pi))), which is
 *             negative for some states above mu and above spin for some
 *             below it.
 * (ELSI numbers them 2, 1, 3, 4.) */
enum {
    ELSI_GPU_OCC_EXPLICIT = 0,
    ELSI_GPU_OCC_FERMI = 1,
    ELSI_GPU_OCC_GAUSSIAN = 2,
    ELSI_GPU_OCC_MP0 = 3,
    ELSI_GPU_OCC_MP1 = 4
};

/* failure codes (positive return values) */
enum {
    ELSI_GPU_ERR_NOT_PD = 1,      /* S not positive definite; info.fail_col = first bad pivot (1-based) */
    ELSI_GPU_ERR_NO_CONV = 2,     /* tridiagonal eigensolver did not converge */
    ELSI_GPU_ERR_REFINE = 3,      /* mixed precision: refinement did not reach refine_tol (outputs
                                     still written; info.refine_step holds the step reached) */
    ELSI_GPU_ERR_MU = 4,          /* mu bisection ran out of steps (outputs still written) */
    ELSI_GPU_ERR_HIP = 5,         /* HIP runtime error */
    ELSI_GPU_ERR_OOM = 6,         /* device memory exhausted */
    ELSI_GPU_ERR_NONFINITE = 7    /* H or S holds NaN or Inf */
};

/* stages timed in elsi_gpu_info.stage_ms (the five steps of Fig. 1 plus the
 * transformations around them) */
enum {
    ELSI_GPU_ST_CHOLESKY = 0,   /* Eq. (10) */
    ELSI_GPU_ST_REDUCE = 1,     /* Eq. (11), H~ = L^-1 H L^-T */
    ELSI_GPU_ST_BAND = 2,       /* step (1): full -> band, Eq. (13) */
    ELSI_GPU_ST_BULGE = 3,      /* step (2): band -> tridiagonal, Eq. (13) */
    ELSI_GPU_ST_TRIDIAG = 4,    /* step (3): divide and conquer */
    ELSI_GPU_ST_OCC = 5,        /* Eq. (17)-(18) */
    ELSI_GPU_ST_BACK_Q2 = 6,    /* step (4) */
    ELSI_GPU_ST_BACK_Q1 = 7,    /* step (5) */
    ELSI_GPU_ST_BACKSUB = 8,    /* c = L^-T c~ */
    ELSI_GPU_ST_DENSITY = 9,    /* Eq. (9) */
    ELSI_GPU_ST_REFINE = 10,    /* FP64 refinement of the mixed-precision path */
    ELSI_GPU_NSTAGES = 11
};

/* arithmetic of elsi_gpu_ev / elsi_gpu_dm (elsi_gpu_set_precision) */
enum { ELSI_GPU_PREC_FP64 = 0, ELSI_GPU_PREC_MIXED = 1 };

typedef struct elsi_gpu_info {
    double stage_ms[ELSI_GPU_NSTAGES]; /* device time per stage of the last call */
    double total_ms;                   /* device time of the last call */
    double mu;                         /* chemical potential of the last dm call (Ha) */
    double energy;                     /* band energy of the last dm call (Ha) */
    double charge_residual;            /* electron surplus left after the fix-up */
    int k_s;                           /* eigenvectors that entered D (f_l > 1e-20) */
    int fail_col;                      /* first non-positive pivot of S (1-based), else 0 */
    int mu_steps;                      /* bisection steps taken */
    int band_width;                    /* b of step (1) */
    int n_basis;
    /* Launch timing (elsi_gpu_set_launch_timing): the GEMM kernel
     * instantiation with the largest summed device time since timing was
     * switched on, its launch count, summed device time and summed
     * algorithmic flops (2mnk per product, lower-triangle entries only for the
     * triangular updates).  Zero / empty while timing is off. */
    int probe_launches;
    double probe_ms;
    double probe_flops;
    char probe_kernel[48];
    /* Mixed precision (elsi_gpu_set_precision): refinement sweeps run, states
     * refined (wanted plus guard), the largest residual norm
     * ||H~ x - theta x||_2 of the wanted states after the last sweep (Ha; a
     * bound on their eigenvalue errors), and the largest weighted Newton
     * step of the wanted states (the estimate of their distance to the exact
     * invariant subspace that decides convergence; weights: the occupations
     * in dm, 1 in ev).  Zero in FP64 mode. */
    int refine_sweeps;
    int refine_states;
    double refine_resid;
    double refine_step;
    /* Singularity check (elsi_gpu_set_singularity): the smallest eigenvalue
     * of S found by the last check (0 when none ran), and N_nonsing, the
     * number of states of the last call (n_basis on the Cholesky route). */
    double overlap_min_eig;
    int n_nonsing;
    /* Mixed precision: the largest weighted Newton step measured in each of
     * the first eight refinement sweeps (0 beyond the last). */
    double refine_hist[8];
} elsi_gpu_info;

/* Create a handle (elsi_init, Sec. 4.4).  n_state: eigenvectors returned by
 * elsi_gpu_ev (1..n_basis); n_electron: electron count for elsi_gpu_dm;
 * hip_stream: the hipStream_t the calls run on (NULL = default stream); the
 * handle also creates a second stream and two events of its own, on which the
 * panel T factors of full -> band, and the block T factors of both
 * back-transformations (beside the tridiagonal solve), run beside the stream's work (the
 * calls still return with everything ordered after their work on hip_stream), and
 * elsi_gpu_finalize releases them.  Defaults: Fermi-Dirac, width 0.01 Ha, occ_accuracy 1e-13,
 * mu_max_steps 100, spin factor 1, band width 64.
 * Errors: -1 h NULL, -2 dtype, -3 n_basis < 1, -4 n_state outside 1..n_basis,
 * -5 n_electron < 0 or above n_basis. */
int elsi_gpu_init(elsi_gpu_handle *h, int dtype, int n_basis, int n_state,
                  double n_electron, void *hip_stream);

/* Device workspace the handle needs for elsi_gpu_ev / elsi_gpu_dm (bytes). */
int elsi_gpu_workspace_size(elsi_gpu_handle h, size_t *bytes);

/* Register a caller-owned device workspace of at least elsi_gpu_workspace_size
 * bytes (e.g. a torch tensor); it must stay valid until elsi_gpu_finalize or
 * the next call of this function.  Without it the library allocates its own
 * workspace on first use and frees it in elsi_gpu_finalize.
 * Errors: -2 NULL pointer, -3 too small. */
int elsi_gpu_set_workspace(elsi_gpu_handle h, void *dev_ptr, size_t bytes);

/* Occupation and chemical potential options (elsi_customize_mu, Sec. 4.6):
 * scheme ELSI_GPU_OCC_*, width = the broadening width in Ha (k_B T for
 * Fermi-Dirac; > 0), occ_accuracy (> 0), mu_max_steps (>= 1), spin_factor
 * (> 0; Fermi-Dirac and Gaussian f range over [0, spin_factor]).
 * Errors: -1 handle, -2 scheme, -3 width, -4 occ_accuracy, -5 mu_max_steps,
 * -6 spin_factor. */
int elsi_gpu_set_occupation(elsi_gpu_handle h, int scheme, double width,
                            double occ_accuracy, int mu_max_steps, double spin_factor);

/* Singularity check of the overlap (Sec. 4.5, Eq. (20); Sec. 4.6
 * no_singularity_check, singularity_tolerance), real handles.  With check = 1
 * every elsi_gpu_ev / elsi_gpu_dm whose S is not already factored first
 * computes all eigenvalues lam of S (by this library's FP64 path, an n^3 cost
 * comparable to the solve).  If the smallest is below tolerance, S is
 * singular for the purpose of the calculation and the Cholesky factorization
 * is replaced by the eigendecomposition S = x lam x^T = X X^T, X = x
 * lam^(1/2), keeping the N_nonsing eigenvectors with lam >= tolerance:
 * H~ = Y^T H Y with Y = x_keep lam_keep^(-1/2) is solved at size N_nonsing
 * (in FP64, whatever the handle's precision), and c = Y c~.  Then eval[0 ..
 * N_nonsing) holds the eigenvalues and eval[N_nonsing .. n) +HUGE_VAL (no
 * state there), occupations beyond N_nonsing are 0, eigenvector columns beyond
 * N_nonsing are 0, S receives X (n x N_nonsing in its first columns, the rest
 * zero) and info.n_nonsing = N_nonsing; with elsi_gpu_set_overlap_factored a
 * later call reuses that X (lam_j = ||X_j||^2).  check = 0 (default): the
 * Cholesky factorization, which reports a non-positive pivot.  Batched calls
 * do not run the check.
 * Errors: -1 handle, -2 check not 0 or 1, or a complex handle, -3 tolerance
 * not > 0. */
int elsi_gpu_set_singularity(elsi_gpu_handle h, int check, double tolerance);

/* overlap_is_unit (Sec. 4.6): S is the identity and is not read. */
int elsi_gpu_set_overlap_is_unit(elsi_gpu_handle h, int flag);

/* S already holds its Cholesky factor L from an earlier call on this handle
 * (the reuse of L across the SCF cycle, Sec. 4.5); the factorization is skipped. */
int elsi_gpu_set_overlap_factored(elsi_gpu_handle h, int flag);

/* Band width b of step (1) (Eq. (13)); 8 <= b <= 64, multiple of 8. */
int elsi_gpu_set_band_width(elsi_gpu_handle h, int b);

/* Arithmetic of elsi_gpu_ev / elsi_gpu_dm on a real handle (the paper's
 * solvers run in one precision; the mixed mode is this library's addition).
 * ELSI_GPU_PREC_FP64 (default): every step in FP64.
 * ELSI_GPU_PREC_MIXED: the matrix products of step (1) (full -> band) and of
 * step (5) (back-transformation by Q1) round their operands to FP32 and
 * multiply and accumulate in FP32 on the matrix cores; Cholesky, reduction
 * (Eq. (10), (11)), steps (2)-(4), storage and everything else stay FP64.
 * The library then carries k' = min(n, k + max(64, ceil(k / 10))) states
 * (k = n_state for ev, k_s for dm) and refines them in FP64 against
 * H~ = L^-1 H L^-T.  Each sweep: CholeskyQR twice, Rayleigh-Ritz with the
 * FP64 solver, residuals r_l = H~ x_l - theta_l x_l, and the Newton
 * correction of the subspace through the factorization H~ ~ Q T Q^T that
 * steps (1)-(3) produced (Q = Q1 Q2, Z the eigenvectors of T of the k'
 * states, P = I - Z Z^T): y_l = -P (T - theta_l)^-1 P Q^T r_l, with the
 * shifted tridiagonal systems solved per state.  When the largest weighted
 * step max_l w_l ||y_l||_2 over the wanted states (w_l = f_l in dm, 1 in ev)
 * is at most refine_tol, or the contraction measured over the last two
 * steps predicts that taking it leaves less than refine_tol
 * (10 (W_s / W_{s-1}) W_s <= refine_tol), that step is taken and one closing
 * Rayleigh-Ritz sweep ends the call with status 0 (an untaken step would be
 * amplified by L^-T in the eigenvectors c = L^-T x); otherwise x_l += Q y_l and the next
 * sweep starts, up to max_refine sweeps in all (default 6; then
 * ELSI_GPU_ERR_REFINE with all outputs written; max_refine = 0 skips the
 * refinement and also ends with ELSI_GPU_ERR_REFINE).  Eigenvalues above the
 * k' refined ones are the FP32-step values.  Needs about 3n^2 more doubles
 * of workspace.  Batched calls always run in FP64.
 * Complex handles: elsi_gpu_dm runs this mode on the real 2n x 2n image of
 * the pencil (FP32 products on the image carry complex64 precision, the
 * refinement complex128); elsi_gpu_ev on complex handles stays FP64.
 * Errors: -1 h NULL, -2 prec unknown, -3 refine_tol not >= 0,
 * -4 max_refine < 0. */
int elsi_gpu_set_precision(elsi_gpu_handle h, int prec, double refine_tol, int max_refine);

/* Measurement aid, not part of the method: on = 1 brackets every GEMM launch
 * with a pair of HIP events on the handle's stream and resets the totals
 * reported in elsi_gpu_info.probe_*; on = 0 stops it.  The totals are
 * harvested (the events synchronized) at the end of each elsi_gpu_ev /
 * elsi_gpu_dm call.  The timing state is process-wide: it covers launches of
 * every handle.  Errors: -1 null handle, -2 on not 0 or 1. */
int elsi_gpu_set_launch_timing(elsi_gpu_handle h, int on);

/* Eigenvalues and eigenvectors (elsi_ev_real / elsi_ev_complex, Sec. 4.5).
 *   H    device, n x n, in; destroyed on exit (complex handles leave it intact);
 *   S    device, n x n, in (SPD, or HPD); on exit holds L of Eq. (10) (lower,
 *        zero above; S = L L^H for complex handles);
 *   eval device, n doubles, out: all eigenvalues, ascending;
 *   evec device, n x n_state, out: S-orthonormal eigenvectors of the lowest
 *        n_state eigenvalues (c^H S c = I).  For complex handles each
 *        eigenvector carries an arbitrary phase; within a group of equal
 *        eigenvalues (to 1e-9 relative) the columns are an orthonormal basis of
 *        the group's eigenspace (groups of more than 32 equal eigenvalues are
 *        not reorthogonalized).
 * Errors: -1 handle, -2 H, -3 S, -4 eval, -5 evec; ELSI_GPU_ERR_NOT_PD, _NO_CONV,
 * _HIP, _OOM, _NONFINITE. */
int elsi_gpu_ev(elsi_gpu_handle h, double *H, double *S, double *eval, double *evec);

/* Density matrix (elsi_dm_real, Sec. 4.5; for complex handles
 * D = sum_l f_l c_l c_l^H, Hermitian).
 *   H, S    as for elsi_gpu_ev;
 *   occ     device, n doubles: in for ELSI_GPU_OCC_EXPLICIT (f of the states in
 *           ascending order, of either sign), out (the broadening scheme's
 *           occupations) otherwise; may be NULL for a broadening scheme;
 *   D       device, n x n, out: both triangles;
 *   eval    device, n doubles, out (may be NULL);
 *   energy  host, out: sum_l f_l eps_l;   mu  host, out (may be NULL).
 * Only the eigenvectors up to the last state with |f_l| > 1e-20 are formed
 * and used for D.
 * Errors: -1 handle, -2 H, -3 S, -4 occ (NULL in explicit mode), -5 D, -7 energy;
 * positive codes as for elsi_gpu_ev, plus ELSI_GPU_ERR_MU (outputs still written). */
int elsi_gpu_dm(elsi_gpu_handle h, double *H, double *S, double *occ, double *D,
                double *eval, double *energy, double *mu);

/* ------------------------------------------------------------------------
 * Batched calls: many independent problems of uneven size in one call, the
 * way ELSI treats k-points and spin channels as independent eigenproblems
 * (Sec. 4.3, parallel modes).  The handle supplies the settings (occupation
 * scheme and parameters, band width, overlap flags); its n_basis, n_state and
 * n_electron are not used.  Problem p has its own column-major device arrays
 * with ld = n[p].  A pool of host worker threads (elsi_gpu_set_batch_workers,
 * default 8), each with its own stream and device workspace (allocated for
 * the duration of the call), solves the problems largest first, so that the
 * kernels of different problems overlap on the device.  The caller's stream
 * is synchronized before the problems start; every output is complete when
 * the call returns.  status[p] (host) receives the return code of problem p
 * as its single-problem call would give it; a failing problem does not stop
 * the others.  Returns 0 when every problem succeeded, else the status of
 * the lowest-index failing problem; negative codes name a bad argument (-3
 * also covers a bad entry of a per-problem array).
 * ------------------------------------------------------------------------ */

/* Worker threads of the batched calls, 1 <= workers <= 16.  Each worker's
 * stream runs on one of the HIP runtime's hardware queues, of which there are
 * GPU_MAX_HW_QUEUES (read from the environment when the runtime starts;
 * 4 unless set): workers beyond that count share queues and their kernels
 * wait for each other, so set it to at least the worker count before the
 * process first uses the GPU.
 * Errors: -1 handle, -2 workers. */
int elsi_gpu_set_batch_workers(elsi_gpu_handle h, int workers);

/* Band widths b of step (1) per problem size for the batched calls (the
 * table an autotuner writes after timing each size bucket).  count entries
 * (0 <= count <= 16; 0 clears the table), host arrays: a problem of size n
 * takes b[i] of the first i with n <= n_max[i]; larger problems, and every
 * problem while the table is empty, take the handle's band width
 * (elsi_gpu_set_band_width).  n_max strictly increasing and >= 1; each b[i]
 * a multiple of 8 in [8, 64].  The table is copied; single-problem calls do
 * not use it.
 * Errors: -1 handle, -2 count, -3 n_max (NULL with count > 0, or not
 * increasing), -4 b (NULL with count > 0, or an invalid width). */
int elsi_gpu_set_batch_band_table(elsi_gpu_handle h, int count, const int *n_max, const int *b);

/* elsi_gpu_ev for count problems: n[p] basis functions, the n_state[p]
 * lowest eigenpairs into eval[p] (n[p] doubles) and evec[p] (n[p] x
 * n_state[p]); H[p] destroyed, S[p] receives L (S may be NULL with the unit
 * overlap flag).  Errors: -1 handle, -2 count < 0, -3 n or a per-problem
 * entry, -4 n_state, -5 H, -6 S, -7 eval, -8 evec, -9 status. */
int elsi_gpu_ev_batched(elsi_gpu_handle h, int count, const int *n, const int *n_state,
                        double *const *H, double *const *S, double *const *eval,
                        double *const *evec, int *status);

/* elsi_gpu_dm for count problems with the handle's broadening scheme (not
 * ELSI_GPU_OCC_EXPLICIT): D[p] (n[p] x n[p], both triangles), eval[p] (may
 * be NULL, or eval itself NULL), energy[p] and mu[p] (host arrays; mu may be
 * NULL).
 * kweight NULL: an independent chemical potential per problem, Eq. (18)
 * with n_electron[p] electrons, and f in [0, spin] as in elsi_gpu_dm.
 * kweight (host, count weights > 0): the problems are the k-points and spin
 * channels of one system sharing one chemical potential (the sum over k-points
 * and spin channels of Sec. 4.5): mu solves
 *   sum_p kweight[p] sum_l f(eps_pl - mu) = sum_p kweight[p] n_electron[p],
 * each problem's occupations include its weight, f_pl = kweight[p] f(eps_pl
 * - mu) (the bisection and the charge fix-up of Sec. 4.5 run over all states
 * of all problems, the fix-up from the last state of the last problem
 * downward), D[p] = sum_l f_pl c_pl c_pl^T (so sum_p tr(D[p] S[p]) is the
 * electron count), energy[p] = sum_l f_pl eps_pl and mu[p] the shared mu.
 * The eigenvalues of every problem are computed first (H and S are read,
 * not destroyed, by that pass), then each problem is solved with its
 * occupations fixed.
 * Errors: -1 handle or explicit occupation scheme, -2 count < 0, -3 n or a
 * per-problem entry, -4 n_electron, -5 a kweight entry not > 0, -6 H, -7 S,
 * -8 D, -10 energy, -12 status. */
int elsi_gpu_dm_batched(elsi_gpu_handle h, int count, const int *n, const double *n_electron,
                        const double *kweight, double *const *H, double *const *S,
                        double *const *D, double *const *eval, double *energy, double *mu,
                        int *status);

/* Timings and diagnostics of the last ev/dm call. */
int elsi_gpu_get_info(elsi_gpu_handle h, elsi_gpu_info *out);

/* Destroy the handle and free what the library allocated (elsi_finalize,
 * Sec. 4.7); *h is set to NULL. */
int elsi_gpu_finalize(elsi_gpu_handle *h);

/* Static text for a return code. */
const char *elsi_gpu_strerror(int status);

/* ------------------------------------------------------------------------
 * Stage entry points: one step of the path each, on caller-owned device
 * buffers, launched on hip_stream and synchronized before returning.  They
 * allocate their own scratch.  Same return conventions as above.
 * ------------------------------------------------------------------------ */

/* C = alpha op(A) op(B) + beta C in FP64 on the matrix cores; ta, tb = 'N' or
 * 'T'; C is m x n.  ta = 'S': A is symmetric with only its lower triangle
 * read (the product Y = A22 V of step (1), Eq. (13)); then k == m and
 * tb == 'N'.  Errors: -1 ta, -2 tb, -3..-5 sizes < 0 (-5 also k != m for 'S'). */
int elsi_gpu_x_dgemm(char ta, char tb, int m, int n, int k, double alpha, const double *A,
                     int lda, const double *B, int ldb, double beta, double *C, int ldc,
                     void *hip_stream);

/* The FP32-arithmetic products of the mixed mode (elsi_gpu_set_precision):
 * as elsi_gpu_x_dgemm with FP64 operands and result, but A and B are rounded
 * to FP32 and multiplied and accumulated in FP32 on the matrix cores; alpha
 * and beta are applied in FP64.  uplo = 1 writes only the entries C(i, j)
 * with i >= j (C square; the strict upper part is left untouched), uplo = 0
 * all of C.  Errors as elsi_gpu_x_dgemm, and -14 uplo not 0 or 1. */
int elsi_gpu_x_gemm_fp32(char ta, char tb, int m, int n, int k, double alpha, const double *A,
                         int lda, const double *B, int ldb, double beta, double *C, int ldc,
                         int uplo, void *hip_stream);

/* S <- L with S = L L^T, Eq. (10) (lower; strict upper set to zero).
 * *fail_col (host, may be NULL) receives the 1-based first bad pivot. */
int elsi_gpu_x_cholesky(int n, double *S, int lds, int *fail_col, void *hip_stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): elsi_gpu_x_cholesky
 * with the same kernels and results, but no hipMalloc, hipFree or other
 * allocating call.  Its scratch (the inverses of the 64 x 64 diagonal blocks
 * of L and the pivot flag, 8 MiB + 256 B) is a fixed device array that each
 * GPU holds until the process ends; the caller passes only S.  Every call on
 * one GPU shares that GPU's array, so calls that overlap on one GPU race.
 * Errors: -1 n < 0 or n > ELSI_GPU_NOALLOC_MAX_N (checked on the host, no
 * GPU call), -2 S NULL, -3 lds < n; 1 S not positive definite (*fail_col as
 * elsi_gpu_x_cholesky), 5 HIP error. */
#define ELSI_GPU_NOALLOC_MAX_N 16384
int elsi_gpu_x_cholesky_noalloc(int n, double *S, int lds, int *fail_col, void *hip_stream);

/* H <- L^-1 H L^-T, Eq. (11); H full symmetric on exit; L from Eq. (10). */
int elsi_gpu_x_reduce(int n, double *H, int ldh, const double *L, int ldl, void *hip_stream);

/* X <- L^-T X (back substitution below Eq. (11)); X is n x k. */
int elsi_gpu_x_backsub(int n, int k, const double *L, int ldl, double *X, int ldx,
                       void *hip_stream);

/* Occupations of a broadening scheme (Eq. (17), Eq. (21), Methfessel-Paxton)
 * and mu, Eq. (18) (Sec. 4.5): eps device (n; ascending within each problem
 * when several are concatenated), weight device (n per-state weights of a mu
 * shared by k-points / spin channels, f_l = w_l f(eps_l); NULL: 1), f device
 * out; mu, k_s (one past the last |f| > 1e-20) to host; returns the status
 * (0, or ELSI_GPU_ERR_MU).  Errors: -1 n, -2 eps, -4 scheme, -5 n_electron,
 * -6 width, -7 spin, -8 occ_accuracy, -9 mu_max_steps, -10 f. */
int elsi_gpu_x_occupations(int n, const double *eps, const double *weight, int scheme, double n_electron,
                           double width, double spin, double occ_accuracy, int mu_max_steps, double *f,
                           double *mu, int *k_s, void *hip_stream);

/* D = sum_{l<k} f_l c_l c_l^T, Eq. (9), for occupations of either sign:
 * C device n x k (ldc), f device (k), D device n x n (ldd), both triangles
 * written. */
int elsi_gpu_x_density(int n, int k, const double *C, int ldc, const double *f, double *D,
                       int ldd, void *hip_stream);

/* Step (1), Eq. (13): band B = Q1^T A Q1 of the symmetric A (lower triangle
 * read, A unchanged) with bandwidth b (1..64); band receives LAPACK lower band
 * storage, band[r + c*ldband] = B(c + r, c) for 0 <= r <= b (ldband >= b+1). */
int elsi_gpu_x_band_reduce(int n, int b, double *A, int lda, double *band, int ldband,
                           void *hip_stream);

/* Steps (1)+(2), Eq. (13): T = Q^T A Q tridiagonal (A unchanged); d (n) and
 * e (n-1) device out, e[i] = T(i+1, i). */
int elsi_gpu_x_tridiagonalize(int n, int b, double *A, int lda, double *d, double *e,
                              void *hip_stream);

/* Schedule of the bulge chasing in step (2), process-wide (a test hook: both
 * compute the same reflectors up to rounding).  0 automatic: the row-window
 * schedule (one workgroup per block row of the band, the band in registers)
 * whenever its grid of (n-2)/b+1 workgroups fits the device at once, else
 * the pipelined-sweep schedule (one workgroup per sweep, blocks through
 * device memory); 1 the same choice; 2 always the pipelined-sweep schedule.
 * Returns -1 for another value. */
int elsi_gpu_x_set_bulge_path(int path);

/* Steps (1)+(2) on A as elsi_gpu_x_tridiagonalize (d, e receive T), then
 * X (n x ncol, ldx, device) <- Q X (trans 0: steps (4) and (5), Q2 then Q1)
 * or Q^T X (trans 1: Q1^T then Q2^T, the map the mixed mode's refinement
 * takes residuals through), Q = Q1 Q2 the product of the reflectors with
 * T = Q^T A Q (Eq. (13)).  slab: columns of X per workgroup in the
 * application of Q2 (0 automatic; 128, 256 or 512).
 * Errors: -1 n < 1, -2 b outside 1..64, -3 A NULL, -4 lda < n, -5 d NULL,
 * -6 e NULL, -7 X NULL, -8 ldx < n, -9 ncol < 0, -10 trans, -11 slab. */
int elsi_gpu_x_backtransform(int n, int b, const double *A, int lda, double *d, double *e,
                             double *X, int ldx, int ncol, int trans, int slab, void *hip_stream);

/* Step (3): eigenvalues w (ascending) and eigenvectors Z (n x n, ldz) of the
 * symmetric tridiagonal (d, e) by divide and conquer. */
int elsi_gpu_x_tridiag_eig(int n, const double *d, const double *e, double *w, double *Z, int ldz,
                           void *hip_stream);

/* FP64 refinement sweeps of the mixed path (elsi_gpu_set_precision) on a
 * caller's subspace: Ht device n x n symmetric (both triangles, ldh; e.g. the
 * output of elsi_gpu_x_reduce), X device n x k (ldx) approximating the
 * invariant subspace of the k lowest eigenvalues, overwritten by the refined
 * vectors (orthonormal, Ritz order); theta (k) and resid (k) device out: Ritz
 * values ascending and ||Ht x_l - theta_l x_l||_2.
 * Q (device n x n, ldq, orthogonal), d (n) and e (n-1) (device) give an
 * approximate factorization Ht ~ Q T Q^T, T = tridiag(e, d, e); each sweep
 * then takes the Newton step y_l = -P (T - theta_l)^-1 P Q^T r_l (Z the
 * eigenvectors of T for its k lowest eigenvalues, P = I - Z Z^T; step (k,
 * device, may be NULL) receives ||y_l||_2) and ends the call with 0 when
 * max_{l < kw} w_l ||y_l||_2 <= tol (weight: device, k values, or NULL for
 * w = 1) after adding that step and one closing Rayleigh-Ritz sweep; until
 * then it adds Q y_l to x_l (only where ||y_l||_2 <= 1/2) and goes on, up to
 * max_sweeps sweeps in all.  Q NULL: one Rayleigh-Ritz sweep (it cannot move
 * span(X)), converged when max_{l < kw} resid_l <= tol.  *sweeps (host, may be
 * NULL) receives the sweeps run.
 * Returns ELSI_GPU_ERR_REFINE when tol was not reached (outputs written; with
 * max_sweeps = 0 nothing is written) or when the columns of X are
 * numerically dependent (the factorization is checked before X is touched:
 * X then holds the vectors of the last completed sweep, theta and resid that
 * sweep's values, and with no completed sweep X is unchanged);
 * ELSI_GPU_ERR_NO_CONV when the eigenvectors of T could not be computed.
 * Errors: -1 n < 0, -2 k outside 0..n, -3 kw outside 0..k, -4 Ht / ldh, -6 X /
 * ldx, -9 ldq, -10 d NULL with Q, -11 e NULL with Q, -13 theta, -14 resid,
 * -16 tol, -17 max_sweeps. */
int elsi_gpu_x_refine(int n, int k, int kw, const double *Ht, int ldh, double *X, int ldx,
                      const double *Q, int ldq, const double *d, const double *e,
                      const double *weight, double *theta, double *resid, double *step, double tol,
                      int max_sweeps, int *sweeps, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ELSI_GPU_H */
