"""Thin ctypes binding of libelsi_gpu (argument marshalling only).

Matrices cross the boundary column-major.  A torch tensor ``X`` of logical
shape (rows, cols) is passed as-is when it is column-major contiguous
(``X.stride() == (1, rows)``, e.g. made by :func:`fortran_empty` or a
symmetric matrix's transpose view); otherwise a column-major copy is made.
All compute happens in the HIP library: this module never computes any part
of the method, and it raises when the library is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libelsi_gpu.so")
_lib = None

REAL64 = 0
COMPLEX128 = 1
OCC_EXPLICIT = 0
OCC_FERMI = 1
OCC_GAUSSIAN = 2
OCC_MP0 = 3
OCC_MP1 = 4
PREC_FP64 = 0
PREC_MIXED = 1
NSTAGES = 11
STAGES = ["cholesky", "reduce", "band", "bulge", "tridiag", "occ", "back_q2", "back_q1",
          "backsub", "density", "refine"]


class ElsiGpuError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.elsi_gpu_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class Info(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double * NSTAGES), ("total_ms", ctypes.c_double),
                ("mu", ctypes.c_double), ("energy", ctypes.c_double),
                ("charge_residual", ctypes.c_double), ("k_s", ctypes.c_int),
                ("fail_col", ctypes.c_int), ("mu_steps", ctypes.c_int),
                ("band_width", ctypes.c_int), ("n_basis", ctypes.c_int),
                ("probe_launches", ctypes.c_int), ("probe_ms", ctypes.c_double),
                ("probe_flops", ctypes.c_double), ("probe_kernel", ctypes.c_char * 48),
                ("refine_sweeps", ctypes.c_int), ("refine_states", ctypes.c_int),
                ("refine_resid", ctypes.c_double), ("refine_step", ctypes.c_double),
                ("overlap_min_eig", ctypes.c_double), ("n_nonsing", ctypes.c_int),
                ("refine_hist", ctypes.c_double * 8)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "stage_ms"}
        d["probe_kernel"] = self.probe_kernel.decode()
        d["refine_hist"] = list(self.refine_hist)
        d["stage_ms"] = {s: self.stage_ms[i] for i, s in enumerate(STAGES)}
        return d


def _ptrs(tensors):
    """Host array of device pointers (double *const *)."""
    arr = (ctypes.c_void_p * len(tensors))()
    for q, t in enumerate(tensors):
        arr[q] = t.data_ptr()
    return arr


def lib():
    """Load libelsi_gpu.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1705_11191_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, c = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_char
        sz = ctypes.c_size_t
        L.elsi_gpu_strerror.restype = ctypes.c_char_p
        L.elsi_gpu_strerror.argtypes = [i]
        L.elsi_gpu_init.argtypes = [ctypes.POINTER(vp), i, i, i, d, vp]
        L.elsi_gpu_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
        L.elsi_gpu_set_workspace.argtypes = [vp, vp, sz]
        L.elsi_gpu_set_occupation.argtypes = [vp, i, d, d, i, d]
        L.elsi_gpu_set_overlap_is_unit.argtypes = [vp, i]
        L.elsi_gpu_set_singularity.argtypes = [vp, i, d]
        L.elsi_gpu_set_overlap_factored.argtypes = [vp, i]
        L.elsi_gpu_set_band_width.argtypes = [vp, i]
        L.elsi_gpu_set_launch_timing.argtypes = [vp, i]
        L.elsi_gpu_set_batch_workers.argtypes = [vp, i]
        L.elsi_gpu_set_batch_band_table.argtypes = [vp, i, vp, vp]
        L.elsi_gpu_set_precision.argtypes = [vp, i, d, i]
        pp, ip, dp = ctypes.POINTER(vp), ctypes.POINTER(i), ctypes.POINTER(d)
        L.elsi_gpu_ev_batched.argtypes = [vp, i, ip, ip, pp, pp, pp, pp, ip]
        L.elsi_gpu_dm_batched.argtypes = [vp, i, ip, dp, dp, pp, pp, pp, pp, dp, dp, ip]
        L.elsi_gpu_ev.argtypes = [vp, vp, vp, vp, vp]
        L.elsi_gpu_dm.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(d), ctypes.POINTER(d)]
        L.elsi_gpu_get_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.elsi_gpu_finalize.argtypes = [ctypes.POINTER(vp)]
        L.elsi_gpu_x_dgemm.argtypes = [c, c, i, i, i, d, vp, i, vp, i, d, vp, i, vp]
        L.elsi_gpu_x_gemm_fp32.argtypes = [c, c, i, i, i, d, vp, i, vp, i, d, vp, i, i, vp]
        L.elsi_gpu_x_cholesky.argtypes = [i, vp, i, ctypes.POINTER(i), vp]
        L.elsi_gpu_x_cholesky_noalloc.argtypes = [i, vp, i, ctypes.POINTER(i), vp]
        L.elsi_gpu_x_reduce.argtypes = [i, vp, i, vp, i, vp]
        L.elsi_gpu_x_backsub.argtypes = [i, i, vp, i, vp, i, vp]
        L.elsi_gpu_x_occupations.argtypes = [i, vp, vp, i, d, d, d, d, i, vp, ctypes.POINTER(d),
                                             ctypes.POINTER(i), vp]
        L.elsi_gpu_x_density.argtypes = [i, i, vp, i, vp, vp, i, vp]
        L.elsi_gpu_x_band_reduce.argtypes = [i, i, vp, i, vp, i, vp]
        L.elsi_gpu_x_tridiagonalize.argtypes = [i, i, vp, i, vp, vp, vp]
        L.elsi_gpu_x_tridiag_eig.argtypes = [i, vp, vp, vp, vp, i, vp]
        L.elsi_gpu_x_refine.argtypes = [i, i, i, vp, i, vp, i, vp, i, vp, vp, vp, vp, vp, vp, d, i,
                                        ctypes.POINTER(i), vp]
        L.elsi_gpu_x_backtransform.argtypes = [i, i, vp, i, vp, vp, vp, i, i, i, i, vp]
        L.elsi_gpu_x_set_bulge_path.argtypes = [i]
        _lib = L
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def fortran_empty(rows: int, cols: int, device="cuda", dtype=torch.float64) -> torch.Tensor:
    """Column-major (rows x cols) tensor: a transposed view of a (cols, rows) buffer."""
    return torch.empty((cols, rows), device=device, dtype=dtype).t()


def as_fortran(X: torch.Tensor) -> torch.Tensor:
    """Column-major version of X (no copy when it already is one)."""
    if X.dim() == 2 and X.stride(0) == 1 and (X.shape[1] <= 1 or X.stride(1) == X.shape[0]):
        return X
    Y = fortran_empty(X.shape[0], X.shape[1], device=X.device, dtype=X.dtype)
    Y.copy_(X)
    return Y


def _check(rc: int, where: str, ok=(0,)):
    if rc not in ok:
        raise ElsiGpuError(rc, where)
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


# ---------------------------------------------------------------------------
# stage entry points
# ---------------------------------------------------------------------------
def dgemm(ta: str, tb: str, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None,
          alpha: float = 1.0, beta: float = 0.0) -> torch.Tensor:
    """C = alpha op(A) op(B) + beta C on the matrix cores (column-major operands)."""
    A, B = as_fortran(A), as_fortran(B)
    m = A.shape[1] if ta == "T" else A.shape[0]
    k = A.shape[0] if ta == "T" else A.shape[1]
    n = B.shape[0] if tb == "T" else B.shape[1]
    if C is None:
        C = fortran_empty(m, n, device=A.device)
        beta = 0.0
    C2 = as_fortran(C)
    rc = lib().elsi_gpu_x_dgemm(ta.encode(), tb.encode(), m, n, k, alpha, _ptr(A), max(1, A.shape[0]),
                                _ptr(B), max(1, B.shape[0]), beta, _ptr(C2), max(1, m), _stream())
    _check(rc, "elsi_gpu_x_dgemm")
    if C2.data_ptr() != C.data_ptr():
        C.copy_(C2)
    return C


def gemm_fp32(ta: str, tb: str, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None,
              alpha: float = 1.0, beta: float = 0.0, uplo: int = 0) -> torch.Tensor:
    """As dgemm, with the operands rounded to FP32 and FP32 matrix-core arithmetic
    (the products of the mixed mode); uplo = 1 writes only the lower triangle."""
    A, B = as_fortran(A), as_fortran(B)
    m = A.shape[1] if ta == "T" else A.shape[0]
    k = A.shape[0] if ta == "T" else A.shape[1]
    n = B.shape[0] if tb == "T" else B.shape[1]
    if C is None:
        C = fortran_empty(m, n, device=A.device)
        C.zero_()
        beta = 0.0
    if not C.t().is_contiguous():
        raise ValueError("C must be column-major (see fortran_empty)")
    rc = lib().elsi_gpu_x_gemm_fp32(ta.encode(), tb.encode(), m, n, k, alpha, _ptr(A), max(1, A.shape[0]),
                                    _ptr(B), max(1, B.shape[0]), beta, _ptr(C), max(1, m), int(uplo), _stream())
    _check(rc, "elsi_gpu_x_gemm_fp32")
    return C


def cholesky(S: torch.Tensor) -> int:
    """S <- L in place (S symmetric, so either layout works); returns 0 or the failing pivot."""
    n = S.shape[0]
    fail = ctypes.c_int(0)
    rc = lib().elsi_gpu_x_cholesky(n, _ptr(S), n, ctypes.byref(fail), _stream())
    _check(rc, "elsi_gpu_x_cholesky", ok=(0, 1))
    return fail.value


NOALLOC_MAX_N = 16384   # ELSI_GPU_NOALLOC_MAX_N


def cholesky_noalloc(S: torch.Tensor) -> int:
    """As cholesky, through the entry point that allocates nothing (its scratch
    is a fixed device array; n <= NOALLOC_MAX_N)."""
    n = S.shape[0]
    fail = ctypes.c_int(0)
    rc = lib().elsi_gpu_x_cholesky_noalloc(n, _ptr(S), n, ctypes.byref(fail), _stream())
    _check(rc, "elsi_gpu_x_cholesky_noalloc", ok=(0, 1))
    return fail.value


def reduce_standard(H: torch.Tensor, L: torch.Tensor) -> None:
    """H <- L^-1 H L^-T in place (H symmetric; L column-major lower)."""
    n = H.shape[0]
    rc = lib().elsi_gpu_x_reduce(n, _ptr(H), n, _ptr(L), n, _stream())
    _check(rc, "elsi_gpu_x_reduce")


def backsub(L: torch.Tensor, X: torch.Tensor) -> None:
    """X <- L^-T X in place (X column-major n x k)."""
    n, k = X.shape
    rc = lib().elsi_gpu_x_backsub(n, k, _ptr(L), n, _ptr(X), n, _stream())
    _check(rc, "elsi_gpu_x_backsub")


def occupations(eps: torch.Tensor, n_electron: float, kT: float, spin: float = 1.0,
                occ_accuracy: float = 1e-13, max_steps: int = 100, scheme: int = None, weight=None):
    """Occupations of a broadening scheme (default Fermi-Dirac) and mu on the
    device; weight: per-state weights of a mu shared by several problems.
    Returns (f, mu, k_s, status)."""
    f = torch.empty_like(eps)
    mu = ctypes.c_double(0.0)
    ks = ctypes.c_int(0)
    scheme = OCC_FERMI if scheme is None else scheme
    rc = lib().elsi_gpu_x_occupations(eps.shape[0], _ptr(eps), _ptr(weight), int(scheme), n_electron, kT, spin,
                                      occ_accuracy, max_steps, _ptr(f), ctypes.byref(mu), ctypes.byref(ks),
                                      _stream())
    _check(rc, "elsi_gpu_x_occupations", ok=(0, 4))
    return f, mu.value, ks.value, rc


def density(C: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
    """D = sum_l f_l c_l c_l^T from column-major C (n x k)."""
    C = as_fortran(C)
    n, k = C.shape
    D = torch.empty((n, n), device=C.device, dtype=torch.float64)
    rc = lib().elsi_gpu_x_density(n, k, _ptr(C), n, _ptr(f), _ptr(D), n, _stream())
    _check(rc, "elsi_gpu_x_density")
    return D


def band_reduce(A: torch.Tensor, b: int) -> torch.Tensor:
    """Band form (LAPACK lower band storage, (b+1) x n column-major) of symmetric A."""
    n = A.shape[0]
    band = fortran_empty(b + 1, n, device=A.device)
    rc = lib().elsi_gpu_x_band_reduce(n, b, _ptr(A), n, _ptr(band), b + 1, _stream())
    _check(rc, "elsi_gpu_x_band_reduce")
    return band


def tridiagonalize(A: torch.Tensor, b: int):
    """(d, e) of the two-stage tridiagonal form of symmetric A."""
    n = A.shape[0]
    d = torch.empty(n, device=A.device, dtype=torch.float64)
    e = torch.empty(max(n - 1, 1), device=A.device, dtype=torch.float64)
    rc = lib().elsi_gpu_x_tridiagonalize(n, b, _ptr(A), n, _ptr(d), _ptr(e), _stream())
    _check(rc, "elsi_gpu_x_tridiagonalize")
    return d, e[: n - 1]


def set_bulge_path(path: int) -> None:
    """Schedule of the bulge chasing, process-wide: 0 automatic, 1 row window
    (when its grid fits the device), 2 pipelined sweeps."""
    _check(lib().elsi_gpu_x_set_bulge_path(int(path)), "elsi_gpu_x_set_bulge_path")


def tridiag_eig(d: torch.Tensor, e: torch.Tensor):
    """Eigenvalues (ascending) and eigenvectors (column-major) of tridiagonal (d, e)."""
    n = d.shape[0]
    w = torch.empty(n, device=d.device, dtype=torch.float64)
    Z = fortran_empty(n, n, device=d.device)
    ee = e if e.numel() > 0 else torch.zeros(1, device=d.device, dtype=torch.float64)
    rc = lib().elsi_gpu_x_tridiag_eig(n, _ptr(d), _ptr(ee), _ptr(w), _ptr(Z), n, _stream())
    _check(rc, "elsi_gpu_x_tridiag_eig")
    return w, Z


def backtransform(A: torch.Tensor, b: int, X: torch.Tensor, trans: bool = False, slab: int = 0):
    """X <- Q X (or Q^T X) in place, Q = Q1 Q2 the reflectors of the two-stage
    tridiagonalization of symmetric A; returns (d, e) of T = Q^T A Q."""
    n = A.shape[0]
    ncol = X.shape[1]
    if not X.t().is_contiguous():
        raise ValueError("X must be column-major (see fortran_empty)")
    d = torch.empty(n, device=A.device, dtype=torch.float64)
    e = torch.empty(max(n - 1, 1), device=A.device, dtype=torch.float64)
    rc = lib().elsi_gpu_x_backtransform(n, b, _ptr(A), n, _ptr(d), _ptr(e), _ptr(X), n, ncol, int(bool(trans)),
                                        int(slab), _stream())
    _check(rc, "elsi_gpu_x_backtransform")
    return d, e[: n - 1]


def refine(Ht: torch.Tensor, X: torch.Tensor, kw: int, tol: float = 1e-10, max_sweeps: int = 4, Q=None, d=None,
           e=None, weight=None):
    """FP64 refinement sweeps of the mixed path on the subspace X (n x k) of the
    symmetric Ht; X is overwritten by the refined vectors.  Q (column-major
    n x n), d, e: an approximate factorization Ht ~ Q T Q^T through which the
    Newton correction runs (None: one Rayleigh-Ritz sweep).  Returns
    (theta, resid, step, sweeps, status) with status 0 or 3 (tolerance not reached)."""
    n = Ht.shape[0]
    k = X.shape[1]
    Ht = as_fortran(Ht)
    if not X.t().is_contiguous():
        raise ValueError("X must be column-major (see fortran_empty)")
    theta = torch.zeros(max(k, 1), device=Ht.device, dtype=torch.float64)
    resid = torch.zeros(max(k, 1), device=Ht.device, dtype=torch.float64)
    step = torch.zeros(max(k, 1), device=Ht.device, dtype=torch.float64)
    sw = ctypes.c_int(0)
    if Q is not None:
        Q = as_fortran(Q)
        ee = e if e.numel() > 0 else torch.zeros(1, device=Ht.device, dtype=torch.float64)
        qargs = (_ptr(Q), max(1, n), _ptr(d), _ptr(ee))
    else:
        qargs = (_ptr(None), max(1, n), _ptr(None), _ptr(None))
    rc = lib().elsi_gpu_x_refine(n, k, kw, _ptr(Ht), max(1, n), _ptr(X), max(1, n), *qargs, _ptr(weight),
                                 _ptr(theta), _ptr(resid), _ptr(step), float(tol), int(max_sweeps),
                                 ctypes.byref(sw), _stream())
    _check(rc, "elsi_gpu_x_refine", ok=(0, 3))
    return theta[:k], resid[:k], step[:k], sw.value, rc


# ---------------------------------------------------------------------------
# handle API
# ---------------------------------------------------------------------------
_live_handles: "weakref.WeakSet[Handle]" = weakref.WeakSet()


def _close_live_handles():
    """Finalize every handle still open at interpreter exit, while the HIP
    runtime is certainly alive (registered after torch is imported, so it
    runs before torch's own exit handlers)."""
    for h in list(_live_handles):
        try:
            h.close()
        except Exception:
            pass


atexit.register(_close_live_handles)


class Handle:
    """One elsi_gpu handle (elsi_init ... elsi_finalize)."""

    def __init__(self, n_basis: int, n_state: int, n_electron: float, stream=None, dtype=REAL64):
        """dtype REAL64 (float64 matrices) or COMPLEX128 (complex128 matrices, which
        must be column-major: a transposed view of a contiguous tensor, see
        fortran_empty / as_fortran)."""
        self._h = ctypes.c_void_p(0)
        s = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
        self.n = n_basis
        self.n_state = n_state
        self.dtype = dtype
        _check(lib().elsi_gpu_init(ctypes.byref(self._h), dtype, n_basis, n_state, n_electron,
                                   ctypes.c_void_p(s)), "elsi_gpu_init")
        _live_handles.add(self)

    def _mat_dtype(self):
        return torch.complex128 if self.dtype == COMPLEX128 else torch.float64

    def _check_input(self, *mats):
        """Complex matrices must be complex128 and column-major (a real symmetric
        matrix reads the same either way; a Hermitian one would read as its
        conjugate)."""
        if self.dtype != COMPLEX128:
            return
        for M in mats:
            if M is None:
                continue
            if M.dtype != torch.complex128 or not M.t().is_contiguous():
                raise ValueError("complex handle: matrices must be column-major complex128 tensors")

    def set_occupation(self, scheme=OCC_FERMI, width=0.01, occ_accuracy=1e-13, mu_max_steps=100,
                       spin_factor=1.0):
        _check(lib().elsi_gpu_set_occupation(self._h, scheme, width, occ_accuracy, mu_max_steps,
                                             spin_factor), "elsi_gpu_set_occupation")

    def set_singularity(self, check=True, tolerance=1e-5):
        """Singularity check of S (Eq. (20)): below `tolerance` the eigendecomposition
        transform replaces the Cholesky factorization (real handles)."""
        _check(lib().elsi_gpu_set_singularity(self._h, int(bool(check)), float(tolerance)), "set_singularity")

    def set_overlap_is_unit(self, flag=True):
        _check(lib().elsi_gpu_set_overlap_is_unit(self._h, int(flag)), "set_overlap_is_unit")

    def set_overlap_factored(self, flag=True):
        _check(lib().elsi_gpu_set_overlap_factored(self._h, int(flag)), "set_overlap_factored")

    def set_band_width(self, b: int):
        _check(lib().elsi_gpu_set_band_width(self._h, b), "set_band_width")

    def set_precision(self, prec=PREC_FP64, refine_tol=1e-10, max_refine=6):
        """PREC_FP64, or PREC_MIXED: FP32 matrix-core products in full -> band and Q1,
        then FP64 refinement (real handles)."""
        _check(lib().elsi_gpu_set_precision(self._h, int(prec), float(refine_tol), int(max_refine)),
               "elsi_gpu_set_precision")

    def set_launch_timing(self, on: bool):
        """Per-launch HIP-event timing of the GEMM kernels (measurement aid)."""
        _check(lib().elsi_gpu_set_launch_timing(self._h, int(bool(on))), "set_launch_timing")

    def workspace_size(self) -> int:
        v = ctypes.c_size_t(0)
        _check(lib().elsi_gpu_workspace_size(self._h, ctypes.byref(v)), "workspace_size")
        return v.value

    def set_workspace(self, buf: torch.Tensor):
        self._ws = buf
        _check(lib().elsi_gpu_set_workspace(self._h, _ptr(buf), buf.numel() * buf.element_size()),
               "set_workspace")

    def ev(self, H: torch.Tensor, S: torch.Tensor, eval_out=None, evec_out=None, ok=(0,)):
        """Eigenpairs; H is destroyed and S receives L.  Returns (eval, evec column-major);
        the return code is kept in self.last_status (codes in `ok` do not raise)."""
        n = self.n
        self._check_input(H, S)
        ev = eval_out if eval_out is not None else torch.empty(n, device=H.device, dtype=torch.float64)
        C = evec_out if evec_out is not None else fortran_empty(n, self.n_state, device=H.device,
                                                                dtype=self._mat_dtype())
        rc = lib().elsi_gpu_ev(self._h, _ptr(H), _ptr(S), _ptr(ev), _ptr(C))
        self.last_status = rc
        _check(rc, "elsi_gpu_ev", ok=ok)
        return ev, C

    def dm(self, H: torch.Tensor, S: torch.Tensor, occ=None, D_out=None, eval_out=None,
           ok=(0,)):
        """Density matrix; returns (D, eval, occ, energy, mu, status)."""
        n = self.n
        self._check_input(H, S)
        D = D_out if D_out is not None else fortran_empty(n, n, device=H.device, dtype=self._mat_dtype())
        ev = eval_out if eval_out is not None else torch.empty(n, device=H.device, dtype=torch.float64)
        f = occ if occ is not None else torch.empty(n, device=H.device, dtype=torch.float64)
        energy = ctypes.c_double(0.0)
        mu = ctypes.c_double(0.0)
        rc = lib().elsi_gpu_dm(self._h, _ptr(H), _ptr(S), _ptr(f), _ptr(D), _ptr(ev),
                               ctypes.byref(energy), ctypes.byref(mu))
        _check(rc, "elsi_gpu_dm", ok=ok)
        return D, ev, f, energy.value, mu.value, rc

    def set_batch_workers(self, workers: int):
        _check(lib().elsi_gpu_set_batch_workers(self._h, workers), "set_batch_workers")

    def set_batch_band_table(self, n_max, b):
        """Band widths of the batched calls per size bucket: a problem of size n
        takes b[i] of the first i with n <= n_max[i] (empty lists clear the table)."""
        n_max, b = [int(x) for x in n_max], [int(x) for x in b]
        if len(n_max) != len(b):
            raise ValueError("n_max and b differ in length")
        cnt = len(n_max)
        arr_n = (ctypes.c_int * max(cnt, 1))(*n_max)
        arr_b = (ctypes.c_int * max(cnt, 1))(*b)
        _check(lib().elsi_gpu_set_batch_band_table(self._h, cnt, arr_n if cnt else None, arr_b if cnt else None),
               "set_batch_band_table")

    def ev_batched(self, Hs, Ss, n_states, ok=(0,)):
        """Batched eigenpairs: returns (evals, evecs column-major, per-problem status, rc)."""
        count = len(Hs)
        n = [int(H.shape[0]) for H in Hs]
        evals = [torch.empty(m, device=Hs[0].device, dtype=torch.float64) for m in n]
        self._check_input(*Hs, *(Ss or []))
        evecs = [fortran_empty(m, int(k), device=Hs[0].device, dtype=self._mat_dtype()) for m, k in zip(n, n_states)]
        status = (ctypes.c_int * count)()
        rc = lib().elsi_gpu_ev_batched(
            self._h, count, (ctypes.c_int * count)(*n), (ctypes.c_int * count)(*[int(k) for k in n_states]),
            _ptrs(Hs), _ptrs(Ss) if Ss is not None else None, _ptrs(evals), _ptrs(evecs), status)
        _check(rc, "elsi_gpu_ev_batched", ok=ok)
        return evals, evecs, list(status), rc

    def dm_batched(self, Hs, Ss, n_electrons, kweight=None, ok=(0,)):
        """Batched density matrices: an independent mu per problem, or with
        kweight one mu shared by all problems (k-points / spin channels, each
        problem's occupations weighted).  Returns (Ds, evals, energies, mus,
        per-problem status, rc)."""
        count = len(Hs)
        n = [int(H.shape[0]) for H in Hs]
        self._check_input(*Hs, *(Ss or []))
        Ds = [fortran_empty(m, m, device=Hs[0].device, dtype=self._mat_dtype()) for m in n]
        evals = [torch.empty(m, device=Hs[0].device, dtype=torch.float64) for m in n]
        energy = (ctypes.c_double * count)()
        mu = (ctypes.c_double * count)()
        status = (ctypes.c_int * count)()
        rc = lib().elsi_gpu_dm_batched(
            self._h, count, (ctypes.c_int * count)(*n), (ctypes.c_double * count)(*[float(x) for x in n_electrons]),
            (ctypes.c_double * count)(*[float(x) for x in kweight]) if kweight is not None else None,
            _ptrs(Hs), _ptrs(Ss) if Ss is not None else None, _ptrs(Ds), _ptrs(evals), energy, mu, status)
        _check(rc, "elsi_gpu_dm_batched", ok=ok)
        return Ds, evals, list(energy), list(mu), list(status), rc

    def info(self) -> dict:
        inf = Info()
        _check(lib().elsi_gpu_get_info(self._h, ctypes.byref(inf)), "get_info")
        return inf.as_dict()

    def close(self):
        if self._h:
            lib().elsi_gpu_finalize(ctypes.byref(self._h))
            self._h = ctypes.c_void_p(0)
        _live_handles.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter shutdown the atexit hook has already closed every
        # live handle; no HIP call is made from a finalizer at that point
        # (the check is bound at definition: module globals may be gone then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
