"""ctypes wrapper of the plain-C FP64 oracle (test infrastructure only).

Every function copies its inputs into Fortran-ordered float64 arrays, calls the
C routine and returns fresh NumPy arrays; nothing here does any arithmetic of
the method itself.  The sections and equations each routine follows are cited
in ``elsi_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "elsi_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i, d = ctypes.c_int, ctypes.c_double
        lib.orc_potrf.argtypes = [i, _dp, i]
        lib.orc_reduce.argtypes = [i, _dp, i, _dp, i]
        lib.orc_tred.argtypes = [i, _dp, i, _dp, _dp, _dp, i]
        lib.orc_tql.argtypes = [i, _dp, _dp, _dp, i]
        lib.orc_backsub.argtypes = [i, i, _dp, i, _dp, i]
        lib.orc_gevp.argtypes = [i, i, _dp, i, _dp, i, _dp, _dp, _ip]
        lib.orc_tridiag_eigvals.argtypes = [i, _dp, _dp, _dp]
        lib.orc_tridiag_eig.argtypes = [i, _dp, _dp, _dp, _dp]
        lib.orc_occupations.argtypes = [i, _dp, d, d, d, d, i, _dp, _dp]
        lib.orc_density.argtypes = [i, i, _dp, i, _dp, _dp, i]
        lib.orc_band_energy.argtypes = [i, _dp, _dp]
        lib.orc_band_energy.restype = d
        lib.orc_dm.argtypes = [i, _dp, i, _dp, i, d, d, d, d, i, _dp, i, _dp, _dp, _dp, _dp, _ip]
        lib.orc_dm_scheme.argtypes = [i, _dp, i, _dp, i, i, d, d, d, d, i, _dp, i, _dp, _dp, _dp, _dp, _ip]
        lib.orc_gevp_checked.argtypes = [i, i, _dp, i, _dp, i, d, _dp, _dp, _ip, _ip]
        lib.orc_dm_checked.argtypes = [i, _dp, i, _dp, i, d, i, d, d, d, d, i, _dp, i, _dp, _dp, _dp, _dp, _ip,
                                       _ip]
        lib.orc_occupations_scheme.argtypes = [i, _dp, _dp, i, d, d, d, d, i, _dp, _dp]
        lib.orc_occupation_value.argtypes = [i, d, d, d, d]
        lib.orc_occupation_value.restype = d
        lib.orc_residual_norms.argtypes = [i, i, _dp, i, _dp, i, _dp, i, _dp, _dp]
        lib.orc_refine.argtypes = [i, i, i, _dp, i, _dp, i, _dp, i, _dp, _dp, _dp, _dp, _dp, _dp, d, i, _ip]
        lib.orc_tridiag_shift_solve.argtypes = [i, _dp, _dp, d, _dp, _dp]
        lib.orc_zpotrf.argtypes = [i, _dp, i]
        lib.orc_zreduce.argtypes = [i, _dp, i, _dp, i]
        lib.orc_ztred.argtypes = [i, _dp, i, _dp, _dp, _dp, i]
        lib.orc_zgevp.argtypes = [i, i, _dp, i, _dp, i, _dp, _dp, _ip]
        lib.orc_zdensity.argtypes = [i, i, _dp, i, _dp, _dp, i]
        lib.orc_zdm.argtypes = [i, _dp, i, _dp, i, d, d, d, d, i, _dp, i, _dp, _dp, _dp, _dp, _ip]
        _lib = lib
    return _lib


def _c128(a) -> np.ndarray:
    return np.array(a, dtype=np.complex128, order="F", copy=True)


def _f64(a) -> np.ndarray:
    return np.array(a, dtype=np.float64, order="F", copy=True)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class OracleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"oracle status {status}: {msg}")
        self.status = status


def potrf(S):
    """Lower Cholesky factor L with S = L L^T (Eq. (10)); raises on a non-positive pivot."""
    A = _f64(S)
    n = A.shape[0]
    info = _load().orc_potrf(n, _p(A), n)
    if info:
        raise OracleError(1, f"S not positive definite at column {info - 1}")
    return A


def reduce_standard(H, L):
    """H~ = L^-1 H L^-T (Eq. (11)), full symmetric."""
    A = _f64(H)
    Lf = _f64(L)
    n = A.shape[0]
    _load().orc_reduce(n, _p(A), n, _p(Lf), n)
    return A


def tred(A):
    """Householder tridiagonalization (Eq. (12)): returns d, e, Q with A = Q T Q^T."""
    W = _f64(A)
    n = W.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1))
    Q = np.zeros((n, n), order="F")
    _load().orc_tred(n, _p(W), n, _p(d), _p(e), _p(Q), n)
    return d, e[: max(n - 1, 0)], Q


def tridiag_eigvals(d, e):
    """Eigenvalues (ascending) of the symmetric tridiagonal (d, e) by implicit QL."""
    d = _f64(d)
    n = d.shape[0]
    ee = np.zeros(max(n, 1))
    ee[: n - 1] = e
    w = np.zeros(n)
    st = _load().orc_tridiag_eigvals(n, _p(d), _p(ee), _p(w))
    if st:
        raise OracleError(st, "QL did not converge")
    return w


def tridiag_eig(d, e):
    """Eigenpairs of the symmetric tridiagonal (d, e): (w ascending, Z column-major)."""
    d = _f64(d)
    n = d.shape[0]
    ee = np.zeros(max(n, 1))
    ee[: n - 1] = e
    w = np.zeros(n)
    Z = np.zeros((n, n), order="F")
    st = _load().orc_tridiag_eig(n, _p(d), _p(ee), _p(w), _p(Z))
    if st:
        raise OracleError(st, "QL did not converge")
    return w, Z


def backsub(L, Z):
    """C = L^-T Z."""
    Lf = _f64(L)
    C = _f64(Z)
    n, k = C.shape
    _load().orc_backsub(n, k, _p(Lf), n, _p(C), n)
    return C


def gevp(H, S, n_state=None):
    """Generalized eigenpairs of Eq. (6): (eval ascending (n), evec n x n_state, L)."""
    Hf = _f64(H)
    Sf = _f64(S)
    n = Hf.shape[0]
    k = n if n_state is None else int(n_state)
    ev = np.zeros(n)
    C = np.zeros((n, max(k, 1)), order="F")
    fail = ctypes.c_int(0)
    st = _load().orc_gevp(n, k, _p(Hf), n, _p(Sf), n, _p(ev), _p(C), ctypes.byref(fail))
    if st == 1:
        raise OracleError(1, f"S not positive definite at column {fail.value - 1}")
    if st:
        raise OracleError(st, "eigensolver failed")
    return ev, C[:, :k], Sf


FERMI, GAUSSIAN, MP0, MP1 = 1, 2, 3, 4   # broadening schemes (Sec. 4.6 broadening_scheme)


def occupations(eps, n_electron, kT, spin=1.0, occ_accuracy=1e-13, max_steps=100, scheme=FERMI, weight=None):
    """Occupations of a broadening scheme (Fermi-Dirac Eq. (17), Gaussian Eq. (21),
    Methfessel-Paxton orders 0 and 1) with mu from Eq. (18); weight: per-state
    weights (k-points / spin channels sharing one mu), f_l = w_l f(eps_l).
    Returns (f, mu, status)."""
    e = _f64(eps)
    n = e.shape[0]
    f = np.zeros(n)
    mu = ctypes.c_double(0.0)
    w = _f64(weight) if weight is not None else None
    st = _load().orc_occupations_scheme(n, _p(e), _p(w) if w is not None else ctypes.POINTER(ctypes.c_double)(),
                                        int(scheme), float(n_electron), float(kT), float(spin),
                                        float(occ_accuracy), int(max_steps), _p(f), ctypes.byref(mu))
    return f, mu.value, st


def occupation_value(scheme, eps, mu, width, spin=1.0):
    """The occupation of one state at eps for chemical potential mu."""
    return float(_load().orc_occupation_value(int(scheme), float(eps), float(mu), float(width), float(spin)))


def density(C, f):
    """D = sum_l f_l c_l c_l^T over f_l > 0 (Eq. (9))."""
    Cf = _f64(C)
    ff = _f64(f)
    n, k = Cf.shape
    D = np.zeros((n, n), order="F")
    _load().orc_density(n, k, _p(Cf), n, _p(ff), _p(D), n)
    return D


def band_energy(f, eps):
    ff = _f64(f)
    e = _f64(eps)
    return float(_load().orc_band_energy(ff.shape[0], _p(ff), _p(e)))


def dm(H, S, n_electron, kT, spin=1.0, occ_accuracy=1e-13, max_steps=100, scheme=FERMI):
    """Density-matrix driver: returns dict(D, eval, occ, energy, mu, status)."""
    Hf = _f64(H)
    Sf = _f64(S)
    n = Hf.shape[0]
    D = np.zeros((n, n), order="F")
    ev = np.zeros(n)
    occ = np.zeros(n)
    energy = ctypes.c_double(0.0)
    mu = ctypes.c_double(0.0)
    fail = ctypes.c_int(0)
    st = _load().orc_dm_scheme(n, _p(Hf), n, _p(Sf), n, int(scheme), float(n_electron), float(kT), float(spin),
                               float(occ_accuracy), int(max_steps), _p(D), n, _p(ev), _p(occ),
                               ctypes.byref(energy), ctypes.byref(mu), ctypes.byref(fail))
    if st in (1, 2):
        raise OracleError(st, "eigensolve failed")
    return dict(D=D, eval=ev, occ=occ, energy=energy.value, mu=mu.value, status=st, L=Sf)


def residual_norms(H, S, X, lam):
    """||H x_j - lam_j S x_j||_2 per column, accumulated in long double."""
    Hf = _f64(H)
    Sf = _f64(S)
    Xf = _f64(X)
    lf = _f64(lam)
    n, k = Xf.shape
    res = np.zeros(k)
    _load().orc_residual_norms(n, k, _p(Hf), n, _p(Sf), n, _p(Xf), n, _p(lf), _p(res))
    return res


# ---------------------------------------------------------------------------
# complex Hermitian path (complex128 arrays; the C side reads them as
# interleaved real/imaginary doubles)
# ---------------------------------------------------------------------------
def refine(Ht, X, kw, tol=1e-10, max_sweeps=4, Q=None, d=None, e=None, weight=None):
    """FP64 refinement sweeps of the subspace X (n x k) of the symmetric Ht:
    CholeskyQR twice, Rayleigh-Ritz, residuals and, given an approximate
    factorization Ht ~ Q T Q^T (Q orthogonal n x n, T = tridiag(e, d, e)),
    the Newton correction through it.  Returns
    (X_refined, theta, res, step, sweeps, status) with status 0 or 3."""
    A = _f64(Ht)
    Xr = _f64(X).copy(order="F")
    n, k = Xr.shape
    theta = np.zeros(max(k, 1))
    res = np.zeros(max(k, 1))
    step = np.zeros(max(k, 1))
    sw = ctypes.c_int(0)
    null = ctypes.POINTER(ctypes.c_double)()
    if Q is not None:
        Qf, df, ef = _f64(Q), _f64(d), _f64(np.append(np.asarray(e, dtype=float), 0.0))
        qargs = (_p(Qf), n, _p(df), _p(ef))
    else:
        qargs = (null, 1, null, null)
    wf = _f64(weight) if weight is not None else None
    st = _load().orc_refine(n, k, int(kw), _p(A), n, _p(Xr), n, *qargs, _p(wf) if wf is not None else null,
                            _p(theta), _p(res), _p(step), float(tol), int(max_sweeps), ctypes.byref(sw))
    return Xr, theta[:k], res[:k], step[:k], sw.value, st


def tridiag_shift_solve(d, e, shift, b):
    """x with (T - shift I) x = b, T = tridiag(e, d, e), by Gaussian elimination
    with partial pivoting."""
    df = _f64(d)
    ef = _f64(np.append(np.asarray(e, dtype=float), 0.0))
    bf = _f64(b)
    x = np.zeros_like(bf)
    _load().orc_tridiag_shift_solve(len(df), _p(df), _p(ef), float(shift), _p(bf), _p(x))
    return x


def zpotrf(S):
    """Complex Cholesky S = L L^H (lower), strict upper triangle zeroed."""
    A = _c128(S)
    st = _load().orc_zpotrf(A.shape[0], _p(A), A.shape[0])
    if st:
        raise OracleError(1, f"S not positive definite at column {st - 1}")
    return A


def zreduce_standard(H, L):
    """H~ = L^-1 H L^-H (Eq. (11)) for Hermitian H, full Hermitian result."""
    Hf = _c128(H)
    Lf = _c128(L)
    n = Hf.shape[0]
    _load().orc_zreduce(n, _p(Hf), n, _p(Lf), n)
    return Hf


def ztred(A):
    """Hermitian Householder tridiagonalization made real: (d, e, Q) with
    A = Q T_r Q^H, T_r real symmetric tridiagonal (d, e)."""
    Af = _c128(A)
    n = Af.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1))
    Q = np.zeros((n, n), dtype=np.complex128, order="F")
    _load().orc_ztred(n, _p(Af), n, _p(d), _p(e), _p(Q), n)
    return d, e[: max(n - 1, 0)], Q


def zgevp(H, S, n_state=None):
    """Complex generalized eigenpairs: (eval ascending (n), evec n x n_state, L)."""
    Hf = _c128(H)
    Sf = _c128(S)
    n = Hf.shape[0]
    k = n if n_state is None else int(n_state)
    ev = np.zeros(n)
    C = np.zeros((n, max(k, 1)), dtype=np.complex128, order="F")
    fail = ctypes.c_int(0)
    st = _load().orc_zgevp(n, k, _p(Hf), n, _p(Sf), n, _p(ev), _p(C), ctypes.byref(fail))
    if st == 1:
        raise OracleError(1, f"S not positive definite at column {fail.value - 1}")
    if st:
        raise OracleError(st, "eigensolver failed")
    return ev, C[:, :k], Sf


def zdensity(C, f):
    """D = sum_l f_l c_l c_l^H over f_l > 0 (Eq. (9), complex)."""
    Cf = _c128(C)
    ff = _f64(f)
    n, k = Cf.shape
    D = np.zeros((n, n), dtype=np.complex128, order="F")
    _load().orc_zdensity(n, k, _p(Cf), n, _p(ff), _p(D), n)
    return D


def zdm(H, S, n_electron, kT, spin=1.0, occ_accuracy=1e-13, max_steps=100):
    """Complex density-matrix driver: returns dict(D, eval, occ, energy, mu, status, L)."""
    Hf = _c128(H)
    Sf = _c128(S)
    n = Hf.shape[0]
    D = np.zeros((n, n), dtype=np.complex128, order="F")
    ev = np.zeros(n)
    occ = np.zeros(n)
    energy = ctypes.c_double(0.0)
    mu = ctypes.c_double(0.0)
    fail = ctypes.c_int(0)
    st = _load().orc_zdm(n, _p(Hf), n, _p(Sf), n, float(n_electron), float(kT), float(spin),
                         float(occ_accuracy), int(max_steps), _p(D), n, _p(ev), _p(occ),
                         ctypes.byref(energy), ctypes.byref(mu), ctypes.byref(fail))
    if st in (1, 2):
        raise OracleError(st, "eigensolve failed")
    return dict(D=D, eval=ev, occ=occ, energy=energy.value, mu=mu.value, status=st, L=Sf)


def dm_shared_mu(Hs, Ss, n_electrons, weights, kT, spin=1.0, occ_accuracy=1e-13, max_steps=100, scheme=FERMI):
    """Density matrices of several problems (k-points / spin channels of one
    system) with one chemical potential (Sec. 4.5, the electron count summed
    over k-points and spin channels): every problem's eigenpairs, then mu over
    all states with each state weighted by its problem's weight and
    N_e = sum_p w_p n_electron_p, then D_p = sum_l f_pl c_pl c_pl^H with the
    weighted occupations f_pl.  Complex (complex128) inputs take the complex
    path.  Returns a list of dict(D, eval, occ, energy) and mu."""
    evs, Cs = [], []
    for H, S in zip(Hs, Ss):
        if np.iscomplexobj(H) or np.iscomplexobj(S):
            ev, C, _ = zgevp(H, S)
        else:
            ev, C, _ = gevp(H, S)
        evs.append(ev)
        Cs.append(C)
    w = np.concatenate([np.full(len(ev), float(wp)) for ev, wp in zip(evs, weights)])
    ne = float(sum(float(wp) * float(n) for wp, n in zip(weights, n_electrons)))
    f, mu, st = occupations(np.concatenate(evs), ne, kT, spin=spin, occ_accuracy=occ_accuracy,
                            max_steps=max_steps, scheme=scheme, weight=w)
    out, o = [], 0
    for ev, C in zip(evs, Cs):
        fp = f[o:o + len(ev)]
        o += len(ev)
        D = zdensity(C, fp) if np.iscomplexobj(C) else density(C, fp)
        out.append(dict(D=D, eval=ev, occ=fp, energy=band_energy(fp, ev)))
    return out, mu, st


def gevp_checked(H, S, tau, n_state=None):
    """Eigenpairs with the singularity check of the overlap (Eq. (20)): the
    Cholesky route when every eigenvalue of S is >= tau, else the
    eigendecomposition transform keeping the n_nonsing eigenvectors of S with
    eigenvalues >= tau.  Returns (eval (n; +inf beyond n_nonsing), evec
    (n x n_state), S_out (L or X), n_nonsing)."""
    Hf, Sf = _f64(H), _f64(S)
    n = Hf.shape[0]
    k = n if n_state is None else int(n_state)
    ev = np.zeros(n)
    C = np.zeros((n, k), order="F")
    m = ctypes.c_int(0)
    fail = ctypes.c_int(0)
    st = _load().orc_gevp_checked(n, k, _p(Hf), n, _p(Sf), n, float(tau), _p(ev), _p(C), ctypes.byref(m),
                                  ctypes.byref(fail))
    if st:
        raise OracleError(st, "eigensolve failed")
    return ev, C, Sf, m.value


def dm_checked(H, S, n_electron, kT, tau, spin=1.0, occ_accuracy=1e-13, max_steps=100, scheme=FERMI):
    """dm with the singularity check (Eq. (20)): returns dict(D, eval, occ,
    energy, mu, status, S_out, n_nonsing)."""
    Hf, Sf = _f64(H), _f64(S)
    n = Hf.shape[0]
    D = np.zeros((n, n), order="F")
    ev = np.zeros(n)
    occ = np.zeros(n)
    energy = ctypes.c_double(0.0)
    mu = ctypes.c_double(0.0)
    m = ctypes.c_int(0)
    fail = ctypes.c_int(0)
    st = _load().orc_dm_checked(n, _p(Hf), n, _p(Sf), n, float(tau), int(scheme), float(n_electron), float(kT),
                                float(spin), float(occ_accuracy), int(max_steps), _p(D), n, _p(ev), _p(occ),
                                ctypes.byref(energy), ctypes.byref(mu), ctypes.byref(m), ctypes.byref(fail))
    if st in (1, 2):
        raise OracleError(st, "eigensolve failed")
    return dict(D=D, eval=ev, occ=occ, energy=energy.value, mu=mu.value, status=st, S_out=Sf, n_nonsing=m.value)
