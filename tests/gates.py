"""Parity gates shared by the GPU tests.

Eigenvalues: 1e-10 Ha for every state with |eps| <= 1 Ha, and 1e-10 relative for
every state that enters the density matrix (when the test passes the
occupations).  The other states with |eps| > 1 Ha are the large eigenvalues
created by the near-singular directions of S; for an eigenvalue of the definite
pencil, a relative backward error eps_mach of S's factorization moves lambda by
up to eps_mach * cond(S) * |lambda|, so every FP64 solver (the oracle included)
carries that much noise there.  Their gate is 1e-10 relative plus
2 eps_mach cond(S).
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(np.float64).eps


def overlap_condition(S) -> float:
    S = np.asarray(S)
    S = S.astype(np.complex128) if np.iscomplexobj(S) else S.astype(np.float64)
    w = np.linalg.eigvalsh(S)
    return float(w[-1] / w[0])


def eig_excess(ev, ref, S, tol: float = 1e-10, occ=None) -> float:
    """max over states of |ev - ref| / allowed; <= 1 passes.

    occ (optional, the reference occupations of the states compared): a state
    with |f| > 1e-20 enters the density matrix and keeps the plain gate
    tol * max(1, |eps|) whatever its size; the conditioning term applies only
    to the others.  (On the small lattice pencils mu lies among the large
    eigenvalues, so occupied states above 1 Ha exist; an independent FP64
    solver, LAPACK, stays within a few percent of the plain gate there.)"""
    ev = np.asarray(ev, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    big = np.abs(ref) > 1.0
    if occ is not None:
        big = big & (np.abs(np.asarray(occ, dtype=np.float64)) <= 1e-20)
    allowed = tol * np.maximum(1.0, np.abs(ref))
    if np.any(big):
        allowed = allowed + np.where(big, 2.0 * EPS * overlap_condition(S) * np.abs(ref), 0.0)
    return float(np.max(np.abs(ev - ref) / allowed))
