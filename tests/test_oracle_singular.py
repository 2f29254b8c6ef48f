"""Pins of the oracle's singularity check and eigendecomposition transform of
the overlap (Sec. 4.5, Eq. (20); Sec. 4.6 singularity_tolerance).

Closed form: duplicating basis functions makes S exactly singular without
changing the physics.  With E (n x n0) the map that copies function idx(a)
into slot a, the duplicated pencil is (E^T-free) H = E H0 E^T, S = E S0 E^T,
its null space is ker E^T, and the transform keeps range(E).  So:
* n_nonsing = n0, and the kept eigenvalues are those of (H0, S0);
* every eigenvector is the minimum-norm coefficient vector of the same
  state, c = E (E^T E)^-1 c0 (a duplicated function's coefficient is split
  evenly between its copies), hence D = M D0 M^T with M = E (E^T E)^-1;
* X X^T = S for the returned X (the dropped eigenvalues are zero).
And with tau below the smallest eigenvalue of S the route is the Cholesky one,
bit for bit.
"""
import numpy as np
import pytest

import oracle as O
from synth import generator as G


def _duplicate(sp, dup):
    n0 = sp.H.shape[0]
    idx = list(range(n0)) + list(dup)
    n = len(idx)
    E = np.zeros((n, n0))
    E[np.arange(n), idx] = 1.0
    return E @ sp.H @ E.T, E @ sp.S @ E.T, E


@pytest.mark.parametrize("dup", [(7,), (3, 40), (5, 5)])
def test_duplicated_basis_functions_closed_form(dup):
    sp = G.make_lattice_system(60, seed=61, kappa=1e3)
    H, S, E = _duplicate(sp, dup)
    n0, n = sp.H.shape[0], H.shape[0]
    ev0, C0, _ = O.gevp(sp.H, sp.S)
    ev, C, X, m = O.gevp_checked(H, S, 1e-10)
    assert m == n0
    assert np.all(np.isinf(ev[n0:])) and np.all(np.abs(C[:, n0:]) == 0.0)
    assert np.abs(ev[:n0] - ev0).max() <= 1e-11 * max(1.0, np.abs(ev0).max())
    M = E @ np.diag(1.0 / np.diag(E.T @ E))
    Cm = M @ C0
    # the same states up to sign, in the minimum-norm coefficients
    dots = np.abs(np.sum((C[:, :n0].T @ S) * Cm.T, axis=1))
    assert np.abs(dots - 1.0).max() <= 1e-9
    assert np.abs(C[:, :n0].T @ S @ C[:, :n0] - np.eye(n0)).max() <= 1e-10
    assert np.abs(X @ X.T - S).max() <= 1e-12 * np.abs(S).max() * n


def test_duplicated_basis_density_matrix():
    sp = G.make_lattice_system(60, seed=62, kappa=1e3)
    H, S, E = _duplicate(sp, (11, 30))
    ref0 = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    r = O.dm_checked(H, S, sp.n_occ, sp.kT, 1e-10)
    M = E @ np.diag(1.0 / np.diag(E.T @ E))
    assert r["n_nonsing"] == 60
    assert np.abs(r["D"] - M @ ref0["D"] @ M.T).max() <= 1e-10
    assert abs(r["mu"] - ref0["mu"]) <= 1e-10 and abs(r["energy"] - ref0["energy"]) <= 1e-10
    assert abs(np.trace(r["D"] @ S) - sp.n_occ) <= 1e-10
    assert np.all(r["occ"][60:] == 0.0)


def test_well_conditioned_overlap_takes_the_cholesky_route():
    sp = G.make_lattice_system(80, seed=63)
    lam_min = np.linalg.eigvalsh(sp.S)[0]
    ev, C, L, m = O.gevp_checked(sp.H, sp.S, 0.5 * lam_min)
    ev0, C0, L0 = O.gevp(sp.H, sp.S)
    assert m == 80
    assert np.array_equal(ev, ev0) and np.array_equal(C, C0) and np.array_equal(L, L0)


def test_tolerance_drops_the_small_eigenvalues():
    """A tau in the first clear gap above the 3rd eigenvalue of S keeps the
    directions above it:
    the kept states are S-orthonormal and lie in the span of the kept
    eigenvectors of S, and their values are the Rayleigh-Ritz values of the
    pencil there, which bound the exact ones from above."""
    sp = G.make_lattice_system(70, seed=64, kappa=1e6)
    lam = np.linalg.eigvalsh(sp.S)
    j = next(j for j in range(2, 69) if lam[j + 1] - lam[j] > 1e-3 * lam[j + 1])
    tau = 0.5 * (lam[j] + lam[j + 1])
    ev, C, X, m = O.gevp_checked(sp.H, sp.S, tau)
    assert m == 70 - (j + 1)
    ev0, _, _ = O.gevp(sp.H, sp.S)
    assert np.all(ev[:m] >= ev0[:m] - 1e-9 * np.maximum(1.0, np.abs(ev0[:m])))
    assert np.abs(C[:, :m].T @ sp.S @ C[:, :m] - np.eye(m)).max() <= 1e-9
    w, V = np.linalg.eigh(sp.S)
    drop = V[:, :j + 1]
    assert np.abs(drop.T @ sp.S @ C[:, :m]).max() <= 1e-9
