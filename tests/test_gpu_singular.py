"""Singularity check of the overlap and the eigendecomposition transform
(Sec. 4.5, Eq. (20)) against the oracle.

The singular pencils duplicate basis functions of a lattice system, so S is
exactly singular and the transformed problem is the original one (the
oracle's closed-form pins hold there).  Gates: the N_nonsing eigenvalues by
gates.eig_excess against the oracle's, +inf beyond them; D within 1e-9; the
returned X satisfies X X^T = S and carries the oracle's column norms (the
kept eigenvalues of S, its columns' signs being free).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from gates import eig_excess
from synth import generator as G

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _duplicate(sp, dup):
    n0 = sp.H.shape[0]
    idx = list(range(n0)) + list(dup)
    E = np.zeros((len(idx), n0))
    E[np.arange(len(idx)), idx] = 1.0
    return E @ sp.H @ E.T, E @ sp.S @ E.T


@pytest.mark.parametrize("n0,dup", [(300, (7, 150, 299)), (520, (3,))])
def test_dm_with_duplicated_basis_functions_vs_oracle(n0, dup):
    from paper_1705_11191_amd import binding as B

    sp = G.make_lattice_system(n0, seed=90 + n0, kappa=1e3)
    H, S = _duplicate(sp, dup)
    n = H.shape[0]
    ref = O.dm_checked(H, S, sp.n_occ, sp.kT, 1e-8)
    h = B.Handle(n, n, sp.n_occ)
    h.set_singularity(True, 1e-8)
    Sd = _dev(S)
    D, ev, f, energy, mu, st = h.dm(_dev(H), Sd)
    info = h.info()
    D, ev, f = D.cpu().numpy(), ev.cpu().numpy(), f.cpu().numpy()
    m = info["n_nonsing"]
    print(f"[singular] n={n} m={m} min eig S {info['overlap_min_eig']:.2e} D err {np.abs(D - ref['D']).max():.2e}",
          flush=True)
    assert st == 0 and m == ref["n_nonsing"] == n0
    assert abs(info["overlap_min_eig"]) <= 1e-10
    assert np.all(np.isinf(ev[m:])) and np.all(f[m:] == 0.0)
    assert eig_excess(ev[:m], ref["eval"][:m], sp.S, occ=ref["occ"][:m]) <= 1.0
    assert np.abs(D - ref["D"]).max() <= 1e-9
    assert abs(energy - ref["energy"]) <= 1e-9 * max(1.0, abs(ref["energy"]))
    X = Sd.cpu().numpy().T   # column-major X in the row-major buffer
    assert np.abs(X[:, m:]).max() == 0.0
    assert np.abs(X @ X.T - S).max() <= 1e-11 * np.abs(S).max()
    Xo = ref["S_out"]
    assert np.allclose(np.sum(X[:, :m] ** 2, 0), np.sum(Xo[:, :m] ** 2, 0), rtol=1e-10, atol=1e-14)
    # a second call reuses X (overlap_factored): the same density matrix
    h.set_overlap_factored(True)
    D2, *_ = h.dm(_dev(H), Sd)
    h.close()
    assert np.abs(D2.cpu().numpy() - D).max() <= 1e-10   # lam_j = ||X_j||^2 is recomputed from X


def test_ev_with_duplicated_basis_functions_vs_oracle():
    from paper_1705_11191_amd import binding as B

    sp = G.make_lattice_system(240, seed=95, kappa=1e3)
    H, S = _duplicate(sp, (10, 11))
    n, k = H.shape[0], 100
    evo, Co, Xo, m = O.gevp_checked(H, S, 1e-8, n_state=k)
    h = B.Handle(n, k, sp.n_occ)
    h.set_singularity(True, 1e-8)
    ev, C = h.ev(_dev(H), _dev(S))
    info = h.info()
    h.close()
    ev, C = ev.cpu().numpy(), C.cpu().numpy()
    assert info["n_nonsing"] == m == 240
    assert eig_excess(ev[:m], evo[:m], sp.S) <= 1.0 and np.all(np.isinf(ev[m:]))
    assert np.abs(C.T @ S @ C - np.eye(k)).max() <= 1e-9
    gap = np.minimum(np.abs(np.diff(evo[:k + 1])[:k]), np.abs(np.diff(evo[:k], prepend=-np.inf)))
    sep = gap > 1e-6
    dots = np.abs(np.sum((C.T @ S) * Co.T, axis=1))
    assert np.all(np.abs(dots[sep] - 1.0) <= 1e-8)


def test_check_on_a_well_conditioned_overlap_takes_the_cholesky_route():
    from paper_1705_11191_amd import binding as B

    sp = G.make_lattice_system(300, seed=96)
    lam_min = np.linalg.eigvalsh(sp.S)[0]
    out = []
    for check in (False, True):
        h = B.Handle(sp.n, sp.n, sp.n_occ)
        h.set_singularity(check, 0.5 * lam_min)
        D, *_ = h.dm(_dev(sp.H), _dev(sp.S))
        out.append((D.cpu().numpy(), h.info()))
        h.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[1][1]["n_nonsing"] == sp.n
    assert abs(out[1][1]["overlap_min_eig"] - lam_min) <= 1e-9 * lam_min


def test_tolerance_above_small_eigenvalues_vs_oracle():
    """A nonsingular S with tau in a wide gap of its spectrum: the directions
    below tau are dropped on both sides alike.  (The lattice basis holds a
    large cluster of eigenvalues of S within 1e-3 of the smallest; a cut inside
    it would not determine the kept subspace in FP64, so tau sits in the widest
    gap above the cluster, whose width bounds the subspace's sensitivity.)"""
    from paper_1705_11191_amd import binding as B

    sp = G.make_lattice_system(260, seed=97, kappa=1e3)
    lam = np.linalg.eigvalsh(sp.S)
    j = 180 + int(np.argmax(np.diff(lam)[180:230]))
    tau = 0.5 * (lam[j] + lam[j + 1])
    ref = O.dm_checked(sp.H, sp.S, sp.n_occ, sp.kT, tau)
    h = B.Handle(sp.n, sp.n, sp.n_occ)
    h.set_singularity(True, tau)
    D, ev, f, energy, mu, st = h.dm(_dev(sp.H), _dev(sp.S))
    info = h.info()
    h.close()
    m = info["n_nonsing"]
    assert st == 0 and m == ref["n_nonsing"] == sp.n - (j + 1)
    assert eig_excess(ev.cpu().numpy()[:m], ref["eval"][:m], sp.S, occ=ref["occ"][:m]) <= 1.0
    assert np.abs(D.cpu().numpy() - ref["D"]).max() <= 1e-9
