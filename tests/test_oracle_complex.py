"""Pins of the oracle's complex Hermitian path (CPU only).

Each check fixes the complex arithmetic against something other than the
complex oracle itself: closed forms (2 x 2 pencil, Toeplitz pencil with a
shared phase), the real oracle (real input seen as complex; the real 2n x 2n
embedding of a complex pencil), an independent library routine (NumPy's
Hermitian eigensolver on the standard form) and invariants (C^H S C = I,
residuals, D Hermitian, tr(D S) = N_e).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle as O
from synth import generator as G


def _embed(Z):
    """Real 2n x 2n image of a complex n x n matrix: z_jk -> [[x, -y], [y, x]] at rows/cols 2j, 2j+1."""
    n = Z.shape[0]
    R = np.zeros((2 * n, 2 * n))
    R[0::2, 0::2] = Z.real
    R[1::2, 1::2] = Z.real
    R[0::2, 1::2] = -Z.imag
    R[1::2, 0::2] = Z.imag
    return R


def _random_pencil(n, seed, kappa=1e3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = (A + A.conj().T) / 2
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    S0 = B @ B.conj().T / n
    w = np.linalg.eigvalsh(S0)
    S = S0 + (w[-1] / kappa) * np.eye(n)
    return H, S


# 2 x 2:  H = [[a, b], [conj b, c]], S = [[1, s], [conj s, 1]]:
#   (1 - |s|^2) lam^2 - (a + c - 2 Re(b conj s)) lam + (a c - |b|^2) = 0
@pytest.mark.parametrize("a,b,c,s", [(1.0, 0.5 + 0.3j, -2.0, 0.3 - 0.2j), (-0.4, 0.7j, 0.9, -0.8j),
                                     (0.25, -1.0 + 1.0j, 0.25, 0.6 + 0.79j)])
def test_zgevp_2x2_closed_form(a, b, c, s):
    A2 = 1 - abs(s) ** 2
    B1 = -(a + c - 2 * (b * np.conj(s)).real)
    C0 = a * c - abs(b) ** 2
    disc = math.sqrt(B1 * B1 - 4 * A2 * C0)
    roots = sorted([(-B1 - disc) / (2 * A2), (-B1 + disc) / (2 * A2)])
    H = np.array([[a, b], [np.conj(b), c]])
    S = np.array([[1.0, s], [np.conj(s), 1.0]])
    ev, C, L = O.zgevp(H, S)
    assert np.abs(ev - roots).max() < 1e-12 * max(1.0, max(abs(r) for r in roots))
    # L closed form: [[1, 0], [conj s, sqrt(1 - |s|^2)]]
    np.testing.assert_allclose(L, [[1.0, 0.0], [np.conj(s), math.sqrt(A2)]], rtol=0, atol=1e-15)


# Toeplitz pencil with one shared phase: beta = b e^{i phi}, sigma = s e^{i phi}; the
# diagonal unitary diag(e^{i j phi}) makes both real, so
#   lam_k = (a + 2 b cos th_k) / (1 + 2 s cos th_k),  th_k = k pi / (N + 1).
@pytest.mark.parametrize("n,a,b,s,phi", [(5, 0.1, -0.7, 0.2, 0.3), (60, -0.3, 0.4, 0.45, 2.0),
                                         (120, 0.2, -0.45, 0.4999, -1.1)])
def test_zgevp_toeplitz_shared_phase_closed_form(n, a, b, s, phi):
    ph = complex(math.cos(phi), math.sin(phi))
    H, S = G.toeplitz_pencil(n, a, b * ph, s * ph)
    th = np.arange(1, n + 1) * np.pi / (n + 1)
    lam = np.sort((a + 2 * b * np.cos(th)) / (1 + 2 * s * np.cos(th)))
    ev, C, _ = O.zgevp(H, S)
    ws = np.linalg.eigvalsh(S)
    kappa = ws[-1] / ws[0]
    assert np.abs(ev - lam).max() <= 1e-13 * np.abs(lam).max() * max(1.0, kappa ** 0.5)


def test_zgevp_real_input_equals_real_oracle():
    sp = G.make_lattice_system(90, seed=3)
    ev_r, C_r, L_r = O.gevp(sp.H, sp.S)
    ev_c, C_c, L_c = O.zgevp(sp.H.astype(np.complex128), sp.S.astype(np.complex128))
    assert np.abs(ev_c - ev_r).max() <= 1e-11 * max(1.0, np.abs(ev_r).max())
    np.testing.assert_allclose(L_c.real, L_r, rtol=0, atol=1e-13)
    assert np.abs(L_c.imag).max() == 0.0
    ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    got = O.zdm(sp.H.astype(np.complex128), sp.S.astype(np.complex128), sp.n_occ, sp.kT)
    assert np.abs(got["D"] - ref["D"]).max() <= 1e-9
    assert abs(got["energy"] - ref["energy"]) <= 1e-9 * max(1.0, abs(ref["energy"]))


def test_zgevp_matches_real_embedding():
    """The real 2n pencil [[Re, -Im], [Im, Re]] has every complex eigenvalue twice."""
    sp = G.make_kpoint_system((2, 3, 3), (0.375, -0.25, 0.25), seed=4, kappa=1e3)
    ev_c, _, _ = O.zgevp(sp.H, sp.S)
    ev_r, _, _ = O.gevp(_embed(sp.H), _embed(sp.S))
    scale = max(1.0, np.abs(ev_c).max())
    assert np.abs(ev_r[0::2] - ev_c).max() <= 1e-11 * scale
    assert np.abs(ev_r[1::2] - ev_c).max() <= 1e-11 * scale


def test_zgevp_vs_numpy_hermitian_eigensolver():
    H, S = _random_pencil(70, seed=8, kappa=1e3)
    Ln = np.linalg.cholesky(S)
    Hs = np.linalg.solve(Ln, np.linalg.solve(Ln, H).conj().T).conj().T
    ref = np.linalg.eigvalsh((Hs + Hs.conj().T) / 2)
    ev, C, _ = O.zgevp(H, S)
    assert np.abs(ev - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n_state", [None, 7])
def test_zgevp_invariants(n_state):
    sp = G.make_kpoint_system((3, 3, 3), (0.125, 0.25, 0.25), seed=2, kappa=1e4)
    ev, C, _ = O.zgevp(sp.H, sp.S, n_state)
    k = C.shape[1]
    G_ = C.conj().T @ sp.S @ C
    assert np.abs(G_ - np.eye(k)).max() <= 1e-10
    R = sp.H @ C - sp.S @ C * ev[:k]
    assert np.abs(R).max() <= 1e-10 * max(1.0, np.abs(ev).max())
    # phase convention: the largest-magnitude entry of every column is real and positive
    imax = np.abs(C).argmax(axis=0)
    top = C[imax, np.arange(k)]
    assert np.all(top.real > 0) and np.abs(top.imag).max() == 0.0


def test_ztred_invariants():
    H, _ = _random_pencil(40, seed=9)
    d, e, Q = O.ztred(H)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(Q.conj().T @ Q - np.eye(40)).max() <= 1e-13
    assert np.abs(Q @ T @ Q.conj().T - H).max() <= 1e-12 * np.abs(H).max()
    assert np.all(e >= 0.0)


def test_zdm_invariants_and_projector():
    sp = G.make_kpoint_system((3, 3, 3), (0.125, 0.25, 0.25), seed=5, kappa=1e4)
    out = O.zdm(sp.H, sp.S, sp.n_occ, sp.kT)
    D = out["D"]
    assert np.abs(D - D.conj().T).max() <= 1e-14 * max(1.0, np.abs(D).max())
    assert abs(np.trace(D @ sp.S).real - sp.n_occ) <= 1e-10 * sp.n_occ
    assert abs(np.trace(D @ sp.S).imag) <= 1e-10
    assert abs(out["energy"] - float(np.dot(out["occ"], out["eval"]))) <= 1e-12 * max(1.0, abs(out["energy"]))
    # against NumPy's eigenvectors of the standard form, mapped back through its own Cholesky
    Ln = np.linalg.cholesky(sp.S)
    Hs = np.linalg.solve(Ln, np.linalg.solve(Ln, sp.H).conj().T).conj().T
    w, Z = np.linalg.eigh((Hs + Hs.conj().T) / 2)
    Cn = np.linalg.solve(Ln.conj().T, Z)
    Dn = (Cn * out["occ"]) @ Cn.conj().T
    assert np.abs(D - Dn).max() <= 1e-9
