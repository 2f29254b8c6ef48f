"""Complex Hermitian pencils (the k-point problems of periodic systems) against
the oracle's native complex path.

The GPU solves the real 2n x 2n image of the pencil; the oracle works in
complex arithmetic throughout (complex Cholesky, Hermitian Householder,
QL), so the two share nothing but the input.  Gates as for the real path:
eigenvalues by gates.eig_excess, D within 1e-9, eigenvectors through C^H S C = I,
residuals and the projector onto gap-separated groups of states.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle as O
from gates import eig_excess
from synth import generator as G

pytestmark = pytest.mark.gpu


def _cdev(A):
    """Column-major complex128 device tensor."""
    from paper_1705_11191_amd import binding as B

    return B.as_fortran(torch.tensor(np.asarray(A, dtype=np.complex128), device="cuda"))


def _kpoint(cells, kpt, seed, kappa=1e6):
    return G.make_kpoint_system(cells, kpt, seed=seed, kappa=kappa)


@pytest.mark.parametrize("cells,kpt,seed", [((2, 3, 3), (0.375, -0.25, 0.25), 1),
                                            ((3, 3, 3), (0.125, 0.25, 0.25), 2),
                                            ((4, 4, 4), (-0.125, 0.25, -0.25), 3)])
def test_complex_dm_vs_oracle(cells, kpt, seed):
    from paper_1705_11191_amd import binding as B

    sp = _kpoint(cells, kpt, seed)
    n = sp.H.shape[0]
    ref = O.zdm(sp.H, sp.S, sp.n_occ, sp.kT)
    h = B.Handle(n, n, sp.n_occ, dtype=B.COMPLEX128)
    S = _cdev(sp.S)
    D, ev, f, energy, mu, st = h.dm(_cdev(sp.H), S)
    h.close()
    assert st == 0
    assert eig_excess(ev.cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
    D = D.cpu().numpy()
    assert np.abs(D - ref["D"]).max() <= 1e-9
    assert np.abs(D - D.conj().T).max() <= 1e-12
    assert abs(energy - ref["energy"]) <= 1e-9 * max(1.0, abs(ref["energy"]))
    assert abs(np.trace(D @ sp.S) - sp.n_occ) <= 1e-10 * max(1.0, sp.n_occ)
    np.testing.assert_allclose(f.cpu().numpy(), ref["occ"], rtol=0, atol=1e-12)
    # S receives the complex Cholesky factor (lower, zero above); as for the
    # real factor, the forward error is about n eps cond(S)^(1/2) |L|
    L = S.cpu().numpy()
    assert np.abs(np.triu(L, 1)).max() == 0.0
    cond = np.linalg.cond(sp.S)
    assert np.abs(L - ref["L"]).max() <= 8 * n * np.finfo(float).eps * math.sqrt(cond) * np.abs(ref["L"]).max()


@pytest.mark.parametrize("n_state", [1, 20, 108])
def test_complex_ev_vs_oracle(n_state):
    from paper_1705_11191_amd import binding as B

    sp = _kpoint((3, 3, 3), (0.125, 0.25, 0.25), 4)
    n = sp.H.shape[0]
    ev_ref, C_ref, _ = O.zgevp(sp.H, sp.S, n_state)
    h = B.Handle(n, n_state, sp.n_occ, dtype=B.COMPLEX128)
    ev, C = h.ev(_cdev(sp.H), _cdev(sp.S))
    h.close()
    ev = ev.cpu().numpy()
    C = C.cpu().numpy()
    assert C.shape == (n, n_state)
    assert eig_excess(ev, ev_ref, sp.S) <= 1.0
    assert np.abs(C.conj().T @ sp.S @ C - np.eye(n_state)).max() <= 1e-8
    R = sp.H @ C - (sp.S @ C) * ev[:n_state]
    assert np.abs(R).max() <= 1e-7 * max(1.0, np.abs(ev).max())
    if n_state == n or ev_ref[n_state] - ev_ref[n_state - 1] > 1e-6:
        P = C @ C.conj().T
        P_ref = C_ref @ C_ref.conj().T
        assert np.abs(P - P_ref).max() <= 1e-8 * max(1.0, np.abs(P_ref).max())


def test_complex_real_input_matches_real_path():
    """k = 0: the complex path on a real pencil gives the real path's results."""
    from paper_1705_11191_amd import binding as B

    sp = _kpoint((3, 3, 3), (0.0, 0.0, 0.0), 5)
    n = sp.H.shape[0]
    Hr = sp.H.real.copy()
    Sr = sp.S.real.copy()
    hr = B.Handle(n, n, sp.n_occ)
    Dr, evr, _, er, mur, _ = hr.dm(torch.tensor(Hr, device="cuda"), torch.tensor(Sr, device="cuda"))
    hr.close()
    hc = B.Handle(n, n, sp.n_occ, dtype=B.COMPLEX128)
    Dc, evc, _, ec, muc, st = hc.dm(_cdev(sp.H), _cdev(sp.S))
    hc.close()
    assert st == 0
    Dc = Dc.cpu().numpy()
    assert np.abs(Dc.real - Dr.cpu().numpy()).max() <= 1e-9
    assert np.abs(Dc.imag).max() <= 1e-9
    assert eig_excess(evc.cpu().numpy(), evr.cpu().numpy(), Sr) <= 1.0
    assert abs(ec - er) <= 1e-9 * max(1.0, abs(er))


def test_complex_degenerate_states_get_an_orthonormal_basis():
    """blockdiag(A, A) x = lam blockdiag(B, B) x: every eigenvalue twice in the
    complex pencil, four times in its real image."""
    from paper_1705_11191_amd import binding as B

    sp = _kpoint((2, 3, 3), (0.375, -0.25, 0.25), 6, kappa=1e4)
    m = sp.H.shape[0]
    n = 2 * m
    H = np.zeros((n, n), dtype=np.complex128)
    S = np.zeros((n, n), dtype=np.complex128)
    H[:m, :m] = sp.H
    H[m:, m:] = sp.H
    S[:m, :m] = sp.S
    S[m:, m:] = sp.S
    k = 40
    ev_ref, _, _ = O.zgevp(sp.H, sp.S)
    h = B.Handle(n, k, 1.0, dtype=B.COMPLEX128)
    ev, C = h.ev(_cdev(H), _cdev(S))
    h.close()
    ev = ev.cpu().numpy()
    C = C.cpu().numpy()
    assert eig_excess(ev, np.repeat(ev_ref, 2), S) <= 1.0
    assert np.abs(C.conj().T @ S @ C - np.eye(k)).max() <= 1e-8
    R = H @ C - (S @ C) * ev[:k]
    assert np.abs(R).max() <= 1e-7 * max(1.0, np.abs(ev).max())


@pytest.mark.parametrize("n,a,b,s,phi", [(40, 0.1, -0.7, 0.2, 0.3), (130, -0.3, 0.4, 0.45, 2.0)])
def test_complex_toeplitz_shared_phase_closed_form(n, a, b, s, phi):
    from paper_1705_11191_amd import binding as B

    ph = complex(math.cos(phi), math.sin(phi))
    H, S = G.toeplitz_pencil(n, a, b * ph, s * ph)
    th = np.arange(1, n + 1) * np.pi / (n + 1)
    lam = np.sort((a + 2 * b * np.cos(th)) / (1 + 2 * s * np.cos(th)))
    h = B.Handle(n, n, 1.0, dtype=B.COMPLEX128)
    ev, _ = h.ev(_cdev(H), _cdev(S))
    h.close()
    ws = np.linalg.eigvalsh(S)
    assert np.abs(ev.cpu().numpy() - lam).max() <= 1e-12 * np.abs(lam).max() * max(1.0, (ws[-1] / ws[0]) ** 0.5)


def test_complex_tiny_closed_forms():
    from paper_1705_11191_amd import binding as B

    # 1 x 1: eps = h / s
    h = B.Handle(1, 1, 0.5, dtype=B.COMPLEX128)
    ev, C = h.ev(_cdev([[-0.3 + 0.0j]]), _cdev([[2.0 + 0.0j]]))
    h.close()
    assert abs(ev.item() + 0.15) <= 1e-15
    # 2 x 2: (1 - |s|^2) lam^2 - (a + c - 2 Re(b conj s)) lam + (a c - |b|^2) = 0
    a, b, c, s = 1.0, 0.5 + 0.3j, -2.0, 0.3 - 0.2j
    A2 = 1 - abs(s) ** 2
    B1 = -(a + c - 2 * (b * np.conj(s)).real)
    C0 = a * c - abs(b) ** 2
    disc = math.sqrt(B1 * B1 - 4 * A2 * C0)
    roots = np.sort([(-B1 - disc) / (2 * A2), (-B1 + disc) / (2 * A2)])
    h = B.Handle(2, 2, 1.0, dtype=B.COMPLEX128)
    ev, C = h.ev(_cdev([[a, b], [np.conj(b), c]]), _cdev([[1.0, s], [np.conj(s), 1.0]]))
    h.close()
    assert np.abs(ev.cpu().numpy() - roots).max() <= 1e-13


def test_complex_factored_overlap_reuse_and_unit_overlap():
    from paper_1705_11191_amd import binding as B

    sp = _kpoint((3, 3, 3), (0.125, 0.25, 0.25), 7)
    n = sp.H.shape[0]
    h = B.Handle(n, n, sp.n_occ, dtype=B.COMPLEX128)
    S = _cdev(sp.S)
    h.dm(_cdev(sp.H), S)
    rng = np.random.default_rng(2)
    H2 = sp.H + np.diag(rng.uniform(-0.01, 0.01, size=n))
    h.set_overlap_factored(True)
    D2, ev2, _, _, _, st = h.dm(_cdev(H2), S)
    h.close()
    ref = O.zdm(H2, sp.S, sp.n_occ, sp.kT)
    assert st == 0
    assert eig_excess(ev2.cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
    assert np.abs(D2.cpu().numpy() - ref["D"]).max() <= 1e-9
    # S = I
    h = B.Handle(n, n, sp.n_occ, dtype=B.COMPLEX128)
    h.set_overlap_is_unit(True)
    D, ev, _, _, _, st = h.dm(_cdev(sp.H), None)
    h.close()
    ref = O.zdm(sp.H, np.eye(n), sp.n_occ, sp.kT)
    assert st == 0
    assert np.abs(D.cpu().numpy() - ref["D"]).max() <= 1e-9


def test_complex_batched_kpoints_vs_oracle():
    from paper_1705_11191_amd import binding as B

    kpts = [(0.125, 0.25, 0.25), (-0.125, 0.25, 0.25), (0.375, -0.25, 0.25), (0.375, 0.25, -0.25)]
    sps = [_kpoint((2, 3, 3), k, 10 + q) for q, k in enumerate(kpts)]
    h = B.Handle(8, 8, 2, dtype=B.COMPLEX128)
    Ds, evals, energy, mu, status, rc = h.dm_batched([_cdev(sp.H) for sp in sps], [_cdev(sp.S) for sp in sps],
                                                     [sp.n_occ for sp in sps])
    h.close()
    assert rc == 0 and status == [0] * len(sps)
    for q, sp in enumerate(sps):
        ref = O.zdm(sp.H, sp.S, sp.n_occ, sp.kT)
        assert eig_excess(evals[q].cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0, q
        assert np.abs(Ds[q].cpu().numpy() - ref["D"]).max() <= 1e-9, q
        assert abs(energy[q] - ref["energy"]) <= 1e-9 * max(1.0, abs(ref["energy"])), q


def test_complex_handle_rejects_row_major_input():
    from paper_1705_11191_amd import binding as B

    h = B.Handle(4, 4, 1.0, dtype=B.COMPLEX128)
    A = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        h.ev(A, A)
    h.close()
