"""Parity of the eigen stages and of the whole ev / dm path against the CPU oracle.

Tolerances follow from backward stability: an orthogonal-transform method
perturbs a symmetric T (or A) by about c n eps ||A||, which moves each
eigenvalue by at most that much; eigenvector residuals are of the same order,
and orthogonality loss is about c n eps.
"""
import math

import numpy as np
import pytest

import oracle as O
from gates import eig_excess
from synth import generator as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _sym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return (A + A.T) / 2


def _band_dense(band, b, n):
    B = np.zeros((n, n))
    for r in range(b + 1):
        for c in range(n - r):
            B[c + r, c] = band[r, c]
            B[c, c + r] = band[r, c]
    return B


@pytest.mark.parametrize("n,b", [(10, 8), (64, 16), (65, 32), (130, 64), (300, 64), (513, 32)])
def test_band_reduce_keeps_spectrum(n, b):
    from paper_1705_11191_amd import binding as B

    A = _sym(n, n + b)
    band = B.band_reduce(_dev(A), b).cpu().numpy()   # (b+1) x n
    Bm = _band_dense(band, min(b, n - 1), n)
    ev_ref = np.linalg.eigvalsh(A)
    d, e, _ = O.tred(Bm)
    ev = O.tridiag_eigvals(d, e)
    assert np.abs(ev - ev_ref).max() <= 64 * n * EPS * np.abs(ev_ref).max()


def _panel_kind_matrix(kind, n, seed):
    """Symmetric matrices whose sub-band panels are full rank, rank deficient or
    strongly graded, so that the panel factorization takes each of its paths
    (the two-pass Cholesky QR and the column-by-column fallback)."""
    rng = np.random.default_rng(seed)
    if kind == "random":
        return _sym(n, seed)
    if kind == "rank40":
        U = np.linalg.qr(rng.standard_normal((n, 40)))[0]
        return U @ np.diag(rng.uniform(-3, 3, 40)) @ U.T
    if kind == "blockdiag":
        A = np.zeros((n, n))
        for o in range(0, n, 100):
            k = min(100, n - o)
            A[o:o + k, o:o + k] = _sym(k, seed + o)
        return A
    if kind == "graded":
        d = np.logspace(0, -6, n)
        return d[:, None] * _sym(n, seed) * d[None, :]
    if kind == "diagonal":
        return np.diag(rng.standard_normal(n))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["random", "rank40", "blockdiag", "graded", "diagonal"])
def test_band_reduce_panel_kinds_keep_spectrum(kind):
    from paper_1705_11191_amd import binding as B

    n, b = 700, 64
    A = _panel_kind_matrix(kind, n, 5)
    band = B.band_reduce(_dev(A), b).cpu().numpy()
    Bm = _band_dense(band, b, n)
    ev_ref = np.linalg.eigvalsh(A)
    d, e, _ = O.tred(Bm)
    ev = O.tridiag_eigvals(d, e)
    assert np.abs(ev - ev_ref).max() <= 64 * n * EPS * np.abs(ev_ref).max()


@pytest.mark.parametrize("n,b", [(2, 8), (3, 8), (17, 8), (64, 64), (100, 32), (257, 64), (600, 64)])
def test_tridiagonalize_keeps_spectrum(n, b):
    from paper_1705_11191_amd import binding as B

    A = _sym(n, 7 * n + b)
    d, e = B.tridiagonalize(_dev(A), b)
    w = O.tridiag_eigvals(d.cpu().numpy(), e.cpu().numpy())
    ref = O.tridiag_eigvals(*O.tred(A)[:2])
    assert np.abs(w - ref).max() <= 64 * n * EPS * np.abs(ref).max()


@pytest.mark.parametrize("n,b", [(3, 8), (17, 8), (100, 32), (257, 64), (600, 64), (777, 24), (1000, 40),
                                 (2049, 64)])
def test_bulge_schedules_agree(n, b):
    """The row-window and pipelined-sweep schedules of the bulge chasing form
    the same reflectors in different summation orders: T agrees entry by entry
    to rounding amplified by the chase (1e-9 ||A||), and both keep the
    oracle's spectrum (64 n eps ||A||)."""
    from paper_1705_11191_amd import binding as B

    A = _sym(n, 11 * n + b)
    ref = O.tridiag_eigvals(*O.tred(A)[:2])
    scale = np.abs(ref).max()
    out = {}
    try:
        for path in (1, 2):
            B.set_bulge_path(path)
            print(f"[bulge] n={n} b={b} path={path}", flush=True)
            d, e = B.tridiagonalize(_dev(A), b)
            out[path] = (d.cpu().numpy(), e.cpu().numpy())
    finally:
        B.set_bulge_path(0)
    for path, (d, e) in out.items():
        w = O.tridiag_eigvals(d, e)
        assert np.abs(w - ref).max() <= 64 * n * EPS * scale, path
    (d1, e1), (d2, e2) = out[1], out[2]
    assert np.abs(d1 - d2).max() <= 1e-9 * scale
    assert np.abs(e1 - e2).max() <= 1e-9 * scale


def _tridiag_cases():
    rng = np.random.default_rng(11)
    cases = []
    for n in [1, 2, 3, 63, 64, 65, 100, 200, 513, 1000]:
        cases.append((f"rand{n}", rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))))
    n = 300   # chain: many close eigenvalue pairs after tearing
    cases.append(("chain300", np.zeros(n), -np.ones(n - 1)))
    e = rng.standard_normal(399)
    e[::7] = 0.0   # exact splits -> deflation
    cases.append(("split400", rng.standard_normal(400), e))
    d = np.repeat([1.0, 2.0, 3.0], 100)   # clusters of equal diagonal entries
    cases.append(("cluster300", d, 1e-9 * rng.standard_normal(299)))
    k = np.arange(257)
    cases.append(("wilk257", np.abs(k - 128.0), np.ones(256)))   # Wilkinson-like, close pairs
    return cases


@pytest.mark.parametrize("name,d,e", _tridiag_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_tridiag_divide_and_conquer(name, d, e):
    from paper_1705_11191_amd import binding as B

    n = d.shape[0]
    w, Z = B.tridiag_eig(_dev(d), _dev(e))
    w = w.cpu().numpy()
    Z = Z.cpu().numpy()
    ref = O.tridiag_eigvals(d, e)
    nrm = max(np.abs(d).max() + 2 * (np.abs(e).max() if e.size else 0.0), 1e-300)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 32 * n * EPS * nrm
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(T @ Z - Z * w).max() <= 32 * n * EPS * nrm
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 32 * n * EPS


@pytest.mark.parametrize("n", [1, 5, 64, 129, 300])
def test_standard_ev_overlap_is_unit(n):
    from paper_1705_11191_amd import binding as B

    A = _sym(n, 3 * n)
    h = B.Handle(n, n, n / 4)
    h.set_overlap_is_unit(True)
    ev, C = h.ev(_dev(A), None)
    h.close()
    ev = ev.cpu().numpy()
    C = C.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    assert np.abs(ev - ref).max() <= 64 * n * EPS * np.abs(ref).max()
    assert np.abs(A @ C - C * ev).max() <= 64 * n * EPS * np.abs(ref).max()
    assert np.abs(C.T @ C - np.eye(n)).max() <= 64 * n * EPS




@pytest.mark.parametrize("kind", ["rank40", "blockdiag", "diagonal"])
def test_standard_ev_panels_that_cholesky_qr_cannot_factor(kind):
    """Rank-deficient panels defeat CholeskyQR2, and inside a solve (not only in
    the stage entry) those panels take the per-column Householder fallback.
    The spectrum and the eigenpairs must come out as for any other matrix."""
    from paper_1705_11191_amd import binding as B

    n = 700
    A = _panel_kind_matrix(kind, n, 9)
    print(f"[ev panels] kind={kind} n={n}", flush=True)
    h = B.Handle(n, n, n / 4)
    h.set_overlap_is_unit(True)
    ev, C = h.ev(_dev(A), None)
    h.close()
    ev = ev.cpu().numpy()
    C = C.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    scale = np.abs(ref).max()
    assert np.abs(ev - ref).max() <= 64 * n * EPS * scale
    assert np.abs(A @ C - C * ev).max() <= 64 * n * EPS * scale
    assert np.abs(C.T @ C - np.eye(n)).max() <= 64 * n * EPS


@pytest.mark.parametrize("b", [64, 32])
def test_ev_config0_vs_oracle(b):
    from paper_1705_11191_amd import binding as B

    sp = G.make_config(0)
    ev_ref, C_ref, _ = O.gevp(sp.H, sp.S)
    h = B.Handle(sp.n, sp.n, sp.n_occ)
    h.set_band_width(b)
    S = _dev(sp.S)
    ev, C = h.ev(_dev(sp.H), S)
    h.close()
    ev = ev.cpu().numpy()
    C = C.cpu().numpy()
    assert eig_excess(ev, ev_ref, sp.S) <= 1.0
    # S-orthonormality, and subspace agreement of the occupied block with the oracle
    assert np.abs(C.T @ sp.S @ C - np.eye(sp.n)).max() <= 1e-8
    k = int(sp.n_occ)
    P = C[:, :k] @ C[:, :k].T
    P_ref = C_ref[:, :k] @ C_ref[:, :k].T
    assert np.abs(P - P_ref).max() <= 1e-8
    # L was written into S (lower, zero above)
    L = S.cpu().numpy().T
    assert np.abs(np.triu(L, 1)).max() == 0.0
    assert np.abs(L @ L.T - sp.S).max() <= 1e-12 * np.abs(sp.S).max() * sp.n


def test_dm_config0_vs_oracle():
    from paper_1705_11191_amd import binding as B

    sp = G.make_config(0)
    ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    h = B.Handle(sp.n, sp.n, sp.n_occ)
    D, ev, f, energy, mu, st = h.dm(_dev(sp.H), _dev(sp.S))
    info = h.info()
    h.close()
    D = D.cpu().numpy()
    ev = ev.cpu().numpy()
    f = f.cpu().numpy()
    assert st == 0
    assert eig_excess(ev, ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
    assert np.abs(D - ref["D"]).max() <= 1e-9
    assert np.abs(D - D.T).max() == 0.0
    assert abs(mu - ref["mu"]) <= 1e-9
    assert abs(energy - ref["energy"]) <= 1e-9
    assert abs(np.trace(D @ sp.S) - sp.n_occ) <= 1e-10
    assert np.abs(f - ref["occ"]).max() <= 1e-12
    # k_s counts f > 1e-20 after the charge fix-up, which removes a surplus of
    # order occ_accuracy from the top states down: states occupied below that
    # level are kept or dropped by rounding, so k_s is bracketed by the states
    # the fix-up cannot remove (f > occ_accuracy) and those with a Fermi-Dirac
    # occupation above the cut before it
    assert info["k_s"] == int(np.sum(f > 1e-20))
    x = (ref["eval"] - ref["mu"]) / sp.kT
    k_hi = int(np.sum(x < -math.log(1e-20)))
    k_lo = int(np.sum(ref["occ"] > 1e-13))
    assert k_lo <= info["k_s"] <= k_hi


def test_dm_explicit_integer_occupations_idempotent():
    from paper_1705_11191_amd import binding as B

    sp = G.make_config(0)
    n, k = sp.n, int(sp.n_occ)
    f = np.zeros(n)
    f[:k] = 1.0
    h = B.Handle(n, n, float(k))
    h.set_occupation(scheme=B.OCC_EXPLICIT)
    D, ev, _, energy, mu, st = h.dm(_dev(sp.H), _dev(sp.S), occ=_dev(f))
    h.close()
    D = D.cpu().numpy()
    assert st == 0
    assert np.abs(D @ sp.S @ D - D).max() <= 1e-9
    assert abs(np.trace(D @ sp.S) - k) <= 1e-10
    assert abs(energy - ev.cpu().numpy()[:k].sum()) <= 1e-10


def test_dm_not_positive_definite_reports_status():
    from paper_1705_11191_amd import binding as B

    sp = G.make_config(0)
    S = sp.S.copy()
    S[100, 100] = -1.0
    h = B.Handle(sp.n, sp.n, sp.n_occ)
    with pytest.raises(B.ElsiGpuError) as ei:
        h.dm(_dev(sp.H), _dev(S))
    assert ei.value.status == 1
    assert h.info()["fail_col"] == 101
    h.close()


def test_dm_nonfinite_input_reports_status():
    from paper_1705_11191_amd import binding as B

    sp = G.make_config(0)
    H = sp.H.copy()
    H[5, 3] = np.nan
    h = B.Handle(sp.n, sp.n, sp.n_occ)
    with pytest.raises(B.ElsiGpuError) as ei:
        h.dm(_dev(H), _dev(sp.S))
    assert ei.value.status == 7
    h.close()
