"""Pins of the CPU oracle against things other than itself.

Each test ties one part of the oracle to a closed form, an exact special case,
an invariant of the mathematics, a brute-force computation in higher or exact
precision, or an independent library route -- chosen so that a dropped term,
a wrong sign or index, or a transposed operand in any oracle step fails at
least one of them.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from synth import generator as G

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ---------------------------------------------------------------------------
# tridiagonal eigensolver (implicit QL): 1D tight-binding chain
#   H = tridiag(t, e0, t):  eps_k = e0 + 2 t cos(k pi / (N+1)),
#   x_k(j) = sqrt(2 / (N+1)) sin(j k pi / (N+1)),  j, k = 1..N
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,e0,t", [(1, 0.3, 1.0), (2, 0.0, -1.0), (7, -0.2, 0.5),
                                    (64, 0.0, -1.0), (257, 1.5, 0.25)])
def test_ql_chain_closed_form(n, e0, t):
    k = np.arange(1, n + 1)
    exact = np.sort(e0 + 2 * t * np.cos(k * np.pi / (n + 1)))
    w, Z = O.tridiag_eig(np.full(n, e0), np.full(n - 1, t))
    assert np.abs(w - exact).max() <= 8 * n * np.finfo(float).eps * (abs(e0) + 2 * abs(t))
    # eigenvectors: compare to the sine vectors up to sign (spectrum is simple);
    # perturbation bound ~ n eps ||T|| / gap (Davis-Kahan)
    j = np.arange(1, n + 1)
    order = np.argsort(e0 + 2 * t * np.cos(k * np.pi / (n + 1)), kind="stable")
    for col, kk in enumerate(k[order]):
        x = math.sqrt(2.0 / (n + 1)) * np.sin(j * kk * np.pi / (n + 1))
        z = Z[:, col]
        gap = np.inf if n == 1 else np.abs(np.delete(exact, col) - exact[col]).min()
        bound = 16 * n * np.finfo(float).eps * (abs(e0) + 2 * abs(t)) / gap
        assert min(np.abs(z - x).max(), np.abs(z + x).max()) < max(bound, 1e-14)


def test_ql_eigvals_only_matches_vectors_path():
    rng = np.random.default_rng(3)
    d, e = rng.standard_normal(40), rng.standard_normal(39)
    w1 = O.tridiag_eigvals(d, e)
    w2, _ = O.tridiag_eig(d, e)
    np.testing.assert_array_equal(w1, w2)


def test_ql_split_matrix_and_zero_offdiag():
    # e = 0 everywhere: eigenvalues are the sorted diagonal, vectors the permutation
    d = np.array([3.0, -1.0, 2.0, -1.0, 0.5])
    w, Z = O.tridiag_eig(d, np.zeros(4))
    np.testing.assert_array_equal(w, np.sort(d, kind="stable"))
    assert np.abs(np.abs(Z) - np.abs(Z).round()).max() == 0.0


# ---------------------------------------------------------------------------
# whole generalized solve: Toeplitz pencil with closed-form spectrum
#   H = tridiag(b, a, b), S = tridiag(s, 1, s), |s| < 1/2:
#   lam_k = (a + 2 b cos th_k) / (1 + 2 s cos th_k), th_k = k pi / (N+1)
#   and S-normalized eigenvectors sin(j th_k) / sqrt((N+1)/2 (1 + 2 s cos th_k)).
# cond(S) = (1 + 2|s| cos(pi/(N+1))) / (1 - 2|s| cos(pi/(N+1))).
# ---------------------------------------------------------------------------
def _sigma_for_cond(n, kappa):
    c = math.cos(math.pi / (n + 1))
    return (kappa - 1) / (kappa + 1) / (2 * c)


@pytest.mark.parametrize("n,a,b,kappa", [(3, 0.1, -0.7, 10.0), (50, -0.3, 0.4, 1e3),
                                         (120, 0.2, -0.45, 1e6)])
def test_gevp_toeplitz_pencil_closed_form(n, a, b, kappa):
    s = _sigma_for_cond(n, kappa)
    H, S = G.toeplitz_pencil(n, a, b, s)
    # closed-form condition number check of the input itself
    ws = np.linalg.eigvalsh(S)
    assert ws[-1] / ws[0] == pytest.approx(kappa, rel=1e-6)
    th = np.arange(1, n + 1) * np.pi / (n + 1)
    lam = (a + 2 * b * np.cos(th)) / (1 + 2 * s * np.cos(th))
    order = np.argsort(lam, kind="stable")
    ev, C, _ = O.gevp(H, S)
    scale = np.abs(lam).max()
    assert np.abs(ev - lam[order]).max() <= 1e-13 * scale * max(1.0, kappa ** 0.5)
    j = np.arange(1, n + 1)
    for col in range(0, n, max(1, n // 10)):
        k = order[col]
        x = np.sin(j * th[k]) / math.sqrt((n + 1) / 2 * (1 + 2 * s * math.cos(th[k])))
        c = C[:, col]
        err = min(np.abs(c - x).max(), np.abs(c + x).max()) / np.abs(x).max()
        assert err < 1e-9 * max(1.0, kappa ** 0.5)


# ---------------------------------------------------------------------------
# 2 x 2 closed form:  H = [[a, b], [b, c]], S = [[1, s], [s, 1]]:
#   (1 - s^2) lam^2 - (a + c - 2 b s) lam + (a c - b^2) = 0
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("a,b,c,s", [(1.0, 0.5, -2.0, 0.3), (-0.4, 0.0, 0.9, -0.8),
                                     (0.25, -1.5, 0.25, 0.999)])
def test_gevp_2x2_closed_form(a, b, c, s):
    A2, B1, C0 = 1 - s * s, -(a + c - 2 * b * s), a * c - b * b
    disc = math.sqrt(B1 * B1 - 4 * A2 * C0)
    roots = sorted([(-B1 - disc) / (2 * A2), (-B1 + disc) / (2 * A2)])
    ev, C, L = O.gevp(np.array([[a, b], [b, c]]), np.array([[1.0, s], [s, 1.0]]))
    assert np.abs(ev - roots).max() < 1e-12 * max(1.0, max(abs(r) for r in roots))
    # L closed form: [[1, 0], [s, sqrt(1 - s^2)]]
    np.testing.assert_allclose(L, [[1.0, 0.0], [s, math.sqrt(1 - s * s)]], rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# Cholesky / reduction special cases and invariants
# ---------------------------------------------------------------------------
def test_identity_overlap_is_exact():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((30, 30))
    H = A + A.T
    L = O.potrf(np.eye(30))
    np.testing.assert_array_equal(L, np.eye(30))
    np.testing.assert_array_equal(O.reduce_standard(H, L), H)


def test_potrf_backward_error_and_failure():
    rng = np.random.default_rng(6)
    B = rng.standard_normal((80, 80))
    S = B @ B.T + 1e-3 * np.eye(80)
    L = O.potrf(S)
    assert np.abs(np.triu(L, 1)).max() == 0.0
    assert np.linalg.norm(L @ L.T - S) / np.linalg.norm(S) < 80 * np.finfo(float).eps
    bad = S.copy()
    bad[10, 10] = -1.0
    with pytest.raises(O.oracle.OracleError) as ei:
        O.potrf(bad)
    assert ei.value.status == 1 and "column 10" in str(ei.value)


def test_reduce_against_explicit_definition():
    # H~ = L^-1 H L^-T: check H~ L^T = L^-1 H, i.e. L H~ L^T = H, to rounding
    rng = np.random.default_rng(7)
    A = rng.standard_normal((60, 60))
    H = A + A.T
    B = rng.standard_normal((60, 60))
    L = O.potrf(B @ B.T + 60 * np.eye(60))
    Ht = O.reduce_standard(H, L)
    np.testing.assert_array_equal(Ht, Ht.T)
    assert np.abs(L @ Ht @ L.T - H).max() < 1e-12 * np.abs(H).max() * 60


# ---------------------------------------------------------------------------
# Householder tridiagonalization: Q orthogonal, A = Q T Q^T, spectrum kept,
# tridiagonal input unchanged up to signs
# ---------------------------------------------------------------------------
def test_tred_invariants():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((70, 70))
    A = A + A.T
    d, e, Q = O.tred(A)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(Q.T @ Q - np.eye(70)).max() < 1e-13
    assert np.abs(Q @ T @ Q.T - A).max() < 1e-12 * np.abs(A).max() * 10
    exact_chain = O.tridiag_eigvals(d, e)
    np.testing.assert_allclose(exact_chain, np.linalg.eigvalsh(A), atol=1e-12 * 70)


def test_tred_on_tridiagonal_input_is_identity_up_to_sign():
    n = 20
    H = G.tight_binding_chain(n, 0.5, -0.3)
    d, e, Q = O.tred(H)
    np.testing.assert_allclose(d, 0.5, atol=1e-15)
    np.testing.assert_allclose(np.abs(e), 0.3, atol=1e-15)
    np.testing.assert_allclose(np.abs(Q), np.eye(n), atol=1e-15)


# ---------------------------------------------------------------------------
# brute force on tiny inputs
#   (1) Sylvester inertia in exact rational arithmetic: the number of
#       eigenvalues of (H, S) below x equals the number of negative pivots of
#       the LDL^T factorization of H - x S.  Bisection with it brackets each
#       eigenvalue independently of every oracle step.
#   (2) 50-digit mpmath eigenvalues of L^-1 H L^-T.
# ---------------------------------------------------------------------------
def _neg_pivots(H, S, x):
    n = len(H)
    A = [[Fraction(H[i][j]) - x * Fraction(S[i][j]) for j in range(n)] for i in range(n)]
    neg = 0
    for k in range(n):
        p = A[k][k]
        if p == 0:
            p = Fraction(1, 10 ** 40)  # perturb an exact zero pivot (measure-zero event)
        if p < 0:
            neg += 1
        for i in range(k + 1, n):
            m = A[i][k] / p
            for j in range(k + 1, n):
                A[i][j] -= m * A[k][j]
    return neg


@pytest.mark.parametrize("n", [3, 4, 5])
def test_gevp_tiny_exact_inertia(n):
    rng = np.random.default_rng(100 + n)
    H = np.round(rng.standard_normal((n, n)) * 8) / 8
    H = (H + H.T) / 2
    B = np.round(rng.standard_normal((n, n)) * 4) / 4
    S = B @ B.T + np.eye(n)
    ev, _, _ = O.gevp(H, S)
    Hq = [[float(v) for v in row] for row in H]
    Sq = [[float(v) for v in row] for row in S]
    for idx, lam in enumerate(ev):
        # exactly idx eigenvalues lie below lam - tol and idx+1 below lam + tol
        tol = Fraction(1, 10 ** 11)
        x = Fraction(lam)
        assert _neg_pivots(Hq, Sq, x - tol) <= idx
        assert _neg_pivots(Hq, Sq, x + tol) >= idx + 1


@pytest.mark.parametrize("n", [2, 6])
def test_gevp_tiny_mpmath(n):
    rng = np.random.default_rng(200 + n)
    A = rng.standard_normal((n, n))
    H = A + A.T
    B = rng.standard_normal((n, n))
    S = B @ B.T + 0.5 * np.eye(n)
    mpmath.mp.dps = 50
    Hm, Sm = mpmath.matrix(H.tolist()), mpmath.matrix(S.tolist())
    Lm = mpmath.cholesky(Sm)
    Li = Lm ** -1
    Am = Li * Hm * Li.T
    Am = (Am + Am.T) / 2
    wm = sorted(float(x) for x in mpmath.eigsy(Am, eigvals_only=True))
    ev, _, _ = O.gevp(H, S)
    assert np.abs(ev - np.array(wm)).max() < 1e-13 * max(1.0, np.abs(wm).max())


# ---------------------------------------------------------------------------
# occupations and chemical potential (Eq. (17), Eq. (18), Sec. 4.5)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [10, 64, 300])
def test_half_filled_chain_mu_is_zero(n):
    # even N, e0 = 0: the spectrum is symmetric about 0 and f(x) + f(-x) = 1,
    # so mu = 0 gives sum f = N/2 exactly
    k = np.arange(1, n + 1)
    eps = np.sort(2 * -1.0 * np.cos(k * np.pi / (n + 1)))
    f, mu, st = O.occupations(eps, n / 2, 0.05)
    assert st == 0
    assert abs(mu) < 1e-13
    assert abs(f.sum() - n / 2) < 1e-13


def test_fermi_dirac_values_and_limits():
    eps = np.array([-50.0, -0.1, 0.0, 0.1, 50.0, 1e4])
    f, mu, st = O.occupations(eps, 2.5, 0.1)
    x = (eps - mu) / 0.1
    expect = np.array([1.0 / (1.0 + math.exp(v)) if v < 700 else 0.0 for v in x])
    # the charge fix-up may lower the topmost occupied state(s) by the small surplus
    assert np.abs(f - expect).max() < 1e-12
    assert f.sum() == pytest.approx(2.5, abs=1e-14)
    assert f[-1] == 0.0 and f[0] == 1.0


def test_spin_factor_scales_occupations():
    eps = np.linspace(-1, 1, 21)
    f1, mu1, _ = O.occupations(eps, 5.0, 0.02, spin=1.0)
    f2, mu2, _ = O.occupations(eps, 10.0, 0.02, spin=2.0)
    assert mu1 == pytest.approx(mu2, abs=1e-12)
    np.testing.assert_allclose(f2, 2 * f1, atol=1e-12)


def test_bisection_step_limit_reports_status_4_and_fixes_charge():
    eps = np.linspace(-1, 1, 41)
    f, mu, st = O.occupations(eps, 7.3, 0.01, max_steps=1)
    assert st == 4
    assert abs(f.sum() - 7.3) < 1e-12   # surplus removed top-down after the bisection


def test_charge_fixup_removes_surplus_from_top():
    # widely spaced levels: at the converged mu the surplus sits in the lowest
    # partially occupied level, and after the fix-up sum f = N_e to rounding
    eps = np.array([-3.0, -2.0, -1.0, 0.0, 1.0, 2.0])
    f, mu, st = O.occupations(eps, 2.0, 1e-3, occ_accuracy=1e-2)
    assert st == 0
    assert abs(f.sum() - 2.0) <= 4 * np.finfo(float).eps
    assert np.all(np.diff(f) <= 0)


# ---------------------------------------------------------------------------
# density matrix (Eq. (9)) and band energy
# ---------------------------------------------------------------------------
def test_density_chain_closed_form():
    n = 30
    H = G.tight_binding_chain(n, 0.0, -1.0)
    r = O.dm(H, np.eye(n), n_electron=n / 2, kT=0.1)
    th = np.arange(1, n + 1) * np.pi / (n + 1)
    eps = -2.0 * np.cos(th)
    x = eps / 0.1
    f = 1.0 / (1.0 + np.exp(x))
    j = np.arange(1, n + 1)
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, np.arange(1, n + 1)) * np.pi / (n + 1))
    D = (V * f) @ V.T
    assert abs(r["mu"]) < 1e-13
    assert np.abs(r["D"] - D).max() < 1e-13
    assert r["energy"] == pytest.approx(float(np.sum(f * eps)), abs=1e-13)


def test_density_invariants_on_generated_system():
    sp = G.make_config(0)
    r = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    D, S, H, f, ev = r["D"], sp.S, sp.H, r["occ"], r["eval"]
    assert np.abs(D - D.T).max() < 1e-15
    assert np.trace(D @ S) == pytest.approx(sp.n_occ, abs=1e-10)
    assert f.sum() == pytest.approx(sp.n_occ, abs=1e-12)
    # tr(D H) = sum f eps (band energy)
    assert np.trace(D @ H) == pytest.approx(r["energy"], abs=1e-9)
    # D S c_l = f_l c_l
    _, C, _ = O.gevp(sp.H, sp.S)
    for l in [0, 50, 127, 128, 140, 300]:
        assert np.abs(D @ S @ C[:, l] - f[l] * C[:, l]).max() < 1e-9 * max(1, np.abs(C[:, l]).max())


def test_density_idempotent_for_integer_occupations():
    sp = G.make_config(0)
    ev, C, _ = O.gevp(sp.H, sp.S)
    nocc = int(sp.n_occ)
    assert ev[nocc] - ev[nocc - 1] > 1e-6
    f = np.zeros(sp.n)
    f[:nocc] = 1.0
    D = O.density(C, f)
    assert np.abs(D @ sp.S @ D - D).max() < 1e-9


# ---------------------------------------------------------------------------
# generated inputs: the oracle against an independent library route (LAPACK
# through SciPy) and the residual certificate
# ---------------------------------------------------------------------------
def test_generated_config0_vs_lapack_and_certificate():
    sp = G.make_config(0)
    ev, C, _ = O.gevp(sp.H, sp.S)
    ref = sl.eigh(sp.H, sp.S, eigvals_only=True, driver="gvd")
    rel = np.abs(ev - ref) / np.maximum(1.0, np.abs(ref))
    assert rel.max() < 1e-10
    # S-orthonormality
    assert np.abs(C.T @ sp.S @ C - np.eye(sp.n)).max() < 1e-8
    # residual certificate (Parlett, residual theorem after the L^-1 transform):
    # for x with x^T S x = 1 some eigenvalue lies within ||H x - lam S x||_{S^-1}
    # of lam; the S^-1 norm is taken through SciPy's own Cholesky factor
    k = 160
    R = sp.H @ C[:, :k] - (sp.S @ C[:, :k]) * ev[:k]
    Ls = sl.cholesky(sp.S, lower=True)
    bound = np.linalg.norm(sl.solve_triangular(Ls, R, lower=True), axis=0)
    assert bound.max() < 1e-10
    # and the plain 2-norm residual agrees with the extended-precision one
    res = O.residual_norms(sp.H, sp.S, C[:, :8], ev[:8])
    np.testing.assert_allclose(res, np.linalg.norm(R[:, :8], axis=0), rtol=0.5, atol=1e-12)
