"""Stage-by-stage parity of the HIP path against the CPU oracle (through the C ABI).

Sizes span several 64/128/256-wide tiles and ragged tails.  Tolerances are
stated per test from the arithmetic: FP64 products accumulate rounding of
order k * eps * |A||B|; solves with L amplify it by cond(L).
"""
import math

import numpy as np
import pytest

import oracle as O
from synth import generator as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _fortran(a):
    from paper_1705_11191_amd.binding import fortran_empty

    t = fortran_empty(a.shape[0], a.shape[1])
    t.copy_(torch.tensor(a, dtype=torch.float64))
    return t


def _spd(n, seed, shift=1.0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    return B @ B.T / n + shift * np.eye(n)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 16), (130, 70, 33), (257, 300, 129),
                                   (512, 40, 700), (33, 513, 5), (200, 200, 0)])
def test_dgemm_all_transposes(ta, tb, m, n, k):
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((k, m) if ta == "T" else (m, k))
    Bm = rng.standard_normal((n, k) if tb == "T" else (k, n))
    C0 = rng.standard_normal((m, n))
    opA = A.T if ta == "T" else A
    opB = Bm.T if tb == "T" else Bm
    ref = 0.7 * opA @ opB - 1.3 * C0
    C = _fortran(C0)
    B.dgemm(ta, tb, _fortran(A), _fortran(Bm), C, alpha=0.7, beta=-1.3)
    got = C.cpu().numpy()
    tol = 4 * max(k, 1) * EPS * (np.abs(opA) @ np.abs(opB)).max() + 8 * EPS * np.abs(C0).max()
    assert np.abs(got - ref).max() <= tol


@pytest.mark.parametrize("m,n", [(1, 1), (63, 64), (130, 70), (300, 64), (517, 33), (1030, 64)])
def test_dgemm_symmetric_lower(m, n):
    """op(A) = the symmetric matrix held in A's lower triangle; the strict upper
    triangle holds NaN and must never be read."""
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(m + 11 * n)
    G = rng.standard_normal((m, m))
    Asym = G + G.T
    A = np.tril(Asym) + np.triu(np.full((m, m), np.nan), 1)
    Bm = rng.standard_normal((m, n))
    C0 = rng.standard_normal((m, n))
    ref = 0.7 * Asym @ Bm - 1.3 * C0
    C = _fortran(C0)
    B.dgemm("S", "N", _fortran(A), _fortran(Bm), C, alpha=0.7, beta=-1.3)
    got = C.cpu().numpy()
    tol = 4 * m * EPS * (np.abs(Asym) @ np.abs(Bm)).max() + 8 * EPS * np.abs(C0).max()
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() <= tol


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 130, 257, 300, 513, 1300])
def test_cholesky_vs_oracle(n):
    from paper_1705_11191_amd import binding as B

    S = _spd(n, n)
    L_ref = O.potrf(S)
    St = _dev(S)
    assert B.cholesky(St) == 0
    L = St.cpu().numpy().T   # back to column-major reading
    # the strict upper triangle is zeroed; lower triangle matches to rounding
    assert np.abs(np.triu(L, 1)).max() == 0.0
    # tol: Cholesky forward error ~ n eps cond(S)^(1/2) |L|
    cond = np.linalg.cond(S)
    assert np.abs(L - L_ref).max() <= 8 * n * EPS * math.sqrt(cond) * np.abs(L_ref).max()


def test_cholesky_reports_first_bad_pivot():
    from paper_1705_11191_amd import binding as B

    S = _spd(200, 3)
    S[150, 150] = -5.0
    St = _dev(S)
    assert B.cholesky(St) == 151


@pytest.mark.parametrize("n", [3, 64, 129, 300, 700, 1100, 1600])
def test_reduce_vs_oracle(n):
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    H = A + A.T
    S = _spd(n, n + 1, shift=0.1)
    L = O.potrf(S)
    ref = O.reduce_standard(H, L)
    # column-major H whose strict upper triangle must not be read
    Ht = _fortran(np.tril(H) + np.triu(np.full((n, n), np.nan), 1))
    B.reduce_standard(Ht, _fortran(L))
    got = Ht.cpu().numpy()
    assert np.abs(got - got.T).max() == 0.0
    condL = np.linalg.cond(L)
    assert np.abs(got - ref).max() <= 16 * n * EPS * condL ** 2 * np.abs(H).max()


@pytest.mark.parametrize("n,k", [(5, 3), (130, 64), (300, 257)])
def test_backsub_vs_oracle(n, k):
    from paper_1705_11191_amd import binding as B

    S = _spd(n, 2 * n)
    L = O.potrf(S)
    rng = np.random.default_rng(k)
    Z = rng.standard_normal((n, k))
    ref = O.backsub(L, Z)
    X = _fortran(Z)
    B.backsub(_fortran(L), X)
    got = X.cpu().numpy()
    condL = np.linalg.cond(L)
    assert np.abs(got - ref).max() <= 16 * n * EPS * condL * np.abs(ref).max()


@pytest.mark.parametrize("n,ne,kT", [(10, 5.0, 0.05), (512, 128.0, 0.01), (3000, 750.5, 0.02)])
def test_occupations_vs_oracle(n, ne, kT):
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(n)
    eps = np.sort(rng.uniform(-1.0, 1.0, n))
    f_ref, mu_ref, st_ref = O.occupations(eps, ne, kT)
    f, mu, ks, st = B.occupations(_dev(eps), ne, kT)
    f = f.cpu().numpy()
    assert st == st_ref == 0
    # summation order differs (tree vs sequential): mu agrees to the count's rounding / slope
    assert abs(mu - mu_ref) <= 1e-12
    assert np.abs(f - f_ref).max() <= 1e-10
    assert abs(f.sum() - ne) <= 1e-12 * max(1.0, ne)
    assert ks == int(np.sum(f > 1e-20))


def test_occupations_step_limit_status():
    from paper_1705_11191_amd import binding as B

    eps = np.linspace(-1, 1, 41)
    f, mu, ks, st = B.occupations(_dev(eps), 7.3, 0.01, max_steps=1)
    assert st == 4
    assert abs(f.cpu().numpy().sum() - 7.3) < 1e-12


@pytest.mark.parametrize("n,k", [(1, 1), (100, 37), (300, 150), (513, 200)])
def test_density_vs_oracle(n, k):
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(n + k)
    C = rng.standard_normal((n, k))
    f = np.sort(rng.uniform(0, 1, k))[::-1].copy()
    ref = O.density(C, f)
    D = B.density(_fortran(C), _dev(f)).cpu().numpy()
    assert np.abs(D - D.T).max() == 0.0
    assert np.abs(D - ref).max() <= 4 * k * EPS * (np.abs(C) ** 2 @ f).max()
