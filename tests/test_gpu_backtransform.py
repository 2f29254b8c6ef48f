"""The back-transformations of steps (4) and (5) and their transposes, and the
size branches that only the large workloads reach on their own.

Q = Q1 Q2 is formed explicitly by applying it to the identity; that Q must be
orthogonal and must tridiagonalize the input (Q^T A Q = T with the returned d
and e), which pins it without reference to the kernels.  Every other
application -- each Q2 column-slab width (128, 256 and 512 columns per
workgroup, each chosen explicitly, and the automatic choice), and the
transposed products Q^T X the mixed mode's refinement uses -- must then equal
NumPy's product with that explicit Q.  Tolerances: products of an orthogonal
matrix with unit-scale columns, 32 n eps.
"""
import numpy as np
import pytest

import oracle as O
from synth import generator as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
N, BW = 1100, 64


def _dev_f(a):
    from paper_1705_11191_amd import binding as B

    a = np.asarray(a, dtype=np.float64)
    t = B.fortran_empty(a.shape[0], a.shape[1])
    t.copy_(torch.tensor(a, device="cuda"))
    return t


@pytest.fixture(scope="module")
def explicit_q():
    from paper_1705_11191_amd import binding as B

    sp = G.make_lattice_system(N, seed=1100)
    A = O.reduce_standard(sp.H, O.potrf(sp.S))
    Ad = torch.tensor(A, device="cuda")
    X = _dev_f(np.eye(N))
    d, e = B.backtransform(Ad, BW, X)
    return A, Ad, X.cpu().numpy(), d.cpu().numpy(), e.cpu().numpy()


def test_explicit_q_is_orthogonal_and_tridiagonalizes(explicit_q):
    A, _, Q, d, e = explicit_q
    assert np.abs(Q.T @ Q - np.eye(N)).max() <= 32 * N * EPS
    T = Q.T @ A @ Q
    scale = np.abs(np.linalg.eigvalsh(A)).max()
    band = np.triu(np.tril(T, 1), -1)
    assert np.abs(T - band).max() <= 64 * N * EPS * scale
    assert np.abs(np.diag(T) - d).max() <= 64 * N * EPS * scale
    assert np.abs(np.diag(T, -1) - e).max() <= 64 * N * EPS * scale


@pytest.mark.parametrize("slab,ncol", [(0, 8200), (512, 8200), (256, 8200), (128, 8200), (256, 2100), (0, 300)])
@pytest.mark.parametrize("trans", [False, True])
def test_every_slab_width_and_the_transpose_match_the_explicit_q(explicit_q, slab, ncol, trans):
    from paper_1705_11191_amd import binding as B

    A, Ad, Q, _, _ = explicit_q
    rng = np.random.default_rng(ncol + slab + int(trans))
    X0 = rng.standard_normal((N, ncol)) / np.sqrt(N)
    X = _dev_f(X0)
    print(f"[backtransform] n={N} ncol={ncol} slab={slab} trans={trans}", flush=True)
    B.backtransform(Ad, BW, X, trans=trans, slab=slab)
    want = (Q.T if trans else Q) @ X0
    err = np.abs(X.cpu().numpy() - want).max()
    assert err <= 32 * N * EPS * np.abs(X0).max(), err


def test_transposed_application_inverts_the_forward_one(explicit_q):
    from paper_1705_11191_amd import binding as B

    _, Ad, _, _, _ = explicit_q
    rng = np.random.default_rng(5)
    X0 = rng.standard_normal((N, 700))
    X = _dev_f(X0)
    B.backtransform(Ad, BW, X)
    B.backtransform(Ad, BW, X, trans=True)
    assert np.abs(X.cpu().numpy() - X0).max() <= 64 * N * EPS * np.abs(X0).max()


@pytest.mark.parametrize("ta", ["N", "T"])
@pytest.mark.parametrize("m,n,k", [(16384 + 77, 64, 300), (20000, 40, 129)])
def test_tall_products_take_the_128x64_tiles(ta, m, n, k):
    """n <= 64 with m >= 16384 selects the 128 x 64 tile instance, otherwise
    reached only at the full-size workloads; ragged m and k."""
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(m + n + k)
    A0 = rng.standard_normal((m, k) if ta == "N" else (k, m))
    B0 = rng.standard_normal((k, n))
    C = B.dgemm(ta, "N", _dev_f(A0), _dev_f(B0))
    want = (A0 if ta == "N" else A0.T) @ B0
    assert np.abs(C.cpu().numpy() - want).max() <= 8 * k * EPS * np.abs(A0).max() * np.abs(B0).max()
