"""The FP32-arithmetic products of the mixed mode (elsi_gpu_x_gemm_fp32).

Reference: the same product in FP64 of the operands rounded to FP32, so the
only difference left is FP32 accumulation.  Bound (round-to-nearest, unit
roundoff u = 2^-24, k products per entry): |C - C_ref| <= gamma_k |op(A)| |op(B)|
with gamma_k = k u / (1 - k u), times |alpha|.  The shapes span several
128 x 128 tiles with ragged tails in m, n and k, and every operand mode.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _dev_f(a):
    from paper_1705_11191_amd import binding as B

    a = np.asarray(a, dtype=np.float64)
    t = B.fortran_empty(a.shape[0], a.shape[1])
    t.copy_(torch.tensor(a, device="cuda"))
    return t


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
@pytest.mark.parametrize("m,n,k", [(300, 200, 129), (1030, 70, 513), (64, 300, 17), (385, 257, 1000)])
def test_gemm_fp32_vs_rounded_fp64(ta, tb, m, n, k):
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((k, m) if ta == "T" else (m, k))
    Bm = rng.standard_normal((n, k) if tb == "T" else (k, n))
    C0 = rng.standard_normal((m, n))
    alpha, beta = -0.75, 0.5
    opA = _r32(A).T if ta == "T" else _r32(A)
    opB = _r32(Bm).T if tb == "T" else _r32(Bm)
    ref = alpha * (opA @ opB) + beta * C0
    bound = abs(alpha) * (k * U32 / (1 - k * U32)) * (np.abs(opA) @ np.abs(opB)) + 1e-15 * np.abs(ref)
    C = _dev_f(C0)
    B.gemm_fp32(ta, tb, _dev_f(A), _dev_f(Bm), C, alpha, beta)
    got = C.cpu().numpy()
    assert np.all(np.abs(got - ref) <= bound)
    # the product really ran in FP32: it differs from the FP64 product of the unrounded operands
    exact = alpha * ((A.T if ta == "T" else A) @ (Bm.T if tb == "T" else Bm)) + beta * C0
    assert np.abs(got - exact).max() > 1e-9


@pytest.mark.parametrize("m,n", [(700, 64), (1100, 129)])
def test_gemm_fp32_symmetric_operand(m, n):
    """ta = 'S': only the lower triangle of A is read (the product Y = A22 V of step (1))."""
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(m + n)
    S = rng.standard_normal((m, m))
    S = (S + S.T) / 2
    A = np.tril(S) + np.triu(np.full((m, m), np.nan), 1)   # the upper part must never be read
    V = rng.standard_normal((m, n))
    ref = _r32(S) @ _r32(V)
    bound = (m * U32 / (1 - m * U32)) * (np.abs(_r32(S)) @ np.abs(_r32(V)))
    C = B.gemm_fp32("S", "N", _dev_f(A), _dev_f(V))
    got = C.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("n,k", [(600, 256), (1000, 128)])
def test_gemm_fp32_lower_triangle_update(n, k):
    """uplo = 1: the rank-k updates of step (1) write only i >= j."""
    from paper_1705_11191_amd import binding as B

    rng = np.random.default_rng(n + k)
    X = rng.standard_normal((n, k))
    Y = rng.standard_normal((n, k))
    C0 = rng.standard_normal((n, n))
    ref = C0 - _r32(X) @ _r32(Y).T
    bound = (k * U32 / (1 - k * U32)) * (np.abs(_r32(X)) @ np.abs(_r32(Y)).T)
    C = _dev_f(C0)
    B.gemm_fp32("N", "T", _dev_f(X), _dev_f(Y), C, -1.0, 1.0, uplo=1)
    got = C.cpu().numpy()
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.all(np.abs(got - ref)[low] <= bound[low])
    assert np.array_equal(got[~low], C0[~low])
