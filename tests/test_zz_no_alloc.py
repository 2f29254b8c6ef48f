"""The allocation-free Cholesky entry point against the allocating one.

elsi_gpu_x_cholesky_noalloc runs the same kernels as elsi_gpu_x_cholesky with
its scratch in a fixed device array, so its factor must equal the allocating
entry point's bit for bit.  Consecutive calls share that array: the second
call of each pair is smaller than the first (stale block inverses of the first
call stay beyond its end), and a failing factorization is followed by a
succeeding one (the pivot flag must have been cleared).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from synth import generator as G

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def _both(S):
    from paper_1705_11191_amd import binding as B

    A1, A2 = S.clone(), S.clone()
    f1 = B.cholesky(A1)
    f2 = B.cholesky_noalloc(A2)
    torch.cuda.synchronize()
    return f1, f2, A1, A2


def test_noalloc_cholesky_equals_allocating_entry_point_on_two_calls():
    """n = 1100 (one 1024-wide outer panel plus a ragged tail, 18 diagonal
    blocks), then n = 300 on the same scratch: identical factors, and the
    factor meets the oracle's to its forward-error scale."""
    for n, seed in ((1100, 3), (300, 4)):
        sp = G.make_lattice_system(n, seed=seed)
        f1, f2, A1, A2 = _both(_dev(sp.S))
        assert f1 == f2 == 0
        assert torch.equal(A1, A2), n
        L = A2.cpu().numpy().T   # the factor is written column-major into the row-major buffer
        Lr = O.potrf(sp.S)
        err = np.abs(np.tril(L) - np.tril(Lr)).max()
        assert err <= 1e-8 * np.abs(Lr).max(), (n, err)


def test_noalloc_cholesky_reports_a_bad_pivot_then_clears_it():
    """A matrix with a negative pivot at column 150 (1-based), then a smaller
    SPD matrix: the second call must succeed, so the flag was reset."""
    rng = np.random.default_rng(7)
    n = 400
    A = rng.standard_normal((n, n))
    S = A @ A.T / n + np.eye(n)
    S[149, 149] = -5.0
    f1, f2, A1, A2 = _both(_dev(S))
    assert f1 == f2 == 150
    sp = G.make_lattice_system(200, seed=5)
    g1, g2, B1, B2 = _both(_dev(sp.S))
    assert g1 == g2 == 0
    assert torch.equal(B1, B2)
