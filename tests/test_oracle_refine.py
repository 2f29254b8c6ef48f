"""Pins of the oracle's FP64 refinement (CholeskyQR twice, Rayleigh-Ritz,
residual norms) against facts that do not come from the oracle itself:

* the closed-form spectrum and eigenvectors of the tridiagonal Toeplitz matrix
  tridiag(t, e0, t): lambda_j = e0 + 2 t cos(j pi / (n + 1)),
  v_j(i) = sin(i j pi / (n + 1));
* the residual bound for symmetric matrices: a unit vector x with Rayleigh
  quotient theta has an eigenvalue within ||A x - theta x||_2;
* Ritz values from a subspace close to the lowest invariant subspace converge
  quadratically in its distance, the residuals linearly;
* CholeskyQR twice leaves the columns orthonormal to rounding even for a
  badly conditioned start.
"""
import numpy as np
import pytest

import oracle as O
from synth import generator as G


def _chain_closed_form(n, e0, t):
    j = np.arange(1, n + 1)
    lam = e0 + 2.0 * t * np.cos(j * np.pi / (n + 1))
    i = np.arange(1, n + 1)[:, None]
    V = np.sin(i * j[None, :] * np.pi / (n + 1)) * np.sqrt(2.0 / (n + 1))
    order = np.argsort(lam)
    return lam[order], V[:, order]


def test_exact_subspace_gives_closed_form_values_in_one_sweep():
    n, k = 60, 9
    e0, t = 0.3, -1.0
    Ht = G.tight_binding_chain(n, e0, t)
    lam, V = _chain_closed_form(n, e0, t)
    rng = np.random.default_rng(1)
    M = rng.standard_normal((k, k)) + 3 * np.eye(k)   # nonsingular mixing
    X0 = V[:, :k] @ M
    X, theta, res, sweeps, st = O.refine(Ht, X0, k, tol=1e-11, max_sweeps=4)
    assert st == 0 and sweeps == 1
    assert np.abs(theta - lam[:k]).max() < 1e-13
    assert res.max() < 1e-12
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-13
    # each refined vector is the closed-form eigenvector up to sign
    overlap = np.abs(np.sum(X * V[:, :k], axis=0))
    assert np.abs(overlap - 1.0).max() < 1e-12


def test_every_ritz_value_lies_within_its_residual_of_the_spectrum():
    n, k = 80, 12
    rng = np.random.default_rng(2)
    A = rng.standard_normal((n, n))
    A = (A + A.T) / 2
    lam = np.linalg.eigvalsh(A)
    X0 = rng.standard_normal((n, k))
    X, theta, res, sweeps, st = O.refine(A, X0, k, tol=0.0, max_sweeps=1)
    assert sweeps == 1 and st == 3
    for th, r in zip(theta, res):
        assert np.abs(lam - th).min() <= r * (1 + 1e-12) + 1e-13
    # the residual is the definition, recomputed here by plain products
    R = A @ X - X * theta
    assert np.allclose(np.linalg.norm(R, axis=0), res, rtol=1e-12, atol=1e-13)
    # Ritz values are ascending and bounded below by the exact ones (Cauchy interlacing)
    assert np.all(np.diff(theta) >= 0)
    assert np.all(theta >= lam[:k] - 1e-12)


def test_quadratic_eigenvalue_convergence_linear_residual():
    n, k = 70, 6
    e0, t = 0.0, 1.0
    Ht = G.tight_binding_chain(n, e0, t)
    lam, V = _chain_closed_form(n, e0, t)
    rng = np.random.default_rng(3)
    E = rng.standard_normal((n, k))
    errs, rs = [], []
    for delta in (1e-3, 1e-4):
        X, theta, res, sweeps, st = O.refine(Ht, V[:, :k] + delta * E, k, tol=0.0, max_sweeps=1)
        errs.append(np.abs(theta - lam[:k]).max())
        rs.append(res.max())
    assert 30 < errs[0] / errs[1] < 300      # ~ delta^2
    assert 3 < rs[0] / rs[1] < 30            # ~ delta


def test_cholesky_qr_twice_orthonormalizes_ill_conditioned_start():
    n, k = 200, 10
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    X0 = Q @ np.diag(np.logspace(0, -6, k)) @ np.linalg.qr(rng.standard_normal((k, k)))[0]
    A = np.diag(np.linspace(-1, 1, n))
    X, theta, res, sweeps, st = O.refine(A, X0, k, tol=0.0, max_sweeps=1)
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-13


def test_stop_rules():
    n, k = 50, 5
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    lam, V = _chain_closed_form(n, 0.0, 1.0)
    rng = np.random.default_rng(5)
    X0 = V[:, :k] + 1e-4 * rng.standard_normal((n, k))
    # no sweeps: not converged, X untouched
    X, theta, res, sweeps, st = O.refine(Ht, X0, k, tol=1e-10, max_sweeps=0)
    assert st == 3 and sweeps == 0 and np.array_equal(X, X0)
    # Rayleigh-Ritz does not change the subspace, so a second sweep could not
    # lower the residual: stop after the first one, not converged
    X, theta, res, sweeps, st = O.refine(Ht, X0, k, tol=1e-14, max_sweeps=4)
    assert st == 3 and sweeps == 1
    # ... and a second call on its output reproduces the same Ritz values
    X2, theta2, res2, sweeps2, st2 = O.refine(Ht, X, k, tol=1e-14, max_sweeps=4)
    assert np.abs(theta2 - theta).max() <= 1e-14 and np.allclose(res2, res, rtol=1e-6, atol=1e-15)
    # a loose tolerance is met after one sweep
    X, theta, res, sweeps, st = O.refine(Ht, X0, k, tol=1e-2, max_sweeps=4)
    assert st == 0 and sweeps == 1
    # only the first kw states decide
    X, theta, res, sweeps, st = O.refine(Ht, V[:, :k], 0, tol=0.0, max_sweeps=3)
    assert st == 0 and sweeps == 1


@pytest.mark.parametrize("n", [120])
def test_dependent_columns_report_failure(n):
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    rng = np.random.default_rng(6)
    # a zero column makes the Gram matrix singular with an exactly zero pivot
    X0 = np.hstack([rng.standard_normal((n, 1)), np.zeros((n, 1)), rng.standard_normal((n, 1))])
    X, theta, res, sweeps, st = O.refine(Ht, X0, 3, tol=1e-10, max_sweeps=2)
    assert st == 3 and sweeps == 0
