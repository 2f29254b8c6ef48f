"""Pins of the oracle's FP64 refinement (CholeskyQR twice, Rayleigh-Ritz,
residuals, and the Newton correction through an approximate factorization
Q T Q^T) against facts that do not come from the oracle itself:

* the closed-form spectrum and eigenvectors of the tridiagonal Toeplitz matrix
  tridiag(t, e0, t): lambda_j = e0 + 2 t cos(j pi / (n + 1)),
  v_j(i) = sin(i j pi / (n + 1));
* the residual bound for symmetric matrices: a unit vector x with Rayleigh
  quotient theta has an eigenvalue within ||A x - theta x||_2;
* Ritz values from a subspace close to the lowest invariant subspace converge
  quadratically in its distance, the residuals linearly;
* CholeskyQR twice leaves the columns orthonormal to rounding even for a
  badly conditioned start;
* Rayleigh-Ritz alone never moves the subspace (the projector onto span(X) is
  the same before and after);
* with an exact factorization the correction equation on the complement is
  solved exactly: the complement component x - Z Z^T x of every vector is
  removed in one step, whatever its size (r = (T - theta) x and the
  complement projector commutes with T);
* with a perturbed T the subspace error contracts per sweep by the
  perturbation over the spectral gap (linear convergence, rate linear in the
  perturbation);
* Gaussian elimination with partial pivoting is backward stable.
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
    X, theta, res, _, sweeps, st = O.refine(Ht, X0, k, tol=1e-11, max_sweeps=4)
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
    X, theta, res, _, sweeps, st = O.refine(A, X0, k, tol=0.0, max_sweeps=1)
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
        X, theta, res, _, sweeps, st = O.refine(Ht, V[:, :k] + delta * E, k, tol=0.0, max_sweeps=1)
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
    X, theta, res, _, sweeps, st = O.refine(A, X0, k, tol=0.0, max_sweeps=1)
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-13


def test_stop_rules():
    n, k = 50, 5
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    lam, V = _chain_closed_form(n, 0.0, 1.0)
    rng = np.random.default_rng(5)
    X0 = V[:, :k] + 1e-4 * rng.standard_normal((n, k))
    # without a factorization there is one Rayleigh-Ritz sweep at most
    # no sweeps: not converged, X untouched
    X, theta, res, _, sweeps, st = O.refine(Ht, X0, k, tol=1e-10, max_sweeps=0)
    assert st == 3 and sweeps == 0 and np.array_equal(X, X0)
    # Rayleigh-Ritz does not change the subspace, so a second sweep could not
    # lower the residual: stop after the first one, not converged
    X, theta, res, _, sweeps, st = O.refine(Ht, X0, k, tol=1e-14, max_sweeps=4)
    assert st == 3 and sweeps == 1
    # ... and a second call on its output reproduces the same Ritz values
    X2, theta2, res2, _, sweeps2, st2 = O.refine(Ht, X, k, tol=1e-14, max_sweeps=4)
    assert np.abs(theta2 - theta).max() <= 1e-14 and np.allclose(res2, res, rtol=1e-6, atol=1e-15)
    # a loose tolerance is met after one sweep
    X, theta, res, _, sweeps, st = O.refine(Ht, X0, k, tol=1e-2, max_sweeps=4)
    assert st == 0 and sweeps == 1
    # only the first kw states decide
    X, theta, res, _, sweeps, st = O.refine(Ht, V[:, :k], 0, tol=0.0, max_sweeps=3)
    assert st == 0 and sweeps == 1


@pytest.mark.parametrize("n", [120])
def test_dependent_columns_report_failure(n):
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    rng = np.random.default_rng(6)
    # a zero column makes the Gram matrix singular with an exactly zero pivot
    X0 = np.hstack([rng.standard_normal((n, 1)), np.zeros((n, 1)), rng.standard_normal((n, 1))])
    X, theta, res, _, sweeps, st = O.refine(Ht, X0, 3, tol=1e-10, max_sweeps=2)
    assert st == 3 and sweeps == 0


def _angle(V, k, X):
    """Largest canonical angle (sine) between span(X) and span(V[:, :k])."""
    Qx, _ = np.linalg.qr(X)
    return np.linalg.norm(V[:, k:].T @ Qx, 2)


def test_rayleigh_ritz_alone_leaves_the_span_unchanged():
    n, k = 80, 10
    rng = np.random.default_rng(21)
    A = rng.standard_normal((n, n))
    A = (A + A.T) / 2
    X0 = rng.standard_normal((n, k))
    X, theta, res, step, sweeps, st = O.refine(A, X0, k, tol=0.0, max_sweeps=3)
    assert sweeps == 1 and st == 3 and np.all(step == 0.0)
    Q0, _ = np.linalg.qr(X0)
    assert np.abs(X @ X.T - Q0 @ Q0.T).max() < 1e-13


@pytest.mark.parametrize("delta", [1e-2, 1e-4])
def test_exact_factorization_removes_the_complement_in_one_step(delta):
    n, k = 60, 8
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    lam, V = _chain_closed_form(n, 0.0, 1.0)
    d, e = np.zeros(n), np.ones(n - 1)
    rng = np.random.default_rng(22)
    X0 = V[:, :k] + delta * (V[:, k:] @ rng.standard_normal((n - k, k)))
    assert _angle(V, k, X0) > 0.5 * delta
    # one correction already lands on the subspace: the second measured step is
    # at rounding level, it is taken, and a closing Rayleigh-Ritz sweep follows
    X, theta, res, step, sweeps, st = O.refine(Ht, X0, k, tol=1e-12, max_sweeps=3, Q=np.eye(n), d=d, e=e)
    assert sweeps == 3 and st == 0 and step.max() < 1e-12
    # with two sweeps there is no room for the closing one: not converged, and
    # the single correction has still removed the complement
    X2, *_, sweeps2, st2 = O.refine(Ht, X0, k, tol=1e-12, max_sweeps=2, Q=np.eye(n), d=d, e=e)
    assert sweeps2 == 2 and st2 == 3 and _angle(V, k, X2) < 1e-13
    assert _angle(V, k, X) < 1e-13
    assert np.abs(theta - lam[:k]).max() < 1e-13


def test_exact_factorization_through_a_general_orthogonal_basis():
    """Ht = Q T Q^T with a random orthogonal Q (not symmetric): the step must
    map the residual with Q^T and back with Q; with Q^T in place of Q the
    subspace does not converge."""
    n, k = 60, 8
    T = G.tight_binding_chain(n, 0.0, 1.0)
    lam, V = _chain_closed_form(n, 0.0, 1.0)
    d, e = np.zeros(n), np.ones(n - 1)
    rng = np.random.default_rng(23)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ T @ Q.T
    X0 = Q @ (V[:, :k] + 1e-3 * (V[:, k:] @ rng.standard_normal((n - k, k))))
    X, theta, res, step, sweeps, st = O.refine(A, X0, k, tol=1e-12, max_sweeps=3, Q=Q, d=d, e=e)
    assert st == 0 and _angle(V, k, Q.T @ X) < 1e-13
    assert np.abs(theta - lam[:k]).max() < 1e-13
    Xw, *_ = O.refine(A, X0, k, tol=0.0, max_sweeps=2, Q=Q.T, d=d, e=e)
    assert _angle(V, k, Q.T @ Xw) > 1e-4


def test_perturbed_factorization_contracts_linearly_in_its_error():
    n, k = 60, 8
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    lam, V = _chain_closed_form(n, 0.0, 1.0)
    gap = lam[k] - lam[k - 1]
    e = np.ones(n - 1)
    rng = np.random.default_rng(24)
    g = rng.standard_normal(n)
    X0 = V[:, :k] + 1e-2 * (V[:, k:] @ rng.standard_normal((n - k, k)))
    worst = {}
    for eta in (1e-3, 1e-5):
        dp = eta * g                      # T' = T + eta diag(g)
        angles = []
        for ms in (1, 2, 3):
            X, *_ = O.refine(Ht, X0, k, tol=0.0, max_sweeps=ms, Q=np.eye(n), d=dp, e=e)
            angles.append(_angle(V, k, X))
        rates = [angles[i + 1] / angles[i] for i in range(2)]
        bound = eta * np.abs(g).max() / gap
        assert max(rates) <= bound, (eta, rates, bound)
        worst[eta] = max(rates)
    # the rate scales with the perturbation
    assert worst[1e-5] < 0.05 * worst[1e-3]
    # ... and the refinement reaches its tolerance and says so
    X, theta, res, step, sweeps, st = O.refine(Ht, X0, k, tol=1e-12, max_sweeps=6, Q=np.eye(n),
                                               d=1e-5 * g, e=e)
    assert st == 0 and sweeps <= 5 and np.abs(theta - lam[:k]).max() < 1e-13


def test_weights_decide_which_steps_count():
    n, k = 50, 6
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    lam, V = _chain_closed_form(n, 0.0, 1.0)
    rng = np.random.default_rng(25)
    X0 = V[:, :k] + 1e-3 * (V[:, k:] @ rng.standard_normal((n - k, k)))
    d, e = np.zeros(n), np.ones(n - 1)
    # zero weights: the first measured step already meets any tolerance; it is
    # taken and one closing sweep follows
    X, theta, res, step, sweeps, st = O.refine(Ht, X0, k, tol=0.0, max_sweeps=4, Q=np.eye(n), d=d, e=e,
                                               weight=np.zeros(k))
    assert st == 0 and sweeps == 2 and step.max() > 1e-5
    # one sweep allowed and a step above tol: not converged, the correction is not applied
    X1, theta1, res1, step1, sweeps1, st1 = O.refine(Ht, X0, k, tol=1e-12, max_sweeps=1, Q=np.eye(n), d=d, e=e)
    assert st1 == 3 and sweeps1 == 1
    Q0, _ = np.linalg.qr(X0)
    assert np.abs(X1 @ X1.T - Q0 @ Q0.T).max() < 1e-13


def test_tridiagonal_shifted_solve_is_backward_stable():
    rng = np.random.default_rng(26)
    n = 70
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    w = np.linalg.eigvalsh(T)
    for s in (0.3, w[10] + 1e-9, w[0] - 0.5):
        b = rng.standard_normal(n)
        x = O.tridiag_shift_solve(d, e, s, b)
        A = T - s * np.eye(n)
        assert np.abs(A @ x - b).max() <= 64 * np.finfo(float).eps * np.abs(A).sum(1).max() * np.abs(x).max()
        if s == 0.3:
            assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-10 * np.abs(x).max()
    # a zero leading diagonal forces the row exchange at the first step
    d0 = np.zeros(4)
    e0 = np.array([1.0, 2.0, 3.0])
    b = np.array([1.0, -2.0, 0.5, 4.0])
    x = O.tridiag_shift_solve(d0, e0, 0.0, b)
    A = np.diag(e0, 1) + np.diag(e0, -1)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-14, atol=1e-14)
    # an exactly singular matrix gets the tiny-pivot guard: finite result
    x = O.tridiag_shift_solve(np.zeros(2), np.zeros(1), 0.0, np.array([1.0, 1.0]))
    assert np.all(np.isfinite(x))


def test_measured_contraction_closes_the_refinement_early():
    """The closing sweep also follows a step W_s > tol when the contraction
    measured over the last two steps predicts that taking it leaves less than
    tol (10 (W_s / W_{s-1}) W_s <= tol); the subspace then still meets tol."""
    n, k = 60, 8
    Ht = G.tight_binding_chain(n, 0.0, 1.0)
    lam, V = _chain_closed_form(n, 0.0, 1.0)
    rng = np.random.default_rng(24)
    g = rng.standard_normal(n)
    X0 = V[:, :k] + 1e-2 * (V[:, k:] @ rng.standard_normal((n - k, k)))
    tol = 1e-12
    X, theta, res, step, sweeps, st = O.refine(Ht, X0, k, tol=tol, max_sweeps=8, Q=np.eye(n), d=1e-5 * g,
                                               e=np.ones(n - 1))
    assert st == 0 and sweeps == 4
    assert step.max() > tol                   # the last measured step itself was above tol ...
    assert _angle(V, k, X) <= tol             # ... and taking it left the subspace within tol
    assert np.abs(theta - lam[:k]).max() < 1e-13
