"""Pins of the oracle's broadening schemes (Sec. 4.6 broadening_scheme; Gaussian
broadening Eq. (21); Methfessel-Paxton orders 0 and 1 from Methfessel &
Paxton, Phys. Rev. B 40, 3616 (1989)) and of the chemical potential shared by
several problems (the k-point / spin sum of Sec. 4.5), each against something
that does not come from the oracle:

* values against 50-digit mpmath erfc / erf and the Hermite series
  S_N = S_0 + sum_n A_n H_{2n-1}(x) e^{-x^2}, A_n = (-1)^n / (n! 4^n sqrt(pi));
* the derivative of the order-1 step against -(A_0 H_0 + A_1 H_2) e^{-x^2};
* the moment property of the order-N approximation to the delta function
  D_N = -dS_N/dx: its moments of order 1..2N+1 vanish (the second moment of
  the Gaussian, N = 0, is 1/2 instead);
* f(x) + f(-x) = spin for every scheme, so a spectrum symmetric about 0 at
  half filling has mu = 0 exactly;
* the closed-form density matrix of the tight-binding chain with the
  (partly negative) order-1 occupations.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle as O
from synth import generator as G

SCHEMES = [O.FERMI, O.GAUSSIAN, O.MP0, O.MP1]
mpmath.mp.dps = 50


def _mp_step(scheme, x):
    x = mpmath.mpf(x)
    if scheme == O.FERMI:
        return 1 / (1 + mpmath.exp(x))
    s0 = (1 - mpmath.erf(x)) / 2            # Eq. (21) as printed
    if scheme in (O.GAUSSIAN, O.MP0):
        return s0
    a1 = mpmath.mpf(-1) / (4 * mpmath.sqrt(mpmath.pi))
    return s0 + a1 * mpmath.hermite(1, x) * mpmath.exp(-x * x)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("x", [-6.0, -2.5, -1.0, -0.3, 0.0, 0.4, 1.0, 2.2, 5.0])
def test_occupation_values_against_mpmath(scheme, x):
    width, spin, mu = 0.01, 2.0, -0.25
    got = O.occupation_value(scheme, mu + x * width, mu, width, spin)
    want = float(spin * _mp_step(scheme, x))
    assert abs(got - want) <= 2e-15 * max(1.0, abs(want)) + 1e-300


def test_order1_derivative_is_the_hermite_delta():
    a0 = 1 / math.sqrt(math.pi)
    a1 = -1 / (4 * math.sqrt(math.pi))
    h = 1e-5
    for x in np.linspace(-3, 3, 25):
        num = (O.occupation_value(O.MP1, x + h, 0.0, 1.0) - O.occupation_value(O.MP1, x - h, 0.0, 1.0)) / (2 * h)
        want = -(a0 * 1.0 + a1 * (4 * x * x - 2)) * math.exp(-x * x)
        assert abs(num - want) <= 1e-9


def _delta_moments(scheme, mmax):
    """Moments int x^m D(x) dx of D = -dS/dx, by Simpson's rule on the exact
    derivative taken from central differences of the oracle's step."""
    x = np.linspace(-9.0, 9.0, 36001)
    h = 1e-6
    D = np.array([-(O.occupation_value(scheme, t + h, 0.0, 1.0) - O.occupation_value(scheme, t - h, 0.0, 1.0))
                  / (2 * h) for t in x])
    dx = x[1] - x[0]
    w = np.ones_like(x)
    w[1:-1:2], w[2:-1:2] = 4, 2
    return [float(np.sum(w * D * x ** m) * dx / 3) for m in range(mmax + 1)]


def test_methfessel_paxton_moments():
    g = _delta_moments(O.GAUSSIAN, 3)
    m1 = _delta_moments(O.MP1, 3)
    assert abs(g[0] - 1) < 1e-8 and abs(g[1]) < 1e-8 and abs(g[2] - 0.5) < 1e-7 and abs(g[3]) < 1e-8
    assert abs(m1[0] - 1) < 1e-8 and max(abs(v) for v in m1[1:]) < 1e-7


@pytest.mark.parametrize("scheme", SCHEMES)
def test_symmetric_spectrum_at_half_filling_has_mu_zero(scheme):
    n = 64
    j = np.arange(1, n + 1)
    eps = np.sort(2.0 * np.cos(j * np.pi / (n + 1)))   # symmetric about 0
    f, mu, st = O.occupations(eps, n / 2, 0.05, scheme=scheme)
    assert st == 0
    assert abs(mu) <= 1e-12
    assert abs(f.sum() - n / 2) <= 1e-12
    # f(x) + f(-x) = spin pairs the states
    assert np.abs(f + f[::-1] - 1.0).max() <= 1e-12


@pytest.mark.parametrize("scheme", SCHEMES)
def test_electron_count_is_exact_after_the_fix_up(scheme):
    rng = np.random.default_rng(4 + scheme)
    eps = np.sort(rng.uniform(-1.0, 1.0, 300))
    f, mu, st = O.occupations(eps, 123.0, 0.02, spin=2.0, scheme=scheme)
    assert st == 0 and abs(f.sum() - 123.0) <= 1e-12


def test_shared_mu_over_weighted_problems():
    """Two problems with weights 1/2 each and N_e = 60: the electron count
    sum_l w_l f(eps_l) is exact, and two identical problems reproduce the
    single problem's mu with half its occupations."""
    rng = np.random.default_rng(9)
    a = np.sort(rng.uniform(-1, 1, 150))
    b = np.sort(rng.uniform(-0.8, 1.2, 150))
    w = np.r_[np.full(150, 0.5), np.full(150, 0.5)]
    f, mu, st = O.occupations(np.r_[a, b], 60.0, 0.01, weight=w)
    assert st == 0 and abs(f.sum() - 60.0) <= 1e-12
    fa = [O.occupation_value(O.FERMI, e, mu, 0.01) for e in a]
    assert np.abs(f[:150] - 0.5 * np.array(fa)).max() <= 1e-12
    f1, mu1, _ = O.occupations(a, 60.0, 0.01)
    f2, mu2, _ = O.occupations(np.r_[a, a], 60.0, 0.01, weight=w)
    assert abs(mu2 - mu1) <= 1e-14
    assert np.abs(f2[:150] - 0.5 * f1).max() <= 1e-13


def test_density_matrix_with_negative_occupations_closed_form():
    """The chain (S = I): D_ij = sum_k f_k (2/(N+1)) sin(i th_k) sin(j th_k)
    with the order-1 occupations, some of them negative."""
    n, ne, width = 40, 17, 0.15
    H = G.tight_binding_chain(n, 0.0, -1.0)
    r = O.dm(H, np.eye(n), ne, width, scheme=O.MP1)
    f = r["occ"]
    assert f.min() < -1e-4                     # the scheme does produce negative occupations
    th = np.arange(1, n + 1) * np.pi / (n + 1)
    lam = -2.0 * np.cos(th)
    order = np.argsort(lam)
    i = np.arange(1, n + 1)[:, None]
    V = np.sqrt(2.0 / (n + 1)) * np.sin(i * th[None, :])[:, order]
    Dcf = (V * f) @ V.T
    assert np.abs(r["D"] - Dcf).max() <= 1e-12
    assert abs(np.trace(r["D"]) - ne) <= 1e-12
