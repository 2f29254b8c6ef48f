"""The seeded input generator: determinism, structure and the conditioning reading."""
import math

import numpy as np
import pytest

from synth import generator as G


def test_chain_config_shape_and_determinism():
    a = G.make_config(0, seed=0)
    b = G.make_config(0, seed=0)
    c = G.make_config(0, seed=1)
    assert a.n == 512 and a.n_occ == 128 and a.kT == 0.01
    np.testing.assert_array_equal(a.H, b.H)
    np.testing.assert_array_equal(a.S, b.S)
    assert np.abs(a.H - c.H).max() > 0


def test_matrices_symmetric_and_diagonals():
    sp = G.make_config(0)
    np.testing.assert_array_equal(sp.H, sp.H.T)
    np.testing.assert_array_equal(sp.S, sp.S.T)
    # normalized s-Gaussians: S_lit,ii = 1, shifted by sigma
    np.testing.assert_allclose(np.diag(sp.S), 1.0 + sp.meta["sigma"], rtol=0, atol=1e-15)
    # on-site energies are in [-15, -5] eV
    h = np.diag(sp.H) / G.HARTREE_PER_EV
    assert h.min() >= -15 and h.max() <= -5


def test_extended_hueckel_offdiagonal_rule():
    sp = G.make_config(0)
    h = np.diag(sp.H)
    i, j = 3, 7
    assert sp.H[i, j] == pytest.approx(1.75 * sp.S[i, j] * (h[i] + h[j]) / 2, rel=1e-15)


def test_condition_number_reading():
    sp = G.make_config(0)
    w = np.linalg.eigvalsh(sp.S)
    assert w[0] > 0
    assert w[-1] / w[0] == pytest.approx(1e6, rel=0.02)


def test_gaussian_overlap_closed_form_two_centres():
    c = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, -0.2]])
    al = np.array([0.7, 1.9])
    S = G.s_gaussian_overlap(c, al)
    a, b = al
    d2 = float(((c[0] - c[1]) ** 2).sum())
    ref = (2 * math.sqrt(a * b) / (a + b)) ** 1.5 * math.exp(-a * b / (a + b) * d2)
    assert S[0, 1] == pytest.approx(ref, rel=1e-15)
    assert S[0, 0] == pytest.approx(1.0, rel=1e-15)


def test_lattice_system_truncation_and_sites():
    sp = G.make_lattice_system(100, seed=3)
    assert sp.n == 100 and sp.meta["n_atoms"] == 7 and sp.n_occ == 25
    pos = G.lattice_positions(547, 2.5, np.zeros((547, 3)))
    assert pos.shape == (547, 3)
    np.testing.assert_array_equal(pos[1], [2.5, 0, 0])
    np.testing.assert_array_equal(pos[9], [0, 2.5, 0])     # m = 9 for 547 atoms
    np.testing.assert_array_equal(pos[81], [0, 0, 2.5])


def test_batch_sizes_range_and_multiple():
    n = G.batch_sizes()
    assert n.shape == (256,)
    assert n.min() >= 255 and n.max() <= 4095
    assert np.all(n % 15 == 0)
    np.testing.assert_array_equal(n, G.batch_sizes())
