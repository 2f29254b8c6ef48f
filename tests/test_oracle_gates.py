"""The eigenvalue gate of the parity tests (tests/gates.py) is relaxed for
unoccupied states above 1 Ha, where the near-singular directions of S make
every FP64 solver noisy; states that enter the density matrix keep the plain
1e-10 relative gate whatever their size.  These CPU checks pin both halves on
the pencils the GPU parity tests use: an independent FP64 solver (LAPACK,
scipy.linalg.eigh on the same pencil) passes the gate against the oracle,
with room to spare on the occupied states; the relaxation is not vacuous (the
kappa = 1e6 pencils have large eigenvalues); and an error of the size the
relaxation would forgive fails the gate when the state is occupied."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from gates import EPS, eig_excess, overlap_condition
from synth import generator as G


def _pencils():
    yield "config0", G.make_config(0)
    for n, seed in [(257, 21), (300, 7), (400, 11), (700, 800)]:
        yield f"lattice{n}", G.make_lattice_system(n, seed=seed)
    yield "lattice700_kappa1e2", G.make_lattice_system(700, seed=800, kappa=1e2)


@pytest.mark.parametrize("name,sp", list(_pencils()), ids=lambda x: x if isinstance(x, str) else "")
def test_independent_solver_passes_the_gate(name, sp):
    ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    ev, f = np.asarray(ref["eval"]), np.asarray(ref["occ"])
    lp = sl.eigh(sp.H, sp.S, eigvals_only=True)
    assert eig_excess(lp, ev, sp.S, occ=f) <= 1.0, name
    occ = np.abs(f) > 1e-20
    # on the states in D LAPACK stays well inside the plain gate
    assert np.max(np.abs(lp - ev)[occ] / (1e-10 * np.maximum(1.0, np.abs(ev[occ])))) <= 0.5, name
    if "kappa1e2" not in name:
        assert (np.abs(ev) > 1.0).any(), name   # the relaxation is exercised


def test_occupied_large_state_keeps_the_plain_gate():
    sp = G.make_lattice_system(300, seed=7)
    ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    ev, f = np.asarray(ref["eval"]), np.asarray(ref["occ"])
    occ_big = np.where((np.abs(f) > 1e-20) & (np.abs(ev) > 1.0))[0]
    empty_big = np.where((np.abs(f) <= 1e-20) & (np.abs(ev) > 1.0))[0]
    assert occ_big.size and empty_big.size
    i, j = occ_big[-1], empty_big[-1]
    # an error of half the conditioning allowance
    for idx in (i, j):
        bad = ev.copy()
        bad[idx] += 0.5 * 2.0 * EPS * overlap_condition(sp.S) * abs(ev[idx])
        excess = eig_excess(bad, ev, sp.S, occ=f)
        if idx == i:
            assert excess > 1.0    # occupied: the plain gate catches it
        else:
            assert excess <= 1.0   # unoccupied: inside the relaxed gate
    # without occupations the gate keeps the relaxation everywhere above 1 Ha
    bad = ev.copy()
    bad[i] += 0.5 * 2.0 * EPS * overlap_condition(sp.S) * abs(ev[i])
    assert eig_excess(bad, ev, sp.S) <= 1.0
