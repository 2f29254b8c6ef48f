"""Batched calls: many independent problems of uneven size in one call.

Each problem must meet the same gates against the oracle as a single call
(eigenvalues as in gates.py, D within 1e-9); the
worker count must not change a single bit (problems share no state); the
block-diagonal pencil solved once must give the union of the spectra of its
blocks solved in a batch; a failing problem reports its own status without
stopping the others.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from gates import eig_excess
from synth import generator as G

pytestmark = pytest.mark.gpu

SIZES = [30, 45, 64, 65, 127, 200, 255, 300, 481]


def _dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def _systems(sizes, seed0=10):
    return [G.make_lattice_system(int(n), seed=seed0 + q) for q, n in enumerate(sizes)]




def _electrons(eps, mu, kT):
    x = (np.asarray(eps) - mu) / kT
    return float(np.sum(np.where(x >= 0, np.exp(-np.abs(x)) / (1 + np.exp(-np.abs(x))),
                                 1 / (1 + np.exp(-np.abs(x))))))


def _check_mu(mu, ref, sp):
    """mu is unique only where the electron count moves with it: inside a wide
    spectral gap every mu reproduces N_e, so there the GPU's mu must give the
    electron count with the oracle's eigenvalues."""
    if abs(mu - ref["mu"]) <= 1e-9:
        return
    assert abs(_electrons(ref["eval"], mu, sp.kT) - sp.n_occ) <= 1e-11


def test_dm_batched_vs_oracle():
    from paper_1705_11191_amd import binding as B

    sps = _systems(SIZES)
    h = B.Handle(8, 8, 2)
    Ds, evals, energy, mu, status, rc = h.dm_batched([_dev(sp.H) for sp in sps], [_dev(sp.S) for sp in sps],
                                                     [sp.n_occ for sp in sps])
    h.close()
    assert rc == 0 and status == [0] * len(sps)
    for q, sp in enumerate(sps):
        ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
        assert eig_excess(evals[q].cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0, q
        D = Ds[q].cpu().numpy()
        assert np.abs(D - ref["D"]).max() <= 1e-9, q
        _check_mu(mu[q], ref, sp)
        assert abs(energy[q] - ref["energy"]) <= 1e-9, q
        assert abs(np.trace(D @ sp.S) - sp.n_occ) <= 1e-10, q


def test_batched_worker_count_changes_no_bit():
    from paper_1705_11191_amd import binding as B

    sps = _systems(SIZES, seed0=40)
    out = []
    for workers in (1, 4):
        h = B.Handle(8, 8, 2)
        h.set_batch_workers(workers)
        Ds, evals, energy, mu, status, rc = h.dm_batched([_dev(sp.H) for sp in sps], [_dev(sp.S) for sp in sps],
                                                         [sp.n_occ for sp in sps])
        h.close()
        assert rc == 0
        out.append(([D.cpu().numpy() for D in Ds], [e.cpu().numpy() for e in evals], energy, mu))
    for q in range(len(sps)):
        assert np.array_equal(out[0][0][q], out[1][0][q]), q
        assert np.array_equal(out[0][1][q], out[1][1][q]), q
    assert out[0][2] == out[1][2] and out[0][3] == out[1][3]


def test_batched_calls_run_fp64_on_a_mixed_handle():
    """The precision setting applies to the single-problem calls only: a handle
    switched to the mixed mode returns the FP64 batched results bit for bit."""
    from paper_1705_11191_amd import binding as B

    sps = _systems(SIZES[:5], seed0=70)
    out = []
    for prec in (B.PREC_FP64, B.PREC_MIXED):
        h = B.Handle(8, 8, 2)
        h.set_batch_workers(2)
        h.set_precision(prec, 1e-10, 4)
        Ds, evals, energy, mu, status, rc = h.dm_batched([_dev(sp.H) for sp in sps], [_dev(sp.S) for sp in sps],
                                                         [sp.n_occ for sp in sps])
        h.close()
        assert rc == 0 and status == [0] * len(sps)
        out.append([D.cpu().numpy() for D in Ds])
    for q in range(len(sps)):
        assert np.array_equal(out[0][q], out[1][q]), q


def test_ev_batched_union_of_block_diagonal():
    """blockdiag(H1, H2, H3) x = lambda blockdiag(S1, S2, S3) x has exactly the
    union of the three spectra."""
    from paper_1705_11191_amd import binding as B

    sizes = [40, 65, 130]
    sps = _systems(sizes, seed0=70)
    h = B.Handle(8, 8, 2)
    evals, evecs, status, rc = h.ev_batched([_dev(sp.H) for sp in sps], [_dev(sp.S) for sp in sps], sizes)
    h.close()
    assert rc == 0 and status == [0, 0, 0]
    n = sum(sizes)
    Hb = np.zeros((n, n))
    Sb = np.zeros((n, n))
    o = 0
    for sp, m in zip(sps, sizes):
        Hb[o:o + m, o:o + m] = sp.H
        Sb[o:o + m, o:o + m] = sp.S
        o += m
    h1 = B.Handle(n, n, 1)
    ev_all, _ = h1.ev(_dev(Hb), _dev(Sb))
    h1.close()
    union = np.sort(np.concatenate([e.cpu().numpy() for e in evals]))
    assert eig_excess(union, ev_all.cpu().numpy(), Sb) <= 1.0
    # each problem's eigenvectors: S-orthonormal and matching the oracle's subspace
    for q, sp in enumerate(sps):
        C = evecs[q].cpu().numpy()
        assert np.abs(C.T @ sp.S @ C - np.eye(sizes[q])).max() <= 1e-8
        ref_ev = O.gevp(sp.H, sp.S, sizes[q])[0]
        assert eig_excess(evals[q].cpu().numpy(), ref_ev, sp.S) <= 1.0


def test_batched_failure_stays_with_its_problem():
    from paper_1705_11191_amd import binding as B

    sps = _systems([50, 70, 90], seed0=90)
    Hs = [_dev(sp.H) for sp in sps]
    Ss = [_dev(sp.S) for sp in sps]
    bad = sps[1].S.copy()
    bad[20, 20] = -1.0                       # not positive definite at pivot 21
    Ss[1] = _dev(bad)
    h = B.Handle(8, 8, 2)
    Ds, evals, energy, mu, status, rc = h.dm_batched(Hs, Ss, [sp.n_occ for sp in sps], ok=(0, 1))
    h.close()
    assert status == [0, 1, 0]
    assert rc == 1
    for q in (0, 2):
        ref = O.dm(sps[q].H, sps[q].S, sps[q].n_occ, sps[q].kT)
        assert np.abs(Ds[q].cpu().numpy() - ref["D"]).max() <= 1e-9


def test_batched_tiny_and_empty():
    from paper_1705_11191_amd import binding as B

    h = B.Handle(8, 8, 2)
    evals, evecs, status, rc = h.ev_batched([], [], [])
    assert rc == 0 and status == []
    # 1 x 1 and 2 x 2 pencils: closed forms
    H1, S1 = np.array([[-0.3]]), np.array([[2.0]])
    H2, S2 = np.array([[1.0, 0.2], [0.2, -0.5]]), np.array([[1.0, 0.1], [0.1, 1.0]])
    evals, evecs, status, rc = h.ev_batched([_dev(H1), _dev(H2)], [_dev(S1), _dev(S2)], [1, 2])
    h.close()
    assert rc == 0 and status == [0, 0]
    assert abs(evals[0].item() - (-0.15)) <= 1e-15
    a, b, c, s = 1.0, 0.2, -0.5, 0.1
    qa, qb, qc = 1 - s * s, -(a + c - 2 * b * s), a * c - b * b
    disc = np.sqrt(qb * qb - 4 * qa * qc)
    lam = np.sort([(-qb - disc) / (2 * qa), (-qb + disc) / (2 * qa)])
    assert np.abs(evals[1].cpu().numpy() - lam).max() <= 1e-14


def test_batched_band_table_routes_each_size_to_its_width():
    """With a table, each problem runs with its bucket's band width: it matches,
    bit for bit, the same problem in a batched call with that width set on the
    handle, and every problem meets the oracle gates."""
    from paper_1705_11191_amd import binding as B

    sizes = [40, 90, 130, 260, 300]
    sps = _systems(sizes, seed0=40)
    ne = [sp.n_occ for sp in sps]

    def run(table=None, b=None):
        h = B.Handle(8, 8, 2)
        if table:
            h.set_batch_band_table(*table)
        if b:
            h.set_band_width(b)
        out = h.dm_batched([_dev(sp.H) for sp in sps], [_dev(sp.S) for sp in sps], ne)
        h.close()
        assert out[5] == 0
        return [D.cpu().numpy() for D in out[0]]

    D_tab = run(table=([64, 256], [16, 32]))
    D16, D32, D64 = run(b=16), run(b=32), run(b=64)
    want = {40: D16, 90: D32, 130: D32, 260: D64, 300: D64}
    for q, n in enumerate(sizes):
        assert np.array_equal(D_tab[q], want[n][q]), n
        ref = O.dm(sps[q].H, sps[q].S, sps[q].n_occ, sps[q].kT)
        assert np.abs(D_tab[q] - ref["D"]).max() <= 1e-9


def test_tuner_sets_a_width_per_bucket_and_caches_it(tmp_path):
    from paper_1705_11191_amd import binding as B
    from paper_1705_11191_amd import tune

    sizes = [60, 100, 200, 300, 520]
    sps = _systems(sizes, seed0=60)
    Hs = [_dev(sp.H) for sp in sps]
    Ss = [_dev(sp.S) for sp in sps]
    H0 = [x.clone() for x in Hs]
    S0 = [x.clone() for x in Ss]
    ne = [sp.n_occ for sp in sps]
    cache = str(tmp_path / "tune.json")
    h = B.Handle(8, 8, 2)
    rec = tune.tune_batch_band_widths(h, Hs, Ss, ne, candidates=(32, 64), per_bucket=2, workers=4,
                                      cache_path=cache)
    assert rec["n_max"] == [512, 1024] and all(b in (32, 64) for b in rec["b"]) and not rec["cached"]
    assert all(torch.equal(a, b) for a, b in zip(Hs, H0)) and all(torch.equal(a, b) for a, b in zip(Ss, S0))
    rec2 = tune.tune_batch_band_widths(h, Hs, Ss, ne, candidates=(32, 64), per_bucket=2, workers=4,
                                       cache_path=cache)
    assert rec2["cached"] and rec2["n_max"] == rec["n_max"] and rec2["b"] == rec["b"]
    Ds, evals, energy, mu, status, rc = h.dm_batched(Hs, Ss, ne)
    h.close()
    assert rc == 0
    for q, sp in enumerate(sps):
        ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
        assert np.abs(Ds[q].cpu().numpy() - ref["D"]).max() <= 1e-9
        assert eig_excess(evals[q].cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
