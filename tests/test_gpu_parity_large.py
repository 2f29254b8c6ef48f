"""Element-wise oracle parity at sizes that take the size branches of the
kernels: N = 3000 (an outer panel of 2048 and a ragged one, 47 band panels;
ev with 2100 states, more than 2048 columns in the back-transformations), a batch
holding an n = 4095 problem (the largest of the benchmark batch), and a
complex pencil of n = 1000.  The oracle needs 10-30 s for each on the host
cores; its results are computed once per module.  Gates as everywhere:
eigenvalues by gates.eig_excess, D within 1e-9, S-orthonormal eigenvectors.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from gates import eig_excess
from synth import generator as G

pytestmark = pytest.mark.gpu

N = 3000


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def big():
    sp = G.make_lattice_system(N, seed=3000)
    print(f"[parity large] oracle dm N={N}", flush=True)
    ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    return sp, ref


def test_dm_n3000_vs_oracle(big):
    from paper_1705_11191_amd import binding as B

    sp, ref = big
    h = B.Handle(N, N, sp.n_occ)
    D, ev, f, energy, mu, st = h.dm(_dev(sp.H), _dev(sp.S))
    h.close()
    D = D.cpu().numpy()
    print(f"[parity large] dm N={N}: D err {np.abs(D - ref['D']).max():.2e} (max |D| {np.abs(ref['D']).max():.1f})",
          flush=True)
    assert st == 0
    assert eig_excess(ev.cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
    assert np.abs(D - ref["D"]).max() <= 1e-9
    assert np.abs(f.cpu().numpy() - ref["occ"]).max() <= 1e-12
    assert abs(energy - ref["energy"]) <= 1e-9 * max(1.0, abs(ref["energy"]))


def test_mixed_dm_n3000_vs_oracle(big):
    from paper_1705_11191_amd import binding as B

    sp, ref = big
    h = B.Handle(N, N, sp.n_occ)
    h.set_precision(B.PREC_MIXED, 1e-10, 6)
    D, ev, f, energy, mu, st = h.dm(_dev(sp.H), _dev(sp.S), ok=(0, 3))
    info = h.info()
    h.close()
    D = D.cpu().numpy()
    ks = info["k_s"]
    print(f"[parity large] mixed dm N={N}: status {st} sweeps {info['refine_sweeps']} step {info['refine_step']:.2e}"
          f" D err {np.abs(D - ref['D']).max():.2e}", flush=True)
    assert st == 0
    assert eig_excess(ev.cpu().numpy()[:ks], ref["eval"][:ks], sp.S, occ=ref["occ"][:ks]) <= 1.0
    assert np.abs(D - ref["D"]).max() <= 1e-9


def test_ev_n3000_with_2100_states_vs_oracle(big):
    from paper_1705_11191_amd import binding as B

    sp, ref = big
    k = 2100
    h = B.Handle(N, k, sp.n_occ)
    ev, C = h.ev(_dev(sp.H), _dev(sp.S))
    h.close()
    ev, C = ev.cpu().numpy(), C.cpu().numpy()
    assert eig_excess(ev, ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
    assert np.abs(C.T @ sp.S @ C - np.eye(k)).max() <= 1e-8
    # eigenvectors of states separated from their neighbours by 1e-6 Ha match
    # the oracle's up to sign (S-inner products of 1 to 1e-8)
    evo, Co, _ = O.gevp(sp.H, sp.S, n_state=k)
    gap = np.minimum(np.abs(np.diff(evo[:k + 1])[:k]), np.abs(np.diff(evo[:k], prepend=-np.inf)))
    sep = gap > 1e-6
    dots = np.abs(np.sum((C.T @ sp.S) * Co.T, axis=1))
    assert np.all(np.abs(dots[sep] - 1.0) <= 1e-8)


def test_batched_with_n4095_vs_oracle():
    from paper_1705_11191_amd import binding as B

    sizes = [4095, 600, 255]
    sps = [G.make_lattice_system(n, seed=4000 + q) for q, n in enumerate(sizes)]
    h = B.Handle(8, 8, 2)
    Ds, evals, energy, mu, status, rc = h.dm_batched([_dev(sp.H) for sp in sps], [_dev(sp.S) for sp in sps],
                                                     [sp.n_occ for sp in sps])
    h.close()
    assert rc == 0 and status == [0, 0, 0]
    for q, sp in enumerate(sps):
        print(f"[parity large] batched oracle n={sp.n}", flush=True)
        ref = O.dm(sp.H, sp.S, sp.n_occ, sp.kT)
        D = Ds[q].cpu().numpy()
        print(f"[parity large] batched n={sp.n}: D err {np.abs(D - ref['D']).max():.2e}", flush=True)
        assert eig_excess(evals[q].cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
        assert np.abs(D - ref["D"]).max() <= 1e-9


def test_complex_dm_n1000_vs_oracle():
    from paper_1705_11191_amd import binding as B

    sp = G.make_kpoint_system((5, 5, 10), (0.125, 0.25, 0.25), seed=1000)
    n = sp.H.shape[0]
    assert n == 1000
    print(f"[parity large] complex oracle n={n}", flush=True)
    ref = O.zdm(sp.H, sp.S, sp.n_occ, sp.kT)
    h = B.Handle(n, n, sp.n_occ, dtype=B.COMPLEX128)
    D, ev, f, energy, mu, st = h.dm(B.as_fortran(torch.tensor(sp.H, device="cuda")),
                                    B.as_fortran(torch.tensor(sp.S, device="cuda")))
    h.close()
    D = D.cpu().numpy()
    print(f"[parity large] complex n={n}: D err {np.abs(D - ref['D']).max():.2e}", flush=True)
    assert st == 0
    assert eig_excess(ev.cpu().numpy(), ref["eval"], sp.S, occ=ref["occ"]) <= 1.0
    assert np.abs(D - ref["D"]).max() <= 1e-9
    assert np.abs(D - D.conj().T).max() <= 1e-12
