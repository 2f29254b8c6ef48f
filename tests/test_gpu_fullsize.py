"""The density-matrix path at its full sizes (3D lattice, N = 8192 and 32768),
in the launch configuration the benchmark times (default handle, band width
64, Fermi-Dirac at kT = 0.01 Ha).

The oracle cannot run at these sizes in a test (about 12.5 N^3 flops on the
host), so the checks are properties that hold at any size, plus sampled
eigenpairs certified one by one:

* ev and dm share steps (0)-(3): their eigenvalues are identical bits;
* D is exactly symmetric; tr(D S) = N_e; the occupations reproduce N_e at the
  returned mu and sum_l f_l eps_l is the returned energy;
* for sampled eigenpairs (lowest, middle of the occupied block, the last
  occupied state, the first empty ones, the last one that enters D) the
  residual r = H c - eps S c is accumulated in long double by the oracle's
  residual routine, and
  - its backward-stability ratio ||r|| / ((||H||_F + |eps| ||S||_F) ||c|| n eps_mach)
    is at most 1 (the LAPACK eigensolver tests accept 30);
  - the sampled columns are S-orthonormal to 1e-8;
  - for samples separated from their neighbours by gap >= 1e-4 Ha in the
    computed spectrum, the quadratic residual bound ||r||_{S^-1}^2 / gap, with
    ||r||_{S^-1}^2 <= ||r||_2^2 / lambda_min(S) and lambda_min(S) >= sigma (the
    shift the generator adds to the positive semidefinite S_lit), is at most
    1e-10 Ha scaled by max(1, |eps|);
* D S c_l = f_l c_l for the sampled eigenvectors.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from synth import generator as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", [1, 2])
def test_fullsize_dm_properties(cfg):
    from paper_1705_11191_amd import binding as B

    dev = torch.device("cuda:0")
    sp = G.make_config(cfg, device=dev)
    n = int(sp.H.shape[0])
    n_occ = int(sp.n_occ)
    print(f"[fullsize] N={n} n_occ={n_occ}", flush=True)
    H0, S0 = sp.H, sp.S
    h = B.Handle(n, n, n_occ)
    D, ev, f, energy, mu, st = h.dm(H0.clone(), S0.clone())
    ks = h.info()["k_s"]
    h.close()
    torch.cuda.empty_cache()
    assert st == 0
    assert bool(torch.all(ev[1:] >= ev[:-1]))
    assert float((D - D.T).abs().max()) == 0.0
    assert abs(float((D * S0).sum()) - n_occ) <= 1e-9
    fe = f.double()
    assert abs(float(fe.sum()) - n_occ) <= 1e-10
    assert abs(float((fe * ev).sum()) - energy) <= 1e-9 * max(1.0, abs(energy))
    x = (ev - mu) / sp.kT
    fd = torch.where(x >= 0, torch.exp(-x) / (1 + torch.exp(-x)), 1 / (1 + torch.exp(x)))
    assert abs(float(fd.sum()) - n_occ) <= 1e-9
    assert ks == int((f > 1e-20).sum())

    # eigenvectors of the lowest k2 states from the ev driver on the same input
    k2 = min(n, ks + 64)
    h2 = B.Handle(n, k2, n_occ)
    ev2, C = h2.ev(H0.clone(), S0.clone())
    h2.close()
    torch.cuda.empty_cache()
    assert torch.equal(ev2, ev)
    idx = sorted({0, 1, n_occ // 2, n_occ - 1, n_occ, min(n_occ + 1, k2 - 1), ks - 1, k2 - 1})
    Cs = C[:, idx].contiguous()
    # D S c = f c on the sample (on the device, in FP64)
    DSc = D @ (S0 @ Cs)
    err = (DSc - Cs * f[idx]).abs().max(dim=0).values
    scale = Cs.abs().max(dim=0).values
    assert bool(torch.all(err <= 1e-8 * torch.clamp(scale, min=1.0))), (err, scale)
    lam = ev[idx].cpu().numpy()
    Xs = Cs.cpu().numpy()
    del D, DSc, C
    torch.cuda.empty_cache()
    Hh = H0.cpu().numpy()
    Sh = S0.cpu().numpy()
    res = O.residual_norms(Hh, Sh, Xs, lam)
    eps = np.finfo(np.float64).eps
    nH = float(np.linalg.norm(Hh))
    nS = float(np.linalg.norm(Sh))
    xnorm = np.linalg.norm(Xs, axis=0)
    ratio = res / ((nH + np.abs(lam) * nS) * xnorm * n * eps)
    G_s = Xs.T @ (Sh @ Xs)
    orth = float(np.abs(G_s - np.eye(len(idx))).max())
    sigma = float(sp.meta["sigma"]) * (1.0 - 1e-6)
    evh = ev.cpu().numpy()
    gap = np.array([min(abs(evh[l] - evh[l - 1]) if l > 0 else np.inf,
                        abs(evh[l + 1] - evh[l]) if l + 1 < n else np.inf) for l in idx])
    quad = res ** 2 / sigma / gap
    print(f"[fullsize] N={n} k_s={ks} ratio {np.array2string(ratio, precision=2)} orth {orth:.1e} "
          f"gap {np.array2string(gap, precision=2)} quadratic bound {np.array2string(quad, precision=2)}",
          flush=True)
    assert np.all(ratio <= 1.0), (idx, ratio)
    assert orth <= 1e-8
    sep = gap >= 1e-4
    assert np.any(sep)
    assert np.all(quad[sep] <= 1e-10 * np.maximum(1.0, np.abs(lam[sep]))), (idx, quad, gap)
