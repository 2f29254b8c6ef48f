"""Synthetic localized-basis H/S pairs standing in for the paper's KS-DFT matrices.

The paper benchmarks on Hamiltonian and overlap matrices produced by FHI-aims
and DGDFT graphene runs (Sec. 5, Table 1); those matrices are not available,
so seeded synthetic matrices of the same kind stand in for them:

* basis functions are normalized s-type Gaussians centred on atoms, so the
  overlap is the integral of Eq. (5) evaluated analytically with the Gaussian
  product theorem:  S_ab = (2 sqrt(a b) / (a + b))^{3/2} exp(-a b / (a + b) |A - B|^2);
* the Hamiltonian is extended-Hueckel-like:  H_ii = h_i,
  H_ij = 1.75 * S_ij * (h_i + h_j) / 2  (i != j), h_i ~ U(-15, -5) eV;
* S is shifted by sigma * I, sigma = lambda_max(S_lit) / kappa, which fixes its
  condition number at about kappa (the literal draw of many same-centre
  exponents is numerically singular).  H is left unchanged because its
  off-diagonal entries use S_ij, i != j, which the shift does not touch.

Random numbers come from ``numpy.random.default_rng(seed)`` in a fixed order:
atom jitter (atoms x 3), exponents (atoms x orbitals), on-site energies (N).
Lengths are in bohr, energies in Hartree (eV are converted on the way in).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HARTREE_PER_EV = 1.0 / 27.211386245988  # CODATA 2018
WH_K = 1.75                             # Wolfsberg-Helmholz constant
DEFAULT_KAPPA = 1.0e6
DEFAULT_KT = 0.01                       # Fermi-Dirac width in Hartree


@dataclass
class SystemSpec:
    """A generated pencil plus the metadata needed to solve and report it."""

    H: np.ndarray
    S: np.ndarray
    n_occ: float
    kT: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.H.shape[0]


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def chain_positions(n_atoms: int, spacing: float, jitter: np.ndarray) -> np.ndarray:
    """Atoms on a line: x_a = spacing * a + jitter_a (only the x jitter is used)."""
    pos = np.zeros((n_atoms, 3))
    pos[:, 0] = spacing * np.arange(n_atoms) + jitter[:, 0]
    return pos


def lattice_positions(n_atoms: int, spacing: float, jitter: np.ndarray) -> np.ndarray:
    """First ``n_atoms`` sites of an m x m x m cubic lattice, x fastest, plus jitter."""
    m = 1
    while m ** 3 < n_atoms:
        m += 1
    idx = np.arange(n_atoms)
    ix, iy, iz = idx % m, (idx // m) % m, idx // (m * m)
    pos = spacing * np.stack([ix, iy, iz], axis=1).astype(np.float64)
    return pos + jitter


# ----------------------------------------------------------------------------
# matrices
# ----------------------------------------------------------------------------
def s_gaussian_overlap(centers: np.ndarray, alphas: np.ndarray, block: int = 2048) -> np.ndarray:
    """Overlap of normalized s-Gaussians (Gaussian product theorem), built in row blocks."""
    n = alphas.shape[0]
    S = np.empty((n, n))
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        a = alphas[i0:i1, None]
        b = alphas[None, :]
        d2 = ((centers[i0:i1, None, :] - centers[None, :, :]) ** 2).sum(axis=2)
        p = a + b
        S[i0:i1] = (2.0 * np.sqrt(a * b) / p) ** 1.5 * np.exp(-(a * b / p) * d2)
    return S


def _lambda_max(S: np.ndarray) -> float:
    """Largest eigenvalue of a symmetric matrix by Lanczos (deterministic start vector)."""
    n = S.shape[0]
    if n <= 64:
        return float(np.linalg.eigvalsh(S)[-1])
    from scipy.sparse.linalg import eigsh

    v0 = np.ones(n) / math.sqrt(n)
    val = eigsh(S, k=1, which="LA", v0=v0, tol=1e-10, return_eigenvectors=False)
    return float(val[0])


def build_system(centers_per_orbital: np.ndarray, alphas: np.ndarray, h: np.ndarray,
                 kappa: float = DEFAULT_KAPPA, block: int = 2048):
    """Return (H, S, sigma) for the given orbital centres, exponents and on-site energies."""
    S = s_gaussian_overlap(centers_per_orbital, alphas, block=block)
    n = S.shape[0]
    sigma = 0.0
    if kappa is not None and kappa > 0:
        sigma = _lambda_max(S) / kappa
    H = np.empty_like(S)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        H[i0:i1] = WH_K * 0.5 * S[i0:i1] * (h[i0:i1, None] + h[None, :])
    di = np.arange(n)
    H[di, di] = h
    S[di, di] += sigma
    return H, S, sigma


def _draw_lattice(n, seed, orbitals_per_atom, spacing, jitter_amp, alpha_lo, alpha_hi):
    n_atoms = -(-n // orbitals_per_atom)
    rng = np.random.default_rng(seed)
    jitter = rng.uniform(-jitter_amp, jitter_amp, size=(n_atoms, 3))
    alphas = rng.uniform(alpha_lo, alpha_hi, size=(n_atoms, orbitals_per_atom)).reshape(-1)[:n]
    h = rng.uniform(-15.0, -5.0, size=n) * HARTREE_PER_EV
    pos = lattice_positions(n_atoms, spacing, jitter)
    centers = np.repeat(pos, orbitals_per_atom, axis=0)[:n]
    return n_atoms, centers, alphas, h


def build_system_torch(centers, alphas, h, kappa=DEFAULT_KAPPA, device="cuda", block=4096,
                       lanczos_steps=80):
    """Same matrices as :func:`build_system`, assembled with torch on ``device``.

    Returns (H, S, sigma) as float64 torch tensors.  lambda_max(S_lit) comes
    from a Lanczos run with full reorthogonalization (deterministic start).
    """
    import torch

    c = torch.as_tensor(centers, dtype=torch.float64, device=device)
    a = torch.as_tensor(alphas, dtype=torch.float64, device=device)
    hh = torch.as_tensor(h, dtype=torch.float64, device=device)
    n = a.shape[0]
    S = torch.empty((n, n), dtype=torch.float64, device=device)
    H = torch.empty((n, n), dtype=torch.float64, device=device)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        ai = a[i0:i1, None]
        p = ai + a[None, :]
        d2 = torch.zeros((i1 - i0, n), dtype=torch.float64, device=device)
        for ax in range(3):
            d2 += (c[i0:i1, ax, None] - c[None, :, ax]) ** 2
        Sb = (2.0 * torch.sqrt(ai * a[None, :]) / p) ** 1.5 * torch.exp(-(ai * a[None, :] / p) * d2)
        S[i0:i1] = Sb
        H[i0:i1] = WH_K * 0.5 * Sb * (hh[i0:i1, None] + hh[None, :])
        del ai, p, d2, Sb
    sigma = 0.0
    if kappa is not None and kappa > 0:
        k = min(lanczos_steps, n)
        Q = torch.zeros((k + 1, n), dtype=torch.float64, device=device)
        alpha = torch.zeros(k, dtype=torch.float64)
        beta = torch.zeros(k, dtype=torch.float64)
        Q[0] = 1.0 / math.sqrt(n)
        m = k
        for j in range(k):
            w = S @ Q[j]
            alpha[j] = torch.dot(w, Q[j]).item()
            w = w - Q[: j + 1].T @ (Q[: j + 1] @ w)
            w = w - Q[: j + 1].T @ (Q[: j + 1] @ w)
            bj = torch.linalg.norm(w).item()
            beta[j] = bj
            if bj < 1e-14:
                m = j + 1
                break
            Q[j + 1] = w / bj
        T = np.diag(alpha[:m].numpy()) + np.diag(beta[: m - 1].numpy(), 1) + np.diag(beta[: m - 1].numpy(), -1)
        sigma = float(np.linalg.eigvalsh(T)[-1]) / kappa
        del Q
    di = torch.arange(n, device=device)
    H[di, di] = hh
    S[di, di] += sigma
    return H, S, sigma


def make_lattice_system(n: int, seed: int, kappa: float = DEFAULT_KAPPA,
                        orbitals_per_atom: int = 15, spacing: float = 2.5,
                        jitter_amp: float = 0.2, alpha_lo: float = 0.2,
                        alpha_hi: float = 3.0, device=None) -> SystemSpec:
    """3D jittered cubic lattice, ``orbitals_per_atom`` s-Gaussians per atom, first n orbitals kept.

    With ``device`` set (a torch device) H and S are torch tensors built there.
    """
    n_atoms, centers, alphas, h = _draw_lattice(n, seed, orbitals_per_atom, spacing, jitter_amp,
                                                alpha_lo, alpha_hi)
    if device is not None:
        H, S, sigma = build_system_torch(centers, alphas, h, kappa, device=device)
    else:
        H, S, sigma = build_system(centers, alphas, h, kappa)
    return SystemSpec(H, S, n_occ=float(n // 4), kT=DEFAULT_KT,
                      meta=dict(kind="lattice3d", n_atoms=n_atoms, seed=seed,
                                kappa=kappa, sigma=sigma, orbitals_per_atom=orbitals_per_atom))


def make_chain_system(seed: int = 0, kappa: float = DEFAULT_KAPPA, n_atoms: int = 128,
                      orbitals_per_atom: int = 4) -> SystemSpec:
    """1D chain: spacing 1.4 bohr, jitter U(+-0.1), 4 s-Gaussians per atom, alpha ~ U(0.3, 2.0)."""
    rng = np.random.default_rng(seed)
    jitter = rng.uniform(-0.1, 0.1, size=(n_atoms, 3))
    alphas = rng.uniform(0.3, 2.0, size=(n_atoms, orbitals_per_atom)).reshape(-1)
    n = n_atoms * orbitals_per_atom
    h = rng.uniform(-15.0, -5.0, size=n) * HARTREE_PER_EV
    pos = chain_positions(n_atoms, 1.4, jitter)
    centers = np.repeat(pos, orbitals_per_atom, axis=0)
    H, S, sigma = build_system(centers, alphas, h, kappa)
    return SystemSpec(H, S, n_occ=float(n // 4), kT=DEFAULT_KT,
                      meta=dict(kind="chain1d", n_atoms=n_atoms, seed=seed,
                                kappa=kappa, sigma=sigma, orbitals_per_atom=orbitals_per_atom))


def batch_sizes(count: int = 256, seed: int = 0, lo: int = 256, hi: int = 4096,
                multiple: int = 15) -> np.ndarray:
    """Problem sizes log-uniform in [lo, hi], rounded to a multiple of ``multiple``."""
    rng = np.random.default_rng(seed)
    raw = np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))
    return (multiple * np.round(raw / multiple)).astype(np.int64)


def make_config(cfg: int, seed: int = 0, kappa: float = DEFAULT_KAPPA, device=None) -> SystemSpec:
    """The single-problem workloads: 0 = 512-orbital chain, 1 = N 8192 lattice, 2 = N 32768 lattice."""
    if cfg == 0:
        return make_chain_system(seed=seed, kappa=kappa)
    if cfg == 1:
        return make_lattice_system(8192, seed, kappa, device=device)
    if cfg == 2:
        return make_lattice_system(32768, seed, kappa, device=device)
    raise ValueError(f"unknown single-problem config {cfg}")


# ----------------------------------------------------------------------------
# closed-form test pencils (inputs only; their exact spectra live in the tests)
# ----------------------------------------------------------------------------
def tight_binding_chain(n: int, eps0: float, t: float) -> np.ndarray:
    """H = tridiag(t, eps0, t), the 1D nearest-neighbour tight-binding chain."""
    H = np.zeros((n, n))
    H[np.arange(n), np.arange(n)] = eps0
    H[np.arange(n - 1), np.arange(1, n)] = t
    H[np.arange(1, n), np.arange(n - 1)] = t
    return H


def toeplitz_pencil(n: int, alpha: float, beta: complex, sigma: complex):
    """H = tridiag(conj(beta), alpha, beta), S = tridiag(conj(sigma), 1, sigma) (upper = beta)."""
    cplx = np.iscomplexobj(beta) or np.iscomplexobj(sigma) or isinstance(beta, complex) \
        or isinstance(sigma, complex)
    dt = np.complex128 if cplx else np.float64
    H = np.zeros((n, n), dtype=dt)
    S = np.zeros((n, n), dtype=dt)
    i = np.arange(n)
    H[i, i] = alpha
    S[i, i] = 1.0
    # column-major reading: entry (row j, col j+1) is the upper one
    H[i[:-1], i[1:]] = beta
    H[i[1:], i[:-1]] = np.conj(beta)
    S[i[:-1], i[1:]] = sigma
    S[i[1:], i[:-1]] = np.conj(sigma)
    return H, S


# ----------------------------------------------------------------------------
# complex Hermitian k-point pencils (periodic cell, Bloch sums)
# ----------------------------------------------------------------------------
def _draw_kpoint_cell(cell_sites, seed, orbitals_per_atom, spacing, jitter_amp, alpha_lo, alpha_hi):
    mx, my, mz = (int(v) for v in cell_sites)
    n_atoms = mx * my * mz
    n = n_atoms * orbitals_per_atom
    rng = np.random.default_rng(seed)
    jitter = rng.uniform(-jitter_amp, jitter_amp, size=(n_atoms, 3))
    alphas = rng.uniform(alpha_lo, alpha_hi, size=(n_atoms, orbitals_per_atom)).reshape(-1)
    h = rng.uniform(-15.0, -5.0, size=n) * HARTREE_PER_EV
    idx = np.arange(n_atoms)
    ix, iy, iz = idx % mx, (idx // mx) % my, idx // (mx * my)
    pos = spacing * np.stack([ix, iy, iz], axis=1).astype(np.float64) + jitter
    centers = np.repeat(pos, orbitals_per_atom, axis=0)
    lat = spacing * np.array([mx, my, mz], dtype=np.float64)
    return (mx, my, mz), centers, alphas, h, lat


MP_KPOINTS_4x2x2 = [(k1, k2, k3) for k1 in (-0.375, -0.125, 0.125, 0.375)
                    for k2 in (-0.25, 0.25) for k3 in (-0.25, 0.25)]


def make_kpoint_system(cell_sites=(3, 3, 3), kpt=(0.125, 0.25, 0.25), seed: int = 0,
                       kappa: float = DEFAULT_KAPPA, orbitals_per_atom: int = 4,
                       spacing: float = 2.5, jitter_amp: float = 0.2, alpha_lo: float = 0.8,
                       alpha_hi: float = 3.0) -> SystemSpec:
    """Complex Hermitian H(k), S(k) of a periodic jittered cubic cell.

    The cell holds cell_sites[0] x cell_sites[1] x cell_sites[2] atoms with
    ``orbitals_per_atom`` s-Gaussians each; the lattice vectors are
    spacing * cell_sites along x, y, z.  With R running over the 27 images
    n_R in {-1, 0, 1}^3 (integer lattice coordinates):
        S(k)_ij = sum_R S_R(i, j) exp(+i 2 pi k . n_R),  S_R(i, j) = overlap of
                  orbital i in the home cell with orbital j in cell R,
        H(k)_ij = sum_R H_R(i, j) exp(+i 2 pi k . n_R),  H_R = 1.75 S_R (h_i + h_j) / 2
                  except H_0(i, i) = h_i,
    and S(k) += sigma I with sigma = lambda_max(S(k)) / kappa.  k is in units
    of the reciprocal lattice; k = 0 gives a real pencil.  Exponents default to
    U(0.8, 3.0) so that the overlaps beyond the 27 images are negligible and
    the truncated Bloch sum stays positive definite (checked).
    Random numbers: jitter (atoms x 3), exponents (atoms x orbitals), on-site
    energies (N), in that order from ``numpy.random.default_rng(seed)``.
    """
    (mx, my, mz), centers, alphas, h, lat = _draw_kpoint_cell(cell_sites, seed, orbitals_per_atom, spacing,
                                                              jitter_amp, alpha_lo, alpha_hi)
    n = h.shape[0]
    k = np.asarray(kpt, dtype=np.float64)
    S = np.zeros((n, n), dtype=np.complex128)
    H = np.zeros((n, n), dtype=np.complex128)
    a = alphas[:, None]
    b = alphas[None, :]
    p = a + b
    pref = (2.0 * np.sqrt(a * b) / p) ** 1.5
    hh = WH_K * 0.5 * (h[:, None] + h[None, :])
    for rx in (-1, 0, 1):
        for ry in (-1, 0, 1):
            for rz in (-1, 0, 1):
                nR = np.array([rx, ry, rz], dtype=np.float64)
                shift = nR * lat
                d2 = ((centers[:, None, :] - (centers[None, :, :] + shift)) ** 2).sum(axis=2)
                SR = pref * np.exp(-(a * b / p) * d2)
                HR = hh * SR
                if rx == 0 and ry == 0 and rz == 0:
                    HR[np.arange(n), np.arange(n)] = h
                ph = np.exp(2j * np.pi * float(k @ nR))
                S += SR * ph
                H += HR * ph
    # exact Hermitian symmetry (the image sum pairs R with -R)
    S = 0.5 * (S + S.conj().T)
    H = 0.5 * (H + H.conj().T)
    w = np.linalg.eigvalsh(S)
    sigma = 0.0
    if kappa is not None and kappa > 0:
        sigma = float(w[-1]) / kappa
    if not (w[0] + sigma > 0.5 * sigma):
        raise ValueError("truncated Bloch sum is not positive definite; use larger exponents or cell")
    S[np.arange(n), np.arange(n)] += sigma
    return SystemSpec(H, S, n_occ=float(n // 4), kT=DEFAULT_KT,
                      meta=dict(kind="kpoint3d", cell_sites=(mx, my, mz), kpt=tuple(k), seed=seed,
                                kappa=kappa, sigma=sigma, orbitals_per_atom=orbitals_per_atom))


def make_kpoint_system_torch(cell_sites=(8, 8, 12), kpt=(0.125, 0.25, 0.25), seed: int = 0,
                             kappa: float = DEFAULT_KAPPA, orbitals_per_atom: int = 15,
                             spacing: float = 2.5, jitter_amp: float = 0.2, alpha_lo: float = 0.8,
                             alpha_hi: float = 3.0, device="cuda", block: int = 2048,
                             lanczos_steps: int = 80) -> SystemSpec:
    """:func:`make_kpoint_system` assembled with torch on ``device`` for large
    cells (default: the 768-atom 8 x 8 x 12 cell, N = 11,520).  H and S are
    column-major complex128 tensors; lambda_max(S(k)) comes from a Lanczos run
    with full reorthogonalization (deterministic start).  The positive
    definiteness check of the small version is skipped (the cell is 20 x 20 x
    30 bohr, far larger than the Gaussians' reach)."""
    import torch

    (mx, my, mz), centers, alphas, h, lat = _draw_kpoint_cell(cell_sites, seed, orbitals_per_atom, spacing,
                                                              jitter_amp, alpha_lo, alpha_hi)
    n = h.shape[0]
    c = torch.as_tensor(centers, dtype=torch.float64, device=device)
    a = torch.as_tensor(alphas, dtype=torch.float64, device=device)
    hh = torch.as_tensor(h, dtype=torch.float64, device=device)
    k = np.asarray(kpt, dtype=np.float64)
    # row-major buffers of the transposes, returned as column-major views
    St = torch.zeros((n, n), dtype=torch.complex128, device=device)
    Ht = torch.zeros((n, n), dtype=torch.complex128, device=device)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        ai = a[i0:i1, None]
        p = ai + a[None, :]
        pref = (2.0 * torch.sqrt(ai * a[None, :]) / p) ** 1.5
        ex = ai * a[None, :] / p
        hw = WH_K * 0.5 * (hh[i0:i1, None] + hh[None, :])
        for rx in (-1, 0, 1):
            for ry in (-1, 0, 1):
                for rz in (-1, 0, 1):
                    nR = np.array([rx, ry, rz], dtype=np.float64)
                    shift = torch.as_tensor(nR * lat, dtype=torch.float64, device=device)
                    d2 = torch.zeros((i1 - i0, n), dtype=torch.float64, device=device)
                    for ax in range(3):
                        d2 += (c[i0:i1, ax, None] - (c[None, :, ax] + shift[ax])) ** 2
                    SR = pref * torch.exp(-ex * d2)
                    HR = hw * SR
                    if rx == 0 and ry == 0 and rz == 0:
                        r = torch.arange(i0, i1, device=device)
                        HR[r - i0, r] = hh[i0:i1]
                    ang = 2.0 * math.pi * float(k @ nR)
                    ph = complex(math.cos(ang), math.sin(ang))
                    # rows i0:i1 of S(k) are columns i0:i1 of the transposed buffer
                    St[:, i0:i1] += (SR * ph).T
                    Ht[:, i0:i1] += (HR * ph).T
                    del d2, SR, HR
        del ai, p, pref, ex, hw
    S = St.t()
    H = Ht.t()
    # exact Hermitian symmetry
    S.copy_(0.5 * (S + S.conj().t()))
    H.copy_(0.5 * (H + H.conj().t()))
    sigma = 0.0
    if kappa is not None and kappa > 0:
        m = min(lanczos_steps, n)
        Q = torch.zeros((m + 1, n), dtype=torch.complex128, device=device)
        alpha = np.zeros(m)
        beta = np.zeros(m)
        Q[0] = 1.0 / math.sqrt(n)
        mm = m
        for j in range(m):
            w = S @ Q[j]
            alpha[j] = torch.vdot(Q[j], w).real.item()
            w = w - Q[: j + 1].T @ (Q[: j + 1].conj() @ w)
            w = w - Q[: j + 1].T @ (Q[: j + 1].conj() @ w)
            bj = torch.linalg.norm(w).item()
            beta[j] = bj
            if bj < 1e-14:
                mm = j + 1
                break
            Q[j + 1] = w / bj
        T = np.diag(alpha[:mm]) + np.diag(beta[: mm - 1], 1) + np.diag(beta[: mm - 1], -1)
        sigma = float(np.linalg.eigvalsh(T)[-1]) / kappa
        del Q
    di = torch.arange(n, device=device)
    S[di, di] += sigma
    return SystemSpec(H, S, n_occ=float(n // 4), kT=DEFAULT_KT,
                      meta=dict(kind="kpoint3d", cell_sites=(mx, my, mz), kpt=tuple(k), seed=seed,
                                kappa=kappa, sigma=sigma, orbitals_per_atom=orbitals_per_atom))
