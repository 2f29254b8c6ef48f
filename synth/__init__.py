"""Seeded synthetic inputs (Hamiltonian / overlap pairs) for the dense Kohn-Sham path.

This package only *builds inputs*: Gaussian-basis overlap matrices, an
extended-Hueckel-like Hamiltonian and the closed-form test pencils.  It holds
none of the solver's arithmetic and is shared by the GPU library's tests and
benchmark and by the CPU oracle's tests alike.
"""
from .generator import (  # noqa: F401
    HARTREE_PER_EV,
    SystemSpec,
    batch_sizes,
    build_system,
    chain_positions,
    lattice_positions,
    make_config,
    make_lattice_system,
    s_gaussian_overlap,
    tight_binding_chain,
    toeplitz_pencil,
)
