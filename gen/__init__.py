"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package only *produces inputs*: molecular-like one- and two-electron
integrals, their Jordan-Wigner image as a list of Pauli strings, network
parameters, and bit-string samples.  It contains none of the variational Monte
Carlo arithmetic (no amplitudes, no local energies, no gradients); both the
CPU oracle and the HIP library consume what it returns.

The Pauli-string encoding used throughout is a pair of 64-bit masks
``(x_mask, z_mask)``: qubit ``j`` is bit ``j``; the single-qubit factor on qubit
``j`` is identity, X, Z or Y for ``(x_j, z_j) = (0,0), (1,0), (0,1), (1,1)``.
Spin-orbital ``j = 2p + sigma`` (``sigma = 0`` up, ``1`` down), so even qubits
carry spin up.  The paper's first qubit ``x_1`` is bit 0.
"""
from .integrals import molecular_integrals
from .jw import jordan_wigner_terms, PauliTerms
from .inputs import (hamiltonian, init_params, param_count, round_bf16, sector_samples,
                     unique_with_counts, CONFIGS, config_inputs)

__all__ = [
    "molecular_integrals", "jordan_wigner_terms", "PauliTerms", "hamiltonian",
    "init_params", "param_count", "round_bf16", "sector_samples", "unique_with_counts",
    "CONFIGS", "config_inputs",
]
