"""Random molecular-like integrals with the locality and symmetry of real ones.

One-electron integrals: a symmetric matrix whose off-diagonal entries decay as
exp(-|p-q|/2) and whose diagonal rises linearly from -2 to -0.5 (orbital
energies sorted ascending).  Two-electron integrals in chemists' notation
(pq|rs): Gaussian entries of standard deviation 0.1 damped by
exp(-(|p-q|+|r-s|)/3), with the full 8-fold permutational symmetry of real
orbitals.  All randomness comes from one NumPy PCG64 stream per seed.
"""
import numpy as np


def molecular_integrals(n_orb: int, seed: int):
    """Return ``(h1[N,N], h2[N,N,N,N])`` in float64 for ``N = n_orb``."""
    N = int(n_orb)
    if N < 1:
        raise ValueError("need at least one spatial orbital")
    rng = np.random.Generator(np.random.PCG64(seed))
    g1 = rng.standard_normal((N, N))
    g2 = rng.standard_normal((N, N, N, N))

    p = np.arange(N)
    hi = np.maximum(p[:, None], p[None, :])
    lo = np.minimum(p[:, None], p[None, :])
    h1 = g1[hi, lo] * np.exp(-np.abs(p[:, None] - p[None, :]) / 2.0)
    if N > 1:
        h1[p, p] = -2.0 + 1.5 * p / (N - 1)
    else:
        h1[0, 0] = -2.0

    # canonical representative of each 8-fold symmetry class: (P>=Q, R>=S,
    # (P,Q) >= (R,S) lexicographically); every member reads the same draw.
    P, Q, R, S = np.meshgrid(p, p, p, p, indexing="ij")
    a, b = np.maximum(P, Q), np.minimum(P, Q)
    c, d = np.maximum(R, S), np.minimum(R, S)
    swap = (a < c) | ((a == c) & (b < d))
    A = np.where(swap, c, a)
    Bb = np.where(swap, d, b)
    C = np.where(swap, a, c)
    D = np.where(swap, b, d)
    damp = np.exp(-(np.abs(P - Q) + np.abs(R - S)) / 3.0)
    h2 = 0.1 * g2[A, Bb, C, D] * damp
    return h1, h2
