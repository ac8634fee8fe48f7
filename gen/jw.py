"""Jordan-Wigner image of a second-quantized molecular Hamiltonian.

The Hamiltonian is

    H = sum_{pq,s} h1[p,q] a+_{ps} a_{qs}
      + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}

with spin-orbital index ``j = 2p + s``.  Under Jordan-Wigner each ladder
operator is a sum of two Pauli strings,

    a+_j = 1/2 Z_{<j} X_j - i/2 Z_{<j} Y_j,   a_j = 1/2 Z_{<j} X_j + i/2 Z_{<j} Y_j,

(|1> = occupied), and a product of ladder operators is expanded numerically in
the ``(x_mask, z_mask)`` representation ``P(x,z) = i^{popcount(x&z)} X^x Z^z``,
for which

    P(x1,z1) P(x2,z2) = i^{x1.z1 + x2.z2 + 2 z1.x2 - x.z} P(x1^x2, z1^z2).

Identical strings are merged by exact grouping, tiny coefficients dropped,
and the (necessarily real) coefficients returned.  This is input preparation
for the synthetic workloads, not part of the variational method.
"""
from dataclasses import dataclass

import numpy as np
import pandas as pd

_U1 = np.uint64(1)


@dataclass
class PauliTerms:
    """A Pauli-string Hamiltonian ``sum_k coeff[k] * P(x_mask[k], z_mask[k])``."""

    n_qubits: int
    x_mask: np.ndarray   # uint64 [K]
    z_mask: np.ndarray   # uint64 [K]
    coeff: np.ndarray    # float64 [K]

    def __len__(self):
        return int(self.x_mask.shape[0])


def _pc(v):
    return np.bitwise_count(v).astype(np.int64)


def _ladder_product(idx, dagger, coef):
    """Expand prod_f a^{dagger_f}_{idx_f} (times coef) into Pauli strings.

    ``idx`` is a list of int64 arrays (one per factor, same length), ``dagger``
    a list of bools.  Returns (x, z, re, im) arrays over tuples x 2^F choices.
    """
    F = len(idx)
    T = idx[0].shape[0]
    xs, zs, res, ims = [], [], [], []
    ej = [np.left_shift(_U1, f.astype(np.uint64)) for f in idx]
    mj = [e - _U1 for e in ej]
    scale = coef * (0.5 ** F)
    real_of = np.array([1.0, 0.0, -1.0, 0.0])
    imag_of = np.array([0.0, 1.0, 0.0, -1.0])
    for choice in range(1 << F):
        e = np.zeros(T, dtype=np.int64)
        x = np.zeros(T, dtype=np.uint64)
        z = np.zeros(T, dtype=np.uint64)
        for f in range(F):
            xf = ej[f]
            if (choice >> f) & 1:
                zf = mj[f] | ej[f]          # Z_{<j} Y_j, prefactor -i (a+) or +i (a)
                ef = 3 if dagger[f] else 1
            else:
                zf = mj[f]                  # Z_{<j} X_j, prefactor 1
                ef = 0
            xn = x ^ xf
            zn = z ^ zf
            e = e + ef + _pc(x & z) + _pc(xf & zf) + 2 * _pc(z & xf) - _pc(xn & zn)
            x, z = xn, zn
        e &= 3
        xs.append(x)
        zs.append(z)
        res.append(scale * real_of[e])
        ims.append(scale * imag_of[e])
    return (np.concatenate(xs), np.concatenate(zs),
            np.concatenate(res), np.concatenate(ims))


def _merge(frames):
    df = pd.concat(frames, ignore_index=True) if len(frames) > 1 else frames[0]
    g = df.groupby(["x", "z"], sort=True)[["re", "im"]].sum()
    out = g.reset_index()
    return out


def _frame(x, z, re, im):
    return pd.DataFrame({"x": x, "z": z, "re": re, "im": im})


def jordan_wigner_terms(h1, h2, drop_tol: float = 1e-10, chunk_pairs: int = 60000):
    """Pauli strings of the spin Hamiltonian built from integrals ``h1, h2``.

    Terms are merged (identical masks summed), entries with
    ``|coeff| < drop_tol`` removed, and the result sorted by (x_mask, z_mask).
    Raises if any merged coefficient keeps an imaginary part.
    """
    N = h1.shape[0]
    n = 2 * N
    if n > 64:
        raise ValueError("at most 64 qubits")
    frames = []

    # one-body: a+_{ps} a_{qs}
    p, q, s = np.meshgrid(np.arange(N), np.arange(N), np.arange(2), indexing="ij")
    p, q, s = p.ravel(), q.ravel(), s.ravel()
    c = h1[p, q]
    frames.append(_frame(*_ladder_product([2 * p + s, 2 * q + s], [True, False], c)))

    # two-body: pair index I=(s,p,q); term(I,J) and term(J,I) are the same
    # operator with the same integral, and term(I,I) vanishes, so sum I<J once.
    pairs = np.arange(2 * N * N)
    ps_, pp_, pq_ = pairs // (N * N), (pairs // N) % N, pairs % N
    I, J = np.triu_indices(2 * N * N, k=1)
    merged = None
    for start in range(0, I.shape[0], chunk_pairs):
        a, b = I[start:start + chunk_pairs], J[start:start + chunk_pairs]
        sp, P, Q = ps_[a], pp_[a], pq_[a]
        st, R, S = ps_[b], pp_[b], pq_[b]
        j1, j2, j3, j4 = 2 * P + sp, 2 * R + st, 2 * S + st, 2 * Q + sp
        keep = (j1 != j2) & (j3 != j4)
        coef = h2[P, Q, R, S]
        keep &= coef != 0.0
        if not np.any(keep):
            continue
        x, z, re, im = _ladder_product(
            [j1[keep], j2[keep], j3[keep], j4[keep]],
            [True, True, False, False], coef[keep])
        frames.append(_frame(x, z, re, im))
        if sum(len(f) for f in frames) > 8_000_000:
            merged = _merge(frames)
            frames = [merged]
    merged = _merge(frames)

    x = merged["x"].to_numpy(dtype=np.uint64)
    z = merged["z"].to_numpy(dtype=np.uint64)
    re = merged["re"].to_numpy(dtype=np.float64)
    im = merged["im"].to_numpy(dtype=np.float64)
    scale = max(1.0, float(np.max(np.abs(re))) if re.size else 1.0)
    if im.size and np.max(np.abs(im)) > 1e-12 * scale:
        raise RuntimeError("Jordan-Wigner expansion left an imaginary coefficient")
    keep = np.abs(re) >= drop_tol
    return PauliTerms(n, x[keep], z[keep], re[keep])
