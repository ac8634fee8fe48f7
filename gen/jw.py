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
_ALL = ~np.uint64(0)


@dataclass
class PauliTerms:
    """A Pauli-string Hamiltonian ``sum_k coeff[k] * P(x_mask[k], z_mask[k])``.

    Masks are uint64 ``[K]`` for up to 64 qubits and uint64 ``[K, W]`` words
    (word w = qubits 64w .. 64w+63) above.
    """

    n_qubits: int
    x_mask: np.ndarray   # uint64 [K] or [K, W]
    z_mask: np.ndarray   # uint64 [K] or [K, W]
    coeff: np.ndarray    # float64 [K]

    def __len__(self):
        return int(self.x_mask.shape[0])


def _pc(v):
    """Population count of [T, W] words, summed over the words."""
    return np.bitwise_count(v).astype(np.int64).sum(axis=1)


def _unit(j, W):
    """Words of the mask with bit j set."""
    out = np.zeros((j.shape[0], W), dtype=np.uint64)
    for w in range(W):
        inw = (j >= 64 * w) & (j < 64 * (w + 1))
        out[inw, w] = np.left_shift(_U1, (j[inw] - 64 * w).astype(np.uint64))
    return out


def _below(j, W):
    """Words of the mask with bits 0 .. j-1 set (the Jordan-Wigner Z string of qubit j)."""
    out = np.zeros((j.shape[0], W), dtype=np.uint64)
    for w in range(W):
        full = j >= 64 * (w + 1)
        out[full, w] = _ALL
        part = (j > 64 * w) & ~full
        out[part, w] = np.left_shift(_U1, (j[part] - 64 * w).astype(np.uint64)) - _U1
    return out


def _ladder_product(idx, dagger, coef, W):
    """Expand prod_f a^{dagger_f}_{idx_f} (times coef) into Pauli strings.

    ``idx`` is a list of int64 arrays (one per factor, same length), ``dagger``
    a list of bools.  Returns (x [., W], z [., W], re, im) over tuples x 2^F
    choices.
    """
    F = len(idx)
    T = idx[0].shape[0]
    xs, zs, res, ims = [], [], [], []
    ej = [_unit(f, W) for f in idx]
    mj = [_below(f, W) for f in idx]
    scale = coef * (0.5 ** F)
    real_of = np.array([1.0, 0.0, -1.0, 0.0])
    imag_of = np.array([0.0, 1.0, 0.0, -1.0])
    for choice in range(1 << F):
        e = np.zeros(T, dtype=np.int64)
        x = np.zeros((T, W), dtype=np.uint64)
        z = np.zeros((T, W), dtype=np.uint64)
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


def _keys(W):
    # most significant word first, so the grouping sorts masks as unsigned integers
    return [f"x{w}" for w in reversed(range(W))] + [f"z{w}" for w in reversed(range(W))]


def _merge(frames, W):
    df = pd.concat(frames, ignore_index=True) if len(frames) > 1 else frames[0]
    g = df.groupby(_keys(W), sort=True)[["re", "im"]].sum()
    out = g.reset_index()
    return out


def _frame(x, z, re, im):
    cols = {f"x{w}": x[:, w] for w in range(x.shape[1])}
    cols.update({f"z{w}": z[:, w] for w in range(z.shape[1])})
    cols.update({"re": re, "im": im})
    return pd.DataFrame(cols)


def jordan_wigner_terms(h1, h2, drop_tol: float = 1e-10, chunk_pairs: int = 60000):
    """Pauli strings of the spin Hamiltonian built from integrals ``h1, h2``.

    Terms are merged (identical masks summed), entries with
    ``|coeff| < drop_tol`` removed, and the result sorted by (x_mask, z_mask).
    Raises if any merged coefficient keeps an imaginary part.
    """
    N = h1.shape[0]
    n = 2 * N
    if n > 128:
        raise ValueError("at most 128 qubits")
    W = (n + 63) // 64
    frames = []

    # one-body: a+_{ps} a_{qs}
    p, q, s = np.meshgrid(np.arange(N), np.arange(N), np.arange(2), indexing="ij")
    p, q, s = p.ravel(), q.ravel(), s.ravel()
    c = h1[p, q]
    frames.append(_frame(*_ladder_product([2 * p + s, 2 * q + s], [True, False], c, W)))

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
            [True, True, False, False], coef[keep], W)
        frames.append(_frame(x, z, re, im))
        if sum(len(f) for f in frames) > 8_000_000:
            merged = _merge(frames, W)
            frames = [merged]
    merged = _merge(frames, W)

    x = np.stack([merged[f"x{w}"].to_numpy(dtype=np.uint64) for w in range(W)], axis=1)
    z = np.stack([merged[f"z{w}"].to_numpy(dtype=np.uint64) for w in range(W)], axis=1)
    if W == 1:
        x, z = x[:, 0], z[:, 0]
    re = merged["re"].to_numpy(dtype=np.float64)
    im = merged["im"].to_numpy(dtype=np.float64)
    scale = max(1.0, float(np.max(np.abs(re))) if re.size else 1.0)
    if im.size and np.max(np.abs(im)) > 1e-12 * scale:
        raise RuntimeError("Jordan-Wigner expansion left an imaginary coefficient")
    keep = np.abs(re) >= drop_tol
    return PauliTerms(n, x[keep], z[keep], re[keep])
