"""Pauli strings, the canonical term set, and dense Hamiltonians (FP64).

Encoding (reading of Sec. 3 and Eq. mtx_element): a Pauli string is a pair of
bit masks (x, z); qubit j is bit j (the paper's x_{j+1}); its factor is
sigma_0, sigma_1, sigma_3, sigma_2 for (x_j, z_j) = (0,0), (1,0), (0,1), (1,1).
With sigma_2 = i sigma_1 sigma_3 the string equals i^{popcount(x&z)} X^x Z^z.

Parity unpinned: nothing here; every function is pinned by tests against the
2x2 matrices of Eq. 1, Kronecker products and fermionic operators.
"""
import numpy as np

# Eq. 1
SIGMA = (
    np.array([[1, 0], [0, 1]], dtype=np.complex128),
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


_W64 = (1 << 64) - 1


def configs(v):
    """Bit strings as an array: uint64 when given as uint64 (up to 64 qubits),
    Python integers (dtype object) when given so (any width).  A uint64
    [B, W] array of words (word w = qubits 64w .. 64w+63) becomes Python
    integers."""
    a = np.asarray(v)
    if a.dtype == object:
        return a
    a = a.astype(np.uint64)
    if a.ndim == 2:
        out = np.empty(a.shape[0], dtype=object)
        for i, row in enumerate(a.tolist()):
            out[i] = sum(int(w) << (64 * k) for k, w in enumerate(row))
        return out
    return a


def popcount(v):
    a = np.asarray(v)
    if a.dtype == object:
        # Python integers: the counts of their 64-bit words, added
        total = np.zeros(a.shape, dtype=np.int64)
        rest = a
        while True:
            word = (rest & _W64).astype(np.uint64)
            total += np.bitwise_count(word).astype(np.int64)
            rest = rest >> 64
            if not np.any(rest != 0):
                return total
    return np.bitwise_count(a.astype(np.uint64)).astype(np.int64)


def pauli_labels(x_mask: int, z_mask: int, n: int):
    """Per-qubit labels p_j in {0,1,2,3} of the string (x_mask, z_mask)."""
    out = []
    for j in range(n):
        xb, zb = (x_mask >> j) & 1, (z_mask >> j) & 1
        out.append({(0, 0): 0, (1, 0): 1, (1, 1): 2, (0, 1): 3}[(xb, zb)])
    return out


def pauli_string_matrix(x_mask: int, z_mask: int, n: int):
    """Dense 2^n matrix of sigma_{p_1} (x) ... (x) sigma_{p_n} (Eq. hamiltonpauli).

    The basis index of |x> is the integer with bit j = x_{j+1}, so qubit j is
    the j-th least significant factor: the Kronecker product is taken with
    qubit n-1 leftmost.
    """
    labels = pauli_labels(x_mask, z_mask, n)
    m = np.array([[1.0 + 0j]])
    for j in reversed(range(n)):
        m = np.kron(m, SIGMA[labels[j]])
    return m


def matrix_element(x, x_mask, z_mask):
    """<x|P|x ^ x_mask> by Eq. mtx_element: (-i)^r prod_{Y,Z positions} (-1)^{x_k}.

    r = number of sigma_2 factors = popcount(x_mask & z_mask); the sign uses
    the row configuration x (reading: the sample is the bra).
    """
    r = bin(int(x_mask) & int(z_mask)).count("1")
    sign = -1.0 if (bin(int(x) & int(z_mask)).count("1") & 1) else 1.0
    return ((-1j) ** r) * sign


def canonical_terms(x_mask, z_mask, coeff, coeff_imag=None, drop_tol=1e-10):
    """Merged, filtered, sorted term set with the i-phase folded in.

    Steps (Sec. 5.1: parse once, keep unique flips, before training):
      1. identical (x, z) merged by sequential FP64 addition in input order;
      2. merged terms with |c| < drop_tol removed;
      3. coefficients must be real (the Pauli coefficients of a Hermitian
         matrix are real, Sec. 3) -- a nonzero imaginary part is an error;
      4. ct = c * (-i)^{popcount(x&z)} (the r-dependent factor of
         Eq. mtx_element), complex in general;
      5. sorted by (x ascending, z ascending) as unsigned integers.
    Returns dict with arrays x, z (uint64, or Python integers when the masks
    are given as Python integers or as [K, W] words), complex128 ct, float64 c.
    """
    x_mask = configs(x_mask)
    z_mask = configs(z_mask)
    wide = x_mask.dtype == object
    coeff = np.asarray(coeff, dtype=np.float64)
    if coeff_imag is not None:
        coeff_imag = np.asarray(coeff_imag, dtype=np.float64)
        if np.any(coeff_imag != 0.0):
            raise ValueError("Pauli coefficients of a Hermitian H must be real")
    acc = {}
    order = []
    for xv, zv, cv in zip(x_mask.tolist(), z_mask.tolist(), coeff.tolist()):
        key = (xv, zv)
        if key in acc:
            acc[key] = acc[key] + cv
        else:
            acc[key] = cv
            order.append(key)
    keys = [k for k in order if abs(acc[k]) >= drop_tol]
    keys.sort()
    x = np.empty(len(keys), dtype=object) if wide else np.zeros(len(keys), dtype=np.uint64)
    z = np.empty(len(keys), dtype=object) if wide else np.zeros(len(keys), dtype=np.uint64)
    for i, k in enumerate(keys):
        x[i], z[i] = k
    c = np.array([acc[k] for k in keys], dtype=np.float64)
    r = popcount(x & z)
    phase = np.array([1, -1j, -1, 1j], dtype=np.complex128)[r % 4]
    return {"x": x, "z": z, "c": c, "ct": c * phase}


def groups(terms):
    """Flip groups of a canonical term set: unique x masks and term ranges."""
    x = terms["x"]
    gx, start = np.unique(x, return_index=True)
    goff = np.append(start, len(x)).astype(np.int64)
    return gx, goff


def dense_hamiltonian(terms, n):
    """Dense H with H[x, x ^ x_k] += ct_k (-1)^{popcount(x & z_k)} (row x is the bra)."""
    if n > 14:
        raise ValueError("dense H only for n <= 14")
    dim = 1 << n
    H = np.zeros((dim, dim), dtype=np.complex128)
    rows = np.arange(dim, dtype=np.uint64)
    for xm, zm, ct in zip(terms["x"], terms["z"], terms["ct"]):
        sign = 1.0 - 2.0 * (popcount(rows & zm) & 1)
        cols = (rows ^ xm).astype(np.int64)
        H[rows.astype(np.int64), cols] += ct * sign
    return H


def sector_basis(n, n_up, n_dn):
    """All n-bit strings with n_up ones on even qubits and n_dn on odd qubits (Eq. hamming_weight_constraint)."""
    allx = np.arange(1 << n, dtype=np.uint64)
    up = np.uint64(int("01" * 32, 2) & ((1 << n) - 1))
    dn = np.uint64(int("10" * 32, 2) & ((1 << n) - 1))
    keep = (popcount(allx & up) == n_up) & (popcount(allx & dn) == n_dn)
    return allx[keep]


def sector_block(terms, basis):
    """Hamiltonian restricted to the span of ``basis`` (sorted uint64 array)."""
    basis = np.asarray(basis, dtype=np.uint64)
    m = len(basis)
    rows = np.arange(m)
    Hs = np.zeros((m, m), dtype=np.complex128)
    for xm, zm, ct in zip(terms["x"], terms["z"], terms["ct"]):
        sign = 1.0 - 2.0 * (popcount(basis & zm) & 1)
        cols = basis ^ xm
        j = np.minimum(np.searchsorted(basis, cols), m - 1)
        hit = basis[j] == cols
        np.add.at(Hs, (rows[hit], j[hit]), ct * sign[hit])
    return Hs
