"""Pins of the oracle's Pauli layer and of the synthetic generator.

Everything is checked against objects built independently of the code under
test: the matrices printed in Eq. 1, Kronecker products, fermionic ladder
operators defined directly on occupation-number states, closed-form counts.
"""
import itertools
import os
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pauli
from gen import molecular_integrals, jordan_wigner_terms


def _read_sigma(golden_dir):
    mats, cur, name = {}, [], None
    for line in open(os.path.join(golden_dir, "pauli_matrices.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("sigma_"):
            name = int(line.split("_")[1])
            cur = []
            mats[name] = cur
            continue
        cur.append([complex(*map(float, e.split(","))) for e in line.split()])
    return {k: np.array(v) for k, v in mats.items()}


def test_sigma_matches_eq1(golden_dir):
    printed = _read_sigma(golden_dir)
    for k in range(4):
        np.testing.assert_array_equal(pauli.SIGMA[k], printed[k])


def _kron_string(labels, golden):
    # qubit j is the j-th least significant tensor factor
    m = np.array([[1.0 + 0j]])
    for j in reversed(range(len(labels))):
        m = np.kron(m, golden[labels[j]])
    return m


def test_matrix_element_rule_all_strings_n3(golden_dir):
    """Eq. mtx_element against Kronecker products for every 3-qubit string and every row."""
    golden = _read_sigma(golden_dir)
    n = 3
    for labels in itertools.product(range(4), repeat=n):
        xm = sum(1 << j for j, p in enumerate(labels) if p in (1, 2))
        zm = sum(1 << j for j, p in enumerate(labels) if p in (2, 3))
        M = _kron_string(labels, golden)
        for x in range(1 << n):
            row = M[x]
            nz = np.nonzero(row)[0]
            assert list(nz) == [x ^ xm]          # one nonzero per row (Sec. 3)
            assert row[x ^ xm] == pauli.matrix_element(x, xm, zm)


def test_dense_builder_matches_kron_sum(golden_dir):
    golden = _read_sigma(golden_dir)
    rng = np.random.default_rng(5)
    n = 4
    xs = rng.integers(0, 16, 30).astype(np.uint64)
    zs = rng.integers(0, 16, 30).astype(np.uint64)
    cs = rng.standard_normal(30)
    terms = pauli.canonical_terms(xs, zs, cs, drop_tol=0.0)
    H = pauli.dense_hamiltonian(terms, n)
    ref = np.zeros((16, 16), dtype=complex)
    for xm, zm, c in zip(terms["x"], terms["z"], terms["c"]):
        labels = pauli.pauli_labels(int(xm), int(zm), n)
        ref += c * _kron_string(labels, golden)
    np.testing.assert_allclose(H, ref, atol=1e-14)


def test_canonical_merge_drop_sort():
    xs = np.array([3, 1, 3, 0, 1, 2], dtype=np.uint64)
    zs = np.array([1, 0, 1, 5, 0, 2], dtype=np.uint64)
    cs = np.array([0.1, 0.2, 0.2, 1e-11, -0.2, 0.5])
    t = pauli.canonical_terms(xs, zs, cs)
    # (1,0): 0.2-0.2 = 0 dropped; (0,5): 1e-11 dropped; (3,1): 0.1+0.2 merged in input order
    assert t["x"].tolist() == [2, 3]
    assert t["z"].tolist() == [2, 1]
    assert t["c"][1] == 0.1 + 0.2
    # (2,2): one Y at qubit 1 -> (-i)^1;  (3,1): one Y -> (-i)
    assert t["ct"][0] == -0.5j and t["ct"][1] == -1j * (0.1 + 0.2)
    with pytest.raises(ValueError):
        pauli.canonical_terms(xs, zs, cs, coeff_imag=np.full(6, 1e-3))


def test_canonical_drop_threshold_after_merge():
    """The 1e-10 cut applies to merged coefficients: 2e-10 stays, 5e-11 goes, and two strings of 6e-11
    that merge to 1.2e-10 stay although each alone would go."""
    xs = np.array([1, 2, 4, 4], dtype=np.uint64)
    zs = np.array([0, 0, 0, 0], dtype=np.uint64)
    cs = np.array([2e-10, 5e-11, 6e-11, 6e-11])
    t = pauli.canonical_terms(xs, zs, cs, drop_tol=1e-10)
    assert t["x"].tolist() == [1, 4]
    assert t["c"].tolist() == [2e-10, 6e-11 + 6e-11]


# ---------------------------------------------------------------- generator

def _ladder_ops(n):
    """Annihilators a_j on the 2^n occupation basis: a_j|x> = (-1)^{sum_{k<j} x_k} |x - e_j>."""
    dim = 1 << n
    ops = []
    for j in range(n):
        rows, cols, vals = [], [], []
        for x in range(dim):
            if (x >> j) & 1:
                sgn = -1.0 if bin(x & ((1 << j) - 1)).count("1") % 2 else 1.0
                rows.append(x ^ (1 << j))
                cols.append(x)
                vals.append(sgn)
        ops.append(sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim)))
    return ops


def _fermionic_h(h1, h2):
    N = h1.shape[0]
    n = 2 * N
    a = _ladder_ops(n)
    ad = [m.T.tocsr() for m in a]
    H = sp.csr_matrix((1 << n, 1 << n))
    for p in range(N):
        for q in range(N):
            for s in range(2):
                H = H + h1[p, q] * (ad[2 * p + s] @ a[2 * q + s])
    for p, q, r, s_ in itertools.product(range(N), repeat=4):
        c = h2[p, q, r, s_]
        for s in range(2):
            for t in range(2):
                H = H + 0.5 * c * (ad[2 * p + s] @ ad[2 * r + t] @ a[2 * s_ + t] @ a[2 * q + s])
    return H.toarray()


@pytest.mark.parametrize("N", [2, 3, 4])
def test_jw_generator_matches_fermionic_hamiltonian(N):
    h1, h2 = molecular_integrals(N, seed=0)
    terms = jordan_wigner_terms(h1, h2, drop_tol=0.0)
    t = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff, drop_tol=0.0)
    H = pauli.dense_hamiltonian(t, 2 * N)
    Hf = _fermionic_h(h1, h2)
    np.testing.assert_allclose(H, Hf, atol=1e-13)
    # Hermitian, real, commutes with the spin-resolved number operators
    assert np.max(np.abs(H - H.conj().T)) <= 1e-13 * np.max(np.abs(H))
    assert np.max(np.abs(H.imag)) < 1e-14
    dim = 1 << (2 * N)
    xs = np.arange(dim, dtype=np.uint64)
    nup = pauli.popcount(xs & np.uint64(0x5555555555555555))
    ndn = pauli.popcount(xs & np.uint64(0xAAAAAAAAAAAAAAAA))
    for occ in (nup, ndn):
        D = np.diag(occ.astype(float))
        assert np.max(np.abs(H @ D - D @ H)) < 1e-12


def k_closed(N):
    return 1 + 2 * N + N * (2 * N - 1) + 4 * (2 * N - 1) * comb(N, 2) + 4 * comb(N, 2) ** 2 + 12 * comb(N, 4)


def g_closed(N):
    # empty flip; same-spin pairs (2 spins); same-spin quadruples; opposite-spin pair pairs
    return 1 + 2 * comb(N, 2) + 2 * comb(N, 4) + comb(N, 2) ** 2


@pytest.mark.parametrize("N", [3, 4, 5, 6])
def test_term_and_group_counts_closed_form(N):
    h1, h2 = molecular_integrals(N, seed=0)
    terms = jordan_wigner_terms(h1, h2)
    t = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    assert len(t["x"]) == k_closed(N)
    gx, goff = pauli.groups(t)
    assert len(gx) == g_closed(N)
    sizes = np.diff(goff)
    pc = pauli.popcount(gx)
    up = pauli.popcount(gx & np.uint64(0x5555555555555555))
    assert sizes[0] == 1 + 2 * N + N * (2 * N - 1)            # diagonal group
    assert np.all(sizes[pc == 2] == 2 * (2 * N - 1))          # singles
    four = pc == 4
    assert np.all(sizes[four & ((up == 4) | (up == 0))] == 6)  # same-spin doubles
    assert np.all(sizes[four & (up == 2)] == 4)                # opposite-spin doubles
    # no odd number of Y factors (real symmetric H)
    assert np.all(pauli.popcount(t["x"] & t["z"]) % 2 == 0)


def test_sector_size_formula_table1(golden_dir):
    """Sector sizes C(n/2, N_up) C(n/2, N_dn) (Sec. 4 Constraints) for Table 1 molecules."""
    for line in open(os.path.join(golden_dir, "paper_counts.txt")):
        if line.startswith("#") or line.startswith("methanol") or not line.strip():
            continue
        name, n, nu, nd = line.split()
        n, nu, nd = int(n), int(nu), int(nd)
        if n > 16:
            continue
        assert len(pauli.sector_basis(n, nu, nd)) == comb(n // 2, nu) * comb(n // 2, nd)


def test_methanol_forward_count(golden_dir):
    line = [l for l in open(os.path.join(golden_dir, "paper_counts.txt")) if l.startswith("methanol")][0]
    kv = dict(f.split("=") for f in line.split()[1:])
    n, K, B = int(kv["n"]), int(kv["K"]), int(kv["B"])
    assert round(B * K / 1e6) == int(kv["forward_inputs_millions"])
    assert abs(4.0 ** n / float(kv["four_pow_n"]) - 1) < 0.01
