"""Pins of the oracle local energy, energy and gradient against invariants of the mathematics."""
from math import comb

import numpy as np
import pytest

from oracle import made, pauli, vmc
from gen import molecular_integrals, jordan_wigner_terms, init_params


def _terms(N, seed=0):
    h1, h2 = molecular_integrals(N, seed)
    t = jordan_wigner_terms(h1, h2)
    return pauli.canonical_terms(t.x_mask, t.z_mask, t.coeff)


def _table_logpsi(basis, vec):
    """log psi for a tabulated amplitude vector over a sorted basis (0 elsewhere)."""
    def f(configs):
        configs = np.asarray(configs, dtype=np.uint64)
        j = np.minimum(np.searchsorted(basis, configs), len(basis) - 1)
        hit = basis[j] == configs
        amp = np.where(hit, vec[j], 0.0)
        with np.errstate(divide="ignore"):
            return np.log(np.abs(amp)), np.angle(amp)
    return f


@pytest.mark.parametrize("N,nu,nd", [(3, 1, 2), (4, 2, 2), (6, 3, 3)])
def test_eigenvector_local_energy_is_lambda_min(N, nu, nd):
    """E_loc(x) = lambda_min for every x where the ground eigenvector is not tiny."""
    terms = _terms(N)
    basis = pauli.sector_basis(2 * N, nu, nd)
    Hs = pauli.sector_block(terms, basis)
    assert np.max(np.abs(Hs - Hs.conj().T)) < 1e-13
    evals, evecs = np.linalg.eigh(Hs)
    psi0 = evecs[:, 0]
    keep = np.abs(psi0) > 1e-8
    el = vmc.local_energy_fn(terms, _table_logpsi(basis, psi0), basis[keep])
    scale = np.max(np.abs(Hs))
    assert np.max(np.abs(el - evals[0])) < 1e-9 * scale * len(basis) ** 0.5


@pytest.mark.parametrize("N,nu,nd,L,h,mode", [(3, 1, 2, 1, 8, 0), (4, 2, 2, 2, 16, 0), (5, 2, 3, 2, 12, 0),
                                              (3, 1, 2, 1, 8, 1), (4, 2, 2, 2, 16, 1)])
def test_exact_mean_of_local_energy(N, nu, nd, L, h, mode):
    """sum_x pi(x) E_loc(x) = <psi|H|psi>/<psi|psi> with zero imaginary part."""
    n = 2 * N
    terms = _terms(N)
    net = made.Net(n=n, n_layers=L, width=h, n_up=nu, n_dn=nd, phase_mode=mode)
    params = init_params(n, L, h, seed=5, std=0.6, phase_mode=mode)
    basis = pauli.sector_basis(n, nu, nd)
    la, ph, _ = made.forward(net, params, basis)
    psi = np.exp(la + 1j * ph)
    Hs = pauli.sector_block(terms, basis)
    ref = np.vdot(psi, Hs @ psi) / np.vdot(psi, psi)
    el = vmc.local_energy(terms, net, params, basis)
    pi = np.abs(psi) ** 2
    mean = np.sum(pi * el) / np.sum(pi)
    assert abs(ref.imag) < 1e-12
    assert abs(mean - ref) < 1e-11 * max(1.0, abs(ref))


def test_single_term_special_cases():
    """H = c Y_j, H = X_j, H = Z-only reduce to closed forms of Eq. local_energy_auto."""
    n = 6
    net = made.Net(n=n, n_layers=2, width=10)
    params = init_params(n, 2, 10, seed=8, std=0.5)
    xs = np.arange(1 << n, dtype=np.uint64)
    la, ph, _ = made.forward(net, params, xs)
    psi = np.exp(la + 1j * ph)
    j, c = 2, 0.7
    tY = pauli.canonical_terms([1 << j], [1 << j], [c])
    el = vmc.local_energy(tY, net, params, xs)
    bit = ((xs >> np.uint64(j)) & np.uint64(1)).astype(int)
    ref = c * (-1j) * (1 - 2 * bit) * psi[(xs ^ np.uint64(1 << j)).astype(int)] / psi
    np.testing.assert_allclose(el, ref, rtol=1e-13, atol=1e-14)
    tX = pauli.canonical_terms([1 << j], [0], [1.0])
    el = vmc.local_energy(tX, net, params, xs)
    np.testing.assert_allclose(el, psi[(xs ^ np.uint64(1 << j)).astype(int)] / psi, rtol=1e-13)
    tZ = pauli.canonical_terms([0, 0], [0b11, 0b100], [0.3, -0.2])
    el = vmc.local_energy(tZ, net, params, xs)
    b0 = (xs & 1).astype(int)
    b1 = ((xs >> np.uint64(1)) & np.uint64(1)).astype(int)
    b2 = ((xs >> np.uint64(2)) & np.uint64(1)).astype(int)
    ref = 0.3 * (1 - 2 * ((b0 + b1) % 2)) - 0.2 * (1 - 2 * b2)
    np.testing.assert_allclose(el, ref, atol=1e-15)


def conn_closed(N, nu, nd):
    t = 1
    for ns in (nu, nd):
        t += ns * (N - ns) + comb(ns, 2) * comb(N - ns, 2)
    return t + nu * (N - nu) * nd * (N - nd)


@pytest.mark.parametrize("N,nu,nd", [(3, 1, 2), (4, 2, 2), (5, 2, 3), (6, 3, 3)])
def test_connected_counts_and_grouped_sum(N, nu, nd):
    """Every sector sample has conn(N, nu, nd) connected configurations; grouped h reproduce E_loc."""
    n = 2 * N
    terms = _terms(N)
    basis = pauli.sector_basis(n, nu, nd)
    rng = np.random.default_rng(1)
    xs = rng.choice(basis, min(25, len(basis)), replace=False)
    diag, ent = vmc.connected(terms, xs, sector_filter=True)
    for gi, xp, hv in ent:
        assert len(gi) + 1 == conn_closed(N, nu, nd)
    # without the filter only exact zeros are dropped; every off-sector h is ~0
    diag2, ent2 = vmc.connected(terms, xs, sector_filter=False)
    np.testing.assert_array_equal(diag, diag2)
    for (g1, _, h1), (g2, _, h2) in zip(ent, ent2):
        extra = np.setdiff1d(g2, g1)
        assert set(g1.tolist()) <= set(g2.tolist())
        if len(extra):
            assert np.max(np.abs(h2[np.isin(g2, extra)])) < 1e-12
    net = made.Net(n=n, n_layers=2, width=12, n_up=nu, n_dn=nd)
    params = init_params(n, 2, 12, seed=3, std=0.5)
    el = vmc.local_energy(terms, net, params, xs)
    la, ph, _ = made.forward(net, params, xs)
    for i, (gi, xp, hv) in enumerate(ent):
        la_p, ph_p, _ = made.forward(net, params, xp)
        r = np.exp((la_p - la[i]) + 1j * (ph_p - ph[i]))
        tot = diag[i] + np.sum(hv * r)
        assert abs(tot - el[i]) < 1e-12 * max(1.0, np.sum(np.abs(hv)))


def test_local_energy_refuses_a_zero_amplitude_sample():
    """E_loc divides by psi(x): a sample outside the network's sector (psi = 0) is an error."""
    N = 3
    n = 2 * N
    terms = _terms(N)
    net = made.Net(n=n, n_layers=1, width=8, n_up=1, n_dn=2)
    params = init_params(n, 1, 8, seed=2, std=0.5)
    good = pauli.sector_basis(n, 1, 2)[:3]
    bad = pauli.sector_basis(n, 2, 1)[:1]
    vmc.local_energy(terms, net, params, good)
    with pytest.raises(ValueError):
        vmc.local_energy(terms, net, params, np.concatenate([good, bad]))


def _complex_terms(n, seed, K=40):
    """Random Pauli strings (odd and even numbers of Y, so complex folded coefficients) with real
    weights, and a pair that cancels: X_0 and X_0 Z_1 at equal weight give h = 0 wherever x_1 = 1."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << n, K).astype(np.uint64)
    z = rng.integers(0, 1 << n, K).astype(np.uint64)
    keep = x != 1
    x = np.append(x[keep], [1, 1]).astype(np.uint64)
    z = np.append(z[keep], [0, 2]).astype(np.uint64)
    c = np.append(rng.standard_normal(keep.sum()), [0.5, 0.5])
    return pauli.canonical_terms(x, z, c)


def test_connected_unfiltered_matches_dense_rows():
    """Without the sector filter, the connected entries of x are exactly the nonzero off-diagonal
    entries of row x of the dense H (built term by term, pinned to Kronecker products), with equal
    values, and the diagonal is H[x, x]; strings with an odd number of Y are included."""
    n = 6
    terms = _complex_terms(n, 4)
    assert np.any(pauli.popcount(terms["x"] & terms["z"]) % 2 == 1)
    H = pauli.dense_hamiltonian(terms, n)
    xs = np.arange(1 << n, dtype=np.uint64)
    diag, ent = vmc.connected(terms, xs, sector_filter=False)
    cancelled = 0
    for i, x in enumerate(xs.tolist()):
        row = H[x]
        assert abs(diag[i] - row[x]) <= 1e-14
        _, xp, hv = ent[i]
        nz = {j for j in np.nonzero(row)[0].tolist() if j != x}
        assert set(xp.tolist()) == nz
        for v, h in zip(xp.tolist(), hv):
            assert abs(h - row[v]) <= 1e-14
        cancelled += (x >> 1) & 1
    assert cancelled > 0                                 # the cancelling group was dropped somewhere


def test_sector_block_is_the_dense_block():
    n = 6
    terms = _complex_terms(n, 5)
    H = pauli.dense_hamiltonian(terms, n)
    for nu, nd in ((2, 1), (1, 2), (3, 3)):
        basis = pauli.sector_basis(n, nu, nd)
        idx = basis.astype(np.int64)
        np.testing.assert_allclose(pauli.sector_block(terms, basis), H[np.ix_(idx, idx)], atol=1e-14, rtol=0)


def test_energy_of_counts_equals_the_expanded_batch():
    """Count weights (the unique-sample buffer's counts) give the estimate of the batch in which each
    sample appears count times: the real and the imaginary mean and W."""
    rng = np.random.default_rng(8)
    el = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    cnt = rng.integers(1, 9, 50)
    E, I, W = vmc.energy(el, cnt)
    E2, I2, W2 = vmc.energy(np.repeat(el, cnt))
    assert W == W2 == cnt.sum()
    assert abs(E - E2) <= 1e-14 and abs(I - I2) <= 1e-14


def test_gradient_matches_fd_of_frozen_surrogate():
    """g equals the central FD (h = 1e-4) of F = sum (w/W) 2[(Re l - E) log|psi| + Im l phi] with E_loc frozen."""
    N, L, h = 4, 2, 16
    n = 2 * N
    terms = _terms(N)
    net = made.Net(n=n, n_layers=L, width=h, n_up=2, n_dn=2)
    params = init_params(n, L, h, seed=13, std=0.3).astype(np.float64)
    basis = pauli.sector_basis(n, 2, 2)
    rng = np.random.default_rng(2)
    xs = rng.choice(basis, 20, replace=False)
    w = rng.integers(1, 5, len(xs)).astype(float)
    el = vmc.local_energy(terms, net, params, xs)
    E, _, W = vmc.energy(el, w)
    g = vmc.gradient(net, params, xs, w, el, E)

    def F(p):
        la, ph, _ = made.forward(net, p, xs)
        return np.sum((w / W) * 2 * ((el.real - E) * la + el.imag * ph))

    idx = rng.choice(len(params), 20, replace=False)
    for k in idx:
        e = np.zeros_like(params)
        e[k] = 1e-4
        fd = (F(params + e) - F(params - e)) / 2e-4
        assert abs(fd - g[k]) < 1e-6 * max(1.0, np.max(np.abs(g)))


@pytest.mark.parametrize("mode", [0, 1])
def test_gradient_matches_fd_of_exact_energy(mode):
    """With exact weights pi over the sector, g = d/dtheta <psi|H|psi> (pins the factor 2 and the real baseline)."""
    N, L, h = 3, 2, 10
    n = 2 * N
    terms = _terms(N)
    net = made.Net(n=n, n_layers=L, width=h, n_up=1, n_dn=2, phase_mode=mode)
    params = init_params(n, L, h, seed=17, std=0.5, phase_mode=mode).astype(np.float64)
    basis = pauli.sector_basis(n, 1, 2)
    Hs = pauli.sector_block(terms, basis)

    def Eexact(p):
        la, ph, _ = made.forward(net, p, basis)
        psi = np.exp(la + 1j * ph)
        return (np.vdot(psi, Hs @ psi) / np.vdot(psi, psi)).real

    la, _, _ = made.forward(net, params, basis)
    pi = np.exp(2 * la)
    el = vmc.local_energy(terms, net, params, basis)
    E, _, _ = vmc.energy(el, pi)
    assert abs(E - Eexact(params)) < 1e-12
    g = vmc.gradient(net, params, basis, pi, el, E)
    rng = np.random.default_rng(4)
    # the last 200 parameters include every phase parameter (the head, and in mode 1 the sub-model)
    picks = np.concatenate([rng.choice(len(params) - 200, 15, replace=False),
                            len(params) - 200 + rng.choice(200, 15, replace=False)])
    for k in picks:
        e = np.zeros_like(params)
        e[k] = 1e-5
        fd = (Eexact(params + e) - Eexact(params - e)) / 2e-5
        assert abs(fd - g[k]) < 1e-7
    # score-function identity: sum_x pi d log pi = 0 (here for log|psi|)
    _, _, cache = made.forward(net, params, basis)
    gs = made.backward(net, params, cache, pi, np.zeros(len(basis)))
    assert np.max(np.abs(gs)) < 1e-12


def test_energy_weights_and_exact_sum():
    el = np.array([1e16 + 1j, 1.0, -1e16 - 1j, 3.0])
    E, I, W = vmc.energy(el, [1, 1, 1, 1])
    assert E == 1.0 and I == 0.0 and W == 4.0


@pytest.mark.parametrize("N,nu,nd", [(3, 1, 2), (4, 2, 2)])
def test_local_energy_scale_is_sum_of_absolute_summands(N, nu, nd):
    """S_i from local_energy(scale=True) equals sum_k |c_k| |psi(x ^ x_k)| / |psi(x)| built from the dense
    sector amplitudes and the unmerged per-term products (the sign and phase drop out of |.|), and
    bounds |E_loc| (the triangle inequality)."""
    n = 2 * N
    terms = _terms(N)
    net = made.Net(n=n, n_layers=2, width=16, n_up=nu, n_dn=nd)
    params = init_params(n, 2, 16, seed=7, std=0.5)
    basis = pauli.sector_basis(n, nu, nd)
    la, ph, _ = made.forward(net, params, basis)
    amp = dict(zip(basis.tolist(), np.exp(la).tolist()))
    el, S = vmc.local_energy(terms, net, params, basis, scale=True)
    assert np.allclose(el, vmc.local_energy(terms, net, params, basis), rtol=0, atol=0)
    for i, x in enumerate(basis.tolist()):
        ref = sum(abs(c) * amp.get(x ^ int(xk), 0.0) / amp[x] for xk, c in zip(terms["x"].tolist(), terms["ct"]))
        assert abs(S[i] - ref) <= 1e-13 * ref
        assert abs(el[i]) <= S[i] * (1 + 1e-13)
