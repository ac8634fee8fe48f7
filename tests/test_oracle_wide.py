"""Pins of the oracle above 64 qubits, where bit strings are Python integers.

The oracle runs the same code for every width; what changes above 64 qubits
is the representation (Python integers in place of uint64), the bit and
population-count helpers and the spin masks.  These tests pin each of them to
brute force, pin the two-word form of the Hamiltonian generator to its
one-word form, and pin the whole local-energy chain across the word boundary
to an eigenvector of the sector block and to relabelling invariance.
"""
import numpy as np
import pytest

from oracle import made, pauli, vmc
from gen import molecular_integrals, jordan_wigner_terms, init_params
from gen.inputs import hamiltonian, sector_samples


def _ints(words):
    """[B, W] uint64 words -> list of Python integers (test-side conversion)."""
    return [sum(int(w) << (64 * k) for k, w in enumerate(row)) for row in np.asarray(words).tolist()]


def _obj(vals):
    a = np.empty(len(vals), dtype=object)
    for i, v in enumerate(vals):
        a[i] = int(v)
    return a


def test_wide_popcount_bits_and_sector_test_by_brute_force():
    rng = np.random.default_rng(7)
    vals = [int(rng.integers(0, 2**63)) | (int(rng.integers(0, 2**63)) << 63) | (int(rng.integers(0, 4)) << 126)
            for _ in range(200)]
    vals += [0, 1 << 64, (1 << 128) - 1, (1 << 64) - 1, 1 << 127]
    a = _obj(vals)
    assert pauli.popcount(a).tolist() == [bin(v).count("1") for v in vals]
    n = 128
    net = made.Net(n=n, n_layers=1, width=8)
    xb = made.bits(net, a)
    assert xb.tolist() == [[(v >> j) & 1 for j in range(n)] for v in vals]
    flips = _obj(vals[::-1])
    ok = vmc.sector_valid(a, flips)
    for v, f, k in zip(vals, vals[::-1], ok.tolist()):
        y = v ^ f
        up = lambda u: sum((u >> j) & 1 for j in range(0, n, 2))
        dn = lambda u: sum((u >> j) & 1 for j in range(1, n, 2))
        assert k == (up(v) == up(y) and dn(v) == dn(y))


def test_words_to_integers():
    w = np.array([[5, 0], [0, 1], [2**64 - 1, 2**63]], dtype=np.uint64)
    assert pauli.configs(w).tolist() == [5, 1 << 64, (2**64 - 1) | (1 << 127)]


def test_two_word_generator_is_the_shifted_one_word_generator():
    """Integrals of 6 orbitals placed on orbitals 30..35 of 36 (qubits 60..71,
    across the word boundary): the Jordan-Wigner strings of the embedded
    system are those of the small system shifted by 60 bits (the Z strings
    below the block cancel in every product of ladder operators), with the
    same coefficients (up to the order in which merged contributions are
    added, which follows the chunking of the pair loop)."""
    m, N, P0 = 6, 36, 30
    h1s, h2s = molecular_integrals(m, 0)
    h1 = np.zeros((N, N))
    h2 = np.zeros((N, N, N, N))
    h1[P0:, P0:] = h1s
    h2[P0:, P0:, P0:, P0:] = h2s
    big = jordan_wigner_terms(h1, h2)
    small = jordan_wigner_terms(h1s, h2s)
    assert big.x_mask.shape == (len(small), 2)
    bx, bz = _ints(big.x_mask), _ints(big.z_mask)
    sx = [int(v) << (2 * P0) for v in small.x_mask.tolist()]
    sz = [int(v) << (2 * P0) for v in small.z_mask.tolist()]
    assert bx == sx and bz == sz
    assert np.max(np.abs(big.coeff - small.coeff)) <= 1e-14 * np.max(np.abs(small.coeff))
    assert any(v >> 64 for v in bx) and any(v & ((1 << 64) - 1) for v in bx)


def test_wide_local_energy_of_the_embedded_eigenvector_is_lambda_min():
    """E_loc over Python-integer bit strings at 72 qubits equals lambda_min of
    the embedded 12-qubit sector block when psi is its ground eigenvector."""
    m, N, P0 = 6, 36, 30
    h1s, h2s = molecular_integrals(m, 0)
    h1 = np.zeros((N, N))
    h2 = np.zeros((N, N, N, N))
    h1[P0:, P0:] = h1s
    h2[P0:, P0:, P0:, P0:] = h2s
    t = jordan_wigner_terms(h1, h2)
    terms = pauli.canonical_terms(t.x_mask, t.z_mask, t.coeff)
    assert terms["x"].dtype == object
    small = pauli.canonical_terms(*[getattr(jordan_wigner_terms(h1s, h2s), k) for k in ("x_mask", "z_mask", "coeff")])
    basis = pauli.sector_basis(2 * m, 3, 3)
    Hs = pauli.sector_block(small, basis)
    evals, evecs = np.linalg.eigh(Hs)
    psi0 = evecs[:, 0]
    shift = 2 * P0
    low = 0b1011_0110_0101                         # fixed occupation of qubits 0..11 (any value)
    table = {(int(b) << shift) | low: v for b, v in zip(basis.tolist(), psi0)}

    def logpsi(cfg):
        amp = np.array([table.get(int(c), 0.0) for c in cfg])
        with np.errstate(divide="ignore"):
            return np.log(np.abs(amp)), np.angle(amp)

    keep = np.abs(psi0) > 1e-8
    samples = _obj([(int(b) << shift) | low for b in basis[keep].tolist()])
    el = vmc.local_energy_fn(terms, logpsi, samples)
    assert np.max(np.abs(el - evals[0])) < 1e-9 * np.max(np.abs(Hs)) * len(basis) ** 0.5


@pytest.mark.parametrize("mode", [0, 1])
def test_wide_matches_narrow_at_12_qubits(mode):
    """Same inputs as uint64 and as Python integers: identical local energies,
    connected sets and gradients (the two representations share every step)."""
    N, L, h = 6, 1, 16
    n = 2 * N
    h1, h2 = molecular_integrals(N, 0)
    t = jordan_wigner_terms(h1, h2)
    tn = pauli.canonical_terms(t.x_mask, t.z_mask, t.coeff)
    tw = pauli.canonical_terms(_obj(t.x_mask.tolist()), _obj(t.z_mask.tolist()), t.coeff)
    net = made.Net(n=n, n_layers=L, width=h, n_up=3, n_dn=3, phase_mode=mode)
    params = init_params(n, L, h, seed=4, std=0.5, phase_mode=mode)
    xs = sector_samples(n, 3, 3, 24, seed=3)
    el_n = vmc.local_energy(tn, net, params, xs)
    el_w = vmc.local_energy(tw, net, params, _obj(xs.tolist()))
    assert np.array_equal(el_n, el_w)
    dn, cn = vmc.connected(tn, xs)
    dw, cw = vmc.connected(tw, _obj(xs.tolist()))
    assert np.array_equal(dn, dw)
    for (gi_n, xp_n, h_n), (gi_w, xp_w, h_w) in zip(cn, cw):
        assert np.array_equal(gi_n, gi_w) and np.array_equal(h_n, h_w)
        assert [int(v) for v in xp_n.tolist()] == [int(v) for v in xp_w.tolist()]
    E, _, _ = vmc.energy(el_n)
    g_n = vmc.gradient(net, params, xs, None, el_n, E)
    g_w = vmc.gradient(net, params, _obj(xs.tolist()), None, el_w, E)
    assert np.array_equal(g_n, g_w)


def _relabel_params(params, n, L, h, pi):
    """Parameters of the same network after qubit j is renamed pi[j]: the
    columns of W_1 and the rows of W_o, b_o are indexed by qubit."""
    p = params.copy()
    W1 = params[:h * n].reshape(h, n)
    p[:h * n] = W1[:, np.argsort(pi)].ravel()
    o = h * n + h + (L - 1) * (h * h + h)
    Wo = params[o:o + n * h].reshape(n, h)
    p[o:o + n * h] = Wo[np.argsort(pi)].ravel()
    bo = params[o + n * h:o + n * h + n]
    p[o + n * h:o + n * h + n] = bo[np.argsort(pi)]
    return p


def _relabel_int(v, pi):
    out = 0
    j = 0
    while v:
        if v & 1:
            out |= 1 << int(pi[j])
        v >>= 1
        j += 1
    return out


def test_wide_local_energy_is_invariant_under_relabelling_across_the_word_boundary():
    """Renaming qubit j to pi(j) = (j + 40) mod 72 (parity kept, so spins are
    kept) in the Hamiltonian, the samples, the sampling order and the
    parameters leaves every local energy unchanged: the renaming moves 32
    qubits from the low word to the high word and 32 the other way."""
    N, L, h = 36, 2, 16
    n = 2 * N
    pi = (np.arange(n) + 40) % n
    t = hamiltonian(N, 0, cutoff=0.05)
    xi, zi = _ints(t.x_mask), _ints(t.z_mask)
    ta = pauli.canonical_terms(_obj(xi), _obj(zi), t.coeff)
    tb = pauli.canonical_terms(_obj([_relabel_int(v, pi) for v in xi]), _obj([_relabel_int(v, pi) for v in zi]),
                               t.coeff)
    order = np.arange(n - 1, -1, -1)
    na = made.Net(n=n, n_layers=L, width=h, n_up=18, n_dn=18, order=order)
    nb = made.Net(n=n, n_layers=L, width=h, n_up=18, n_dn=18, order=pi[order])
    pa = init_params(n, L, h, seed=6, std=0.3)
    pb = _relabel_params(pa, n, L, h, pi)
    xs = _ints(sector_samples(n, 18, 18, 6, seed=9))
    la, fa = vmc.log_psi(na, pa, _obj(xs))
    lb, fb = vmc.log_psi(nb, pb, _obj([_relabel_int(v, pi) for v in xs]))
    assert np.allclose(la, lb, rtol=0, atol=1e-12) and np.allclose(fa, fb, rtol=0, atol=1e-12)
    ea = vmc.local_energy(ta, na, pa, _obj(xs))
    eb = vmc.local_energy(tb, nb, pb, _obj([_relabel_int(v, pi) for v in xs]))
    scale = np.sum(np.abs(t.coeff))
    assert np.max(np.abs(ea - eb)) < 1e-12 * scale


def test_wide_sampler_counter_and_properties():
    """The sampler's counter carries the configuration's high word in its third
    word (zero up to 64 qubits, so one-word draws are unchanged); at 66 qubits
    with an unbounded buffer every draw is kept (counts sum to n_draws), the
    configurations are distinct and in the sector, and the draws of the first
    position split binomially with the network's conditional there."""
    from oracle import sampler
    x = (1 << 63) | 12345
    assert sampler.split_draws(1000, 0.3, x, 5, 9) == sampler.binomial(1000, 0.3, sampler.Uniforms((x, 5, 0), (9, 0)))
    xw = x | (7 << 64)
    assert sampler.split_draws(1000, 0.3, xw, 5, 9) == sampler.binomial(1000, 0.3, sampler.Uniforms((x, 5, 7), (9, 0)))
    assert sampler.split_draws(1000, 0.3, xw, 5, 9) != sampler.split_draws(1000, 0.3, x, 5, 9) or \
        sampler.split_draws(1000, 0.3, xw, 6, 9) != sampler.split_draws(1000, 0.3, x, 6, 9)
    n, L, h, draws = 66, 1, 16, 20000
    net = made.Net(n=n, n_layers=L, width=h, n_up=2, n_dn=2)
    params = init_params(n, L, h, seed=3, std=0.5)
    xs, cs = sampler.sample(net, params, draws, seed=4, max_unique=10**9)
    assert xs.dtype == object and int(cs.sum()) == draws and np.all(cs > 0)
    assert len(set(int(v) for v in xs)) == len(xs)
    xb = made.bits(net, xs)
    assert np.all(xb[:, 0::2].sum(axis=1) == 2) and np.all(xb[:, 1::2].sum(axis=1) == 2)
    assert any(int(v) >> 64 for v in xs)
    q0 = int(net.order[0])
    p0 = float(sampler.conditionals(net, params, pauli.configs(np.zeros((1, 2), dtype=np.uint64)), 0)[0])
    k1 = int(cs[xb[:, q0] == 1].sum())
    assert abs(k1 - draws * p0) <= 5 * np.sqrt(draws * p0 * (1 - p0))
