"""Pins of the FP64 reference sampler (Sec. 4, Sampling) to things outside it."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import made, pauli, sampler
from gen import init_params


def test_philox4x64_matches_numpy_philox():
    # numpy's Philox is Philox4x64-10 and advances the 256-bit counter before each block
    for key, start in (([0x1234, 0x5678], [0, 0, 0, 0]), ([2**64 - 1, 7], [2**64 - 1, 5, 9, 0]),
                       ([0, 0], [3, 0, 0, 2**63])):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(start, dtype=np.uint64))
        raw = bg.random_raw(4 * 5)
        ctr = start[0] + (start[1] << 64) + (start[2] << 128) + (start[3] << 192)
        for b in range(5):
            ctr = (ctr + 1) % (1 << 256)
            words = [(ctr >> (64 * i)) & (2**64 - 1) for i in range(4)]
            out = sampler.philox4x64_10(words, key)
            assert [int(v) for v in raw[4 * b:4 * b + 4]] == out


@pytest.mark.parametrize("c,p", [(1, 0.3), (7, 0.5), (50, 0.1), (400, 0.05), (10**6, 1e-5), (31, 0.97)])
def test_binomial_small_mean_is_exact_inversion(c, p):
    rng = np.random.default_rng(c)
    for u in rng.random(300):
        k = sampler.binomial(c, p, float(u), 0.5)
        if p <= 0.5:
            assert k == int(stats.binom.ppf(u, c, p))
        else:                                # reflected: c - Bin(c, 1 - p) on the same uniform
            assert k == c - int(stats.binom.ppf(u, c, 1 - p))


def test_binomial_large_mean_moments():
    c, p = 10**7, 0.3
    ks = np.array([sampler.binomial(c, p, sampler.uniform53(w[0]), sampler.uniform53(w[1]))
                   for w in (sampler.philox4x64_10((i, 0, 0, 0), (99, 0)) for i in range(4000))])
    m, v = c * p, c * p * (1 - p)
    assert abs(ks.mean() - m) < 5 * math.sqrt(v / len(ks))
    assert abs(ks.var() / v - 1) < 0.1
    assert ks.min() >= 0 and ks.max() <= c
    # p and 1 - p mirror each other on the same uniforms
    assert sampler.binomial(c, 0.7, 0.25, 0.6) == c - sampler.binomial(c, 0.3, 0.25, 0.6)


def _exact_pi(net, params):
    basis = pauli.sector_basis(net.n, net.n_up, net.n_dn)
    la, _, _ = made.forward(net, params, basis)
    return basis, np.exp(2 * la)


def test_sampler_matches_exact_distribution_8_qubits():
    net = made.Net(n=8, n_layers=2, width=32, n_up=2, n_dn=2)
    params = init_params(8, 2, 32, seed=5, std=0.5)
    basis, pi = _exact_pi(net, params)
    assert abs(pi.sum() - 1) < 1e-12
    N = 200000
    xs, cs = sampler.sample(net, params, N, seed=11, max_unique=10**6)
    assert cs.sum() == N and len(np.unique(xs)) == len(xs)
    idx = np.searchsorted(basis, xs)
    assert np.all(basis[idx] == xs)                 # every draw lies in the (2, 2) sector
    counts = np.zeros(len(basis))
    counts[idx] = cs
    chi2 = np.sum((counts - N * pi) ** 2 / (N * pi))
    assert chi2 < stats.chi2.ppf(0.999, len(basis) - 1)


def test_sampler_bounded_buffer():
    net = made.Net(n=12, n_layers=1, width=64, n_up=3, n_dn=3)
    params = init_params(12, 1, 64, seed=2, std=0.5)
    xs, cs = sampler.sample(net, params, 10**6, seed=3, max_unique=50)
    assert 0 < len(xs) <= 50 and len(np.unique(xs)) == len(xs)
    assert np.all(cs > 0) and cs.sum() <= 10**6
    basis = pauli.sector_basis(12, 3, 3)
    assert np.all(np.isin(xs, basis))
    # same seed, same result; another seed, another result
    xs2, cs2 = sampler.sample(net, params, 10**6, seed=3, max_unique=50)
    assert np.array_equal(xs, xs2) and np.array_equal(cs, cs2)
    xs3, _ = sampler.sample(net, params, 10**6, seed=4, max_unique=50)
    assert not np.array_equal(np.sort(xs), np.sort(xs3)) or len(xs) < 50
