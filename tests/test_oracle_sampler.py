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


def test_uniform53_is_numpys_double_conversion():
    """A word becomes a double in [0, 1) as NumPy's generators make it from the same Philox words."""
    for key in ([3, 4], [2**64 - 1, 0]):
        bg1 = np.random.Philox(key=np.array(key, dtype=np.uint64))
        bg2 = np.random.Philox(key=np.array(key, dtype=np.uint64))
        raw = bg1.random_raw(256)
        assert [sampler.uniform53(int(w)) for w in raw] == np.random.Generator(bg2).random(256).tolist()


class _Given:
    """Uniforms given in advance (for the inversion branch: one per draw)."""

    def __init__(self, *vals):
        self.vals = list(vals)

    def next(self):
        return self.vals.pop(0)


@pytest.mark.parametrize("c,p", [(1, 0.3), (7, 0.5), (50, 0.1), (400, 0.05), (10**6, 1e-5), (31, 0.97)])
def test_binomial_small_mean_is_exact_inversion(c, p):
    rng = np.random.default_rng(c)
    for u in rng.random(300):
        k = sampler.binomial(c, p, _Given(float(u)))
        if p <= 0.5:
            assert k == int(stats.binom.ppf(u, c, p))
        else:                                # reflected: c - Bin(c, 1 - p) on the same uniform
            assert k == c - int(stats.binom.ppf(u, c, 1 - p))


def test_log_fact_ratio_against_sums_of_logs():
    """log(a!/b!) from the Stirling form equals the exactly summed log(b+1) + ... + log(a), also next to
    10^12 where a difference of two lgamma values would keep only ~1e-4 absolute accuracy."""
    for a, b in ((5, 0), (15, 3), (16, 15), (40, 17), (1000, 900), (10**6 + 300, 10**6),
                 (10**12 + 4000, 10**12), (10**12, 10**12 - 3000), (4 * 10**11 + 20, 4 * 10**11 - 50)):
        ref = math.fsum(math.log(i) for i in range(b + 1, a + 1))
        got = sampler.log_fact_ratio(a, b)
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)), (a, b, got, ref)
    # the Stirling correction's series and its lgamma form agree where they meet, to the rounding of the
    # lgamma form (a difference of numbers of size lgamma(x))
    for k in range(16, 40):
        x = k + 1.0
        direct = math.lgamma(x) - ((k + 0.5) * math.log(x) - x + 0.5 * math.log(2 * math.pi))
        assert abs(sampler._stirling_corr(k) - direct) < 8 * 2.0**-52 * math.lgamma(x)


def _chi2_binom(ks, c, p, bins=24):
    """Chi-square statistic of draws against Bin(c, p) over bins of about equal probability; (stat, dof)."""
    qs = np.linspace(0, 1, bins + 1)[1:-1]
    edges = np.unique(stats.binom.ppf(qs, c, p).astype(np.int64))
    cdf = np.concatenate([[0.0], stats.binom.cdf(edges, c, p), [1.0]])
    expect = np.diff(cdf) * len(ks)
    got = np.bincount(np.searchsorted(edges, ks, side="left"), minlength=len(expect))
    return float(np.sum((got - expect) ** 2 / expect)), len(expect) - 1


@pytest.mark.parametrize("c,p", [(100, 0.4), (10**4, 0.01), (10**7, 0.3), (10**12, 0.37), (10**12, 1e-9),
                                 (5 * 10**5, 0.93)])
def test_binomial_large_mean_matches_distribution(c, p):
    """Draws of the rejection branch (c q >= 32) against scipy's binomial distribution: chi-square over 24
    bins of about equal probability from 6,000 draws of seeded counters, and the first two moments."""
    ks = np.array([sampler.binomial(c, p, sampler.Uniforms((i, 3, 0), (99, 0))) for i in range(6000)])
    assert ks.min() >= 0 and ks.max() <= c
    chi2, dof = _chi2_binom(ks, c, p)
    assert chi2 < stats.chi2.ppf(0.999, dof), (chi2, dof)
    m, v = c * p, c * p * (1 - p)
    assert abs(ks.mean() - m) < 5 * math.sqrt(v / len(ks))
    assert abs(ks.var() / v - 1) < 0.1


class _Rejected(Exception):
    pass


class _FirstAttempt:
    """The uniforms (u, v) of one attempt of the rejection branch; a second attempt raises."""

    def __init__(self, u, v):
        self.vals = [u, v]

    def next(self):
        if not self.vals:
            raise _Rejected
        return self.vals.pop(0)


def _attempt(c, p, u, v):
    try:
        return sampler.binomial(c, p, _FirstAttempt(u, v))
    except _Rejected:
        return None


def _accept_level(c, p, u):
    """A(u): the first attempt at (u, v) is accepted exactly for v <= A(u) (bisection on v)."""
    if _attempt(c, p, u, 0.0) is None:
        return 0.0
    lo, hi = 0.0, 1.0
    for _ in range(48):
        mid = 0.5 * (lo + hi)
        if _attempt(c, p, u, mid) is None:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def _first_u(c, p, k):
    """Smallest u whose candidate is k or above (the candidate rises with u; above u = 1/2 a
    rejected candidate lies past c)."""
    lo, hi = 1e-12, 1.0 - 1e-12
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        kk = _attempt(c, p, mid, 0.0)
        if (kk is not None and kk >= k) or (kk is None and mid > 0.5):
            hi = mid
        else:
            lo = mid
    return hi


@pytest.mark.parametrize("c,p,spread,tol", [(60, 0.45, 0, 1e-7), (1001, 0.3, 5, 1e-6), (10**7, 0.3, 4.5, 1e-6),
                                            (10**9, 0.001, 4.5, 1e-6), (10**12, 0.37, 4.5, 2e-4)])
def test_binomial_rejection_branch_is_exact(c, p, spread, tol):
    """The output distribution of the rejection branch, computed rather than sampled.  Attempts take
    fresh uniforms, so a draw is distributed as the first attempt's candidate given that it is
    accepted: P(k) is proportional to the integral of A(u) over the u whose candidate is k.  Both
    the candidate boundaries and A come from the branch's own decisions (bisection); the integral
    is Gauss-Legendre quadrature.  Hormann's BTRS is exact, so P(k) / Bin(k; c, p) is the same for
    every k (at c = 60 every k of probability above 1e-8: further out the candidate intervals shrink
    toward the 2^-53 grain of the uniforms; a band of +-`spread` standard deviations otherwise).  At
    10^12 the candidate's double-precision rounding (~4e-5 of one count) bounds the agreement."""
    mu, sd = c * p, math.sqrt(c * p * (1 - p))
    if spread == 0:
        ks = [k for k in range(c + 1) if stats.binom.pmf(k, c, p) > 1e-8]
    elif c <= 2000:
        ks = list(range(int(mu - spread * sd), int(mu + spread * sd) + 1))
    else:
        ks = sorted(set(int(round(mu + z * sd)) for z in np.linspace(-spread, spread, 31)))
    x, w = np.polynomial.legendre.leggauss(8)
    ratio = []
    for k in ks:
        a, b = _first_u(c, p, k), _first_u(c, p, k + 1)
        tot = 0.0
        for s in range(6):
            lo, hi = a + (b - a) * s / 6, a + (b - a) * (s + 1) / 6
            for xi, wi in zip(x, w):
                tot += 0.5 * (hi - lo) * wi * _accept_level(c, p, 0.5 * (lo + hi) + 0.5 * (hi - lo) * xi)
        ratio.append(tot / stats.binom.pmf(k, c, p))
    ratio = np.array(ratio)
    assert (ratio.max() - ratio.min()) / ratio.mean() <= tol


def test_binomial_reflection_and_counter_words():
    c = 10**7
    for i in range(50):
        # p and 1 - p mirror each other on the same uniforms
        assert sampler.binomial(c, 0.7, sampler.Uniforms((i, 0, 0), (5, 0))) == \
            c - sampler.binomial(c, 0.3, sampler.Uniforms((i, 0, 0), (5, 0)))
    # successive uniforms walk the four words of block 0, then block 1
    u = sampler.Uniforms((11, 2, 3), (7, 8))
    b0, b1 = sampler.philox4x64_10((11, 2, 3, 0), (7, 8)), sampler.philox4x64_10((11, 2, 3, 1), (7, 8))
    assert [u.next() for _ in range(6)] == [sampler.uniform53(w) for w in b0 + b1[:2]]
    # degenerate conditionals: no draws, certain outcomes, NaN (treated as no draws)
    assert sampler.binomial(0, 0.3, _Given()) == 0 and sampler.binomial(9, 0.0, _Given()) == 0
    assert sampler.binomial(9, 1.0, _Given()) == 9 and sampler.binomial(9, float("nan"), _Given()) == 0


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


def test_sampler_elimination_keeps_the_most_draws():
    """A buffer bounded below the unique count of one sampling position keeps the children with the
    most draws.  Unique counts never fall from one position to the next (each parent with draws
    keeps a child), so with the bound between the counts before and at the last position t* where
    the unbounded run grows, only t* eliminates, and every later position gives each kept entry one
    child with all its draws (the split of a parent depends on its configuration and count only).
    The bounded result is then the unbounded one's configurations whose prefixes at t* have the
    largest counts, ties at the threshold taken in buffer order."""
    net = made.Net(n=10, n_layers=2, width=24, n_up=2, n_dn=3)
    params = init_params(10, 2, 24, seed=8, std=0.6)
    xs, cs = sampler.sample(net, params, 20000, seed=5, max_unique=10**6)
    masks = [0]
    for t in range(net.n):
        masks.append(masks[-1] | (1 << int(net.order[t])))
    sizes = [len(np.unique(xs & np.uint64(m))) for m in masks]
    assert sizes == sorted(sizes) and sizes[-1] == len(xs)
    ts = max(t for t in range(1, net.n + 1) if sizes[t] > sizes[t - 1])
    assert sizes[ts:] == [len(xs)] * (net.n + 1 - ts)   # after t* each entry has a single child
    order = np.sort(cs)[::-1]
    cands = [u for u in range(sizes[ts - 1], sizes[ts]) if order[u - 1] > order[u]]
    assert cands                                         # a bound with no tie at the threshold
    for U in cands[:3]:
        bx, bc = sampler.sample(net, params, 20000, seed=5, max_unique=U)
        keep = cs >= order[U - 1]
        assert len(bx) == U == keep.sum()
        got = dict(zip(bx.tolist(), bc.tolist()))
        assert got == dict(zip(xs[keep].tolist(), cs[keep].tolist()))
    # Ties at the threshold are kept in buffer order.  Children with a 0 at the position just
    # placed come before those with a 1, each in parent order, so an entry's place at t* is
    # ordered by its bits at positions t*-1, t*-2, ..., 0.
    pos_bits = [[(int(v) >> int(net.order[t])) & 1 for t in range(ts - 1, -1, -1)] for v in xs.tolist()]
    place = sorted(range(len(xs)), key=lambda i: pos_bits[i])
    rank = np.empty(len(xs), dtype=np.int64)
    rank[place] = np.arange(len(xs))
    ties = [u for u in range(sizes[ts - 1], sizes[ts]) if order[u - 1] == order[u]]
    assert ties
    for U in ties[:3]:
        bx, bc = sampler.sample(net, params, 20000, seed=5, max_unique=U)
        want = sorted(range(len(xs)), key=lambda i: (-cs[i], rank[i]))[:U]
        assert dict(zip(bx.tolist(), bc.tolist())) == {int(xs[i]): int(cs[i]) for i in want}


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
