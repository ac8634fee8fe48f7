"""Unique-sample autoregressive sampler, FP64 CPU reference (Sec. 4, Sampling).

Test infrastructure only: used by tests/ (not by the library).

The sampler keeps a buffer of distinct configurations with occurrence counts.
It starts from one configuration (all qubits 0) carrying all n_draws draws.
At step t (sampling position t, qubit q = order[t]):
  * every buffer entry is doubled into a child with x_q = 0 and a child with
    x_q = 1;
  * the draws of the entry are split between the two children by Bernoulli
    sampling of each draw with the conditional probability of x_q = 1 given
    the entry's earlier positions, i.e. a binomial draw; the conditional is
    the network's sigmoid(o_q), replaced by 0 or 1 where the Hamming-weight
    modifier (Eq. modifier) forces the value;
  * children without draws are dropped; if more than max_unique remain, the
    ones with the fewest draws are eliminated.
Readings (also listed in the design notes): the starting configuration is all
zeros; ties in the elimination are broken by the buffer order, which is the
order of the configurations' bits in sampling order (all children with x_q = 0
before those with x_q = 1, each group in parent order); the random numbers
come from a counter-based generator keyed by the seed and indexed by (parent
configuration, t), so a draw does not depend on where the entry sits in the
buffer.

Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011), counter (x_parent mod 2^64, t,
x_parent >> 64, j) (the third word is zero up to 64 qubits), key (seed, 0);
block j = 0, 1, ... gives four 64-bit words, each a uniform in [0, 1) from its
top 53 bits.  Binomial draw Bin(c, p), q = min(p, 1 - p), reflected (c - k)
when p > 1/2, exact in both branches:
  * c q < 32: inversion of the distribution function summed from k = 0 with
    the first uniform of block 0 (stopping where the terms underflow to zero,
    which bounds the search when u lies above the rounded total);
  * otherwise Hormann's BTRS, transformed rejection with squeeze (W. Hormann,
    "The generation of binomial random variates", J. Statist. Comput. Simul.
    46 (1993) 101-110): each attempt takes the next two uniforms (block 0's
    words 0 and 1, then 2 and 3, then block 1's ...), accepts in the squeeze
    region, else compares log V with the log of the probability ratio
    f(k)/f(m) at the mode m.  That log is written as differences of
    log-factorials, log(a!/b!) = d log(b+1) + (a + 1/2) log1p(d/(b+1)) - d +
    fc(a) - fc(b) with d = a - b and fc the Stirling correction, so that its
    rounding stays at the size of the result for counts up to 10^12 (the
    difference of two lgamma values of 10^12 would lose five digits).
    Attempts are capped at 4096 (never reached in practice: each accepts with
    probability above 0.75); at the cap the draw is the mode.
"""
import math

import numpy as np

from . import made
from .pauli import configs


def _as_configs(vals, n):
    if n <= 64:
        return np.array(vals, dtype=np.uint64)
    out = np.empty(len(vals), dtype=object)
    for i, v in enumerate(vals):
        out[i] = int(v)
    return out

_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1
SMALL_MEAN = 32.0


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds: four 64-bit output words."""
    c = [int(v) & _MASK for v in ctr]
    k = [int(v) & _MASK for v in key]
    for r in range(10):
        if r > 0:
            k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & _MASK]
    return c


def uniform53(word):
    """[0, 1) from the top 53 bits of a 64-bit word."""
    return (int(word) >> 11) * (1.0 / 9007199254740992.0)


def _stirling_corr(k):
    """fc(k) = log(k!) - [(k + 1/2) log(k + 1) - (k + 1) + log(2 pi) / 2]."""
    if k < 16:
        return math.lgamma(k + 1.0) - ((k + 0.5) * math.log(k + 1.0) - (k + 1.0) + 0.5 * math.log(2.0 * math.pi))
    x = k + 1.0
    x2 = x * x
    return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0 - (1.0 / 1680.0) / x2) / x2) / x2) / x


def log_fact_ratio(a, b):
    """log(a! / b!) for integers a >= b >= 0 (stable when a - b << b)."""
    d = a - b
    if d == 0:
        return 0.0
    return (d * math.log(b + 1.0) + (a + 0.5) * math.log1p(d / (b + 1.0)) - d
            + _stirling_corr(a) - _stirling_corr(b))


class Uniforms:
    """The uniforms of one draw: words of Philox blocks j = 0, 1, ... of a counter."""

    def __init__(self, ctr3, key):
        self.ctr3, self.key, self.j, self.words = list(ctr3), key, 0, []

    def next(self):
        if not self.words:
            self.words = philox4x64_10(self.ctr3 + [self.j], self.key)
            self.j += 1
        return uniform53(self.words.pop(0))


MAX_ATTEMPTS = 4096


def _btrs(n, p, uni):
    """Bin(n, p) for p <= 1/2 and n p >= SMALL_MEAN by Hormann's BTRS."""
    q = 1.0 - p
    spq = math.sqrt(n * p * q)
    b = 1.15 + 2.53 * spq
    a = -0.0873 + 0.0248 * b + 0.01 * p
    c = n * p + 0.5
    vr = 0.92 - 4.2 / b
    alpha = (2.83 + 5.1 / b) * spq
    lpq = math.log(p / q)
    m = math.floor((n + 1) * p)
    for _ in range(MAX_ATTEMPTS):
        u = uni.next() - 0.5
        v = uni.next()
        us = 0.5 - abs(u)
        k = math.floor((2.0 * a / us + b) * u + c if us > 0.0 else -1.0)   # us = 0 only at u = -1/2
        if us >= 0.07 and v <= vr:
            return k
        if k < 0 or k > n:
            continue
        v = v * alpha / (a / (us * us) + b)
        # log f(k)/f(m) = log(m!/k!) + log((n-m)!/(n-k)!) + (k - m) log(p/q)
        if k >= m:
            lr = -log_fact_ratio(k, m) + log_fact_ratio(n - m, n - k)
        else:
            lr = log_fact_ratio(m, k) - log_fact_ratio(n - k, n - m)
        if v == 0.0 or math.log(v) <= lr + (k - m) * lpq:                     # log 0 = -inf
            return k
    return m


def binomial(c, p, uni):
    """Bin(c, p) with the uniforms of `uni` (see the module docstring)."""
    c = int(c)
    if c == 0 or not (p > 0.0):
        return 0
    if not (p < 1.0):
        return c
    flip = p > 0.5
    q = 1.0 - p if flip else p
    if c * q < SMALL_MEAN:
        u1 = uni.next()
        r = q / (1.0 - q)
        pk = math.exp(c * math.log1p(-q))
        F = pk
        k = 0
        while u1 > F and k < c and pk > 0.0:   # past the underflowing tail every term is 0
            pk *= r * (c - k) / (k + 1)
            k += 1
            F += pk
    else:
        k = _btrs(c, q, uni)
    return c - k if flip else k


def split_draws(count, p1, x_parent, t, seed):
    """Draws of the child with x = 1 out of `count`."""
    x_parent = int(x_parent)
    return binomial(count, p1, Uniforms((x_parent & _MASK, t, x_parent >> 64), (seed, 0)))


def conditionals(net: made.Net, params, xs, t):
    """P(x_{order[t]} = 1 | earlier positions) for each configuration of xs."""
    xs = configs(xs)
    _, _, cache = made.forward(net, params, xs)
    q = net.order[t]
    o = cache["o"][:, q]
    p = 1.0 / (1.0 + np.exp(-o))
    free, _, one = made.constraint(net, cache["xb"], forced_values=True)
    return np.where(free[:, q], p, np.where(one[:, q], 1.0, 0.0))


def sample(net: made.Net, params, n_draws, seed, max_unique):
    """(configurations [U], counts int64 [U]) in buffer order; configurations are
    uint64 up to 64 qubits and Python integers (dtype object) above."""
    xs = [0]
    cs = [int(n_draws)]
    for t in range(net.n):
        q = int(net.order[t])   # a Python integer: the child bit 1 << q for any qubit
        p = conditionals(net, params, _as_configs(xs, net.n), t)
        c1 = [split_draws(c, float(p[i]), x, t, seed) for i, (x, c) in enumerate(zip(xs, cs))]
        kids = [(x, c - k) for x, c, k in zip(xs, cs, c1)] + \
               [(x | (1 << q), k) for x, k in zip(xs, c1)]
        kids = [(x, c) for x, c in kids if c > 0]
        if len(kids) > max_unique:
            # keep the max_unique largest counts; among equal counts the earlier entries
            keep = sorted(range(len(kids)), key=lambda i: (-kids[i][1], i))[:max_unique]
            kids = [kids[i] for i in sorted(keep)]
        xs = [x for x, _ in kids]
        cs = [c for _, c in kids]
    return _as_configs(xs, net.n), np.array(cs, dtype=np.int64)
