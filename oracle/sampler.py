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
x_parent >> 64, 0) (the last two words are zero up to 64 qubits), key (seed, 0).  Binomial draw Bin(c, p) from the counter's first two outputs:
with q = min(p, 1 - p), inversion of the distribution function summed from
k = 0 when c q < 32 (stopping where the terms underflow to zero, which bounds
the search when u lies above the rounded total), otherwise the normal approximation
floor(c q + z sqrt(c q (1 - q)) + 1/2) clamped to [0, c] with z from the
Box-Muller transform; reflected (c - k) when p > 1/2.
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


def binomial(c, p, u1, u2):
    """Bin(c, p) from two uniforms in [0, 1) (see the module docstring)."""
    c = int(c)
    if c == 0 or p <= 0.0:
        return 0
    if p >= 1.0:
        return c
    flip = p > 0.5
    q = 1.0 - p if flip else p
    if c * q < SMALL_MEAN:
        r = q / (1.0 - q)
        pk = math.exp(c * math.log1p(-q))
        F = pk
        k = 0
        while u1 > F and k < c and pk > 0.0:   # past the underflowing tail every term is 0
            pk *= r * (c - k) / (k + 1)
            k += 1
            F += pk
    else:
        z = math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)
        k = math.floor(c * q + z * math.sqrt(c * q * (1.0 - q)) + 0.5)
        k = min(max(k, 0), c)
    return c - k if flip else k


def split_draws(count, p1, x_parent, t, seed):
    """Draws of the child with x = 1 out of `count`."""
    x_parent = int(x_parent)
    w = philox4x64_10((x_parent & _MASK, t, x_parent >> 64, 0), (seed, 0))
    return binomial(count, p1, uniform53(w[0]), uniform53(w[1]))


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
