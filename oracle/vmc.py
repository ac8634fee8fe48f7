"""Local energy, energy estimate and VMC gradient, plain FP64 (Sec. 3, Sec. 5).

Readings taken here:
  * samples carry weights w_i (occurrence counts of a unique-sample buffer,
    Sec. 4 Sampling; default 1) and averages divide by W = sum w_i in place of
    the 1/B of Eq. total_energy_sum;
  * the reported objective is E = <H> (twice the L of Sec. 3) and the reported
    gradient is grad E = 2 Re E[(l - b) conj(sigma)] with the real scalar
    baseline b = E-bar (Eq. grad with b = E[l]);
  * the local energy runs term by term over the full merged term set exactly as
    Alg. 1 / Eq. local_energy_auto, with psi evaluated once per distinct
    connected configuration (the unique-flip buffer of Sec. 5.1 is a cache of
    the same values); a term whose flip is empty contributes its matrix element
    times one.
"""
import math

import numpy as np

from . import made
from .pauli import popcount, groups, configs

UP_MASK = np.uint64(0x5555555555555555)
DN_MASK = np.uint64(0xAAAAAAAAAAAAAAAA)
# the same masks over 128 qubits, for bit strings held as Python integers
UP_MASK_WIDE = int("01" * 64, 2)
DN_MASK_WIDE = int("10" * 64, 2)


def log_psi(net, params, configs_in, rows=32768):
    """Complex log psi for each configuration; -inf real part off-sector.

    Configurations that contradict a forced value of the modifier have
    amplitude 0 whatever the network outputs, so the network is evaluated
    only on the others (in batches of ``rows``); the values are those of
    ``made.forward``.
    """
    cfg = configs(configs_in)
    la = np.full(len(cfg), -np.inf)
    phi = np.zeros(len(cfg))
    _, bad = made.constraint(net, made.bits(net, cfg))
    idx = np.nonzero(~bad)[0]
    for s in range(0, len(idx), rows):
        sel = idx[s:s + rows]
        a, p, _ = made.forward(net, params, cfg[sel])
        la[sel] = a
        phi[sel] = p
    return la, phi


def local_energy(terms, net, params, samples, batch_terms=4_000_000, scale=False):
    """E_loc(x_i) = sum_k ct_k (-1)^{popcount(x_i & z_k)} psi(x_i ^ x_k) / psi(x_i)  (Eq. local_energy_auto).

    Returns complex128 [B].  Raises on a zero-amplitude sample.  With
    ``scale``, returns (E_loc, S) with S_i = sum_k |summand_k|, the magnitude
    the rounding of the K-term sum is relative to.
    """
    return local_energy_fn(terms, lambda c: log_psi(net, params, c), samples, batch_terms, scale)


def local_energy_fn(terms, logpsi, samples, batch_terms=4_000_000, scale=False):
    """Eq. local_energy_auto for any amplitude given as ``logpsi(configs) -> (log|psi|, phase)``."""
    samples = configs(samples)
    xk, zk, ct = terms["x"], terms["z"], terms["ct"]
    la_s, ph_s = logpsi(samples)
    if np.any(~np.isfinite(la_s)):
        raise ValueError("sample with zero amplitude")
    out = np.empty(len(samples), dtype=np.complex128)
    S = np.empty(len(samples))
    K = len(xk)
    per = max(1, batch_terms // max(K, 1))
    for start in range(0, len(samples), per):
        xs = samples[start:start + per]
        xp = xs[:, None] ^ xk[None, :]                       # Alg. 1: X xor F^{1,2}
        sign = 1.0 - 2.0 * (popcount(xs[:, None] & zk[None, :]) & 1)   # Eq. mtx_element
        uniq, inv = np.unique(xp.ravel(), return_inverse=True)
        la_u, ph_u = logpsi(uniq)
        la_p = la_u[inv].reshape(xp.shape)
        ph_p = ph_u[inv].reshape(xp.shape)
        ls = la_s[start:start + per][:, None]
        ps = ph_s[start:start + per][:, None]
        with np.errstate(invalid="ignore"):
            ratio = np.where(np.isfinite(la_p),
                             np.exp((la_p - ls) + 1j * (ph_p - ps)), 0.0)
        summand = ct[None, :] * sign * ratio
        for i in range(xs.shape[0]):
            out[start + i] = complex(math.fsum(summand[i].real), math.fsum(summand[i].imag))
            if scale:
                S[start + i] = math.fsum(np.abs(summand[i]))
    return (out, S) if scale else out


def energy(eloc, weights=None):
    """(E-bar, mean imaginary part, W): weighted sample means (Eq. total_energy_sum), exact summation."""
    eloc = np.asarray(eloc, dtype=np.complex128)
    w = np.ones(len(eloc)) if weights is None else np.asarray(weights, dtype=np.float64)
    W = math.fsum(w)
    E = math.fsum(w * eloc.real) / W
    I = math.fsum(w * eloc.imag) / W
    return E, I, W


def gradient(net, params, samples, weights, eloc, ebar):
    """grad E = 2 Re sum_i (w_i/W)(E_loc,i - E-bar) conj(d log psi(x_i))  (Eq. grad, x2, b = E-bar).

    = sum_i (w_i/W) * 2 * [(Re l_i - E-bar) d log|psi_i| + Im l_i d phi_i].
    """
    w = np.ones(len(samples)) if weights is None else np.asarray(weights, dtype=np.float64)
    W = math.fsum(w)
    _, _, cache = made.forward(net, params, samples)
    g_la = 2.0 * (w / W) * (eloc.real - ebar)
    g_ph = 2.0 * (w / W) * eloc.imag
    return made.backward(net, params, cache, g_la, g_ph)


def sector_valid(x, flip):
    """Integer spin-sector test: the flip keeps the number of up and down electrons."""
    x = configs(x)
    y = x ^ configs(flip)
    up, dn = (UP_MASK_WIDE, DN_MASK_WIDE) if y.dtype == object else (UP_MASK, DN_MASK)
    return (popcount(x & up) == popcount(y & up)) & \
           (popcount(x & dn) == popcount(y & dn))


def connected(terms, samples, sector_filter=True):
    """Per-sample connected entries in canonical order, for bit-exact checks.

    For each sample x and each flip group g (groups by x mask ascending, terms
    inside by z ascending): h_g(x) = sum_{k in g} ct_k (-1)^{popcount(x & z_k)},
    summed sequentially in that order in FP64 (real and imaginary parts
    separately).  The empty flip gives the diagonal element.  A non-empty group
    is kept when it passes the spin-sector test (``sector_filter``) or, without
    the filter, when h != 0.

    Returns (diag[B] complex, list over samples of (group index array,
    x' array, h complex array)).
    """
    gx, goff = groups(terms)
    zk, ct = terms["z"], terms["ct"]
    samples = configs(samples)
    B = len(samples)
    G = len(gx)
    H = np.zeros((B, G), dtype=np.complex128)
    for g in range(G):
        a, b = goff[g], goff[g + 1]
        sign = 1.0 - 2.0 * (popcount(samples[:, None] & zk[None, a:b]) & 1)
        contrib = ct[None, a:b] * sign
        re = np.add.accumulate(contrib.real, axis=1)[:, -1]   # sequential order
        im = np.add.accumulate(contrib.imag, axis=1)[:, -1]
        H[:, g] = re + 1j * im
    diag = np.zeros(B, dtype=np.complex128)
    has_diag = G > 0 and gx[0] == 0
    if has_diag:
        diag = H[:, 0].copy()
    out = []
    gstart = 1 if has_diag else 0
    for i in range(B):
        gi = np.arange(gstart, G)
        if sector_filter:
            keep = sector_valid(np.full(len(gi), samples[i], dtype=samples.dtype), gx[gi])
        else:
            keep = H[i, gi] != 0
        gi = gi[keep]
        out.append((gi, samples[i] ^ gx[gi], H[i, gi]))
    return diag, out
