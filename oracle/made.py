"""Masked autoregressive amplitude/phase network in FP64 (Sec. 4).

Definition (readings of Sec. 4, Architecture and Constraints):
  * input s = 2x - 1, column j = qubit j (the paper feeds alternating +-1
    values, Sec. 4 Sampling);
  * the autoregressive order ``order`` lists qubits in sampling order; the
    default is the reverse order n-1, ..., 0 (the paper samples starting from
    the n-th qubit, Sec. 4); qubit j has degree d(j) = 1 + its position;
  * hidden unit k of every hidden layer has degree m_k = 1 + (k mod (n-1))
    (MADE's mask rule; the paper leaves the degree assignment open);
  * masks: first layer [m_k >= d(j)], hidden layers [m_k >= m_k'], conditional
    head [d(j) > m_k], phase head [m_k <= n-2] (the phase is a function of the
    first n-2 entries in sampling order, one value per completion of the last
    two, Sec. 4 Architecture);
  * a_l = ReLU((M_l*W_l) a_{l-1} + b_l), l = 1..L;  o = (M_o*W_o) a_L + b_o;
    p = (M_phi*W_phi) a_L + b_phi;
  * pi_j(x_j = 1 | earlier) = sigmoid(o_j);  log f = i phi + 1/2 sum log pi
    (Sec. 4, the complex logarithm of the model output), the sum running over
    the positions left free by the Hamming-weight modifier (Eq. modifier):
    forced positions have modified conditional 1 and contribute log 1 = 0,
    and a configuration that contradicts a forced value has amplitude 0;
  * modifier, per spin s of the qubit at position t (even qubits are spin
    up): with c_s ones already placed on spin-s qubits and r_s spin-s
    positions still to come after t, the value is forced to 0 when
    c_s >= n_s and forced to 1 when c_s + r_s < n_s;
  * phi = p[2 x_{order[n-2]} + x_{order[n-1]}], used as a real angle.

Two readings of the phase network (Sec. 4, Architecture):
  * phase_mode 0: the phase head above reads the shared masked trunk;
  * phase_mode 1: the paper's separate phase sub-model, a plain MLP whose
    input is the first n-2 entries in sampling order, v_t = s_{order[t]}
    for t < n-2, with the same depth L and width h as the modulus network:
    c_1 = ReLU(V_1 v + e_1), c_l = ReLU(V_l c_{l-1} + e_l), p = W_phi c_L +
    b_phi.  Its input already excludes the last two positions, so its layers
    carry no masks; the modulus network keeps the trunk and the conditional
    head and has no phase head.

Parameters are the flat layout W_1, b_1, ..., W_L, b_L, W_o, b_o, then (mode
1 only) V_1, e_1, ..., V_L, e_L, then W_phi, b_phi, with weights row-major
[out][in] (V_1 is [h][n-2]).

The forward runs in float64 or complex128 (complex-step derivative checks);
the reverse pass is written out by hand.
"""
from dataclasses import dataclass, field

import numpy as np

from .pauli import configs


@dataclass
class Net:
    n: int
    n_layers: int
    width: int
    n_up: int = -1
    n_dn: int = -1
    order: np.ndarray = field(default=None)
    phase_mode: int = 0

    def __post_init__(self):
        if self.order is None:
            self.order = np.arange(self.n - 1, -1, -1)
        self.order = np.asarray(self.order, dtype=np.int64)
        if sorted(self.order.tolist()) != list(range(self.n)):
            raise ValueError("order must be a permutation of the qubits")
        if self.n < 2:
            raise ValueError("need at least two qubits")
        if self.phase_mode not in (0, 1):
            raise ValueError("phase_mode is 0 (shared trunk) or 1 (separate sub-model)")

    @property
    def constrained(self):
        return self.n_up >= 0 and self.n_dn >= 0


def unpack(net: Net, params):
    """Split the flat parameter vector into
    ([(W_l, b_l)] * L, (W_o, b_o), (W_phi, b_phi), [(V_l, e_l)] * L or [])."""
    p = np.asarray(params)
    n, h, L = net.n, net.width, net.n_layers
    off = 0

    def take(rows, cols):
        nonlocal off
        W = p[off:off + rows * cols].reshape(rows, cols)
        off += rows * cols
        b = p[off:off + rows]
        off += rows
        return W, b

    layers = [take(h, n if l == 0 else h) for l in range(L)]
    head_o = take(n, h)
    phase_layers = [take(h, n - 2 if l == 0 else h) for l in range(L)] if net.phase_mode == 1 else []
    head_p = take(4, h)
    if off != p.shape[0]:
        raise ValueError(f"parameter vector has {p.shape[0]} entries, layout needs {off}")
    return layers, head_o, head_p, phase_layers


def n_params(net: Net):
    n, h, L = net.n, net.width, net.n_layers
    total = h * n + h + (L - 1) * (h * h + h) + n * h + n + 4 * h + 4
    if net.phase_mode == 1:
        total += h * (n - 2) + h + (L - 1) * (h * h + h)
    return total


def masks(net: Net):
    """(M_1, [M_l for hidden l >= 2], M_o, M_phi) as float64 0/1 arrays."""
    n, h = net.n, net.width
    pos = np.empty(n, dtype=np.int64)
    pos[net.order] = np.arange(n)
    d = 1 + pos                                   # degree of qubit j
    m = 1 + (np.arange(h) % (n - 1))              # degree of hidden unit k
    M1 = (m[:, None] >= d[None, :]).astype(np.float64)
    Mh = (m[:, None] >= m[None, :]).astype(np.float64)
    Mo = (d[:, None] > m[None, :]).astype(np.float64)
    if net.phase_mode == 1:
        Mp = np.ones((4, h))                      # the sub-model's head reads all its units
    else:
        Mp = np.repeat((m <= n - 2)[None, :], 4, axis=0).astype(np.float64)
    return M1, Mh, Mo, Mp


def bits(net: Net, samples):
    s = configs(samples)
    if s.dtype == object:
        # Python integers (any width): bits of each 64-bit word in turn
        out = np.zeros((s.shape[0], net.n), dtype=np.int64)
        for w in range((net.n + 63) // 64):
            word = ((s >> (64 * w)) & ((1 << 64) - 1)).astype(np.uint64)
            j = np.arange(min(64, net.n - 64 * w), dtype=np.uint64)
            out[:, 64 * w:64 * w + j.shape[0]] = (word[:, None] >> j[None, :]) & np.uint64(1)
        return out
    j = np.arange(net.n, dtype=np.uint64)
    return ((s[:, None] >> j[None, :]) & np.uint64(1)).astype(np.int64)


def constraint(net: Net, xb, forced_values=False):
    """Per-sample, per-qubit (free, violated) flags of the modifier (Eq. modifier);
    with forced_values also the value each forced qubit is forced to (True = 1).
    The flags of the qubit at position t depend only on the bits before t."""
    B, n = xb.shape
    free = np.ones((B, n), dtype=bool)
    bad = np.zeros(B, dtype=bool)
    one = np.zeros((B, n), dtype=bool)
    if not net.constrained:
        return (free, bad, one) if forced_values else (free, bad)
    target = (net.n_up, net.n_dn)
    placed = np.zeros((B, 2), dtype=np.int64)
    spin_of = np.arange(n) % 2
    remaining = np.array([np.sum(spin_of == 0), np.sum(spin_of == 1)])
    for t in range(n):
        j = net.order[t]
        s = spin_of[j]
        remaining[s] -= 1                          # spin-s positions after t
        c = placed[:, s]
        force0 = c >= target[s]
        force1 = c + remaining[s] < target[s]
        xj = xb[:, j]
        bad |= (force0 & (xj == 1)) | (force1 & (xj == 0))
        free[:, j] = ~(force0 | force1)
        one[:, j] = force1
        placed[:, s] += xj
    return (free, bad, one) if forced_values else (free, bad)


def _softplus(z):
    """log(1 + e^z), stable, valid for float64 and complex128 arguments."""
    z = np.asarray(z)
    out = np.empty_like(z)
    pos = np.real(z) > 0
    with np.errstate(over="ignore", invalid="ignore"):
        out[pos] = z[pos] + np.log1p(np.exp(-z[pos]))
        out[~pos] = np.log1p(np.exp(z[~pos]))
    return out


def _relu(z):
    return np.where(np.real(z) > 0, z, 0)


def forward(net: Net, params, samples, dtype=np.float64):
    """log|psi| (float64, -inf off-sector), phi, and the activations for backward."""
    layers, (Wo, bo), (Wp, bp), phase_layers = unpack(net, np.asarray(params).astype(dtype))
    M1, Mh, Mo, Mp = masks(net)
    xb = bits(net, samples)
    s = (2 * xb - 1).astype(dtype)
    acts = [s]
    pre = []
    a = s
    for li, (W, b) in enumerate(layers):
        M = M1 if li == 0 else Mh
        z = a @ (M * W).T + b
        pre.append(z)
        a = _relu(z)
        acts.append(a)
    o = a @ (Mo * Wo).T + bo
    pacts, ppre = [], []
    if net.phase_mode == 1:
        c = s[:, net.order[:net.n - 2]]             # first n-2 entries in sampling order
        pacts.append(c)
        for V, e in phase_layers:
            z = c @ V.T + e
            ppre.append(z)
            c = _relu(z)
            pacts.append(c)
        p = c @ (Mp * Wp).T + bp
    else:
        p = a @ (Mp * Wp).T + bp
    free, bad = constraint(net, xb)
    # log pi_j(x_j) = -softplus(-o) if x_j = 1 else -softplus(o)
    lp = np.where(xb == 1, -_softplus(-o), -_softplus(o))
    logabs = 0.5 * np.sum(np.where(free, lp, 0), axis=1)
    sel = 2 * xb[:, net.order[net.n - 2]] + xb[:, net.order[net.n - 1]]
    phi = p[np.arange(len(sel)), sel]
    if np.issubdtype(np.dtype(dtype), np.floating):
        logabs = np.where(bad, -np.inf, logabs)
    cache = dict(acts=acts, pre=pre, o=o, p=p, xb=xb, free=free, bad=bad, sel=sel, pacts=pacts, ppre=ppre)
    return logabs, phi, cache


def backward(net: Net, params, cache, g_logabs, g_phi):
    """Gradient of sum_i g_logabs[i] log|psi_i| + g_phi[i] phi_i w.r.t. the flat parameters.

    d log|psi| / d o_j = 1/2 [j free] (x_j - sigmoid(o_j)); d phi / d p_c = [c == sel].
    ReLU'(0) = 0; masked-out weights receive zero gradient.
    """
    layers, (Wo, bo), (Wp, bp), phase_layers = unpack(net, np.asarray(params, dtype=np.float64))
    M1, Mh, Mo, Mp = masks(net)
    acts, pre, o, xb, free, sel = (cache[k] for k in ("acts", "pre", "o", "xb", "free", "sel"))
    if np.any(cache["bad"]):
        raise ValueError("gradient of a zero-amplitude configuration")
    g_logabs = np.asarray(g_logabs, dtype=np.float64)
    g_phi = np.asarray(g_phi, dtype=np.float64)
    sig = 1.0 / (1.0 + np.exp(-o))
    d_o = g_logabs[:, None] * 0.5 * free * (xb - sig)
    d_p = np.zeros((len(sel), 4))
    d_p[np.arange(len(sel)), sel] = g_phi
    aL = acts[-1]
    phase_in = cache["pacts"][-1] if net.phase_mode == 1 else aL
    gWp = (d_p.T @ phase_in) * Mp
    gbp = d_p.sum(axis=0)
    gWo = (d_o.T @ aL) * Mo
    gbo = d_o.sum(axis=0)

    def through(stack, inputs, pres, d_a, mask_of):
        """Reverse pass through ReLU layers; returns [(gW, gb)] in forward order."""
        out = []
        for li in reversed(range(len(stack))):
            W, _ = stack[li]
            M = mask_of(li)
            d_z = d_a * (pres[li] > 0)
            out.append(((d_z.T @ inputs[li]) * M, d_z.sum(axis=0)))
            d_a = d_z @ (M * W)
        return out[::-1]

    d_a = d_o @ (Mo * Wo)
    if net.phase_mode == 0:
        d_a = d_a + d_p @ (Mp * Wp)
    trunk = through(layers, acts, pre, d_a, lambda li: M1 if li == 0 else Mh)
    flat = []
    for gW, gb in trunk:
        flat += [gW.ravel(), gb]
    flat += [gWo.ravel(), gbo]
    if net.phase_mode == 1:
        ones = lambda li: 1.0
        sub = through(phase_layers, cache["pacts"], cache["ppre"], d_p @ Wp, ones)
        for gW, gb in sub:
            flat += [gW.ravel(), gb]
    flat += [gWp.ravel(), gbp]
    return np.concatenate(flat)
