"""Pins of the oracle network: normalization, autoregressive structure, derivatives."""
import itertools

import numpy as np
import pytest

from oracle import made, pauli
from gen import init_params


def _net(n=8, L=2, h=16, nu=2, nd=2, order=None):
    return made.Net(n=n, n_layers=L, width=h, n_up=nu, n_dn=nd, order=order)


@pytest.mark.parametrize("n,nu,nd,order_kind", [(8, 2, 2, "rev"), (10, 2, 3, "rev"),
                                                (8, 1, 3, "rand"), (6, 3, 0, "fwd")])
def test_constrained_distribution_normalized(n, nu, nd, order_kind):
    """sum over the sector of pi-hat = 1 and pi-hat = 0 outside it (Sec. 4, Eq. modifier)."""
    order = {"rev": None, "fwd": np.arange(n),
             "rand": np.random.default_rng(3).permutation(n)}[order_kind]
    net = _net(n=n, nu=nu, nd=nd, order=order)
    params = init_params(n, net.n_layers, net.width, seed=11, std=0.5)
    allx = np.arange(1 << n, dtype=np.uint64)
    la, _, _ = made.forward(net, params, allx)
    prob = np.exp(2 * la)
    insec = np.zeros(1 << n, dtype=bool)
    insec[pauli.sector_basis(n, nu, nd).astype(np.int64)] = True
    assert np.all(prob[~insec] == 0.0)
    assert abs(prob[insec].sum() - 1.0) < 1e-12


def test_unconstrained_distribution_normalized():
    n = 7
    net = made.Net(n=n, n_layers=3, width=12)
    params = init_params(n, 3, 12, seed=4, std=0.7)
    la, _, _ = made.forward(net, params, np.arange(1 << n, dtype=np.uint64))
    assert abs(np.exp(2 * la).sum() - 1.0) < 1e-12


def test_autoregressive_dependence():
    """o at position t depends only on earlier positions; p only on the first n-2."""
    n = 9
    order = np.random.default_rng(1).permutation(n)
    net = made.Net(n=n, n_layers=3, width=20, order=order)
    params = init_params(n, 3, 20, seed=2, std=0.5)
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 1 << n, 50).astype(np.uint64)
    _, _, c0 = made.forward(net, params, xs)
    for t in range(n):
        q = order[t]
        flipped = xs ^ np.uint64(1 << int(q))
        _, _, c1 = made.forward(net, params, flipped)
        earlier = order[:t + 1]      # o of positions <= t must not change
        np.testing.assert_array_equal(c0["o"][:, earlier], c1["o"][:, earlier])
        if t >= n - 2:
            np.testing.assert_array_equal(c0["p"], c1["p"])
        else:
            assert np.any(c0["p"] != c1["p"])


def test_single_layer_is_paper_two_layer_mlp():
    """L = 1 is exactly Input -> MaskedFC1 -> ReLU -> MaskedFC2 (Sec. 4 Architecture)."""
    n, h = 6, 10
    net = made.Net(n=n, n_layers=1, width=h, n_up=-1, n_dn=-1)
    params = init_params(n, 1, h, seed=9, std=0.4).astype(np.float64)
    assert len(params) == made.n_params(net)
    W1 = params[:h * n].reshape(h, n)
    b1 = params[h * n:h * n + h]
    off = h * n + h
    Wo = params[off:off + n * h].reshape(n, h)
    bo = params[off + n * h: off + n * h + n]
    M1, _, Mo, _ = made.masks(net)
    x = np.uint64(0b101101)
    s = np.array([1.0 if (int(x) >> j) & 1 else -1.0 for j in range(n)])
    a = np.maximum((M1 * W1) @ s + b1, 0)
    o = (Mo * Wo) @ a + bo
    sig = 1 / (1 + np.exp(-o))
    bits = np.array([(int(x) >> j) & 1 for j in range(n)])
    ref = 0.5 * np.sum(np.log(np.where(bits == 1, sig, 1 - sig)))
    la, _, _ = made.forward(net, params, np.array([x]))
    assert abs(la[0] - ref) < 1e-13


@pytest.mark.parametrize("L,constrained", [(1, True), (2, True), (3, False)])
def test_backward_matches_complex_step(L, constrained):
    """Hand reverse pass vs complex-step derivatives (h = 1e-30) on random parameters."""
    n, h = 8, 14
    net = _net(n=n, L=L, h=h, nu=2 if constrained else -1, nd=2 if constrained else -1)
    params = init_params(n, L, h, seed=21, std=0.4).astype(np.float64)
    rng = np.random.default_rng(7)
    basis = pauli.sector_basis(n, 2, 2) if constrained else np.arange(1 << n, dtype=np.uint64)
    xs = rng.choice(basis, 12, replace=False)
    ga = rng.standard_normal(len(xs))
    gp = rng.standard_normal(len(xs))
    _, _, cache = made.forward(net, params, xs)
    g = made.backward(net, params, cache, ga, gp)
    idx = rng.choice(len(params), 40, replace=False)
    hstep = 1e-30
    for k in idx:
        pc = params.astype(np.complex128)
        pc[k] += 1j * hstep
        la, ph, _ = made.forward(net, pc, xs, dtype=np.complex128)
        F = np.sum(ga * la) + np.sum(gp * ph)
        assert abs(F.imag / hstep - g[k]) <= 1e-12 * max(1.0, abs(g[k]))
    # masked-out weights get exactly zero gradient
    M1 = made.masks(net)[0]
    gW1 = g[:h * n].reshape(h, n)
    assert np.all(gW1[M1 == 0] == 0)
