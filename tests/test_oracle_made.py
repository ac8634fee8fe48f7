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


@pytest.mark.parametrize("n,L,h", [(8, 3, 16), (6, 2, 5), (10, 2, 40)])
def test_every_hidden_unit_reaches_an_output(n, L, h):
    """No hidden unit is cut off: following the masks back from the conditionals reaches every unit of
    every hidden layer, and every unit sees at least one input (MADE keeps hidden degrees within
    1 .. n-1, so that each unit feeds some later conditional)."""
    for order in (None, np.random.default_rng(n).permutation(n)):
        net = made.Net(n=n, n_layers=L, width=h, order=order)
        M1, Mh, Mo, _ = made.masks(net)
        reach = Mo > 0                                   # [n, h]: conditional j reads unit k of layer L
        assert reach.any(axis=0).all()
        for _ in range(L - 1):
            reach = (reach.astype(np.float64) @ Mh) > 0  # units of the layer below
            assert reach.any(axis=0).all()
        assert (M1 > 0).any(axis=1).all()


def test_relu_kink_takes_the_left_derivative():
    """A unit whose pre-activation is exactly zero on every sample (zero incoming weights and bias)
    passes no gradient to its incoming weights: the reverse pass takes the derivative from the left
    of the kink, where the unit stays off and log psi does not change, while from the right it does."""
    n, L, h = 8, 2, 14
    net = _net(n=n, L=L, h=h)
    params = init_params(n, L, h, seed=5, std=0.4).astype(np.float64)
    xs = pauli.sector_basis(n, 2, 2)[::5]
    rng = np.random.default_rng(9)
    ga, gp = rng.standard_normal(len(xs)), rng.standard_normal(len(xs))
    k1, k2 = 3, 2                                        # a layer-1 unit and a layer-2 unit
    b1 = h * n
    w2 = b1 + h
    b2 = w2 + h * h
    params[k1 * n:(k1 + 1) * n] = 0.0
    params[b1 + k1] = 0.0
    params[w2 + k2 * h:w2 + (k2 + 1) * h] = 0.0
    params[b2 + k2] = 0.0
    _, _, cache = made.forward(net, params, xs)
    g = made.backward(net, params, cache, ga, gp)

    def F(p):
        la, ph, _ = made.forward(net, p, xs)
        return np.sum(ga * la) + np.sum(gp * ph)

    for bias in (b1 + k1, b2 + k2):
        left, right = params.copy(), params.copy()
        left[bias] -= 1e-3
        right[bias] += 1e-3
        assert F(left) == F(params)                      # the unit stays off
        assert abs(F(right) - F(params)) > 1e-9          # and matters once it is on
        assert g[bias] == 0.0
    assert np.all(g[k1 * n:(k1 + 1) * n] == 0.0)
    assert np.all(g[w2 + k2 * h:w2 + (k2 + 1) * h] == 0.0)


def test_phase_submodel_single_layer_is_paper_mlp():
    """phase_mode 1, L = 1: the phase is Input[n-2] -> FC1 -> ReLU -> FC2 -> [4] on the
    first n-2 entries in sampling order (Sec. 4 Architecture), and the modulus is the
    shared-trunk network's with the same trunk and conditional head."""
    n, h = 7, 9
    order = np.random.default_rng(5).permutation(n)
    net = made.Net(n=n, n_layers=1, width=h, order=order, phase_mode=1)
    params = init_params(n, 1, h, seed=3, std=0.5, phase_mode=1).astype(np.float64)
    assert len(params) == made.n_params(net)
    off = h * n + h + n * h + n                 # trunk and conditional head
    V1 = params[off:off + h * (n - 2)].reshape(h, n - 2)
    e1 = params[off + h * (n - 2):off + h * (n - 2) + h]
    o2 = off + h * (n - 2) + h
    Wp = params[o2:o2 + 4 * h].reshape(4, h)
    bp = params[o2 + 4 * h:o2 + 4 * h + 4]
    assert o2 + 4 * h + 4 == len(params)
    xs = np.random.default_rng(6).integers(0, 1 << n, 20).astype(np.uint64)
    la, ph, _ = made.forward(net, params, xs)
    for i, x in enumerate(xs):
        bitsx = [(int(x) >> j) & 1 for j in range(n)]
        v = np.array([2.0 * bitsx[order[t]] - 1.0 for t in range(n - 2)])
        c = np.maximum(V1 @ v + e1, 0.0)
        p = Wp @ c + bp
        sel = 2 * bitsx[order[n - 2]] + bitsx[order[n - 1]]
        assert abs(ph[i] - p[sel]) < 1e-13
    # modulus: the shared-trunk net with the same trunk and head gives the same log|psi|
    net0 = made.Net(n=n, n_layers=1, width=h, order=order, phase_mode=0)
    p0 = np.concatenate([params[:off], Wp.ravel(), bp])
    la0, _, _ = made.forward(net0, p0, xs)
    np.testing.assert_array_equal(la, la0)


def test_phase_submodel_dependence():
    """phase_mode 1: the 4-vector p depends on the first n-2 positions only, and every
    one of them enters."""
    n = 8
    order = np.random.default_rng(2).permutation(n)
    net = made.Net(n=n, n_layers=2, width=16, order=order, phase_mode=1)
    params = init_params(n, 2, 16, seed=8, std=0.5, phase_mode=1)
    xs = np.random.default_rng(3).integers(0, 1 << n, 40).astype(np.uint64)
    _, _, c0 = made.forward(net, params, xs)
    for t in range(n):
        _, _, c1 = made.forward(net, params, xs ^ np.uint64(1 << int(order[t])))
        if t >= n - 2:
            np.testing.assert_array_equal(c0["p"], c1["p"])
        else:
            assert np.any(c0["p"] != c1["p"])


@pytest.mark.parametrize("L,constrained", [(1, True), (2, True), (3, False)])
def test_phase_submodel_backward_matches_complex_step(L, constrained):
    n, h = 8, 12
    net = made.Net(n=n, n_layers=L, width=h, n_up=2 if constrained else -1, n_dn=2 if constrained else -1,
                   phase_mode=1)
    params = init_params(n, L, h, seed=31, std=0.4, phase_mode=1).astype(np.float64)
    rng = np.random.default_rng(9)
    basis = pauli.sector_basis(n, 2, 2) if constrained else np.arange(1 << n, dtype=np.uint64)
    xs = rng.choice(basis, 12, replace=False)
    ga = rng.standard_normal(len(xs))
    gp = rng.standard_normal(len(xs))
    _, _, cache = made.forward(net, params, xs)
    g = made.backward(net, params, cache, ga, gp)
    nphase = h * (n - 2) + h + (L - 1) * (h * h + h) + 4 * h + 4
    idx = np.concatenate([rng.choice(len(params) - nphase, 20, replace=False),
                          len(params) - nphase + rng.choice(nphase, 30, replace=False)])
    for k in idx:
        pc = params.astype(np.complex128)
        pc[k] += 1j * 1e-30
        la, ph, _ = made.forward(net, pc, xs, dtype=np.complex128)
        F = np.sum(ga * la) + np.sum(gp * ph)
        assert abs(F.imag / 1e-30 - g[k]) <= 1e-12 * max(1.0, abs(g[k]))
    # the trunk gets nothing from the phase: with g_logabs = 0 its gradient is zero
    g_ph = made.backward(net, params, cache, np.zeros(len(xs)), gp)
    ntrunk = len(params) - nphase
    assert np.all(g_ph[:ntrunk] == 0) and np.any(g_ph[ntrunk:] != 0)
