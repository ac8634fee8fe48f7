"""Pins of the Adam oracle (Kingma and Ba, Algorithm 1; Sec. 6)."""
import numpy as np
import torch

from oracle import adam


def test_first_step_moves_by_lr_times_sign():
    # with zero moments the bias-corrected ratio is g / (|g| + eps)
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(1000).astype(np.float32)
    g = rng.standard_normal(1000) * 10.0 ** rng.integers(-3, 3, 1000)
    lr, eps = 1e-3, 1e-8
    t1, m, v = adam.step(theta, g, np.zeros(1000), np.zeros(1000), 1, lr=lr, eps=eps)
    expect = (theta.astype(np.float64) - lr * g / (np.abs(g) + eps)).astype(np.float32)
    assert np.array_equal(t1, expect)
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.01 * g * g, rtol=1e-14)


def test_constant_gradient_keeps_unit_ratio():
    # m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so every step moves by lr g / (|g| + eps)
    g = np.array([3.0, -0.5, 2e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    th = np.zeros(3, dtype=np.float32)
    for t in range(1, 30):
        th_new, m, v = adam.step(th, g, m, v, t, lr=1e-2, eps=0.0)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13)
        assert np.allclose(v, (1 - 0.99 ** t) * g * g, rtol=1e-13)
        step = th_new.astype(np.float64) - th.astype(np.float64)
        assert np.allclose(step, -1e-2 * np.sign(g), rtol=1e-5, atol=2e-7)
        th = th_new


def test_matches_torch_adam():
    """Several steps against torch.optim.Adam (the same algorithm, a library
    implementation: it updates m by linear interpolation and forms the
    denominator as sqrt(v)/sqrt(1 - b2^t) + eps) run in FP64 on the CPU.  The
    moments agree to rounding at the scale of the gradients; the oracle's
    parameters are rounded to FP32 after every step, so they stay within half
    an FP32 ulp per step of torch's FP64 trajectory."""
    rng = np.random.default_rng(1)
    n = 4096
    th = rng.standard_normal(n).astype(np.float32)
    p = torch.tensor(th.astype(np.float64), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.99), eps=1e-8)
    m = np.zeros(n)
    v = np.zeros(n)
    gmax = np.zeros(n)
    bound = np.zeros(n)
    for t in range(1, 9):
        g = rng.standard_normal(n) * 10.0 ** rng.integers(-4, 1, n)
        gmax = np.maximum(gmax, np.abs(g))
        p.grad = torch.tensor(g)
        opt.step()
        th_prev = th
        th, m, v = adam.step(th, g, m, v, t)
        bound += 0.5 * np.spacing(np.maximum(np.abs(th_prev), np.abs(th))).astype(np.float64)
        st = opt.state[p]
        assert np.all(np.abs(st["exp_avg"].numpy() - m) <= 1e-15 * gmax)
        assert np.all(np.abs(st["exp_avg_sq"].numpy() - v) <= 1e-15 * gmax ** 2)
        assert np.all(np.abs(th.astype(np.float64) - p.detach().numpy()) <= bound * 1.001 + 1e-15)
