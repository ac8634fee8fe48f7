"""GPU unique-sample autoregressive sampler (Sec. 4, Sampling) against the oracle.

With the FP64 network the GPU conditionals equal the oracle's to ~1e-15, and
both sides draw from the same counter-based generator with the same binomial
rule, so the sampled configurations and their counts are compared exactly
(buffer order included).  At 60 qubits (BF16 network) the checks are the
properties every output must have.
"""
import numpy as np
import pytest
import torch

from oracle import made, pauli, sampler
from gen import init_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2208_05637_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def ctx(nqs):
    return nqs.Context(0)


def _plan(nqs, ctx, n, L, h, nu, nd, prec, order=None):
    H = nqs.Hamiltonian(n, [1], [0], [1.0]).upload(ctx)      # the sampler does not use H
    return nqs.Plan(ctx, H, L, h, nu, nd, prec, max_batch=16, order=order), H


@pytest.mark.parametrize("n,L,h,nu,nd,draws,umax,order_seed", [
    (12, 1, 64, 3, 3, 10**6, 40, None),          # elimination active from early on
    (12, 1, 64, 3, 3, 10**6, 10**4, None),       # no elimination: all draws kept
    (12, 1, 64, 3, 3, 10**12, 10**4, None),      # counts up to 10^12: the rejection branch throughout
    (16, 2, 128, 4, 4, 10**9, 300, None),
    (12, 2, 64, 2, 4, 10**5, 64, 3),             # random sampling order, unequal sector
    (10, 1, 64, 3, 2, 7, 1000, None)])           # fewer draws than states
def test_sampler_matches_oracle_fp64(nqs, ctx, n, L, h, nu, nd, draws, umax, order_seed):
    order = None if order_seed is None else np.random.default_rng(order_seed).permutation(n)
    plan, H = _plan(nqs, ctx, n, L, h, nu, nd, "fp64", order)
    params = init_params(n, L, h, seed=n + L, std=0.5)
    x, w = nqs.sample(plan, torch.from_numpy(params).cuda(), draws, seed=12345, max_unique=umax)
    xg = x.cpu().numpy().view(np.uint64)
    wg = w.cpu().numpy()
    net = made.Net(n=n, n_layers=L, width=h, n_up=nu, n_dn=nd, order=order)
    xr, cr = sampler.sample(net, params, draws, seed=12345, max_unique=umax)
    print(f"n={n}: {len(xr)} unique of {draws} draws (cap {umax}); GPU {len(xg)}")
    assert np.array_equal(xg, xr)
    assert np.array_equal(wg, cr.astype(np.float64))


def test_sampler_single_entry_buffer(nqs, ctx):
    plan, H = _plan(nqs, ctx, 8, 1, 64, 2, 2, "fp64")
    params = init_params(8, 1, 64, seed=1, std=0.5)
    x, w = nqs.sample(plan, torch.from_numpy(params).cuda(), 1000, seed=5, max_unique=1)
    assert x.numel() == 1 and w.item() > 0
    net = made.Net(n=8, n_layers=1, width=64, n_up=2, n_dn=2)
    xr, cr = sampler.sample(net, params, 1000, seed=5, max_unique=1)
    assert int(x.cpu().numpy().view(np.uint64)[0]) == int(xr[0]) and w.item() == cr[0]


def test_sampler_60_qubits_bf16_network(nqs, ctx):
    """65,536-entry buffer at 60 qubits: unique, in the (15, 15) sector, positive counts."""
    n, L, h = 60, 4, 1024
    plan, H = _plan(nqs, ctx, n, L, h, 15, 15, "bf16w")
    params = init_params(n, L, h, seed=1, dtype="bf16")
    p = torch.from_numpy(params).cuda()
    nqs.sample(plan, p, 10**6, seed=1, max_unique=1024)          # warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    x, w = nqs.sample(plan, p, 10**12, seed=2, max_unique=65536)
    e1.record()
    torch.cuda.synchronize()
    xs = x.cpu().numpy().view(np.uint64)
    ws = w.cpu().numpy()
    print(f"60 qubits: {len(xs)} unique configurations from 1e12 draws in {e0.elapsed_time(e1):.1f} ms")
    assert len(xs) == 65536 and len(np.unique(xs)) == len(xs)
    up = np.array([bin(int(v) & 0x5555555555555555).count("1") for v in xs])
    dn = np.array([bin(int(v) & 0xAAAAAAAAAAAAAAAA).count("1") for v in xs])
    assert np.all(up == 15) and np.all(dn == 15)
    assert np.all(ws > 0) and ws.sum() <= 1e12
    # the sampled configurations have non-zero amplitude under the same network
    lp = nqs.log_psi(plan, p, x).cpu().numpy()
    assert np.all(np.isfinite(lp[:, 0]))
