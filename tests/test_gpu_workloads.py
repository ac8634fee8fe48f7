"""GPU checks on the benchmark workloads, through the C ABI.

Each workload runs at its full batch in the launch configuration that
bench.py times (plan defaults); outputs the oracle can compute one by one
(a few samples' local energies, FP64) are compared, together with properties
that hold at any size (every sample has exactly the planned number of
connected configurations; the energy equals the weighted mean of the
returned local energies; no device error flag).
"""
import math

import numpy as np
import pytest
import torch

from oracle import made, pauli, vmc
from gen import config_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    import paper_2208_05637_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def ctx(nqs):
    return nqs.Context(0)


def _run(nqs, ctx, name, precision=None, batch=None):
    terms, params, xs, w, cfg = config_inputs(name, batch=batch)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    prec = precision or cfg["precision"]
    plan = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], prec, max_batch=len(xs),
                    dedup=cfg["dedup"])
    p = torch.from_numpy(params).cuda()
    energy, grad, eloc = nqs.energy_grad(plan, p, xs, w)
    torch.cuda.synchronize()
    assert nqs.device_status(plan) == 0
    return terms, params, xs, w, cfg, plan, energy.cpu().numpy(), grad.cpu().numpy(), eloc.cpu().numpy()


def _oracle_eloc(terms, cfg, params, xs):
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    net = made.Net(n=cfg["n"], n_layers=cfg["L"], width=cfg["h"], n_up=cfg["n_up"], n_dn=cfg["n_dn"])
    return vmc.local_energy(ref, net, params, xs)


def _closed_conn(N, nu, nd):
    t = 1
    for s in (nu, nd):
        t += s * (N - s) + math.comb(s, 2) * math.comb(N - s, 2)
    return t + nu * (N - nu) * nd * (N - nd)


@pytest.mark.parametrize("name,prec,tol", [
    # per-sample |dE_loc| bars: FP32 / split-BF16 carry ~1e-6 relative error in
    # log psi, the local energy sums ~1e4 terms of size ~1e-2 with random signs
    ("c3", "bf16w", 2e-3), ("c3", "bf16x3", 2e-3), ("c3", "fp32", 2e-3), ("c3", "bf16", 0.5)])
def test_40_qubits_full_batch_sampled(nqs, ctx, name, prec, tol):
    terms, params, xs, w, cfg, plan, energy, grad, eloc = _run(nqs, ctx, name, prec)
    N = cfg["N"]
    assert plan.entries_per_sample == _closed_conn(N, N // 2, N // 2) - 1
    # energy is the weighted mean of the returned local energies
    E = math.fsum(w * eloc[:, 0]) / math.fsum(w)
    assert abs(E - energy[0]) <= 1e-12 * abs(E)
    idx = np.array([0, len(xs) // 2, len(xs) - 1])
    el_ref = _oracle_eloc(terms, cfg, params, xs[idx])
    d = np.abs(eloc[idx, 0] + 1j * eloc[idx, 1] - el_ref)
    print(f"{name} {prec}: sampled |dE_loc| = {d}, E = {energy[0]:.10f}")
    assert np.all(d <= tol)
    assert np.all(np.isfinite(grad))


def test_four_instances_one_call(nqs, ctx):
    """16/28/44/64 qubits, each with its own H, network and samples, in one nqs_energy_grad_multi."""
    items, refs = [], []
    plans = []
    for name, B in (("c5a", 512), ("c5b", 256), ("c5c", 128), ("c5d", 64)):
        terms, params, xs, w, cfg = config_inputs(name, batch=B)
        H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
        plan = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], cfg["precision"],
                        max_batch=len(xs), dedup=cfg["dedup"])
        plans.append((plan, H))
        dev = ctx.device
        it = dict(plan=plan, params=torch.from_numpy(params).to(dev),
                  samples=torch.from_numpy(xs.view(np.int64)).to(dev),
                  weights=torch.from_numpy(w).to(dev),
                  eloc=torch.empty((len(xs), 2), dtype=torch.float64, device=dev),
                  energy=torch.empty(3, dtype=torch.float64, device=dev),
                  grad=torch.empty(plan.n_params, dtype=torch.float64, device=dev))
        items.append(it)
        refs.append((terms, params, xs, w, cfg))
    ws = nqs.multi_workspace(items)
    nqs.energy_grad_multi(items, ws)
    torch.cuda.synchronize()
    for it, (terms, params, xs, w, cfg) in zip(items, refs):
        el = it["eloc"].cpu().numpy()
        # each instance equals its own single-instance call
        e1, g1, l1 = nqs.energy_grad(it["plan"], it["params"], it["samples"], it["weights"])
        assert torch.equal(l1, it["eloc"]) and torch.equal(g1, it["grad"]) and torch.equal(e1, it["energy"])
        el_ref = _oracle_eloc(terms, cfg, params, xs[:2])
        d = np.abs(el[:2, 0] + 1j * el[:2, 1] - el_ref)
        print(f"{cfg['n']} qubits: |dE_loc| = {d}")
        assert np.all(d <= 2e-3)


def test_60_qubits_full_batch_sampled(nqs, ctx):
    """The benchmark's workload at full size, in its launch configuration: 65,536 unique
    configurations drawn from the 60-qubit BF16 network by the GPU sampler (10^12 draws),
    energy and gradient over all of them; sampled local energies against the oracle."""
    terms, params, _, _, cfg = config_inputs("c4")
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    mk = lambda mb: nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], cfg["precision"],
                             max_batch=mb, dedup=cfg["dedup"])
    p = torch.from_numpy(params).cuda()
    x, w = nqs.sample(mk(16), p, 10**12, seed=2, max_unique=cfg["B"])
    assert x.numel() == cfg["B"] and float(w.sum()) <= 1e12 and bool((w > 0).all())
    plan = mk(cfg["B"])
    N = cfg["N"]
    assert plan.entries_per_sample == _closed_conn(N, N // 2, N // 2) - 1
    assert plan.kernel_info()["waves_per_block"] == 16 and plan.chunk_samples == (256 << 20) // 73125
    energy, grad, eloc = nqs.energy_grad(plan, p, x, w)
    torch.cuda.synchronize()
    assert nqs.device_status(plan) == 0
    energy, grad, eloc, wn = energy.cpu().numpy(), grad.cpu().numpy(), eloc.cpu().numpy(), w.cpu().numpy()
    E = math.fsum(wn * eloc[:, 0]) / math.fsum(wn)
    assert abs(E - energy[0]) <= 1e-12 * abs(E) and energy[2] == math.fsum(wn)
    xs = x.cpu().numpy().view(np.uint64)
    idx = np.array([0, len(xs) - 1])
    el_ref = _oracle_eloc(terms, cfg, params, xs[idx])
    d = np.abs(eloc[idx, 0] + 1j * eloc[idx, 1] - el_ref)
    print(f"c4 bf16w, 65,536 sampled configurations: sampled |dE_loc| = {d}, E = {energy[0]:.10f}")
    assert np.all(d <= 1e-3)
    assert np.all(np.isfinite(grad))
