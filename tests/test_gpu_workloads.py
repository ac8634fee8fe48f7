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
