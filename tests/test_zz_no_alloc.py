"""GPU checks of the allocation-free entry point (nqs_energy_grad_noalloc),
through the C ABI: its results equal nqs_energy_grad's on a caller workspace,
bit for bit, on two calls in a row (the second with a smaller batch, so the
shared static workspace holds the first call's contents), and they meet the
FP64 oracle bars; a plan whose workspace exceeds the static array is refused
before anything runs."""
import math

import numpy as np
import pytest
import torch

from gen import hamiltonian, init_params, sector_samples, unique_with_counts
from oracle import made, pauli, vmc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    import paper_2208_05637_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def ctx(nqs):
    return nqs.Context(0)


@pytest.mark.parametrize("prec,L,h,dedup", [("fp64", 1, 64, True), ("bf16w", 2, 256, False)])
def test_noalloc_equals_workspace_call(nqs, ctx, prec, L, h, dedup):
    N, n = 6, 12
    terms = hamiltonian(N, 0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    params = init_params(n, L, h, seed=1, dtype="bf16" if prec == "bf16w" else "fp32")
    xs, w = unique_with_counts(sector_samples(n, 3, 3, 2000, seed=2))
    assert len(xs) > 300
    plan = nqs.Plan(ctx, H, L, h, 3, 3, prec, max_batch=len(xs), dedup=dedup)
    assert plan.workspace_size(len(xs)) <= nqs._lib.NQS_NOALLOC_SCRATCH_BYTES
    p = torch.from_numpy(params).cuda()
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    net = made.Net(n=n, n_layers=L, width=h, n_up=3, n_dn=3)
    for B in (len(xs), 123):       # the second call is smaller and runs on the first call's leftovers
        print(f"noalloc {prec}: B = {B}", flush=True)
        e1, g1, l1 = nqs.energy_grad(plan, p, xs[:B], w[:B])
        e2, g2, l2, fl = nqs.energy_grad_noalloc(plan, p, xs[:B], w[:B])
        torch.cuda.synchronize()
        assert int(fl.item()) == 0
        assert torch.equal(e1, e2) and torch.equal(g1, g2) and torch.equal(l1, l2)
        if prec == "fp64":
            el_ref = vmc.local_energy(ref, net, params, xs[:B])
            E_ref, _, _ = vmc.energy(el_ref, w[:B])
            g_ref = vmc.gradient(net, params, xs[:B], w[:B], el_ref, E_ref)
            assert abs(e2[0].item() - E_ref) <= 1e-10 * abs(E_ref)
            g = g2.cpu().numpy()
            assert np.linalg.norm(g - g_ref) <= 1e-9 * np.linalg.norm(g_ref)


def test_noalloc_refuses_a_plan_beyond_the_array(nqs, ctx):
    terms = hamiltonian(12, 0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    plan = nqs.Plan(ctx, H, 2, 256, 6, 6, "fp32", max_batch=8192, dedup=True)
    B = 8192
    assert plan.workspace_size(B) > nqs._lib.NQS_NOALLOC_SCRATCH_BYTES
    p = torch.from_numpy(init_params(24, 2, 256, seed=1)).cuda()
    xs, w = unique_with_counts(sector_samples(24, 6, 6, B, seed=2))
    energy = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(nqs.NQSError, match="WORKSPACE_TOO_SMALL"):
        nqs.energy_grad_noalloc(plan, p, xs, w, energy=energy)
    torch.cuda.synchronize()
    assert torch.equal(energy.cpu(), torch.full((3,), 7.0, dtype=torch.float64))
