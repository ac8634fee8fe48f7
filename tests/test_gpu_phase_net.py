"""The separate phase sub-model (Sec. 4, Architecture; NQS_PHASE_SEPARATE) on
the GPU against the oracle, through the C ABI: log psi of every precision,
FP64 local energies, energy and gradient, the BF16-weight path's energy and
gradient, the multi-instance call, the sampler and launch-grouping
invariance."""
import numpy as np
import pytest
import torch

from oracle import made, pauli, sampler, vmc
from gen import hamiltonian, init_params, sector_samples, unique_with_counts

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


def _ham(nqs, ctx, N, seed=0):
    terms = hamiltonian(N, seed)
    return nqs.Hamiltonian.from_terms(terms).upload(ctx), pauli.canonical_terms(terms.x_mask, terms.z_mask,
                                                                                terms.coeff)


def _net(n, L, h, nu, nd, order=None):
    return made.Net(n=n, n_layers=L, width=h, n_up=nu, n_dn=nd, order=order, phase_mode=1)


@pytest.mark.parametrize("prec,h,L,std,tol,pdtype", [
    ("fp64", 64, 1, 0.3, 1e-12, "fp32"), ("fp64", 128, 2, 0.3, 1e-12, "fp32"),
    ("fp32", 256, 2, 0.3, 2e-5, "fp32"), ("bf16x3", 512, 2, 0.1, 5e-4, "fp32"),
    ("bf16w", 1024, 2, 0.1, 5e-4, "bf16"), ("bf16", 256, 3, 0.1, 0.05, "fp32")])
def test_log_psi_parity(nqs, ctx, prec, h, L, std, tol, pdtype):
    N = 6
    n = 2 * N
    H, ref = _ham(nqs, ctx, N)
    order = np.random.default_rng(h + L).permutation(n) if h == 128 else None
    plan = nqs.Plan(ctx, H, L, h, 3, 3, prec, max_batch=16, order=order, phase_mode="separate")
    params = init_params(n, L, h, seed=7, std=std, dtype=pdtype, phase_mode=1)
    assert plan.n_params == len(params)
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 1 << n, 3000).astype(np.uint64)      # in and out of sector, ragged tile
    xs[:400] = pauli.sector_basis(n, 3, 3)
    la_ref, ph_ref, _ = made.forward(_net(n, L, h, 3, 3, order), params, xs)
    out = nqs.log_psi(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    fin = np.isfinite(la_ref)
    assert np.array_equal(np.isfinite(out[:, 0]), fin)
    err_la = np.max(np.abs(out[fin, 0] - la_ref[fin]))
    err_ph = np.max(np.abs(out[:, 1] - ph_ref))
    print(f"separate phase net, {prec} h={h} L={L}: max|d log|psi|| = {err_la:.3e}, max|d phi| = {err_ph:.3e}")
    assert err_la <= tol and err_ph <= tol


def test_energy_and_gradient_fp64_12_qubits(nqs, ctx):
    N, n, L, h = 6, 12, 2, 64
    H, ref = _ham(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, L, h, 3, 3, "fp64", max_batch=1024, dedup=True, phase_mode=1)
    params = init_params(n, L, h, seed=1, std=0.3, phase_mode=1)
    xs, w = unique_with_counts(sector_samples(n, 3, 3, 1024, seed=2))
    net = _net(n, L, h, 3, 3)
    el_ref = vmc.local_energy(ref, net, params, xs)
    E_ref, I_ref, W_ref = vmc.energy(el_ref, w)
    g_ref = vmc.gradient(net, params, xs, w, el_ref, E_ref)
    energy, grad, el = nqs.energy_grad(plan, torch.from_numpy(params).cuda(), xs, w)
    el = el.cpu().numpy()
    energy = energy.cpu().numpy()
    grad = grad.cpu().numpy()
    # rounding scale of each local energy: sum over terms of |summand|
    la, _, _ = made.forward(net, params, xs[:32])
    S = np.array([np.sum(np.abs(ref["ct"]) * np.nan_to_num(np.exp(made.forward(net, params, x ^ ref["x"])[0] - la[i])))
                  for i, x in enumerate(xs[:32])])
    err = np.abs(el[:, 0] + 1j * el[:, 1] - el_ref)
    gerr = np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref)
    print(f"separate phase net fp64: max |dE_loc|/S = {np.max(err[:32] / S):.3e}, E = {energy[0]:.15f} "
          f"(oracle {E_ref:.15f}), |dg|/|g| = {gerr:.3e}")
    assert np.all(err[:32] <= 1e-10 * S)
    assert abs(energy[0] - E_ref) <= 1e-10 * max(1.0, abs(E_ref))
    assert abs(energy[1] - I_ref) <= 1e-10 * max(1.0, abs(E_ref))
    assert energy[2] == W_ref
    assert gerr <= 1e-9
    nphase = h * (n - 2) + h + (L - 1) * (h * h + h) + 4 * h + 4
    assert np.any(grad[-nphase:] != 0)
    assert nqs.device_status(plan) == 0


def test_energy_bf16_weights_16_qubits(nqs, ctx):
    N, n, L, h = 8, 16, 3, 512
    H, ref = _ham(nqs, ctx, N, seed=1)
    plan = nqs.Plan(ctx, H, L, h, 4, 4, "bf16w", max_batch=64, dedup=True, phase_mode=1)
    params = init_params(n, L, h, seed=1, dtype="bf16", phase_mode=1)
    xs, w = unique_with_counts(sector_samples(n, 4, 4, 64, seed=2))
    net = _net(n, L, h, 4, 4)
    el_ref = vmc.local_energy(ref, net, params, xs)
    E_ref, _, _ = vmc.energy(el_ref, w)
    g_ref = vmc.gradient(net, params, xs, w, el_ref, E_ref)
    energy, grad, _ = nqs.energy_grad(plan, torch.from_numpy(params).cuda(), xs, w)
    dE = abs(energy[0].item() - E_ref)
    gerr = np.linalg.norm(grad.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    print(f"separate phase net bf16w: |dE| = {dE:.3e} Ha, |dg|/|g| = {gerr:.3e}")
    assert dE <= 1e-4 and gerr <= 1e-3


def test_multi_with_separate_phase_net_equals_single(nqs, ctx):
    """A separate-phase instance adds a second segment (its phase network) to each launch group."""
    items, keep = [], []
    specs = [(6, 0, "bf16w", 512, 2, 200, 1), (7, 1, "bf16w", 512, 2, 150, 0), (5, 2, "fp32", 256, 1, 120, 1),
             (6, 3, "bf16w", 512, 3, 90, 1), (8, 4, "bf16w", 512, 2, 60, 1), (5, 5, "bf16w", 512, 1, 80, 1)]
    for N, seed, prec, h, L, B, mode in specs:
        n = 2 * N
        H, _ = _ham(nqs, ctx, N, seed)
        xs, w = unique_with_counts(sector_samples(n, N // 2, N // 2, B, seed=seed + 10))
        plan = nqs.Plan(ctx, H, L, h, N // 2, N // 2, prec, max_batch=len(xs),
                        chunk_samples=max(8, len(xs) // 3), phase_mode=mode)
        dev = ctx.device
        pd = "bf16" if prec == "bf16w" else "fp32"
        it = dict(plan=plan, params=torch.from_numpy(init_params(n, L, h, seed=seed, dtype=pd, phase_mode=mode)).to(dev),
                  samples=torch.from_numpy(xs.view(np.int64)).to(dev), weights=torch.from_numpy(w).to(dev),
                  eloc=torch.empty((len(xs), 2), dtype=torch.float64, device=dev),
                  energy=torch.empty(3, dtype=torch.float64, device=dev),
                  grad=torch.empty(plan.n_params, dtype=torch.float64, device=dev))
        items.append(it)
        keep.append(H)
    nqs.energy_grad_multi(items)
    torch.cuda.synchronize()
    for it in items:
        e1, g1, l1 = nqs.energy_grad(it["plan"], it["params"], it["samples"], it["weights"])
        assert torch.equal(l1, it["eloc"]) and torch.equal(g1, it["grad"]) and torch.equal(e1, it["energy"])
        assert nqs.device_status(it["plan"]) == 0


def test_sampler_fp64_equals_oracle(nqs, ctx):
    n, L, h = 10, 2, 64
    H, _ = _ham(nqs, ctx, n // 2)
    plan = nqs.Plan(ctx, H, L, h, 2, 3, "fp64", max_batch=16, phase_mode=1)
    params = init_params(n, L, h, seed=4, std=0.5, phase_mode=1)
    x, w = nqs.sample(plan, torch.from_numpy(params).cuda(), 10**7, seed=77, max_unique=60)
    xr, cr = sampler.sample(_net(n, L, h, 2, 3), params, 10**7, seed=77, max_unique=60)
    assert np.array_equal(x.cpu().numpy().view(np.uint64), xr)
    assert np.array_equal(w.cpu().numpy(), cr.astype(np.float64))


def test_launch_grouping_invariance(nqs, ctx):
    N, B = 22, 16
    n = 2 * N
    H, _ = _ham(nqs, ctx, N, 3)
    xs = sector_samples(n, N // 2, N // 2, B, seed=8)
    plan = nqs.Plan(ctx, H, 3, 512, N // 2, N // 2, "bf16w", max_batch=B, phase_mode=1)
    p = torch.from_numpy(init_params(n, 3, 512, seed=2, dtype="bf16", phase_mode=1)).cuda()
    con = nqs.connected(plan, xs)
    ne = int(con["n_entries"].item())
    ent = con["x"][:ne].contiguous()
    M = plan.kernel_info()["rows_per_block"]
    whole = nqs.log_psi(plan, p, ent)
    step = 37 * M + 5
    parts = torch.cat([nqs.log_psi(plan, p, ent[i:i + step]) for i in range(0, ne, step)])
    torch.cuda.synchronize()
    assert torch.equal(whole, parts)
