"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (derived from the arithmetic of each path):
  * integer / bit work (connected sets, dedup sets): bit-exact;
  * matrix elements h and the diagonal: bit-exact (same sequential FP64
    order as the oracle);
  * FP64 network: log psi to 1e-12 absolute; E_loc to 1e-10 relative to the
    sum of absolute summands S_i (the rounding scale of the sum);
  * FP32 network: log psi 2e-5 absolute (FP32 accumulation over <= 1024
    terms per unit, ~60 log-sigmoids summed in FP64); E_loc 1e-4 * S_i;
  * split-BF16 (hi*hi + hi*lo + lo*hi) network: same bars as FP32 but 4x looser;
  * plain BF16 network: 8-bit mantissa activations; bars stated per test.
"""
import math

import numpy as np
import pytest
import torch

from oracle import made, pauli, vmc
from gen import hamiltonian, init_params, round_bf16, sector_samples, unique_with_counts

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


def _setup(nqs, ctx, N, seed=0, **plan_kw):
    terms = hamiltonian(N, seed)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    return terms, H, ref


def _oracle_net(n, L, h, nu, nd, order=None):
    return made.Net(n=n, n_layers=L, width=h, n_up=nu, n_dn=nd, order=order)


@pytest.mark.parametrize("prec,h,L,std,tol", [
    ("fp64", 64, 1, 0.3, 1e-12), ("fp64", 128, 2, 0.3, 1e-12), ("fp64", 512, 3, 0.1, 1e-12),
    ("fp64", 1024, 2, 0.1, 1e-12),
    ("fp32", 128, 2, 0.3, 2e-5), ("fp32", 256, 3, 0.3, 2e-5), ("fp32", 1024, 2, 0.1, 2e-5),
    # split bf16 keeps ~16 mantissa bits per operand: a few 1e-5 relative on logits of O(10)
    ("bf16x3", 256, 2, 0.3, 5e-4), ("bf16x3", 1024, 2, 0.1, 5e-4),
    # bf16 activations carry 8 bits: relative 2^-9 per rounding, summed over ~n log-sigmoids
    ("bf16", 256, 2, 0.1, 0.05), ("bf16", 512, 3, 0.1, 0.05), ("bf16", 1024, 4, 0.1, 0.05)])
@pytest.mark.parametrize("constrained", [True, False])
def test_log_psi_parity(nqs, ctx, prec, h, L, std, tol, constrained):
    N = 6
    n = 2 * N
    terms, H, ref = _setup(nqs, ctx, N)
    nu, nd = (3, 3) if constrained else (-1, -1)
    order = np.random.default_rng(h + L).permutation(n) if h == 128 else None
    plan = nqs.Plan(ctx, H, L, h, nu, nd, prec, max_batch=4096, order=order)
    params = init_params(n, L, h, seed=7, std=std)
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 1 << n, 3000).astype(np.uint64)      # in and out of sector, ragged tile
    xs[:400] = pauli.sector_basis(n, 3, 3)
    la_ref, ph_ref, _ = made.forward(_oracle_net(n, L, h, nu, nd, order), params, xs)
    out = nqs.log_psi(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    fin = np.isfinite(la_ref)
    assert np.array_equal(np.isfinite(out[:, 0]), fin)
    err_la = np.max(np.abs(out[fin, 0] - la_ref[fin]))
    err_ph = np.max(np.abs(out[:, 1] - ph_ref))
    print(f"{prec} h={h} L={L}: max|d log|psi|| = {err_la:.3e}, max|d phi| = {err_ph:.3e}")
    assert err_la <= tol and err_ph <= tol


@pytest.mark.parametrize("h,L", [(256, 2), (512, 3), (1024, 2)])
def test_log_psi_parity_bf16_weights(nqs, ctx, h, L):
    """BF16 network (BF16-valued weights): only the activations are split, so
    the bar of the split-BF16 path holds (weights carry no rounding at all)."""
    N = 6
    n = 2 * N
    terms, H, ref = _setup(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, L, h, 3, 3, "bf16w", max_batch=16)
    params = init_params(n, L, h, seed=7, dtype="bf16")
    rng = np.random.default_rng(3)
    xs = rng.integers(0, 1 << n, 2100).astype(np.uint64)
    xs[:400] = pauli.sector_basis(n, 3, 3)
    la_ref, ph_ref, _ = made.forward(_oracle_net(n, L, h, 3, 3), params, xs)
    out = nqs.log_psi(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    fin = np.isfinite(la_ref)
    assert np.array_equal(np.isfinite(out[:, 0]), fin)
    err_la = np.max(np.abs(out[fin, 0] - la_ref[fin]))
    err_ph = np.max(np.abs(out[:, 1] - ph_ref))
    print(f"bf16w h={h} L={L}: max|d log|psi|| = {err_la:.3e}, max|d phi| = {err_ph:.3e}")
    assert err_la <= 5e-4 and err_ph <= 5e-4


def _weight_entries(n, L, h):
    """Boolean mask of the weight (not bias) entries of the flat parameter layout."""
    m = []
    for l in range(L):
        m += [True] * (h * (n if l == 0 else h)) + [False] * h
    m += [True] * (n * h) + [False] * n + [True] * (4 * h) + [False] * 4
    return np.array(m)


def test_bf16_weights_round_parameters(nqs, ctx):
    """The BF16 network takes each weight as the parameter rounded to BF16
    (biases unrounded): FP32 parameters and their weight-rounded copy give
    identical log psi, energy and gradient."""
    N, n, L, h = 6, 12, 2, 256
    terms, H, ref = _setup(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, L, h, 3, 3, "bf16w", max_batch=200)
    p = init_params(n, L, h, seed=11)
    wmask = _weight_entries(n, L, h)
    assert wmask.size == p.size
    q = p.copy()
    q[wmask] = round_bf16(p[wmask])
    assert not np.array_equal(p, q)
    xs, w = unique_with_counts(sector_samples(n, 3, 3, 200, seed=4))
    a = [t.clone() for t in nqs.energy_grad(plan, torch.from_numpy(p).cuda(), xs, w)]
    b = nqs.energy_grad(plan, torch.from_numpy(q).cuda(), xs, w)
    assert all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("N,B,filt", [(6, 257, True), (6, 100, False), (12, 70, True)])
def test_connected_bit_exact(nqs, ctx, N, B, filt):
    n = 2 * N
    terms = hamiltonian(N, 0)
    H = nqs.Hamiltonian.from_terms(terms, conserves_spin=filt).upload(ctx)
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    plan = nqs.Plan(ctx, H, 1, 64, N // 2, N // 2, "fp64", max_batch=B, chunk_samples=B, dedup=True)
    xs = sector_samples(n, N // 2, N // 2, B, seed=5)
    out = nqs.connected(plan, xs)
    diag_ref, ent = vmc.connected(ref, xs, sector_filter=filt)
    torch.cuda.synchronize()
    ne = int(out["n_entries"].item())
    assert ne == sum(len(e[0]) for e in ent)
    diag = out["diag"].cpu().numpy()
    assert np.array_equal(diag[:, 0], diag_ref.real) and np.array_equal(diag[:, 1], diag_ref.imag)
    es = out["sample"][:ne].cpu().numpy()
    ex = out["x"][:ne].cpu().numpy().view(np.uint64)
    eh = out["h"][:ne].cpu().numpy()
    pos = 0
    for i, (gi, xp, hv) in enumerate(ent):
        k = len(gi)
        assert np.all(es[pos:pos + k] == i)
        assert np.array_equal(ex[pos:pos + k], xp)                # canonical order, bit-exact
        assert np.array_equal(eh[pos:pos + k, 0], hv.real)
        assert np.array_equal(eh[pos:pos + k, 1], hv.imag)
        pos += k
    nu = int(out["n_unique"].item())
    uniq = np.sort(out["unique"][:nu].cpu().numpy().view(np.uint64))
    assert np.array_equal(uniq, np.unique(ex))
    eu = out["entry_unique"][:ne].cpu().numpy()
    assert np.array_equal(out["unique"][:nu].cpu().numpy().view(np.uint64)[eu], ex)
    # the distinct configurations are listed in the order of their first entries
    _, first = np.unique(ex, return_index=True)
    assert np.array_equal(out["unique"][:nu].cpu().numpy().view(np.uint64), ex[np.sort(first)])


def test_entry_bound_equals_closed_form(nqs, ctx):
    for N, nu, nd in [(6, 3, 3), (12, 6, 6), (8, 3, 5)]:
        terms = hamiltonian(N, 0)
        H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
        plan = nqs.Plan(ctx, H, 1, 64, nu, nd, "fp64", max_batch=16)
        conn = 1 + sum(s * (N - s) + math.comb(s, 2) * math.comb(N - s, 2) for s in (nu, nd)) \
            + nu * (N - nu) * nd * (N - nd)
        assert plan.entries_per_sample == conn - 1


def test_reduce_table_eigenvector(nqs, ctx):
    """E_loc == lambda_min on the GPU ratio-reduce when psi is the exact ground vector."""
    N, n = 6, 12
    terms, H, ref = _setup(nqs, ctx, N)
    basis = pauli.sector_basis(n, 3, 3)
    Hs = pauli.sector_block(ref, basis)
    ev, V = np.linalg.eigh(Hs)
    psi0 = V[:, 0]
    xs = basis[np.abs(psi0) > 1e-8]
    plan = nqs.Plan(ctx, H, 1, 64, 3, 3, "fp64", max_batch=len(xs), chunk_samples=len(xs))
    out = nqs.connected(plan, xs)
    ne = int(out["n_entries"].item())
    ex = out["x"][:ne].cpu().numpy().view(np.uint64)

    def logtab(c):
        j = np.minimum(np.searchsorted(basis, c), len(basis) - 1)
        a = np.where(basis[j] == c, psi0[j], 0.0)
        with np.errstate(divide="ignore"):
            return np.stack([np.log(np.abs(a)), np.angle(a)], axis=1)

    lps = torch.from_numpy(logtab(xs)).cuda()
    lpe = torch.from_numpy(logtab(ex)).cuda()
    el = nqs.reduce_table(plan, lps, lpe, out["diag"], out["sample"][:ne], out["h"][:ne], ne).cpu().numpy()
    scale = np.max(np.abs(Hs)) * math.sqrt(len(basis))
    assert np.max(np.abs(el[:, 0] - ev[0])) < 1e-9 * scale
    assert np.max(np.abs(el[:, 1])) < 1e-9 * scale


def _eloc_scale(ref, net, params, xs):
    """S_i = sum_k |summand_k| of Eq. local_energy_auto (the rounding scale)."""
    la, ph, _ = made.forward(net, params, xs)
    out = []
    for i, x in enumerate(xs):
        xp = x ^ ref["x"]
        l2, _, _ = made.forward(net, params, xp)
        with np.errstate(invalid="ignore"):
            r = np.where(np.isfinite(l2), np.exp(l2 - la[i]), 0.0)
        out.append(np.sum(np.abs(ref["ct"]) * r))
    return np.array(out)


@pytest.mark.parametrize("dedup,chunk", [(True, 0), (False, 300)])
def test_local_energy_fp64_12_qubits(nqs, ctx, dedup, chunk):
    """12 qubits, 1024 sector-uniform samples, L=1, h=64, FP64: |dE_loc| <= 1e-10 S_i."""
    N, n, L, h = 6, 12, 1, 64
    terms, H, ref = _setup(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, L, h, 3, 3, "fp64", max_batch=1024, dedup=dedup, chunk_samples=chunk)
    params = init_params(n, L, h, seed=1)
    xs = sector_samples(n, 3, 3, 1024, seed=2)
    net = _oracle_net(n, L, h, 3, 3)
    el_ref = vmc.local_energy(ref, net, params, xs)
    el = nqs.local_energy(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    S = _eloc_scale(ref, net, params, xs[:64])
    err = np.abs((el[:, 0] + 1j * el[:, 1]) - el_ref)
    print(f"max |dE_loc| = {err.max():.3e}, max relative to S_i = {np.max(err[:64] / S):.3e}")
    assert np.all(err[:64] <= 1e-10 * S)
    assert err.max() <= 1e-10 * np.max(S)
    assert nqs.device_status(plan) == 0


def test_energy_and_gradient_fp64_12_qubits(nqs, ctx):
    N, n, L, h = 6, 12, 1, 64
    terms, H, ref = _setup(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, L, h, 3, 3, "fp64", max_batch=1024, dedup=True)
    params = init_params(n, L, h, seed=1)
    xs, w = unique_with_counts(sector_samples(n, 3, 3, 1024, seed=2))
    net = _oracle_net(n, L, h, 3, 3)
    el_ref = vmc.local_energy(ref, net, params, xs)
    E_ref, I_ref, W_ref = vmc.energy(el_ref, w)
    g_ref = vmc.gradient(net, params, xs, w, el_ref, E_ref)
    energy, grad, el = nqs.energy_grad(plan, torch.from_numpy(params).cuda(), xs, w)
    energy = energy.cpu().numpy()
    grad = grad.cpu().numpy()
    print(f"E = {energy[0]:.15f} (oracle {E_ref:.15f}); |dg|/|g| = "
          f"{np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref):.3e}")
    assert abs(energy[0] - E_ref) <= 1e-10 * max(1.0, abs(E_ref))
    assert abs(energy[1] - I_ref) <= 1e-10 * max(1.0, abs(E_ref))
    assert energy[2] == W_ref
    assert np.linalg.norm(grad - g_ref) <= 1e-9 * np.linalg.norm(g_ref)
    M1 = made.masks(net)[0]
    assert np.all(grad[:h * n].reshape(h, n)[M1 == 0] == 0.0)


def test_energy_and_gradient_fp32_24_qubits_subset(nqs, ctx):
    """24 qubits, L=2, h=256, FP32 network, 96 samples with count weights."""
    N, n, L, h = 12, 24, 2, 256
    terms, H, ref = _setup(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, L, h, 6, 6, "fp32", max_batch=96, chunk_samples=40)
    params = init_params(n, L, h, seed=1)
    xs, w = unique_with_counts(sector_samples(n, 6, 6, 96, seed=2))
    net = _oracle_net(n, L, h, 6, 6)
    el_ref = vmc.local_energy(ref, net, params, xs)
    E_ref, _, _ = vmc.energy(el_ref, w)
    g_ref = vmc.gradient(net, params, xs, w, el_ref, E_ref)
    energy, grad, el = nqs.energy_grad(plan, torch.from_numpy(params).cuda(), xs, w)
    el = el.cpu().numpy()
    err = np.abs(el[:, 0] + 1j * el[:, 1] - el_ref)
    S = _eloc_scale(ref, net, params, xs[:8])
    gerr = np.linalg.norm(grad.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    dE = abs(energy[0].item() - E_ref)
    print(f"fp32: max |dE_loc|/S = {np.max(err[:8] / S):.3e}, |dE| = {dE:.3e}, |dg|/|g| = {gerr:.3e}")
    assert np.all(err[:8] <= 1e-4 * S)
    assert dE <= 1e-4
    assert gerr <= 1e-4


@pytest.mark.parametrize("prec,tol_e,pdtype", [("bf16x3", 1e-4, "fp32"), ("bf16", 5e-2, "fp32"),
                                               ("bf16w", 1e-4, "bf16")])
def test_energy_bf16_paths_16_qubits(nqs, ctx, prec, tol_e, pdtype):
    N, n, L, h = 8, 16, 3, 512
    terms, H, ref = _setup(nqs, ctx, N, seed=1)
    plan = nqs.Plan(ctx, H, L, h, 4, 4, prec, max_batch=64, dedup=True)
    params = init_params(n, L, h, seed=1, dtype=pdtype)
    xs, w = unique_with_counts(sector_samples(n, 4, 4, 64, seed=2))
    net = _oracle_net(n, L, h, 4, 4)
    el_ref = vmc.local_energy(ref, net, params, xs)
    E_ref, _, _ = vmc.energy(el_ref, w)
    g_ref = vmc.gradient(net, params, xs, w, el_ref, E_ref)
    energy, grad, el = nqs.energy_grad(plan, torch.from_numpy(params).cuda(), xs, w)
    dE = abs(energy[0].item() - E_ref)
    gerr = np.linalg.norm(grad.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    print(f"{prec}: |dE| = {dE:.3e} Ha, |dg|/|g| = {gerr:.3e}")
    assert dE <= tol_e
    if prec != "bf16":
        assert gerr <= 1e-3


def test_edge_cases(nqs, ctx):
    N, n = 6, 12
    terms, H, ref = _setup(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, 1, 64, 3, 3, "fp64", max_batch=64)
    params = torch.from_numpy(init_params(n, 1, 64, seed=1)).cuda()
    # empty batch
    out = nqs.local_energy(plan, params, np.zeros(0, dtype=np.uint64))
    assert out.shape == (0, 2)
    # a zero-amplitude (out-of-sector) sample raises the device flag, others unaffected
    xs = sector_samples(n, 3, 3, 5, seed=9)
    bad = xs.copy()
    bad[2] = np.uint64(0b111)          # 2 up, 1 down electrons
    el = nqs.local_energy(plan, params, bad).cpu().numpy()
    assert nqs.device_status(plan) & 1
    assert np.isnan(el[2, 0])
    good = nqs.local_energy(plan, params, xs).cpu().numpy()
    assert np.all(el[[0, 1, 3, 4]] == good[[0, 1, 3, 4]])
    assert nqs.device_status(plan) == 0
    # too small a workspace is rejected on the host
    import ctypes as C
    from paper_2208_05637_amd import _lib
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    st = plan.lib.nqs_local_energy(plan.handle, C.c_void_p(params.data_ptr()), C.c_void_p(0), 0,
                                   C.c_void_p(0), C.c_void_p(ws.data_ptr()), 1024)
    assert st == 4
    # batch above the plan's maximum
    with pytest.raises(_lib.NQSError):
        nqs.local_energy(plan, params, sector_samples(n, 3, 3, 65, seed=1))


@pytest.mark.parametrize("prec,h", [("bf16", 256), ("bf16", 1024), ("bf16x3", 512), ("bf16w", 1024),
                                    ("fp32", 1024), ("fp64", 1024)])
def test_deterministic(nqs, ctx, prec, h):
    """Two calls give bit-identical results (covers shapes whose head is split over k)."""
    N, n, L = 8, 16, 2
    terms, H, ref = _setup(nqs, ctx, N, seed=1)
    plan = nqs.Plan(ctx, H, L, h, 4, 4, prec, max_batch=300, dedup=True, chunk_samples=128)
    params = torch.from_numpy(init_params(n, L, h, seed=1)).cuda()
    xs, w = unique_with_counts(sector_samples(n, 4, 4, 300, seed=2))
    e1, g1, l1 = [t.clone() for t in nqs.energy_grad(plan, params, xs, w)]
    e2, g2, l2 = nqs.energy_grad(plan, params, xs, w)
    assert torch.equal(e1, e2) and torch.equal(g1, g2) and torch.equal(l1, l2)


def test_graph_capture_replay_matches_eager(nqs, ctx):
    N, n, L, h = 8, 16, 2, 256
    terms, H, ref = _setup(nqs, ctx, N, seed=1)
    xs, w = unique_with_counts(sector_samples(n, 4, 4, 200, seed=2))
    B = len(xs)
    plan = nqs.Plan(ctx, H, L, h, 4, 4, "bf16", max_batch=B, dedup=True, chunk_samples=64)
    params = torch.from_numpy(init_params(n, L, h, seed=1)).cuda()
    xt = torch.from_numpy(xs.view(np.int64)).cuda()
    wt = torch.from_numpy(w).cuda()
    eager = [t.clone() for t in nqs.energy_grad(plan, params, xt, wt)]
    energy = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty(plan.n_params, dtype=torch.float64, device="cuda")
    eloc = torch.empty((B, 2), dtype=torch.float64, device="cuda")
    plan.workspace()
    s = torch.cuda.Stream()
    ctx.use_stream(s)
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            nqs.energy_grad(plan, params, xt, wt, eloc=eloc, energy=energy, grad=grad)
    finally:
        ctx.use_stream(torch.cuda.current_stream())
    for rep in range(3):
        energy.zero_(); grad.zero_(); eloc.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(energy, eager[0]) and torch.equal(grad, eager[1]) and torch.equal(eloc, eager[2])
        _ = nqs.local_energy(plan, params, xt)     # eager work between replays
        torch.cuda.synchronize()


def test_autograd_function(nqs, ctx):
    N, n, L, h = 6, 12, 1, 64
    terms, H, ref = _setup(nqs, ctx, N)
    plan = nqs.Plan(ctx, H, L, h, 3, 3, "fp64", max_batch=200)
    xs, w = unique_with_counts(sector_samples(n, 3, 3, 200, seed=3))
    p = torch.from_numpy(init_params(n, L, h, seed=1)).cuda().requires_grad_(True)
    E, eloc = nqs.EnergyFn.apply(p, xs, w, plan)
    (3.0 * E).backward()
    _, g, _ = nqs.energy_grad(plan, p.detach(), xs, w)
    assert torch.allclose(p.grad.double(), 3.0 * g, rtol=1e-6, atol=1e-9)


def test_dedup_at_64_qubits_with_the_all_ones_configuration(nqs, ctx):
    """Exactly 64 qubits, where every 64-bit word is a configuration: a Hamiltonian of two-qubit X strings
    (no sector filter) whose flips take several samples to the all-ones string.  The distinct connected
    configurations equal np.unique of the entries (all-ones included), the entry map and first-entry order
    are exact, and the FP64 local energies with dedup on equal those with it off bit for bit."""
    n = 64
    rng = np.random.default_rng(11)
    pairs = [(0, 5), (3, 9), (62, 63), (17, 40), (8, 33)]
    xm = np.array([(1 << a) | (1 << b) for a, b in pairs], dtype=np.uint64)
    zm = np.array([(1 << (7 * k % 64)) for k in range(len(pairs))], dtype=np.uint64)
    cf = rng.normal(size=len(pairs))
    H = nqs.Hamiltonian(n, np.concatenate([xm, [0]]).astype(np.uint64), np.concatenate([zm, [3]]).astype(np.uint64),
                        np.concatenate([cf, [0.7]]), conserves_spin=False).upload(ctx)
    ones = np.uint64(2**64 - 1)
    xs = [ones ^ m for m in xm] + [ones] + list(rng.integers(0, 2**63, size=40, dtype=np.uint64) * np.uint64(2))
    xs = np.unique(np.array(xs, dtype=np.uint64))
    B = len(xs)
    mk = lambda d: nqs.Plan(ctx, H, 1, 64, -1, -1, "fp64", max_batch=B, chunk_samples=B, dedup=d)
    out = nqs.connected(mk(True), xs)
    torch.cuda.synchronize()
    ne, nu = int(out["n_entries"].item()), int(out["n_unique"].item())
    ex = out["x"][:ne].cpu().numpy().view(np.uint64)
    u = out["unique"][:nu].cpu().numpy().view(np.uint64)
    assert ne == B * len(pairs) and int(np.sum(ex == ones)) == len(pairs)
    assert np.array_equal(np.sort(u), np.unique(ex)) and ones in u
    eu = out["entry_unique"][:ne].cpu().numpy()
    assert np.array_equal(u[eu], ex)
    _, first = np.unique(ex, return_index=True)
    assert np.array_equal(u, ex[np.sort(first)])
    params = torch.from_numpy(init_params(n, 1, 64, seed=1, std=0.2)).cuda()
    e_on = nqs.local_energy(mk(True), params, xs)
    e_off = nqs.local_energy(mk(False), params, xs)
    torch.cuda.synchronize()
    assert torch.equal(e_on, e_off) and bool(torch.isfinite(e_on).all())


@pytest.mark.parametrize("n,K,B", [(12, 400, 90), (70, 500, 40)])
def test_connected_bit_exact_complex(nqs, ctx, n, K, B):
    """Random Pauli strings, many with an odd number of Y (imaginary folded coefficients), no sector filter,
    one and two 64-bit words, on samples that include neighbours of each other: connected sets, h (real and
    imaginary parts) and the diagonal bit-exact against the oracle; FP64 local energies with dedup on equal
    those with it off."""
    rng = np.random.default_rng(n + 3)
    W = 1 if n <= 64 else 2
    full = (1 << n) - 1

    def rnd():
        return (int(rng.integers(0, 2**62)) | (int(rng.integers(0, 2**62)) << 62)) & full

    # few distinct flips (several terms per group), sparse z masks
    flips = [0] + [rnd() & rnd() & rnd() for _ in range(K // 8)]
    xm = [flips[int(rng.integers(0, len(flips)))] for _ in range(K)]
    zm = [rnd() & rnd() for _ in range(K)]
    cf = rng.normal(size=K)
    ref = pauli.canonical_terms(np.array(xm, dtype=object), np.array(zm, dtype=object), cf)
    assert np.any(ref["ct"].imag != 0) and np.any(ref["ct"].real != 0)
    to_w = (lambda v: np.array(v, dtype=np.uint64)) if W == 1 else \
        (lambda v: np.array([[(a >> (64 * w)) & ((1 << 64) - 1) for w in range(2)] for a in v], dtype=np.uint64))
    H = nqs.Hamiltonian(n, to_w(xm), to_w(zm), cf, conserves_spin=False).upload(ctx)
    base = [rnd() for _ in range(B // 2)]
    xs_int = base + [b ^ flips[1 + k % (len(flips) - 1)] for k, b in enumerate(base)]
    xs_int = list(dict.fromkeys(xs_int))
    B = len(xs_int)
    xs = to_w(xs_int)
    plan = nqs.Plan(ctx, H, 1, 64, -1, -1, "fp64", max_batch=B, chunk_samples=B, dedup=True)
    out = nqs.connected(plan, xs)
    diag_ref, ent = vmc.connected(ref, np.array(xs_int, dtype=object) if W == 2 else xs, sector_filter=False)
    torch.cuda.synchronize()
    ne = int(out["n_entries"].item())
    assert ne == sum(len(e[0]) for e in ent)
    diag = out["diag"].cpu().numpy()
    assert np.array_equal(diag[:, 0], diag_ref.real) and np.array_equal(diag[:, 1], diag_ref.imag)
    ex = out["x"][:ne].cpu().numpy().view(np.uint64)
    ex = ex.reshape(-1).tolist() if W == 1 else [int(r[0]) | (int(r[1]) << 64) for r in ex.tolist()]
    eh = out["h"][:ne].cpu().numpy()
    es = out["sample"][:ne].cpu().numpy()
    pos = 0
    for i, (gi, xp, hv) in enumerate(ent):
        k = len(gi)
        assert np.all(es[pos:pos + k] == i)
        assert ex[pos:pos + k] == [int(v) for v in xp]
        assert np.array_equal(eh[pos:pos + k, 0], hv.real) and np.array_equal(eh[pos:pos + k, 1], hv.imag)
        pos += k
    params = torch.from_numpy(init_params(n, 1, 64, seed=2, std=0.2)).cuda()
    e_on = nqs.local_energy(plan, params, xs)
    off = nqs.Plan(ctx, H, 1, 64, -1, -1, "fp64", max_batch=B, chunk_samples=max(1, B // 3), dedup=False)
    e_off = nqs.local_energy(off, params, xs)
    torch.cuda.synchronize()
    assert nqs.device_status(plan) == 0 and nqs.device_status(off) == 0
    assert torch.equal(e_on, e_off) and bool(torch.isfinite(e_on).all())
