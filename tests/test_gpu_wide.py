"""GPU parity above 64 qubits (bit strings of two 64-bit words) against the
FP64 oracle, through the C ABI.

Workload: a sparser synthetic molecule on 76 qubits, the size of the paper's
largest system (Sec. 6): 38 spatial orbitals, two-electron integrals of
magnitude below 0.05 set to zero before the Jordan-Wigner expansion (about
25,000 merged terms, 3,600 flip groups, ~1,500 connected configurations per
sample), samples uniform in the (19, 19) sector.  The Z strings of the
expansion cross the word boundary, so every kernel sees both words.  Edge
widths: 65 qubits (one bit in the second word) and 128 (both words full).

Tolerances are those of the one-word parity tests: bit-exact connected sets
and matrix elements; FP64 log psi 1e-12, E_loc 1e-10 of the summand scale
S_i, gradient 1e-9 relative; FP32 2e-5.  The split-BF16 kinds keep the
per-position bound of the 12-qubit tests (5e-4 over 12 positions): log|psi|
is half a sum of one log-sigmoid per free position, each off by the logit's
rounding, so the bar is 5e-4 n / 12.
"""
import numpy as np
import pytest
import torch

from oracle import made, pauli, vmc
from gen.inputs import hamiltonian, init_params, sector_samples, unique_with_counts

pytestmark = pytest.mark.gpu

N76, CUT = 38, 0.05


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


@pytest.fixture(scope="module")
def h76(nqs, ctx):
    terms = hamiltonian(N76, 0, cutoff=CUT)
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    return terms, H, ref


def _ints(words):
    return [int(r[0]) | (int(r[1]) << 64) for r in np.asarray(words).view(np.uint64).tolist()]


def _words(ints, W=2):
    return np.array([[(v >> (64 * w)) & ((1 << 64) - 1) for w in range(W)] for v in ints], dtype=np.uint64)


def _random_strings(n, count, rng):
    """Uniform n-bit strings as [count, 2] words."""
    ints = [int(rng.integers(0, 2**63)) | (int(rng.integers(0, 2**63)) << 63) | (int(rng.integers(0, 4)) << 126)
            for _ in range(count)]
    return _words([v & ((1 << n) - 1) for v in ints])


def _z_only_ham(nqs, ctx, n):
    """A one-term Hamiltonian (Z on the last qubit) to carry n for a plan."""
    x = np.zeros((1, 2), dtype=np.uint64)
    z = _words([1 << (n - 1)])
    return nqs.Hamiltonian(n, x, z, [1.0]).upload(ctx)


@pytest.mark.parametrize("filt", [True, False])
def test_wide_connected_bit_exact(nqs, ctx, h76, filt):
    terms, _, ref = h76
    n = 2 * N76
    H = nqs.Hamiltonian.from_terms(terms, conserves_spin=filt).upload(ctx)
    B = 70
    plan = nqs.Plan(ctx, H, 1, 64, 19, 19, "fp64", max_batch=B, chunk_samples=B, dedup=True)
    assert plan.dedup
    xs = sector_samples(n, 19, 19, B, seed=5)
    # samples 1..8: connected configurations of sample 0, so the chunk shares configurations
    _, ent0 = vmc.connected(ref, xs[:1])
    xs[1:9] = _words([int(v) for v in ent0[0][1][:8].tolist()])
    out = nqs.connected(plan, xs)
    diag_ref, ent = vmc.connected(ref, xs, sector_filter=filt)
    torch.cuda.synchronize()
    ne = int(out["n_entries"].item())
    assert ne == sum(len(e[0]) for e in ent)
    diag = out["diag"].cpu().numpy()
    assert np.array_equal(diag[:, 0], diag_ref.real) and np.array_equal(diag[:, 1], diag_ref.imag)
    es = out["sample"][:ne].cpu().numpy()
    ex = _ints(out["x"][:ne].cpu().numpy())
    eh = out["h"][:ne].cpu().numpy()
    pos = 0
    for i, (gi, xp, hv) in enumerate(ent):
        k = len(gi)
        assert np.all(es[pos:pos + k] == i)
        assert ex[pos:pos + k] == [int(v) for v in xp]      # canonical order, bit-exact
        assert np.array_equal(eh[pos:pos + k, 0], hv.real)
        assert np.array_equal(eh[pos:pos + k, 1], hv.imag)
        pos += k
    assert any(v >> 64 for v in ex) and any(v & 1 for v in ex)
    # dedup: the distinct configurations in the order of their first entries, and each entry's index
    nu = int(out["n_unique"].item())
    uq = _ints(out["unique"][:nu].cpu().numpy())
    first = list(dict.fromkeys(ex))
    assert uq == first and nu < ne
    eu = out["entry_unique"][:ne].cpu().numpy()
    assert [uq[j] for j in eu.tolist()] == ex


@pytest.mark.parametrize("n,prec,h,L,order_kind,tol", [
    (76, "fp64", 64, 2, "reverse", 1e-12), (76, "fp64", 128, 1, "identity", 1e-12),
    (76, "fp64", 64, 2, "random", 1e-12), (65, "fp64", 64, 2, "reverse", 1e-12),
    (128, "fp64", 256, 2, "reverse", 1e-12), (128, "fp64", 64, 1, "random", 1e-12),
    (76, "fp32", 256, 2, "random", 2e-5), (100, "fp32", 1024, 2, "reverse", 2e-5),
    (76, "bf16x3", 256, 2, "reverse", 5e-4 * 76 / 12), (76, "bf16w", 512, 3, "reverse", 5e-4 * 76 / 12),
    (128, "bf16w", 1024, 2, "random", 5e-4 * 128 / 12)])
@pytest.mark.parametrize("constrained", [True, False])
def test_wide_log_psi_parity(nqs, ctx, n, prec, h, L, order_kind, tol, constrained):
    H = _z_only_ham(nqs, ctx, n)
    rng = np.random.default_rng(n + h + L)
    order = {"reverse": None, "identity": np.arange(n), "random": rng.permutation(n)}[order_kind]
    nu, nd = ((n + 1) // 4, n // 4) if constrained else (-1, -1)
    plan = nqs.Plan(ctx, H, L, h, nu, nd, prec, max_batch=16, order=order)
    params = init_params(n, L, h, seed=7, std=0.1 if h >= 512 else 0.3,
                         dtype="bf16" if prec == "bf16w" else "fp32")
    count = 1100                                             # several tiles and a ragged tail
    xs = _random_strings(n, count, rng)
    if constrained:
        xs[:600] = sector_samples(n, nu, nd, 600, seed=n)
    net = made.Net(n=n, n_layers=L, width=h, n_up=nu, n_dn=nd, order=order)
    la_ref, ph_ref, _ = made.forward(net, params, xs)
    out = nqs.log_psi(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    fin = np.isfinite(la_ref)
    assert np.array_equal(np.isfinite(out[:, 0]), fin)
    if constrained:
        assert fin[:600].all() and not fin.all()
    err_la = np.max(np.abs(out[fin, 0] - la_ref[fin]))
    err_ph = np.max(np.abs(out[:, 1] - ph_ref))
    print(f"n={n} {prec} h={h} L={L} {order_kind}: max|d log|psi|| = {err_la:.3e}, max|d phi| = {err_ph:.3e}")
    assert err_la <= tol and err_ph <= tol


@pytest.mark.parametrize("mode", [0, 1])
def test_wide_log_psi_separate_phase_network(nqs, ctx, mode):
    n, L, h = 76, 2, 128
    H = _z_only_ham(nqs, ctx, n)
    plan = nqs.Plan(ctx, H, L, h, 19, 19, "fp64", max_batch=16, phase_mode=mode)
    params = init_params(n, L, h, seed=3, std=0.3, phase_mode=mode)
    xs = sector_samples(n, 19, 19, 300, seed=4)
    net = made.Net(n=n, n_layers=L, width=h, n_up=19, n_dn=19, phase_mode=mode)
    la_ref, ph_ref, _ = made.forward(net, params, xs)
    out = nqs.log_psi(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    assert np.max(np.abs(out[:, 0] - la_ref)) <= 1e-12 and np.max(np.abs(out[:, 1] - ph_ref)) <= 1e-12


def _eloc_scale(ref, net, params, xs):
    """S_i = sum_k |summand_k| of Eq. local_energy_auto (the rounding scale)."""
    xi = pauli.configs(xs)
    la, _, _ = made.forward(net, params, xi)
    out = []
    for i, x in enumerate(xi):
        l2, _, _ = made.forward(net, params, x ^ ref["x"])
        with np.errstate(invalid="ignore"):
            r = np.where(np.isfinite(l2), np.exp(l2 - la[i]), 0.0)
        out.append(np.sum(np.abs(ref["ct"]) * r))
    return np.array(out)


@pytest.mark.parametrize("chunk", [0, 40])
def test_wide_local_energy_fp64(nqs, ctx, h76, chunk):
    """76 qubits, FP64 network: |dE_loc| <= 1e-10 S_i (chunk 40: three chunks, ragged tail)."""
    terms, H, ref = h76
    n, L, h, B = 2 * N76, 2, 64, 96
    plan = nqs.Plan(ctx, H, L, h, 19, 19, "fp64", max_batch=B, chunk_samples=chunk)
    params = init_params(n, L, h, seed=1, std=0.3)
    xs = sector_samples(n, 19, 19, B, seed=2)
    net = made.Net(n=n, n_layers=L, width=h, n_up=19, n_dn=19)
    el_ref = vmc.local_energy(ref, net, params, xs)
    el = nqs.local_energy(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    S = _eloc_scale(ref, net, params, xs[:16])
    err = np.abs((el[:, 0] + 1j * el[:, 1]) - el_ref)
    print(f"max |dE_loc| = {err.max():.3e}, max relative to S_i = {np.max(err[:16] / S):.3e}")
    assert np.all(err[:16] <= 1e-10 * S)
    assert err.max() <= 1e-10 * np.max(S)
    assert nqs.device_status(plan) == 0


def test_wide_energy_and_gradient_fp64(nqs, ctx, h76):
    terms, H, ref = h76
    n, L, h = 2 * N76, 2, 64
    plan = nqs.Plan(ctx, H, L, h, 19, 19, "fp64", max_batch=128)
    params = init_params(n, L, h, seed=1, std=0.3)
    xs, w = unique_with_counts(np.concatenate([sector_samples(n, 19, 19, 100, seed=2)] * 2)[:150])
    net = made.Net(n=n, n_layers=L, width=h, n_up=19, n_dn=19)
    el_ref = vmc.local_energy(ref, net, params, xs)
    E_ref, I_ref, W_ref = vmc.energy(el_ref, w)
    g_ref = vmc.gradient(net, params, xs, w, el_ref, E_ref)
    energy, grad, el = nqs.energy_grad(plan, torch.from_numpy(params).cuda(), xs, w)
    energy = energy.cpu().numpy()
    grad = grad.cpu().numpy()
    print(f"E = {energy[0]:.15f} (oracle {E_ref:.15f}); |dg|/|g| = "
          f"{np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref):.3e}")
    assert np.max(w) == 2.0 and energy[2] == W_ref
    assert abs(energy[0] - E_ref) <= 1e-10 * max(1.0, abs(E_ref))
    assert abs(energy[1] - I_ref) <= 1e-10 * max(1.0, abs(E_ref))
    assert np.linalg.norm(grad - g_ref) <= 1e-9 * np.linalg.norm(g_ref)


def test_wide_energy_bf16_weights(nqs, ctx, h76):
    """The timed network kind (BF16 weights, split activations) at 76 qubits:
    |dE| <= 1e-4 Ha and the gradient to 1e-3 relative, as at 16 qubits."""
    terms, H, ref = h76
    n, L, h = 2 * N76, 3, 512
    plan = nqs.Plan(ctx, H, L, h, 19, 19, "bf16w", max_batch=64)
    params = init_params(n, L, h, seed=1, dtype="bf16")
    xs, w = unique_with_counts(sector_samples(n, 19, 19, 64, seed=2))
    net = made.Net(n=n, n_layers=L, width=h, n_up=19, n_dn=19)
    el_ref = vmc.local_energy(ref, net, params, xs)
    E_ref, _, _ = vmc.energy(el_ref, w)
    g_ref = vmc.gradient(net, params, xs, w, el_ref, E_ref)
    energy, grad, el = nqs.energy_grad(plan, torch.from_numpy(params).cuda(), xs, w)
    dE = abs(energy[0].item() - E_ref)
    gerr = np.linalg.norm(grad.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    print(f"bf16w 76 qubits: |dE| = {dE:.3e} Ha, |dg|/|g| = {gerr:.3e}")
    assert dE <= 1e-4 and gerr <= 1e-3


def test_wide_rejections(nqs, ctx, h76):
    """Two-word plans reject one-word sample arrays."""
    terms, H, ref = h76
    n = 2 * N76
    plan = nqs.Plan(ctx, H, 1, 64, 19, 19, "fp64", max_batch=8, dedup="auto")
    params = torch.from_numpy(init_params(n, 1, 64, seed=1)).cuda()
    xs = torch.from_numpy(sector_samples(n, 19, 19, 4, seed=1).view(np.int64)).cuda()
    with pytest.raises(ValueError):
        nqs.local_energy(plan, params, xs.reshape(-1))          # one word per sample


def test_wide_multi_instance_equal_single(nqs, ctx, h76):
    """One nqs_energy_grad_multi call over a 12-qubit instance, a 76-qubit one
    and a 76-qubit one with the separate phase network (two-word instances run
    their forwards as launches of their own): every output equal bit for bit
    to the instance's single call."""
    terms76, H76, _ = h76
    t12 = hamiltonian(6, 0)
    H12 = nqs.Hamiltonian.from_terms(t12).upload(ctx)
    dev = ctx.device
    items = []
    for H, n, nu, prec, h, L, mode, B in ((H12, 12, 3, "fp64", 64, 1, 0, 90), (H76, 76, 19, "fp64", 64, 2, 0, 40),
                                          (H76, 76, 19, "bf16w", 512, 2, 1, 30)):
        plan = nqs.Plan(ctx, H, L, h, nu, nu, prec, max_batch=B, chunk_samples=max(8, B // 3), phase_mode=mode)
        xs = sector_samples(n, nu, nu, B, seed=n + B)
        params = init_params(n, L, h, seed=2, std=0.3 if h < 512 else 0.1, phase_mode=mode,
                             dtype="bf16" if prec == "bf16w" else "fp32")
        items.append(dict(plan=plan, params=torch.from_numpy(params).to(dev),
                          samples=torch.from_numpy(np.ascontiguousarray(xs).view(np.int64)).to(dev),
                          weights=torch.ones(B, dtype=torch.float64, device=dev),
                          eloc=torch.empty((B, 2), dtype=torch.float64, device=dev),
                          energy=torch.empty(3, dtype=torch.float64, device=dev),
                          grad=torch.empty(plan.n_params, dtype=torch.float64, device=dev)))
    nqs.energy_grad_multi(items)
    torch.cuda.synchronize()
    for it in items:
        e1, g1, l1 = nqs.energy_grad(it["plan"], it["params"], it["samples"], it["weights"])
        assert torch.equal(l1, it["eloc"]) and torch.equal(g1, it["grad"]) and torch.equal(e1, it["energy"])
        assert nqs.device_status(it["plan"]) == 0


@pytest.mark.parametrize("n,L,h,nu,nd,draws,umax,order_seed", [
    (66, 2, 64, 3, 2, 100000, 10**6, None), (76, 1, 128, 19, 19, 10**9, 300, 7), (128, 1, 64, 4, 4, 5000, 64, 3)])
def test_wide_sampler_matches_oracle_fp64(nqs, ctx, n, L, h, nu, nd, draws, umax, order_seed):
    """The GPU sampler on two-word strings with the FP64 network: the same
    configurations and counts as the oracle sampler, draw for draw (an
    unbounded buffer at 66 qubits; elimination at 76 and 128)."""
    order = None if order_seed is None else np.random.default_rng(order_seed).permutation(n)
    H = _z_only_ham(nqs, ctx, n)
    plan = nqs.Plan(ctx, H, L, h, nu, nd, "fp64", max_batch=16, order=order)
    params = init_params(n, L, h, seed=n + L, std=0.5)
    x, w = nqs.sample(plan, torch.from_numpy(params).cuda(), draws, seed=12345, max_unique=umax)
    xg = _ints(x.cpu().numpy())
    from oracle import sampler
    net = made.Net(n=n, n_layers=L, width=h, n_up=nu, n_dn=nd, order=order)
    xr, cr = sampler.sample(net, params, draws, seed=12345, max_unique=umax)
    print(f"n={n}: {len(xr)} unique of {draws} draws (cap {umax}); GPU {len(xg)}")
    assert xg == [int(v) for v in xr.tolist()]
    assert np.array_equal(w.cpu().numpy(), cr.astype(np.float64))
    assert any(v >> 64 for v in xg)


@pytest.mark.parametrize("prec,h,L", [("fp64", 64, 2), ("bf16w", 512, 3)])
def test_wide_dedup_on_off_bit_identical(nqs, ctx, h76, prec, h, L):
    """Dedup only regroups rows: with two-word keys the local energies are bit
    for bit those without it, over several chunks of samples drawn from the
    network, with eight connected configurations of the first sample placed
    after it so that the first chunk shares configurations."""
    terms, H, ref = h76
    n = 2 * N76
    params = torch.from_numpy(init_params(n, L, h, seed=1, std=0.3 if h < 512 else 0.1,
                                          dtype="bf16" if prec == "bf16w" else "fp32")).cuda()
    mk = lambda d: nqs.Plan(ctx, H, L, h, 19, 19, prec, max_batch=200, dedup=d, chunk_samples=64)
    x, w = nqs.sample(mk(False), params, 10**9, seed=3, max_unique=200)
    nb = nqs.connected(mk(False), x[:1])["x"][:8]
    x = torch.cat([x[:1], nb, x[1:]])[:200].contiguous()
    pd = mk(True)
    e_on = nqs.local_energy(pd, params, x)
    e_off = nqs.local_energy(mk(False), params, x)
    con = nqs.connected(mk(True), x[:64])
    ne, nu = int(con["n_entries"].item()), int(con["n_unique"].item())
    print(f"{prec}: 200 sampled configurations, first chunk {ne} entries, {nu} distinct ({ne / nu:.2f})")
    assert pd.dedup and nu < ne
    assert torch.equal(e_on, e_off)
    assert nqs.device_status(pd) == 0


def test_wide_graph_capture_replay_matches_eager(nqs, ctx, h76):
    """A 76-qubit energy-and-gradient step (dedup on, three chunks) captured in
    a HIP graph: every replay equals the eager call, with eager work between
    replays."""
    terms, H, ref = h76
    n, L, h = 2 * N76, 2, 256
    dev = ctx.device
    params = torch.from_numpy(init_params(n, L, h, seed=1, std=0.2)).to(dev)
    plan = nqs.Plan(ctx, H, L, h, 19, 19, "fp32", max_batch=96, dedup=True, chunk_samples=32)
    xt, wt = nqs.sample(plan, params, 10**8, seed=6, max_unique=96)
    B = xt.shape[0]
    eager = [t.clone() for t in nqs.energy_grad(plan, params, xt, wt)]
    energy = torch.empty(3, dtype=torch.float64, device=dev)
    grad = torch.empty(plan.n_params, dtype=torch.float64, device=dev)
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev)
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


def test_wide_autotune_choices(nqs, ctx, h76):
    """The autotuner on a two-word plan (dedup auto) times every candidate;
    for one workgroup shape the dedup and chunk choices give the same local
    energies bit for bit (they only regroup rows), and the two shapes (whose
    head sums its k slices in another order) agree to the 1e-3 bar of the
    sampled full-size checks."""
    terms, H, ref = h76
    n, L, h = 2 * N76, 2, 512
    dev = ctx.device
    params = torch.from_numpy(init_params(n, L, h, seed=1, dtype="bf16")).to(dev)
    plan = nqs.Plan(ctx, H, L, h, 19, 19, "bf16w", max_batch=64, dedup="auto", chunk_samples=32)
    xs = torch.from_numpy(sector_samples(n, 19, 19, 64, seed=8).view(np.int64)).to(dev)
    rep = plan.autotune(params, xs)
    assert len(rep["candidates"]) >= 4
    by_shape = {}
    for c in rep["candidates"]:
        plan.configure(waves_per_block=c["waves_per_block"], rows_per_block=c["rows_per_block"], dedup=c["dedup"],
                       chunk_samples=c["chunk_samples"], resident=c["resident"])
        el = nqs.local_energy(plan, params, xs).clone()
        first = by_shape.setdefault((c["waves_per_block"], c["rows_per_block"]), el)
        assert torch.equal(el, first), c
    shapes = list(by_shape.values())
    assert len(shapes) == 4      # 8 or 16 waves x tiles of 64 or 32 rows at h = 512
    d = max(float((a - shapes[0]).abs().max()) for a in shapes[1:])
    print(f"76 qubits: max |dE_loc| between the workgroup shapes = {d:.3e}")
    assert d <= 1e-3
    assert nqs.device_status(plan) == 0
