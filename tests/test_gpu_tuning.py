"""GPU checks of the tunable parts of the path, through the C ABI.

* every forward variant (waves per workgroup) against the oracle, at the
  same bars as the default variant;
* dedup on/off and the two chunk sizes the autotuner may pick give
  bit-identical local energies (they change only which rows are evaluated
  together, never a row's arithmetic or a sample's summation order);
* the autotuner times every candidate, applies the fastest and caches it;
* the forward's two grids (one workgroup per tile; resident workgroups
  looping over tiles) give bit-identical rows;
* the multi-instance call with instances of different precisions (several
  forward launch groups) equals single-instance calls bit for bit;
* dedup's look-back to the previous chunk evaluates exactly the distinct
  connected configurations that chunk did not (counted here from the oracle's
  connected sets) and changes no local energy, in single and multi calls.
"""
import numpy as np
import pytest
import torch

from oracle import made, pauli, vmc
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


@pytest.mark.parametrize("prec,h,L,tol", [
    ("fp32", 256, 2, 2e-5), ("fp32", 1024, 2, 2e-5),
    ("bf16x3", 256, 2, 5e-4), ("bf16x3", 512, 3, 5e-4), ("bf16x3", 1024, 2, 5e-4),
    ("bf16", 256, 2, 0.05), ("bf16", 512, 3, 0.05), ("bf16", 1024, 3, 0.05)])
def test_forward_variants_log_psi(nqs, ctx, prec, h, L, tol):
    N = 6
    n = 2 * N
    terms = hamiltonian(N, 0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    plan = nqs.Plan(ctx, H, L, h, 3, 3, prec, max_batch=16)
    params = init_params(n, L, h, seed=7, std=0.1)
    rng = np.random.default_rng(2)
    xs = rng.integers(0, 1 << n, 2500).astype(np.uint64)       # ragged last tile
    xs[:400] = pauli.sector_basis(n, 3, 3)
    la_ref, ph_ref, _ = made.forward(made.Net(n=n, n_layers=L, width=h, n_up=3, n_dn=3), params, xs)
    fin = np.isfinite(la_ref)
    p = torch.from_numpy(params).cuda()
    info = plan.kernel_info()
    default, full = info["waves_per_block"], info["rows_per_block"]
    tiles = [full] + ([full // 2] if full >= 64 else [])          # the half tile keeps 32 rows or more
    for waves, rows in [(w_, r_) for w_ in (default, 8 if default == 16 else 16) for r_ in tiles]:
        plan.configure(waves_per_block=waves, rows_per_block=rows)
        assert plan.kernel_info()["waves_per_block"] == waves and plan.kernel_info()["rows_per_block"] == rows
        out = nqs.log_psi(plan, p, xs).cpu().numpy()
        assert np.array_equal(np.isfinite(out[:, 0]), fin)
        e1 = np.max(np.abs(out[fin, 0] - la_ref[fin]))
        e2 = np.max(np.abs(out[:, 1] - ph_ref))
        print(f"{prec} h={h} waves={waves} rows={rows}: {e1:.3e} {e2:.3e}")
        assert e1 <= tol and e2 <= tol


def test_configure_rejects_bad_values(nqs, ctx):
    terms = hamiltonian(6, 0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    plan = nqs.Plan(ctx, H, 1, 64, 3, 3, "fp64", max_batch=64, dedup=False, chunk_samples=40)
    with pytest.raises(nqs.NQSError):
        plan.configure(waves_per_block=16)          # the FP64 forward has one variant
    with pytest.raises(nqs.NQSError):
        plan.configure(rows_per_block=8)            # no tile of 8 rows
    with pytest.raises(nqs.NQSError):
        plan.configure(dedup=True)                  # no dedup tables in this plan's workspace
    with pytest.raises(nqs.NQSError):
        plan.configure(chunk_samples=41)            # above the created chunk
    with pytest.raises(nqs.NQSError):
        plan.configure(chunk_samples=19)            # below half of it
    plan.configure(chunk_samples=20)
    assert plan.chunk_samples == 20


def test_dedup_and_chunk_bit_identical(nqs, ctx):
    """40 qubits: the four (dedup, chunk) choices give identical local energies."""
    N = 20
    n = 2 * N
    terms = hamiltonian(N, 0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    xs, w = unique_with_counts(sector_samples(n, N // 2, N // 2, 300, seed=9))
    plan = nqs.Plan(ctx, H, 2, 256, N // 2, N // 2, "bf16x3", max_batch=len(xs), dedup="auto",
                    chunk_samples=64)
    p = torch.from_numpy(init_params(n, 2, 256, seed=3)).cuda()
    outs = {}
    for dedup in (False, True):
        for chunk in (64, 32):
            plan.configure(dedup=dedup, chunk_samples=chunk)
            assert plan.dedup == dedup and plan.chunk_samples == chunk
            outs[(dedup, chunk)] = nqs.local_energy(plan, p, xs)
    torch.cuda.synchronize()
    assert nqs.device_status(plan) == 0
    first = outs[(False, 64)]
    for k, v in outs.items():
        assert torch.equal(v, first), k


def test_autotune_times_candidates_and_caches(nqs, ctx):
    N = 12
    n = 2 * N
    terms = hamiltonian(N, 0)
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    xs, w = unique_with_counts(sector_samples(n, N // 2, N // 2, 512, seed=4))
    plan = nqs.Plan(ctx, H, 2, 512, N // 2, N // 2, "bf16x3", max_batch=len(xs), dedup="auto",
                    chunk_samples=128)
    params = init_params(n, 2, 512, seed=5)
    p = torch.from_numpy(params).cuda()
    rep = plan.autotune(p, xs, force=True)
    cands = rep["candidates"]
    # workgroup shapes (8 or 16 waves x tiles of 64 or 32 rows) x dedup on/off x chunk {128, 64} x grid (one
    # workgroup per tile, resident)
    assert len(cands) == 32 and not rep["from_cache"]
    assert sorted({(c["waves_per_block"], c["rows_per_block"], c["dedup"], c["chunk_samples"], c["resident"])
                   for c in cands}) == \
        sorted((w_, m_, d_, c_, r_) for w_ in (8, 16) for m_ in (64, 32) for d_ in (False, True) for c_ in (128, 64)
               for r_ in (False, True))
    assert rep["probe_samples"] == min(len(xs), 256)
    assert all(c["ms"] > 0 for c in cands)
    best = cands[rep["chosen"]]
    assert best["ms"] == min(c["ms"] for c in cands)
    info = plan.kernel_info()
    assert info["tuned"] and info["waves_per_block"] == best["waves_per_block"]
    assert info["rows_per_block"] == best["rows_per_block"]
    assert plan.dedup == best["dedup"] and plan.chunk_samples == best["chunk_samples"]
    assert info["resident"] == best["resident"]
    print("autotune:", [(c["waves_per_block"], c["rows_per_block"], c["dedup"], c["chunk_samples"], c["resident"],
                         round(c["ms"], 3)) for c in cands], "chosen", rep["chosen"])
    # a second plan of the same shape takes the cached choice without timing
    plan2 = nqs.Plan(ctx, H, 2, 512, N // 2, N // 2, "bf16x3", max_batch=len(xs), dedup="auto",
                     chunk_samples=128)
    rep2 = plan2.autotune(p, xs)
    assert rep2["from_cache"] and plan2.kernel_info()["waves_per_block"] == best["waves_per_block"]
    assert plan2.kernel_info()["rows_per_block"] == best["rows_per_block"]
    assert plan2.kernel_info()["resident"] == best["resident"]
    # the tuned plan is still correct
    el = nqs.local_energy(plan2, p, xs).cpu().numpy()
    net = made.Net(n=n, n_layers=2, width=512, n_up=N // 2, n_dn=N // 2)
    el_ref = vmc.local_energy(ref, net, params, xs[:3])
    d = np.abs(el[:3, 0] + 1j * el[:3, 1] - el_ref)
    print("tuned |dE_loc|:", d)
    assert np.all(d <= 1e-3)


def test_multi_mixed_precisions_equal_single(nqs, ctx):
    """Instances of two precisions and two widths (three launch groups)."""
    items = []
    specs = [(6, 0, "fp32", 256, 2, 300), (7, 1, "bf16x3", 512, 2, 200), (8, 2, "bf16x3", 512, 2, 150),
             (5, 3, "fp64", 128, 1, 100)]
    keep = []
    for k, (N, seed, prec, h, L, B) in enumerate(specs):
        n = 2 * N
        terms = hamiltonian(N, seed)
        H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
        xs, w = unique_with_counts(sector_samples(n, N // 2, N // 2, B, seed=seed + 10))
        plan = nqs.Plan(ctx, H, L, h, N // 2, N // 2, prec, max_batch=len(xs), chunk_samples=max(8, len(xs) // 3))
        # the two split-BF16 instances differ only in the forward's grid: two launch groups
        plan.configure(resident=(k in (1, 3)))
        dev = ctx.device
        it = dict(plan=plan, params=torch.from_numpy(init_params(n, L, h, seed=seed)).to(dev),
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


@pytest.mark.parametrize("N,B,order_seed", [(22, 24, None), (32, 12, None), (20, 24, 5)])
def test_forward_launch_grouping_invariance(nqs, ctx, N, B, order_seed):
    """The connected-configuration rows give bit-identical log psi whether one
    launch evaluates all of them or several launches evaluate slices, and
    whether the grid holds one workgroup per tile or resident workgroups that
    loop over tiles (every row's arithmetic is independent of the others and
    of the grid)."""
    n = 2 * N
    terms = hamiltonian(N, 3)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    order = None if order_seed is None else np.random.default_rng(order_seed).permutation(n)
    xs = sector_samples(n, N // 2, N // 2, B, seed=8)
    for prec, h in (("bf16w", 512), ("bf16x3", 512), ("fp32", 256)):
        plan = nqs.Plan(ctx, H, 3, h, N // 2, N // 2, prec, max_batch=B, order=order)
        p = torch.from_numpy(init_params(n, 3, h, seed=2, dtype="bf16" if prec == "bf16w" else "fp32")).cuda()
        con = nqs.connected(plan, xs)
        ne = int(con["n_entries"].item())
        ent = con["x"][:ne].contiguous()
        M = plan.kernel_info()["rows_per_block"]
        whole = nqs.log_psi(plan, p, ent)
        step = 37 * M + 5          # ragged slices: tile boundaries shift between launches
        parts = torch.cat([nqs.log_psi(plan, p, ent[i:i + step]) for i in range(0, ne, step)])
        plan.configure(resident=True)
        assert plan.kernel_info()["resident"]
        res = nqs.log_psi(plan, p, ent)
        res_parts = torch.cat([nqs.log_psi(plan, p, ent[i:i + step]) for i in range(0, ne, step)])
        torch.cuda.synchronize()
        assert torch.equal(whole, parts), (prec, N)
        assert torch.equal(whole, res) and torch.equal(whole, res_parts), (prec, N, "resident")


def test_forward_launch_split_beyond_32_bit_work_items(nqs, ctx):
    """2^27 + 3 * 4096 rows need more than 2^32 work-items at 32 rows per 1,024-lane
    workgroup, so the forward is split into two dispatches; the rows cycle through all
    4,096 12-qubit configurations, so every row must equal its copy in the first cycle
    (bit for bit), and the first cycle the oracle."""
    n, L, h = 12, 1, 1024
    terms = hamiltonian(6, 0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    plan = nqs.Plan(ctx, H, L, h, -1, -1, "bf16w", max_batch=16)
    assert plan.kernel_info()["rows_per_block"] == 32 and plan.kernel_info()["waves_per_block"] == 16
    params = init_params(n, L, h, seed=3, dtype="bf16")
    rows = (1 << 27) + 3 * 4096
    assert (rows // 32) * 1024 > 2**32
    xs = torch.arange(rows, device="cuda", dtype=torch.int64) % 4096
    out = nqs.log_psi(plan, torch.from_numpy(params).cuda(), xs)
    torch.cuda.synchronize()
    first = out[:4096]
    assert torch.equal(out.view(-1, 4096, 2), first.unsqueeze(0).expand(rows // 4096, 4096, 2))
    la_ref, ph_ref, _ = made.forward(made.Net(n=n, n_layers=L, width=h), params, np.arange(4096, dtype=np.uint64))
    f = first.cpu().numpy()
    assert np.max(np.abs(f[:, 0] - la_ref)) <= 5e-4 and np.max(np.abs(f[:, 1] - ph_ref)) <= 5e-4
    # the resident grid takes all 2^22 + 384 tiles in one dispatch
    plan.configure(resident=True)
    out2 = nqs.log_psi(plan, torch.from_numpy(params).cuda(), xs)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    del out, out2, xs


def _lookback_rows(ref, xs, chunk):
    """Forward rows of a dedup call with look-back: the B sample rows, then
    per chunk its distinct connected configurations less those of the chunk
    before it (connected sets from the oracle, spin-sector filtered)."""
    _, ent = vmc.connected(ref, xs, sector_filter=True)
    rows, prev = len(xs), set()
    for c0 in range(0, len(xs), chunk):
        cur = set()
        for gi, xp, hv in ent[c0:c0 + chunk]:
            cur.update(int(v) for v in xp)
        rows += len(cur - prev)
        prev = cur
    return rows


@pytest.mark.parametrize("N,B,chunk,seed", [(6, 400, 40, 1), (6, 400, 7, 2), (10, 600, 64, 3), (12, 256, 30, 4)])
def test_dedup_look_back_rows_and_values(nqs, ctx, N, B, chunk, seed):
    """Samples in an order that makes neighbouring chunks share connected
    configurations: every sector configuration of 12 qubits, shuffled, and
    sampler-like streams at 20 and 24 qubits (each sample one excitation away
    from the one before)."""
    n = 2 * N
    terms = hamiltonian(N, 0)
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    H = nqs.Hamiltonian.from_terms(terms, conserves_spin=True).upload(ctx)
    rng = np.random.default_rng(seed)
    if N == 6:
        xs = pauli.sector_basis(n, 3, 3).astype(np.uint64)
        xs = xs[rng.permutation(len(xs))][:B]
    else:
        x = sector_samples(n, N // 2, N // 2, 1, seed=seed)[0]
        seen, out = set(), []
        while len(out) < B:           # a walk over single same-spin hops
            if int(x) not in seen:
                seen.add(int(x))
                out.append(x)
            bits = [b for b in range(n) if (int(x) >> b) & 1]
            i = int(rng.choice(bits))
            holes = [b for b in range(i % 2, n, 2) if not (int(x) >> b) & 1]
            j = int(rng.choice(holes))
            x = np.uint64(int(x) ^ (1 << i) ^ (1 << j))
        xs = np.array(out, dtype=np.uint64)
    B = len(xs)
    w = np.full(B, 1.0 / B)
    p = torch.from_numpy(init_params(n, 1, 64, seed=seed)).cuda()
    on = nqs.Plan(ctx, H, 1, 64, N // 2, N // 2, "fp64", max_batch=B, chunk_samples=chunk, dedup=True)
    off = nqs.Plan(ctx, H, 1, 64, N // 2, N // 2, "fp64", max_batch=B, chunk_samples=chunk, dedup=False)
    on.profile(True)
    e_on = nqs.local_energy(on, p, xs)
    torch.cuda.synchronize()
    prof = on.profile_read()
    on.profile(False)
    e_off = nqs.local_energy(off, p, xs)
    torch.cuda.synchronize()
    assert nqs.device_status(on) == 0 and nqs.device_status(off) == 0
    assert torch.equal(e_on, e_off)
    nchunks = (B + chunk - 1) // chunk
    assert prof["forward_launches"] == 1 + nchunks
    expect = _lookback_rows(ref, xs, chunk)
    print(f"N={N} B={B} chunk={chunk}: {int(prof['forward_rows'])} forward rows, expected {expect}")
    assert int(prof["forward_rows"]) == expect
    # the multi-instance form: two instances with different chunkings, one with look-back
    dev = ctx.device
    items = []
    for plan in (on, off):
        items.append(dict(plan=plan, params=p, samples=torch.from_numpy(xs.view(np.int64)).to(dev),
                          weights=torch.from_numpy(w).to(dev),
                          eloc=torch.empty((B, 2), dtype=torch.float64, device=dev),
                          energy=torch.empty(3, dtype=torch.float64, device=dev),
                          grad=torch.empty(on.n_params, dtype=torch.float64, device=dev)))
    ws = nqs.multi_workspace(items)
    nqs.energy_grad_multi(items, ws)
    torch.cuda.synchronize()
    assert nqs.multi_device_status(items, ws) == 0
    for it in items:
        assert torch.equal(it["eloc"], e_off)


def test_dedup_look_back_with_empty_chunks(nqs, ctx):
    """A Hamiltonian of Z strings only: no chunk has a connected configuration, so every dedup and
    look-back set is empty; the local energies are the diagonal (bit-exact against the oracle's sum)
    and the forward evaluates the samples alone."""
    n = 12
    rng = np.random.default_rng(21)
    zm = np.array([int(v) for v in rng.integers(1, 1 << n, 30)], dtype=np.uint64)
    cf = rng.normal(size=30)
    H = nqs.Hamiltonian(n, np.zeros(30, dtype=np.uint64), zm, cf, conserves_spin=False).upload(ctx)
    ref = pauli.canonical_terms(np.zeros(30, dtype=np.uint64), zm, cf)
    xs = pauli.sector_basis(n, 3, 3).astype(np.uint64)[:50]
    plan = nqs.Plan(ctx, H, 1, 64, -1, -1, "fp64", max_batch=len(xs), chunk_samples=7, dedup=True)
    p = torch.from_numpy(init_params(n, 1, 64, seed=4)).cuda()
    plan.profile(True)
    el = nqs.local_energy(plan, p, xs)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    assert nqs.device_status(plan) == 0
    diag, ent = vmc.connected(ref, xs, sector_filter=False)
    assert all(len(e[0]) == 0 for e in ent)
    out = el.cpu().numpy()
    assert np.array_equal(out[:, 0], diag.real) and np.array_equal(out[:, 1], diag.imag)
    assert int(prof["forward_rows"]) == len(xs)


def test_multi_half_tiles_equal_single(nqs, ctx):
    """Instances whose forwards run the half tile (32 rows at h = 512) in one multi-instance call: the
    multi-segment form of the half-tile kernels against single calls, bit for bit."""
    items, keep = [], []
    for k, (N, seed, waves) in enumerate([(7, 1, 16), (8, 2, 16), (6, 3, 8)]):
        n = 2 * N
        terms = hamiltonian(N, seed)
        H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
        xs, w = unique_with_counts(sector_samples(n, N // 2, N // 2, 150, seed=seed + 20))
        plan = nqs.Plan(ctx, H, 2, 512, N // 2, N // 2, "bf16x3", max_batch=len(xs), dedup=True,
                        chunk_samples=max(8, len(xs) // 3))
        plan.configure(waves_per_block=waves, rows_per_block=32, resident=(k != 1))
        assert plan.kernel_info()["rows_per_block"] == 32
        dev = ctx.device
        items.append(dict(plan=plan, params=torch.from_numpy(init_params(n, 2, 512, seed=seed)).to(dev),
                          samples=torch.from_numpy(xs.view(np.int64)).to(dev), weights=torch.from_numpy(w).to(dev),
                          eloc=torch.empty((len(xs), 2), dtype=torch.float64, device=dev),
                          energy=torch.empty(3, dtype=torch.float64, device=dev),
                          grad=torch.empty(plan.n_params, dtype=torch.float64, device=dev)))
        keep.append(H)
    ws = nqs.multi_workspace(items)
    nqs.energy_grad_multi(items, ws)
    torch.cuda.synchronize()
    assert nqs.multi_device_status(items, ws) == 0
    for it in items:
        e1, g1, l1 = nqs.energy_grad(it["plan"], it["params"], it["samples"], it["weights"])
        assert torch.equal(l1, it["eloc"]) and torch.equal(g1, it["grad"]) and torch.equal(e1, it["energy"])


@pytest.mark.parametrize("prec,h,waves", [("bf16x3", 512, 16), ("bf16w", 512, 16), ("bf16", 1024, 16),
                                          ("fp32", 256, 8)])
def test_half_tile_repeatable(nqs, ctx, prec, h, waves):
    """The half-tile shapes give the same local energies on every call (five calls, resident grid and one
    workgroup per tile), within 5e-4 of the full tile's."""
    N = 8
    n = 2 * N
    terms = hamiltonian(N, 0)
    H = nqs.Hamiltonian.from_terms(terms).upload(ctx)
    xs, w = unique_with_counts(sector_samples(n, N // 2, N // 2, 300, seed=6))
    plan = nqs.Plan(ctx, H, 2, h, N // 2, N // 2, prec, max_batch=len(xs), dedup=True, chunk_samples=100)
    p = torch.from_numpy(init_params(n, 2, h, seed=2, dtype="bf16" if prec == "bf16w" else "fp32")).cuda()
    full = plan.kernel_info()["rows_per_block"]
    ref = nqs.local_energy(plan, p, xs).clone()
    for resident in (True, False):
        plan.configure(waves_per_block=waves, rows_per_block=full // 2, resident=resident)
        first = nqs.local_energy(plan, p, xs).clone()
        for _ in range(4):
            assert torch.equal(nqs.local_energy(plan, p, xs), first)
        tol = 0.05 if prec == "bf16" else 5e-4
        assert float((first - ref).abs().max()) <= tol
    assert nqs.device_status(plan) == 0
