"""GPU parity of the structured matrix elements (NQS_H_TABLES) against the
FP64 oracle, through the C ABI.

The tables give h_g(x) of Eq. mtx_element summed over a flip group in another
order (sub-group by sub-group), so the bars are:
  * connected configurations and their samples: bit-exact (integer work);
  * h and the diagonal: 2 m eps sum_k |c_k| per group (m terms; the rounding
    of two summation orders of the same m terms);
  * E_loc of the FP64 network: 1e-10 S_i, as without tables;
  * with the BF16-weight network at 60 qubits: local energies within 1e-9 of
    the term-list path's (which differ only by the rounding of h).
"""
import numpy as np
import pytest
import torch

from oracle import made, pauli, vmc
from gen.inputs import config_inputs, hamiltonian, init_params, sector_samples

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


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


def _ints(a, W):
    a = np.asarray(a).view(np.uint64)
    if W == 1:
        return [int(v) for v in a.tolist()]
    return [int(r[0]) | (int(r[1]) << 64) for r in a.tolist()]


def _bounds(ref):
    """Per group: 2 m eps sum |c| over the group's terms."""
    gx, goff = pauli.groups(ref)
    m = np.diff(goff)
    s = np.add.reduceat(np.abs(ref["c"]), goff[:-1]) if len(gx) else np.zeros(0)
    return 2 * m * EPS * s


@pytest.mark.parametrize("N,cutoff,B", [(6, 0.0, 257), (12, 0.0, 70), (38, 0.05, 40)])
def test_tables_connected(nqs, ctx, N, cutoff, B):
    n = 2 * N
    W = 1 if n <= 64 else 2
    terms = hamiltonian(N, 0, cutoff=cutoff)
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    H = nqs.Hamiltonian.from_terms(terms, tables=True).upload(ctx)
    plan = nqs.Plan(ctx, H, 1, 64, N // 2, N // 2, "fp64", max_batch=B, chunk_samples=B)
    xs = sector_samples(n, N // 2, N // 2, B, seed=5)
    out = nqs.connected(plan, xs)
    diag_ref, ent = vmc.connected(ref, xs)
    bound = _bounds(ref)
    torch.cuda.synchronize()
    ne = int(out["n_entries"].item())
    assert ne == sum(len(e[0]) for e in ent)
    diag = out["diag"].cpu().numpy()
    assert np.all(np.abs(diag[:, 0] + 1j * diag[:, 1] - diag_ref) <= bound[0])
    es = out["sample"][:ne].cpu().numpy()
    ex = _ints(out["x"][:ne].cpu().numpy(), W)
    eh = out["h"][:ne].cpu().numpy()
    pos, worst = 0, 0.0
    for i, (gi, xp, hv) in enumerate(ent):
        k = len(gi)
        assert np.all(es[pos:pos + k] == i)
        assert ex[pos:pos + k] == [int(v) for v in xp.tolist()]
        d = np.abs(eh[pos:pos + k, 0] + 1j * eh[pos:pos + k, 1] - hv)
        assert np.all(d <= bound[gi])
        worst = max(worst, float(np.max(d / np.maximum(bound[gi], 1e-300))) if k else 0.0)
        pos += k
    print(f"N={N}: {ne} entries, max |dh| / bound = {worst:.3f}")


@pytest.mark.parametrize("N,cutoff,L,h,B", [(6, 0.0, 1, 64, 512), (38, 0.05, 2, 64, 48)])
def test_tables_local_energy_fp64(nqs, ctx, N, cutoff, L, h, B):
    n = 2 * N
    terms = hamiltonian(N, 0, cutoff=cutoff)
    ref = pauli.canonical_terms(terms.x_mask, terms.z_mask, terms.coeff)
    H = nqs.Hamiltonian.from_terms(terms, tables=True).upload(ctx)
    plan = nqs.Plan(ctx, H, L, h, N // 2, N // 2, "fp64", max_batch=B, dedup=n < 64)
    params = init_params(n, L, h, seed=1, std=0.3)
    xs = sector_samples(n, N // 2, N // 2, B, seed=2)
    net = made.Net(n=n, n_layers=L, width=h, n_up=N // 2, n_dn=N // 2)
    el_ref = vmc.local_energy(ref, net, params, xs)
    el = nqs.local_energy(plan, torch.from_numpy(params).cuda(), xs).cpu().numpy()
    # S_i: sum of |summand| over the terms (the rounding scale of the sum)
    xi = pauli.configs(xs[:8])
    la, _, _ = made.forward(net, params, xi)
    S = []
    for i, x in enumerate(xi):
        l2, _, _ = made.forward(net, params, x ^ ref["x"])
        with np.errstate(invalid="ignore"):
            S.append(np.sum(np.abs(ref["ct"]) * np.where(np.isfinite(l2), np.exp(l2 - la[i]), 0.0)))
    S = np.array(S)
    err = np.abs(el[:, 0] + 1j * el[:, 1] - el_ref)
    print(f"n={n} tables: max |dE_loc| = {err.max():.3e}, relative to S_i {np.max(err[:8] / S):.3e}")
    assert np.all(err[:8] <= 1e-10 * S) and err.max() <= 1e-10 * S.max()
    assert nqs.device_status(plan) == 0


def test_tables_match_term_list_at_60_qubits(nqs, ctx):
    """The benchmark's 60-qubit Hamiltonian and BF16-weight network on 256
    sector samples: local energies with tables equal those from the term list
    to 1e-9 (only h's rounding differs), energy and gradient likewise."""
    terms, params, _, _, cfg = config_inputs("c4")
    p = torch.from_numpy(params).cuda()
    xs = sector_samples(cfg["n"], cfg["n_up"], cfg["n_dn"], 256, seed=4)
    res = []
    for tables in (False, True):
        H = nqs.Hamiltonian.from_terms(terms, tables=tables).upload(ctx)
        plan = nqs.Plan(ctx, H, cfg["L"], cfg["h"], cfg["n_up"], cfg["n_dn"], cfg["precision"], max_batch=256)
        e, g, el = nqs.energy_grad(plan, p, xs)
        torch.cuda.synchronize()
        assert nqs.device_status(plan) == 0
        res.append((e.cpu().numpy(), g.cpu().numpy(), el.cpu().numpy()))
        del plan, H
    (e0, g0, l0), (e1, g1, l1) = res
    d = np.max(np.abs(l0 - l1))
    print(f"60 qubits: max |dE_loc| tables vs term list = {d:.3e}, |dE| = {abs(e0[0] - e1[0]):.3e}")
    assert d <= 1e-9 * max(1.0, np.max(np.abs(l0)))
    assert abs(e0[0] - e1[0]) <= 1e-9 * abs(e0[0])
    assert np.linalg.norm(g0 - g1) <= 1e-7 * np.linalg.norm(g0)
