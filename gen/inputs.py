"""Workload recipes: Hamiltonians, parameters, samples and weights.

The parameter layout is the library's flat FP32 layout: for each hidden layer
l = 1..L the weight W_l (row-major [h][in_l], in_1 = n, else h) then its bias
b_l [h]; then the conditional head W_o [n][h], b_o [n]; then the phase head
W_phi [4][h], b_phi [4]; with a separate phase network (phase_mode 1) its
layers V_1 [h][n-2], e_1 [h], ..., V_L [h][h], e_L [h] sit between the
conditional head and W_phi.  All entries are drawn i.i.d. N(0, 0.1^2) in float32;
for the workloads whose network is BF16, every entry is then rounded to the
nearest BF16 value (the parameters of that network are BF16 values, held in
float32 storage).

Samples are bit strings packed into uint64 (bit j = qubit j), drawn uniformly
from the (n_up, n_dn) spin sector: up electrons on even qubits, down electrons
on odd qubits.
"""
from functools import lru_cache

import numpy as np

from .integrals import molecular_integrals
from .jw import jordan_wigner_terms, PauliTerms


@lru_cache(maxsize=8)
def _hamiltonian_cached(n_orb, seed, drop_tol, cutoff):
    h1, h2 = molecular_integrals(n_orb, seed)
    if cutoff > 0.0:
        h2 = np.where(np.abs(h2) >= cutoff, h2, 0.0)
    return jordan_wigner_terms(h1, h2, drop_tol=drop_tol)


def hamiltonian(n_orb: int, seed: int = 0, drop_tol: float = 1e-10, cutoff: float = 0.0) -> PauliTerms:
    """Merged Pauli-string Hamiltonian on ``2*n_orb`` qubits (cached per process).

    ``cutoff`` > 0 zeroes the two-electron integrals of magnitude below it
    before the expansion (a sparser synthetic molecule with fewer terms; the
    8-fold symmetry is kept, since symmetric entries are equal).
    """
    return _hamiltonian_cached(int(n_orb), int(seed), float(drop_tol), float(cutoff))


def words(n: int) -> int:
    """64-bit words per bit string of n qubits."""
    return (int(n) + 63) // 64


def param_count(n: int, n_layers: int, width: int, phase_mode: int = 0) -> int:
    h = width
    total = h * n + h
    total += (n_layers - 1) * (h * h + h)
    total += n * h + n
    total += 4 * h + 4
    if phase_mode == 1:             # separate phase network: V_1 [h][n-2], e_1, then (L-1) x [h][h], [h]
        total += h * (n - 2) + h + (n_layers - 1) * (h * h + h)
    return total


def round_bf16(a):
    """Nearest BF16 values (ties to even) of a float32 array, as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def init_params(n: int, n_layers: int, width: int, seed: int = 1, std: float = 0.1, dtype: str = "fp32",
                phase_mode: int = 0):
    """N(0, std^2) parameters in float32; dtype "bf16" rounds them to BF16 values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = (std * rng.standard_normal(param_count(n, n_layers, width, phase_mode))).astype(np.float32)
    if dtype == "bf16":
        p = round_bf16(p)
    elif dtype != "fp32":
        raise ValueError(f"unknown parameter dtype {dtype}")
    return p


def sector_samples(n: int, n_up: int, n_dn: int, count: int, seed: int = 2):
    """``count`` i.i.d. uniform draws from the (n_up, n_dn) sector.

    uint64 [count] for n <= 64, else uint64 [count, W] words (word w holds
    qubits 64w .. 64w+63)."""
    N = n // 2
    if not (0 <= n_up <= N and 0 <= n_dn <= N):
        raise ValueError("sector outside the orbital range")
    W = words(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((count, W), dtype=np.uint64)
    for spin, ne in ((0, n_up), (1, n_dn)):
        if ne == 0:
            continue
        keys = rng.random((count, N))
        chosen = np.argsort(keys, axis=1)[:, :ne]          # uniform ne-subset
        qubits = 2 * chosen + spin
        for w in range(W):
            inw = (qubits >= 64 * w) & (qubits < 64 * (w + 1))
            bits = np.where(inw, np.left_shift(np.uint64(1), (qubits - 64 * w).clip(0, 63).astype(np.uint64)),
                            np.uint64(0))
            out[:, w] |= np.bitwise_or.reduce(bits, axis=1)
    return out[:, 0].copy() if W == 1 else out


def unique_with_counts(samples):
    """Distinct samples in ascending order (as unsigned integers) and their counts."""
    a = np.asarray(samples, dtype=np.uint64)
    if a.ndim == 1:
        u, c = np.unique(a, return_counts=True)
        return u, c.astype(np.float64)
    u, c = np.unique(a[:, ::-1], axis=0, return_counts=True)   # most significant word first
    return np.ascontiguousarray(u[:, ::-1]), c.astype(np.float64)


# The five workloads: spatial orbitals N (n = 2N qubits, half filling),
# integral seed, batch, hidden layers L, width h, arithmetic of the path,
# parameter values (FP32, or BF16 for the BF16 networks).
CONFIGS = {
    "c1": dict(N=6, seed=0, B=1024, L=1, h=64, precision="fp64", dedup=True,
               weights="ones", params="fp32"),
    "c2": dict(N=12, seed=0, B=8192, L=2, h=256, precision="fp32", dedup=False,
               weights="counts", params="fp32"),
    "c3": dict(N=20, seed=0, B=32768, L=3, h=512, precision="bf16w", dedup=True,
               weights="counts", params="bf16"),
    "c4": dict(N=30, seed=0, B=65536, L=4, h=1024, precision="bf16w", dedup="auto",
               weights="counts", params="bf16"),
    "c5a": dict(N=8, seed=1, B=4096, L=3, h=512, precision="bf16w", dedup=True,
                weights="counts", params="bf16"),
    "c5b": dict(N=14, seed=2, B=16384, L=3, h=512, precision="bf16w", dedup=False,
                weights="counts", params="bf16"),
    "c5c": dict(N=22, seed=3, B=32768, L=3, h=512, precision="bf16w", dedup=False,
                weights="counts", params="bf16"),
    "c5d": dict(N=32, seed=4, B=16384, L=3, h=512, precision="bf16w", dedup=False,
                weights="counts", params="bf16"),
}


def config_inputs(name: str, batch: int = None, sample_seed: int = 2, param_seed: int = 1):
    """(PauliTerms, params f32, samples u64, weights f64, cfg) for a workload."""
    cfg = dict(CONFIGS[name])
    N = cfg["N"]
    n = 2 * N
    ham = hamiltonian(N, cfg["seed"])
    B = cfg["B"] if batch is None else int(batch)
    params = init_params(n, cfg["L"], cfg["h"], seed=param_seed, dtype=cfg["params"])
    raw = sector_samples(n, N // 2, N // 2, B, seed=sample_seed)
    if cfg["weights"] == "counts":
        samples, weights = unique_with_counts(raw)
    else:
        samples, weights = raw, np.ones(B, dtype=np.float64)
    cfg["n"] = n
    cfg["n_up"] = N // 2
    cfg["n_dn"] = N // 2
    return ham, params, samples, weights, cfg
