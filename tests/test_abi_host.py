"""Host-side checks of the C ABI (no GPU needed): exported symbols, the
Hamiltonian canonicalisation against the oracle (bit-exact), parameter
layout, error statuses."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import pauli, made
from gen import molecular_integrals, jordan_wigner_terms, param_count as gen_param_count

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2208_05637_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libnqs.so not built: run python -m paper_2208_05637_amd.build")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    header = open(os.path.join(ROOT, "include", "nqs.h")).read()
    names = set(re.findall(r"\b(nqs_[a-z_0-9]+)\s*\(", header))
    assert len(names) >= 20
    for name in sorted(names):
        assert hasattr(lib, name), name
    from paper_2208_05637_amd import _lib
    assert names == set(_lib.SIGNATURES)


def _ham(n, x, z, c, ci=None, tol=1e-10, flags=1):
    from paper_2208_05637_amd import Hamiltonian
    return Hamiltonian(n, x, z, c, coeff_imag=ci, drop_tol=tol, conserves_spin=bool(flags))


@pytest.mark.parametrize("N", [3, 6, 12])
def test_canonical_tensor_bit_exact_vs_oracle(lib, N):
    h1, h2 = molecular_integrals(N, seed=0)
    t = jordan_wigner_terms(h1, h2, drop_tol=0.0)
    # shuffle and split coefficients so the merge step has real work
    rng = np.random.default_rng(N)
    perm = rng.permutation(len(t))
    x = np.concatenate([t.x_mask[perm], t.x_mask[perm[: len(perm) // 3]]])
    z = np.concatenate([t.z_mask[perm], t.z_mask[perm[: len(perm) // 3]]])
    c = np.concatenate([t.coeff[perm], 0.25 * t.coeff[perm[: len(perm) // 3]]])
    ref = pauli.canonical_terms(x, z, c)
    gx, goff = pauli.groups(ref)
    H = _ham(2 * N, x, z, c)
    ex = H.export()
    assert H.K == len(ref["x"]) and H.G == len(gx) and not H.has_imag
    np.testing.assert_array_equal(ex["gx"], gx)
    np.testing.assert_array_equal(ex["goff"], goff)
    np.testing.assert_array_equal(ex["tz"], ref["z"])
    assert np.array_equal(ex["tre"], ref["ct"].real)      # bit-exact, same merge order
    assert np.array_equal(ex["tim"], ref["ct"].imag)


def _words_to_ints(a):
    return [int(r[0]) | (int(r[1]) << 64) for r in np.asarray(a).tolist()]


@pytest.mark.parametrize("cutoff", [0.05])
def test_two_word_canonical_tensor_bit_exact_vs_oracle(lib, cutoff):
    """76 qubits: masks of two words, merged, folded, sorted as 128-bit
    unsigned integers and grouped exactly as the oracle does with Python
    integers."""
    from gen.inputs import hamiltonian
    t = hamiltonian(38, 0, cutoff=cutoff)
    rng = np.random.default_rng(76)
    perm = rng.permutation(len(t))
    x = np.concatenate([t.x_mask[perm], t.x_mask[perm[: len(perm) // 3]]])
    z = np.concatenate([t.z_mask[perm], t.z_mask[perm[: len(perm) // 3]]])
    c = np.concatenate([t.coeff[perm], 0.25 * t.coeff[perm[: len(perm) // 3]]])
    ref = pauli.canonical_terms(x, z, c)
    assert ref["x"].dtype == object
    gx, goff = pauli.groups(ref)
    H = _ham(76, x, z, c)
    ex = H.export()
    assert H.K == len(ref["x"]) and H.G == len(gx)
    assert ex["gx"].shape == (H.G, 2) and ex["tz"].shape == (H.K, 2)
    assert _words_to_ints(ex["gx"]) == [int(v) for v in gx]
    np.testing.assert_array_equal(ex["goff"], goff)
    assert _words_to_ints(ex["tz"]) == [int(v) for v in ref["z"]]
    assert np.array_equal(ex["tre"], ref["ct"].real)
    assert np.array_equal(ex["tim"], ref["ct"].imag)
    assert any(int(v) >> 64 for v in gx) and H.G > 1000


def test_two_word_odd_y_fold(lib):
    """A Y on qubit 100 and one on qubit 3: (-i)^2 = -1; a lone Y on qubit 70: -i."""
    x = np.array([[1 << 3, 1 << 36], [0, 1 << 6]], dtype=np.uint64)
    z = np.array([[1 << 3, 1 << 36], [0, 1 << 6]], dtype=np.uint64)
    c = np.array([0.5, 0.25])
    H = _ham(101, x, z, c)
    ref = pauli.canonical_terms(x, z, c)
    ex = H.export()
    assert H.has_imag
    assert np.array_equal(ex["tre"], ref["ct"].real) and np.array_equal(ex["tim"], ref["ct"].imag)
    assert sorted(ref["ct"].tolist(), key=abs) == [-0.25j, -0.5 + 0j]


def test_odd_y_terms_fold_into_imaginary_plane(lib):
    x = np.array([0b10, 0b11, 0b1], dtype=np.uint64)
    z = np.array([0b10, 0b01, 0b1], dtype=np.uint64)
    c = np.array([0.5, 0.25, -2.0])
    H = _ham(2, x, z, c)
    ref = pauli.canonical_terms(x, z, c)
    ex = H.export()
    assert H.has_imag
    assert np.array_equal(ex["tre"], ref["ct"].real)
    assert np.array_equal(ex["tim"], ref["ct"].imag)


def test_error_statuses(lib):
    from paper_2208_05637_amd import NQSError
    with pytest.raises(NQSError) as e:
        _ham(3, [1], [0], [1.0], ci=[1e-3])
    assert e.value.status == 3            # NQS_ERR_NOT_HERMITIAN
    with pytest.raises(NQSError) as e:
        _ham(129, np.array([[1, 0, 0]], dtype=np.uint64), np.zeros((1, 3), dtype=np.uint64), [1.0])
    assert e.value.status == 2            # NQS_ERR_UNSUPPORTED
    with pytest.raises(NQSError) as e:   # acts on qubit 70 of a 70-qubit system
        _ham(70, np.array([[0, 1 << 6]], dtype=np.uint64), np.zeros((1, 2), dtype=np.uint64), [1.0])
    assert e.value.status == 1
    with pytest.raises(ValueError):       # 70 qubits take two words per mask
        _ham(70, [1], [0], [1.0])
    with pytest.raises(NQSError) as e:
        _ham(3, [8], [0], [1.0])          # acts on qubit 3 of a 3-qubit system
    assert e.value.status == 1
    with pytest.raises(NQSError):
        _ham(3, [1], [0], [float("nan")])


@pytest.mark.parametrize("n,L,h,prec,mode", [(12, 1, 64, "fp64", 0), (24, 2, 256, "fp32", 0),
                                             (60, 4, 1024, "bf16", 0), (64, 3, 512, "bf16x3", 0),
                                             (12, 1, 64, "fp64", 1), (60, 4, 1024, "bf16w", 1)])
def test_param_layout(lib, n, L, h, prec, mode):
    from paper_2208_05637_amd import param_count
    want = made.n_params(made.Net(n=n, n_layers=L, width=h, phase_mode=mode))
    assert param_count(n, L, h, prec, phase_mode=mode) == want == gen_param_count(n, L, h, mode)


def test_phase_mode_rejected_values(lib):
    from paper_2208_05637_amd import param_count, NQSError
    with pytest.raises(NQSError):
        param_count(12, 1, 64, "fp64", phase_mode=2)
    with pytest.raises(NQSError):
        param_count(2, 1, 64, "fp64", phase_mode=1)     # no first n-2 entries


def test_unsupported_width_rejected(lib):
    from paper_2208_05637_amd import param_count, NQSError
    with pytest.raises(NQSError):
        param_count(12, 1, 100, "bf16")
    # above 64 qubits the 256-row tiles of BF16 at width 256 and FP32 at width
    # 128 leave no LDS for the head of 132 outputs
    for prec, h in (("bf16", 256), ("fp32", 128)):
        assert param_count(64, 1, h, prec) > 0
        with pytest.raises(NQSError):
            param_count(65, 1, h, prec)
    with pytest.raises(NQSError):
        param_count(129, 1, 64, "fp64")


@pytest.mark.parametrize("n,L,h,prec,mode", [(76, 3, 512, "bf16w", 0), (65, 1, 64, "fp64", 0),
                                             (128, 2, 256, "fp32", 1), (100, 2, 512, "bf16", 0)])
def test_param_layout_above_64_qubits(lib, n, L, h, prec, mode):
    from paper_2208_05637_amd import param_count
    want = made.n_params(made.Net(n=n, n_layers=L, width=h, phase_mode=mode))
    assert param_count(n, L, h, prec, phase_mode=mode) == want == gen_param_count(n, L, h, mode)


def test_adam_rejects_arguments_on_the_host(lib):
    import ctypes as C
    z = C.c_void_p(0)
    assert lib.nqs_adam_step(z, 0, z, z, z, z, 1, 1e-3, 0.9, 0.99, 1e-8) == 1     # NULL context


def test_binding_rejects_tensors_the_kernels_would_overrun():
    import torch
    from paper_2208_05637_amd.api import _dev_tensor
    ok = torch.zeros(6, dtype=torch.float64)
    assert _dev_tensor(ok, "eloc", torch.float64, 6, "cpu") is ok
    for bad, why in ((torch.zeros(5, dtype=torch.float64), "short"),
                     (torch.zeros(6, dtype=torch.float32), "dtype"),
                     (torch.zeros(12, dtype=torch.float64)[::2], "strided")):
        with pytest.raises(ValueError):
            _dev_tensor(bad, why, torch.float64, 6, "cpu")
