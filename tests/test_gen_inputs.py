"""Host checks of the seeded input generator (no GPU)."""
import numpy as np
import torch

from gen import CONFIGS, config_inputs, init_params, param_count, round_bf16


def test_round_bf16_is_torch_bfloat16_rne():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(20000).astype(np.float32) * s for s in (1e-3, 0.1, 10.0)])
    # exact ties: low half-word 0x8000 rounds to the even neighbour
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    a = np.concatenate([a, ties, -ties])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(round_bf16(a), ref)
    assert np.array_equal(round_bf16(ref), ref)        # BF16 values are fixed points


def test_bf16_parameters_are_bf16_values():
    p = init_params(12, 2, 64, seed=3, dtype="bf16")
    assert p.dtype == np.float32 and p.size == param_count(12, 2, 64)
    assert np.all((p.view(np.uint32) & 0xFFFF) == 0)
    q = init_params(12, 2, 64, seed=3)
    assert np.array_equal(round_bf16(q), p)


def test_config_parameter_kinds():
    for name, cfg in CONFIGS.items():
        assert cfg["params"] == ("bf16" if cfg["precision"] == "bf16w" else "fp32"), name
    terms, params, xs, w, cfg = config_inputs("c1", batch=64)
    assert params.size == param_count(cfg["n"], cfg["L"], cfg["h"])
    assert len(xs) == 64 and np.all(w == 1.0)
