"""GPU Adam step (nqs_adam_step) against the FP64 Adam oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import adam

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


# 3,276,864 = the parameter count of the 60-qubit, L = 4, h = 1,024 network
@pytest.mark.parametrize("n", [1, 1000, 65537, 3276864])
def test_adam_matches_oracle(nqs, ctx, n):
    rng = np.random.default_rng(n)
    th = (rng.standard_normal(n) * 0.1).astype(np.float32)
    p = torch.from_numpy(th.copy()).cuda()
    opt = nqs.Adam(ctx, p, lr=1e-3, betas=(0.9, 0.99), eps=1e-8)
    m = np.zeros(n)
    v = np.zeros(n)
    for t in range(1, 4):
        g = rng.standard_normal(n) * 10.0 ** rng.integers(-6, 2, n)
        if n > 10:
            g[:3] = 0.0                        # zero gradient: no move at step 1
        opt.step(torch.from_numpy(g).cuda())
        th, m, v = adam.step(th, g, m, v, t)
        torch.cuda.synchronize()
        mg, vg, pg = opt.m.cpu().numpy(), opt.v.cpu().numpy(), p.cpu().numpy()
        assert np.array_equal(mg, m) and np.array_equal(vg, v), t
        ulps = np.abs(pg.view(np.int32).astype(np.int64) - th.view(np.int32).astype(np.int64))
        print(f"n={n} t={t}: params differing from the oracle: {np.count_nonzero(ulps)}, max {ulps.max()} ulp")
        assert ulps.max() <= 1
        th = pg.copy()                          # continue both from the same parameters


def test_adam_empty_and_bad_arguments(nqs, ctx):
    import ctypes as C
    lib = ctx.lib
    z = C.c_void_p(0)
    assert lib.nqs_adam_step(ctx.handle, 0, z, z, z, z, 1, 1e-3, 0.9, 0.99, 1e-8) == 0   # nothing to do
    p = torch.zeros(4, device="cuda")
    g = torch.zeros(4, dtype=torch.float64, device="cuda")
    ptr = lambda t: C.c_void_p(t.data_ptr())
    m, v = torch.zeros_like(g), torch.zeros_like(g)
    for step, lr, b1, b2, eps in ((0, 1e-3, 0.9, 0.99, 1e-8), (1, -1.0, 0.9, 0.99, 1e-8),
                                  (1, 1e-3, 1.0, 0.99, 1e-8), (1, 1e-3, 0.9, -0.1, 1e-8),
                                  (1, 1e-3, 0.9, 0.99, float("nan"))):
        assert lib.nqs_adam_step(ctx.handle, 4, ptr(p), ptr(g), ptr(m), ptr(v), step, lr, b1, b2, eps) == 1
    assert lib.nqs_adam_step(ctx.handle, 4, z, ptr(g), ptr(m), ptr(v), 1, 1e-3, 0.9, 0.99, 1e-8) == 1
