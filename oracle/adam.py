"""Adam update, FP64 CPU reference (Kingma and Ba, ICLR 2015, Algorithm 1;
the paper's optimiser, Sec. 6: learning rate 1e-3, betas (0.9, 0.99)).

Test infrastructure only: used by tests/ (not by the library).

For a step t >= 1 with gradient g:
  m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
  m_hat = m / (1 - b1^t),   v_hat = v / (1 - b2^t),
  theta <- theta - lr m_hat / (sqrt(v_hat) + eps).
The parameters are FP32 values; the update is formed in FP64 and the result
rounded to the nearest FP32 value.
"""
import numpy as np


def step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.99, eps=1e-8):
    """(theta' f32, m' f64, v' f64) after step t (t counts from 1)."""
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    upd = lr * m_hat / (np.sqrt(v_hat) + eps)
    theta = (np.asarray(theta, dtype=np.float32).astype(np.float64) - upd).astype(np.float32)
    return theta, m, v
