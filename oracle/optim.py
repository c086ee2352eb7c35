"""Adam in float64 (test infrastructure only): the update the fine-tuning step
applies to every parameter (Kingma and Ba's algorithm with bias correction)."""
from __future__ import annotations

import numpy as np


def adam(p, grads, lr, b1=0.9, b2=0.999, eps=1e-15):
    """Applies the gradients of successive steps; returns (p, m, v)."""
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t, g in enumerate(grads, start=1):
        g = np.asarray(g, dtype=np.float64)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v
