"""Spectral norm of a dense complex matrix by power iteration on K^H K (FP64).

Used only to choose the synthetic reflection kernel's scale so that the
Marchenko operator of Eq.5 is well conditioned (sigma(M) within [1-q, 1+q]
when ||K_f||_2 <= q for every slice).  Test/setup infrastructure only.
"""
from __future__ import annotations

import numpy as np


def spectral_norm(K: np.ndarray, iters: int = 60, seed: int = 0) -> float:
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(K.shape[1]) + 1j * rng.standard_normal(K.shape[1])
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = K.conj().T @ (K @ v)
        lam = np.linalg.norm(w)
        v = w / lam
    return float(np.sqrt(lam))
