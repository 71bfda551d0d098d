"""Oracle for the Marchenko block operator of Eq.5, FP64 (test infrastructure only).

    [Theta R f_d+]   [ I          -Theta R ] [f- ]
    [      0     ] = [ -Theta R*   I       ] [f_m+]

R applies the MDC of Eq.3 with the reflection kernel; R* applies it with the
complex-conjugated kernel (conjugation only, no transpose: a correlation in
time).  Theta is the time-space window that keeps, for each trace s and
virtual point v, the samples before the direct arrival.

Readings taken where the paper is silent:
  * Theta is a hard 0/1 window on the circular two-sided time axis:
    Theta[t, s, v] = 1 when |lag(t)| < onset[s, v], lag(t) = t for t < nt/2
    and t - nt otherwise; onsets arrive as integers so both sides agree.
  * The adjoint follows from the block structure with Theta real diagonal:
    M^H = [[I, -(R*)^H Theta], [-R^H Theta, I]].

Vectors are pairs (block0, block1), each of shape [nt, n, nv].
"""
from __future__ import annotations

import numpy as np

from .mdc import mdc_adjoint, mdc_forward


def lag_index(nt: int) -> np.ndarray:
    t = np.arange(nt)
    return np.where(t < nt / 2, t, t - nt)


def theta(nt: int, onset: np.ndarray) -> np.ndarray:
    """Theta[t, s, v] in {0, 1} from integer onsets [n, nv].

    onset >= 0: the two-sided Marchenko window |lag| < onset (Eq.5).  onset < 0: the
    one-sided window 0 <= lag < -onset, a causal time-domain preconditioner for the
    MDD unknown (Discussion section).
    """
    lag = lag_index(nt)[:, None, None]
    on = np.asarray(onset)[None, :, :]
    two = np.abs(lag) < on
    one = (lag >= 0) & (lag < -on)
    return np.where(on >= 0, two, one).astype(np.float64)


def forward(K: np.ndarray, onset: np.ndarray, fm: np.ndarray, fp: np.ndarray):
    """M [f-, f_m+] = (f- - Theta R f_m+,  -Theta R* f- + f_m+)."""
    th = theta(fm.shape[0], onset)
    o0 = fm - th * mdc_forward(K, fp)
    o1 = -th * mdc_forward(np.conj(K), fm) + fp
    return o0, o1


def adjoint(K: np.ndarray, onset: np.ndarray, d0: np.ndarray, d1: np.ndarray):
    """M^H [d0, d1] = (d0 - (R*)^H Theta d1,  -R^H Theta d0 + d1)."""
    th = theta(d0.shape[0], onset)
    i0 = d0 - mdc_adjoint(np.conj(K), th * d1)
    i1 = -mdc_adjoint(K, th * d0) + d1
    return i0, i1


def data(K: np.ndarray, onset: np.ndarray, fd_plus: np.ndarray):
    """Right-hand side d = (Theta R f_d+, 0)."""
    th = theta(fd_plus.shape[0], onset)
    return th * mdc_forward(K, fd_plus), np.zeros_like(fd_plus)


def neumann(K: np.ndarray, onset: np.ndarray, d0: np.ndarray, d1: np.ndarray,
            nterms: int):
    """Forward-only scheme: f = sum_{k<nterms} B^k d with B = I - M (needs rho(B) < 1)."""
    acc0, acc1 = d0.copy(), d1.copy()
    t0, t1 = d0.copy(), d1.copy()
    for _ in range(nterms - 1):
        m0, m1 = forward(K, onset, t0, t1)
        t0, t1 = t0 - m0, t1 - m1
        acc0 += t0
        acc1 += t1
    return acc0, acc1


def greens(K: np.ndarray, fm: np.ndarray, fplus: np.ndarray):
    """Eq.6: (-g-, g+*) = (f- - R f+, -R* f- + f+), returned as (g-, g+*)."""
    gm = -(fm - mdc_forward(K, fplus))
    gpc = -mdc_forward(np.conj(K), fm) + fplus
    return gm, gpc
