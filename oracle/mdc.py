"""Oracle for the MDC operator, FP64 (test infrastructure only).

Follows the Theory section: Eq.2 (frequency-domain form), Eq.3 (forward and
adjoint chains F^H I^H K I F and F^H I^H K^H I F), Eq.4 (one dense slice per
frequency) and the orthogonal real-FFT remark of the batch-matrix-multiply
section (1/sqrt(nt) both ways, positive frequencies only).

Readings taken where the paper is silent:
  * the convolution is circular of length nt (no implicit padding);
  * the inverse real transform discards the imaginary parts of the DC and
    Nyquist bins, which makes it exactly adjoint to the truncated forward
    transform in the weighted inner product; no separate time reversal is
    needed for the adjoint.

Layouts: time vectors x[t, r, v] (nt x n_R x n_A); spectra X[f, r, v]
(nfmax x n_R x n_A); kernel K[f, s, r] (nfmax x n_B x n_R), with the
integration weight dx_R already multiplied in.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(nt: int, nfmax: int, sign: float = -1.0) -> np.ndarray:
    """E[f, t] = exp(sign * 2 pi i ((f t) mod nt) / nt), f < nfmax, t < nt.

    The product f*t is reduced modulo nt before scaling so that every phase is
    an exact multiple of 2 pi / nt in [0, 2 pi).
    """
    f = np.arange(nfmax, dtype=np.int64)[:, None]
    t = np.arange(nt, dtype=np.int64)[None, :]
    ph = ((f * t) % nt).astype(np.float64) / nt
    return np.exp(sign * 2j * np.pi * ph)


def band_weights(nt: int, nfmax: int) -> np.ndarray:
    """c_f: 1 for the DC bin and (nt even) the Nyquist bin, 2 for every other bin."""
    c = np.full(nfmax, 2.0)
    c[0] = 1.0
    if nt % 2 == 0 and nfmax > nt // 2:
        c[nt // 2] = 1.0
    return c


def rfft_trunc(x: np.ndarray, nfmax: int) -> np.ndarray:
    """I_wmax F x: X[f, ...] = nt^-1/2 sum_t x[t, ...] exp(-2 pi i f t / nt), f < nfmax."""
    nt = x.shape[0]
    if not 1 <= nfmax <= nt // 2 + 1:
        raise ValueError("nfmax must lie in [1, nt//2 + 1]")
    E = dft_matrix(nt, nfmax, -1.0)
    X = E @ x.reshape(nt, -1).astype(np.float64)
    return (X / np.sqrt(nt)).reshape((nfmax,) + x.shape[1:])


def irfft_pad(X: np.ndarray, nt: int) -> np.ndarray:
    """F^H I^H X: y[t, ...] = nt^-1/2 sum_{f<nfmax} c_f Re(X[f, ...] exp(+2 pi i f t / nt))."""
    nfmax = X.shape[0]
    if not 1 <= nfmax <= nt // 2 + 1:
        raise ValueError("nfmax must lie in [1, nt//2 + 1]")
    Einv = dft_matrix(nt, nfmax, +1.0).T  # [t, f]
    c = band_weights(nt, nfmax)
    Z = (c[:, None] * X.reshape(nfmax, -1))
    y = np.real(Einv @ Z)
    return (y / np.sqrt(nt)).reshape((nt,) + X.shape[1:])


def kernel_apply(K: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Batch matrix multiply: Y[f] = K[f] @ X[f] for every frequency slice (Eq.4)."""
    nf, ns, nr = K.shape
    Xf = X.reshape(nf, nr, -1)
    Y = np.matmul(K, Xf)
    return Y.reshape((nf, ns) + X.shape[2:])


def kernel_apply_adjoint(K: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Transpose and complex conjugate per slice: X[f] = K[f]^H @ Y[f]."""
    nf, ns, nr = K.shape
    Yf = Y.reshape(nf, ns, -1)
    X = np.matmul(np.conj(np.transpose(K, (0, 2, 1))), Yf)
    return X.reshape((nf, nr) + Y.shape[2:])


def mdc_forward(K: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Eq.3 forward: g = F^H I^H K I F f, with x[t, r, (v)] -> y[t, s, (v)]."""
    nt = x.shape[0]
    nfmax = K.shape[0]
    return irfft_pad(kernel_apply(K, rfft_trunc(x, nfmax)), nt)


def mdc_adjoint(K: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Eq.3 adjoint: f = F^H I^H K^H I F g, with y[t, s, (v)] -> x[t, r, (v)]."""
    nt = y.shape[0]
    nfmax = K.shape[0]
    return irfft_pad(kernel_apply_adjoint(K, rfft_trunc(y, nfmax)), nt)


# ----------------------------------------------------------------------------
# Time-domain definition (Eq.1) as brute-force circular sums, for tiny inputs.
# ----------------------------------------------------------------------------
def conv_time(k: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y[t, s, v] = sum_r sum_tau k[(t - tau) mod nt, s, r] x[tau, r, v] (plain loops)."""
    nt, ns, nr = k.shape
    x3 = x.reshape(nt, nr, -1)
    y = np.zeros((nt, ns, x3.shape[2]))
    for t in range(nt):
        for tau in range(nt):
            y[t] += k[(t - tau) % nt] @ x3[tau]
    return y.reshape((nt, ns) + x.shape[2:])


def corr_time(k: np.ndarray, y: np.ndarray) -> np.ndarray:
    """x[tau, r, v] = sum_s sum_t k[(t - tau) mod nt, s, r] y[t, s, v] (plain loops)."""
    nt, ns, nr = k.shape
    y3 = y.reshape(nt, ns, -1)
    x = np.zeros((nt, nr, y3.shape[2]))
    for tau in range(nt):
        for t in range(nt):
            x[tau] += k[(t - tau) % nt].T @ y3[t]
    return x.reshape((nt, nr) + y.shape[2:])
