"""Pins for the FP64 MDC oracle (CPU).

Each test checks the oracle against something other than itself: numpy's FFT
(a library routine the oracle does not use), brute-force circular sums of the
time-domain definition (Eq.1), closed forms (delta and shift kernels, the
Ricker spectrum), and invariants (adjointness, Parseval, idempotence).
A dropped c_f weight, a wrong exponent sign, a missing conjugate or a
transposed kernel each fail at least one of them.
"""
import numpy as np
import pytest

from oracle import mdc as om
from paper_2011_11120_amd import synth


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("nt", [8, 9, 64, 63, 512])
def test_rfft_trunc_matches_numpy_rfft(nt):
    x = synth.gaussian((nt, 5, 3))
    ref = np.fft.rfft(x, axis=0, norm="ortho")
    for nfmax in (1, nt // 3 + 1, nt // 2 + 1):
        got = om.rfft_trunc(x, nfmax)
        assert got.shape == (nfmax, 5, 3)
        assert rel(got, ref[:nfmax]) < 1e-13


@pytest.mark.parametrize("nt", [8, 9, 64, 63, 512])
def test_irfft_pad_matches_numpy_irfft(nt):
    nf_full = nt // 2 + 1
    for nfmax in (1, nt // 3 + 1, nf_full):
        X = synth.gaussian((nfmax, 4, 2)) + 1j * synth.gaussian((nfmax, 4, 2), seed=5)
        Xp = np.zeros((nf_full, 4, 2), dtype=complex)
        Xp[:nfmax] = X
        ref = np.fft.irfft(Xp, n=nt, axis=0, norm="ortho")
        assert rel(om.irfft_pad(X, nt), ref) < 1e-13


def test_band_weights():
    assert list(om.band_weights(8, 5)) == [1, 2, 2, 2, 1]
    assert list(om.band_weights(9, 5)) == [1, 2, 2, 2, 2]
    assert list(om.band_weights(8, 3)) == [1, 2, 2]


def test_round_trip_full_band_is_identity():
    for nt in (16, 17):
        x = synth.gaussian((nt, 6))
        assert rel(om.irfft_pad(om.rfft_trunc(x, nt // 2 + 1), nt), x) < 1e-14


def test_parseval_full_band():
    nt = 64
    x = synth.gaussian((nt, 7))
    X = om.rfft_trunc(x, nt // 2 + 1)
    c = om.band_weights(nt, nt // 2 + 1)
    assert abs(np.sum(x * x) - np.sum(c[:, None] * np.abs(X) ** 2)) < 1e-11 * np.sum(x * x)


def _c1(nfmax=33, nx_r=None):
    """c1-shaped problem: nt = 64, dt = 4 ms, 8x8 grid, dx = 20 m, 3 events per trace."""
    nt, dt, dx = 64, 0.004, 20.0
    G = synth.c1_time_kernel(nt=nt, nx=8, dt=dt, dx=dx, nx_r=nx_r)
    k = dt * dx * dx * G  # weighted time kernel: integral over tau and x_R (Eq.1)
    # Kernel preprocessing (time -> frequency) through numpy's FFT, not the oracle's DFT.
    K = np.fft.rfft(k, axis=0)[:nfmax]
    return nt, k, K


def _band_limit(k, nfmax):
    nt = k.shape[0]
    Kf = np.fft.rfft(k, axis=0)
    Kf[nfmax:] = 0
    return np.fft.irfft(Kf, n=nt, axis=0)


def test_forward_equals_bruteforce_convolution_full_band():
    nt, k, K = _c1()
    x = synth.ricker_spikes(nt, 64, 1)
    y = om.mdc_forward(K, x)
    assert rel(y, om.conv_time(k, x)) < 1e-12


def test_adjoint_equals_bruteforce_correlation_full_band():
    nt, k, K = _c1()
    y = synth.gaussian((nt, 64, 1))
    x = om.mdc_adjoint(K, y)
    assert rel(x, om.corr_time(k, y)) < 1e-12


def test_forward_adjoint_bruteforce_truncated_band():
    nfmax = 20
    nt, k, K = _c1(nfmax)
    kL = _band_limit(k, nfmax)
    x = synth.ricker_spikes(nt, 64, 2)
    y = synth.gaussian((nt, 64, 2))
    assert rel(om.mdc_forward(K, x), om.conv_time(kL, x)) < 1e-12
    assert rel(om.mdc_adjoint(K, y), om.corr_time(kL, y)) < 1e-12


def test_rectangular_kernel_bruteforce():
    """ns != nr: a transposed kernel cannot even be applied."""
    nt, dt, dx = 32, 0.004, 20.0
    G = synth.c1_time_kernel(nt=nt, nx=3, nx_r=4, dt=dt, dx=dx)  # ns = 9, nr = 16
    k = dt * dx * dx * G
    K = np.fft.rfft(k, axis=0)
    x = synth.gaussian((nt, 16, 2))
    y = synth.gaussian((nt, 9, 2), seed=7)
    assert rel(om.mdc_forward(K, x), om.conv_time(k, x)) < 1e-12
    assert rel(om.mdc_adjoint(K, y), om.corr_time(k, y)) < 1e-12


@pytest.mark.parametrize("nt", [64, 63])
def test_delta_kernel_is_identity_or_projector(nt):
    n = 5
    x = synth.gaussian((nt, n, 2))
    full = nt // 2 + 1
    K = np.broadcast_to(np.eye(n), (full, n, n)).astype(complex)
    assert rel(om.mdc_forward(K, x), x) < 1e-13
    assert rel(om.mdc_adjoint(K, x), x) < 1e-13
    nf = full // 2
    P = om.mdc_forward(K[:nf], x)
    assert rel(om.mdc_forward(K[:nf], P), P) < 1e-13  # idempotent band-limit projector
    assert rel(P, x) > 0.1


def test_shift_kernel_is_circular_shift():
    nt, n, t0 = 64, 4, 5
    f = np.arange(nt // 2 + 1)
    K = np.exp(-2j * np.pi * f * t0 / nt)[:, None, None] * np.eye(n)[None]
    x = synth.gaussian((nt, n))
    assert rel(om.mdc_forward(K, x), np.roll(x, t0, axis=0)) < 1e-13
    assert rel(om.mdc_adjoint(K, x), np.roll(x, -t0, axis=0)) < 1e-13


@pytest.mark.parametrize("nt,nfmax", [(64, 33), (64, 20), (63, 17), (512, 150)])
def test_dot_product_adjoint(nt, nfmax):
    ns, nr, nv = 7, 11, 3
    K = synth.random_complex_kernel(nfmax, ns, nr)
    x = synth.gaussian((nt, nr, nv))
    y = synth.gaussian((nt, ns, nv), seed=9)
    lhs = np.vdot(om.mdc_forward(K, x), y)
    rhs = np.vdot(x, om.mdc_adjoint(K, y))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_conjugate_kernel_is_correlation():
    """R* (conjugated kernel, no transpose) equals convolution with the time-reversed kernel."""
    nt, k, K = _c1()
    k_rev = np.roll(k[::-1], 1, axis=0)  # k[(-t) mod nt]
    x = synth.ricker_spikes(nt, 64, 1)
    assert rel(om.mdc_forward(np.conj(K), x), om.conv_time(k_rev, x)) < 1e-12


def test_columns_are_independent():
    nt, nfmax, n = 64, 20, 6
    K = synth.random_complex_kernel(nfmax, n, n)
    x = synth.gaussian((nt, n, 4))
    Y = om.mdc_forward(K, x)
    for v in range(4):
        assert rel(om.mdc_forward(K, x[:, :, v]), Y[:, :, v]) < 1e-14


def test_ricker_closed_form_spectrum_matches_sampled_dft():
    """Ricker spectrum used by the frequency-domain kernel generator vs DFT of samples."""
    nt, dt, fp, t0 = 1024, 0.004, 15.0, 1.0
    t = np.arange(nt) * dt
    w = synth.ricker(t - t0, fp)
    f = np.arange(nt // 2 + 1) / (nt * dt)
    Wd = dt * np.fft.rfft(w)
    Wc = synth.ricker_spectrum(f, fp) * np.exp(-2j * np.pi * f * t0)
    assert np.max(np.abs(Wd - Wc)) < 1e-12 * np.max(np.abs(Wc))


def test_frequency_kernel_matches_dft_of_time_traces():
    """Closed-form K equals dt*dA*DFT of the sampled hyperbolic-event traces (noise off)."""
    spec = synth.KernelSpec(nt=512, nfmax=150, nx=3, noise=0.0)
    K = synth.kernel_full(spec)
    gx, gy = synth.grid_xy(3, 3, spec.dx)
    tau = synth.event_times(spec.events, gx, gy, gx, gy)
    t = np.arange(spec.nt) * spec.dt
    G = np.einsum("k,tksr->tsr", spec.events.amp, synth.ricker(t[:, None, None, None] - tau[None], spec.fp))
    Kt = spec.dt * spec.dA * np.fft.rfft(G, axis=0)[:150]
    assert rel(K, Kt) < 1e-9
