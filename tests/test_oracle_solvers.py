"""Pins for the LSQR / CGLS / Marchenko / Neumann oracles (CPU).

LSQR is checked against scipy.sparse.linalg.lsqr (same algorithm, independent
code) iterate by iterate, against numpy.linalg.lstsq once converged, and
against CGLS (identical iterates in exact arithmetic).  The Marchenko block
operator of Eq.5 is checked against a dense matrix assembled entry by entry
from time-domain convolution and correlation matrices, by its dot-product
test, by K = 0 giving M = I, and by the forward-only Neumann series reaching
the least-squares solution when ||Theta R|| < 1.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import lsqr as ol
from oracle import marchenko as om
from oracle import mdc as omdc
from paper_2011_11120_amd import synth


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def _dense_problem(m=40, n=25, seed=3):
    A = synth.gaussian((m, n), seed=seed)
    b = synth.gaussian((m,), seed=seed + 1)
    return A, b


@pytest.mark.parametrize("niter", [1, 3, 7, 15])
def test_lsqr_matches_scipy_iterates(niter):
    A, b = _dense_problem()
    x, _ = ol.lsqr(lambda v: [A @ v[0]], lambda u: [A.T @ u[0]], [b], niter)
    ref = spla.lsqr(A, b, damp=0.0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=niter)[0]
    assert rel(x[0], ref) < 1e-12


def test_lsqr_converges_to_lstsq():
    A, b = _dense_problem(30, 12)
    x, hist = ol.lsqr(lambda v: [A @ v[0]], lambda u: [A.T @ u[0]], [b], 40)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    assert rel(x[0], ref) < 1e-10
    assert abs(hist[-1] - np.linalg.norm(A @ ref - b)) < 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("niter", [1, 4, 10])
def test_lsqr_equals_cgls(niter):
    A, b = _dense_problem(60, 25, seed=11)
    xl, _ = ol.lsqr(lambda v: [A @ v[0]], lambda u: [A.T @ u[0]], [b], niter)
    xc, _ = ol.cgls(lambda v: [A @ v[0]], lambda u: [A.T @ u[0]], [b], niter)
    assert rel(xl[0], xc[0]) < 1e-10


def _conv_matrix(k):
    """Dense matrix of x -> conv_time(k, x) for one virtual point, built entry by entry."""
    nt, ns, nr = k.shape
    M = np.zeros((nt * ns, nt * nr))
    for t in range(nt):
        for tau in range(nt):
            M[t * ns:(t + 1) * ns, tau * nr:(tau + 1) * nr] = k[(t - tau) % nt]
    return M


def _marchenko_case(nt=16, nx=2, nv=1, scale=1.0):
    dt, dx = 0.004, 20.0
    G = synth.c1_time_kernel(nt=nt, nx=nx, dt=dt, dx=dx)
    k = scale * dt * dx * dx * G / np.abs(G).max()
    K = np.fft.rfft(k, axis=0)
    n = nx * nx
    onset = (3 + np.arange(n * nv) % 4).reshape(n, nv).astype(np.int32)
    return k, K, onset


def test_marchenko_matches_dense_block_matrix():
    nt = 16
    k, K, onset = _marchenko_case(nt)
    n = k.shape[1]
    R = _conv_matrix(k)
    k_rev = np.roll(k[::-1], 1, axis=0)  # R*: correlation = convolution with k(-t)
    Rs = _conv_matrix(k_rev)
    th = np.diag(om.theta(nt, onset)[:, :, 0].ravel())
    I = np.eye(nt * n)
    M = np.block([[I, -th @ R], [-th @ Rs, I]])
    fm = synth.gaussian((nt, n, 1))
    fp = synth.gaussian((nt, n, 1), seed=4)
    o0, o1 = om.forward(K, onset, fm, fp)
    ref = M @ np.concatenate([fm.ravel(), fp.ravel()])
    assert rel(np.concatenate([o0.ravel(), o1.ravel()]), ref) < 1e-12
    i0, i1 = om.adjoint(K, onset, fm, fp)
    refa = M.T @ np.concatenate([fm.ravel(), fp.ravel()])
    assert rel(np.concatenate([i0.ravel(), i1.ravel()]), refa) < 1e-12


def test_marchenko_dot_product():
    nt = 64
    k, K, onset = _marchenko_case(nt, nx=3, nv=2)
    K = K[:20]
    n = 9
    a = [synth.gaussian((nt, n, 2), seed=s) for s in (1, 2)]
    b = [synth.gaussian((nt, n, 2), seed=s) for s in (3, 4)]
    Ma = om.forward(K, onset, *a)
    MHb = om.adjoint(K, onset, *b)
    lhs = sum(np.vdot(p, q) for p, q in zip(Ma, b))
    rhs = sum(np.vdot(p, q) for p, q in zip(a, MHb))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_marchenko_zero_kernel_is_identity():
    nt, n = 32, 4
    K = np.zeros((10, n, n), dtype=complex)
    onset = np.full((n, 1), 5, dtype=np.int32)
    d = [synth.gaussian((nt, n, 1), seed=s) for s in (1, 2)]
    x, hist = ol.lsqr(lambda v: list(om.forward(K, onset, *v)),
                      lambda u: list(om.adjoint(K, onset, *u)), d, 1)
    assert rel(x[0], d[0]) < 1e-14 and rel(x[1], d[1]) < 1e-14
    assert hist[-1] < 1e-12


def test_neumann_series_equals_lsqr_solution():
    nt = 32
    k, K, onset = _marchenko_case(nt, nx=2, nv=1)
    n = 4
    K = K / max(np.linalg.norm(K[f], 2) for f in range(K.shape[0])) * 0.5
    fd = synth.ricker_spikes(nt, n, 1)
    d = list(om.data(K, onset, fd))
    xn = om.neumann(K, onset, *d, nterms=60)
    xl, _ = ol.lsqr(lambda v: list(om.forward(K, onset, *v)),
                    lambda u: list(om.adjoint(K, onset, *u)), d, 60)
    assert rel(xn[0], xl[0]) < 1e-10 and rel(xn[1], xl[1]) < 1e-10
    r = om.forward(K, onset, *xl)
    assert rel(r[0], d[0]) < 1e-10


def _block_parts(nt=16, nx=2, nv=1):
    """Time-domain R and R* matrices (entry by entry) of the case, with Theta as a diagonal."""
    k, K, onset = _marchenko_case(nt, nx=nx, nv=nv)
    R = _conv_matrix(k)
    Rs = _conv_matrix(np.roll(k[::-1], 1, axis=0))  # R*: correlation = convolution with k(-t)
    return k, K, onset, R, Rs


def test_greens_match_dense_eq6_block_matrix():
    """Eq.6 with f- != 0: [-g-; g+*] = [[I, -R], [-R*, I]] [f-; f+], R and R* assembled entry by entry."""
    nt = 16
    k, K, onset, R, Rs = _block_parts(nt)
    n = k.shape[1]
    I = np.eye(nt * n)
    B = np.block([[I, -R], [-Rs, I]])
    fm = synth.gaussian((nt, n, 1), seed=21)
    fplus = synth.gaussian((nt, n, 1), seed=22)
    gm, gpc = om.greens(K, fm, fplus)
    lhs = B @ np.concatenate([fm.ravel(), fplus.ravel()])
    assert rel(-gm.ravel(), lhs[: nt * n]) < 1e-12
    assert rel(gpc.ravel(), lhs[nt * n:]) < 1e-12
    # the two blocks use different operators: R and R* differ for this kernel, so swapping them,
    # or dropping the f- terms, changes the result well beyond rounding
    assert rel(R @ fplus.ravel(), Rs @ fplus.ravel()) > 0.1
    assert rel(-gm.ravel(), (fm.ravel() - Rs @ fplus.ravel())) > 0.1
    assert rel(gpc.ravel(), fplus.ravel() - R @ fm.ravel()) > 0.1
    assert rel(gpc.ravel(), fplus.ravel()) > 0.1


def test_marchenko_data_matches_dense_theta_r():
    """Right-hand side of Eq.5: (Theta R f_d+, 0) from the entry-by-entry convolution matrix."""
    nt = 16
    k, K, onset, R, Rs = _block_parts(nt)
    n = k.shape[1]
    th = om.theta(nt, onset)
    fd = synth.ricker_spikes(nt, n, 1)
    d0, d1 = om.data(K, onset, fd)
    ref = th[:, :, 0].ravel() * (R @ fd.ravel())
    assert rel(d0.ravel(), ref) < 1e-12
    assert np.all(d1 == 0) and d1.shape == fd.shape
    # the window removes part of the product and R* differs from R on this input
    assert rel(d0.ravel(), R @ fd.ravel()) > 0.1
    assert rel(d0.ravel(), th[:, :, 0].ravel() * (Rs @ fd.ravel())) > 0.1


@pytest.mark.parametrize("shape,scale", [((12, 12), 3.7), ((9, 14), 0.21), ((20, 7), 11.0)])
def test_spectral_norm_matches_svd(shape, scale):
    """Power iteration on K^H K returns the largest singular value (not its square)."""
    from oracle import power
    K = scale * (synth.gaussian(shape, seed=41) + 1j * synth.gaussian(shape, seed=42))
    ref = np.linalg.norm(K, 2)
    assert abs(ref - 1.0) > 0.5  # so that the norm and its square differ
    assert abs(power.spectral_norm(K, iters=400) - ref) < 1e-9 * ref


def test_greens_single_scattering():
    """Eq.6 with f- = 0 and f+ = f_d+ gives g- = R f_d+ (single-scattering redatuming)."""
    nt = 32
    k, K, _ = _marchenko_case(nt)
    fd = synth.ricker_spikes(nt, 4, 1)
    gm, gpc = om.greens(K, np.zeros_like(fd), fd)
    assert rel(gm, omdc.conv_time(k, fd)) < 1e-12
    assert rel(gpc, fd) < 1e-14


def test_window_encoding_by_enumeration():
    """Two-sided (onset >= 0) and one-sided causal (onset < 0) windows, sample by sample."""
    nt = 12
    onset = np.array([[0, 3], [-1, -4], [-12, 7]], dtype=np.int32)
    th = om.theta(nt, onset)
    for s in range(3):
        for v in range(2):
            o = onset[s, v]
            for t in range(nt):
                lag = t if t < nt // 2 else t - nt
                keep = abs(lag) < o if o >= 0 else 0 <= lag < -o
                assert th[t, s, v] == (1.0 if keep else 0.0)
    assert np.array_equal(th[:, 2, 0], (np.arange(nt) < nt // 2).astype(float))


def test_causal_preconditioned_lsqr_is_restricted_lstsq():
    """LSQR on C P (P the causal window) converges to least squares over the causal samples only."""
    nt, nx = 16, 2
    k, K, _ = _marchenko_case(nt=nt, nx=nx, scale=3.0)
    n = nx * nx
    pre = np.full((n, 1), -nt, dtype=np.int32)
    P = om.theta(nt, pre)
    b = synth.gaussian((nt, n, 1), seed=31)
    A = lambda v: [omdc.mdc_forward(K, P * v[0])]
    AH = lambda u: [P * omdc.mdc_adjoint(K, u[0])]
    x, _ = ol.lsqr(A, AH, [b], 80)
    assert np.all(x[0][nt // 2:] == 0)
    C = _conv_matrix(k)
    cols = np.concatenate([np.arange(t * n, (t + 1) * n) for t in range(nt // 2)])
    z = np.linalg.lstsq(C[:, cols], b[:, :, 0].ravel(), rcond=None)[0]
    assert rel(x[0][: nt // 2, :, 0].ravel(), z) < 1e-8
