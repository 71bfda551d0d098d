"""GPU parity of the Marchenko operator (Eq.5) and of device LSQR against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import lsqr as ol
from oracle import marchenko as omc
from oracle import mdc as om
from oracle import power
from paper_2011_11120_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def mdcmod(gpu):
    from paper_2011_11120_amd import mdc
    return mdc


def marchenko_case(nt=64, nfmax=25, nx=6, nv=3, seed=0, q=0.5):
    n = nx * nx
    K = synth.random_complex_kernel(nfmax, n, n, seed=seed)
    K *= q / max(power.spectral_norm(K[f], iters=80) for f in range(nfmax))
    onset = (4 + (np.arange(n * nv) * 7) % (nt // 2 - 4)).reshape(n, nv).astype(np.int32)
    return K, onset


def op_for(mdcmod, K, nt, max_cols):
    nf, ns, nr = K.shape
    op = mdcmod.MdcOp(nt, nf, ns, nr, max_cols=max_cols)
    op.set_kernel(dev(K, torch.complex64))
    return op


@pytest.mark.parametrize("nt,nfmax,nx,nv", [(64, 25, 6, 3), (128, 65, 5, 1), (256, 60, 8, 5)])
def test_marchenko_forward_adjoint(mdcmod, nt, nfmax, nx, nv):
    print(f"marchenko nt={nt} nfmax={nfmax} nx={nx} nv={nv}", flush=True)
    K, onset = marchenko_case(nt, nfmax, nx, nv)
    n = nx * nx
    op = op_for(mdcmod, K, nt, 2 * nv)
    a0, a1 = synth.gaussian((nt, n, nv), seed=1), synth.gaussian((nt, n, nv), seed=2)
    g0, g1 = op.marchenko(dev(onset, torch.int32), dev(a0), dev(a1))
    r0, r1 = omc.forward(K, onset, a0, a1)
    assert relmax(host(g0), r0) < TOL and relmax(host(g1), r1) < TOL
    h0, h1 = op.marchenko(dev(onset, torch.int32), dev(a0), dev(a1), adjoint=True)
    s0, s1 = omc.adjoint(K, onset, a0, a1)
    assert relmax(host(h0), s0) < TOL and relmax(host(h1), s1) < TOL


def test_lsqr_mdc_matches_oracle(mdcmod):
    nt, nfmax, n, nv, niter = 64, 20, 36, 2, 12
    K = synth.random_complex_kernel(nfmax, n, n, seed=3)
    op = op_for(mdcmod, K, nt, nv)
    b = synth.gaussian((nt, n, nv), seed=4)
    x, hist = op.lsqr(dev(b), niter, nv=nv)
    xr, hr = ol.lsqr(lambda v: [om.mdc_forward(K, v[0])], lambda u: [om.mdc_adjoint(K, u[0])], [b], niter)
    assert rel2(host(x), xr[0]) < TOL
    assert np.max(np.abs(host(hist) - hr) / hr[0]) < TOL


@pytest.mark.parametrize("niter", [0, 1, 15])
def test_lsqr_marchenko_matches_oracle(mdcmod, niter):
    nt, nfmax, nx, nv = 64, 25, 5, 2
    K, onset = marchenko_case(nt, nfmax, nx, nv, seed=5)
    n = nx * nx
    op = op_for(mdcmod, K, nt, 2 * nv)
    fd = synth.ricker_spikes(nt, n, nv)
    d0, d1 = omc.data(K, onset, fd)
    b = np.stack([d0, d1])
    x, hist = op.lsqr(dev(b), niter, kind=mdcmod.MDC_OP_MARCHENKO, nv=nv, onset=dev(onset, torch.int32))
    A = lambda v: list(omc.forward(K, onset, *v))
    AH = lambda u: list(omc.adjoint(K, onset, *u))
    xr, hr = ol.lsqr(A, AH, [d0, d1], niter)
    xg = host(x)
    if niter == 0:
        assert np.all(xg == 0)
    else:
        assert rel2(xg, np.stack(xr)) < TOL
    assert np.max(np.abs(host(hist) - hr) / hr[0]) < TOL


def test_lsqr_zero_kernel_returns_data(mdcmod):
    nt, nfmax, n, nv = 32, 10, 16, 1
    K = np.zeros((nfmax, n, n), dtype=complex)
    op = op_for(mdcmod, K, nt, 2)
    onset = np.full((n, nv), 5, dtype=np.int32)
    b = np.stack([synth.gaussian((nt, n, nv), seed=s) for s in (1, 2)])
    x, hist = op.lsqr(dev(b), 3, kind=mdcmod.MDC_OP_MARCHENKO, nv=nv, onset=dev(onset, torch.int32))
    assert relmax(host(x), b) < 1e-6
    assert host(hist)[-1] < 1e-5 * host(hist)[0]


def test_lsqr_graph_replays_match_eager(mdcmod, monkeypatch):
    """Iterations 2..niter replay one captured graph; every replay equals the eager run bitwise."""
    nt, nfmax, nx, nv, niter = 64, 25, 5, 2, 9
    K, onset = marchenko_case(nt, nfmax, nx, nv, seed=7)
    n = nx * nx
    op = op_for(mdcmod, K, nt, 2 * nv)
    on = dev(onset, torch.int32)
    fd = synth.ricker_spikes(nt, n, nv)
    d0, d1 = omc.data(K, onset, fd)
    b = dev(np.stack([d0, d1]))
    monkeypatch.setenv("MDC_LSQR_GRAPH", "0")
    xe, he = op.lsqr(b, niter, kind=mdcmod.MDC_OP_MARCHENKO, nv=nv, onset=on)
    xe, he = xe.clone(), he.clone()
    monkeypatch.setenv("MDC_LSQR_GRAPH", "1")
    xg = torch.empty_like(xe)
    hg = torch.empty_like(he)
    other = dev(synth.gaussian((nt, n, nv), seed=9))
    for rep in range(3):
        xg.zero_()
        op.lsqr(b, niter, kind=mdcmod.MDC_OP_MARCHENKO, nv=nv, onset=on, out=(xg, hg))
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and torch.equal(hg, he), f"replay {rep}"
        op.forward(other)  # eager work between replays
        torch.cuda.synchronize()


# (kind, nt, nfmax, ns, nr, nv): rectangular MDC with an odd trace count (scalar epilogue), with a
# vector epilogue, with wide tiles and more than a thousand partial-sum slots; Marchenko blocks.
FUSED_CASES = [
    ("mdc", 64, 20, 35, 29, 1),
    ("mdc", 64, 20, 36, 40, 3),
    ("mdc", 64, 20, 1030, 1030, 8),
    ("marchenko", 64, 25, 25, 25, 2),
    ("marchenko", 128, 40, 49, 49, 3),
]


@pytest.mark.parametrize("solver", ["lsqr", "cgls"])
@pytest.mark.parametrize("case", FUSED_CASES, ids=lambda c: "-".join(map(str, c)))
def test_fused_norms_match_separate_passes_and_oracle(mdcmod, monkeypatch, case, solver):
    """The recurrences and norms fused into the inverse transforms equal the separate vector passes
    (same per-element arithmetic, partial sums grouped differently) and the FP64 oracle."""
    kind, nt, nfmax, ns, nr, nv = case
    print(f"fused {solver} {case}", flush=True)
    niter = 6
    op, b, args, A, AH, bl = solver_case(mdcmod, case)
    run = op.lsqr if solver == "lsqr" else op.cgls
    monkeypatch.delenv("MDC_LSQR_FUSE", raising=False)
    xf, hf = run(dev(b), niter, **args)
    xf, hf = host(xf), host(hf)
    monkeypatch.setenv("MDC_LSQR_FUSE", "0")
    xs, hs = run(dev(b), niter, **args)
    xs, hs = host(xs), host(hs)
    monkeypatch.delenv("MDC_LSQR_FUSE", raising=False)
    assert rel2(xf, xs) < 1e-6
    assert np.max(np.abs(hf - hs)) / hs[0] < 1e-6
    xr, hr = (ol.lsqr if solver == "lsqr" else ol.cgls)(A, AH, bl, niter)
    assert rel2(xf, np.stack(xr) if kind == "marchenko" else xr[0]) < TOL
    assert np.max(np.abs(hf - hr) / hr[0]) < TOL


# 2209 traces x 4 points = 8836 traces per block: 16-trace tiles with a partly filled last tile on the
# 16-byte path (the cases above pad only on the narrow-tile and scalar paths)
TILED_PAD_CASES = [("mdc", 64, 10, 2209, 2209, 4), ("marchenko", 64, 10, 2209, 2209, 4)]


@pytest.mark.parametrize("fuse", ["1", "0"])
@pytest.mark.parametrize("case", FUSED_CASES + TILED_PAD_CASES, ids=lambda c: "-".join(map(str, c)))
def test_tiled_vectors_match_plain_layout(mdcmod, monkeypatch, case, fuse):
    """LSQR keeps its Krylov vectors in the transforms' tiled layout (tiles of whole trace groups,
    zero padding traces, converted at the boundary); the caller's layout (MDC_LSQR_TILED=0) gives
    the same solution and residual history (the same per-element arithmetic; only the vector norms
    outside the transforms are summed in another order), for odd and padded trace counts."""
    print(f"tiled {case} fuse={fuse}", flush=True)
    niter = 6
    op, b, args, _, _, _ = solver_case(mdcmod, case)
    monkeypatch.setenv("MDC_LSQR_FUSE", fuse)
    monkeypatch.delenv("MDC_LSQR_TILED", raising=False)
    xt, ht = op.lsqr(dev(b), niter, **args)
    xt, ht = host(xt), host(ht)
    monkeypatch.setenv("MDC_LSQR_TILED", "0")
    xp, hp = op.lsqr(dev(b), niter, **args)
    xp, hp = host(xp), host(hp)
    monkeypatch.delenv("MDC_LSQR_TILED", raising=False)
    monkeypatch.delenv("MDC_LSQR_FUSE", raising=False)
    assert rel2(xt, xp) < 1e-6
    assert np.max(np.abs(ht - hp)) / hp[0] < 1e-6


@pytest.mark.parametrize("niter", [0, 1, 2])
def test_tiled_short_solves(mdcmod, monkeypatch, niter):
    """Solves that end before the captured iteration graph (0, 1 iterations) or right after its
    first replay still write their tiled iterate back: x = 0 and phibar_0 = ||b|| after none, and
    the caller's-layout run equals the tiled one after one or two."""
    op, b, args, _, _, _ = solver_case(mdcmod, ("marchenko", 64, 25, 25, 25, 3))
    monkeypatch.delenv("MDC_LSQR_TILED", raising=False)
    xt, ht = op.lsqr(dev(b), niter, **args)
    xt, ht = host(xt), host(ht)
    monkeypatch.setenv("MDC_LSQR_TILED", "0")
    xp, hp = op.lsqr(dev(b), niter, **args)
    xp, hp = host(xp), host(hp)
    monkeypatch.delenv("MDC_LSQR_TILED", raising=False)
    assert abs(ht[0] - np.linalg.norm(b.ravel())) < 1e-6 * ht[0]
    if niter == 0:
        assert np.all(xt == 0) and np.all(xp == 0)
    else:
        assert rel2(xt, xp) < 1e-6
    assert np.max(np.abs(ht - hp)) / hp[0] < 1e-6


def solver_case(mdcmod, case):
    """Operator, right-hand side, solver arguments and oracle operator of one FUSED_CASES entry."""
    kind, nt, nfmax, ns, nr, nv = case
    if kind == "mdc":
        K = synth.random_complex_kernel(nfmax, ns, nr, seed=11)
        K *= 0.8 / max(power.spectral_norm(K[f], iters=40) for f in range(nfmax))
        op = op_for(mdcmod, K, nt, nv)
        b = synth.gaussian((nt, ns, nv), seed=12)
        args = dict(nv=nv)
        A = lambda v: [om.mdc_forward(K, v[0])]
        AH = lambda u: [om.mdc_adjoint(K, u[0])]
        bl = [b]
    else:
        K, onset = marchenko_case(nt, nfmax, int(round(ns ** 0.5)), nv, seed=13)
        op = op_for(mdcmod, K, nt, 2 * nv)
        fd = synth.ricker_spikes(nt, ns, nv)
        d0, d1 = omc.data(K, onset, fd)
        b = np.stack([d0, d1])
        args = dict(kind=mdcmod.MDC_OP_MARCHENKO, nv=nv, onset=dev(onset, torch.int32))
        A = lambda v: list(omc.forward(K, onset, *v))
        AH = lambda u: list(omc.adjoint(K, onset, *u))
        bl = [d0, d1]
    return op, b, args, A, AH, bl
