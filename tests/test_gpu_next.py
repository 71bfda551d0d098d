"""Widened rows: kernel from time traces, Green's functions (Eq.6), Neumann scheme,
CGLS (the paper's solver), and MDD (Eq.8) chained after Marchenko redatuming."""
import numpy as np
import pytest
import torch

from oracle import lsqr as ol
from oracle import marchenko as omc
from oracle import mdc as om
from oracle import power
from paper_2011_11120_amd import synth, workloads

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


@pytest.mark.parametrize("nx_r,temp", [(4, False), (3, True)])
def test_kernel_from_time_traces_bruteforce(mdcmod, nx_r, temp):
    """K = dt dA DFT(traces) through the library's FFT; the operator equals Eq.1's sums."""
    nt, dt, dx = 64, 0.004, 20.0
    G = synth.c1_time_kernel(nt=nt, nx=3, nx_r=nx_r, dt=dt, dx=dx)
    ns, nr = G.shape[1], G.shape[2]
    k = dt * dx * dx * G
    op = mdcmod.MdcOp(nt, nt // 2 + 1, ns, nr, max_cols=2)
    tmp = torch.empty(8 * (nt // 2 + 1) * ns * nr, dtype=torch.uint8, device="cuda") if temp else None
    mdcmod.mdc_set_kernel_time(op.handle, dev(G), scale=dt * dx * dx, temp=tmp)
    x = synth.gaussian((nt, nr, 2), seed=1)
    y = synth.gaussian((nt, ns, 2), seed=2)
    assert relmax(host(op.forward(dev(x))), om.conv_time(k, x)) < TOL
    assert relmax(host(op.adjoint(dev(y))), om.corr_time(k, y)) < TOL
    # conj: traces of g(-t) give the kernel of g
    G_rev = np.roll(G[::-1], 1, axis=0)
    op2 = mdcmod.MdcOp(nt, nt // 2 + 1, ns, nr, max_cols=2)
    mdcmod.mdc_set_kernel_time(op2.handle, dev(G_rev), conj=True, scale=dt * dx * dx, temp=tmp)
    assert relmax(host(op2.forward(dev(x))), om.conv_time(k, x)) < TOL


def test_kernel_from_time_traces_truncated_fp16s(mdcmod):
    nt, nfmax, ns, nr = 128, 40, 20, 12
    g = synth.gaussian((nt, ns, nr), seed=3)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, prec="fp16s")
    tmp = torch.empty(8 * nfmax * ns * nr, dtype=torch.uint8, device="cuda")
    mdcmod.mdc_set_kernel_time(op.handle, dev(g), scale=0.5, temp=tmp)
    K = 0.5 * np.fft.rfft(g, axis=0)[:nfmax]
    x = synth.gaussian((nt, nr, 1), seed=4)
    assert relmax(host(op.forward(dev(x))), om.mdc_forward(K, x)) < 2e-3
    with pytest.raises(mdcmod.MdcError):
        mdcmod.mdc_set_kernel_time(op.handle, dev(g))  # 16-bit storage needs a temp buffer


def marchenko_kernel(nt, nfmax, n, seed, q):
    K = synth.random_complex_kernel(nfmax, n, n, seed=seed)
    return K * (q / max(power.spectral_norm(K[f], iters=80) for f in range(nfmax)))


def test_greens_match_oracle(mdcmod):
    nt, nfmax, n, nv = 64, 25, 36, 3
    K = marchenko_kernel(nt, nfmax, n, 1, 0.5)
    op = mdcmod.MdcOp(nt, nfmax, n, n, max_cols=2 * nv)
    op.set_kernel(dev(K, torch.complex64))
    fm = synth.gaussian((nt, n, nv), seed=1)
    fd = synth.ricker_spikes(nt, n, nv)
    fmp = synth.gaussian((nt, n, nv), seed=2)
    gm, gp = op.greens(dev(fm), dev(fd), dev(fmp))
    rm, rp = omc.greens(K, fm, fd + fmp)
    assert relmax(host(gm), rm) < TOL and relmax(host(gp), rp) < TOL


def test_neumann_matches_oracle(mdcmod):
    nt, nfmax, nx, nv = 64, 25, 5, 2
    n = nx * nx
    K = marchenko_kernel(nt, nfmax, n, 3, 0.4)
    onset = (4 + (np.arange(n * nv) * 5) % 24).reshape(n, nv).astype(np.int32)
    op = mdcmod.MdcOp(nt, nfmax, n, n, max_cols=2 * nv)
    op.set_kernel(dev(K, torch.complex64))
    d0, d1 = omc.data(K, onset, synth.ricker_spikes(nt, n, nv))
    f = op.neumann(dev(onset, torch.int32), dev(np.stack([d0, d1])), 12)
    r0, r1 = omc.neumann(K, onset, d0, d1, 12)
    assert rel2(host(f), np.stack([r0, r1])) < TOL


@pytest.mark.parametrize("kind", ["mdc", "marchenko"])
def test_cgls_matches_oracle(mdcmod, kind):
    nt, nfmax, nx, nv, niter = 64, 25, 5, 2, 10
    n = nx * nx
    K = marchenko_kernel(nt, nfmax, n, 5, 0.5)
    op = mdcmod.MdcOp(nt, nfmax, n, n, max_cols=2 * nv)
    op.set_kernel(dev(K, torch.complex64))
    if kind == "mdc":
        b = synth.gaussian((nt, n, nv), seed=6)
        x, h = op.cgls(dev(b), niter, nv=nv)
        xr, hr = ol.cgls(lambda v: [om.mdc_forward(K, v[0])], lambda u: [om.mdc_adjoint(K, u[0])], [b], niter)
        xr = xr[0]
    else:
        onset = (4 + (np.arange(n * nv) * 5) % 24).reshape(n, nv).astype(np.int32)
        d0, d1 = omc.data(K, onset, synth.ricker_spikes(nt, n, nv))
        x, h = op.cgls(dev(np.stack([d0, d1])), niter, kind=mdcmod.MDC_OP_MARCHENKO, nv=nv,
                       onset=dev(onset, torch.int32))
        xr, hr = ol.cgls(lambda v: list(omc.forward(K, onset, *v)), lambda u: list(omc.adjoint(K, onset, *u)),
                         [d0, d1], niter)
        xr = np.stack(xr)
    assert rel2(host(x), xr) < TOL
    assert np.max(np.abs(host(h) - hr) / hr[0]) < TOL


def test_marchenko_greens_mdd_chain_matches_oracle(mdcmod):
    """Receiver-side redatuming (Eq.5, LSQR) -> Green's functions (Eq.6) -> source-side MDD
    (Eq.8: kernel G+ from the g+* traces, LSQR over all focusing points as virtual sources)."""
    # record of 1.024 s: the direct arrivals from 650 m (0.33-0.4 s) fit inside it
    case = workloads.marchenko_case(nx=6, nt=256, nfmax=70, d=1, px=4, py=2,
                                    kappa_value=workloads.kappa("c4") * 8.0)
    nt, n, nF = case.spec.nt, case.n, case.nv
    dAF = 20.0 * 20.0
    op = mdcmod.MdcOp(nt, case.spec.nfmax, n, n, max_cols=2 * nF)
    op.synth_kernel(case.spec)
    on = dev(case.onset, torch.int32)
    dg = op.marchenko_data(on, dev(case.fd))
    f, _ = op.lsqr(dg, 12, kind=mdcmod.MDC_OP_MARCHENKO, nv=nF, onset=on)
    gm, gpc = op.greens(f[0].contiguous(), dev(case.fd), f[1].contiguous())
    mdd = mdcmod.MdcOp(nt, case.spec.nfmax, n, nF, max_cols=nF)
    mdcmod.mdc_set_kernel_time(mdd.handle, gpc, conj=True, scale=dAF)
    r, _ = mdd.lsqr(gm, 15, nv=nF)
    # the same chain in the oracle (FP64), from the same seeded inputs
    K = synth.kernel_block(case.spec, np.arange(case.spec.nfmax), case.idx, case.idx)
    d0, d1 = omc.data(K, case.onset, case.fd)
    fo, _ = ol.lsqr(lambda v: list(omc.forward(K, case.onset, *v)),
                    lambda u: list(omc.adjoint(K, case.onset, *u)), [d0, d1], 12)
    gmo, gpco = omc.greens(K, fo[0], case.fd + fo[1])
    Kmdd = dAF * np.conj(om.rfft_trunc(gpco, case.spec.nfmax) * np.sqrt(nt))
    ro, _ = ol.lsqr(lambda v: [om.mdc_forward(Kmdd, v[0])], lambda u: [om.mdc_adjoint(Kmdd, u[0])], [gmo], 15)
    print(f"stage errors: f {rel2(host(f), np.stack(fo)):.2e} g- {rel2(host(gm), gmo):.2e} "
          f"g+* {rel2(host(gpc), gpco):.2e}", flush=True)
    assert np.linalg.norm(ro[0]) > 1e-6 * np.linalg.norm(gmo)  # a non-trivial reflectivity
    err = rel2(host(r), ro[0])
    print(f"MDD chain: relative error {err:.2e}", flush=True)
    assert err < 1e-4
    # adjoint-only imaging (correlation, the MDD section's adjoint) equals the oracle's
    img = mdd.adjoint(gm)
    assert relmax(host(img), om.mdc_adjoint(Kmdd, gmo)) < 1e-4
    # MDD with the causal time preconditioner (the reflectivity lives at non-negative times)
    causal = np.full((nF, nF), -nt, dtype=np.int32)
    rc, _ = mdd.lsqr(gm, 15, nv=nF, onset=dev(causal, torch.int32))
    P = omc.theta(nt, causal)
    rco, _ = ol.lsqr(lambda v: [om.mdc_forward(Kmdd, P * v[0])], lambda u: [P * om.mdc_adjoint(Kmdd, u[0])],
                     [gmo], 15)
    rcg = host(rc)
    assert np.all(rcg[nt // 2:] == 0)
    err = rel2(rcg, rco[0])
    print(f"causal MDD chain: relative error {err:.2e}", flush=True)
    assert err < 1e-4


@pytest.mark.parametrize("solver", ["lsqr", "cgls"])
def test_preconditioned_mdc_solvers_match_oracle(mdcmod, solver):
    """Plain-MDC solves with a model window P (one-sided and two-sided onsets mixed)."""
    nt, nfmax, ns, nr, nv, niter = 64, 25, 20, 12, 3, 10
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=41)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=nv)
    op.set_kernel(dev(K, torch.complex64))
    pre = (np.arange(nr * nv).reshape(nr, nv) % 7 - 3) * 5
    pre[0, 0] = -nt
    pre = pre.astype(np.int32)
    b = synth.gaussian((nt, ns, nv), seed=42)
    run = op.lsqr if solver == "lsqr" else op.cgls
    x, hist = run(dev(b), niter, nv=nv, onset=dev(pre, torch.int32))
    P = omc.theta(nt, pre)
    ref = ol.lsqr if solver == "lsqr" else ol.cgls
    xr, hr = ref(lambda v: [om.mdc_forward(K, P * v[0])], lambda u: [P * om.mdc_adjoint(K, u[0])], [b], niter)
    xg = host(x)
    assert np.all(xg[P == 0] == 0)
    assert rel2(xg, xr[0]) < TOL
    assert np.max(np.abs(host(hist) - hr) / hr[0]) < TOL


def test_irregular_geometry_voronoi_weights(mdcmod):
    """Irregular receivers (a random half of the lattice) with Voronoi areal weights per column."""
    from paper_2011_11120_amd import geometry
    spec = synth.KernelSpec(nt=128, nfmax=40, nx=8, dx=15.0, nev=6, kappa=1.0)
    idx = synth.irregular_subset(spec.nx, spec.nx, 0.5)
    gx, gy = synth.grid_xy(spec.nx, spec.nx, spec.dx)
    w = geometry.voronoi_areas(gx[idx], gy[idx], bounds=(-7.5, 112.5, -7.5, 112.5), pixel=0.5)
    K = synth.kernel_block(spec, np.arange(spec.nfmax), np.arange(spec.n), idx)
    op = mdcmod.MdcOp(spec.nt, spec.nfmax, spec.n, idx.size, max_cols=3)
    op.set_kernel(dev(K, torch.complex64), col_weight=dev(w))
    Kw = K * w[None, None, :]
    x = synth.gaussian((spec.nt, idx.size, 3), seed=21)
    y = synth.gaussian((spec.nt, spec.n, 3), seed=22)
    assert relmax(host(op.forward(dev(x))), om.mdc_forward(Kw, x)) < TOL
    assert relmax(host(op.adjoint(dev(y))), om.mdc_adjoint(Kw, y)) < TOL
