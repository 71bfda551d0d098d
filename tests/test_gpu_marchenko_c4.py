"""Marchenko LSQR workloads (Eq.5, 32 focusing points, full / 2x / 4x decimated grids).

Reduced sizes: the whole LSQR run is compared with the FP64 oracle's LSQR,
iterate for iterate (FP32 vectors, FP64 scalars: tolerance 1e-5 on the
solution).  Full size (nt=1024, nfmax=250, 50 x 50 traces, nv=32): the
Marchenko apply is compared on sampled (trace, point) pairs, the operator
passes the dot-product test, and the solve satisfies the LSQR identity
||d - M x|| = phibar.  On the 4x decimated full-size grid (626 traces, the
same 32 points and 30 iterations) the whole solve is compared with the FP64
oracle's LSQR in every storage format: FP32 to 1e-5, the 16-bit formats to
the 1e-3 model-error budget, with the phibar history checked iterate by
iterate.
"""
import numpy as np
import pytest
import torch

from oracle import lsqr as ol
from oracle import marchenko as omc
from oracle import mdc as om
from paper_2011_11120_amd import synth, workloads

pytestmark = pytest.mark.gpu


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.fixture(scope="module")
def mdcmod(gpu):
    from paper_2011_11120_amd import mdc
    return mdc


def build(mdcmod, case):
    op = mdcmod.MdcOp(case.spec.nt, case.spec.nfmax, case.n, case.n, max_cols=2 * case.nv)
    op.synth_kernel(case.spec, s_index=case.idx, r_index=case.idx)
    return op


@pytest.mark.parametrize("d", [1, 2, 4])
def test_reduced_marchenko_lsqr_matches_oracle(mdcmod, d):
    print(f"reduced marchenko d={d}", flush=True)
    case = workloads.marchenko_case(nx=12, nt=256, nfmax=70, d=d, px=4, py=2,
                                    kappa_value=workloads.kappa("c4") * 8.0)
    op = build(mdcmod, case)
    on = dev(case.onset, torch.int32)
    dg = op.marchenko_data(on, dev(case.fd))
    K = synth.kernel_block(case.spec, np.arange(case.spec.nfmax), case.idx, case.idx)
    d0, d1 = omc.data(K, case.onset, case.fd)
    dh = dg.cpu().numpy().astype(np.float64)
    assert relmax(dh[0], d0) < 1e-5 and np.all(dh[1] == 0)
    niter = 20
    x, hist = op.lsqr(dg, niter, kind=mdcmod.MDC_OP_MARCHENKO, nv=case.nv, onset=on)
    xr, hr = ol.lsqr(lambda v: list(omc.forward(K, case.onset, *v)),
                     lambda u: list(omc.adjoint(K, case.onset, *u)), [d0, d1], niter)
    assert rel2(x.cpu().numpy().astype(np.float64), np.stack(xr)) < 1e-5
    assert np.max(np.abs(hist.cpu().numpy() - hr) / hr[0]) < 1e-5
    assert hr[-1] < 0.5 * hr[0]  # the solve makes progress (well-conditioned M)
    op.close()


@pytest.fixture(scope="module")
def c4(mdcmod):
    case = workloads.marchenko_case(kappa_value=workloads.kappa("c4"))
    print(f"c4: n={case.n} nv={case.nv}", flush=True)
    op = build(mdcmod, case)
    yield case, op
    op.close()


def test_c4_marchenko_apply_sampled(c4):
    case, op = c4
    nt, n, nv = case.spec.nt, case.n, case.nv
    a0 = synth.gaussian((nt, n, nv), seed=1)
    a1 = synth.gaussian((nt, n, nv), seed=2)
    on = dev(case.onset, torch.int32)
    g0, g1 = op.marchenko(on, dev(a0), dev(a1))
    h0, h1 = op.marchenko(on, dev(a0), dev(a1), adjoint=True)
    torch.cuda.synchronize()
    rows = np.array([0, 1249, 2499])
    vs = np.array([0, 17, 31])
    allf = np.arange(case.spec.nfmax)
    Krows = synth.kernel_block(case.spec, allf, rows, case.idx)       # [f, rows, all]
    th = omc.theta(nt, case.onset[rows][:, vs])
    # forward rows: o0 = a0 - Theta R a1 ; o1 = a1 - Theta R* a0
    r0 = a0[:, rows][:, :, vs] - th * om.mdc_forward(Krows, a1[:, :, vs])
    r1 = a1[:, rows][:, :, vs] - th * om.mdc_forward(np.conj(Krows), a0[:, :, vs])
    assert relmax(g0[:, rows][:, :, vs].cpu().numpy(), r0) < 1e-5
    assert relmax(g1[:, rows][:, :, vs].cpu().numpy(), r1) < 1e-5
    # adjoint rows need kernel columns: i1 = a1 - R^H Theta a0 ; i0 = a0 - R*^H Theta a1
    Kcols = synth.kernel_block(case.spec, allf, case.idx, rows)       # [f, all, rows]
    thf = omc.theta(nt, case.onset[:, vs])
    s1 = a1[:, rows][:, :, vs] - om.mdc_adjoint(Kcols, thf * a0[:, :, vs])
    s0 = a0[:, rows][:, :, vs] - om.mdc_adjoint(np.conj(Kcols), thf * a1[:, :, vs])
    assert relmax(h1[:, rows][:, :, vs].cpu().numpy(), s1) < 1e-5
    assert relmax(h0[:, rows][:, :, vs].cpu().numpy(), s0) < 1e-5


def test_c4_dot_product(c4):
    case, op = c4
    nt, n, nv = case.spec.nt, case.n, case.nv
    on = dev(case.onset, torch.int32)
    a = [synth.gaussian((nt, n, nv), seed=s) for s in (3, 4)]
    b = [synth.gaussian((nt, n, nv), seed=s) for s in (5, 6)]
    Ma = op.marchenko(on, dev(a[0]), dev(a[1]))
    MHb = op.marchenko(on, dev(b[0]), dev(b[1]), adjoint=True)
    lhs = sum(np.vdot(p.cpu().numpy().astype(np.float64), q) for p, q in zip(Ma, b))
    rhs = sum(np.vdot(p, q.cpu().numpy().astype(np.float64)) for p, q in zip(a, MHb))
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_c4_lsqr_residual_identity(mdcmod, c4):
    case, op = c4
    on = dev(case.onset, torch.int32)
    dg = op.marchenko_data(on, dev(case.fd))
    x, hist = op.lsqr(dg, 30, kind=mdcmod.MDC_OP_MARCHENKO, nv=case.nv, onset=on)
    m0, m1 = op.marchenko(on, x[0].contiguous(), x[1].contiguous())
    res = torch.sqrt(((dg[0].double() - m0.double()) ** 2).sum() + ((dg[1].double() - m1.double()) ** 2).sum())
    h = hist.cpu().numpy()
    assert np.all(np.diff(h) <= 1e-6 * h[0])               # phibar never increases
    assert h[-1] < 1e-2 * h[0]                              # 30 iterations converge on M with ||K_f|| <= 0.5
    assert abs(float(res) - h[-1]) < 1e-4 * h[0]            # ||d - M x|| == phibar (exact arithmetic identity)


@pytest.mark.parametrize("prec", ["bf16x2", "fp16s", "fp16"])
def test_c4_low_precision_solution_matches_fp32(mdcmod, c4, prec):
    """Full size, 30 iterations: the solution with a 16-bit stored kernel stays within the 1e-3
    relative model error of the FP32 solution (same right-hand side, same onsets)."""
    case, op = c4
    on = dev(case.onset, torch.int32)
    dg = op.marchenko_data(on, dev(case.fd))
    x32, _ = op.lsqr(dg, 30, kind=mdcmod.MDC_OP_MARCHENKO, nv=case.nv, onset=on)
    x32 = x32.cpu().numpy().astype(np.float64)
    print(f"c4 {prec}: generating kernel on device", flush=True)
    lp = mdcmod.MdcOp(case.spec.nt, case.spec.nfmax, case.n, case.n, max_cols=2 * case.nv, prec=prec)
    lp.synth_kernel(case.spec, s_index=case.idx, r_index=case.idx)
    xl, hist = lp.lsqr(dg, 30, kind=mdcmod.MDC_OP_MARCHENKO, nv=case.nv, onset=on)
    err = rel2(xl.cpu().numpy().astype(np.float64), x32)
    print(f"c4 {prec}: relative model difference to FP32 {err:.2e}", flush=True)
    assert err < 1e-3
    h = hist.cpu().numpy()
    assert h[-1] < 1e-2 * h[0]
    lp.close()


@pytest.fixture(scope="module")
def c4d4_oracle():
    """FP64 oracle LSQR on the 4x decimated full-size Marchenko problem (host, about a minute)."""
    import time
    case = workloads.marchenko_case(d=4, kappa_value=workloads.kappa("c4"))
    t0 = time.perf_counter()
    K = synth.kernel_block(case.spec, np.arange(case.spec.nfmax), case.idx, case.idx)
    Kc = np.conj(K)
    print(f"c4 d4 oracle: kernel {K.shape} generated in {time.perf_counter() - t0:.1f} s", flush=True)
    th = omc.theta(case.spec.nt, case.onset)
    # the oracle's Marchenko blocks (Eq.5) with the conjugated kernel formed once
    fwd = lambda v: [v[0] - th * om.mdc_forward(K, v[1]), -th * om.mdc_forward(Kc, v[0]) + v[1]]
    adj = lambda u: [u[0] - om.mdc_adjoint(Kc, th * u[1]), -om.mdc_adjoint(K, th * u[0]) + u[1]]
    calls = [0]

    def fwd_p(v):
        calls[0] += 1
        if calls[0] % 5 == 0:
            print(f"c4 d4 oracle: iteration {calls[0]} of 30 ({time.perf_counter() - t0:.0f} s)", flush=True)
        return fwd(v)

    d0, d1 = omc.data(K, case.onset, case.fd)
    xr, hr = ol.lsqr(fwd_p, adj, [d0, d1], 30)
    print(f"c4 d4 oracle: done in {time.perf_counter() - t0:.1f} s, phibar {hr[0]:.3e} -> {hr[-1]:.3e}", flush=True)
    return case, d0, np.stack(xr), hr


@pytest.mark.parametrize("prec,tol_data,tol", [("fp32", 1e-5, 1e-5), ("fp16s", 2e-3, 1e-3), ("bf16x2", 2e-5, 1e-3)])
def test_c4_d4_full_size_lsqr_matches_oracle(mdcmod, c4d4_oracle, prec, tol_data, tol):
    case, d0, xr, hr = c4d4_oracle
    print(f"c4 d4 {prec}: n={case.n} nv={case.nv}", flush=True)
    op = mdcmod.MdcOp(case.spec.nt, case.spec.nfmax, case.n, case.n, max_cols=2 * case.nv, prec=prec)
    op.synth_kernel(case.spec, s_index=case.idx, r_index=case.idx)
    on = dev(case.onset, torch.int32)
    dg = op.marchenko_data(on, dev(case.fd))
    e_data = relmax(dg[0].cpu().numpy().astype(np.float64), d0)
    x, hist = op.lsqr(dg, 30, kind=mdcmod.MDC_OP_MARCHENKO, nv=case.nv, onset=on)
    err = rel2(x.cpu().numpy().astype(np.float64), xr)
    eh = float(np.max(np.abs(hist.cpu().numpy() - hr)) / hr[0])
    print(f"c4 d4 {prec}: data {e_data:.2e}, model error {err:.2e}, phibar history {eh:.2e}", flush=True)
    assert e_data < tol_data
    assert err < tol
    assert eh < tol
    assert hr[-1] < 1e-2 * hr[0]
    op.close()
