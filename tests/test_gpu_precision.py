"""Reduced-precision kernel storage (FP16 with per-frequency power-of-two scale, BF16, BF16 hi+lo).

Per-apply bound for the split low-precision formats: max-norm relative error <= 2e-3
against the FP64 oracle; BF16 hi+lo keeps close to FP32 (<= 2e-5).  LSQR with a
16-bit kernel: relative model error <= 1e-3 after the same iteration count.
The error of each case is printed so the run log records it.
"""
import numpy as np
import pytest
import torch

from oracle import lsqr as ol
from oracle import marchenko as omc
from oracle import mdc as om
from paper_2011_11120_amd import synth, workloads

pytestmark = pytest.mark.gpu

TOL = {"bf16x2": 2e-5, "fp16s": 2e-3, "bf16": 8e-3, "fp16": 2e-3}


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


SHAPES = [(64, 20, 40, 40, 1), (128, 40, 130, 98, 3), (128, 40, 129, 257, 9),
          (256, 60, 300, 200, 64), (128, 30, 200, 130, 65), (64, 20, 70, 30, 17),
          (64, 16, 512, 256, 24)]  # whole 256-row tiles in both directions (no idle row blocks)


@pytest.mark.parametrize("prec", ["bf16x2", "fp16s", "bf16", "fp16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_formats_match_oracle(mdcmod, prec, shape):
    nt, nfmax, ns, nr, nv = shape
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=ns + nv)
    K *= np.exp(np.linspace(0, 8, nfmax))[:, None, None]  # spread magnitudes across frequencies
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=nv, prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    x = synth.gaussian((nt, nr, nv), seed=3)
    y = synth.gaussian((nt, ns, nv), seed=4)
    ef = relmax(host(op.forward(dev(x))), om.mdc_forward(K, x))
    ea = relmax(host(op.adjoint(dev(y))), om.mdc_adjoint(K, y))
    print(f"{prec} {shape}: forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef < TOL[prec] and ea < TOL[prec]
    op.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x2", "fp16s", "bf16"])
@pytest.mark.parametrize("nv", [3, 5, 6, 7])
def test_streaming_widths_match_oracle(mdcmod, monkeypatch, prec, nv):
    """Every width below 9 streams the kernel once, for every storage format."""
    monkeypatch.setenv("MDC_PRODUCT", "gemv")
    nt, nfmax, ns, nr = 128, 30, 75, 133
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=7 * nv)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=nv, prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    x = synth.gaussian((nt, nr, nv), seed=8)
    y = synth.gaussian((nt, ns, nv), seed=9)
    ef = relmax(host(op.forward(dev(x))), om.mdc_forward(K, x))
    ea = relmax(host(op.adjoint(dev(y))), om.mdc_adjoint(K, y))
    tol = 1e-5 if prec == "fp32" else TOL[prec]
    print(f"streaming {prec} nv={nv}: forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef < tol and ea < tol
    op.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x2", "fp16s"])
@pytest.mark.parametrize("nv", [5, 8])
def test_streaming_chunks_match_oracle(mdcmod, monkeypatch, prec, nv):
    """Wide column groups over reductions longer than one LDS chunk: the forward stages X in chunks
    of 4096 / nv positions (two or three here, the last one short) with several positions per lane
    in flight, the adjoint stages Y in chunks of 4096 / nv rows (two here)."""
    monkeypatch.setenv("MDC_PRODUCT", "gemv")
    nt, nfmax, ns, nr = 64, 8, 900, 1100
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=11 * nv)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=nv, prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    x = synth.gaussian((nt, nr, nv), seed=12)
    y = synth.gaussian((nt, ns, nv), seed=13)
    ef = relmax(host(op.forward(dev(x))), om.mdc_forward(K, x))
    ea = relmax(host(op.adjoint(dev(y))), om.mdc_adjoint(K, y))
    tol = 1e-5 if prec == "fp32" else TOL[prec]
    print(f"chunked streaming {prec} nv={nv}: forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef < tol and ea < tol
    op.close()


@pytest.mark.parametrize("prec,tol", [("bf16x2", 1e-5), ("fp16s", 1e-5), ("bf16", 1e-5), ("fp16", 2.0 ** -11)])
def test_formats_dot_product(mdcmod, prec, tol):
    """The forward and adjoint read the same stored kernel, so the pair stays adjoint; with FP16
    spectra (one product) only up to the rounding of the spectra, 2^-11 relative."""
    nt, nfmax, ns, nr, nv = 128, 40, 150, 90, 12
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=1)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=nv, prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    x = synth.gaussian((nt, nr, nv), seed=5)
    y = synth.gaussian((nt, ns, nv), seed=6)
    lhs = np.vdot(host(op.forward(dev(x))), y)
    rhs = np.vdot(x, host(op.adjoint(dev(y))))
    print(f"dot test {prec}: {abs(lhs - rhs) / abs(lhs):.2e}", flush=True)
    assert abs(lhs - rhs) < tol * abs(lhs)


@pytest.mark.parametrize("prec,tol", [("bf16x2", 2.0 ** -15), ("fp16s", 2.0 ** -10), ("bf16", 2.0 ** -7),
                                      ("fp16", 2.0 ** -10)])
def test_generator_formats(mdcmod, prec, tol):
    spec = synth.KernelSpec(nt=256, nfmax=60, nx=12)
    op = mdcmod.MdcOp(spec.nt, spec.nfmax, spec.n, spec.n, prec=prec)
    op.synth_kernel(spec)
    rng = np.random.default_rng(1)
    for f, s, r in zip(rng.integers(1, 60, 40), rng.integers(0, 144, 40), rng.integers(0, 144, 40)):
        ref = synth.kernel_block(spec, [f], [s], [r])[0, 0, 0]
        got = mdcmod.mdc_kernel_element(op.handle, int(f), int(s), int(r))
        assert abs(got.real - ref.real) <= tol * abs(ref.real) + 1e-12 * abs(ref)
        assert abs(got.imag - ref.imag) <= tol * abs(ref.imag) + 1e-12 * abs(ref)
    op.close()


@pytest.mark.parametrize("prec", ["bf16x2", "fp16s", "fp16"])
def test_marchenko_lsqr_low_precision(mdcmod, prec):
    case = workloads.marchenko_case(nx=12, nt=256, nfmax=70, d=1, px=4, py=4,
                                    kappa_value=workloads.kappa("c4") * 8.0)
    op = mdcmod.MdcOp(case.spec.nt, case.spec.nfmax, case.n, case.n, max_cols=2 * case.nv, prec=prec)
    op.synth_kernel(case.spec, s_index=case.idx, r_index=case.idx)
    on = dev(case.onset, torch.int32)
    dg = op.marchenko_data(on, dev(case.fd))
    x, _ = op.lsqr(dg, 20, kind=mdcmod.MDC_OP_MARCHENKO, nv=case.nv, onset=on)
    K = synth.kernel_block(case.spec, np.arange(case.spec.nfmax), case.idx, case.idx)
    d0, d1 = omc.data(K, case.onset, case.fd)
    xr, _ = ol.lsqr(lambda v: list(omc.forward(K, case.onset, *v)),
                    lambda u: list(omc.adjoint(K, case.onset, *u)), [d0, d1], 20)
    err = rel2(host(x), np.stack(xr))
    print(f"marchenko lsqr {prec}: model error {err:.2e}", flush=True)
    assert err < 1e-3
    op.close()


@pytest.mark.parametrize("prec", ["fp16s", "fp16"])
def test_fp16_spectra_scale_is_per_column(mdcmod, monkeypatch, prec):
    """On the FP16 matrix cores each column's spectra get their own power-of-two scale, so a
    column's result does not depend on the magnitude of the columns batched with it: the first
    columns of a product [A | 2^20 B] equal the product of A alone, bit for bit."""
    monkeypatch.setenv("MDC_PRODUCT", "gemm")
    nt, nfmax, ns, nr, na, nb = 128, 30, 140, 100, 5, 11
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=23)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=na + nb, prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    xa = synth.gaussian((nt, nr, na), seed=24)
    xb = synth.gaussian((nt, nr, nb), seed=25) * 2.0 ** 20
    for adjoint in (False, True):
        n_in = ns if adjoint else nr
        a = synth.gaussian((nt, n_in, na), seed=26) if adjoint else xa
        b = synth.gaussian((nt, n_in, nb), seed=27) * 2.0 ** 20 if adjoint else xb
        apply = op.adjoint if adjoint else op.forward
        alone = host(apply(dev(a)))
        mixed = host(apply(dev(np.concatenate([a, b], axis=2))))
        assert np.array_equal(mixed[:, :, :na], alone)
        ref = (om.mdc_adjoint if adjoint else om.mdc_forward)(K, a)
        assert relmax(alone, ref) < TOL[prec]
    op.close()


@pytest.mark.parametrize("prec", ["bf16x2", "fp16s", "bf16", "fp16"])
@pytest.mark.parametrize("nv", [9, 64, 130])
def test_eight_wave_gemm16_matches_oracle(mdcmod, monkeypatch, prec, nv):
    """The 16-bit matrix-core product with eight waves of 32 rows per workgroup (family 2),
    forced at several widths (one, one full and three column tiles), against the oracle."""
    monkeypatch.setenv("MDC_PRODUCT", "gemm32")
    nt, nfmax, ns, nr = 128, 24, 300, 230
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=31 + nv)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=nv, prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    x = synth.gaussian((nt, nr, nv), seed=32)
    y = synth.gaussian((nt, ns, nv), seed=33)
    ef = relmax(host(op.forward(dev(x))), om.mdc_forward(K, x))
    ea = relmax(host(op.adjoint(dev(y))), om.mdc_adjoint(K, y))
    print(f"eight-wave gemm16 {prec} nv={nv}: forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef < TOL[prec] and ea < TOL[prec]
    op.close()
