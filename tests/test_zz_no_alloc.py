"""The allocation-free apply (static device scratch) against the workspace apply, through the C-ABI.

Both run the same kernels on the same inputs, so the outputs must agree bit for bit.  Two calls in
a row (the second narrower) check that a call does not depend on what the previous call left in
the shared scratch.  Sizes beyond the scratch are refused before anything is launched.
"""
import numpy as np
import pytest
import torch

from paper_2011_11120_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdcmod(gpu):
    from paper_2011_11120_amd import mdc
    return mdc


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "bf16x2"])
@pytest.mark.parametrize("widths", [(24, 5), (3, 1)])
def test_noalloc_matches_workspace_apply(mdcmod, prec, widths):
    nt, nfmax, ns, nr = 256, 60, 150, 130
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=17)
    op = mdcmod.MdcOp(nt, nfmax, ns, nr, max_cols=max(widths), prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    for call, nv in enumerate(widths):
        print(f"noalloc {prec} call {call}: nv={nv}", flush=True)
        x = dev(synth.gaussian((nt, nr, nv), seed=30 + nv))
        y = dev(synth.gaussian((nt, ns, nv), seed=40 + nv))
        ref_f, ref_a = op.forward(x), op.adjoint(y)
        got_f = torch.full((nt, ns, nv), np.nan, dtype=torch.float32, device="cuda")
        got_a = torch.full((nt, nr, nv), np.nan, dtype=torch.float32, device="cuda")
        mdcmod.mdc_apply_noalloc(op.handle, 0, x, got_f, nv)
        mdcmod.mdc_apply_noalloc(op.handle, 1, y, got_a, nv)
        torch.cuda.synchronize()
        assert torch.equal(got_f, ref_f)
        assert torch.equal(got_a, ref_a)
    op.close()


def test_noalloc_refuses_sizes_beyond_the_scratch(mdcmod):
    nt, nfmax, n = 128, 60, 1000
    op = mdcmod.MdcOp(nt, nfmax, n, n, max_cols=1)
    per_col = nfmax * 2 * n * 8
    nv = mdcmod.MDC_NOALLOC_SCRATCH_BYTES // per_col + 1
    x = torch.zeros((nt, n, nv), dtype=torch.float32, device="cuda")
    y = torch.zeros((nt, n, nv), dtype=torch.float32, device="cuda")
    with pytest.raises(mdcmod.MdcError) as ei:
        mdcmod.mdc_apply_noalloc(op.handle, 0, x, y, nv)
    assert ei.value.status == mdcmod.MDC_ENOMEM and "static scratch" in str(ei.value)
    op.close()
