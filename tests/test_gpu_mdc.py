"""GPU parity of the MDC operator against the FP64 oracle (through the C-ABI).

Tolerance (FP32 path): max-norm relative error <= 1e-5, i.e.
max|y_gpu - y_ref| <= 1e-5 * max|y_ref|; the FP32 arithmetic (kernel rounded
once, FFT with FP32 twiddles, FP32 accumulation) lands near 1e-6.
"""
import numpy as np
import pytest
import torch

from oracle import mdc as om
from paper_2011_11120_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def mdcmod(gpu):
    from paper_2011_11120_amd import mdc
    return mdc


def make_op(mdcmod, K, nt, max_cols=1):
    nf, ns, nr = K.shape
    op = mdcmod.MdcOp(nt, nf, ns, nr, max_cols=max_cols)
    op.set_kernel(dev(K, torch.complex64))
    return op


def _c1(nfmax):
    nt, dt, dx = 64, 0.004, 20.0
    G = synth.c1_time_kernel(nt=nt, nx=8, dt=dt, dx=dx)
    return nt, np.fft.rfft(dt * dx * dx * G, axis=0)[:nfmax]


@pytest.mark.parametrize("nfmax", [33, 20])
def test_c1_forward_adjoint(mdcmod, nfmax):
    nt, K = _c1(nfmax)
    print(f"c1 nfmax={nfmax}", flush=True)
    op = make_op(mdcmod, K, nt)
    x = synth.ricker_spikes(nt, 64, 1)
    y = synth.gaussian((nt, 64, 1))
    yg = host(op.forward(dev(x)))
    xg = host(op.adjoint(dev(y)))
    assert relmax(yg, om.mdc_forward(K, x)) < TOL
    assert relmax(xg, om.mdc_adjoint(K, y)) < TOL


# (nt, nfmax, ns, nr, nv): ragged row groups, column tiles, chunk boundaries, several column groups
SHAPES = [
    (16, 9, 5, 2, 1),
    (32, 17, 33, 66, 1),
    (64, 20, 48, 36, 1),
    (128, 65, 130, 98, 3),
    (256, 100, 203, 300, 2),
    (512, 40, 17, 4098, 1),     # more than one LDS chunk of X in the forward product
    (512, 40, 4100, 18, 1),     # more than one LDS chunk of Y in the adjoint product
    (1024, 60, 70, 130, 4),
    (2048, 30, 20, 32, 1),
    (64, 33, 40, 40, 8),
    (64, 20, 40, 40, 13),       # 8 + 5 column groups
    (128, 30, 70, 94, 6),       # one streaming pass of 6 columns
    (64, 20, 45, 37, 7),        # one streaming pass of 7 columns, odd nr
    (64, 25, 25, 25, 1),        # odd nr: padded rows
    (128, 40, 31, 129, 3),      # odd nr, ragged column tile
    (128, 30, 90, 258, 5),
    (128, 40, 1030, 1030, 9),   # wide FFT blocks, n*nv not a multiple of 4 (scalar FFT path)
    (64, 20, 2050, 2050, 4),    # wide FFT blocks, vector path, ragged last block
    (512, 100, 64, 72, 132),    # wide FFT tiles at nt = 512 (n * nv >= 8192), GEMM with a ragged column tile
    (1024, 200, 64, 64, 130),   # wide FFT tiles at nt = 1024
    (2048, 300, 40, 33, 260),   # wide FFT tiles at nt = 2048
]


@pytest.mark.parametrize("shape", SHAPES)
def test_random_kernels_match_oracle(mdcmod, shape):
    nt, nfmax, ns, nr, nv = shape
    print(f"shape {shape}", flush=True)
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=nt + ns)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, nr, nv), seed=3)
    y = synth.gaussian((nt, ns, nv), seed=4)
    yg = host(op.forward(dev(x)))
    xg = host(op.adjoint(dev(y)))
    assert relmax(yg, om.mdc_forward(K, x)) < TOL
    assert relmax(xg, om.mdc_adjoint(K, y)) < TOL


def test_unaligned_vectors_use_scalar_path(mdcmod):
    nt, nfmax, n, nv = 64, 20, 40, 2
    K = synth.random_complex_kernel(nfmax, n, n, seed=14)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, n, nv), seed=15)
    buf = torch.zeros(x.size + 1, dtype=torch.float32, device="cuda")
    xin = buf[1:]
    xin.copy_(dev(x).reshape(-1))
    obuf = torch.zeros(x.size + 1, dtype=torch.float32, device="cuda")
    yout = obuf[1:]
    mdcmod.mdc_forward(op.handle, xin, yout, nv)
    assert relmax(host(yout).reshape(nt, n, nv), om.mdc_forward(K, x)) < TOL


def test_gpu_dot_product_test(mdcmod):
    nt, nfmax, ns, nr, nv = 256, 80, 96, 130, 3
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=5)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, nr, nv), seed=6)
    y = synth.gaussian((nt, ns, nv), seed=7)
    lhs = np.vdot(host(op.forward(dev(x))), y)
    rhs = np.vdot(x, host(op.adjoint(dev(y))))
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_columns_match_single_column_applies(mdcmod):
    nt, nfmax, n, nv = 128, 40, 64, 6
    K = synth.random_complex_kernel(nfmax, n, n, seed=8)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, n, nv), seed=9)
    Y = host(op.forward(dev(x)))
    for v in range(nv):
        yv = host(op.forward(dev(x[:, :, v:v + 1])))
        assert relmax(yv[:, :, 0], Y[:, :, v]) < 1e-6


def test_deterministic(mdcmod):
    nt, nfmax, n = 256, 100, 300
    K = synth.random_complex_kernel(nfmax, n, n, seed=10)
    op = make_op(mdcmod, K, nt, max_cols=2)
    y = dev(synth.gaussian((nt, n, 2), seed=11))
    a = op.adjoint(y).clone()
    b = op.adjoint(y).clone()
    assert torch.equal(a, b)


def test_scale_and_column_weights(mdcmod):
    nt, nfmax, n = 64, 20, 12
    K = synth.random_complex_kernel(nfmax, n, n, seed=12)
    w = 1.0 + np.arange(n) / n
    op = mdcmod.MdcOp(nt, nfmax, n, n)
    op.set_kernel(dev(K, torch.complex64), scale=2.5, col_weight=dev(w))
    x = synth.gaussian((nt, n, 1), seed=13)
    ref = om.mdc_forward(2.5 * K * w[None, None, :], x)
    assert relmax(host(op.forward(dev(x))), ref) < TOL


def test_errors_raise(mdcmod):
    nt, nfmax, n = 64, 20, 12
    K = synth.random_complex_kernel(nfmax, n, n)
    op = make_op(mdcmod, K, nt, max_cols=2)
    x = dev(synth.gaussian((nt, n, 3)))
    y = torch.empty((nt, n, 3), device="cuda")
    with pytest.raises(mdcmod.MdcError) as ei:
        mdcmod.mdc_forward(op.handle, x, y, 3)
    assert ei.value.status == mdcmod.MDC_EINVAL
    fresh = mdcmod.MdcOp(nt, nfmax, n, n)
    with pytest.raises(mdcmod.MdcError):
        fresh.forward(dev(synth.gaussian((nt, n, 1))))


# ---------------------------------------------------------------- c2 size ----
C2 = dict(nt=512, nfmax=150, nx=40)


def c2_spec():
    return synth.KernelSpec(nt=C2["nt"], nfmax=C2["nfmax"], nx=C2["nx"])


def c2_input(spec, nv=1):
    gx, gy = synth.grid_xy(spec.nx, spec.nx, spec.dx)
    c = (spec.nx - 1) * spec.dx / 2
    td = synth.direct_traveltime(gx, gy, np.full(nv, c), np.full(nv, c), np.full(nv, 650.0), 2400.0)
    return synth.direct_focusing(spec.nt, td, spec.dt)


@pytest.fixture(scope="module")
def c2op(mdcmod):
    spec = c2_spec()
    op = mdcmod.MdcOp(spec.nt, spec.nfmax, spec.n, spec.n, max_cols=1)
    op.synth_kernel(spec)
    return spec, op


def test_device_generator_matches_host_generator(mdcmod, c2op):
    spec, op = c2op
    rng = np.random.default_rng(0)
    fs = rng.integers(0, spec.nfmax, 64)
    ss = rng.integers(0, spec.n, 64)
    rs = rng.integers(0, spec.n, 64)
    for f, s, r in zip(fs, ss, rs):
        ref = synth.kernel_block(spec, [f], [s], [r])[0, 0, 0]
        got = mdcmod.mdc_kernel_element(op.handle, int(f), int(s), int(r))
        assert abs(got - ref) <= 1.2e-7 * abs(ref) + 1e-30


def test_c2_full_size_sampled_rows_and_columns(c2op):
    """Full c2 apply (the configuration the benchmark times) vs the oracle on sampled traces."""
    spec, op = c2op
    x = c2_input(spec)
    y_in = synth.gaussian((spec.nt, spec.n, 1), seed=2)
    yg = host(op.forward(dev(x)))
    xg = host(op.adjoint(dev(y_in)))
    idx = np.array([0, 1, 39, 40, 799, 800, 1234, 1598, 1599])
    allf = np.arange(spec.nfmax)
    allr = np.arange(spec.n)
    Krows = synth.kernel_block(spec, allf, idx, allr)
    yref = om.mdc_forward(Krows, x)
    assert relmax(yg[:, idx], yref) < TOL
    Kcols = synth.kernel_block(spec, allf, allr, idx)
    xref = om.mdc_adjoint(Kcols, y_in)
    assert relmax(xg[:, idx], xref) < TOL


def test_c2_dot_product(c2op):
    spec, op = c2op
    x = synth.gaussian((spec.nt, spec.n, 1), seed=5)
    y = synth.gaussian((spec.nt, spec.n, 1), seed=6)
    lhs = np.vdot(host(op.forward(dev(x))), y)
    rhs = np.vdot(x, host(op.adjoint(dev(y))))
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


# ------------------------------------------------------- matrix-core path ----
GEMM_SHAPES = [
    (64, 20, 40, 40, 9),        # just above the streaming range
    (64, 25, 130, 66, 16),      # ragged 128-row tile, ragged 16-column slab
    (128, 40, 129, 257, 33),    # odd nr (padded rows), ragged everything
    (256, 60, 300, 200, 64),    # one full 64-column tile
    (128, 30, 200, 130, 65),    # two column tiles, second with one column
    (64, 20, 17, 300, 130),     # three column tiles, tiny ns
    (64, 16, 256, 128, 24),     # whole 128-row tiles in both directions (no idle waves)
]


@pytest.mark.parametrize("shape", GEMM_SHAPES)
def test_gemm_kernels_match_oracle(mdcmod, shape):
    nt, nfmax, ns, nr, nv = shape
    print(f"gemm shape {shape}", flush=True)
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=nt + nr)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, nr, nv), seed=3)
    y = synth.gaussian((nt, ns, nv), seed=4)
    yg = host(op.forward(dev(x)))
    xg = host(op.adjoint(dev(y)))
    assert relmax(yg, om.mdc_forward(K, x)) < TOL
    assert relmax(xg, om.mdc_adjoint(K, y)) < TOL


@pytest.mark.parametrize("nv", [1, 3, 8])
def test_gemm_forced_for_few_columns(mdcmod, monkeypatch, nv):
    """The matrix-core kernels on column counts the streaming kernels normally take."""
    monkeypatch.setenv("MDC_PRODUCT", "gemm")
    nt, nfmax, ns, nr = 128, 40, 150, 98
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=21)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, nr, nv), seed=5)
    y = synth.gaussian((nt, ns, nv), seed=6)
    assert relmax(host(op.forward(dev(x))), om.mdc_forward(K, x)) < TOL
    assert relmax(host(op.adjoint(dev(y))), om.mdc_adjoint(K, y)) < TOL


@pytest.mark.parametrize("nv", [9, 24])
def test_gemv_forced_for_many_columns(mdcmod, monkeypatch, nv):
    monkeypatch.setenv("MDC_PRODUCT", "gemv")
    nt, nfmax, n = 64, 20, 70
    K = synth.random_complex_kernel(nfmax, n, n, seed=22)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, n, nv), seed=7)
    assert relmax(host(op.forward(dev(x))), om.mdc_forward(K, x)) < TOL


# ---------------------------------------------------------------- c3 size ----
# per-apply max-norm bounds of the storage formats (FP32: the FP32 path's 1e-5)
C3_TOL = {"fp32": TOL, "bf16x2": 2e-5, "fp16s": 2e-3, "bf16": 8e-3, "fp16": 2e-3}


@pytest.mark.parametrize("prec", ["fp32", "bf16x2", "fp16s", "bf16", "fp16"])
def test_c3_full_size_sampled(mdcmod, prec):
    """nt=1024, nfmax=300, ns=nr=3600, nv=64 on the matrix cores, every storage format; sampled
    (trace, point) pairs of the forward and adjoint against the FP64 oracle."""
    spec = synth.KernelSpec(nt=1024, nfmax=300, nx=60)
    n, nv = spec.n, 64
    print(f"c3 {prec}: generating kernel on device", flush=True)
    op = mdcmod.MdcOp(spec.nt, spec.nfmax, n, n, max_cols=nv, prec=prec)
    op.synth_kernel(spec)
    x = synth.ricker_spikes(spec.nt, n, nv, dt=spec.dt)
    y_in = synth.gaussian((spec.nt, n, nv), seed=2)
    yg = op.forward(dev(x))
    xg = op.adjoint(dev(y_in))
    torch.cuda.synchronize()
    idx = np.array([0, 127, 128, 1800, 3599])
    vs = np.array([0, 31, 63])
    allf, alln = np.arange(spec.nfmax), np.arange(n)
    print("c3: oracle rows", flush=True)
    yref = om.mdc_forward(synth.kernel_block(spec, allf, idx, alln), x[:, :, vs])
    ysub = yg[:, idx][:, :, vs].cpu().numpy().astype(np.float64)
    ef = relmax(ysub, yref)
    print("c3: oracle columns", flush=True)
    xref = om.mdc_adjoint(synth.kernel_block(spec, allf, alln, idx), y_in[:, :, vs])
    xsub = xg[:, idx][:, :, vs].cpu().numpy().astype(np.float64)
    ea = relmax(xsub, xref)
    print(f"c3 {prec}: forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef < C3_TOL[prec] and ea < C3_TOL[prec]
    op.close()


@pytest.mark.parametrize("nv", [9, 33, 64, 65])
def test_gemm32_tiles_match_oracle(mdcmod, monkeypatch, nv):
    monkeypatch.setenv("MDC_PRODUCT", "gemm32")
    nt, nfmax, ns, nr = 128, 40, 150, 98
    K = synth.random_complex_kernel(nfmax, ns, nr, seed=31)
    op = make_op(mdcmod, K, nt, max_cols=nv)
    x = synth.gaussian((nt, nr, nv), seed=5)
    y = synth.gaussian((nt, ns, nv), seed=6)
    assert relmax(host(op.forward(dev(x))), om.mdc_forward(K, x)) < TOL
    assert relmax(host(op.adjoint(dev(y))), om.mdc_adjoint(K, y)) < TOL


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_autotune_table_cache_and_parity(mdcmod, tmp_path, prec):
    nt, nfmax, n, maxc = 128, 40, 130, 64
    K = synth.random_complex_kernel(nfmax, n, n, seed=32)
    op = mdcmod.MdcOp(nt, nfmax, n, n, max_cols=maxc, prec=prec)
    op.set_kernel(dev(K, torch.complex64))
    cache = tmp_path / "tune.jsonl"
    assert mdcmod.mdc_autotune(op.handle, cache) is True
    table = mdcmod.mdc_tune_table(op.handle)
    print(f"{prec} tuning table (ncols, fwd family, adj family): {table}", flush=True)
    assert [t[0] for t in table][-1] == maxc and all(f in (0, 1, 2) for t in table for f in t[1:])
    op2 = mdcmod.MdcOp(nt, nfmax, n, n, max_cols=maxc, prec=prec)
    op2.set_kernel(dev(K, torch.complex64))
    assert mdcmod.mdc_autotune(op2.handle, cache) is False
    assert mdcmod.mdc_tune_table(op2.handle) == table
    tol = 1e-5 if prec == "fp32" else 2e-3
    for nv in (1, 5, 20, 64):
        x = synth.gaussian((nt, n, nv), seed=nv)
        assert relmax(host(op.forward(dev(x))), om.mdc_forward(K, x)) < tol
        assert relmax(host(op.adjoint(dev(x))), om.mdc_adjoint(K, x)) < tol
