"""A served request at the full size of the served-stream workload, against the FP64 oracle.

The grid is 100 x 100 traces (nt = 1024, nfmax = 200, kernel scale of that workload).  The checked
request has 5 focusing points, decimation 4 and 10 LSQR iterations; it shares the server with
wider requests so that its lattice level's steps run the matrix-core product (up to 42 columns)
and the wide-tile transforms of the full-size run, and its 12500 traces per block fill the last
16-trace tile of its tiled vectors only partly (padding traces).  Its solution on the 2500-trace lattice and its
phibar history are compared with the oracle's LSQR on the same decimated problem: FP32 to 1e-5,
FP16S to the 1e-3 model-error budget.  The FP32 run also solves the request alone on the full
grid (zero traces off the lattice) and checks that it equals the lattice-level solution.
"""
import time

import numpy as np
import pytest
import torch

from oracle import lsqr as ol
from oracle import marchenko as omc
from oracle import mdc as om
from paper_2011_11120_amd import synth, workloads

pytestmark = pytest.mark.gpu

NX, NT, NF = 100, 1024, 200


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def mdcmod(gpu):
    from paper_2011_11120_amd import mdc
    return mdc


def checked_points():
    vx, vy, vz = synth.virtual_points(NX, NX, 20.0, 8, 8)
    return vx[:5], vy[:5], vz[:5]


@pytest.fixture(scope="module")
def oracle_c5():
    """FP64 oracle LSQR of the checked request on its lattice (host: about two minutes)."""
    t0 = time.perf_counter()
    kap = workloads.kappa("c5")
    spec = workloads.marchenko_spec(nx=NX, nt=NT, nfmax=NF, d=4, kappa_value=kap)
    vx, vy, vz = checked_points()
    idx, onset, fd = workloads.serve_request_inputs(NX, NT, 4, vx, vy, vz)
    K = synth.kernel_block(spec, np.arange(NF), idx, idx)
    Kc = np.conj(K)
    print(f"c5 oracle: lattice kernel {K.shape} in {time.perf_counter() - t0:.0f} s", flush=True)
    on, f = onset[idx], fd[:, idx]
    th = omc.theta(NT, on)
    fwd = lambda v: [v[0] - th * om.mdc_forward(K, v[1]), -th * om.mdc_forward(Kc, v[0]) + v[1]]
    adj = lambda u: [u[0] - om.mdc_adjoint(Kc, th * u[1]), -om.mdc_adjoint(K, th * u[0]) + u[1]]
    d0, d1 = omc.data(K, on, f)
    x, h = ol.lsqr(fwd, adj, [d0, d1], 10)
    print(f"c5 oracle: LSQR done in {time.perf_counter() - t0:.0f} s, phibar {h[0]:.3e} -> {h[-1]:.3e}",
          flush=True)
    del K, Kc
    return kap, idx, np.stack(x), h


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp16s", 1e-3)])
def test_c5_size_served_request_matches_oracle(mdcmod, oracle_c5, prec, tol):
    kap, idx, xr, hr = oracle_c5
    torch.cuda.empty_cache()
    spec = workloads.marchenko_spec(nx=NX, nt=NT, nfmax=NF, kappa_value=kap)
    print(f"c5 {prec}: generating the {NX * NX}-trace kernel on the device", flush=True)
    op = mdcmod.MdcOp(NT, NF, NX * NX, NX * NX, max_cols=64, prec=prec)
    op.synth_kernel(spec)
    srv = mdcmod.Server(op, NX, arena_bytes=12 << 30, sublattice=4)
    vx, vy, vz = synth.virtual_points(NX, NX, 20.0, 8, 8)
    rid = srv.submit(*checked_points(), 10, 4)
    ballast = [srv.submit(vx[8:16], vy[8:16], vz[8:16], 10, 4), srv.submit(vx[16:24], vy[16:24], vz[16:24], 12, 4),
               srv.submit(vx[24:28], vy[24:28], vz[24:28], 10, 1)]
    srv.drain()
    st = srv.stats()
    assert st["completed"] == 4 and st["max_active"] >= 2
    x, h = srv.result(rid)
    xg = x.cpu().numpy().astype(np.float64)
    err = rel2(xg[:, :, idx], xr)
    eh = float(np.max(np.abs(h.cpu().numpy() - hr)) / hr[0])
    print(f"c5 {prec}: model error {err:.2e}, phibar history {eh:.2e}, {st['steps']} steps", flush=True)
    assert err < tol and eh < tol
    off = np.setdiff1d(np.arange(NX * NX), idx)
    assert np.all(xg[:, :, off] == 0)
    srv.close()
    del srv, x, h
    torch.cuda.empty_cache()
    if prec == "fp32":  # the same request alone, on the full grid with zero traces off the lattice
        full = mdcmod.Server(op, NX, arena_bytes=20 << 30, sublattice=0)
        rf = full.submit(*checked_points(), 10, 4)
        full.drain()
        ef = rel2(full.result(rf)[0].cpu().numpy().astype(np.float64), xg)
        print(f"c5 fp32: full-grid encoding vs lattice level {ef:.2e}", flush=True)
        assert ef < 1e-5
        full.close()
    op.close()
    del op
    torch.cuda.empty_cache()
