"""Synthetic workloads (inputs only) for the benchmark and the parity tests.

Each builder returns seeded inputs of the shape and structure of the paper's
experiments (co-located square grids, hyperbolic-event reflection kernels,
focusing points at z_F = 650 m, time-reversed direct arrivals, hard
direct-arrival windows, regular decimation with a d-times larger areal
element).  No operator arithmetic happens here.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np

from . import synth

# Package data: the synthetic kernel scales, written by tests/golden/make_kappa.py.
_KAPPA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "kappa.json")


def kappa(name: str) -> float:
    """Kernel scale chosen so that max_f ||K_f||_2 is about 0.5 (see tests/golden/make_kappa.py)."""
    with open(_KAPPA) as fh:
        return float(json.load(fh)[name]["kappa"])


@dataclass
class MarchenkoCase:
    spec: synth.KernelSpec
    idx: np.ndarray      # kept full-grid trace indices (sources = receivers)
    onset: np.ndarray    # [n_d, nv] int32
    fd: np.ndarray       # [nt, n_d, nv] direct focusing function
    td: np.ndarray       # [n_d, nv] direct-arrival times

    @property
    def n(self) -> int:
        return int(self.idx.size)

    @property
    def nv(self) -> int:
        return int(self.onset.shape[1])


# Zero-offset times of the reflection events of the Marchenko workloads, as fractions of the
# record length T = nt dt: U(0.02 T, 0.25 T) = 0.08 - 1.0 s at nt = 1024, dt = 4 ms, so part of
# the reflected energy (the overburden above the 650 m focusing level) arrives before the direct
# arrival from the focusing points (0.33 - 0.45 s) and falls inside the window Theta.
MARCHENKO_T0 = (0.02, 0.25)


def marchenko_spec(nx=50, nt=1024, nfmax=250, d=1, kappa_value=1.0, dt=0.004, dx=20.0) -> synth.KernelSpec:
    return synth.KernelSpec(nt=nt, nfmax=nfmax, nx=nx, dt=dt, dx=dx, kappa=kappa_value, area_scale=float(d),
                            t0_lo=MARCHENKO_T0[0], t0_hi=MARCHENKO_T0[1])


def marchenko_case(nx=50, nt=1024, nfmax=250, d=1, px=8, py=4, kappa_value=1.0, c=2000.0,
                   dt=0.004, dx=20.0, eps=6) -> MarchenkoCase:
    """Receiver-side redatuming problem of Eq.5 on an nx-by-nx grid decimated by d."""
    spec = marchenko_spec(nx, nt, nfmax, d, kappa_value, dt, dx)
    idx = np.nonzero(synth.decimation_mask(nx, nx, d))[0]
    gx, gy = synth.grid_xy(nx, nx, dx)
    vx, vy, vz = synth.virtual_points(nx, nx, dx, px, py)
    td = synth.direct_traveltime(gx[idx], gy[idx], vx, vy, vz, c)
    onset = synth.window_onset(td, dt, eps)
    fd = synth.direct_focusing(nt, td, dt)
    return MarchenkoCase(spec, idx, onset, fd, td)


def serve_request_inputs(nx, nt, decim, vx, vy, vz, dx=20.0, dt=0.004, c=2000.0, eps=6, fp=20.0):
    """Host twin of the server's per-request inputs on the full grid.

    Returns (idx, onset, fd): kept trace indices of the decimation lattice, and the onsets
    [n, nv] and initial focusing functions [nt, n, nv] on the full grid (zero off the lattice).
    """
    n = nx * nx
    keep = synth.decimation_mask(nx, nx, decim)
    gx, gy = synth.grid_xy(nx, nx, dx)
    td = synth.direct_traveltime(gx, gy, np.asarray(vx, float), np.asarray(vy, float), np.asarray(vz, float), c)
    onset = synth.window_onset(td, dt, eps)
    onset[~keep] = 0
    fd = synth.direct_focusing(nt, td, dt, fp)
    fd[:, ~keep] = 0.0
    return np.nonzero(keep)[0], onset.astype(np.int32), fd
