"""Seeded synthetic inputs for the MDC / Marchenko / LSQR path (host, FP64).

This module generates *inputs* only: acquisition geometry, Ricker wavelets,
hyperbolic-event kernels, focusing functions, window onsets and decimation
masks.  It holds none of the operator's arithmetic (no DFT of the input
vector, no per-frequency product, no inverse transform, no solver), so the
FP64 oracle and the HIP path can both draw their inputs from it without
sharing any of the method.

The paper's finite-difference dataset (Benchmarking section, Table 1) is not
available; these generators stand in for it with the same structure:
co-located square source/receiver grids, reflection kernels made of
hyperbolic events with a deconvolved (Ricker-shaped) spectrum, focusing
functions that are time-reversed direct arrivals from a subsurface point at
z_F = 650 m (MDD application section), and a 20 Hz Ricker for the input
wavelet (Benchmarking section).

Random numbers come from one counter-based generator: the SplitMix64
finaliser of Steele, Lea & Flood ("Fast splittable pseudorandom number
generators", OOPSLA 2014) keyed by (seed, stream, counter), turned into
uniforms on (0, 1) with 53 bits, and into normals by the Box-Muller
transform.  The device generator in the HIP library implements the same
published definition independently; tests compare sampled elements.
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import os
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------- RNG ----
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_STREAM_MUL = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Stream identifiers (one independent sequence per kind of draw).
STREAM_EVENT_AMP = 1
STREAM_EVENT_T0 = 2
STREAM_EVENT_V = 3
STREAM_KNOISE = 4
STREAM_C1_AMP = 5
STREAM_X_TIME = 6
STREAM_X_AMP = 7
STREAM_GAUSS = 8
STREAM_SERVE = 9

# Seeds (one per role).
SEED_KERNEL = 0
SEED_X = 1
SEED_Y = 2
SEED_SERVE = 3


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (wrapping uint64 arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def rng_bits(seed: int, stream: int, counter) -> np.ndarray:
    """64 random bits for each counter value of the (seed, stream) sequence."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = _mix64(np.uint64(seed) * _GOLDEN + np.uint64(stream + 1) * _STREAM_MUL)
        return _mix64(key + (c + np.uint64(1)) * _GOLDEN)


def rng_uniform(seed: int, stream: int, counter) -> np.ndarray:
    """Uniform double in the open interval (0, 1): ((bits >> 11) + 0.5) / 2**53."""
    b = rng_bits(seed, stream, counter) >> np.uint64(11)
    return (b.astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def rng_normal(seed: int, stream: int, index) -> np.ndarray:
    """Standard normal number `index` of the stream (Box-Muller, cosine branch).

    Normal j consumes uniforms 2j and 2j+1: sqrt(-2 ln u0) * cos(2 pi u1).
    """
    j = np.asarray(index, dtype=np.uint64)
    u0 = rng_uniform(seed, stream, j * np.uint64(2))
    u1 = rng_uniform(seed, stream, j * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


# ------------------------------------------------------------ wavelets ----
def ricker(t, fp: float) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 fp^2 t^2) exp(-pi^2 fp^2 t^2), peak at t = 0."""
    a = (np.pi * fp * np.asarray(t, dtype=np.float64)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ricker_spectrum(f, fp: float) -> np.ndarray:
    """Continuous Fourier transform of `ricker` (e^{-2 pi i f t} convention).

    W(f) = 2 f^2 / (sqrt(pi) fp^3) * exp(-f^2 / fp^2); real and non-negative.
    """
    f = np.asarray(f, dtype=np.float64)
    return 2.0 * f * f / (math.sqrt(math.pi) * fp ** 3) * np.exp(-(f * f) / (fp * fp))


# ------------------------------------------------------------ geometry ----
def grid_xy(nx: int, ny: int, dx: float = 20.0):
    """Surface lattice (ix*dx, iy*dx); trace index r = ix*ny + iy."""
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    return (ix.ravel() * dx).astype(np.float64), (iy.ravel() * dx).astype(np.float64)


def decimation_mask(nx: int, ny: int, d: int) -> np.ndarray:
    """Regular sub-sampling of an nx-by-ny trace lattice by a factor d in {1, 2, 4}.

    d = 2 keeps (ix + iy) even (quincunx), d = 4 keeps (ix - iy) = 0 mod 4.  On the
    paper's 99 x 99 grid these keep 4901 and 2451 traces, the Sub2 and Sub4 counts of
    Table 1; the areal element of a kept trace grows to d * dx^2.
    """
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ix, iy = ix.ravel(), iy.ravel()
    if d == 1:
        return np.ones(nx * ny, dtype=bool)
    if d == 2:
        return (ix + iy) % 2 == 0
    if d == 4:
        return (ix - iy) % 4 == 0
    raise ValueError("decimation factor must be 1, 2 or 4")


def virtual_points(nx: int, ny: int, dx: float, px: int, py: int, dpx: float = 20.0,
                   zf: float = 650.0):
    """px-by-py focusing points at depth zf on a dpx grid centred under the array."""
    cx = (nx - 1) * dx / 2.0
    cy = (ny - 1) * dx / 2.0
    ax = cx + (np.arange(px) - (px - 1) / 2.0) * dpx
    ay = cy + (np.arange(py) - (py - 1) / 2.0) * dpx
    gx, gy = np.meshgrid(ax, ay, indexing="ij")
    return gx.ravel(), gy.ravel(), np.full(px * py, zf)


def direct_traveltime(rx, ry, vx, vy, vz, c: float):
    """Straight-ray traveltime [n, nv] from each surface trace to each virtual point."""
    h2 = (rx[:, None] - vx[None, :]) ** 2 + (ry[:, None] - vy[None, :]) ** 2
    return np.sqrt(h2 + vz[None, :] ** 2) / c


# -------------------------------------------------------------- events ----
@dataclass
class Events:
    """Hyperbolic reflection events tau_k(h) = sqrt(t0_k^2 + h^2 / v_k^2)."""
    amp: np.ndarray
    t0: np.ndarray
    v: np.ndarray


def make_events(nev: int, T: float, seed: int = SEED_KERNEL, t0_lo: float = 0.15, t0_hi: float = 0.5) -> Events:
    """nev events: amplitudes N(0,1); t0 ~ U(t0_lo T, t0_hi T) and v ~ U(1500, 3000) m/s, both sorted."""
    k = np.arange(nev)
    amp = rng_normal(seed, STREAM_EVENT_AMP, k)
    t0 = np.sort(T * (t0_lo + (t0_hi - t0_lo) * rng_uniform(seed, STREAM_EVENT_T0, k)))
    v = np.sort(1500.0 + 1500.0 * rng_uniform(seed, STREAM_EVENT_V, k))
    return Events(amp, t0, v)


def event_times(ev: Events, sx, sy, rx, ry) -> np.ndarray:
    """tau[k, s, r] for the given source and receiver coordinates."""
    h2 = (sx[:, None] - rx[None, :]) ** 2 + (sy[:, None] - ry[None, :]) ** 2
    return np.sqrt(ev.t0[:, None, None] ** 2 + h2[None] / ev.v[:, None, None] ** 2)


# -------------------------------------------------------- kernel specs ----
@dataclass
class KernelSpec:
    """Frequency-domain synthetic reflection kernel on a co-located square grid.

    K[f, s, r] = kappa * dA * W(f_f) * sum_k a_k exp(-2 pi i f_f tau_k(s, r))
                 + noise * sigma_f * (n1 + i n2) / sqrt(2)
    with f_f = f / (nt dt), W the Ricker spectrum at fp, sigma_f = kappa dA W(f_f)
    sqrt(sum a_k^2) and (n1, n2) the normals 2q and 2q+1 of the noise stream at
    q = (f*n + s)*n + r (full-grid indices).  This is dA times the band-limited
    spectrum of sum_k a_k w(t - tau_k), i.e. dt*dA*DFT of the sampled traces for
    events well inside the record.
    """
    nt: int
    nfmax: int
    nx: int
    dt: float = 0.004
    dx: float = 20.0
    nev: int = 20
    fp: float = 15.0
    noise: float = 0.05
    kappa: float = 1.0
    seed: int = SEED_KERNEL
    area_scale: float = 1.0
    t0_lo: float = 0.15
    t0_hi: float = 0.5
    events: Events = field(default=None)

    def __post_init__(self):
        if self.events is None:
            self.events = make_events(self.nev, self.nt * self.dt, self.seed, self.t0_lo, self.t0_hi)

    @property
    def n(self) -> int:
        return self.nx * self.nx

    @property
    def dA(self) -> float:
        """Areal element of a trace: dx^2, times d for a grid decimated by d."""
        return self.dx * self.dx * self.area_scale


def kernel_block(spec: KernelSpec, f_idx, s_idx, r_idx) -> np.ndarray:
    """K[f, s, r] (complex128) on the outer product of the given full-grid indices."""
    f_idx = np.atleast_1d(np.asarray(f_idx, dtype=np.int64))
    s_idx = np.atleast_1d(np.asarray(s_idx, dtype=np.int64))
    r_idx = np.atleast_1d(np.asarray(r_idx, dtype=np.int64))
    gx, gy = grid_xy(spec.nx, spec.nx, spec.dx)
    tau = event_times(spec.events, gx[s_idx], gy[s_idx], gx[r_idx], gy[r_idx])  # [k,s,r]
    ev = spec.events
    out = np.empty((f_idx.size, s_idx.size, r_idx.size), dtype=np.complex128)
    n = spec.n
    rms = math.sqrt(float(np.sum(ev.amp ** 2)))

    def one_bin(i):
        f = f_idx[i]
        ff = f / (spec.nt * spec.dt)
        wf = spec.kappa * spec.dA * float(ricker_spectrum(ff, spec.fp))
        acc = np.zeros((s_idx.size, r_idx.size), dtype=np.complex128)
        for k in range(ev.amp.size):
            cyc = ff * tau[k]
            frac = cyc - np.floor(cyc)
            acc += ev.amp[k] * (np.cos(2 * np.pi * frac) - 1j * np.sin(2 * np.pi * frac))
        q = (np.uint64(f) * np.uint64(n) + s_idx.astype(np.uint64)[:, None]) * np.uint64(n) \
            + r_idx.astype(np.uint64)[None, :]
        n1 = rng_normal(spec.seed, STREAM_KNOISE, q * np.uint64(2))
        n2 = rng_normal(spec.seed, STREAM_KNOISE, q * np.uint64(2) + np.uint64(1))
        sig = spec.noise * wf * rms / math.sqrt(2.0)
        out[i] = wf * acc + sig * (n1 + 1j * n2)

    # bins are independent; numpy releases the GIL inside these array expressions, so large
    # blocks are generated by a few threads (the values do not depend on the thread count)
    workers = min(16, os.cpu_count() or 1, f_idx.size) if s_idx.size * r_idx.size >= 1 << 16 else 1
    if workers > 1:
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one_bin, range(f_idx.size)))
    else:
        for i in range(f_idx.size):
            one_bin(i)
    return out


def kernel_full(spec: KernelSpec) -> np.ndarray:
    """Whole K[nfmax, n, n] (only for sizes that fit comfortably on the host)."""
    idx = np.arange(spec.n)
    return kernel_block(spec, np.arange(spec.nfmax), idx, idx)


# ------------------------------------------- small time-domain kernel ----
def c1_time_kernel(nt: int = 64, nx: int = 8, dt: float = 0.004, dx: float = 20.0,
                   nev: int = 3, fp: float = 15.0, seed: int = SEED_KERNEL,
                   nx_r: int | None = None) -> np.ndarray:
    """G[t, s, r] = sum_{k<nev} a_{srk} ricker(t dt - tau_k(s, r)), a ~ N(0,1) per (s, r, k).

    Sources on an nx-by-nx grid, receivers on nx_r-by-nx_r (default nx).  Per-trace random
    amplitudes make the kernel non-symmetric, so a transposed operand cannot hide.
    """
    nx_r = nx if nx_r is None else nx_r
    T = nt * dt
    ev = make_events(nev, T, seed)
    sx, sy = grid_xy(nx, nx, dx)
    rx, ry = grid_xy(nx_r, nx_r, dx)
    tau = event_times(ev, sx, sy, rx, ry)  # [k, s, r]
    ns, nr = sx.size, rx.size
    q = (np.arange(ns)[:, None] * nr + np.arange(nr)[None, :])[None] * nev \
        + np.arange(nev)[:, None, None]
    a = rng_normal(seed, STREAM_C1_AMP, q)  # [k, s, r]
    t = np.arange(nt) * dt
    return np.einsum("ksr,tksr->tsr", a, ricker(t[:, None, None, None] - tau[None], fp))


# -------------------------------------------------- focusing functions ----
def ricker_spikes(nt: int, n: int, nv: int, dt: float = 0.004, nspk: int = 3,
                  fp: float = 20.0, seed: int = SEED_X) -> np.ndarray:
    """x[t, r, v]: nspk Ricker(fp) spikes per trace at U(0.1T, 0.9T) with N(0,1) amplitudes."""
    T = nt * dt
    j = np.arange(n * nv * nspk).reshape(n, nv, nspk)
    tj = T * (0.1 + 0.8 * rng_uniform(seed, STREAM_X_TIME, j))
    aj = rng_normal(seed, STREAM_X_AMP, j)
    t = np.arange(nt) * dt
    return np.einsum("rvj,trvj->trv", aj, ricker(t[:, None, None, None] - tj[None], fp))


def lag_seconds(nt: int, dt: float) -> np.ndarray:
    """Two-sided circular time axis: t*dt for t < nt/2, (t - nt)*dt otherwise."""
    t = np.arange(nt)
    return np.where(t < nt / 2, t, t - nt) * dt


def direct_focusing(nt: int, td: np.ndarray, dt: float = 0.004, fp: float = 20.0) -> np.ndarray:
    """f_d+[t, r, v] = ricker(lag(t) + td[r, v]): the time-reversed direct arrival."""
    lag = lag_seconds(nt, dt)
    return ricker(lag[:, None, None] + td[None], fp)


def window_onset(td: np.ndarray, dt: float = 0.004, eps: int = 6) -> np.ndarray:
    """Integer onset o[s, v] = round(td / dt) - eps of the hard Marchenko window.

    The window keeps samples with |lag(t)| < o: everything strictly before the
    direct arrival minus eps samples (about 1.5 periods of the 15 Hz wavelet).
    """
    return np.maximum(np.rint(td / dt).astype(np.int32) - eps, 0).astype(np.int32)


def gaussian(shape, seed: int = SEED_Y, stream: int = STREAM_GAUSS) -> np.ndarray:
    """N(0,1) array of the given shape (C order counter = flat index)."""
    n = int(np.prod(shape))
    return rng_normal(seed, stream, np.arange(n)).reshape(shape)


def random_complex_kernel(nfmax: int, ns: int, nr: int, seed: int = SEED_KERNEL) -> np.ndarray:
    """Dense N(0,1) complex kernel with ns != nr allowed (for transpose traps)."""
    re = gaussian((nfmax, ns, nr), seed, STREAM_KNOISE)
    im = gaussian((nfmax, ns, nr), seed + 1000, STREAM_KNOISE)
    return re + 1j * im


def irregular_subset(nx: int, ny: int, fraction: float = 0.5, seed: int = SEED_KERNEL) -> np.ndarray:
    """Sorted indices of a random `fraction` of an nx-by-ny trace lattice (irregular geometry)."""
    n = nx * ny
    keys = rng_uniform(seed, STREAM_SERVE + 1, np.arange(n))
    return np.sort(np.argsort(keys)[: int(round(fraction * n))])
