"""ctypes binding of libmdcgpu.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts PyTorch
device tensors into raw pointers and the current HIP stream into a handle,
and raises when a call fails.  PyTorch provides device memory and streams.
If the library has not been built, importing the binding raises: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdcgpu.so")

MDC_OK, MDC_EINVAL, MDC_ENOMEM, MDC_EDEVICE, MDC_EBUSY, MDC_ENOTREADY, MDC_ECANCELED, MDC_ENOTSUP = \
    0, -1, -2, -3, -4, -5, -6, -7
MDC_FP32, MDC_FP16S, MDC_BF16, MDC_BF16X2, MDC_FP16 = 0, 1, 2, 3, 4
MDC_OP_MDC, MDC_OP_MARCHENKO = 0, 1
MDC_NOALLOC_SCRATCH_BYTES = 64 << 20  # static scratch of mdc_apply_noalloc (include/mdc.h)
PREC = {"fp32": MDC_FP32, "fp16s": MDC_FP16S, "bf16": MDC_BF16, "bf16x2": MDC_BF16X2, "fp16": MDC_FP16}


class MdcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class mdc_desc(C.Structure):
    _fields_ = [("nt", C.c_int), ("nfmax", C.c_int), ("ns", C.c_int), ("nr", C.c_int),
                ("max_cols", C.c_int), ("prec", C.c_int)]


class mdc_synth_desc(C.Structure):
    _fields_ = [("nx", C.c_int), ("dt", C.c_double), ("dx", C.c_double), ("fp", C.c_double),
                ("kappa", C.c_double), ("noise", C.c_double), ("area", C.c_double),
                ("seed", C.c_uint64), ("nev", C.c_int),
                ("amp", C.POINTER(C.c_double)), ("t0", C.POINTER(C.c_double)),
                ("vel", C.POINTER(C.c_double)),
                ("s_index", C.c_void_p), ("r_index", C.c_void_p)]


class lsqr_desc(C.Structure):
    _fields_ = [("kind", C.c_int), ("nv", C.c_int), ("niter", C.c_int), ("onset", C.c_void_p)]


class serve_geometry(C.Structure):
    _fields_ = [("nx", C.c_int), ("dx", C.c_double), ("dt", C.c_double), ("c", C.c_double),
                ("eps", C.c_int), ("fp", C.c_double), ("sublattice", C.c_int)]


class serve_req(C.Structure):
    _fields_ = [("nv", C.c_int), ("niter", C.c_int), ("decim", C.c_int),
                ("vx", C.POINTER(C.c_double)), ("vy", C.POINTER(C.c_double)), ("vz", C.POINTER(C.c_double)),
                ("x_out", C.c_void_p), ("hist", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2011_11120_amd.build (no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i, d, st = C.c_void_p, C.c_int, C.c_double, C.c_int
    sig = {
        "mdc_last_error": (C.c_char_p, []),
        "mdc_query_sizes": (st, [C.POINTER(mdc_desc), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "mdc_create": (st, [C.POINTER(mdc_desc), vp, vp, vp, C.POINTER(vp)]),
        "mdc_set_kernel": (st, [vp, vp, d, vp, vp]),
        "mdc_synth_kernel": (st, [vp, C.POINTER(mdc_synth_desc), vp]),
        "mdc_kernel_element": (st, [vp, i, i, i, vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
        "mdc_forward": (st, [vp, vp, vp, i, vp]),
        "mdc_adjoint": (st, [vp, vp, vp, i, vp]),
        "mdc_apply_noalloc": (st, [vp, i, vp, vp, i, vp]),
        "mch_forward": (st, [vp, vp, i, vp, vp, vp, vp, vp]),
        "mch_adjoint": (st, [vp, vp, i, vp, vp, vp, vp, vp]),
        "mch_data": (st, [vp, vp, i, vp, vp, vp, vp]),
        "mdc_profile": (st, [vp, i]),
        "mdc_profile_read": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
        "mdc_destroy": (st, [vp]),
        "mdc_autotune": (st, [vp, C.c_char_p, vp, C.POINTER(C.c_int)]),
        "mdc_tune_table": (st, [vp, i, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int)]),
        "lsqr_query_sizes": (st, [vp, C.POINTER(lsqr_desc), C.POINTER(C.c_size_t)]),
        "lsqr_solve": (st, [vp, C.POINTER(lsqr_desc), vp, vp, vp, vp, C.c_size_t, vp]),
        "cgls_solve": (st, [vp, C.POINTER(lsqr_desc), vp, vp, vp, vp, C.c_size_t, vp]),
        "mdc_set_kernel_time": (st, [vp, vp, i, d, vp, vp, C.c_size_t, vp]),
        "mch_greens": (st, [vp, i, vp, vp, vp, vp, vp, vp]),
        "mch_neumann_query": (st, [vp, i, C.POINTER(C.c_size_t)]),
        "mch_neumann": (st, [vp, vp, i, vp, vp, i, vp, C.c_size_t, vp]),
        "serve_request_bytes": (st, [vp, i, C.POINTER(C.c_size_t)]),
        "serve_level_bytes": (st, [vp, i, C.POINTER(C.c_size_t)]),
        "serve_phase_stats": (st, [vp, C.POINTER(C.c_long), C.POINTER(C.c_long), C.POINTER(C.c_double)]),
        "serve_create": (st, [vp, C.POINTER(serve_geometry), vp, C.c_size_t, C.POINTER(vp)]),
        "serve_submit": (st, [vp, C.POINTER(serve_req), C.POINTER(C.c_uint64)]),
        "serve_poll": (st, [vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
        "serve_cancel": (st, [vp, C.c_uint64]),
        "serve_drain": (st, [vp]),
        "serve_stats": (st, [vp, i, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                             C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_long)]),
        "serve_graph_stats": (st, [vp, C.POINTER(C.c_long), C.POINTER(C.c_long)]),
        "serve_destroy": (st, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTS = ("mdc_last_error", "mdc_query_sizes", "mdc_create", "mdc_set_kernel", "mdc_synth_kernel",
           "mdc_kernel_element", "mdc_forward", "mdc_adjoint", "mdc_apply_noalloc", "mch_forward", "mch_adjoint", "mch_data",
           "mdc_profile", "mdc_profile_read", "mdc_destroy", "mdc_autotune", "mdc_tune_table",
           "lsqr_query_sizes", "lsqr_solve", "cgls_solve", "mdc_set_kernel_time", "mch_greens",
           "mch_neumann_query", "mch_neumann",
           "serve_request_bytes", "serve_level_bytes", "serve_create", "serve_submit", "serve_poll",
           "serve_cancel", "serve_drain", "serve_stats", "serve_phase_stats", "serve_graph_stats", "serve_destroy")


def _check(status: int):
    if status != MDC_OK:
        raise MdcError(status, _lib.mdc_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ----------------------------------------------------------- same-name API ----
def mdc_last_error() -> str:
    return _lib.mdc_last_error().decode()


def mdc_query_sizes(desc: mdc_desc):
    res, work = C.c_size_t(0), C.c_size_t(0)
    _check(_lib.mdc_query_sizes(C.byref(desc), C.byref(res), C.byref(work)))
    return res.value, work.value


def mdc_create(desc: mdc_desc, resident, workspace, stream=None):
    h = C.c_void_p()
    _check(_lib.mdc_create(C.byref(desc), _ptr(resident), _ptr(workspace), _stream(stream), C.byref(h)))
    return h


def mdc_set_kernel(h, K, scale=1.0, col_weight=None, stream=None):
    _check(_lib.mdc_set_kernel(h, _ptr(K), float(scale), _ptr(col_weight), _stream(stream)))


def mdc_synth_kernel(h, sd: mdc_synth_desc, stream=None):
    _check(_lib.mdc_synth_kernel(h, C.byref(sd), _stream(stream)))


def mdc_kernel_element(h, f, s, r, stream=None):
    re, im = C.c_float(), C.c_float()
    _check(_lib.mdc_kernel_element(h, f, s, r, _stream(stream), C.byref(re), C.byref(im)))
    return complex(re.value, im.value)


def mdc_forward(h, x, y, nv, stream=None):
    _check(_lib.mdc_forward(h, _ptr(x), _ptr(y), int(nv), _stream(stream)))


def mdc_adjoint(h, y, x, nv, stream=None):
    _check(_lib.mdc_adjoint(h, _ptr(y), _ptr(x), int(nv), _stream(stream)))


def mdc_apply_noalloc(h, adjoint, x, y, nv, stream=None):
    _check(_lib.mdc_apply_noalloc(h, 1 if adjoint else 0, _ptr(x), _ptr(y), int(nv), _stream(stream)))


def mch_forward(h, onset, nv, in0, in1, out0, out1, stream=None):
    _check(_lib.mch_forward(h, _ptr(onset), int(nv), _ptr(in0), _ptr(in1), _ptr(out0), _ptr(out1),
                            _stream(stream)))


def mch_adjoint(h, onset, nv, in0, in1, out0, out1, stream=None):
    _check(_lib.mch_adjoint(h, _ptr(onset), int(nv), _ptr(in0), _ptr(in1), _ptr(out0), _ptr(out1),
                            _stream(stream)))


def mch_data(h, onset, nv, fd, d0, d1, stream=None):
    _check(_lib.mch_data(h, _ptr(onset), int(nv), _ptr(fd), _ptr(d0), _ptr(d1), _stream(stream)))


def mdc_profile(h, enable: bool):
    _check(_lib.mdc_profile(h, 1 if enable else 0))


def mdc_profile_read(h):
    ms = (C.c_double * 4)()
    cnt = (C.c_int * 4)()
    _check(_lib.mdc_profile_read(h, ms, cnt))
    return list(ms), list(cnt)


def mdc_autotune(h, cache_path=None, stream=None) -> bool:
    """Returns True when the table was measured, False when it came from the cache."""
    m = C.c_int(0)
    _check(_lib.mdc_autotune(h, None if cache_path is None else str(cache_path).encode(), _stream(stream),
                             C.byref(m)))
    return bool(m.value)


def mdc_tune_table(h):
    cnt = C.c_int(0)
    _check(_lib.mdc_tune_table(h, 0, C.byref(cnt), None, None, None))
    n = cnt.value
    a, b, c = (C.c_int * max(n, 1))(), (C.c_int * max(n, 1))(), (C.c_int * max(n, 1))()
    _check(_lib.mdc_tune_table(h, n, C.byref(cnt), a, b, c))
    return [(a[i], b[i], c[i]) for i in range(n)]


def mdc_destroy(h):
    _check(_lib.mdc_destroy(h))


def lsqr_query_sizes(h, ld: lsqr_desc) -> int:
    n = C.c_size_t(0)
    _check(_lib.lsqr_query_sizes(h, C.byref(ld), C.byref(n)))
    return n.value


def lsqr_solve(h, ld: lsqr_desc, b, x, hist, work, stream=None):
    _check(_lib.lsqr_solve(h, C.byref(ld), _ptr(b), _ptr(x), _ptr(hist), _ptr(work),
                           C.c_size_t(work.numel() * work.element_size()), _stream(stream)))


def cgls_solve(h, ld: lsqr_desc, b, x, hist, work, stream=None):
    _check(_lib.cgls_solve(h, C.byref(ld), _ptr(b), _ptr(x), _ptr(hist), _ptr(work),
                           C.c_size_t(work.numel() * work.element_size()), _stream(stream)))


def mdc_set_kernel_time(h, g, conj=False, scale=1.0, col_weight=None, temp=None, stream=None):
    nb = 0 if temp is None else temp.numel() * temp.element_size()
    _check(_lib.mdc_set_kernel_time(h, _ptr(g), 1 if conj else 0, float(scale), _ptr(col_weight), _ptr(temp),
                                    C.c_size_t(nb), _stream(stream)))


def mch_greens(h, nv, fminus, fd, fm, gminus, gplus_conj, stream=None):
    _check(_lib.mch_greens(h, int(nv), _ptr(fminus), _ptr(fd), _ptr(fm), _ptr(gminus), _ptr(gplus_conj),
                           _stream(stream)))


def mch_neumann_query(h, nv) -> int:
    n = C.c_size_t(0)
    _check(_lib.mch_neumann_query(h, int(nv), C.byref(n)))
    return n.value


def mch_neumann(h, onset, nv, d, f, nterms, work, stream=None):
    _check(_lib.mch_neumann(h, _ptr(onset), int(nv), _ptr(d), _ptr(f), int(nterms), _ptr(work),
                            C.c_size_t(work.numel() * work.element_size()), _stream(stream)))


def serve_request_bytes(h, nv) -> int:
    n = C.c_size_t(0)
    _check(_lib.serve_request_bytes(h, int(nv), C.byref(n)))
    return n.value


def serve_level_bytes(h, decim) -> int:
    n = C.c_size_t(0)
    _check(_lib.serve_level_bytes(h, int(decim), C.byref(n)))
    return n.value


def serve_phase_stats(srv):
    rs, dfr, dfs = C.c_long(), C.c_long(), C.c_double()
    _check(_lib.serve_phase_stats(srv, C.byref(rs), C.byref(dfr), C.byref(dfs)))
    return {"request_steps": rs.value, "deferred": dfr.value, "deferred_s": dfs.value}


def serve_create(h, geom: serve_geometry, arena):
    srv = C.c_void_p()
    _check(_lib.serve_create(h, C.byref(geom), _ptr(arena), C.c_size_t(arena.numel() * arena.element_size()),
                             C.byref(srv)))
    return srv


def serve_submit(srv, req: serve_req) -> int:
    rid = C.c_uint64(0)
    _check(_lib.serve_submit(srv, C.byref(req), C.byref(rid)))
    return rid.value


def serve_poll(srv, rid):
    """Returns (done, latency_s): done = 1 finished, 0 running, -1 cancelled/failed."""
    done, lat = C.c_int(0), C.c_double(0.0)
    st = _lib.serve_poll(srv, C.c_uint64(rid), C.byref(done), C.byref(lat))
    if st not in (MDC_OK, MDC_ENOTREADY, MDC_ECANCELED):
        _check(st)
    return done.value, lat.value


def serve_cancel(srv, rid):
    _check(_lib.serve_cancel(srv, C.c_uint64(rid)))


def serve_drain(srv):
    _check(_lib.serve_drain(srv))


def serve_stats(srv, skip=0):
    sps, p50, p99 = C.c_double(), C.c_double(), C.c_double()
    done, mact, steps = C.c_int(), C.c_int(), C.c_long()
    _check(_lib.serve_stats(srv, int(skip), C.byref(sps), C.byref(p50), C.byref(p99), C.byref(done),
                            C.byref(mact), C.byref(steps)))
    return {"solves_per_s": sps.value, "p50_s": p50.value, "p99_s": p99.value, "completed": done.value,
            "max_active": mact.value, "steps": steps.value}


def serve_graph_stats(srv):
    cap, rep = C.c_long(), C.c_long()
    _check(_lib.serve_graph_stats(srv, C.byref(cap), C.byref(rep)))
    return {"captured": cap.value, "replayed": rep.value}


def serve_destroy(srv):
    _check(_lib.serve_destroy(srv))


class Server:
    """Owns the arena (PyTorch) and the library server over an MdcOp."""

    def __init__(self, op, nx, arena_bytes=None, dx=20.0, dt=0.004, c=2000.0, eps=6, fp=20.0, arena=None,
                 sublattice=0):
        """sublattice: decimation levels (2, 4 or 6 for both) solved on their own lattice with a
        kernel gathered into the arena; arena_bytes counts the request slots only, the levels'
        bytes (serve_level_bytes) are added to it."""
        self.op = op
        self.nt, self.n = op.nt, op.ns
        if arena is None:
            extra = sum(serve_level_bytes(op.handle, d) for d in (2, 4) if sublattice & d)
            arena = torch.empty(int(arena_bytes) + extra, dtype=torch.uint8, device="cuda")
        self.arena = arena
        torch.cuda.synchronize()
        self.handle = serve_create(op.handle, serve_geometry(nx, dx, dt, c, eps, fp, sublattice), self.arena)
        self._keep = {}

    def submit(self, vx, vy, vz, niter, decim=1, x_out=None, hist=True):
        import numpy as np
        nv = len(vx)
        if x_out is None:
            x_out = torch.zeros((2, self.nt, self.n, nv), dtype=torch.float32, device="cuda")
        h = torch.zeros(niter + 1, dtype=torch.float64, device="cuda") if hist else None
        torch.cuda.synchronize()
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (vx, vy, vz)]
        req = serve_req(nv, niter, decim, *[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs],
                        x_out.data_ptr(), None if h is None else h.data_ptr())
        rid = serve_submit(self.handle, req)
        self._keep[rid] = (x_out, h)
        return rid

    def result(self, rid):
        return self._keep[rid]

    def release(self, rid):
        """Drop this wrapper's reference to a finished request's output buffers."""
        self._keep.pop(rid, None)

    def poll(self, rid):
        return serve_poll(self.handle, rid)

    def cancel(self, rid):
        serve_cancel(self.handle, rid)

    def drain(self):
        serve_drain(self.handle)

    def stats(self, skip=0):
        return serve_stats(self.handle, skip)

    def graph_stats(self):
        return serve_graph_stats(self.handle)

    def phase_stats(self):
        return serve_phase_stats(self.handle)

    def close(self):
        if self.handle is not None:
            serve_destroy(self.handle)
            self.handle = None


# ------------------------------------------------------------ convenience ----
class MdcOp:
    """Owns the device buffers (PyTorch) of one operator and its library handle.

    prec: storage format of the resident kernel, one of PREC's names ("fp32", "fp16s",
    "bf16", "bf16x2", "fp16") or an mdc_prec value.
    """

    def __init__(self, nt, nfmax, ns, nr, max_cols=1, prec="fp32", device="cuda"):
        self.desc = mdc_desc(nt, nfmax, ns, nr, max_cols, PREC[prec] if isinstance(prec, str) else prec)
        res, work = mdc_query_sizes(self.desc)
        self.resident = torch.empty(max(res, 256), dtype=torch.uint8, device=device)
        self.workspace = torch.empty(max(work, 256), dtype=torch.uint8, device=device)
        self.handle = mdc_create(self.desc, self.resident, self.workspace)
        self.nt, self.nfmax, self.ns, self.nr, self.max_cols = nt, nfmax, ns, nr, max_cols
        self._lsqr_work = None

    def set_kernel(self, K, scale=1.0, col_weight=None):
        """K: complex64 device tensor [nfmax][ns][nr]."""
        if K.dtype != torch.complex64 or tuple(K.shape) != (self.nfmax, self.ns, self.nr):
            raise ValueError("K must be complex64 [nfmax, ns, nr]")
        mdc_set_kernel(self.handle, K.contiguous(), scale, col_weight)

    def synth_kernel(self, spec, s_index=None, r_index=None, area=None):
        """Generate synth.KernelSpec-defined K on the device (FP64, rounded once)."""
        import numpy as np
        ev = spec.events
        amp = np.ascontiguousarray(ev.amp, dtype=np.float64)
        t0 = np.ascontiguousarray(ev.t0, dtype=np.float64)
        vel = np.ascontiguousarray(ev.v, dtype=np.float64)
        self._si = None if s_index is None else torch.as_tensor(s_index, dtype=torch.int32).cuda()
        self._ri = None if r_index is None else torch.as_tensor(r_index, dtype=torch.int32).cuda()
        sd = mdc_synth_desc(spec.nx, spec.dt, spec.dx, spec.fp, spec.kappa, spec.noise,
                            spec.dA if area is None else area, spec.seed, amp.size,
                            amp.ctypes.data_as(C.POINTER(C.c_double)),
                            t0.ctypes.data_as(C.POINTER(C.c_double)),
                            vel.ctypes.data_as(C.POINTER(C.c_double)),
                            None if self._si is None else self._si.data_ptr(),
                            None if self._ri is None else self._ri.data_ptr())
        mdc_synth_kernel(self.handle, sd)

    def forward(self, x, y=None):
        nv = x.numel() // (self.nt * self.nr)
        if y is None:
            y = torch.empty((self.nt, self.ns, nv), dtype=torch.float32, device=x.device)
        mdc_forward(self.handle, x, y, nv)
        return y

    def adjoint(self, y, x=None):
        nv = y.numel() // (self.nt * self.ns)
        if x is None:
            x = torch.empty((self.nt, self.nr, nv), dtype=torch.float32, device=y.device)
        mdc_adjoint(self.handle, y, x, nv)
        return x

    def marchenko(self, onset, in0, in1, adjoint=False):
        nv = onset.shape[1]
        o0, o1 = torch.empty_like(in0), torch.empty_like(in1)
        (mch_adjoint if adjoint else mch_forward)(self.handle, onset, nv, in0, in1, o0, o1)
        return o0, o1

    def marchenko_data(self, onset, fd):
        nv = onset.shape[1]
        d = torch.empty((2,) + tuple(fd.shape), dtype=torch.float32, device=fd.device)
        mch_data(self.handle, onset, nv, fd, d[0], d[1])
        return d

    def lsqr(self, b, niter, kind=MDC_OP_MDC, nv=1, onset=None, hist=True, out=None):
        """LSQR on the device; out=(x, hist) reuses result buffers (and the captured iteration graph)."""
        ld = lsqr_desc(kind, nv, niter, None if onset is None else onset.data_ptr())
        need = lsqr_query_sizes(self.handle, ld)
        if self._lsqr_work is None or self._lsqr_work.numel() < need:
            self._lsqr_work = torch.empty(need, dtype=torch.uint8, device=b.device)
        if out is not None:
            x, h = out
        else:
            if kind == MDC_OP_MARCHENKO:
                x = torch.empty((2, self.nt, self.nr, nv), dtype=torch.float32, device=b.device)
            else:
                x = torch.empty((self.nt, self.nr, nv), dtype=torch.float32, device=b.device)
            h = torch.empty(niter + 1, dtype=torch.float64, device=b.device) if hist else None
        lsqr_solve(self.handle, ld, b, x, h, self._lsqr_work)
        return x, h

    def cgls(self, b, niter, kind=MDC_OP_MDC, nv=1, onset=None):
        ld = lsqr_desc(kind, nv, niter, None if onset is None else onset.data_ptr())
        need = lsqr_query_sizes(self.handle, ld)
        if self._lsqr_work is None or self._lsqr_work.numel() < need:
            self._lsqr_work = torch.empty(need, dtype=torch.uint8, device=b.device)
        shape = (2, self.nt, self.nr, nv) if kind == MDC_OP_MARCHENKO else (self.nt, self.nr, nv)
        x = torch.empty(shape, dtype=torch.float32, device=b.device)
        h = torch.empty(niter + 1, dtype=torch.float64, device=b.device)
        cgls_solve(self.handle, ld, b, x, h, self._lsqr_work)
        return x, h

    def greens(self, fminus, fd, fm):
        nv = fminus.shape[-1]
        gm, gp = torch.empty_like(fminus), torch.empty_like(fminus)
        mch_greens(self.handle, nv, fminus, fd, fm, gm, gp)
        return gm, gp

    def neumann(self, onset, d, nterms):
        nv = onset.shape[1]
        work = torch.empty(mch_neumann_query(self.handle, nv), dtype=torch.uint8, device=d.device)
        f = torch.empty_like(d)
        mch_neumann(self.handle, onset, nv, d, f, nterms, work)
        return f

    def close(self):
        if self.handle is not None:
            mdc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
