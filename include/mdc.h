/*
 * mdc.h -- C ABI of the MI355X (gfx950) multi-dimensional convolution library.
 *
 * The operator (Theory section, Eq.2-4) maps a real input x[t][r][v]
 * (nt x nr x nv, time outermost) to y[t][s][v] (nt x ns x nv):
 *
 *   forward  y = F^H I^H K I F x      (Eq.3, left)
 *   adjoint  x = F^H I^H K^H I F y    (Eq.3, right)
 *
 * F is the orthogonal real FFT along t (scaled by nt^-1/2 both ways,
 * positive frequencies only), I keeps the first nfmax bins and its adjoint
 * zero-pads, and K is block diagonal with one dense complex slice K_f
 * (ns x nr) per retained frequency (Eq.4), already multiplied by the
 * integration weight dx_R.  The inverse transform takes the real parts of
 * the DC and Nyquist bins, so the adjoint is exact: no time reversal is
 * applied besides the conjugate transpose of each slice.
 *
 * Memory: the library never allocates device memory.  The caller obtains
 * sizes from mdc_query_sizes / lsqr_query_sizes / serve_request_bytes and
 * passes device buffers it owns (e.g. from PyTorch); the library never frees
 * them.  Host-side handles (mdc_op, mdc_server) are owned by the library
 * and released by the matching *_destroy call.
 *
 * Streams: every `stream` argument is a hipStream_t passed as void* (NULL is
 * the default stream).  Calls only enqueue work and return; results are
 * ready when the stream reaches that point.  One mdc_op owns one workspace,
 * so applies on the same op must be issued in order on one stream; distinct
 * ops (each with its own workspace) may run concurrently.
 *
 * Alignment: buffers the library carves into pieces (resident, workspace, the
 * solver work buffers, the serving arena) must be 256-byte aligned.  Vector
 * arguments need only element (4-byte) alignment: the transforms move four
 * traces per 16-byte access when the pointer and the trace count allow it and
 * fall back to element accesses otherwise, and the Marchenko solvers pass the
 * second block of a vector as an element offset into the first.
 *
 * Errors: every function returns an mdc_status; nothing throws.  On error
 * no work has been enqueued (argument checks run first) except for
 * MDC_EDEVICE, which reports a failed launch.  mdc_last_error() returns a
 * thread-local description of the last failure.
 *
 * Layouts (row-major, last index fastest):
 *   time vectors   float   [nt][n][nv]
 *   kernel input   float2  [nfmax][ns][nr]   (complex64: re, im)
 *   onsets         int32   [n][nv]           (window half-width in samples)
 *
 * Windows: an onset o >= 0 keeps the samples with |lag(t)| < o (two-sided); an
 * onset o < 0 keeps 0 <= lag(t) < -o (one-sided, causal), with lag(t) = t for
 * t < nt/2 and t - nt otherwise.
 */
#ifndef MDC_H
#define MDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MDC_OK = 0,
  MDC_EINVAL = -1,     /* bad argument: null/misaligned pointer, size out of range */
  MDC_ENOMEM = -2,     /* a buffer is too small, or a request can never fit its budget */
  MDC_EDEVICE = -3,    /* a HIP launch or runtime call failed */
  MDC_EBUSY = -4,      /* the object is in use (server still has requests) */
  MDC_ENOTREADY = -5,  /* a served request has not finished yet */
  MDC_ECANCELED = -6,  /* a served request was cancelled or failed */
  MDC_ENOTSUP = -7     /* a valid but unsupported combination (e.g. nt not a power of 2) */
} mdc_status;

/* Storage format of the resident kernel.  Products always accumulate in FP32.
 *   MDC_FP32   complex64, 8 bytes per element.
 *   MDC_FP16S  FP16 pairs scaled by a power of two per frequency slice (4 bytes).
 *   MDC_BF16   BF16 pairs (4 bytes).
 *   MDC_BF16X2 BF16 hi + lo pairs, hi = RNE(k), lo = RNE(k - hi) (8 bytes).
 *   MDC_FP16   the MDC_FP16S kernel; on the matrix cores the spectra are rounded
 *              once to FP16 (power-of-two scale per frequency) instead of split
 *              into hi + lo, so the product takes one pass instead of two (about
 *              2^-11 relative error per apply instead of 2^-12).  Forward and
 *              adjoint round different spectra, so on the matrix cores this
 *              format is adjoint only up to that rounding (dot-product test
 *              about 1e-4, against 1e-6 for the other formats); an iterative
 *              solver on it converges to a slightly perturbed normal equation.  */
typedef enum { MDC_FP32 = 0, MDC_FP16S = 1, MDC_BF16 = 2, MDC_BF16X2 = 3, MDC_FP16 = 4 } mdc_prec;

typedef struct mdc_op mdc_op;

typedef struct {
  int nt;        /* time samples; a power of two in [16, 2048] */
  int nfmax;     /* retained bins, 1 <= nfmax <= nt/2 + 1 (Eq.2, omega_max) */
  int ns;        /* rows of each slice: output traces x_B */
  int nr;        /* columns of each slice: integration traces x_R */
  int max_cols;  /* widest column count (virtual points, fused blocks) per apply, >= 1 */
  mdc_prec prec; /* resident storage format */
} mdc_desc;

/* Thread-local text of the last error (never NULL). */
const char* mdc_last_error(void);

/* Bytes of the resident buffer (kernel + tables, 256-byte aligned pieces) and
 * of the per-apply workspace (spectra of max_cols columns; for the 16-bit
 * formats also one spectrum split into 16-bit hi and lo parts, padded to
 * multiples of 64 columns and 96 traces, and nfmax per-frequency maxima, for
 * the matrix-core product). */
mdc_status mdc_query_sizes(const mdc_desc* desc, size_t* resident_bytes, size_t* workspace_bytes);

/* Create an operator over caller-owned device buffers `resident` and `workspace`
 * (256-byte aligned, at least the queried sizes).  Writes the FFT tables into
 * `resident` on `stream`.  The kernel itself is loaded by mdc_set_kernel or
 * mdc_synth_kernel before the first apply. */
mdc_status mdc_create(const mdc_desc* desc, void* resident, void* workspace, void* stream,
                      mdc_op** out);

/* Load the kernel (Eq.4 slices, integration weight included) from a device array
 * K [nfmax][ns][nr] complex64, multiplying element (f, s, r) by
 * scale * (col_weight ? col_weight[r] : 1) (Theory section: constant or
 * receiver-dependent dx_R pre-multiplied into the columns), and converting it to
 * the storage format.  col_weight is a device array of nr floats or NULL.
 * K may be released once the stream passes this call. */
mdc_status mdc_set_kernel(mdc_op* op, const void* K, double scale, const float* col_weight,
                          void* stream);

/* Synthetic hyperbolic-event reflection kernel generated on the device in FP64
 * and rounded once to the storage format (a stand-in for the paper's
 * finite-difference data; see the header comment of the generator):
 *   K[f,s,r] = kappa dA W(f/(nt dt)) sum_k a_k exp(-2 pi i f tau_k(s,r)/(nt dt))
 *              + noise sigma_f (n1 + i n2)/sqrt(2)
 * on a square grid of nx*nx traces with spacing dx; rows and columns are the
 * full-grid trace indices s_index[i], r_index[j] (device int32 arrays of ns and
 * nr entries, or NULL for the identity).  The noise normals come from the
 * SplitMix64 counter generator keyed by (seed, stream 4, counter 2q, 2q+1),
 * q = (f * nx^2 + s) * nx^2 + r. */
typedef struct {
  int nx;              /* grid side; full grid has nx*nx traces */
  double dt, dx;       /* sampling (s, m) */
  double fp;           /* Ricker peak frequency of the kernel spectrum (Hz) */
  double kappa;        /* overall scale */
  double noise;        /* relative noise level */
  double area;         /* dA: areal element multiplied in (m^2) */
  uint64_t seed;
  int nev;             /* number of events (<= 64) */
  const double* amp;   /* host arrays of nev entries: amplitudes, */
  const double* t0;    /*   zero-offset times (s), */
  const double* vel;   /*   moveout velocities (m/s) */
  const int* s_index;  /* device, ns entries or NULL */
  const int* r_index;  /* device, nr entries or NULL */
} mdc_synth_desc;
mdc_status mdc_synth_kernel(mdc_op* op, const mdc_synth_desc* sd, void* stream);

/* Kernel from time-domain traces g[t][s][r] (device float, nt x ns x nr): each trace is
 * transformed with the library's real FFT, K[f][s][r] = scale * col_weight[r] *
 * sum_t g[t][s][r] exp(-2 pi i f t / nt) for f < nfmax (conjugated when conj != 0, which
 * turns traces of g(-t) into the kernel of g), then stored in the op's format: the
 * time-to-frequency preprocessing of the kernel (batch-matmul section), with
 * scale = dt * dA for Eq.1's integral.  temp: device scratch of 8*nfmax*ns*nr bytes,
 * or NULL for complex64 storage with nr a multiple of 4 (transformed in place). */
mdc_status mdc_set_kernel_time(mdc_op* op, const float* g, int conj, double scale, const float* col_weight,
                               void* temp, size_t temp_bytes, void* stream);

/* Read back element (f, s, r) of the resident kernel as complex64 (host
 * pointers re/im; synchronises the stream).  For tests of the loaders. */
mdc_status mdc_kernel_element(mdc_op* op, int f, int s, int r, void* stream, float* re, float* im);

/* Forward (Eq.3 left): y[t][s][v] from x[t][r][v], 1 <= nv <= max_cols.
 * x and y are device float arrays and must not overlap. */
mdc_status mdc_forward(mdc_op* op, const float* x, float* y, int nv, void* stream);

/* Adjoint (Eq.3 right): x[t][r][v] from y[t][s][v]. */
mdc_status mdc_adjoint(mdc_op* op, const float* y, float* x, int nv, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mdc_forward (adjoint = 0) or mdc_adjoint
 * (adjoint = 1) with the apply's spectra in a static device array of the library instead of the
 * op's workspace.  The array holds 64 MiB (MDC_NOALLOC_SCRATCH_BYTES) on every GPU the library
 * runs on, until the process ends; an apply whose spectra need more (nfmax * (ns + nr) * nv * 8
 * bytes, plus the 16-bit split buffers) returns MDC_ENOMEM.  nv is not bounded by the op's
 * max_cols.  The call allocates nothing; the array's device address is looked up once per device
 * (at mdc_create, else at the first call).  All calls on one GPU share the array: calls that
 * overlap on one GPU (different streams, threads or ops) race and must be serialised by the
 * caller.  The op's own workspace is not touched, so mdc_forward / mdc_adjoint may overlap it. */
#define MDC_NOALLOC_SCRATCH_BYTES (64u << 20)
mdc_status mdc_apply_noalloc(mdc_op* op, int adjoint, const float* in, float* out, int nv, void* stream);

/* Marchenko operator of Eq.5 on a square op (ns == nr == n) with 2*nv <= max_cols:
 *   forward  (o0, o1) = (in0 - Theta R in1,  in1 - Theta R* in0)
 *   adjoint  (o0, o1) = (in0 - R*^H Theta in1,  in1 - R^H Theta in0)
 * R uses the kernel, R* its complex conjugate (no transpose).  Theta[t][s][v] = 1
 * when |lag(t)| < onset[s][v] (onset >= 0; the window encoding above).
 * One pass over the kernel serves both blocks (columns [R-input | conj R*-input]).
 * All arrays are device arrays [nt][n][nv]; outputs must not alias inputs. */
mdc_status mch_forward(mdc_op* op, const int* onset, int nv, const float* in0, const float* in1,
                       float* out0, float* out1, void* stream);
mdc_status mch_adjoint(mdc_op* op, const int* onset, int nv, const float* in0, const float* in1,
                       float* out0, float* out1, void* stream);

/* Right-hand side of Eq.5: d0 = Theta R fd, d1 = 0, with fd [nt][n][nv] the
 * direct (initial) focusing function; nv <= max_cols. */
mdc_status mch_data(mdc_op* op, const int* onset, int nv, const float* fd, float* d0, float* d1, void* stream);

/* Green's functions of Eq.6 from the focusing functions (square op, 2*nv <= max_cols):
 *   g- = R f+ - f-,   g+* = f+ - R* f-,   f+ = fd + fm
 * (the sign convention of Eq.6: [-g-; g+*] = [[I, -R], [-R*, I]] [f-; f+]).  All arrays
 * are device [nt][n][nv]; gminus and gplus_conj must not alias the inputs. */
mdc_status mch_greens(mdc_op* op, int nv, const float* fminus, const float* fd, const float* fm, float* gminus,
                      float* gplus_conj, void* stream);

/* Forward-only (Neumann) scheme for Eq.5: f = sum_{k<nterms} B^k d with B = I - M,
 * i.e. B [a0; a1] = [Theta R a1; Theta R* a0]; converges when rho(B) < 1 (Applications:
 * Neumann vs gradient solvers).  d, f: device [2][nt][n][nv]; work from
 * mch_neumann_query. */
mdc_status mch_neumann_query(const mdc_op* op, int nv, size_t* work_bytes);
mdc_status mch_neumann(mdc_op* op, const int* onset, int nv, const float* d, float* f, int nterms, void* work,
                       size_t work_bytes, void* stream);

/* Per-stage timing with HIP events on the apply stream (for measurement).
 * enable != 0 starts recording; mdc_profile_read synchronises and returns the
 * summed milliseconds and launch counts of each stage since the last read:
 * [0] forward FFT, [1] kernel product (forward form), [2] kernel product
 * (adjoint form), [3] inverse FFT. */
mdc_status mdc_profile(mdc_op* op, int enable);
mdc_status mdc_profile_read(mdc_op* op, double ms[4], int counts[4]);

/* Autotuner of the per-frequency product (the batch matrix multiplication of
 * Eq.4).  For column counts 1, 2, 3, 4, 6, 8, 12, ... up to max_cols and both
 * directions it times each kernel family on this op's resident kernel -- the
 * streaming kernels (family 0) and two matrix-core variants: 64- and 32-column tiles
 * for complex64 storage, four waves of 64 rows and eight waves of 32 rows per
 * workgroup for the 16-bit formats (families 1 and 2) -- and keeps the fastest per
 * width; later applies of N columns use the entry of the smallest tuned
 * width >= N.  With cache_path non-NULL, a JSON line per (arch, format, shape) is
 * read if present (*measured = 0) or appended after measuring (*measured = 1).
 * Synchronises the stream; overwrites the op's workspace.  Without tuning, up to 8
 * columns use family 0 and wider products family 1. */
mdc_status mdc_autotune(mdc_op* op, const char* cache_path, void* stream, int* measured);
/* The tuning table: count entries; arrays of at least `cap` ints (or NULL). */
mdc_status mdc_tune_table(const mdc_op* op, int cap, int* count, int* ncols, int* fwd_family, int* adj_family);

mdc_status mdc_destroy(mdc_op* op);

/* ----------------------------------------------------------------- LSQR ----
 * LSQR (Paige & Saunders 1982; damping 0, x0 = 0, fixed niter) on the MDC
 * operator (kind MDC_OP_MDC: A = C, model [nt][nr][nv], data [nt][ns][nv]) or
 * on the Marchenko operator (kind MDC_OP_MARCHENKO: A = M, model and data two
 * blocks [2][nt][n][nv]).  Vectors are FP32 on the device; alpha, beta, rho,
 * rhobar, c, s, theta, phi, phibar and the norms are FP64 on the device.  The
 * host does not synchronise inside the solve.  The paper runs CGLS for 10
 * iterations (Applications section); LSQR produces the same iterates in exact
 * arithmetic. */
typedef enum { MDC_OP_MDC = 0, MDC_OP_MARCHENKO = 1 } mdc_opkind;
typedef struct {
  mdc_opkind kind;
  int nv;             /* virtual points */
  int niter;          /* iterations (>= 0) */
  const int* onset;   /* MDC_OP_MARCHENKO: window onsets [n][nv] (device), required.
                         MDC_OP_MDC: optional model preconditioner P [nr][nv] (device) in the
                         same encoding, so the solve is min ||b - C P z||, x = P z (Discussion
                         section: causal time windowing of the MDD unknown); NULL = none */
} lsqr_desc;

/* Bytes of the workspace lsqr_solve needs for this descriptor. */
mdc_status lsqr_query_sizes(const mdc_op* op, const lsqr_desc* ld, size_t* work_bytes);

/* b: data (device, float); x: model output (device, float, overwritten);
 * hist: device double array of niter+1 entries receiving phibar (the residual
 * norm estimate) after each iteration, or NULL; work: device workspace.
 * The three-term recurrences and their norms run inside the operator's inverse
 * transform (environment MDC_LSQR_FUSE=0 runs them as separate vector passes:
 * the same per-element arithmetic, norms summed in a different grouping), and
 * iterations after the first replay a captured graph (MDC_LSQR_GRAPH=0 runs
 * them eagerly).  The Krylov vectors and the iterate live in the workspace in the
 * transforms' tiled layout (each transform workgroup reads or writes one contiguous
 * tile of traces); b is converted on entry and x written at the end
 * (MDC_LSQR_TILED=0 keeps the [nt][n][nv] layout throughout, for comparison). */
mdc_status lsqr_solve(mdc_op* op, const lsqr_desc* ld, const float* b, float* x, double* hist,
                      void* work, size_t work_bytes, void* stream);

/* CGLS, the solver the paper runs (Applications: 10 iterations): conjugate gradients on
 * the normal equations, x0 = 0, fixed niter, same operators, layouts and workspace size
 * (lsqr_query_sizes) as lsqr_solve; hist receives ||b - A x_i|| for i = 0..niter.
 * FP32 vectors, FP64 scalars on the device. */
mdc_status cgls_solve(mdc_op* op, const lsqr_desc* ld, const float* b, float* x, double* hist, void* work,
                      size_t work_bytes, void* stream);

/* -------------------------------------------------------------- serving ----
 * A server runs Marchenko LSQR solves (Eq.5) for requests that arrive over
 * time against one resident kernel (a square op over a full nx*nx grid).
 * Every step is one pass over the kernel serving the columns of every admitted
 * request (forward and adjoint steps alternate; each request advances one
 * operator application per step), so concurrent requests share the kernel
 * reads (Discussion: many focusing points per pass, independent groups of
 * points).  Each request keeps its own Krylov vectors and FP64 scalars in a
 * slot of the caller's arena; admission is FIFO by slot size and by the op's
 * column budget (2*nv columns per request, max_cols in total).  A request
 * draws its inputs on the device from its focusing points: direct traveltime
 * td = |x_r - x_v| / c, window onsets max(rint(td/dt) - eps, 0), initial
 * focusing function ricker_fp(lag(t) dt + td); decimation by 2 or 4 keeps the
 * lattice traces of the paper's Sub2/Sub4 geometries with areal element d dx^2.
 * A request's result depends only on its own columns (same alone or in a mix,
 * up to the rounding of the product family chosen by the total width).
 * The server owns the op and its workspace while it exists.  A worker thread
 * and a HIP stream of the library run the steps. */
typedef struct mdc_server mdc_server;
typedef struct {
  int nx;            /* grid side (nx*nx == op ns == op nr) */
  double dx, dt;     /* trace spacing (m), time sampling (s) */
  double c;          /* direct-arrival velocity (m/s) */
  int eps;           /* window margin in samples */
  double fp;         /* peak frequency of the initial focusing wavelet (Hz) */
  int sublattice;    /* decimation levels solved on their own lattice: 0, 2, 4 or 2|4.  For such
                        a level serve_create gathers the lattice's kernel rows and columns once
                        into the arena (serve_level_bytes), and its requests run their
                        transforms, product and Krylov vectors on the lattice's traces only
                        (the Sub2 / Sub4 problems of Table 1: 1/d of the traces, 1/d^2 of the
                        kernel).  Other decimated requests run on the full grid with zero
                        traces off the lattice. */
} serve_geometry;
typedef struct {
  int nv;                  /* focusing points, 1..64 */
  int niter;               /* LSQR iterations, >= 0 */
  int decim;               /* 1, 2 or 4 */
  const double *vx, *vy, *vz;  /* host arrays of nv coordinates (m), copied at submit */
  float* x_out;            /* device [2][nt][n][nv]: solution (f-, f_m+); ready when polled done */
  double* hist;            /* device [niter+1] residual-norm history, or NULL */
} serve_req;

/* Arena bytes one request of nv points occupies on the full grid (an upper bound for lattice
 * levels, whose four vectors have 1/d the length); the vectors are held in the transforms'
 * tiled layout and the solution is written to x_out when the request finishes. */
mdc_status serve_request_bytes(const mdc_op* op, int nv, size_t* bytes);
/* Arena bytes serve_create reserves for the lattice level of decimation 2 or 4 (index tables
 * and the gathered kernel in the op's storage format). */
mdc_status serve_level_bytes(const mdc_op* op, int decim, size_t* bytes);
/* arena: caller-owned device buffer (256-byte aligned) for the lattice levels (first) and the
 * request slots.  The op's kernel must be loaded and its load synchronised: the lattice levels
 * are gathered from it, on the server's stream, before the call returns.  MDC_ENOMEM when the
 * arena cannot hold the levels asked for. */
mdc_status serve_create(mdc_op* op, const serve_geometry* g, void* arena, size_t arena_bytes, mdc_server** out);
/* Queue a request (MDC_ENOMEM if it can never fit the arena or the column budget). Buffers
 * must be ready (their producers synchronised) before the call. */
mdc_status serve_submit(mdc_server* srv, const serve_req* req, uint64_t* id);
/* done = 1 and MDC_OK when finished (latency = completion - submission, seconds);
 * done = 0 and MDC_ENOTREADY while queued or running; done = -1 and MDC_ECANCELED.  A finished
 * request is reported once: the server then releases it, and a later poll or cancel of the
 * same id returns MDC_EINVAL (unknown id), so a long-running server holds only live requests. */
mdc_status serve_poll(mdc_server* srv, uint64_t id, int* done, double* latency_s);
/* Cancel a queued or running request; it leaves at the next step boundary. */
mdc_status serve_cancel(mdc_server* srv, uint64_t id);
/* Block until every submitted request has finished or been cancelled. */
mdc_status serve_drain(mdc_server* srv);
/* Completed solves per second (first submission to last completion), median and 99th
 * percentile latency over completions after the first `skip`, completion count, the
 * largest number of simultaneously admitted requests, and the number of steps run. */
mdc_status serve_stats(mdc_server* srv, int skip, double* solves_per_s, double* p50_s, double* p99_s,
                       int* completed, int* max_active, long* steps);
/* Lockstep phases.  Every admitted request applies the operator in the step's direction and new
 * requests (which start with a forward application) join at forward steps, so each pass over
 * the kernel serves every admitted request.  request_steps: requests served, summed over steps;
 * deferred: requests that could have been admitted during an adjoint step and waited for it;
 * deferred_s: the time they waited, summed (the latency a pass serving both directions at once
 * would remove). */
mdc_status serve_phase_stats(mdc_server* srv, long* request_steps, long* deferred, double* deferred_s);
/* Steps captured into hipGraphs and steps replayed from them so far.  Within a fixed set
 * of active requests every forward and every adjoint step enqueues the same launches: the
 * first step of such a composition runs eagerly, the second is captured, later ones replay
 * the graph (environment MDC_SERVE_GRAPH=0 runs every step eagerly). */
mdc_status serve_graph_stats(mdc_server* srv, long* captured, long* replayed);

/* Stop the worker (cancelling what is left) and release the handle. */
mdc_status serve_destroy(mdc_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* MDC_H */
