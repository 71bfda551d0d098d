// C ABI of the MDC library: argument checks, buffer carving and the order of
// launches of each apply (Eq.3 chain: truncated real FFT, per-frequency
// product, zero-padded inverse FFT with fused epilogue).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "store.hpp"



namespace mdc {

static thread_local char g_err[512] = "no error";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

mdc_status fail(mdc_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

mdc_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MDC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return MDC_OK;
}

size_t store_bytes(const mdc_desc& d) {
  const size_t elems = (size_t)d.nfmax * d.ns * kernel_ld(d.nr);
  switch (d.prec) {
    case MDC_FP32: return elems * 8;
    case MDC_FP16S: return elems * 4;
    case MDC_FP16: return elems * 4;
    case MDC_BF16: return elems * 4;
    case MDC_BF16X2: return elems * 8;
  }
  return 0;
}

// Product families: the streaming kernels (0), and the matrix-core kernels: FP32 with 64-column
// (1) or 32-column (2) tiles; 16-bit formats with four waves of 64 rows (1) or eight waves of
// 32 rows (2) per workgroup.
enum Family { kFamGemv = 0, kFamGemm64 = 1, kFamGemm32 = 2 };
// Default crossover without tuning: streaming kernels up to 8 columns.
static constexpr int kGemvMaxCols = 8;

// d: the op's descriptor, or a copy whose max_cols sizes the split-spectra buffer bsplit.
static mdc_status run_family(const mdc_op* op, int fam, int adjoint, const float2* in, float2* out, int ncols,
                             hipStream_t st, const mdc_desc& d, unsigned int* bsplit) {
  const int ldk = kernel_ld(d.nr);
  if (fam == kFamGemv) return gemv_launch(d, op->kstore, op->fscale, ldk, adjoint, in, out, ncols, st);
  if (d.prec == MDC_FP32)
    return gemm_launch(d, static_cast<const float2*>(op->kstore), ldk, adjoint, in, out, ncols, st,
                       fam == kFamGemm32 ? 32 : 64);
  return gemm16_launch(d, op->kstore, op->fscale, ldk, adjoint, in, out, ncols, bsplit, fam == kFamGemm32 ? 1 : 0,
                       st);
}

int forced_family(const mdc_op* op) {
  if (const char* e = getenv("MDC_PRODUCT")) {  // forced family (tests)
    if (!strcmp(e, "gemv")) return kFamGemv;
    if (!strcmp(e, "gemm")) return kFamGemm64;
    if (!strcmp(e, "gemm32")) return kFamGemm32;
  }
  return -1;
}

int choose_family(const mdc_op* op, int adjoint, int ncols) {
  const int forced = forced_family(op);
  if (forced >= 0) return forced;
  const auto& ns = op->tune_ncols;
  if (!ns.empty()) {
    size_t i = 0;
    while (i + 1 < ns.size() && ns[i] < ncols) ++i;  // smallest tuned width >= ncols (else the widest)
    return op->tune_family[adjoint ? 1 : 0][i];
  }
  return ncols > kGemvMaxCols ? kFamGemm64 : kFamGemv;
}

mdc_status product_launch(const mdc_op* op, int adjoint, const float2* in, float2* out, int ncols, hipStream_t st) {
  return run_family(op, choose_family(op, adjoint, ncols), adjoint, in, out, ncols, st, op->d, op->bsplit);
}

// Time one family at one width on the op's own kernel (ms per launch, best of 3).
float time_family(mdc_op* op, int fam, int adjoint, int ncols, hipStream_t st) {
  float2* in = adjoint ? op->specS : op->specR;
  float2* out = adjoint ? op->specR : op->specS;
  hipEvent_t a = nullptr, b = nullptr;
  float best = 3.0e38f;  // a family that cannot be timed is never chosen
  if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
      run_family(op, fam, adjoint, in, out, ncols, st, op->d, op->bsplit) == MDC_OK) {  // warm-up
    for (int rep = 0; rep < 3; ++rep) {
      float ms = 0.f;
      if (hipEventRecord(a, st) != hipSuccess ||
          run_family(op, fam, adjoint, in, out, ncols, st, op->d, op->bsplit) != MDC_OK ||
          hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
          hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        best = 3.0e38f;
        break;
      }
      best = ms < best ? ms : best;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return best;
}

}  // namespace mdc

using namespace mdc;

namespace {

constexpr size_t kAlign = 256;

mdc_status check_desc(const mdc_desc* d) {
  if (!d) return fail(MDC_EINVAL, "descriptor is NULL");
  if (d->nt < 16 || d->nt > 2048 || (d->nt & (d->nt - 1)) != 0)
    return fail(MDC_ENOTSUP, "nt=%d: must be a power of two in [16, 2048]", d->nt);
  if (d->nfmax < 1 || d->nfmax > d->nt / 2 + 1) return fail(MDC_EINVAL, "nfmax=%d outside [1, nt/2+1]", d->nfmax);
  if (d->ns < 1 || d->nr < 1) return fail(MDC_EINVAL, "ns=%d, nr=%d must be positive", d->ns, d->nr);
  if (d->max_cols < 1 || d->max_cols > 4096) return fail(MDC_EINVAL, "max_cols=%d outside [1, 4096]", d->max_cols);
  if (d->prec < MDC_FP32 || d->prec > MDC_FP16) return fail(MDC_EINVAL, "unknown storage format %d", (int)d->prec);
  return MDC_OK;
}

struct Layout {
  size_t tw, fscale, kstore, resident;
  size_t specR, specS, bsplit, work;
};

Layout layout_of(const mdc_desc& d) {
  Layout L{};
  size_t off = 0;
  L.tw = off; off = align_up(off + (size_t)d.nt * 8, kAlign);
  L.fscale = off; off = align_up(off + (size_t)d.nfmax * 4, kAlign);
  L.kstore = off; off = align_up(off + store_bytes(d), kAlign);
  L.resident = off;
  off = 0;
  L.specR = off; off = align_up(off + (size_t)d.nfmax * d.nr * d.max_cols * 8, kAlign);
  L.specS = off; off = align_up(off + (size_t)d.nfmax * d.ns * d.max_cols * 8, kAlign);
  L.bsplit = off;
  if (d.prec != MDC_FP32) off = align_up(off + gemm16_split_bytes(d), kAlign);
  L.work = off;
  return L;
}

hipEvent_t take_event(mdc_op* op) {
  if (!op->pool.empty()) {
    hipEvent_t e = op->pool.back();
    op->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Scoped stage timer: records an event pair around the launches of one stage.
struct Stage {
  mdc_op* op;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Stage(mdc_op* o, int s, hipStream_t stream) : op(o), stage(s), st(stream) {
    if (op->prof) {
      a = take_event(op);
      if (a && hipEventRecord(a, st) != hipSuccess) {  // unrecorded: this stage goes untimed
        op->pool.push_back(a);
        a = nullptr;
      }
    }
  }
  ~Stage() {
    if (op->prof && a) {
      hipEvent_t b = take_event(op);
      if (b && hipEventRecord(b, st) == hipSuccess) {
        op->evs.push_back({stage, a, b});
      } else {
        op->pool.push_back(a);
        if (b) op->pool.push_back(b);
      }
    }
  }
};

mdc_status check_vec(const void* p, const char* name) {
  if (!p) return fail(MDC_EINVAL, "%s is NULL", name);
  if (!aligned(p, 4)) return fail(MDC_EINVAL, "%s is not 4-byte aligned", name);
  return MDC_OK;
}

// Spectra buffers of one apply: the op's workspace, or another buffer carved the same way for a
// descriptor copy d whose max_cols is the apply's width.
struct Spectra {
  float2 *R, *S;
  unsigned int* split;
  mdc_desc d;
};

// pre: optional window [nr][nv] on the model side (a time-domain preconditioner P, so the
// operator is C P, adjoint P C^H), or nullptr.  ws: spectra buffers replacing the op's workspace.
// tiled: in and out in the tiled time layout of the solvers (fft_tile), else [nt][n][nv].
mdc_status apply_plain(mdc_op* op, const float* in, float* out, int nv, int adjoint, hipStream_t st,
                       const int* pre = nullptr, const double* in_scale = nullptr, const Recur* rec = nullptr,
                       const Spectra* ws = nullptr, int tiled = 0) {
  const mdc_desc& d = op->d;
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded (mdc_set_kernel / mdc_synth_kernel)");
  if (nv < 1 || nv > (ws ? ws->d.max_cols : d.max_cols))
    return fail(MDC_EINVAL, "nv=%d outside [1, max_cols=%d]", nv, ws ? ws->d.max_cols : d.max_cols);
  mdc_status s;
  if ((s = check_vec(in, "input")) != MDC_OK) return s;
  if ((s = check_vec(out, "output")) != MDC_OK) return s;
  const int nin = adjoint ? d.ns : d.nr;
  const int nout = adjoint ? d.nr : d.ns;
  float2* sR = ws ? ws->R : op->specR;
  float2* sS = ws ? ws->S : op->specS;
  float2* spec_in = adjoint ? sS : sR;
  float2* spec_out = adjoint ? sR : sS;
  {
    Stage t(op, 0, st);
    FftSeg seg{in, adjoint ? nullptr : pre, 0, 0, in_scale, tiled};
    if ((s = rfft_launch(op->tw, d.nt, d.nfmax, nin, nv, nv, seg, spec_in, st)) != MDC_OK) return s;
  }
  {
    Stage t(op, adjoint ? 2 : 1, st);
    s = ws ? run_family(op, choose_family(op, adjoint, nv), adjoint, spec_in, spec_out, nv, st, ws->d, ws->split)
           : product_launch(op, adjoint, spec_in, spec_out, nv, st);
    if (s != MDC_OK) return s;
  }
  {
    Stage t(op, 3, st);
    IfftSeg seg{out, nullptr, adjoint ? pre : nullptr, 0, 0, 1.0f};
    seg.tiled = tiled;
    attach_recur(seg, rec, 0);
    if ((s = irfft_launch(op->tw, d.nt, d.nfmax, nout, nv, nv, seg, spec_out, st)) != MDC_OK) return s;
  }
  return MDC_OK;
}

// Marchenko block operator (Eq.5): one kernel pass with columns [block for R | conj block for R*].
mdc_status apply_marchenko(mdc_op* op, const int* onset, int nv, const float* in0, const float* in1, float* out0,
                           float* out1, int adjoint, hipStream_t st, int mode = 0,
                           const double* in_scale = nullptr, const Recur* rec = nullptr, int tiled = 0) {
  const mdc_desc& d = op->d;
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  if (d.ns != d.nr) return fail(MDC_EINVAL, "Marchenko operator needs ns == nr (got %d, %d)", d.ns, d.nr);
  if (nv < 1 || 2 * nv > d.max_cols) return fail(MDC_EINVAL, "2*nv=%d outside [2, max_cols=%d]", 2 * nv, d.max_cols);
  mdc_status s;
  if ((s = check_vec(onset, "onset")) != MDC_OK) return s;
  if ((s = check_vec(in0, "in0")) != MDC_OK) return s;
  if ((s = check_vec(in1, "in1")) != MDC_OK) return s;
  if ((s = check_vec(out0, "out0")) != MDC_OK) return s;
  if ((s = check_vec(out1, "out1")) != MDC_OK) return s;
  const int n = d.ns, N = 2 * nv;
  float2* spec_in = adjoint ? op->specS : op->specR;
  float2* spec_out = adjoint ? op->specR : op->specS;
  {
    Stage t(op, 0, st);
    // forward: R acts on in1, R* on in0; adjoint: R^H on Theta in0, R*^H on Theta in1
    const int* pre = adjoint ? onset : nullptr;
    FftSeg a{adjoint ? in0 : in1, pre, 0, 0, in_scale, tiled};
    FftSeg b{adjoint ? in1 : in0, pre, 1, nv, in_scale, tiled};
    if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, a, spec_in, st)) != MDC_OK) return s;
    if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, b, spec_in, st)) != MDC_OK) return s;
  }
  {
    Stage t(op, adjoint ? 2 : 1, st);
    if ((s = product_launch(op, adjoint, spec_in, spec_out, N, st)) != MDC_OK) return s;
  }
  {
    Stage t(op, 3, st);
    const int* post = adjoint ? nullptr : onset;
    // forward: out0 = in0 - Theta R in1 (cols 0..nv), out1 = in1 - Theta R* in0 (cols nv..2nv, conj)
    // adjoint: out1 = in1 - R^H Theta in0 (cols 0..nv), out0 = in0 - R*^H Theta in1 (cols nv..2nv, conj)
    // mode 1 (Neumann term B = I - M): no identity blocks, + sign
    const float sg = mode == 1 ? 1.0f : -1.0f;
    IfftSeg a{adjoint ? out1 : out0, mode == 1 ? nullptr : (adjoint ? in1 : in0), post, 0, 0, sg, 1.0f, in_scale};
    IfftSeg b{adjoint ? out0 : out1, mode == 1 ? nullptr : (adjoint ? in0 : in1), post, 1, nv, sg, 1.0f, in_scale};
    a.tiled = b.tiled = tiled;
    attach_recur(a, rec, 0);
    attach_recur(b, rec, irfft_blocks(d.nt, n, nv));
    if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, a, spec_out, st)) != MDC_OK) return s;
    if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, b, spec_out, st)) != MDC_OK) return s;
  }
  return MDC_OK;
}

__global__ void fill_zero(float* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.f;
}

// d0 = Theta R fd, d1 = 0 (right-hand side of the Marchenko system).
mdc_status apply_mch_data(mdc_op* op, const int* onset, int nv, const float* fd, float* d0, float* d1,
                          hipStream_t st) {
  const mdc_desc& d = op->d;
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  if (d.ns != d.nr) return fail(MDC_EINVAL, "Marchenko operator needs ns == nr (got %d, %d)", d.ns, d.nr);
  if (nv < 1 || nv > d.max_cols) return fail(MDC_EINVAL, "nv=%d outside [1, max_cols=%d]", nv, d.max_cols);
  mdc_status s;
  if ((s = check_vec(onset, "onset")) != MDC_OK) return s;
  if ((s = check_vec(fd, "fd")) != MDC_OK) return s;
  if ((s = check_vec(d0, "d0")) != MDC_OK) return s;
  if ((s = check_vec(d1, "d1")) != MDC_OK) return s;
  const int n = d.ns;
  {
    Stage t(op, 0, st);
    FftSeg a{fd, nullptr, 0, 0};
    if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, nv, nv, a, op->specR, st)) != MDC_OK) return s;
  }
  {
    Stage t(op, 1, st);
    if ((s = product_launch(op, 0, op->specR, op->specS, nv, st)) != MDC_OK) return s;
  }
  {
    Stage t(op, 3, st);
    IfftSeg a{d0, nullptr, onset, 0, 0, 1.0f};
    if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, nv, nv, a, op->specS, st)) != MDC_OK) return s;
  }
  hipLaunchKernelGGL(fill_zero, dim3(1024), dim3(256), 0, st, d1, (size_t)d.nt * n * nv);
  return check_launch("fill_zero");
}

// Scaled conversion of a complex64 kernel [nfmax][ns][nr] into the resident store
// [nfmax][ns][ldk] (pad columns zero), through one of the storage formats.
template <typename Store>
__global__ void load_kernel(const float2* K, Store out, int nfmax, int ns, int nr, int ldk, double scale,
                            const float* __restrict__ w) {
  const size_t count = (size_t)nfmax * ns * ldk;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const size_t row = i / (size_t)ldk;
    const int r = (int)(i - row * (size_t)ldk);
    const int f = (int)(row / (size_t)ns), s = (int)(row - (size_t)f * ns);
    double re = 0.0, im = 0.0;
    if (r < nr) {
      const double m = scale * (w ? (double)w[r] : 1.0);
      const float2 k = K[row * nr + r];
      // round the scaled value to complex64 first, as a caller-scaled complex64 kernel would be
      re = (double)(float)(k.x * m);
      im = (double)(float)(k.y * m);
    }
    out.put(f, s, r, re, im);
  }
}

template <typename Store>
mdc_status launch_load(mdc_op* op, const float2* K, double scale, const float* w, hipStream_t st) {
  const mdc_desc& d = op->d;
  StoreRef ref{op->kstore, op->fscale, d.nfmax, d.ns, d.nr, kernel_ld(d.nr)};
  hipLaunchKernelGGL(load_kernel<Store>, dim3(4096), dim3(256), 0, st, K, Store(ref), d.nfmax, d.ns, d.nr,
                     kernel_ld(d.nr), scale, w);
  return check_launch("load_kernel");
}

__global__ void add2(float* __restrict__ out, const float* __restrict__ a, const float* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = a[i] + b[i];
}

__global__ void copy2(float* __restrict__ a, float* __restrict__ b, const float* __restrict__ src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float v = src[i];
    a[i] = v;
    b[i] = v;
  }
}

__global__ void acc_add(float* __restrict__ f, const float* __restrict__ t, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) f[i] += t[i];
}

// Eq.6: g- = R f+ - f-,  g+* = f+ - R* f-,  f+ = fd + fm (formed in gpc first).
mdc_status apply_greens(mdc_op* op, int nv, const float* fminus, const float* fd, const float* fm, float* gminus,
                        float* gpc, hipStream_t st) {
  const mdc_desc& d = op->d;
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  if (d.ns != d.nr) return fail(MDC_EINVAL, "Green's functions need ns == nr");
  if (nv < 1 || 2 * nv > d.max_cols) return fail(MDC_EINVAL, "2*nv=%d outside [2, max_cols=%d]", 2 * nv, d.max_cols);
  mdc_status s;
  if ((s = check_vec(fminus, "fminus")) != MDC_OK || (s = check_vec(fd, "fd")) != MDC_OK ||
      (s = check_vec(fm, "fm")) != MDC_OK || (s = check_vec(gminus, "gminus")) != MDC_OK ||
      (s = check_vec(gpc, "gplus_conj")) != MDC_OK)
    return s;
  const int n = d.ns, N = 2 * nv;
  hipLaunchKernelGGL(add2, dim3(1024), dim3(256), 0, st, gpc, fd, fm, (size_t)d.nt * n * nv);
  if ((s = check_launch("add2")) != MDC_OK) return s;
  FftSeg a{gpc, nullptr, 0, 0};
  FftSeg b{fminus, nullptr, 1, nv};
  if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, a, op->specR, st)) != MDC_OK) return s;
  if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, b, op->specR, st)) != MDC_OK) return s;
  if ((s = product_launch(op, 0, op->specR, op->specS, N, st)) != MDC_OK) return s;
  IfftSeg ga{gminus, fminus, nullptr, 0, 0, 1.0f, -1.0f};
  IfftSeg gb{gpc, gpc, nullptr, 1, nv, -1.0f, 1.0f};
  if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, ga, op->specS, st)) != MDC_OK) return s;
  return irfft_launch(op->tw, d.nt, d.nfmax, n, nv, N, gb, op->specS, st);
}

// f = sum_{k < nterms} B^k d with B = I - M (forward-only scheme; needs rho(B) < 1).
mdc_status apply_neumann(mdc_op* op, const int* onset, int nv, const float* dvec, float* f, int nterms, void* work,
                         size_t work_bytes, hipStream_t st) {
  const mdc_desc& d = op->d;
  const size_t blk = (size_t)d.nt * d.ns * nv, vec = 2 * blk;
  const size_t need = 2 * align_up(vec * 4, 256);
  if (!work || !aligned(work, 256)) return fail(MDC_EINVAL, "work must be non-NULL and 256-byte aligned");
  if (work_bytes < need) return fail(MDC_ENOMEM, "work has %zu bytes, %zu needed", work_bytes, need);
  if (nterms < 1) return fail(MDC_EINVAL, "nterms must be >= 1");
  mdc_status s;
  if ((s = check_vec(dvec, "d")) != MDC_OK || (s = check_vec(f, "f")) != MDC_OK) return s;
  float* t = static_cast<float*>(work);
  float* t2 = reinterpret_cast<float*>(static_cast<char*>(work) + align_up(vec * 4, 256));
  hipLaunchKernelGGL(copy2, dim3(1024), dim3(256), 0, st, f, t, dvec, vec);
  for (int k = 1; k < nterms; ++k) {
    if ((s = apply_marchenko(op, onset, nv, t, t + blk, t2, t2 + blk, 0, st, 1)) != MDC_OK) return s;
    hipLaunchKernelGGL(acc_add, dim3(1024), dim3(256), 0, st, f, t2, vec);
    float* tmp = t;
    t = t2;
    t2 = tmp;
  }
  return check_launch("neumann");
}

// Kernel of a sub-grid: dst[f][i][j] = src[f][idx[i]][idx[j]] for i, j < nsub (pad columns zero),
// copied word for word in the storage format.  KIND 0: 8-byte elements (complex64), 1: 4-byte
// pairs (FP16S, FP16, BF16), 2: BF16 hi + lo rows stored in groups of four complex values.
template <int KIND>
__global__ void gather_sub_kernel(const unsigned int* __restrict__ src, unsigned int* __restrict__ dst,
                                  const int* __restrict__ idx, int nfmax, int ns, int ldk, int nsub, int ldks) {
  const size_t count = (size_t)nfmax * nsub * ldks;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const size_t row = e / (size_t)ldks;
    const int j = (int)(e - row * (size_t)ldks);
    const int f = (int)(row / (size_t)nsub), i = (int)(row - (size_t)f * nsub);
    const bool in = j < nsub;
    const size_t srow = (size_t)f * ns + idx[i];
    const int r = in ? idx[j] : 0;
    if constexpr (KIND == 0) {
      const uint2 v = in ? reinterpret_cast<const uint2*>(src)[srow * ldk + r] : make_uint2(0u, 0u);
      reinterpret_cast<uint2*>(dst)[row * ldks + j] = v;
    } else if constexpr (KIND == 1) {
      dst[row * ldks + j] = in ? src[srow * ldk + r] : 0u;
    } else {
      const unsigned int* sr = src + srow * (size_t)ldk * 2;
      unsigned int* dr = dst + row * (size_t)ldks * 2;
      const int gs = (r >> 2) * 8 + (r & 3), gd = (j >> 2) * 8 + (j & 3);
      dr[gd] = in ? sr[gs] : 0u;
      dr[gd + 4] = in ? sr[gs + 4] : 0u;
    }
  }
}

}  // namespace

namespace mdc {

size_t sub_op_resident_bytes(const mdc_op* parent, int nsub) {
  mdc_desc d = parent->d;
  d.ns = d.nr = nsub;
  return layout_of(d).resident;
}

mdc_status sub_op_create(const mdc_op* parent, const int* idx, int nsub, void* resident, hipStream_t st,
                         mdc_op** out) {
  const mdc_desc& pd = parent->d;
  if (pd.ns != pd.nr || nsub < 1 || nsub > pd.ns) return fail(MDC_EINVAL, "sub-grid of %d traces", nsub);
  if (!resident || !aligned(resident, kAlign)) return fail(MDC_EINVAL, "sub-grid resident must be 256-byte aligned");
  mdc_desc d = pd;
  d.ns = d.nr = nsub;
  const Layout L = layout_of(d);
  mdc_op* op = new (std::nothrow) mdc_op();
  if (!op) return fail(MDC_ENOMEM, "host allocation failed");
  op->d = d;
  op->resident = static_cast<char*>(resident);
  op->work = parent->work;  // every piece of the sub-grid workspace fits in the parent's
  op->tw = reinterpret_cast<float2*>(op->resident + L.tw);
  op->fscale = reinterpret_cast<float*>(op->resident + L.fscale);
  op->kstore = op->resident + L.kstore;
  op->specR = reinterpret_cast<float2*>(op->work + L.specR);
  op->specS = reinterpret_cast<float2*>(op->work + L.specS);
  op->bsplit = d.prec != MDC_FP32 ? reinterpret_cast<unsigned int*>(op->work + L.bsplit) : nullptr;
  op->prof = false;
  op->tw_host = parent->tw_host;
  op->tune_ncols = parent->tune_ncols;
  op->tune_family[0] = parent->tune_family[0];
  op->tune_family[1] = parent->tune_family[1];
  bool ok = hipMemcpyAsync(op->tw, parent->tw, (size_t)d.nt * sizeof(float2), hipMemcpyDeviceToDevice, st) ==
                hipSuccess &&
            hipMemcpyAsync(op->fscale, parent->fscale, (size_t)d.nfmax * 4, hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (!ok) {
    delete op;
    return fail(MDC_EDEVICE, "copying the sub-grid tables failed");
  }
  const unsigned int* src = static_cast<const unsigned int*>(parent->kstore);
  unsigned int* dst = static_cast<unsigned int*>(op->kstore);
  const int ldk = kernel_ld(pd.nr), ldks = kernel_ld(nsub);
  const dim3 grid(4096), block(256);
  switch (d.prec) {
    case MDC_FP32:
      hipLaunchKernelGGL(gather_sub_kernel<0>, grid, block, 0, st, src, dst, idx, d.nfmax, pd.ns, ldk, nsub, ldks);
      break;
    case MDC_BF16X2:
      hipLaunchKernelGGL(gather_sub_kernel<2>, grid, block, 0, st, src, dst, idx, d.nfmax, pd.ns, ldk, nsub, ldks);
      break;
    default:
      hipLaunchKernelGGL(gather_sub_kernel<1>, grid, block, 0, st, src, dst, idx, d.nfmax, pd.ns, ldk, nsub, ldks);
      break;
  }
  const mdc_status s = check_launch("gather_sub_kernel");
  if (s != MDC_OK) {
    delete op;
    return s;
  }
  op->kernel_ready = parent->kernel_ready;
  *out = op;
  return MDC_OK;
}

mdc_status lsqr_check(const mdc_op* op, const mdc_desc& d, const lsqr_desc* ld);
size_t lsqr_work_bytes(const mdc_desc& d, const lsqr_desc& ld);
mdc_status lsqr_run(mdc_op* op, const mdc_desc& d, const lsqr_desc& ld, const float* b, float* x, double* hist,
                    void* work, hipStream_t st);
mdc_status cgls_run(mdc_op* op, const mdc_desc& d, const lsqr_desc& ld, const float* b, float* x, double* hist,
                    void* work, hipStream_t st);

// One application of the solver's operator (MDC or Marchenko) to in_scale * in (in_scale a
// device scalar, or nullptr for 1); Marchenko vectors are two contiguous blocks of `half`
// elements; tiled: vectors in the tiled time layout (fft_tile).
mdc_status apply_op(mdc_op* op, int kind, const int* onset, int nv, int adjoint, const float* in, float* out,
                    size_t half, hipStream_t st, const double* in_scale, const Recur* rec, int tiled) {
  if (kind == MDC_OP_MARCHENKO)
    return apply_marchenko(op, onset, nv, in, in + half, out, out + half, adjoint, st, 0, in_scale, rec, tiled);
  return apply_plain(op, in, out, nv, adjoint, st, onset, in_scale, rec, nullptr, tiled);
}
}  // namespace mdc

namespace {

// Spectra of mdc_apply_noalloc: a fixed device array instead of caller memory.  In host code the
// array's name is not a device address; the address comes from hipGetSymbolAddress, once per
// device, with that device current.  Every launch writes all of the scratch it later reads
// (transforms, split pass, per-frequency maxima), so nothing needs clearing between calls.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

mdc_status scratch_on_device(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(MDC_EDEVICE, "no usable current device for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MDC_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MDC_OK;
}

}  // namespace

extern "C" {

const char* mdc_last_error(void) { return g_err; }

mdc_status mdc_query_sizes(const mdc_desc* desc, size_t* resident_bytes, size_t* workspace_bytes) {
  mdc_status s = check_desc(desc);
  if (s != MDC_OK) return s;
  const Layout L = layout_of(*desc);
  if (resident_bytes) *resident_bytes = L.resident;
  if (workspace_bytes) *workspace_bytes = L.work;
  return MDC_OK;
}

mdc_status mdc_create(const mdc_desc* desc, void* resident, void* workspace, void* stream, mdc_op** out) {
  mdc_status s = check_desc(desc);
  if (s != MDC_OK) return s;
  if (!out) return fail(MDC_EINVAL, "out is NULL");
  if (!resident || !aligned(resident, kAlign)) return fail(MDC_EINVAL, "resident must be non-NULL and 256-byte aligned");
  if (!workspace || !aligned(workspace, kAlign)) return fail(MDC_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  const Layout L = layout_of(*desc);
  mdc_op* op = new (std::nothrow) mdc_op();
  if (!op) return fail(MDC_ENOMEM, "host allocation failed");
  op->d = *desc;
  op->resident = static_cast<char*>(resident);
  op->work = static_cast<char*>(workspace);
  op->tw = reinterpret_cast<float2*>(op->resident + L.tw);
  op->fscale = reinterpret_cast<float*>(op->resident + L.fscale);
  op->kstore = op->resident + L.kstore;
  op->specR = reinterpret_cast<float2*>(op->work + L.specR);
  op->specS = reinterpret_cast<float2*>(op->work + L.specS);
  op->bsplit = desc->prec != MDC_FP32 ? reinterpret_cast<unsigned int*>(op->work + L.bsplit) : nullptr;
  op->kernel_ready = false;
  op->prof = false;
  // FFT table in FP64, rounded once: tw[k] = exp(-2 pi i k / nt)
  op->tw_host.resize(desc->nt);
  for (int k = 0; k < desc->nt; ++k) {
    const double a = -2.0 * M_PI * (double)k / (double)desc->nt;
    op->tw_host[k] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(op->tw, op->tw_host.data(), (size_t)desc->nt * sizeof(float2), hipMemcpyHostToDevice, st) !=
      hipSuccess) {
    delete op;
    return fail(MDC_EDEVICE, "uploading FFT table failed");
  }
  // set-up of the static scratch of mdc_apply_noalloc on this device (its address is looked up
  // here, outside any capture; a failure is reported by mdc_apply_noalloc itself)
  char* sp = nullptr;
  (void)scratch_on_device(&sp);
  *out = op;
  return MDC_OK;
}

mdc_status mdc_set_kernel(mdc_op* op, const void* K, double scale, const float* col_weight, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  if (!K || !aligned(K, 8)) return fail(MDC_EINVAL, "K must be non-NULL and 8-byte aligned");
  if (col_weight && !aligned(col_weight, 4)) return fail(MDC_EINVAL, "col_weight must be 4-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const float2* k = static_cast<const float2*>(K);
  mdc_status s = MDC_OK;
  switch (op->d.prec) {
    case MDC_FP32: s = launch_load<StoreF32>(op, k, scale, col_weight, st); break;
    case MDC_BF16: s = launch_load<StoreBF16>(op, k, scale, col_weight, st); break;
    case MDC_BF16X2: s = launch_load<StoreBF16X2>(op, k, scale, col_weight, st); break;
    case MDC_FP16S:
    case MDC_FP16:
      if (hipMemsetAsync(op->fscale, 0, (size_t)op->d.nfmax * 4, st) != hipSuccess)
        return fail(MDC_EDEVICE, "clearing the scale table failed");
      if ((s = launch_load<StoreMax>(op, k, scale, col_weight, st)) != MDC_OK) return s;
      if ((s = fp16_scales_launch(op->fscale, op->d.nfmax, st)) != MDC_OK) return s;
      s = launch_load<StoreF16S>(op, k, scale, col_weight, st);
      break;
  }
  if (s == MDC_OK) op->kernel_ready = true;
  return s;
}

mdc_status mdc_set_kernel_time(mdc_op* op, const float* g, int conj, double scale, const float* col_weight, void* temp,
                               size_t temp_bytes, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  const mdc_desc& d = op->d;
  if (!g || !aligned(g, 4)) return fail(MDC_EINVAL, "g must be non-NULL and 4-byte aligned");
  const size_t need = (size_t)8 * d.nfmax * d.ns * d.nr;
  const bool in_place = temp == nullptr;
  if (in_place && !(d.prec == MDC_FP32 && d.nr % 4 == 0))
    return fail(MDC_EINVAL, "temp may be NULL only for complex64 storage with nr a multiple of 4");
  if (!in_place && (!aligned(temp, 256) || temp_bytes < need))
    return fail(MDC_ENOMEM, "temp needs %zu bytes, 256-byte aligned", need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float2* spec = in_place ? static_cast<float2*>(op->kstore) : static_cast<float2*>(temp);
  // orthogonal FFT of every trace (s, r), then x sqrt(nt): the unnormalised DFT of Eq.2's kernel
  FftSeg seg{g, nullptr, conj ? 1 : 0, 0};
  mdc_status s = rfft_launch(op->tw, d.nt, d.nfmax, d.ns, d.nr, d.nr, seg, spec, st);
  if (s != MDC_OK) return s;
  return mdc_set_kernel(op, spec, scale * std::sqrt((double)d.nt), col_weight, stream);
}

mdc_status mch_greens(mdc_op* op, int nv, const float* fminus, const float* fd, const float* fm, float* gminus,
                      float* gplus_conj, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  return apply_greens(op, nv, fminus, fd, fm, gminus, gplus_conj, static_cast<hipStream_t>(stream));
}

mdc_status mch_neumann_query(const mdc_op* op, int nv, size_t* work_bytes) {
  if (!op || !work_bytes) return fail(MDC_EINVAL, "NULL argument");
  *work_bytes = 2 * align_up((size_t)2 * op->d.nt * op->d.ns * nv * 4, 256);
  return MDC_OK;
}

mdc_status mch_neumann(mdc_op* op, const int* onset, int nv, const float* d, float* f, int nterms, void* work,
                       size_t work_bytes, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  if (op->d.ns != op->d.nr) return fail(MDC_EINVAL, "Marchenko operator needs ns == nr");
  if (nv < 1 || 2 * nv > op->d.max_cols) return fail(MDC_EINVAL, "2*nv outside [2, max_cols]");
  return apply_neumann(op, onset, nv, d, f, nterms, work, work_bytes, static_cast<hipStream_t>(stream));
}

mdc_status mdc_synth_kernel(mdc_op* op, const mdc_synth_desc* sd, void* stream) {
  if (!op || !sd) return fail(MDC_EINVAL, "op or descriptor is NULL");
  StoreRef ref{op->kstore, op->fscale, op->d.nfmax, op->d.ns, op->d.nr, kernel_ld(op->d.nr)};
  mdc_status s = synth_launch(op->d, *sd, ref, static_cast<hipStream_t>(stream));
  if (s == MDC_OK) op->kernel_ready = true;
  return s;
}

mdc_status mdc_kernel_element(mdc_op* op, int f, int s, int r, void* stream, float* re, float* im) {
  if (!op || !re || !im) return fail(MDC_EINVAL, "NULL argument");
  const mdc_desc& d = op->d;
  if (f < 0 || f >= d.nfmax || s < 0 || s >= d.ns || r < 0 || r >= d.nr) return fail(MDC_EINVAL, "index out of range");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int ldk = kernel_ld(d.nr);
  const size_t row = (size_t)f * d.ns + s;
  const char* base = static_cast<const char*>(op->kstore);
  unsigned int w[2] = {0u, 0u};
  float2 v{0.f, 0.f};
  float sf = 1.f;
  bool ok = true;
  switch (d.prec) {
    case MDC_FP32:
      ok = hipMemcpyAsync(&v, base + (row * ldk + r) * 8, 8, hipMemcpyDeviceToHost, st) == hipSuccess;
      break;
    case MDC_FP16S:
    case MDC_FP16:
      ok = hipMemcpyAsync(&w[0], base + (row * ldk + r) * 4, 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
           hipMemcpyAsync(&sf, op->fscale + f, 4, hipMemcpyDeviceToHost, st) == hipSuccess;
      break;
    case MDC_BF16:
      ok = hipMemcpyAsync(&w[0], base + (row * ldk + r) * 4, 4, hipMemcpyDeviceToHost, st) == hipSuccess;
      break;
    case MDC_BF16X2: {
      const size_t g = row * (size_t)ldk * 8 + (size_t)(r >> 2) * 32 + (r & 3) * 4;
      ok = hipMemcpyAsync(&w[0], base + g, 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
           hipMemcpyAsync(&w[1], base + g + 16, 4, hipMemcpyDeviceToHost, st) == hipSuccess;
      break;
    }
  }
  if (!ok || hipStreamSynchronize(st) != hipSuccess) return fail(MDC_EDEVICE, "reading kernel element failed");
  auto bf = [](unsigned int h) {
    const unsigned int u = h << 16;
    float x;
    memcpy(&x, &u, 4);
    return x;
  };
  auto hf = [](unsigned int h) {
    _Float16 x;
    const unsigned short b = (unsigned short)h;
    memcpy(&x, &b, 2);
    return (float)x;
  };
  switch (d.prec) {
    case MDC_FP32: *re = v.x; *im = v.y; break;
    case MDC_FP16S:
    case MDC_FP16: *re = hf(w[0] & 0xFFFFu) / sf; *im = hf(w[0] >> 16) / sf; break;
    case MDC_BF16: *re = bf(w[0] & 0xFFFFu); *im = bf(w[0] >> 16); break;
    case MDC_BF16X2: *re = bf(w[0] & 0xFFFFu) + bf(w[1] & 0xFFFFu); *im = bf(w[0] >> 16) + bf(w[1] >> 16); break;
  }
  return MDC_OK;
}

mdc_status mdc_forward(mdc_op* op, const float* x, float* y, int nv, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  return apply_plain(op, x, y, nv, 0, static_cast<hipStream_t>(stream));
}

mdc_status mdc_adjoint(mdc_op* op, const float* y, float* x, int nv, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  return apply_plain(op, y, x, nv, 1, static_cast<hipStream_t>(stream));
}

mdc_status mdc_apply_noalloc(mdc_op* op, int adjoint, const float* in, float* out, int nv, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  if (adjoint != 0 && adjoint != 1) return fail(MDC_EINVAL, "adjoint must be 0 or 1");
  if (nv < 1) return fail(MDC_EINVAL, "nv=%d must be positive", nv);
  Spectra ws{};
  ws.d = op->d;
  ws.d.max_cols = nv;  // the buffers are carved for this width only
  const Layout L = layout_of(ws.d);
  if (L.work > kScratchBytes)
    return fail(MDC_ENOMEM, "an apply of %d columns needs %zu bytes of spectra; the static scratch holds %zu", nv,
                L.work, kScratchBytes);
  char* base = nullptr;
  mdc_status s = scratch_on_device(&base);
  if (s != MDC_OK) return s;
  ws.R = reinterpret_cast<float2*>(base + L.specR);
  ws.S = reinterpret_cast<float2*>(base + L.specS);
  ws.split = op->d.prec != MDC_FP32 ? reinterpret_cast<unsigned int*>(base + L.bsplit) : nullptr;
  return apply_plain(op, in, out, nv, adjoint, static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr, &ws);
}

mdc_status mch_forward(mdc_op* op, const int* onset, int nv, const float* in0, const float* in1, float* out0,
                       float* out1, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  return apply_marchenko(op, onset, nv, in0, in1, out0, out1, 0, static_cast<hipStream_t>(stream));
}

mdc_status mch_adjoint(mdc_op* op, const int* onset, int nv, const float* in0, const float* in1, float* out0,
                       float* out1, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  return apply_marchenko(op, onset, nv, in0, in1, out0, out1, 1, static_cast<hipStream_t>(stream));
}

mdc_status mch_data(mdc_op* op, const int* onset, int nv, const float* fd, float* d0, float* d1, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  return apply_mch_data(op, onset, nv, fd, d0, d1, static_cast<hipStream_t>(stream));
}

static void tune_key(const mdc_op* op, char* buf, size_t n) {
  const mdc_desc& d = op->d;
  snprintf(buf, n, "gfx950 prec=%d nt=%d nfmax=%d ns=%d nr=%d max_cols=%d", (int)d.prec, d.nt, d.nfmax, d.ns, d.nr,
           d.max_cols);
}

// Parse `"name": [a, b, ...]` from a JSON line into v.
static bool parse_array(const char* line, const char* name, std::vector<int>& v) {
  char pat[64];
  snprintf(pat, sizeof pat, "\"%s\": [", name);
  const char* p = strstr(line, pat);
  if (!p) return false;
  p += strlen(pat);
  v.clear();
  while (*p && *p != ']') {
    char* end = nullptr;
    const long x = strtol(p, &end, 10);
    if (end == p) return false;
    v.push_back((int)x);
    p = end;
    while (*p == ',' || *p == ' ') ++p;
  }
  return *p == ']';
}

mdc_status mdc_autotune(mdc_op* op, const char* cache_path, void* stream, int* measured) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  char key[160];
  tune_key(op, key, sizeof key);
  if (measured) *measured = 0;
  if (cache_path) {
    if (FILE* fh = fopen(cache_path, "r")) {
      char line[8192];
      char kpat[200];
      snprintf(kpat, sizeof kpat, "\"key\": \"%s\"", key);
      bool found = false;
      while (fgets(line, sizeof line, fh)) {
        if (!strstr(line, kpat)) continue;
        std::vector<int> nc, fw, ad;
        if (parse_array(line, "ncols", nc) && parse_array(line, "fwd", fw) && parse_array(line, "adj", ad) &&
            !nc.empty() && nc.size() == fw.size() && nc.size() == ad.size()) {
          op->tune_ncols = nc;
          op->tune_family[0] = fw;
          op->tune_family[1] = ad;
          op->tune_gen += 1;
          found = true;
        }
      }
      fclose(fh);
      if (found) return MDC_OK;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  static const int cand[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  std::vector<int> nc;
  for (int c : cand)
    if (c <= op->d.max_cols) nc.push_back(c);
  if (nc.empty() || nc.back() != op->d.max_cols) nc.push_back(op->d.max_cols);
  const std::vector<int> fams = {kFamGemv, kFamGemm64, kFamGemm32};
  std::vector<int> best[2];
  for (int dir = 0; dir < 2; ++dir) {
    for (int n : nc) {
      int bf = -1;
      float bt = 3.0e38f;
      for (int fam : fams) {
        if (fam == kFamGemv && n > 16) continue;  // streaming kernels re-read the kernel every 8 columns
        if (fam == kFamGemm32 && n > 64 && op->d.prec == MDC_FP32) continue;  // 32-column FP32 tiles
        const float t = time_family(op, fam, dir, n, st);
        if (t < bt) { bt = t; bf = fam; }
      }
      if (bf < 0) return fail(MDC_EDEVICE, "autotune: no product family ran");
      best[dir].push_back(bf);
    }
  }
  if (hipGetLastError() != hipSuccess) return fail(MDC_EDEVICE, "autotune: a timing launch failed");
  op->tune_ncols = nc;
  op->tune_family[0] = best[0];
  op->tune_family[1] = best[1];
  op->tune_gen += 1;
  if (measured) *measured = 1;
  if (cache_path) {
    if (FILE* fh = fopen(cache_path, "a")) {
      fprintf(fh, "{\"key\": \"%s\", \"ncols\": [", key);
      for (size_t i = 0; i < nc.size(); ++i) fprintf(fh, "%s%d", i ? ", " : "", nc[i]);
      fprintf(fh, "], \"fwd\": [");
      for (size_t i = 0; i < nc.size(); ++i) fprintf(fh, "%s%d", i ? ", " : "", best[0][i]);
      fprintf(fh, "], \"adj\": [");
      for (size_t i = 0; i < nc.size(); ++i) fprintf(fh, "%s%d", i ? ", " : "", best[1][i]);
      fprintf(fh, "]}\n");
      fclose(fh);
    }
  }
  return MDC_OK;
}

mdc_status mdc_tune_table(const mdc_op* op, int cap, int* count, int* ncols, int* fwd_family, int* adj_family) {
  if (!op || !count) return fail(MDC_EINVAL, "NULL argument");
  *count = (int)op->tune_ncols.size();
  for (int i = 0; i < *count && i < cap; ++i) {
    if (ncols) ncols[i] = op->tune_ncols[i];
    if (fwd_family) fwd_family[i] = op->tune_family[0][i];
    if (adj_family) adj_family[i] = op->tune_family[1][i];
  }
  return MDC_OK;
}

mdc_status mdc_profile(mdc_op* op, int enable) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  op->prof = enable != 0;
  return MDC_OK;
}

mdc_status mdc_profile_read(mdc_op* op, double ms[4], int counts[4]) {
  if (!op || !ms || !counts) return fail(MDC_EINVAL, "NULL argument");
  for (int i = 0; i < 4; ++i) { ms[i] = 0.0; counts[i] = 0; }
  mdc_status st = MDC_OK;
  for (auto& e : op->evs) {
    float t = 0.f;
    if (hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) {
      st = fail(MDC_EDEVICE, "reading profile events failed");
    } else {
      ms[e.stage] += t;
      counts[e.stage] += 1;
    }
    op->pool.push_back(e.a);
    op->pool.push_back(e.b);
  }
  op->evs.clear();
  return st;
}

mdc_status lsqr_query_sizes(const mdc_op* op, const lsqr_desc* ld, size_t* work_bytes) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  mdc_status s = lsqr_check(op, op->d, ld);
  if (s != MDC_OK) return s;
  if (!work_bytes) return fail(MDC_EINVAL, "work_bytes is NULL");
  *work_bytes = lsqr_work_bytes(op->d, *ld);
  return MDC_OK;
}

mdc_status lsqr_solve(mdc_op* op, const lsqr_desc* ld, const float* b, float* x, double* hist, void* work,
                      size_t work_bytes, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  mdc_status s = lsqr_check(op, op->d, ld);
  if (s != MDC_OK) return s;
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  if ((s = check_vec(b, "b")) != MDC_OK) return s;
  if ((s = check_vec(x, "x")) != MDC_OK) return s;
  if (!work || !aligned(work, 256)) return fail(MDC_EINVAL, "work must be non-NULL and 256-byte aligned");
  if (work_bytes < lsqr_work_bytes(op->d, *ld))
    return fail(MDC_ENOMEM, "work has %zu bytes, %zu needed", work_bytes, lsqr_work_bytes(op->d, *ld));
  if (hist && !aligned(hist, 8)) return fail(MDC_EINVAL, "hist must be 8-byte aligned");
  return lsqr_run(op, op->d, *ld, b, x, hist, work, static_cast<hipStream_t>(stream));
}

mdc_status cgls_solve(mdc_op* op, const lsqr_desc* ld, const float* b, float* x, double* hist, void* work,
                      size_t work_bytes, void* stream) {
  if (!op) return fail(MDC_EINVAL, "op is NULL");
  mdc_status s = lsqr_check(op, op->d, ld);
  if (s != MDC_OK) return s;
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  if ((s = check_vec(b, "b")) != MDC_OK) return s;
  if ((s = check_vec(x, "x")) != MDC_OK) return s;
  if (!work || !aligned(work, 256)) return fail(MDC_EINVAL, "work must be non-NULL and 256-byte aligned");
  if (work_bytes < lsqr_work_bytes(op->d, *ld))
    return fail(MDC_ENOMEM, "work has %zu bytes, %zu needed", work_bytes, lsqr_work_bytes(op->d, *ld));
  if (hist && !aligned(hist, 8)) return fail(MDC_EINVAL, "hist must be 8-byte aligned");
  return cgls_run(op, op->d, *ld, b, x, hist, work, static_cast<hipStream_t>(stream));
}

mdc_status mdc_destroy(mdc_op* op) {
  if (!op) return MDC_OK;
  if (op->lsqr_exec) (void)hipGraphExecDestroy(op->lsqr_exec);
  if (op->cap_stream) {
    (void)hipStreamSynchronize(op->cap_stream);
    (void)hipStreamDestroy(op->cap_stream);
  }
  for (auto& e : op->evs) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto e : op->pool) (void)hipEventDestroy(e);
  delete op;
  return MDC_OK;
}

}  // extern "C"
