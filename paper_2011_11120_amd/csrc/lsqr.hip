// LSQR on the device (Paige & Saunders, ACM TOMS 8(1) 1982; damping 0, x0 = 0,
// fixed iteration count).  The paper solves the Marchenko equations (Eq.5)
// and the MDD equations (Eq.8) with a gradient solver (CGLS, 10 iterations);
// LSQR yields the same iterates in exact arithmetic.
//
// Vectors are FP32; every scalar of the recurrence (alpha, beta, rho, rhobar,
// c, s, theta, phi, phibar) and every norm is FP64 and lives on the device,
// so the host enqueues the whole solve without synchronising.  Norms are
// reduced in two fixed-shape stages (per-block FP64 partials, then one block),
// so results do not depend on scheduling.  By default the three-term
// recurrences and their partial norms run inside the operator's inverse
// transform (one partial per transform workgroup), leaving one x/w update
// pass per iteration.
#include <cmath>
#include <cstdlib>

#include "common.hpp"

namespace mdc {

mdc_status apply_op(mdc_op* op, int kind, const int* onset, int nv, int adjoint, const float* in, float* out,
                    size_t half, hipStream_t st, const double* in_scale = nullptr, const Recur* rec = nullptr,
                    int tiled = 0);

namespace {

constexpr int kThreads = 256;
constexpr int kParts = 1024;  // blocks of the first reduction stage

struct Scalars {
  double alpha, beta, rhobar, phibar;
  double cx, cw;        // x += cx w ; w = v + cw w
  double inv;           // reciprocal of the last norm (or 1 when it was 0)
  double uinv, vinv;    // 1/beta, 1/alpha: u and v are stored unnormalised (beta u, alpha v)
  int iter, pad;        // completed iterations (device-side, so every iteration's launches are identical)
  double gamma, qn, sn, rn;  // CGLS: ||s||^2 of the last step, last norms of q, s, r
  double part[kParts];  // stage-1 partial sums
};

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;  // valid in thread 0
}

// out = x + coef * y  (coef = sgn * (*c1 or 1) * (*c2 or 1)); partial sum of out^2
__global__ __launch_bounds__(kThreads) void lin_norm(float* out, const float* x, const float* y,
                                                     const double* __restrict__ c1, const double* __restrict__ c2,
                                                     double sgn, size_t n, Scalars* sc) {
  __shared__ double sh[kThreads / 64];
  const float coef = (float)(sgn * (c1 ? *c1 : 1.0) * (c2 ? *c2 : 1.0));
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    const float v = x[i] + coef * y[i];
    out[i] = v;
    acc += (double)v * (double)v;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) sc->part[blockIdx.x] = t;
}

// partial sums of x^2
__global__ __launch_bounds__(kThreads) void sumsq(const float* __restrict__ x, size_t n, Scalars* sc) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    acc += (double)x[i] * (double)x[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) sc->part[blockIdx.x] = t;
}

// norm = sqrt(sum of partials) into *dst; *inv = 1/norm (1 if norm == 0)
__global__ __launch_bounds__(kThreads) void finish_norm(const double* __restrict__ part, double* dst, double* inv,
                                                        int nparts) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  // eight loads in flight per thread (clamped, unconditional), added in the order of a plain strided loop
  for (int i0 = threadIdx.x; i0 < nparts; i0 += kThreads * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[i0 + u * kThreads < nparts ? i0 + u * kThreads : 0];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * kThreads < nparts) acc += v[u];
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(t);
    *dst = nrm;
    *inv = nrm > 0.0 ? 1.0 / nrm : 1.0;
  }
}

// w = v (= vinv * stored v), x = 0, phibar = beta, rhobar = alpha
__global__ __launch_bounds__(kThreads) void init_xw(float* __restrict__ x, float* __restrict__ w,
                                                    const float* __restrict__ v, size_t n, Scalars* sc,
                                                    double* hist) {
  const float vi = (float)sc->vinv;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    x[i] = 0.f;
    w[i] = v[i] * vi;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->phibar = sc->beta;
    sc->rhobar = sc->alpha;
    sc->iter = 0;
    if (hist) hist[0] = sc->beta;
  }
}

// Plane rotation of one LSQR step, in FP64, one thread.
__global__ void givens(Scalars* sc, double* hist) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int it = ++sc->iter;
  const double alpha = sc->alpha, beta = sc->beta, rhobar = sc->rhobar, phibar = sc->phibar;
  const double rho = hypot(rhobar, beta);
  if (rho > 0.0) {
    const double c = rhobar / rho, s = beta / rho;
    const double theta = s * alpha;
    const double phi = c * phibar;
    sc->rhobar = -c * alpha;
    sc->phibar = s * phibar;
    sc->cx = phi / rho;
    sc->cw = -theta / rho;
  } else {  // exact solution reached: leave x unchanged
    sc->cx = 0.0;
    sc->cw = 0.0;
  }
  if (hist) hist[it] = sc->phibar;
}

// x += cx w ; w = v + cw w  (v = vinv * stored v)
__global__ __launch_bounds__(kThreads) void update_xw(float* __restrict__ x, float* __restrict__ w,
                                                      const float* __restrict__ v, size_t n, const Scalars* sc) {
  const float cx = (float)sc->cx, cw = (float)sc->cw, vi = (float)sc->vinv;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    const float wi = w[i];
    x[i] += cx * wi;
    w[i] = v[i] * vi + cw * wi;
  }
}
void launch_update_xw(float* x, float* w, const float* v, size_t n, const Scalars* sc, hipStream_t st) {
  const size_t b = (n + kThreads - 1) / kThreads;
  const int gd = (int)(b < (size_t)kParts ? (b == 0 ? 1 : b) : kParts);
  hipLaunchKernelGGL(update_xw, dim3(gd), dim3(kThreads), 0, st, x, w, v, n, sc);
}

// ---------------------------------------------------------------- CGLS ----
// gamma = ||s||^2 (start), hist[0] = ||r||
__global__ void cg_init(Scalars* sc, double* hist) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  sc->gamma = sc->sn * sc->sn;
  sc->iter = 0;
  if (hist) hist[0] = sc->rn;
}
// alpha = gamma / ||q||^2
__global__ void cg_alpha(Scalars* sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double delta = sc->qn * sc->qn;
  sc->alpha = delta > 0.0 ? sc->gamma / delta : 0.0;
}
// x += alpha p ; r -= alpha q
__global__ __launch_bounds__(kThreads) void cg_xr(float* __restrict__ x, const float* __restrict__ p,
                                                  float* __restrict__ r, const float* __restrict__ q, size_t nm,
                                                  size_t nd, const Scalars* sc) {
  const float a = (float)sc->alpha;
  const size_t n = nm > nd ? nm : nd;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    if (i < nm) x[i] += a * p[i];
    if (i < nd) r[i] -= a * q[i];
  }
}
// beta = ||s||^2 / gamma ; gamma = ||s||^2 ; hist[it] = ||r||
__global__ void cg_beta(Scalars* sc, double* hist) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double g = sc->sn * sc->sn;
  sc->beta = sc->gamma > 0.0 ? g / sc->gamma : 0.0;
  sc->gamma = g;
  const int it = ++sc->iter;
  if (hist) hist[it] = sc->rn;
}

inline int grid_for(size_t n) {
  const size_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < (size_t)kParts ? (b == 0 ? 1 : b) : kParts);
}

}  // namespace

size_t lsqr_scalars_bytes() { return align_up(sizeof(Scalars), 256); }

const double* lsqr_uinv(const LsqrState& s) { return &static_cast<Scalars*>(s.sc)->uinv; }
const double* lsqr_vinv(const LsqrState& s) { return &static_cast<Scalars*>(s.sc)->vinv; }

// The Paige-Saunders recurrences with u and v stored unnormalised: the stored u is
// beta u and the stored v is alpha v; uinv = 1/beta and vinv = 1/alpha are applied by
// every consumer as it reads them (the operator's input transform and identity terms,
// the next recurrence, the w update), which saves a read-write pass over each vector.

// beta u = b (u holds b on entry)
void lsqr_after_b(const LsqrState& s, hipStream_t st) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  const int gd = grid_for(s.data);
  hipLaunchKernelGGL(sumsq, dim3(gd), dim3(kThreads), 0, st, s.u, s.data, sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->beta, &sc->uinv, gd);
}

// alpha v = t2 (= A^H u), w = v, x = 0
void lsqr_after_init_adj(const LsqrState& s, hipStream_t st) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  const int gm = grid_for(s.model);
  hipLaunchKernelGGL(lin_norm, dim3(gm), dim3(kThreads), 0, st, s.v, s.t2, s.t2, (const double*)nullptr,
                     (const double*)nullptr, 0.0, s.model, sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->alpha, &sc->vinv, gm);
  hipLaunchKernelGGL(init_xw, dim3(gm), dim3(kThreads), 0, st, s.x, s.w, s.v, s.model, sc, s.hist);
}

// beta u = t - alpha u  (t = A v; the stored previous u times uinv is u)
void lsqr_after_fwd(const LsqrState& s, hipStream_t st) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  const int gd = grid_for(s.data);
  hipLaunchKernelGGL(lin_norm, dim3(gd), dim3(kThreads), 0, st, s.u, s.t, s.u, (const double*)&sc->alpha,
                     (const double*)&sc->uinv, -1.0, s.data, sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->beta, &sc->uinv, gd);
}

// alpha v = t2 - beta v  (t2 = A^H u); rotation; x += phi/rho w; w = v - theta/rho w
void lsqr_after_adj(const LsqrState& s, hipStream_t st) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  const int gm = grid_for(s.model);
  hipLaunchKernelGGL(lin_norm, dim3(gm), dim3(kThreads), 0, st, s.v, s.t2, s.v, (const double*)&sc->beta,
                     (const double*)&sc->vinv, -1.0, s.model, sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->alpha, &sc->vinv, gm);
  hipLaunchKernelGGL(givens, dim3(1), dim3(64), 0, st, sc, s.hist);
  launch_update_xw(s.x, s.w, s.v, s.model, sc, st);
}

// The same recurrences fused into the applies: the forward apply's inverse transform forms
// beta u = A v - alpha u in place and the adjoint's alpha v = A^H u - beta v, each workgroup
// leaving the FP64 sum of its squares in rpart; these finish the norms (and the rotation).
Recur lsqr_recur_fwd(const LsqrState& s) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  return Recur{&sc->alpha, &sc->uinv, -1.0f, s.rpart};
}
Recur lsqr_recur_adj(const LsqrState& s) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  return Recur{&sc->beta, &sc->vinv, -1.0f, s.rpart};
}
Recur lsqr_recur_init(const LsqrState& s) { return Recur{nullptr, nullptr, 0.f, s.rpart}; }
// alpha v = A^H u written by the adjoint itself; w = v, x = 0
void lsqr_after_init_adj_fused(const LsqrState& s, hipStream_t st) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  const int gm = grid_for(s.model);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, s.rpart, &sc->alpha, &sc->vinv, s.nparts_adj);
  hipLaunchKernelGGL(init_xw, dim3(gm), dim3(kThreads), 0, st, s.x, s.w, s.v, s.model, sc, s.hist);
}
void lsqr_after_fwd_fused(const LsqrState& s, hipStream_t st) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, s.rpart, &sc->beta, &sc->uinv, s.nparts_fwd);
}
void lsqr_after_adj_fused(const LsqrState& s, hipStream_t st) {
  Scalars* sc = static_cast<Scalars*>(s.sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, s.rpart, &sc->alpha, &sc->vinv, s.nparts_adj);
  hipLaunchKernelGGL(givens, dim3(1), dim3(64), 0, st, sc, s.hist);
  launch_update_xw(s.x, s.w, s.v, s.model, sc, st);
}

namespace {

struct Sizes {
  size_t model, data;        // element counts
  int qm, qd;                // traces per block of a model / data vector
  size_t bm, bd;             // elements per block (tiled: whole tiles)
  int blocks;                // blocks per vector (2 for the Marchenko system)
  int parts_fwd, parts_adj;  // partial-sum slots of the fused recurrences
};

// tiled: vectors in the transforms' tiled time layout (whole tiles, zero padding traces).
Sizes sizes_of(const mdc_desc& d, const lsqr_desc& ld, bool tiled) {
  Sizes z{};
  auto blk = [&](int q) { return tiled ? tiled_len(d.nt, q) : (size_t)d.nt * q; };
  if (ld.kind == MDC_OP_MARCHENKO) {
    z.qm = z.qd = d.ns * ld.nv;
    z.blocks = 2;
    z.parts_fwd = z.parts_adj = 2 * irfft_blocks(d.nt, d.ns, ld.nv);
  } else {
    z.qm = d.nr * ld.nv;
    z.qd = d.ns * ld.nv;
    z.blocks = 1;
    z.parts_fwd = irfft_blocks(d.nt, d.ns, ld.nv);
    z.parts_adj = irfft_blocks(d.nt, d.nr, ld.nv);
  }
  z.bm = blk(z.qm);
  z.bd = blk(z.qd);
  z.model = z.blocks * z.bm;
  z.data = z.blocks * z.bd;
  return z;
}

size_t parts_bytes_of(const Sizes& z) {
  return align_up((size_t)(z.parts_fwd > z.parts_adj ? z.parts_fwd : z.parts_adj) * sizeof(double), 256);
}

// Sized for the tiled layout (never smaller than the plain one) plus the solution in that layout.
size_t work_bytes_of(const Sizes& z) {
  size_t b = lsqr_scalars_bytes();
  b += 2 * align_up(z.data * 4, 256);   // u, t
  b += 3 * align_up(z.model * 4, 256);  // v, w, t2
  b += parts_bytes_of(z);               // partial sums of the fused recurrences
  b += align_up(z.model * 4, 256);      // x in the tiled layout (copied to the caller's x at the end)
  return b;
}

}  // namespace

mdc_status lsqr_check(const mdc_op* op, const mdc_desc& d, const lsqr_desc* ld) {
  if (!op || !ld) return fail(MDC_EINVAL, "NULL argument");
  if (ld->kind != MDC_OP_MDC && ld->kind != MDC_OP_MARCHENKO) return fail(MDC_EINVAL, "unknown operator kind");
  if (ld->niter < 0) return fail(MDC_EINVAL, "niter must be >= 0");
  if (ld->kind == MDC_OP_MARCHENKO) {
    if (d.ns != d.nr) return fail(MDC_EINVAL, "Marchenko needs ns == nr");
    if (ld->nv < 1 || 2 * ld->nv > d.max_cols) return fail(MDC_EINVAL, "2*nv outside [2, max_cols]");
    if (!ld->onset) return fail(MDC_EINVAL, "Marchenko needs onsets");
  } else if (ld->nv < 1 || ld->nv > d.max_cols) {
    return fail(MDC_EINVAL, "nv outside [1, max_cols]");
  }
  return MDC_OK;
}

size_t lsqr_work_bytes(const mdc_desc& d, const lsqr_desc& ld) { return work_bytes_of(sizes_of(d, ld, true)); }

__global__ void zero_vec(float* __restrict__ x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = 0.f;
}

__global__ void copy_f32(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Block b of a vector between the caller's layout [nt][Q] and the tiled layout (tiles of T
// traces, [nt][T] each, tile_len = nt * T): to_tiles writes every element of the tiled block,
// zeros on the padding traces; from_tiles writes the caller's block.
__global__ void to_tiles(float* __restrict__ dst, const float* __restrict__ src, int nt, int Q, int T,
                         size_t blk_tiled, size_t blk_plain, int blocks) {
  const size_t tile_len = (size_t)nt * T, total = blk_tiled * blocks;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / blk_tiled, e = i - b * blk_tiled;
    const size_t j = e / tile_len, r = e - j * tile_len;
    const int t = (int)(r / T), q = (int)(j * T + (r - (size_t)t * T));
    dst[i] = q < Q ? src[b * blk_plain + (size_t)t * Q + q] : 0.f;
  }
}
__global__ void from_tiles(float* __restrict__ dst, const float* __restrict__ src, int nt, int Q, int T,
                           size_t blk_tiled, size_t blk_plain, int blocks) {
  const size_t total = blk_plain * blocks;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / blk_plain, e = i - b * blk_plain;
    const int t = (int)(e / Q), q = (int)(e - (size_t)t * Q);
    dst[i] = src[b * blk_tiled + (size_t)(q / T) * nt * T + (size_t)t * T + (q % T)];
  }
}

void launch_to_tiles(float* dst, const float* src, int nt, int Q, int blocks, hipStream_t st) {
  const size_t blk = tiled_len(nt, Q);
  hipLaunchKernelGGL(to_tiles, dim3(grid_for(blk * blocks)), dim3(kThreads), 0, st, dst, src, nt, Q, fft_tile(nt, Q),
                     blk, (size_t)nt * Q, blocks);
}
void launch_from_tiles(float* dst, const float* src, int nt, int Q, int blocks, hipStream_t st) {
  const size_t blk = tiled_len(nt, Q);
  hipLaunchKernelGGL(from_tiles, dim3(grid_for((size_t)nt * Q * blocks)), dim3(kThreads), 0, st, dst, src, nt, Q,
                     fft_tile(nt, Q), blk, (size_t)nt * Q, blocks);
}

mdc_status lsqr_run(mdc_op* op, const mdc_desc& d, const lsqr_desc& ld, const float* b, float* x, double* hist,
                    void* work, hipStream_t st) {
  // Krylov vectors in the transforms' tiled layout (each transform workgroup reads or writes one
  // contiguous tile); MDC_LSQR_TILED=0 keeps the caller's [nt][n][nv] layout throughout.
  const char* tl = getenv("MDC_LSQR_TILED");
  const int tiled = (tl && tl[0] == '0') ? 0 : 1;
  const Sizes z = sizes_of(d, ld, tiled != 0);
  const Sizes zt = sizes_of(d, ld, true);  // the workspace layout (lsqr_work_bytes)
  char* p = static_cast<char*>(work);
  LsqrState S{};
  S.sc = p;
  p += lsqr_scalars_bytes();
  S.u = reinterpret_cast<float*>(p); p += align_up(zt.data * 4, 256);
  S.t = reinterpret_cast<float*>(p); p += align_up(zt.data * 4, 256);
  S.v = reinterpret_cast<float*>(p); p += align_up(zt.model * 4, 256);
  S.w = reinterpret_cast<float*>(p); p += align_up(zt.model * 4, 256);
  S.t2 = reinterpret_cast<float*>(p); p += align_up(zt.model * 4, 256);
  const char* f = getenv("MDC_LSQR_FUSE");
  if (!(f && f[0] == '0')) {
    S.rpart = reinterpret_cast<double*>(p);
    S.nparts_fwd = z.parts_fwd;
    S.nparts_adj = z.parts_adj;
  }
  p += parts_bytes_of(zt);
  S.x = tiled ? reinterpret_cast<float*>(p) : x;
  S.hist = hist;
  S.model = z.model;
  S.data = z.data;
  const int kind = ld.kind;
  const size_t half = z.bm;  // Marchenko block size (model == data)
  mdc_status s;

  if (tiled) {
    // u = b in tiles; the transforms write only the traces of a vector, so the padding traces
    // of every vector they write start at zero (the recurrences keep them there)
    launch_to_tiles(S.u, b, d.nt, z.qd, z.blocks, st);
    hipLaunchKernelGGL(zero_vec, dim3(grid_for(z.model)), dim3(kThreads), 0, st, S.v, z.model);
    if (!S.rpart) {  // the separate-pass recurrences read the transforms' outputs t and t2 whole
      hipLaunchKernelGGL(zero_vec, dim3(grid_for(z.data)), dim3(kThreads), 0, st, S.t, z.data);
      hipLaunchKernelGGL(zero_vec, dim3(grid_for(z.model)), dim3(kThreads), 0, st, S.t2, z.model);
    }
  } else {
    hipLaunchKernelGGL(copy_f32, dim3(grid_for(z.data)), dim3(kThreads), 0, st, S.u, b, z.data);
  }
  lsqr_after_b(S, st);
  if (S.rpart) {
    const Recur ri = lsqr_recur_init(S);
    if ((s = apply_op(op, kind, ld.onset, ld.nv, 1, S.u, S.v, half, st, lsqr_uinv(S), &ri, tiled)) != MDC_OK)
      return s;
    lsqr_after_init_adj_fused(S, st);
  } else {
    if ((s = apply_op(op, kind, ld.onset, ld.nv, 1, S.u, S.t2, half, st, lsqr_uinv(S), nullptr, tiled)) != MDC_OK)
      return s;
    lsqr_after_init_adj(S, st);
  }
  if ((s = check_launch("lsqr init")) != MDC_OK) return s;
  auto iteration = [&](hipStream_t q) -> mdc_status {
    mdc_status e;
    if (S.rpart) {
      const Recur rf = lsqr_recur_fwd(S);
      if ((e = apply_op(op, kind, ld.onset, ld.nv, 0, S.v, S.u, half, q, lsqr_vinv(S), &rf, tiled)) != MDC_OK)
        return e;
      lsqr_after_fwd_fused(S, q);
      const Recur ra = lsqr_recur_adj(S);
      if ((e = apply_op(op, kind, ld.onset, ld.nv, 1, S.u, S.v, half, q, lsqr_uinv(S), &ra, tiled)) != MDC_OK)
        return e;
      lsqr_after_adj_fused(S, q);
      return check_launch("lsqr iteration");
    }
    if ((e = apply_op(op, kind, ld.onset, ld.nv, 0, S.v, S.t, half, q, lsqr_vinv(S), nullptr, tiled)) != MDC_OK)
      return e;
    lsqr_after_fwd(S, q);
    if ((e = apply_op(op, kind, ld.onset, ld.nv, 1, S.u, S.t2, half, q, lsqr_uinv(S), nullptr, tiled)) != MDC_OK)
      return e;
    lsqr_after_adj(S, q);
    return check_launch("lsqr iteration");
  };
  // the solution in the caller's layout (after the last iteration on the stream)
  auto finish = [&]() -> mdc_status {
    if (!tiled) return MDC_OK;
    launch_from_tiles(x, S.x, d.nt, z.qm, z.blocks, st);
    return check_launch("lsqr solution");
  };
  if (ld.niter >= 1 && (s = iteration(st)) != MDC_OK) return s;  // eager: every kernel variant initialised
  if (ld.niter < 2) return finish();
  const char* g = getenv("MDC_LSQR_GRAPH");
  const bool use_graph = !op->prof && !(g && g[0] == '0');
  if (!use_graph) {
    for (int it = 2; it <= ld.niter; ++it)
      if ((s = iteration(st)) != MDC_OK) return s;
    return finish();
  }
  // Capture one iteration (identical launches every time: the iteration counter lives on the
  // device) on the op's private stream, then replay it on the caller's stream.
  const LsqrGraphKey key{kind, ld.nv, S.rpart != nullptr, tiled, op->tune_gen, forced_family(op), ld.onset, work, x, hist, b};
  if (!op->lsqr_exec || !(op->lsqr_key == key)) {
    if (op->lsqr_exec) {
      (void)hipGraphExecDestroy(op->lsqr_exec);
      op->lsqr_exec = nullptr;
    }
    if (!op->cap_stream && hipStreamCreate(&op->cap_stream) != hipSuccess)
      return fail(MDC_EDEVICE, "creating the capture stream failed");
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(MDC_EDEVICE, "hipStreamBeginCapture failed");
    const mdc_status cs = iteration(op->cap_stream);
    const hipError_t ce = hipStreamEndCapture(op->cap_stream, &graph);
    if (cs != MDC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    if (ce != hipSuccess || !graph) return fail(MDC_EDEVICE, "hipStreamEndCapture failed");
    const hipError_t ie = hipGraphInstantiate(&op->lsqr_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      op->lsqr_exec = nullptr;
      return fail(MDC_EDEVICE, "hipGraphInstantiate failed");
    }
    op->lsqr_key = key;
  }
  for (int it = 2; it <= ld.niter; ++it)
    if (hipGraphLaunch(op->lsqr_exec, st) != hipSuccess) return fail(MDC_EDEVICE, "hipGraphLaunch failed");
  return finish();
}

// CGLS (the paper's solver): conjugate gradients on the normal equations, x0 = 0, fixed niter.
// Vectors FP32 (r, q data-sized; s, p model-sized); gamma, alpha, beta and the norms FP64.
mdc_status cgls_run(mdc_op* op, const mdc_desc& d, const lsqr_desc& ld, const float* b, float* x, double* hist,
                    void* work, hipStream_t st) {
  const Sizes z = sizes_of(d, ld, false);  // the caller's layout (within the workspace sized for tiles)
  char* w = static_cast<char*>(work);
  Scalars* sc = reinterpret_cast<Scalars*>(w);
  w += lsqr_scalars_bytes();
  float* r = reinterpret_cast<float*>(w); w += align_up(z.data * 4, 256);
  float* q = reinterpret_cast<float*>(w); w += align_up(z.data * 4, 256);
  float* sv = reinterpret_cast<float*>(w); w += align_up(z.model * 4, 256);
  float* p = reinterpret_cast<float*>(w); w += align_up(z.model * 4, 256);
  // ||q|| and ||s|| from partial sums the inverse transforms leave (no separate pass)
  const char* f = getenv("MDC_LSQR_FUSE");
  double* rpart = (f && f[0] == '0') ? nullptr : reinterpret_cast<double*>(w);
  const Recur rnorm{nullptr, nullptr, 0.f, rpart};
  const Recur* rn = rpart ? &rnorm : nullptr;
  const size_t half = z.model / 2;
  const int gd = grid_for(z.data), gm = grid_for(z.model), gx = grid_for(z.model > z.data ? z.model : z.data);
  mdc_status s;
  // r = b ; s = A^H r ; p = s ; x = 0
  hipLaunchKernelGGL(copy_f32, dim3(gd), dim3(kThreads), 0, st, r, b, z.data);
  hipLaunchKernelGGL(sumsq, dim3(gd), dim3(kThreads), 0, st, r, z.data, sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->rn, &sc->inv, gd);
  if ((s = apply_op(op, ld.kind, ld.onset, ld.nv, 1, r, sv, half, st)) != MDC_OK) return s;
  hipLaunchKernelGGL(lin_norm, dim3(gm), dim3(kThreads), 0, st, p, sv, sv, (const double*)nullptr, (const double*)nullptr, 0.0, z.model, sc);
  hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->sn, &sc->inv, gm);
  hipLaunchKernelGGL(zero_vec, dim3(gm), dim3(kThreads), 0, st, x, z.model);
  hipLaunchKernelGGL(cg_init, dim3(1), dim3(64), 0, st, sc, hist);
  for (int it = 1; it <= ld.niter; ++it) {
    // q = A p ; alpha = gamma / ||q||^2 ; x += alpha p ; r -= alpha q
    if ((s = apply_op(op, ld.kind, ld.onset, ld.nv, 0, p, q, half, st, nullptr, rn)) != MDC_OK) return s;
    if (rpart) {
      hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, rpart, &sc->qn, &sc->inv, z.parts_fwd);
    } else {
      hipLaunchKernelGGL(sumsq, dim3(gd), dim3(kThreads), 0, st, q, z.data, sc);
      hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->qn, &sc->inv, gd);
    }
    hipLaunchKernelGGL(cg_alpha, dim3(1), dim3(64), 0, st, sc);
    hipLaunchKernelGGL(cg_xr, dim3(gx), dim3(kThreads), 0, st, x, p, r, q, z.model, z.data, sc);
    hipLaunchKernelGGL(sumsq, dim3(gd), dim3(kThreads), 0, st, r, z.data, sc);
    hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->rn, &sc->inv, gd);
    // s = A^H r ; beta = ||s||^2 / gamma ; p = s + beta p
    if ((s = apply_op(op, ld.kind, ld.onset, ld.nv, 1, r, sv, half, st, nullptr, rn)) != MDC_OK) return s;
    if (rpart) {
      hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, rpart, &sc->sn, &sc->inv, z.parts_adj);
    } else {
      hipLaunchKernelGGL(sumsq, dim3(gm), dim3(kThreads), 0, st, sv, z.model, sc);
      hipLaunchKernelGGL(finish_norm, dim3(1), dim3(kThreads), 0, st, sc->part, &sc->sn, &sc->inv, gm);
    }
    hipLaunchKernelGGL(cg_beta, dim3(1), dim3(64), 0, st, sc, hist);
    hipLaunchKernelGGL(lin_norm, dim3(gm), dim3(kThreads), 0, st, p, sv, p, (const double*)&sc->beta, (const double*)nullptr, 1.0, z.model, sc);
    if ((s = check_launch("cgls iteration")) != MDC_OK) return s;
  }
  return MDC_OK;
}

}  // namespace mdc
