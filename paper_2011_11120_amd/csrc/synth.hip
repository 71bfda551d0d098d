// Device generator of the synthetic reflection kernel (input data, untimed
// setup).  It stands in for the paper's finite-difference dataset
// (Benchmarking section), which is not available: a sum of hyperbolic events
// with a deconvolved Ricker-shaped spectrum plus complex Gaussian noise,
//
//   K[f,s,r] = kappa dA W(f_f) sum_k a_k exp(-2 pi i f_f tau_k(s,r))
//              + noise sigma_f (n1 + i n2) / sqrt(2),
//   tau_k = sqrt(t0_k^2 + h^2 / v_k^2),  f_f = f / (nt dt),
//   W(f) = 2 f^2 / (sqrt(pi) fp^3) exp(-f^2 / fp^2)   (Ricker spectrum),
//   sigma_f = kappa dA W(f_f) sqrt(sum_k a_k^2),
//
// evaluated in FP64 and rounded once to the storage format.  The noise uses the
// SplitMix64 output finaliser (Steele, Lea & Flood, OOPSLA 2014) as a
// counter-based generator keyed by (seed, stream, counter): 53-bit uniforms on
// (0,1) and Box-Muller normals (cosine branch).  Normal j of a stream takes
// uniforms 2j and 2j+1; n1, n2 are normals 2q and 2q+1 of stream 4 with
// q = (f * N + s) * N + r over the full N = nx^2 grid.
#include <cmath>

#include "common.hpp"
#include "store.hpp"

namespace mdc {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kStreamMul = 0xD1B54A32D192ED03ull;
constexpr int kNoiseStream = 4;
constexpr int kMaxEvents = 64;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform(uint64_t key, uint64_t counter) {
  const uint64_t b = mix64(key + (counter + 1ull) * kGolden) >> 11;
  return ((double)b + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double normal(uint64_t key, uint64_t j) {
  const double u0 = uniform(key, 2ull * j);
  const double u1 = uniform(key, 2ull * j + 1ull);
  return sqrt(-2.0 * log(u0)) * cos(2.0 * M_PI * u1);
}

struct SynthArgs {
  int nfmax, ns, nr, ldk, nt, nx, nev;
  double dt, dx, fp, kappa, noise, area;
  uint64_t key;
  double amp[kMaxEvents], t0sq[kMaxEvents], inv_v2[kMaxEvents];
};

template <typename Store>
__global__ __launch_bounds__(256) void synth_kernel(SynthArgs a, const int* __restrict__ s_index,
                                                    const int* __restrict__ r_index, Store out) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (r >= a.ldk) return;
  if (r >= a.nr) {  // zero pad columns
    for (int f = 0; f < a.nfmax; ++f) out.put(f, s, r, 0.0, 0.0);
    return;
  }
  const int sg = s_index ? s_index[s] : s;
  const int rg = r_index ? r_index[r] : r;
  const double sx = (double)(sg / a.nx) * a.dx, sy = (double)(sg % a.nx) * a.dx;
  const double rx = (double)(rg / a.nx) * a.dx, ry = (double)(rg % a.nx) * a.dx;
  const double h2 = (sx - rx) * (sx - rx) + (sy - ry) * (sy - ry);
  double tau[kMaxEvents];
  double rms2 = 0.0;
  for (int k = 0; k < a.nev; ++k) {
    tau[k] = sqrt(a.t0sq[k] + h2 * a.inv_v2[k]);
    rms2 += a.amp[k] * a.amp[k];
  }
  const double rms = sqrt(rms2);
  const uint64_t N = (uint64_t)a.nx * (uint64_t)a.nx;
  for (int f = 0; f < a.nfmax; ++f) {
    const double ff = (double)f / ((double)a.nt * a.dt);
    const double wf = a.kappa * a.area * (2.0 * ff * ff / (sqrt(M_PI) * a.fp * a.fp * a.fp)) *
                      exp(-(ff * ff) / (a.fp * a.fp));
    double re = 0.0, im = 0.0;
    for (int k = 0; k < a.nev; ++k) {
      const double cyc = ff * tau[k];
      const double frac = cyc - floor(cyc);
      re += a.amp[k] * cos(2.0 * M_PI * frac);
      im -= a.amp[k] * sin(2.0 * M_PI * frac);
    }
    const uint64_t q = ((uint64_t)f * N + (uint64_t)sg) * N + (uint64_t)rg;
    const double n1 = normal(a.key, 2ull * q);
    const double n2 = normal(a.key, 2ull * q + 1ull);
    const double sig = a.noise * wf * rms / sqrt(2.0);
    out.put(f, s, r, wf * re + sig * n1, wf * im + sig * n2);
  }
}

}  // namespace

mdc_status synth_launch(const mdc_desc& d, const mdc_synth_desc& sd, const StoreRef& st_ref, hipStream_t st) {
  if (sd.nev < 0 || sd.nev > kMaxEvents) return fail(MDC_EINVAL, "nev=%d must lie in [0, %d]", sd.nev, kMaxEvents);
  if (sd.nev > 0 && (!sd.amp || !sd.t0 || !sd.vel)) return fail(MDC_EINVAL, "event arrays must not be NULL");
  if (sd.nx <= 0) return fail(MDC_EINVAL, "nx must be positive");
  if (!sd.s_index && d.ns > sd.nx * sd.nx) return fail(MDC_EINVAL, "ns exceeds the nx*nx grid");
  if (!sd.r_index && d.nr > sd.nx * sd.nx) return fail(MDC_EINVAL, "nr exceeds the nx*nx grid");
  SynthArgs a{};
  a.nfmax = d.nfmax; a.ns = d.ns; a.nr = d.nr; a.ldk = st_ref.ldk; a.nt = d.nt; a.nx = sd.nx; a.nev = sd.nev;
  a.dt = sd.dt; a.dx = sd.dx; a.fp = sd.fp; a.kappa = sd.kappa; a.noise = sd.noise; a.area = sd.area;
  // key = mix64(seed * golden + (stream + 1) * stream_mul), as for every stream of the generator
  {
    uint64_t z = sd.seed * kGolden + (uint64_t)(kNoiseStream + 1) * kStreamMul;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    a.key = z ^ (z >> 31);
  }
  for (int k = 0; k < sd.nev; ++k) {
    a.amp[k] = sd.amp[k];
    a.t0sq[k] = sd.t0[k] * sd.t0[k];
    a.inv_v2[k] = 1.0 / (sd.vel[k] * sd.vel[k]);
  }
  const dim3 grid((st_ref.ldk + 255) / 256, d.ns);
  switch (d.prec) {
    case MDC_FP32:
      hipLaunchKernelGGL(synth_kernel<StoreF32>, grid, dim3(256), 0, st, a, sd.s_index, sd.r_index, StoreF32(st_ref));
      break;
    case MDC_BF16:
      hipLaunchKernelGGL(synth_kernel<StoreBF16>, grid, dim3(256), 0, st, a, sd.s_index, sd.r_index, StoreBF16(st_ref));
      break;
    case MDC_BF16X2:
      hipLaunchKernelGGL(synth_kernel<StoreBF16X2>, grid, dim3(256), 0, st, a, sd.s_index, sd.r_index,
                         StoreBF16X2(st_ref));
      break;
    case MDC_FP16S:
    case MDC_FP16: {
      // two passes: per-frequency maxima, power-of-two scales, then the scaled FP16 values
      if (hipMemsetAsync(st_ref.fscale, 0, (size_t)d.nfmax * 4, st) != hipSuccess)
        return fail(MDC_EDEVICE, "clearing the scale table failed");
      hipLaunchKernelGGL(synth_kernel<StoreMax>, grid, dim3(256), 0, st, a, sd.s_index, sd.r_index, StoreMax(st_ref));
      mdc_status s = check_launch("synth_kernel (max)");
      if (s != MDC_OK) return s;
      if ((s = fp16_scales_launch(st_ref.fscale, d.nfmax, st)) != MDC_OK) return s;
      hipLaunchKernelGGL(synth_kernel<StoreF16S>, grid, dim3(256), 0, st, a, sd.s_index, sd.r_index, StoreF16S(st_ref));
      break;
    }
  }
  return check_launch("synth_kernel");
}

}  // namespace mdc
