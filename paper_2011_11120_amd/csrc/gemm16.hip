// Per-frequency complex kernel product on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulate) for the 16-bit storage formats:
// the reduced-precision variants of the many-point product (Eq.4 slices).
//
// Operands are split into bf16 hi + lo parts so the product keeps close to
// FP32 accuracy (the split-operand scheme of Henry, Tang & Heinecke,
// ARITH 2019):  K X ~ Khi Xhi + Khi Xlo + Klo Xhi.
//   BF16X2: K stored as hi + lo (8 bytes per complex), three products.
//   FP16S:  K stored as FP16 scaled by a power of two per frequency (4 bytes);
//           every FP16 value splits exactly into bf16 hi + lo in registers,
//           three products, the scale divided out of the result.
//   BF16:   K stored as bf16 (4 bytes), two products (Khi Xhi + Khi Xlo).
// The spectra X (or Y) arrive in FP32 and are split when staged into LDS.
//
// The complex product is the same real embedding as the FP32 kernel: the
// interleaved kernel is a real ns x 2nr matrix, and the B operand is built
// from complex values at fragment-read time (forward: (c, -d) / (d, c) pairs;
// adjoint: (e, f) / (f, -e) pairs), here by flipping and swapping the halves of
// 32-bit bf16 pairs.  One MFMA k-step consumes 16 complex kernel columns.
// Tiles: 128 output rows x 64 complex columns per 256-thread workgroup (four
// waves of 64 x 64 real outputs), 32-column slabs staged through LDS (the
// adjoint stages the kernel transposed so fragments stay contiguous), register
// prefetch of the next slab, XCD-aware workgroup numbering.
#include "common.hpp"
#include "store.hpp"

namespace mdc {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int BM = 128;  // output rows per workgroup
constexpr int BN = 64;   // complex output columns per workgroup
constexpr int BK = 32;   // complex reduction columns per slab
constexpr int LDW = 36;  // 32-bit words per LDS row: 32 complex + 4 pad

__device__ __forceinline__ unsigned int split_lo(float x, unsigned int hb) {
  return bf16_rne_bits(x - bf16_bits_to_f(hb));
}
// (re, im) FP32 -> hi and lo bf16 pair words
__device__ __forceinline__ void split_pair(float re, float im, unsigned int& hi, unsigned int& lo) {
  const unsigned int hr = bf16_rne_bits(re), hm = bf16_rne_bits(im);
  hi = hr | (hm << 16);
  lo = split_lo(re, hr) | (split_lo(im, hm) << 16);
}
__device__ __forceinline__ unsigned int swap16(unsigned int w) { return (w >> 16) | (w << 16); }

template <int FMT>
constexpr int a_loads() { return FMT == MDC_BF16X2 ? 8 : 4; }

template <int FMT, bool ADJ>
__global__ __launch_bounds__(kThreads, 2) void gemm16_kernel(const char* __restrict__ K, const float* __restrict__ fscale,
                                                             int ns, int nr, int ldk, const float2* __restrict__ Bsrc,
                                                             float2* __restrict__ Cdst, int ncols, int tiles_m,
                                                             int tiles_n, int nblocks) {
  __shared__ __attribute__((aligned(16))) unsigned int Ah[BM * LDW];
  __shared__ __attribute__((aligned(16))) unsigned int Al[BM * LDW];
  __shared__ __attribute__((aligned(16))) unsigned int Bh[BN * LDW];
  __shared__ __attribute__((aligned(16))) unsigned int Bl[BN * LDW];
  constexpr bool HAS_LO = FMT != MDC_BF16;

  const int b = blockIdx.x;
  const int q8 = nblocks >> 3, rem = nblocks & 7, xcd = b & 7;
  const int L = xcd * q8 + min(xcd, rem) + (b >> 3);
  const int tiles_per_f = tiles_m * tiles_n;
  const int f = L / tiles_per_f;
  const int t = L - f * tiles_per_f;
  const int mt = t % tiles_m, nt = t / tiles_m;
  const int M = ADJ ? nr : ns;
  const int KD = ADJ ? ns : nr;
  const int m0 = mt * BM, n0 = nt * BN;
  const size_t rowb = (FMT == MDC_BF16X2) ? (size_t)ldk * 8 : (size_t)ldk * 4;
  const char* Kf = K + (size_t)f * ns * rowb;
  const float2* Bf = Bsrc + (size_t)f * KD * ncols;
  float* Cf = reinterpret_cast<float*>(Cdst + (size_t)f * M * ncols);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, kb = lane >> 4;

  u4v pa[a_loads<FMT>()];
  float2 pb[8];

  auto load_slab = [&](int k0) {
#pragma unroll
    for (int q = 0; q < a_loads<FMT>(); ++q) {
      const int idx = tid + kThreads * q;
      u4v v = u4v{0u, 0u, 0u, 0u};
      if constexpr (FMT == MDC_BF16X2) {
        if (!ADJ) {
          const int row = idx >> 4, c = idx & 15, gi = c >> 1, half = c & 1;
          const int m = m0 + row, col = k0 + 4 * gi;
          if (m < ns && col < ldk)
            v = *reinterpret_cast<const u4v*>(Kf + (size_t)m * rowb + (size_t)(col >> 2) * 32 + half * 16);
        } else {  // consecutive lanes take consecutive kernel rows (conflict-free transposed LDS stores)
          const int srow = idx & 31, c = idx >> 5, gi = c >> 1, half = c & 1;
          const int s = k0 + srow, col = m0 + 4 * gi;
          if (s < ns && col < ldk)
            v = *reinterpret_cast<const u4v*>(Kf + (size_t)s * rowb + (size_t)(col >> 2) * 32 + half * 16);
        }
      } else {
        if (!ADJ) {
          const int row = idx >> 3, c4 = idx & 7;
          const int m = m0 + row, col = k0 + 4 * c4;
          if (m < ns && col < ldk) v = *reinterpret_cast<const u4v*>(Kf + (size_t)m * rowb + (size_t)col * 4);
        } else {
          const int srow = idx & 31, c4 = idx >> 5;
          const int s = k0 + srow, col = m0 + 4 * c4;
          if (s < ns && col < ldk) v = *reinterpret_cast<const u4v*>(Kf + (size_t)s * rowb + (size_t)col * 4);
        }
      }
      pa[q] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + kThreads * q;
      const int krow = idx & 31, c2 = idx >> 5;  // consecutive lanes: consecutive LDS words
      const int kk = k0 + krow, v = n0 + 2 * c2;
      const float2* src = Bf + (size_t)kk * ncols;
      pb[2 * q] = (kk < KD && v < ncols) ? src[v] : make_float2(0.f, 0.f);
      pb[2 * q + 1] = (kk < KD && v + 1 < ncols) ? src[v + 1] : make_float2(0.f, 0.f);
    }
  };

  auto store_slab = [&]() {
#pragma unroll
    for (int q = 0; q < a_loads<FMT>(); ++q) {
      const int idx = tid + kThreads * q;
      const u4v v = pa[q];
      const unsigned int w[4] = {v.x, v.y, v.z, v.w};
      unsigned int hi[4], lo[4];
      unsigned int* dst_h;
      unsigned int* dst_l;
      int rowl, coll;  // forward: (row, first column) ; adjoint: (first r, s)
      if constexpr (FMT == MDC_BF16X2) {
        const int half = ADJ ? ((idx >> 5) & 1) : (idx & 1);
        if (!ADJ) { rowl = idx >> 4; coll = 4 * ((idx & 15) >> 1); }
        else { coll = idx & 31; rowl = 4 * ((idx >> 5) >> 1); }
#pragma unroll
        for (int h = 0; h < 4; ++h) hi[h] = w[h];
        dst_h = half ? Al : Ah;
        dst_l = nullptr;
      } else {
        if (!ADJ) { rowl = idx >> 3; coll = 4 * (idx & 7); }
        else { coll = idx & 31; rowl = 4 * (idx >> 5); }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          if constexpr (FMT == MDC_FP16S) {
            const float re = f16_bits_to_f(w[h] & 0xFFFFu), im = f16_bits_to_f(w[h] >> 16);
            split_pair(re, im, hi[h], lo[h]);  // exact: an FP16 value is bf16 hi + lo
          } else {
            hi[h] = w[h];
            lo[h] = 0u;
          }
        }
        dst_h = Ah;
        dst_l = HAS_LO ? Al : nullptr;
      }
      if (!ADJ) {
        *reinterpret_cast<u4v*>(&dst_h[rowl * LDW + coll]) = u4v{hi[0], hi[1], hi[2], hi[3]};
        if (dst_l) *reinterpret_cast<u4v*>(&dst_l[rowl * LDW + coll]) = u4v{lo[0], lo[1], lo[2], lo[3]};
      } else {  // transposed: A[r][s]
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          dst_h[(rowl + h) * LDW + coll] = hi[h];
          if (dst_l) dst_l[(rowl + h) * LDW + coll] = lo[h];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + kThreads * q;
      const int krow = idx & 31, c2 = idx >> 5;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        unsigned int hi, lo;
        split_pair(pb[2 * q + h].x, pb[2 * q + h].y, hi, lo);
        Bh[(2 * c2 + h) * LDW + krow] = hi;
        Bl[(2 * c2 + h) * LDW + krow] = lo;
      }
    }
  };

  f4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  const int nslabs = (KD + BK - 1) / BK;
  load_slab(0);
  for (int sl = 0; sl < nslabs; ++sl) {
    __syncthreads();  // previous slab fully consumed
    store_slab();
    __syncthreads();
    if (sl + 1 < nslabs) load_slab((sl + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int wo = ks * 16 + 4 * kb;  // word offset of this lane's 4 complex values
      bf8v ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) {
        const int row = wm * 64 + mi * 16 + li;
        ah[mi] = __builtin_bit_cast(bf8v, *reinterpret_cast<const u4v*>(&Ah[row * LDW + wo]));
        if constexpr (HAS_LO) al[mi] = __builtin_bit_cast(bf8v, *reinterpret_cast<const u4v*>(&Al[row * LDW + wo]));
      }
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) {
        const int n = wn * 64 + ni * 16 + li;  // real column within the tile
        const int v = n >> 1, jj = n & 1;
        u4v wh = *reinterpret_cast<const u4v*>(&Bh[v * LDW + wo]);
        u4v wl = *reinterpret_cast<const u4v*>(&Bl[v * LDW + wo]);
        if (!ADJ) {
          if (jj == 0) { wh ^= 0x80000000u; wl ^= 0x80000000u; }   // (c, -d)
          else {                                                     // (d, c)
            wh = u4v{swap16(wh.x), swap16(wh.y), swap16(wh.z), swap16(wh.w)};
            wl = u4v{swap16(wl.x), swap16(wl.y), swap16(wl.z), swap16(wl.w)};
          }
        } else if (jj == 1) {                                        // (f, -e)
          wh = u4v{swap16(wh.x), swap16(wh.y), swap16(wh.z), swap16(wh.w)} ^ 0x80000000u;
          wl = u4v{swap16(wl.x), swap16(wl.y), swap16(wl.z), swap16(wl.w)} ^ 0x80000000u;
        }
        bh[ni] = __builtin_bit_cast(bf8v, wh);
        bl[ni] = __builtin_bit_cast(bf8v, wl);
      }
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bl[ni], acc[mi][ni], 0, 0, 0);
          if constexpr (HAS_LO)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mi], bh[ni], acc[mi][ni], 0, 0, 0);
        }
    }
  }

  const float osc = (FMT == MDC_FP16S) ? 1.0f / fscale[f] : 1.0f;
  // D[i][j] of a 16x16 block: j = lane % 16, i = 4 * (lane / 16) + e
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int n = 2 * n0 + wn * 64 + ni * 16 + li;
      const int v = n >> 1;
      if (v >= ncols) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm * 64 + mi * 16 + 4 * kb + e;
        if (row < M) Cf[((size_t)row * ncols + v) * 2 + (n & 1)] = acc[mi][ni][e] * osc;
      }
    }
}

template <int FMT>
mdc_status launch_fmt(const mdc_desc& d, const char* K, const float* fscale, int ldk, int adjoint, const float2* in,
                      float2* out, int ncols, hipStream_t st) {
  const int M = adjoint ? d.nr : d.ns;
  const int tiles_m = (M + BM - 1) / BM;
  const int tiles_n = (ncols + BN - 1) / BN;
  const long nb = (long)tiles_m * tiles_n * d.nfmax;
  if (nb > 0x7fffffffL) return fail(MDC_ENOTSUP, "too many GEMM tiles");
  const int nblocks = (int)nb;
  if (adjoint)
    hipLaunchKernelGGL((gemm16_kernel<FMT, true>), dim3(nblocks), dim3(kThreads), 0, st, K, fscale, d.ns, d.nr, ldk,
                       in, out, ncols, tiles_m, tiles_n, nblocks);
  else
    hipLaunchKernelGGL((gemm16_kernel<FMT, false>), dim3(nblocks), dim3(kThreads), 0, st, K, fscale, d.ns, d.nr, ldk,
                       in, out, ncols, tiles_m, tiles_n, nblocks);
  return check_launch("gemm16_kernel");
}

__global__ void fp16_scales_kernel(float* fscale, int nfmax) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfmax) return;
  const float mx = __uint_as_float(reinterpret_cast<const unsigned int*>(fscale)[f]);
  // largest power of two s with mx * s <= 2^15 (FP16 max is 65504)
  float s = 1.0f;
  if (mx > 0.f) {
    int e;
    frexpf(mx, &e);  // mx in [2^(e-1), 2^e)
    s = ldexpf(1.0f, 15 - e);
  }
  fscale[f] = s;
}

}  // namespace

mdc_status fp16_scales_launch(float* fscale, int nfmax, hipStream_t st) {
  hipLaunchKernelGGL(fp16_scales_kernel, dim3((nfmax + 255) / 256), dim3(256), 0, st, fscale, nfmax);
  return check_launch("fp16_scales_kernel");
}

mdc_status gemm16_launch(const mdc_desc& d, const void* K, const float* fscale, int ldk, int adjoint,
                         const float2* in, float2* out, int ncols, hipStream_t st) {
  const char* k = static_cast<const char*>(K);
  switch (d.prec) {
    case MDC_FP16S: return launch_fmt<MDC_FP16S>(d, k, fscale, ldk, adjoint, in, out, ncols, st);
    case MDC_BF16: return launch_fmt<MDC_BF16>(d, k, fscale, ldk, adjoint, in, out, ncols, st);
    case MDC_BF16X2: return launch_fmt<MDC_BF16X2>(d, k, fscale, ldk, adjoint, in, out, ncols, st);
    default: return fail(MDC_EINVAL, "gemm16: not a 16-bit format");
  }
}

}  // namespace mdc
