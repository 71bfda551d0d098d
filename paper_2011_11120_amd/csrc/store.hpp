// Resident kernel storage formats (the rounding of K to its stored form).
#pragma once
#include <hip/hip_fp16.h>

#include "common.hpp"

namespace mdc {

// Rows of the stored kernel are padded to ldk = nr rounded up to a multiple of 4
// (16-byte aligned rows for every format); pad columns hold zeros.
inline int kernel_ld(int nr) { return (nr + 3) & ~3; }

struct StoreRef {
  void* base;      // start of the stored kernel [nfmax][ns][ldk]
  float* fscale;   // per-frequency scale (FP16S), else nullptr
  int nfmax, ns, nr, ldk;
};

// ------------------------------------------------------------- 16-bit ---
__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_bits_to_f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f16_rne_bits(float f) { return (uint32_t)__half_as_ushort(__float2half_rn(f)); }
__device__ __forceinline__ float f16_bits_to_f(uint32_t h) { return __half2float(__ushort_as_half((unsigned short)h)); }

// Bytes of one stored row of ldk complex values.
inline size_t row_bytes(mdc_prec p, int ldk) {
  return (p == MDC_FP32 || p == MDC_BF16X2) ? (size_t)ldk * 8 : (size_t)ldk * 4;
}

// complex64, RNE from FP64
struct StoreF32 {
  float2* p;
  int ns, ldk;
  explicit StoreF32(const StoreRef& r) : p(static_cast<float2*>(r.base)), ns(r.ns), ldk(r.ldk) {}
  __device__ __forceinline__ void put(int f, int s, int r, double re, double im) const {
    p[((size_t)f * ns + s) * ldk + r] = make_float2((float)re, (float)im);
  }
};

// FP16 pairs (re low half, im high half) of k * s_f, s_f = fscale[f] a power of two.
struct StoreF16S {
  uint32_t* p;
  const float* fscale;
  int ns, ldk;
  explicit StoreF16S(const StoreRef& r)
      : p(static_cast<uint32_t*>(r.base)), fscale(r.fscale), ns(r.ns), ldk(r.ldk) {}
  __device__ __forceinline__ void put(int f, int s, int r, double re, double im) const {
    const float sf = fscale[f];
    const uint32_t a = f16_rne_bits((float)re * sf), b = f16_rne_bits((float)im * sf);
    p[((size_t)f * ns + s) * ldk + r] = a | (b << 16);
  }
};

// BF16 pairs of the complex64 value.
struct StoreBF16 {
  uint32_t* p;
  int ns, ldk;
  explicit StoreBF16(const StoreRef& r) : p(static_cast<uint32_t*>(r.base)), ns(r.ns), ldk(r.ldk) {}
  __device__ __forceinline__ void put(int f, int s, int r, double re, double im) const {
    p[((size_t)f * ns + s) * ldk + r] = bf16_rne_bits((float)re) | (bf16_rne_bits((float)im) << 16);
  }
};

// BF16 hi + lo of the complex64 value g: hi = RNE(g), lo = RNE(g - hi).  Rows are stored in
// groups of four complex values: 16 bytes of hi pairs followed by 16 bytes of lo pairs.
struct StoreBF16X2 {
  uint32_t* p;
  int ns, ldk;
  explicit StoreBF16X2(const StoreRef& r) : p(static_cast<uint32_t*>(r.base)), ns(r.ns), ldk(r.ldk) {}
  __device__ __forceinline__ void put(int f, int s, int r, double re, double im) const {
    const float gr = (float)re, gi = (float)im;
    const uint32_t hr = bf16_rne_bits(gr), hi = bf16_rne_bits(gi);
    const uint32_t lr = bf16_rne_bits(gr - bf16_bits_to_f(hr)), li = bf16_rne_bits(gi - bf16_bits_to_f(hi));
    uint32_t* row = p + ((size_t)f * ns + s) * (size_t)ldk * 2;
    const int g = r >> 2, j = r & 3;
    row[g * 8 + j] = hr | (hi << 16);
    row[g * 8 + 4 + j] = lr | (li << 16);
  }
};

// Records max(|re|, |im|) per frequency (first pass of FP16S): fscale viewed as uint bits.
struct StoreMax {
  unsigned int* mx;
  explicit StoreMax(const StoreRef& r) : mx(reinterpret_cast<unsigned int*>(r.fscale)) {}
  __device__ __forceinline__ void put(int f, int, int, double re, double im) const {
    const float m = fmaxf(fabsf((float)re), fabsf((float)im));
    atomicMax(mx + f, __float_as_uint(m));
  }
};

size_t store_bytes(const mdc_desc& d);
mdc_status synth_launch(const mdc_desc& d, const mdc_synth_desc& sd, const StoreRef& st_ref, hipStream_t st);
mdc_status gemv_launch(const mdc_desc& d, const void* K, const float* fscale, int ldk, int adjoint,
                       const float2* in, float2* out, int ncols, hipStream_t st);

// Per-frequency FP16 scale from the maxima left by StoreMax: s_f = 2^e with max * s_f <= 2^15.
mdc_status fp16_scales_launch(float* fscale, int nfmax, hipStream_t st);
// bsplit: workspace of gemm16_split_bytes(d) bytes receiving the split spectra of each launch.
size_t gemm16_split_bytes(const mdc_desc& d);
// variant 0: four waves of 64 output rows per workgroup; 1: eight waves of 32 rows.
mdc_status gemm16_launch(const mdc_desc& d, const void* K, const float* fscale, int ldk, int adjoint,
                         const float2* in, float2* out, int ncols, unsigned int* bsplit, int variant, hipStream_t st);
mdc_status gemm_launch(const mdc_desc& d, const float2* K, int ldk, int adjoint, const float2* in, float2* out,
                       int ncols, hipStream_t st, int bn);

}  // namespace mdc
