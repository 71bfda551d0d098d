// Resident kernel storage formats (the rounding of K to its stored form).
#pragma once
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

// complex64, RNE from FP64
struct StoreF32 {
  float2* p;
  int ns, ldk;
  explicit StoreF32(const StoreRef& r) : p(static_cast<float2*>(r.base)), ns(r.ns), ldk(r.ldk) {}
  __device__ __forceinline__ void put(int f, int s, int r, double re, double im) const {
    p[((size_t)f * ns + s) * ldk + r] = make_float2((float)re, (float)im);
  }
};

size_t store_bytes(const mdc_desc& d);
mdc_status synth_launch(const mdc_desc& d, const mdc_synth_desc& sd, const StoreRef& st_ref, hipStream_t st);
mdc_status gemv_launch(const mdc_desc& d, const float2* K, int ldk, int adjoint, const float2* in, float2* out,
                       int ncols, hipStream_t st);

mdc_status gemm_launch(const mdc_desc& d, const float2* K, int ldk, int adjoint, const float2* in, float2* out,
                       int ncols, hipStream_t st);

}  // namespace mdc
