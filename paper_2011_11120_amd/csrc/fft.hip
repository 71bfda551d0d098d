// Orthogonal real FFT along the (outermost) time axis, truncated to nfmax bins,
// and its zero-padded inverse (Eq.3: I F and F^H I^H; batch-matmul section:
// orthogonal real transform, 1/sqrt(nt) both ways, positive frequencies only).
//
// A length-nt real trace is packed into M = nt/2 complex points
// z[m] = x[2m] + i x[2m+1] and transformed by a radix-4 (plus one radix-2)
// Stockham FFT held in LDS; a split step then yields the nt/2+1 real-signal
// bins, of which only the first nfmax are written.  The inverse runs the same
// steps backwards from zero-padded bins, dropping the imaginary parts of the
// DC and Nyquist bins (what makes the pair exactly adjoint).
//
// Layout: each workgroup owns CB consecutive traces (consecutive (n, v)
// columns of the [nt][n][nv] array), so every global access of a time row or
// a spectral row is contiguous across lanes.  LDS holds z as [M][CB] complex.
// Twiddles come from an FP64-built table rounded once to FP32:
// tw[k] = exp(-2 pi i k / nt).
#include <climits>

#include "common.hpp"

namespace mdc {
namespace {

constexpr int kThreads = 256;

template <int M>
constexpr int log2c() {
  int l = 0;
  for (int v = M; v > 1; v >>= 1) ++l;
  return l;
}

// y = DFT_4(a) with sign DIR (-1 forward, +1 inverse), in place.
template <int DIR>
__device__ __forceinline__ void bfly4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), d = csub(a1, a3);
  // DIR * i * d
  const float2 id = (DIR < 0) ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, id);
  a3 = csub(t1, id);
}

// Complete M-point Stockham FFT (unnormalised) of the CB columns in lds[M][CB].
template <int M, int CB, int DIR>
__device__ __forceinline__ void fft_lds(float2* lds, const float2* __restrict__ tw, int tid) {
  constexpr int LOG = log2c<M>();
  int Ns = 1;
  if constexpr (LOG % 2 == 1) {
    constexpr int NB = (M / 2) * CB;
    constexpr int BPT = (NB + kThreads - 1) / kThreads;
    float2 v0[BPT], v1[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int b = tid + i * kThreads;
      if (b < NB) {
        const int col = b % CB, j = b / CB;
        v0[i] = lds[j * CB + col];
        v1[i] = lds[(j + M / 2) * CB + col];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int b = tid + i * kThreads;
      if (b < NB) {
        const int col = b % CB, j = b / CB;
        lds[(2 * j) * CB + col] = cadd(v0[i], v1[i]);
        lds[(2 * j + 1) * CB + col] = csub(v0[i], v1[i]);
      }
    }
    __syncthreads();
    Ns = 2;
  }
  constexpr int NB = (M / 4) * CB;
  constexpr int BPT = (NB + kThreads - 1) / kThreads;
  for (; Ns < M; Ns *= 4) {
    const int tstep = 2 * (M / (4 * Ns));  // tw index stride per unit of r*k
    float2 v[BPT][4];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int b = tid + i * kThreads;
      if (b < NB) {
        const int col = b % CB, j = b / CB;
        const int k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[i][r] = lds[(j + r * (M / 4)) * CB + col];
        if (Ns > 1) {
#pragma unroll
          for (int r = 1; r < 4; ++r) {
            float2 w = tw[r * k * tstep];
            if (DIR > 0) w = cconj(w);
            v[i][r] = cmul(v[i][r], w);
          }
        }
        bfly4<DIR>(v[i][0], v[i][1], v[i][2], v[i][3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int b = tid + i * kThreads;
      if (b < NB) {
        const int col = b % CB, j = b / CB;
        const int k = j & (Ns - 1);
        const int base = (j - k) * 4 + k;
#pragma unroll
        for (int r = 0; r < 4; ++r) lds[(base + r * Ns) * CB + col] = v[i][r];
      }
    }
    __syncthreads();
  }
}

template <int M, int CB>
__global__ __launch_bounds__(kThreads) void rfft_trunc_kernel(
    const float* __restrict__ x, const int* __restrict__ onset, int conj, const float2* __restrict__ tw,
    int nfmax, int n, int nv, int ldc, int c0, float scale, float2* __restrict__ spec) {
  extern __shared__ float2 lds[];
  constexpr int NT = 2 * M;
  constexpr int ROWS = kThreads / CB;
  const int Q = n * nv;
  const int tid = threadIdx.x;
  const int col = tid % CB;
  const int q = blockIdx.x * CB + col;
  const bool qok = q < Q;
  const int on = (onset != nullptr && qok) ? onset[q] : INT_MAX;

  for (int m = tid / CB; m < M; m += ROWS) {
    float a = 0.f, b = 0.f;
    if (qok) {
      a = x[(size_t)(2 * m) * Q + q];
      b = x[(size_t)(2 * m + 1) * Q + q];
      if (onset != nullptr) {
        if (!in_window(2 * m, NT, on)) a = 0.f;
        if (!in_window(2 * m + 1, NT, on)) b = 0.f;
      }
    }
    lds[m * CB + col] = make_float2(a, b);
  }
  __syncthreads();
  fft_lds<M, CB, -1>(lds, tw, tid);

  const int r = q / nv, v = q - (q / nv) * nv;
  for (int k = tid / CB; k < nfmax; k += ROWS) {
    const float2 zk = lds[(k & (M - 1)) * CB + col];
    const float2 zc = cconj(lds[((M - k) & (M - 1)) * CB + col]);
    const float2 e = cscale(cadd(zk, zc), 0.5f);
    const float2 d = csub(zk, zc);
    const float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // d / (2i)
    float2 X = cscale(cadd(e, cmul(tw[k], o)), scale);
    if (conj) X = cconj(X);
    if (qok) spec[((size_t)k * n + r) * ldc + c0 + v] = X;
  }
}

template <int M, int CB>
__global__ __launch_bounds__(kThreads) void irfft_pad_kernel(
    const float2* __restrict__ spec, int ldc, int c0, int conj, const float2* __restrict__ tw, int nfmax,
    int n, int nv, float scale, float* __restrict__ out, const float* __restrict__ ident,
    const int* __restrict__ onset, float sign) {
  extern __shared__ float2 lds[];
  constexpr int NT = 2 * M;
  constexpr int ROWS = kThreads / CB;
  const int Q = n * nv;
  const int tid = threadIdx.x;
  const int col = tid % CB;
  const int q = blockIdx.x * CB + col;
  const bool qok = q < Q;
  const int r = q / nv, v = q - (q / nv) * nv;

  auto bin = [&](int k) -> float2 {
    if (!qok || k >= nfmax) return make_float2(0.f, 0.f);
    float2 X = spec[((size_t)k * n + r) * ldc + c0 + v];
    if (conj) X.y = -X.y;
    if (k == 0 || k == M) X.y = 0.f;  // the inverse real transform keeps only Re of DC/Nyquist
    return X;
  };
  // Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) exp(+2 pi i k / nt)
  for (int k = tid / CB; k <= M / 2; k += ROWS) {
    const float2 a = bin(k), b = bin(M - k);
    {
      const float2 e = cadd(a, cconj(b));
      const float2 o = cmul(csub(a, cconj(b)), cconj(tw[k]));
      lds[k * CB + col] = make_float2(e.x - o.y, e.y + o.x);
    }
    if (k > 0 && k < M / 2) {
      const float2 e = cadd(b, cconj(a));
      const float2 o = cmul(csub(b, cconj(a)), cconj(tw[M - k]));
      lds[(M - k) * CB + col] = make_float2(e.x - o.y, e.y + o.x);
    }
  }
  __syncthreads();
  fft_lds<M, CB, +1>(lds, tw, tid);

  if (!qok) return;
  const int on = (onset != nullptr) ? onset[q] : INT_MAX;
  for (int m = tid / CB; m < M; m += ROWS) {
    const float2 z = lds[m * CB + col];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = 2 * m + h;
      float val = (h == 0 ? z.x : z.y) * scale;
      if (onset != nullptr && !in_window(t, NT, on)) val = 0.f;
      val *= sign;
      const size_t idx = (size_t)t * Q + q;
      if (ident != nullptr) val += ident[idx];
      out[idx] = val;
    }
  }
}

template <int M>
constexpr int cols_per_block() { return M >= 1024 ? 8 : 16; }

template <int M>
mdc_status rfft_one(const float2* tw, int nfmax, int n, int nv, int ldc, const FftSeg& s, float2* spec,
                    hipStream_t st) {
  constexpr int CB = cols_per_block<M>();
  const int Q = n * nv;
  const size_t lds = (size_t)M * CB * sizeof(float2);
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void*)rfft_trunc_kernel<M, CB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  const float scale = (float)(1.0 / __builtin_sqrt((double)(2 * M)));
  hipLaunchKernelGGL((rfft_trunc_kernel<M, CB>), dim3((Q + CB - 1) / CB), dim3(kThreads), lds, st, s.in, s.onset,
                     s.conj, tw, nfmax, n, nv, ldc, s.c0, scale, spec);
  return check_launch("rfft_trunc_kernel");
}

template <int M>
mdc_status irfft_one(const float2* tw, int nfmax, int n, int nv, int ldc, const IfftSeg& s, const float2* spec,
                     hipStream_t st) {
  constexpr int CB = cols_per_block<M>();
  const int Q = n * nv;
  const size_t lds = (size_t)M * CB * sizeof(float2);
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void*)irfft_pad_kernel<M, CB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  const float scale = (float)(1.0 / __builtin_sqrt((double)(2 * M)));
  hipLaunchKernelGGL((irfft_pad_kernel<M, CB>), dim3((Q + CB - 1) / CB), dim3(kThreads), lds, st, spec, ldc, s.c0,
                     s.conj, tw, nfmax, n, nv, scale, s.out, s.ident, s.onset, s.sign);
  return check_launch("irfft_pad_kernel");
}

}  // namespace

mdc_status rfft_launch(const float2* tw, int nt, int nfmax, int n, int nv, int ldc, const FftSeg& seg,
                       float2* spec, hipStream_t st) {
  switch (nt) {
    case 16: return rfft_one<8>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 32: return rfft_one<16>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 64: return rfft_one<32>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 128: return rfft_one<64>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 256: return rfft_one<128>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 512: return rfft_one<256>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 1024: return rfft_one<512>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 2048: return rfft_one<1024>(tw, nfmax, n, nv, ldc, seg, spec, st);
    default: return fail(MDC_ENOTSUP, "nt=%d: the FFT supports powers of two in [16, 2048]", nt);
  }
}

mdc_status irfft_launch(const float2* tw, int nt, int nfmax, int n, int nv, int ldc, const IfftSeg& seg,
                        const float2* spec, hipStream_t st) {
  switch (nt) {
    case 16: return irfft_one<8>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 32: return irfft_one<16>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 64: return irfft_one<32>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 128: return irfft_one<64>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 256: return irfft_one<128>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 512: return irfft_one<256>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 1024: return irfft_one<512>(tw, nfmax, n, nv, ldc, seg, spec, st);
    case 2048: return irfft_one<1024>(tw, nfmax, n, nv, ldc, seg, spec, st);
    default: return fail(MDC_ENOTSUP, "nt=%d: the FFT supports powers of two in [16, 2048]", nt);
  }
}

}  // namespace mdc
