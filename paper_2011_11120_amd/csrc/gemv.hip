// Per-frequency complex kernel product for few columns (Eq.4: one dense slice
// per frequency; matrix-vector form when n_xA = 1).  Every element of K_f is
// read exactly once per apply, in both directions, so the product runs at the
// HBM streaming rate (about 1 flop per byte).
//
// Forward  Y_f[s][c] = sum_r K_f[s][r] X_f[r][c]        (row dot products)
// Adjoint  X_f[r][c] = sum_s conj(K_f[s][r]) Y_f[s][c]  (column sums)
//
// Forward: a wave owns RW rows at a time; lanes stride along the row with
// 16-byte non-temporal loads (a group of VEC complex values: two in complex64,
// four in a 16-bit format), the column block of X_f sits in LDS column-major
// (each lane reads its VEC values of a column as 16-byte pieces, consecutive
// lanes on consecutive pieces) and is reused by the RW rows; the wave's partial
// sums of all its rows and columns are closed together by recursive halving
// (n values in n - 1 exchanges).  Rows in flight are held as the stored words
// and widened where they are consumed; wide column groups load several
// reduction positions per lane before consuming any.
// Adjoint: a workgroup owns 64*VEC consecutive columns of K_f for all rows
// (column-block ownership), its four waves split the rows, Y_f sits in LDS and
// is read as a broadcast, and the four partial sums are added in a fixed
// order, so results are deterministic (no atomics).  16-bit formats are
// widened to FP32 in registers; products accumulate in FP32; the FP16 format's
// power-of-two frequency scale is divided out of each result.
#include "common.hpp"
#include "store.hpp"

namespace mdc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kStage = 8;  // loads in flight per thread when a spectra chunk is staged in LDS

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef unsigned int vu4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ vf4 ldnt_f4(const void* p) { return __builtin_nontemporal_load(static_cast<const vf4*>(p)); }
__device__ __forceinline__ vu4 ldnt_u4(const void* p) { return __builtin_nontemporal_load(static_cast<const vu4*>(p)); }

// Kernel formats: VEC complex values per 16-byte group (32 bytes for hi + lo).  Loads keep the
// stored words (Raw: 16 or 32 bytes per group, so rows in flight cost no more registers than
// their bytes); unpack widens them to FP32 where they are consumed.
struct Raw2 {
  vu4 h, l;
};
template <int FMT> struct KF;
template <> struct KF<MDC_FP32> {
  static constexpr int VEC = 2, GROUP_BYTES = 16;
  using Raw = vf4;
  __device__ static Raw load(const char* g) { return ldnt_f4(g); }
  __device__ static Raw zero() { return vf4{0.f, 0.f, 0.f, 0.f}; }
  __device__ static void unpack(const Raw& v, float2 (&k)[2]) {
    k[0] = make_float2(v.x, v.y);
    k[1] = make_float2(v.z, v.w);
  }
};
template <> struct KF<MDC_FP16S> {
  static constexpr int VEC = 4, GROUP_BYTES = 16;
  using Raw = vu4;
  __device__ static Raw load(const char* g) { return ldnt_u4(g); }
  __device__ static Raw zero() { return vu4{0u, 0u, 0u, 0u}; }
  __device__ static void unpack(const Raw& v, float2 (&k)[4]) {
    const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) k[j] = make_float2(f16_bits_to_f(w[j] & 0xFFFFu), f16_bits_to_f(w[j] >> 16));
  }
};
template <> struct KF<MDC_BF16> {
  static constexpr int VEC = 4, GROUP_BYTES = 16;
  using Raw = vu4;
  __device__ static Raw load(const char* g) { return ldnt_u4(g); }
  __device__ static Raw zero() { return vu4{0u, 0u, 0u, 0u}; }
  __device__ static void unpack(const Raw& v, float2 (&k)[4]) {
    const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) k[j] = make_float2(__uint_as_float(w[j] << 16), __uint_as_float(w[j] & 0xFFFF0000u));
  }
};
template <> struct KF<MDC_BF16X2> {
  static constexpr int VEC = 4, GROUP_BYTES = 32;
  using Raw = Raw2;
  __device__ static Raw load(const char* g) { return Raw2{ldnt_u4(g), ldnt_u4(g + 16)}; }
  __device__ static Raw zero() { return Raw2{vu4{0u, 0u, 0u, 0u}, vu4{0u, 0u, 0u, 0u}}; }
  __device__ static void unpack(const Raw& v, float2 (&k)[4]) {
    const unsigned int wh[4] = {v.h.x, v.h.y, v.h.z, v.h.w}, wl[4] = {v.l.x, v.l.y, v.l.z, v.l.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      k[j] = make_float2(__uint_as_float(wh[j] << 16) + __uint_as_float(wl[j] << 16),
                         __uint_as_float(wh[j] & 0xFFFF0000u) + __uint_as_float(wl[j] & 0xFFFF0000u));
  }
};

template <int FMT>
__device__ __forceinline__ float out_scale(const float* fscale, int f) {
  if constexpr (FMT == MDC_FP16S) return 1.0f / fscale[f];  // exact: a power of two
  else return 1.0f;
}

// Sums each of NP values across the wave by recursive halving: at the exchange with offset O a
// lane keeps half of the values it holds (the upper half where bit O of the lane is set) and adds
// its partner's copy of that half, so NP values take NP - 1 exchanges instead of 6 NP.  Once the
// values are down to one per lane the remaining offsets finish a plain butterfly.  On return v[0]
// holds the sum of value lane >> (6 - log2 NP), the same on every lane of a group of 64 / NP.
template <int M, int O>
struct WaveHalve {
  template <int NP>
  __device__ static __forceinline__ void run(float (&v)[NP], int lane) {
    if constexpr (M > 1) {
      const bool hi = (lane & O) != 0;
#pragma unroll
      for (int k = 0; k < M / 2; ++k) {
        const float send = hi ? v[k] : v[k + M / 2];
        const float keep = hi ? v[k + M / 2] : v[k];
        v[k] = keep + __shfl_xor(send, O, 64);
      }
      WaveHalve<M / 2, O / 2>::run(v, lane);
    } else if constexpr (O > 0) {
      v[0] += __shfl_xor(v[0], O, 64);
      WaveHalve<1, O / 2>::run(v, lane);
    }
  }
};

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }
constexpr int log2_exact(int n) { return n <= 1 ? 0 : 1 + log2_exact(n / 2); }

// ---------------------------------------------------------------- forward ---
// UP reduction positions per lane are loaded (UP x RW groups of K in flight) before any is consumed.
template <int FMT, int NC, int RW, int UP>
__global__ __launch_bounds__(kThreads) void gemv_fwd_kernel(const char* __restrict__ K, const float* __restrict__ fscale,
                                                            const float2* __restrict__ X, float2* __restrict__ Y,
                                                            int ns, int nr, int ldk, int ldc, int col0,
                                                            int groups_per_block, int rc) {
  using F = KF<FMT>;
  constexpr int VEC = F::VEC;
  // chunk of X_f column-major, column c at c * xst: a lane reads its VEC reduction values of a
  // column as 16-byte pieces, consecutive lanes on consecutive pieces (no bank conflicts); the
  // stride rc + 2 keeps columns 16-byte aligned and spreads the staging writes over the banks
  extern __shared__ __attribute__((aligned(16))) float2 xs[];  // [NC][rc + 2]
  const int xst = rc + 2;
  const int f = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const size_t rowb = (size_t)(ldk / VEC) * F::GROUP_BYTES;
  const char* Kf = K + (size_t)f * ns * rowb;
  const float2* Xf = X + (size_t)f * nr * ldc;
  float2* Yf = Y + (size_t)f * ns * ldc;
  const int nchunks = (ldk + rc - 1) / rc;
  const int rows_per_group = kWaves * RW;
  const float osc = out_scale<FMT>(fscale, f);

  for (int g = 0; g < groups_per_block; ++g) {
    const int sbase = (blockIdx.x * groups_per_block + g) * rows_per_group + wave * RW;
    if ((blockIdx.x * groups_per_block + g) * rows_per_group >= ns) break;  // uniform per block
    float acc[RW][NC][2];
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[i][c][0] = acc[i][c][1] = 0.f;

    for (int ch = 0; ch < nchunks; ++ch) {
      const int r0 = ch * rc;
      const int rlen = min(rc, ldk - r0);  // a multiple of 4: ldk and rc are
      if (nchunks > 1 || g == 0) {
        __syncthreads();
        // kStage loads per thread issued before their stores: one round trip per kStage elements.
        // The loads are unconditional (an element past the chunk or past nr reads X_f[0][col0] and is
        // replaced by zero), so none of them waits for the others.
        const int ne = rlen * NC;
        for (int e0 = threadIdx.x; e0 < ne; e0 += kThreads * kStage) {
          float2 t[kStage];
#pragma unroll
          for (int u = 0; u < kStage; ++u) {
            const int e = e0 + u * kThreads, rr = e / NC, c = e - (e / NC) * NC;
            const bool ok = e < ne && r0 + rr < nr;
            const float2 v = Xf[ok ? (size_t)(r0 + rr) * ldc + col0 + c : (size_t)col0];
            t[u] = ok ? v : make_float2(0.f, 0.f);
          }
#pragma unroll
          for (int u = 0; u < kStage; ++u) {
            const int e = e0 + u * kThreads, rr = e / NC, c = e - (e / NC) * NC;
            if (e < ne) xs[c * xst + rr] = t[u];
          }
        }
        __syncthreads();
      }
      const int npos = rlen / VEC;
      for (int p0 = lane; p0 < npos; p0 += 64 * UP) {
        typename F::Raw kr[UP][RW];
#pragma unroll
        for (int u = 0; u < UP; ++u)
#pragma unroll
          for (int i = 0; i < RW; ++i) {
            const int s = sbase + i, p = p0 + 64 * u;
            kr[u][i] = (s < ns && (UP == 1 || p < npos))
                           ? F::load(Kf + (size_t)s * rowb + (size_t)(r0 / VEC + p) * F::GROUP_BYTES)
                           : F::zero();
          }
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const int p = p0 + 64 * u;
          if (UP > 1 && p >= npos) continue;
          if constexpr (UP == 1) {  // all columns' X values held, rows widened one at a time
            float2 xv[NC][VEC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
              for (int j = 0; j < VEC; j += 2) {
                const float4 t = *reinterpret_cast<const float4*>(&xs[c * xst + VEC * p + j]);
                xv[c][j] = make_float2(t.x, t.y);
                xv[c][j + 1] = make_float2(t.z, t.w);
              }
#pragma unroll
            for (int i = 0; i < RW; ++i) {
              float2 kv[VEC];
              F::unpack(kr[u][i], kv);
#pragma unroll
              for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                  acc[i][c][0] += kv[j].x * xv[c][j].x - kv[j].y * xv[c][j].y;
                  acc[i][c][1] += kv[j].x * xv[c][j].y + kv[j].y * xv[c][j].x;
                }
            }
          } else {  // all rows widened, X read one column at a time
            float2 kv[RW][VEC];
#pragma unroll
            for (int i = 0; i < RW; ++i) F::unpack(kr[u][i], kv[i]);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              float2 xv[VEC];
#pragma unroll
              for (int j = 0; j < VEC; j += 2) {
                const float4 t = *reinterpret_cast<const float4*>(&xs[c * xst + VEC * p + j]);
                xv[j] = make_float2(t.x, t.y);
                xv[j + 1] = make_float2(t.z, t.w);
              }
#pragma unroll
              for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                  acc[i][c][0] += kv[i][j].x * xv[j].x - kv[i][j].y * xv[j].y;
                  acc[i][c][1] += kv[i][j].x * xv[j].y + kv[i][j].y * xv[j].x;
                }
            }
          }
        }
      }
    }
    // value (i * NC + c) * 2 + z of every lane summed across the wave; one lane per value stores it
    constexpr int NV = RW * NC * 2, NP = pow2_at_least(NV), SH = 6 - log2_exact(NP);
    float v[NP];
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[(i * NC + c) * 2] = acc[i][c][0];
        v[(i * NC + c) * 2 + 1] = acc[i][c][1];
      }
#pragma unroll
    for (int k = NV; k < NP; ++k) v[k] = 0.f;
    WaveHalve<NP, 32>::run(v, lane);
    const int idx = lane >> SH;
    if ((lane & ((1 << SH) - 1)) == 0 && idx < NV) {
      const int ic = idx >> 1, i = ic / NC, c = ic - (ic / NC) * NC;
      const int s = sbase + i;
      if (s < ns) reinterpret_cast<float*>(Yf)[((size_t)s * ldc + col0 + c) * 2 + (idx & 1)] = v[0] * osc;
    }
  }
}

// ---------------------------------------------------------------- adjoint ---
// Workgroup = (column tile of 64*VEC, frequency).  UR rows of K are loaded back
// to back by each wave before they are consumed.
template <int FMT, int NC, int UR>
__global__ __launch_bounds__(kThreads) void gemv_adj_kernel(const char* __restrict__ K, const float* __restrict__ fscale,
                                                            const float2* __restrict__ Y, float2* __restrict__ X,
                                                            int ns, int nr, int ldk, int ldc, int col0, int rcy) {
  using F = KF<FMT>;
  constexpr int VEC = F::VEC;
  extern __shared__ float2 sh[];  // ys[rcy][NC], then partials of two waves [2][VEC*NC*2][64]
  float2* ys = sh;
  const int f = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const size_t rowb = (size_t)(ldk / VEC) * F::GROUP_BYTES;
  const char* Kf = K + (size_t)f * ns * rowb;
  const float2* Yf = Y + (size_t)f * ns * ldc;
  float2* Xf = X + (size_t)f * nr * ldc;
  const int p = blockIdx.x * 64 + lane;  // group: columns VEC*p .. VEC*p + VEC-1
  const bool pok = VEC * p < nr;

  float acc[VEC][NC][2];
#pragma unroll
  for (int h = 0; h < VEC; ++h)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[h][c][0] = acc[h][c][1] = 0.f;

  for (int s0 = 0; s0 < ns; s0 += rcy) {
    const int slen = min(rcy, ns - s0);
    __syncthreads();
    const int ne = slen * NC;
    // kStage unconditional loads per thread before their stores (past the chunk: Y_f[s0][col0], unused)
    for (int e0 = threadIdx.x; e0 < ne; e0 += kThreads * kStage) {
      float2 t[kStage];
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int e = e0 + u * kThreads, ss = e / NC, c = e - (e / NC) * NC;
        t[u] = Yf[e < ne ? (size_t)(s0 + ss) * ldc + col0 + c : (size_t)s0 * ldc + col0];
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int e = e0 + u * kThreads;
        if (e < ne) ys[e] = t[u];
      }
    }
    __syncthreads();
    // wave w takes rows w*UR .. w*UR+UR-1, then every kWaves*UR rows
    for (int sb = wave * UR; sb < slen; sb += kWaves * UR) {
      typename F::Raw kr[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int ss = sb + u;
        kr[u] = (pok && ss < slen) ? F::load(Kf + (size_t)(s0 + ss) * rowb + (size_t)p * F::GROUP_BYTES) : F::zero();
      }
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int ss = min(sb + u, slen - 1);  // rows past the end carry k = 0
        float2 kv[VEC];
        F::unpack(kr[u], kv);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const float2 y = ys[ss * NC + c];
#pragma unroll
          for (int h = 0; h < VEC; ++h) {
            // conj(k) * y = (kr yr + ki yi) + i (kr yi - ki yr)
            acc[h][c][0] += kv[h].x * y.x + kv[h].y * y.y;
            acc[h][c][1] += kv[h].x * y.y - kv[h].y * y.x;
          }
        }
      }
    }
  }
  // fixed-order reduction of the four waves' partials, (p0 + p1) + (p2 + p3), in two rounds so that
  // LDS holds two waves' partials at a time (at 16-bit widths above 4 the four would take 40-64 KB
  // and halve the workgroups per CU)
  float* part = reinterpret_cast<float*>(sh);
  constexpr int NV = VEC * NC * 2;
  __syncthreads();
  if (wave & 1) {
#pragma unroll
    for (int h = 0; h < VEC; ++h)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int z = 0; z < 2; ++z) part[((wave >> 1) * NV + (h * NC + c) * 2 + z) * 64 + lane] = acc[h][c][z];
  }
  __syncthreads();
  if (!(wave & 1)) {  // wave 0: p0 + p1, wave 2: p2 + p3
#pragma unroll
    for (int h = 0; h < VEC; ++h)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int z = 0; z < 2; ++z) acc[h][c][z] += part[((wave >> 1) * NV + (h * NC + c) * 2 + z) * 64 + lane];
  }
  __syncthreads();
  if (wave == 2) {
#pragma unroll
    for (int h = 0; h < VEC; ++h)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int z = 0; z < 2; ++z) part[((h * NC + c) * 2 + z) * 64 + lane] = acc[h][c][z];
  }
  __syncthreads();
  if (wave == 0 && pok) {
    const float osc = out_scale<FMT>(fscale, f);
#pragma unroll
    for (int h = 0; h < VEC; ++h)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int k = ((h * NC + c) * 2) * 64 + lane;
        const float re = (acc[h][c][0] + part[k]) * osc;
        const float im = (acc[h][c][1] + part[k + 64]) * osc;
        if (VEC * p + h < nr) Xf[(size_t)(VEC * p + h) * ldc + col0 + c] = make_float2(re, im);
      }
  }
}

template <int FMT, int NC>
mdc_status gemv_group(const mdc_desc& d, const char* K, const float* fscale, int ldk, int adjoint, const float2* in,
                      float2* out, int ldc, int col0, hipStream_t st) {
  constexpr int VEC = KF<FMT>::VEC;
  if (!adjoint) {
    // rows per wave: 4 while a row's products fit (NC * VEC <= 8), else 2 with UP positions per lane
    // in flight (as many as one chunk spans, at most 128 bytes of K per lane)
    constexpr int RW = (NC * VEC <= 8) ? 4 : 2;
    // chunk of the reduction held in LDS, a multiple of 4 (equal chunks sized to the reduction, which
    // raise the occupancy, measured 0.5-6% slower at 1, 2 and 8 columns on the 40 x 40 grid)
    constexpr int RC = (4096 / NC) & ~3;
    constexpr int UPC = RC / VEC / 64, UPB = 128 / (RW * KF<FMT>::GROUP_BYTES);
    constexpr int UP = (NC * VEC <= 8) ? 1 : (UPC < 1 ? 1 : (UPC < UPB ? UPC : UPB));
    const int rc = RC;
    const int rows_per_group = kWaves * RW;
    const int ngroups = (d.ns + rows_per_group - 1) / rows_per_group;
    int gpb = (int)((long)ngroups * d.nfmax / 4096);
    gpb = gpb < 1 ? 1 : (gpb > 8 ? 8 : gpb);
    const int nblk = (ngroups + gpb - 1) / gpb;
    const size_t lds = (size_t)(rc + 2) * NC * sizeof(float2);
    hipLaunchKernelGGL((gemv_fwd_kernel<FMT, NC, RW, UP>), dim3(nblk, d.nfmax), dim3(kThreads), lds, st, K, fscale, in,
                       out, d.ns, d.nr, ldk, ldc, col0, gpb, rc);
    return check_launch("gemv_fwd_kernel");
  }
  // rows of K in flight per wave: 16 for the narrowest column groups (measured about 1% faster than
  // 8 on the single-column workload), fewer where each row brings more registers
  constexpr int UR = (NC * VEC >= 16) ? 4 : (NC * VEC <= 4 ? 16 : 8);
  const int rcy = 4096 / NC;
  const size_t lds_y = (size_t)rcy * NC * sizeof(float2);
  const size_t lds_p = (size_t)2 * VEC * NC * 2 * 64 * sizeof(float);  // two waves' partials
  const size_t lds = lds_y > lds_p ? lds_y : lds_p;
  const int nblk = ((d.nr + VEC - 1) / VEC + 63) / 64;
  hipLaunchKernelGGL((gemv_adj_kernel<FMT, NC, UR>), dim3(nblk, d.nfmax), dim3(kThreads), lds, st, K, fscale, in,
                     out, d.ns, d.nr, ldk, ldc, col0, rcy);
  return check_launch("gemv_adj_kernel");
}

template <int FMT>
mdc_status gemv_fmt(const mdc_desc& d, const char* K, const float* fscale, int ldk, int adjoint, const float2* in,
                    float2* out, int ncols, hipStream_t st) {
  // one pass over the kernel for every group of up to 8 columns (any width below 9 reads K once)
  int c0 = 0;
  while (c0 < ncols) {
    const int nc = ncols - c0 >= 8 ? 8 : ncols - c0;
    mdc_status s;
    switch (nc) {
      case 8: s = gemv_group<FMT, 8>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
      case 7: s = gemv_group<FMT, 7>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
      case 6: s = gemv_group<FMT, 6>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
      case 5: s = gemv_group<FMT, 5>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
      case 4: s = gemv_group<FMT, 4>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
      case 3: s = gemv_group<FMT, 3>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
      case 2: s = gemv_group<FMT, 2>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
      default: s = gemv_group<FMT, 1>(d, K, fscale, ldk, adjoint, in, out, ncols, c0, st); break;
    }
    if (s != MDC_OK) return s;
    c0 += nc;
  }
  return MDC_OK;
}

}  // namespace

// Few-column product (ncols columns in groups of at most 8, one kernel pass each), any storage format.
mdc_status gemv_launch(const mdc_desc& d, const void* K, const float* fscale, int ldk, int adjoint, const float2* in,
                       float2* out, int ncols, hipStream_t st) {
  const char* k = static_cast<const char*>(K);
  switch (d.prec) {
    case MDC_FP32: return gemv_fmt<MDC_FP32>(d, k, fscale, ldk, adjoint, in, out, ncols, st);
    case MDC_FP16S:  // the spectra stay FP32 here: both FP16 formats take this path
    case MDC_FP16: return gemv_fmt<MDC_FP16S>(d, k, fscale, ldk, adjoint, in, out, ncols, st);
    case MDC_BF16: return gemv_fmt<MDC_BF16>(d, k, fscale, ldk, adjoint, in, out, ncols, st);
    case MDC_BF16X2: return gemv_fmt<MDC_BF16X2>(d, k, fscale, ldk, adjoint, in, out, ncols, st);
  }
  return fail(MDC_EINVAL, "unknown storage format");
}

}  // namespace mdc
