// Per-frequency complex kernel product for few columns (Eq.4: one dense slice
// per frequency; matrix-vector form when n_xA = 1).  Every element of K_f is
// read exactly once per apply, in both directions, so the product runs at the
// HBM streaming rate (about 1 flop per byte).
//
// Forward  Y_f[s][c] = sum_r K_f[s][r] X_f[r][c]        (row dot products)
// Adjoint  X_f[r][c] = sum_s conj(K_f[s][r]) Y_f[s][c]  (column sums)
//
// Forward: a wave owns RW rows at a time; lanes stride along the row with
// 16-byte loads (two complex values), the column block of X_f sits in LDS
// and is reused by the RW rows; a butterfly reduction across the wave closes
// each row.  Adjoint: a workgroup owns 128 consecutive columns of K_f for all
// rows (the "column-block ownership" layout), its four waves split the rows,
// Y_f sits in LDS and is read as a broadcast, and the four partial sums are
// added in a fixed order, so results are deterministic (no atomics).
#include "common.hpp"

namespace mdc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

typedef float vf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ldg_stream(const float4* p) {
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- forward ---
// Requires nr even (16-byte aligned rows).  NC columns, RW rows per wave.
template <int NC, int RW>
__global__ __launch_bounds__(kThreads) void gemv_fwd_kernel(const float2* __restrict__ K,
                                                            const float2* __restrict__ X,
                                                            float2* __restrict__ Y, int ns, int nr, int ldk,
                                                            int ldc, int col0, int groups_per_block, int rc) {
  extern __shared__ float2 xs[];  // [rc][NC]
  const int f = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const float2* Kf = K + (size_t)f * ns * ldk;
  const float2* Xf = X + (size_t)f * nr * ldc;
  float2* Yf = Y + (size_t)f * ns * ldc;
  const int nchunks = (ldk + rc - 1) / rc;
  const int rows_per_group = kWaves * RW;

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
      const int rlen = min(rc, ldk - r0);  // even: ldk and rc are
      if (nchunks > 1 || g == 0) {
        __syncthreads();
        for (int e = threadIdx.x; e < rlen * NC; e += kThreads) {
          const int rr = e / NC, c = e - (e / NC) * NC;
          xs[e] = (r0 + rr < nr) ? Xf[(size_t)(r0 + rr) * ldc + col0 + c] : make_float2(0.f, 0.f);
        }
        __syncthreads();
      }
      const int npos = rlen >> 1;  // float4 positions in this chunk
      for (int p = lane; p < npos; p += 64) {
        float4 kv[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
          const int s = sbase + i;
          kv[i] = (s < ns) ? ldg_stream(reinterpret_cast<const float4*>(Kf + (size_t)s * ldk + r0) + p)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const float2 x0 = xs[(2 * p) * NC + c];
          const float2 x1 = xs[(2 * p + 1) * NC + c];
#pragma unroll
          for (int i = 0; i < RW; ++i) {
            acc[i][c][0] += kv[i].x * x0.x - kv[i].y * x0.y + kv[i].z * x1.x - kv[i].w * x1.y;
            acc[i][c][1] += kv[i].x * x0.y + kv[i].y * x0.x + kv[i].z * x1.y + kv[i].w * x1.x;
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float re = wave_sum(acc[i][c][0]);
        const float im = wave_sum(acc[i][c][1]);
        const int s = sbase + i;
        if (lane == 0 && s < ns) Yf[(size_t)s * ldc + col0 + c] = make_float2(re, im);
      }
  }
}

// ---------------------------------------------------------------- adjoint ---
// Requires nr even.  Workgroup = (column tile of 128, frequency).  UR rows of
// K are loaded back to back by each wave before they are consumed.
template <int NC, int UR>
__global__ __launch_bounds__(kThreads) void gemv_adj_kernel(const float2* __restrict__ K,
                                                            const float2* __restrict__ Y,
                                                            float2* __restrict__ X, int ns, int nr, int ldk,
                                                            int ldc, int col0, int rcy) {
  extern __shared__ float2 sh[];  // ys[rcy][NC], then partials [kWaves][64][2][NC]
  float2* ys = sh;
  const int f = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const float2* Kf = K + (size_t)f * ns * ldk;
  const float2* Yf = Y + (size_t)f * ns * ldc;
  float2* Xf = X + (size_t)f * nr * ldc;
  const int p = blockIdx.x * 64 + lane;  // float4 position = columns 2p, 2p+1
  const bool pok = 2 * p < nr;

  float acc[2][NC][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[h][c][0] = acc[h][c][1] = 0.f;

  for (int s0 = 0; s0 < ns; s0 += rcy) {
    const int slen = min(rcy, ns - s0);
    __syncthreads();
    for (int e = threadIdx.x; e < slen * NC; e += kThreads) {
      const int ss = e / NC, c = e - (e / NC) * NC;
      ys[e] = Yf[(size_t)(s0 + ss) * ldc + col0 + c];
    }
    __syncthreads();
    // wave w takes rows w, w+4, w+8, ... of the chunk, UR at a time
    for (int sb = wave * UR; sb < slen; sb += kWaves * UR) {
      float4 kv[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int ss = sb + u;
        kv[u] = (pok && ss < slen)
                    ? ldg_stream(reinterpret_cast<const float4*>(Kf + (size_t)(s0 + ss) * ldk) + p)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int ss = min(sb + u, slen - 1);  // rows past the end carry kv = 0
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const float2 y = ys[ss * NC + c];
          // conj(k) * y = (kr yr + ki yi) + i (kr yi - ki yr)
          acc[0][c][0] += kv[u].x * y.x + kv[u].y * y.y;
          acc[0][c][1] += kv[u].x * y.y - kv[u].y * y.x;
          acc[1][c][0] += kv[u].z * y.x + kv[u].w * y.y;
          acc[1][c][1] += kv[u].z * y.y - kv[u].w * y.x;
        }
      }
    }
  }
  // fixed-order reduction of the four waves' partials
  __syncthreads();
  float* part = reinterpret_cast<float*>(sh);  // [kWaves][2*NC*2][64]
  constexpr int NV = 2 * NC * 2;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int z = 0; z < 2; ++z) part[(wave * NV + (h * NC + c) * 2 + z) * 64 + lane] = acc[h][c][z];
  __syncthreads();
  if (wave == 0 && pok) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        float v[2];
#pragma unroll
        for (int z = 0; z < 2; ++z) {
          const int k = ((h * NC + c) * 2 + z) * 64 + lane;
          v[z] = ((part[k] + part[NV * 64 + k]) + (part[2 * NV * 64 + k] + part[3 * NV * 64 + k]));
        }
        if (2 * p + h < nr) Xf[(size_t)(2 * p + h) * ldc + col0 + c] = make_float2(v[0], v[1]);
      }
  }
}

template <int NC>
mdc_status gemv_group(const mdc_desc& d, const float2* K, int ldk, int adjoint, const float2* in, float2* out,
                      int ldc, int col0, hipStream_t st) {
  if (!adjoint) {
    constexpr int RW = (NC >= 4) ? 2 : 4;
    const int rc = 4096 / NC;
    const int rows_per_group = kWaves * RW;
    const int ngroups = (d.ns + rows_per_group - 1) / rows_per_group;
    int gpb = (int)((long)ngroups * d.nfmax / 4096);
    gpb = gpb < 1 ? 1 : (gpb > 8 ? 8 : gpb);
    const int nblk = (ngroups + gpb - 1) / gpb;
    const size_t lds = (size_t)rc * NC * sizeof(float2);
    hipLaunchKernelGGL((gemv_fwd_kernel<NC, RW>), dim3(nblk, d.nfmax), dim3(kThreads), lds, st, K, in, out, d.ns,
                       d.nr, ldk, ldc, col0, gpb, rc);
    return check_launch("gemv_fwd_kernel");
  }
  constexpr int UR = (NC >= 4) ? 4 : 8;
  const int rcy = 4096 / NC;
  const size_t lds_y = (size_t)rcy * NC * sizeof(float2);
  const size_t lds_p = (size_t)kWaves * 2 * NC * 2 * 64 * sizeof(float);
  const size_t lds = lds_y > lds_p ? lds_y : lds_p;
  const int nblk = ((d.nr + 1) / 2 + 63) / 64;
  hipLaunchKernelGGL((gemv_adj_kernel<NC, UR>), dim3(nblk, d.nfmax), dim3(kThreads), lds, st, K, in, out, d.ns, d.nr,
                     ldk, ldc, col0, rcy);
  return check_launch("gemv_adj_kernel");
}

}  // namespace

// Few-column product (ncols columns in groups of 8, 4, 2, 1).
mdc_status gemv_launch(const mdc_desc& d, const float2* K, int ldk, int adjoint, const float2* in, float2* out,
                       int ncols, hipStream_t st) {
  int c0 = 0;
  while (c0 < ncols) {
    const int rem = ncols - c0;
    mdc_status s;
    if (rem >= 8) { s = gemv_group<8>(d, K, ldk, adjoint, in, out, ncols, c0, st); c0 += 8; }
    else if (rem >= 4) { s = gemv_group<4>(d, K, ldk, adjoint, in, out, ncols, c0, st); c0 += 4; }
    else if (rem >= 2) { s = gemv_group<2>(d, K, ldk, adjoint, in, out, ncols, c0, st); c0 += 2; }
    else { s = gemv_group<1>(d, K, ldk, adjoint, in, out, ncols, c0, st); c0 += 1; }
    if (s != MDC_OK) return s;
  }
  return MDC_OK;
}

}  // namespace mdc
