// Per-frequency complex kernel product for many columns on the matrix cores
// (Eq.4 slices; the matrix-matrix form the paper uses when several virtual
// points are solved together, Benchmarking and Discussion sections).
//
// The complex product is run as one real GEMM on v_mfma_f32_16x16x4f32 (FP32
// in, FP32 accumulate) without repacking the kernel: K_f stored as interleaved
// (re, im) pairs is read as a real ns x 2nr matrix.
//
//   forward  Y = K X:    A[s][2r+j] = K[s][r].(re,im)_j,
//                        B[2r][2v] = c,  B[2r][2v+1] = d,  B[2r+1][2v] = -d,  B[2r+1][2v+1] = c
//                        (X[r][v] = c + i d); the real result C[s][2v+j] is Y[s][v] interleaved.
//   adjoint  X = K^H Y:  A[r][2s+j] = K[s][r].(re,im)_j  (the same memory, read along s),
//                        B[2s][2v] = e,  B[2s][2v+1] = f,  B[2s+1][2v] = f,  B[2s+1][2v+1] = -e
//                        (Y[s][v] = e + i f).
//
// One MFMA k-step of depth 4 consumes two complex columns of the kernel.  The
// spectra are embedded into the real B matrix once, when a slab is stored to
// LDS, so fragment reads are plain loads with no arithmetic between the
// matrix operations; each k-step's fragments are read while the previous
// step's MFMAs run, the reads interleaved with them. Tiles: a 256-thread
// workgroup computes 128 output rows x BN complex columns (BN = 64 or 32; four
// waves of 64 x BN real outputs), stepping through the reduction 16 complex
// columns at a time with double-buffered LDS and a register prefetch of the
// next slab. Workgroups are numbered so that all tiles of one frequency run on
// the same XCD (hardware deals workgroups round-robin over the 8 XCDs), which
// keeps that frequency's spectrum panel in one L2.
#include "common.hpp"

namespace mdc {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int BM = 128;        // output rows per workgroup
constexpr int BK = 16;         // complex reduction columns per slab
constexpr int A_FWD_LD = 34;   // floats per A row (forward): 2*BK + 2, so a fragment read hits 32 banks
constexpr int A_ADJ_LD = 288;  // floats per A row (adjoint): 2*BM + 32 pad
constexpr int A_FLOATS = 4608; // >= BM*A_FWD_LD, == BK*A_ADJ_LD

// BN complex output columns per workgroup (64 or 32; the autotuner picks).
template <bool ADJ, int BN>
__global__ __launch_bounds__(kThreads, 2) void gemm_f32_kernel(const float2* __restrict__ K, int ns, int nr, int ldk,
                                                               const float2* __restrict__ Bsrc,
                                                               float2* __restrict__ Cdst, int ncols, int tiles_m,
                                                               int tiles_n, int nblocks) {
  // The spectra slab is stored already embedded as the real 2BK x 2BN matrix B (row 2k + part,
  // column 2v + j), so a B fragment is one plain LDS read; the row stride 2BN + 16 puts the four
  // k rows of a fragment read 16 banks apart.
  constexpr int BRL = 2 * BN + 16;    // floats per embedded B row
  constexpr int NI = BN / 16;         // 16-real-column MFMA blocks per wave (a wave covers BN real columns)
  constexpr int B_LOADS = BK * BN / kThreads;
  __shared__ __attribute__((aligned(16))) float As[2][A_FLOATS];
  __shared__ __attribute__((aligned(16))) float Br[2][2 * BK * BRL];

  // XCD-aware numbering: hardware block b runs on XCD b % 8; give each XCD a contiguous
  // range of logical tiles (bijective for any nblocks).
  const int b = blockIdx.x;
  const int q8 = nblocks >> 3, rem = nblocks & 7, xcd = b & 7;
  const int L = xcd * q8 + min(xcd, rem) + (b >> 3);
  const int tiles_per_f = tiles_m * tiles_n;
  const int f = L / tiles_per_f;
  const int t = L - f * tiles_per_f;
  // column tiles of one row block are adjacent, so they run together on one XCD and
  // share that block's kernel rows through L2 instead of each reading them from HBM
  const int nt = t % tiles_n, mt = t / tiles_n;
  const int M = ADJ ? nr : ns;
  const int KD = ADJ ? ns : nr;
  const int m0 = mt * BM, n0 = nt * BN;
  const float2* Kf = K + (size_t)f * ns * ldk;
  const float2* Bf = Bsrc + (size_t)f * KD * ncols;
  float* Cf = reinterpret_cast<float*>(Cdst + (size_t)f * M * ncols);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;

  float4 pa[4];
  float2 pb[B_LOADS];
  auto load_slab = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + kThreads * q;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (!ADJ) {
        const int row = idx >> 3, c4 = idx & 7;
        const int m = m0 + row, rr = k0 + 2 * c4;
        if (m < ns && rr < ldk) v = *reinterpret_cast<const float4*>(Kf + (size_t)m * ldk + rr);
      } else {
        const int srow = idx >> 6, c4 = idx & 63;
        const int s = k0 + srow, r = m0 + 2 * c4;
        if (s < ns && r < ldk) v = *reinterpret_cast<const float4*>(Kf + (size_t)s * ldk + r);
      }
      pa[q] = v;
    }
#pragma unroll
    for (int q = 0; q < B_LOADS; ++q) {
      const int idx = tid + kThreads * q;
      const int rr = idx / BN, c = idx % BN;
      const int kk = k0 + rr, v = n0 + c;
      pb[q] = (kk < KD && v < ncols) ? Bf[(size_t)kk * ncols + v] : make_float2(0.f, 0.f);
    }
  };
  auto store_slab = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + kThreads * q;
      if (!ADJ) {  // two 8-byte stores (rows are 8-byte aligned at stride 34)
        float* dst = &As[buf][(idx >> 3) * A_FWD_LD + 4 * (idx & 7)];
        *reinterpret_cast<float2*>(dst) = make_float2(pa[q].x, pa[q].y);
        *reinterpret_cast<float2*>(dst + 2) = make_float2(pa[q].z, pa[q].w);
      } else {
        *reinterpret_cast<float4*>(&As[buf][(idx >> 6) * A_ADJ_LD + 4 * (idx & 63)]) = pa[q];
      }
    }
    // real embedding of X[k][v] = c + i d:  forward rows (c, d | -d, c), adjoint rows (c, d | d, -c)
#pragma unroll
    for (int q = 0; q < B_LOADS; ++q) {
      const int idx = tid + kThreads * q;
      const int rr = idx / BN, c = idx % BN;
      const float2 z = pb[q];
      float* row0 = &Br[buf][(2 * rr) * BRL + 2 * c];
      *reinterpret_cast<float2*>(row0) = z;
      *reinterpret_cast<float2*>(row0 + BRL) = ADJ ? make_float2(z.y, -z.x) : make_float2(-z.y, z.x);
    }
  };

  f4v acc[4][NI];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  // fragments of k-step ks (real reduction rows 4 ks .. 4 ks + 3; this lane's row is 4 ks + lk)
  struct Frag {
    float a[4], b[NI];
  };
  auto read_frag = [&](Frag& F, int buf, int ks) {
    const float* A = As[buf];
    const float* B = Br[buf];
    const int kr = 4 * ks + lk;  // = 2 cc + part with cc = 2 ks + lk / 2, part = lk % 2
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
      const int row = wm * 64 + mi * 16 + li;
      F.a[mi] = ADJ ? A[(kr >> 1) * A_ADJ_LD + 2 * row + (kr & 1)] : A[row * A_FWD_LD + kr];
    }
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) F.b[ni] = B[kr * BRL + wn * BN + ni * 16 + li];
  };

  // A wave whose 64 rows all lie past the last output row (in the last row tile when M is not a
  // multiple of BM) skips the matrix operations; it still takes part in the slab loads.
  const bool active = m0 + __builtin_amdgcn_readfirstlane(wm) * 64 < M;
  const int nslabs = (KD + BK - 1) / BK;
  load_slab(0);
  store_slab(0);
  __syncthreads();
  Frag F[2];
  for (int sl = 0; sl < nslabs; ++sl) {
    const int buf = sl & 1;
    if (sl + 1 < nslabs) load_slab((sl + 1) * BK);
    if (active) {
      read_frag(F[0], buf, 0);
#pragma unroll
      for (int ks = 0; ks < BK / 2; ++ks) {
        // the next k-step's fragments are read while this step's matrix operations run, one
        // LDS read issued between every MPR of them
        if (ks + 1 < BK / 2) read_frag(F[(ks + 1) & 1], buf, ks + 1);
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
          for (int ni = 0; ni < NI; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(F[ks & 1].a[mi], F[ks & 1].b[ni], acc[mi][ni], 0, 0, 0);
        if (ks + 1 < BK / 2) {
          constexpr int NR = 4 + NI, MPR = 4 * NI / NR;  // fragment reads, matrix operations per read
#pragma unroll
          for (int i = 0; i < NR; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, MPR, 0);  // matrix operations
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);    // one LDS read
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (sl + 1 < nslabs) store_slab(buf ^ 1);
    __syncthreads();
  }

  // D[i][j] of a 16x16 block: j = lane % 16, i = 4 * (lane / 16) + e
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int n = 2 * n0 + wn * (BN) + ni * 16 + li;  // real output column
      const int v = n >> 1;
      if (v >= ncols) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm * 64 + mi * 16 + 4 * lk + e;
        if (row < M) Cf[((size_t)row * ncols + v) * 2 + (n & 1)] = acc[mi][ni][e];
      }
    }
}

template <int BN>
mdc_status gemm_bn(const mdc_desc& d, const float2* K, int ldk, int adjoint, const float2* in, float2* out, int ncols,
                   hipStream_t st) {
  const int M = adjoint ? d.nr : d.ns;
  const int tiles_m = (M + BM - 1) / BM;
  const int tiles_n = (ncols + BN - 1) / BN;
  const long nb = (long)tiles_m * tiles_n * d.nfmax;
  if (nb > 0x7fffffffL) return fail(MDC_ENOTSUP, "too many GEMM tiles");
  const int nblocks = (int)nb;
  if (adjoint)
    hipLaunchKernelGGL((gemm_f32_kernel<true, BN>), dim3(nblocks), dim3(kThreads), 0, st, K, d.ns, d.nr, ldk, in, out,
                       ncols, tiles_m, tiles_n, nblocks);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<false, BN>), dim3(nblocks), dim3(kThreads), 0, st, K, d.ns, d.nr, ldk, in,
                       out, ncols, tiles_m, tiles_n, nblocks);
  return check_launch("gemm_f32_kernel");
}

}  // namespace

// bn: 64 or 32 complex columns per workgroup.
mdc_status gemm_launch(const mdc_desc& d, const float2* K, int ldk, int adjoint, const float2* in, float2* out,
                       int ncols, hipStream_t st, int bn) {
  if (bn == 32) return gemm_bn<32>(d, K, ldk, adjoint, in, out, ncols, st);
  return gemm_bn<64>(d, K, ldk, adjoint, in, out, ncols, st);
}

}  // namespace mdc
