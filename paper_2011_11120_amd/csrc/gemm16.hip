// Per-frequency complex kernel product on the 16-bit matrix cores for the
// reduced-precision storage formats: the many-point product (Eq.4 slices)
// with a kernel of 4 or 8 bytes per complex value.
//
// Operands are split into hi + lo parts so the product keeps close to FP32
// accuracy (the split-operand scheme of Henry, Tang & Heinecke, ARITH 2019),
// FP32 accumulation throughout:
//   BF16X2: K stored as bf16 hi + lo (8 bytes per complex); spectra split into
//           bf16 hi + lo; three products Khi Xhi + Khi Xlo + Klo Xhi
//           (v_mfma_f32_32x32x16_bf16).
//   BF16:   K stored as bf16 (4 bytes); two products Khi Xhi + Khi Xlo.
//   FP16S:  K stored as FP16 of K * 2^e_f (4 bytes, power-of-two scale per
//           frequency); spectra split into FP16 hi + lo of X * 2^s_fv, s_fv from the
//           maximum of column v at frequency f; two products on
//           v_mfma_f32_32x32x16_f16; both scales divided out of the result (exact,
//           powers of two).  The spectra scale is per column, so the rounding of a
//           column does not depend on the other columns of the product (requests
//           batched together round as they would alone).
//   FP16:   the FP16S kernel and scales, spectra rounded once to FP16 (the hi part
//           of the split): one product Khi Xhi.
//
// The complex product is the real embedding used by the FP32 kernel: the
// interleaved kernel is a real ns x 2nr matrix (forward) or its transpose
// (adjoint), and the spectra enter as 2x2 real blocks, forward (c, -d | d, c),
// adjoint (e, f | f, -e).
//
// Data flow per apply:
//  1. bsplit_kernel transposes the FP32 spectra [f][k][v] into split pair words
//     [f][v][k/4][hi 4 words | lo 4 words], zero-padded to whole tiles, so every
//     row tile stages them with plain 16-byte copies (FP16S first takes the
//     per-column maxima, spec_max_kernel).
//  2. gemm16_kernel: a 256-thread workgroup computes 256 output rows x 64 complex
//     columns of one frequency.  Wave w owns rows 64w .. 64w + 63 (two blocks of
//     32 rows) for all 64 complex columns, as eight 32x32 MFMA blocks: block ni
//     holds the real part (ni even) or imaginary part (ni odd) of complex columns
//     32 (ni / 2) .. 32 (ni / 2) + 31.
//     * The kernel is never shared between waves, so it bypasses LDS: each lane
//       loads its own fragment registers five 16-column k-steps ahead of use
//       (ring of six register sets).  Forward: four consecutive complex values
//       of one kernel row; adjoint: one kernel column at four consecutive rows.
//     * The split spectra go through LDS, triple-buffered per 32-column slab,
//       both embedded variants stored side by side (the sign/swap is applied
//       once per slab at the store, not per fragment).  Spectra fragments are
//       read one half-step (8 complex columns) ahead of their MFMAs.
//     * The 32x32 MFMA shape issues back to back from one wave per SIMD, so the
//       inner loop holds only fragment loads and MFMAs; one workgroup per CU
//       leaves each wave the register file for the deep ring and accumulators.
//     * Loads are never predicated (a predicated load makes the compiler wait
//       for every outstanding load at the merge, draining the ring): indices
//       past the end are clamped onto valid kernel data, which meets zero
//       spectra or feeds outputs that are not stored.
//     * Workgroups are numbered so that the row tiles of one frequency run on
//       one XCD (hardware deals workgroups round-robin over the 8 XCDs), which
//       keeps that frequency's spectra in one L2.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.hpp"
#include "store.hpp"

namespace mdc {
namespace {

typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int BM = 256;                 // output rows per workgroup (4 waves x 64)
constexpr int BN = 64;                  // complex output columns per workgroup
constexpr int BK = 32;                  // complex reduction columns per LDS slab
constexpr int KSTEP_PAD = 96;           // reduction length padded to six 16-column k-steps
constexpr int LDB = 36;                 // words per LDS row: 32 reduction indices + 4 pad
constexpr int HALF = 2 * BN * LDB;      // one (hi or lo) slab: 128 real columns
constexpr int BUF = 2 * HALF + 64;      // hi | lo, lo shifted by 32 banks (conflict-free stores)

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

// Power-of-two scale of the FP16 spectra split: largest s = 2^e with max * s <= 2^14.
__device__ __forceinline__ float spec_scale(float mx) {
  if (!(mx > 0.f)) return 1.0f;
  int e;
  frexpf(mx, &e);  // mx in [2^(e-1), 2^e)
  return ldexpf(1.0f, 14 - e);
}

// RB: 32-row blocks per wave.  RB = 2: four waves of 64 rows (one per SIMD, deep register ring);
// RB = 1: eight waves of 32 rows (two per SIMD, half the registers each).
template <int FMT, bool ADJ, int RB>
__global__ __launch_bounds__(BM / (32 * RB) * 64, 1) void gemm16_kernel(const char* __restrict__ K,
                                                             const float* __restrict__ fscale,
                                                             const float* __restrict__ bmax, int ns, int nr, int ldk,
                                                             const unsigned int* __restrict__ Bp, int KG, int NCP,
                                                             float2* __restrict__ Cdst, int ncols, int tiles_m,
                                                             int tiles_n, int nblocks) {
  __shared__ __attribute__((aligned(16))) unsigned int Bs[3 * BUF];
  constexpr bool X2 = FMT == MDC_BF16X2;
  constexpr bool F16 = FMT == MDC_FP16S || FMT == MDC_FP16;
  constexpr bool ONE = FMT == MDC_FP16;  // spectra hi part only: one product
  using frag = typename std::conditional<F16, h8v, bf8v>::type;
  constexpr int NTH = BM / (32 * RB) * 64;  // threads per workgroup
  constexpr int NA = (X2 ? 2 : 1) * 2 * RB;  // u4v per lane per k-step: RB row blocks x 2 k-halves (x hi, lo)
  constexpr int NB = 1024 / NTH;             // 16-byte spectra pieces per thread per slab

  const int b = blockIdx.x;
  const int q8 = nblocks >> 3, rem = nblocks & 7, xcd = b & 7;
  const int L = xcd * q8 + min(xcd, rem) + (b >> 3);
  const int tiles_per_f = tiles_m * tiles_n;
  const int f = L / tiles_per_f;
  const int t = L - f * tiles_per_f;
  // column tiles of one row block are adjacent, so they run together on one XCD and
  // share that block's kernel rows through L2 instead of each reading them from HBM
  const int nt = t % tiles_n, mt = t / tiles_n;
  const int m0 = mt * BM, n0 = nt * BN;
  const int M = ADJ ? nr : ns;
  const size_t rowb = X2 ? (size_t)ldk * 8 : (size_t)ldk * 4;
  const unsigned int* Bf = Bp + ((size_t)f * NCP + n0) * KG * 8;
  float* Cf = reinterpret_cast<float*>(Cdst + (size_t)f * M * ncols);
  const char* Kf = K + (size_t)f * ns * rowb;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, kh = lane >> 5;
  const int nsteps = KG >> 2;  // 16-column k-steps, a multiple of 6
  const int nslabs = nsteps >> 1;

  // this lane's RB output rows (kernel rows forward, kernel columns adjoint), clamped
  size_t aoff[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int rr = min(m0 + wave * 32 * RB + rb * 32 + l32, M - 1);
    aoff[rb] = !ADJ ? (size_t)rr * rowb : (X2 ? (size_t)(rr >> 2) * 32 + (rr & 3) * 4 : (size_t)rr * 4);
  }
  // kernel fragments of k-step j: r[q] (q = 2 rb + h) holds the lane's four reduction
  // indices 16 j + 8 h + 4 kh .. + 3 of row block rb (X2: r[2q] hi, r[2q + 1] lo)
  auto load_a = [&](int j, u4v (&r)[NA]) {
#pragma unroll
    for (int q = 0; q < 2 * RB; ++q) {
      const int h = q & 1, rb = q >> 1;
      const int g = 4 * min(j, nsteps - 1) + 2 * h + kh;  // group of four reduction indices
      if constexpr (!ADJ) {
        const char* p = Kf + aoff[rb] + (size_t)min(g, (ldk >> 2) - 1) * (X2 ? 32 : 16);
        r[X2 ? 2 * q : q] = *reinterpret_cast<const u4v*>(p);
        if constexpr (X2) r[2 * q + 1] = *reinterpret_cast<const u4v*>(p + 16);
      } else {
        unsigned int wh[4], wl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const char* p = Kf + (size_t)min(4 * g + i, ns - 1) * rowb + aoff[rb];
          wh[i] = *reinterpret_cast<const unsigned int*>(p);
          if constexpr (X2) wl[i] = *reinterpret_cast<const unsigned int*>(p + 16);
        }
        r[X2 ? 2 * q : q] = u4v{wh[0], wh[1], wh[2], wh[3]};
        if constexpr (X2) r[2 * q + 1] = u4v{wl[0], wl[1], wl[2], wl[3]};
      }
    }
  };
  // split spectra of one slab: 64 columns x 8 groups x (hi, lo), NB 16-byte pieces per thread
  u4v pb[NB];
  auto load_b = [&](int sl) {
    const int g0 = min(sl, nslabs - 1) * (BK / 4);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int idx = tid + NTH * q;
      const int v = idx >> 4, gi = (idx & 15) >> 1, half = idx & 1;
      pb[q] = *reinterpret_cast<const u4v*>(Bf + ((size_t)v * KG + g0 + gi) * 8 + half * 4);
    }
  };
  // both embedded variants: forward (c, -d) | (d, c), adjoint (e, f) | (f, -e)
  auto store_b = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int idx = tid + NTH * q;
      const int v = idx >> 4, gi = (idx & 15) >> 1, half = idx & 1;
      const u4v w = pb[q];
      const u4v sw = u4v{swap16(w.x), swap16(w.y), swap16(w.z), swap16(w.w)};
      const int row0 = (v >> 5) * 64 + (v & 31);
      unsigned int* base = Bs + buf * BUF + half * (HALF + 32) + 4 * gi;
      *reinterpret_cast<u4v*>(base + row0 * LDB) = ADJ ? w : w ^ 0x80000000u;
      *reinterpret_cast<u4v*>(base + (row0 + 32) * LDB) = ADJ ? sw ^ 0x80000000u : sw;
    }
  };
  // spectra fragments of one half-step (k-step ks of a slab, half h) from LDS buffer buf
  struct Frags {
    frag hi[4], lo[4];
  };
  auto read_b = [&](Frags& F, int buf, int ks, int h) {
    const unsigned int* Bh = Bs + buf * BUF;
    const unsigned int* Bl = Bh + HALF + 32;
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int off = (ni * 32 + l32) * LDB + ks * 16 + 8 * h + 4 * kh;
      F.hi[ni] = __builtin_bit_cast(frag, *reinterpret_cast<const u4v*>(Bh + off));
      if constexpr (!ONE) F.lo[ni] = __builtin_bit_cast(frag, *reinterpret_cast<const u4v*>(Bl + off));
    }
  };

  f16v acc[RB][4];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[rb][i][e] = 0.f;

  auto mma = [](frag a, frag bb, f16v c) {
    if constexpr (F16) return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, bb, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, c, 0, 0, 0);
  };
  // Row blocks that hold no output row (the last row tile when M is not a multiple of BM)
  // skip their matrix operations; their clamped loads and the cooperative spectra staging
  // run as in every other block.
  bool rvalid[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) rvalid[rb] = m0 + __builtin_amdgcn_readfirstlane(wave) * 32 * RB + rb * 32 < M;
  auto compute = [&](const u4v (&r)[NA], const Frags& F, int h) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (!rvalid[rb]) continue;
      const int q = 2 * rb + h;
      const frag ah = __builtin_bit_cast(frag, r[X2 ? 2 * q : q]);
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc[rb][ni] = mma(ah, F.hi[ni], acc[rb][ni]);
      if constexpr (!ONE) {
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[rb][ni] = mma(ah, F.lo[ni], acc[rb][ni]);
      }
      if constexpr (X2) {
        const frag al = __builtin_bit_cast(frag, r[2 * q + 1]);
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[rb][ni] = mma(al, F.hi[ni], acc[rb][ni]);
      }
    }
  };

  // Pipeline: kernel fragments five k-steps ahead in a ring of six register sets;
  // spectra staged from memory at the start of slab sl, stored to LDS buffer
  // (sl + 2) % 3 at its end; spectra fragments read one half-step ahead.  An
  // iteration covers six k-steps = three slabs = one turn of both rings, so every
  // ring and buffer index below is a compile-time constant.
  u4v ring[6][NA];
  Frags F[2];
#pragma unroll
  for (int i = 0; i < 5; ++i) load_a(i, ring[i]);
  load_b(0);
  store_b(0);
  load_b(1);
  store_b(1);
  __syncthreads();
  read_b(F[0], 0, 0, 0);
  for (int j = 0; j < nsteps; j += 6) {
#pragma unroll
    for (int p = 0; p < 12; ++p) {  // half-step p: k-step i = p / 2 of the iteration, half h = p % 2
      const int i = p >> 1, h = p & 1, s3 = p >> 2;
      const int st = j + i;
      if ((p & 3) == 0) load_b((st >> 1) + 2);
      if (h == 0) load_a(st + 5, ring[(i + 5) % 6]);  // the set freed by step st - 1
      __builtin_amdgcn_sched_barrier(0);
      const int np = p + 1;  // next half-step (np == 12: first of the next iteration, buffer 0)
      read_b(F[np & 1], (np >> 2) % 3, (np >> 1) & 1, np & 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(ring[i], F[p & 1], h);
      __builtin_amdgcn_sched_barrier(0);
      if ((p & 3) == 3) {
        store_b((s3 + 2) % 3);
        __syncthreads();
      }
    }
  }

  // D of a 32x32 block: column = lane % 32, row = 8 (e / 4) + 4 (lane / 32) + e % 4
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int v = n0 + (ni >> 1) * 32 + l32;
      if (v >= ncols) continue;
      // FP16: divide out the kernel's and the column's power-of-two scales
      const float osc = F16 ? 1.0f / (fscale[f] * spec_scale(bmax[(size_t)f * NCP + v])) : 1.0f;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + wave * 32 * RB + rb * 32 + 8 * (e >> 2) + 4 * kh + (e & 3);
        if (row < M) Cf[((size_t)row * ncols + v) * 2 + (ni & 1)] = acc[rb][ni][e] * osc;
      }
    }
}

// Split spectra X[f][k][ncols] (complex FP32) into Bp[f][v][g][8]: words 0-3 the hi pair
// words (re | im << 16) of k = 4g..4g+3, words 4-7 the lo pair words, v < NCP, g < KG, zero
// outside [KD) x [ncols).  bf16: hi = RNE(x), lo = RNE(x - hi).  FP16 (F16): the same of
// x * s_fv with s_fv = spec_scale(bmax[f][v]).  One workgroup transposes a 64 (k) x 64 (v)
// tile through LDS.
template <bool F16>
__global__ __launch_bounds__(kThreads) void bsplit_kernel(const float2* __restrict__ X, int KD, int ncols, int KG,
                                                          int NCP, const float* __restrict__ bmax,
                                                          unsigned int* __restrict__ Bp) {
  __shared__ float2 tile[64][65];
  const int f = blockIdx.z, k0 = blockIdx.x * 64, v0 = blockIdx.y * 64;
  const float2* Xf = X + (size_t)f * KD * ncols;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int idx = tid + kThreads * i;
    const int kk = idx >> 6, v = idx & 63;
    const int k = k0 + kk, c = v0 + v;
    tile[kk][v] = (k < KD && c < ncols) ? Xf[(size_t)k * ncols + c] : make_float2(0.f, 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int task = tid + kThreads * i;
    const int g = task & 15, v = task >> 4;
    const int gg = (k0 >> 2) + g;
    if (gg >= KG) continue;
    const float sc = F16 ? spec_scale(bmax[(size_t)f * NCP + v0 + v]) : 1.0f;
    unsigned int hi[4], lo[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      if constexpr (F16) {
        const float re = tile[4 * g + h][v].x * sc, im = tile[4 * g + h][v].y * sc;
        const unsigned int hr = f16_rne_bits(re), hm = f16_rne_bits(im);
        hi[h] = hr | (hm << 16);
        lo[h] = f16_rne_bits(re - f16_bits_to_f(hr)) | (f16_rne_bits(im - f16_bits_to_f(hm)) << 16);
      } else {
        split_pair(tile[4 * g + h][v].x, tile[4 * g + h][v].y, hi[h], lo[h]);
      }
    }
    unsigned int* dst = Bp + (((size_t)f * NCP + v0 + v) * KG + gg) * 8;
    *reinterpret_cast<u4v*>(dst) = u4v{hi[0], hi[1], hi[2], hi[3]};
    *reinterpret_cast<u4v*>(dst + 4) = u4v{lo[0], lo[1], lo[2], lo[3]};
  }
}

__global__ void zero_floats(float* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// bmax[f][v] = max |re|, |im| over column v of the spectrum slice of frequency f (X[f][k][v],
// k < KD), v < ncols (bmax zeroed first; columns past ncols keep 0).  A workgroup covers 64
// columns of one frequency and one chunk of kchunk reduction rows (its four waves stride over
// them); chunks combine by an atomic maximum, which is exact and order independent for
// non-negative floats compared as integers.
__global__ __launch_bounds__(kThreads) void spec_max_kernel(const float2* __restrict__ X, int KD, int ncols, int NCP,
                                                            int kchunk, float* __restrict__ bmax) {
  __shared__ float part[kThreads / 64][64];
  const int f = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v = blockIdx.x * 64 + lane;
  const float2* Xf = X + (size_t)f * KD * ncols;
  const int k0 = blockIdx.z * kchunk, k1 = min(KD, k0 + kchunk);
  float m = 0.f;
  if (v < ncols)
    for (int k = k0 + wave; k < k1; k += kThreads / 64) {
      const float2 z = Xf[(size_t)k * ncols + v];
      m = fmaxf(m, fmaxf(fabsf(z.x), fabsf(z.y)));
    }
  part[wave][lane] = m;
  __syncthreads();
  if (wave == 0 && v < ncols) {
    m = fmaxf(fmaxf(part[0][lane], part[1][lane]), fmaxf(part[2][lane], part[3][lane]));
    atomicMax(reinterpret_cast<unsigned int*>(bmax) + (size_t)f * NCP + v, __float_as_uint(m));
  }
}

size_t split_cols(const mdc_desc& d) { return (size_t)(d.max_cols + BN - 1) / BN * BN; }

// Bytes of the split spectra: nfmax x (max_cols rounded up to BN) x (reduction rounded up to
// KSTEP_PAD) x 8.
size_t split_data_bytes(const mdc_desc& d) {
  const size_t kdp = (size_t)((d.ns > d.nr ? d.ns : d.nr) + KSTEP_PAD - 1) / KSTEP_PAD * KSTEP_PAD;
  return (size_t)d.nfmax * split_cols(d) * kdp * 8;
}

template <int FMT, bool ADJ, int RB>
void launch_gemm16(const char* K, const float* fscale, const float* bmax, const mdc_desc& d, int ldk,
                   const unsigned int* bsplit, int KG, int NCP, float2* out, int ncols, int tiles_m, int tiles_n,
                   int nblocks, hipStream_t st) {
  constexpr int NTH = BM / (32 * RB) * 64;
  hipLaunchKernelGGL((gemm16_kernel<FMT, ADJ, RB>), dim3(nblocks), dim3(NTH), 0, st, K, fscale, bmax, d.ns, d.nr, ldk,
                     bsplit, KG, NCP, out, ncols, tiles_m, tiles_n, nblocks);
}

// variant 0: four waves of 64 rows per workgroup; variant 1: eight waves of 32 rows.
template <int FMT>
mdc_status launch_fmt(const mdc_desc& d, const char* K, const float* fscale, int ldk, int adjoint, const float2* in,
                      float2* out, int ncols, unsigned int* bsplit, int variant, hipStream_t st) {
  const int M = adjoint ? d.nr : d.ns;
  const int KD = adjoint ? d.ns : d.nr;
  const int tiles_m = (M + BM - 1) / BM;
  const int tiles_n = (ncols + BN - 1) / BN;
  const int NCP = tiles_n * BN;
  const int KG = (KD + KSTEP_PAD - 1) / KSTEP_PAD * (KSTEP_PAD / 4);
  const long nb = (long)tiles_m * tiles_n * d.nfmax;
  if (nb > 0x7fffffffL) return fail(MDC_ENOTSUP, "too many GEMM tiles");
  const int nblocks = (int)nb;
  float* bmax = reinterpret_cast<float*>(reinterpret_cast<char*>(bsplit) + align_up(split_data_bytes(d), 256));
  const dim3 sgrid((KG * 4 + 63) / 64, NCP / 64, d.nfmax);
  if constexpr (FMT == MDC_FP16S || FMT == MDC_FP16) {
    const int nmax = d.nfmax * NCP;
    hipLaunchKernelGGL(zero_floats, dim3((nmax + 255) / 256), dim3(256), 0, st, bmax, nmax);
    const int kchunk = 256, nch = (KD + kchunk - 1) / kchunk;
    hipLaunchKernelGGL(spec_max_kernel, dim3(NCP / 64, d.nfmax, nch), dim3(kThreads), 0, st, in, KD, ncols, NCP,
                       kchunk, bmax);
    hipLaunchKernelGGL(bsplit_kernel<true>, sgrid, dim3(kThreads), 0, st, in, KD, ncols, KG, NCP, bmax, bsplit);
  } else {
    hipLaunchKernelGGL(bsplit_kernel<false>, sgrid, dim3(kThreads), 0, st, in, KD, ncols, KG, NCP, bmax, bsplit);
  }
  mdc_status s = check_launch("bsplit_kernel");
  if (s != MDC_OK) return s;
  if (variant == 1) {
    if (adjoint) launch_gemm16<FMT, true, 1>(K, fscale, bmax, d, ldk, bsplit, KG, NCP, out, ncols, tiles_m, tiles_n, nblocks, st);
    else launch_gemm16<FMT, false, 1>(K, fscale, bmax, d, ldk, bsplit, KG, NCP, out, ncols, tiles_m, tiles_n, nblocks, st);
  } else {
    if (adjoint) launch_gemm16<FMT, true, 2>(K, fscale, bmax, d, ldk, bsplit, KG, NCP, out, ncols, tiles_m, tiles_n, nblocks, st);
    else launch_gemm16<FMT, false, 2>(K, fscale, bmax, d, ldk, bsplit, KG, NCP, out, ncols, tiles_m, tiles_n, nblocks, st);
  }
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

size_t gemm16_split_bytes(const mdc_desc& d) {
  return align_up(split_data_bytes(d), 256) + align_up((size_t)d.nfmax * split_cols(d) * 4, 256);
}

mdc_status gemm16_launch(const mdc_desc& d, const void* K, const float* fscale, int ldk, int adjoint,
                         const float2* in, float2* out, int ncols, unsigned int* bsplit, int variant, hipStream_t st) {
  const char* k = static_cast<const char*>(K);
  switch (d.prec) {
    case MDC_FP16S: return launch_fmt<MDC_FP16S>(d, k, fscale, ldk, adjoint, in, out, ncols, bsplit, variant, st);
    case MDC_FP16: return launch_fmt<MDC_FP16>(d, k, fscale, ldk, adjoint, in, out, ncols, bsplit, variant, st);
    case MDC_BF16: return launch_fmt<MDC_BF16>(d, k, fscale, ldk, adjoint, in, out, ncols, bsplit, variant, st);
    case MDC_BF16X2: return launch_fmt<MDC_BF16X2>(d, k, fscale, ldk, adjoint, in, out, ncols, bsplit, variant, st);
    default: return fail(MDC_EINVAL, "gemm16: not a 16-bit format");
  }
}

}  // namespace mdc
