// Orthogonal real FFT along the (outermost) time axis, truncated to nfmax bins,
// and its zero-padded inverse (Eq.3: I F and F^H I^H; batch-matmul section:
// orthogonal real transform, 1/sqrt(nt) both ways, positive frequencies only).
//
// A length-nt real trace is packed into M = nt/2 complex points
// z[m] = x[2m] + i x[2m+1] and transformed by a radix-8 (plus one radix-2 or 4)
// Stockham FFT held in LDS; a split step then yields the nt/2+1 real-signal
// bins, of which only the first nfmax are written.  The inverse runs the same
// steps backwards from zero-padded bins, dropping the imaginary parts of the
// DC and Nyquist bins (what makes the pair exactly adjoint).  Its epilogue
// applies the window Theta, the sign and the identity term of the Marchenko
// blocks and, inside the solvers, the vector recurrence out += c * out_old
// with one FP64 partial sum of out^2 per workgroup (the next norm).
//
// Layout: each workgroup owns CB consecutive traces (consecutive (n, v)
// columns of the [nt][n][nv] array), so every global access of a time row or
// a spectral row is contiguous across lanes; with 16-byte vectors a thread
// moves four traces of one time row.  The solvers' vectors may instead be
// tiled (fft_tile): the workgroup's CB traces then form one contiguous
// [nt][CB] tile, and its time-domain reads and writes one contiguous block.  Long transforms with wide tiles run one
// wave per trace of the tile.  All global loads of a thread are issued
// before any is consumed.  LDS holds z as [M][CB] complex plus the twiddle
// table tw[k] = exp(-2 pi i k / nt) (built in FP64, rounded once to FP32).
#include <climits>
#include <cmath>

#include "common.hpp"

namespace mdc {
namespace {

constexpr int kThreads = 256;  // threads per workgroup of the narrow tiles and short transforms

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
  const float2 id = (DIR < 0) ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);  // DIR * i * d
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, id);
  a3 = csub(t1, id);
}

// y = DFT_8(v) with sign DIR, in place: two DFT_4 of the even and odd points and one
// radix-2 combination with w8^k = exp(DIR 2 pi i k / 8).
template <int DIR>
__device__ __forceinline__ void bfly8(float2 (&v)[8]) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  bfly4<DIR>(e0, e1, e2, e3);
  bfly4<DIR>(o0, o1, o2, o3);
  constexpr float h = 0.70710678118654752f;  // 1 / sqrt(2)
  // w8^1 o1, w8^2 o2 = DIR i o2, w8^3 o3
  const float2 t1 = (DIR < 0) ? make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x))
                              : make_float2(h * (o1.x - o1.y), h * (o1.y + o1.x));
  const float2 t2 = (DIR < 0) ? make_float2(o2.y, -o2.x) : make_float2(-o2.y, o2.x);
  const float2 t3 = (DIR < 0) ? make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y))
                              : make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

// One radix-R Stockham pass (R = 2, 4 or 8) of the CB columns in lds[M][CB], from
// sub-transforms of size Ns to size R Ns.  tws: twiddle table exp(-2 pi i k / (2M)).
template <int M, int CB, int DIR, int R, int NTH>
__device__ __forceinline__ void stockham_pass(float2* lds, const float2* tws, int tid, int Ns) {
  constexpr int NB = (M / R) * CB;
  constexpr int BPT = (NB + NTH - 1) / NTH;
  const int tstep = 2 * (M / (R * Ns));  // table stride per unit of r*k
  float2 v[BPT][R];
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int b = tid + i * NTH;
    if (b < NB) {
      const int col = b % CB, j = b / CB;
      const int k = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[(j + r * (M / R)) * CB + col];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tws[r * k * tstep];
          if (DIR > 0) w = cconj(w);
          v[i][r] = cmul(v[i][r], w);
        }
      }
      if constexpr (R == 8) {
        bfly8<DIR>(v[i]);
      } else if constexpr (R == 4) {
        bfly4<DIR>(v[i][0], v[i][1], v[i][2], v[i][3]);
      } else {
        const float2 a = v[i][0];
        v[i][0] = cadd(a, v[i][1]);
        v[i][1] = csub(a, v[i][1]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int b = tid + i * NTH;
    if (b < NB) {
      const int col = b % CB, j = b / CB;
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(base + r * Ns) * CB + col] = v[i][r];
    }
  }
  __syncthreads();
}

// Complete M-point Stockham FFT (unnormalised) of the CB columns in lds[M][CB]: radix-8
// passes, preceded by one radix-2 or radix-4 pass when log2(M) is not a multiple of 3
// (M = 512: three passes through LDS instead of five radix-4/2 ones).
template <int M, int CB, int DIR, int NTH>
__device__ __forceinline__ void fft_lds(float2* lds, const float2* tws, int tid) {
  constexpr int LOG = log2c<M>();
  int Ns = 1;
  if constexpr (LOG % 3 == 1) {
    stockham_pass<M, CB, DIR, 2, NTH>(lds, tws, tid, Ns);
    Ns = 2;
  } else if constexpr (LOG % 3 == 2) {
    stockham_pass<M, CB, DIR, 4, NTH>(lds, tws, tid, Ns);
    Ns = 4;
  }
  for (; Ns < M; Ns *= 8) stockham_pass<M, CB, DIR, 8, NTH>(lds, tws, tid, Ns);
}

// The 2M-entry twiddle table copied to LDS in two halves: load() issues this thread's entries
// (clamped addresses, unconditional) before the tile's own loads, store() writes them to LDS once
// the tile's loads are in flight, so the table's round trip overlaps the tile's.
template <int M, int NTH>
struct TwiddleStage {
  static constexpr int N = (2 * M + NTH - 1) / NTH;
  float2 t[N];
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int tid) {
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = tw[min(tid + i * NTH, 2 * M - 1)];
  }
  __device__ __forceinline__ void store(float2* tws, int tid) const {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (tid + i * NTH < 2 * M) tws[tid + i * NTH] = t[i];
  }
};

// Workgroup number with neighbouring trace groups on the same XCD (hardware deals
// workgroups round-robin over the 8 XCDs): two neighbours share 128-byte lines of
// every time row, which one L2 then fetches and writes back once.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int q8 = nb >> 3, rem = nb & 7, xcd = b & 7;
  return xcd * q8 + min(xcd, rem) + (b >> 3);
}

// Element (t, q) of a time-domain array of Q traces: row-major [nt][Q], or tiled (solver
// vectors): tiles of CB consecutive traces, each tile [nt][CB] contiguous.
template <int CB, int NT>
__device__ __forceinline__ size_t time_index(int t, int q, int Q, int tiled) {
  return tiled ? (size_t)(q / CB) * (NT * CB) + (size_t)t * CB + (q % CB) : (size_t)t * Q + q;
}


// ----------------------------------------------------------------- forward ---
// VEC: Q % 4 == 0 and x 16-byte aligned (four traces per 16-byte load);
// CONTIG: the bins of a trace pair (q, q+1), q even, are adjacent and 16-byte
// aligned in the spectrum (one segment with Q even, or nv, ldc and c0 all even)
// and go out as one 16-byte store.
template <int M, int CB, bool VEC, bool CONTIG, int NTH>
__global__ __launch_bounds__(NTH) void rfft_trunc_kernel(
    const float* __restrict__ x, const int* __restrict__ onset, int conj, const float2* __restrict__ tw,
    int nfmax, int n, int nv, int ldc, int c0, float scale, float2* __restrict__ spec,
    const double* __restrict__ dscale, int tiled) {
  extern __shared__ __attribute__((aligned(16))) float2 sh[];
  float2* lds = sh;            // [M][CB]
  float2* tws = sh + M * CB;   // [2M]
  constexpr int NT = 2 * M;
  const int Q = n * nv;
  const int tid = threadIdx.x;
  const int q0 = xcd_block() * CB;
  TwiddleStage<M, NTH> twl;
  twl.load(tw, tid);
  const float ds = dscale != nullptr ? (float)*dscale : 1.0f;

  if constexpr (VEC) {
    constexpr int CG = CB / 4;                 // 4-trace groups per row
    constexpr int TASKS = M * CG;              // (m, group) pairs
    constexpr int TPT = (TASKS + NTH - 1) / NTH;
    float4 ra[TPT], rb[TPT];
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int task = tid + i * NTH;
      const int m = task / CG, g = task - (task / CG) * CG;
      const int q = q0 + 4 * g;
      ra[i] = rb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (task < TASKS && q < Q) {  // Q % 4 == 0: the whole group is in range
        ra[i] = *reinterpret_cast<const float4*>(x + time_index<CB, NT>(2 * m, q, Q, tiled));
        rb[i] = *reinterpret_cast<const float4*>(x + time_index<CB, NT>(2 * m + 1, q, Q, tiled));
      }
    }
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int task = tid + i * NTH;
      if (task >= TASKS) continue;
      const int m = task / CG, g = task - (task / CG) * CG;
      const int q = q0 + 4 * g;
      float a[4] = {ra[i].x * ds, ra[i].y * ds, ra[i].z * ds, ra[i].w * ds};
      float b[4] = {rb[i].x * ds, rb[i].y * ds, rb[i].z * ds, rb[i].w * ds};
      if (onset != nullptr && q < Q) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int on = onset[q + h];
          if (!in_window(2 * m, NT, on)) a[h] = 0.f;
          if (!in_window(2 * m + 1, NT, on)) b[h] = 0.f;
        }
      }
      float4* dst = reinterpret_cast<float4*>(&lds[m * CB + 4 * g]);
      dst[0] = make_float4(a[0], b[0], a[1], b[1]);
      dst[1] = make_float4(a[2], b[2], a[3], b[3]);
    }
  } else {
    const int col = tid % CB;
    const int q = q0 + col;
    const bool qok = q < Q;
    const int on = (onset != nullptr && qok) ? onset[q] : INT_MAX;
    constexpr int ROWS = NTH / CB;
    constexpr int TPT = (M + ROWS - 1) / ROWS;
    float ra[TPT], rb[TPT];
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int m = tid / CB + i * ROWS;
      ra[i] = rb[i] = 0.f;
      if (m < M && qok) {
        ra[i] = x[time_index<CB, NT>(2 * m, q, Q, tiled)];
        rb[i] = x[time_index<CB, NT>(2 * m + 1, q, Q, tiled)];
      }
    }
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int m = tid / CB + i * ROWS;
      if (m >= M) continue;
      float a = ra[i] * ds, b = rb[i] * ds;
      if (!in_window(2 * m, NT, on)) a = 0.f;
      if (!in_window(2 * m + 1, NT, on)) b = 0.f;
      lds[m * CB + col] = make_float2(a, b);
    }
  }
  twl.store(tws, tid);
  __syncthreads();
  fft_lds<M, CB, -1, NTH>(lds, tws, tid);

  // split step: X_k = E_k + exp(-2 pi i k / nt) O_k for k < nfmax, two traces per task
  constexpr int CP = CB / 2;
  for (int task = tid; task < nfmax * CP; task += NTH) {
    const int k = task / CP, p = task - (task / CP) * CP;
    const float2 w = tws[k];
    float2 X[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = 2 * p + h;
      const float2 zk = lds[(k & (M - 1)) * CB + col];
      const float2 zc = cconj(lds[((M - k) & (M - 1)) * CB + col]);
      const float2 e = cscale(cadd(zk, zc), 0.5f);
      const float2 d = csub(zk, zc);
      const float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // d / (2i)
      X[h] = cscale(cadd(e, cmul(w, o)), scale);
      if (conj) X[h] = cconj(X[h]);
    }
    const int q = q0 + 2 * p;
    if (CONTIG) {
      // traces q, q+1 (q even) are adjacent spectral columns (see CONTIG above)
      if (q + 1 < Q) {
        const int r = q / nv, v = q - r * nv;
        *reinterpret_cast<float4*>(spec + ((size_t)k * n + r) * ldc + c0 + v) =
            make_float4(X[0].x, X[0].y, X[1].x, X[1].y);
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int qq = q + h;
        if (qq < Q) {
          const int r = qq / nv, v = qq - (qq / nv) * nv;
          spec[((size_t)k * n + r) * ldc + c0 + v] = X[h];
        }
      }
    }
  }
}

// ----------------------------------------------------------------- inverse ---
template <int M, int CB, bool VEC, bool CONTIG, int NTH>
__global__ __launch_bounds__(NTH) void irfft_pad_kernel(
    const float2* __restrict__ spec, int ldc, int c0, int conj, const float2* __restrict__ tw, int nfmax,
    int n, int nv, float scale, float* out, const float* ident,
    const int* __restrict__ onset, float sign, float iscale0, const double* __restrict__ ident_dscale,
    const double* __restrict__ acc_c1, const double* __restrict__ acc_c2, float acc_sgn, double* __restrict__ part,
    int tiled) {
  extern __shared__ __attribute__((aligned(16))) float2 sh[];
  __shared__ double red[NTH / 64];
  float2* lds = sh;
  float2* tws = sh + M * CB;
  constexpr int NT = 2 * M;
  const int Q = n * nv;
  const int tid = threadIdx.x;
  const int q0 = xcd_block() * CB;
  TwiddleStage<M, NTH> twl;
  twl.load(tw, tid);
  const float iscale = ident_dscale != nullptr ? iscale0 * (float)*ident_dscale : iscale0;
  // fused recurrence: out += coef * out_old, coefficient formed in FP64 as the separate pass does
  const bool acc = acc_c1 != nullptr;
  const float coef = acc ? (float)((double)acc_sgn * *acc_c1 * (acc_c2 != nullptr ? *acc_c2 : 1.0)) : 0.f;
  double ssq = 0.0;

  // Bins k and M - k of the trace pair (q, q + 1); every load of the tile is issued before
  // any is consumed, from clamped addresses (unpredicated), invalid bins zeroed afterwards.
  auto bin2 = [&](int k, int q, float2& X0, float2& X1) {
    const int kc = min(k, nfmax - 1);
    if (CONTIG) {  // pair of adjacent, 16-byte aligned columns (see the forward split step)
      const int qc = min(q, Q - 2);
      const int r = qc / nv, v = qc - r * nv;
      const float4 w = *reinterpret_cast<const float4*>(spec + ((size_t)kc * n + r) * ldc + c0 + v);
      const bool ok = k < nfmax && q + 1 < Q;
      X0 = ok ? make_float2(w.x, w.y) : make_float2(0.f, 0.f);
      X1 = ok ? make_float2(w.z, w.w) : make_float2(0.f, 0.f);
    } else {
      const int qa = min(q, Q - 1), qb = min(q + 1, Q - 1);
      const float2 a = spec[((size_t)kc * n + qa / nv) * ldc + c0 + qa % nv];
      const float2 b = spec[((size_t)kc * n + qb / nv) * ldc + c0 + qb % nv];
      X0 = (k < nfmax && q < Q) ? a : make_float2(0.f, 0.f);
      X1 = (k < nfmax && q + 1 < Q) ? b : make_float2(0.f, 0.f);
    }
  };
  // Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) exp(+2 pi i k / nt), two traces per task
  constexpr int CP = CB / 2;
  constexpr int NMAIN = (M / 2) * CP;  // k = 0 .. M/2 - 1; the middle bin k = M/2 follows
  constexpr int ITER = (NMAIN + NTH - 1) / NTH;
  float2 ga[ITER][2], gb[ITER][2], gm[2];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int task = min(tid + it * NTH, NMAIN - 1);
    const int k = task / CP, p = task - (task / CP) * CP;
    bin2(k, q0 + 2 * p, ga[it][0], ga[it][1]);
    bin2(M - k, q0 + 2 * p, gb[it][0], gb[it][1]);
  }
  // the middle bin M/2 is its own mirror: every thread loads it for trace pair min(tid, CP - 1)
  bin2(M / 2, q0 + 2 * min(tid, CP - 1), gm[0], gm[1]);
  twl.store(tws, tid);
  __syncthreads();
  auto split = [&](int k, int p, float2 (&a)[2], float2 (&b)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (conj) { a[h].y = -a[h].y; b[h].y = -b[h].y; }
      if (k == 0) { a[h].y = 0.f; b[h].y = 0.f; }  // only Re of DC (bin 0) and Nyquist (bin M)
    }
    const float2 wk = cconj(tws[k]), wmk = cconj(tws[M - k]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = 2 * p + h;
      {
        const float2 e = cadd(a[h], cconj(b[h]));
        const float2 o = cmul(csub(a[h], cconj(b[h])), wk);
        lds[k * CB + col] = make_float2(e.x - o.y, e.y + o.x);
      }
      if (k > 0 && k < M / 2) {
        const float2 e = cadd(b[h], cconj(a[h]));
        const float2 o = cmul(csub(b[h], cconj(a[h])), wmk);
        lds[(M - k) * CB + col] = make_float2(e.x - o.y, e.y + o.x);
      }
    }
  };
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int task = tid + it * NTH;
    if (task >= NMAIN) continue;
    const int k = task / CP, p = task - (task / CP) * CP;
    float2 a[2] = {ga[it][0], ga[it][1]}, b[2] = {gb[it][0], gb[it][1]};
    split(k, p, a, b);
  }
  if (tid < CP) {
    float2 a[2] = {gm[0], gm[1]}, b[2] = {gm[0], gm[1]};
    split(M / 2, tid, a, b);
  }
  __syncthreads();
  fft_lds<M, CB, +1, NTH>(lds, tws, tid);

  // y[2m] = Re z[m] / sqrt(nt), y[2m+1] = Im z[m] / sqrt(nt); epilogue out = ident + sign * Theta * y
  if constexpr (VEC) {
    constexpr int CG = CB / 4;
    constexpr int TASKS = M * CG;
    for (int task = tid; task < TASKS; task += NTH) {
      const int m = task / CG, g = task - (task / CG) * CG;
      const int q = q0 + 4 * g;
      if (q >= Q) continue;
      const float4 z01 = *reinterpret_cast<const float4*>(&lds[m * CB + 4 * g]);
      const float4 z23 = *reinterpret_cast<const float4*>(&lds[m * CB + 4 * g + 2]);
      float e0[4] = {z01.x, z01.z, z23.x, z23.z};
      float e1[4] = {z01.y, z01.w, z23.y, z23.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        e0[h] *= scale * sign;
        e1[h] *= scale * sign;
        if (onset != nullptr) {
          const int on = onset[q + h];
          if (!in_window(2 * m, NT, on)) e0[h] = 0.f;
          if (!in_window(2 * m + 1, NT, on)) e1[h] = 0.f;
        }
      }
      const size_t i0 = time_index<CB, NT>(2 * m, q, Q, tiled), i1 = time_index<CB, NT>(2 * m + 1, q, Q, tiled);
      float4 o0 = make_float4(e0[0], e0[1], e0[2], e0[3]);
      float4 o1 = make_float4(e1[0], e1[1], e1[2], e1[3]);
      if (ident != nullptr) {
        const float4 d0 = *reinterpret_cast<const float4*>(ident + i0);
        const float4 d1 = *reinterpret_cast<const float4*>(ident + i1);
        o0 = make_float4(o0.x + iscale * d0.x, o0.y + iscale * d0.y, o0.z + iscale * d0.z, o0.w + iscale * d0.w);
        o1 = make_float4(o1.x + iscale * d1.x, o1.y + iscale * d1.y, o1.z + iscale * d1.z, o1.w + iscale * d1.w);
      }
      if (acc) {
        const float4 p0 = *reinterpret_cast<const float4*>(out + i0);
        const float4 p1 = *reinterpret_cast<const float4*>(out + i1);
        o0 = make_float4(o0.x + coef * p0.x, o0.y + coef * p0.y, o0.z + coef * p0.z, o0.w + coef * p0.w);
        o1 = make_float4(o1.x + coef * p1.x, o1.y + coef * p1.y, o1.z + coef * p1.z, o1.w + coef * p1.w);
      }
      *reinterpret_cast<float4*>(out + i0) = o0;
      *reinterpret_cast<float4*>(out + i1) = o1;
      if (part != nullptr)
        ssq += (double)o0.x * o0.x + (double)o0.y * o0.y + (double)o0.z * o0.z + (double)o0.w * o0.w +
               (double)o1.x * o1.x + (double)o1.y * o1.y + (double)o1.z * o1.z + (double)o1.w * o1.w;
    }
  } else {
    const int col = tid % CB;
    const int q = q0 + col;
    if (q < Q) {
      const int on = (onset != nullptr) ? onset[q] : INT_MAX;
      for (int m = tid / CB; m < M; m += NTH / CB) {
        const float2 z = lds[m * CB + col];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int t = 2 * m + h;
          float val = (h == 0 ? z.x : z.y) * scale * sign;
          if (!in_window(t, NT, on)) val = 0.f;
          const size_t idx = time_index<CB, NT>(t, q, Q, tiled);
          if (ident != nullptr) val += iscale * ident[idx];
          if (acc) val += coef * out[idx];
          out[idx] = val;
          if (part != nullptr) ssq += (double)val * val;
        }
      }
    }
  }
  // per-workgroup partial sum of out^2 (fixed reduction order: deterministic)
  if (part != nullptr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ssq += __shfl_xor(ssq, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = ssq;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < NTH / 64; ++w) t += red[w];
      part[blockIdx.x] = t;
    }
  }
}

// Wide width: 16 traces (64-byte pieces of every time row), or 8 where a 16-trace tile
// would leave one workgroup per CU (M >= 1024).
template <int M, bool INV>
constexpr int wide_cb() { return M >= 1024 ? 8 : 16; }

// Threads per workgroup: one wave per trace for the wide tiles of the long transforms (more
// waves to keep loads in flight and the LDS passes short: at M = 512 the forward runs 14-26%
// and the inverse 30% faster than with four waves per tile), else four waves.
template <int M, int CB>
constexpr int fft_nth() { return (M >= 256 && CB >= 8) ? 64 * CB : kThreads; }

template <int M, bool INV>
int pick_cb(int Q) {
  constexpr int maxcb = wide_cb<M, INV>();
  if (Q >= 256 * 2 * maxcb) return maxcb;
  return 4;
}

template <int M, int CB, bool VEC, bool CONTIG, int NTH>
mdc_status rfft_run(const float2* tw, int nfmax, int n, int nv, int ldc, const FftSeg& s, float2* spec,
                    hipStream_t st) {
  const int Q = n * nv;
  const size_t lds = ((size_t)M * CB + 2 * M) * sizeof(float2);
  const float scale = (float)(1.0 / std::sqrt((double)(2 * M)));
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)rfft_trunc_kernel<M, CB, VEC, CONTIG, NTH>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
      return fail(MDC_EDEVICE, "rfft_trunc_kernel: %zu bytes of LDS refused: %s", lds, hipGetErrorString(e));
    attr = true;
  }
  hipLaunchKernelGGL((rfft_trunc_kernel<M, CB, VEC, CONTIG, NTH>), dim3((Q + CB - 1) / CB), dim3(NTH), lds, st, s.in,
                     s.onset, s.conj, tw, nfmax, n, nv, ldc, s.c0, scale, spec, s.dscale, s.tiled);
  return check_launch("rfft_trunc_kernel");
}

template <int M, int CB, int NTH>
mdc_status rfft_cb(const float2* tw, int nfmax, int n, int nv, int ldc, const FftSeg& s, float2* spec,
                   hipStream_t st) {
  const int Q = n * nv;
  const bool vec = (Q % 4 == 0) && aligned(s.in, 16);
  // pairs contiguous: one segment (ldc == nv, c0 == 0, Q even), or nv, ldc, c0 all even
  const bool contig = aligned(spec, 16) && ((ldc == nv && s.c0 == 0 && Q % 2 == 0) ||
                                            (nv % 2 == 0 && ldc % 2 == 0 && s.c0 % 2 == 0));
  if (vec && contig) return rfft_run<M, CB, true, true, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
  if (vec) return rfft_run<M, CB, true, false, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
  if (contig) return rfft_run<M, CB, false, true, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
  return rfft_run<M, CB, false, false, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
}

template <int M>
mdc_status rfft_one(const float2* tw, int nfmax, int n, int nv, int ldc, const FftSeg& s, float2* spec,
                    hipStream_t st) {
  constexpr int WIDE = wide_cb<M, false>();
  if (pick_cb<M, false>(n * nv) == WIDE) return rfft_cb<M, WIDE, fft_nth<M, WIDE>()>(tw, nfmax, n, nv, ldc, s, spec, st);
  return rfft_cb<M, 4, kThreads>(tw, nfmax, n, nv, ldc, s, spec, st);
}

template <int M, int CB, bool VEC, bool CONTIG, int NTH>
mdc_status irfft_run(const float2* tw, int nfmax, int n, int nv, int ldc, const IfftSeg& s, const float2* spec,
                     hipStream_t st) {
  const int Q = n * nv;
  const size_t lds = ((size_t)M * CB + 2 * M) * sizeof(float2);
  const float scale = (float)(1.0 / std::sqrt((double)(2 * M)));
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)irfft_pad_kernel<M, CB, VEC, CONTIG, NTH>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
      return fail(MDC_EDEVICE, "irfft_pad_kernel: %zu bytes of LDS refused: %s", lds, hipGetErrorString(e));
    attr = true;
  }
  hipLaunchKernelGGL((irfft_pad_kernel<M, CB, VEC, CONTIG, NTH>), dim3((Q + CB - 1) / CB), dim3(NTH), lds, st, spec,
                     ldc, s.c0, s.conj, tw, nfmax, n, nv, scale, s.out, s.ident, s.onset, s.sign, s.ident_scale,
                     s.ident_dscale, s.acc_c1, s.acc_c2, s.acc_sgn, s.part, s.tiled);
  return check_launch("irfft_pad_kernel");
}

template <int M, int CB, int NTH>
mdc_status irfft_cb(const float2* tw, int nfmax, int n, int nv, int ldc, const IfftSeg& s, const float2* spec,
                    hipStream_t st) {
  const int Q = n * nv;
  const bool vec = (Q % 4 == 0) && aligned(s.out, 16) && (s.ident == nullptr || aligned(s.ident, 16));
  // pairs contiguous: one segment (ldc == nv, c0 == 0, Q even), or nv, ldc, c0 all even
  const bool contig = aligned(spec, 16) && ((ldc == nv && s.c0 == 0 && Q % 2 == 0) ||
                                            (nv % 2 == 0 && ldc % 2 == 0 && s.c0 % 2 == 0));
  if (vec && contig) return irfft_run<M, CB, true, true, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
  if (vec) return irfft_run<M, CB, true, false, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
  if (contig) return irfft_run<M, CB, false, true, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
  return irfft_run<M, CB, false, false, NTH>(tw, nfmax, n, nv, ldc, s, spec, st);
}

template <int M>
int irfft_blocks_m(int Q) {
  const int cb = pick_cb<M, true>(Q);
  return (Q + cb - 1) / cb;
}

template <int M>
mdc_status irfft_one(const float2* tw, int nfmax, int n, int nv, int ldc, const IfftSeg& s, const float2* spec,
                     hipStream_t st) {
  constexpr int WIDE = wide_cb<M, true>();
  if (pick_cb<M, true>(n * nv) == WIDE) return irfft_cb<M, WIDE, fft_nth<M, WIDE>()>(tw, nfmax, n, nv, ldc, s, spec, st);
  return irfft_cb<M, 4, kThreads>(tw, nfmax, n, nv, ldc, s, spec, st);
}

}  // namespace

int irfft_blocks(int nt, int n, int nv) {
  const int Q = n * nv;
  switch (nt) {
    case 16: return irfft_blocks_m<8>(Q);
    case 32: return irfft_blocks_m<16>(Q);
    case 64: return irfft_blocks_m<32>(Q);
    case 128: return irfft_blocks_m<64>(Q);
    case 256: return irfft_blocks_m<128>(Q);
    case 512: return irfft_blocks_m<256>(Q);
    case 1024: return irfft_blocks_m<512>(Q);
    case 2048: return irfft_blocks_m<1024>(Q);
    default: return 0;
  }
}

int fft_tile(int nt, int Q) {
  switch (nt) {
    case 16: return pick_cb<8, false>(Q);
    case 32: return pick_cb<16, false>(Q);
    case 64: return pick_cb<32, false>(Q);
    case 128: return pick_cb<64, false>(Q);
    case 256: return pick_cb<128, false>(Q);
    case 512: return pick_cb<256, false>(Q);
    case 1024: return pick_cb<512, false>(Q);
    case 2048: return pick_cb<1024, false>(Q);
    default: return 4;  // not a supported length (the transforms refuse it)
  }
}

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
