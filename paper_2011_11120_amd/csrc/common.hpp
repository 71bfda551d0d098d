// Shared device/host helpers of the HIP library (not used by the oracle).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/mdc.h"

// What a captured LSQR iteration graph depends on (pointers are baked into its nodes).
// The product family of every apply is fixed at capture time, so the key also holds the
// tuning-table generation and the forced-family switch.
struct LsqrGraphKey {
  int kind, nv, fused, tiled, tune_gen, forced;
  const void *onset, *work, *x, *hist, *b;
  bool operator==(const LsqrGraphKey& o) const {
    return kind == o.kind && nv == o.nv && fused == o.fused && tiled == o.tiled && tune_gen == o.tune_gen &&
           forced == o.forced &&
           onset == o.onset && work == o.work && x == o.x && hist == o.hist && b == o.b;
  }
};

// Operator state (host side; device buffers are caller-owned).
struct mdc_op {
  mdc_desc d;
  char* resident;
  char* work;
  float2* tw;        // [nt] exp(-2 pi i k / nt)
  float* fscale;     // [nfmax] per-frequency storage scale (FP16S), else unused
  void* kstore;      // stored kernel
  float2* specR;     // [nfmax][nr][max_cols]
  float2* specS;     // [nfmax][ns][max_cols]
  unsigned int* bsplit;  // split spectra of the 16-bit matrix-core product (16-bit formats), else nullptr
  bool kernel_ready;
  std::vector<float2> tw_host;
  // profiling
  bool prof;
  struct Ev { int stage; hipEvent_t a, b; };
  std::vector<Ev> evs;
  std::vector<hipEvent_t> pool;
  // product family per column bucket and direction (filled by mdc_autotune)
  std::vector<int> tune_ncols;
  std::vector<int> tune_family[2];
  int tune_gen = 0;  // bumped whenever the table changes
  // LSQR iteration graph (captured on cap_stream, replayed on the caller's stream)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t lsqr_exec = nullptr;
  LsqrGraphKey lsqr_key{};
};

namespace mdc {

// ------------------------------------------------------------ status -------
void set_error(const char* fmt, ...);
mdc_status fail(mdc_status st, const char* fmt, ...);
mdc_status check_launch(const char* what);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// ----------------------------------------------------- complex helpers -----
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ---------------------------------------------------- window (Theta) -------
// Theta[t][s][v] = 1 when |lag(t)| < onset, lag(t) = t (t < nt/2) else t - nt.
// A negative onset -h selects the one-sided (causal) window 0 <= lag(t) < h, the
// time-domain preconditioner that confines a solution to non-negative times.
__device__ __forceinline__ bool in_window(int t, int nt, int onset) {
  const bool causal = 2 * t < nt;
  if (onset < 0) return causal && t < -onset;
  return (causal ? t : nt - t) < onset;
}

// --------------------------------------------------------- launchers -------
// Spectra are complex64 [nfmax][n][ldc]; a segment is a run of nv columns
// starting at column c0, fed from/to a time-domain array [nt][n][nv].
struct FftSeg {
  const float* in;     // time-domain input [nt][n][nv]
  const int* onset;    // optional pre-window [n][nv] (adjoint Marchenko), or nullptr
  int conj;            // conjugate the spectrum
  int c0;              // first spectral column
  const double* dscale = nullptr;  // optional device scalar multiplying the input as it is read
  int tiled = 0;       // input in the tiled layout (fft_tile), else [nt][n][nv]
};
struct IfftSeg {
  float* out;          // time-domain output [nt][n][nv]
  const float* ident;  // optional identity term: out = ident_scale * ident + sign * Theta * y
  const int* onset;    // optional post-window [n][nv], or nullptr
  int conj;            // conjugate the spectrum before the inverse
  int c0;              // first spectral column
  float sign;          // multiplier of the transformed term
  float ident_scale = 1.0f;
  const double* ident_dscale = nullptr;  // optional device scalar multiplying ident as it is read
  // Optional fused recurrence (LSQR / CGLS): with acc_c1 set, out = (the above) + acc_sgn *
  // (*acc_c1) * (*acc_c2 or 1) * out_old, read and written at the same index; with part set,
  // each workgroup writes the FP64 sum of its out^2 to part[workgroup] (irfft_blocks slots).
  const double* acc_c1 = nullptr;
  const double* acc_c2 = nullptr;
  float acc_sgn = 0.f;
  double* part = nullptr;
  int tiled = 0;       // out, ident in the tiled layout (fft_tile), else [nt][n][nv]
};

// Fused recurrence handed to an apply: out = op(in) + sgn * (*c1) * (*c2 or 1) * out (c1 may be
// null: no update), with per-workgroup partial sums of out^2 at part (one run of slots per
// inverse-transform segment, in segment order; irfft_blocks slots each).
struct Recur {
  const double* c1;
  const double* c2;
  float sgn;
  double* part;
};

// Attach a fused recurrence to an inverse-transform segment; slot is its first partial-sum slot.
inline void attach_recur(IfftSeg& seg, const Recur* rec, int slot) {
  if (!rec) return;
  seg.acc_c1 = rec->c1;
  seg.acc_c2 = rec->c2;
  seg.acc_sgn = rec->sgn;
  seg.part = rec->part ? rec->part + slot : nullptr;
}

// FFT tables in the resident buffer: tw[k] = exp(-2 pi i k / nt), k < nt.
mdc_status rfft_launch(const float2* tw, int nt, int nfmax, int n, int nv, int ldc, const FftSeg& seg,
                       float2* spec, hipStream_t st);
mdc_status irfft_launch(const float2* tw, int nt, int nfmax, int n, int nv, int ldc, const IfftSeg& seg,
                        const float2* spec, hipStream_t st);
// Workgroups of one inverse launch over n * nv traces (slots of its partial sums).
int irfft_blocks(int nt, int n, int nv);
// Tiled time layout of the solvers' vectors: the Q traces in tiles of T = fft_tile(nt, Q)
// consecutive traces (the transforms' workgroup width), tile j holding [nt][T] floats at
// j * nt * T; the traces of the last tile past Q are padding and hold zeros.  A vector block
// then takes tiled_len(nt, Q) floats, and every transform reads or writes whole tiles.
int fft_tile(int nt, int Q);
inline size_t tiled_len(int nt, int Q) {
  const int T = fft_tile(nt, Q);
  return (size_t)nt * ((size_t)(Q + T - 1) / T) * T;
}
// Between `blocks` consecutive blocks of [nt][Q] floats and their tiled form (tiled_len each):
// to_tiles writes whole tiles (zero padding traces), from_tiles the [nt][Q] blocks.
void launch_to_tiles(float* dst, const float* src, int nt, int Q, int blocks, hipStream_t st);
void launch_from_tiles(float* dst, const float* src, int nt, int Q, int blocks, hipStream_t st);

// Kernel product over all frequencies: forward Y_f = K_f X_f (ns x nr times nr x ncols),
// adjoint X_f = K_f^H Y_f.  Spectra [nfmax][n][ncols].  The kernel family comes from the
// op's tuning table (mdc_autotune), else from the default crossover.
mdc_status product_launch(const mdc_op* op, int adjoint, const float2* in, float2* out, int ncols, hipStream_t st);
// Product family forced by the environment (MDC_PRODUCT = gemv | gemm | gemm32), or -1.
int forced_family(const mdc_op* op);

// Operator on a sub-grid of a square operator (rows and columns idx, nsub traces): its kernel is
// gathered from the parent's resident kernel into `resident` (sub_op_resident_bytes) on `st`, the
// tables and tuning are copied, and the parent's workspace is shared, so applies of the two must
// not overlap.  Released with mdc_destroy.
size_t sub_op_resident_bytes(const mdc_op* parent, int nsub);
mdc_status sub_op_create(const mdc_op* parent, const int* idx, int nsub, void* resident, hipStream_t st,
                         mdc_op** out);

// Device state of one LSQR solve (all pointers are device memory).
struct LsqrState {
  void* sc;                    // FP64 scalars + reduction partials (lsqr_scalars_bytes())
  float *u, *t, *v, *w, *t2;   // data-size u, t; model-size v, w, t2 (t, t2 unused when fused)
  float* x;                    // solution (model size)
  double* hist;                // phibar history (niter + 1) or nullptr
  size_t model, data;          // element counts
  double* rpart = nullptr;     // partial sums of the fused recurrences (or nullptr: separate passes)
  int nparts_fwd = 0, nparts_adj = 0;  // slots the forward / adjoint apply fills
};
size_t lsqr_scalars_bytes();
// Device scalars 1/beta and 1/alpha: u and v are kept unnormalised and every consumer scales
// them as it reads them (no separate normalisation pass).
const double* lsqr_uinv(const LsqrState& s);
const double* lsqr_vinv(const LsqrState& s);
void lsqr_after_b(const LsqrState& s, hipStream_t st);
void lsqr_after_init_adj(const LsqrState& s, hipStream_t st);
void lsqr_after_fwd(const LsqrState& s, hipStream_t st);
void lsqr_after_adj(const LsqrState& s, hipStream_t st);
// Recurrences fused into the applies' inverse transforms; these finish the norms only.
Recur lsqr_recur_init(const LsqrState& s);
Recur lsqr_recur_fwd(const LsqrState& s);
Recur lsqr_recur_adj(const LsqrState& s);
void lsqr_after_init_adj_fused(const LsqrState& s, hipStream_t st);
void lsqr_after_fwd_fused(const LsqrState& s, hipStream_t st);
void lsqr_after_adj_fused(const LsqrState& s, hipStream_t st);

}  // namespace mdc
