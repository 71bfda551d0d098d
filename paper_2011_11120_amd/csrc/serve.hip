// Serving loop for Marchenko redatuming solves (Eq.5) against one resident kernel.
//
// The paper groups focusing points into independent inversions (Discussion:
// embarrassingly parallel groups of points, each solved as one problem, and
// many points per kernel pass because matrix-matrix products beat repeated
// matrix-vector ones).  Here requests of uneven size (points, iterations,
// decimation) arrive while others run; every step is one pass over the kernel
// that serves the columns of every admitted request:
//
//   * the step direction alternates forward / adjoint; a request advances one
//     operator application per step (data Theta R fd, then A^H u, then
//     A v / A^H u per LSQR iteration), so all admitted requests share the pass;
//   * each request's traces are transformed into its own column range of one
//     spectral array, one product (GEMV or MFMA GEMM by total width) runs over
//     all columns, and each request's inverse transform applies its own window,
//     decimation scale and keep mask;
//   * every request keeps its own FP64 LSQR scalars and Krylov vectors on the
//     device, in a slot of the caller-provided arena; admission is FIFO by
//     arena footprint and column budget; results of a request depend only on
//     its own columns.
//
// A request decimated by d solves the problem of its lattice (the Sub2 / Sub4
// geometries of Table 1, areal element d dx^2) in one of two ways:
//   * on a sub-grid level prepared at creation: the lattice's traces only, with
//     the kernel rows and columns of the lattice gathered once into the arena, so
//     the request's product, transforms and vectors all shrink by d (d^2 fewer
//     kernel multiply-adds per column); its solution is scattered back onto the
//     full grid (zeros elsewhere) when it finishes;
//   * on the full grid: traces outside the lattice have zero inputs, zero window
//     and a zero keep mask on adjoint outputs, which equals the decimated
//     problem but pays the full-grid product.
// Requests of different levels share a step; each level runs its own product.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "common.hpp"

namespace mdc {
namespace {

constexpr int kMaxPoints = 64;
constexpr int kThreads = 256;

struct PointArgs {
  double vx[kMaxPoints], vy[kMaxPoints], vz[kMaxPoints];
};

__device__ __forceinline__ bool lattice_keep(int r, int nx, int d) {
  const int ix = r / nx, iy = r - (r / nx) * nx;
  if (d == 2) return ((ix + iy) & 1) == 0;
  if (d == 4) return (((ix - iy) % 4) + 4) % 4 == 0;
  return true;
}

// Trace i of the request's problem is full-grid trace idx[i] (a lattice level) or i (the full
// grid, n = nx^2, traces off the lattice of d masked out); trace q = i nv + v.
// onset[q] = max(rint(td/dt) - eps, 0) on kept traces, 0 elsewhere; keep[q] = nt or 0;
// fd(t, q) = ricker(lag(t) dt + td) on kept traces, 0 elsewhere, written in the tiled layout
// (tiles of T traces, zero padding traces); td = |x_r - x_v| / c (FP64, no contraction, so the
// integer onsets match a host computation exactly).
__global__ __launch_bounds__(kThreads) void request_inputs(int nt, int nx, double dx, double dt, double c, int eps,
                                                           double fp, int d, int n, const int* __restrict__ idx,
                                                           int nv, PointArgs P, int T, int* __restrict__ onset,
                                                           int* __restrict__ keep, float* __restrict__ fd) {
  const size_t Q = (size_t)n * nv, tile = (size_t)nt * T;
  const size_t total = (Q + T - 1) / T * tile;
  for (size_t e = blockIdx.x * (size_t)kThreads + threadIdx.x; e < total; e += (size_t)gridDim.x * kThreads) {
    const size_t j = e / tile, rr = e - j * tile;
    const int t = (int)(rr / T);
    const size_t q = j * T + (rr - (size_t)t * T);
    if (q >= Q) {
      fd[e] = 0.f;
      continue;
    }
    const int i = (int)(q / nv), v = (int)(q - (size_t)i * nv);
    const int r = idx ? idx[i] : i;
    const bool kept = idx ? true : lattice_keep(r, nx, d);
    const double rx = (double)(r / nx) * dx, ry = (double)(r % nx) * dx;
    const double ax = __dadd_rn(rx, -P.vx[v]), ay = __dadd_rn(ry, -P.vy[v]);
    const double h2 = __dadd_rn(__dadd_rn(__dmul_rn(ax, ax), __dmul_rn(ay, ay)), __dmul_rn(P.vz[v], P.vz[v]));
    const double td = __ddiv_rn(sqrt(h2), c);
    if (t == 0) {
      int o = (int)rint(__ddiv_rn(td, dt)) - eps;
      o = o < 0 ? 0 : o;
      onset[q] = kept ? o : 0;
      keep[q] = kept ? nt : 0;
    }
    float val = 0.f;
    if (kept) {
      const double lag = (double)((2 * t < nt) ? t : t - nt) * dt;
      const double a = M_PI * fp * (lag + td);
      const double a2 = a * a;
      val = (float)((1.0 - 2.0 * a2) * exp(-a2));
    }
    fd[e] = val;
  }
}

__global__ void zero_f32(float* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.f;
}

// out[b][t][r][v] = x_b(t, pos[r] nv + v) where the full-grid trace r is on the lattice
// (pos[r] >= 0), 0 elsewhere: a lattice solution (two blocks of blk floats in the tiled layout,
// tiles of T traces) written onto the full grid [2][nt][n][nv].
__global__ __launch_bounds__(kThreads) void scatter_lattice(const float* __restrict__ x, float* __restrict__ out,
                                                            const int* __restrict__ pos, int nt, int n, int nv,
                                                            int T, size_t blk) {
  const size_t total = 2ull * nt * n * nv;
  for (size_t e = blockIdx.x * (size_t)kThreads + threadIdx.x; e < total; e += (size_t)gridDim.x * kThreads) {
    const size_t bt = e / ((size_t)n * nv);  // block * nt + t
    const size_t q = e - bt * (size_t)n * nv;
    const int r = (int)(q / nv), v = (int)(q - (size_t)r * nv);
    const int b = (int)(bt / nt), t = (int)(bt - (size_t)b * nt);
    const int p = pos[r];
    const size_t qs = (size_t)p * nv + v;  // lattice trace
    out[e] = p >= 0 ? x[b * blk + qs / T * ((size_t)nt * T) + (size_t)t * T + qs % T] : 0.f;
  }
}

enum Phase { kQueued, kData, kInitAdj, kIterF, kIterA, kDone, kCanceled };

// A problem size the server solves on: the full grid (the server's op) or a lattice level.
struct Level {
  mdc_op* op = nullptr;     // operator of the level
  int n = 0;                // traces
  int* idx = nullptr;       // device [n]: trace -> full-grid trace (lattice levels only)
  int* pos = nullptr;       // device [nx^2]: full-grid trace -> lattice position or -1
};
constexpr int kLevels = 3;  // full grid, lattice of d = 2, lattice of d = 4

int level_of(int decim) { return decim == 4 ? 2 : (decim == 2 ? 1 : 0); }

struct Request {
  uint64_t id;
  int nv, niter, decim;
  int lv = 0;             // level it is solved on (0: full grid)
  int n = 0;              // traces of its problem
  PointArgs pts;
  float* x_out;
  double* hist;
  size_t slot_off = 0, slot_bytes = 0;
  int* onset = nullptr;
  int* keep = nullptr;
  LsqrState S{};
  Phase phase = kQueued;
  int it = 0;             // completed LSQR iterations
  int c0 = 0;             // first spectral column in the current step
  bool cancel = false;
  bool deferred = false;  // waited for an adjoint step before admission (lockstep phases)
  bool finished = false;  // left the server (done or cancelled); set under the lock
  std::chrono::steady_clock::time_point arrival, finish;
};

// Partial-sum slots of one request's fused recurrences (two inverse segments per apply).
int parts_for(int nt, int n, int nv) { return 2 * irfft_blocks(nt, n, nv); }

// Arena bytes of a request on n traces: onsets, keep mask, scalars, partial sums, and the
// vectors u, v, w (recurrences fused into the applies) and x, all in the transforms' tiled
// layout (x is written onto the caller's output, [2][nt][nx^2][nv], when the request finishes).
size_t slot_bytes_for(int nt, int n, int nv) {
  const size_t vec = 2 * tiled_len(nt, n * nv) * 4;  // two Marchenko blocks
  size_t b = 2 * align_up((size_t)n * nv * 4, 256);
  b += lsqr_scalars_bytes();
  b += align_up((size_t)parts_for(nt, n, nv) * sizeof(double), 256);
  b += 4 * align_up(vec, 256);
  return b;
}

// First-fit allocator over [0, size) with coalescing.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool fits(size_t bytes) const {
    for (const auto& kv : free_)
      if (kv.second >= bytes) return true;
    return false;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

}  // namespace
}  // namespace mdc

using namespace mdc;

struct mdc_server {
  mdc_op* op = nullptr;
  serve_geometry g{};
  char* arena_base = nullptr;
  size_t arena_bytes = 0;
  size_t reserved = 0;                   // arena bytes held by the lattice levels
  Arena arena;
  Level lv[kLevels];
  int device = 0;
  hipStream_t stream = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false;
  uint64_t next_id = 1;
  std::deque<Request*> queue;            // waiting for admission (FIFO)
  std::vector<Request*> active;          // admitted, running
  std::map<uint64_t, Request*> all;      // every request ever submitted
  std::vector<double> latencies;         // completion order
  std::chrono::steady_clock::time_point first_arrival, last_finish;
  bool any_arrival = false;
  int outstanding = 0;
  int max_active = 0;
  long steps = 0;
  bool forward_next = true;
  mdc_status error = MDC_OK;
  // Steps replayed from captured graphs, keyed by direction and the (request, phase) list:
  // within a fixed set of active requests every forward and every adjoint step enqueues the
  // same launches.  A key's first step runs eagerly, its second is captured.
  std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
  std::map<std::vector<uint64_t>, int> seen;
  bool graphs_ok = true;
  std::atomic<long> captured{0}, replayed{0};
  // Lockstep phases: every admitted request applies the operator in the step's direction, and
  // new requests (whose first application is a forward one) are admitted at forward steps only.
  // A request that could have been admitted during an adjoint step waits for that step: the
  // only delay a pass serving both directions at once would remove.
  long deferred = 0;
  double deferred_s = 0.0;
  long request_steps = 0;               // sum over steps of the requests served
};

namespace {

int cols_for(const Request* r) { return r->phase == kData ? r->nv : 2 * r->nv; }

bool wants_forward(const Request* r) { return r->phase == kData || r->phase == kIterF; }

// Enqueue the launches of one level's requests in a step (all in the same direction): their
// transforms into consecutive column ranges of the level's spectra, one product over all of
// them, and their inverse transforms with the LSQR recurrences.  Only launches: the phase
// transitions are applied afterwards by advance().
mdc_status enqueue_level(mdc_server* S, const Level& L, std::vector<Request*>& part, bool fwd, hipStream_t st) {
  mdc_op* op = L.op;
  const mdc_desc& d = op->d;
  const int n = L.n;
  int N = 0;
  for (Request* r : part) {
    r->c0 = N;
    N += cols_for(r);
  }
  float2* spec_in = fwd ? op->specR : op->specS;
  float2* spec_out = fwd ? op->specS : op->specR;
  mdc_status s;
  for (Request* r : part) {
    const size_t half = tiled_len(d.nt, n * r->nv);  // one block of a request vector (tiled layout)
    if (r->phase == kData) {
      FftSeg a{r->S.w, nullptr, 0, r->c0, nullptr, 1};  // fd was generated into w (block 0)
      if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, a, spec_in, st)) != MDC_OK) return s;
    } else if (fwd) {  // R on v1, R* on v0 (stored v times 1/alpha)
      FftSeg a{r->S.v + half, nullptr, 0, r->c0, lsqr_vinv(r->S), 1};
      FftSeg b{r->S.v, nullptr, 1, r->c0 + r->nv, lsqr_vinv(r->S), 1};
      if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, a, spec_in, st)) != MDC_OK) return s;
      if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, b, spec_in, st)) != MDC_OK) return s;
    } else {  // R^H on Theta u0, R*^H on Theta u1 (stored u times 1/beta)
      FftSeg a{r->S.u, r->onset, 0, r->c0, lsqr_uinv(r->S), 1};
      FftSeg b{r->S.u + half, r->onset, 1, r->c0 + r->nv, lsqr_uinv(r->S), 1};
      if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, a, spec_in, st)) != MDC_OK) return s;
      if ((s = rfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, b, spec_in, st)) != MDC_OK) return s;
    }
  }
  if ((s = product_launch(op, fwd ? 0 : 1, spec_in, spec_out, N, st)) != MDC_OK) return s;
  for (Request* r : part) {
    const size_t half = tiled_len(d.nt, n * r->nv);
    const float dsc = (float)r->decim;
    if (r->phase == kData) {  // u0 = d Theta R fd, u1 = 0 ; then beta u = b
      IfftSeg a{r->S.u, nullptr, r->onset, 0, r->c0, dsc};
      a.tiled = 1;
      if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, a, spec_out, st)) != MDC_OK) return s;
      hipLaunchKernelGGL(zero_f32, dim3(1024), dim3(kThreads), 0, st, r->S.u + half, half);
      lsqr_after_b(r->S, st);
    } else if (fwd) {  // beta u = A v - alpha u: [v0 - d Theta R v1 ; v1 - d Theta R* v0] - alpha u, in place
      const Recur rec = lsqr_recur_fwd(r->S);
      IfftSeg a{r->S.u, r->S.v, r->onset, 0, r->c0, -dsc, 1.0f, lsqr_vinv(r->S)};
      IfftSeg b{r->S.u + half, r->S.v + half, r->onset, 1, r->c0 + r->nv, -dsc, 1.0f, lsqr_vinv(r->S)};
      a.tiled = b.tiled = 1;
      attach_recur(a, &rec, 0);
      attach_recur(b, &rec, r->S.nparts_fwd / 2);
      if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, a, spec_out, st)) != MDC_OK) return s;
      if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, b, spec_out, st)) != MDC_OK) return s;
      lsqr_after_fwd_fused(r->S, st);
    } else {  // alpha v = A^H u - beta v: [u0 - d keep R*^H Theta u1 ; u1 - d keep R^H Theta u0] - beta v
      const int* km = (r->decim > 1 && r->lv == 0) ? r->keep : nullptr;  // lattice levels hold no other traces
      const Recur rec = r->phase == kInitAdj ? lsqr_recur_init(r->S) : lsqr_recur_adj(r->S);
      IfftSeg a{r->S.v + half, r->S.u + half, km, 0, r->c0, -dsc, 1.0f, lsqr_uinv(r->S)};
      IfftSeg b{r->S.v, r->S.u, km, 1, r->c0 + r->nv, -dsc, 1.0f, lsqr_uinv(r->S)};
      a.tiled = b.tiled = 1;
      attach_recur(a, &rec, 0);
      attach_recur(b, &rec, r->S.nparts_adj / 2);
      if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, a, spec_out, st)) != MDC_OK) return s;
      if ((s = irfft_launch(op->tw, d.nt, d.nfmax, n, r->nv, N, b, spec_out, st)) != MDC_OK) return s;
      if (r->phase == kInitAdj) lsqr_after_init_adj_fused(r->S, st);
      else lsqr_after_adj_fused(r->S, st);
    }
  }
  return check_launch("serve step");
}

// One step: the levels present run one after another on the serving stream (they share the
// op's workspace).
mdc_status enqueue_step(mdc_server* S, std::vector<Request*>& part, bool fwd, hipStream_t st) {
  for (int l = 0; l < kLevels; ++l) {
    std::vector<Request*> group;
    for (Request* r : part)
      if (r->lv == l) group.push_back(r);
    if (group.empty()) continue;
    const mdc_status s = enqueue_level(S, S->lv[l], group, fwd, st);
    if (s != MDC_OK) return s;
  }
  return MDC_OK;
}

// Phase transitions of the requests of a step that has been enqueued.
void advance(std::vector<Request*>& part, bool fwd) {
  for (Request* r : part) {
    if (r->phase == kData) {
      r->phase = kInitAdj;
    } else if (fwd) {
      r->phase = kIterA;
    } else if (r->phase == kInitAdj) {
      r->phase = r->niter > 0 ? kIterF : kDone;
    } else {
      r->it += 1;
      r->phase = r->it >= r->niter ? kDone : kIterF;
    }
  }
}

void drop_graphs(mdc_server* S) {
  for (auto& kv : S->graphs) (void)hipGraphExecDestroy(kv.second);
  S->graphs.clear();
}

// One step: replayed from its captured graph when this composition has run before.
mdc_status run_step(mdc_server* S, std::vector<Request*>& part, bool fwd) {
  hipStream_t st = S->stream;
  const char* g = getenv("MDC_SERVE_GRAPH");
  const bool use = S->graphs_ok && !S->op->prof && !(g && g[0] == '0');
  mdc_status s = MDC_OK;
  if (!use) {
    s = enqueue_step(S, part, fwd, st);
  } else {
    std::vector<uint64_t> key{fwd ? 1ull : 0ull};
    for (Request* r : part) {
      key.push_back(r->id);
      key.push_back((uint64_t)r->phase);
    }
    auto hit = S->graphs.find(key);
    if (hit != S->graphs.end()) {
      S->replayed += 1;
      if (hipGraphLaunch(hit->second, st) != hipSuccess) s = fail(MDC_EDEVICE, "hipGraphLaunch failed");
    } else if (S->seen[key]++ == 0) {  // first occurrence: eager (initialises every kernel variant)
      s = enqueue_step(S, part, fwd, st);
    } else {
      if (S->graphs.size() >= 32) drop_graphs(S);  // compositions come and go; keep the cache small
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        const mdc_status cs = enqueue_step(S, part, fwd, st);
        ok = hipStreamEndCapture(st, &graph) == hipSuccess && graph != nullptr && cs == MDC_OK;
        ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
      }
      if (ok) {
        S->graphs[key] = exec;
        S->captured += 1;
        if (hipGraphLaunch(exec, st) != hipSuccess) s = fail(MDC_EDEVICE, "hipGraphLaunch failed");
      } else {  // capture unavailable: run eagerly from now on (nothing of the capture executed)
        (void)hipGetLastError();  // clear the failed capture's error
        S->graphs_ok = false;
        s = enqueue_step(S, part, fwd, st);
      }
    }
    if (S->seen.size() > 4096) S->seen.clear();
  }
  advance(part, fwd);
  return s;
}

size_t request_bytes(const mdc_server* S, const Request* r) { return slot_bytes_for(S->op->d.nt, r->n, r->nv); }

// Give a request its arena slot and generate its inputs (called with the lock held).
bool admit(mdc_server* S, Request* r) {
  const mdc_desc& d = S->op->d;
  size_t off;
  const size_t bytes = request_bytes(S, r);
  if (!S->arena.alloc(bytes, &off)) return false;
  r->slot_off = off;
  r->slot_bytes = bytes;
  char* p = S->arena_base + off;
  const int n = r->n;
  const size_t vec = 2 * tiled_len(d.nt, n * r->nv);
  r->onset = reinterpret_cast<int*>(p); p += align_up((size_t)n * r->nv * 4, 256);
  r->keep = reinterpret_cast<int*>(p); p += align_up((size_t)n * r->nv * 4, 256);
  r->S.sc = p; p += lsqr_scalars_bytes();
  r->S.rpart = reinterpret_cast<double*>(p); p += align_up((size_t)parts_for(d.nt, n, r->nv) * sizeof(double), 256);
  r->S.nparts_fwd = r->S.nparts_adj = parts_for(d.nt, n, r->nv);
  r->S.u = reinterpret_cast<float*>(p); p += align_up(vec * 4, 256);
  r->S.v = reinterpret_cast<float*>(p); p += align_up(vec * 4, 256);
  r->S.w = reinterpret_cast<float*>(p); p += align_up(vec * 4, 256);
  r->S.t = r->S.t2 = nullptr;
  r->S.x = reinterpret_cast<float*>(p);
  r->S.hist = r->hist;
  r->S.model = r->S.data = vec;
  // the transforms write only the traces of u and v: their padding traces start at zero
  hipLaunchKernelGGL(zero_f32, dim3(1024), dim3(kThreads), 0, S->stream, r->S.u, vec);
  hipLaunchKernelGGL(zero_f32, dim3(1024), dim3(kThreads), 0, S->stream, r->S.v, vec);
  hipLaunchKernelGGL(request_inputs, dim3(2048), dim3(kThreads), 0, S->stream, d.nt, S->g.nx, S->g.dx, S->g.dt,
                     S->g.c, S->g.eps, S->g.fp, r->decim, n, (const int*)S->lv[r->lv].idx, r->nv, r->pts,
                     fft_tile(d.nt, n * r->nv), r->onset, r->keep, r->S.w);
  r->phase = kData;
  return true;
}

// A finished request's solution (tiled, on its level's traces) onto the caller's full-grid output.
void finish_output(mdc_server* S, const Request* r) {
  const int nt = S->op->d.nt;
  if (r->lv == 0) {
    launch_from_tiles(r->x_out, r->S.x, nt, r->n * r->nv, 2, S->stream);
    return;
  }
  const Level& L = S->lv[r->lv];
  hipLaunchKernelGGL(scatter_lattice, dim3(2048), dim3(kThreads), 0, S->stream, (const float*)r->S.x, r->x_out,
                     (const int*)L.pos, nt, S->op->d.ns, r->nv, fft_tile(nt, L.n * r->nv),
                     tiled_len(nt, L.n * r->nv));
}

void release(mdc_server* S, Request* r) {
  if (r->slot_bytes) S->arena.release(r->slot_off, r->slot_bytes);
  r->slot_bytes = 0;
}

void worker_main(mdc_server* S) {
  (void)hipSetDevice(S->device);  // the device serve_create ran on, current there
  const int max_cols = S->op->d.max_cols;
  while (true) {
    std::vector<Request*> part, deferred_now;
    bool fwd;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->active.empty(); });
      if (S->stop) break;
      // cancelled requests leave at step boundaries
      for (auto it = S->active.begin(); it != S->active.end();) {
        if ((*it)->cancel) {
          (*it)->phase = kCanceled;
          (*it)->finished = true;
          release(S, *it);
          S->outstanding -= 1;
          it = S->active.erase(it);
          S->done_cv.notify_all();
        } else {
          ++it;
        }
      }
      if (S->active.empty()) S->forward_next = true;
      fwd = S->forward_next;
      int cols = 0;
      for (Request* r : S->active) cols += 2 * r->nv;
      if (!fwd) {  // lockstep: queued requests that would fit now wait for this adjoint step
        int c = cols;
        for (Request* r : S->queue) {
          if (r->cancel) continue;
          if (c + 2 * r->nv > max_cols || !S->arena.fits(request_bytes(S, r))) break;
          c += 2 * r->nv;
          deferred_now.push_back(r);
        }
      }
      if (fwd) {  // admission (new requests start with the forward data step)
        while (!S->queue.empty()) {
          Request* r = S->queue.front();
          if (r->cancel) {
            r->phase = kCanceled;
            r->finished = true;
            S->outstanding -= 1;
            S->queue.pop_front();
            S->done_cv.notify_all();
            continue;
          }
          if (cols + 2 * r->nv > max_cols || !admit(S, r)) break;
          cols += 2 * r->nv;
          S->active.push_back(r);
          S->queue.pop_front();
        }
      }
      for (Request* r : S->active)
        if (wants_forward(r) == fwd) part.push_back(r);
      if ((int)S->active.size() > S->max_active) S->max_active = (int)S->active.size();
      S->forward_next = !fwd;
      if (part.empty()) continue;
      S->request_steps += (long)part.size();
    }
    const auto step_start = std::chrono::steady_clock::now();
    mdc_status st = run_step(S, part, fwd);
    if (st == MDC_OK)
      for (Request* r : part)
        if (r->phase == kDone) finish_output(S, r);
    // always wait for the step, also after a failed launch, before any slot can be reused
    const hipError_t se = hipStreamSynchronize(S->stream);
    if (st == MDC_OK && se != hipSuccess) st = fail(MDC_EDEVICE, "serve step failed: %s", hipGetErrorString(se));
    const auto now = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    S->steps += 1;
    for (Request* r : deferred_now) {  // still queued (admission happens under this lock)
      if (!r->deferred) S->deferred += 1;
      r->deferred = true;
      S->deferred_s += std::chrono::duration<double>(now - step_start).count();
    }
    if (st != MDC_OK) {  // fail every running request; the server stays up for new ones
      S->error = st;
      for (Request* r : part) r->phase = kCanceled;
    }
    for (auto it = S->active.begin(); it != S->active.end();) {
      Request* r = *it;
      if (r->phase == kDone || r->phase == kCanceled) {
        r->finish = now;
        r->finished = true;
        if (r->phase == kDone) {
          S->latencies.push_back(std::chrono::duration<double>(r->finish - r->arrival).count());
          S->last_finish = now;
        }
        release(S, r);
        S->outstanding -= 1;
        it = S->active.erase(it);
        S->done_cv.notify_all();
      } else {
        ++it;
      }
    }
  }
}

// Full-grid traces of the lattice of decimation d (the Sub2 / Sub4 rule), in trace order.
std::vector<int> lattice_traces(int nx, int d) {
  std::vector<int> idx;
  for (int r = 0; r < nx * nx; ++r) {
    const int ix = r / nx, iy = r % nx;
    const bool keep = d == 2 ? ((ix + iy) & 1) == 0 : (((ix - iy) % 4) + 4) % 4 == 0;
    if (keep) idx.push_back(r);
  }
  return idx;
}

size_t level_bytes(const mdc_op* op, int nx, int d) {
  const size_t nsub = lattice_traces(nx, d).size();
  return align_up(nsub * 4, 256) + align_up((size_t)nx * nx * 4, 256) + sub_op_resident_bytes(op, (int)nsub);
}

// Carve a lattice level out of the arena: index tables and the gathered kernel.
mdc_status make_level(mdc_server* S, int d) {
  const int nx = S->g.nx, n = nx * nx;
  const std::vector<int> idx = lattice_traces(nx, d);
  std::vector<int> pos(n, -1);
  for (size_t i = 0; i < idx.size(); ++i) pos[idx[i]] = (int)i;
  const size_t bytes = level_bytes(S->op, nx, d);
  size_t off;
  if (!S->arena.alloc(bytes, &off))
    return fail(MDC_ENOMEM, "lattice level d=%d needs %zu bytes of the arena", d, bytes);
  S->reserved += bytes;
  Level& L = S->lv[level_of(d)];
  char* p = S->arena_base + off;
  L.n = (int)idx.size();
  L.idx = reinterpret_cast<int*>(p); p += align_up(idx.size() * 4, 256);
  L.pos = reinterpret_cast<int*>(p); p += align_up((size_t)n * 4, 256);
  if (hipMemcpyAsync(L.idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, S->stream) != hipSuccess ||
      hipMemcpyAsync(L.pos, pos.data(), (size_t)n * 4, hipMemcpyHostToDevice, S->stream) != hipSuccess ||
      hipStreamSynchronize(S->stream) != hipSuccess)  // the host tables go out of scope
    return fail(MDC_EDEVICE, "uploading the lattice tables failed");
  return sub_op_create(S->op, L.idx, L.n, p, S->stream, &L.op);
}

}  // namespace

extern "C" {

mdc_status serve_request_bytes(const mdc_op* op, int nv, size_t* bytes) {
  if (!op || !bytes) return fail(MDC_EINVAL, "NULL argument");
  if (nv < 1 || nv > kMaxPoints) return fail(MDC_EINVAL, "nv=%d outside [1, %d]", nv, kMaxPoints);
  *bytes = slot_bytes_for(op->d.nt, op->d.ns, nv);
  return MDC_OK;
}

mdc_status serve_level_bytes(const mdc_op* op, int decim, size_t* bytes) {
  if (!op || !bytes) return fail(MDC_EINVAL, "NULL argument");
  if (decim != 2 && decim != 4) return fail(MDC_EINVAL, "decimation must be 2 or 4");
  const int nx = (int)std::lround(std::sqrt((double)op->d.ns));
  if (nx * nx != op->d.ns || op->d.ns != op->d.nr) return fail(MDC_EINVAL, "not a square grid operator");
  *bytes = level_bytes(op, nx, decim);
  return MDC_OK;
}

mdc_status serve_create(mdc_op* op, const serve_geometry* g, void* arena, size_t arena_bytes, mdc_server** out) {
  if (!op || !g || !out) return fail(MDC_EINVAL, "NULL argument");
  if (op->d.ns != op->d.nr) return fail(MDC_EINVAL, "serving needs a square operator (ns == nr)");
  if (g->nx <= 0 || g->nx * g->nx != op->d.ns) return fail(MDC_EINVAL, "grid nx=%d does not match ns=%d", g->nx, op->d.ns);
  if (!(g->dt > 0) || !(g->dx > 0) || !(g->c > 0) || g->eps < 0) return fail(MDC_EINVAL, "bad geometry");
  if (!arena || !aligned(arena, 256)) return fail(MDC_EINVAL, "arena must be non-NULL and 256-byte aligned");
  if (!op->kernel_ready) return fail(MDC_EINVAL, "kernel not loaded");
  if (g->sublattice & ~6) return fail(MDC_EINVAL, "sublattice=%d: a combination of 2 and 4", g->sublattice);
  mdc_server* S = new (std::nothrow) mdc_server();
  if (!S) return fail(MDC_ENOMEM, "host allocation failed");
  S->op = op;
  S->g = *g;
  S->arena_base = static_cast<char*>(arena);
  S->arena_bytes = arena_bytes / 256 * 256;
  S->arena.reset(S->arena_bytes);
  S->lv[0].op = op;
  S->lv[0].n = op->d.ns;
  if (hipGetDevice(&S->device) != hipSuccess || hipStreamCreate(&S->stream) != hipSuccess) {
    delete S;
    return fail(MDC_EDEVICE, "creating the serving stream failed");
  }
  for (int dd : {2, 4}) {
    if (!(g->sublattice & dd)) continue;
    const mdc_status ls = make_level(S, dd);
    if (ls != MDC_OK) {
      (void)hipStreamSynchronize(S->stream);
      for (auto& L : S->lv)
        if (L.op && L.op != op) mdc_destroy(L.op);
      (void)hipStreamDestroy(S->stream);
      delete S;
      return ls;
    }
  }
  if (hipStreamSynchronize(S->stream) != hipSuccess) {
    for (auto& L : S->lv)
      if (L.op && L.op != op) mdc_destroy(L.op);
    (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(MDC_EDEVICE, "preparing the lattice levels failed");
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return MDC_OK;
}

mdc_status serve_submit(mdc_server* S, const serve_req* q, uint64_t* id) {
  if (!S || !q || !id) return fail(MDC_EINVAL, "NULL argument");
  if (q->nv < 1 || q->nv > kMaxPoints) return fail(MDC_EINVAL, "nv=%d outside [1, %d]", q->nv, kMaxPoints);
  if (q->niter < 0) return fail(MDC_EINVAL, "niter must be >= 0");
  if (q->decim != 1 && q->decim != 2 && q->decim != 4) return fail(MDC_EINVAL, "decimation must be 1, 2 or 4");
  if (!q->vx || !q->vy || !q->vz) return fail(MDC_EINVAL, "virtual point arrays must not be NULL");
  if (!q->x_out || !aligned(q->x_out, 16)) return fail(MDC_EINVAL, "x_out must be non-NULL and 16-byte aligned");
  if (q->hist && !aligned(q->hist, 8)) return fail(MDC_EINVAL, "hist must be 8-byte aligned");
  if (2 * q->nv > S->op->d.max_cols) return fail(MDC_ENOMEM, "2*nv=%d exceeds the column budget %d", 2 * q->nv, S->op->d.max_cols);
  Request* r = new (std::nothrow) Request();
  if (!r) return fail(MDC_ENOMEM, "host allocation failed");
  r->nv = q->nv;
  r->niter = q->niter;
  r->decim = q->decim;
  r->lv = S->lv[level_of(q->decim)].op ? level_of(q->decim) : 0;
  r->n = S->lv[r->lv].n;
  const size_t need = request_bytes(S, r);
  if (need > S->arena_bytes - S->reserved) {
    delete r;
    return fail(MDC_ENOMEM, "request needs %zu bytes, the arena has %zu free of levels", need,
                S->arena_bytes - S->reserved);
  }
  for (int v = 0; v < q->nv; ++v) {
    r->pts.vx[v] = q->vx[v];
    r->pts.vy[v] = q->vy[v];
    r->pts.vz[v] = q->vz[v];
  }
  r->x_out = q->x_out;
  r->hist = q->hist;
  r->arrival = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete r;
      return fail(MDC_EBUSY, "server is shutting down");
    }
    r->id = S->next_id++;
    *id = r->id;
    if (!S->any_arrival) {
      S->first_arrival = r->arrival;
      S->any_arrival = true;
    }
    S->all[r->id] = r;
    S->queue.push_back(r);
    S->outstanding += 1;
  }
  S->cv.notify_all();
  return MDC_OK;
}

mdc_status serve_poll(mdc_server* S, uint64_t id, int* done, double* latency_s) {
  if (!S || !done) return fail(MDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return fail(MDC_EINVAL, "unknown request id %llu", (unsigned long long)id);
  Request* r = it->second;
  if (!r->finished) {
    *done = 0;
    return MDC_ENOTREADY;
  }
  // a finished request is reported once and then released
  const bool ok = r->phase == kDone;
  const double lat = std::chrono::duration<double>(r->finish - r->arrival).count();
  S->all.erase(it);
  delete r;
  if (ok) {
    *done = 1;
    if (latency_s) *latency_s = lat;
    return MDC_OK;
  }
  *done = -1;
  return fail(MDC_ECANCELED, "request %llu was cancelled or failed", (unsigned long long)id);
}

mdc_status serve_cancel(mdc_server* S, uint64_t id) {
  if (!S) return fail(MDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return fail(MDC_EINVAL, "unknown request id %llu", (unsigned long long)id);
  it->second->cancel = true;
  S->cv.notify_all();
  return MDC_OK;
}

mdc_status serve_drain(mdc_server* S) {
  if (!S) return fail(MDC_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  S->done_cv.wait(lk, [&] { return S->outstanding == 0; });
  return S->error == MDC_OK ? MDC_OK : fail(S->error, "a serving step failed");
}

mdc_status serve_stats(mdc_server* S, int skip, double* solves_per_s, double* p50_s, double* p99_s, int* completed,
                       int* max_active, long* steps) {
  if (!S) return fail(MDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  std::vector<double> lat(S->latencies.begin() + std::min<size_t>(skip < 0 ? 0 : skip, S->latencies.size()),
                          S->latencies.end());
  if (completed) *completed = (int)S->latencies.size();
  if (max_active) *max_active = S->max_active;
  if (steps) *steps = S->steps;
  if (solves_per_s) {
    const double span = S->any_arrival ? std::chrono::duration<double>(S->last_finish - S->first_arrival).count() : 0.0;
    *solves_per_s = span > 0 ? (double)S->latencies.size() / span : 0.0;
  }
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double p) {
    if (lat.empty()) return 0.0;
    const double pos = p * (double)(lat.size() - 1);
    const size_t i = (size_t)pos;
    const double fr = pos - (double)i;
    return i + 1 < lat.size() ? lat[i] * (1 - fr) + lat[i + 1] * fr : lat[i];
  };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  return MDC_OK;
}

mdc_status serve_phase_stats(mdc_server* S, long* request_steps, long* deferred, double* deferred_s) {
  if (!S) return fail(MDC_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (request_steps) *request_steps = S->request_steps;
  if (deferred) *deferred = S->deferred;
  if (deferred_s) *deferred_s = S->deferred_s;
  return MDC_OK;
}

mdc_status serve_graph_stats(mdc_server* S, long* captured, long* replayed) {
  if (!S) return fail(MDC_EINVAL, "NULL server");
  if (captured) *captured = S->captured.load();
  if (replayed) *replayed = S->replayed.load();
  return MDC_OK;
}

mdc_status serve_destroy(mdc_server* S) {
  if (!S) return MDC_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipStreamSynchronize(S->stream);
  drop_graphs(S);
  (void)hipStreamDestroy(S->stream);
  for (auto& L : S->lv)
    if (L.op && L.op != S->op) mdc_destroy(L.op);
  for (auto& kv : S->all) delete kv.second;
  delete S;
  return MDC_OK;
}

}  // extern "C"
