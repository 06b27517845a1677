// C ABI of the reconstruction library: argument validation, memory layout of
// the caller-owned plan and workspace buffers, and the enqueue order of the
// kernels.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/recon.h"
#include "kernels.hpp"

using namespace recon;

namespace {

thread_local std::string g_last_error;

recon_status_t fail(recon_status_t s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

recon_status_t hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return RECON_E_HIP;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
  } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int default_L(int N) {
  int L = 64;
  while (L < 2 * N - 1) L *= 2;
  return L;
}

int base_prec(int32_t prec) { return prec & ~RECON_ITER_FP64; }
bool iter_f64(int32_t prec) { return (prec & RECON_ITER_FP64) != 0; }

// A plan / workspace precision: one of the NUDFT precisions, optionally with
// the FP64 iteration (FP64 adjoint only, L <= 1024).
bool valid_prec(int32_t prec, int32_t L) {
  const int b = base_prec(prec);
  if (b < RECON_FP32 || b > RECON_FP64) return false;
  if (iter_f64(prec) && (b != RECON_FP64 || L > 1024)) return false;
  return true;
}

recon_status_t check_geometry(int64_t M, int32_t N, int32_t L) {
  if (N < 2 || N > 1024) return fail(RECON_E_RANGE, "N must be in [2, 1024]");
  if (!is_pow2(L) || L < 64 || L > 2048)
    return fail(RECON_E_RANGE, "L must be a power of two in [64, 2048]");
  if (L < 2 * N - 1) return fail(RECON_E_RANGE, "L must be >= 2N-1");
  if (M < 1 || M > (int64_t)0x7fffffff) return fail(RECON_E_RANGE, "M must be in [1, 2^31-1]");
  return RECON_OK;
}

struct PlanLayout {
  size_t k, ex, ey, tw, khat, at, xs, ph, tw64, khat64, total;
};

PlanLayout plan_layout(int64_t M, int32_t N, int32_t L, int32_t prec_full) {
  PlanLayout p{};
  const int prec = base_prec(prec_full);
  size_t off = 0;
  p.k = off;
  off = align_up(off + (size_t)M * 2 * sizeof(double));
  p.ex = off;
  off = align_up(off + (size_t)M * N * sizeof(float2));
  p.ey = off;
  off = align_up(off + (size_t)M * N * sizeof(float2));
  p.tw = off;
  off = align_up(off + (size_t)L * sizeof(float2));
  p.khat = off;
  off = align_up(off + (size_t)L * L * sizeof(float));
  p.at = p.xs = 0;
  if (prec == RECON_BF16X3 || prec == RECON_FP16X3) {
    p.at = off;
    off = align_up(off + 4 * (size_t)N * split_pad_M(M) * 2);
    p.xs = off;
    off = align_up(off + 4 * (size_t)M * split_pad_N(N) * 2);
  }
  p.ph = 0;
  if (prec == RECON_FP64) {  // phase tables of the FP64 adjoint
    p.ph = off;
    off = align_up(off + 2 * (size_t)M * phase_record(N) * sizeof(double2));
  }
  p.tw64 = p.khat64 = 0;
  if (iter_f64(prec_full)) {  // FP64 twiddles and spectrum of the FP64 iteration
    p.tw64 = off;
    off = align_up(off + (size_t)L * sizeof(double2));
    p.khat64 = off;
    off = align_up(off + (size_t)L * L * sizeof(double));
  }
  p.total = off;
  return p;
}

struct WsLayout {
  size_t b, x[2], r, d[2], qd, T, p1, p3, p4, pg0, pobj, params, yy, yyp, sc, adj, xb, total;
  int rows, nb1, nb3, nb4, adj_splits;
};

// Images and the row-transform intermediate hold complex64 values, or
// complex128 with the FP64 iteration (f64).  hq: two more images after the
// common layout (frozen image and gradient of the half-quadratic solver).
WsLayout ws_layout(int64_t M, int32_t N, int32_t L, int32_t B, bool f64, bool hq = false) {
  WsLayout w{};
  const size_t es = f64 ? sizeof(double2) : sizeof(float2);
  const size_t img = (size_t)B * N * N * es;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  w.b = take(img);
  w.x[0] = take(img);
  w.x[1] = take(img);
  w.r = take(img);
  w.d[0] = take(img);
  w.d[1] = take(img);
  w.qd = take(img);
  w.T = take((size_t)B * N * L * es);
  w.rows = fft_rows_per_block(L);  // rows per block of every per-row kernel
  w.nb1 = cdiv(N, w.rows);
  w.nb3 = L / fft_cols_per_block(L, f64);  // <d, Qd> partials come from the column pass
  w.nb4 = cdiv(N, w.rows);
  w.p1 = take((size_t)B * w.nb1 * 3 * sizeof(double));
  w.p3 = take((size_t)B * w.nb3 * sizeof(double));
  w.p4 = take((size_t)B * w.nb4 * 4 * sizeof(double));
  w.pg0 = take((size_t)B * w.nb4 * sizeof(double));
  w.pobj = take((size_t)B * w.nb4 * 4 * sizeof(double));
  w.params = take((size_t)B * sizeof(FrameParam));
  w.yy = take((size_t)B * sizeof(double));
  w.yyp = take((size_t)B * sumsq_parts() * sizeof(double));
  w.sc = take((size_t)B * sizeof(float));
  w.adj_splits = adjoint_splits(M, N);
  {
    // FP64 complex split-K partials serve every adjoint precision; the FP64
    // adjoint has a launch shape of its own: room for the larger of the two
    auto part_frames = [B](int splits, int group) -> size_t {
      const int frames = group < B ? group : B;
      return splits > 1 ? (size_t)splits * frames : 0;
    };
    const size_t a32 = part_frames(w.adj_splits, adjoint_group(M, N));
    const size_t a64 = part_frames(adjoint64_splits(M, N), adjoint64_group(M, N));
    w.adj = take((a32 > a64 ? a32 : a64) * N * N * sizeof(double2));
  }
  w.xb = 0;
  if (hq) w.xb = take(img);
  w.total = off;
  return w;
}

struct GramWsLayout {
  size_t part, emb, emb2, total;
  int splits;
};

GramWsLayout gram_ws_layout(int64_t M, int32_t N, int32_t L) {
  GramWsLayout g{};
  g.splits = gram_splits(M, N);
  size_t off = 0;
  g.part = off;
  off = align_up(off + (size_t)g.splits * 4 * N * N * sizeof(double));
  g.emb = off;
  off = align_up(off + (size_t)L * L * sizeof(double2));
  g.emb2 = off;
  off = align_up(off + (size_t)L * L * sizeof(double2));
  g.total = off;
  return g;
}

// Event traces of kernel kinds (recon_trace_enable / recon_trace_enable_set):
// per kind, up to `capacity` pairs of events recorded around its launches.
constexpr int TK_KINDS = 7;
struct Trace {
  std::mutex mu;
  unsigned mask = 0;  // enabled kinds
  int first = -1;     // kind read by recon_trace_read
  int capacity = 0;
  int used[TK_KINDS] = {};
  std::vector<hipEvent_t> ev[TK_KINDS];  // 2 per record
} g_trace;

struct TraceScope {
  hipEvent_t stop = nullptr;
  hipStream_t s;
  TraceScope(int kernel, hipStream_t st) : s(st) {
    if (!(g_trace.mask & (1u << kernel))) return;
    std::lock_guard<std::mutex> lk(g_trace.mu);
    if (!(g_trace.mask & (1u << kernel)) || g_trace.used[kernel] >= g_trace.capacity) return;
    const int i = g_trace.used[kernel]++;
    (void)hipEventRecord(g_trace.ev[kernel][2 * i], s);
    stop = g_trace.ev[kernel][2 * i + 1];
  }
  ~TraceScope() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

enum { TK_DIR = 0, TK_COL = 1, TK_ROWINV = 2, TK_UPDATE = 3, TK_ADJ = 4, TK_GRAM = 5, TK_FWD = 6 };

struct SolveCtx {
  int B = 0;
  int phi = 0;
  int iters = 0;                 // iterations run so far on this workspace (k)
  bool has_y = false;
  bool bg = false;               // some frame has the background penalty on (lambda0 > 0)
  bool pool = false;             // slot pool of the serving path
  std::vector<int32_t> start_at;  // per slot (pool only): k at admission
  std::vector<int32_t> stop_at;   // per slot (pool only): k at which the slot stops
};

// ---- convolution gridding / NUFFT geometry ---------------------------------
constexpr int GRID_TILE = 32;    // grid tile side of the spreading kernel
constexpr int GRID_GROUP = 16;   // frames gridded per round (bounds the workspace)

struct GridGeom {
  int64_t M;
  int Nout, G, W, h, phase;
  double beta;
};

struct GridLayout {
  size_t k, base, wy, wx, pf, toff, tent, deap, tw, total;
  int ntiles;
};

// Kaiser-Bessel shape for width W at oversampling sigma (minimal-oversampling rule).
double kb_beta(int W, double sigma) {
  const double a = (double)W / sigma * (sigma - 0.5);
  return M_PI * std::sqrt(a * a - 0.8);
}

// Fourier transform of the Kaiser-Bessel kernel (closed form).
double kb_hat(double nu, int W, double beta) {
  const double z2 = beta * beta - (M_PI * W * nu) * (M_PI * W * nu);
  if (z2 > 1e-12) {
    const double z = std::sqrt(z2);
    return W * std::sinh(z) / z;
  }
  if (z2 < -1e-12) {
    const double z = std::sqrt(-z2);
    return W * std::sin(z) / z;
  }
  return (double)W;
}

GridLayout grid_layout(const GridGeom& g) {
  GridLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  l.ntiles = (g.G / GRID_TILE) * (g.G / GRID_TILE);
  l.k = take((size_t)g.M * 2 * sizeof(double));
  l.base = take((size_t)g.M * sizeof(int2));
  l.wy = take((size_t)g.M * g.W * sizeof(double));
  l.wx = take((size_t)g.M * g.W * sizeof(double));
  l.pf = take((size_t)g.M * sizeof(double2));
  l.toff = take((size_t)(l.ntiles + 1) * sizeof(int));
  l.tent = take((size_t)g.M * 4 * sizeof(int));  // a footprint touches at most 2 x 2 tiles
  l.deap = take((size_t)g.Nout * sizeof(double));
  l.tw = take((size_t)g.G * sizeof(double2));
  l.total = off;
  return l;
}

recon_status_t check_grid_geom(const GridGeom& g) {
  if (g.M < 1 || g.M > (int64_t)0x1fffffff) return fail(RECON_E_RANGE, "M must be in [1, 2^29-1]");
  if (!is_pow2(g.G) || g.G < 64 || g.G > 2048)
    return fail(RECON_E_RANGE, "grid size must be a power of two in [64, 2048]");
  if (g.Nout < 2 || 2 * g.Nout > g.G) return fail(RECON_E_RANGE, "need 2 <= N and 2 N <= grid size");
  if (g.W < 2 || g.W > 16) return fail(RECON_E_RANGE, "kernel width must be in [2, 16]");
  if (!(g.beta > 0.0) || !std::isfinite(g.beta)) return fail(RECON_E_RANGE, "bad kernel shape");
  return RECON_OK;
}

// Per-tile sample lists (host counting sort), apodization correction and
// FFT twiddles uploaded to mem; per-sample weights computed on the device.
// Synchronises `s` (host staging buffers).
recon_status_t build_grid(const GridGeom& g, const double* traj, char* mem, const GridLayout& l,
                          hipStream_t s) {
  const int nt = g.G / GRID_TILE;
  std::vector<int> cnt((size_t)l.ntiles + 1, 0);
  std::vector<int> tiles((size_t)g.M * 4);
  std::vector<unsigned char> ntl((size_t)g.M);
  for (int64_t i = 0; i < g.M; ++i) {
    int ty[2], tx[2], ny = 0, nx = 0;
    const double u[2] = {(double)g.G * traj[2 * i + 1], (double)g.G * traj[2 * i]};
    for (int ax = 0; ax < 2; ++ax) {
      const int64_t g0 = (int64_t)std::floor(u[ax] - 0.5 * g.W) + 1;
      int* t = ax == 0 ? ty : tx;
      int& n = ax == 0 ? ny : nx;
      for (int j = 0; j < g.W; ++j) {
        const int gi = (int)(((g0 + j) % g.G + g.G) % g.G);
        const int ti = gi / GRID_TILE;
        bool seen = false;
        for (int q = 0; q < n; ++q) seen |= t[q] == ti;
        if (!seen) t[n++] = ti;
      }
    }
    int c = 0;
    for (int a = 0; a < ny; ++a)
      for (int b = 0; b < nx; ++b) {
        const int tile = ty[a] * nt + tx[b];
        tiles[(size_t)i * 4 + c++] = tile;
        ++cnt[tile + 1];
      }
    ntl[i] = (unsigned char)c;
  }
  for (int t = 0; t < l.ntiles; ++t) cnt[t + 1] += cnt[t];
  std::vector<int> toff(cnt);
  std::vector<int> tent((size_t)cnt[l.ntiles]);
  for (int64_t i = 0; i < g.M; ++i)
    for (int c = 0; c < ntl[i]; ++c) tent[cnt[tiles[(size_t)i * 4 + c]]++] = (int)i;
  std::vector<double> deap(g.Nout);
  for (int n = 0; n < g.Nout; ++n) deap[n] = 1.0 / kb_hat((double)(n - g.h) / g.G, g.W, g.beta);
  std::vector<double2> tw(g.G);
  for (int i = 0; i < g.G; ++i) {
    const double a = -2.0 * M_PI * (double)i / (double)g.G;
    tw[i] = make_double2(std::cos(a), std::sin(a));
  }
  hipError_t e = hipMemcpyAsync(mem + l.k, traj, (size_t)g.M * 2 * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(mem + l.toff, toff.data(), toff.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !tent.empty())
    e = hipMemcpyAsync(mem + l.tent, tent.data(), tent.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(mem + l.deap, deap.data(), deap.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(mem + l.tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_grid_weights(g.M, g.G, g.W, g.beta, g.h, g.phase,
                            reinterpret_cast<const double*>(mem + l.k),
                            reinterpret_cast<int2*>(mem + l.base), reinterpret_cast<double*>(mem + l.wy),
                            reinterpret_cast<double*>(mem + l.wx),
                            reinterpret_cast<double2*>(mem + l.pf), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "grid plan");
  return RECON_OK;
}

// Type-1 sums of B frames (or of the real weights when y == NULL, B = 1) in
// rounds of GRID_GROUP frames.  gridbuf: [GRID_GROUP][G][G], rows:
// [GRID_GROUP][G][Nout] (FP64 complex).
template <typename O>
recon_status_t grid_type1(const GridGeom& g, const char* mem, const GridLayout& l, const float2* y,
                          const double* w, double scale, int B, O* out, double2* gridbuf,
                          double2* rows, hipStream_t s) {
  for (int f0 = 0; f0 < B; f0 += GRID_GROUP) {
    const int nb = B - f0 < GRID_GROUP ? B - f0 : GRID_GROUP;
    HIP_TRY(launch_grid_spread(g.G, g.W, nb, g.M, reinterpret_cast<const int*>(mem + l.toff),
                               reinterpret_cast<const int*>(mem + l.tent),
                               reinterpret_cast<const int2*>(mem + l.base),
                               reinterpret_cast<const double*>(mem + l.wy),
                               reinterpret_cast<const double*>(mem + l.wx),
                               reinterpret_cast<const double2*>(mem + l.pf),
                               y ? y + (size_t)f0 * g.M : nullptr, w, scale, gridbuf, s));
    HIP_TRY(launch_grid_fft(g.G, g.Nout, g.h, nb, gridbuf, rows,
                            reinterpret_cast<const double*>(mem + l.deap),
                            out + (size_t)f0 * g.Nout * g.Nout,
                            reinterpret_cast<const double2*>(mem + l.tw), s));
  }
  return RECON_OK;
}

int grid_default_G(int Nout) {
  int G = 64;
  while (G < 2 * Nout) G *= 2;
  return G;
}

}  // namespace

struct recon_grid_s {
  GridGeom geom;
  GridLayout lay;
  char* mem;
};

namespace {

struct GridWs {
  size_t grid, rows, total;
};

GridWs grid_ws_layout(const GridGeom& g, int B) {
  GridWs w{};
  const int nb = B < GRID_GROUP ? B : GRID_GROUP;
  size_t off = 0;
  w.grid = off;
  off = align_up(off + (size_t)nb * g.G * g.G * sizeof(double2));
  w.rows = off;
  off = align_up(off + (size_t)nb * g.G * g.Nout * sizeof(double2));
  w.total = off;
  return w;
}

// Geometry of the lag-kernel type-1 sum of a plan: 2N outputs (lags
// -N .. N-1), grid >= 4N, no sample phase.
GridGeom lag_geom(int64_t M, int N, int W) {
  GridGeom g{};
  g.M = M;
  g.Nout = 2 * N;
  g.G = grid_default_G(2 * N);
  g.W = W;
  g.h = N;
  g.phase = 0;
  g.beta = kb_beta(W, (double)g.G / g.Nout);
  return g;
}

struct GramNufftWs {
  GridGeom geom;
  GridLayout lay;
  size_t gplan, ones, grid, rows, lag2n, emb, emb2, total;
};

GramNufftWs gram_nufft_layout(int64_t M, int N, int L, int W) {
  GramNufftWs w{};
  w.geom = lag_geom(M, N, W);
  w.lay = grid_layout(w.geom);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  w.gplan = take(w.lay.total);
  w.ones = take((size_t)M * sizeof(double));
  w.grid = take((size_t)w.geom.G * w.geom.G * sizeof(double2));
  w.rows = take((size_t)w.geom.G * w.geom.Nout * sizeof(double2));
  w.lag2n = take((size_t)w.geom.Nout * w.geom.Nout * sizeof(double2));
  w.emb = take((size_t)L * L * sizeof(double2));
  w.emb2 = take((size_t)L * L * sizeof(double2));
  w.total = off;
  return w;
}

}  // namespace

struct recon_plan_s {
  int64_t M;
  int32_t N, L, prec;  // prec: NUDFT precision (without RECON_ITER_FP64)
  bool f64 = false;    // FP64 iteration
  char* mem;
  size_t mem_bytes;
  PlanLayout lay;
  bool gram_done = false;
  std::mutex mu;
  std::unordered_map<void*, SolveCtx> solves;

  double* k() const { return reinterpret_cast<double*>(mem + lay.k); }
  float2* ex() const { return reinterpret_cast<float2*>(mem + lay.ex); }
  float2* ey() const { return reinterpret_cast<float2*>(mem + lay.ey); }
  float2* tw() const { return reinterpret_cast<float2*>(mem + lay.tw); }
  float* khat() const { return reinterpret_cast<float*>(mem + lay.khat); }
  void* at() const { return mem + lay.at; }
  void* xs() const { return mem + lay.xs; }
  double2* ph() const { return reinterpret_cast<double2*>(mem + lay.ph); }
  double2* tw64() const { return reinterpret_cast<double2*>(mem + lay.tw64); }
  double* khat64() const { return reinterpret_cast<double*>(mem + lay.khat64); }
  int32_t prec_full() const { return prec | (f64 ? RECON_ITER_FP64 : 0); }
  bool split() const { return prec == RECON_BF16X3 || prec == RECON_FP16X3; }
  int table_prec() const { return prec; }
  bool has_tables() const { return split(); }
};

namespace {

struct Ws {
  WsLayout lay;
  char* base;
  float2* img(size_t off) const { return reinterpret_cast<float2*>(base + off); }
  double2* img64(size_t off) const { return reinterpret_cast<double2*>(base + off); }
  template <typename C>
  C* at(size_t off) const { return reinterpret_cast<C*>(base + off); }
  double* dbl(size_t off) const { return reinterpret_cast<double*>(base + off); }
  FrameParam* params() const { return reinterpret_cast<FrameParam*>(base + lay.params); }
};

// Plans whose adjoint is FP32 or split-precision take at most this many
// frames per adjoint, forward or solve call.
constexpr int32_t MAX_BATCH_NON_FP64 = 64;

recon_status_t check_batch(recon_plan_t p, int32_t B) {
  if (p->prec != RECON_FP64 && B > MAX_BATCH_NON_FP64)
    return fail(RECON_E_ARG, "plans with an FP32 or split-precision adjoint take at most 64 "
                             "frames per adjoint, forward or solve call");
  return RECON_OK;
}

recon_status_t check_ws(recon_plan_t p, void* ws, size_t ws_bytes, int32_t B, Ws* out,
                        bool hq = false) {
  if (!ws) return fail(RECON_E_ARG, "workspace is NULL");
  if (B < 1) return fail(RECON_E_ARG, "B must be >= 1");
  out->lay = ws_layout(p->M, p->N, p->L, B, p->f64, hq);
  if (ws_bytes < out->lay.total)
    return fail(RECON_E_NOMEM, hq ? "workspace smaller than recon_hq_workspace_bytes"
                                  : "workspace smaller than recon_workspace_bytes");
  out->base = static_cast<char*>(ws);
  return RECON_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Q v for B frames into out (T: N x L scratch per frame); optional <v, Qv> partials.
recon_status_t gram_apply(recon_plan_t p, const float2* v, float2* out, int B, float2* T,
                          double* p3, hipStream_t s) {
  HIP_TRY(launch_rowfft_plain(p->L, p->N, B, v, T, p->tw(), s));
  {
    TraceScope ts(TK_COL, s);
    HIP_TRY(launch_colpass(p->L, p->N, B, T, p->khat(), p3, p->tw(), nullptr, 0, s));
  }
  {
    TraceScope ts(TK_ROWINV, s);
    HIP_TRY(launch_rowifft(p->L, p->N, B, T, out, p->tw(), nullptr, 0, s));
  }
  return RECON_OK;
}

// The same in FP64 (the FP64 iteration's warm start).
recon_status_t gram_apply64(recon_plan_t p, const double2* v, double2* out, int B, double2* T,
                            hipStream_t s) {
  HIP_TRY(launch_rowfft_plain(p->L, p->N, B, v, T, p->tw64(), s));
  HIP_TRY(launch_colpass(p->L, p->N, B, T, p->khat64(), nullptr, p->tw64(), nullptr, 0, s));
  HIP_TRY(launch_rowifft(p->L, p->N, B, T, out, p->tw64(), nullptr, 0, s));
  return RECON_OK;
}

// b = A^H y kept in FP64 for the FP64 iteration (FP64 adjoint only).
recon_status_t adjoint_traced64(recon_plan_t p, const float2* y, int B, double2* b, void* part,
                                hipStream_t s) {
  TraceScope ts(TK_ADJ, s);
  HIP_TRY(launch_adjoint_f64(p->M, p->N, B, p->ph(), y, b, static_cast<double2*>(part), s));
  return RECON_OK;
}

recon_status_t adjoint_traced(recon_plan_t p, const float2* y, int B, float2* b, void* part,
                              float* sc, hipStream_t s) {
  TraceScope ts(TK_ADJ, s);
  if (p->split())
    HIP_TRY(launch_adjoint_split(p->prec, p->M, p->N, B, p->at(), p->ex(), y, sc, b,
                                 static_cast<float2*>(part), s));
  else if (p->prec == RECON_FP64)
    HIP_TRY(launch_adjoint_f64(p->M, p->N, B, p->ph(), y, b, static_cast<double2*>(part), s));
  else
    HIP_TRY(launch_adjoint_f32(p->M, p->N, B, p->ex(), p->ey(), y, b, static_cast<float2*>(part), s));
  return RECON_OK;
}

}  // namespace

extern "C" {

size_t recon_plan_bytes(int64_t M, int32_t N, int32_t L, int32_t prec) {
  if (L == 0) L = default_L(N);
  if (check_geometry(M, N, L) != RECON_OK) return 0;
  if (!valid_prec(prec, L)) return 0;
  return plan_layout(M, N, L, prec).total;
}

size_t recon_gram_workspace_bytes(int64_t M, int32_t N, int32_t L) {
  if (L == 0) L = default_L(N);
  if (check_geometry(M, N, L) != RECON_OK) return 0;
  return gram_ws_layout(M, N, L).total;
}

size_t recon_workspace_bytes(int64_t M, int32_t N, int32_t L, int32_t B, int32_t prec) {
  if (L == 0) L = default_L(N);
  if (check_geometry(M, N, L) != RECON_OK || B < 1) return 0;
  if (!valid_prec(prec, L)) return 0;
  return ws_layout(M, N, L, B, iter_f64(prec)).total;
}

size_t recon_hq_workspace_bytes(int64_t M, int32_t N, int32_t L, int32_t B, int32_t prec) {
  if (L == 0) L = default_L(N);
  if (check_geometry(M, N, L) != RECON_OK || B < 1) return 0;
  if (!valid_prec(prec, L)) return 0;
  return ws_layout(M, N, L, B, iter_f64(prec), true).total;
}

recon_status_t recon_plan(const double* traj, int64_t M, int32_t N, int32_t L, int32_t prec,
                          void* plan_mem, size_t plan_mem_bytes, void* stream,
                          recon_plan_t* out) {
  g_last_error.clear();
  if (!traj || !plan_mem || !out) return fail(RECON_E_ARG, "NULL argument");
  if (L == 0) L = default_L(N);
  recon_status_t st = check_geometry(M, N, L);
  if (st != RECON_OK) return st;
  if (!valid_prec(prec, L))
    return fail(RECON_E_ARG, "unknown precision (RECON_ITER_FP64 needs RECON_FP64 and L <= 1024)");
  for (int64_t i = 0; i < 2 * M; ++i) {
    const double v = traj[i];
    if (!std::isfinite(v) || std::fabs(v) > 0.5)
      return fail(RECON_E_RANGE, "trajectory entries must be finite with |k| <= 0.5");
  }
  const PlanLayout lay = plan_layout(M, N, L, prec);
  if (plan_mem_bytes < lay.total) return fail(RECON_E_NOMEM, "plan memory smaller than recon_plan_bytes");
  auto* p = new recon_plan_s();
  p->M = M;
  p->N = N;
  p->L = L;
  p->prec = base_prec(prec);
  p->f64 = iter_f64(prec);
  p->mem = static_cast<char*>(plan_mem);
  p->mem_bytes = plan_mem_bytes;
  p->lay = lay;
  hipStream_t s = as_stream(stream);
  std::vector<float2> tw(L);
  for (int i = 0; i < L; ++i) {
    const double a = -2.0 * M_PI * (double)i / (double)L;
    tw[i] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  std::vector<double2> tw64(p->f64 ? L : 0);
  for (int i = 0; i < (int)tw64.size(); ++i) {
    const double a = -2.0 * M_PI * (double)i / (double)L;
    tw64[i] = make_double2(std::cos(a), std::sin(a));
  }
  hipError_t e = hipMemcpyAsync(p->k(), traj, (size_t)M * 2 * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->tw(), tw.data(), (size_t)L * sizeof(float2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && p->f64)
    e = hipMemcpyAsync(p->tw64(), tw64.data(), (size_t)L * sizeof(double2), hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess) e = launch_tables_f32(M, N, p->k(), p->ex(), p->ey(), s);
  if (e == hipSuccess && p->has_tables())
    e = launch_tables_split(p->table_prec(), M, N, p->k(), p->at(), p->xs(), s);
  if (e == hipSuccess && p->prec == RECON_FP64)
    e = launch_phase_tables_f64(M, N, p->k(), p->ph(), s);
  // The host copies above read caller and local memory: finish before return.
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "recon_plan");
  }
  *out = p;
  return RECON_OK;
}

recon_status_t recon_plan_info(recon_plan_t p, int64_t* M, int32_t* N, int32_t* L, int32_t* prec) {
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  if (M) *M = p->M;
  if (N) *N = p->N;
  if (L) *L = p->L;
  if (prec) *prec = p->prec_full();
  return RECON_OK;
}

void recon_plan_destroy(recon_plan_t p) { delete p; }

recon_status_t recon_gram_kernel(recon_plan_t p, void* ws, size_t ws_bytes, float* khat_out,
                                 double* lag_out, void* stream) {
  g_last_error.clear();
  if (!p || !ws) return fail(RECON_E_ARG, "NULL argument");
  const GramWsLayout g = gram_ws_layout(p->M, p->N, p->L);
  if (ws_bytes < g.total) return fail(RECON_E_NOMEM, "gram workspace smaller than recon_gram_workspace_bytes");
  hipStream_t s = as_stream(stream);
  char* base = static_cast<char*>(ws);
  double* part = reinterpret_cast<double*>(base + g.part);
  double2* emb = reinterpret_cast<double2*>(base + g.emb);
  double2* emb2 = reinterpret_cast<double2*>(base + g.emb2);
  {
    TraceScope ts(TK_GRAM, s);
    HIP_TRY(launch_gram_f64(p->M, p->N, p->k(), part, g.splits, s));
  }
  HIP_TRY(launch_gram_assemble(p->N, p->L, part, g.splits, lag_out, emb, s));
  HIP_TRY(launch_spectrum_f64(p->L, emb, emb2, p->khat(), khat_out,
                              p->f64 ? p->khat64() : nullptr, s));
  p->gram_done = true;
  return RECON_OK;
}

recon_status_t recon_adjoint(recon_plan_t p, const float* y, int32_t B, float* b, double* yy_out,
                             void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p || !y || !b) return fail(RECON_E_ARG, "NULL argument");
  Ws w;
  recon_status_t st = check_ws(p, ws, ws_bytes, B, &w);
  if (st == RECON_OK) st = check_batch(p, B);
  if (st != RECON_OK) return st;
  hipStream_t s = as_stream(stream);
  const float2* y2 = reinterpret_cast<const float2*>(y);
  if (yy_out) HIP_TRY(launch_sumsq(p->M, B, y2, w.dbl(w.lay.yyp), yy_out, s));
  return adjoint_traced(p, y2, B, reinterpret_cast<float2*>(b), w.img(w.lay.adj),
                        reinterpret_cast<float*>(w.base + w.lay.sc), s);
}

recon_status_t recon_forward(recon_plan_t p, const float* x, int32_t B, float* y, void* ws,
                             size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p || !x || !y) return fail(RECON_E_ARG, "NULL argument");
  Ws w;
  recon_status_t st = check_ws(p, ws, ws_bytes, B, &w);
  if (st == RECON_OK) st = check_batch(p, B);
  if (st != RECON_OK) return st;
  TraceScope ts(TK_FWD, as_stream(stream));
  if (p->has_tables())
    HIP_TRY(launch_forward_split(p->table_prec(), p->M, p->N, B, p->xs(), p->ey(),
                                 reinterpret_cast<const float2*>(x),
                                 reinterpret_cast<float*>(w.base + w.lay.sc),
                                 reinterpret_cast<float2*>(y), as_stream(stream)));
  else
    HIP_TRY(launch_forward_f32(p->M, p->N, B, p->ex(), p->ey(), reinterpret_cast<const float2*>(x),
                               reinterpret_cast<float2*>(y), as_stream(stream)));
  return RECON_OK;
}

recon_status_t recon_gram_apply(recon_plan_t p, const float* v, int32_t B, float* Qv, void* ws,
                                size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p || !v || !Qv) return fail(RECON_E_ARG, "NULL argument");
  if (v == Qv) return fail(RECON_E_ARG, "v and Qv may not alias");
  if (!p->gram_done) return fail(RECON_E_STATE, "recon_gram_kernel has not been called");
  Ws w;
  recon_status_t st = check_ws(p, ws, ws_bytes, B, &w);
  if (st != RECON_OK) return st;
  return gram_apply(p, reinterpret_cast<const float2*>(v), reinterpret_cast<float2*>(Qv), B,
                    w.img(w.lay.T), nullptr, as_stream(stream));
}

// ---- allocation-free Gram apply --------------------------------------------
// The row-pass intermediate of recon_gram_apply_noalloc lives in this
// file-scope device array (one copy per GPU, for the life of the process).
// Host code never uses its name as an address: the device address is taken
// once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this GPU's scratch array (looked up on first use).
static recon_status_t scratch_on_current_device(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RECON_E_RANGE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(RECON_E_HIP, "hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RECON_OK;
}

extern "C" size_t recon_gram_apply_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" recon_status_t recon_gram_apply_noalloc(recon_plan_t p, const float* v, int32_t B,
                                                   float* Qv, void* stream) {
  g_last_error.clear();
  if (!p || !v || !Qv) return fail(RECON_E_ARG, "NULL argument");
  if (v == Qv) return fail(RECON_E_ARG, "v and Qv may not alias");
  if (B < 1) return fail(RECON_E_ARG, "B must be >= 1");
  if (!p->gram_done) return fail(RECON_E_STATE, "recon_gram_kernel has not been called");
  const size_t need = (size_t)B * p->N * p->L * sizeof(float2);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(RECON_E_RANGE, "B * N * L * 8 bytes exceeds the 64 MiB scratch of "
                               "recon_gram_apply_noalloc (use fewer frames per call)");
  void* T = nullptr;
  recon_status_t st = scratch_on_current_device(&T);
  if (st != RECON_OK) return st;
  return gram_apply(p, reinterpret_cast<const float2*>(v), reinterpret_cast<float2*>(Qv), B,
                    static_cast<float2*>(T), nullptr, as_stream(stream));
}

// lambda0 >= 0 and, when it is > 0, alpha0 > 0 (the background term).
static recon_status_t check_background(double lambda0, double alpha0) {
  if (!(lambda0 >= 0.0) || !std::isfinite(lambda0)) return fail(RECON_E_RANGE, "lambda0 must be >= 0");
  if (lambda0 > 0.0 && (!(alpha0 > 0.0) || !std::isfinite(alpha0)))
    return fail(RECON_E_RANGE, "alpha0 must be > 0");
  return RECON_OK;
}

// b given in complex64 (b_in) or, for the FP64 iteration, in complex128
// (b_in64); otherwise b = A^H y.
static recon_status_t solve_begin(recon_plan_t p, const float* y, const float* b_in,
                                  const double* b_in64, int32_t B, double lambda, double delta,
                                  double lambda0, double alpha0, int32_t phi, const float* x0,
                                  void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  if (!y && !b_in && !b_in64) return fail(RECON_E_ARG, "need y or b");
  if (b_in64 && !p->f64) return fail(RECON_E_ARG, "an FP64 b needs a plan with RECON_ITER_FP64");
  if (!p->gram_done) return fail(RECON_E_STATE, "recon_gram_kernel has not been called");
  if (phi < 0 || phi > 2) return fail(RECON_E_ARG, "unknown penalty");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(RECON_E_RANGE, "lambda must be >= 0");
  if (phi != RECON_PHI_QUADRATIC && (!(delta > 0.0) || !std::isfinite(delta)))
    return fail(RECON_E_RANGE, "delta must be > 0");
  recon_status_t st = check_background(lambda0, alpha0);
  if (st != RECON_OK) return st;
  Ws w;
  st = check_ws(p, ws, ws_bytes, B, &w);
  if (st == RECON_OK) st = check_batch(p, B);
  if (st != RECON_OK) return st;
  hipStream_t s = as_stream(stream);
  const int N = p->N;
  const size_t n_img = (size_t)B * N * N;
  double* yy = w.dbl(w.lay.yy);
  if (y) {
    const float2* y2 = reinterpret_cast<const float2*>(y);
    HIP_TRY(launch_sumsq(p->M, B, y2, w.dbl(w.lay.yyp), yy, s));
    recon_status_t r =
        p->f64 ? adjoint_traced64(p, y2, B, w.img64(w.lay.b), w.img(w.lay.adj), s)
               : adjoint_traced(p, y2, B, w.img(w.lay.b), w.img(w.lay.adj),
                                reinterpret_cast<float*>(w.base + w.lay.sc), s);
    if (r != RECON_OK) return r;
  } else if (b_in64) {
    HIP_TRY(hipMemcpyAsync(w.img64(w.lay.b), b_in64, n_img * sizeof(double2),
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_zero_f64((size_t)B, yy, s));
  } else {
    const float2* b2 = reinterpret_cast<const float2*>(b_in);
    if (p->f64)
      HIP_TRY(launch_widen(n_img, b2, w.img64(w.lay.b), s));
    else
      HIP_TRY(hipMemcpyAsync(w.img(w.lay.b), b2, n_img * sizeof(float2), hipMemcpyDeviceToDevice,
                             s));
    HIP_TRY(launch_zero_f64((size_t)B, yy, s));
  }
  HIP_TRY(launch_set_params(B, lambda, delta, lambda0, lambda0 > 0.0 ? alpha0 : 1.0, INT32_MAX,
                            w.params(), s));
  if (p->f64) {
    // x0 widened into the second iterate buffer (free before iteration 1)
    const double2* x0w = nullptr;
    const double2* qx0 = nullptr;
    if (x0) {
      HIP_TRY(launch_widen(n_img, reinterpret_cast<const float2*>(x0), w.img64(w.lay.x[1]), s));
      x0w = w.img64(w.lay.x[1]);
      recon_status_t r = gram_apply64(p, x0w, w.img64(w.lay.qd), B, w.img64(w.lay.T), s);
      if (r != RECON_OK) return r;
      qx0 = w.img64(w.lay.qd);
    }
    HIP_TRY(launch_init(phi, N, w.lay.rows, B, w.img64(w.lay.b), x0w, qx0, w.img64(w.lay.x[0]),
                        w.img64(w.lay.r), w.img64(w.lay.d[0]), w.dbl(w.lay.p4),
                        w.dbl(w.lay.pg0), w.params(), s));
  } else {
    const float2* qx0 = nullptr;
    if (x0) {
      recon_status_t r = gram_apply(p, reinterpret_cast<const float2*>(x0), w.img(w.lay.qd), B,
                                    w.img(w.lay.T), nullptr, s);
      if (r != RECON_OK) return r;
      qx0 = w.img(w.lay.qd);
    }
    HIP_TRY(launch_init(phi, N, w.lay.rows, B, w.img(w.lay.b),
                        reinterpret_cast<const float2*>(x0), qx0, w.img(w.lay.x[0]),
                        w.img(w.lay.r), w.img(w.lay.d[0]), w.dbl(w.lay.p4), w.dbl(w.lay.pg0),
                        w.params(), s));
  }
  std::lock_guard<std::mutex> lk(p->mu);
  SolveCtx& c = p->solves[ws];
  c = SolveCtx{};
  c.B = B;
  c.phi = phi;
  c.iters = 0;
  c.has_y = y != nullptr;
  c.bg = lambda0 > 0.0;
  return RECON_OK;
}

recon_status_t recon_solve_begin(recon_plan_t p, const float* y, const float* b_in, int32_t B,
                                 double lambda, double delta, double lambda0, double alpha0,
                                 int32_t phi, const float* x0, void* ws, size_t ws_bytes,
                                 void* stream) {
  return solve_begin(p, y, b_in, nullptr, B, lambda, delta, lambda0, alpha0, phi, x0, ws,
                     ws_bytes, stream);
}

recon_status_t recon_solve_begin_b64(recon_plan_t p, const double* b, int32_t B, double lambda,
                                     double delta, double lambda0, double alpha0, int32_t phi,
                                     const float* x0, void* ws, size_t ws_bytes, void* stream) {
  if (!b) {
    g_last_error.clear();
    return fail(RECON_E_ARG, "NULL b");
  }
  return solve_begin(p, nullptr, nullptr, b, B, lambda, delta, lambda0, alpha0, phi, x0, ws,
                     ws_bytes, stream);
}

static recon_status_t get_ctx(recon_plan_t p, void* ws, SolveCtx* out) {
  std::lock_guard<std::mutex> lk(p->mu);
  auto it = p->solves.find(ws);
  if (it == p->solves.end()) return fail(RECON_E_STATE, "recon_solve_begin has not been called on this workspace");
  *out = it->second;
  return RECON_OK;
}

}  // extern "C"

// Iterations k0 .. k0+iters-1 of the pseudo-conjugate gradient on every frame
// of the workspace (frames with stop_at <= k are skipped by the kernels).
// C: float2 (FP32 iteration, plan twiddles/spectrum in FP32) or double2.
template <typename C, typename K>
static recon_status_t run_iterations_t(recon_plan_t p, const SolveCtx& c, const Ws& w, int k0,
                                       int iters, const C* tw, const K* khat, hipStream_t s) {
  const int N = p->N, L = p->L;
  // A slot pool launches over slots 0 .. (highest slot still running) only:
  // the slots above it are idle for the whole call, and their blocks would
  // only start and exit.  (The scheduler fills the lowest free slot first.)
  int B = c.B;
  if (c.pool) {
    int hi = 0;
    for (int sl = 0; sl < c.B; ++sl)
      if (c.stop_at[sl] > k0) hi = sl + 1;
    if (hi == 0) return RECON_OK;  // nothing running
    B = hi;
  }
  C* T = w.at<C>(w.lay.T);
  C* r = w.at<C>(w.lay.r);
  for (int it = 0; it < iters; ++it) {
    const int k = k0 + it;
    C* d_old = w.at<C>(w.lay.d[k & 1]);
    C* d_new = w.at<C>(w.lay.d[(k + 1) & 1]);
    C* x_old = w.at<C>(w.lay.x[k & 1]);
    C* x_new = w.at<C>(w.lay.x[(k + 1) & 1]);
    {
      TraceScope ts(TK_DIR, s);
      HIP_TRY(launch_dir_rowfft(L, c.phi, N, B, r, d_old, d_new, x_old, T, w.dbl(w.lay.p4),
                                w.lay.nb4, w.dbl(w.lay.p1), w.params(), tw, k, c.bg, s));
    }
    {
      TraceScope ts(TK_COL, s);
      HIP_TRY(launch_colpass(L, N, B, T, khat, w.dbl(w.lay.p3), tw, w.params(), k, s));
    }
    {
      TraceScope ts(TK_UPDATE, s);
      HIP_TRY(launch_update(L, c.phi, N, B, T, x_old, x_new, d_new, r, w.dbl(w.lay.p1),
                            w.lay.nb1, w.dbl(w.lay.p3), w.lay.nb3, w.dbl(w.lay.p4), w.params(),
                            tw, k, c.bg, s));
    }
  }
  return RECON_OK;
}

// Half-quadratic minimisation: `outer` times, freeze the penalty weights at
// the current image and run `inner` linear-CG steps on the surrogate; then
// the true gradient's norm into the update partials (for the statistics).
// An inner step is the conjugate-gradient step's three kernels with the
// weights taken from the frozen image xb.  The step counter k advances by
// one per inner step (x, d buffers as in run_iterations).
template <typename C, typename K>
static recon_status_t run_hq_t(recon_plan_t p, const SolveCtx& c, const Ws& w, int k0, int outer,
                               int inner, const C* tw, const K* khat, hipStream_t s) {
  const int N = p->N, L = p->L, B = c.B, R = w.lay.rows;
  C* T = w.at<C>(w.lay.T);
  C* r = w.at<C>(w.lay.r);
  C* xb = w.at<C>(w.lay.xb);
  int k = k0;
  for (int o = 0; o < outer; ++o) {
    HIP_TRY(launch_hq_freeze(N, B, w.lay.nb4, w.at<C>(w.lay.x[k & 1]), xb, w.dbl(w.lay.p4), s));
    for (int it = 0; it < inner; ++it, ++k) {
      C* d_old = w.at<C>(w.lay.d[k & 1]);
      C* d_new = w.at<C>(w.lay.d[(k + 1) & 1]);
      C* x_old = w.at<C>(w.lay.x[k & 1]);
      C* x_new = w.at<C>(w.lay.x[(k + 1) & 1]);
      {
        TraceScope ts(TK_DIR, s);
        HIP_TRY(launch_dir_rowfft(L, c.phi, N, B, r, d_old, d_new, x_old, T, w.dbl(w.lay.p4),
                                  w.lay.nb4, w.dbl(w.lay.p1), w.params(), tw, k, c.bg, s, xb));
      }
      {
        TraceScope ts(TK_COL, s);
        HIP_TRY(launch_colpass(L, N, B, T, khat, w.dbl(w.lay.p3), tw, w.params(), k, s));
      }
      {
        TraceScope ts(TK_UPDATE, s);
        HIP_TRY(launch_update(L, c.phi, N, B, T, x_old, x_new, d_new, r, w.dbl(w.lay.p1),
                              w.lay.nb1, w.dbl(w.lay.p3), w.lay.nb3, w.dbl(w.lay.p4), w.params(),
                              tw, k, c.bg, s, xb));
      }
    }
  }
  HIP_TRY(launch_hq_gnorm(c.phi, N, R, B, w.at<C>(w.lay.x[k & 1]), r, w.dbl(w.lay.p4),
                          w.params(), c.bg, s));
  return RECON_OK;
}

extern "C" {

static recon_status_t run_iterations(recon_plan_t p, const SolveCtx& c, const Ws& w, int k0,
                                     int iters, hipStream_t s) {
  if (p->f64) return run_iterations_t(p, c, w, k0, iters, p->tw64(), p->khat64(), s);
  return run_iterations_t(p, c, w, k0, iters, p->tw(), p->khat(), s);
}

static recon_status_t run_hq(recon_plan_t p, const SolveCtx& c, const Ws& w, int k0, int outer,
                             int inner, hipStream_t s) {
  if (p->f64) return run_hq_t(p, c, w, k0, outer, inner, p->tw64(), p->khat64(), s);
  return run_hq_t(p, c, w, k0, outer, inner, p->tw(), p->khat(), s);
}

// Copy (FP32 iteration) or round (FP64 iteration) n complex values of the
// workspace at `off` to the complex64 buffer out.
static recon_status_t copy_out(recon_plan_t p, const Ws& w, size_t off, size_t n, float2* out,
                               hipStream_t s) {
  if (p->f64) {
    HIP_TRY(launch_narrow(n, w.img64(off), out, s));
  } else if (out != w.img(off)) {
    HIP_TRY(hipMemcpyAsync(out, w.img(off), n * sizeof(float2), hipMemcpyDeviceToDevice, s));
  }
  return RECON_OK;
}

recon_status_t recon_solve_iterate(recon_plan_t p, int32_t iters, void* ws, size_t ws_bytes,
                                   void* stream) {
  g_last_error.clear();
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  if (iters < 0) return fail(RECON_E_ARG, "iters must be >= 0");
  SolveCtx c;
  recon_status_t st = get_ctx(p, ws, &c);
  if (st != RECON_OK) return st;
  if (c.pool) return fail(RECON_E_STATE, "workspace is a slot pool: use recon_pool_step");
  Ws w;
  st = check_ws(p, ws, ws_bytes, c.B, &w);
  if (st != RECON_OK) return st;
  st = run_iterations(p, c, w, c.iters, iters, as_stream(stream));
  if (st != RECON_OK) return st;
  std::lock_guard<std::mutex> lk(p->mu);
  p->solves[ws].iters = c.iters + iters;
  return RECON_OK;
}

recon_status_t recon_solve_hq_iterate(recon_plan_t p, int32_t outer, int32_t inner, void* ws,
                                      size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  if (outer < 0 || inner < 0) return fail(RECON_E_ARG, "outer and inner must be >= 0");
  if ((int64_t)outer * inner > INT32_MAX) return fail(RECON_E_RANGE, "too many iterations");
  SolveCtx c;
  recon_status_t st = get_ctx(p, ws, &c);
  if (st != RECON_OK) return st;
  if (c.pool) return fail(RECON_E_STATE, "workspace is a slot pool");
  if ((int64_t)c.iters + (int64_t)outer * inner > INT32_MAX)
    return fail(RECON_E_RANGE, "iteration counter overflow");
  Ws w;
  st = check_ws(p, ws, ws_bytes, c.B, &w, true);
  if (st != RECON_OK) return st;
  st = run_hq(p, c, w, c.iters, outer, inner, as_stream(stream));
  if (st != RECON_OK) return st;
  std::lock_guard<std::mutex> lk(p->mu);
  p->solves[ws].iters = c.iters + outer * inner;
  return RECON_OK;
}

recon_status_t recon_solve_export(recon_plan_t p, int32_t field, float* out, void* ws,
                                  size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p || !out) return fail(RECON_E_ARG, "NULL argument");
  SolveCtx c;
  recon_status_t st = get_ctx(p, ws, &c);
  if (st != RECON_OK) return st;
  if (c.pool) return fail(RECON_E_STATE, "workspace is a slot pool: use recon_pool_retire");
  Ws w;
  st = check_ws(p, ws, ws_bytes, c.B, &w);
  if (st != RECON_OK) return st;
  hipStream_t s = as_stream(stream);
  const size_t n = (size_t)c.B * p->N * p->N;
  const int k = c.iters;
  float2* o = reinterpret_cast<float2*>(out);
  switch (field) {
    case 0: return copy_out(p, w, w.lay.x[k & 1], n, o, s);
    case 1: return copy_out(p, w, w.lay.r, n, o, s);
    case 2:
    case 3: {
      const int dir = field == 3;
      if (p->f64)
        HIP_TRY(launch_export(c.phi, p->N, w.lay.rows, c.B, w.img64(w.lay.x[k & 1]),
                              w.img64(w.lay.r), dir ? w.img64(w.lay.d[k & 1]) : nullptr,
                              w.dbl(w.lay.p4), w.lay.nb4, w.params(), o, dir, s));
      else
        HIP_TRY(launch_export(c.phi, p->N, w.lay.rows, c.B, w.img(w.lay.x[k & 1]),
                              w.img(w.lay.r), dir ? w.img(w.lay.d[k & 1]) : nullptr,
                              w.dbl(w.lay.p4), w.lay.nb4, w.params(), o, dir, s));
      return RECON_OK;
    }
    case 4: return copy_out(p, w, w.lay.b, n, o, s);
    default: return fail(RECON_E_ARG, "unknown field");
  }
}

// Objective partials and stats of B frames starting at frame f0 of the
// workspace, whose current iterate sits in x buffer xi.
static recon_status_t stats_of(recon_plan_t p, const SolveCtx& c, const Ws& w, int f0, int B,
                               int xi, int iters, recon_stats_t* stats, hipStream_t s) {
  const int N = p->N;
  const size_t fo = (size_t)f0 * N * N;
  double* pobj = w.dbl(w.lay.pobj) + (size_t)f0 * w.lay.nb4 * 4;
  if (p->f64)
    HIP_TRY(launch_objective(c.phi, N, w.lay.rows, B, w.img64(w.lay.x[xi]) + fo,
                             w.img64(w.lay.b) + fo, w.img64(w.lay.r) + fo, pobj,
                             w.params() + f0, s));
  else
    HIP_TRY(launch_objective(c.phi, N, w.lay.rows, B, w.img(w.lay.x[xi]) + fo,
                             w.img(w.lay.b) + fo, w.img(w.lay.r) + fo, pobj, w.params() + f0,
                             s));
  HIP_TRY(launch_stats(B, pobj, w.lay.nb4, w.dbl(w.lay.p4) + (size_t)f0 * w.lay.nb4 * 4,
                       w.lay.nb4, w.dbl(w.lay.pg0) + (size_t)f0 * w.lay.nb4, w.lay.nb4,
                       w.dbl(w.lay.yy) + f0, iters, w.params() + f0, stats, s));
  return RECON_OK;
}

recon_status_t recon_solve_end(recon_plan_t p, float* x_out, recon_stats_t* stats, void* ws,
                               size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  SolveCtx c;
  recon_status_t st = get_ctx(p, ws, &c);
  if (st != RECON_OK) return st;
  if (c.pool) return fail(RECON_E_STATE, "workspace is a slot pool: use recon_pool_retire");
  Ws w;
  st = check_ws(p, ws, ws_bytes, c.B, &w);
  if (st != RECON_OK) return st;
  hipStream_t s = as_stream(stream);
  const int k = c.iters;
  if (stats) {
    st = stats_of(p, c, w, 0, c.B, k & 1, k, stats, s);
    if (st != RECON_OK) return st;
  }
  if (x_out)
    return copy_out(p, w, w.lay.x[k & 1], (size_t)c.B * p->N * p->N,
                    reinterpret_cast<float2*>(x_out), s);
  return RECON_OK;
}

recon_status_t recon_solve(recon_plan_t p, const float* y, int32_t B, double lambda, double delta,
                           int32_t iters, int32_t phi, float* x, int32_t x_in_is_x0, void* ws,
                           size_t ws_bytes, recon_stats_t* stats, void* stream) {
  if (!p || !y || !x) return fail(RECON_E_ARG, "NULL argument");
  if (iters < 0) return fail(RECON_E_ARG, "iters must be >= 0");
  recon_status_t st = recon_solve_begin(p, y, nullptr, B, lambda, delta, 0.0, 1.0, phi,
                                        x_in_is_x0 ? x : nullptr, ws, ws_bytes, stream);
  if (st != RECON_OK) return st;
  st = recon_solve_iterate(p, iters, ws, ws_bytes, stream);
  if (st != RECON_OK) return st;
  return recon_solve_end(p, x, stats, ws, ws_bytes, stream);
}

recon_status_t recon_solve_hq(recon_plan_t p, const float* y, int32_t B, double lambda,
                              double delta, int32_t outer, int32_t inner, int32_t phi, float* x,
                              int32_t x_in_is_x0, void* ws, size_t ws_bytes, recon_stats_t* stats,
                              void* stream) {
  if (!p || !y || !x) return fail(RECON_E_ARG, "NULL argument");
  if (outer < 0 || inner < 0) return fail(RECON_E_ARG, "outer and inner must be >= 0");
  if (B >= 1 && ws_bytes < ws_layout(p->M, p->N, p->L, B, p->f64, true).total)
    return fail(RECON_E_NOMEM, "workspace smaller than recon_hq_workspace_bytes");
  recon_status_t st = recon_solve_begin(p, y, nullptr, B, lambda, delta, 0.0, 1.0, phi,
                                        x_in_is_x0 ? x : nullptr, ws, ws_bytes, stream);
  if (st != RECON_OK) return st;
  st = recon_solve_hq_iterate(p, outer, inner, ws, ws_bytes, stream);
  if (st != RECON_OK) return st;
  return recon_solve_end(p, x, stats, ws, ws_bytes, stream);
}

// ---- slot pools (continuous batching) -------------------------------------

recon_status_t recon_pool_reset(recon_plan_t p, int32_t B, int32_t phi, void* ws, size_t ws_bytes,
                                void* stream) {
  g_last_error.clear();
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  if (!p->gram_done) return fail(RECON_E_STATE, "recon_gram_kernel has not been called");
  if (phi < 0 || phi > 2) return fail(RECON_E_ARG, "unknown penalty");
  Ws w;
  recon_status_t st = check_ws(p, ws, ws_bytes, B, &w);
  if (st != RECON_OK) return st;
  // every slot idle: stop_at = 0
  HIP_TRY(launch_set_params(B, 0.0, 1.0, 0.0, 1.0, 0, w.params(), as_stream(stream)));
  std::lock_guard<std::mutex> lk(p->mu);
  SolveCtx& c = p->solves[ws];
  c = SolveCtx{};
  c.B = B;
  c.phi = phi;
  c.iters = 0;
  c.pool = true;
  c.start_at.assign(B, 0);
  c.stop_at.assign(B, 0);
  return RECON_OK;
}

static recon_status_t get_pool(recon_plan_t p, void* ws, SolveCtx* out) {
  recon_status_t st = get_ctx(p, ws, out);
  if (st != RECON_OK) return st;
  if (!out->pool) return fail(RECON_E_STATE, "workspace is not a slot pool (recon_pool_reset)");
  return RECON_OK;
}

recon_status_t recon_pool_admit(recon_plan_t p, int32_t slot, const float* y, double lambda,
                                double delta, double lambda0, double alpha0, int32_t iters,
                                void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p || !y) return fail(RECON_E_ARG, "NULL argument");
  SolveCtx c;
  recon_status_t st = get_pool(p, ws, &c);
  if (st != RECON_OK) return st;
  if (slot < 0 || slot >= c.B) return fail(RECON_E_RANGE, "slot out of range");
  if (c.stop_at[slot] > c.iters) return fail(RECON_E_STATE, "slot is busy");
  if (iters < 0 || (int64_t)c.iters + iters > INT32_MAX) return fail(RECON_E_RANGE, "bad iteration count");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(RECON_E_RANGE, "lambda must be >= 0");
  if (c.phi != RECON_PHI_QUADRATIC && (!(delta > 0.0) || !std::isfinite(delta)))
    return fail(RECON_E_RANGE, "delta must be > 0");
  st = check_background(lambda0, alpha0);
  if (st != RECON_OK) return st;
  Ws w;
  st = check_ws(p, ws, ws_bytes, c.B, &w);
  if (st != RECON_OK) return st;
  hipStream_t s = as_stream(stream);
  const int N = p->N;
  const size_t fo = (size_t)slot * N * N;
  const int k = c.iters;
  const float2* y2 = reinterpret_cast<const float2*>(y);
  HIP_TRY(launch_sumsq(p->M, 1, y2, w.dbl(w.lay.yyp) + (size_t)slot * sumsq_parts(),
                       w.dbl(w.lay.yy) + slot, s));
  st = p->f64 ? adjoint_traced64(p, y2, 1, w.img64(w.lay.b) + fo, w.img(w.lay.adj), s)
              : adjoint_traced(p, y2, 1, w.img(w.lay.b) + fo, w.img(w.lay.adj),
                               reinterpret_cast<float*>(w.base + w.lay.sc) + slot, s);
  if (st != RECON_OK) return st;
  const int stop = k + iters;
  HIP_TRY(launch_set_params(1, lambda, delta, lambda0, lambda0 > 0.0 ? alpha0 : 1.0, stop,
                            w.params() + slot, s));
  double* p4 = w.dbl(w.lay.p4) + (size_t)slot * w.lay.nb4 * 4;
  double* pg0 = w.dbl(w.lay.pg0) + (size_t)slot * w.lay.nb4;
  if (p->f64)
    HIP_TRY(launch_init(c.phi, N, w.lay.rows, 1, w.img64(w.lay.b) + fo, nullptr, nullptr,
                        w.img64(w.lay.x[k & 1]) + fo, w.img64(w.lay.r) + fo,
                        w.img64(w.lay.d[k & 1]) + fo, p4, pg0, w.params() + slot, s));
  else
    HIP_TRY(launch_init(c.phi, N, w.lay.rows, 1, w.img(w.lay.b) + fo, nullptr, nullptr,
                        w.img(w.lay.x[k & 1]) + fo, w.img(w.lay.r) + fo,
                        w.img(w.lay.d[k & 1]) + fo, p4, pg0, w.params() + slot, s));
  std::lock_guard<std::mutex> lk(p->mu);
  p->solves[ws].start_at[slot] = k;
  p->solves[ws].stop_at[slot] = stop;
  if (lambda0 > 0.0) p->solves[ws].bg = true;  // until the pool is reset
  return RECON_OK;
}

recon_status_t recon_pool_step(recon_plan_t p, int32_t iters, void* ws, size_t ws_bytes,
                               void* stream) {
  g_last_error.clear();
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  if (iters < 0) return fail(RECON_E_ARG, "iters must be >= 0");
  SolveCtx c;
  recon_status_t st = get_pool(p, ws, &c);
  if (st != RECON_OK) return st;
  if ((int64_t)c.iters + iters > INT32_MAX) return fail(RECON_E_RANGE, "iteration counter overflow");
  Ws w;
  st = check_ws(p, ws, ws_bytes, c.B, &w);
  if (st != RECON_OK) return st;
  st = run_iterations(p, c, w, c.iters, iters, as_stream(stream));
  if (st != RECON_OK) return st;
  std::lock_guard<std::mutex> lk(p->mu);
  p->solves[ws].iters = c.iters + iters;
  return RECON_OK;
}

recon_status_t recon_pool_retire(recon_plan_t p, int32_t slot, float* x_out, recon_stats_t* stats,
                                 void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(RECON_E_ARG, "NULL plan");
  SolveCtx c;
  recon_status_t st = get_pool(p, ws, &c);
  if (st != RECON_OK) return st;
  if (slot < 0 || slot >= c.B) return fail(RECON_E_RANGE, "slot out of range");
  const int stop = c.stop_at[slot];
  if (stop > c.iters) return fail(RECON_E_STATE, "slot has not finished its iterations");
  Ws w;
  st = check_ws(p, ws, ws_bytes, c.B, &w);
  if (st != RECON_OK) return st;
  hipStream_t s = as_stream(stream);
  const int N = p->N;
  const size_t fo = (size_t)slot * N * N;
  if (stats) {
    st = stats_of(p, c, w, slot, 1, stop & 1, stop - c.start_at[slot], stats, s);
    if (st != RECON_OK) return st;
  }
  if (x_out) {
    const size_t off = w.lay.x[stop & 1] + fo * (p->f64 ? sizeof(double2) : sizeof(float2));
    return copy_out(p, w, off, (size_t)N * N, reinterpret_cast<float2*>(x_out), s);
  }
  return RECON_OK;
}

int64_t recon_pool_iteration(recon_plan_t p, void* ws) {
  SolveCtx c;
  if (!p || get_ctx(p, ws, &c) != RECON_OK) return -1;
  return c.iters;
}

static void trace_clear() {
  for (auto& v : g_trace.ev) {
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
    v.clear();
  }
  for (int& u : g_trace.used) u = 0;
  g_trace.mask = 0;
  g_trace.first = -1;
  g_trace.capacity = 0;
}

recon_status_t recon_trace_enable_set(uint32_t mask, int32_t capacity) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_trace.mu);
  trace_clear();
  if (mask == 0) return RECON_OK;
  if ((mask >> TK_KINDS) != 0 || capacity < 1) return fail(RECON_E_ARG, "bad trace request");
  for (int k = 0; k < TK_KINDS; ++k) {
    if (!(mask & (1u << k))) continue;
    g_trace.ev[k].resize(2 * (size_t)capacity);
    for (auto& e : g_trace.ev[k]) {
      const hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) {
        e = nullptr;
        trace_clear();
        return hip_fail(err, "hipEventCreate");
      }
    }
    if (g_trace.first < 0) g_trace.first = k;
  }
  g_trace.capacity = capacity;
  g_trace.mask = mask;
  return RECON_OK;
}

recon_status_t recon_trace_enable(int32_t kernel, int32_t capacity) {
  if (kernel < 0) return recon_trace_enable_set(0, 0);
  if (kernel >= TK_KINDS) return fail(RECON_E_ARG, "bad trace request");
  return recon_trace_enable_set(1u << kernel, capacity);
}

int32_t recon_trace_read_kind(int32_t kernel, float* ms_out, int32_t n) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  if (!ms_out || n < 0 || kernel < 0 || kernel >= TK_KINDS) return -1;
  if (!(g_trace.mask & (1u << kernel))) return 0;
  const int m = g_trace.used[kernel] < n ? g_trace.used[kernel] : n;
  const auto& ev = g_trace.ev[kernel];
  for (int i = 0; i < m; ++i) {
    if (hipEventSynchronize(ev[2 * i + 1]) != hipSuccess) return -1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) return -1;
    ms_out[i] = ms;
  }
  return m;
}

int32_t recon_trace_read(float* ms_out, int32_t n) {
  int first;
  {
    std::lock_guard<std::mutex> lk(g_trace.mu);
    first = g_trace.first;
  }
  if (first < 0) return (ms_out && n >= 0) ? 0 : -1;
  return recon_trace_read_kind(first, ms_out, n);
}

// ---- convolution gridding / NUFFT ------------------------------------------

static GridGeom adjoint_geom(int64_t M, int32_t N, int32_t G, int32_t W, double beta) {
  GridGeom g{};
  g.M = M;
  g.Nout = N;
  g.G = G ? G : grid_default_G(N);
  g.W = W;
  g.h = N / 2;
  g.phase = 1;
  g.beta = beta > 0.0 ? beta : kb_beta(W, (double)g.G / N);
  return g;
}

size_t recon_grid_bytes(int64_t M, int32_t N, int32_t G, int32_t W) {
  const GridGeom g = adjoint_geom(M, N, G, W, 0.0);
  if (N < 2 || W < 2 || W > 16 || check_grid_geom(g) != RECON_OK) return 0;
  return grid_layout(g).total;
}

recon_status_t recon_grid_plan(const double* traj, int64_t M, int32_t N, int32_t G, int32_t W,
                               double beta, void* mem, size_t mem_bytes, void* stream,
                               recon_grid_t* out) {
  g_last_error.clear();
  if (!traj || !mem || !out) return fail(RECON_E_ARG, "NULL argument");
  if (N < 2) return fail(RECON_E_RANGE, "N must be >= 2");
  if (W < 2 || W > 16) return fail(RECON_E_RANGE, "kernel width must be in [2, 16]");
  if (beta < 0.0 || !std::isfinite(beta)) return fail(RECON_E_RANGE, "beta must be >= 0");
  const GridGeom g = adjoint_geom(M, N, G, W, beta);
  recon_status_t st = check_grid_geom(g);
  if (st != RECON_OK) return st;
  for (int64_t i = 0; i < 2 * M; ++i) {
    const double v = traj[i];
    if (!std::isfinite(v) || std::fabs(v) > 0.5)
      return fail(RECON_E_RANGE, "trajectory entries must be finite with |k| <= 0.5");
  }
  const GridLayout l = grid_layout(g);
  if (mem_bytes < l.total) return fail(RECON_E_NOMEM, "grid memory smaller than recon_grid_bytes");
  st = build_grid(g, traj, static_cast<char*>(mem), l, as_stream(stream));
  if (st != RECON_OK) return st;
  auto* p = new recon_grid_s();
  p->geom = g;
  p->lay = l;
  p->mem = static_cast<char*>(mem);
  *out = p;
  return RECON_OK;
}

void recon_grid_destroy(recon_grid_t g) { delete g; }

recon_status_t recon_grid_info(recon_grid_t g, int32_t* G, int32_t* W, double* beta) {
  if (!g) return fail(RECON_E_ARG, "NULL grid plan");
  if (G) *G = g->geom.G;
  if (W) *W = g->geom.W;
  if (beta) *beta = g->geom.beta;
  return RECON_OK;
}

size_t recon_grid_workspace_bytes(recon_grid_t g, int32_t B) {
  if (!g || B < 1) return 0;
  return grid_ws_layout(g->geom, B).total;
}

recon_status_t recon_grid_adjoint(recon_grid_t g, const float* y, const double* w, int32_t B,
                                  float* out, void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!g || !y || !out || !ws) return fail(RECON_E_ARG, "NULL argument");
  if (B < 1) return fail(RECON_E_ARG, "B must be >= 1");
  const GridWs wl = grid_ws_layout(g->geom, B);
  if (ws_bytes < wl.total) return fail(RECON_E_NOMEM, "workspace smaller than recon_grid_workspace_bytes");
  char* base = static_cast<char*>(ws);
  return grid_type1(g->geom, g->mem, g->lay, reinterpret_cast<const float2*>(y), w,
                    1.0 / g->geom.Nout, B, reinterpret_cast<float2*>(out),
                    reinterpret_cast<double2*>(base + wl.grid),
                    reinterpret_cast<double2*>(base + wl.rows), as_stream(stream));
}

recon_status_t recon_grid_adjoint64(recon_grid_t g, const float* y, const double* w, int32_t B,
                                    double* out, void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!g || !y || !out || !ws) return fail(RECON_E_ARG, "NULL argument");
  if (B < 1) return fail(RECON_E_ARG, "B must be >= 1");
  const GridWs wl = grid_ws_layout(g->geom, B);
  if (ws_bytes < wl.total) return fail(RECON_E_NOMEM, "workspace smaller than recon_grid_workspace_bytes");
  char* base = static_cast<char*>(ws);
  return grid_type1(g->geom, g->mem, g->lay, reinterpret_cast<const float2*>(y), w,
                    1.0 / g->geom.Nout, B, reinterpret_cast<double2*>(out),
                    reinterpret_cast<double2*>(base + wl.grid),
                    reinterpret_cast<double2*>(base + wl.rows), as_stream(stream));
}

recon_status_t recon_grid_density(recon_grid_t g, int32_t iters, double* w, void* ws,
                                  size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!g || !w || !ws) return fail(RECON_E_ARG, "NULL argument");
  if (iters < 1) return fail(RECON_E_ARG, "iters must be >= 1");
  const GridWs wl = grid_ws_layout(g->geom, 1);
  if (ws_bytes < wl.total) return fail(RECON_E_NOMEM, "workspace smaller than recon_grid_workspace_bytes");
  hipStream_t s = as_stream(stream);
  const GridGeom& gg = g->geom;
  const GridLayout& l = g->lay;
  double2* grid = reinterpret_cast<double2*>(static_cast<char*>(ws) + wl.grid);
  const double sigma = (double)gg.G / gg.Nout;
  const double h0 = kb_hat(0.0, gg.W, gg.beta);
  const double final_scale = h0 * h0 * h0 * h0 / (sigma * sigma);
  HIP_TRY(launch_fill_f64((size_t)gg.M, 1.0, w, s));
  for (int it = 0; it < iters; ++it) {
    HIP_TRY(launch_grid_spread(gg.G, gg.W, 1, gg.M, reinterpret_cast<const int*>(g->mem + l.toff),
                               reinterpret_cast<const int*>(g->mem + l.tent),
                               reinterpret_cast<const int2*>(g->mem + l.base),
                               reinterpret_cast<const double*>(g->mem + l.wy),
                               reinterpret_cast<const double*>(g->mem + l.wx),
                               reinterpret_cast<const double2*>(g->mem + l.pf), nullptr, w, 1.0,
                               grid, s));
    HIP_TRY(launch_dcf_update(gg.G, gg.W, gg.M, reinterpret_cast<const int2*>(g->mem + l.base),
                              reinterpret_cast<const double*>(g->mem + l.wy),
                              reinterpret_cast<const double*>(g->mem + l.wx), grid, w,
                              it + 1 == iters ? final_scale : 1.0, s));
  }
  return RECON_OK;
}

size_t recon_gram_nufft_workspace_bytes(int64_t M, int32_t N, int32_t L, int32_t W) {
  if (L == 0) L = default_L(N);
  if (check_geometry(M, N, L) != RECON_OK || W < 2 || W > 16) return 0;
  const GramNufftWs w = gram_nufft_layout(M, N, L, W);
  if (check_grid_geom(w.geom) != RECON_OK) return 0;
  return w.total;
}

recon_status_t recon_gram_kernel_nufft(recon_plan_t p, int32_t W, void* ws, size_t ws_bytes,
                                       float* khat_out, double* lag_out, void* stream) {
  g_last_error.clear();
  if (!p || !ws) return fail(RECON_E_ARG, "NULL argument");
  if (W < 2 || W > 16) return fail(RECON_E_RANGE, "kernel width must be in [2, 16]");
  const GramNufftWs w = gram_nufft_layout(p->M, p->N, p->L, W);
  recon_status_t st = check_grid_geom(w.geom);
  if (st != RECON_OK) return st;
  if (ws_bytes < w.total) return fail(RECON_E_NOMEM, "workspace smaller than recon_gram_nufft_workspace_bytes");
  hipStream_t s = as_stream(stream);
  char* base = static_cast<char*>(ws);
  // the trajectory is on the device in the plan; the host binning needs it
  std::vector<double> traj((size_t)p->M * 2);
  HIP_TRY(hipMemcpyAsync(traj.data(), p->k(), traj.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  char* gmem = base + w.gplan;
  st = build_grid(w.geom, traj.data(), gmem, w.lay, s);
  if (st != RECON_OK) return st;
  double* ones = reinterpret_cast<double*>(base + w.ones);
  HIP_TRY(launch_fill_f64((size_t)p->M, 1.0, ones, s));
  double2* lag2n = reinterpret_cast<double2*>(base + w.lag2n);
  {
    TraceScope ts(TK_GRAM, s);
    st = grid_type1(w.geom, gmem, w.lay, nullptr, ones, 1.0 / ((double)p->N * p->N), 1, lag2n,
                    reinterpret_cast<double2*>(base + w.grid),
                    reinterpret_cast<double2*>(base + w.rows), s);
    if (st != RECON_OK) return st;
  }
  double2* emb = reinterpret_cast<double2*>(base + w.emb);
  HIP_TRY(launch_lag_embed(p->N, p->L, lag2n, lag_out, emb, s));
  HIP_TRY(launch_spectrum_f64(p->L, emb, reinterpret_cast<double2*>(base + w.emb2), p->khat(),
                              khat_out, p->f64 ? p->khat64() : nullptr, s));
  p->gram_done = true;
  return RECON_OK;
}

const char* recon_status_string(recon_status_t s) {
  switch (s) {
    case RECON_OK: return "ok";
    case RECON_E_ARG: return "invalid argument";
    case RECON_E_RANGE: return "size or value out of range";
    case RECON_E_NOMEM: return "buffer too small";
    case RECON_E_HIP: return "HIP runtime error";
    case RECON_E_STATE: return "call order violated";
    case RECON_E_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

const char* recon_last_error(void) { return g_last_error.c_str(); }

const char* recon_version(void) { return "recon-mi355x 0.1 (gfx950)"; }

}  // extern "C"
