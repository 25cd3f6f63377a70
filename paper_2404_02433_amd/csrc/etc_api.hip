// Host side of the ETC library: plan, preparation, PCG driver, results.
// All solver arithmetic runs in the kernels of etc_kernels.hpp; the host only
// validates, sizes, launches and polls the device state every few passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "etc.h"
#include "etc_kernels.hpp"

using namespace etc;

namespace {

thread_local std::string g_err;

etc_status fail(etc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(ETC_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(name)                                                                         \
  do {                                                                                          \
    hipError_t e_ = hipGetLastError();                                                          \
    if (e_ != hipSuccess) return fail(ETC_E_HIP, std::string("launch ") + name + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kThreads = 256;
// Isotropic stencil tile width (b; tiles of 16 a rows): float32 lines
// longer than 256 take 128 (fewer halo lines: 0.35 against 0.36 ms at
// 512^3), shorter ones 64 (fewer idle lanes on ragged tiles: 48^3 to 256^3
// run 3-22 % faster); float64 keeps 64 (register footprint).
constexpr int stencil_tbw(size_t elt, int nb) { return (elt == 4 && nb > 256) ? 128 : 64; }
constexpr int kStencilTAH = 16;
constexpr int kMaxGridStride = 2048;   // grid of the grid-stride reduction kernels
constexpr int kThomasP = 32;           // most partitions per line in the tridiagonal kernel

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Launch shapes.  Every grid carries the instance index of a batch in its
// last dimension; nX is the number of blocks (= partial sums) per instance.
struct LaunchCfg {
  // operator: block (64, 4) over 64 x 16 tiles; residual: 64 x 4 tiles
  int stencilTBW;  // isotropic stencil tile width (b)
  dim3 gridRes;    // isotropic float64 residual (64-wide tiles), nRes blocks per instance
  int nRes;
  dim3 gridA;
  int nA_max;  // partials of the stencil at its smallest chunk (autotuner candidates)
  int kchunk, nA;
  dim3 gridR;
  int kchunkR, nR;
  // rows
  int rpb, nrows;
  dim3 gridRows;
  int nRows;
  size_t ldsRows;
  // columns
  int tb, colThreads;
  dim3 gridCols;
  size_t ldsCols;
  int colsPers;  // blocks of the persistent column kernels (0: one block per tile)
  // tridiagonal
  dim3 gridThomas;  // persistent blocks per instance (x) times instances (z)
  int tvar;         // variant (ThomasVariants): block of thomasTB modes x thomasP partitions
  int thomasTB, thomasP;
  int Puse, maxm, nThomas, thomasTiles;
  int nThomasMax;  // tiles per instance of the narrowest block shape (autotuner candidates)
  // grid-stride kernels
  dim3 gridStride;
  int nStride;
  dim3 gridKeff;
  int nKeff;
  // extrema: tiles of 256 plane positions x chunks of extChunk planes
  dim3 gridExt;
  int extChunk, nExt;
};

}  // namespace

struct etc_plan {
  Geo g;
  int64_t n_user[3];
  int axis;
  etc_precision prec;
  etc_dtype in_dt;
  etc_options opt;
  hipStream_t stream;
  // memory
  bool own_ws;
  char* ws;
  size_t ws_bytes;
  void* kap_s[3];      // storage precision: load-axis, a and b components (alias when isotropic)
  double* kap_hi[3];   // float64 copies when the storage rounds the input, else nullptr
  bool ortho;
  double* src;         // canonical volume source, or nullptr
  double* pin_face;    // Dirichlet values per first/last-layer face ([a][b]), or nullptr
  double* pout_face;
  double* p;
  void *r, *w, *q, *t;
  void *tw_a, *tw_b;
  double* partials;
  int max_partials;
  DevState* st;
  double* hist;
  double* padj;       // adjoint state (want_grad), else nullptr
  void* dlt;          // mixed form: float32 solution increment since the last refinement
  DevState* st_host;  // pinned, one per instance (st_local for a scratch-array plan)
  bool no_alloc;       // plan of etc_solve_static: scratch-array workspace, pageable state mirror
  DevState st_local;
  DctPlan dpa, dpb;
  LaunchCfg lc;
  int nseg;                    // instances in the batch (1 for a single RVE)
  int hstride;                 // residual-history entries per instance
  std::vector<double> kref;    // 5 per instance (load-axis, a, b, in, out)
  double* kref_d;              // device copy
  std::vector<double> lam_lo, lam_hi;
  bool any_done;  // some instance had converged at the last poll (batch plans)
  // host copies of the uploaded tables (kept until the plan ends, so that
  // their asynchronous uploads need no wait)
  std::vector<unsigned char> tw_a_h, tw_b_h;
  bool solved;
  int last_iters;              // max over instances
  int last_status;             // worst over instances
  // captured passes (use_graph): one graph per (solution buffer, Dirichlet
  // pair, whether an instance of the batch has converged: the column
  // transforms launched differ)
  hipStream_t cstream;         // capture/replay stream owned by the plan (or nullptr)
  struct GraphEntry {
    double* p;
    double p_in, p_out;
    bool any_done;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  int tuned;  // 1: launch shapes chosen by the autotuner
  // mixed-size ensemble: one batch plan per distinct shape (groups), all on
  // this plan's stream and solved together by multi-group launches; empty
  // for every other plan
  std::vector<etc_plan*> groups;
  std::vector<int> inst_group, inst_local;  // ensemble instance (input order) -> group, index in it
  std::vector<int> multi_thomas_per;         // persistent tridiagonal blocks per instance of each group
  // kernel timer
  int timer_id;
  std::vector<hipEvent_t> ev;
  int ev_used;
  double timer_ms;
  int timer_launches;
};

namespace {

size_t elt_size(etc_precision prec) { return prec == ETC_MIXED ? sizeof(float) : sizeof(double); }

// Transform lengths with compile-time DCT kernels (the benchmark edge and the
// ensemble edges); any other length runs the run-time-shaped kernels.
template <class T, bool ROWS, class F>
bool ct_dispatch(int, int, F&) {
  return false;
}
template <class T, bool ROWS, class F, int N0, int... Ns>
bool ct_dispatch(int N, int shape, F& f) {
  if (N == N0 && shape == (ROWS ? DctShape<T, N0>::rows : DctShape<T, N0>::cols)) {
    f(std::integral_constant<int, N0>{});
    return true;
  }
  return ct_dispatch<T, ROWS, F, Ns...>(N, shape, f);
}
// Calls f(std::integral_constant<int, NC>) with NC = N if N has compile-time
// kernels whose lines (columns) per block equal `shape`, else with NC = 0.
template <class T, bool ROWS, class F>
void with_ct_len(int N, int shape, F&& f) {
  if (!ct_dispatch<T, ROWS, F, 512, 256, 128, 64, 160, 96, 48>(N, shape, f)) f(std::integral_constant<int, 0>{});
}

// Factor M into the radices of the LDS FFT; false if a prime factor > 5 remains.
bool factor_radices(int M, DctPlan& dp) {
  dp.nst = 0;
  int m = M;
  const int pref[] = {16, 8, 4, 2, 3, 5};
  for (int r : pref) {
    while (m % r == 0 && m >= r) {
      if (dp.nst >= 8) return false;
      dp.R[dp.nst++] = r;
      m /= r;
    }
  }
  return m == 1;
}

DctPlan make_dct_plan(int N) {
  DctPlan dp{};
  dp.N = N;
  dp.M = N / 2;
  dp.fft = 0;
  if (N >= 2 && N % 2 == 0 && factor_radices(N / 2, dp)) dp.fft = 1;
  // lines too long for one pass of a stage even one at a time take the
  // direct route
  if (dp.fft && fft_lines_cap(dp.M, 256) < 1) dp.fft = 0;
  if (dp.fft) {
    dp.lstride = fft_lstride(dp.M);  // complex slots per line
  } else {
    dp.nst = 0;
    dp.lstride = (N + 1) / 2 + 1;  // complex slots holding N reals
  }
  return dp;
}

struct Sizes {
  size_t off_kap_s, off_kap_hi, off_src, off_faces, off_p, off_r, off_w, off_q, off_t, off_tw_a, off_tw_b,
      off_kref, off_part, off_st, off_hist, off_padj, off_dlt, total;
  int max_partials;
};

void canonical_dims(const int64_t n[3], int axis, int& nL, int& na, int& nb) {
  nL = (int)n[axis];
  int o[2], c = 0;
  for (int d = 0; d < 3; ++d)
    if (d != axis) o[c++] = (int)n[d];
  na = o[0];
  nb = o[1];
}

// Stencil launch for plane chunks of `kchunk` (tiles of 64 b x 16 a).
void set_stencil_chunk(LaunchCfg& lc, const Geo& g, int kchunk) {
  const int tbw = lc.stencilTBW;
  const int gx = (g.nb + tbw - 1) / tbw, gy = (g.na + kStencilTAH - 1) / kStencilTAH;
  const int nch = (g.nL + kchunk - 1) / kchunk;
  lc.kchunk = kchunk;
  lc.gridA = dim3(gx, gy, nch * g.nseg);
  lc.nA = gx * gy * nch;
  // the float64-arithmetic residual keeps 64-wide tiles (register footprint)
  const int gx64 = (g.nb + 63) / 64;
  lc.gridRes = dim3(gx64, gy, nch * g.nseg);
  lc.nRes = gx64 * gy * nch;
}

// Variant of the tridiagonal kernel for blocks of tb modes x p partitions
// on a load axis of nL rows: the exact one when every partition has the same
// rows, else the smallest bound that holds them; -1 when none is compiled.
template <class S> int thomas_pick(int tb, int p, int nL) {
  const int Puse = std::max(1, std::min(p, nL / 2));
  const int m = (nL + Puse - 1) / Puse;
  int best = -1;
  for (int i = 0; i < ThomasVariants<S>::n; ++i) {
    const ThomasVariant& v = ThomasVariants<S>::v[i];
    if (v.tb != tb || v.p != p) continue;
    if (v.exact) {
      if (Puse == p && nL == p * v.rows) return i;
    } else if (v.rows >= m && (best < 0 || v.rows < ThomasVariants<S>::v[best].rows)) {
      best = i;
    }
  }
  return best;
}

// Block shape of the tridiagonal kernel by load-axis length, from timings of
// every compiled shape on batches of cubes (the autotuner may pick another):
// 32 x 8 up to 128 rows and at 160 and 256 (8 partitions of 20 or 32 rows),
// 16 x 16 up to 192, 32 x 16 up to 256 and at 512 (16 partitions of 32
// rows), else 32 partitions of 32 (float32) or 16 (float64) modes.
void thomas_default_shape(int nL, size_t elt, int& tb, int& p) {
  if (nL <= 128 || nL == 160 || nL == 256) tb = 32, p = 8;
  else if (nL <= 192) tb = 16, p = 16;
  else if (nL <= 256 || nL == 512) tb = 32, p = 16;
  else tb = elt == 4 ? 32 : 16, p = kThomasP;
}

// Launch shape of the tridiagonal kernel for tb x p blocks; false when no
// variant of that shape holds this load axis.
bool set_thomas(LaunchCfg& lc, const Geo& g, size_t elt, int tb, int p) {
  const int v = elt == 4 ? thomas_pick<float>(tb, p, g.nL) : thomas_pick<double>(tb, p, g.nL);
  if (v < 0) return false;
  lc.tvar = v;
  lc.thomasTB = tb;
  lc.thomasP = p;
  lc.Puse = std::max(1, std::min(p, g.nL / 2));
  lc.maxm = (g.nL + lc.Puse - 1) / lc.Puse;
  lc.thomasTiles = (g.nb + tb - 1) / tb;
  lc.nThomas = lc.thomasTiles * g.na;                // tiles (and partial sums) per instance
  lc.gridThomas = dim3(lc.nThomas, 1, g.nseg);       // capped to the resident blocks at setup
  return true;
}

LaunchCfg make_launch(const Geo& g, const DctPlan& dpa, const DctPlan& dpb, size_t elt, bool ortho) {
  LaunchCfg lc{};
  const size_t cx_sz = 2 * elt;
  const int ns = g.nseg;
  // operator (tiles of stencil_tbw b x kStencilTAH a; the orthotropic
  // kernels keep 64 x 16 and 64 x 4): aim for >= ~2048 blocks over the batch
  // with chunks of at least 16 planes, and go down to 8 planes while there
  // are fewer than 512 (single RVEs up to 128^3: 22 instead of 32 us at
  // 128^3, while 8-plane chunks at 256^3 are no faster)
  lc.stencilTBW = ortho ? 64 : stencil_tbw(elt, g.nb);
  const int gx = (g.nb + lc.stencilTBW - 1) / lc.stencilTBW, gy = (g.na + kStencilTAH - 1) / kStencilTAH;
  const int64_t cols = (int64_t)gx * gy * ns;
  int kchunk = g.nL;
  auto blocks = [&](int kc) { return cols * ((g.nL + kc - 1) / kc); };
  // (never below 8 planes: the partial sums are sized for chunks of 8)
  while ((kchunk > 16 && blocks(kchunk) < 2048) || ((kchunk + 1) / 2 >= 8 && blocks(kchunk) < 512))
    kchunk = (kchunk + 1) / 2;
  set_stencil_chunk(lc, g, kchunk);
  lc.nA_max = ((g.nb + 63) / 64) * gy * ((g.nL + std::min(8, g.nL) - 1) / std::min(8, g.nL));
  {
    const int gy4 = (g.na + 3) / 4;
    int kc4 = g.nL;
    while (kc4 > 8 && (int64_t)gx * gy4 * ns * ((g.nL + kc4 - 1) / kc4) < 4096) kc4 = (kc4 + 1) / 2;
    const int nch4 = (g.nL + kc4 - 1) / kc4;
    lc.kchunkR = kc4;
    lc.gridR = dim3(gx, gy4, nch4 * ns);
    lc.nR = gx * gy4 * nch4;
  }
  // rows (b axis); the same shape rules as the compile-time kernels
  static_assert(kThreads == 256, "row kernels are shaped for 256 threads");
  {
    const size_t line_bytes = (size_t)dpb.lstride * cx_sz;
    int rpb = rows_lines(dpb.M, dpb.lstride, (int)elt, dpb.fft != 0);
    lc.nrows = g.nL * g.na;
    rpb = std::min(rpb, lc.nrows);
    lc.rpb = rpb;
    lc.nRows = (lc.nrows + rpb - 1) / rpb;
    lc.gridRows = dim3(lc.nRows, ns);
    lc.ldsRows = (size_t)rpb * line_bytes;
  }
  // columns (a axis); float32 columns use 512-thread blocks so 32-wide tiles
  // (128-byte rows) still fit one pass per FFT stage
  {
    const size_t line_bytes = (size_t)dpa.lstride * cx_sz;
    lc.colThreads = cols_threads((int)elt);
    int tb = cols_tile(dpa.M, dpa.lstride, (int)elt, dpa.fft != 0);
    tb = std::min(tb, g.nb);
    lc.tb = tb;
    lc.gridCols = dim3((g.nb + tb - 1) / tb, g.nL * ns, 1);
    lc.ldsCols = (size_t)tb * line_bytes;
  }
  // tridiagonal
  {
    int tb = 0, p = 0;
    thomas_default_shape(g.nL, elt, tb, p);
    lc.tvar = -1;  // stays -1 when no compiled variant holds the load axis (setup refuses the plan)
    if (!set_thomas(lc, g, elt, tb, p)) (void)set_thomas(lc, g, elt, elt == 4 ? 32 : 16, kThomasP);
    lc.nThomasMax = ((g.nb + 15) / 16) * g.na;  // no compiled shape has fewer than 16 modes
  }
  int64_t gs = (g.V + kThreads - 1) / kThreads;
  lc.nStride = (int)std::min<int64_t>(gs, std::max<int64_t>(8, kMaxGridStride / ns));
  lc.gridStride = dim3(lc.nStride, ns);
  int64_t gk = (g.plane + kThreads - 1) / kThreads;
  lc.nKeff = (int)std::min<int64_t>(gk, 1024);
  lc.gridKeff = dim3(lc.nKeff, ns);
  // extrema of one instance: about kMaxGridStride blocks, every one a whole
  // tile of plane positions marching over a chunk of the load axis
  {
    const int64_t tiles = (g.plane + kThreads - 1) / kThreads;
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(g.nL, kMaxGridStride / tiles));
    lc.extChunk = (int)((g.nL + nch - 1) / nch);
    lc.gridExt = dim3((unsigned)tiles, (unsigned)((g.nL + lc.extChunk - 1) / lc.extChunk));
    lc.nExt = (int)(lc.gridExt.x * lc.gridExt.y);
  }
  return lc;
}

// Largest number of partial sums any kernel writes per instance.
int max_partials_of(const LaunchCfg& lc) {
  int64_t m = 1024;
  m = std::max<int64_t>(m, lc.nA);
  m = std::max<int64_t>(m, lc.nA_max);
  m = std::max<int64_t>(m, lc.nR);
  m = std::max<int64_t>(m, lc.nRows);
  m = std::max<int64_t>(m, lc.nThomas);
  m = std::max<int64_t>(m, lc.nThomasMax);
  m = std::max<int64_t>(m, (int64_t)lc.nStride * 12);
  m = std::max<int64_t>(m, (int64_t)lc.nKeff * 2);
  m = std::max<int64_t>(m, (int64_t)lc.nExt * 12);
  return (int)m;
}

etc_status validate(const int64_t n[3], int axis, const etc_options& o) {
  if (!n) return fail(ETC_E_INVALID, "n is NULL");
  if (axis < 0 || axis > 2) return fail(ETC_E_INVALID, "axis must be 0, 1 or 2");
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1) return fail(ETC_E_INVALID, "every dimension must be >= 1");
  if (n[axis] < 2) return fail(ETC_E_INVALID, "the load axis needs at least 2 voxels");
  for (int d = 0; d < 3; ++d)
    if (n[d] > (1 << 20)) return fail(ETC_E_UNSUPPORTED, "dimension too large");
  int nL, na, nb;
  canonical_dims(n, axis, nL, na, nb);
  if ((int64_t)na * nb > (int64_t)1 << 31) return fail(ETC_E_UNSUPPORTED, "transverse plane too large");
  if (na > 65535) return fail(ETC_E_UNSUPPORTED, "transverse axis a longer than 65535");
  if (nL > kThomasP * 64) return fail(ETC_E_UNSUPPORTED, "load axis longer than 2048");
  if (o.precision == ETC_MIXED && nL > kThomasP * 16)
    return fail(ETC_E_UNSUPPORTED, "mixed form: load axis longer than 512");
  if (!(o.rtol > 0.0) || !std::isfinite(o.rtol)) return fail(ETC_E_INVALID, "rtol must be > 0");
  if (o.max_iter < 0) return fail(ETC_E_INVALID, "max_iter must be >= 0");
  if (o.precision != ETC_FP64 && o.precision != ETC_MIXED) return fail(ETC_E_INVALID, "bad precision");
  if (o.precond != ETC_PC_DCT && o.precond != ETC_PC_NONE) return fail(ETC_E_INVALID, "bad preconditioner");
  if (o.kref_mode == ETC_KREF_USER)
    for (int i = 0; i < 5; ++i)
      if (!(o.kref_user[i] > 0.0) || !std::isfinite(o.kref_user[i]))
        return fail(ETC_E_INVALID, "kref_user entries must be finite and > 0");
  for (int d = 0; d < 3; ++d)
    if (o.L[d] < 0.0 || !std::isfinite(o.L[d])) return fail(ETC_E_INVALID, "L must be >= 0");
  const bool anyL = o.L[0] != 0.0 || o.L[1] != 0.0 || o.L[2] != 0.0;
  if (anyL && !(o.L[0] > 0.0 && o.L[1] > 0.0 && o.L[2] > 0.0))
    return fail(ETC_E_INVALID, "L must be all zero or all positive");
  return ETC_OK;
}

struct ProblemShape {
  bool ortho, src, faces;
};

// Geometry of one instance (nseg instances of it in a batch).
Geo make_geo(const int64_t n[3], int axis, int nseg) {
  int nL, na, nb;
  canonical_dims(n, axis, nL, na, nb);
  Geo g{};
  g.nL = nL;
  g.na = na;
  g.nb = nb;
  g.plane = (int64_t)na * nb;
  g.V = g.plane * nL;
  g.nseg = nseg;
  return g;
}

Sizes plan_sizes(const int64_t n[3], int axis, etc_dtype dt, const etc_options& o, ProblemShape ps, int nseg) {
  const Geo g = make_geo(n, axis, nseg);
  const int na = g.na, nb = g.nb;
  const size_t es = elt_size(o.precision);
  DctPlan dpa = make_dct_plan(na), dpb = make_dct_plan(nb);
  LaunchCfg lc = make_launch(g, dpa, dpb, es, ps.ortho);
  Sizes s{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o2 = off;
    off += align_up(bytes);
    return o2;
  };
  const size_t V = (size_t)g.V * nseg;  // every volume array holds the whole batch
  const int ncomp = ps.ortho ? 3 : 1;
  s.off_kap_s = take(ncomp * V * es);
  s.off_kap_hi = take((o.precision == ETC_MIXED && dt == ETC_F64) ? ncomp * V * sizeof(double) : 0);
  s.off_src = take(ps.src ? V * sizeof(double) : 0);
  s.off_faces = take(ps.faces ? 2 * (size_t)g.plane * sizeof(double) : 0);
  s.off_p = take(V * sizeof(double));
  s.off_r = take(V * es);
  s.off_w = take(V * es);
  s.off_q = take(V * es);
  s.off_t = take(V * es);
  s.off_tw_a = take((size_t)4 * na * 2 * es);
  s.off_tw_b = take((size_t)4 * nb * 2 * es);
  s.off_kref = take((size_t)5 * nseg * sizeof(double));
  s.max_partials = max_partials_of(lc);
  s.off_part = take((size_t)s.max_partials * nseg * sizeof(double));
  s.off_st = take(sizeof(DevState) * nseg);
  s.off_hist = take((size_t)(o.max_iter + 2) * nseg * sizeof(double));
  s.off_padj = take(o.want_grad ? V * sizeof(double) : 0);
  s.off_dlt = take(o.precision == ETC_MIXED ? V * sizeof(float) : 0);
  s.total = off;
  return s;
}

template <class T> void fill_twiddles(std::vector<cx<T>>& tw, int N) {
  tw.resize((size_t)4 * N);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < 4 * N; ++j) {
    const long double ang = -2.0L * pi * (long double)j / (4.0L * (long double)N);
    tw[j].re = (T)std::cos(ang);
    tw[j].im = (T)std::sin(ang);
  }
}

// ------------------------------------------------------------------ launches
template <class S> struct Ops {
  using T = S;

  static Kap<S> kap(const etc_plan* P) {
    Kap<S> k;
    k.L = (const S*)P->kap_s[0];
    k.A = (const S*)P->kap_s[1];
    k.B = (const S*)P->kap_s[2];
    k.hL = P->kap_hi[0];
    k.hA = P->kap_hi[1];
    k.hB = P->kap_hi[2];
    return k;
  }

  static Rhs rhs(const etc_plan* P) { return Rhs{P->src, P->pin_face, P->pout_face}; }

  // canonical copy of one instance of a user-layout array (dtype In)
  template <class In, class Out>
  static etc_status canon_one(etc_plan* P, const In* src, Out* dst, double* dst_hi) {
    Geo g = P->g;
    g.nseg = 1;
    if (P->axis == 2) {
      dim3 grid((g.nL + 31) / 32, (g.nb + 31) / 32, g.na);
      k_canon_axis2<In, Out><<<grid, dim3(32, 8), 0, P->stream>>>(src, dst, dst_hi, g);
    } else {
      k_canon_rows<In, Out><<<P->lc.nStride, kThreads, 0, P->stream>>>(src, dst, dst_hi, P->axis, g);
    }
    LAUNCHCHK("canon");
    return ETC_OK;
  }

  // Canonical copies of instance `inst` (conductivity components, source)
  // and its family extrema into the first 12 * nExt partials.
  // inst_src: this instance's own conductivity array (isotropic batches
  // whose instances are not back to back), else nullptr
  static etc_status canon(etc_plan* P, const void* const comp_user[3], const double* source, int inst,
                          const void* inst_src = nullptr) {
    const int64_t off = (int64_t)inst * P->g.V;
    const size_t in_es = (P->in_dt == ETC_F64) ? sizeof(double) : sizeof(float);
    for (int c = 0; c < (P->ortho ? 3 : 1); ++c) {
      const char* src = inst_src ? (const char*)inst_src : (const char*)comp_user[c] + (size_t)off * in_es;
      S* dst = (S*)P->kap_s[c] + off;
      double* dhi = P->kap_hi[c] ? P->kap_hi[c] + off : nullptr;
      etc_status s = (P->in_dt == ETC_F64) ? canon_one<double, S>(P, (const double*)src, dst, dhi)
                                           : canon_one<float, S>(P, (const float*)src, dst, dhi);
      if (s) return s;
    }
    if (source) {
      etc_status s = canon_one<double, double>(P, source + off, P->src + off, nullptr);
      if (s) return s;
    }
    Kap<S> k = kap(P);
    k.L += off;
    k.A += off;
    k.B += off;
    if (k.hL) k.hL += off;
    if (k.hA) k.hA += off;
    if (k.hB) k.hB += off;
    Geo g = P->g;
    g.nseg = 1;
    k_extrema<S><<<P->lc.gridExt, kThreads, 0, P->stream>>>(g, k, P->partials, P->lc.extChunk);
    LAUNCHCHK("extrema");
    return ETC_OK;
  }

  // Dynamic LDS above 64 KiB must be requested per kernel (gfx950 has 160 KiB
  // per CU): the run-time-shaped kernels and the compile-time ones of this length.
  static etc_status lds_limits(etc_plan* P) {
    const int cols = (int)P->lc.ldsCols, rows = (int)P->lc.ldsRows;
    hipError_t e = hipSuccess;
    auto set = [&](const void* fn, int bytes) {
      if (e == hipSuccess) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    };
    if (cols > 65536) {
      auto f = [&](auto nc) {
        constexpr int NC = decltype(nc)::value;
        set((const void*)&k_cols<S, T, -1, NC>, cols);
        set((const void*)&k_cols<S, T, +1, NC>, cols);
      };
      f(std::integral_constant<int, 0>{});
      with_ct_len<T, false>(P->dpa.N, P->lc.tb, f);
    }
    with_cols_pf(P, [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      set((const void*)&k_cols_pf<S, T, -1, NC>, ColsPf<T, NC>::bytes);
      set((const void*)&k_cols_pf<S, T, +1, NC>, ColsPf<T, NC>::bytes);
    });
    if (rows > 65536) {
      auto f = [&](auto nc) {
        constexpr int NC = decltype(nc)::value;
        set((const void*)&k_rows_fwd<S, T, 0, NC>, rows);
        set((const void*)&k_rows_fwd<S, T, 1, NC>, rows);
        set((const void*)&k_rows_inv<S, T, 0, NC>, rows);
        set((const void*)&k_rows_inv<S, T, 1, NC>, rows);
      };
      f(std::integral_constant<int, 0>{});
      with_ct_len<T, true>(P->dpb.N, P->lc.rpb, f);
    }
    if (e != hipSuccess) return fail(ETC_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    return ETC_OK;
  }

  // DCT launches: compile-time kernels for the common lengths, else the
  // run-time-shaped ones.
  template <int MODE>
  static void rows_fwd(etc_plan* P, const S* src, S* dst, S* r, const S* q, double* partials, const DevState* st,
                       int gate) {
    const LaunchCfg& lc = P->lc;
    const cx<T>* twb = (const cx<T>*)P->tw_b;
    with_ct_len<T, true>(P->dpb.N, lc.rpb, [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      k_rows_fwd<S, T, MODE, NC><<<lc.gridRows, kThreads, lc.ldsRows, P->stream>>>(
          P->g, P->dpb, twb, src, dst, lc.rpb, lc.nrows, r, q, partials, st, gate);
    });
  }
  template <int MODE>
  static void rows_inv(etc_plan* P, const S* src, S* dst, S* x, const DevState* st, int gate) {
    const LaunchCfg& lc = P->lc;
    const cx<T>* twb = (const cx<T>*)P->tw_b;
    with_ct_len<T, true>(P->dpb.N, lc.rpb, [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      k_rows_inv<S, T, MODE, NC><<<lc.gridRows, kThreads, lc.ldsRows, P->stream>>>(P->g, P->dpb, twb, src, dst,
                                                                                 lc.rpb, lc.nrows, x, st, gate);
    });
  }
  // Calls f(std::integral_constant<int, NC>) when the plan's column
  // transforms can run the persistent kernel: a compile-time length, whole
  // tiles, and the twiddles fitting beside two tiles per CU.
  template <class F>
  static void with_cols_pf(const etc_plan* P, F&& f) {
    if (P->g.plane >= ((int64_t)1 << 31) || P->g.nb % P->lc.tb != 0) return;
    with_ct_len<T, false>(P->dpa.N, P->lc.tb, [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      if constexpr (NC > 0) {
        using Sh = DctShape<T, NC>;
        constexpr int NT = Sh::col_threads, VW = 16 / (int)sizeof(S);
        if constexpr ((Sh::cols * NC) % NT == 0 && NT % Sh::cols == 0 && Sh::M % 2 == 0 &&
                      (Sh::cols * (Sh::M / 2)) % NT == 0 && Sh::cols % VW == 0 &&
                      NC % (NT / (Sh::cols / VW)) == 0 && 2 * ColsPf<T, NC>::bytes <= 160 * 1024)
          f(nc);
      }
    });
  }

  template <int DIR>
  static void cols(etc_plan* P, S* t, const DevState* st, int gate) {
    const LaunchCfg& lc = P->lc;
    const cx<T>* twa = (const cx<T>*)P->tw_a;
    // A batch runs the persistent kernel only while no instance had
    // converged at the last poll, and without its exit test: it cannot skip
    // the tiles of one instance and keep the same stores per tile, and
    // transforming the scratch rows of an instance that has just converged
    // changes nothing it still uses.  Refinement-only launches keep the
    // gated kernel.
    const bool single = P->g.nseg == 1;
    if (lc.colsPers > 0 && (single || (gate <= 1 && !P->any_done))) {
      bool done = false;
      with_cols_pf(P, [&](auto nc) {
        constexpr int NC = decltype(nc)::value;
        const int ntx = (int)lc.gridCols.x, ntiles = (int)(lc.gridCols.x * lc.gridCols.y);
        k_cols_pf<S, T, DIR, NC><<<lc.colsPers, lc.colThreads, ColsPf<T, NC>::bytes, P->stream>>>(
            P->g, twa, t, ntx, ntiles, single ? st : nullptr, single ? gate : 0);
        done = true;
      });
      if (done) return;
    }
    with_ct_len<T, false>(P->dpa.N, lc.tb, [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      k_cols<S, T, DIR, NC><<<lc.gridCols, lc.colThreads, lc.ldsCols, P->stream>>>(P->g, P->dpa, twa, t, lc.tb, st,
                                                                                  gate);
    });
  }

  static RefMedium ref(const etc_plan* P) {
    RefMedium rm;
    rm.kref = P->kref_d;
    rm.step_a = 1.5707963267948966 / (double)P->g.na;
    rm.step_b = 1.5707963267948966 / (double)P->g.nb;
    rm.dot_scale = 4.0 / ((double)P->g.na * (double)P->g.nb);
    return rm;
  }

  // Tridiagonal kernel of this plan's variant (block shape and partition rows).
  template <class F>
  static void with_thomas(const LaunchCfg& lc, F&& f) {
    with_thomas_variant<S>(lc.tvar, [&](auto ic) {
      constexpr ThomasVariant v = ThomasVariants<S>::v[decltype(ic)::value];
      f(&k_thomas<S, v.tb, v.p, v.rows, v.exact>);
    });
  }

  // Setup-time autotuner: time the stencil for plane chunks of 8 .. nL and
  // the tridiagonal kernel for every compiled block shape that holds the load
  // axis, each with persistent grids of 1x and 2x the resident blocks and
  // one block per tile, on this plan's own buffers, and keep the fastest of
  // each (cached per problem shape for the process).
  struct Tuned {
    int kchunk, thomas_tb, thomas_p, thomas_x;
  };
  static etc_status autotune(etc_plan* P) {
    // shared by every plan of the process (plans may be set up from several threads)
    static std::mutex mu;
    static std::vector<std::pair<std::vector<int64_t>, Tuned>> cache;
    LaunchCfg& lc = P->lc;
    const Geo& g = P->g;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const std::vector<int64_t> key = {dev, g.nL, g.na, g.nb, P->nseg, (int64_t)sizeof(S), P->ortho ? 1 : 0,
                                      P->opt.thomas_modes, P->opt.thomas_parts};
    {
      std::lock_guard<std::mutex> lock(mu);
      for (auto& e : cache)
        if (e.first == key) {
          set_stencil_chunk(lc, g, e.second.kchunk);
          if (!set_thomas(lc, g, sizeof(S), e.second.thomas_tb, e.second.thomas_p))
            return fail(ETC_E_UNSUPPORTED, "autotune: cached tridiagonal shape no longer valid");
          lc.gridThomas.x = e.second.thomas_x;
          P->tuned = 1;
          return ETC_OK;
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    etc_status s = ETC_OK;
    auto time_it = [&](auto&& launch) -> float {
      launch();
      (void)hipEventRecord(e0, P->stream);
      for (int i = 0; i < 3; ++i) launch();
      (void)hipEventRecord(e1, P->stream);
      float ms = 0.0f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 1e30f;
      return ms;
    };
    const size_t vb = (size_t)g.V * P->nseg * sizeof(S);
    if (hipMemsetAsync(P->w, 0, vb, P->stream) != hipSuccess || hipMemsetAsync(P->t, 0, vb, P->stream) != hipSuccess)
      s = fail(ETC_E_HIP, "autotune: memset failed");
    // stencil chunk
    Tuned best{lc.kchunk, lc.thomasTB, lc.thomasP, (int)lc.gridThomas.x};
    if (!s) {
      float tbest = 1e30f;
      for (int kc = std::min(8, g.nL);; kc *= 2) {
        const int kcc = std::min(kc, g.nL);
        set_stencil_chunk(lc, g, kcc);
        if (lc.gridA.z <= 65535) {
          const float ms = time_it([&] { (void)apply_A_launch(P, (const S*)P->w, (S*)P->q, nullptr, nullptr, 0); });
          if (ms < tbest) {
            tbest = ms;
            best.kchunk = kcc;
          }
        }
        if (kcc >= g.nL) break;
      }
      set_stencil_chunk(lc, g, best.kchunk);
    }
    // tridiagonal block shape and grid
    if (!s) {
      float tbest = 1e30f;
      std::vector<std::pair<int, int>> shapes;
      for (const ThomasVariant& v : ThomasVariants<S>::v)
        if (std::find(shapes.begin(), shapes.end(), std::make_pair(v.tb, v.p)) == shapes.end())
          shapes.push_back({v.tb, v.p});
      const bool fixed = P->opt.thomas_modes || P->opt.thomas_parts;
      for (const auto& sh : shapes) {
        if (fixed && sh != std::make_pair(P->opt.thomas_modes, P->opt.thomas_parts)) continue;
        if (!set_thomas(lc, g, sizeof(S), sh.first, sh.second)) continue;
        if ((s = thomas_grid(P))) break;
        const int resident = (int)lc.gridThomas.x;
        const int cands[3] = {resident, std::min(lc.nThomas, 2 * resident), lc.nThomas};
        for (int c : cands) {
          lc.gridThomas.x = c;
          const float ms = time_it([&] { (void)thomas(P, (S*)P->t, nullptr, nullptr, 0); });
          if (ms < tbest) {
            tbest = ms;
            best.thomas_tb = sh.first;
            best.thomas_p = sh.second;
            best.thomas_x = c;
          }
        }
      }
      if (!set_thomas(lc, g, sizeof(S), best.thomas_tb, best.thomas_p) && !s)
        s = fail(ETC_E_UNSUPPORTED, "autotune: no tridiagonal shape");
      lc.gridThomas.x = best.thomas_x;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    HIPCHK(hipGetLastError());
    {
      std::lock_guard<std::mutex> lock(mu);
      cache.push_back({key, best});
    }
    P->tuned = 1;
    return ETC_OK;
  }

  // Persistent grid of the column kernels: the blocks that fit on
  // the device at once (both directions), at most one per tile.
  static etc_status cols_grid(etc_plan* P) {
    LaunchCfg& lc = P->lc;
    lc.colsPers = 0;
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipError_t e = hipSuccess;
    int occ = 0;
    with_cols_pf(P, [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      int o1 = 0, o2 = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o1, (const void*)&k_cols_pf<S, T, -1, NC>, lc.colThreads,
                                                       ColsPf<T, NC>::bytes);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o2, (const void*)&k_cols_pf<S, T, +1, NC>, lc.colThreads,
                                                         ColsPf<T, NC>::bytes);
      occ = std::min(o1, o2);
    });
    if (e != hipSuccess) return fail(ETC_E_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
    if (occ > 0) {
      const int64_t ntiles = (int64_t)lc.gridCols.x * lc.gridCols.y;
      lc.colsPers = (int)std::min<int64_t>(ntiles, (int64_t)cus * occ);
    }
    return ETC_OK;
  }

  // Persistent grid of the tridiagonal kernel: the blocks that fit on the device at once.
  static etc_status thomas_grid(etc_plan* P) {
    LaunchCfg& lc = P->lc;
    int dev = 0, cus = 0, occ = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipError_t e = hipSuccess;
    with_thomas(lc, [&](auto fn) {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)fn, lc.thomasTB * lc.thomasP, 0);
    });
    if (e != hipSuccess) return fail(ETC_E_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
    const int ns = P->nseg;
    const int resident = std::max(1, cus * std::max(1, occ));
    const int per = std::max(1, std::min(lc.nThomas, (resident + ns - 1) / ns));
    lc.gridThomas = dim3(per, 1, ns);
    return ETC_OK;
  }

  static etc_status thomas(etc_plan* P, S* t, double* partials, const DevState* st, int gate) {
    const LaunchCfg& lc = P->lc;
    const RefMedium rm = ref(P);
    const int threads = lc.thomasTB * lc.thomasP;
    if (lc.tvar < 0 || lc.tvar >= ThomasVariants<S>::n) return fail(ETC_E_UNSUPPORTED, "no tridiagonal variant");
    with_thomas(lc, [&](auto fn) {
      fn<<<lc.gridThomas, threads, 0, P->stream>>>(P->g, rm, t, lc.Puse, partials, st, gate, lc.thomasTiles,
                                                   lc.nThomas);
    });
    LAUNCHCHK("thomas");
    return ETC_OK;
  }

  // finalize over every instance: n partials each, `pstride` apart
  static etc_status fin(etc_plan* P, int op, int n, int64_t pstride, const double* partials = nullptr) {
    k_fin<<<P->nseg, 1024, 0, P->stream>>>(op, partials ? partials : P->partials, n, pstride, P->st, P->hist,
                                           P->hstride);
    LAUNCHCHK("finalize");
    return ETC_OK;
  }

  static void timer_begin(etc_plan* P, int id) {
    if (P->timer_id == id && P->ev_used + 2 <= (int)P->ev.size()) (void)hipEventRecord(P->ev[P->ev_used], P->stream);
  }
  static void timer_end(etc_plan* P, int id) {
    if (P->timer_id == id && P->ev_used + 2 <= (int)P->ev.size()) {
      (void)hipEventRecord(P->ev[P->ev_used + 1], P->stream);
      P->ev_used += 2;
    }
  }

  // Preconditioner of the initial pass (and of etc_apply_Minv):
  // t = DCT_b(src); t = DCT_a(t); Thomas; t = DCT_a^{-1}(t); dst = DCT_b^{-1}(t).
  static etc_status precond(etc_plan* P, const S* src, S* dst, const DevState* st, int gate,
                            int fin_op) {
    const LaunchCfg& lc = P->lc;
    S* t = (S*)P->t;
    rows_fwd<0>(P, src, t, nullptr, nullptr, nullptr, st, gate);
    LAUNCHCHK("rows_fwd");
    cols<-1>(P, t, st, gate);
    LAUNCHCHK("cols_fwd");
    etc_status s = thomas(P, t, P->partials, st, gate);
    if (s) return s;
    s = fin(P, fin_op, lc.nThomas, lc.nThomas);
    if (s) return s;
    cols<+1>(P, t, st, gate);
    LAUNCHCHK("cols_inv");
    rows_inv<0>(P, t, dst, nullptr, st, gate);
    LAUNCHCHK("rows_inv");
    return ETC_OK;
  }

  // Initial pass: p = p0 (or 0), r = b - A p, z = M^{-1} r, w = z, rho = r.z.
  static etc_status init(etc_plan* P, const double* p0_user) {
    const LaunchCfg& lc = P->lc;
    const Geo& g = P->g;
    S* r = (S*)P->r;
    S* w = (S*)P->w;
    k_init<S><<<lc.gridStride, kThreads, 0, P->stream>>>(g, P->p, r, kap(P), rhs(P), (S*)P->dlt, P->partials);
    LAUNCHCHK("init");
    etc_status s = fin(P, FIN_BNORM, lc.nStride, lc.nStride);
    if (s) return s;
    if (p0_user) {
      // canonical copy of p0 into p (double), then r = b - A p0
      for (int inst = 0; inst < P->nseg; ++inst) {
        s = canon_one<double, double>(P, p0_user + (int64_t)inst * g.V, P->p + (int64_t)inst * g.V, nullptr);
        if (s) return s;
      }
      s = residual(P, r, nullptr, 0);
      if (s) return s;
      // relative residual of the warm start
      if ((s = fin(P, FIN_RR0, residual_parts(P), residual_parts(P)))) return s;
    }
    if (P->opt.precond == ETC_PC_NONE) {
      k_norm2<S><<<lc.gridStride, kThreads, 0, P->stream>>>(g, r, P->partials, P->st);
      LAUNCHCHK("norm2");
      if ((s = fin(P, FIN_RHO0, lc.nStride, lc.nStride))) return s;
      k_dir_plain<S><<<lc.gridStride, kThreads, 0, P->stream>>>(g, r, w, P->st, 1);
      LAUNCHCHK("dir");
      return ETC_OK;
    }
    return precond(P, r, w, P->st, 1, FIN_RHO0);
  }

  // The vector the update step accumulates into: p (FP64) or the float32
  // increment (mixed).
  static S* xsol(etc_plan* P) { return P->dlt ? (S*)P->dlt : (S*)(void*)P->p; }

  // fold the float32 increment (and, with_w, this pass's alpha w) into p
  static etc_status flush(etc_plan* P, bool with_w) {
    k_flush<<<P->lc.gridStride, kThreads, 0, P->stream>>>(P->g, P->p, (float*)P->dlt,
                                                           with_w ? (const float*)P->w : nullptr, P->st);
    LAUNCHCHK("flush");
    return ETC_OK;
  }

  // the solution update a pass that stopped at its residual test left undone
  static etc_status fixup(etc_plan* P) {
    k_fixup<S><<<P->lc.gridStride, kThreads, 0, P->stream>>>(P->g, xsol(P), (const S*)P->w, P->st);
    LAUNCHCHK("fixup");
    return ETC_OK;
  }

  // One pass of plain CG (z = r).
  static etc_status iteration_plain(etc_plan* P) {
    const LaunchCfg& lc = P->lc;
    const Geo& g = P->g;
    S* r = (S*)P->r;
    S* w = (S*)P->w;
    S* q = (S*)P->q;
    etc_status s;
    if ((s = apply_A_launch(P, w, q, P->partials, P->st, 1))) return s;
    if ((s = fin(P, FIN_ALPHA, lc.nA, lc.nA))) return s;
    k_update_plain<S><<<lc.gridStride, kThreads, 0, P->stream>>>(g, xsol(P), w, r, q, P->partials, P->st);
    LAUNCHCHK("update");
    if ((s = fin(P, FIN_RR, lc.nStride, lc.nStride))) return s;
    if (P->prec == ETC_MIXED) {
      if ((s = flush(P, false))) return s;
      if ((s = residual(P, r, P->st, 2))) return s;
      if ((s = fin(P, FIN_REFINE, residual_parts(P), residual_parts(P)))) return s;
    }
    k_norm2<S><<<lc.gridStride, kThreads, 0, P->stream>>>(g, r, P->partials, P->st);
    LAUNCHCHK("norm2");
    if ((s = fin(P, FIN_BETA, lc.nStride, lc.nStride))) return s;
    k_dir_plain<S><<<lc.gridStride, kThreads, 0, P->stream>>>(g, r, w, P->st, 0);
    LAUNCHCHK("dir");
    return ETC_OK;
  }

  // One PCG pass (alg:pcg loop body) on the device.
  static etc_status iteration(etc_plan* P) {
    if (P->opt.precond == ETC_PC_NONE) return iteration_plain(P);
    const LaunchCfg& lc = P->lc;
    S* r = (S*)P->r;
    S* w = (S*)P->w;
    S* q = (S*)P->q;
    S* t = (S*)P->t;
    etc_status s;
    // q = A w, alpha = rho / (w . q)
    timer_begin(P, 1);
    s = apply_A_launch(P, w, q, P->partials, P->st, 1);
    timer_end(P, 1);
    if (s) return s;
    if ((s = fin(P, FIN_ALPHA, lc.nA, lc.nA))) return s;
    // r -= alpha q, ||r||^2, t = DCT_b(r)
    timer_begin(P, 2);
    rows_fwd<1>(P, nullptr, t, r, q, P->partials, P->st, 1);
    timer_end(P, 2);
    LAUNCHCHK("update_rows_fwd");
    if ((s = fin(P, FIN_RR, lc.nRows, lc.nRows))) return s;
    if (P->prec == ETC_MIXED) {
      // fold the increment and alpha w into p, replace r by the float64 true
      // residual when requested, and redo DCT_b
      if ((s = flush(P, true))) return s;
      if ((s = residual(P, r, P->st, 2))) return s;
      if ((s = fin(P, FIN_REFINE, residual_parts(P), residual_parts(P)))) return s;
      rows_fwd<0>(P, r, t, nullptr, nullptr, nullptr, P->st, 2);
      LAUNCHCHK("rows_fwd_refine");
    }
    timer_begin(P, 3);
    cols<-1>(P, t, P->st, 1);
    timer_end(P, 3);
    LAUNCHCHK("cols_fwd");
    timer_begin(P, 4);
    s = thomas(P, t, P->partials, P->st, 1);
    timer_end(P, 4);
    if (s) return s;
    if ((s = fin(P, FIN_BETA, lc.nThomas, lc.nThomas))) return s;
    timer_begin(P, 5);
    cols<+1>(P, t, P->st, 1);
    timer_end(P, 5);
    LAUNCHCHK("cols_inv");
    // w = DCT_b^{-1}(t) + beta w
    timer_begin(P, 6);
    rows_inv<1>(P, t, w, xsol(P), P->st, 1);
    timer_end(P, 6);
    LAUNCHCHK("rows_inv_dir");
    return ETC_OK;
  }

  static etc_status keff(etc_plan* P, bool energy) {
    const LaunchCfg& lc = P->lc;
    k_keff<S><<<lc.gridKeff, kThreads, 0, P->stream>>>(P->g, P->p, kap(P), rhs(P), P->partials);
    LAUNCHCHK("keff");
    etc_status s;
    if ((s = fin(P, FIN_ACC0, lc.nKeff, 2 * lc.nKeff))) return s;
    if ((s = fin(P, FIN_ACC1, lc.nKeff, 2 * lc.nKeff, P->partials + lc.nKeff))) return s;
    if (energy) {
      k_energy<S><<<lc.gridStride, kThreads, 0, P->stream>>>(P->g, P->p, kap(P), rhs(P), P->partials);
      LAUNCHCHK("energy");
      if ((s = fin(P, FIN_ACC2, lc.nStride, lc.nStride))) return s;
    }
    return ETC_OK;
  }

  template <class O>
  static etc_status grad(etc_plan* P, O* out_user, double c) {
    k_grad<S, O><<<P->lc.gridStride, kThreads, 0, P->stream>>>(P->g, P->p, P->padj, kap(P), c, P->axis, out_user);
    LAUNCHCHK("grad");
    return ETC_OK;
  }

  static etc_status apply_A_launch(etc_plan* P, const S* x, S* y, double* partials, const DevState* st, int gate) {
    const LaunchCfg& lc = P->lc;
    if (P->ortho)
      k_apply_A<S, S, true><<<lc.gridA, dim3(64, 4), 0, P->stream>>>(P->g, x, kap(P), y, partials, st, gate, lc.kchunk);
    else {
      auto launch = [&](auto tbw) {
        constexpr int TBW = decltype(tbw)::value;
        k_apply_A_iso<S, false, S, TBW, kStencilTAH><<<lc.gridA, dim3(TBW, kStencilTAH / 4), 0, P->stream>>>(
            P->g, x, kap(P), (const S*)P->kap_s[0], rhs(P), y, partials, st, gate, lc.kchunk);
      };
      if constexpr (sizeof(S) == 4) {
        if (lc.stencilTBW == 128) launch(std::integral_constant<int, 128>{});
        else launch(std::integral_constant<int, 64>{});
      } else {
        launch(std::integral_constant<int, 64>{});
      }
    }
    LAUNCHCHK("apply_A");
    return ETC_OK;
  }

  // partial sums the residual kernel writes per instance
  static int residual_parts(const etc_plan* P) { return P->ortho ? P->lc.nR : P->lc.nRes; }

  static etc_status residual(etc_plan* P, S* r, const DevState* st, int gate) {
    const LaunchCfg& lc = P->lc;
    if (P->ortho)
      k_residual<S, true><<<lc.gridR, dim3(64, 4), 0, P->stream>>>(P->g, P->p, kap(P), rhs(P), r, P->partials, st, gate,
                                                                   lc.kchunkR);
    else {
      // kappa at its input precision (the float64 copy of a float64 input);
      // without a source and face data b needs no reads of its own
      const bool plain = !P->src && !P->pin_face && !P->pout_face;
      auto launch = [&](auto pl, const auto* ks) {
        using KT = typename std::remove_cv<typename std::remove_pointer<decltype(ks)>::type>::type;
        k_apply_A_iso<S, true, KT, 64, kStencilTAH, decltype(pl)::value>
            <<<lc.gridRes, dim3(64, kStencilTAH / 4), 0, P->stream>>>(P->g, P->p, kap(P), ks, rhs(P), r, P->partials,
                                                                      st, gate, lc.kchunk);
      };
      if (const double* hi = P->kap_hi[0]) {
        if (plain) launch(std::true_type{}, hi);
        else launch(std::false_type{}, hi);
      } else {
        const S* ks = (const S*)P->kap_s[0];
        if (plain) launch(std::true_type{}, ks);
        else launch(std::false_type{}, ks);
      }
    }
    LAUNCHCHK("residual");
    return ETC_OK;
  }

  static etc_status apply_A(etc_plan* P, const void* x, void* y, bool dot) {
    const LaunchCfg& lc = P->lc;
    etc_status s = apply_A_launch(P, (const S*)x, (S*)y, dot ? P->partials : nullptr, nullptr, 0);
    if (s) return s;
    if (dot) return fin(P, FIN_ACC3, lc.nA, lc.nA);
    return ETC_OK;
  }

  // ------------------------------------------ multi-group (ensemble) passes
  // Every kernel of a pass is launched once for all groups of an ensemble
  // plan E; group gi's blocks follow group gi-1's in the flat grid.
  static void add_group(GroupMap& gm, int gi, dim3 grid, unsigned& total) {
    gm.start[gi] = total;
    gm.grid[gi] = grid;
    total += grid.x * grid.y * grid.z;
    gm.ng = gi + 1;
    gm.start[gi + 1] = total;
  }
  // compile-time length a group's transforms run in a multi-group launch
  // (0: the run-time-shaped kernel)
  static int nc_rows(const etc_plan* P) {
    int v = 0;
    with_ct_len<T, true>(P->dpb.N, P->lc.rpb, [&](auto nc) { v = decltype(nc)::value; });
    return multi_nc(v) ? v : 0;
  }
  static int nc_cols(const etc_plan* P) {
    int v = 0;
    with_ct_len<T, false>(P->dpa.N, P->lc.tb, [&](auto nc) { v = decltype(nc)::value; });
    return multi_nc(v) ? v : 0;
  }
  // Launch set-up of an ensemble solve: dynamic LDS limits of the
  // multi-group transforms and the persistent blocks of the tridiagonal
  // kernel per group.
  static etc_status multi_prepare(etc_plan* E) {
    // Each group keeps the persistent grid it would have alone (blocks per
    // instance filling the device): on the 64-RVE GRF ensemble (edges
    // 48-160) that ran faster than one block per tile, or than the device's
    // resident blocks shared out in proportion to each group's rows
    // (139 against 123 RVEs/s, timed with 32 partitions per line in every
    // group).
    E->multi_thomas_per.clear();
    for (const etc_plan* P : E->groups) E->multi_thomas_per.push_back((int)P->lc.gridThomas.x);
    return multi_lds(E);
  }

  static etc_status multi_lds(const etc_plan* E) {
    size_t rows = 0, cols = 0;
    for (const etc_plan* P : E->groups) {
      rows = std::max(rows, P->lc.ldsRows);
      cols = std::max(cols, P->lc.ldsCols);
    }
    hipError_t e = hipSuccess;
    auto set = [&](const void* fn, size_t bytes) {
      if (e == hipSuccess && bytes > 65536) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    };
    set((const void*)&k_rows_fwd_multi<S, T, 0>, rows);
    set((const void*)&k_rows_fwd_multi<S, T, 1>, rows);
    set((const void*)&k_rows_inv_multi<S, T, 1>, rows);
    set((const void*)&k_cols_multi<S, T, -1>, cols);
    set((const void*)&k_cols_multi<S, T, +1>, cols);
    if (e != hipSuccess) return fail(ETC_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    return ETC_OK;
  }

  static etc_status stencil_multi(etc_plan* E) {
    GroupMap gm{};
    StencilMulti<S, S, S> m{};
    unsigned tot = 0;
    for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
      etc_plan* P = E->groups[gi];
      add_group(gm, gi, P->lc.gridA, tot);
      m.a[gi] = StencilArgs<S, S, S>{P->g, (const S*)P->w, kap(P), (const S*)P->kap_s[0], rhs(P), (S*)P->q,
                                     P->partials, P->st, P->lc.kchunk};
    }
    // one tile width for all groups (etc_setup_ensemble makes them agree)
    auto launch = [&](auto tbw) {
      constexpr int TBW = decltype(tbw)::value;
      k_apply_A_iso_multi<S, false, S, TBW, kStencilTAH><<<tot, dim3(TBW, kStencilTAH / 4), 0, E->stream>>>(gm, m, 1);
    };
    if constexpr (sizeof(S) == 4) {
      if (E->groups[0]->lc.stencilTBW == 128) launch(std::integral_constant<int, 128>{});
      else launch(std::integral_constant<int, 64>{});
    } else {
      launch(std::integral_constant<int, 64>{});
    }
    LAUNCHCHK("apply_A_multi");
    return ETC_OK;
  }

  // mixed form: r = b - A p in float64 arithmetic where a refinement is due
  template <class KT>
  static etc_status residual_multi_kt(etc_plan* E) {
    GroupMap gm{};
    StencilMulti<S, double, KT> m{};
    unsigned tot = 0;
    for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
      etc_plan* P = E->groups[gi];
      add_group(gm, gi, P->lc.gridRes, tot);
      const KT* ks = std::is_same<KT, double>::value ? (const KT*)(const void*)P->kap_hi[0] : (const KT*)P->kap_s[0];
      m.a[gi] = StencilArgs<S, double, KT>{P->g, P->p, kap(P), ks, rhs(P), (S*)P->r, P->partials, P->st, P->lc.kchunk};
    }
    bool plain = true;  // no group has a source or face data
    for (etc_plan* P : E->groups) plain = plain && !P->src && !P->pin_face && !P->pout_face;
    if (plain)
      k_apply_A_iso_multi<S, true, KT, 64, kStencilTAH, true><<<tot, dim3(64, kStencilTAH / 4), 0, E->stream>>>(gm, m, 2);
    else
      k_apply_A_iso_multi<S, true, KT, 64, kStencilTAH><<<tot, dim3(64, kStencilTAH / 4), 0, E->stream>>>(gm, m, 2);
    LAUNCHCHK("residual_multi");
    return ETC_OK;
  }
  static etc_status residual_multi(etc_plan* E) {
    return E->groups[0]->kap_hi[0] ? residual_multi_kt<double>(E) : residual_multi_kt<S>(E);
  }

  // n(P): partial sums per instance of the reducing kernel just launched
  template <class F>
  static etc_status fin_multi(etc_plan* E, int op, F&& n) {
    GroupMap gm{};
    FinMulti m{};
    unsigned tot = 0;
    for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
      etc_plan* P = E->groups[gi];
      add_group(gm, gi, dim3(P->nseg, 1, 1), tot);
      const int np = n(P);
      m.a[gi] = FinArgs{P->partials, np, np, P->st, P->hist, P->hstride};
    }
    k_fin_multi<<<tot, 1024, 0, E->stream>>>(gm, m, op);
    LAUNCHCHK("finalize_multi");
    return ETC_OK;
  }

  template <int MODE>
  static etc_status rows_fwd_multi(etc_plan* E, int gate) {
    GroupMap gm{};
    RowsMulti<S, T> m{};
    unsigned tot = 0;
    size_t lds = 0;
    for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
      etc_plan* P = E->groups[gi];
      add_group(gm, gi, P->lc.gridRows, tot);
      lds = std::max(lds, P->lc.ldsRows);
      m.a[gi] = RowsArgs<S, T>{P->g, P->dpb, (const cx<T>*)P->tw_b, MODE == 1 ? nullptr : (const S*)P->r,
                               (S*)P->t, P->lc.rpb, P->lc.nrows, MODE == 1 ? (S*)P->r : nullptr,
                               MODE == 1 ? (const S*)P->q : nullptr, MODE == 1 ? P->partials : nullptr, P->st,
                               nc_rows(P)};
    }
    k_rows_fwd_multi<S, T, MODE><<<tot, kThreads, lds, E->stream>>>(gm, m, gate);
    LAUNCHCHK("rows_fwd_multi");
    return ETC_OK;
  }

  static etc_status rows_inv_multi(etc_plan* E) {
    GroupMap gm{};
    RowsMulti<S, T> m{};
    unsigned tot = 0;
    size_t lds = 0;
    for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
      etc_plan* P = E->groups[gi];
      add_group(gm, gi, P->lc.gridRows, tot);
      lds = std::max(lds, P->lc.ldsRows);
      m.a[gi] = RowsArgs<S, T>{P->g, P->dpb, (const cx<T>*)P->tw_b, (const S*)P->t, (S*)P->w, P->lc.rpb,
                               P->lc.nrows, xsol(P), nullptr, nullptr, P->st, nc_rows(P)};
    }
    k_rows_inv_multi<S, T, 1><<<tot, kThreads, lds, E->stream>>>(gm, m, 1);
    LAUNCHCHK("rows_inv_multi");
    return ETC_OK;
  }

  template <int DIR>
  static etc_status cols_multi(etc_plan* E) {
    GroupMap gm{};
    ColsMulti<S, T> m{};
    unsigned tot = 0;
    size_t lds = 0;
    for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
      etc_plan* P = E->groups[gi];
      add_group(gm, gi, P->lc.gridCols, tot);
      lds = std::max(lds, P->lc.ldsCols);
      m.a[gi] = ColsArgs<S, T>{P->g, P->dpa, (const cx<T>*)P->tw_a, (S*)P->t, P->lc.tb, P->st, nc_cols(P)};
    }
    k_cols_multi<S, T, DIR><<<tot, E->groups[0]->lc.colThreads, lds, E->stream>>>(gm, m, 1);
    LAUNCHCHK("cols_multi");
    return ETC_OK;
  }

  // One launch per tridiagonal variant among the groups (each group runs the
  // variant its own plan launches).
  static etc_status thomas_multi(etc_plan* E) {
    std::vector<int> vars;
    for (const etc_plan* P : E->groups)
      if (std::find(vars.begin(), vars.end(), P->lc.tvar) == vars.end()) vars.push_back(P->lc.tvar);
    for (int var : vars) {
      GroupMap gm{};
      ThomasMulti<S> m{};
      unsigned tot = 0;
      int j = 0;
      for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
        etc_plan* P = E->groups[gi];
        const LaunchCfg& lc = P->lc;
        if (lc.tvar != var) continue;
        add_group(gm, j, dim3(E->multi_thomas_per[gi], 1, P->nseg), tot);
        m.a[j++] = ThomasArgs<S>{P->g, ref(P), (S*)P->t, lc.Puse, P->partials, P->st, lc.thomasTiles, lc.nThomas,
                                 var};
      }
      bool launched = false;
      with_thomas_variant<S>(var, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        // ensemble load axes stop at 512: partitions of at most 16 rows, or
        // exact partitions of more (20 or 32 rows)
        if constexpr (ThomasVariants<S>::v[I].rows <= 16 || ThomasVariants<S>::v[I].exact) {
          k_thomas_multi<S, I><<<tot, ThomasVariants<S>::v[I].threads(), 0, E->stream>>>(gm, m, 1);
          launched = true;
        }
      });
      if (!launched) return fail(ETC_E_UNSUPPORTED, "ensemble: no tridiagonal variant");
      LAUNCHCHK("thomas_multi");
    }
    return ETC_OK;
  }

  static etc_status flush_multi(etc_plan* E) {
    GroupMap gm{};
    FlushMulti m{};
    unsigned tot = 0;
    for (int gi = 0; gi < (int)E->groups.size(); ++gi) {
      etc_plan* P = E->groups[gi];
      add_group(gm, gi, P->lc.gridStride, tot);
      m.a[gi] = FlushArgs{P->g, P->p, (float*)P->dlt, (const float*)P->w, P->st};
    }
    k_flush_multi<<<tot, kThreads, 0, E->stream>>>(gm, m);
    LAUNCHCHK("flush_multi");
    return ETC_OK;
  }

  // One PCG pass (alg:pcg loop body) for every instance of every group.
  static etc_status iteration_multi(etc_plan* E) {
    etc_status s;
    if ((s = stencil_multi(E))) return s;
    if ((s = fin_multi(E, FIN_ALPHA, [](const etc_plan* P) { return P->lc.nA; }))) return s;
    if ((s = rows_fwd_multi<1>(E, 1))) return s;
    if ((s = fin_multi(E, FIN_RR, [](const etc_plan* P) { return P->lc.nRows; }))) return s;
    if (E->prec == ETC_MIXED) {
      if ((s = flush_multi(E))) return s;
      if ((s = residual_multi(E))) return s;
      if ((s = fin_multi(E, FIN_REFINE, [](const etc_plan* P) { return residual_parts(P); }))) return s;
      if ((s = rows_fwd_multi<0>(E, 2))) return s;
    }
    if ((s = cols_multi<-1>(E))) return s;
    if ((s = thomas_multi(E))) return s;
    if ((s = fin_multi(E, FIN_BETA, [](const etc_plan* P) { return P->lc.nThomas; }))) return s;
    if ((s = cols_multi<+1>(E))) return s;
    return rows_inv_multi(E);
  }

  // dK/dkappa of one instance of a batch plan into `out` (user layout)
  template <class O>
  static etc_status grad_instance(etc_plan* P, int inst, O* out, double c) {
    Geo g1 = P->g;
    g1.nseg = 1;
    const int64_t off = (int64_t)inst * P->g.V;
    Kap<S> k = kap(P);
    k.shift(off);
    k_grad<S, O><<<dim3(P->lc.nStride, 1), kThreads, 0, P->stream>>>(g1, P->p + off, P->padj + off, k, c, P->axis, out);
    LAUNCHCHK("grad");
    return ETC_OK;
  }
};

}  // namespace

// ================================================================== C ABI
extern "C" {

void etc_options_default(etc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = ETC_FP64;
  o->kref_mode = ETC_KREF_MID;
  for (int i = 0; i < 5; ++i) o->kref_user[i] = 1.0;
  o->rtol = 1e-6;
  o->max_iter = 1000;
  o->refine_every = 20;
  o->poll_every = 8;
  o->stream = nullptr;
  o->want_grad = 0;
  o->precond = ETC_PC_DCT;
  o->use_graph = 0;
  o->autotune = 0;
  o->thomas_modes = 0;
  o->thomas_parts = 0;
}

etc_status etc_launch_info(const etc_plan* P, int* kchunk, int* thomas_blocks, int* tuned, int* thomas_modes,
                           int* thomas_parts) {
  if (P && !P->groups.empty()) return fail(ETC_E_INVALID, "not defined for an ensemble plan (use the batch calls)");
  if (!P) return fail(ETC_E_INVALID, "plan is NULL");
  if (kchunk) *kchunk = P->lc.kchunk;
  if (thomas_blocks) *thomas_blocks = (int)P->lc.gridThomas.x;
  if (tuned) *tuned = P->tuned;
  if (thomas_modes) *thomas_modes = P->lc.thomasTB;
  if (thomas_parts) *thomas_parts = P->lc.thomasP;
  return ETC_OK;
}

const char* etc_last_error(void) { return g_err.c_str(); }

const char* etc_version(void) { return "etc-mi355x 0.1 (gfx950)"; }

static ProblemShape shape_of(const etc_problem* pr) {
  ProblemShape ps{false, false, false};
  if (pr) {
    ps.ortho = pr->kappa[1] != nullptr || pr->kappa[2] != nullptr;
    ps.src = pr->source != nullptr;
    ps.faces = pr->p_in_face != nullptr || pr->p_out_face != nullptr;
  }
  return ps;
}

etc_status etc_workspace_size_ex(const etc_problem* pr, const int64_t n[3], etc_dtype dt, int axis,
                                 const etc_options* opt, size_t* bytes) {
  etc_options o;
  if (opt) o = *opt;
  else etc_options_default(&o);
  if (!bytes) return fail(ETC_E_INVALID, "bytes is NULL");
  etc_status s = validate(n, axis, o);
  if (s) return s;
  *bytes = plan_sizes(n, axis, dt, o, shape_of(pr), 1).total;
  return ETC_OK;
}

etc_status etc_workspace_size(const int64_t n[3], etc_dtype dt, int axis, const etc_options* opt, size_t* bytes) {
  return etc_workspace_size_ex(nullptr, n, dt, axis, opt, bytes);
}

etc_status etc_workspace_size_batch(const int64_t n[3], int nbatch, etc_dtype dt, int axis, const etc_options* opt,
                                    size_t* bytes) {
  etc_options o;
  if (opt) o = *opt;
  else etc_options_default(&o);
  if (!bytes) return fail(ETC_E_INVALID, "bytes is NULL");
  if (nbatch < 1 || nbatch > 4096) return fail(ETC_E_INVALID, "nbatch must be in 1..4096");
  etc_status s = validate(n, axis, o);
  if (s) return s;
  *bytes = plan_sizes(n, axis, dt, o, ProblemShape{false, false, false}, nbatch).total;
  return ETC_OK;
}

}  // extern "C"

// inst_kappa: per-instance conductivity pointers of a batch whose instances
// are not stored back to back (isotropic only), else nullptr
static etc_status setup_impl(const etc_problem* pr, etc_dtype dt, const int64_t n[3], int nseg, etc_bc bc, int axis,
                             const etc_options* opt, etc_plan** out, bool no_alloc = false,
                             const void* const* inst_kappa = nullptr) {
  if (!out) return fail(ETC_E_INVALID, "plan is NULL");
  *out = nullptr;
  if (!pr) return fail(ETC_E_INVALID, "problem is NULL");
  const ProblemShape ps = shape_of(pr);
  if (ps.ortho) {
    for (int d = 0; d < 3; ++d)
      if (!pr->kappa[d]) return fail(ETC_E_INVALID, "an orthotropic problem needs all three kappa components");
  } else if (!pr->kappa[0]) {
    return fail(ETC_E_INVALID, "kappa is NULL");
  }
  if (dt != ETC_F64 && dt != ETC_F32) return fail(ETC_E_INVALID, "bad dtype");
  etc_options o;
  if (opt) o = *opt;
  else etc_options_default(&o);
  etc_status s = validate(n, axis, o);
  if (s) return s;
  if (!(bc.p_in != bc.p_out) || !std::isfinite(bc.p_in) || !std::isfinite(bc.p_out))
    return fail(ETC_E_INVALID, "p_in and p_out must be finite and differ");
  if (o.poll_every < 1) o.poll_every = 1;
  if (o.want_grad && (ps.ortho || ps.src || ps.faces))
    return fail(ETC_E_UNSUPPORTED, "etc_grad covers isotropic kappa with constant Dirichlet data only");
  if (nseg > 1 && (ps.ortho || ps.src || ps.faces))
    return fail(ETC_E_UNSUPPORTED, "batches take isotropic kappa with constant Dirichlet data");

  etc_plan* P = new etc_plan();
  P->opt = o;
  P->axis = axis;
  P->in_dt = dt;
  P->prec = o.precision;
  P->stream = (hipStream_t)o.stream;
  P->timer_id = 0;
  P->ev_used = 0;
  P->nseg = nseg;
  P->hstride = o.max_iter + 2;
  for (int d = 0; d < 3; ++d) P->n_user[d] = n[d];
  P->g = make_geo(n, axis, nseg);
  Geo& g = P->g;
  const int na = g.na, nb = g.nb;
  {
    double h_user[3] = {1.0, 1.0, 1.0};
    if (o.L[0] > 0.0)
      for (int d = 0; d < 3; ++d) h_user[d] = o.L[d] / (double)n[d];
    int order[3] = {axis, 0, 0}, c = 1;
    for (int d = 0; d < 3; ++d)
      if (d != axis) order[c++] = d;
    g.fL = 1.0 / (h_user[order[0]] * h_user[order[0]]);
    g.fa = 1.0 / (h_user[order[1]] * h_user[order[1]]);
    g.fb = 1.0 / (h_user[order[2]] * h_user[order[2]]);
  }
  g.p_in = bc.p_in;
  g.p_out = bc.p_out;
  const size_t es = elt_size(P->prec);
  P->dpa = make_dct_plan(na);
  P->dpb = make_dct_plan(nb);
  P->lc = make_launch(g, P->dpa, P->dpb, es, ps.ortho);
  if (((o.thomas_modes || o.thomas_parts) && !set_thomas(P->lc, g, es, o.thomas_modes, o.thomas_parts)) ||
      P->lc.tvar < 0) {
    delete P;
    return fail(ETC_E_UNSUPPORTED, "no compiled tridiagonal block of that shape holds this load axis");
  }
  if (P->lc.gridCols.y > 65535 || P->lc.gridA.z > 65535) {
    delete P;
    return fail(ETC_E_UNSUPPORTED, "batch too large: load planes times instances exceeds 65535");
  }

  Sizes sz = plan_sizes(n, axis, dt, o, ps, nseg);
  P->max_partials = sz.max_partials;
  if (o.workspace) {
    if (o.workspace_bytes < sz.total) {
      delete P;
      return fail(ETC_E_NOMEM, "workspace smaller than etc_workspace_size");
    }
    P->own_ws = false;
    P->ws = (char*)o.workspace;
    P->ws_bytes = o.workspace_bytes;
  } else {
    P->own_ws = true;
    if (hipMalloc((void**)&P->ws, sz.total) != hipSuccess) {
      delete P;
      return fail(ETC_E_NOMEM, "hipMalloc of the workspace failed");
    }
    P->ws_bytes = sz.total;
  }
  P->no_alloc = no_alloc;
  if (no_alloc) {
    // one instance; its state is read back into pageable host memory
    P->st_host = &P->st_local;
  } else if (hipHostMalloc((void**)&P->st_host, sizeof(DevState) * nseg, hipHostMallocDefault) != hipSuccess) {
    if (P->own_ws) (void)hipFree(P->ws);
    delete P;
    return fail(ETC_E_NOMEM, "pinned host allocation failed");
  }
  char* b = P->ws;
  P->ortho = ps.ortho;
  {
    const size_t vbytes = (size_t)g.V * nseg * es;
    const bool hi = (P->prec == ETC_MIXED && dt == ETC_F64);
    for (int c = 0; c < 3; ++c) {
      const int cc = ps.ortho ? c : 0;
      P->kap_s[c] = b + sz.off_kap_s + cc * vbytes;
      P->kap_hi[c] = hi ? (double*)(b + sz.off_kap_hi) + (size_t)cc * g.V * nseg : nullptr;
    }
  }
  P->src = ps.src ? (double*)(b + sz.off_src) : nullptr;
  P->pin_face = ps.faces ? (double*)(b + sz.off_faces) : nullptr;
  P->pout_face = ps.faces ? (double*)(b + sz.off_faces) + g.plane : nullptr;
  P->p = (double*)(b + sz.off_p);
  P->r = b + sz.off_r;
  P->w = b + sz.off_w;
  P->q = b + sz.off_q;
  P->t = b + sz.off_t;
  P->tw_a = b + sz.off_tw_a;
  P->tw_b = b + sz.off_tw_b;
  P->kref_d = (double*)(b + sz.off_kref);
  P->partials = (double*)(b + sz.off_part);
  P->st = (DevState*)(b + sz.off_st);
  P->hist = (double*)(b + sz.off_hist);
  P->padj = o.want_grad ? (double*)(b + sz.off_padj) : nullptr;
  P->dlt = (P->prec == ETC_MIXED) ? (void*)(b + sz.off_dlt) : nullptr;

  auto bail = [&](etc_status st) {
    etc_destroy(P);
    return st;
  };

  s = (P->prec == ETC_MIXED) ? Ops<float>::lds_limits(P) : Ops<double>::lds_limits(P);
  if (s) return bail(s);
  s = (P->prec == ETC_MIXED) ? Ops<float>::thomas_grid(P) : Ops<double>::thomas_grid(P);
  if (s) return bail(s);
  s = (P->prec == ETC_MIXED) ? Ops<float>::cols_grid(P) : Ops<double>::cols_grid(P);
  if (s) return bail(s);
  P->tuned = 0;
  if (o.autotune) {
    s = (P->prec == ETC_MIXED) ? Ops<float>::autotune(P) : Ops<double>::autotune(P);
    if (s) return bail(s);
  }
  if (ps.faces) {
    // face data: [a][b] over the transverse axes in user order (constant pair where NULL)
    std::vector<double> pin((size_t)g.plane, bc.p_in), pout((size_t)g.plane, bc.p_out);
    if (hipMemcpyAsync(P->pin_face, pin.data(), pin.size() * sizeof(double), hipMemcpyHostToDevice, P->stream) !=
            hipSuccess ||
        hipMemcpyAsync(P->pout_face, pout.data(), pout.size() * sizeof(double), hipMemcpyHostToDevice, P->stream) !=
            hipSuccess ||
        (pr->p_in_face && hipMemcpyAsync(P->pin_face, pr->p_in_face, (size_t)g.plane * sizeof(double),
                                         hipMemcpyDeviceToDevice, P->stream) != hipSuccess) ||
        (pr->p_out_face && hipMemcpyAsync(P->pout_face, pr->p_out_face, (size_t)g.plane * sizeof(double),
                                          hipMemcpyDeviceToDevice, P->stream) != hipSuccess) ||
        hipStreamSynchronize(P->stream) != hipSuccess)
      return bail(fail(ETC_E_HIP, "copying the Dirichlet face data failed"));
  }
  // DCT twiddle tables (independent of kappa): built on the host while the device makes
  // the canonical copy of the first instance, uploaded behind it
  auto upload_tables = [&]() -> etc_status {
    if (P->prec == ETC_MIXED) {
      std::vector<cx<float>> a, c;
      fill_twiddles(a, na);
      fill_twiddles(c, nb);
      P->tw_a_h.assign((unsigned char*)a.data(), (unsigned char*)(a.data() + a.size()));
      P->tw_b_h.assign((unsigned char*)c.data(), (unsigned char*)(c.data() + c.size()));
    } else {
      std::vector<cx<double>> a, c;
      fill_twiddles(a, na);
      fill_twiddles(c, nb);
      P->tw_a_h.assign((unsigned char*)a.data(), (unsigned char*)(a.data() + a.size()));
      P->tw_b_h.assign((unsigned char*)c.data(), (unsigned char*)(c.data() + c.size()));
    }
    if (hipMemcpyAsync(P->tw_a, P->tw_a_h.data(), P->tw_a_h.size(), hipMemcpyHostToDevice, P->stream) !=
            hipSuccess ||
        hipMemcpyAsync(P->tw_b, P->tw_b_h.data(), P->tw_b_h.size(), hipMemcpyHostToDevice, P->stream) !=
            hipSuccess)
      return fail(ETC_E_HIP, "uploading the tables failed");
    return ETC_OK;
  };
  // canonical copies, extrema and reference parameters, instance by instance
  P->kref.assign((size_t)5 * nseg, 1.0);
  P->lam_lo.assign(nseg, 1.0);
  P->lam_hi.assign(nseg, 1.0);
  {
    // user component order -> canonical (load axis, a, b)
    const void* comp[3] = {pr->kappa[0], pr->kappa[0], pr->kappa[0]};
    if (ps.ortho) {
      int order[3] = {axis, 0, 0}, c = 1;
      for (int d = 0; d < 3; ++d)
        if (d != axis) order[c++] = d;
      for (int d = 0; d < 3; ++d) comp[d] = pr->kappa[order[d]];
    }
    std::vector<double> part((size_t)P->lc.nExt * 12);
    for (int inst = 0; inst < nseg; ++inst) {
      s = (P->prec == ETC_MIXED) ? Ops<float>::canon(P, comp, pr->source, inst, inst_kappa ? inst_kappa[inst] : nullptr)
                                 : Ops<double>::canon(P, comp, pr->source, inst, inst_kappa ? inst_kappa[inst] : nullptr);
      if (s) return bail(s);
      if (inst == 0 && (s = upload_tables())) return bail(s);
      if (hipMemcpyAsync(part.data(), P->partials, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                         P->stream) != hipSuccess ||
          hipStreamSynchronize(P->stream) != hipSuccess)
        return bail(fail(ETC_E_HIP, "reading the extrema failed"));
      double mn[5], mx[5], bad = 0.0;
      for (int f = 0; f < 5; ++f) {
        mn[f] = INFINITY;
        mx[f] = -INFINITY;
      }
      for (int blk = 0; blk < P->lc.nExt; ++blk) {
        for (int f = 0; f < 5; ++f) {
          mn[f] = std::fmin(mn[f], part[(size_t)blk * 12 + 2 * f]);
          mx[f] = std::fmax(mx[f], part[(size_t)blk * 12 + 2 * f + 1]);
        }
        bad += part[(size_t)blk * 12 + 10];
      }
      if (bad > 0.0) return bail(fail(ETC_E_INVALID, "kappa holds values that are <= 0, NaN or Inf"));
      double* kr = &P->kref[(size_t)5 * inst];
      for (int f = 0; f < 5; ++f) {
        const bool empty = !(mn[f] <= mx[f]);
        if (o.kref_mode == ETC_KREF_USER) kr[f] = o.kref_user[f];
        else if (o.kref_mode == ETC_KREF_ONE || empty) kr[f] = 1.0;
        else kr[f] = std::sqrt(mn[f] * mx[f]);
      }
      double lo = INFINITY, hi = -INFINITY;
      for (int f = 0; f < 5; ++f) {
        if (!(mn[f] <= mx[f])) continue;
        lo = std::fmin(lo, mn[f] / kr[f]);
        hi = std::fmax(hi, mx[f] / kr[f]);
      }
      P->lam_lo[inst] = lo;
      P->lam_hi[inst] = hi;
    }
  }
  // reference parameters of every instance (no wait: the plan keeps the
  // host copy, and etc_destroy synchronises before releasing it)
  if (hipMemcpyAsync(P->kref_d, P->kref.data(), P->kref.size() * sizeof(double), hipMemcpyHostToDevice,
                     P->stream) != hipSuccess)
    return bail(fail(ETC_E_HIP, "uploading the reference parameters failed"));
  P->solved = false;
  *out = P;
  return ETC_OK;
}

static etc_status reset_state(etc_plan* P) {
  DevState h{};
  h.rtol = P->opt.rtol;
  h.max_iter = P->opt.max_iter;
  h.refine_every = (P->prec == ETC_MIXED) ? std::max(0, P->opt.refine_every) : 0;
  h.mixed = (P->prec == ETC_MIXED) ? 1 : 0;
  for (int i = 0; i < P->nseg; ++i) P->st_host[i] = h;
  P->any_done = false;
  HIPCHK(hipMemcpyAsync(P->st, P->st_host, sizeof(DevState) * P->nseg, hipMemcpyHostToDevice, P->stream));
  return ETC_OK;
}

static etc_status pull_state(etc_plan* P) {
  HIPCHK(hipMemcpyAsync(P->st_host, P->st, sizeof(DevState) * P->nseg, hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  return ETC_OK;
}

// Graph of `poll_every` passes for the current solution buffer and Dirichlet
// pair, captured on first use and kept until etc_destroy.  Capture needs a
// stream other than the null stream: a plan on the null stream captures and
// replays on a blocking stream of its own, which the null stream orders
// against implicitly.  `*ls` receives the stream to launch the graph on.
static etc_status graph_for(etc_plan* P, hipGraphExec_t* out, hipStream_t* ls) {
  hipStream_t cs = P->stream;
  if (!cs) {
    if (!P->cstream) HIPCHK(hipStreamCreate(&P->cstream));
    cs = P->cstream;
  }
  *ls = cs;
  for (auto& e : P->graphs)
    if (e.p == P->p && e.p_in == P->g.p_in && e.p_out == P->g.p_out && e.any_done == P->any_done) {
      *out = e.exec;
      return ETC_OK;
    }
  const hipStream_t saved = P->stream;
  P->stream = cs;
  etc_plan::GraphEntry e{P->p, P->g.p_in, P->g.p_out, P->any_done, nullptr, nullptr};
  etc_status s = ETC_OK;
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    for (int i = 0; i < P->opt.poll_every && s == ETC_OK; ++i)
      s = (P->prec == ETC_MIXED) ? Ops<float>::iteration(P) : Ops<double>::iteration(P);
    hipError_t he2 = hipStreamEndCapture(cs, &e.graph);
    if (he2 != hipSuccess && s == ETC_OK)
      s = fail(ETC_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he2));
  } else {
    s = fail(ETC_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(he));
  }
  P->stream = saved;
  if (s) {
    if (e.graph) (void)hipGraphDestroy(e.graph);
    return s;
  }
  if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(e.graph);
    return fail(ETC_E_HIP, "hipGraphInstantiate failed");
  }
  P->graphs.push_back(e);
  *out = e.exec;
  return ETC_OK;
}

extern "C" {

etc_status etc_setup(const void* kappa, etc_dtype dt, const int64_t n[3], etc_bc bc, int axis,
                     const etc_options* opt, etc_plan** out) {
  etc_problem pr;
  std::memset(&pr, 0, sizeof(pr));
  pr.kappa[0] = kappa;
  return setup_impl(&pr, dt, n, 1, bc, axis, opt, out);
}

etc_status etc_setup_ex(const etc_problem* pr, etc_dtype dt, const int64_t n[3], etc_bc bc, int axis,
                        const etc_options* opt, etc_plan** out) {
  return setup_impl(pr, dt, n, 1, bc, axis, opt, out);
}

etc_status etc_setup_batch(const void* kappa, etc_dtype dt, const int64_t n[3], int nbatch, etc_bc bc, int axis,
                           const etc_options* opt, etc_plan** out) {
  if (nbatch < 1 || nbatch > 4096) return fail(ETC_E_INVALID, "nbatch must be in 1..4096");
  etc_problem pr;
  std::memset(&pr, 0, sizeof(pr));
  pr.kappa[0] = kappa;
  return setup_impl(&pr, dt, n, nbatch, bc, axis, opt, out);
}

// Groups of a mixed-size ensemble: the instances of each distinct shape, in
// the order of first appearance, then sorted largest group first (its
// blocks lead every multi-group launch); workspace ranges per group.
struct EnsembleLayout {
  std::vector<std::vector<int64_t>> dims;  // user dims per group
  std::vector<std::vector<int>> members;   // instance indices per group
  std::vector<int> inst_group, inst_local;
  std::vector<size_t> ws_off, ws_size;
  size_t total = 0;
};

static etc_status ensemble_layout(const int64_t* dims, int count, etc_dtype dt, int axis, const etc_options& o,
                                  EnsembleLayout& L) {
  if (!dims) return fail(ETC_E_INVALID, "dims is NULL");
  if (count < 1 || count > 4096) return fail(ETC_E_INVALID, "count must be in 1..4096");
  if (dt != ETC_F64 && dt != ETC_F32) return fail(ETC_E_INVALID, "bad dtype");
  std::vector<std::vector<int64_t>> gd;
  std::vector<std::vector<int>> gm;
  for (int i = 0; i < count; ++i) {
    const int64_t* n = dims + 3 * (size_t)i;
    etc_status s = validate(n, axis, o);
    if (s) return s;
    if (n[axis] > kThomasP * 16)
      return fail(ETC_E_UNSUPPORTED, "ensemble RVEs take load axes up to 512 voxels");
    std::vector<int64_t> key(n, n + 3);
    size_t gi = 0;
    while (gi < gd.size() && gd[gi] != key) ++gi;
    if (gi == gd.size()) {
      gd.push_back(key);
      gm.emplace_back();
    }
    gm[gi].push_back(i);
  }
  if ((int)gd.size() > kMaxGroups)
    return fail(ETC_E_UNSUPPORTED, "an ensemble takes at most " + std::to_string(kMaxGroups) + " distinct RVE shapes");
  std::vector<size_t> order(gd.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  auto voxels = [&](size_t g) { return gd[g][0] * gd[g][1] * gd[g][2] * (int64_t)gm[g].size(); };
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return voxels(a) > voxels(b); });
  L = EnsembleLayout{};
  L.inst_group.assign(count, 0);
  L.inst_local.assign(count, 0);
  for (size_t k = 0; k < order.size(); ++k) {
    const size_t g = order[k];
    L.dims.push_back(gd[g]);
    L.members.push_back(gm[g]);
    for (size_t j = 0; j < gm[g].size(); ++j) {
      L.inst_group[gm[g][j]] = (int)k;
      L.inst_local[gm[g][j]] = (int)j;
    }
    const size_t sz = align_up(plan_sizes(gd[g].data(), axis, dt, o, ProblemShape{false, false, false},
                                          (int)gm[g].size()).total);
    L.ws_off.push_back(L.total);
    L.ws_size.push_back(sz);
    L.total += sz;
  }
  return ETC_OK;
}

// Captured passes of an ensemble plan (use_graph), keyed like a plan's own
// graphs by the first group's solution buffer and the Dirichlet pair (the
// adjoint solve swaps both).
static etc_status ensemble_graph(etc_plan* E, hipGraphExec_t* out, hipStream_t* ls) {
  hipStream_t cs = E->stream;
  if (!cs) {
    if (!E->cstream) HIPCHK(hipStreamCreate(&E->cstream));
    cs = E->cstream;
  }
  *ls = cs;
  etc_plan* G0 = E->groups[0];
  for (auto& e : E->graphs)
    if (e.p == G0->p && e.p_in == G0->g.p_in && e.p_out == G0->g.p_out) {
      *out = e.exec;
      return ETC_OK;
    }
  const hipStream_t saved = E->stream;
  E->stream = cs;
  etc_plan::GraphEntry e{G0->p, G0->g.p_in, G0->g.p_out, false, nullptr, nullptr};
  etc_status s = ETC_OK;
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    for (int i = 0; i < E->opt.poll_every && s == ETC_OK; ++i)
      s = (E->prec == ETC_MIXED) ? Ops<float>::iteration_multi(E) : Ops<double>::iteration_multi(E);
    hipError_t he2 = hipStreamEndCapture(cs, &e.graph);
    if (he2 != hipSuccess && s == ETC_OK)
      s = fail(ETC_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he2));
  } else {
    s = fail(ETC_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(he));
  }
  E->stream = saved;
  if (s) {
    if (e.graph) (void)hipGraphDestroy(e.graph);
    return s;
  }
  if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(e.graph);
    return fail(ETC_E_HIP, "hipGraphInstantiate failed");
  }
  E->graphs.push_back(e);
  *out = e.exec;
  return ETC_OK;
}

// PCG for every instance of every group of an ensemble plan: each kernel of
// a pass is one launch for the whole ensemble; the host reads every group's
// device state once per `poll_every` passes.
static etc_status solve_ensemble(etc_plan* E, etc_result* res) {
  etc_status s;
  const bool mixed = E->prec == ETC_MIXED;
  for (etc_plan* P : E->groups) {
    if ((s = reset_state(P))) return s;
    if ((s = mixed ? Ops<float>::init(P, nullptr) : Ops<double>::init(P, nullptr))) return s;
  }
  if ((s = mixed ? Ops<float>::multi_prepare(E) : Ops<double>::multi_prepare(E))) return s;
  hipGraphExec_t exec = nullptr;
  hipStream_t gstream = nullptr;
  if (E->opt.use_graph) {
    if ((s = ensemble_graph(E, &exec, &gstream))) return s;
    if (gstream != E->stream) HIPCHK(hipStreamSynchronize(E->stream));
  }
  int enq = 0;
  const int chunk = E->opt.poll_every;
  for (;;) {
    for (etc_plan* P : E->groups)
      HIPCHK(hipMemcpyAsync(P->st_host, P->st, sizeof(DevState) * P->nseg, hipMemcpyDeviceToHost, E->stream));
    HIPCHK(hipStreamSynchronize(E->stream));
    bool all_done = true;
    for (etc_plan* P : E->groups)
      for (int i = 0; i < P->nseg; ++i) all_done = all_done && P->st_host[i].done;
    if (all_done || enq > E->opt.max_iter) break;
    if (exec) {
      HIPCHK(hipGraphLaunch(exec, gstream));
    } else {
      for (int i = 0; i < chunk; ++i)
        if ((s = mixed ? Ops<float>::iteration_multi(E) : Ops<double>::iteration_multi(E))) return s;
    }
    enq += chunk;
  }
  for (etc_plan* P : E->groups)
    if ((s = mixed ? Ops<float>::fixup(P) : Ops<double>::fixup(P))) return s;
  HIPCHK(hipStreamSynchronize(E->stream));
  int iters = 0, status = ST_OK;
  for (etc_plan* P : E->groups) {
    int gi = 0, gs = ST_OK;
    for (int i = 0; i < P->nseg; ++i) {
      const DevState& h = P->st_host[i];
      gi = std::max(gi, h.iter);
      const int st = h.done ? h.status : ST_NOT_CONVERGED;
      if (st == ST_BREAKDOWN) gs = ST_BREAKDOWN;
      else if (st == ST_NOT_CONVERGED && gs == ST_OK) gs = ST_NOT_CONVERGED;
    }
    P->last_iters = gi;
    P->last_status = gs;
    P->solved = gs != ST_BREAKDOWN;
    iters = std::max(iters, gi);
    if (gs == ST_BREAKDOWN) status = ST_BREAKDOWN;
    else if (gs == ST_NOT_CONVERGED && status == ST_OK) status = ST_NOT_CONVERGED;
  }
  E->last_iters = iters;
  E->last_status = status;
  if (res) {
    const etc_plan* P0 = E->groups[E->inst_group[0]];
    const int j0 = E->inst_local[0];
    res->iters = P0->st_host[j0].iter;
    res->status = status;
    res->relres = P0->st_host[j0].relres;
    for (int i = 0; i < 5; ++i) res->kref[i] = P0->kref[(size_t)5 * j0 + i];
    res->lambda_lo = P0->lam_lo[j0];
    res->lambda_hi = P0->lam_hi[j0];
  }
  if (status == ST_BREAKDOWN) {
    E->solved = false;
    return fail(ETC_E_BREAKDOWN, "PCG breakdown (non-positive or non-finite scalar)");
  }
  E->solved = true;
  if (status == ST_NOT_CONVERGED) {
    g_err = "iteration cap reached";
    return ETC_NOT_CONVERGED;
  }
  return ETC_OK;
}

etc_status etc_workspace_size_ensemble(const int64_t* dims, int count, etc_dtype dt, int axis, const etc_options* opt,
                                       size_t* bytes) {
  if (!bytes) return fail(ETC_E_INVALID, "bytes is NULL");
  etc_options o;
  if (opt) o = *opt;
  else etc_options_default(&o);
  EnsembleLayout L;
  etc_status s = ensemble_layout(dims, count, dt, axis, o, L);
  if (s) return s;
  *bytes = L.total;
  return ETC_OK;
}

etc_status etc_setup_ensemble(const void* const* kappa, const int64_t* dims, int count, etc_dtype dt, etc_bc bc,
                              int axis, const etc_options* opt, etc_plan** out) {
  if (!out) return fail(ETC_E_INVALID, "plan is NULL");
  *out = nullptr;
  if (!kappa) return fail(ETC_E_INVALID, "kappa is NULL");
  etc_options o;
  if (opt) o = *opt;
  else etc_options_default(&o);
  EnsembleLayout L;
  etc_status s = ensemble_layout(dims, count, dt, axis, o, L);
  if (s) return s;
  for (int i = 0; i < count; ++i)
    if (!kappa[i]) return fail(ETC_E_INVALID, "kappa[" + std::to_string(i) + "] is NULL");
  if (o.workspace && o.workspace_bytes < L.total) return fail(ETC_E_NOMEM, "workspace smaller than etc_workspace_size_ensemble");
  if (o.poll_every < 1) o.poll_every = 1;
  etc_plan* E = new etc_plan();
  E->opt = o;
  E->axis = axis;
  E->in_dt = dt;
  E->prec = o.precision;
  E->stream = (hipStream_t)o.stream;
  E->nseg = count;
  E->hstride = o.max_iter + 2;
  E->own_ws = false;
  E->solved = false;
  for (size_t gi = 0; gi < L.dims.size(); ++gi) {
    etc_options og = o;
    og.use_graph = 0;  // the ensemble captures its own passes
    if (o.workspace) {
      og.workspace = (char*)o.workspace + L.ws_off[gi];
      og.workspace_bytes = L.ws_size[gi];
    }
    std::vector<const void*> ptrs;
    for (int i : L.members[gi]) ptrs.push_back(kappa[i]);
    etc_problem pr;
    std::memset(&pr, 0, sizeof(pr));
    pr.kappa[0] = ptrs[0];
    etc_plan* G = nullptr;
    s = setup_impl(&pr, dt, L.dims[gi].data(), (int)ptrs.size(), bc, axis, &og, &G, false, ptrs.data());
    if (s) {
      const std::string msg = g_err;
      etc_destroy(E);
      return fail(s, msg);
    }
    E->groups.push_back(G);
  }
  // the isotropic stencil runs as one launch for all groups: one tile width
  // (128 if any group's lines are long enough for it; wider tiles need fewer
  // partial sums, so every group's buffers still suffice)
  {
    int tbw = 64;
    for (etc_plan* G : E->groups)
      if (!G->ortho) tbw = std::max(tbw, G->lc.stencilTBW);
    for (etc_plan* G : E->groups)
      if (!G->ortho && G->lc.stencilTBW != tbw) {
        G->lc.stencilTBW = tbw;
        set_stencil_chunk(G->lc, G->g, G->lc.kchunk);
      }
  }
  E->inst_group = L.inst_group;
  E->inst_local = L.inst_local;
  *out = E;
  return ETC_OK;
}

etc_status etc_solve(etc_plan* P, const double* p0, etc_result* res) {
  if (!P) return fail(ETC_E_INVALID, "plan is NULL");
  if (!P->groups.empty()) {
    if (p0) return fail(ETC_E_UNSUPPORTED, "an ensemble plan starts from p0 = 0");
    return solve_ensemble(P, res);
  }
  etc_status s = reset_state(P);
  if (s) return s;
  // kernel timer events
  if (P->timer_id > 0) {
    const size_t need = (size_t)2 * (P->opt.max_iter + 2);
    while (P->ev.size() < need) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      P->ev.push_back(e);
    }
  }
  P->ev_used = 0;
  s = (P->prec == ETC_MIXED) ? Ops<float>::init(P, p0) : Ops<double>::init(P, p0);
  if (s) return s;
  int enq = 0;
  const int chunk = P->opt.poll_every;
  hipGraphExec_t exec = nullptr;
  hipStream_t gstream = nullptr;
  if (P->opt.use_graph && P->timer_id == 0) {
    if ((s = graph_for(P, &exec, &gstream))) return s;
    if (gstream != P->stream) HIPCHK(hipStreamSynchronize(P->stream));
  }
  for (;;) {
    if ((s = pull_state(P))) return s;
    bool all_done = true;
    for (int i = 0; i < P->nseg; ++i) all_done = all_done && P->st_host[i].done;
    const bool was_done = P->any_done;
    for (int i = 0; i < P->nseg; ++i) P->any_done = P->any_done || P->st_host[i].done;
    if (all_done || enq > P->opt.max_iter) break;
    if (exec && P->any_done != was_done) {
      // an instance has converged: from here the passes gate the column
      // transforms, which is another captured graph
      if ((s = graph_for(P, &exec, &gstream))) return s;
    }
    if (exec) {
      HIPCHK(hipGraphLaunch(exec, gstream));
    } else {
      for (int i = 0; i < chunk; ++i) {
        s = (P->prec == ETC_MIXED) ? Ops<float>::iteration(P) : Ops<double>::iteration(P);
        if (s) return s;
      }
    }
    enq += chunk;
  }
  if (P->opt.precond == ETC_PC_DCT) {
    s = (P->prec == ETC_MIXED) ? Ops<float>::fixup(P) : Ops<double>::fixup(P);
    if (s) return s;
    HIPCHK(hipStreamSynchronize(P->stream));
  }
  int iters = 0, status = ST_OK;
  for (int i = 0; i < P->nseg; ++i) {
    const DevState& h = P->st_host[i];
    iters = std::max(iters, h.iter);
    const int st = h.done ? h.status : ST_NOT_CONVERGED;
    if (st == ST_BREAKDOWN) status = ST_BREAKDOWN;
    else if (st == ST_NOT_CONVERGED && status == ST_OK) status = ST_NOT_CONVERGED;
  }
  P->last_iters = iters;
  P->last_status = status;
  if (P->timer_id > 0) {
    double tot = 0.0;
    for (int i = 0; i + 1 < P->ev_used; i += 2) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, P->ev[i], P->ev[i + 1]));
      tot += ms;
    }
    P->timer_ms = tot;
    P->timer_launches = P->ev_used / 2;
  }
  if (res) {
    res->iters = P->st_host[0].iter;
    res->status = P->last_status;
    res->relres = P->st_host[0].relres;
    for (int i = 0; i < 5; ++i) res->kref[i] = P->kref[i];
    res->lambda_lo = P->lam_lo[0];
    res->lambda_hi = P->lam_hi[0];
  }
  if (P->last_status == ST_BREAKDOWN) {
    P->solved = false;
    return fail(ETC_E_BREAKDOWN, "PCG breakdown (non-positive or non-finite scalar)");
  }
  P->solved = true;
  if (P->last_status == ST_NOT_CONVERGED) {
    g_err = "iteration cap reached";
    return ETC_NOT_CONVERGED;
  }
  return ETC_OK;
}

etc_status etc_batch_results(const etc_plan* P, int* iters, int* status, double* relres) {
  if (!P) return fail(ETC_E_INVALID, "plan is NULL");
  if (!P->groups.empty()) {
    for (size_t i = 0; i < P->inst_group.size(); ++i) {
      const DevState& h = P->groups[P->inst_group[i]]->st_host[P->inst_local[i]];
      if (iters) iters[i] = h.iter;
      if (status) status[i] = h.done ? h.status : ST_NOT_CONVERGED;
      if (relres) relres[i] = h.relres;
    }
    return ETC_OK;
  }
  for (int i = 0; i < P->nseg; ++i) {
    const DevState& h = P->st_host[i];
    if (iters) iters[i] = h.iter;
    if (status) status[i] = h.done ? h.status : ST_NOT_CONVERGED;
    if (relres) relres[i] = h.relres;
  }
  return ETC_OK;
}

static etc_status keff_all(etc_plan* P, bool energy) {
  if (!P->solved) return fail(ETC_E_STATE, "etc_keff before a successful etc_solve");
  etc_status s = (P->prec == ETC_MIXED) ? Ops<float>::keff(P, energy) : Ops<double>::keff(P, energy);
  if (s) return s;
  return pull_state(P);
}

etc_status etc_keff(etc_plan* P, double* k_out, double* k_in, double* k_energy) {
  if (!P) return fail(ETC_E_INVALID, "plan is NULL");
  if (P && !P->groups.empty()) return fail(ETC_E_INVALID, "not defined for an ensemble plan (use the batch calls)");
  if (!k_out) return fail(ETC_E_INVALID, "k_out is NULL");
  etc_status s = keff_all(P, k_energy != nullptr);
  if (s) return s;
  const Geo& g = P->g;
  const double dp = g.p_in - g.p_out;
  const double scale = (double)g.nL / ((double)g.na * (double)g.nb * dp);
  *k_out = scale * P->st_host[0].k_acc[0];
  if (k_in) *k_in = scale * P->st_host[0].k_acc[1];
  if (k_energy) *k_energy = scale / g.fL * P->st_host[0].k_acc[2] / dp;
  return ETC_OK;
}

etc_status etc_keff_batch(etc_plan* P, double* k_out, double* k_in) {
  if (!P) return fail(ETC_E_INVALID, "plan is NULL");
  if (!k_out) return fail(ETC_E_INVALID, "k_out is NULL");
  if (!P->groups.empty()) {
    if (!P->solved) return fail(ETC_E_STATE, "etc_keff_batch before a successful etc_solve");
    for (etc_plan* G : P->groups) {
      etc_status s = keff_all(G, false);
      if (s) return s;
    }
    for (size_t i = 0; i < P->inst_group.size(); ++i) {
      const etc_plan* G = P->groups[P->inst_group[i]];
      const Geo& g = G->g;
      const double scale = (double)g.nL / ((double)g.na * (double)g.nb * (g.p_in - g.p_out));
      const DevState& h = G->st_host[P->inst_local[i]];
      k_out[i] = scale * h.k_acc[0];
      if (k_in) k_in[i] = scale * h.k_acc[1];
    }
    return ETC_OK;
  }
  etc_status s = keff_all(P, false);
  if (s) return s;
  const Geo& g = P->g;
  const double scale = (double)g.nL / ((double)g.na * (double)g.nb * (g.p_in - g.p_out));
  for (int i = 0; i < P->nseg; ++i) {
    k_out[i] = scale * P->st_host[i].k_acc[0];
    if (k_in) k_in[i] = scale * P->st_host[i].k_acc[1];
  }
  return ETC_OK;
}

// user-layout copy of instance `inst` of a (batch) plan's canonical vector
static etc_status decanon_instance(const etc_plan* P, const double* vec, int inst, double* dst) {
  Geo g = P->g;
  g.nseg = 1;
  const double* src = vec + (int64_t)inst * g.V;
  if (P->axis == 2) {
    dim3 grid((g.nL + 31) / 32, (g.nb + 31) / 32, g.na);
    k_decanon_axis2<<<grid, dim3(32, 8), 0, P->stream>>>(src, dst, g);
  } else {
    k_decanon_rows<<<P->lc.nStride, kThreads, 0, P->stream>>>(src, dst, P->axis, g);
  }
  LAUNCHCHK("decanon");
  return ETC_OK;
}

etc_status etc_get_solution(const etc_plan* P, double* p) {
  if (!P || !p) return fail(ETC_E_INVALID, "NULL argument");
  if (!P->solved) return fail(ETC_E_STATE, "etc_get_solution before a successful etc_solve");
  if (!P->groups.empty()) {
    int64_t off = 0;
    for (size_t i = 0; i < P->inst_group.size(); ++i) {
      const etc_plan* G = P->groups[P->inst_group[i]];
      etc_status s = decanon_instance(G, G->p, P->inst_local[i], p + off);
      if (s) return s;
      off += G->g.V;
    }
    return ETC_OK;
  }
  for (int inst = 0; inst < P->nseg; ++inst) {
    etc_status s = decanon_instance(P, P->p, inst, p + (int64_t)inst * P->g.V);
    if (s) return s;
  }
  return ETC_OK;
}

etc_status etc_residual_history(const etc_plan* P, double* hist, int cap, int* count) {
  if (!P || !hist || !count) return fail(ETC_E_INVALID, "NULL argument");
  if (!P->groups.empty()) {
    // instance 0 of the ensemble (input order)
    const etc_plan* G = P->groups[P->inst_group[0]];
    const int j = P->inst_local[0];
    int n = std::min(cap, G->st_host[j].iter + 1);
    if (n < 0) n = 0;
    if (n > 0) {
      HIPCHK(hipMemcpyAsync(hist, G->hist + (int64_t)j * G->hstride, n * sizeof(double), hipMemcpyDeviceToHost,
                            G->stream));
      HIPCHK(hipStreamSynchronize(G->stream));
    }
    *count = n;
    return ETC_OK;
  }
  int n = std::min(cap, P->st_host[0].iter + 1);
  if (n < 0) n = 0;
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(hist, P->hist, n * sizeof(double), hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipStreamSynchronize(P->stream));
  }
  *count = n;
  return ETC_OK;
}

extern "C++" template <class O>
static etc_status grad_ensemble(etc_plan* E, O* out) {
  for (etc_plan* G : E->groups)
    if (!G->padj) return fail(ETC_E_STATE, "etc_grad needs a plan made with want_grad = 1");
  if (!E->solved) return fail(ETC_E_STATE, "etc_grad before a successful etc_solve");
  // adjoint solves of every instance together: Dirichlet pair (0, 1),
  // solutions into padj
  struct Saved { Geo g; int iters, status; std::vector<DevState> st; };
  std::vector<Saved> sv;
  for (etc_plan* G : E->groups) {
    sv.push_back(Saved{G->g, G->last_iters, G->last_status, std::vector<DevState>(G->st_host, G->st_host + G->nseg)});
    std::swap(G->p, G->padj);
    G->g.p_in = 0.0;
    G->g.p_out = 1.0;
  }
  const int iters0 = E->last_iters, status0 = E->last_status;
  etc_status s = solve_ensemble(E, nullptr);
  for (size_t gi = 0; gi < E->groups.size(); ++gi) {
    etc_plan* G = E->groups[gi];
    std::swap(G->p, G->padj);
    G->g = sv[gi].g;
    G->last_iters = sv[gi].iters;
    G->last_status = sv[gi].status;
    std::copy(sv[gi].st.begin(), sv[gi].st.end(), G->st_host);
    G->solved = true;
  }
  E->last_iters = iters0;
  E->last_status = status0;
  E->solved = true;
  if (s != ETC_OK && s != ETC_NOT_CONVERGED) return s;
  int64_t off = 0;
  for (size_t i = 0; i < E->inst_group.size(); ++i) {
    etc_plan* G = E->groups[E->inst_group[i]];
    const Geo& g = G->g;
    const double c = (double)g.nL / ((double)g.na * (double)g.nb * (g.p_in - g.p_out));
    s = (G->prec == ETC_MIXED) ? Ops<float>::grad_instance(G, E->inst_local[i], out + off, c)
                               : Ops<double>::grad_instance(G, E->inst_local[i], out + off, c);
    if (s) return s;
    off += g.V;
  }
  HIPCHK(hipStreamSynchronize(E->stream));
  return ETC_OK;
}

etc_status etc_grad(etc_plan* P, double* dk_dkappa) { return etc_grad_as(P, dk_dkappa, ETC_F64); }

etc_status etc_grad_as(etc_plan* P, void* dk_dkappa, etc_dtype out_dt) {
  if (!P || !dk_dkappa) return fail(ETC_E_INVALID, "NULL argument");
  if (out_dt != ETC_F64 && out_dt != ETC_F32) return fail(ETC_E_INVALID, "bad output dtype");
  if (!P->groups.empty())
    return out_dt == ETC_F64 ? grad_ensemble(P, (double*)dk_dkappa) : grad_ensemble(P, (float*)dk_dkappa);
  if (!P->padj) return fail(ETC_E_STATE, "etc_grad needs a plan made with want_grad = 1");
  if (!P->solved) return fail(ETC_E_STATE, "etc_grad before a successful etc_solve");
  // adjoint solve: the primal system with Dirichlet pair (0, 1), solution into padj
  const Geo g0 = P->g;
  const int iters0 = P->last_iters, status0 = P->last_status;
  const int timer0 = P->timer_id;
  std::vector<DevState> st0(P->st_host, P->st_host + P->nseg);
  std::swap(P->p, P->padj);
  P->g.p_in = 0.0;
  P->g.p_out = 1.0;
  P->timer_id = 0;
  etc_status s = etc_solve(P, nullptr, nullptr);
  std::swap(P->p, P->padj);
  P->g = g0;
  P->timer_id = timer0;
  P->last_iters = iters0;
  P->last_status = status0;
  std::copy(st0.begin(), st0.end(), P->st_host);
  P->solved = true;
  if (s != ETC_OK && s != ETC_NOT_CONVERGED) return s;
  const double c = (double)g0.nL / ((double)g0.na * (double)g0.nb * (g0.p_in - g0.p_out));
  if (out_dt == ETC_F64)
    s = (P->prec == ETC_MIXED) ? Ops<float>::grad(P, (double*)dk_dkappa, c) : Ops<double>::grad(P, (double*)dk_dkappa, c);
  else
    s = (P->prec == ETC_MIXED) ? Ops<float>::grad(P, (float*)dk_dkappa, c) : Ops<double>::grad(P, (float*)dk_dkappa, c);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(P->stream));
  return ETC_OK;
}

etc_status etc_apply_A(etc_plan* P, const void* x, void* y, double* xAx) {
  if (P && !P->groups.empty()) return fail(ETC_E_INVALID, "not defined for an ensemble plan (use the batch calls)");
  if (!P || !x || !y) return fail(ETC_E_INVALID, "NULL argument");
  if (x == y) return fail(ETC_E_INVALID, "x and y must not alias");
  etc_status s = (P->prec == ETC_MIXED) ? Ops<float>::apply_A(P, x, y, xAx != nullptr)
                                        : Ops<double>::apply_A(P, x, y, xAx != nullptr);
  if (s) return s;
  if (xAx) {
    if ((s = pull_state(P))) return s;
    double sum = 0.0;
    for (int i = 0; i < P->nseg; ++i) sum += P->st_host[i].k_acc[3];
    *xAx = sum;
  }
  return ETC_OK;
}

etc_status etc_apply_Minv(etc_plan* P, const void* r, void* z, double* rz) {
  if (P && !P->groups.empty()) return fail(ETC_E_INVALID, "not defined for an ensemble plan (use the batch calls)");
  if (!P || !r || !z) return fail(ETC_E_INVALID, "NULL argument");
  if (r == z) return fail(ETC_E_INVALID, "r and z must not alias");
  if (P->opt.precond == ETC_PC_NONE) {
    HIPCHK(hipMemcpyAsync(z, r, (size_t)P->g.V * P->nseg * elt_size(P->prec), hipMemcpyDeviceToDevice, P->stream));
    if (rz) return fail(ETC_E_UNSUPPORTED, "no dot without a preconditioner");
    return ETC_OK;
  }
  etc_status s = (P->prec == ETC_MIXED) ? Ops<float>::precond(P, (const float*)r, (float*)z, P->st, 0, FIN_ACC3)
                                        : Ops<double>::precond(P, (const double*)r, (double*)z, P->st, 0, FIN_ACC3);
  if (s) return s;
  if (rz) {
    if ((s = pull_state(P))) return s;
    double sum = 0.0;
    for (int i = 0; i < P->nseg; ++i) sum += P->st_host[i].k_acc[3];
    *rz = sum;
  }
  return ETC_OK;
}

etc_status etc_set_kernel_timer(etc_plan* P, int kernel_id) {
  if (P && !P->groups.empty()) return fail(ETC_E_INVALID, "not defined for an ensemble plan (use the batch calls)");
  if (!P) return fail(ETC_E_INVALID, "plan is NULL");
  if (kernel_id < 0 || kernel_id > 6) return fail(ETC_E_INVALID, "kernel_id must be 0..6");
  P->timer_id = kernel_id;
  return ETC_OK;
}

etc_status etc_kernel_time(const etc_plan* P, double* total_ms, int* launches) {
  if (!P || !total_ms || !launches) return fail(ETC_E_INVALID, "NULL argument");
  *total_ms = P->timer_ms;
  *launches = P->timer_launches;
  return ETC_OK;
}

etc_status etc_copy_f64(const double* src, double* dst, int64_t n, void* stream) {
  if (!src || !dst || n < 0) return fail(ETC_E_INVALID, "bad copy arguments");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return fail(ETC_E_INVALID, "copy buffers must be 16-byte aligned");
  int64_t gs = std::min<int64_t>((n / 2 + 4 * kThreads - 1) / (4 * kThreads), 16384);
  if (gs < 1) gs = 1;
  k_copy<<<(int)gs, kThreads, 0, (hipStream_t)stream>>>(src, dst, n);
  LAUNCHCHK("copy");
  return ETC_OK;
}

}  // extern "C"

// Workspace of etc_solve_static: one array per GPU, held until the process
// ends.  In host code the name `scratch` is only a stand-in for the symbol;
// its device address comes from hipGetSymbolAddress, once per device, and
// only that address is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[ETC_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
etc_status static_scratch(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ETC_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(ETC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ETC_OK;
}
}  // namespace

extern "C" {

etc_status etc_solve_static(const void* kappa, etc_dtype dt, const int64_t n[3], etc_bc bc, int axis,
                            const etc_options* opt, double* p, double* k_out, double* k_in, etc_result* res) {
  if (!k_out) return fail(ETC_E_INVALID, "k_out is NULL");
  etc_options o;
  if (opt) o = *opt;
  else etc_options_default(&o);
  if (o.workspace) return fail(ETC_E_INVALID, "etc_solve_static uses its own scratch array: workspace must be NULL");
  if (o.autotune || o.use_graph || o.want_grad)
    return fail(ETC_E_INVALID, "etc_solve_static: autotune, use_graph and want_grad must be 0");
  size_t need = 0;
  etc_status s = etc_workspace_size(n, dt, axis, &o, &need);
  if (s) return s;
  if (need > (size_t)ETC_STATIC_SCRATCH_BYTES)
    return fail(ETC_E_UNSUPPORTED, "problem needs " + std::to_string(need) + " bytes of scratch; etc_solve_static holds " +
                                       std::to_string((size_t)ETC_STATIC_SCRATCH_BYTES));
  void* ws = nullptr;
  if ((s = static_scratch(&ws))) return s;
  o.workspace = ws;
  o.workspace_bytes = ETC_STATIC_SCRATCH_BYTES;
  etc_problem pr;
  std::memset(&pr, 0, sizeof(pr));
  pr.kappa[0] = kappa;
  etc_plan* P = nullptr;
  if ((s = setup_impl(&pr, dt, n, 1, bc, axis, &o, &P, true))) return s;
  const etc_status st = etc_solve(P, nullptr, res);
  if (st < 0) {
    const std::string msg = g_err;
    etc_destroy(P);
    return fail(st, msg);
  }
  s = etc_keff(P, k_out, k_in, nullptr);
  if (s == ETC_OK && p) s = etc_get_solution(P, p);
  const std::string msg = g_err;
  etc_destroy(P);
  if (s) return fail(s, msg);
  if (st == ETC_NOT_CONVERGED) g_err = "iteration cap reached";
  return st;
}

void etc_destroy(etc_plan* P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->stream);
  for (etc_plan* G : P->groups) etc_destroy(G);
  P->groups.clear();
  for (auto& e : P->graphs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
  }
  if (P->cstream) {
    (void)hipStreamSynchronize(P->cstream);
    (void)hipStreamDestroy(P->cstream);
  }
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  if (P->own_ws && P->ws) (void)hipFree(P->ws);
  if (P->st_host && !P->no_alloc) (void)hipHostFree(P->st_host);
  delete P;
}

}  // extern "C"
