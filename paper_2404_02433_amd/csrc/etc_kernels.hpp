// HIP kernels of the TPFA / DCT-preconditioned CG solver (gfx950).
//
// Data live in the canonical layout [k][a][b] (load axis k slowest, b
// contiguous).  S is the storage type of the iteration vectors (double for the
// FP64 form, float for the mixed form); the solution p is always double.
// Every reduction writes one partial per block; a one-block finalize kernel
// sums them in a fixed order, so results are bitwise reproducible.
#pragma once
#include <type_traits>

#include "etc_common.hpp"
#include "etc_fft.hpp"

namespace etc {

// Kernels launched inside the solve loop return at once when the device state
// says the solve is over (gate 1) or, for refinement work, when no refinement
// was requested in this pass (gate 2).  Standalone calls pass st = nullptr.
__device__ __forceinline__ bool gated_out(const DevState* st, int gate) {
  if (st == nullptr || gate == 0) return false;
  if (st->done) return true;
  if (gate == 2 && !st->refine) return true;
  return false;
}

// Conductivity views: storage-precision arrays of the load-axis component L
// and the two transverse components A, B (all three alias one array for an
// isotropic medium), and float64 copies when the storage rounds the input
// (null otherwise).
template <class S> struct Kap {
  const S* L;
  const S* A;
  const S* B;
  const double* hL;
  const double* hA;
  const double* hB;
  __device__ __forceinline__ double dL(int64_t i) const { return hL ? hL[i] : (double)L[i]; }
  __device__ __forceinline__ double dA(int64_t i) const { return hA ? hA[i] : (double)A[i]; }
  __device__ __forceinline__ double dB(int64_t i) const { return hB ? hB[i] : (double)B[i]; }
  // view of instance s of a batch (instances are V voxels apart)
  __host__ __device__ __forceinline__ void shift(int64_t off) {
    L += off;
    A += off;
    B += off;
    if (hL) hL += off;
    if (hA) hA += off;
    if (hB) hB += off;
  }
};

// Right-hand-side data beyond the constant Dirichlet pair, all nullable:
// a volume source per voxel (canonical layout) and Dirichlet values per face
// of the first and last load layers ([a][b]).
struct Rhs {
  const double* src;
  const double* pin;
  const double* pout;
};

// b at canonical index i (load layer k, transverse offset col): the source
// plus 2 kappa~ p_D on the Dirichlet layers (eq:flux with face data p_D).
template <class S>
__device__ __forceinline__ double rhs_at(const Geo& g, const Kap<S>& kp, const Rhs& rh, int64_t i, int64_t k,
                                         int64_t col) {
  double bv = rh.src ? rh.src[i] : 0.0;
  if (k == 0) bv += 2.0 * g.fL * kp.dL(i) * (rh.pin ? rh.pin[col] : g.p_in);
  if (k == g.nL - 1) bv += 2.0 * g.fL * kp.dL(i) * (rh.pout ? rh.pout[col] : g.p_out);
  return bv;
}

// ===================================================================== setup
// Canonical copy of the user's array (load axis -> slowest).  user dims:
// axis 0: (nL, na, nb); axis 1: (na, nL, nb).  Coalesced over b.
template <class In, class S>
__global__ void k_canon_rows(const In* __restrict__ src, S* __restrict__ dst, double* __restrict__ dst_hi, int axis,
                             Geo g) {
  if (axis == 0) {  // same layout: a converting copy
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride) {
      const double v = (double)src[i];
      dst[i] = (S)v;
      if (dst_hi) dst_hi[i] = v;
    }
    return;
  }
  // rows (k, a) over the blocks, b over the threads
  const int nrows = g.nL * g.na;
  for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
    const int k = row / g.na, a = row - k * g.na;
    const int64_t di = (int64_t)row * g.nb, si = ((int64_t)a * g.nL + k) * g.nb;
    for (int b = threadIdx.x; b < g.nb; b += blockDim.x) {
      const double v = (double)src[si + b];
      dst[di + b] = (S)v;
      if (dst_hi) dst_hi[di + b] = v;
    }
  }
}

// axis 2: user dims (na, nb, nL); 32x32 tile transpose of (b, k) per a.
template <class In, class S>
__global__ void k_canon_axis2(const In* __restrict__ src, S* __restrict__ dst, double* __restrict__ dst_hi, Geo g) {
  __shared__ double tile[32][33];
  const int64_t a = blockIdx.z;
  const int b0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int b = b0 + j, k = k0 + threadIdx.x;
    if (b < g.nb && k < g.nL) tile[j][threadIdx.x] = (double)src[(a * g.nb + b) * g.nL + k];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int k = k0 + j, b = b0 + threadIdx.x;
    if (k < g.nL && b < g.nb) {
      const double v = tile[threadIdx.x][j];
      const int64_t di = ((int64_t)k * g.na + a) * g.nb + b;
      dst[di] = (S)v;
      if (dst_hi) dst_hi[di] = v;
    }
  }
}

// Inverse permutation for the solution / gradient (double -> user layout).
__global__ void k_decanon_rows(const double* __restrict__ src, double* __restrict__ dst, int axis, Geo g) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride) {
    const int64_t k = i / g.plane, rem = i - k * g.plane;
    const int64_t a = rem / g.nb, b = rem - a * g.nb;
    const int64_t di = axis == 0 ? i : (a * g.nL + k) * g.nb + b;
    dst[di] = src[i];
  }
}

__global__ void k_decanon_axis2(const double* __restrict__ src, double* __restrict__ dst, Geo g) {
  __shared__ double tile[32][33];
  const int64_t a = blockIdx.z;
  const int b0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int k = k0 + j, b = b0 + threadIdx.x;
    if (k < g.nL && b < g.nb) tile[j][threadIdx.x] = src[((int64_t)k * g.na + a) * g.nb + b];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int b = b0 + j, k = k0 + threadIdx.x;
    if (b < g.nb && k < g.nL) dst[(a * g.nb + b) * g.nL + k] = tile[threadIdx.x][j];
  }
}

// Conductivity reads of k_extrema with one storage type for the three
// families; ISO: one array for all three (one load per voxel and neighbour).
template <class T, bool ISO> struct KapRead {
  const T *L, *A, *B;
  __device__ __forceinline__ double dL(int64_t i) const { return (double)L[i]; }
  __device__ __forceinline__ double dA(int64_t i) const { return (double)(ISO ? L : A)[i]; }
  __device__ __forceinline__ double dB(int64_t i) const { return (double)(ISO ? L : B)[i]; }
};

template <class KA>
__device__ __forceinline__ void extrema_walk(const Geo& g, const KA& kp, int kchunk, double (&mn)[5],
                                             double (&mx)[5], double& bad) {
  {
    const int nblk = gridDim.x * gridDim.y;
    const int id = xcd_tile(blockIdx.x + gridDim.x * blockIdx.y, nblk);
    const int tile = id % gridDim.x, chunk = id / gridDim.x;
    const int64_t pos = (int64_t)tile * blockDim.x + threadIdx.x;
    const int k0 = chunk * kchunk, k1 = min(g.nL, k0 + kchunk);
    if (pos < g.plane) {
      const int a = (int)(pos / g.nb), b = (int)(pos - (int64_t)a * g.nb);
      double prev = k0 > 0 ? kp.dL((int64_t)(k0 - 1) * g.plane + pos) : 1.0;
      constexpr int UX = 4;  // planes per trip, all loads issued before any use
      for (int kb = k0; kb < k1; kb += UX) {
        double kc[UX], ka[UX], kbb[UX], na_[UX], nb_[UX];
#pragma unroll
        for (int u = 0; u < UX; ++u) {
          if (kb + u < k1) {
            const int64_t i = (int64_t)(kb + u) * g.plane + pos;
            kc[u] = kp.dL(i);
            ka[u] = kp.dA(i);
            kbb[u] = kp.dB(i);
            na_[u] = a > 0 ? kp.dA(i - g.nb) : 1.0;
            nb_[u] = b > 0 ? kp.dB(i - 1) : 1.0;
          }
        }
#pragma unroll
        for (int u = 0; u < UX; ++u) {
          const int k = kb + u;
          if (k >= k1) continue;
          if (!(kc[u] > 0.0) || !isfinite(kc[u]) || !(ka[u] > 0.0) || !isfinite(ka[u]) || !(kbb[u] > 0.0) ||
              !isfinite(kbb[u]))
            bad += 1.0;
          if (k > 0) {
            const double t = g.fL * hface(kc[u], prev);
            mn[0] = fmin(mn[0], t);
            mx[0] = fmax(mx[0], t);
          }
          prev = kc[u];
          if (a > 0) {
            const double t = g.fa * hface(ka[u], na_[u]);
            mn[1] = fmin(mn[1], t);
            mx[1] = fmax(mx[1], t);
          }
          if (b > 0) {
            const double t = g.fb * hface(kbb[u], nb_[u]);
            mn[2] = fmin(mn[2], t);
            mx[2] = fmax(mx[2], t);
          }
          if (k == 0) {
            mn[3] = fmin(mn[3], g.fL * kc[u]);
            mx[3] = fmax(mx[3], g.fL * kc[u]);
          }
          if (k == g.nL - 1) {
            mn[4] = fmin(mn[4], g.fL * kc[u]);
            mx[4] = fmax(mx[4], g.fL * kc[u]);
          }
        }
      }
    }
  }
}

// Extrema of the five coefficient families (scaled harmonic faces normal to
// L, a, b; scaled load-axis conductivity of the first and last layers) and a
// count of invalid conductivities (<= 0, NaN, Inf).  12 partials per block:
// [minL maxL mina maxa minb maxb minin maxin minout maxout invalid unused].
// Block (256 threads) = 256 consecutive positions of a plane, marching over
// a chunk of `kchunk` planes (grid: plane tiles x chunks, tiles of one XCD
// adjacent): the load-axis neighbour is the thread's previous value and the
// a and b neighbours lie in lines that this XCD's blocks read at about the
// same time, so each conductivity comes from HBM about once.
template <class S>
__global__ __launch_bounds__(256) void k_extrema(Geo g, Kap<S> kp, double* __restrict__ partials, int kchunk) {
  double mn[5], mx[5];
  for (int f = 0; f < 5; ++f) {
    mn[f] = __builtin_huge_val();
    mx[f] = -__builtin_huge_val();
  }
  double bad = 0.0;
  // the float64 copy of the mixed form when there is one, else the stored arrays
  if (kp.hL && kp.hA && kp.hB) {
    if (kp.hA == kp.hL && kp.hB == kp.hL) extrema_walk(g, KapRead<double, true>{kp.hL, kp.hA, kp.hB}, kchunk, mn, mx, bad);
    else extrema_walk(g, KapRead<double, false>{kp.hL, kp.hA, kp.hB}, kchunk, mn, mx, bad);
  } else if (!kp.hL && !kp.hA && !kp.hB) {
    if (kp.A == kp.L && kp.B == kp.L) extrema_walk(g, KapRead<S, true>{kp.L, kp.A, kp.B}, kchunk, mn, mx, bad);
    else extrema_walk(g, KapRead<S, false>{kp.L, kp.A, kp.B}, kchunk, mn, mx, bad);
  } else {
    extrema_walk(g, kp, kchunk, mn, mx, bad);
  }
  __shared__ double red[12][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int f = 0; f < 5; ++f) {
    double a = mn[f], b = mx[f];
    for (int off = 32; off > 0; off >>= 1) {
      a = fmin(a, __shfl_down(a, off, 64));
      b = fmax(b, __shfl_down(b, off, 64));
    }
    if (lane == 0) {
      red[2 * f][wid] = a;
      red[2 * f + 1][wid] = b;
    }
  }
  double c = wave_sum(bad);
  if (lane == 0) red[10][wid] = c;
  __syncthreads();
  if (threadIdx.x < 11) {
    const int q = threadIdx.x;
    double v = red[q][0];
    for (int w = 1; w < 4; ++w) {
      if (q == 10) v += red[q][w];
      else if (q & 1) v = fmax(v, red[q][w]);
      else v = fmin(v, red[q][w]);
    }
    partials[(int64_t)(blockIdx.x + gridDim.x * blockIdx.y) * 12 + q] = v;
  }
}

// p = 0, r = b (source plus 2 kappa~ p_in on the first load layer and
// 2 kappa~ p_out on the last), partial ||b||^2.
template <class S>
__global__ __launch_bounds__(256) void k_init(Geo g, double* __restrict__ p, S* __restrict__ r, Kap<S> kp, Rhs rh,
                                              S* __restrict__ dlt, double* __restrict__ partials) {
  __shared__ double red[16];
  // instance blockIdx.y of a batch
  {
    const int64_t off = (int64_t)blockIdx.y * g.V;
    p += off;
    r += off;
    if (dlt) dlt += off;
    kp.shift(off);
    partials += (int64_t)blockIdx.y * gridDim.x;
  }
  double acc = 0.0;
  // rows (k, a) over the blocks, b over the threads (one index split per row)
  const int nrows = g.nL * g.na;
  for (int row = blockIdx.x; row < nrows; row += gridDim.x) {
    const int k = row / g.na;
    const int64_t r0 = (int64_t)row * g.nb, c0 = (int64_t)(row - k * g.na) * g.nb;
    for (int b = threadIdx.x; b < g.nb; b += blockDim.x) {
      const int64_t i = r0 + b;
      const double bv = rhs_at(g, kp, rh, i, (int64_t)k, c0 + b);
      p[i] = 0.0;
      if (dlt) dlt[i] = S(0);
      const S bs = (S)bv;
      r[i] = bs;
      acc += (double)bs * (double)bs;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ================================================================== operator
// q = A w (7-point TPFA stencil, harmonic-mean faces recomputed from kappa)
// with the partial w . q of each block, for orthotropic kappa (the isotropic
// operator is k_apply_A_iso below).
// 2.5D tiling: a block of 64 x 4 threads owns a tile of 64 (b) x 16 (a)
// columns (4 rows per thread) and marches along k over `kchunk` planes.  The
// current plane of w and kappa sits in LDS with a one-voxel halo (lateral
// neighbours); planes k-1 and k+1 stay in registers.  Tile centres are
// prefetched two planes ahead and halos one plane ahead, so every HBM value is
// read once per sweep plus the halo rows.  (ORTHO: the a and b faces use their
// own conductivity components, read from the caches.)
constexpr int ATB = 64, ATA = 16, ARPT = 4;  // tile width (b), height (a), rows per thread

template <class S, class C, bool ORTHO>
__global__ __launch_bounds__(256) void k_apply_A(Geo g, const S* __restrict__ w, Kap<S> kp, S* __restrict__ q,
                                                 double* __restrict__ partials, const DevState* __restrict__ st,
                                                 int gate, int kchunk) {
  // tile (bx, by, bz), bz = instance * chunks + chunk (instances of a batch
  // are V apart), renumbered so that neighbouring tiles share an XCD; the
  // partial sums are stored by tile so that each instance's are contiguous
  const int ntile = gridDim.x * gridDim.y * gridDim.z;
  const int tile = xcd_tile(flat_block(), ntile);
  const int bx = tile % gridDim.x, by = (tile / gridDim.x) % gridDim.y, bz = tile / (gridDim.x * gridDim.y);
  const int nch = (g.nL + kchunk - 1) / kchunk;
  const int inst = bz / nch, chunk = bz - inst * nch;
  if (st) st += inst;
  if (gated_out(st, gate)) return;
  {
    const int64_t off = (int64_t)inst * g.V;
    w += off;
    q += off;
    kp.shift(off);
  }
  __shared__ C tw_[ATA + 2][ATB + 2];
  __shared__ C tk_[ATA + 2][ATB + 2];
  __shared__ double red[16];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int b0 = bx * ATB, a0 = by * ATA;
  const int b = b0 + tx;
  const int k0 = chunk * kchunk;
  const int k1 = min(g.nL, k0 + kchunk);
  const S* __restrict__ ks = kp.L;
  const S* __restrict__ ka = ORTHO ? kp.A : kp.L;
  const S* __restrict__ kb = ORTHO ? kp.B : kp.L;
  const C fL = (C)g.fL, fa = (C)g.fa, fb = (C)g.fb;
  const bool bok = b < g.nb;
  bool rok[ARPT];
  int64_t col[ARPT];
#pragma unroll
  for (int j = 0; j < ARPT; ++j) {
    const int a = a0 + ty + 4 * j;
    rok[j] = bok && a < g.na;
    col[j] = (int64_t)a * g.nb + b;
  }
  // halo element of this thread: top row (ty 0), bottom row (ty 1), left
  // column (ty 2, tx < 16), right column (ty 3, tx < 16)
  int hr = -1, hc = -1;
  int64_t hcol = 0;
  {
    int ha = -1, hb = -1;
    if (ty == 0) { ha = a0 - 1; hb = b; hr = 0; hc = tx + 1; }
    else if (ty == 1) { ha = a0 + ATA; hb = b; hr = ATA + 1; hc = tx + 1; }
    else if (tx < ATA) { ha = a0 + tx; hb = (ty == 2) ? b0 - 1 : b0 + ATB; hr = tx + 1; hc = (ty == 2) ? 0 : ATB + 1; }
    if (ha < 0 || ha >= g.na || hb < 0 || hb >= g.nb) hr = -1;
    else hcol = (int64_t)ha * g.nb + hb;
  }
  auto ld = [&](const S* __restrict__ arr, int k, int64_t c, bool ok, C dflt) -> C {
    return (ok && k >= 0 && k < g.nL) ? (C)arr[(int64_t)k * g.plane + c] : dflt;
  };
  C wm[ARPT], km[ARPT], wc[ARPT], kc[ARPT], wn[ARPT], kn[ARPT];
#pragma unroll
  for (int j = 0; j < ARPT; ++j) {
    wm[j] = ld(w, k0 - 1, col[j], rok[j], C(0));
    km[j] = ld(ks, k0 - 1, col[j], rok[j], C(1));
    wc[j] = ld(w, k0, col[j], rok[j], C(0));
    kc[j] = ld(ks, k0, col[j], rok[j], C(1));
    wn[j] = ld(w, k0 + 1, col[j], rok[j], C(0));
    kn[j] = ld(ks, k0 + 1, col[j], rok[j], C(1));
  }
  C hw = ld(w, k0, hcol, hr >= 0, C(0)), hk = ld(ks, k0, hcol, hr >= 0, C(1));
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    // prefetch: centres of plane k+2, halo of plane k+1
    C wnn[ARPT], knn[ARPT];
    const bool more = k + 1 < k1;
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      wnn[j] = ld(w, k + 2, col[j], rok[j] && more, C(0));
      knn[j] = ld(ks, k + 2, col[j], rok[j] && more, C(1));
    }
    const C hwn = ld(w, k + 1, hcol, hr >= 0 && more, C(0)), hkn = ld(ks, k + 1, hcol, hr >= 0 && more, C(1));
    __syncthreads();  // previous plane's LDS reads are done
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      tw_[1 + ty + 4 * j][1 + tx] = wc[j];
      tk_[1 + ty + 4 * j][1 + tx] = kc[j];
    }
    if (hr >= 0) {
      tw_[hr][hc] = hw;
      tk_[hr][hc] = hk;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      if (rok[j]) {
        const int a = a0 + ty + 4 * j;
        const int r = 1 + ty + 4 * j, cc = 1 + tx;
        const C w0 = wc[j], k0v = kc[j];
        C qv;
        if (k > 0) qv = fL * harm(k0v, km[j]) * (w0 - wm[j]);
        else qv = C(2) * fL * k0v * w0;
        if (k + 1 < g.nL) qv += fL * harm(k0v, kn[j]) * (w0 - wn[j]);
        else qv += C(2) * fL * k0v * w0;
        if (ORTHO) {
          const int64_t ii = (int64_t)k * g.plane + col[j];
          const C kac = (C)ka[ii], kbc = (C)kb[ii];
          if (a > 0) qv += fa * harm(kac, (C)ka[ii - g.nb]) * (w0 - tw_[r - 1][cc]);
          if (a + 1 < g.na) qv += fa * harm(kac, (C)ka[ii + g.nb]) * (w0 - tw_[r + 1][cc]);
          if (b > 0) qv += fb * harm(kbc, (C)kb[ii - 1]) * (w0 - tw_[r][cc - 1]);
          if (b + 1 < g.nb) qv += fb * harm(kbc, (C)kb[ii + 1]) * (w0 - tw_[r][cc + 1]);
        } else {
          if (a > 0) qv += fa * harm(k0v, tk_[r - 1][cc]) * (w0 - tw_[r - 1][cc]);
          if (a + 1 < g.na) qv += fa * harm(k0v, tk_[r + 1][cc]) * (w0 - tw_[r + 1][cc]);
          if (b > 0) qv += fb * harm(k0v, tk_[r][cc - 1]) * (w0 - tw_[r][cc - 1]);
          if (b + 1 < g.nb) qv += fb * harm(k0v, tk_[r][cc + 1]) * (w0 - tw_[r][cc + 1]);
        }
        const S qs = (S)qv;
        q[(int64_t)k * g.plane + col[j]] = qs;
        acc += (double)w0 * (double)qs;
      }
    }
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      wm[j] = wc[j];
      km[j] = kc[j];
      wc[j] = wn[j];
      kc[j] = kn[j];
      wn[j] = wnn[j];
      kn[j] = knn[j];
    }
    hw = hwn;
    hk = hkn;
  }
  if (partials) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[tile] = s;
  }
}

// Isotropic operator with every face coefficient computed once: block
// (TBW, TAH / 4) owns a TBW (b) x TAH (a) tile, and thread (x, y) holds the
// four consecutive rows a0 + 4y .. a0 + 4y + 3 of column b0 + x.  Load-axis
// faces are carried from one plane to the next, the faces between a thread's
// own rows are shared in registers (five a faces per four voxels), each b
// face is computed by its left voxel and passed on by a lane shift, and the
// four faces left of a wave's first column by its lanes 0..3.  Out-of-range
// neighbours read finite defaults from LDS and get a zero coefficient.
//
// RES = true: the float64 true residual r = b - A p of the mixed form (p
// float64, kappa read as KT, arithmetic in C = double, r stored as S, partial
// ||r||^2); RES = false: q = A w with the partial w . q, all in S.
template <class S, bool RES, class KT, int TBW, int TAH, class BG, bool PLAIN = false>
__device__ __forceinline__ void k_apply_A_iso_body(const BG bg, Geo g, const typename std::conditional<RES, double, S>::type* __restrict__ w,
                                                     Kap<S> kp, const KT* __restrict__ ks, Rhs rh,
                                                     S* __restrict__ q, double* __restrict__ partials,
                                                     const DevState* __restrict__ st, int gate, int kchunk) {
  using C = typename std::conditional<RES, double, S>::type;
  const int ntile = bg.gx() * bg.gy() * bg.gz();
  const int tile = xcd_tile(bg.flat(), ntile);
  const int bx = tile % bg.gx(), by = (tile / bg.gx()) % bg.gy(), bz = tile / (bg.gx() * bg.gy());
  const int nch = (g.nL + kchunk - 1) / kchunk;
  const int inst = bz / nch, chunk = bz - inst * nch;
  if (st) st += inst;
  if (gated_out(st, gate)) return;
  {
    const int64_t off = (int64_t)inst * g.V;
    w += off;
    q += off;
    ks += off;
    kp.shift(off);
    if (RES && rh.src) rh.src += off;
  }
  static_assert(TAH % ARPT == 0 && TAH >= 16 && TBW >= TAH && TBW % 64 == 0, "tile shape");
  // two LDS planes, used alternately: a plane is written while the previous
  // one may still be read, so one barrier per plane suffices
  __shared__ C tw2_[2][TAH + 2][TBW + 2];
  __shared__ C tk2_[2][TAH + 2][TBW + 2];
  __shared__ double red[16];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int b0 = bx * TBW, a0 = by * TAH;
  const int b = b0 + tx;
  const int k0 = chunk * kchunk;
  const int k1 = min(g.nL, k0 + kchunk);
  const C fL = (C)g.fL, fa = (C)g.fa, fb = (C)g.fb;
  const int64_t plane = g.plane;
  const bool bok = b < g.nb;
  const int abase = a0 + ARPT * ty;  // first row of this thread
  const int rbase = 1 + ARPT * ty;   // its LDS row
  bool rok[ARPT];
  int64_t col[ARPT];
#pragma unroll
  for (int j = 0; j < ARPT; ++j) {
    rok[j] = bok && (abase + j) < g.na;
    col[j] = (int64_t)(abase + j) * g.nb + b;
  }
  // halo slot of this thread (always written: loaded value or a default):
  // top row (ty 0), bottom row (ty 1), left column (ty 2, tx < 16), right
  // column (ty 3, tx < 16)
  int hr = -1, hc = 0;
  bool hok = false;
  int64_t hcol = 0;
  {
    int ha = -1, hb = -1;
    if (ty == 0) { ha = a0 - 1; hb = b; hr = 0; hc = tx + 1; }
    else if (ty == 1) { ha = a0 + TAH; hb = b; hr = TAH + 1; hc = tx + 1; }
    else if (ty <= 3 && tx < TAH) {
      ha = a0 + tx; hb = (ty == 2) ? b0 - 1 : b0 + TBW; hr = tx + 1; hc = (ty == 2) ? 0 : TBW + 1;
    }
    hok = hr >= 0 && ha >= 0 && ha < g.na && hb >= 0 && hb < g.nb;
    if (hok) hcol = (int64_t)ha * g.nb + hb;
  }
  auto ld = [&](const auto* __restrict__ arr, int k, int64_t c, bool ok, C dflt) -> C {
    return (ok && k >= 0 && k < g.nL) ? (C)arr[(int64_t)k * plane + c] : dflt;
  };
  // which faces exist
  const bool bl_ok = b0 + tx > 0, br_ok = b + 1 < g.nb;
  bool fa_ok[ARPT + 1];
#pragma unroll
  for (int i = 0; i <= ARPT; ++i) {
    const int ar = abase + i;  // face between rows ar - 1 and ar
    fa_ok[i] = ar >= 1 && ar < g.na;
  }
  C wm[ARPT], wc[ARPT], kc[ARPT], wn[ARPT], kn[ARPT], tdn[ARPT];
#pragma unroll
  for (int j = 0; j < ARPT; ++j) {
    wm[j] = ld(w, k0 - 1, col[j], rok[j], C(0));
    const C km = ld(ks, k0 - 1, col[j], rok[j], C(1));
    wc[j] = ld(w, k0, col[j], rok[j], C(0));
    kc[j] = ld(ks, k0, col[j], rok[j], C(1));
    wn[j] = ld(w, k0 + 1, col[j], rok[j], C(0));
    kn[j] = ld(ks, k0 + 1, col[j], rok[j], C(1));
    // face below plane k0: interior harmonic mean or the Dirichlet face 2 kappa
    tdn[j] = (k0 > 0) ? hface(km, kc[j]) : C(2) * kc[j];
  }
  C hw = ld(w, k0, hcol, hok, C(0)), hk = ld(ks, k0, hcol, hok, C(1));
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    // prefetch: centres of plane k+2, halo of plane k+1
    C wnn[ARPT], knn[ARPT];
    const bool more = k + 1 < k1;
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      wnn[j] = ld(w, k + 2, col[j], rok[j] && more, C(0));
      knn[j] = ld(ks, k + 2, col[j], rok[j] && more, C(1));
    }
    const C hwn = ld(w, k + 1, hcol, hok && more, C(0)), hkn = ld(ks, k + 1, hcol, hok && more, C(1));
    // this plane's buffer was last read two planes ago, before the barrier
    // that followed the previous plane's writes
    C(&tw_)[TAH + 2][TBW + 2] = tw2_[(k - k0) & 1];
    C(&tk_)[TAH + 2][TBW + 2] = tk2_[(k - k0) & 1];
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      tw_[rbase + j][1 + tx] = wc[j];
      tk_[rbase + j][1 + tx] = kc[j];
    }
    if (hr >= 0) {
      tw_[hr][hc] = hw;
      tk_[hr][hc] = hk;
    }
    __syncthreads();
    const int cc = 1 + tx;
    // load-axis face above this plane (Dirichlet face 2 kappa on the last layer)
    C tup[ARPT];
#pragma unroll
    for (int j = 0; j < ARPT; ++j) tup[j] = (k + 1 < g.nL) ? hface(kc[j], kn[j]) : C(2) * kc[j];
    // a faces: fa_[i] between rows i - 1 and i of this thread (i = 0: the row above)
    C fav[ARPT + 1];
    fav[0] = fa_ok[0] ? hface(tk_[rbase - 1][cc], kc[0]) : C(0);
#pragma unroll
    for (int i = 1; i < ARPT; ++i) fav[i] = fa_ok[i] ? hface(kc[i - 1], kc[i]) : C(0);
    fav[ARPT] = fa_ok[ARPT] ? hface(kc[ARPT - 1], tk_[rbase + ARPT][cc]) : C(0);
    // b faces: right face here, left face from the lane to the left; lanes
    // 0..3 compute the faces left of column b0 for rows 0..3 of this wave
    C fr[ARPT], fl[ARPT];
#pragma unroll
    for (int j = 0; j < ARPT; ++j) fr[j] = br_ok ? hface(kc[j], tk_[rbase + j][cc + 1]) : C(0);
    const int lane = tx & 63, cw = 1 + (tx - lane);  // LDS column of the wave's first lane
    const int hl = lane & (ARPT - 1);
    const C edge = hface(tk_[rbase + hl][cw - 1], tk_[rbase + hl][cw]);
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      const C up = __shfl_up(fr[j], 1, 64);
      const C e = __shfl(edge, j, 64);
      fl[j] = bl_ok ? (lane == 0 ? e : up) : C(0);
    }
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      const int r = rbase + j;
      const C w0 = wc[j];
      const C wa_ = (j == 0) ? tw_[r - 1][cc] : wc[j - 1];
      const C wb_ = (j == ARPT - 1) ? tw_[r + 1][cc] : wc[j + 1];
      C qv = fL * (tdn[j] * (w0 - wm[j]) + tup[j] * (w0 - wn[j]));
      qv += fa * (fav[j] * (w0 - wa_) + fav[j + 1] * (w0 - wb_));
      qv += fb * (fl[j] * (w0 - tw_[r][cc - 1]) + fr[j] * (w0 - tw_[r][cc + 1]));
      if (rok[j]) {
        const int64_t gi = (int64_t)k * plane + col[j];
        if constexpr (RES) {
          // PLAIN: no source and constant Dirichlet data, so b is the
          // boundary term of the first and last layers, whose conductivity
          // is this voxel's (the same value rhs_at reads)
          double bv;
          if constexpr (PLAIN) {
            bv = 0.0;
            if (k == 0) bv += 2.0 * g.fL * (double)kc[j] * g.p_in;
            if (k == g.nL - 1) bv += 2.0 * g.fL * (double)kc[j] * g.p_out;
          } else {
            bv = rhs_at(g, kp, rh, gi, k, col[j]);
          }
          const S rs = (S)(bv - qv);
          q[gi] = rs;
          acc += (double)rs * (double)rs;
        } else {
          const S qs = (S)qv;
          q[gi] = qs;
          acc += (double)w0 * (double)qs;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < ARPT; ++j) {
      tdn[j] = tup[j];
      wm[j] = wc[j];
      wc[j] = wn[j];
      kc[j] = kn[j];
      wn[j] = wnn[j];
      kn[j] = knn[j];
    }
    hw = hwn;
    hk = hkn;
  }
  if (partials) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[tile] = s;
  }
}

template <class S, bool RES, class KT, int TBW, int TAH, bool PLAIN = false>
__global__ __launch_bounds__(TBW*(TAH / 4)) void k_apply_A_iso(Geo g, const typename std::conditional<RES, double, S>::type* __restrict__ w,
                                                     Kap<S> kp, const KT* __restrict__ ks, Rhs rh,
                                                     S* __restrict__ q, double* __restrict__ partials,
                                                     const DevState* __restrict__ st, int gate, int kchunk) {
  k_apply_A_iso_body<S, RES, KT, TBW, TAH, HwGrid, PLAIN>(HwGrid{}, g, w, kp, ks, rh, q, partials, st, gate, kchunk);
}

// r = b - A p in double arithmetic (p double, kappa at its input precision),
// stored at S precision, with the partial ||r||^2, for orthotropic kappa (the
// isotropic residual is k_apply_A_iso<S, true>).  Columns of 64 b x 4 a
// march along k; lateral neighbours come through the caches (tiles
// renumbered per XCD as in k_apply_A).
template <class S, bool ORTHO>
__global__ __launch_bounds__(256) void k_residual(Geo g, const double* __restrict__ p, Kap<S> kp, Rhs rh,
                                                  S* __restrict__ r, double* __restrict__ partials,
                                                  const DevState* __restrict__ st, int gate, int kchunk) {
  const int tile = xcd_tile(flat_block(), gridDim.x * gridDim.y * gridDim.z);
  const int bx = tile % gridDim.x, by = (tile / gridDim.x) % gridDim.y, bz = tile / (gridDim.x * gridDim.y);
  const int nch = (g.nL + kchunk - 1) / kchunk;
  const int inst = bz / nch, chunk = bz - inst * nch;
  if (st) st += inst;
  if (gated_out(st, gate)) return;
  {
    const int64_t off = (int64_t)inst * g.V;
    p += off;
    r += off;
    kp.shift(off);
    if (rh.src) rh.src += off;
  }
  __shared__ double red[16];
  const int b = bx * 64 + threadIdx.x;
  const int a = by * 4 + threadIdx.y;
  const int k0 = chunk * kchunk;
  const int k1 = min(g.nL, k0 + kchunk);
  const bool valid = (a < g.na) && (b < g.nb);
  double acc = 0.0;
  if (valid) {
    const int64_t col = (int64_t)a * g.nb + b;
    int64_t i = (int64_t)k0 * g.plane + col;
    double pc = p[i], kc = kp.dL(i);
    double pm = 0.0, km = 1.0;
    if (k0 > 0) {
      pm = p[i - g.plane];
      km = kp.dL(i - g.plane);
    }
    // load-axis face below the current plane (carried from plane to plane)
    double tdn = (k0 > 0) ? hface(kc, km) : 2.0 * kc;
    double pp = 0.0, kpp = 1.0;
    if (k0 + 1 < g.nL) {
      pp = p[i + g.plane];
      kpp = kp.dL(i + g.plane);
    }
    for (int k = k0; k < k1; ++k, i += g.plane) {
      // prefetch the plane after next
      double pn = 0.0, kn = 1.0;
      if (k + 2 < g.nL && k + 1 < k1) {
        pn = p[i + 2 * g.plane];
        kn = kp.dL(i + 2 * g.plane);
      }
      const double tup = (k + 1 < g.nL) ? hface(kc, kpp) : 2.0 * kc;
      double qv = g.fL * (tdn * (pc - pm) + tup * (pc - pp));
      const double kac = ORTHO ? kp.dA(i) : kc, kbc = ORTHO ? kp.dB(i) : kc;
      if (ORTHO) {
        if (a > 0) qv += g.fa * hface(kac, kp.dA(i - g.nb)) * (pc - p[i - g.nb]);
        if (a + 1 < g.na) qv += g.fa * hface(kac, kp.dA(i + g.nb)) * (pc - p[i + g.nb]);
        if (b > 0) qv += g.fb * hface(kbc, kp.dB(i - 1)) * (pc - p[i - 1]);
        if (b + 1 < g.nb) qv += g.fb * hface(kbc, kp.dB(i + 1)) * (pc - p[i + 1]);
      } else {
        if (a > 0) qv += g.fa * hface(kc, kp.dL(i - g.nb)) * (pc - p[i - g.nb]);
        if (a + 1 < g.na) qv += g.fa * hface(kc, kp.dL(i + g.nb)) * (pc - p[i + g.nb]);
        if (b > 0) qv += g.fb * hface(kc, kp.dL(i - 1)) * (pc - p[i - 1]);
        if (b + 1 < g.nb) qv += g.fb * hface(kc, kp.dL(i + 1)) * (pc - p[i + 1]);
      }
      const S rs = (S)(rhs_at(g, kp, rh, i, k, col) - qv);
      r[i] = rs;
      acc += (double)rs * (double)rs;
      tdn = tup;
      pm = pc;
      pc = pp;
      kc = kpp;
      pp = pn;
      kpp = kn;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[tile] = s;
}

// ============================================================ DCT along rows
// Global loads are issued in batches of UNR per thread before their LDS
// stores, so every wave keeps several HBM requests in flight.
constexpr int UNR = 8;

// Compile-time shape of the DCT kernels: NC = 0 takes every length and
// launch shape from the plan at run time; NC > 0 fixes the transform length
// (even, FFT route) and with it the line stride and lines per block.
template <class T, int NC> struct DctShape {
  static constexpr bool ct = NC > 0;
  static constexpr int M = NC / 2;
  static constexpr int ls = ct ? fft_lstride(M) : 0;
  static constexpr int rows = ct ? rows_lines(M, ls, (int)sizeof(T), true) : 0;
  static constexpr int cols = ct ? cols_tile(M, ls, (int)sizeof(T), true) : 0;
  static constexpr int col_threads = cols_threads((int)sizeof(T));
  // loads per thread that cover a whole block in one batch (all in flight)
  static constexpr int row_elems = ct ? (rows * NC + 255) / 256 : 0;
  static constexpr int row_items = ct ? (rows * (M / 2 + 1) + 255) / 256 : 0;
  static constexpr int col_elems = ct ? (cols * NC + col_threads - 1) / col_threads : 0;
  static constexpr int col_items = ct ? (cols * (M / 2 + 1) + col_threads - 1) / col_threads : 0;
};

// Unroll of a load batch: the whole block when the shape is compile-time
// (capped by a register budget of `cap` values per thread), else `dflt`.
__host__ __device__ constexpr int batch_of(int whole, int cap, int dflt) {
  return whole > 0 ? (whole < cap ? whole : cap) : dflt;
}

// 16-byte vector of storage values (global loads and stores of 4 float32 or
// 2 float64 per lane).
template <class S> struct alignas(16) V16 {
  static constexpr int n = 16 / (int)sizeof(S);
  S v[n];
};
template <class S> __device__ __forceinline__ V16<S> ld16(const S* p) { return *reinterpret_cast<const V16<S>*>(p); }
template <class S> __device__ __forceinline__ void st16(S* p, const V16<S>& x) { *reinterpret_cast<V16<S>*>(p) = x; }

// Rows are the contiguous b lines; a block owns `rpb` whole rows.
// MODE 0: t = DCT_b(src).  MODE 1 (fused PCG update): r -= alpha q, partial
// ||r||^2, t = DCT_b(r).  (The solution update x += alpha w is done by the
// backward row transform, which reads w anyway.)
template <class S, class T, int MODE, int NC, class BG>
__device__ __forceinline__ void k_rows_fwd_body(const BG bg, Geo g, DctPlan dp, const cx<T>* __restrict__ tw,
                                                  const S* __restrict__ src, S* __restrict__ dst, int rpb, int nrows,
                                                  S* __restrict__ r, const S* __restrict__ q,
                                                  double* __restrict__ partials, const DevState* __restrict__ st,
                                                  int gate) {
  using Sh = DctShape<T, NC>;
  // instance bg.by() of a batch
  if (st) st += bg.by();
  if (gated_out(st, gate)) return;
  {
    const int64_t off = (int64_t)bg.by() * g.V;
    if (src) src += off;
    dst += off;
    if (MODE == 1) {
      r += off;
      q += off;
      partials += (int64_t)bg.by() * bg.gx();
    }
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  __shared__ double red[16];
  const int tid = threadIdx.x;
  constexpr int nthr = 256;
  const int N = Sh::ct ? NC : dp.N;
  const int M = Sh::ct ? Sh::M : dp.M;
  const bool fft = Sh::ct ? true : (dp.fft != 0);
  const int ls = Sh::ct ? Sh::ls : dp.lstride;
  const int rpbv = Sh::ct ? Sh::rows : rpb;
  const int64_t row0 = (int64_t)bg.bx() * rpbv;
  const int lines = (int)min((int64_t)rpbv, (int64_t)nrows - row0);
  const int64_t base = row0 * N;
  const int total = lines * N;
  double acc = 0.0;
  double alpha = 0.0;
  if (MODE == 1) alpha = st->alpha;
  // load (and update) the rows into LDS, reordered for the FFT route; each
  // batch issues all its loads before the first use (64 registers of values)
  constexpr int U = (MODE == 1) ? batch_of(Sh::row_elems, 16, 4) : batch_of(Sh::row_elems, 64 / ((int)sizeof(S) / 4), UNR);
  auto put = [&](int e, T v) {
    const int line = e / N, j = e - line * N;
    T* L = reinterpret_cast<T*>(buf + line * ls);
    if (fft) L[vpos(dct_perm(j, N))] = v;
    else L[j] = v;
  };
  if constexpr (Sh::ct) {
    // compile-time lengths (multiples of 4): 16-byte accesses, batches of
    // UV vectors per thread
    using Vt = V16<S>;
    constexpr int VW = Vt::n;
    constexpr int UV = (MODE == 1) ? 16 / VW : 32 / VW;
    for (int v0 = tid; v0 * VW < total; v0 += nthr * UV) {
      Vt a[UV], b[UV];
#pragma unroll
      for (int u = 0; u < UV; ++u) {
        const int e = (v0 + u * nthr) * VW;
        if (e < total) {
          if (MODE == 1) {
            a[u] = ld16(r + base + e);
            b[u] = ld16(q + base + e);
          } else {
            a[u] = ld16(src + base + e);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UV; ++u) {
        const int e = (v0 + u * nthr) * VW;
        if (e < total) {
          if (MODE == 1) {
            Vt o;
#pragma unroll
            for (int i = 0; i < VW; ++i) {
              o.v[i] = (S)((double)a[u].v[i] - alpha * (double)b[u].v[i]);
              acc += (double)o.v[i] * (double)o.v[i];
              put(e + i, (T)o.v[i]);
            }
            st16(r + base + e, o);
          } else {
#pragma unroll
            for (int i = 0; i < VW; ++i) put(e + i, (T)a[u].v[i]);
          }
        }
      }
    }
  } else
  for (int e0 = tid; e0 < total; e0 += nthr * U) {
    if (MODE == 1) {
      S rv[U], qv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * nthr;
        if (e < total) {
          rv[u] = r[base + e];
          qv[u] = q[base + e];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * nthr;
        if (e < total) {
          const S rs = (S)((double)rv[u] - alpha * (double)qv[u]);
          r[base + e] = rs;
          acc += (double)rs * (double)rs;
          put(e, (T)rs);
        }
      }
    } else {
      S xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * nthr;
        if (e < total) xv[u] = src[base + e];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * nthr;
        if (e < total) put(e, (T)xv[u]);
      }
    }
  }
  __syncthreads();
  if (fft) {
    if constexpr (Sh::ct) lds_fft_ct<T, -1, Sh::M, Sh::rows, nthr, Sh::ls>(buf, tw, tid);
    else lds_fft<T, -1>(buf, lines, ls, dp, tw, tid, nthr);
    const int nit = M / 2 + 1;
    for (int e = tid; e < lines * nit; e += nthr) {
      const int line = e / nit, k = e - line * nit;
      S* out = dst + base + (int64_t)line * N;
      dct_post(buf + line * ls, k, N, M, tw, [&](int idx, T v) { out[idx] = (S)v; });
    }
  } else {
    const int N4 = 4 * N;
    for (int e = tid; e < total; e += nthr) {
      const int line = e / N, k = e - line * N;
      const T* L = reinterpret_cast<const T*>(buf + line * ls);
      T s = T(0);
      for (int n = 0; n < N; ++n) s += L[n] * tw[((2 * n + 1) * k) % N4].re;
      dst[base + e] = (S)s;
    }
  }
  if (MODE == 1) {
    const double s = block_sum(acc, red);
    if (tid == 0) partials[bg.bx()] = s;
  }
}

template <class S, class T, int MODE, int NC = 0>
__global__ __launch_bounds__(256) void k_rows_fwd(Geo g, DctPlan dp, const cx<T>* __restrict__ tw,
                                                  const S* __restrict__ src, S* __restrict__ dst, int rpb, int nrows,
                                                  S* __restrict__ r, const S* __restrict__ q,
                                                  double* __restrict__ partials, const DevState* __restrict__ st,
                                                  int gate) {
  k_rows_fwd_body<S, T, MODE, NC, HwGrid>(HwGrid{}, g, dp, tw, src, dst, rpb, nrows, r, q, partials, st, gate);
}

// Inverse along rows.  MODE 0: dst = DCT_b^{-1}(src).  MODE 1: dst holds w on
// entry; x += alpha w (the solution update of this pass; skipped when a
// refinement already folded it into p), then w = z + beta w with
// z = DCT_b^{-1}(src) (never stored).  x is the solution p in the FP64 form
// and the float32 increment since the last refinement in the mixed form.
template <class S, class T, int MODE, int NC, class BG>
__device__ __forceinline__ void k_rows_inv_body(const BG bg, Geo g, DctPlan dp, const cx<T>* __restrict__ tw,
                                                  const S* __restrict__ src, S* __restrict__ dst, int rpb, int nrows,
                                                  S* __restrict__ xs, const DevState* __restrict__ st, int gate) {
  using Sh = DctShape<T, NC>;
  if (st) st += bg.by();
  if (gated_out(st, gate)) return;
  {
    const int64_t off = (int64_t)bg.by() * g.V;
    src += off;
    dst += off;
    if (MODE == 1) xs += off;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  constexpr int nthr = 256;
  const int N = Sh::ct ? NC : dp.N;
  const int M = Sh::ct ? Sh::M : dp.M;
  const bool fft = Sh::ct ? true : (dp.fft != 0);
  const int ls = Sh::ct ? Sh::ls : dp.lstride;
  const int rpbv = Sh::ct ? Sh::rows : rpb;
  const int64_t row0 = (int64_t)bg.bx() * rpbv;
  const int lines = (int)min((int64_t)rpbv, (int64_t)nrows - row0);
  const int64_t base = row0 * N;
  const int total = lines * N;
  double beta = 0.0, alpha = 0.0;
  if (MODE == 1) {
    beta = st->beta;
    alpha = st->refine ? 0.0 : st->alpha;  // a refinement already moved p
  }
  if (fft) {
    const int nit = M / 2 + 1;
    const int items = lines * nit;
    constexpr int UI = batch_of(Sh::row_items, 64 / (4 * ((int)sizeof(S) / 4)), 4);
    for (int e0 = tid; e0 < items; e0 += nthr * UI) {
      T xv[UI][4];
#pragma unroll
      for (int u = 0; u < UI; ++u) {
        const int e = e0 + u * nthr;
        if (e < items) {
          const int line = e / nit, k = e - line * nit;
          const S* in = src + base + (int64_t)line * N;
          int i0, i1, i2, i3;
          pre_inv_idx(k, N, M, i0, i1, i2, i3);
          xv[u][0] = (T)in[i0];
          xv[u][1] = (T)in[i1];
          xv[u][2] = (T)in[i2];
          xv[u][3] = (T)in[i3];
        }
      }
#pragma unroll
      for (int u = 0; u < UI; ++u) {
        const int e = e0 + u * nthr;
        if (e < items) {
          const int line = e / nit, k = e - line * nit;
          dct_pre_inv_vals(buf + line * ls, k, M, tw, xv[u][0], xv[u][1], xv[u][2], xv[u][3]);
        }
      }
    }
    __syncthreads();
    if constexpr (Sh::ct) lds_fft_ct<T, +1, Sh::M, Sh::rows, nthr, Sh::ls>(buf, tw, tid);
    else lds_fft<T, +1>(buf, lines, ls, dp, tw, tid, nthr);
    const T invM = T(1) / T(M);
    constexpr int UO = (MODE == 1) ? batch_of(Sh::row_elems, 32 / ((int)sizeof(S) / 4), UNR / 2)
                                   : batch_of(Sh::row_elems, 64 / ((int)sizeof(S) / 4), UNR);
    if constexpr (Sh::ct) {
      // 16-byte accesses (compile-time lengths are multiples of 4)
      using Vt = V16<S>;
      constexpr int VW = Vt::n;
      constexpr int UV = 32 / VW;
      for (int v0 = tid; v0 * VW < total; v0 += nthr * UV) {
        Vt wa[UV], xa[UV];
        if (MODE == 1) {
#pragma unroll
          for (int u = 0; u < UV; ++u) {
            const int e = (v0 + u * nthr) * VW;
            if (e < total) {
              wa[u] = ld16(dst + base + e);
              xa[u] = ld16(xs + base + e);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < UV; ++u) {
          const int e = (v0 + u * nthr) * VW;
          if (e < total) {
            const int line = e / N, j0 = e - line * N;
            const T* L = reinterpret_cast<const T*>(buf + line * ls);
            Vt wo, xo;
#pragma unroll
            for (int i = 0; i < VW; ++i) {
              const T z = L[vpos(dct_perm(j0 + i, N))] * invM;
              if (MODE == 1) {
                xo.v[i] = (S)((double)xa[u].v[i] + alpha * (double)wa[u].v[i]);
                wo.v[i] = (S)((double)z + beta * (double)wa[u].v[i]);
              } else {
                wo.v[i] = (S)z;
              }
            }
            st16(dst + base + e, wo);
            if (MODE == 1) st16(xs + base + e, xo);
          }
        }
      }
    } else {
    S wv[UO], xv[UO];
    for (int e0 = tid; e0 < total; e0 += nthr * UO) {
      if (MODE == 1) {
#pragma unroll
        for (int u = 0; u < UO; ++u) {
          const int e = e0 + u * nthr;
          if (e < total) {
            wv[u] = dst[base + e];
            xv[u] = xs[base + e];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UO; ++u) {
        const int e = e0 + u * nthr;
        if (e < total) {
          const int line = e / N, j = e - line * N;
          const T* L = reinterpret_cast<const T*>(buf + line * ls);
          const T z = L[vpos(dct_perm(j, N))] * invM;
          if (MODE == 1) {
            xs[base + e] = (S)((double)xv[u] + alpha * (double)wv[u]);
            dst[base + e] = (S)((double)z + beta * (double)wv[u]);
          } else {
            dst[base + e] = (S)z;
          }
        }
      }
    }
    }
  } else {
    for (int e = tid; e < total; e += nthr) {
      const int line = e / N, j = e - line * N;
      T* L = reinterpret_cast<T*>(buf + line * ls);
      L[j] = (T)src[base + e];
    }
    __syncthreads();
    const int N4 = 4 * N;
    const T sc = T(2) / T(N);
    for (int e = tid; e < total; e += nthr) {
      const int line = e / N, n = e - line * N;
      const T* L = reinterpret_cast<const T*>(buf + line * ls);
      T s = T(0.5) * L[0];
      for (int k = 1; k < N; ++k) s += L[k] * tw[((2 * n + 1) * k) % N4].re;
      const T z = sc * s;
      const int64_t gi = base + e;
      if (MODE == 1) {
        const double wv = (double)dst[gi];
        xs[gi] = (S)((double)xs[gi] + alpha * wv);
        dst[gi] = (S)((double)z + beta * wv);
      } else {
        dst[gi] = (S)z;
      }
    }
  }
}

template <class S, class T, int MODE, int NC = 0>
__global__ __launch_bounds__(256) void k_rows_inv(Geo g, DctPlan dp, const cx<T>* __restrict__ tw,
                                                  const S* __restrict__ src, S* __restrict__ dst, int rpb, int nrows,
                                                  S* __restrict__ xs, const DevState* __restrict__ st, int gate) {
  k_rows_inv_body<S, T, MODE, NC, HwGrid>(HwGrid{}, g, dp, tw, src, dst, rpb, nrows, xs, st, gate);
}

// ========================================================= DCT along columns
// Strided axis a, in place.  A block owns `tb` adjacent b columns of one
// plane: every LDS line is one column (length na).  Element e
// of a block is (row n, column c) = (e / tb, e % tb); columns beyond the
// right edge of the plane are skipped.
template <class S, class T, int DIR, int NC, class BG>
__device__ __forceinline__ void k_cols_body(const BG bg, Geo g, DctPlan dp, const cx<T>* __restrict__ tw, S* __restrict__ data,
                                              int tb, const DevState* __restrict__ st, int gate) {
  using Sh = DctShape<T, NC>;
  // tile (column block bx, global plane) with tiles renumbered per XCD so
  // that tiles sharing 128-byte lines run on one XCD together; instances of a
  // batch hold nL planes each
  const int tile = xcd_tile(bg.bx() + bg.gx() * bg.by(), bg.gx() * bg.gy());
  const int bx = tile % bg.gx(), plane = tile / bg.gx();
  if (st) st += plane / g.nL;
  if (gated_out(st, gate)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int nthr = Sh::ct ? Sh::col_threads : (int)blockDim.x;
  const int N = Sh::ct ? NC : dp.N;  // = na
  const int M = Sh::ct ? Sh::M : dp.M;
  const bool fft = Sh::ct ? true : (dp.fft != 0);
  const int ls = Sh::ct ? Sh::ls : dp.lstride;
  const int tbv = Sh::ct ? Sh::cols : tb;
  const int b0 = bx * tbv;
  const int lines = min(tbv, g.nb - b0);
  S* pl = data + (int64_t)plane * g.plane + b0;
  const int total = tbv * N;
  if (DIR < 0) {
    constexpr int UC = batch_of(Sh::col_elems, 64 / ((int)sizeof(S) / 4), UNR);
    for (int e0 = tid; e0 < total; e0 += nthr * UC) {
      S x[UC];
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int e = e0 + u * nthr;
        const int n = e / tbv, c = e - n * tbv;
        if (e < total && c < lines) x[u] = pl[(int64_t)n * g.nb + c];
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int e = e0 + u * nthr;
        const int n = e / tbv, c = e - n * tbv;
        if (e < total && c < lines) {
          T* L = reinterpret_cast<T*>(buf + c * ls);
          if (fft) L[vpos(dct_perm(n, N))] = (T)x[u];
          else L[n] = (T)x[u];
        }
      }
    }
    __syncthreads();
    if (fft) {
      if constexpr (Sh::ct) lds_fft_ct<T, -1, Sh::M, Sh::cols, Sh::col_threads, Sh::ls>(buf, tw, tid);
      else lds_fft<T, -1>(buf, lines, ls, dp, tw, tid, nthr);
      const int nit = M / 2 + 1;
      for (int e = tid; e < tbv * nit; e += nthr) {
        const int k = e / tbv, c = e - k * tbv;
        if (c < lines)
          dct_post(buf + c * ls, k, N, M, tw, [&](int idx, T v) { pl[(int64_t)idx * g.nb + c] = (S)v; });
      }
    } else {
      const int N4 = 4 * N;
      for (int e = tid; e < total; e += nthr) {
        const int k = e / tbv, c = e - k * tbv;
        if (c >= lines) continue;
        const T* L = reinterpret_cast<const T*>(buf + c * ls);
        T s = T(0);
        for (int n = 0; n < N; ++n) s += L[n] * tw[((2 * n + 1) * k) % N4].re;
        pl[(int64_t)k * g.nb + c] = (S)s;
      }
    }
  } else {
    if (fft) {
      const int nit = M / 2 + 1;
      const int items = tbv * nit;
      constexpr int UI = batch_of(Sh::col_items, 64 / (4 * ((int)sizeof(S) / 4)), 4);
      for (int e0 = tid; e0 < items; e0 += nthr * UI) {
        T xv[UI][4];
#pragma unroll
        for (int u = 0; u < UI; ++u) {
          const int e = e0 + u * nthr;
          const int k = e / tbv, c = e - k * tbv;
          if (e < items && c < lines) {
            int i0, i1, i2, i3;
            pre_inv_idx(k, N, M, i0, i1, i2, i3);
            xv[u][0] = (T)pl[(int64_t)i0 * g.nb + c];
            xv[u][1] = (T)pl[(int64_t)i1 * g.nb + c];
            xv[u][2] = (T)pl[(int64_t)i2 * g.nb + c];
            xv[u][3] = (T)pl[(int64_t)i3 * g.nb + c];
          }
        }
#pragma unroll
        for (int u = 0; u < UI; ++u) {
          const int e = e0 + u * nthr;
          const int k = e / tbv, c = e - k * tbv;
          if (e < items && c < lines)
            dct_pre_inv_vals(buf + c * ls, k, M, tw, xv[u][0], xv[u][1], xv[u][2], xv[u][3]);
        }
      }
      __syncthreads();
      if constexpr (Sh::ct) lds_fft_ct<T, +1, Sh::M, Sh::cols, Sh::col_threads, Sh::ls>(buf, tw, tid);
      else lds_fft<T, +1>(buf, lines, ls, dp, tw, tid, nthr);
      const T invM = T(1) / T(M);
      for (int e = tid; e < total; e += nthr) {
        const int n = e / tbv, c = e - n * tbv;
        if (c >= lines) continue;
        const T* L = reinterpret_cast<const T*>(buf + c * ls);
        pl[(int64_t)n * g.nb + c] = (S)(L[vpos(dct_perm(n, N))] * invM);
      }
    } else {
      for (int e = tid; e < total; e += nthr) {
        const int n = e / tbv, c = e - n * tbv;
        if (c >= lines) continue;
        T* L = reinterpret_cast<T*>(buf + c * ls);
        L[n] = (T)pl[(int64_t)n * g.nb + c];
      }
      __syncthreads();
      const int N4 = 4 * N;
      const T sc = T(2) / T(N);
      for (int e = tid; e < total; e += nthr) {
        const int n = e / tbv, c = e - n * tbv;
        if (c >= lines) continue;
        const T* L = reinterpret_cast<const T*>(buf + c * ls);
        T s = T(0.5) * L[0];
        for (int k = 1; k < N; ++k) s += L[k] * tw[((2 * n + 1) * k) % N4].re;
        pl[(int64_t)n * g.nb + c] = (S)(sc * s);
      }
    }
  }
}

template <class S, class T, int DIR, int NC = 0>
__global__ __launch_bounds__(512) void k_cols(Geo g, DctPlan dp, const cx<T>* __restrict__ tw, S* __restrict__ data,
                                              int tb, const DevState* __restrict__ st, int gate) {
  k_cols_body<S, T, DIR, NC, HwGrid>(HwGrid{}, g, dp, tw, data, tb, st, gate);
}

// Persistent column transforms (compile-time lengths, whole tiles; a batch
// runs them without the per-instance exit test).
// Block x takes tiles x, x + gridDim.x, ... and loads the next tile's inputs
// into registers while the current one is transformed in LDS.  The loads of
// a tile are only useful in flight if nothing after them forces a wait for
// them: one counter tracks vector loads and stores in issue order, so every
// tile issues the same number of global stores (the host runs these kernels
// on whole tiles only; the column clamp below would make a ragged tile's
// extra lanes repeat its last column), the twiddles come from LDS, and the
// forward outputs are grouped four to an item.  LDS:
// the tile, every 8th twiddle (FFT stages) and the twiddles of the DCT
// pre/post steps (float32: the first 2N; float64: the two short tables of
// DctTw, which keep two tiles per CU).
template <class T, int NC> struct ColsPf {
  using Sh = DctShape<T, NC>;
  static constexpr bool full = sizeof(T) == 4;
  static constexpr int tile_slots = Sh::cols * Sh::ls;
  static constexpr int dct_slots = full ? 2 * NC : 2 * (Sh::M + 1);
  static constexpr int bytes = (tile_slots + Sh::M + dct_slots) * 2 * (int)sizeof(T);
};

template <class S, class T, int DIR, int NC>
__global__ __launch_bounds__((DctShape<T, NC>::col_threads), (DctShape<T, NC>::col_threads / 128)) void k_cols_pf(Geo g, const cx<T>* __restrict__ tw, S* __restrict__ data,
                                                    int ntx, int ntiles, const DevState* __restrict__ st, int gate) {
  using Sh = DctShape<T, NC>;
  static_assert(NC > 0, "compile-time lengths only");
  constexpr int N = NC, M = Sh::M, LS = Sh::ls, TBV = Sh::cols, NTHR = Sh::col_threads;
  constexpr int total = TBV * N;            // inputs (outputs) of a tile
  constexpr int items = TBV * (M / 2 + 1);  // pre- (post-) processing items of a tile
  static_assert(total % NTHR == 0 && NTHR % TBV == 0 && M % 2 == 0 && (TBV * (M / 2)) % NTHR == 0, "tile shape");
  constexpr int UE = total / NTHR;
  constexpr int UP = TBV * (M / 2) / NTHR;  // forward items of four outputs per thread
  constexpr int UI = (items + NTHR - 1) / NTHR;
  // forward inputs: 16-byte loads of VW adjacent columns (whole tiles)
  constexpr int VW = 16 / (int)sizeof(S), CQ = TBV / VW, RPR = NTHR / CQ, UV = N / RPR;
  static_assert(TBV % VW == 0 && NTHR % CQ == 0 && N % RPR == 0, "forward load shape");
  // backward inputs of float32 columns of 256 or more: 16-byte loads as well,
  // VW adjacent columns of one item's four rows (items4 pairs of column group
  // and item); 271 against 277 us at 512^3.  Shorter or float64 columns keep
  // one column per lane (the wider loads cost them occupancy or registers).
  constexpr bool BV = DIR > 0 && sizeof(S) == 4 && NC >= 256;
  constexpr int IQ = TBV / VW, items4 = IQ * (M / 2 + 1), UB = (items4 + NTHR - 1) / NTHR;
  constexpr int NV = (DIR < 0 || BV) ? 1 : 4 * UI;
  if (gated_out(st, gate)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* twc = buf + ColsPf<T, NC>::tile_slots;  // twc[j] = tw[8 j], j < M
  cx<T>* tlo = twc + M;                           // tlo[j] = tw[j], j < 2N (float32) or j <= M
  cx<T>* tq = tlo + M + 1;                        // (float64) tq[j] = tw[4 j], j <= M
  int tid = threadIdx.x;
  for (int j = tid; j < M; j += NTHR) twc[j] = tw[8 * j];
  if constexpr (ColsPf<T, NC>::full) {
    for (int j = tid; j < 2 * N; j += NTHR) tlo[j] = tw[j];
  } else {
    for (int j = tid; j <= M; j += NTHR) {
      tlo[j] = tw[j];
      tq[j] = tw[4 * j];
    }
  }
  __syncthreads();
  using TwD = typename std::conditional<ColsPf<T, NC>::full, const cx<T>*, DctTw<T>>::type;
  TwD twd;
  if constexpr (ColsPf<T, NC>::full) twd = tlo;
  else twd = DctTw<T>{tlo, tq, M};
  uint32_t nb = (uint32_t)g.nb;

  // tile -> first element and the last real column (offsets in a plane fit 32 bits)
  auto locate = [&](int tile, S*& pl, int& last) {
    const int bx = tile % ntx, plane = tile / ntx;
    const int b0 = bx * TBV;
    last = min(TBV, g.nb - b0) - 1;
    pl = data + (int64_t)plane * g.plane + b0;
  };
  S x[NV];
  V16<S> xb[BV ? UB : 1][4];
  V16<S> xv[DIR < 0 ? UV : 1];
  auto load = [&](const S* pl, int last, uint32_t nb) {
    const uint32_t c = (uint32_t)min(tid % TBV, last);
    if constexpr (DIR < 0) {
      const uint32_t c4 = VW * (uint32_t)(tid % CQ), r0 = (uint32_t)(tid / CQ);
#pragma unroll
      for (int u = 0; u < UV; ++u) xv[u] = ld16(pl + (r0 + (uint32_t)(u * RPR)) * nb + c4);
    } else if constexpr (BV) {
      (void)c;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int e = tid + u * NTHR;
        if (e < items4) {
          int i0, i1, i2, i3;
          const uint32_t c4 = VW * (uint32_t)(e % IQ);
          pre_inv_idx(e / IQ, N, M, i0, i1, i2, i3);
          xb[u][0] = ld16(pl + (uint32_t)i0 * nb + c4);
          xb[u][1] = ld16(pl + (uint32_t)i1 * nb + c4);
          xb[u][2] = ld16(pl + (uint32_t)i2 * nb + c4);
          xb[u][3] = ld16(pl + (uint32_t)i3 * nb + c4);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < UI; ++u) {
        const int e = tid + u * NTHR;
        if (e < items) {
          int i0, i1, i2, i3;
          pre_inv_idx(e / TBV, N, M, i0, i1, i2, i3);
          x[4 * u + 0] = pl[(uint32_t)i0 * nb + c];
          x[4 * u + 1] = pl[(uint32_t)i1 * nb + c];
          x[4 * u + 2] = pl[(uint32_t)i2 * nb + c];
          x[4 * u + 3] = pl[(uint32_t)i3 * nb + c];
        }
      }
    }
  };

  // inputs in registers -> LDS lines
  auto stage = [&]() {
    if constexpr (DIR < 0) {
      const int c4 = VW * (tid % CQ), r0 = tid / CQ;
#pragma unroll
      for (int u = 0; u < UV; ++u) {
        const int pos = vpos(dct_perm(r0 + u * RPR, N));
#pragma unroll
        for (int j = 0; j < VW; ++j) reinterpret_cast<T*>(buf + (c4 + j) * LS)[pos] = (T)xv[u].v[j];
      }
    } else if constexpr (BV) {
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int e = tid + u * NTHR;
        if (e < items4) {
          const int k = e / IQ, c4 = VW * (e % IQ);
#pragma unroll
          for (int j = 0; j < VW; ++j)
            dct_pre_inv_vals(buf + (c4 + j) * LS, k, M, twd, (T)xb[u][0].v[j], (T)xb[u][1].v[j], (T)xb[u][2].v[j],
                             (T)xb[u][3].v[j]);
        }
      }
    } else {
      const int c = tid % TBV;
#pragma unroll
      for (int u = 0; u < UI; ++u) {
        const int e = tid + u * NTHR;
        if (e < items)
          dct_pre_inv_vals(buf + c * LS, e / TBV, M, twd, (T)x[4 * u], (T)x[4 * u + 1], (T)x[4 * u + 2],
                           (T)x[4 * u + 3]);
      }
    }
  };

  // The first tile is staged before the loop; inside it the next tile's
  // loads are issued before the transform and staged after the stores, so
  // every wait for them leaves the stores of the tile in flight.
  int tile = blockIdx.x;
  S* pl = data;
  int last = 0;
  if (tile < ntiles) {
    locate(tile, pl, last);
    load(pl, last, nb);
    stage();
  }
  __syncthreads();
  for (; tile < ntiles; tile += gridDim.x) {
    // per-thread offsets are recomputed every tile rather than held in
    // registers across the loop
    asm volatile("" : "+v"(tid), "+s"(nb));
    const int c = tid % TBV;
    const cx<T>* Lc = buf + c * LS;
    // the next tile's inputs -> registers, in flight during the transform
    const int tn = tile + gridDim.x;
    S* pln = data;
    int lastn = 0;
    if (tn < ntiles) {
      locate(tn, pln, lastn);
      load(pln, lastn, nb);
    }
    lds_fft_ct<T, DIR, M, TBV, NTHR, LS, 0, 1, 1>(buf, twc, tid);
    const uint32_t cg = (uint32_t)min(c, last);
    if constexpr (DIR < 0) {
      // items of exactly four outputs, stored straight from registers
#pragma unroll
      for (int u = 0; u < UP; ++u) {
        const int k = tid / TBV + u * (NTHR / TBV);
        dct_post4(Lc, k, N, M, twd, [&](int idx, T v) { pl[(uint32_t)idx * nb + cg] = (S)v; });
      }
    } else {
      const T invM = T(1) / T(M);
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const int n = tid / TBV + u * (NTHR / TBV);
        pl[(uint32_t)n * nb + cg] = (S)(reinterpret_cast<const T*>(Lc)[vpos(dct_perm(n, N))] * invM);
      }
    }
    __syncthreads();  // every read of this tile's LDS lines is done
    if (tn < ntiles) stage();
    __syncthreads();
    pl = pln;
    last = lastn;
  }
}

// =================================================================== Thomas

// lambda(k) = 2 (1 - cos(k pi / N)) = 4 sin^2(k pi / (2 N)), the eigenvalues
// of the 1D Neumann matrix (Section "Preconditioner system solver"), for
// 0 <= k < N, with step = pi / (2 N).  The argument lies in [0, pi/2), where
// the Taylor series of sin through x^23 is exact to double rounding (the
// next term is below 1e-19 of the sum); Horner in x^2.  No memory access,
// so the tridiagonal kernel forms a mode's shift without a load.
__device__ __forceinline__ double neumann_lambda(int k, double step) {
  const double x = (double)k * step;
  const double x2 = x * x;
  double sp = 1.0 / 25852016738884976640000.0;          // 1/23!
  sp = fma(sp, -x2, 1.0 / 51090942171709440000.0);      // 1/21!
  sp = fma(sp, -x2, 1.0 / 121645100408832000.0);        // 1/19!
  sp = fma(sp, -x2, 1.0 / 355687428096000.0);           // 1/17!
  sp = fma(sp, -x2, 1.0 / 1307674368000.0);             // 1/15!
  sp = fma(sp, -x2, 1.0 / 6227020800.0);                // 1/13!
  sp = fma(sp, -x2, 1.0 / 39916800.0);                  // 1/11!
  sp = fma(sp, -x2, 1.0 / 362880.0);                    // 1/9!
  sp = fma(sp, -x2, 1.0 / 5040.0);                      // 1/7!
  sp = fma(sp, -x2, 1.0 / 120.0);                       // 1/5!
  sp = fma(sp, -x2, 1.0 / 6.0);                         // 1/3!
  sp = fma(sp, -x2, 1.0);
  const double sn = x * sp;
  return 4.0 * sn * sn;
}

// Solve T_{a',b'} z = t along k for every transverse mode (a', b'), in place,
// with double arithmetic.  T = s I + kL tridiag(-1, 2, -1), first and last
// diagonal entries s + kL + 2 kin and s + kL + 2 kout, s = lam_a ka + lam_b kb.
//
// Partitioned elimination keeps every value in registers: the block holds TB
// adjacent modes (lines, coalesced) times P partitions of each line.  A
// partition is `len` interior rows followed by one separator row (none for
// the last partition).  Phase 1: each thread loads its rows and runs the LU
// sweep of its interior block M = L D L^T (pivots kept).  The same sweep
// gives both ends of y = M^{-1} t and the corner entries of M^{-1}: with
// g = L^{-1} e_1 (a running product of the multipliers), y_1 = sum_j g_j d_j,
// (M^{-1})_{11} = sum_j g_j^2 / u_j, (M^{-1})_{1,len} = g_len / u_len.  The
// separators then form a symmetric tridiagonal Schur complement, solved by
// parallel cyclic reduction with one thread per separator.  Phase 2: each
// thread moves its two separator couplings to the right-hand side and
// re-solves its block with the stored pivots.
//
// Also returns the partial of r . z per tile: by the DCT's Parseval relation
// it equals (4 / (na nb)) sum alpha_a' alpha_b' t . z over modes, t the
// transformed r; per partition, t . z = t^T M^{-1} t + (coupling) * (ends of
// M^{-1} t).
//
// The mode's shift s comes from eigenvalues computed in registers
// (neumann_lambda), not from a table in memory.
//
// Blocks are persistent: block x of instance z handles tiles x, x + gridDim.x,
// ... (a tile is TB modes b' of one mode a'; consecutive blocks take adjacent
// tiles, so the rows in flight at one time cover long runs of each plane).
// PF: the block loads the next tile's rows into registers before it works on
// the current one, so HBM traffic overlaps the elimination (float32 rows;
// float64 rows would cost the registers of a second block per CU, which hides
// latency better).  Loads and stores share one in-order counter per wave, so
// the prefetched rows are taken (waited for) before the current tile's
// stores are issued, and the shift needs no load: a wait placed after the
// stores would also wait for them to drain.  EXACT: nL = P * MAXM (every
// partition has MAXM rows), which removes the ragged-length guards.
template <class S, int TB, int P, int MAXM, bool EXACT, bool PF, class BG>
__device__ __forceinline__ void k_thomas_body(const BG bg, Geo g, RefMedium rm, S* __restrict__ t, int Puse,
                                                  double* __restrict__ partials, const DevState* __restrict__ st,
                                                  int gate, int ntx, int ntiles, double (&sh)[6][P][TB + 1],
                                                  double* red) {
  static_assert(64 % P == 0, "the P threads of a line must sit in one wave");
  // instance bg.bz() of a batch
  if (st) st += bg.bz();
  if (gated_out(st, gate)) return;
  t += (int64_t)bg.bz() * g.V;
  if (partials) partials += (int64_t)bg.bz() * ntiles;
  const double* kr = rm.kref + 5 * bg.bz();
  const int tid = threadIdx.x;
  const int l = tid % TB, p = tid / TB;
  const int nL = g.nL;
  const int m = EXACT ? MAXM : (nL + Puse - 1) / Puse;
  const int Peff = EXACT ? P : (nL + m - 1) / m;
  const int start = p * m;
  const bool pok = p < Peff;
  const bool right = pok && (p < Peff - 1);  // partition ends in a separator row
  const int endp = min(start + m, nL);
  const int lenp = pok ? (endp - start - (right ? 1 : 0)) : 0;
  const double kL = kr[0], ka = kr[1], kb = kr[2];
  const double aoff = -kL;
  const double a2 = kL * kL;
  const double Dint0 = 2.0 * kL;
  // extra diagonal of the first row of the line (k = 0) and of the last (k = nL - 1)
  const double dfirst = (start == 0) ? (kr[3] * 2.0 - kL) : 0.0;
  const double dlast = (pok && !right) ? (kr[4] * 2.0 - kL) : 0.0;
  const int64_t plane = g.plane;
  const int nsep = Peff - 1;
  // pivots' reciprocals: float32 rows take one Newton step, float64 rows two
  auto rcp = [](double u) {
    if constexpr (sizeof(S) == 4) return frcp1(u);
    else return frcp(u);
  };

  auto row_ok = [&](int j) { return EXACT ? (j < MAXM - 1 || !right) : (j < lenp); };
  auto load = [&](int tile, S* v, S& vs) {
    const int bm = (tile % ntx) * TB + l, am = tile / ntx;
    if (pok && bm < g.nb) {
      const S* src = t + (int64_t)start * plane + (int64_t)am * g.nb + bm;
#pragma unroll
      for (int j = 0; j < MAXM; ++j)
        if (row_ok(j)) v[j] = src[(int64_t)j * plane];
      if (right) vs = src[(int64_t)(endp - 1 - start) * plane];
    }
  };

  // PF: the next tile's rows are prefetched into registers (when they fit)
  // tiles of one round are renumbered so that each XCD holds a contiguous
  // range (adjacent tiles share 128-byte lines when TB * sizeof(S) < 128)
  S cur[MAXM], cur_s = S(0);
  int tile = bg.bx();
  if (PF && tile < ntiles) {
    load(tile, cur, cur_s);
    // wait for the first tile here, outside the loop, so that the loop head
    // never waits (a wait there would also cover the previous tile's stores)
#pragma unroll
    for (int j = 0; j < MAXM; ++j) asm volatile("" ::"v"(cur[j]));
    asm volatile("" ::"v"(cur_s));
  }
  for (; tile < ntiles; tile += bg.gx()) {
    const int bm = (tile % ntx) * TB + l, am = tile / ntx;
    const bool line_ok = bm < g.nb;
    const bool active = line_ok && pok;
    const bool has_right = active && right;
    const int len = active ? lenp : 0;
    // the mode's shift from the eigenvalues computed in registers: a load here
    // would wait behind the previous tile's stores in the in-order counter
    const double sft = line_ok ? (neumann_lambda(am, rm.step_a) * ka + neumann_lambda(bm, rm.step_b) * kb) : 0.0;
    const double Dint = sft + Dint0;
    S nxt[PF ? MAXM : 1], nxt_s = S(0);
    if constexpr (PF) {
      // this tile's rows arrived before the loop head (first tile) or were
      // taken before the previous tile's stores; the shift is in registers
      asm volatile("" ::"v"(Dint));
      const int tn = tile + bg.gx();
      if (tn < ntiles) load(tn, nxt, nxt_s);
    } else {
      load(tile, cur, cur_s);
    }
    // register arrays are only ever indexed by unrolled constants
    double dv[MAXM], invu[MAXM];
    double quad = 0.0, ts = 0.0, y_last = 0.0, y_first = 0.0, m11 = 0.0, gj = 1.0;
    if (active) {
      ts = (double)cur_s;
      // LU sweep of the partition block M = L D L^T: pivots u_j (kept as
      // 1/u_j), d_j = (L D)^{-1} t, t^T M^{-1} t = sum d_j f_j (f = L^{-1} t)
      double dprev = 0.0, iu = 0.0;
#pragma unroll
      for (int j = 0; j < MAXM; ++j) {
        if (EXACT || j < len) {
          if (!EXACT || j < MAXM - 1 || !has_right) {
            double u = Dint;
            double f = (double)cur[j];
            if (j == 0) {
              u += dfirst;
            } else {
              u -= a2 * iu;
              f -= aoff * dprev;
              gj *= -(aoff * iu);
            }
            if (j == (EXACT ? MAXM - 1 : len - 1)) u += dlast;
            iu = rcp(u);
            invu[j] = iu;
            dprev = f * iu;
            quad += dprev * f;
            y_first += gj * dprev;
            m11 += gj * gj * iu;
          }
        }
      }
      y_last = dprev;
      // what the separators need of this partition (stored as they are:
      // storing the separator's partial sums instead made the compiler
      // spill hundreds of registers in the guarded float64 variants)
      sh[0][p][l] = y_first;
      sh[1][p][l] = y_last;
      sh[2][p][l] = m11;
      sh[3][p][l] = iu;       // (M^{-1})_{len,len}
      sh[4][p][l] = gj * iu;  // (M^{-1})_{1,len}
      sh[5][p][l] = ts;
    }
    __syncthreads();
    // Separator q (the last row of partition q) couples to q - 1 and q + 1:
    // L_q x_{q-1} + B_q x_q + U_q x_{q+1} = r_q.  Parallel cyclic reduction:
    // at stride h every row eliminates its neighbours q - h and q + h, so
    // after ceil(log2 nsep) steps each row stands alone.  Threads take the
    // separators line by line (thread = line * P + separator): a line's
    // separators sit in P adjacent lanes of one wave, which exchange rows
    // through shared memory with wave-level ordering only, no block barrier.
    if constexpr (MAXM <= 16 || EXACT) {
      const int q = tid % P, ls = tid / P;
      const int bs = (tile % ntx) * TB + ls;  // the separator's mode b'
      const bool sep = bs < g.nb && q < nsep;
      double Lq = 0.0, Bq = 1.0, Uq = 0.0, rq = 0.0;
      if (sep) {
        // the separator is an interior row (never k = 0 or nL - 1); its
        // line's diagonal is formed again (the thread worked another line)
        const double Ds = Dint0 + neumann_lambda(am, rm.step_a) * ka + neumann_lambda(bs, rm.step_b) * kb;
        Lq = (q > 0) ? -a2 * sh[4][q][ls] : 0.0;
        Bq = Ds - a2 * (sh[3][q][ls] + sh[2][q + 1][ls]);
        Uq = (q + 1 < nsep) ? -a2 * sh[4][q + 1][ls] : 0.0;
        rq = sh[5][q][ls] - aoff * sh[1][q][ls] - aoff * sh[0][q + 1][ls];
      }
      for (int h = 1; h < nsep; h <<= 1) {
        wave_sync();  // every lane has read the slots the writes below replace
        // each row publishes its L, U, r scaled by its 1/B
        const double iB = rcp(Bq);
        if (sep) {
          sh[0][q][ls] = Lq * iB;
          sh[1][q][ls] = Uq * iB;
          sh[2][q][ls] = rq * iB;
        }
        wave_sync();
        if (sep) {
          double nL_ = 0.0, nU = 0.0, nB = Bq, nr = rq;
          if (q - h >= 0) {
            nL_ = -Lq * sh[0][q - h][ls];
            nB -= Lq * sh[1][q - h][ls];
            nr -= Lq * sh[2][q - h][ls];
          }
          if (q + h < nsep) {
            nU = -Uq * sh[1][q + h][ls];
            nB -= Uq * sh[0][q + h][ls];
            nr -= Uq * sh[2][q + h][ls];
          }
          Lq = nL_;
          Uq = nU;
          Bq = nB;
          rq = nr;
        }
      }
      // separator value x_q (slot 5 of partition q was read only by this thread)
      if (sep) sh[5][q][ls] = rq / Bq;
    } else {
      // guarded partitions longer than 16 rows (load axes beyond 512):
      // separator q is taken by the thread of partition q, rows exchanged
      // through shared memory with block barriers
      const int q = p;
      const bool sep = line_ok && q < nsep;
      double Lq = 0.0, Bq = 1.0, Uq = 0.0, rq = 0.0;
      if (sep) {
        Lq = (q > 0) ? -a2 * sh[4][q][l] : 0.0;
        Bq = Dint - a2 * (sh[3][q][l] + sh[2][q + 1][l]);
        Uq = (q + 1 < nsep) ? -a2 * sh[4][q + 1][l] : 0.0;
        rq = sh[5][q][l] - aoff * sh[1][q][l] - aoff * sh[0][q + 1][l];
      }
      for (int h = 1; h < nsep; h <<= 1) {
        __syncthreads();  // every read of the previous contents is done
        const double iB = rcp(Bq);
        if (sep) {
          sh[0][q][l] = Lq;
          sh[1][q][l] = Uq;
          sh[2][q][l] = rq;
          sh[3][q][l] = iB;
        }
        __syncthreads();
        if (sep) {
          double nL_ = 0.0, nU = 0.0, nB = Bq, nr = rq;
          if (q - h >= 0) {
            const double al = -Lq * sh[3][q - h][l];
            nL_ = al * sh[0][q - h][l];
            nB += al * sh[1][q - h][l];
            nr += al * sh[2][q - h][l];
          }
          if (q + h < nsep) {
            const double ga = -Uq * sh[3][q + h][l];
            nU = ga * sh[1][q + h][l];
            nB += ga * sh[0][q + h][l];
            nr += ga * sh[2][q + h][l];
          }
          Lq = nL_;
          Uq = nU;
          Bq = nB;
          rq = nr;
        }
      }
      __syncthreads();
      if (sep) sh[5][q][l] = rq / Bq;
    }
    __syncthreads();
    double acc = 0.0, zr = 0.0;
    if (active) {
      const double zl = (p > 0) ? sh[5][p - 1][l] : 0.0;
      zr = has_right ? sh[5][p][l] : 0.0;
      const double c1 = -aoff * zl, cm = -aoff * zr;
      // z = M^{-1} (t + c1 e_1 + cm e_len): forward elimination with the
      // couplings at both ends, then back substitution, both with the stored
      // pivots
      const int lastj = EXACT ? (has_right ? MAXM - 2 : MAXM - 1) : len - 1;
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < MAXM; ++j) {
        if ((EXACT && (j < MAXM - 1 || !has_right)) || (!EXACT && j < len)) {
          double f = (double)cur[j];
          f += (j == 0) ? c1 : -aoff * d;
          if (j == lastj) f += cm;
          d = f * invu[j];
          if constexpr (sizeof(S) == 8) cur[j] = d;  // float64 rows: in place
          else dv[j] = d;
        }
      }
      double z = 0.0;
#pragma unroll
      for (int j = MAXM - 1; j >= 0; --j) {
        if ((EXACT && (j < MAXM - 1 || !has_right)) || (!EXACT && j < len)) {
          if constexpr (sizeof(S) == 8) {
            z = (j == lastj) ? (double)cur[j] : ((double)cur[j] - aoff * invu[j] * z);
            cur[j] = z;
          } else {
            z = (j == lastj) ? dv[j] : (dv[j] - aoff * invu[j] * z);
            cur[j] = (S)z;  // this tile's rows are dead after the forward pass
          }
        }
      }
      const double wa = (am == 0) ? 0.5 : 1.0, wb = (bm == 0) ? 0.5 : 1.0;
      acc = wa * wb * (quad + c1 * y_first + cm * y_last + (has_right ? ts * zr : 0.0));
    }
    if constexpr (PF) {
      // Loads and stores share one in-order counter per wave: take the
      // prefetched tile now, on every path, so that no later wait for it
      // also waits for this tile's stores.
#pragma unroll
      for (int j = 0; j < MAXM; ++j) asm volatile("" ::"v"(nxt[j]) : "memory");
      asm volatile("" ::"v"(nxt_s) : "memory");
    }
    if (active) {
      S* dst = t + (int64_t)start * plane + (int64_t)am * g.nb + bm;
#pragma unroll
      for (int j = 0; j < MAXM; ++j)
        if ((EXACT && (j < MAXM - 1 || !has_right)) || (!EXACT && j < len))
          dst[(int64_t)j * plane] = cur[j];
      if (has_right) dst[(int64_t)(endp - 1 - start) * plane] = (S)zr;
    }
    if (partials) {
      const double sum = block_sum(acc, red);
      if (tid == 0) partials[tile] = sum * rm.dot_scale;
    }
    __syncthreads();  // the next tile rewrites sh
    if constexpr (PF) {
#pragma unroll
      for (int j = 0; j < MAXM; ++j) cur[j] = nxt[j];
      cur_s = nxt_s;
    }
  }
}

// Partitions of more than 16 rows take up to 256 registers per thread (one
// 512-thread block per CU): their rows stay in registers without spills.
template <class S, int TB, int P, int MAXM, bool EXACT, bool PF = ((EXACT && sizeof(S) == 4) || MAXM <= 8),
          int MINW = (MAXM > 16 ? 2 : 4)>
__global__ __launch_bounds__(TB* P, MINW) void k_thomas(Geo g, RefMedium rm, S* __restrict__ t, int Puse,
                                                  double* __restrict__ partials, const DevState* __restrict__ st,
                                                  int gate, int ntx, int ntiles) {
  // per (partition, mode): y_1, y_len, (M^-1)_11, (M^-1)_len,len,
  // (M^-1)_1,len, t of the separator row, then the separator value; padded
  // against bank conflicts when the separator threads read a line's partitions
  __shared__ double sh[6][P][TB + 1];
  __shared__ double red[16];
  k_thomas_body<S, TB, P, MAXM, EXACT, PF, HwGrid>(HwGrid{}, g, rm, t, Puse, partials, st, gate, ntx, ntiles, sh, red);
}

// Compiled variants of the tridiagonal kernel: TB modes times P partitions
// per block and the rows of a partition (an upper bound, or the exact count
// when every partition has it, nL = P * rows).  Fewer partitions mean fewer
// reduction steps and less repeated pivot work; smaller blocks let several
// run on one CU, so the barriers of one overlap the arithmetic of another.
// Measured on batches of cubes (float32 rows, microseconds per solve of the
// whole batch): 64^3 x 16: 47 (32 x 32) -> 18 (32 x 8); 96^3 x 12: 139 ->
// 32 (32 x 8); 128^3 x 8: 96 -> 36 (32 x 8); 160^3 x 6: 208 -> 70 (16 x 16);
// 256^3 x 2: 113 -> 70 (32 x 16); 512^3: 32 x 32 stays the fastest of these.  Float64
// rows: 32 x 8 up to 128, 16 x 16 at 160, 32 x 16 at 256, 16 x 32 beyond.
// At 512 rows, 32 x 16 with exact partitions of 32 rows (512 threads, up to
// 256 registers, one block per CU) beats 32 partitions of 16: 281 against
// 315 us (float32 rows) and 451 against 567 us (float64).  Likewise 32 x 8
// with exact partitions of 20 rows at 160 and of 32 at 256 (256 threads,
// up to 256 registers): 160^3 x 6: 70 -> 52 us (float32), 93 -> 85
// (float64); 256^3 x 2: 71 -> 64 us (float32), 109 -> 103 (float64).
struct ThomasVariant {
  int tb, p, rows;
  bool exact;
  constexpr int threads() const { return tb * p; }
};
template <class S> struct ThomasVariants;
// Float32 guarded partitions stop at 16 rows (load axes up to 512): the
// 32 x 32 variant of up to 32 rows (1024 threads, 193 spilled registers)
// faulted on its first run and is not compiled.  Exact partitions of 20 and
// 32 rows (at most 512 threads) are.
template <> struct ThomasVariants<float> {
  static constexpr ThomasVariant v[] = {
      {32, 32, 16, true}, {32, 32, 8, true},   {32, 32, 5, true},   {32, 32, 4, true},  {32, 32, 3, true},
      {32, 32, 2, true},  {32, 32, 4, false},  {32, 32, 8, false},  {32, 32, 16, false},
      {32, 8, 16, true},  {32, 8, 12, true},   {32, 8, 8, true},    {32, 8, 6, true},   {32, 8, 4, false},
      {32, 8, 8, false},  {32, 8, 16, false},
      {16, 16, 16, true}, {16, 16, 10, true},  {16, 16, 4, false},  {16, 16, 8, false}, {16, 16, 16, false},
      {64, 8, 16, true},  {64, 8, 12, true},   {64, 8, 8, true},    {64, 8, 6, true},   {64, 8, 4, false},
      {64, 8, 8, false},  {64, 8, 16, false},
      {32, 16, 16, true}, {32, 16, 10, true},  {32, 16, 4, false},  {32, 16, 8, false}, {32, 16, 16, false},
      {32, 16, 32, true}, {32, 8, 20, true},   {32, 8, 32, true}};
  static constexpr int n = sizeof(v) / sizeof(v[0]);
};
template <> struct ThomasVariants<double> {
  static constexpr ThomasVariant v[] = {
      {16, 32, 16, true}, {16, 32, 8, true},   {16, 32, 5, true},   {16, 32, 4, true},  {16, 32, 3, true},
      {16, 32, 2, true},  {16, 32, 4, false},  {16, 32, 8, false},  {16, 32, 16, false}, {16, 32, 32, false},
      {16, 32, 64, false},
      {32, 8, 16, true},  {32, 8, 12, true},   {32, 8, 8, true},    {32, 8, 6, true},   {32, 8, 4, false},
      {32, 8, 8, false},  {32, 8, 16, false},
      {16, 16, 16, true}, {16, 16, 10, true},  {16, 16, 4, false},  {16, 16, 8, false}, {16, 16, 16, false},
      {32, 16, 16, true}, {32, 16, 10, true},  {32, 16, 4, false},  {32, 16, 8, false}, {32, 16, 16, false},
      {32, 16, 32, true}, {32, 8, 20, true},   {32, 8, 32, true}};
  static constexpr int n = sizeof(v) / sizeof(v[0]);
};

// f(std::integral_constant<int, i>) for the variant index i == idx (none when
// idx is out of range); the caller reads ThomasVariants<S>::v[i] as constants.
template <class S, int I = 0, class F>
__host__ __device__ __forceinline__ void with_thomas_variant(int idx, F&& f) {
  if constexpr (I < ThomasVariants<S>::n) {
    if (idx == I) f(std::integral_constant<int, I>{});
    else with_thomas_variant<S, I + 1>(idx, static_cast<F&&>(f));
  }
}


// ================================================================ finalize
enum FinOp { FIN_BNORM = 0, FIN_RHO0, FIN_ALPHA, FIN_RR, FIN_REFINE, FIN_BETA, FIN_RR0, FIN_ACC0, FIN_ACC1, FIN_ACC2, FIN_ACC3 };

// One block of 1024 threads sums n partials in a fixed order and applies the
// scalar step of the iteration to the device state.
// Block s handles instance s of a batch: partials + s * pstride, state s,
// history row s (hstride entries).
template <class BG>
__device__ __forceinline__ void k_fin_body(const BG bg, int op, const double* __restrict__ partials, int n, int64_t pstride,
                                              DevState* st, double* __restrict__ hist, int hstride) {
  __shared__ double red[16];
  partials += (int64_t)bg.bx() * pstride;
  st += bg.bx();
  hist += (int64_t)bg.bx() * hstride;
  if (op == FIN_REFINE) {
    if (st->done || !st->refine) return;
  } else if (op == FIN_ALPHA || op == FIN_RR || op == FIN_BETA || op == FIN_RHO0) {
    if (st->done) return;
  }
  double v = 0.0;
  // eight loads in flight before the first add, the adds in the order of a
  // plain strided loop (the same sum bit for bit)
  const int step = blockDim.x;
  int i = threadIdx.x;
  for (; i + 7 * step < n; i += 8 * step) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = partials[i + u * step];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += x[u];
  }
  for (; i < n; i += step) v += partials[i];
  const double s = block_sum(v, red);
  if (threadIdx.x != 0) return;
  switch (op) {
    case FIN_BNORM: {
      st->bnorm2 = s;
      st->rr = s;
      st->relres = 1.0;
      hist[0] = 1.0;
      if (!(s > 0.0) || !isfinite(s)) {
        st->done = 1;
        st->status = ST_BREAKDOWN;
      } else if (st->rtol >= 1.0) {
        st->done = 1;
      }
      break;
    }
    case FIN_RHO0: {
      st->rho = s;
      if (!(s > 0.0) || !isfinite(s)) {
        st->done = 1;
        st->status = ST_BREAKDOWN;
      } else if (st->max_iter <= 0) {
        st->done = 1;
        st->status = ST_NOT_CONVERGED;
      }
      break;
    }
    case FIN_RR0: {
      // residual of a warm start p0
      st->rr = s;
      const double rel = sqrt(s / st->bnorm2);
      st->relres = rel;
      hist[0] = rel;
      if (rel <= st->rtol) st->done = 1;
      break;
    }
    case FIN_ALPHA: {
      st->wq = s;
      if (!(s > 0.0) || !isfinite(s)) {
        st->done = 1;
        st->status = ST_BREAKDOWN;
      } else {
        st->alpha = st->rho / s;
      }
      break;
    }
    case FIN_RR: {
      st->rr = s;
      const int it = st->iter + 1;
      st->iter = it;
      const double rel = sqrt(s / st->bnorm2);
      st->relres = rel;
      hist[it] = rel;
      if (!isfinite(rel)) {
        st->done = 1;
        st->status = ST_BREAKDOWN;
        break;
      }
      const bool conv = rel <= st->rtol;
      if (!st->mixed) {
        // the solution update of this pass happens in the backward row
        // transform, which no longer runs: leave it to the fix-up kernel
        if (conv) {
          st->done = 1;
          st->status = ST_OK;
          st->pending = 1;
        } else if (it >= st->max_iter) {
          st->done = 1;
          st->status = ST_NOT_CONVERGED;
          st->pending = 1;
        }
      } else {
        st->refine = (conv || it >= st->max_iter || (st->refine_every > 0 && it % st->refine_every == 0)) ? 1 : 0;
      }
      break;
    }
    case FIN_REFINE: {
      st->rr_true = s;
      const double rel = sqrt(s / st->bnorm2);
      st->relres = rel;
      hist[st->iter] = rel;
      if (rel <= st->rtol) {
        st->done = 1;
        st->status = ST_OK;
      } else if (st->iter >= st->max_iter || !isfinite(rel)) {
        st->done = 1;
        st->status = isfinite(rel) ? ST_NOT_CONVERGED : ST_BREAKDOWN;
      }
      break;
    }
    case FIN_BETA: {
      if (!(s > 0.0) || !isfinite(s)) {
        st->done = 1;
        st->status = ST_BREAKDOWN;
      } else {
        st->beta = s / st->rho;
        st->rho = s;
      }
      break;
    }
    default: st->k_acc[op - FIN_ACC0] = s; break;
  }
}

__global__ __launch_bounds__(1024) void k_fin(int op, const double* __restrict__ partials, int n, int64_t pstride,
                                              DevState* st, double* __restrict__ hist, int hstride) {
  k_fin_body<HwGrid>(HwGrid{}, op, partials, n, pstride, st, hist, hstride);
}

// ===================================================================== K_eff
// Flux sums over the two Dirichlet layers: comp 0 = sum 2 kappa (p_last -
// p_out), comp 1 = sum 2 kappa (p_in - p_first).  Partials [2][nblk].
template <class S>
__global__ __launch_bounds__(256) void k_keff(Geo g, const double* __restrict__ p, Kap<S> kp, Rhs rh,
                                              double* __restrict__ partials) {
  __shared__ double red[16];
  // instance blockIdx.y: partials [instance][2][gridDim.x]
  p += (int64_t)blockIdx.y * g.V;
  kp.shift((int64_t)blockIdx.y * g.V);
  partials += (int64_t)blockIdx.y * 2 * gridDim.x;
  double ao = 0.0, ai = 0.0;
  const int64_t last = (int64_t)(g.nL - 1) * g.plane;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.plane; i += (int64_t)gridDim.x * blockDim.x) {
    const double po = rh.pout ? rh.pout[i] : g.p_out, pi = rh.pin ? rh.pin[i] : g.p_in;
    ao += 2.0 * kp.dL(last + i) * (p[last + i] - po);
    ai += 2.0 * kp.dL(i) * (pi - p[i]);
  }
  const double so = block_sum(ao, red);
  const double si = block_sum(ai, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = so;
    partials[gridDim.x + blockIdx.x] = si;
  }
}

// Dissipation sum over every face (internal faces counted once from their
// upper cell, plus the Dirichlet faces), double arithmetic.
template <class S>
__global__ __launch_bounds__(256) void k_energy(Geo g, const double* __restrict__ p, Kap<S> kp, Rhs rh,
                                                double* __restrict__ partials) {
  __shared__ double red[16];
  p += (int64_t)blockIdx.y * g.V;
  kp.shift((int64_t)blockIdx.y * g.V);
  partials += (int64_t)blockIdx.y * gridDim.x;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride) {
    const int64_t k = i / g.plane, rem = i - k * g.plane;
    const int64_t a = rem / g.nb, b = rem - a * g.nb;
    const double kc = kp.dL(i), pc = p[i];
    if (k > 0) {
      const double d = pc - p[i - g.plane];
      acc += g.fL * harm(kc, kp.dL(i - g.plane)) * d * d;
    } else {
      const double d = pc - (rh.pin ? rh.pin[rem] : g.p_in);
      acc += 2.0 * g.fL * kc * d * d;
    }
    if (k == g.nL - 1) {
      const double d = pc - (rh.pout ? rh.pout[rem] : g.p_out);
      acc += 2.0 * g.fL * kc * d * d;
    }
    if (a > 0) {
      const double d = pc - p[i - g.nb];
      acc += g.fa * harm(kp.dA(i), kp.dA(i - g.nb)) * d * d;
    }
    if (b > 0) {
      const double d = pc - p[i - 1];
      acc += g.fb * harm(kp.dB(i), kp.dB(i - 1)) * d * d;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Gradient of K_out with respect to every voxel conductivity (adjoint form).
// K_out = c sum_last 2 kappa (p - p_out), c = nL / (na nb (p_in - p_out)).
// With A lambda = dK/dp (= 2 c kappa on the last layer), lambda = (c / fL) phi
// where phi solves the primal system with Dirichlet pair (0, 1).  Then
//   dK/dkappa_v = [v last] 2 c (p_v - p_out)
//               - sum_{faces F of v} dkappa_F/dkappa_v (p_v - p_n)(lambda_v - lambda_n)
//               - [v first] 2 fL (p_v - p_in) lambda_v - [v last] 2 fL (p_v - p_out) lambda_v,
// dkappa_F/dkappa_v = f_d 2 kappa_n^2 / (kappa_v + kappa_n)^2 for a
// harmonic-mean face.  Reads the canonical layout, writes `out` (type O) in
// the user layout of load axis `axis`; double arithmetic.
template <class S, class O>
__global__ __launch_bounds__(256) void k_grad(Geo g, const double* __restrict__ p, const double* __restrict__ phi,
                                              Kap<S> kp, double c, int axis, O* __restrict__ out) {
  {
    const int64_t off = (int64_t)blockIdx.y * g.V;
    p += off;
    phi += off;
    kp.shift(off);
    out += off;
  }
  const double lsc = c / g.fL;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride) {
    const int64_t k = i / g.plane, rem = i - k * g.plane;
    const int64_t a = rem / g.nb, b = rem - a * g.nb;
    const double kv = kp.dL(i), pv = p[i], lv = lsc * phi[i];
    double gv = 0.0;
    auto face = [&](int64_t n, double f) {
      const double kn = kp.dL(n);
      const double sden = kv + kn;
      gv -= f * 2.0 * kn * kn / (sden * sden) * (pv - p[n]) * (lv - lsc * phi[n]);
    };
    if (k > 0) face(i - g.plane, g.fL);
    if (k + 1 < g.nL) face(i + g.plane, g.fL);
    if (a > 0) face(i - g.nb, g.fa);
    if (a + 1 < g.na) face(i + g.nb, g.fa);
    if (b > 0) face(i - 1, g.fb);
    if (b + 1 < g.nb) face(i + 1, g.fb);
    if (k == 0) gv -= 2.0 * g.fL * (pv - g.p_in) * lv;
    if (k == g.nL - 1) gv += 2.0 * c * (pv - g.p_out) - 2.0 * g.fL * (pv - g.p_out) * lv;
    const int64_t ui = axis == 0 ? i : (axis == 1 ? (a * g.nL + k) * g.nb + b : (a * g.nb + b) * g.nL + k);
    out[ui] = (O)gv;
  }
}

// Unpreconditioned form (z = r), used to compare with plain CG:
// p += alpha w, r -= alpha q, partial ||r||^2.
template <class S>
__global__ __launch_bounds__(256) void k_update_plain(Geo g, S* __restrict__ p, const S* __restrict__ w,
                                                      S* __restrict__ r, const S* __restrict__ q,
                                                      double* __restrict__ partials, const DevState* __restrict__ st) {
  st += blockIdx.y;
  if (st->done) return;
  {
    const int64_t off = (int64_t)blockIdx.y * g.V;
    p += off;
    w += off;
    r += off;
    q += off;
    partials += (int64_t)blockIdx.y * gridDim.x;
  }
  __shared__ double red[16];
  const double alpha = st->alpha;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride) {
    p[i] = (S)((double)p[i] + alpha * (double)w[i]);
    const S rs = (S)((double)r[i] - alpha * (double)q[i]);
    r[i] = rs;
    acc += (double)rs * (double)rs;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// partial x . x
template <class S>
__global__ __launch_bounds__(256) void k_norm2(Geo g, const S* __restrict__ x, double* __restrict__ partials,
                                               const DevState* __restrict__ st) {
  if (st) st += blockIdx.y;
  if (st && st->done) return;
  x += (int64_t)blockIdx.y * g.V;
  partials += (int64_t)blockIdx.y * gridDim.x;
  __shared__ double red[16];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride)
    acc += (double)x[i] * (double)x[i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// w = r + beta w (init: w = r)
template <class S>
__global__ __launch_bounds__(256) void k_dir_plain(Geo g, const S* __restrict__ r, S* __restrict__ w,
                                                   const DevState* __restrict__ st, int init) {
  st += blockIdx.y;
  if (st->done) return;
  r += (int64_t)blockIdx.y * g.V;
  w += (int64_t)blockIdx.y * g.V;
  const double beta = st->beta;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride)
    w[i] = init ? r[i] : (S)((double)r[i] + beta * (double)w[i]);
}

// Mixed form, at a refinement: p += increment, increment = 0 (float64 p).
template <class BG>
__device__ __forceinline__ void k_flush_body(const BG bg, Geo g, double* __restrict__ p, float* __restrict__ dlt,
                                               const float* __restrict__ w, const DevState* __restrict__ st) {
  st += bg.by();
  if (st->done || !st->refine) return;
  p += (int64_t)bg.by() * g.V;
  dlt += (int64_t)bg.by() * g.V;
  if (w) w += (int64_t)bg.by() * g.V;
  // w given: this pass's alpha w is folded in here too (the backward row
  // transform then skips it)
  const double alpha = w ? st->alpha : 0.0;
  const int64_t stride = (int64_t)bg.gx() * blockDim.x;
  for (int64_t i = (int64_t)bg.bx() * blockDim.x + threadIdx.x; i < g.V; i += stride) {
    double v = p[i] + (double)dlt[i];
    if (w) v += alpha * (double)w[i];
    p[i] = v;
    dlt[i] = 0.0f;
  }
}

__global__ __launch_bounds__(256) void k_flush(Geo g, double* __restrict__ p, float* __restrict__ dlt,
                                               const float* __restrict__ w, const DevState* __restrict__ st) {
  k_flush_body<HwGrid>(HwGrid{}, g, p, dlt, w, st);
}

// x += alpha w for the instances whose last pass ended before its backward
// row transform (the float64 form stops right after the residual test).
template <class S>
__global__ __launch_bounds__(256) void k_fixup(Geo g, S* __restrict__ x, const S* __restrict__ w,
                                               const DevState* __restrict__ st) {
  st += blockIdx.y;
  if (!st->pending) return;
  x += (int64_t)blockIdx.y * g.V;
  w += (int64_t)blockIdx.y * g.V;
  const double alpha = st->alpha;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += stride)
    x[i] = (S)((double)x[i] + alpha * (double)w[i]);
}

// Plain copy (bandwidth calibration of the hardware byte counters).
// 16-byte accesses, four per thread in flight; src and dst 16-byte aligned.
__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  constexpr int U = 4;
  const int64_t nv = n / 2;
  const V16<double>* s2 = reinterpret_cast<const V16<double>*>(src);
  V16<double>* d2 = reinterpret_cast<V16<double>*>(dst);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * U;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x * U + threadIdx.x; i0 < nv; i0 += stride) {
    V16<double> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * blockDim.x < nv) v[u] = s2[i0 + u * blockDim.x];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * blockDim.x < nv) d2[i0 + u * blockDim.x] = v[u];
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) dst[n - 1] = src[n - 1];
}

// ================================================= multi-group (ensemble) launches
// An ensemble of RVEs of several sizes keeps one batch of same-size RVEs per
// size (a group).  Each kernel of a pass is then launched once for the whole
// ensemble: the flat block index selects the group and a block of that
// group's own grid, and the group's arguments (geometry, buffers, transform
// plan, device state) come from a table in the kernel arguments.  The body
// that runs is the single-group kernel's, with the compile-time variant the
// group would use on its own (DCT length, partition length).
constexpr int kMaxGroups = 8;

struct GroupMap {
  int ng;
  unsigned start[kMaxGroups + 1];  // first flat block of each group; start[ng] = total
  dim3 grid[kMaxGroups];           // each group's own grid
  __device__ __forceinline__ int find(SubGrid& sg) const {
    const unsigned b = blockIdx.x;
    int gi = 0;
#pragma unroll
    for (int i = 1; i < kMaxGroups; ++i) gi = (i < ng && b >= start[i]) ? i : gi;
    const unsigned local = b - start[gi];
    const dim3 gd = grid[gi];
    sg.b = dim3(local % gd.x, (local / gd.x) % gd.y, local / (gd.x * gd.y));
    sg.g = gd;
    return gi;
  }
};

template <class S, class W, class KT> struct StencilArgs {
  Geo g;
  const W* w;
  Kap<S> kp;
  const KT* ks;
  Rhs rh;
  S* q;
  double* partials;
  const DevState* st;
  int kchunk;
};
template <class S, class W, class KT> struct StencilMulti { StencilArgs<S, W, KT> a[kMaxGroups]; };

template <class S, bool RES, class KT, int TBW, int TAH, bool PLAIN = false>
__global__ __launch_bounds__(TBW*(TAH / 4)) void k_apply_A_iso_multi(
    GroupMap gm, StencilMulti<S, typename std::conditional<RES, double, S>::type, KT> m, int gate) {
  SubGrid sg;
  const auto& x = m.a[gm.find(sg)];
  k_apply_A_iso_body<S, RES, KT, TBW, TAH, SubGrid, PLAIN>(sg, x.g, x.w, x.kp, x.ks, x.rh, x.q, x.partials, x.st,
                                                          gate, x.kchunk);
}

template <class S, class T> struct RowsArgs {
  Geo g;
  DctPlan dp;
  const cx<T>* tw;
  const S* src;
  S* dst;
  int rpb, nrows;
  S* aux;            // forward: r (MODE 1); backward: the solution accumulator
  const S* q;
  double* partials;
  const DevState* st;
  int nc;            // compile-time length of the group's row kernels (0: run-time shaped)
};
template <class S, class T> struct RowsMulti { RowsArgs<S, T> a[kMaxGroups]; };

// Calls f(std::integral_constant<int, NC>) for the ensemble lengths with
// compile-time kernels (up to 160: the longer ones would raise the register
// count of every multi-group launch), else with NC = 0 (run-time shaped).
__host__ __device__ constexpr bool multi_nc(int nc) { return nc == 160 || nc == 128 || nc == 96 || nc == 64 || nc == 48; }
template <class F> __device__ __forceinline__ void with_nc(int nc, F&& f) {
  switch (nc) {
    case 160: f(std::integral_constant<int, 160>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 96: f(std::integral_constant<int, 96>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 48: f(std::integral_constant<int, 48>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
  }
}

template <class S, class T, int MODE>
__global__ __launch_bounds__(256) void k_rows_fwd_multi(GroupMap gm, RowsMulti<S, T> m, int gate) {
  SubGrid sg;
  const auto& x = m.a[gm.find(sg)];
  with_nc(x.nc, [&](auto nc) {
    k_rows_fwd_body<S, T, MODE, decltype(nc)::value, SubGrid>(sg, x.g, x.dp, x.tw, x.src, x.dst, x.rpb, x.nrows,
                                                                x.aux, x.q, x.partials, x.st, gate);
  });
}

template <class S, class T, int MODE>
__global__ __launch_bounds__(256) void k_rows_inv_multi(GroupMap gm, RowsMulti<S, T> m, int gate) {
  SubGrid sg;
  const auto& x = m.a[gm.find(sg)];
  with_nc(x.nc, [&](auto nc) {
    k_rows_inv_body<S, T, MODE, decltype(nc)::value, SubGrid>(sg, x.g, x.dp, x.tw, x.src, x.dst, x.rpb, x.nrows,
                                                                x.aux, x.st, gate);
  });
}

template <class S, class T> struct ColsArgs {
  Geo g;
  DctPlan dp;
  const cx<T>* tw;
  S* data;
  int tb;
  const DevState* st;
  int nc;
};
template <class S, class T> struct ColsMulti { ColsArgs<S, T> a[kMaxGroups]; };

template <class S, class T, int DIR>
__global__ __launch_bounds__(512) void k_cols_multi(GroupMap gm, ColsMulti<S, T> m, int gate) {
  SubGrid sg;
  const auto& x = m.a[gm.find(sg)];
  with_nc(x.nc, [&](auto nc) {
    k_cols_body<S, T, DIR, decltype(nc)::value, SubGrid>(sg, x.g, x.dp, x.tw, x.data, x.tb, x.st, gate);
  });
}

template <class S> struct ThomasArgs {
  Geo g;
  RefMedium rm;
  S* t;
  int Puse;
  double* partials;
  const DevState* st;
  int ntx, ntiles;
  int variant;  // index into ThomasVariants<S> (the launch's own)
};
template <class S> struct ThomasMulti { ThomasArgs<S> a[kMaxGroups]; };

// The groups of one launch share its variant I (a launch per variant the
// groups use): one body per kernel keeps each variant's register allocation
// that of its single-group kernel (a kernel holding several bodies takes
// the register pressure of the worst and spills in all of them).
template <class S, int I>
__global__ __launch_bounds__(ThomasVariants<S>::v[I].threads(), (ThomasVariants<S>::v[I].rows > 16 ? 2 : 4)) void
k_thomas_multi(GroupMap gm, ThomasMulti<S> m, int gate) {
  constexpr ThomasVariant v = ThomasVariants<S>::v[I];
  constexpr bool PF = (v.exact && sizeof(S) == 4) || v.rows <= 8;
  __shared__ double sh[6][v.p][v.tb + 1];
  __shared__ double red[16];
  SubGrid sg;
  const auto& x = m.a[gm.find(sg)];
  k_thomas_body<S, v.tb, v.p, v.rows, v.exact, PF, SubGrid>(sg, x.g, x.rm, x.t, x.Puse, x.partials, x.st, gate, x.ntx,
                                                             x.ntiles, sh, red);
}

struct FinArgs {
  const double* partials;
  int n;
  int64_t pstride;
  DevState* st;
  double* hist;
  int hstride;
};
struct FinMulti { FinArgs a[kMaxGroups]; };

// one block per instance of the ensemble (group grids (instances, 1, 1))
__global__ __launch_bounds__(1024) void k_fin_multi(GroupMap gm, FinMulti m, int op) {
  SubGrid sg;
  const auto& x = m.a[gm.find(sg)];
  k_fin_body<SubGrid>(sg, op, x.partials, x.n, x.pstride, x.st, x.hist, x.hstride);
}

struct FlushArgs {
  Geo g;
  double* p;
  float* dlt;
  const float* w;
  const DevState* st;
};
struct FlushMulti { FlushArgs a[kMaxGroups]; };

__global__ __launch_bounds__(256) void k_flush_multi(GroupMap gm, FlushMulti m) {
  SubGrid sg;
  const auto& x = m.a[gm.find(sg)];
  k_flush_body<SubGrid>(sg, x.g, x.p, x.dlt, x.w, x.st);
}

}  // namespace etc
