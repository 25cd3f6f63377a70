// Batched DCT-II / DCT-III engine for lines staged in LDS (gfx950).
//
// Forward transform (scale 1):   X[k] = sum_n x[n] cos(pi (2n+1) k / (2N))
// Backward transform (scale 2/N, alpha_0 = 1/2) is its exact inverse; both are
// the 1D pair of the paper's Section "Preconditioner system solver".
//
// Route for even N (M = N/2): reorder x into v (even samples ascending, odd
// samples descending), read v as M complex values z[n] = v[2n] + i v[2n+1],
// run an M-point complex FFT (Stockham, radices 2/3/4/5/8/16, in LDS), then
// split the half-length spectrum and rotate by exp(-i pi k / 2N).  The
// backward transform runs the same steps in reverse.  Lengths whose half does
// not factor into those radices (and odd N) use the O(N^2) definition.
#pragma once
#include <hip/hip_runtime.h>

namespace etc {

template <class T> struct cx {
  T re, im;
};

template <class T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
template <class T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by DIR * i  (DIR = -1: forward transform sign)
template <int DIR, class T> __device__ __forceinline__ cx<T> rot_i(cx<T> a) {
  return DIR < 0 ? cx<T>{a.im, -a.re} : cx<T>{-a.im, a.re};
}

// Stage plan of one transform length, passed by value to kernels.
struct DctPlan {
  int N;        // transform length
  int M;        // N / 2 on the FFT route
  int fft;      // 1: FFT route, 0: O(N^2) definition
  int nst;      // number of radix stages (product of R[] = M)
  int R[8];
  int lstride;  // LDS stride of one line, in elements of the line buffer
};

// LDS index padding: one spare slot after every 16 complex values keeps
// power-of-two strided accesses from landing in one bank group.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// ----------------------------------------------------------------- codelets
template <int DIR, class T> __device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int DIR, class T> __device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = rot_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int DIR, class T> __device__ __forceinline__ void dft3(cx<T>* v) {
  const T s60 = T(0.86602540378443864676372317075294);
  cx<T> t1 = cadd(v[1], v[2]);
  cx<T> t2 = {v[0].re - T(0.5) * t1.re, v[0].im - T(0.5) * t1.im};
  cx<T> t3 = cscale(rot_i<DIR>(csub(v[1], v[2])), s60);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}

template <int DIR, class T> __device__ __forceinline__ void dft5(cx<T>* v) {
  const T c1 = T(0.30901699437494742410229341718282), c2 = T(-0.80901699437494742410229341718282);
  const T s1 = T(0.95105651629515357211643933337938), s2 = T(0.58778525229247312916870595463907);
  cx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]), t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  cx<T> a = {v[0].re + c1 * t1.re + c2 * t2.re, v[0].im + c1 * t1.im + c2 * t2.im};
  cx<T> b = {v[0].re + c2 * t1.re + c1 * t2.re, v[0].im + c2 * t1.im + c1 * t2.im};
  cx<T> u = rot_i<DIR>(cx<T>{s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im});
  cx<T> w = rot_i<DIR>(cx<T>{s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im});
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(a, u);
  v[4] = csub(a, u);
  v[2] = cadd(b, w);
  v[3] = csub(b, w);
}

template <int DIR, class T> __device__ __forceinline__ void dft8(cx<T>* v) {
  const T h = T(0.70710678118654752440084436210485);
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // o_k *= exp(DIR 2 pi i k / 8)
  o1 = cmul(o1, cx<T>{h, T(DIR) * h});
  o2 = rot_i<DIR>(o2);
  o3 = cmul(o3, cx<T>{-h, T(DIR) * h});
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <int DIR, class T> __device__ __forceinline__ void dft16(cx<T>* v) {
  // n = 4 n1 + n2, k = k1 + 4 k2
  const T c1 = T(0.92387953251128675612818318939679), s1 = T(0.38268343236508977172845998403040);
  const T h = T(0.70710678118654752440084436210485);
  cx<T> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cx<T> a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
    dft4<DIR>(a0, a1, a2, a3);
    y[n2][0] = a0;
    y[n2][1] = a1;
    y[n2][2] = a2;
    y[n2][3] = a3;
  }
  // twiddles exp(DIR 2 pi i n2 k1 / 16), n2 k1 in {1,2,3,4,6,9}
  const T sg = T(DIR);
  y[1][1] = cmul(y[1][1], cx<T>{c1, sg * s1});
  y[1][2] = cmul(y[1][2], cx<T>{h, sg * h});
  y[1][3] = cmul(y[1][3], cx<T>{s1, sg * c1});
  y[2][1] = cmul(y[2][1], cx<T>{h, sg * h});
  y[2][2] = rot_i<DIR>(y[2][2]);
  y[2][3] = cmul(y[2][3], cx<T>{-h, sg * h});
  y[3][1] = cmul(y[3][1], cx<T>{s1, sg * c1});
  y[3][2] = cmul(y[3][2], cx<T>{-h, sg * h});
  y[3][3] = cmul(y[3][3], cx<T>{-c1, -sg * s1});
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1];
    dft4<DIR>(a0, a1, a2, a3);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

template <int R, int DIR, class T> __device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 5) dft5<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else dft16<DIR>(v);
}

// ------------------------------------------------------------ Stockham stage
// One radix-R stage over `lines` lines of M complex values (LDS, padded),
// line stride `ls` (complex units).  `tw[j]` = exp(-2 pi i j / (8M)).
// Every thread must call it (it contains barriers).
// Complex values a thread may hold in one stage.
template <class T> struct stage_cap {
  static constexpr int v = 16;
};
template <class T, int R> struct ipt_of {
  static constexpr int v = (R >= stage_cap<T>::v) ? 1 : (stage_cap<T>::v / R);
};

// Items per thread of a radix-R stage: a stage over `lines` lines of M points
// fits one pass when lines * M <= stage_cap * nthr.  Not inlined, so each
// radix gets its own register allocation.
template <class T, int R, int DIR, int IPT = ipt_of<T, R>::v>
__device__ __attribute__((noinline)) void fft_stage(cx<T>* buf, int lines, int ls, int M, int Ns, const cx<T>* __restrict__ tw,
                                          int tid, int nthr) {
  const int per_line = M / R;
  const int items = lines * per_line;
  const int step = M / (Ns * R);
  cx<T> v[IPT][R];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int it = tid + i * nthr;
    if (it < items) {
      const int line = it / per_line, j = it - line * per_line;
      const cx<T>* L = buf + line * ls;
      const int jm = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = L[lpad(j + r * per_line)];
      if (jm != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[8 * jm * r * step];
          if (DIR > 0) w.im = -w.im;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      dftR<R, DIR>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int it = tid + i * nthr;
    if (it < items) {
      const int line = it / per_line, j = it - line * per_line;
      cx<T>* L = buf + line * ls;
      const int jm = j % Ns;
      const int idxD = (j / Ns) * Ns * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) L[lpad(idxD + r * Ns)] = v[i][r];
    }
  }
  __syncthreads();
}

// All stages of an M-point FFT on `lines` LDS lines (natural-order output).
template <class T, int DIR>
__device__ void lds_fft(cx<T>* buf, int lines, int ls, const DctPlan& dp, const cx<T>* __restrict__ tw, int tid,
                        int nthr) {
  int Ns = 1;
  for (int s = 0; s < dp.nst; ++s) {
    const int R = dp.R[s];
    switch (R) {
      case 2: fft_stage<T, 2, DIR>(buf, lines, ls, dp.M, Ns, tw, tid, nthr); break;
      case 3: fft_stage<T, 3, DIR>(buf, lines, ls, dp.M, Ns, tw, tid, nthr); break;
      case 4: fft_stage<T, 4, DIR>(buf, lines, ls, dp.M, Ns, tw, tid, nthr); break;
      case 5: fft_stage<T, 5, DIR>(buf, lines, ls, dp.M, Ns, tw, tid, nthr); break;
      case 8: fft_stage<T, 8, DIR>(buf, lines, ls, dp.M, Ns, tw, tid, nthr); break;
      default: fft_stage<T, 16, DIR>(buf, lines, ls, dp.M, Ns, tw, tid, nthr); break;
    }
    Ns *= R;
  }
}

// ------------------------------------------------ compile-time specialisation
// For the common lengths the whole stage schedule is fixed at compile time:
// line count, line stride, radices and stage strides are constants, so every
// index split (line, butterfly, twiddle) is a shift or a constant multiply.
// The launch shapes below are shared with the host so that both sides agree.
struct RadixPlan {
  int n;  // number of stages, -1 if M has a prime factor > 5
  int r[8];
};

__host__ __device__ constexpr RadixPlan radix_plan(int M) {
  RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
  int m = M;
  const int pref[6] = {16, 8, 4, 2, 3, 5};
  for (int i = 0; i < 6; ++i)
    while (m % pref[i] == 0 && m >= pref[i]) {
      if (p.n >= 8) return RadixPlan{-1, {0, 0, 0, 0, 0, 0, 0, 0}};
      p.r[p.n++] = pref[i];
      m /= pref[i];
    }
  if (m != 1) p.n = -1;
  return p;
}

// LDS slots (complex) per line of M complex values: padded, odd.
__host__ __device__ constexpr int fft_lstride(int M) {
  const int ls = (M - 1) + ((M - 1) >> 4) + 1;
  return (ls % 2 == 0) ? ls + 1 : ls;
}

// Most lines that one pass of every stage of an M-point FFT covers with
// nthr threads: a radix-R stage of the run-time route holds 16 / R (at
// least 1) butterflies per thread, so lines * (M / R) <= (16 / R) * nthr
// for each radix of the plan (radices 3 and 5 bind below lines * M = 16 nthr).
// 0 when not even one line fits.
__host__ __device__ constexpr int fft_lines_cap(int M, int nthr) {
  const RadixPlan p = radix_plan(M);
  int c = 16 * nthr / M;
  for (int i = 0; i < p.n; ++i) {
    const int R = p.r[i];
    const int ci = (R >= 16 ? 1 : 16 / R) * nthr / (M / R);
    if (ci < c) c = ci;
  }
  return c;
}

// Lines per block of the row transforms (256 threads): an LDS budget of
// 48 KiB and one pass of every FFT stage.
__host__ __device__ constexpr int rows_lines(int M, int ls, int elt, bool fft) {
  const int line_bytes = ls * 2 * elt;
  int r = (48 * 1024) / line_bytes;
  if (r < 1) r = 1;
  if (fft) {
    int c = fft_lines_cap(M, 256);
    if (c < 1) c = 1;
    if (c < r) r = c;
  }
  return r < 64 ? r : 64;
}

// Columns per block of the column transforms (256 threads in float64, 512 in
// float32): an LDS budget of 80 KiB, one pass of every FFT stage, 16 or 32
// columns when they fit (whole 128-byte rows).
__host__ __device__ constexpr int cols_threads(int elt) { return elt == 4 ? 512 : 256; }
__host__ __device__ constexpr int cols_tile(int M, int ls, int elt, bool fft) {
  const int line_bytes = ls * 2 * elt;
  int tb = (80 * 1024) / line_bytes;
  if (tb < 1) tb = 1;
  if (fft) {
    int c = fft_lines_cap(M, cols_threads(elt));
    if (c < 1) c = 1;
    if (c < tb) tb = c;
  }
  if (tb > 32) tb = 32;
  if (tb >= 16) tb = 16 * (tb / 16);
  else if (tb >= 8) tb = 8;
  return tb;
}

// One radix-R Stockham stage over LINES lines of M points (line stride LS),
// all shapes compile-time.  Same data flow as fft_stage.
// TWS: twiddle j of a stage is tw[TWS * j] (8 for the plan's table of 4N
// entries, 1 for a table of its every 8th entry).
template <class T, int R, int DIR, int M, int NS, int LINES, int NTHR, int LS, int TWS = 8>
__device__ __forceinline__ void fft_stage_ct(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  constexpr int per_line = M / R;
  constexpr int items = LINES * per_line;
  constexpr int step = M / (NS * R);
  constexpr int IPT = (items + NTHR - 1) / NTHR;
  cx<T> v[IPT][R];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int it = tid + i * NTHR;
    if (items % NTHR == 0 || it < items) {
      const int line = it / per_line, j = it - line * per_line;
      const cx<T>* L = buf + line * LS;
      const int jm = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = L[lpad(j + r * per_line)];
      if (NS > 1 && jm != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[TWS * step * r * jm];
          if (DIR > 0) w.im = -w.im;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      dftR<R, DIR>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int it = tid + i * NTHR;
    if (items % NTHR == 0 || it < items) {
      const int line = it / per_line, j = it - line * per_line;
      cx<T>* L = buf + line * LS;
      const int jm = j % NS;
      const int idxD = (j / NS) * NS * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) L[lpad(idxD + r * NS)] = v[i][r];
    }
  }
  __syncthreads();
}

template <class T, int DIR, int M, int LINES, int NTHR, int LS, int S = 0, int NS = 1, int TWS = 8>
__device__ __forceinline__ void lds_fft_ct(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  constexpr RadixPlan rp = radix_plan(M);
  static_assert(rp.n > 0, "length not supported by the compile-time route");
  if constexpr (S < rp.n) {
    constexpr int R = rp.r[S];
    fft_stage_ct<T, R, DIR, M, NS, LINES, NTHR, LS, TWS>(buf, tw, tid);
    lds_fft_ct<T, DIR, M, LINES, NTHR, LS, S + 1, NS * R, TWS>(buf, tw, tid);
  }
}

// Position of input sample j in the reordered sequence v (FFT route).
__device__ __forceinline__ int dct_perm(int j, int N) { return (j & 1) ? (N - 1 - (j >> 1)) : (j >> 1); }

// Real offset (in T units) of v[m] inside a padded complex line.
__device__ __forceinline__ int vpos(int m) { return 2 * lpad(m >> 1) + (m & 1); }

// Forward post-processing of one item k in [0, M/2]: from the half-length
// spectrum Z (LDS line) produce the outputs X[k], X[N-k], X[M-k], X[M+k].
// `emit(index, value)` stores one output.
// Twiddles exp(-i pi j / 2N) of the DCT pre/post steps from two short
// tables: j <= M (lo) and the multiples of 4 up to 4M (q, entry j / 4) --
// every index those steps use.
template <class T> struct DctTw {
  const cx<T>* lo;
  const cx<T>* q;
  int M;
  __device__ __forceinline__ cx<T> operator[](int j) const { return j <= M ? lo[j] : q[j >> 2]; }
};

// W with X[k] = Re W, X[N-k] = -Im W, from A = Z[k] and B = Z[M-k].  (TW:
// a twiddle table pointer, or DctTw.)
template <class T, class TW>
__device__ __forceinline__ cx<T> dct_post_w(cx<T> A, cx<T> B, int k, const TW& tw) {
  const T half = T(0.5);
  cx<T> s = cadd(A, cconj(B)), d = csub(A, cconj(B));
  cx<T> V = csub(cscale(s, half), cscale(rot_i<+1>(cmul(tw[4 * k], d)), half));
  return cmul(tw[k], V);
}

template <class T, class Emit>
__device__ __forceinline__ void dct_post(const cx<T>* Z, int k, int N, int M, const cx<T>* __restrict__ tw, Emit emit) {
  if (k == 0) {
    cx<T> z0 = Z[lpad(0)];
    emit(0, z0.re + z0.im);
    // X[M] = Re(exp(-i pi/4) (Re z0 - Im z0))
    emit(M, (z0.re - z0.im) * tw[M].re);
    return;
  }
  const int k2 = M - k;
  cx<T> A = Z[lpad(k)], B = Z[lpad(k2)];
  {
    const cx<T> W = dct_post_w(A, B, k, tw);
    emit(k, W.re);
    emit(N - k, -W.im);
  }
  if (k2 != k) {
    const cx<T> W = dct_post_w(B, A, k2, tw);
    emit(k2, W.re);
    emit(N - k2, -W.im);
  }
}

// The same outputs in items of exactly four (M even), without branches:
// item 0 covers k = 0 and k = M/2, item k in [1, M/2) covers k and M - k.
template <class T, class TW, class Emit>
__device__ __forceinline__ void dct_post4(const cx<T>* Z, int k, int N, int M, const TW& tw, Emit emit) {
  const bool z = k == 0;
  const int h = M / 2, k2 = z ? h : M - k;
  const cx<T> A = Z[lpad(k)], B = Z[lpad(k2)];
  const cx<T> W = dct_post_w(A, B, k, tw);               // k > 0: X[k], X[N-k]
  const cx<T> W2 = dct_post_w(B, z ? B : A, k2, tw);     // X[k2], X[N-k2] (k = 0: X[M/2], X[N-M/2])
  emit(k, z ? A.re + A.im : W.re);                       // k = 0: X[0]
  emit(z ? M : N - k, z ? (A.re - A.im) * tw[M].re : -W.im);  // k = 0: X[M]
  emit(k2, W2.re);
  emit(N - k2, -W2.im);
}

// Backward pre-processing of one item k in [0, M/2] from the four inputs
// xk = X[k], xnk = X[N-k], xk2 = X[M-k], xnk2 = X[M+k] (for k = 0: X[0], X[M]
// in xk, xk2); writes Z[k] and Z[M-k] to the LDS line.
template <class T, class TW>
__device__ __forceinline__ void dct_pre_inv_vals(cx<T>* Z, int k, int M, const TW& tw, T xk, T xnk, T xk2, T xnk2) {
  const T half = T(0.5);
  if (k == 0) {
    cx<T> V0 = {xk, T(0)};
    // V[M] = exp(i pi/4) (X[M] - i X[M]) = sqrt(2) X[M]
    cx<T> VM = cmul(cconj(tw[M]), cx<T>{xk2, -xk2});
    cx<T> E = cscale(cadd(V0, cconj(VM)), half);
    cx<T> O = cscale(csub(V0, cconj(VM)), half);
    Z[lpad(0)] = cadd(E, rot_i<+1>(O));
    return;
  }
  const int k2 = M - k;
  cx<T> Vk = cmul(cconj(tw[k]), cx<T>{xk, -xnk});
  cx<T> Vk2 = cmul(cconj(tw[k2]), cx<T>{xk2, -xnk2});
  {
    cx<T> E = cscale(cadd(Vk, cconj(Vk2)), half);
    cx<T> O = cscale(cmul(cconj(tw[4 * k]), csub(Vk, cconj(Vk2))), half);
    Z[lpad(k)] = cadd(E, rot_i<+1>(O));
  }
  if (k2 != k) {
    cx<T> E = cscale(cadd(Vk2, cconj(Vk)), half);
    cx<T> O = cscale(cmul(cconj(tw[4 * k2]), csub(Vk2, cconj(Vk))), half);
    Z[lpad(k2)] = cadd(E, rot_i<+1>(O));
  }
}

// Indices of the four inputs of backward item k (k = 0 uses slots 0 and 2).
__device__ __forceinline__ void pre_inv_idx(int k, int N, int M, int& i0, int& i1, int& i2, int& i3) {
  if (k == 0) {
    i0 = 0;
    i1 = 0;
    i2 = M;
    i3 = M;
  } else {
    i0 = k;
    i1 = N - k;
    i2 = M - k;
    i3 = M + k;
  }
}

}  // namespace etc
