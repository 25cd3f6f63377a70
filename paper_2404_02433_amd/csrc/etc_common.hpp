// Shared device/host definitions of the ETC (effective thermal conductivity)
// library: grid geometry, device-resident solver state, block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace etc {

// Canonical layout [k][a][b]: k = load (Dirichlet) axis, slowest; b contiguous.
struct Geo {
  int nL, na, nb;
  int64_t plane;      // na * nb
  int64_t V;          // nL * na * nb (one instance)
  int nseg;           // instances stacked along the load axis (a batch of same-size RVEs)
  double fL, fa, fb;  // 1 / h^2 per canonical axis (scaled conductivity factors)
  double p_in, p_out;
};

// Reference-medium parameters (per instance: kL ka kb kin kout) and what the
// tridiagonal kernel needs to form a mode's shift lambda_a ka + lambda_b kb
// (lambda(k) = 4 sin^2(k step), step = pi / (2 N) per transverse axis) and to
// scale its r . z partials.  Kernel arguments, so they sit in scalar registers.
struct RefMedium {
  const double* kref;      // 5 per instance
  double step_a, step_b;   // pi / (2 na), pi / (2 nb)
  double dot_scale;        // 4 / (na nb), Parseval weight of the transformed dot product
};

// Solver state kept in device memory so the host never waits per dot product.
struct DevState {
  double rho;          // r . z of the current iterate
  double alpha, beta;  // step and direction coefficients of the current pass
  double wq;           // w . A w
  double rr;           // ||r||^2 of the recursively updated residual
  double rr_true;      // ||b - A p||^2 at the last refinement (mixed form)
  double bnorm2;       // ||b||^2
  double relres;       // last relative residual written to the history
  double rtol;
  double k_acc[4];     // result accumulators (flux sums, dissipation)
  int iter;            // completed passes (products A w)
  int done;            // 1: every later kernel of the solve returns at once
  int status;          // 0 ok, 1 not converged, -4 breakdown
  int refine;          // 1: the true residual is recomputed in this pass
  int max_iter;
  int refine_every;    // 0: never (FP64 form)
  int mixed;
  int pending;         // 1: the last pass's x += alpha w is still to be applied
};

enum { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = -4 };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Orders the shared-memory accesses of one wave: accesses before it complete
// (and are visible to the wave's other lanes) before any after it.  Lanes
// that exchange data through shared memory within one wave need this, not a
// block barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Deterministic block sum: fixed shuffle tree per wave, then the wave sums in
// order.  Result valid in thread 0.  `lds` holds >= 16 doubles.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  v = wave_sum(v);
  if ((tid & 63) == 0) lds[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    const int nw = (nthr + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += lds[i];
  }
  __syncthreads();
  return s;
}

__device__ __forceinline__ int flat_block() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// Block index and grid seen by a kernel body.  HwGrid: the launch's own
// (the hardware registers, read where used).  SubGrid: one group's share of
// a launch that covers several groups, each with a grid of its own.
struct HwGrid {
  __device__ __forceinline__ unsigned bx() const { return blockIdx.x; }
  __device__ __forceinline__ unsigned by() const { return blockIdx.y; }
  __device__ __forceinline__ unsigned bz() const { return blockIdx.z; }
  __device__ __forceinline__ unsigned gx() const { return gridDim.x; }
  __device__ __forceinline__ unsigned gy() const { return gridDim.y; }
  __device__ __forceinline__ unsigned gz() const { return gridDim.z; }
  __device__ __forceinline__ int flat() const { return flat_block(); }
};
struct SubGrid {
  dim3 b, g;
  __device__ __forceinline__ unsigned bx() const { return b.x; }
  __device__ __forceinline__ unsigned by() const { return b.y; }
  __device__ __forceinline__ unsigned bz() const { return b.z; }
  __device__ __forceinline__ unsigned gx() const { return g.x; }
  __device__ __forceinline__ unsigned gy() const { return g.y; }
  __device__ __forceinline__ unsigned gz() const { return g.z; }
  __device__ __forceinline__ int flat() const { return (int)(b.x + g.x * (b.y + g.y * b.z)); }
};

// Work-groups are dealt to the 8 XCDs round-robin by flat id.  Renumber so
// that each XCD receives one contiguous range of tiles: tiles that share halo
// lines then run on the same XCD at about the same time and meet in its L2.
// A bijection of [0, total) for any total.
__device__ __forceinline__ int xcd_tile(int id, int total) {
  constexpr int NX = 8;
  const int x = id % NX, j = id / NX;
  const int per = total / NX, rem = total % NX;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
}

template <class T> __device__ __forceinline__ double to_d(T v) { return static_cast<double>(v); }

// Harmonic-mean face conductivity 2 k1 k2 / (k1 + k2) of two cells.
template <class C> __device__ __forceinline__ C harm(C k1, C k2) {
  return C(2) * k1 * k2 / (k1 + k2);
}

// Reciprocal: hardware estimate refined by two Newton steps (within one ulp
// of the correctly rounded quotient for positive normal arguments).
__device__ __forceinline__ double frcp(double u) {
  double r = __builtin_amdgcn_rcp(u);
  double e = fma(-u, r, 1.0);
  r = fma(r, e, r);
  e = fma(-u, r, 1.0);
  return fma(r, e, r);
}
// float32: the hardware reciprocal (1 ulp)
__device__ __forceinline__ float frcp(float u) { return __builtin_amdgcn_rcpf(u); }
// Reciprocal with one Newton step: the estimate's relative error (below 5e-8
// measured) squares to a few 1e-15, ample where the values are stored as
// float32 afterwards.
__device__ __forceinline__ double frcp1(double u) {
  const double r = __builtin_amdgcn_rcp(u);
  return fma(r, fma(-u, r, 1.0), r);
}

// Face coefficient of the hot operator: the harmonic mean through the
// reciprocal above.  Symmetric in its arguments bit for bit (the product and
// the sum commute, the factor 2 is exact).
template <class C> __device__ __forceinline__ C hface(C k1, C k2) {
  return C(2) * k1 * k2 * frcp(k1 + k2);
}

}  // namespace etc
