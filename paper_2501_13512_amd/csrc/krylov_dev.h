// Device-side pieces of the BiCGSTAB step shared by the vector kernels and
// by the FFT passes that fuse vector updates and inner products.
//
// Reductions: every workgroup of a system writes its partial sum; a finalize
// kernel (one workgroup per system, all systems of a solve in one launch)
// sums the partials in a fixed order (deterministic, no atomics or
// device-scope fences) and applies the scalar step of the iteration.
#pragma once
#include "kernels.h"

namespace vie {

constexpr int NPART = 4;   // doubles per partial

// Sum NV doubles over the workgroup (any size <= 1024); valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sm[16][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  // lanes that exist in this wavefront (the last one may be partial)
  const int live = min(64, (int)blockDim.x - wid * 64);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double o = __shfl_down(v[k], off, 64);
      if (lane + off < live) v[k] += o;
    }
  __syncthreads();   // sm may still be read by a previous call
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sm[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double a = sm[0][k];
      for (int w = 1; w < nw; ++w) a += sm[w][k];
      v[k] = a;
    }
  }
}

// Workgroup `tile` of `ntiles` of system `sys` writes its partial sum (plain
// stores; the finalize kernel that reads them runs after this kernel ends).
// Tile 0 also records how many partials the system has.
template <int NV>
__device__ __forceinline__ void write_partial(double (&v)[NV], double* partials, int64_t pstride, int* ntile,
                                              int sys, int64_t tile, int64_t ntiles) {
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
    double* p = partials + sys * pstride + tile * NPART;
#pragma unroll
    for (int k = 0; k < NV; ++k) p[k] = v[k];
    if (tile == 0) ntile[sys] = (int)ntiles;
  }
}

// Sum of system `sys`'s partials in a fixed order; valid in thread 0.
template <int NV>
__device__ __forceinline__ void final_sum(const double* partials, int64_t pstride, const int* ntile, int sys,
                                          double (&v)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const int nt = ntile[sys];
  for (int c = threadIdx.x; c < nt; c += blockDim.x) {
    const double* p = partials + sys * pstride + (int64_t)c * NPART;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += p[k];
  }
  block_sum<NV>(v);
}

// As write_partial, without recording the partial count (a consumer in the
// same kernel may still read the count of another buffer).
template <int NV>
__device__ __forceinline__ void write_partial_at(double (&v)[NV], double* partials, int64_t pstride, int sys,
                                                 int64_t tile) {
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
    double* p = partials + sys * pstride + tile * NPART;
#pragma unroll
    for (int k = 0; k < NV; ++k) p[k] = v[k];
  }
}

// final_sum broadcast to every thread of the workgroup (all threads call).
template <int NV>
__device__ __forceinline__ void final_sum_all(const double* partials, int64_t pstride, const int* ntile, int sys,
                                              double (&v)[NV]) {
  __shared__ double bc[NV];
  final_sum<NV>(partials, pstride, ntile, sys, v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) bc[k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = bc[k];
  __syncthreads();
}

__device__ __forceinline__ c128 cdiv(c128 a, c128 b) {
  const double s = fabs(b.x) + fabs(b.y);
  const double br = b.x / s, bi = b.y / s, ar = a.x / s, ai = a.y / s;
  const double d = br * br + bi * bi;
  return mk<double>((ar * br + ai * bi) / d, (ai * br - ar * bi) / d);
}

// alpha = rho / <rhat, v> inside a product's first pass (in_mode 3): every
// workgroup of the system sums the <rhat, v> partials of the previous
// product in the same order; the owner (the system's first workgroup) counts
// the step and records alpha, or the breakdown.  All threads call; returns
// false on breakdown (<rhat, v> = 0).
__device__ __forceinline__ bool fused_alpha(const KBatch& k, int sys, bool owner, c128* alpha) {
  double v[2];
  final_sum_all<2>(k.partials, k.pstride, k.ntile, sys, v);
  KState& st = k.st[sys];
  const c128 den = mk<double>(v[0], v[1]);
  const bool ok = !(den.x == 0.0 && den.y == 0.0);
  *alpha = ok ? cdiv(st.rho, den) : mk<double>(0.0, 0.0);
  if (owner && threadIdx.x == 0) {
    st.iters += 1;
    if (ok)
      st.alpha = *alpha;
    else
      k.status[sys] = ST_BREAKDOWN;
  }
  return ok;
}

// ---- scalar steps (thread 0 of the finishing workgroup) ----

// alpha = rho / <rhat, v>; counts the step
__device__ __forceinline__ void fin_alpha(KState& k, int* status, const double* v) {
  k.iters += 1;
  const c128 den = mk<double>(v[0], v[1]);
  if (den.x == 0.0 && den.y == 0.0)
    *status = ST_BREAKDOWN;
  else
    k.alpha = cdiv(k.rho, den);
}

// half-step test on ||s||
__device__ __forceinline__ void fin_s(KState& k, int* status, double s2) {
  k.snorm = sqrt(s2) / k.nb;
  if (k.snorm <= k.tol) *status = ST_HALF;
}

// omega = <t, s> / <t, t>
__device__ __forceinline__ void fin_omega(KState& k, int* status, const double* v) {
  if (v[2] == 0.0)
    *status = ST_BREAKDOWN;
  else
    k.omega = mk<double>(v[0] / v[2], v[1] / v[2]);
}

// new rho = <rhat, r>, ||r||; convergence, breakdown, cap, next beta
__device__ __forceinline__ void fin_xr(KState& k, int* status, const double* v) {
  k.rnorm = sqrt(v[2]) / k.nb;
  k.rho_old = k.rho;
  k.rho = mk<double>(v[0], v[1]);
  const bool om0 = k.omega.x == 0.0 && k.omega.y == 0.0;
  const bool rho0 = k.rho.x == 0.0 && k.rho.y == 0.0;
  if (k.rnorm <= k.tol)
    *status = ST_CONVERGED;
  else if (om0 || rho0 || !(k.rnorm == k.rnorm))
    *status = ST_BREAKDOWN;
  else if (k.iters >= k.maxit)
    *status = ST_MAXIT;
  else
    k.beta = cdiv(k.rho, k.rho_old) * cdiv(k.alpha, k.omega);
}

// end of a CGS step (r recomputed as b - A x): new rho = <rhat, r>, ||r||;
// convergence, breakdown, cap, beta = rho' / rho
__device__ __forceinline__ void fin_cgs(KState& k, int* status, const double* v) {
  k.rnorm = sqrt(v[2]) / k.nb;
  k.rho_old = k.rho;
  k.rho = mk<double>(v[0], v[1]);
  const bool rho0 = k.rho.x == 0.0 && k.rho.y == 0.0;
  if (k.rnorm <= k.tol)
    *status = ST_CONVERGED;
  else if (rho0 || !(k.rnorm == k.rnorm))
    *status = ST_BREAKDOWN;
  else if (k.iters >= k.maxit)
    *status = ST_MAXIT;
  else
    k.beta = cdiv(k.rho, k.rho_old);
}

}  // namespace vie
