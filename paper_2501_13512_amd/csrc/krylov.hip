// BiCGSTAB vector operations and reductions for batches of independent
// systems, and the gather/scatter between the outer vector and the blocks of
// the block-diagonal preconditioner (Sec. II-B, eqs. (10)-(11)).
//
// Every reduction is deterministic: each workgroup reduces a fixed chunk of
// 2048 elements (wavefront shuffles, then LDS) into a partial, and a finalize
// kernel with one workgroup per system sums the partials in a fixed order and
// applies the scalar step of the iteration.  No floating-point atomics.
// Elementwise kernels issue all loads of a thread's elements before their
// stores, so the loads overlap (the vectors may alias as far as the compiler
// knows).
//
// BiCGSTAB (van der Vorst), right-preconditioned, per system:
//   rho = <rhat, r>; p = r + beta (p - omega v); y = K^{-1} p; v = A y;
//   alpha = rho / <rhat, v>; s = r - alpha v; [||s|| <= tol ||b||: x += alpha y]
//   z = K^{-1} s; t = A z; omega = <t, s> / <t, t>;
//   x += alpha y + omega z; r = s - omega t; beta = (rho'/rho)(alpha/omega).
//
// Conjugate gradient squared (Sonneveld), right-preconditioned, per system:
//   u = r + beta q; p = u + beta (q + beta p); v = A K^{-1} p;
//   alpha = rho / <rhat, v>; q = u - alpha v; x += alpha K^{-1} (u + q);
//   r = b - A x; rho' = <rhat, r>; beta = rho' / rho.
#include <stdexcept>
#include <string>

#include "krylov_dev.h"

namespace vie {

constexpr int KT = 256;               // threads per workgroup
constexpr int KEPT = 8;               // elements per thread
constexpr int KCH = KT * KEPT;        // elements per chunk

__host__ __device__ inline int64_t chunks_of(int64_t n) { return (n + KCH - 1) / KCH; }
int64_t krylov_chunks(int64_t n) { return chunks_of(n); }

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

// chunk / system decomposition of a (chunks x nsys) grid
#define KRYLOV_INDEX                                         \
  const int64_t chunks = chunks_of(n);                       \
  const int sys = (int)(blockIdx.x / chunks);                \
  const int64_t chunk = blockIdx.x - (int64_t)sys * chunks;  \
  const int64_t base = (int64_t)sys * n;                     \
  const int64_t i0 = chunk * KCH + threadIdx.x;

// ---------------------------------------------------------------- init
__global__ void __launch_bounds__(KT) kk_init(KBatch k, const int* gate, const c128* b, c128* x, c128* r,
                                              c128* rhat) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  if (gate && *gate != ST_ACTIVE) return;
  double acc[1] = {0.0};
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      const c128 v = b[base + i];
      x[base + i] = mk<double>(0.0, 0.0);
      r[base + i] = v;
      rhat[base + i] = v;
      acc[0] += abs2(v);
    }
  }
  write_partial<1>(acc, k.partials, k.pstride, k.ntile, sys, chunk, chunks);
}

void k_init(const KBatch& k, const c128* b, c128* x, c128* r, c128* rhat, const int* gate, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_init, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, gate, b, x, r, rhat);
  check_launch("krylov init");
}

// ---------------------------------------------------------------- finalize
__global__ void __launch_bounds__(KT) kk_finalize(KBatch k, int kind, const int* gate, double tol, int maxit) {
  const int sys = blockIdx.x;
  const int stt = k.status[sys];
  KState& st = k.st[sys];
  if (kind == FIN_INIT) {
    if (gate && *gate != ST_ACTIVE) {
      if (threadIdx.x == 0) k.status[sys] = ST_IDLE;
      return;
    }
    double v[1];
    final_sum<1>(k.partials, k.pstride, k.ntile, sys, v);
    if (threadIdx.x == 0) {
      const double nb = sqrt(v[0]);
      st.nb = nb;
      st.rho = mk<double>(v[0], 0.0);
      st.rho_old = mk<double>(1.0, 0.0);
      st.alpha = mk<double>(1.0, 0.0);
      st.omega = mk<double>(1.0, 0.0);
      st.beta = mk<double>(0.0, 0.0);
      st.rnorm = nb > 0.0 ? 1.0 : 0.0;
      st.snorm = st.rnorm;
      st.tol = tol;
      st.iters = 0;
      st.maxit = maxit;
      st.pending = 0;
      k.status[sys] = nb > 0.0 ? ST_ACTIVE : ST_CONVERGED;
    }
    return;
  }
  if (kind == FIN_XR && stt == ST_HALF) {
    if (threadIdx.x == 0) {
      st.rnorm = st.snorm;
      k.status[sys] = ST_CONVERGED;
    }
    return;
  }
  if (stt != ST_ACTIVE) return;
  if (kind == FIN_ALPHA) {
    double v[2];
    final_sum<2>(k.partials, k.pstride, k.ntile, sys, v);
    if (threadIdx.x == 0) fin_alpha(st, &k.status[sys], v);
  } else if (kind == FIN_S) {
    double v[1];
    final_sum<1>(k.partials, k.pstride, k.ntile, sys, v);
    if (threadIdx.x == 0) fin_s(st, &k.status[sys], v[0]);
  } else if (kind == FIN_OMEGA) {
    double v[3];
    final_sum<3>(k.partials, k.pstride, k.ntile, sys, v);
    if (threadIdx.x == 0) fin_omega(st, &k.status[sys], v);
  } else if (kind == FIN_SOMEGA) {
    double v[4];
    final_sum<4>(k.partials, k.pstride, k.ntile, sys, v);
    if (threadIdx.x == 0) {
      fin_s(st, &k.status[sys], v[3]);
      if (k.status[sys] == ST_ACTIVE) fin_omega(st, &k.status[sys], v);
    }
  } else if (kind == FIN_CGS) {
    double v[3];
    final_sum<3>(k.partials, k.pstride, k.ntile, sys, v);
    if (threadIdx.x == 0) fin_cgs(st, &k.status[sys], v);
  } else {
    double v[3];
    final_sum<3>(k.partials, k.pstride, k.ntile, sys, v);
    if (threadIdx.x == 0) fin_xr(st, &k.status[sys], v);
  }
}

void k_finalize(const KBatch& k, FinKind kind, hipStream_t s, const int* gate, double tol, int maxit) {
  if (k.nsys <= 0) return;
  hipLaunchKernelGGL(kk_finalize, dim3(k.nsys), dim3(KT), 0, s, k, (int)kind, gate, tol, maxit);
  check_launch("krylov finalize");
}

// ---------------------------------------------------------------- p update
__global__ void __launch_bounds__(KT) kk_update_p(KBatch k, const c128* r, const c128* v, c128* p) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  (void)chunk;
  if (k.status[sys] != ST_ACTIVE) return;
  const KState& st = k.st[sys];
  const bool first = st.iters == 0;
  const c128 beta = st.beta, omega = st.omega;
  c128 rv[KEPT], pv[KEPT], vv[KEPT];
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      rv[j] = r[base + i];
      if (!first) {
        pv[j] = p[base + i];
        vv[j] = v[base + i];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) p[base + i] = first ? rv[j] : rv[j] + beta * (pv[j] - omega * vv[j]);
  }
}

void k_update_p(const KBatch& k, const c128* r, const c128* v, c128* p, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_update_p, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, r, v, p);
  check_launch("krylov p");
}

// ---------------------------------------------------------------- s update
__global__ void __launch_bounds__(KT) kk_update_s(KBatch k, const c128* r, const c128* v, c128* sv) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  if (k.status[sys] != ST_ACTIVE) return;
  const c128 alpha = k.st[sys].alpha;
  double acc[1] = {0.0};
  c128 rv[KEPT], vv[KEPT];
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      rv[j] = r[base + i];
      vv[j] = v[base + i];
    }
  }
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      const c128 sval = rv[j] - alpha * vv[j];
      sv[base + i] = sval;
      acc[0] += abs2(sval);
    }
  }
  write_partial<1>(acc, k.partials, k.pstride, k.ntile, sys, chunk, chunks);
}

void k_update_s(const KBatch& k, const c128* r, const c128* v, c128* sv, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_update_s, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, r, v, sv);
  check_launch("krylov s");
}

// ---------------------------------------------------------------- x, r update
__global__ void __launch_bounds__(KT) kk_update_xr(KBatch k, c128* x, const c128* y, const c128* z, c128* r,
                                                   const c128* sv, const c128* t, const c128* rhat) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  const int stt = k.status[sys];
  if (stt == ST_HALF) {
    const c128 alpha = k.st[sys].alpha;
    c128 xv[KEPT], yv[KEPT];
#pragma unroll
    for (int j = 0; j < KEPT; ++j) {
      const int64_t i = i0 + (int64_t)j * KT;
      if (i < n) {
        xv[j] = x[base + i];
        yv[j] = y[base + i];
      }
    }
#pragma unroll
    for (int j = 0; j < KEPT; ++j) {
      const int64_t i = i0 + (int64_t)j * KT;
      if (i < n) x[base + i] = xv[j] + alpha * yv[j];
    }
    return;
  }
  if (stt != ST_ACTIVE) return;
  const c128 alpha = k.st[sys].alpha, omega = k.st[sys].omega;
  double acc[3] = {0.0, 0.0, 0.0};
  // two halves of KEPT/2 elements: all loads of a half before its stores
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    constexpr int HE = KEPT / 2;
    c128 xv[HE], yv[HE], zv[HE], sw[HE], tv[HE], hv[HE];
#pragma unroll
    for (int j = 0; j < HE; ++j) {
      const int64_t i = i0 + (int64_t)(h * HE + j) * KT;
      if (i < n) {
        xv[j] = x[base + i];
        yv[j] = y[base + i];
        zv[j] = z[base + i];
        sw[j] = sv[base + i];
        tv[j] = t[base + i];
        hv[j] = rhat[base + i];
      }
    }
#pragma unroll
    for (int j = 0; j < HE; ++j) {
      const int64_t i = i0 + (int64_t)(h * HE + j) * KT;
      if (i < n) {
        x[base + i] = xv[j] + alpha * yv[j] + omega * zv[j];
        const c128 rv = sw[j] - omega * tv[j];
        r[base + i] = rv;
        const c128 d = cdot1(hv[j], rv);
        acc[0] += d.x;
        acc[1] += d.y;
        acc[2] += abs2(rv);
      }
    }
  }
  write_partial<3>(acc, k.partials, k.pstride, k.ntile, sys, chunk, chunks);
}

void k_update_xr(const KBatch& k, c128* x, const c128* y, const c128* z, c128* r, const c128* sv, const c128* t,
                 const c128* rhat, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_update_xr, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, x, y, z, r, sv, t, rhat);
  check_launch("krylov xr");
}

// ---------------------------------------------------------------- fused step end
// The half-step test and omega (FIN_SOMEGA) formed in every workgroup of the
// x, r update from the second product's partials; r's partials go to the
// second buffer (the first is still being read by other workgroups).
// ZS: z and s are one vector (the unpreconditioned steps of the inner
// solves), loaded once.
template <bool ZS>
__global__ void __launch_bounds__(KT) kk_update_xr_fused(KBatch k, c128* x, const c128* y, const c128* z, c128* r,
                                                         const c128* sv, const c128* t, const c128* rhat) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  if (k.status[sys] != ST_ACTIVE) return;
  constexpr int HE = KEPT / 2;
  c128 xv[HE], yv[HE], zv[HE], sw[HE], tv[HE], hv[HE];
  // the loads of the first half are in flight while the partials are summed
  auto load = [&](int h) {
#pragma unroll
    for (int j = 0; j < HE; ++j) {
      const int64_t i = i0 + (int64_t)(h * HE + j) * KT;
      if (i < n) {
        xv[j] = x[base + i];
        yv[j] = y[base + i];
        zv[j] = z[base + i];
        if constexpr (!ZS) sw[j] = sv[base + i];
        tv[j] = t[base + i];
        hv[j] = rhat[base + i];
      }
    }
  };
  load(0);
  double v[4];   // <t, s> (re, im), <t, t>, ||s||^2
  final_sum_all<4>(k.partials, k.pstride, k.ntile, sys, v);
  KState& st = k.st[sys];
  const bool owner = chunk == 0 && threadIdx.x == 0;
  const double snorm = sqrt(v[3]) / st.nb;
  const c128 alpha = st.alpha;
  if (snorm <= st.tol) {   // converged at the half step: x += alpha y
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) load(1);
#pragma unroll
      for (int j = 0; j < HE; ++j) {
        const int64_t i = i0 + (int64_t)(h * HE + j) * KT;
        if (i < n) x[base + i] = xv[j] + alpha * yv[j];
      }
    }
    if (owner) {
      st.snorm = snorm;
      st.pending = ST_HALF;
    }
    return;
  }
  if (v[2] == 0.0) {   // <t, t> = 0: breakdown, x and r stay
    if (owner) {
      st.snorm = snorm;
      st.pending = ST_BREAKDOWN;
    }
    return;
  }
  const c128 omega = mk<double>(v[0] / v[2], v[1] / v[2]);
  if (owner) {
    st.snorm = snorm;
    st.omega = omega;
    st.pending = 0;
  }
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h) load(1);
#pragma unroll
    for (int j = 0; j < HE; ++j) {
      const int64_t i = i0 + (int64_t)(h * HE + j) * KT;
      if (i < n) {
        x[base + i] = xv[j] + alpha * yv[j] + omega * zv[j];
        const c128 rv = (ZS ? zv[j] : sw[j]) - omega * tv[j];
        r[base + i] = rv;
        const c128 d = cdot1(hv[j], rv);
        acc[0] += d.x;
        acc[1] += d.y;
        acc[2] += abs2(rv);
      }
    }
  }
  write_partial_at<3>(acc, k.partials2, k.pstride, sys, chunk);
}

void k_update_xr_fused(const KBatch& k, c128* x, const c128* y, const c128* z, c128* r, const c128* sv,
                       const c128* t, const c128* rhat, hipStream_t s) {
  if (!k.partials2) throw std::runtime_error("fused x, r update: no second partial buffer");
  const int64_t chunks = chunks_of(k.n);
  if (z == sv)
    hipLaunchKernelGGL(kk_update_xr_fused<true>, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, x, y, z, r,
                       sv, t, rhat);
  else
    hipLaunchKernelGGL(kk_update_xr_fused<false>, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, x, y, z, r,
                       sv, t, rhat);
  check_launch("krylov xr (fused)");
}

// One workgroup finishes the step of every system: pending half-step or
// breakdown outcomes, else FIN_XR from the second partial buffer
// (chunks_of(n) partials per system, summed in a fixed order), then the
// number of systems still ACTIVE.  Short partial lists (the block systems):
// one thread per system, all systems at once, the partials loaded eight at a
// time and added in order; long ones (full grids): one wavefront per system,
// the partials split over its lanes.
constexpr int kStepEndThreadChunks = 32;

__device__ __forceinline__ void step_end_one(KBatch& k, int sys, const double* v) {
  KState& st = k.st[sys];
  int status = ST_ACTIVE;
  fin_xr(st, &status, v);
  k.status[sys] = status;
}

__global__ void __launch_bounds__(KT) kk_step_end(KBatch k, int* count_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = KT / 64;
  const int64_t chunks = chunks_of(k.n);
  if (chunks <= kStepEndThreadChunks) {
    for (int sys = threadIdx.x; sys < k.nsys; sys += KT) {
      if (k.status[sys] != ST_ACTIVE) continue;
      KState& st = k.st[sys];
      const int pend = st.pending;
      if (pend != 0) {
        if (pend == ST_HALF) {
          st.rnorm = st.snorm;
          k.status[sys] = ST_CONVERGED;
        } else {
          k.status[sys] = ST_BREAKDOWN;
        }
        st.pending = 0;
        continue;
      }
      const double* p = k.partials2 + sys * k.pstride;
      double v[3] = {0.0, 0.0, 0.0};
      for (int64_t c0 = 0; c0 < chunks; c0 += 8) {
        double q[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (c0 + u < chunks)
#pragma unroll
            for (int e = 0; e < 3; ++e) q[u][e] = p[(c0 + u) * NPART + e];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (c0 + u < chunks)
#pragma unroll
            for (int e = 0; e < 3; ++e) v[e] += q[u][e];
      }
      step_end_one(k, sys, v);
    }
  } else {
  for (int sys = wave; sys < k.nsys; sys += NW) {
    if (k.status[sys] != ST_ACTIVE) continue;   // uniform in the wavefront
    KState& st = k.st[sys];
    const int pend = st.pending;
    if (pend != 0) {
      if (lane == 0) {
        if (pend == ST_HALF) {
          st.rnorm = st.snorm;
          k.status[sys] = ST_CONVERGED;
        } else {
          k.status[sys] = ST_BREAKDOWN;
        }
        st.pending = 0;
      }
      continue;
    }
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t c = lane; c < chunks; c += 64) {
      const double* p = k.partials2 + sys * k.pstride + c * NPART;
      v[0] += p[0];
      v[1] += p[1];
      v[2] += p[2];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double o = __shfl_down(v[q], off, 64);
        if (lane + off < 64) v[q] += o;
      }
    if (lane == 0) step_end_one(k, sys, v);
  }
  }
  if (!count_out) return;
  __syncthreads();
  int act = 0;
  for (int sys = threadIdx.x; sys < k.nsys; sys += KT) act += k.status[sys] == ST_ACTIVE ? 1 : 0;
  __shared__ int cnt[NW];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) act += __shfl_down(act, off, 64);
  if (lane == 0) cnt[wave] = act;
  __syncthreads();
  if (threadIdx.x == 0) {
    int total = 0;
    for (int w = 0; w < NW; ++w) total += cnt[w];
    *count_out = total;
  }
}

void k_step_end(const KBatch& k, int* count_out, hipStream_t s) {
  if (k.nsys <= 0) return;
  if (!k.partials2) throw std::runtime_error("step end: no second partial buffer");
  hipLaunchKernelGGL(kk_step_end, dim3(1), dim3(KT), 0, s, k, count_out);
  check_launch("krylov step end");
}

// ---------------------------------------------------------------- CGS
__global__ void __launch_bounds__(KT) kk_cgs_up(KBatch k, const c128* r, c128* u, const c128* q, c128* p) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  (void)chunk;
  if (k.status[sys] != ST_ACTIVE) return;
  const bool first = k.st[sys].iters == 0;
  const c128 beta = k.st[sys].beta;
  c128 rv[KEPT], qv[KEPT], pv[KEPT];
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      rv[j] = r[base + i];
      if (!first) {
        qv[j] = q[base + i];
        pv[j] = p[base + i];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      if (first) {
        u[base + i] = rv[j];
        p[base + i] = rv[j];
      } else {
        const c128 uv = rv[j] + beta * qv[j];
        u[base + i] = uv;
        p[base + i] = uv + beta * (qv[j] + beta * pv[j]);
      }
    }
  }
}

void cgs_update_up(const KBatch& k, const c128* r, c128* u, const c128* q, c128* p, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_cgs_up, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, r, u, q, p);
  check_launch("cgs u, p");
}

__global__ void __launch_bounds__(KT) kk_cgs_q(KBatch k, const c128* u, const c128* v, c128* q, c128* w) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  (void)chunk;
  if (k.status[sys] != ST_ACTIVE) return;
  const c128 alpha = k.st[sys].alpha;
  c128 uv[KEPT], vv[KEPT];
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      uv[j] = u[base + i];
      vv[j] = v[base + i];
    }
  }
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      const c128 qv = uv[j] - alpha * vv[j];
      q[base + i] = qv;
      w[base + i] = uv[j] + qv;
    }
  }
}

void cgs_update_q(const KBatch& k, const c128* u, const c128* v, c128* q, c128* w, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_cgs_q, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, u, v, q, w);
  check_launch("cgs q");
}

__global__ void __launch_bounds__(KT) kk_cgs_x(KBatch k, c128* x, const c128* uh) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  (void)chunk;
  if (k.status[sys] != ST_ACTIVE) return;
  const c128 alpha = k.st[sys].alpha;
  c128 xv[KEPT], hv[KEPT];
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      xv[j] = x[base + i];
      hv[j] = uh[base + i];
    }
  }
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) x[base + i] = xv[j] + alpha * hv[j];
  }
}

void cgs_update_x(const KBatch& k, c128* x, const c128* uh, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_cgs_x, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, x, uh);
  check_launch("cgs x");
}

__global__ void __launch_bounds__(KT) kk_cgs_r(KBatch k, const c128* b, const c128* t, c128* r, const c128* rhat) {
  const int64_t n = k.n;
  KRYLOV_INDEX
  if (k.status[sys] != ST_ACTIVE) return;
  double acc[3] = {0.0, 0.0, 0.0};
  c128 bv[KEPT], tv[KEPT], hv[KEPT];
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      bv[j] = b[base + i];
      tv[j] = t[base + i];
      hv[j] = rhat[base + i];
    }
  }
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) {
      const c128 rv = bv[j] - tv[j];
      r[base + i] = rv;
      const c128 d = cdot1(hv[j], rv);
      acc[0] += d.x;
      acc[1] += d.y;
      acc[2] += abs2(rv);
    }
  }
  write_partial<3>(acc, k.partials, k.pstride, k.ntile, sys, chunk, chunks);
}

void cgs_update_r(const KBatch& k, const c128* b, const c128* t, c128* r, const c128* rhat, hipStream_t s) {
  const int64_t chunks = chunks_of(k.n);
  hipLaunchKernelGGL(kk_cgs_r, dim3((unsigned)(chunks * k.nsys)), dim3(KT), 0, s, k, b, t, r, rhat);
  check_launch("cgs r");
}

// ---------------------------------------------------------------- bookkeeping
__global__ void __launch_bounds__(KT) kk_record_inner(const int* gate, const KState* st, const int* slots,
                                                      int nslots, int64_t* acc, int32_t* hist, int64_t hist_cap) {
  if (gate && *gate != ST_ACTIVE) return;
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < nslots; j += KT) v[0] += (double)st[slots[j]].iters;
  block_sum<1>(v);
  __shared__ int64_t len;
  if (threadIdx.x == 0) {
    acc[0] += (int64_t)v[0];
    acc[1] += 1;
    len = acc[2];
    acc[2] = len + nslots;
  }
  __syncthreads();
  if (hist && len + nslots <= hist_cap)
    for (int j = threadIdx.x; j < nslots; j += KT) hist[len + j] = st[slots[j]].iters;
}

void record_inner(const int* gate, const KState* st, const int* slots, int nslots, int64_t* acc, int32_t* hist,
                  int64_t hist_cap, hipStream_t s) {
  hipLaunchKernelGGL(kk_record_inner, dim3(1), dim3(KT), 0, s, gate, st, slots, nslots, acc, hist, hist_cap);
  check_launch("record inner");
}

// ---------------------------------------------------------------- helpers
__global__ void __launch_bounds__(KT) kk_count_active(const int* status, int n, int* out) {
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += KT) v[0] += status[i] == ST_ACTIVE ? 1.0 : 0.0;
  block_sum<1>(v);
  if (threadIdx.x == 0) *out = (int)v[0];
}

void count_active(const int* status, int n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(kk_count_active, dim3(1), dim3(KT), 0, s, status, n, out);
  check_launch("count active");
}

__global__ void kk_total_field(const c128* P, const c128* chi, c128* e, int64_t nv, int ncomp, int64_t cper) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * ncomp) return;
  const c128 ci = chi[i % cper];
  e[i] = (ci.x == 0.0 && ci.y == 0.0) ? mk<double>(0.0, 0.0) : P[i] * ci;
}

void total_field(const c128* P, const c128* chi_inv, c128* e, int64_t nv, int ncomp, hipStream_t s, int64_t cper) {
  const int64_t n = nv * ncomp;
  if (cper <= 0) cper = nv;
  hipLaunchKernelGGL(kk_total_field, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, chi_inv, e, nv, ncomp,
                     cper);
  check_launch("total field");
}

__global__ void kk_masked_copy(const c128* e, const c128* chi, c128* b, int64_t nv, int64_t cper) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nv) return;
  const c128 ci = chi[i % cper];
  b[i] = (ci.x == 0.0 && ci.y == 0.0) ? mk<double>(0.0, 0.0) : e[i];
}

__global__ void kk_zero_outer_faces(c128* e, int nx, int ny, int nz) {
  const int64_t nv = (int64_t)nx * ny * nz;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
  if (x == nx - 1) e[v] = mk<double>(0.0, 0.0);
  if (y == ny - 1) e[nv + v] = mk<double>(0.0, 0.0);
  if (z == nz - 1) e[2 * nv + v] = mk<double>(0.0, 0.0);
}

void zero_outer_faces(c128* e, int nx, int ny, int nz, hipStream_t s) {
  const int64_t nv = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(kk_zero_outer_faces, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, e, nx, ny, nz);
  check_launch("zero outer faces");
}

void masked_copy(const c128* e, const c128* chi_inv, c128* b, int64_t nv, hipStream_t s, int64_t cper) {
  if (cper <= 0) cper = nv;
  hipLaunchKernelGGL(kk_masked_copy, dim3((unsigned)((3 * nv + 255) / 256)), dim3(256), 0, s, e, chi_inv, b, nv,
                     cper);
  check_launch("masked copy");
}

__global__ void kk_sub(const c128* b, const c128* a, c128* r, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - a[i];
}
void sub_vec(const c128* b, const c128* a, c128* r, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(kk_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b, a, r, n);
  check_launch("sub");
}

// dst[(c nrhs + r) nv + i] = src[(3 r + c) nv + i], zero for stopped systems
__global__ void kk_batch_to_stacked(const c128* src, c128* dst, int nrhs, int64_t nv, const int* status) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = 3 * (int64_t)nrhs * nv;
  if (j >= total) return;
  const int64_t c = j / ((int64_t)nrhs * nv);
  const int64_t rem = j - c * nrhs * nv;
  const int64_t r = rem / nv, i = rem - r * nv;
  const bool live = status == nullptr || status[r] == ST_ACTIVE;
  dst[j] = live ? src[(3 * r + c) * nv + i] : mk<double>(0.0, 0.0);
}

__global__ void kk_stacked_to_batch(const c128* src, c128* dst, int nrhs, int64_t nv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // batch index
  const int64_t total = 3 * (int64_t)nrhs * nv;
  if (j >= total) return;
  const int64_t r = j / (3 * nv);
  const int64_t rem = j - r * 3 * nv;
  const int64_t c = rem / nv, i = rem - c * nv;
  dst[j] = src[(c * nrhs + r) * nv + i];
}

void batch_to_stacked(const c128* src, c128* dst, int nrhs, int64_t nv, const int* status, hipStream_t s) {
  const int64_t total = 3 * (int64_t)nrhs * nv;
  hipLaunchKernelGGL(kk_batch_to_stacked, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, nrhs, nv,
                     status);
  check_launch("batch to stacked");
}

void stacked_to_batch(const c128* src, c128* dst, int nrhs, int64_t nv, hipStream_t s) {
  const int64_t total = 3 * (int64_t)nrhs * nv;
  hipLaunchKernelGGL(kk_stacked_to_batch, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, nrhs, nv);
  check_launch("stacked to batch");
}

__global__ void kk_add(c128* x, const c128* d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] + d[i];
}
void add_vec(c128* x, const c128* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(kk_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, d, n);
  check_launch("add");
}

// ||v||^2 of one vector: partials, then one workgroup sums them in order
__global__ void __launch_bounds__(KT) kk_norm2(int64_t n, const c128* v, double* partials) {
  KRYLOV_INDEX
  double acc[1] = {0.0};
#pragma unroll
  for (int j = 0; j < KEPT; ++j) {
    const int64_t i = i0 + (int64_t)j * KT;
    if (i < n) acc[0] += abs2(v[base + i]);
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) partials[chunk * NPART] = acc[0];
}

__global__ void __launch_bounds__(KT) kk_norm2_fin(int64_t n, const double* partials, double* out) {
  const int64_t chunks = chunks_of(n);
  double v[1] = {0.0};
  for (int64_t c = threadIdx.x; c < chunks; c += KT) v[0] += partials[c * NPART];
  block_sum<1>(v);
  if (threadIdx.x == 0) *out = v[0];
}

void norm2(const c128* v, int64_t n, double* partials, double* out, hipStream_t s) {
  const int64_t chunks = chunks_of(n);
  hipLaunchKernelGGL(kk_norm2, dim3((unsigned)chunks), dim3(KT), 0, s, n, v, partials);
  hipLaunchKernelGGL(kk_norm2_fin, dim3(1), dim3(KT), 0, s, n, partials, out);
  check_launch("norm2");
}

// ---------------------------------------------------------------- blocks
__device__ __forceinline__ int64_t block_local(const BlockMap& m, int k, int x, int y, int z, int* g, int* sysi,
                                               int64_t* bnv) {
  *g = m.block_group[k];
  *sysi = m.block_sys[k];
  const int4 o = m.block_origin[k];
  const int4 b = m.gbox[*g];
  *bnv = (int64_t)b.x * b.y * b.z;
  return ((int64_t)(z - o.z) * b.y + (y - o.y)) * b.x + (x - o.x);
}

__global__ void kk_gather(BlockMap m, const c128* w, c128* const* gdst) {
  const int64_t nv = (int64_t)m.nx * m.ny * m.nz;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int x = (int)(v % m.nx), y = (int)((v / m.nx) % m.ny), z = (int)(v / ((int64_t)m.nx * m.ny));
  if (m.faces) {   // each component to the block owning its face
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = m.block_id[c * nv + v];
      if (k < 0) continue;
      int g, sysi;
      int64_t bnv;
      const int64_t loc = block_local(m, k, x, y, z, &g, &sysi, &bnv);
      gdst[g][(int64_t)sysi * 3 * bnv + c * bnv + loc] = w[c * nv + v];
    }
    return;
  }
  const int k = m.block_id[v];
  if (k < 0) return;
  int g, sysi;
  int64_t bnv;
  const int64_t loc = block_local(m, k, x, y, z, &g, &sysi, &bnv);
  c128* dst = gdst[g] + (int64_t)sysi * 3 * bnv + loc;
#pragma unroll
  for (int c = 0; c < 3; ++c) dst[c * bnv] = w[c * nv + v];
}

void block_gather(const BlockMap& m, const c128* w, c128* const* gdst, hipStream_t s) {
  const int64_t nv = (int64_t)m.nx * m.ny * m.nz;
  hipLaunchKernelGGL(kk_gather, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, m, w, gdst);
  check_launch("gather");
}

__global__ void kk_scatter(BlockMap m, c128* const* gsrc, c128* y) {
  const int64_t nv = (int64_t)m.nx * m.ny * m.nz;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  if (m.faces) {
    const int x = (int)(v % m.nx), yy = (int)((v / m.nx) % m.ny), z = (int)(v / ((int64_t)m.nx * m.ny));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = m.block_id[c * nv + v];
      c128 val = mk<double>(0.0, 0.0);
      if (k >= 0) {
        int g, sysi;
        int64_t bnv;
        const int64_t loc = block_local(m, k, x, yy, z, &g, &sysi, &bnv);
        val = gsrc[g][(int64_t)sysi * 3 * bnv + c * bnv + loc];
      }
      y[c * nv + v] = val;
    }
    return;
  }
  const int k = m.block_id[v];
  if (k < 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c * nv + v] = mk<double>(0.0, 0.0);
    return;
  }
  const int x = (int)(v % m.nx), yy = (int)((v / m.nx) % m.ny), z = (int)(v / ((int64_t)m.nx * m.ny));
  int g, sysi;
  int64_t bnv;
  const int64_t loc = block_local(m, k, x, yy, z, &g, &sysi, &bnv);
  const c128* src = gsrc[g] + (int64_t)sysi * 3 * bnv + loc;
#pragma unroll
  for (int c = 0; c < 3; ++c) y[c * nv + v] = src[c * bnv];
}

__global__ void kk_gather_sets(const c128* w, int nx, int ny, int nz, int bx, int by, int bz, int nsys,
                               const int4* origin, const c128* chi, c128* gdst) {
  const int64_t bnv = (int64_t)bx * by * bz;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)nsys * bnv) return;
  const c128 ci = chi[j];
  if (ci.x == 0.0 && ci.y == 0.0) return;   // not in the set (stays zero)
  const int64_t q = j / bnv, pos = j - q * bnv;
  const int x = (int)(pos % bx), y = (int)((pos / bx) % by), z = (int)(pos / ((int64_t)bx * by));
  const int4 o = origin[q];
  const int X = o.x + x, Y = o.y + y, Z = o.z + z;
  if (X >= nx || Y >= ny || Z >= nz) return;
  const int64_t nv = (int64_t)nx * ny * nz;
  const int64_t v = ((int64_t)Z * ny + Y) * nx + X;
  c128* dst = gdst + q * 3 * bnv + pos;
#pragma unroll
  for (int c = 0; c < 3; ++c) dst[c * bnv] = w[c * nv + v];
}

void gather_sets(const c128* w, int nx, int ny, int nz, int bx, int by, int bz, int nsys, const int4* origin,
                 const c128* chi, c128* gdst, hipStream_t s) {
  const int64_t total = (int64_t)nsys * bx * by * bz;
  if (total == 0) return;
  hipLaunchKernelGGL(kk_gather_sets, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, w, nx, ny, nz, bx, by,
                     bz, nsys, origin, chi, gdst);
  check_launch("gather sets");
}

void block_scatter(const BlockMap& m, c128* const* gsrc, c128* y, hipStream_t s) {
  const int64_t nv = (int64_t)m.nx * m.ny * m.nz;
  hipLaunchKernelGGL(kk_scatter, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, m, gsrc, y);
  check_launch("scatter");
}

}  // namespace vie
