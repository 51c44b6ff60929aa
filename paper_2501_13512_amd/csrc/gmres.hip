// Flexible GMRES(m) for the outer solve (a solver variant next to the
// paper's BiCGSTAB of Sec. II-B): right preconditioned with the block
// preconditioner of eq. (10), whose inner iterative solves make it change
// from step to step, so the preconditioned vectors z_j are kept (Saad's
// flexible form).  The Arnoldi vector of each step is orthogonalised by
// classical Gram-Schmidt applied twice (two passes of batched inner products
// and one batched update each, instead of j + 1 dependent dot products);
// the Hessenberg column, the Givens rotations and the residual estimate are
// updated on the device by one thread, which also sets the solve's status,
// so steps the host enqueues past the end are skipped.  Reductions are
// per-workgroup partials summed in a fixed order (deterministic).
#include <stdexcept>
#include <string>

#include "krylov_dev.h"

namespace vie {

constexpr int GT = 256;               // threads per workgroup
constexpr int GEPT = 8;               // elements per thread
constexpr int GCH = GT * GEPT;        // elements per chunk
constexpr int GDOT = 8;               // inner products per multi-dot launch

int64_t gmres_chunks(int64_t n) { return (n + GCH - 1) / GCH; }

static void check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

__device__ __forceinline__ c128 hcol(const GmresDev& d, int i, int j) { return d.H[(int64_t)j * (d.m + 1) + i]; }
__device__ __forceinline__ void hset(const GmresDev& d, int i, int j, c128 v) { d.H[(int64_t)j * (d.m + 1) + i] = v; }

// part[(i * nchunk + chunk) * 2 + {re, im}] = chunk's part of <V_i, w>, i in [i0, i0 + cnt)
__global__ void __launch_bounds__(GT) kg_mdot(GmresDev d, const c128* w, int i0, int cnt) {
  if (*d.status != ST_ACTIVE) return;
  const int64_t chunk = blockIdx.x;
  double acc[2 * GDOT];
#pragma unroll
  for (int q = 0; q < 2 * GDOT; ++q) acc[q] = 0.0;
#pragma unroll
  for (int e = 0; e < GEPT; ++e) {
    const int64_t i = chunk * GCH + (int64_t)e * GT + threadIdx.x;
    if (i >= d.n) break;
    const c128 wv = w[i];
#pragma unroll
    for (int q = 0; q < GDOT; ++q)
      if (q < cnt) {
        const c128 t = cdot1(d.V[(int64_t)(i0 + q) * d.n + i], wv);
        acc[2 * q] += t.x;
        acc[2 * q + 1] += t.y;
      }
  }
  block_sum<2 * GDOT>(acc);
  if (threadIdx.x == 0)
    for (int q = 0; q < cnt; ++q) {
      double* p = d.part + ((int64_t)(i0 + q) * d.nchunk + chunk) * 2;
      p[0] = acc[2 * q];
      p[1] = acc[2 * q + 1];
    }
}

// c[i] = sum over chunks (fixed order); h[i] = c[i] (first pass) or h[i] + c[i]
__global__ void __launch_bounds__(GT) kg_mdot_fin(GmresDev d, int accumulate) {
  if (*d.status != ST_ACTIVE) return;
  const int i = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int64_t c = threadIdx.x; c < d.nchunk; c += GT) {
    const double* p = d.part + ((int64_t)i * d.nchunk + c) * 2;
    v[0] += p[0];
    v[1] += p[1];
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    const c128 val = mk<double>(v[0], v[1]);
    d.c[i] = val;
    d.h[i] = accumulate ? d.h[i] + val : val;
  }
}

// w -= sum_{i < cnt} c_i V_i
__global__ void __launch_bounds__(GT) kg_maxpy(GmresDev d, c128* w, int cnt) {
  if (*d.status != ST_ACTIVE) return;
  const int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (i >= d.n) return;
  c128 acc = w[i];
  for (int q = 0; q < cnt; ++q) acc = acc - d.c[q] * d.V[(int64_t)q * d.n + i];
  w[i] = acc;
}

// Column j of the Hessenberg matrix from h and ||w|| (scal[0] = ||w||^2),
// earlier rotations, a new rotation, the residual estimate and the status.
__global__ void kg_arnoldi(GmresDev d, int j) {
  if (threadIdx.x != 0 || *d.status != ST_ACTIVE) return;
  GmresState& s = *d.st;
  const double hn = sqrt(d.scal[0]);
  for (int i = 0; i <= j; ++i) hset(d, i, j, d.h[i]);
  hset(d, j + 1, j, mk<double>(hn, 0.0));
  for (int i = 0; i < j; ++i) {
    const c128 a0 = hcol(d, i, j), a1 = hcol(d, i + 1, j);
    const double c = d.cs[i];
    const c128 sn = d.sn[i];
    hset(d, i, j, c * a0 + sn * a1);
    hset(d, i + 1, j, c * a1 - conj(sn) * a0);
  }
  // rotation zeroing H[j+1, j] (real, >= 0)
  const c128 a = hcol(d, j, j);
  const double b = hn;
  double c;
  c128 sn;
  const double aa = sqrt(abs2(a));
  if (b == 0.0) {
    c = 1.0;
    sn = mk<double>(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    sn = mk<double>(1.0, 0.0);
  } else {
    const double dd = hypot(aa, b);
    c = aa / dd;
    sn = mk<double>(a.x / aa * b / dd, a.y / aa * b / dd);   // (a / |a|) conj(b) / d, b real
  }
  d.cs[j] = c;
  d.sn[j] = sn;
  hset(d, j, j, c * a + sn * mk<double>(b, 0.0));
  hset(d, j + 1, j, mk<double>(0.0, 0.0));
  const c128 gj = d.g[j];
  d.g[j + 1] = mk<double>(0.0, 0.0) - conj(sn) * gj;
  d.g[j] = c * gj;
  s.iters += 1;
  s.k = j + 1;
  s.hnext = hn;
  const double res = sqrt(abs2(d.g[j + 1])) / s.nb;
  s.relres = res;
  int st = ST_ACTIVE;
  if (res <= s.tol)
    st = ST_CONVERGED;
  else if (!(res == res))
    st = ST_BREAKDOWN;
  else if (s.iters >= s.maxit)
    st = ST_MAXIT;
  else if (hn == 0.0 || j + 1 == d.m)
    st = ST_RESTART;   // cycle full, or an invariant subspace: update x and restart from b - A x
  *d.status = st;
}

// v *= 1 / hnext while the solve goes on (the next Arnoldi vector)
__global__ void __launch_bounds__(GT) kg_scale(GmresDev d, c128* v) {
  if (*d.status != ST_ACTIVE) return;
  const int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (i >= d.n) return;
  const double f = 1.0 / d.st->hnext;
  v[i] = f * v[i];
}

// (Re)start from scal[0] = ||r||^2: g = (beta, 0, ...), status.  The first
// start also sets ||b||, the tolerance and the step cap.
__global__ void kg_start(GmresDev d, int first, double tol, int maxit) {
  if (threadIdx.x != 0) return;
  GmresState& s = *d.st;
  const double beta = sqrt(d.scal[0]);
  if (first) {
    s.nb = beta;
    s.iters = 0;
    s.tol = tol;
    s.maxit = maxit;
  }
  for (int i = 0; i <= d.m; ++i) d.g[i] = mk<double>(0.0, 0.0);
  d.g[0] = mk<double>(beta, 0.0);
  s.k = 0;
  s.hnext = beta;
  s.relres = s.nb > 0.0 ? beta / s.nb : 0.0;
  int st = ST_ACTIVE;
  if (s.nb == 0.0 || s.relres <= s.tol)
    st = ST_CONVERGED;
  else if (s.iters >= s.maxit)
    st = ST_MAXIT;
  *d.status = st;
}

// y = H[:k, :k]^{-1} g[:k] (back substitution, k = columns of this cycle).
// A zero pivot (the flexible Arnoldi relation turned singular: a
// preconditioned direction added nothing new) drops that direction and marks
// the solve as broken down.
__global__ void kg_solve_y(GmresDev d) {
  if (threadIdx.x != 0) return;
  const int k = d.st->k;
  for (int i = k - 1; i >= 0; --i) {
    c128 acc = d.g[i];
    for (int q = i + 1; q < k; ++q) acc = acc - hcol(d, i, q) * d.y[q];
    const c128 piv = hcol(d, i, i);
    if (piv.x == 0.0 && piv.y == 0.0) {
      d.y[i] = mk<double>(0.0, 0.0);
      *d.status = ST_BREAKDOWN;
    } else {
      d.y[i] = cdiv(acc, piv);
    }
  }
}

// x += sum_{i < k} y_i B_i  (B = Z with a preconditioner, V without)
__global__ void __launch_bounds__(GT) kg_update_x(GmresDev d, c128* x, const c128* B) {
  const int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (i >= d.n) return;
  const int k = d.st->k;
  c128 acc = x[i];
  for (int q = 0; q < k; ++q) acc = acc + d.y[q] * B[(int64_t)q * d.n + i];
  x[i] = acc;
}

static unsigned blocks_of(int64_t n) { return (unsigned)((n + GT - 1) / GT); }

void gmres_orthogonalise(const GmresDev& d, c128* w, int j, hipStream_t s) {
  for (int pass = 0; pass < 2; ++pass) {
    for (int i0 = 0; i0 <= j; i0 += GDOT) {
      const int cnt = (j + 1 - i0) < GDOT ? (j + 1 - i0) : GDOT;
      hipLaunchKernelGGL(kg_mdot, dim3((unsigned)d.nchunk), dim3(GT), 0, s, d, (const c128*)w, i0, cnt);
    }
    hipLaunchKernelGGL(kg_mdot_fin, dim3(j + 1), dim3(GT), 0, s, d, pass);
    hipLaunchKernelGGL(kg_maxpy, dim3(blocks_of(d.n)), dim3(GT), 0, s, d, w, j + 1);
  }
  check("gmres orthogonalise");
}

void gmres_arnoldi(const GmresDev& d, c128* w, int j, hipStream_t s) {
  hipLaunchKernelGGL(kg_arnoldi, dim3(1), dim3(64), 0, s, d, j);
  hipLaunchKernelGGL(kg_scale, dim3(blocks_of(d.n)), dim3(GT), 0, s, d, w);
  check("gmres arnoldi");
}

void gmres_start(const GmresDev& d, c128* v0, bool first, double tol, int maxit, hipStream_t s) {
  hipLaunchKernelGGL(kg_start, dim3(1), dim3(64), 0, s, d, first ? 1 : 0, tol, maxit);
  hipLaunchKernelGGL(kg_scale, dim3(blocks_of(d.n)), dim3(GT), 0, s, d, v0);
  check("gmres start");
}

void gmres_update(const GmresDev& d, c128* x, const c128* B, hipStream_t s) {
  hipLaunchKernelGGL(kg_solve_y, dim3(1), dim3(64), 0, s, d);
  hipLaunchKernelGGL(kg_update_x, dim3(blocks_of(d.n)), dim3(GT), 0, s, d, x, B);
  check("gmres update");
}

}  // namespace vie
