// Inner block solves (Sec. II-B, eqs. (10)-(11)) with one workgroup per block.
//
// The paper solves every block of the block-diagonal preconditioner
// independently (one OpenMP thread per block).  Here a workgroup runs the
// whole unpreconditioned BiCGSTAB of one block — the FFT product on the
// block's box (the same five passes as the full-grid product, each a loop
// over the box's pencils), the vector updates and the inner products — with
// workgroup barriers only: no kernel launches, no device-wide
// synchronisation, one launch per preconditioner application for all small
// blocks.  Global memory written by one pass is read by the next after a
// barrier; all waves of a workgroup share one CU's vector cache, so a
// workgroup-scope fence (part of the barrier) makes the writes visible.
//
// The FFT lengths of the box are template parameters (LX = LY for the x and
// y axes, LZ); blocks whose lengths have no instantiation use the batched
// multi-workgroup kernels instead.
#include <stdexcept>
#include <string>

#include "fft_core.h"
#include "krylov_dev.h"

namespace vie {

constexpr int BT = 512;   // threads per block-solver workgroup

constexpr int cmin_i(int a, int b) { return a < b ? a : b; }

// Pencils transformed at once by the row and column passes: every thread
// busy, at most 4096 elements of LDS.
template <int L>
constexpr int wg_pencils() {
  constexpr int T = PlanInfo<L>::max_butterflies;
  return cmin_i(BT / T, 4096 / L);
}

template <typename R>
__device__ __forceinline__ cx<R> zero_c() {
  return mk<R>(R(0), R(0));
}

// Sum over the workgroup, result broadcast to every thread.
template <int NV>
__device__ __forceinline__ void wg_allsum(double (&v)[NV]) {
  __shared__ double bc[NV];
  block_sum<NV>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) bc[k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = bc[k];
  __syncthreads();
}

// ---------------------------------------------------------------- passes
// Contiguous pencils (rows): pencil i of `count`, elements along memory.
template <typename R, int L, int DIR, class Load, class Store>
__device__ __forceinline__ void wg_rows(int count, Load ld, Store st, cx<R>* lds, const cx<R>* tw) {
  constexpr int T = PlanInfo<L>::max_butterflies;
  constexpr int PP = wg_pencils<L>();
  static_assert(PP >= 1, "pencil too long");
  const int p = threadIdx.x / T, t = threadIdx.x - p * T;
  for (int c0 = 0; c0 < count; c0 += PP) {
    const int i = c0 + p;
    const bool valid = p < PP && i < count;
    const int ii = valid ? i : 0;
    auto l = [&](int n) -> cx<R> { return ld(ii, n); };
    auto s = [&](int k, cx<R> v) { st(ii, k, v); };
    fft_pencil<R, L, T, DIR>(l, s, lds + (p < PP ? p : 0) * L, 1, t, valid, tw);
    __syncthreads();
  }
}

// Strided pencils (columns): column i of `count`; LDS [L][PP] for adjacent
// columns in adjacent threads.
template <typename R, int L, int DIR, class Load, class Store>
__device__ __forceinline__ void wg_cols(int count, Load ld, Store st, cx<R>* lds, const cx<R>* tw) {
  constexpr int T = PlanInfo<L>::max_butterflies;
  constexpr int PP = wg_pencils<L>();
  const int p = threadIdx.x % PP, t = threadIdx.x / PP;
  for (int c0 = 0; c0 < count; c0 += PP) {
    const int i = c0 + p;
    const bool valid = t < T && i < count;
    const int ii = valid ? i : 0;
    auto l = [&](int n) -> cx<R> { return ld(ii, n); };
    auto s = [&](int k, cx<R> v) { st(ii, k, v); };
    fft_pencil<R, L, T, DIR>(l, s, lds + p, PP, t, valid, tw);
    __syncthreads();
  }
}

// y = A x on one block's box: pruned x, y forward; z forward + spectral
// multiply + z inverse; y, x inverse + crop + local term (the full-grid
// product's arithmetic, in one workgroup).
template <typename R, int LX, int LZ>
__device__ void wg_matvec(const BlockSolveArgs& a, int sys, const c128* xin, c128* yout, cx<R>* lds) {
  constexpr int LY = LX;
  const int bx = a.bx, by = a.by, bz = a.bz;
  const int64_t bnv = (int64_t)bx * by * bz;
  cx<R>* w = (cx<R>*)a.work + (int64_t)sys * 3 * bz * LY * LX;
  const c128* chi = a.chi + sys * bnv;
  const cx<R>* twx = (const cx<R>*)a.twx;
  const cx<R>* twz = (const cx<R>*)a.twz;
  // pass 1: rows (c, z, y) of bx voxels -> LX
  wg_rows<R, LX, -1>(
      3 * bz * by, [&](int i, int n) -> cx<R> { return n < bx ? cvt<R>(xin[(int64_t)i * bx + n]) : zero_c<R>(); },
      [&](int i, int k, cx<R> v) {
        const int cz = i / by, y = i - cz * by;
        w[((int64_t)cz * LY + y) * LX + k] = v;
      },
      lds, twx);
  // pass 2: columns (c, z, x) along y: by -> LY
  wg_cols<R, LY, -1>(
      3 * bz * LX,
      [&](int i, int n) -> cx<R> {
        const int cz = i / LX, xq = i - cz * LX;
        return n < by ? w[((int64_t)cz * LY + n) * LX + xq] : zero_c<R>();
      },
      [&](int i, int k, cx<R> v) {
        const int cz = i / LX, xq = i - cz * LX;
        w[((int64_t)cz * LY + k) * LX + xq] = v;
      },
      lds, twx);
  // pass 3: columns (qy, qx) along z for the three components, multiply
  {
    constexpr int T = PlanInfo<LZ>::max_butterflies;
    constexpr int ZP = cmin_i(BT / (3 * T), 64);
    const int comp = threadIdx.x / (T * ZP);
    const int rem = threadIdx.x - comp * (T * ZP);
    const int p = rem % ZP, t = rem / ZP;
    const int64_t plane = (int64_t)LY * LX;
    const int cols = LY * LX;
    const cx<R>* spec = (const cx<R>*)a.spec;
    constexpr int HX = LX / 2, HY = LY / 2, HZ = LZ / 2;
    constexpr int64_t OX = HX + 1, OY = HY + 1;
    constexpr int64_t OCT = OX * OY * (HZ + 1);
    for (int c0 = 0; c0 < cols; c0 += ZP) {
      const int col = c0 + p;
      const bool valid = comp < 3 && col < cols;
      const int cc = valid ? col : 0;
      const int ccomp = comp < 3 ? comp : 0;
      cx<R>* base = w + (int64_t)ccomp * bz * plane + cc;
      cx<R>* slot = lds + ccomp * LZ * ZP + p;
      auto ldg = [&](int n) -> cx<R> { return n < bz ? base[n * plane] : zero_c<R>(); };
      auto sts = [&](int k, cx<R> v) { slot[k * ZP] = v; };
      fft_pencil<R, LZ, T, -1, false, true>(ldg, sts, slot, ZP, t, valid, twz);
      for (int i = threadIdx.x; i < LZ * ZP; i += BT) {
        const int qz = i / ZP, pp = i - qz * ZP;
        const int c2 = c0 + pp;
        if (c2 >= cols) continue;
        const int qy = c2 / LX, qx = c2 - qy * LX;
        const int fx = qx <= HX ? qx : LX - qx, fy = qy <= HY ? qy : LY - qy, fz = qz <= HZ ? qz : LZ - qz;
        const R sx = qx <= HX ? R(1) : R(-1), sy = qy <= HY ? R(1) : R(-1), sz = qz <= HZ ? R(1) : R(-1);
        const int64_t o = ((int64_t)fz * OY + fy) * OX + fx;
        const cx<R> sxx = spec[o], syy = spec[3 * OCT + o], szz = spec[5 * OCT + o];
        const cx<R> sxy = (sx * sy) * spec[OCT + o];
        const cx<R> sxz = (sx * sz) * spec[2 * OCT + o];
        const cx<R> syz = (sy * sz) * spec[4 * OCT + o];
        const int e = qz * ZP + pp;
        const cx<R> X = lds[e], Y = lds[LZ * ZP + e], Z = lds[2 * LZ * ZP + e];
        lds[e] = sxx * X + sxy * Y + sxz * Z;
        lds[LZ * ZP + e] = sxy * X + syy * Y + syz * Z;
        lds[2 * LZ * ZP + e] = sxz * X + syz * Y + szz * Z;
      }
      __syncthreads();
      auto lds_ld = [&](int n) -> cx<R> { return slot[n * ZP]; };
      auto stg = [&](int k, cx<R> v) {
        if (k < bz) base[k * plane] = v;
      };
      fft_pencil<R, LZ, T, +1, true, false>(lds_ld, stg, slot, ZP, t, valid, twz);
      __syncthreads();
    }
  }
  // pass 4: columns along y, inverse: LY -> by
  wg_cols<R, LY, +1>(
      3 * bz * LX,
      [&](int i, int n) -> cx<R> {
        const int cz = i / LX, xq = i - cz * LX;
        return w[((int64_t)cz * LY + n) * LX + xq];
      },
      [&](int i, int k, cx<R> v) {
        if (k < by) {
          const int cz = i / LX, xq = i - cz * LX;
          w[((int64_t)cz * LY + k) * LX + xq] = v;
        }
      },
      lds, twx);
  // pass 5: rows along x, inverse, crop, scale, local term, mask
  const double scale = 1.0 / ((double)LX * LY * LZ);
  wg_rows<R, LX, +1>(
      3 * bz * by,
      [&](int i, int n) -> cx<R> {
        const int cz = i / by, y = i - cz * by;
        return w[((int64_t)cz * LY + y) * LX + n];
      },
      [&](int i, int k, cx<R> v) {
        if (k < bx) {
          const int64_t e = (int64_t)i * bx + k;
          const int64_t vox = e % bnv;
          const c128 ci = chi[vox];
          c128 out = mk<double>(0.0, 0.0);
          if (ci.x != 0.0 || ci.y != 0.0) out = xin[e] * ci - scale * cvt<double>(v);
          yout[e] = out;
        }
      },
      lds, twx);
}

template <typename R, int LX, int LZ>
__global__ void __launch_bounds__(BT) k_block_solve(BlockSolveArgs a) {
  constexpr int ES = (int)sizeof(cx<R>);
  constexpr int TZ = PlanInfo<LZ>::max_butterflies;
  constexpr int ZP = cmin_i(BT / (3 * TZ), 64);
  constexpr int LDS_XY = wg_pencils<LX>() * LX;
  constexpr int LDS_Z = 3 * LZ * ZP;
  constexpr int LDS_N = LDS_XY > LDS_Z ? LDS_XY : LDS_Z;
  static_assert(LDS_N * ES <= 96 * 1024, "block solver LDS too large");
  __shared__ cx<R> lds[LDS_N];
  const int sys = blockIdx.x;
  const int64_t n = a.n;
  const int64_t o = (int64_t)sys * n;
  c128 *x = a.x + o, *r = a.r + o, *rh = a.rhat + o, *p = a.p + o, *v = a.v + o, *s = a.s + o, *t = a.t + o;
  const c128* b = a.b + o;
  KState& ks = a.st[sys];
  if (a.gate && *a.gate != ST_ACTIVE) {
    if (threadIdx.x == 0) a.status[sys] = ST_IDLE;
    return;
  }
  // x = 0, r = rhat = b, ||b||
  double acc1[1] = {0.0};
  for (int64_t i = threadIdx.x; i < n; i += BT) {
    const c128 bv = b[i];
    x[i] = mk<double>(0.0, 0.0);
    r[i] = bv;
    rh[i] = bv;
    acc1[0] += abs2(bv);
  }
  wg_allsum<1>(acc1);
  const double nb = sqrt(acc1[0]);
  c128 rho = mk<double>(acc1[0], 0.0), alpha = mk<double>(1.0, 0.0), omega = mk<double>(1.0, 0.0);
  c128 beta = mk<double>(0.0, 0.0);
  int status = nb > 0.0 ? (a.maxit > 0 ? ST_ACTIVE : ST_MAXIT) : ST_CONVERGED;
  int it = 0;
  double rnorm = nb > 0.0 ? 1.0 : 0.0;
  while (status == ST_ACTIVE) {
    // p = r + beta (p - omega v)   (p = r on the first step)
    for (int64_t i = threadIdx.x; i < n; i += BT) p[i] = it == 0 ? r[i] : r[i] + beta * (p[i] - omega * v[i]);
    __syncthreads();
    wg_matvec<R, LX, LZ>(a, sys, p, v, lds);
    __syncthreads();
    double d2[2] = {0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += BT) {
      const c128 d = cdot1(rh[i], v[i]);
      d2[0] += d.x;
      d2[1] += d.y;
    }
    wg_allsum<2>(d2);
    ++it;
    if (d2[0] == 0.0 && d2[1] == 0.0) {
      status = ST_BREAKDOWN;
      break;
    }
    alpha = cdiv(rho, mk<double>(d2[0], d2[1]));
    double s2[1] = {0.0};
    for (int64_t i = threadIdx.x; i < n; i += BT) {
      const c128 sv = r[i] - alpha * v[i];
      s[i] = sv;
      s2[0] += abs2(sv);
    }
    wg_allsum<1>(s2);
    const double snorm = sqrt(s2[0]) / nb;
    if (snorm <= a.tol) {
      for (int64_t i = threadIdx.x; i < n; i += BT) x[i] = x[i] + alpha * p[i];
      rnorm = snorm;
      status = ST_CONVERGED;
      break;
    }
    wg_matvec<R, LX, LZ>(a, sys, s, t, lds);
    __syncthreads();
    double d3[3] = {0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += BT) {
      const c128 tv = t[i];
      const c128 d = cdot1(tv, s[i]);
      d3[0] += d.x;
      d3[1] += d.y;
      d3[2] += abs2(tv);
    }
    wg_allsum<3>(d3);
    if (d3[2] == 0.0) {
      status = ST_BREAKDOWN;
      break;
    }
    omega = mk<double>(d3[0] / d3[2], d3[1] / d3[2]);
    double q3[3] = {0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += BT) {
      x[i] = x[i] + alpha * p[i] + omega * s[i];
      const c128 rv = s[i] - omega * t[i];
      r[i] = rv;
      const c128 d = cdot1(rh[i], rv);
      q3[0] += d.x;
      q3[1] += d.y;
      q3[2] += abs2(rv);
    }
    wg_allsum<3>(q3);
    const c128 rho_new = mk<double>(q3[0], q3[1]);
    rnorm = sqrt(q3[2]) / nb;
    const bool om0 = omega.x == 0.0 && omega.y == 0.0;
    const bool rho0 = rho_new.x == 0.0 && rho_new.y == 0.0;
    if (rnorm <= a.tol) {
      status = ST_CONVERGED;
    } else if (om0 || rho0 || !(rnorm == rnorm)) {
      status = ST_BREAKDOWN;
    } else if (it >= a.maxit) {
      status = ST_MAXIT;
    } else {
      beta = cdiv(rho_new, rho) * cdiv(alpha, omega);
    }
    rho = rho_new;
  }
  if (threadIdx.x == 0) {
    ks.nb = nb;
    ks.iters = it;
    ks.rnorm = rnorm;
    ks.tol = a.tol;
    ks.maxit = a.maxit;
    ks.rho = rho;
    ks.alpha = alpha;
    ks.omega = omega;
    a.status[sys] = status;
  }
}

// ---------------------------------------------------------------- dispatch
// One workgroup streams its system's whole working set through one CU, so
// the kernel only pays off for small boxes: at most kMaxPadded padded
// elements per system (three components), where a batched step would be
// dominated by launch latency.
constexpr int64_t kMaxPadded = 8192;

// (lx == ly, lz) pairs reachable under that limit
#define VIE_BLOCK_SHAPES(F)                                                                                 \
  F(8, 8) F(8, 12) F(8, 16) F(8, 24) F(8, 32) F(12, 8) F(12, 12) F(12, 16) F(12, 24) F(12, 32) F(16, 8)    \
      F(16, 12) F(16, 16) F(16, 24) F(24, 8)

bool block_solver_supported(int lx, int ly, int lz, int bz) {
  if (lx != ly || 3LL * bz * lx * ly > kMaxPadded) return false;
#define C(a, b) \
  if (lx == a && lz == b) return true;
  VIE_BLOCK_SHAPES(C)
#undef C
  return false;
}

template <typename R>
void block_solve(const BlockSolveArgs& a, int lx, int lz, hipStream_t s) {
  if (a.nsys <= 0) return;
#define C(A, B)                                                                                                 \
  if (lx == A && lz == B) {                                                                                     \
    hipLaunchKernelGGL((k_block_solve<R, A, B>), dim3(a.nsys), dim3(BT), 0, s, a);                              \
    hipError_t e = hipGetLastError();                                                                           \
    if (e != hipSuccess) throw std::runtime_error(std::string("block solver launch: ") + hipGetErrorString(e)); \
    return;                                                                                                     \
  }
  VIE_BLOCK_SHAPES(C)
#undef C
  throw std::runtime_error("block solver: no kernel for these FFT lengths");
}

template void block_solve<float>(const BlockSolveArgs&, int, int, hipStream_t);
template void block_solve<double>(const BlockSolveArgs&, int, int, hipStream_t);

}  // namespace vie
