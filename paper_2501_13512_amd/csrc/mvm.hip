// FFT-accelerated product with the discretised VIE operator, and the setup of
// the Green-tensor spectra.
//
// Operator (eqs. (2)-(4) and (6) of the paper, unknown P = J/(j omega eps0)):
//   (A x)_m = x_m / chi_m - sum_n T(m - n) x_n   on the scatterer voxels,
//   (A x)_m = 0                                   on vacuum voxels.
// The sum is a 3-D convolution with the block-Toeplitz kernel T (Sec. I),
// done as a circulant convolution on a (lx, ly, lz) grid with L >= 2n - 1 per
// axis, in five passes over HBM:
//   1. x forward, pruned: rows of nx voxels, zero-padded to lx;
//   2. y forward, pruned: only the nz non-zero z-planes exist;
//   3. z forward + 3x3 symmetric spectral multiply + z inverse, fused in one
//      workgroup per (y-fold, tile of x-folds): the four mirror columns
//      (+-qx, +-qy) of the three components sit in LDS together, so each
//      value of the octant spectrum (q in [0, L/2]^3, parity signs for the
//      odd components: T_xy is odd in x and y, ...) is read once;
//   4. y inverse, cropped to ny rows;
//   5. x inverse, cropped to nx, scaled by 1/(lx ly lz), fused with the
//      local term and the vacuum mask, written as c128.
#include <cmath>
#include <stdexcept>
#include <string>

#include "api_lock.h"
#include "fft_core.h"
#include "krylov_dev.h"

namespace vie {

int smallest_fft_length(int min_len, bool xy) {
  for (int L : kFftLengths)
    if (L >= min_len && !(xy && L == 36)) return L;
  return -1;
}

// ------------------------------------------------------------------ geometry
constexpr int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p *= 2;
  return p;
}
constexpr int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <typename R, int L>
struct Geo {
  static constexpr int T = PlanInfo<L>::max_butterflies;  // threads per pencil
  static constexpr int ES = (int)sizeof(cx<R>);
  // rows (contiguous pencils): ~256 threads, LDS [ROWP][L]
  static constexpr int ROWP = cmax(1, cmin(256 / T, (64 * 1024) / (L * ES)));
  // columns (strided pencils), LDS [L][COLP]: at least 128 contiguous bytes
  // per row of the tile (one full cache line) when 64 KB of LDS allow it,
  // with TC <= T threads per column (several butterflies per thread when
  // T * COLP would exceed 1024 threads)
  static constexpr int LDS_COLS = cmax(1, (64 * 1024) / (L * ES));
  static constexpr int COLP = cmax(1, pow2_floor(cmin(LDS_COLS, cmax(128 / ES, cmin(cmax(16, 256 / T), 512 / T)))));
  static constexpr int TC = cmin(T, cmax(1, 1024 / COLP));
};

__device__ __forceinline__ bool sys_active(const int* status, int s) {
  return status == nullptr || status[s] == ST_ACTIVE;
}

// n / d by one multiply-high: m = ceil(2^32 / d) for d >= 2, m = 0 for d = 1.
// With n = q d + r, n m / 2^32 = n / d + n (m - 2^32 / d) / 2^32 and the
// second term is below n / 2^32, so the floor is q whenever n d < 2^32.
// The plane kernels' element, row and plane indices stay far inside that
// range (checked when they are launched).
inline unsigned div_magic(int d) { return d <= 1 ? 0u : (unsigned)(((1ull << 32) + (unsigned)d - 1) / (unsigned)d); }
__device__ __forceinline__ unsigned udiv_m(unsigned n, unsigned m) { return m ? __umulhi(n, m) : n; }

template <typename R>
__device__ __forceinline__ cx<R> czero() {
  return mk<R>(R(0), R(0));
}

// ------------------------------------------------------------------ kernels
template <typename R>
struct RowArgs {
  int nx, ny, nz, lx, ly;
  int64_t vstride, cstride, wstride;
  const c128* x;
  c128* y;
  const c128* chi_inv;
  cx<R>* work;
  const int* status;
  const cx<R>* tw;
  int mask_input;
  int chi3;   // 1/chi per component ([3][nz][ny][nx]: rooftop faces) instead of per voxel
  // division constants of the plane kernels (udiv_m): nx ny, nx, ny, nz
  unsigned m_pe, m_nx, m_ny, m_nz;
  double scale;
  // BiCGSTAB work fused into pass 1 (in_mode) and pass 5 (out_mode)
  int in_mode, out_mode;
  const c128* r;
  c128* p;
  const c128* v;
  const c128* rhat;
  const c128* s;
  KBatch k;
};

// Pass 1: x forward with zero padding nx -> lx, c128 -> R.  With a fused
// BiCGSTAB update (in_mode 1: p, in_mode 2: s) the new vector is formed in a
// pre-pass that issues all loads of a chunk of elements before storing it to
// HBM and to the pencil's LDS slot; the transform then starts from LDS.
template <typename R, int L>
__global__ void __launch_bounds__((Geo<R, L>::T * Geo<R, L>::ROWP)) k_row_fwd(RowArgs<R> a) {
  using G = Geo<R, L>;
  constexpr int T = G::T;
  __shared__ cx<R> lds[G::ROWP * L];
  const int rows = 3 * a.nz * a.ny;
  const int tiles = (rows + G::ROWP - 1) / G::ROWP;
  const int sys = blockIdx.x / tiles, tile = blockIdx.x - sys * tiles;
  if (!sys_active(a.status, sys)) return;
  const int p = threadIdx.x / T, t = threadIdx.x - p * T;
  const int row = tile * G::ROWP + p;
  const bool valid = row < rows;
  const int rr = valid ? row : 0;
  const int c = rr / (a.nz * a.ny), zy = rr - c * (a.nz * a.ny);
  const int z = zy / a.ny, yy = zy - z * a.ny;
  const int64_t vrow = sys * a.vstride + (int64_t)rr * a.nx;
  cx<R>* w = a.work + sys * a.wstride + ((int64_t)(c * a.nz + z) * a.ly + yy) * a.lx;
  cx<R>* slot = lds + p * L;
  const int nx = a.nx;
  const int mode = a.in_mode;
  auto st = [&](int k, cx<R> v) { w[k] = v; };
  if (mode == 0) {
    const c128* xin = a.x + vrow;
    const c128* chi = a.chi_inv + sys * a.cstride + (int64_t)(a.chi3 ? rr : zy) * a.nx;
    const bool msk = a.mask_input != 0;
    auto ld = [&](int n) -> cx<R> {
      if (n < nx) {
        c128 v = xin[n];
        if (msk) {
          c128 ci = chi[n];
          if (ci.x == 0.0 && ci.y == 0.0) v = mk<double>(0.0, 0.0);
        }
        return cvt<R>(v);
      }
      return czero<R>();
    };
    fft_pencil<R, L, T, -1>(ld, st, slot, 1, t, valid, a.tw);
    return;
  }
  const KState& ks = a.k.st[sys];
  const bool first = mode == 1 && ks.iters == 0;
  double acc = 0.0;
  constexpr int E = (L + T - 1) / T;   // elements per thread
  constexpr int CH = 4;                // elements per load batch
  c128 rv[CH], pv[CH], vv[CH];
  auto load = [&](int j0) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int n = t + (j0 + u) * T;
      if (valid && j0 + u < E && n < nx) {
        rv[u] = a.r[vrow + n];
        if (!first) vv[u] = a.v[vrow + n];
        if (mode == 1 && !first) pv[u] = a.p[vrow + n];
      }
    }
  };
  load(0);   // in flight while alpha is formed
  c128 c1;
  if (mode == 3) {   // alpha from the last product's partials (FIN_ALPHA fused)
    if (!fused_alpha(a.k, sys, tile == 0, &c1)) return;
  } else {
    c1 = mode == 1 ? ks.beta : ks.alpha;
  }
  const c128 c2 = ks.omega;
#pragma unroll
  for (int j0 = 0; j0 < E; j0 += CH) {
    if (j0 > 0) load(j0);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int n = t + (j0 + u) * T;
      if (valid && j0 + u < E && n < L) {
        if (n < nx) {
          c128 val;
          if (mode == 1)
            val = first ? rv[u] : rv[u] + c1 * (pv[u] - c2 * vv[u]);   // p = r + beta (p - omega v)
          else
            val = rv[u] - c1 * vv[u];                                    // s = r - alpha v
          a.p[vrow + n] = val;
          slot[n] = cvt<R>(val);
          acc += abs2(val);
        } else {
          slot[n] = czero<R>();
        }
      }
    }
  }
  __syncthreads();
  auto ld = [&](int n) -> cx<R> { return slot[n]; };
  fft_pencil<R, L, T, -1, true, false>(ld, st, slot, 1, t, valid, a.tw);
  if (mode == 2) {
    double sum[1] = {acc};
    write_partial<1>(sum, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  }
}

// Pass 5: x inverse, crop lx -> nx, y = x/chi - scale * Q on the mask, 0 off
// it.  The cropped transform lands in LDS; a post-pass issues the loads of
// 1/chi, x and (fused inner products) rhat or s for a chunk of elements
// before storing y.
template <typename R, int L>
__global__ void __launch_bounds__((Geo<R, L>::T * Geo<R, L>::ROWP)) k_row_inv_local(RowArgs<R> a) {
  using G = Geo<R, L>;
  constexpr int T = G::T;
  __shared__ cx<R> lds[G::ROWP * L];
  const int rows = 3 * a.nz * a.ny;
  const int tiles = (rows + G::ROWP - 1) / G::ROWP;
  const int sys = blockIdx.x / tiles, tile = blockIdx.x - sys * tiles;
  if (!sys_active(a.status, sys)) return;
  const int p = threadIdx.x / T, t = threadIdx.x - p * T;
  const int row = tile * G::ROWP + p;
  const bool valid = row < rows;
  const int rr = valid ? row : 0;
  const int c = rr / (a.nz * a.ny), zy = rr - c * (a.nz * a.ny);
  const int z = zy / a.ny, yy = zy - z * a.ny;
  const int64_t vrow = sys * a.vstride + (int64_t)rr * a.nx;
  const c128* chi = a.chi_inv + sys * a.cstride + (int64_t)(a.chi3 ? rr : zy) * a.nx;
  const cx<R>* w = a.work + sys * a.wstride + ((int64_t)(c * a.nz + z) * a.ly + yy) * a.lx;
  cx<R>* slot = lds + p * L;
  const int nx = a.nx;
  auto ld = [&](int n) -> cx<R> { return w[n]; };
  auto sts = [&](int k, cx<R> v) {
    if (k < nx) slot[k] = v;
  };
  fft_pencil<R, L, T, +1, false, true>(ld, sts, slot, 1, t, valid, a.tw);

  const double scale = a.scale;
  const int mode = a.out_mode;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  constexpr int E = (L + T - 1) / T;
  constexpr int CH = 4;
#pragma unroll
  for (int j0 = 0; j0 < E; j0 += CH) {
    c128 ci[CH], xv[CH], ov[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int k = t + (j0 + u) * T;
      if (valid && j0 + u < E && k < nx) {
        ci[u] = chi[k];
        xv[u] = a.x[vrow + k];
        if (mode == 1 || mode == 3) ov[u] = a.rhat[vrow + k];
        if (mode == 2 || mode == 4) ov[u] = a.s[vrow + k];
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int k = t + (j0 + u) * T;
      if (valid && j0 + u < E && k < nx) {
        c128 out = mk<double>(0.0, 0.0);
        if (mode == 3)   // field at every voxel: E_inc + sum T P
          out = ov[u] + scale * cvt<double>(slot[k]);
        else if (ci[u].x != 0.0 || ci[u].y != 0.0)
          out = xv[u] * ci[u] - scale * cvt<double>(slot[k]);
        a.y[vrow + k] = out;
        if (mode == 1) {          // <rhat, y>
          const c128 d = cdot1(ov[u], out);
          acc[0] += d.x;
          acc[1] += d.y;
        } else if (mode == 2 || mode == 4) {   // <y, s>, <y, y> (and ||s||^2)
          const c128 d = cdot1(out, ov[u]);
          acc[0] += d.x;
          acc[1] += d.y;
          acc[2] += abs2(out);
          if (mode == 4) acc[3] += abs2(ov[u]);
        }
      }
    }
  }
  if (mode == 1) {
    double sum[2] = {acc[0], acc[1]};
    write_partial<2>(sum, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  } else if (mode == 2) {
    double sum[3] = {acc[0], acc[1], acc[2]};
    write_partial<3>(sum, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  } else if (mode == 4) {
    write_partial<4>(acc, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  }
}

// ------------------------------------------------------------------ plane passes
// Small square transforms (lx = ly <= 64): the x and y transforms of a
// z-plane run in one kernel with the plane in LDS, so passes 1 + 2 become
// k_plane_fwd and passes 4 + 5 become k_plane_inv_local (one launch and one
// trip through HBM fewer each way; same BiCGSTAB fusion as the row kernels).
// A workgroup takes NPL consecutive planes (c, z) of one system; LDS holds
// them as [NPL][L][L + 1] (rows padded against bank conflicts on columns).
// Variant PV sets NPL: 0 as many planes as 48 KB of LDS hold (at most 16),
// 1 at most two, 2 one plane.  Fewer planes per workgroup mean more, shorter
// workgroups: the product's latency falls when few systems are active (two
// 32 x 32 planes of a 16 x 16 box take 3 transform rounds of 32 pencils
// where five planes take 8), at the cost of more workgroups to dispatch.
template <typename R, int L, int PV>
struct PlaneGeo {
  static constexpr int ES = (int)sizeof(cx<R>);
  static constexpr int LP = L + 1;
  static constexpr int NPL_LDS = cmax(1, cmin(16, (48 * 1024) / (L * LP * ES)));
  static constexpr int NPL = PV == 0 ? NPL_LDS : (PV == 1 ? cmin(2, NPL_LDS) : 1);
  static constexpr int BT = 256;
  static constexpr int T = PlanInfo<L>::max_butterflies;
  static constexpr int PP = BT / T;
  static_assert(BT % T == 0, "pencil threads must divide the workgroup");
};

template <typename R, int L, int PV>
__global__ void __launch_bounds__((PlaneGeo<R, L, PV>::BT)) k_plane_fwd(RowArgs<R> a) {
  using G = PlaneGeo<R, L, PV>;
  constexpr int T = G::T, PP = G::PP, LP = G::LP, NPL = G::NPL, BT = G::BT;
  __shared__ cx<R> lds[NPL * L * LP];
  const int planes = 3 * a.nz;
  const int tiles = (planes + NPL - 1) / NPL;
  const int sys = blockIdx.x / tiles, tile = blockIdx.x - sys * tiles;
  if (!sys_active(a.status, sys)) return;
  const int pl0 = tile * NPL, npl = min(NPL, planes - pl0);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int pe = ny * nx;
  const int ne = npl * pe;
  const int64_t v0 = sys * a.vstride + (int64_t)pl0 * pe;
  const int mode = a.in_mode;
  double acc = 0.0;
  // zero the padding columns [nx, L) of rows y < ny
  const int padw = L - nx;
  for (int e = threadIdx.x; e < npl * ny * padw; e += BT) {
    const int row = e / padw, xx = nx + (e - row * padw);
    const int q = (int)udiv_m((unsigned)row, a.m_ny);
    lds[q * L * LP + (row - q * ny) * LP + xx] = czero<R>();
  }
  auto lds_at = [&](int e) -> cx<R>* {
    const int q = (int)udiv_m((unsigned)e, a.m_pe), rem = e - q * pe, y = (int)udiv_m((unsigned)rem, a.m_nx);
    return lds + (q * L + y) * LP + (rem - y * nx);
  };
  if (mode == 0) {
    const c128* chi = a.chi_inv + sys * a.cstride;
    const bool msk = a.mask_input != 0;
    for (int e = threadIdx.x; e < ne; e += BT) {
      c128 v = a.x[v0 + e];
      if (msk) {
        const int q = (int)udiv_m((unsigned)e, a.m_pe);
        const int zq = pl0 + q;
        const int z = a.chi3 ? zq : zq - nz * (int)udiv_m((unsigned)zq, a.m_nz);
        const c128 ci = chi[(int64_t)z * pe + (e - q * pe)];
        if (ci.x == 0.0 && ci.y == 0.0) v = mk<double>(0.0, 0.0);
      }
      *lds_at(e) = cvt<R>(v);
    }
  } else {
    const KState& ks = a.k.st[sys];
    const bool first = mode == 1 && ks.iters == 0;
    constexpr int CH = 4;
    c128 rv[CH], pv[CH], vv[CH];
    auto load = [&](int e0) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = e0 + u * BT + (int)threadIdx.x;
        if (e < ne) {
          rv[u] = a.r[v0 + e];
          if (!first) vv[u] = a.v[v0 + e];
          if (mode == 1 && !first) pv[u] = a.p[v0 + e];
        }
      }
    };
    load(0);   // in flight while alpha is formed
    c128 c1;
    if (mode == 3) {   // alpha from the last product's partials (FIN_ALPHA fused)
      if (!fused_alpha(a.k, sys, tile == 0, &c1)) return;
    } else {
      c1 = mode == 1 ? ks.beta : ks.alpha;
    }
    const c128 c2 = ks.omega;
    for (int e0 = 0; e0 < ne; e0 += CH * BT) {
      if (e0 > 0) load(e0);
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = e0 + u * BT + (int)threadIdx.x;
        if (e < ne) {
          c128 val;
          if (mode == 1)
            val = first ? rv[u] : rv[u] + c1 * (pv[u] - c2 * vv[u]);   // p = r + beta (p - omega v)
          else
            val = rv[u] - c1 * vv[u];                                    // s = r - alpha v
          a.p[v0 + e] = val;
          *lds_at(e) = cvt<R>(val);
          acc += abs2(val);
        }
      }
    }
  }
  __syncthreads();
  // x transforms of the rows y < ny, in place.  Consecutive lanes take
  // consecutive rows (a row's threads are PP lanes apart), so the threads
  // that a stage with fewer butterflies leaves idle form whole wavefronts,
  // which skip it; the row stride LP keeps the lanes' LDS banks distinct.
  {
    const int p = threadIdx.x % PP, t = threadIdx.x / PP;
    const int nrows = npl * ny;
    for (int r0 = 0; r0 < nrows; r0 += PP) {
      const int row = r0 + p;
      const bool valid = p < PP && row < nrows;
      const int rr = valid ? row : 0;
      const int rq = (int)udiv_m((unsigned)rr, a.m_ny);
      cx<R>* slot = lds + (rq * L + (rr - rq * ny)) * LP;
      auto ld = [&](int n) -> cx<R> { return slot[n]; };
      auto st = [&](int k, cx<R> v) { slot[k] = v; };
      fft_pencil<R, L, T, -1, true, true>(ld, st, slot, 1, t, valid, a.tw);
    }
  }
  // y transforms of the L columns (rows >= ny are zero), out to HBM
  {
    const int p = threadIdx.x % PP, t = threadIdx.x / PP;
    const int ncols = npl * L;
    cx<R>* w = a.work + sys * a.wstride + (int64_t)pl0 * L * L;
    for (int c0 = 0; c0 < ncols; c0 += PP) {
      const int col = c0 + p;
      const bool valid = t < T && col < ncols;
      const int cc = valid ? col : 0;
      const int q = cc / L, xq = cc - q * L;
      cx<R>* slot = lds + q * L * LP + xq;
      cx<R>* wc = w + (int64_t)q * L * L + xq;
      auto ld = [&](int n) -> cx<R> { return n < ny ? slot[n * LP] : czero<R>(); };
      auto st = [&](int k, cx<R> v) { wc[k * L] = v; };
      fft_pencil<R, L, T, -1, true, false>(ld, st, slot, LP, t, valid, a.tw);
    }
  }
  if (mode == 2) {
    double sum[1] = {acc};
    write_partial<1>(sum, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  }
}

template <typename R, int L, int PV>
__global__ void __launch_bounds__((PlaneGeo<R, L, PV>::BT)) k_plane_inv_local(RowArgs<R> a) {
  using G = PlaneGeo<R, L, PV>;
  constexpr int T = G::T, PP = G::PP, LP = G::LP, NPL = G::NPL, BT = G::BT;
  __shared__ cx<R> lds[NPL * L * LP];
  const int planes = 3 * a.nz;
  const int tiles = (planes + NPL - 1) / NPL;
  const int sys = blockIdx.x / tiles, tile = blockIdx.x - sys * tiles;
  if (!sys_active(a.status, sys)) return;
  const int pl0 = tile * NPL, npl = min(NPL, planes - pl0);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int pe = ny * nx;
  const int ne = npl * pe;
  const int64_t v0 = sys * a.vstride + (int64_t)pl0 * pe;
  // y inverse of the L columns from HBM, rows k < ny kept in LDS
  {
    const int p = threadIdx.x % PP, t = threadIdx.x / PP;
    const int ncols = npl * L;
    const cx<R>* w = a.work + sys * a.wstride + (int64_t)pl0 * L * L;
    for (int c0 = 0; c0 < ncols; c0 += PP) {
      const int col = c0 + p;
      const bool valid = t < T && col < ncols;
      const int cc = valid ? col : 0;
      const int q = cc / L, xq = cc - q * L;
      cx<R>* slot = lds + q * L * LP + xq;
      const cx<R>* wc = w + (int64_t)q * L * L + xq;
      auto ld = [&](int n) -> cx<R> { return wc[n * L]; };
      auto st = [&](int k, cx<R> v) {
        if (k < ny) slot[k * LP] = v;
      };
      fft_pencil<R, L, T, +1, false, true>(ld, st, slot, LP, t, valid, a.tw);
    }
  }
  // x inverse of the rows y < ny, in place, cropped to nx (lanes over rows
  // as in the forward kernel)
  {
    const int p = threadIdx.x % PP, t = threadIdx.x / PP;
    const int nrows = npl * ny;
    for (int r0 = 0; r0 < nrows; r0 += PP) {
      const int row = r0 + p;
      const bool valid = p < PP && row < nrows;
      const int rr = valid ? row : 0;
      const int rq = (int)udiv_m((unsigned)rr, a.m_ny);
      cx<R>* slot = lds + (rq * L + (rr - rq * ny)) * LP;
      auto ld = [&](int n) -> cx<R> { return slot[n]; };
      auto st = [&](int k, cx<R> v) {
        if (k < nx) slot[k] = v;
      };
      fft_pencil<R, L, T, +1, true, true>(ld, st, slot, 1, t, valid, a.tw);
    }
  }
  // y = x/chi - scale Q on the mask, fused inner products
  const double scale = a.scale;
  const int mode = a.out_mode;
  const c128* chi = a.chi_inv + sys * a.cstride;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  constexpr int CH = 4;
  for (int e0 = 0; e0 < ne; e0 += CH * BT) {
    c128 ci[CH], xv[CH], ov[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = e0 + u * BT + (int)threadIdx.x;
      if (e < ne) {
        const int q = (int)udiv_m((unsigned)e, a.m_pe), zq = pl0 + q;
        ci[u] = chi[(int64_t)(a.chi3 ? zq : zq - nz * (int)udiv_m((unsigned)zq, a.m_nz)) * pe + (e - q * pe)];
        xv[u] = a.x[v0 + e];
        if (mode == 1 || mode == 3) ov[u] = a.rhat[v0 + e];
        if (mode == 2 || mode == 4) ov[u] = a.s[v0 + e];
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = e0 + u * BT + (int)threadIdx.x;
      if (e < ne) {
        const int q = (int)udiv_m((unsigned)e, a.m_pe), rem = e - q * pe, y = (int)udiv_m((unsigned)rem, a.m_nx);
        const cx<R> qv = lds[(q * L + y) * LP + (rem - y * nx)];
        c128 out = mk<double>(0.0, 0.0);
        if (mode == 3)   // field at every voxel: E_inc + sum T P
          out = ov[u] + scale * cvt<double>(qv);
        else if (ci[u].x != 0.0 || ci[u].y != 0.0)
          out = xv[u] * ci[u] - scale * cvt<double>(qv);
        a.y[v0 + e] = out;
        if (mode == 1) {          // <rhat, y>
          const c128 d = cdot1(ov[u], out);
          acc[0] += d.x;
          acc[1] += d.y;
        } else if (mode == 2 || mode == 4) {   // <y, s>, <y, y> (and ||s||^2)
          const c128 d = cdot1(out, ov[u]);
          acc[0] += d.x;
          acc[1] += d.y;
          acc[2] += abs2(out);
          if (mode == 4) acc[3] += abs2(ov[u]);
        }
      }
    }
  }
  if (mode == 1) {
    double sum[2] = {acc[0], acc[1]};
    write_partial<2>(sum, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  } else if (mode == 2) {
    double sum[3] = {acc[0], acc[1], acc[2]};
    write_partial<3>(sum, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  } else if (mode == 4) {
    write_partial<4>(acc, a.k.partials, a.k.pstride, a.k.ntile, sys, tile, tiles);
  }
}

// In-place FFT of full-length rows (spectra setup).
template <typename R, int L>
__global__ void __launch_bounds__((Geo<R, L>::T * Geo<R, L>::ROWP)) k_row_full(cx<R>* data, int64_t rows,
                                                                           const cx<R>* tw) {
  using G = Geo<R, L>;
  __shared__ cx<R> lds[G::ROWP * L];
  const int p = threadIdx.x / G::T, t = threadIdx.x - p * G::T;
  const int64_t row = (int64_t)blockIdx.x * G::ROWP + p;
  const bool valid = row < rows;
  cx<R>* d = data + (valid ? row : 0) * L;
  auto ld = [&](int n) -> cx<R> { return d[n]; };
  auto st = [&](int k, cx<R> v) { d[k] = v; };
  fft_pencil<R, L, G::T, -1>(ld, st, lds + p * L, 1, t, valid, tw);
}

// Strided pencils, in place: per system, data[outer][L][inner]; element n of
// column (o, i) at o*L*inner + n*inner + i.  Reads n < n_in (zero beyond),
// writes k < n_out.  Passes 2 and 4, and the y/z passes of the setup.
template <typename R>
struct ColArgs {
  cx<R>* data;
  int outer, inner, n_in, n_out;
  int64_t stride;
  const int* status;
  const cx<R>* tw;
  int nsys;
};

template <typename R, int L, int DIR>
__global__ void __launch_bounds__((Geo<R, L>::TC * Geo<R, L>::COLP)) k_col(ColArgs<R> a) {
  using G = Geo<R, L>;
  __shared__ cx<R> lds[G::COLP * L];
  const int64_t cols = (int64_t)a.outer * a.inner;
  const int64_t tiles = (cols + G::COLP - 1) / G::COLP;
  const int sys = (int)(blockIdx.x / tiles);
  const int64_t tile = blockIdx.x - (int64_t)sys * tiles;
  if (!sys_active(a.status, sys)) return;
  const int p = threadIdx.x % G::COLP, t = threadIdx.x / G::COLP;
  const int64_t col = tile * G::COLP + p;
  const bool valid = col < cols;
  const int64_t cc = valid ? col : 0;
  const int64_t o = cc / a.inner, i = cc - o * a.inner;
  cx<R>* base = a.data + sys * a.stride + o * (int64_t)L * a.inner + i;
  const int inner = a.inner, n_in = a.n_in, n_out = a.n_out;
  auto ld = [&](int n) -> cx<R> { return n < n_in ? base[(int64_t)n * inner] : czero<R>(); };
  auto st = [&](int k, cx<R> v) {
    if (k < n_out) base[(int64_t)k * inner] = v;
  };
  fft_pencil<R, L, G::TC, DIR>(ld, st, lds + p, G::COLP, t, valid, a.tw);
}

// Pass 3: z forward (nz -> LZ), spectral multiply, z inverse (LZ -> nz).
//
// The spectrum is stored for q in [0, L/2] per axis only; the other octants
// are the same values with a sign (S_ij(L - q) = +-S_ij(q)).  An axis of
// length L is covered by folds f in [0, nfold(L)); fold f stands for column
// f (mirror 0) and column L - f (mirror 1), both using spectral index f.
// For even L fold 0's mirror is the Nyquist column L/2 (spectral index L/2,
// sign +); for odd L fold 0 has no mirror.  A workgroup takes one y-fold and
// ZP consecutive x-folds and transforms all four mirror columns
// (+-qx, +-qy) of the three components, so each spectrum value is loaded
// once and applied to up to 8 points (+-qx, +-qy, qz and LZ - qz).
__host__ __device__ constexpr int nfold(int L) { return (L % 2 == 0) ? L / 2 : (L + 1) / 2; }

struct FoldCol {
  int col;  // column index, -1 if absent
  int sf;   // spectral (octant) index
  int sg;   // parity sign for components odd in this axis
};

__device__ __forceinline__ FoldCol fold_col(int f, int m, int L) {
  if (m == 0) return {f, f, 1};
  if (f > 0) return {L - f, f, -1};
  if ((L & 1) == 0 && L >= 2) return {L / 2, L / 2, 1};
  return {-1, 0, 1};
}

// Element i of an array whose byte size is below 4 GiB: the byte offset is
// formed in 32 bits, so the access can use a uniform base register plus a
// 32-bit per-lane offset.
template <typename T>
__device__ __forceinline__ T* elem(T* base, unsigned i) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T* elem(const T* base, unsigned i) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}

// Workgroup b of n runs on XCD b % 8 (round-robin dispatch).  Renumber so
// that each XCD takes one contiguous range of the logical order: work that
// shares data then shares that XCD's L2.
__device__ __forceinline__ int xcd_chunked(int b, int n) {
  constexpr int NX = 8;
  const int q = n / NX, r = n - q * NX;
  const int x = b % NX, l = b / NX;
  return x * q + min(x, r) + l;
}

// Logical row i -> qy in the order 0, 1, L-1, 2, L-2, ...: rows that share
// an octant row of the spectra (qy and L - qy) are adjacent.
__device__ __forceinline__ int mirror_paired_row(int i, int L) {
  if (i == 0) return 0;
  const int k = (i + 1) >> 1;
  return (i & 1) ? k : L - k;
}

// Variant 0: one tile of ZP columns per workgroup, three components side by
// side; each point loads its spectrum values.  Tiles run along mirror-paired
// rows, chunked per XCD, so the four mirror columns that use one octant
// spectrum value are transformed on one XCD close together in time and the
// value is fetched from HBM about once.
// Column-set variants (V = 0, 2, 3, 4): ZP columns per workgroup, TZ threads
// per column and component, PF: spectrum values loaded into registers
// before the data (their latency overlaps the forward transform).
//   0: wide tiles (up to 1024 threads), max_butterflies threads per column
//   2: wide tiles, min_butterflies rounded up to a power of two threads per
//      column, prefetch (for L = 48: 4 threads, so a 16-column tile of the
//      three components fills three whole wavefronts and each thread takes
//      four radix-3 butterflies, where 3 threads leave a quarter of the
//      third wavefront idle and take six butterflies, the last for one
//      thread in three)
//   3: one cache line of columns, min_butterflies threads, prefetch
//   4: one cache line of columns, max_butterflies threads
template <typename R, int LZ, int V>
struct ZColGeo {
  static constexpr int T = PlanInfo<LZ>::max_butterflies;
  static constexpr int TB = V == 2 ? cmin(T, pow2_ceil(PlanInfo<LZ>::min_butterflies)) : PlanInfo<LZ>::min_butterflies;
  static constexpr int ES = (int)sizeof(cx<R>);
  static constexpr int LDS_ZP = cmax(1, (144 * 1024) / (3 * LZ * ES));
  static constexpr int LINE = cmax(1, pow2_floor(cmin(LDS_ZP, 128 / ES)));
  static constexpr int WIDE = cmax(1, pow2_floor(cmin(LDS_ZP, cmin(64, cmax(128 / ES, 1024 / (3 * T))))));
  static constexpr int ZP = (V == 3 || V == 4) ? LINE : WIDE;
  static constexpr int TZ = (V == 2 || V == 3) ? cmin(TB, cmax(1, 1024 / (3 * ZP)))
                                               : cmin(T, pow2_floor(cmax(1, 1024 / (3 * ZP))));
  static constexpr bool PF = V == 2 || V == 3;
};

// Variant 1 (mirror columns): geometry.
template <typename R, int LZ>
struct ZGeo {
  static constexpr int T = PlanInfo<LZ>::max_butterflies;
  static constexpr int ES = (int)sizeof(cx<R>);
  static constexpr int ZP = cmax(1, pow2_floor(cmin(64, cmin(1024 / (3 * T), (144 * 1024) / (12 * LZ * ES)))));
};

template <typename R>
struct ZArgs {
  int nz, ly, lx;
  int variant;   // 0, 2, 3, 4: column sets (ZColGeo); 1: mirror columns
  int rooftop;   // spectral multiply of the rooftop discretisation (column sets only)
  int64_t wstride, sstride;
  cx<R>* work;
  const cx<R>* spec;
  const cx<R>* const* spec_tab;   // per-system spectra (null: spec + sys sstride)
  const int* status;
  const cx<R>* tw;
};

template <typename R, int LZ>
__global__ void __launch_bounds__((3 * ZGeo<R, LZ>::T * ZGeo<R, LZ>::ZP)) k_zconv_mirror(ZArgs<R> a) {
  using G = ZGeo<R, LZ>;
  constexpr int T = G::T, ZP = G::ZP;
  constexpr int SLOT = LZ * ZP;           // one (mirror, component) pencil set
  __shared__ cx<R> lds[12 * SLOT];        // [mirror 4][component 3][qz][p]
  const int lx = a.lx, ly = a.ly, nz = a.nz;
  const int nfx = nfold(lx), nfy = nfold(ly);
  const int xt = (nfx + ZP - 1) / ZP;
  const int per_sys = nfy * xt;
  const int sys = blockIdx.x / per_sys;
  const int rr = blockIdx.x - sys * per_sys;
  const int fy = rr / xt, ft = rr - fy * xt;
  if (!sys_active(a.status, sys)) return;
  const int comp = threadIdx.x / (T * ZP);
  const int rem = threadIdx.x - comp * (T * ZP);
  const int p = rem % ZP, t = rem / ZP;
  const int fx = ft * ZP + p;
  const bool pvalid = fx < nfx;
  const int64_t plane = (int64_t)ly * lx;
  cx<R>* wsys = a.work + sys * a.wstride + (int64_t)comp * nz * plane;

  // forward along z of the four mirror columns, into LDS
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const FoldCol cxm = fold_col(fx, m & 1, lx), cym = fold_col(fy, m >> 1, ly);
    const bool valid = pvalid && cxm.col >= 0 && cym.col >= 0;
    cx<R>* base = wsys + (valid ? (int64_t)cym.col * lx + cxm.col : 0);
    cx<R>* slot = lds + (m * 3 + comp) * SLOT + p;
    auto ldg = [&](int n) -> cx<R> { return n < nz ? base[n * plane] : czero<R>(); };
    auto sts = [&](int k, cx<R> v) { slot[k * ZP] = v; };
    fft_pencil<R, LZ, T, -1, false, true>(ldg, sts, slot, ZP, t, valid, a.tw);
  }

  // Q = S X at every point of the four columns; one spectrum load per
  // (fold x, fold y, fold z), reused for its mirrors
  const int64_t ox = lx / 2 + 1, oy = ly / 2 + 1;
  const int64_t oct = ox * oy * (LZ / 2 + 1);
  const cx<R>* spec = a.spec_tab ? a.spec_tab[sys] : a.spec + sys * a.sstride;
  constexpr int NFZ = nfold(LZ);
  for (int i = threadIdx.x; i < NFZ * ZP; i += 3 * T * ZP) {
    const int fz = i / ZP, pp = i - fz * ZP;
    const int fxx = ft * ZP + pp;
    if (fxx >= nfx) continue;
    int64_t o_prev = -1;
    cx<R> sxx, sxy, sxz, syy, syz, szz;
#pragma unroll
    for (int mz = 0; mz < 2; ++mz) {
      const FoldCol czm = fold_col(fz, mz, LZ);
      if (czm.col < 0) continue;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const FoldCol cxm = fold_col(fxx, m & 1, lx), cym = fold_col(fy, m >> 1, ly);
        if (cxm.col < 0 || cym.col < 0) continue;
        const int64_t o = ((int64_t)czm.sf * oy + cym.sf) * ox + cxm.sf;
        if (o != o_prev) {
          sxx = spec[o];
          sxy = spec[oct + o];
          sxz = spec[2 * oct + o];
          syy = spec[3 * oct + o];
          syz = spec[4 * oct + o];
          szz = spec[5 * oct + o];
          o_prev = o;
        }
        const R gxy = R(cxm.sg * cym.sg), gxz = R(cxm.sg * czm.sg), gyz = R(cym.sg * czm.sg);
        const cx<R> axy = gxy * sxy, axz = gxz * sxz, ayz = gyz * syz;
        cx<R>* e = lds + m * 3 * SLOT + czm.col * ZP + pp;
        const cx<R> X = e[0], Y = e[SLOT], Z = e[2 * SLOT];
        e[0] = sxx * X + axy * Y + axz * Z;
        e[SLOT] = axy * X + syy * Y + ayz * Z;
        e[2 * SLOT] = axz * X + ayz * Y + szz * Z;
      }
    }
  }
  __syncthreads();

  // inverse along z, cropped to nz, back to HBM
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const FoldCol cxm = fold_col(fx, m & 1, lx), cym = fold_col(fy, m >> 1, ly);
    const bool valid = pvalid && cxm.col >= 0 && cym.col >= 0;
    cx<R>* base = wsys + (valid ? (int64_t)cym.col * lx + cxm.col : 0);
    cx<R>* slot = lds + (m * 3 + comp) * SLOT + p;
    auto lds_ld = [&](int n) -> cx<R> { return slot[n * ZP]; };
    auto stg = [&](int k, cx<R> v) {
      if (k < nz) base[k * plane] = v;
    };
    fft_pencil<R, LZ, T, +1, true, false>(lds_ld, stg, slot, ZP, t, valid, a.tw);
  }
}

// K = 0: the collocated dyadic multiply (six octant spectra of the symmetric
// tensor).  K = 1: the rooftop discretisation, whose spectral operator is
// G'(q) (X_c - conj(b_c) sum_j b_j X_j) with G' = k0^2 dV FFT(g~) (one even
// octant spectrum) and b_j = (1 - exp(-2 pi i q_j / L_j)) / (k0 d_j), the
// symbol of the cell divergence of face values; -conj(b_c) is the symbol of
// the face gradient of cell values.  The spectrum buffer holds the octant of
// G' followed by the full-length tables b_x[lx], b_y[ly], b_z[lz].
template <typename R, int LZ, int V, int K>
__global__ void __launch_bounds__((3 * ZColGeo<R, LZ, V>::TZ * ZColGeo<R, LZ, V>::ZP)) k_zconv_col(ZArgs<R> a) {
  using G = ZColGeo<R, LZ, V>;
  constexpr int T = G::TZ, ZP = G::ZP;
  constexpr int NT = 3 * T * ZP;
  constexpr int HZ = LZ / 2;
  constexpr int NFT = NT / ZP;                    // fold walkers per column
  constexpr int NF = (HZ + 1 + NFT - 1) / NFT;    // folds per walker
  __shared__ cx<R> lds[3 * LZ * ZP];
  const int cols = a.ly * a.lx;
  const int tiles = (cols + ZP - 1) / ZP;
  // Tile-major logical order (the grid is tiles x systems): each XCD takes
  // a contiguous range of tiles of every system, so the systems still
  // active are spread over all XCDs whichever they are, and the group's
  // shared spectrum columns of a tile are reused from that XCD's L2 by the
  // consecutive workgroups of the other systems.
  const int nsys = (int)gridDim.x / tiles;
  const int g = __builtin_amdgcn_readfirstlane(xcd_chunked(blockIdx.x, gridDim.x));   // uniform
  const int tile = g / nsys, sys = g - tile * nsys;
  if (!sys_active(a.status, sys)) return;
  const int comp = threadIdx.x / (T * ZP);
  const int rem = threadIdx.x - comp * (T * ZP);
  const int p = rem % ZP, t = rem / ZP;
  const int col = tile * ZP + p;   // logical column
  const bool valid = col < cols;
  // element offsets in 32 bits from the system's base (one system's work
  // buffer holds < 2^31 elements), so loads use a uniform base + offset
  const unsigned plane = (unsigned)a.ly * (unsigned)a.lx;
  unsigned pcol = 0;               // its place in the plane
  if (valid) {
    const int i = col / a.lx;
    pcol = (unsigned)(mirror_paired_row(i, a.ly) * a.lx + (col - i * a.lx));
  }
  cx<R>* const wsys = a.work + sys * a.wstride;
  const unsigned coff = (unsigned)comp * (unsigned)a.nz * plane + pcol;
  cx<R>* slot = lds + comp * LZ * ZP + p;
  const int nz = a.nz;

  // The multiply's view: a thread keeps one column (qx, qy) and walks the
  // z-folds fz = j, j + NFT, ...: each spectrum value serves qz = fz and
  // qz = LZ - fz.
  const int lx = a.lx, ly = a.ly;
  const int hx = lx / 2, hy = ly / 2;
  const int64_t ox = hx + 1, oy = hy + 1;
  const int64_t oct = ox * oy * (HZ + 1);
  const int pp = threadIdx.x % ZP, j0 = threadIdx.x / ZP;
  const int c2 = tile * ZP + pp;
  const bool cvalid = c2 < cols;
  R sx = R(1), sy = R(1);
  const cx<R>* const sp = a.spec_tab ? a.spec_tab[sys] : a.spec + sys * a.sstride;
  unsigned soff = 0;
  cx<R> bx = czero<R>(), by = czero<R>();   // K = 1: difference symbols of the column
  const unsigned oct32 = (unsigned)oct, fzs = (unsigned)(oy * ox);
  if (cvalid) {
    const int i2 = c2 / lx;
    const int qy = mirror_paired_row(i2, ly), qx = c2 - i2 * lx;
    const int fx = qx <= hx ? qx : lx - qx, fy = qy <= hy ? qy : ly - qy;
    sx = qx <= hx ? R(1) : R(-1);
    sy = qy <= hy ? R(1) : R(-1);
    soff = (unsigned)(fy * ox + fx);
    if constexpr (K == 1) {
      bx = *elem(sp, oct32 + (unsigned)qx);
      by = *elem(sp, oct32 + (unsigned)(lx + qy));
    }
  }
  constexpr int NS = K == 1 ? 3 : 6;
  // K = 0: spectrum values (xx, xy, xz, yy, yz, zz, parity signs of qx, qy
  // applied); K = 1: G'(fz), b_z(fz), b_z(LZ - fz)
  auto spec_at = [&](int fz, cx<R>* sv) {
    const unsigned o = soff + (unsigned)fz * fzs;
    if constexpr (K == 1) {
      const unsigned bz0 = oct32 + (unsigned)(lx + ly);
      sv[0] = *elem(sp, o);
      sv[1] = *elem(sp, bz0 + (unsigned)fz);
      sv[2] = *elem(sp, bz0 + (unsigned)(fz == 0 ? 0 : LZ - fz));
    } else {
      sv[0] = *elem(sp, o);
      sv[1] = (sx * sy) * *elem(sp, oct32 + o);
      sv[2] = sx * *elem(sp, 2 * oct32 + o);
      sv[3] = *elem(sp, 3 * oct32 + o);
      sv[4] = sy * *elem(sp, 4 * oct32 + o);
      sv[5] = *elem(sp, 5 * oct32 + o);
    }
  };
  cx<R> pre[G::PF ? NF : 1][NS];
  if constexpr (G::PF) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int fz = j0 + f * NFT;
      if (cvalid && fz <= HZ) spec_at(fz, pre[f]);
    }
  }

  // forward along z into the component's LDS slot
  // first-stage element n = t + (a constant of the unrolled stage): offsets
  // split into a per-thread part and a uniform part
  const unsigned toff = coff + (unsigned)t * plane;
  auto ldg = [&](int n) -> cx<R> {
    return n < nz ? *elem(wsys, toff + (unsigned)(n - t) * plane) : czero<R>();
  };
  auto sts = [&](int k, cx<R> v) { slot[k * ZP] = v; };
  fft_pencil<R, LZ, T, -1, false, true>(ldg, sts, slot, ZP, t, valid, a.tw);

  // Q(q) = S(q) X(q), S symmetric 3x3 from the octant with parity signs
  if constexpr (K == 1) if (cvalid) {
    cx<R>* e0 = lds + pp;
    const cx<R> cbx = conj(bx), cby = conj(by);
    auto roof = [&](cx<R>* e, cx<R> gq, cx<R> bz) {
      const cx<R> X = e[0], Y = e[LZ * ZP], Z = e[2 * LZ * ZP];
      const cx<R> d = bx * X + by * Y + bz * Z;   // divergence
      e[0] = gq * (X - cbx * d);
      e[LZ * ZP] = gq * (Y - cby * d);
      e[2 * LZ * ZP] = gq * (Z - conj(bz) * d);
    };
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int fz = j0 + f * NFT;
      if (fz > HZ) break;
      cx<R> sl[NS];
      const cx<R>* sv = sl;
      if constexpr (G::PF)
        sv = pre[f];
      else
        spec_at(fz, sl);
      roof(e0 + fz * ZP, sv[0], sv[1]);
      const int qz2 = LZ - fz;
      if (fz > 0 && qz2 != fz) roof(e0 + qz2 * ZP, sv[0], sv[2]);
    }
  }
  if constexpr (K == 0) if (cvalid) {
    cx<R>* e0 = lds + pp;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int fz = j0 + f * NFT;
      if (fz > HZ) break;
      cx<R> sl[NS];
      const cx<R>* sv = sl;
      if constexpr (G::PF)
        sv = pre[f];
      else
        spec_at(fz, sl);
      const cx<R> sxx = sv[0], sxy = sv[1], sxz = sv[2], syy = sv[3], syz = sv[4], szz = sv[5];
      {
        cx<R>* e = e0 + fz * ZP;   // qz = fz: sz = +1
        const cx<R> X = e[0], Y = e[LZ * ZP], Z = e[2 * LZ * ZP];
        e[0] = sxx * X + sxy * Y + sxz * Z;
        e[LZ * ZP] = sxy * X + syy * Y + syz * Z;
        e[2 * LZ * ZP] = sxz * X + syz * Y + szz * Z;
      }
      const int qz2 = LZ - fz;
      if (fz > 0 && qz2 != fz) {   // qz = LZ - fz: sz = -1
        cx<R>* e = e0 + qz2 * ZP;
        const cx<R> X = e[0], Y = e[LZ * ZP], Z = e[2 * LZ * ZP];
        e[0] = sxx * X + sxy * Y - sxz * Z;
        e[LZ * ZP] = sxy * X + syy * Y - syz * Z;
        e[2 * LZ * ZP] = szz * Z - sxz * X - syz * Y;
      }
    }
  }
  __syncthreads();
  // inverse along z, cropped to nz
  auto lds_ld = [&](int n) -> cx<R> { return slot[n * ZP]; };
  auto stg = [&](int k, cx<R> v) {
    if (k < nz) *elem(wsys, toff + (unsigned)(k - t) * plane) = v;
  };
  fft_pencil<R, LZ, T, +1, true, false>(lds_ld, stg, slot, ZP, t, valid, a.tw);
}

// ------------------------------------------------------------------ launchers
#define VIE_L_CASES(F)                                                                                    \
  F(1) F(2) F(3) F(4) F(6) F(8) F(12) F(16) F(24) F(32) F(36) F(48) F(64) F(72) F(96) F(128) F(144) F(192) F(256) \
      F(288) F(384) F(512)

[[noreturn]] static void bad_length(const char* what, int L) {
  throw std::runtime_error(std::string("unsupported FFT length for ") + what + ": " + std::to_string(L));
}

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

template <typename R>
static void launch_row_fwd(int L, const RowArgs<R>& a, int nsys, hipStream_t s) {
  switch (L) {
#define C(l)                                                                   \
  case l: {                                                                    \
    using G = Geo<R, l>;                                                       \
    const int rows = 3 * a.nz * a.ny, tiles = (rows + G::ROWP - 1) / G::ROWP;  \
    hipLaunchKernelGGL((k_row_fwd<R, l>), dim3(tiles * nsys), dim3(G::T * G::ROWP), 0, s, a); \
    break;                                                                     \
  }
    VIE_L_CASES(C)
#undef C
    default:
      bad_length("x pass", L);
  }
  check_launch("x forward");
}

template <typename R>
static void launch_row_inv(int L, const RowArgs<R>& a, int nsys, hipStream_t s) {
  switch (L) {
#define C(l)                                                                   \
  case l: {                                                                    \
    using G = Geo<R, l>;                                                       \
    const int rows = 3 * a.nz * a.ny, tiles = (rows + G::ROWP - 1) / G::ROWP;  \
    hipLaunchKernelGGL((k_row_inv_local<R, l>), dim3(tiles * nsys), dim3(G::T * G::ROWP), 0, s, a); \
    break;                                                                     \
  }
    VIE_L_CASES(C)
#undef C
    default:
      bad_length("x pass", L);
  }
  check_launch("x inverse");
}

template <typename R, int DIR>
static void launch_col(int L, const ColArgs<R>& a, hipStream_t s) {
  switch (L) {
#define C(l)                                                                        \
  case l: {                                                                         \
    using G = Geo<R, l>;                                                            \
    const int64_t cols = (int64_t)a.outer * a.inner;                                \
    const int64_t tiles = (cols + G::COLP - 1) / G::COLP;                           \
    hipLaunchKernelGGL((k_col<R, l, DIR>), dim3((unsigned)(tiles * a.nsys)), dim3(G::TC * G::COLP), 0, s, a); \
    break;                                                                          \
  }
    VIE_L_CASES(C)
#undef C
    default:
      bad_length("column pass", L);
  }
  check_launch("column pass");
}

constexpr int kZVariants = kZPassVariants;   // 0, 2, 3, 4: column sets; 1: mirror columns

template <typename R, int L, int V>
static void launch_zcol(const ZArgs<R>& a, int nsys, hipStream_t s) {
  using G = ZColGeo<R, L, V>;
  const int cols = a.ly * a.lx;
  const int blocks = ((cols + G::ZP - 1) / G::ZP) * nsys;
  if (a.rooftop)
    hipLaunchKernelGGL((k_zconv_col<R, L, V, 1>), dim3(blocks), dim3(3 * G::TZ * G::ZP), 0, s, a);
  else
    hipLaunchKernelGGL((k_zconv_col<R, L, V, 0>), dim3(blocks), dim3(3 * G::TZ * G::ZP), 0, s, a);
}

template <typename R>
static void launch_zconv(int L, const ZArgs<R>& a, int nsys, hipStream_t s) {
  const int nfy = nfold(a.ly), nfx = nfold(a.lx);
  switch (L) {
#define C(l)                                                                                      \
  case l: {                                                                                       \
    if (a.variant == 1) {                                                                         \
      if (a.rooftop) throw std::runtime_error("z pass: no mirror-column variant for rooftop spectra"); \
      using G = ZGeo<R, l>;                                                                       \
      const int blocks = nfy * ((nfx + G::ZP - 1) / G::ZP) * nsys;                                \
      hipLaunchKernelGGL((k_zconv_mirror<R, l>), dim3(blocks), dim3(3 * G::T * G::ZP), 0, s, a);  \
    } else if (l < 32 || a.variant == 0) {                                                        \
      launch_zcol<R, l, 0>(a, nsys, s);                                                           \
    } else if (a.variant == 2) {                                                                  \
      launch_zcol<R, l, (l < 32 ? 0 : 2)>(a, nsys, s);                                            \
    } else if (a.variant == 3) {                                                                  \
      launch_zcol<R, l, (l < 32 ? 0 : 3)>(a, nsys, s);                                            \
    } else {                                                                                      \
      launch_zcol<R, l, (l < 32 ? 0 : 4)>(a, nsys, s);                                            \
    }                                                                                             \
    break;                                                                                        \
  }
    VIE_L_CASES(C)
#undef C
    default:
      bad_length("z pass", L);
  }
  check_launch("z pass");
}

#define VIE_PLANE_CASES(F) F(8) F(12) F(16) F(24) F(32) F(48) F(64)

bool plane_supported(int lx, int ly) {
  if (lx != ly) return false;
#define C(l) \
  if (lx == l) return true;
  VIE_PLANE_CASES(C)
#undef C
  return false;
}

template <typename R, int L, int PV>
static void launch_plane_pv(bool fwd, const RowArgs<R>& a, int nsys, hipStream_t s) {
  using G = PlaneGeo<R, L, PV>;
  const int tiles = (3 * a.nz + G::NPL - 1) / G::NPL;
  if (fwd)
    hipLaunchKernelGGL((k_plane_fwd<R, L, PV>), dim3(tiles * nsys), dim3(G::BT), 0, s, a);
  else
    hipLaunchKernelGGL((k_plane_inv_local<R, L, PV>), dim3(tiles * nsys), dim3(G::BT), 0, s, a);
}

template <typename R>
static void launch_plane(bool fwd, int L, int pv, const RowArgs<R>& a, int nsys, hipStream_t s) {
  if (pv < 0 || pv >= kPlaneVariants) throw std::runtime_error("plane variant out of range");
  // udiv_m's range: element indices below 16 nx ny planes' worth, row
  // indices below 16 ny, plane indices below 3 nz
  const uint64_t pe = (uint64_t)a.nx * (uint64_t)a.ny;
  if (16 * pe * pe >= (1ull << 32) || 16 * (uint64_t)a.ny * a.ny >= (1ull << 32) || 3 * (uint64_t)a.nz * a.nz >= (1ull << 32))
    throw std::runtime_error("plane pass: box too large for its index arithmetic");
  switch (L) {
#define C(l)                                                 \
  case l: {                                                  \
    if (pv == 0)                                             \
      launch_plane_pv<R, l, 0>(fwd, a, nsys, s);             \
    else if (pv == 1)                                        \
      launch_plane_pv<R, l, 1>(fwd, a, nsys, s);             \
    else                                                     \
      launch_plane_pv<R, l, 2>(fwd, a, nsys, s);             \
    break;                                                   \
  }
    VIE_PLANE_CASES(C)
#undef C
    default:
      bad_length("plane pass", L);
  }
  check_launch("plane pass");
}

static void mark(hipEvent_t* ev, int i, hipStream_t s) {
  if (ev && hipEventRecord(ev[i], s) != hipSuccess) throw std::runtime_error("hipEventRecord failed");
}

template <typename R>
static RowArgs<R> row_args(const MvmBatch<R>& b, const KBatch* k, const FuseArgs& f, const c128* x, c128* y,
                           bool mask_input) {
  RowArgs<R> ra{};
  ra.nx = b.nx;
  ra.ny = b.ny;
  ra.nz = b.nz;
  ra.lx = b.lx;
  ra.ly = b.ly;
  ra.vstride = b.vstride;
  ra.cstride = b.cstride;
  ra.wstride = b.wstride;
  ra.x = x;
  ra.y = y;
  ra.chi_inv = b.chi_inv;
  ra.work = b.work;
  ra.status = b.status;
  ra.tw = b.tw->table[b.lx];
  ra.mask_input = mask_input ? 1 : 0;
  ra.chi3 = b.rooftop;
  ra.m_pe = div_magic(b.nx * b.ny);
  ra.m_nx = div_magic(b.nx);
  ra.m_ny = div_magic(b.ny);
  ra.m_nz = div_magic(b.nz);
  ra.scale = 1.0 / ((double)b.lx * (double)b.ly * (double)b.lz);
  ra.r = f.r;
  ra.p = f.p;
  ra.v = f.v;
  ra.rhat = f.rhat;
  ra.s = f.s;
  if (k) ra.k = *k;
  return ra;
}

template <typename R>
void mvm_pass1(const MvmBatch<R>& b, const KBatch* k, const FuseArgs& f, const c128* x, bool mask_input,
               hipStream_t s) {
  if (b.nsys <= 0) return;
  if (f.in_mode == 0 && !x) throw std::runtime_error("mvm_pass1: missing input");
  if (f.in_mode != 0 && (!k || !f.r || !f.v || !f.p))
    throw std::runtime_error("mvm_pass1: missing fused vectors");
  RowArgs<R> ra = row_args<R>(b, k, f, x, nullptr, mask_input);
  ra.in_mode = f.in_mode;
  if (b.plane)
    launch_plane<R>(true, b.lx, b.pvariant, ra, b.nsys, s);
  else
    launch_row_fwd<R>(b.lx, ra, b.nsys, s);
}

template <typename R>
void mvm_mid(const MvmBatch<R>& b, hipStream_t s) {
  if (b.nsys <= 0) return;
  ColArgs<R> ca{};
  ca.data = b.work;
  ca.outer = 3 * b.nz;
  ca.inner = b.lx;
  ca.n_in = b.ny;
  ca.n_out = b.ly;
  ca.stride = b.wstride;
  ca.status = b.status;
  ca.tw = b.tw->table[b.ly];
  ca.nsys = b.nsys;
  if (!b.plane) launch_col<R, -1>(b.ly, ca, s);

  ZArgs<R> za{};
  za.nz = b.nz;
  za.ly = b.ly;
  za.lx = b.lx;
  za.variant = b.zvariant;
  za.wstride = b.wstride;
  za.sstride = b.sstride;
  za.work = b.work;
  za.spec = b.spec;
  za.spec_tab = b.spec_tab;
  za.rooftop = b.rooftop;
  za.status = b.status;
  za.tw = b.tw->table[b.lz];
  launch_zconv<R>(b.lz, za, b.nsys, s);

  ca.n_in = b.ly;
  ca.n_out = b.ny;
  if (!b.plane) launch_col<R, +1>(b.ly, ca, s);
}

template <typename R>
void mvm_pass5(const MvmBatch<R>& b, const KBatch* k, const FuseArgs& f, const c128* x, c128* y, hipStream_t s) {
  if (b.nsys <= 0) return;
  if (!x || !y) throw std::runtime_error("mvm_pass5: missing vectors");
  if ((f.out_mode == 1 || f.out_mode == 2 || f.out_mode == 4) && !k)
    throw std::runtime_error("mvm_pass5: missing Krylov batch");
  if (((f.out_mode == 1 || f.out_mode == 3) && !f.rhat) || ((f.out_mode == 2 || f.out_mode == 4) && !f.s))
    throw std::runtime_error("mvm_pass5: missing fused vectors");
  RowArgs<R> ra = row_args<R>(b, k, f, x, y, false);
  ra.out_mode = f.out_mode;
  if (b.plane)
    launch_plane<R>(false, b.lx, b.pvariant, ra, b.nsys, s);
  else
    launch_row_inv<R>(b.lx, ra, b.nsys, s);
}

template <typename R>
void mvm(const MvmBatch<R>& b, const c128* x, c128* y, bool mask_input, hipStream_t s, hipEvent_t* ev) {
  if (b.nsys <= 0) return;
  const FuseArgs none{0, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
  mark(ev, 0, s);
  mvm_pass1<R>(b, nullptr, none, x, mask_input, s);
  mark(ev, 1, s);
  if (!ev) {
    mvm_mid<R>(b, s);
  } else {
    // per-pass events for measurement
    ColArgs<R> ca{};
    ca.data = b.work;
    ca.outer = 3 * b.nz;
    ca.inner = b.lx;
    ca.n_in = b.ny;
    ca.n_out = b.ly;
    ca.stride = b.wstride;
    ca.status = b.status;
    ca.tw = b.tw->table[b.ly];
    ca.nsys = b.nsys;
    if (!b.plane) launch_col<R, -1>(b.ly, ca, s);
    mark(ev, 2, s);
    ZArgs<R> za{};
    za.nz = b.nz;
    za.ly = b.ly;
    za.lx = b.lx;
    za.variant = b.zvariant;
    za.wstride = b.wstride;
    za.sstride = b.sstride;
    za.work = b.work;
    za.spec = b.spec;
    za.spec_tab = b.spec_tab;
    za.rooftop = b.rooftop;
    za.status = b.status;
    za.tw = b.tw->table[b.lz];
    launch_zconv<R>(b.lz, za, b.nsys, s);
    mark(ev, 3, s);
    ca.n_in = b.ly;
    ca.n_out = b.ny;
    if (!b.plane) launch_col<R, +1>(b.ly, ca, s);
    mark(ev, 4, s);
  }
  mvm_pass5<R>(b, nullptr, none, x, y, s);
  mark(ev, 5, s);
}

// Autotuning of the z pass: time each variant on the batch's own work buffer
// (contents are overwritten; call before the buffer holds live data) and
// return the faster one.
template <typename R>
int tune_zpass(const MvmBatch<R>& b, hipStream_t s, float* ms_out) {
  if (ms_out)
    for (int v = 0; v < kZPassVariants; ++v) ms_out[v] = -1.0f;
  if (b.nsys <= 0) return 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  {
    ApiShared api;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      throw std::runtime_error("hipEventCreate failed");
  }
  float best = 1e30f;
  int best_v = 0;
  for (int v = 0; v < kZVariants; ++v) {
    if (v >= 2 && b.lz < 32) break;   // short columns: variants 0 and 1 only
    if (v == 1 && b.rooftop) continue;   // column sets only
    ZArgs<R> za{};
    za.nz = b.nz;
    za.ly = b.ly;
    za.lx = b.lx;
    za.variant = v;
    za.wstride = b.wstride;
    za.sstride = b.sstride;
    za.work = b.work;
    za.spec = b.spec;
    za.spec_tab = b.spec_tab;
    za.rooftop = b.rooftop;
    za.status = nullptr;
    za.tw = b.tw->table[b.lz];
    launch_zconv<R>(b.lz, za, b.nsys, s);   // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < 3; ++r) launch_zconv<R>(b.lz, za, b.nsys, s);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms_out) ms_out[v] = ms;
    if (ms < best) {
      best = ms;
      best_v = v;
    }
  }
  {
    ApiShared api;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return best_v;
}
template int tune_zpass<float>(const MvmBatch<float>&, hipStream_t, float*);
template int tune_zpass<double>(const MvmBatch<double>&, hipStream_t, float*);

// Autotuning of the plane kernels (batches with b.plane): time the forward
// and inverse plane passes of each variant (plain product, every system
// active) on the batch's own work buffer, x as input and y as output (all
// overwritten; call before they hold live data); returns the fastest.
template <typename R>
int tune_plane(const MvmBatch<R>& b, const c128* x, c128* y, hipStream_t s, float* ms_out) {
  if (ms_out)
    for (int v = 0; v < kPlaneVariants; ++v) ms_out[v] = -1.0f;
  if (b.nsys <= 0 || !b.plane) return 0;
  if (!x || !y) throw std::runtime_error("tune_plane: missing vectors");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  {
    ApiShared api;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      throw std::runtime_error("hipEventCreate failed");
  }
  MvmBatch<R> bb = b;
  bb.status = nullptr;
  const FuseArgs none{0, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
  float best = 1e30f;
  int best_v = 0;
  for (int v = 0; v < kPlaneVariants; ++v) {
    bb.pvariant = v;
    auto run = [&]() {
      mvm_pass1<R>(bb, nullptr, none, x, false, s);
      mvm_pass5<R>(bb, nullptr, none, x, y, s);
    };
    run();   // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < 3; ++r) run();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms_out) ms_out[v] = ms;
    if (ms < best) {
      best = ms;
      best_v = v;
    }
  }
  {
    ApiShared api;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return best_v;
}

#define VIE_MVM_INST(R)                                                                                           \
  template void mvm<R>(const MvmBatch<R>&, const c128*, c128*, bool, hipStream_t, hipEvent_t*);                  \
  template void mvm_pass1<R>(const MvmBatch<R>&, const KBatch*, const FuseArgs&, const c128*, bool, hipStream_t); \
  template void mvm_mid<R>(const MvmBatch<R>&, hipStream_t);                                                     \
  template void mvm_pass5<R>(const MvmBatch<R>&, const KBatch*, const FuseArgs&, const c128*, c128*, hipStream_t);
VIE_MVM_INST(float)
VIE_MVM_INST(double)
#undef VIE_MVM_INST
template int tune_plane<float>(const MvmBatch<float>&, const c128*, c128*, hipStream_t, float*);
template int tune_plane<double>(const MvmBatch<double>&, const c128*, c128*, hipStream_t, float*);

int64_t mvm_row_tiles(int lx, int nz, int ny) {
  const int64_t rows = 3 * (int64_t)nz * ny;
  if (plane_supported(lx, lx)) {   // plane kernels: at most one workgroup per plane
    switch (lx) {
#define C(l)                                                                                 \
  case l: {                                                                                  \
    const int rp = cmin(Geo<float, l>::ROWP, Geo<double, l>::ROWP);                          \
    return std::max<int64_t>((rows + rp - 1) / rp, 3 * (int64_t)nz);                        \
  }
      VIE_PLANE_CASES(C)
#undef C
    }
  }
  switch (lx) {
#define C(l)                                                                            \
  case l: {                                                                             \
    const int rp = cmin(Geo<float, l>::ROWP, Geo<double, l>::ROWP);                     \
    return (rows + rp - 1) / rp;                                                        \
  }
    VIE_L_CASES(C)
#undef C
    default:
      bad_length("x pass", lx);
  }
}

// ------------------------------------------------------------------ spectra setup
// T(m) of the discretised dyadic Green's function (eq. (1) with the scalar
// Green's function after it), collocated voxels: for m != 0 the dyadic
// (I + grad grad / k0^2) g sampled at the centre separation R times
// k0^2 dV,
//   g [ (1 - j/u - 1/u^2) I + (3/u^2 + 3j/u - 1) Rhat Rhat ],  u = k0 |R|;
// for m = 0 the integral of k0^2 G over the equal-volume sphere,
//   ((2 (1 + j k0 a) exp(-j k0 a) - 3) / 3) I,  a = (3 dV / 4 pi)^(1/3).
// Slot s of an axis of n voxels embedded in length L holds offset s (s < n),
// s - L (s > L - n), nothing otherwise.  Output [6][lz][ly][lx], component
// order xx, xy, xz, yy, yz, zz.
__device__ __forceinline__ int slot_offset(int s, int n, int L, bool* ok) {
  if (s < n) {
    *ok = true;
    return s;
  }
  if (s > L - n) {
    *ok = true;
    return s - L;
  }
  *ok = false;
  return 0;
}

__global__ void k_green_embed(c128* out, int nx, int ny, int nz, int lx, int ly, int lz, double dx, double dy,
                              double dz, double k0) {
  const int64_t npts = (int64_t)lx * ly * lz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  const int sx = (int)(i % lx);
  const int sy = (int)((i / lx) % ly);
  const int sz = (int)(i / ((int64_t)lx * ly));
  bool okx, oky, okz;
  const int mx = slot_offset(sx, nx, lx, &okx);
  const int my = slot_offset(sy, ny, ly, &oky);
  const int mz = slot_offset(sz, nz, lz, &okz);
  double t[6] = {0, 0, 0, 0, 0, 0};
  double ti[6] = {0, 0, 0, 0, 0, 0};
  if (okx && oky && okz) {
    const double dV = dx * dy * dz;
    if (mx == 0 && my == 0 && mz == 0) {
      const double a = cbrt(3.0 * dV / (4.0 * M_PI));
      const double x = k0 * a;
      double sn, cs;
      sincos(x, &sn, &cs);
      // (1 + j x) exp(-j x) = (cos x + x sin x) + j (x cos x - sin x)
      const double re = (2.0 * (cs + x * sn) - 3.0) / 3.0;
      const double im = 2.0 * (x * cs - sn) / 3.0;
      t[0] = t[3] = t[5] = re;
      ti[0] = ti[3] = ti[5] = im;
    } else {
      const double Rx = mx * dx, Ry = my * dy, Rz = mz * dz;
      const double R = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
      const double u = k0 * R;
      double sn, cs;
      sincos(u, &sn, &cs);
      const double inv4piR = 1.0 / (4.0 * M_PI * R);
      // pref = k0^2 dV g = k0^2 dV exp(-j u) / (4 pi R)
      const double pr = k0 * k0 * dV * cs * inv4piR, pi = -k0 * k0 * dV * sn * inv4piR;
      const double iu = 1.0 / u, iu2 = iu * iu;
      const double ar = 1.0 - iu2, ai = -iu;          // 1 - j/u - 1/u^2
      const double br = 3.0 * iu2 - 1.0, bi = 3.0 * iu;  // 3/u^2 + 3j/u - 1
      const double rh[3] = {Rx / R, Ry / R, Rz / R};
      const int ci[6] = {0, 0, 0, 1, 1, 2}, cj[6] = {0, 1, 2, 1, 2, 2};
      for (int c = 0; c < 6; ++c) {
        const double rr = rh[ci[c]] * rh[cj[c]];
        double fr = br * rr, fi = bi * rr;
        if (ci[c] == cj[c]) {
          fr += ar;
          fi += ai;
        }
        t[c] = pr * fr - pi * fi;
        ti[c] = pr * fi + pi * fr;
      }
    }
  }
  for (int c = 0; c < 6; ++c) out[c * npts + i] = mk<double>(t[c], ti[c]);
}

__global__ void k_extract_octant(const c128* full, c128* s64, c64* s32, int lx, int ly, int lz, int ncomp) {
  const int ox = lx / 2 + 1, oy = ly / 2 + 1, oz = lz / 2 + 1;
  const int64_t oct = (int64_t)ox * oy * oz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncomp * oct) return;
  const int c = (int)(i / oct);
  const int64_t r = i - c * oct;
  const int fx = (int)(r % ox), fy = (int)((r / ox) % oy), fz = (int)(r / ((int64_t)ox * oy));
  const c128 v = full[(int64_t)c * lx * ly * lz + ((int64_t)fz * ly + fy) * lx + fx];
  if (s64) s64[i] = v;
  if (s32) s32[i] = cvt<float>(v);
}

template <int L>
static void launch_row_full_L(c128* data, int64_t rows, const c128* tw, hipStream_t s) {
  using G = Geo<double, L>;
  const int64_t blocks = (rows + G::ROWP - 1) / G::ROWP;
  hipLaunchKernelGGL((k_row_full<double, L>), dim3((unsigned)blocks), dim3(G::T * G::ROWP), 0, s, data, rows, tw);
}

static void launch_row_full(int L, c128* data, int64_t rows, const c128* tw, hipStream_t s) {
  switch (L) {
#define C(l)                                  \
  case l:                                     \
    launch_row_full_L<l>(data, rows, tw, s); \
    break;
    VIE_L_CASES(C)
#undef C
    default:
      bad_length("setup x pass", L);
  }
  check_launch("setup x pass");
}

void green_spectra(int nx, int ny, int nz, int lx, int ly, int lz, double dx, double dy, double dz, double k0,
                   c128* scratch, c128* spec64, c64* spec32, const TwiddleSet<double>& tw, hipStream_t s) {
  const int64_t npts = (int64_t)lx * ly * lz;
  hipLaunchKernelGGL(k_green_embed, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, scratch, nx, ny, nz, lx,
                     ly, lz, dx, dy, dz, k0);
  check_launch("green embed");
  launch_row_full(lx, scratch, 6 * (int64_t)ly * lz, tw.table[lx], s);
  ColArgs<double> ca{};
  ca.data = scratch;
  ca.outer = 6 * lz;
  ca.inner = lx;
  ca.n_in = ly;
  ca.n_out = ly;
  ca.stride = 0;
  ca.status = nullptr;
  ca.tw = tw.table[ly];
  ca.nsys = 1;
  launch_col<double, -1>(ly, ca, s);
  ca.outer = 6;
  ca.inner = lx * ly;
  ca.n_in = lz;
  ca.n_out = lz;
  ca.tw = tw.table[lz];
  launch_col<double, -1>(lz, ca, s);
  const int64_t oct = 6 * (int64_t)(lx / 2 + 1) * (ly / 2 + 1) * (lz / 2 + 1);
  hipLaunchKernelGGL(k_extract_octant, dim3((unsigned)((oct + 255) / 256)), dim3(256), 0, s, scratch, spec64, spec32,
                     lx, ly, lz, 6);
  check_launch("octant");
}

// Rooftop discretisation (Sec. II-A, eq. (5)): the scalar kernel
// k0^2 dV g~(m), g~ the scalar Green's function at the centre separation for
// m != 0 and its mean over the sphere of the cell's volume at m = 0,
//   k0^2 dV g~(0) = (1 + j k0 a) exp(-j k0 a) - 1,  a = (3 dV / 4 pi)^(1/3)
// (the radial integral of r exp(-j k0 r) from 0 to a).  Same slot layout as
// k_green_embed, one component.
__global__ void k_green_embed_scalar(c128* out, int nx, int ny, int nz, int lx, int ly, int lz, double dx, double dy,
                                     double dz, double k0) {
  const int64_t npts = (int64_t)lx * ly * lz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  const int sx = (int)(i % lx);
  const int sy = (int)((i / lx) % ly);
  const int sz = (int)(i / ((int64_t)lx * ly));
  bool okx, oky, okz;
  const int mx = slot_offset(sx, nx, lx, &okx);
  const int my = slot_offset(sy, ny, ly, &oky);
  const int mz = slot_offset(sz, nz, lz, &okz);
  double re = 0.0, im = 0.0;
  if (okx && oky && okz) {
    const double dV = dx * dy * dz;
    if (mx == 0 && my == 0 && mz == 0) {
      const double x = k0 * cbrt(3.0 * dV / (4.0 * M_PI));
      double sn, cs;
      sincos(x, &sn, &cs);
      re = cs + x * sn - 1.0;
      im = x * cs - sn;
    } else {
      const double Rx = mx * dx, Ry = my * dy, Rz = mz * dz;
      const double R = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
      double sn, cs;
      sincos(k0 * R, &sn, &cs);
      const double f = k0 * k0 * dV / (4.0 * M_PI * R);
      re = f * cs;
      im = -f * sn;
    }
  }
  out[i] = mk<double>(re, im);
}

// b_j(q) = (1 - exp(-2 pi i q / L_j)) / (k0 d_j) for q in [0, L_j), the three
// axes one after the other: 1 - cos t = 2 sin^2(t / 2) keeps the small
// symbols accurate.
__global__ void k_diff_symbols(c128* s64, c64* s32, int lx, int ly, int lz, double dx, double dy, double dz,
                               double k0) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= lx + ly + lz) return;
  int q = i, L = lx;
  double d = dx;
  if (q >= lx) {
    q -= lx;
    L = ly;
    d = dy;
    if (q >= ly) {
      q -= ly;
      L = lz;
      d = dz;
    }
  }
  double sh, ch, sf, cf;
  sincospi((double)q / L, &sh, &ch);
  sincospi(2.0 * q / L, &sf, &cf);
  const c128 b = mk<double>(2.0 * sh * sh / (k0 * d), sf / (k0 * d));
  if (s64) s64[i] = b;
  if (s32) s32[i] = cvt<float>(b);
}

void green_spectrum_rooftop(int nx, int ny, int nz, int lx, int ly, int lz, double dx, double dy, double dz,
                            double k0, c128* scratch, c128* spec64, c64* spec32, const TwiddleSet<double>& tw,
                            hipStream_t s) {
  const int64_t npts = (int64_t)lx * ly * lz;
  hipLaunchKernelGGL(k_green_embed_scalar, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, scratch, nx, ny,
                     nz, lx, ly, lz, dx, dy, dz, k0);
  check_launch("rooftop embed");
  launch_row_full(lx, scratch, (int64_t)ly * lz, tw.table[lx], s);
  ColArgs<double> ca{};
  ca.data = scratch;
  ca.outer = lz;
  ca.inner = lx;
  ca.n_in = ly;
  ca.n_out = ly;
  ca.stride = 0;
  ca.status = nullptr;
  ca.tw = tw.table[ly];
  ca.nsys = 1;
  launch_col<double, -1>(ly, ca, s);
  ca.outer = 1;
  ca.inner = lx * ly;
  ca.n_in = lz;
  ca.n_out = lz;
  ca.tw = tw.table[lz];
  launch_col<double, -1>(lz, ca, s);
  const int64_t oct = (int64_t)(lx / 2 + 1) * (ly / 2 + 1) * (lz / 2 + 1);
  hipLaunchKernelGGL(k_extract_octant, dim3((unsigned)((oct + 255) / 256)), dim3(256), 0, s, scratch, spec64, spec32,
                     lx, ly, lz, 1);
  check_launch("rooftop octant");
  hipLaunchKernelGGL(k_diff_symbols, dim3((unsigned)((lx + ly + lz + 255) / 256)), dim3(256), 0, s,
                     spec64 ? spec64 + oct : nullptr, spec32 ? spec32 + oct : nullptr, lx, ly, lz, dx, dy, dz, k0);
  check_launch("rooftop symbols");
}

}  // namespace vie
