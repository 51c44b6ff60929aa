// Device FFT core: small DFTs in registers and a compile-time mixed-radix
// Stockham pipeline for one pencil.
//
// The 3-D convolution that accelerates the VIE product (the Toeplitz + FFT
// statement of Sec. I of the paper) is built from 1-D pencils of length
// L = 2^a 3^b.  A pencil is transformed by a chain of radix stages
// (autosort Stockham form): stage s with radix R and p = product of the
// earlier radices reads element b + m*L/R (m < R) for butterfly b, twiddles
// it by w^(m k) with w = exp(-+2 pi i / (p R)), k = b mod p, applies a
// length-R DFT and writes element (b - k) R + k + m p.  The first stage reads
// through a caller-supplied loader (HBM, coalesced across threads) and the
// last stage writes through a caller-supplied storer; the stages in between
// exchange data through LDS.  DIR = -1 is the forward transform
// exp(-2 pi i k n / L), DIR = +1 the unnormalised inverse.
#pragma once
#include "cx.h"

namespace vie {

// ---------------------------------------------------------------- small DFTs
template <int DIR, typename R>
__host__ __device__ __forceinline__ cx<R> rot_q(cx<R> a) {  // a * exp(DIR * i pi / 2)
  return DIR < 0 ? mul_mi(a) : mul_i(a);
}

template <int RAD, int DIR, typename R>
__host__ __device__ __forceinline__ void dft(cx<R>* v) {
  if constexpr (RAD == 1) {
  } else if constexpr (RAD == 2) {
    cx<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (RAD == 3) {
    const R c = R(-0.5);
    const R s = DIR < 0 ? R(-0.86602540378443864676) : R(0.86602540378443864676);
    cx<R> t1 = v[1] + v[2], t2 = v[1] - v[2];
    cx<R> m = v[0] + c * t1;
    cx<R> j = mk<R>(-s * t2.y, s * t2.x);  // i * s * t2
    v[0] = v[0] + t1;
    v[1] = m + j;
    v[2] = m - j;
  } else if constexpr (RAD == 4) {
    cx<R> e0 = v[0] + v[2], e1 = v[0] - v[2];
    cx<R> o0 = v[1] + v[3], o1 = rot_q<DIR>(v[1] - v[3]);
    v[0] = e0 + o0;
    v[2] = e0 - o0;
    v[1] = e1 + o1;
    v[3] = e1 - o1;
  } else if constexpr (RAD == 8) {
    cx<R> e[4] = {v[0], v[2], v[4], v[6]};
    cx<R> o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, DIR>(e);
    dft<4, DIR>(o);
    const R h = R(0.70710678118654752440);
    const R sg = DIR < 0 ? R(-1) : R(1);
    cx<R> t1 = mk<R>(h * (o[1].x - sg * o[1].y), h * (o[1].y + sg * o[1].x));       // w8^1
    cx<R> t2 = rot_q<DIR>(o[2]);                                                    // w8^2
    cx<R> t3 = mk<R>(h * (-o[3].x - sg * o[3].y), h * (-o[3].y + sg * o[3].x));     // w8^3
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + t1;
    v[5] = e[1] - t1;
    v[2] = e[2] + t2;
    v[6] = e[2] - t2;
    v[3] = e[3] + t3;
    v[7] = e[3] - t3;
  } else if constexpr (RAD == 16) {
    cx<R> e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<8, DIR>(e);
    dft<8, DIR>(o);
    const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173);
    const R h = R(0.70710678118654752440);
    const R sg = DIR < 0 ? R(-1) : R(1);
    // w16^k = cos(2 pi k/16) + sg * i sin(2 pi k/16)
    const R cr[8] = {R(1), c1, h, s1, R(0), -s1, -h, -c1};
    const R ci[8] = {R(0), s1, h, c1, R(1), c1, h, s1};
    v[0] = e[0] + o[0];
    v[8] = e[0] - o[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      cx<R> t;
      if (k == 4) {
        t = rot_q<DIR>(o[4]);
      } else {
        const R wr = cr[k], wi = sg * ci[k];
        t = mk<R>(o[k].x * wr - o[k].y * wi, o[k].x * wi + o[k].y * wr);
      }
      v[k] = e[k] + t;
      v[k + 8] = e[k] - t;
    }
  } else {
    static_assert(RAD == 2, "unsupported radix");
  }
}

// ---------------------------------------------------------------- plans
template <int... Rs>
struct Radices {};

template <int L>
struct Plan;
template <> struct Plan<1> { using type = Radices<>; };
template <> struct Plan<2> { using type = Radices<2>; };
template <> struct Plan<3> { using type = Radices<3>; };
template <> struct Plan<4> { using type = Radices<4>; };
template <> struct Plan<6> { using type = Radices<2, 3>; };
template <> struct Plan<8> { using type = Radices<8>; };
template <> struct Plan<12> { using type = Radices<4, 3>; };
template <> struct Plan<16> { using type = Radices<16>; };
template <> struct Plan<24> { using type = Radices<8, 3>; };
template <> struct Plan<32> { using type = Radices<8, 4>; };
template <> struct Plan<36> { using type = Radices<4, 3, 3>; };
template <> struct Plan<48> { using type = Radices<16, 3>; };
template <> struct Plan<64> { using type = Radices<8, 8>; };
template <> struct Plan<72> { using type = Radices<8, 3, 3>; };
template <> struct Plan<96> { using type = Radices<8, 4, 3>; };
template <> struct Plan<128> { using type = Radices<16, 8>; };
template <> struct Plan<144> { using type = Radices<16, 3, 3>; };
template <> struct Plan<192> { using type = Radices<16, 4, 3>; };
template <> struct Plan<256> { using type = Radices<16, 16>; };
template <> struct Plan<288> { using type = Radices<8, 4, 3, 3>; };
template <> struct Plan<384> { using type = Radices<16, 8, 3>; };
template <> struct Plan<512> { using type = Radices<8, 8, 8>; };

template <class Rad>
struct RadInfo;
template <>
struct RadInfo<Radices<>> {
  static constexpr int nstages = 0;
  static constexpr int rmin = 1 << 30;
  static constexpr int rmax = 1;
};
template <int R0, int... Rs>
struct RadInfo<Radices<R0, Rs...>> {
  static constexpr int nstages = 1 + sizeof...(Rs);
  static constexpr int rmin = R0 < RadInfo<Radices<Rs...>>::rmin ? R0 : RadInfo<Radices<Rs...>>::rmin;
  static constexpr int rmax = R0 > RadInfo<Radices<Rs...>>::rmax ? R0 : RadInfo<Radices<Rs...>>::rmax;
};

// Largest number of butterflies of any stage = L / smallest radix; a pencil
// uses at most that many threads.  With min_butterflies (L / largest radix)
// threads no thread idles in any stage; stages with more butterflies then
// give each thread several.
template <int L>
struct PlanInfo {
  using rad = typename Plan<L>::type;
  static constexpr int nstages = RadInfo<rad>::nstages;
  static constexpr int max_butterflies = nstages == 0 ? 1 : L / RadInfo<rad>::rmin;
  static constexpr int min_butterflies = nstages == 0 ? 1 : L / RadInfo<rad>::rmax;
};

// ---------------------------------------------------------------- pipeline
// Twiddle table tw[t] = exp(-2 pi i t / L), t < L, in HBM (shared, cached).
template <int DIR, typename R>
__device__ __forceinline__ cx<R> twiddle(const cx<R>* __restrict__ tw, int idx) {
  cx<R> w = tw[(unsigned)idx];   // unsigned 32-bit offset from a uniform base
  return DIR < 0 ? w : conj(w);
}

// One stage.  Threads t < T of a pencil cooperate; `lds` points at element 0
// of this pencil's LDS slot and consecutive elements are `ls` apart.  All
// threads of the workgroup must call every stage (barriers inside).
// LDLDS: the loader reads this pencil's LDS slot; STLDS: the storer writes
// it.  Then the first (last) stage separates its reads from its writes by a
// barrier, since the transform runs in place in the slot.
template <typename R, int L, int T, int DIR, int RAD, int P, bool FIRST, bool LAST, bool LDLDS, bool STLDS,
          class Load, class Store>
__device__ __forceinline__ void fft_stage(Load& ld, Store& st, cx<R>* lds, int ls, int t, bool tvalid,
                                          const cx<R>* __restrict__ tw) {
  constexpr int NB = L / RAD;
  constexpr int NPT = (NB + T - 1) / T;
  constexpr bool READS_SLOT = !FIRST || LDLDS;
  constexpr bool WRITES_SLOT = !LAST || STLDS;
  cx<R> v[NPT][RAD];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int b = t + q * T;
    if (tvalid && (NB % T == 0 || b < NB)) {
#pragma unroll
      for (int m = 0; m < RAD; ++m) {
        const int idx = b + m * NB;
        if constexpr (FIRST)
          v[q][m] = ld(idx);
        else
          v[q][m] = lds[idx * ls];
      }
    }
  }
  if constexpr (READS_SLOT && WRITES_SLOT) __syncthreads();
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int b = t + q * T;
    if (tvalid && (NB % T == 0 || b < NB)) {
      const int k = (P == 1) ? 0 : (b % P);
      if constexpr (P > 1) {
        constexpr int TS = L / (P * RAD);
#pragma unroll
        for (int m = 1; m < RAD; ++m) v[q][m] = v[q][m] * twiddle<DIR>(tw, m * k * TS);
      }
      dft<RAD, DIR>(v[q]);
      const int j = (b - k) * RAD + k;
#pragma unroll
      for (int m = 0; m < RAD; ++m) {
        if constexpr (LAST)
          st(j + m * P, v[q][m]);
        else
          lds[(j + m * P) * ls] = v[q][m];
      }
    }
  }
  if constexpr (WRITES_SLOT) __syncthreads();
}

template <typename R, int L, int T, int DIR, int P, bool FIRST, bool LDLDS, bool STLDS, class Load, class Store,
          int RAD, int... Rest>
__device__ __forceinline__ void fft_stages(Load& ld, Store& st, cx<R>* lds, int ls, int t, bool tvalid,
                                           const cx<R>* __restrict__ tw, Radices<RAD, Rest...>) {
  constexpr bool LAST = sizeof...(Rest) == 0;
  fft_stage<R, L, T, DIR, RAD, P, FIRST, LAST, LDLDS, STLDS>(ld, st, lds, ls, t, tvalid, tw);
  if constexpr (!LAST)
    fft_stages<R, L, T, DIR, P * RAD, false, LDLDS, STLDS>(ld, st, lds, ls, t, tvalid, tw, Radices<Rest...>{});
}

// Transform one pencil of length L: x_n = ld(n) (n < L) -> st(k, X_k).
// Threads t in [0, T) of the pencil take part; tvalid = false threads still
// hit the barriers but touch no data.  The pencil's LDS slot is the exchange
// buffer between stages; see fft_stage for LDLDS / STLDS.
template <typename R, int L, int T, int DIR, bool LDLDS = false, bool STLDS = false, class Load, class Store>
__device__ __forceinline__ void fft_pencil(Load ld, Store st, cx<R>* lds, int ls, int t, bool tvalid,
                                           const cx<R>* __restrict__ tw) {
  using rad = typename Plan<L>::type;
  if constexpr (RadInfo<rad>::nstages == 0) {
    if (tvalid && t == 0) st(0, ld(0));
    if constexpr (STLDS) __syncthreads();
  } else {
    fft_stages<R, L, T, DIR, 1, true, LDLDS, STLDS>(ld, st, lds, ls, t, tvalid, tw, rad{});
  }
}

}  // namespace vie
