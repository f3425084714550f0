// Batched complex FFTs of small length N held in LDS (gfx950).
//
// A workgroup transforms `cnt` sequences of length N that live in LDS at
// positions addr(t, e) (t = sequence, e = element).  Each Stockham stage of
// radix R reads all of its R-point butterflies into registers, waits at a
// barrier, then writes them back in place: one LDS buffer suffices (planes of
// 72 x 72 complex doubles use 83 KB), and the output is in natural order.
//
// Stage with radix R after sub-transforms of size P have been formed
// (P = product of earlier radices), butterfly i in [0, N/R), k = i mod P:
//     v_r = x[i + r N/R] * w_N^(r k N/(P R)),  r = 0..R-1
//     y[(i - k) R + k + r P] = sum_s v_s exp(SIGN 2 pi i r s / R)
// SIGN = -1 is the forward transform, +1 the unnormalised inverse.
#pragma once
#include "common.h"

namespace lgw {

template <int... Rs> struct RList {};

// Radix plans of the supported grid sizes (products of 2, 3, 4, 5).
template <int N> struct Plan;
template <> struct Plan<16> { using type = RList<4, 4>; };
template <> struct Plan<24> { using type = RList<4, 3, 2>; };
template <> struct Plan<32> { using type = RList<4, 4, 2>; };
template <> struct Plan<40> { using type = RList<4, 5, 2>; };
template <> struct Plan<48> { using type = RList<4, 4, 3>; };
template <> struct Plan<64> { using type = RList<4, 4, 4>; };
template <> struct Plan<72> { using type = RList<4, 3, 3, 2>; };

// --- small DFTs ----------------------------------------------------------
template <int R, int SIGN, typename T> struct Dft;

template <int SIGN, typename T> struct Dft<2, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* a) {
    cplx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  }
};

template <int SIGN, typename T> struct Dft<3, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* a) {
    const T h = T(0.5);
    const T s = T(0.86602540378443864676);   // sqrt(3)/2
    cplx<T> t1 = a[1] + a[2];
    cplx<T> t2 = a[1] - a[2];
    cplx<T> m = a[0] - h * t1;
    cplx<T> q = muli<SIGN>(s * t2);
    a[0] = a[0] + t1;
    a[1] = m + q;
    a[2] = m - q;
  }
};

template <int SIGN, typename T> struct Dft<4, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* a) {
    cplx<T> t0 = a[0] + a[2];
    cplx<T> t1 = a[0] - a[2];
    cplx<T> t2 = a[1] + a[3];
    cplx<T> t3 = muli<SIGN>(a[1] - a[3]);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
  }
};

template <int SIGN, typename T> struct Dft<5, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* a) {
    const T c1 = T(0.30901699437494742410);   // cos(2 pi / 5)
    const T c2 = T(-0.80901699437494742410);  // cos(4 pi / 5)
    const T s1 = T(0.95105651629515357212);   // sin(2 pi / 5)
    const T s2 = T(0.58778525229247312917);   // sin(4 pi / 5)
    cplx<T> t1 = a[1] + a[4], t2 = a[2] + a[3];
    cplx<T> t3 = a[1] - a[4], t4 = a[2] - a[3];
    cplx<T> A1 = a[0] + c1 * t1 + c2 * t2;
    cplx<T> A2 = a[0] + c2 * t1 + c1 * t2;
    cplx<T> B1 = muli<SIGN>(s1 * t3 + s2 * t4);
    cplx<T> B2 = muli<SIGN>(s2 * t3 - s1 * t4);
    a[0] = a[0] + t1 + t2;
    a[1] = A1 + B1;
    a[4] = A1 - B1;
    a[2] = A2 + B2;
    a[3] = A2 - B2;
  }
};

// --- one stage ----------------------------------------------------------
// TFAST: consecutive threads take consecutive sequences (use when elements
// are strided and sequences are adjacent); otherwise consecutive butterflies
// of one sequence (elements adjacent).
template <typename T, int N, int R, int P, int SIGN, int NT, int MAXCNT, bool TFAST, class Addr>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, const cplx<T>* tw, int cnt, Addr addr) {
  constexpr int M = N / R;
  constexpr int MAXB = (MAXCNT * M + NT - 1) / NT;
  constexpr int TWS = N / (P * R);
  const int tid = threadIdx.x;
  const int nb = cnt * M;
  cplx<T> v[MAXB][R];
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int b = tid + k * NT;
    if (b < nb) {
      int t, i;
      if (TFAST) { t = b % cnt; i = b / cnt; } else { i = b % M; t = b / M; }
      const int kk = i % P;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = buf[addr(t, i + r * M)];
      if (P > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[r * kk * TWS];
          if (SIGN > 0) w.y = -w.y;
          v[k][r] = v[k][r] * w;
        }
      }
      Dft<R, SIGN, T>::run(v[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int b = tid + k * NT;
    if (b < nb) {
      int t, i;
      if (TFAST) { t = b % cnt; i = b / cnt; } else { i = b % M; t = b / M; }
      const int kk = i % P;
      const int j = (i - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[addr(t, j + r * P)] = v[k][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int P, int SIGN, int NT, int MAXCNT, bool TFAST, class Addr>
__device__ __forceinline__ void fft_run(RList<>, cplx<T>*, const cplx<T>*, int, Addr) {}

template <typename T, int N, int P, int SIGN, int NT, int MAXCNT, bool TFAST, class Addr, int R0, int... Rs>
__device__ __forceinline__ void fft_run(RList<R0, Rs...>, cplx<T>* buf, const cplx<T>* tw, int cnt, Addr addr) {
  fft_stage<T, N, R0, P, SIGN, NT, MAXCNT, TFAST>(buf, tw, cnt, addr);
  fft_run<T, N, P * R0, SIGN, NT, MAXCNT, TFAST>(RList<Rs...>{}, buf, tw, cnt, addr);
}

// In-place FFTs of `cnt` (<= MAXCNT) sequences.  The caller must have synced
// the buffer before the call; the call ends with a barrier.
// tw[j] = exp(-2 pi i j / N) (forward table; the inverse conjugates it).
template <typename T, int N, int SIGN, int NT, int MAXCNT, bool TFAST, class Addr>
__device__ __forceinline__ void fft_lds(cplx<T>* buf, const cplx<T>* tw, int cnt, Addr addr) {
  fft_run<T, N, 1, SIGN, NT, MAXCNT, TFAST>(typename Plan<N>::type{}, buf, tw, cnt, addr);
}

}  // namespace lgw
