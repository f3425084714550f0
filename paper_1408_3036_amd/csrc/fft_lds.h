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

// Radix plans of the supported grid sizes: two Stockham stages N = A * B,
// each an in-register DFT (composite radices 6 = 3*2, 8 = 4*2, 9 = 3*3).
template <int N> struct Plan;
template <> struct Plan<16> { using type = RList<4, 4>; };
template <> struct Plan<24> { using type = RList<6, 4>; };
template <> struct Plan<32> { using type = RList<8, 4>; };
template <> struct Plan<40> { using type = RList<8, 5>; };
template <> struct Plan<48> { using type = RList<8, 6>; };
template <> struct Plan<64> { using type = RList<8, 8>; };
template <> struct Plan<72> { using type = RList<8, 9>; };
template <int R0, int R1> constexpr int first_of(RList<R0, R1>) { return R0; }
template <int R0, int R1> constexpr int second_of(RList<R0, R1>) { return R1; }

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

// W_R^e = cos(2 pi e / R) + SIGN i sin(2 pi e / R) for the composite radices
template <int R> struct TwC;
template <> struct TwC<6> {
  static constexpr double c[3] = {1.0, 0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.86602540378443864676, 0.86602540378443864676};
};
template <> struct TwC<8> {
  static constexpr double c[4] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440};
  static constexpr double s[4] = {0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440};
};
template <> struct TwC<9> {
  static constexpr double c[5] = {1.0, 0.76604444311897803520, 0.17364817766693034885, -0.5,
                                  -0.93969262078590838405};
  static constexpr double s[5] = {0.0, 0.64278760968653932632, 0.98480775301220805936,
                                  0.86602540378443864676, 0.34202014332566873304};
};

// DFT of R = R1 * R2 points from R2 DFTs of R1 points (subsequences
// a[R2 m + l]), twiddles W_R^(l k1), then R1 DFTs of R2 points:
//   y[k1 + R1 k2] = sum_l W_R^(l k1) (sum_m a[R2 m + l] W_R1^(m k1)) W_R2^(l k2)
template <int R1, int R2, int SIGN, typename T>
__device__ __forceinline__ void dft_composite(cplx<T>* a) {
  constexpr int R = R1 * R2;
  cplx<T> b[R2][R1];
#pragma unroll
  for (int l = 0; l < R2; ++l) {
#pragma unroll
    for (int m = 0; m < R1; ++m) b[l][m] = a[m * R2 + l];
    Dft<R1, SIGN, T>::run(b[l]);
  }
#pragma unroll
  for (int l = 1; l < R2; ++l) {
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      const int e = l * k1;
      const cplx<T> w{T(TwC<R>::c[e]), T(SIGN * TwC<R>::s[e])};
      b[l][k1] = b[l][k1] * w;
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cplx<T> c[R2];
#pragma unroll
    for (int l = 0; l < R2; ++l) c[l] = b[l][k1];
    Dft<R2, SIGN, T>::run(c);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = c[k2];
  }
}

template <int SIGN, typename T> struct Dft<6, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* a) { dft_composite<3, 2, SIGN, T>(a); }
};
template <int SIGN, typename T> struct Dft<8, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* a) { dft_composite<4, 2, SIGN, T>(a); }
};
template <int SIGN, typename T> struct Dft<9, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* a) { dft_composite<3, 3, SIGN, T>(a); }
};

// --- one stage ----------------------------------------------------------
// Stage with explicit load/store functors: ld(t, e) -> value, st(t, e, v).
// MID: barrier between the load and the store phase (in-place in LDS).
// TFAST: consecutive threads take consecutive sequences (use when elements
// are strided and sequences are adjacent); otherwise consecutive butterflies
// of one sequence (elements adjacent).
template <typename T, int N, int R, int P, int SIGN, int NT, int MAXCNT, bool TFAST, bool MID, class Ld, class St>
__device__ __forceinline__ void fft_stage_ls(const cplx<T>* tw, int cnt, Ld ld, St st) {
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
      for (int r = 0; r < R; ++r) v[k][r] = ld(t, i + r * M);
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
  if (MID) __syncthreads();
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int b = tid + k * NT;
    if (b < nb) {
      int t, i;
      if (TFAST) { t = b % cnt; i = b / cnt; } else { i = b % M; t = b / M; }
      const int kk = i % P;
      const int j = (i - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) st(t, j + r * P, v[k][r]);
    }
  }
  __syncthreads();
}

// Global-memory ends of a transform that reads and writes through an index
// map (index < 0: no element there).  A thread loads all its indices before
// any value that depends on them, so it waits on memory twice per stage
// rather than once per element (an element-by-element gather serialises an
// index load and a value load per element).

// The indices of a thread's elements in a stage of radix R after
// sub-transforms of size P (the output positions of fft_stage_ls).
template <int N, int R, int P, int NT, int MAXCNT, bool TFAST, class Idx>
__device__ __forceinline__ void stage_out_index(int cnt, Idx idx, int (&ci)[(MAXCNT * (N / R) + NT - 1) / NT][R]) {
  constexpr int M = N / R;
  constexpr int MAXB = (MAXCNT * M + NT - 1) / NT;
  const int nb = cnt * M;
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    // threads past the last butterfly load the first one's indices (always
    // valid) and drop them: the loads stay unconditional and independent
    const int b = threadIdx.x + k * NT;
    const int bb = b < nb ? b : 0;
    int t, i;
    if (TFAST) { t = bb % cnt; i = bb / cnt; } else { i = bb % M; t = bb / M; }
    const int kk = i % P;
    const int j = (i - kk) * R + kk;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = idx(t, j + r * P);
      ci[k][r] = b < nb ? c : -1;
    }
  }
}

// The indices of a thread's elements in a first stage (P = 1) of radix R
// (the input positions of fft_stage_ls).
template <int N, int R, int NT, int MAXCNT, bool TFAST, class Idx>
__device__ __forceinline__ void stage_in_index(int cnt, Idx idx, int (&ci)[(MAXCNT * (N / R) + NT - 1) / NT][R]) {
  constexpr int M = N / R;
  constexpr int MAXB = (MAXCNT * M + NT - 1) / NT;
  const int nb = cnt * M;
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int b = threadIdx.x + k * NT;
    const int bb = b < nb ? b : 0;   // as in stage_out_index
    int t, i;
    if (TFAST) { t = bb % cnt; i = bb / cnt; } else { i = bb % M; t = bb / M; }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = idx(t, i + r * M);
      ci[k][r] = b < nb ? c : -1;
    }
  }
}

// First stage (P = 1, no twiddles) with its inputs gathered from src[ci]
// (ci from stage_in_index with the same parameters; zero where negative),
// results stored by st(t, e, v), closing barrier as in fft_stage_ls.
template <typename T, int N, int R, int SIGN, int NT, int MAXCNT, bool TFAST, class St>
__device__ __forceinline__ void fft_stage_gather(int cnt, const int (&ci)[(MAXCNT * (N / R) + NT - 1) / NT][R],
                                                 const cplx<T>* __restrict__ src, St st) {
  constexpr int M = N / R;
  constexpr int MAXB = (MAXCNT * M + NT - 1) / NT;
  const int nb = cnt * M;
  cplx<T> v[MAXB][R];
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = ci[k][r];
      const cplx<T> x = src[c >= 0 ? c : 0];   // src[0] exists; its value is discarded
      v[k][r] = c >= 0 ? x : cplx<T>{0, 0};
    }
  }
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < nb) {
      int t, i;
      if (TFAST) { t = b % cnt; i = b / cnt; } else { i = b % M; t = b / M; }
      Dft<R, SIGN, T>::run(v[k]);
      const int j = i * R;
#pragma unroll
      for (int r = 0; r < R; ++r) st(t, j + r, v[k][r]);
    }
  }
  __syncthreads();
}

// Last stage with its outputs scattered to dst[ci] (ci from stage_out_index
// with the same parameters, loaded ahead by the caller; negative: dropped).
// No closing barrier: nothing in the workgroup reads the results.
template <typename T, int N, int R, int P, int SIGN, int NT, int MAXCNT, bool TFAST, class Ld>
__device__ __forceinline__ void fft_stage_scatter(const cplx<T>* tw, int cnt, Ld ld,
                                                  const int (&ci)[(MAXCNT * (N / R) + NT - 1) / NT][R],
                                                  cplx<T>* __restrict__ dst) {
  constexpr int M = N / R;
  constexpr int MAXB = (MAXCNT * M + NT - 1) / NT;
  constexpr int TWS = N / (P * R);
  const int nb = cnt * M;
  cplx<T> v[MAXB][R];
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < nb) {
      int t, i;
      if (TFAST) { t = b % cnt; i = b / cnt; } else { i = b % M; t = b / M; }
      const int kk = i % P;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = ld(t, i + r * M);
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
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (ci[k][r] >= 0) dst[ci[k][r]] = v[k][r];
  }
}

template <typename T, int N, int R, int P, int SIGN, int NT, int MAXCNT, bool TFAST, class Addr>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, const cplx<T>* tw, int cnt, Addr addr) {
  fft_stage_ls<T, N, R, P, SIGN, NT, MAXCNT, TFAST, true>(
      tw, cnt, [&](int t, int e) { return buf[addr(t, e)]; },
      [&](int t, int e, cplx<T> x) { buf[addr(t, e)] = x; });
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

// Single stage with explicit radix R and sub-transform size P (building block
// of kernels that fuse work between stages).
template <typename T, int N, int R, int P, int SIGN, int NT, int MAXCNT, bool TFAST, class Addr>
__device__ __forceinline__ void fft_one_stage(cplx<T>* buf, const cplx<T>* tw, int cnt, Addr addr) {
  fft_stage<T, N, R, P, SIGN, NT, MAXCNT, TFAST>(buf, tw, cnt, addr);
}

// Row filter: in place on `cnt` rows, y <- FFT(m * IFFT(y)) pointwise
// multiplier m (unnormalised transforms).  The inverse uses the reversed plan
// {B, A} so that its last stage and the forward first stage (both radix A)
// touch the same elements {i + r B}: that pair runs in registers around the
// multiply, three LDS round trips in all.  mul(t, e) returns the real factor.
template <typename T, int N, int NT, int MAXCNT, class Addr, class Mul>
__device__ __forceinline__ void fft_filter_rows(cplx<T>* buf, const cplx<T>* tw, int cnt, Addr addr, Mul mul) {
  constexpr int A = first_of(typename Plan<N>::type{});
  constexpr int B = second_of(typename Plan<N>::type{});
  // inverse stage 1: radix B, P = 1
  fft_stage<T, N, B, 1, +1, NT, MAXCNT, false>(buf, tw, cnt, addr);
  // inverse stage 2 (radix A, P = B) + multiply + forward stage 1 (radix A, P = 1)
  {
    constexpr int MAXB = (MAXCNT * B + NT - 1) / NT;
    const int nb = cnt * B;
    cplx<T> v[MAXB][A];
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      const int b = threadIdx.x + k * NT;
      if (b < nb) {
        const int i = b % B, t = b / B;
#pragma unroll
        for (int r = 0; r < A; ++r) v[k][r] = buf[addr(t, i + r * B)];
#pragma unroll
        for (int r = 1; r < A; ++r) {
          cplx<T> w = tw[r * i];
          w.y = -w.y;
          v[k][r] = v[k][r] * w;
        }
        Dft<A, +1, T>::run(v[k]);
#pragma unroll
        for (int r = 0; r < A; ++r) v[k][r] = mul(t, i + r * B) * v[k][r];
        Dft<A, -1, T>::run(v[k]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      const int b = threadIdx.x + k * NT;
      if (b < nb) {
        const int i = b % B, t = b / B;
#pragma unroll
        for (int r = 0; r < A; ++r) buf[addr(t, i * A + r)] = v[k][r];
      }
    }
    __syncthreads();
  }
  // forward stage 2: radix B, P = A
  fft_stage<T, N, B, A, -1, NT, MAXCNT, false>(buf, tw, cnt, addr);
}

// The row filter when only the rows' elements e in {0..h} U {N-h..N-1} carry
// data: the first stage reads those and takes zeros for the rest (which are
// never read from LDS, so they need not be cleared), the last stage stores
// only those outputs.  Same arithmetic as fft_filter_rows otherwise.
// TFAST: consecutive threads take consecutive rows (with a row stride of
// N + 1 elements the lanes of one LDS access then fall in distinct banks for
// every stage, including the stride-R stores of the stages with P = 1); else
// consecutive butterflies of one row.
template <typename T, int N, int NT, int MAXCNT, bool TFAST, class Addr, class Mul>
__device__ __forceinline__ void fft_filter_rows_pruned(cplx<T>* buf, const cplx<T>* tw, int cnt, int h, Addr addr,
                                                       Mul mul) {
  constexpr int A = first_of(typename Plan<N>::type{});
  constexpr int B = second_of(typename Plan<N>::type{});
  auto live = [h](int e) { return e <= h || e >= N - h; };
  // inverse stage 1: radix B, P = 1
  fft_stage_ls<T, N, B, 1, +1, NT, MAXCNT, TFAST, true>(
      tw, cnt, [&](int t, int e) { return live(e) ? buf[addr(t, e)] : cplx<T>{0, 0}; },
      [&](int t, int e, cplx<T> x) { buf[addr(t, e)] = x; });
  // inverse stage 2 (radix A, P = B) + multiply + forward stage 1 (radix A, P = 1)
  {
    constexpr int MAXB = (MAXCNT * B + NT - 1) / NT;
    const int nb = cnt * B;
    cplx<T> v[MAXB][A];
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      const int b = threadIdx.x + k * NT;
      if (b < nb) {
        const int t = TFAST ? b % cnt : b / B, i = TFAST ? b / cnt : b % B;
#pragma unroll
        for (int r = 0; r < A; ++r) v[k][r] = buf[addr(t, i + r * B)];
#pragma unroll
        for (int r = 1; r < A; ++r) {
          cplx<T> w = tw[r * i];
          w.y = -w.y;
          v[k][r] = v[k][r] * w;
        }
        Dft<A, +1, T>::run(v[k]);
#pragma unroll
        for (int r = 0; r < A; ++r) v[k][r] = mul(t, i + r * B) * v[k][r];
        Dft<A, -1, T>::run(v[k]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXB; ++k) {
      const int b = threadIdx.x + k * NT;
      if (b < nb) {
        const int t = TFAST ? b % cnt : b / B, i = TFAST ? b / cnt : b % B;
#pragma unroll
        for (int r = 0; r < A; ++r) buf[addr(t, i * A + r)] = v[k][r];
      }
    }
    __syncthreads();
  }
  // forward stage 2: radix B, P = A
  fft_stage_ls<T, N, B, A, -1, NT, MAXCNT, TFAST, true>(
      tw, cnt, [&](int t, int e) { return buf[addr(t, e)]; },
      [&](int t, int e, cplx<T> x) {
        if (live(e)) buf[addr(t, e)] = x;
      });
}

}  // namespace lgw
