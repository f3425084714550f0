// Shared device/host definitions of the lgw HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lgw {

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cplx {
  T x, y;
};
using z64 = cplx<double>;
using z32 = cplx<float>;

template <typename T> __host__ __device__ __forceinline__ cplx<T> mk(T a, T b) { return {a, b}; }
template <typename T> __host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.x, -a.y}; }
// conj(a) * b
template <typename T> __host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// multiply by +i (s=+1) or -i (s=-1)
template <int S, typename T> __host__ __device__ __forceinline__ cplx<T> muli(cplx<T> a) {
  return S > 0 ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}
template <typename T> __host__ __device__ __forceinline__ T norm2(cplx<T> a) { return a.x * a.x + a.y * a.y; }
template <typename T, typename U> __host__ __device__ __forceinline__ cplx<T> cvt(cplx<U> a) {
  return {static_cast<T>(a.x), static_cast<T>(a.y)};
}

// Plane-wave geometry shared by the transform kernels.  The sphere is stored
// in lexicographic order of the signed integer triples (mx, my, mz), so each
// z-column (mx, my) is a contiguous run mz = -h..h and the index of -m is
// npw - 1 - index(m).
struct Geom {
  int N;            // grid points per axis (cubic grid)
  int npw;          // plane waves in the sphere
  int ncols;        // z-columns holding at least one plane wave
  int hx, hy;       // max |mx|, max |my| over the sphere
  const int* col_start;  // [ncols] first sphere index of the column
  const int* col_h;      // [ncols] column holds mz in [-h, h]
  const int* col_pos;    // [ncols] (mx mod N) * N + (my mod N)
  const double* kin;     // [npw] |K|^2 / 2
  const int* col_of;     // [N * N] column at plane position x * N + y, -1 where none
};

// LDS position of element e of a length-N line with one pad slot every 8
// elements: Stockham stages write at strides of the radix, and the pad keeps
// 16-byte accesses at stride 8 off a single bank group.
__host__ __device__ constexpr int skew(int e) { return e + (e >> 3); }

// Map a "system" (one right-hand side of a batched solve) to its storage slot.
__device__ __forceinline__ int sys_of(const int* act, int b) { return act ? act[b] : b; }

}  // namespace lgw
